#!/usr/bin/env python3
"""Benchmark: FP64 ray-steps/s of the compiled-graph ray tracer on one MI355X.

One benchmark step = one full trace of the workload (every ray advanced by
every step of its integrator) with inputs resident in HBM.  Default workload:
the 3-D stratified layer, 1,048,576 rays x 10,000 RK4 steps, every 100th
state stored (101 snapshots, 5.08 GB).  Other workloads (--config 1..5) are
available for separate runs; 4 and 5 add the adjoint pass (fwd+adj).

Printed: one JSON line with the persistent-kernel throughput, the plain
one-launch-per-step comparator, a roofline entry for the dominant kernel
(FP64 vector ALU bound, flops counted from the compiled graph) and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 128 flop/clk x 2.4 GHz
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="2")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed plain-form traces")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=0, help="oracle sample size (0 = auto)")
    ap.add_argument("--traffic", default="",
                    help="HBM-traffic summary (default: profiles/traffic_<kernel>_<workload>.txt)")
    ap.add_argument("--rays", type=int, default=0, help="trace only the first N rays of the workload (0 = all)")
    ap.add_argument("--block", type=int, default=0, help="fix the block size (0 = autotuned)")
    ap.add_argument("--rpl", type=int, default=0, help="fix rays per lane (0 = autotuned)")
    ap.add_argument("--compact", type=int, default=0, help="fix the compaction interval (0 = autotuned)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle sample time")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the single precision side measurement (RK4 forward workloads)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the ray tracer runs on one GPU; --gpus must be 1 "
                          "(sharding rays over several GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    from paper_2508_15967_amd import media, raygraph as rgb, workloads as W

    w = W.make(args.config)
    full_size = not (0 < args.rays < w.n)
    if not full_size:
        w = w.subset(args.rays)
    adjoint = args.config in ("4", "5")
    dev = torch.device("cuda:0")
    g, D, params = media.build(w.medium)
    t0 = time.time()
    prog = g.compile(D, want_adjoint=adjoint)
    compile_s = time.time() - t0
    info = prog.info()
    n, d, ny = w.n, w.dim, 2 * w.dim
    x0 = torch.from_numpy(w.x0).to(dev)
    k0 = torch.from_numpy(w.k0).to(dev)
    om = torch.from_numpy(w.omega).to(dev)
    pt = [torch.from_numpy(p).to(dev) for p in params]
    kw = dict(integrator=w.integrator, dt=w.dt, n_steps=w.n_steps, h0=w.h0, rtol=w.rtol,
              atol=w.atol, hmin=w.hmin)
    if w.budget is not None:
        kw["budget"] = torch.from_numpy(w.budget.astype(np.int32)).to(dev)
    if w.box_lo is not None:
        kw["box"] = (list(w.box_lo), list(w.box_hi))
    outs = {"x_out": torch.empty((d, n), dtype=torch.float64, device=dev),
            "k_out": torch.empty((d, n), dtype=torch.float64, device=dev),
            "t_out": torch.empty(n, dtype=torch.float64, device=dev),
            "status_out": torch.empty(n, dtype=torch.int32, device=dev),
            "steps_out": torch.empty(n, dtype=torch.int32, device=dev)}
    if w.integrator == W.DOPRI54:
        outs["attempts_out"] = torch.empty(n, dtype=torch.int32, device=dev)
    if w.store_every > 0:
        ns = w.n_steps // w.store_every + 1
        outs["traj"] = torch.empty((ns, ny, n), dtype=torch.float64, device=dev)
        kw["store_every"] = w.store_every
    ckpt = None
    if adjoint:
        nc = (w.n_steps + w.ckpt_every - 1) // w.ckpt_every
        ckpt = torch.empty((nc, ny + 1, n), dtype=torch.float64, device=dev)
        kw["checkpoint_every"] = w.ckpt_every
        kw["checkpoints"] = ckpt
    stream = torch.cuda.current_stream()

    def make(mode):
        return prog.make_desc(x0, k0, om, pt, mode=mode, use_hipgraph=True, block=args.block,
                              rays_per_lane=args.rpl, compact_interval=args.compact, **kw, **outs)

    if args.calib_copy_mb > 0:
        src = torch.ones(args.calib_copy_mb * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    desc = make(rgb.PERSISTENT)
    adj = {}
    if adjoint:
        tx = torch.from_numpy(w.targets).to(dev)
        adj = {"lx": torch.empty((d, n), dtype=torch.float64, device=dev),
               "gx0": torch.empty((d, n), dtype=torch.float64, device=dev),
               "gk0": torch.empty((d, n), dtype=torch.float64, device=dev),
               "gp": [torch.empty_like(p) for p in pt], "tx": tx}

    def fwd():
        prog.trace_desc(desc, stream)

    def bwd():
        # dL/dx_end of L = sum |x_end - target|^2
        torch.mul(outs["x_out"] - adj["tx"], 2.0, out=adj["lx"])
        prog.adjoint_desc(desc, adj["lx"], None, adj["gx0"], adj["gk0"], adj["gp"], stream)

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    progress(f"workload {w.name}: {n} rays, compiled in {compile_s:.1f} s")
    # warmup (includes autotuning and hipGraph capture on the first call)
    t0 = time.time()
    for _ in range(max(args.warmup, 1)):
        fwd()
        if adjoint:
            bwd()
    torch.cuda.synchronize()
    warm_s = time.time() - t0
    launch = prog.last_launch()

    # timed region
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    evb = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)] if adjoint else []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    progress(f"warmup done in {warm_s:.1f} s")
    for i in range(args.steps):
        ev[i][0].record(stream)
        fwd()
        ev[i][1].record(stream)
        if adjoint:
            evb[i][0].record(stream)
            bwd()
            evb[i][1].record(stream)
    torch.cuda.synchronize()
    progress("timed steps done")
    wall = time.perf_counter() - t0
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    bwd_ms = float(np.mean([a.elapsed_time(b) for a, b in evb])) if adjoint else 0.0

    st = outs["status_out"].cpu().numpy()
    steps = outs["steps_out"].cpu().numpy().astype(np.int64)
    ray_steps = int(steps.sum())
    ms_per_step = wall * 1e3 / args.steps
    value = ray_steps * args.steps / wall

    if w.integrator == W.RK4:
        flops_alg = info["rk4_step_flops_alg"] * ray_steps
        flops_iss = info["rk4_step_flops_issued"] * ray_steps
    else:
        # every attempt (accepted or rejected) costs one attempt's flops
        attempts = int(outs["attempts_out"].cpu().numpy().astype(np.int64).sum())
        flops_alg = info["dopri_attempt_flops_alg"] * attempts
        flops_iss = info["dopri_attempt_flops_issued"] * attempts
    # ray-invariant operations (constants, parameters, omega only) run once
    # per ray, outside the step loop
    inv_fwd = info["rhs_flops_ray_invariant"] * n
    flops_alg += inv_fwd
    flops_iss += inv_fwd
    if adjoint:
        inv_adj = (info["rhs_flops_ray_invariant"] + info["vjp_flops_ray_invariant"]) * n
        flops_alg_adj = info["adj_step_flops_alg"] * ray_steps + inv_adj
        flops_iss_adj = info["adj_step_flops_issued"] * ray_steps + inv_adj
    # the roofline entry is for the dominant kernel of one step
    if w.integrator == W.RK4:
        kname = "rg_rk4_r%d" % launch["rays_per_lane"]
    else:
        kname = "rg_dopri_persistent"
    kernel_ms, k_alg, k_iss = fwd_ms, flops_alg, flops_iss
    if adjoint and bwd_ms > fwd_ms:
        kname, kernel_ms, k_alg, k_iss = "rg_rk4_adjoint", bwd_ms, flops_alg_adj, flops_iss_adj
    achieved = k_alg / (kernel_ms * 1e-3) / 1e12
    achieved_iss = k_iss / (kernel_ms * 1e-3) / 1e12

    # HBM bytes per launch of that kernel from the rocprofv3 FETCH_SIZE and
    # WRITE_SIZE passes (calibrated against a copy of known size), valid
    # only for the source they were taken on
    def profile_entry(path):
        """key: value pairs of a committed counter summary, if it was taken on
        this kernel, workload and generated source"""
        if not (os.path.exists(path) and full_size):
            return None
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                key, val = line.split(":", 1)
                kv[key.strip()] = val.strip()
        ok = (kv.get("source_hash") == "%016x" % info["source_hash"] and kv.get("kernel") == kname
              and kv.get("workload") == w.name)
        return kv if ok else None

    tkv = profile_entry(args.traffic or os.path.join(ROOT, "profiles", f"traffic_{kname}_{w.name}.txt"))
    traffic = float(tkv["hbm_bytes_per_launch"]) if tkv else None
    # FP64 flops per ray-step counted by the hardware (SQ_INSTS_VALU_FLOPS_FP64)
    fkv = profile_entry(os.path.join(ROOT, "profiles", f"fp64_{kname}_{w.name}.txt"))
    hw_flops = float(fkv["fp64_flops_per_ray_step"]) if fkv else None

    result = {
        "metric": ("FP64 ray-steps/s (persistent fused RK4, one launch per trace)" if w.integrator == W.RK4 else
                   "FP64 accepted ray-steps/s (persistent Dormand-Prince 5(4) with in-kernel refill)"),
        "value": value, "unit": "ray-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n_rays": n, "integrator": "RK4" if w.integrator == W.RK4 else "DOPRI54",
                   "n_steps": w.n_steps, "dt": w.dt, "store_every": w.store_every,
                   "ray_steps_per_trace": ray_steps, "adjoint": adjoint,
                   **({"attempts_per_trace": attempts} if w.integrator == W.DOPRI54 else {})},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": kname, "kernel_ms": kernel_ms,
                     "flops_per_ray_step_alg": k_alg / max(ray_steps, 1),
                     "achieved_issued": achieved_iss, "frac_issued": achieved_iss / PEAK_FP64_TFLOPS,
                     "hw_fp64_flops_per_ray_step": hw_flops,
                     "frac_hw": (hw_flops * ray_steps / (kernel_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS
                                 if hw_flops else None)},
        "launch": launch, "compile_s": compile_s, "warmup_s": warm_s,
        "source_hash": "%016x" % info["source_hash"],
        "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
    }
    if adjoint:
        tot_ms = fwd_ms + bwd_ms
        result["metric"] = "FP64 ray-steps/s fwd+adjoint (persistent RK4 + checkpointed discrete adjoint)"
        result["value"] = value
        result["fwd"] = {"ray_steps_per_s": ray_steps / (fwd_ms * 1e-3), "ms": fwd_ms}
        result["fwd_adj"] = {"ray_steps_per_s": ray_steps / (tot_ms * 1e-3), "ms": tot_ms,
                             "adj_ms": bwd_ms,
                             "tflops_alg": (flops_alg + flops_alg_adj) / (tot_ms * 1e-3) / 1e12,
                             "tflops_issued": (flops_iss + flops_iss_adj) / (tot_ms * 1e-3) / 1e12}
        result["fwd_adj"]["frac_alg"] = result["fwd_adj"]["tflops_alg"] / PEAK_FP64_TFLOPS
        result["fwd_adj"]["frac_issued"] = result["fwd_adj"]["tflops_issued"] / PEAK_FP64_TFLOPS

    # hand-derived-derivative kernels for the anisotropic medium (speed
    # reference for the compiled kernels on the same inputs)
    if args.config == "5":
        progress("hand-derived kernels")
        from paper_2508_15967_amd import hand
        hm = hand.medium_struct(w.medium)
        hx, hk = torch.empty_like(x0), torch.empty_like(k0)
        hcp = torch.empty_like(ckpt)
        hgx, hgk, hgs = torch.empty_like(x0), torch.empty_like(k0), torch.empty_like(pt[0])
        hl = torch.empty_like(x0)
        def hand_fwd():
            hand.trace(hm, x0, k0, om, pt[0], w.dt, w.n_steps, hx, hk, w.ckpt_every, hcp, stream=stream)
        def hand_bwd():
            torch.mul(hx - adj["tx"], 2.0, out=hl)
            hand.adjoint(hm, om, pt[0], w.dt, w.n_steps, w.ckpt_every, hcp, hl, None, hgx, hgk, hgs,
                         stream=stream)
        hand_fwd(); hand_bwd()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream); hand_fwd(); e[1].record(stream); hand_bwd(); e[2].record(stream)
        torch.cuda.synchronize()
        hf, hb = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
        result["hand"] = {"fwd_ms": hf, "adj_ms": hb,
                          "fwd_ray_steps_per_s": ray_steps / (hf * 1e-3),
                          "fwd_adj_ray_steps_per_s": ray_steps / ((hf + hb) * 1e-3),
                          "compiled_over_hand_fwd": hf / fwd_ms,
                          "compiled_over_hand_fwd_adj": (hf + hb) / (fwd_ms + bwd_ms)}

    # single precision variant (float state and right-hand side, same outputs
    # in double, D residual monitored in double): a side line, not the metric
    if not args.no_fp32 and w.integrator == W.RK4 and not adjoint and w.medium.kind != W.SPLINE2D:
        prog32 = g.compile(D, fp32=True)
        x64, k64 = outs["x_out"].clone(), outs["k_out"].clone()
        desc32 = prog32.make_desc(x0, k0, om, pt, mode=rgb.PERSISTENT, use_hipgraph=True,
                                  precision=rgb.FP32, block=args.block, **kw, **outs)
        prog32.trace_desc(desc32, stream)  # warm: tuning and capture
        torch.cuda.synchronize()
        e32 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        for a_, b_ in e32:
            a_.record(stream)
            prog32.trace_desc(desc32, stream)
            b_.record(stream)
        torch.cuda.synchronize()
        ms32 = float(np.mean([a_.elapsed_time(b_) for a_, b_ in e32]))
        steps32 = int(outs["steps_out"].cpu().numpy().astype(np.int64).sum())
        dx = torch.linalg.vector_norm(outs["x_out"] - x64, dim=0) / torch.clamp(
            torch.linalg.vector_norm(x64, dim=0), min=1.0)
        result["fp32"] = {"value": steps32 / (ms32 * 1e-3), "unit": "ray-steps/s", "ms_per_trace": ms32,
                          "speedup_vs_fp64": fwd_ms / ms32, "launch": prog32.last_launch(),
                          "median_rel_dev_x_vs_fp64": float(dx.median()),
                          "frac_rays_dev_x_gt_1e-3": float((dx > 1e-3).double().mean())}
        outs["x_out"].copy_(x64)
        outs["k_out"].copy_(k64)

    # plain one-launch-per-step comparator on the same GPU and inputs
    if not args.no_plain:
        progress("plain comparator")
        pdesc = prog.make_desc(x0, k0, om, pt, mode=rgb.PLAIN, use_hipgraph=False, **kw, **outs)
        prog.trace_desc(pdesc, stream)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            prog.trace_desc(pdesc, stream)
        torch.cuda.synchronize()
        pw = (time.perf_counter() - t0) / args.plain_steps
        psteps = int(outs["steps_out"].cpu().numpy().astype(np.int64).sum())
        result["plain"] = {"value": psteps / pw, "ms_per_trace": pw * 1e3,
                           "launches_per_trace": w.n_steps + 2 if w.integrator == W.RK4 else None}
        # forward against forward
        result["speedup_vs_plain"] = (pw * 1e3 / psteps) / (fwd_ms / ray_steps)
        if adjoint:
            # the adjoint in its per-step form on the plain forward's checkpoints
            def plain_bwd():
                torch.mul(outs["x_out"] - adj["tx"], 2.0, out=adj["lx"])
                prog.adjoint_desc(pdesc, adj["lx"], None, adj["gx0"], adj["gk0"], adj["gp"], stream)
            plain_bwd()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.plain_steps):
                plain_bwd()
            torch.cuda.synchronize()
            pb = (time.perf_counter() - t0) / args.plain_steps
            result["plain"]["adj_ms"] = pb * 1e3
            result["plain"]["fwd_adj_value"] = psteps / (pw + pb)
            result["plain"]["adj_launches"] = 2 * w.n_steps + 2 * ((w.n_steps + w.ckpt_every - 1) // w.ckpt_every) + 3
            result["speedup_vs_plain_fwd_adj"] = (pw + pb) * 1e3 / (fwd_ms + bwd_ms)

    # CPU oracle on a bounded sample of the same workload: a pilot run sizes
    # the sample to about --cpu-seconds of work on all host cores
    if not args.no_cpu:
        progress("oracle sample on the host cores")
        from oracle import pyoracle
        pyoracle.build(force=False)
        cores = pyoracle.threads()

        def oracle_run(m):
            ws = w.subset(min(m, w.n))
            t0 = time.perf_counter()
            ro = pyoracle.trace(ws)
            if adjoint:
                lam = np.concatenate([2 * (ro["x"] - ws.targets), np.zeros_like(ro["k"])])
                pyoracle.adjoint(ws, lam)
            return ws, ro, time.perf_counter() - t0

        m = args.cpu_rays
        if not m:
            # pilot runs grow until one takes a second, then one sized run
            m = min(w.n, 4 * cores)
            while True:
                _, _, ps = oracle_run(m)
                if ps >= 1.0 or m >= w.n:
                    break
                m = min(w.n, m * 8)
            m = int(min(w.n, max(m, m * args.cpu_seconds / max(ps, 1e-3))))
        ws, ro, cs = oracle_run(m)
        if not args.cpu_rays and cs < 0.5 * args.cpu_seconds and m < w.n:
            # the pilots' per-ray time was off (start-up costs): size again
            m = int(min(w.n, m * args.cpu_seconds / max(cs, 1e-3)))
            ws, ro, cs = oracle_run(m)
        crs = int(ro["steps"].astype(np.int64).sum())
        result["cpu_baseline"] = {"value": crs / cs, "unit": "ray-steps/s" + (" (fwd+adj)" if adjoint else ""),
                                  "cores": cores, "kind": "oracle",
                                  "sample": f"first {ws.n} of {w.n} rays of {w.name}, all steps"
                                            f"{' fwd+adj' if adjoint else ''}, {cs:.1f} s"}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
