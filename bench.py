#!/usr/bin/env python3
"""Benchmark: FP64 ray-steps/s of the compiled-graph ray tracer on one MI355X,
forward and forward+adjoint, against the FP64 vector peak and against the
one-launch-per-step form.

One benchmark step = one full forward trace of the workload followed by its
checkpointed discrete adjoint (every ray advanced by every step, then swept
back), with inputs resident in HBM.  Default workload: the anisotropic medium
k.A(x).k - omega^2 with 16 Gaussian blobs, 1,048,576 rays x 20,000 RK4
steps, checkpoints every 10 steps, gradients of L = sum |x_end - target|^2
with respect to the launch states and the 16 blob scales.  A ray-step is one
ray advanced by one accepted step; for forward+adjoint the forward's
ray-steps are counted once.

Printed: one JSON line with the persistent-kernel throughput (forward and
forward+adjoint), the roofline entry of the dominant kernel (the adjoint;
FP64 vector ALU bound, flops counted from the compiled graph), the plain
one-launch-per-step comparator, the hand-derived kernels on the same inputs,
the CPU oracle timed on a bounded sample of the same workload, and the
stratified-layer forward (1,048,576 rays x 10,000 steps) as a nested entry.
Other workloads: --config 1..5 | cp (the cold-plasma workload; its k_x is
found by the library's Newton solve before tracing, off the clock).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 128 flop/clk x 2.4 GHz
METRIC = "FP64 ray-steps/s fwd and fwd+adjoint; % FP64 vector peak vs plain launch"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="5")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed plain-form traces")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-hand", action="store_true", help="skip the hand-derived kernels (workload 5)")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the nested stratified-layer forward entry")
    ap.add_argument("--cpu-rays", type=int, default=0, help="oracle sample size (0 = auto)")
    ap.add_argument("--traffic", default="",
                    help="HBM-traffic summary (default: profiles/traffic_<kernel>_<workload>.txt)")
    ap.add_argument("--rays", type=int, default=0, help="trace only the first N rays of the workload (0 = all)")
    ap.add_argument("--block", type=int, default=0, help="fix the block size (0 = autotuned)")
    ap.add_argument("--rpl", type=int, default=0, help="fix rays per lane (0 = autotuned)")
    ap.add_argument("--compact", type=int, default=0, help="fix the compaction interval (0 = autotuned)")
    ap.add_argument("--min-waves", type=int, default=0,
                    help="4: the RK4 kernel variant built for at least four waves per SIMD (0 = autotuned)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle sample time")
    ap.add_argument("--ckpt-every", type=int, default=0,
                    help="adjoint checkpoint interval in steps (0 = the workload's, 100)")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the single precision side measurement (RK4 forward workloads)")
    return ap.parse_args()


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


class Bench:
    """One workload on the GPU: inputs, outputs and descriptors, and the
    measurements of the persistent path, the plain comparator and the
    roofline entry."""

    def __init__(self, cfg, args, rays=0, full_workload=True):
        import torch
        from paper_2508_15967_amd import media, workloads as W
        self.torch, self.W, self.args, self.cfg = torch, W, args, cfg
        w = W.make(cfg)
        self.full_size = not (0 < rays < w.n)
        if not self.full_size:
            w = w.subset(rays)
        if args.ckpt_every > 0 and w.ckpt_every > 0:
            w.ckpt_every = args.ckpt_every
        self.w = w
        self.adjoint = cfg in ("4", "5") and full_workload
        dev = self.dev = torch.device("cuda:0")
        g, D, params = media.build(w.medium)
        self.g, self.D = g, D
        t0 = time.time()
        self.prog = g.compile(D, want_adjoint=self.adjoint)
        self.compile_s = time.time() - t0
        self.info = self.prog.info()
        n, d, ny = w.n, w.dim, 2 * w.dim
        self.x0 = torch.from_numpy(w.x0).to(dev)
        self.k0 = torch.from_numpy(w.k0).to(dev)
        self.om = torch.from_numpy(w.omega).to(dev)
        self.pt = [torch.from_numpy(p).to(dev) for p in params]
        self.newton = None
        if w.solve_k >= 0:
            # launch conditions: the wavevector component solve_k by Newton's
            # method on D = 0 from the branch-selecting guess (setup, untimed)
            it, Dres, mx = self.prog.solve_k(self.x0, self.k0, self.om, self.pt, component=w.solve_k,
                                             tol=1e-15, max_iter=60)
            torch.cuda.synchronize()
            self.newton = {"component": w.solve_k, "max_abs_D": float(mx.item()),
                           "unconverged": int((it < 0).sum().item()), "max_iters": int(it.max().item())}
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
        self.ckpt = None
        if self.adjoint:
            nc = (w.n_steps + w.ckpt_every - 1) // w.ckpt_every
            self.ckpt = torch.empty((nc, ny + 1, n), dtype=torch.float64, device=dev)
            kw["checkpoint_every"] = w.ckpt_every
            kw["checkpoints"] = self.ckpt
        self.kw, self.outs = kw, outs
        self.stream = torch.cuda.current_stream()
        self.desc = self.make(0, args.block, args.rpl, args.compact, args.min_waves)
        if self.adjoint:
            self.adj = {"lx": torch.empty((d, n), dtype=torch.float64, device=dev),
                        "gx0": torch.empty((d, n), dtype=torch.float64, device=dev),
                        "gk0": torch.empty((d, n), dtype=torch.float64, device=dev),
                        "gp": [torch.empty_like(p) for p in self.pt],
                        "tx": torch.from_numpy(w.targets).to(dev)}

    def make(self, mode, block=0, rpl=0, compact=0, min_waves=0):
        return self.prog.make_desc(self.x0, self.k0, self.om, self.pt, mode=mode, use_hipgraph=True,
                                   block=block, rays_per_lane=rpl, compact_interval=compact,
                                   min_waves_per_simd=min_waves, **self.kw, **self.outs)

    def fwd(self, desc=None):
        self.prog.trace_desc(desc or self.desc, self.stream)

    def bwd(self, desc=None):
        # dL/dx_end of L = sum |x_end - target|^2
        a = self.adj
        self.torch.mul(self.outs["x_out"] - a["tx"], 2.0, out=a["lx"])
        self.prog.adjoint_desc(desc or self.desc, a["lx"], None, a["gx0"], a["gk0"], a["gp"], self.stream)

    def run(self, steps, warmup):
        """Warm-up (autotuning and hipGraph capture on the first call), then
        `steps` timed steps bracketed by synchronisations; kernel times from
        HIP events on the stream the kernels run on."""
        torch = self.torch
        t0 = time.time()
        for _ in range(max(warmup, 1)):
            self.fwd()
            if self.adjoint:
                self.bwd()
        torch.cuda.synchronize()
        self.warm_s = time.time() - t0
        self.launch = self.prog.last_launch()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        evb = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)] if self.adjoint else []
        torch.cuda.synchronize()
        progress(f"{self.w.name}: warmup done in {self.warm_s:.1f} s")
        t0 = time.perf_counter()
        for i in range(steps):
            ev[i][0].record(self.stream)
            self.fwd()
            ev[i][1].record(self.stream)
            if self.adjoint:
                evb[i][0].record(self.stream)
                self.bwd()
                evb[i][1].record(self.stream)
        torch.cuda.synchronize()
        self.wall = time.perf_counter() - t0
        progress(f"{self.w.name}: timed steps done")
        self.fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        self.bwd_ms = float(np.mean([a.elapsed_time(b) for a, b in evb])) if self.adjoint else 0.0
        self.steps = steps
        self.status = self.outs["status_out"].cpu().numpy()
        self.ray_steps = int(self.outs["steps_out"].cpu().numpy().astype(np.int64).sum())
        self.attempts = (int(self.outs["attempts_out"].cpu().numpy().astype(np.int64).sum())
                         if "attempts_out" in self.outs else None)

    def flops(self):
        """Algorithmic and issued flops of one forward and of one adjoint."""
        info, n = self.info, self.w.n
        if self.w.integrator == self.W.RK4:
            f_alg = info["rk4_step_flops_alg"] * self.ray_steps
            f_iss = info["rk4_step_flops_issued"] * self.ray_steps
        else:
            # every attempt (accepted or rejected) costs one attempt's flops
            f_alg = info["dopri_attempt_flops_alg"] * self.attempts
            f_iss = info["dopri_attempt_flops_issued"] * self.attempts
        # ray-invariant operations (constants, parameters, omega only) run
        # once per ray, outside the step loop
        inv = info["rhs_flops_ray_invariant"] * n
        out = {"fwd": (f_alg + inv, f_iss + inv)}
        if self.adjoint:
            inv_a = (info["rhs_flops_ray_invariant"] + info["vjp_flops_ray_invariant"]) * n
            out["adj"] = (info["adj_step_flops_alg"] * self.ray_steps + inv_a,
                          info["adj_step_flops_issued"] * self.ray_steps + inv_a)
        return out

    def profile_entry(self, path, kname):
        """key: value pairs of a committed counter summary, if it was taken on
        this kernel, workload and generated source"""
        if not (os.path.exists(path) and self.full_size):
            return None
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                key, val = line.split(":", 1)
                kv[key.strip()] = val.strip()
        ok = (kv.get("source_hash") == "%016x" % self.info["source_hash"] and kv.get("kernel") == kname
              and kv.get("workload") == self.w.name)
        return kv if ok else None

    def roofline(self, kname, kernel_ms, f_alg, f_iss, traffic_path=""):
        achieved = f_alg / (kernel_ms * 1e-3) / 1e12
        achieved_iss = f_iss / (kernel_ms * 1e-3) / 1e12
        # HBM bytes per launch of that kernel from the rocprofv3 FETCH_SIZE and
        # WRITE_SIZE passes (calibrated against a copy of known size), valid
        # only for the source they were taken on
        tkv = self.profile_entry(traffic_path or os.path.join(ROOT, "profiles", f"traffic_{kname}_{self.w.name}.txt"),
                                 kname)
        traffic = float(tkv["hbm_bytes_per_launch"]) if tkv else None
        # FP64 flops per ray-step counted by the hardware (SQ_INSTS_VALU_FLOPS_FP64)
        fkv = self.profile_entry(os.path.join(ROOT, "profiles", f"fp64_{kname}_{self.w.name}.txt"), kname)
        hw = float(fkv["fp64_flops_per_ray_step"]) if fkv else None
        rs = max(self.ray_steps, 1)
        return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic, "kernel": kname,
                "kernel_ms": kernel_ms, "flops_per_ray_step_alg": f_alg / rs,
                "flops_per_ray_step_issued": f_iss / rs,
                "achieved_issued": achieved_iss, "frac_issued": achieved_iss / PEAK_FP64_TFLOPS,
                "hw_fp64_flops_per_ray_step": hw,
                "frac_hw": (hw * self.ray_steps / (kernel_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS
                            if hw else None),
                "hbm_gbs": (traffic / (kernel_ms * 1e-3) / 1e9 if traffic else None)}

    def fwd_kernel(self):
        if self.w.integrator == self.W.RK4:
            if self.launch.get("min_waves_per_simd") == 4:
                return "rg_rk4_r1o4"
            return "rg_rk4_r%d" % self.launch["rays_per_lane"]
        return "rg_dopri_persistent"

    def plain(self):
        """The paper's one launch per step on the same GPU and inputs."""
        torch = self.torch
        progress(f"{self.w.name}: plain comparator")
        pdesc = self.make(1)
        pdesc.use_hipgraph = 0
        self.fwd(pdesc)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(self.args.plain_steps):
            self.fwd(pdesc)
        torch.cuda.synchronize()
        pw = (time.perf_counter() - t0) / self.args.plain_steps
        psteps = int(self.outs["steps_out"].cpu().numpy().astype(np.int64).sum())
        out = {"value": psteps / pw, "ms_per_trace": pw * 1e3,
               "launches_per_trace": self.w.n_steps + 2 if self.w.integrator == self.W.RK4 else None,
               "speedup_vs_plain": (pw * 1e3 / psteps) / (self.fwd_ms / self.ray_steps)}
        if self.w.integrator == self.W.RK4 and psteps == self.w.n * self.w.n_steps:
            # every launch reads and writes each ray's state (2 dim doubles),
            # t, status and step count and reads omega; plus the stored
            # snapshots and checkpoints
            ny = 2 * self.w.dim
            b = 16 * ny + 40
            if self.w.store_every > 0:
                b += 8 * ny / self.w.store_every
            if self.adjoint:
                b += 8 * (ny + 1) / self.w.ckpt_every
            out["alg_bytes_per_ray_step"] = b
            out["hbm_gbs_alg"] = b * psteps / pw / 1e9
        if self.adjoint:
            # the adjoint in its per-step form on the plain forward's checkpoints
            self.bwd(pdesc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(self.args.plain_steps):
                self.bwd(pdesc)
            torch.cuda.synchronize()
            pb = (time.perf_counter() - t0) / self.args.plain_steps
            out["adj_ms"] = pb * 1e3
            out["fwd_adj_value"] = psteps / (pw + pb)
            out["adj_launches"] = (2 * self.w.n_steps + 2 * ((self.w.n_steps + self.w.ckpt_every - 1)
                                                             // self.w.ckpt_every) + 3)
            out["speedup_vs_plain_fwd_adj"] = (pw + pb) * 1e3 / (self.fwd_ms + self.bwd_ms)
        return out

    def fp32(self):
        """Single precision variant (float state and right-hand side, same
        outputs in double, D residual monitored in double): a side line."""
        torch, outs = self.torch, self.outs
        prog32 = self.g.compile(self.D, fp32=True)
        x64, k64 = outs["x_out"].clone(), outs["k_out"].clone()
        desc32 = prog32.make_desc(self.x0, self.k0, self.om, self.pt, mode=0, use_hipgraph=True,
                                  precision=1, block=self.args.block, **self.kw, **outs)
        prog32.trace_desc(desc32, self.stream)  # warm: tuning and capture
        torch.cuda.synchronize()
        e32 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2)]
        for a_, b_ in e32:
            a_.record(self.stream)
            prog32.trace_desc(desc32, self.stream)
            b_.record(self.stream)
        torch.cuda.synchronize()
        ms32 = float(np.mean([a_.elapsed_time(b_) for a_, b_ in e32]))
        steps32 = int(outs["steps_out"].cpu().numpy().astype(np.int64).sum())
        dx = torch.linalg.vector_norm(outs["x_out"] - x64, dim=0) / torch.clamp(
            torch.linalg.vector_norm(x64, dim=0), min=1.0)
        res = {"value": steps32 / (ms32 * 1e-3), "unit": "ray-steps/s", "ms_per_trace": ms32,
               "speedup_vs_fp64": self.fwd_ms / ms32, "launch": prog32.last_launch(),
               "median_rel_dev_x_vs_fp64": float(dx.median()),
               "frac_rays_dev_x_gt_1e-3": float((dx > 1e-3).double().mean())}
        outs["x_out"].copy_(x64)
        outs["k_out"].copy_(k64)
        return res

    def hand(self):
        """Hand-derived-derivative kernels for the anisotropic medium: the
        speed reference for the compiled kernels on the same inputs."""
        torch, w, a = self.torch, self.w, self.adj
        progress("hand-derived kernels")
        from paper_2508_15967_amd import hand
        hm = hand.medium_struct(w.medium)
        hx, hk = torch.empty_like(self.x0), torch.empty_like(self.k0)
        hcp = self.ckpt  # the compiled runs are done; their checkpoints are rewritten by the plain leg
        hgx, hgk, hgs = torch.empty_like(self.x0), torch.empty_like(self.k0), torch.empty_like(self.pt[0])
        hl = torch.empty_like(self.x0)
        hws = torch.empty(hand.workspace_size(w.n, w.ckpt_every), dtype=torch.uint8, device=self.dev)

        def hand_fwd():
            hand.trace(hm, self.x0, self.k0, self.om, self.pt[0], w.dt, w.n_steps, hx, hk, w.ckpt_every, hcp,
                       stream=self.stream)

        def hand_bwd():
            torch.mul(hx - a["tx"], 2.0, out=hl)
            hand.adjoint(hm, self.om, self.pt[0], w.dt, w.n_steps, w.ckpt_every, hcp, hl, None, hgx, hgk, hgs,
                         stream=self.stream, workspace=hws)
        hand_fwd()
        hand_bwd()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(self.stream)
        hand_fwd()
        e[1].record(self.stream)
        hand_bwd()
        e[2].record(self.stream)
        torch.cuda.synchronize()
        hf, hb = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
        return {"fwd_ms": hf, "adj_ms": hb, "fwd_ray_steps_per_s": self.ray_steps / (hf * 1e-3),
                "fwd_adj_ray_steps_per_s": self.ray_steps / ((hf + hb) * 1e-3),
                "compiled_over_hand_fwd": hf / self.fwd_ms,
                "compiled_over_hand_fwd_adj": (hf + hb) / (self.fwd_ms + self.bwd_ms)}

    def cpu_baseline(self):
        """The oracle on a bounded sample of the same workload: a pilot run
        sizes the sample to about --cpu-seconds of work on all host cores."""
        progress("oracle sample on the host cores")
        from oracle import pyoracle
        pyoracle.build(force=False)
        cores = pyoracle.threads()
        w, args, adjoint = self.w, self.args, self.adjoint

        def oracle_run(m):
            ws = w.subset(min(m, w.n))
            if w.solve_k >= 0:  # the oracle's own Newton launch conditions (untimed setup)
                ws.k0, _, _ = pyoracle.newton_k(ws.medium, ws.x0, ws.k0, ws.omega, component=w.solve_k,
                                                tol=1e-15, max_iter=60)
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
        return {"value": crs / cs, "unit": "ray-steps/s" + (" (fwd+adj)" if adjoint else ""),
                "cores": cores, "cpu_model": cpu_model(), "kind": "oracle",
                "sample": f"first {ws.n} of {w.n} rays of {w.name}, all steps"
                          f"{' fwd+adj' if adjoint else ''}, {cs:.1f} s"}

    def release(self):
        for k in list(self.__dict__):
            if k not in ("args", "torch", "W"):
                delattr(self, k)
        self.torch.cuda.empty_cache()


def forward_entry(b: Bench, with_plain=True, with_fp32=False):
    """Forward-only measurement of a workload as a dict."""
    fl = b.flops()
    kname = b.fwd_kernel()
    e = {"workload": b.w.name, "n_rays": b.w.n, "n_steps": b.w.n_steps, "dt": b.w.dt,
         "integrator": "RK4" if b.w.integrator == b.W.RK4 else "DOPRI54",
         "store_every": b.w.store_every, "ray_steps_per_trace": b.ray_steps,
         "value": b.ray_steps / (b.fwd_ms * 1e-3), "unit": "ray-steps/s", "ms_per_trace": b.fwd_ms,
         "roofline": b.roofline(kname, b.fwd_ms, *fl["fwd"]), "launch": b.launch,
         "source_hash": "%016x" % b.info["source_hash"]}
    if b.attempts is not None:
        e["attempts_per_trace"] = b.attempts
    if with_fp32:
        e["fp32"] = b.fp32()
    if with_plain:
        e["plain"] = b.plain()
    return e


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the ray tracer runs on one GPU; --gpus must be 1 "
                          "(sharding rays over several GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    from paper_2508_15967_amd import workloads as W

    if args.calib_copy_mb > 0:
        src = torch.ones(args.calib_copy_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    b = Bench(args.config, args, rays=args.rays)
    w = b.w
    progress(f"workload {w.name}: {w.n} rays, compiled in {b.compile_s:.1f} s")
    b.run(args.steps, args.warmup)
    fl = b.flops()
    value = b.ray_steps * args.steps / b.wall
    kname = b.fwd_kernel()
    cfg = {"workload": w.name, "n_rays": w.n, "integrator": "RK4" if w.integrator == W.RK4 else "DOPRI54",
           "n_steps": w.n_steps, "dt": w.dt, "store_every": w.store_every,
           "ray_steps_per_trace": b.ray_steps, "adjoint": b.adjoint}
    if b.attempts is not None:
        cfg["attempts_per_trace"] = b.attempts
    result = {
        "metric": METRIC, "value": value, "unit": "ray-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": b.wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg,
    }
    if b.adjoint:
        cfg["checkpoint_every"] = w.ckpt_every
        cfg["gradients"] = "dL/dx0, dL/dk0, dL/dtheta of L = sum |x_end - target|^2"
        tot_ms = b.fwd_ms + b.bwd_ms
        fa, fi = fl["fwd"][0] + fl["adj"][0], fl["fwd"][1] + fl["adj"][1]
        result["fwd"] = {"value": b.ray_steps / (b.fwd_ms * 1e-3), "ms": b.fwd_ms,
                         "roofline": b.roofline(kname, b.fwd_ms, *fl["fwd"])}
        result["fwd_adj"] = {"value": b.ray_steps / (tot_ms * 1e-3), "ms": tot_ms, "adj_ms": b.bwd_ms,
                             "tflops_alg": fa / (tot_ms * 1e-3) / 1e12,
                             "tflops_issued": fi / (tot_ms * 1e-3) / 1e12}
        result["fwd_adj"]["frac_alg"] = result["fwd_adj"]["tflops_alg"] / PEAK_FP64_TFLOPS
        result["fwd_adj"]["frac_issued"] = result["fwd_adj"]["tflops_issued"] / PEAK_FP64_TFLOPS
        # the dominant kernel of a step: the adjoint
        result["roofline"] = b.roofline("rg_rk4_adjoint", b.bwd_ms, *fl["adj"], traffic_path=args.traffic)
    else:
        result["metric"] = METRIC + " (forward only for this workload)"
        result["roofline"] = b.roofline(kname, b.fwd_ms, *fl["fwd"], traffic_path=args.traffic)
    result.update({"launch": b.launch, "compile_s": b.compile_s, "warmup_s": b.warm_s,
                   "source_hash": "%016x" % b.info["source_hash"],
                   "status_counts": {int(k): int(v) for k, v in zip(*np.unique(b.status, return_counts=True))}})
    if b.newton:
        result["newton_launch"] = b.newton
    if args.config == "5" and b.adjoint and not args.no_hand:
        result["hand"] = b.hand()
    if (not args.no_fp32 and w.integrator == W.RK4 and not b.adjoint
            and w.medium.kind != W.SPLINE2D):
        result["fp32"] = b.fp32()
    if not args.no_plain:
        p = b.plain()
        result["plain"] = p
        result["speedup_vs_plain"] = p.pop("speedup_vs_plain")
        if b.adjoint:
            result["speedup_vs_plain_fwd_adj"] = p.pop("speedup_vs_plain_fwd_adj")
    if not args.no_cpu:
        result["cpu_baseline"] = b.cpu_baseline()
    b.release()

    # the stratified layer forward (1,048,576 rays x 10,000 RK4 steps, 101
    # snapshots stored) as a nested entry of the default run
    if args.config == "5" and not args.no_side and not (0 < args.rays):
        s = Bench("2", args)
        progress(f"side workload {s.w.name}: {s.w.n} rays")
        s.run(args.steps, args.warmup)
        result["strat3d_fwd"] = forward_entry(s, with_plain=not args.no_plain, with_fp32=not args.no_fp32)
        s.release()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
