"""Launch-shape invariance and boundary behaviour on the GPU.

Each ray's arithmetic does not depend on which lane, wave or launch runs
it, so every tuning variant (block size, rays per lane, compaction
interval), the plain one-launch-per-step form, hipGraph replay and a trace
split in two and resumed must give bitwise-identical results."""
import numpy as np
import pytest

from paper_2508_15967_amd import raygraph as rgb
from paper_2508_15967_amd import workloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _same(a, b, keys=("x", "k", "t", "status", "steps")):
    for k in keys:
        assert np.array_equal(a[k], b[k]), k


def test_rk4_variants_bitwise():
    w = W.make("2", 5000)  # ragged: not a multiple of any block size
    w.n_steps = 400
    base = U.gpu_trace(w, block=256, rays_per_lane=1, store=True)
    for block in (64, 128, 512):
        for rpl in (1, 2, 4):
            print(f"[case] rk4 block={block} rpl={rpl}", flush=True)
            _same(base, U.gpu_trace(w, block=block, rays_per_lane=rpl, store=True), ("x", "k", "t", "traj"))
    for block in (256, 512):  # the kernel variant built for at least four waves per SIMD
        print(f"[case] rk4 block={block} min_waves_per_simd=4", flush=True)
        _same(base, U.gpu_trace(w, block=block, rays_per_lane=1, min_waves_per_simd=4, store=True),
              ("x", "k", "t", "traj"))
    pl = U.gpu_trace(w, mode=rgb.PLAIN, block=128, store=True)
    _same(base, pl, ("x", "k", "t", "status", "steps", "traj"))
    gr = U.gpu_trace(w, block=256, rays_per_lane=2, use_hipgraph=True, store=True)
    _same(base, gr, ("x", "k", "traj"))
    gr2 = U.gpu_trace(w, block=256, rays_per_lane=2, use_hipgraph=True, store=True)  # replay
    _same(base, gr2, ("x", "k", "traj"))


def test_rk4_autotuned_matches_fixed():
    w = W.make("1b", 1000)
    w.n_steps = 300
    a = U.gpu_trace(w)
    b = U.gpu_trace(w, block=64, rays_per_lane=1)
    _same(a, b)
    # the anisotropic medium's forward (natural register count above 128:
    # the four-wave variant differs in code, not in results)
    w5 = W.make("5", 3000)
    w5.n_steps = 200
    a5 = U.gpu_trace(w5, block=256, rays_per_lane=1)
    _same(a5, U.gpu_trace(w5, block=256, rays_per_lane=1, min_waves_per_simd=4))
    _same(a5, U.gpu_trace(w5))


def test_split_and_resume_bitwise():
    w = W.make("4", 3000)
    w.n_steps = 600
    full = U.gpu_trace(w, block=128, rays_per_lane=1)
    w1 = w.subset(w.n)
    w1.n_steps = 250
    a = U.gpu_trace(w1, block=128, rays_per_lane=1)
    w2 = w.subset(w.n)
    w2.x0, w2.k0 = a["x"], a["k"]
    w2.n_steps = 350
    b = U.gpu_trace(w2, block=128, rays_per_lane=1, t0=U.dev(a["t"]))
    assert np.array_equal(full["x"], b["x"]) and np.array_equal(full["k"], b["k"])
    assert np.array_equal(full["t"], b["t"])


def test_dopri_variants_bitwise():
    w = W.make("3", 6000)
    base = U.gpu_trace(w, block=128, compact_interval=32)
    for block, C in ((64, 8), (256, 128), (128, -1), (512, 1)):
        print(f"[case] dopri block={block} C={C}", flush=True)
        _same(base, U.gpu_trace(w, block=block, compact_interval=C))
    _same(base, U.gpu_trace(w, block=128, compact_interval=32, use_hipgraph=True))
    _same(base, U.gpu_trace(w, block=128, compact_interval=32, use_hipgraph=True))
    _same(base, U.gpu_trace(w, mode=rgb.PLAIN, block=256))


def test_status_paths_match_oracle(oracle):
    """Non-finite input, a start outside the box and a one-step budget give the
    same statuses, step counts and final states as the oracle."""
    w = W.make("3", 256)
    w.x0 = w.x0.copy()
    w.k0 = w.k0.copy()
    w.budget = w.budget.copy()
    w.x0[0, 0] = np.nan           # non-finite start
    w.x0[2, 1] = -1.0             # below the box floor
    w.budget[2] = 1               # one accepted step
    w.k0[:, 3] = [np.inf, 0, 0]   # non-finite wavevector
    g = U.gpu_trace(w, block=64, compact_interval=16)
    o = oracle.trace(w)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["steps"], o["steps"])
    assert g["status"][0] == rgb.RAY_NONFINITE and g["status"][3] == rgb.RAY_NONFINITE
    assert g["status"][1] == rgb.RAY_EXITED_BOX and g["steps"][1] == 1
    assert g["status"][2] == rgb.RAY_BUDGET and g["steps"][2] == 1
    fin = np.isfinite(o["x"]).all(0) & np.isfinite(o["k"]).all(0)
    ex, ek = U.ray_errors(g, o, w.omega, w.dim)
    assert ex[fin].max() < U.TOL and ek[fin].max() < U.TOL
    # rays frozen at a non-finite state: the same state, NaN for NaN
    for key in ("x", "k"):
        assert np.array_equal(g[key][:, ~fin], o[key][:, ~fin], equal_nan=True), key
    assert np.array_equal(g["t"][~fin], o["t"][~fin])
    # RK4 with a non-finite start freezes at the start with NONFINITE
    w4 = W.make("1", 64)
    w4.x0 = w4.x0.copy()
    w4.x0[1, 5] = np.nan
    w4.n_steps = 50
    g4 = U.gpu_trace(w4, block=64, rays_per_lane=1)
    o4 = oracle.trace(w4)
    assert np.array_equal(g4["status"], o4["status"]) and g4["status"][5] == rgb.RAY_NONFINITE
    assert np.array_equal(g4["steps"], o4["steps"])


def test_empty_and_single_ray(oracle):
    torch = U.torch_mod()
    w = W.make("1", 1)
    w.n_steps = 100
    g = U.gpu_trace(w)
    o = oracle.trace(w)
    ex, ek = U.ray_errors(g, o, w.omega, w.dim)
    assert ex.max() < U.TOL and ek.max() < U.TOL
    _, _, prog, _ = U.program(w)
    e = torch.empty((2, 0), dtype=torch.float64, device="cuda")
    d = prog.make_desc(e, e, torch.empty(0, dtype=torch.float64, device="cuda"), dt=1e-3, n_steps=10,
                       x_out=e, k_out=e)
    prog.trace_desc(d)  # zero rays is a no-op


@pytest.mark.parametrize("mode", [rgb.PERSISTENT, rgb.PLAIN])
def test_zero_steps(mode):
    """n_steps = 0, the degenerate trace: the endpoints are the launch
    states (bitwise), no step is taken, and the adjoint is the identity map
    (dL/dx0 = dL/dx_end, dL/dk0 = dL/dk_end) with zero parameter
    gradients."""
    torch = U.torch_mod()
    w = W.make("5", 96)
    w.n_steps = 0
    print(f"[case] zero steps mode={mode}", flush=True)
    _, _, prog, params = U.program(w, want_adjoint=True)
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    pt = [U.dev(p) for p in params]
    out = prog.trace(x0, k0, om, pt, dt=w.dt, n_steps=0, checkpoint_every=10, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(out["x"], x0) and torch.equal(out["k"], k0)
    assert int(out["steps"].abs().max()) == 0 and int(out["status"].abs().max()) == 0
    assert float(out["t"].abs().max()) == 0.0
    lx = (2.0 * (out["x"] - U.dev(w.targets))).contiguous()
    lk = torch.ones_like(k0)
    gx0, gk0 = torch.empty_like(x0), torch.empty_like(k0)
    gp = [torch.full_like(p, 5.0) for p in pt]
    prog.adjoint_desc(out["_desc"], lx, lk, gx0, gk0, gp)
    torch.cuda.synchronize()
    assert torch.equal(gx0, lx) and torch.equal(gk0, lk)
    assert all(float(g.abs().max()) == 0.0 for g in gp)


def test_boundary_rejects_bad_buffers():
    """Host pointers, undersized device buffers and overlapping outputs are
    refused before any launch (RG_EINVAL), with a message."""
    torch = U.torch_mod()
    w = W.make("1", 128)
    _, _, prog, _ = U.program(w)
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    xo = torch.empty((2, 128), dtype=torch.float64, device="cuda")
    ko = torch.empty((2, 128), dtype=torch.float64, device="cuda")
    d = prog.make_desc(x0, k0, om, dt=1e-3, n_steps=10, x_out=xo, k_out=ko)
    host = np.zeros((2, 128))
    d.x_out = host.ctypes.data
    with pytest.raises(rgb.RayGraphError) as e:
        prog.trace_desc(d)
    assert e.value.status == rgb.RG_EINVAL and "device memory" in str(e.value)
    small = torch.empty(2 * 128 - 1, dtype=torch.float64, device="cuda")
    # a separate allocation that is too small for 2 x 128 doubles
    torch.cuda.empty_cache()
    d = prog.make_desc(x0, k0, om, dt=1e-3, n_steps=10, x_out=xo, k_out=ko)
    d.n_rays = 1 << 30  # claims far more rays than the buffers hold
    with pytest.raises(rgb.RayGraphError) as e:
        prog.trace_desc(d)
    assert e.value.status == rgb.RG_EINVAL and "smaller than required" in str(e.value)
    del small
    d = prog.make_desc(x0, k0, om, dt=1e-3, n_steps=10, x_out=xo, k_out=ko, block=96)
    with pytest.raises(rgb.RayGraphError):
        prog.trace_desc(d)
    # outputs may not overlap inputs or each other (the autotuner's sample
    # runs write the outputs before the trace reads its inputs)
    for xo2, ko2, what in ((x0, ko, "overlaps input x0"), (xo, xo, "overlaps k_out")):
        d = prog.make_desc(x0, k0, om, dt=1e-3, n_steps=10, x_out=xo2, k_out=ko2)
        with pytest.raises(rgb.RayGraphError) as e:
            prog.trace_desc(d)
        assert e.value.status == rgb.RG_EINVAL and what in str(e.value), str(e.value)


@pytest.mark.parametrize("cfg,n,steps", [("4", 1000, 300), ("5", 300, 300)])
def test_plain_adjoint_matches_persistent(cfg, n, steps):
    """The per-step-launch adjoint (fwd.mode = RG_PLAIN) against the
    persistent one on the same forward (ragged ray counts): per-ray
    gradients bitwise, parameter gradients up to the summation order."""
    torch = U.torch_mod()
    w = W.make(cfg, n)
    w.n_steps = steps
    print(f"[case] plain adjoint cfg={cfg} n={n} steps={steps}", flush=True)
    _, _, prog, params = U.program(w, want_adjoint=True)
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    pt = [U.dev(p) for p in params]
    out = prog.trace(x0, k0, om, pt, dt=w.dt, n_steps=w.n_steps, checkpoint_every=100)
    lx = (2.0 * (out["x"] - U.dev(w.targets))).contiguous()
    res = []
    for mode in (rgb.PERSISTENT, rgb.PLAIN):
        desc = out["_desc"]
        desc.mode = mode
        gx0, gk0 = torch.empty_like(x0), torch.empty_like(k0)
        gp = [torch.empty_like(p) for p in pt]
        prog.adjoint_desc(desc, lx, None, gx0, gk0, gp)
        torch.cuda.synchronize()
        res.append((gx0.cpu().numpy(), gk0.cpu().numpy(), [g.cpu().numpy() for g in gp]))
    (ax, ak, ap), (bx, bk, bp) = res
    assert np.array_equal(ax, bx) and np.array_equal(ak, bk)
    for p1, p2 in zip(ap, bp):
        assert np.abs(p1 - p2).max() <= 1e-12 * np.abs(p1).max()


def test_step_underflow_matches_oracle(oracle):
    """Dormand-Prince with a tolerance the first steps cannot meet and a
    floor hmin on the step size: about half the rays end with
    RAY_STEP_UNDERFLOW after a run of rejected attempts, the others leave
    the box.  Statuses, accepted steps, attempts and end states as the
    oracle's (same controller decisions; the parity rules of the
    Dormand-Prince tests for a decision that rounding flips)."""
    from tests.test_gpu_parity import _dopri_check
    w = W.make("3", 2048)
    w.rtol = w.atol = 1e-11
    w.h0, w.hmin = 2.0, 0.05
    print("[case] step underflow", flush=True)
    g = U.gpu_trace(w, block=128, compact_interval=8)
    bad, o = U.ill_conditioned(oracle, w)
    _dopri_check(oracle, w, g, o, bad, 0.99)
    n_uf = int((g["status"] == rgb.RAY_STEP_UNDERFLOW).sum())
    assert 0.2 * w.n < n_uf < 0.8 * w.n, n_uf
    assert abs(int((o["status"] == rgb.RAY_STEP_UNDERFLOW).sum()) - n_uf) <= 2


@pytest.mark.parametrize("t_end", [3.7, 35.0])
def test_t_end_stop_matches_oracle(oracle, t_end):
    """Dormand-Prince with an end time: the last step is shortened to land on
    t_end (status RAY_OK, t == t_end exactly on both sides); with the later
    end time about half the rays leave the box first."""
    from tests.test_gpu_parity import _dopri_check
    w = W.make("3", 2048)
    print(f"[case] t_end {t_end}", flush=True)
    g = U.gpu_trace(w, block=256, compact_interval=8, t_end=t_end)
    bad, o = U.ill_conditioned(oracle, w, t_end=t_end)
    _dopri_check(oracle, w, g, o, bad, 0.99)
    done = g["status"] == rgb.RAY_OK
    assert done.sum() > 0.4 * w.n and np.all(g["t"][done] == t_end)
    assert np.array_equal(done, o["status"] == rgb.RAY_OK)
    if t_end > 10:
        assert (g["status"] == rgb.RAY_EXITED_BOX).sum() > 0.3 * w.n


def test_trace_stats_and_kernel_time():
    """rg_trace_stats reduces a finished trace's statuses, steps and attempts
    on the GPU: the same counts, sums and maxima as numpy over the outputs;
    rg_last_launch reports the last call's device time once it has run."""
    torch = U.torch_mod()
    w = W.make("3", 6000)
    _, _, prog, _ = U.program(w)
    g = U.gpu_trace(w, block=128, compact_interval=8)
    desc = g["_t"]["_desc"]
    torch.cuda.synchronize()
    ms = prog.last_launch()["last_kernel_ms"]
    assert ms > 0.0, ms
    st = prog.trace_stats(desc)
    for s in range(5):
        assert st["by_status"][s] == int((g["status"] == s).sum()), s
    assert st["other_status"] == 0
    assert st["steps"] == int(g["steps"].astype(np.int64).sum())
    assert st["attempts"] == int(g["attempts"].astype(np.int64).sum())
    assert st["rejected"] == st["attempts"] - st["steps"] > 0
    assert st["max_steps"] == int(g["steps"].max()) and st["max_attempts"] == int(g["attempts"].max())
    # fixed-step RK4: steps only, attempts 0
    w2 = W.make("2", 3000)
    w2.n_steps = 200
    g2 = U.gpu_trace(w2, block=256, rays_per_lane=1)
    _, _, prog2, _ = U.program(w2)
    st2 = prog2.trace_stats(g2["_t"]["_desc"])
    assert st2["by_status"][0] == 3000 and st2["steps"] == 3000 * 200 and st2["attempts"] == 0
    assert st2["max_steps"] == 200


@pytest.mark.parametrize("cfg", ["2", "3"])
def test_hipgraph_replays_match_eager(cfg):
    """One descriptor traced again and again with use_hipgraph: the first
    call captures the launch sequence (for Dormand-Prince the fill kernel
    that resets the refill queue, then the persistent kernel), the later
    calls replay the cached graph.  Between the replays the program runs
    eager work (a direct trace and a point evaluation) and the host
    synchronises; the outputs are overwritten with NaN before each replay,
    and every replay equals the eager trace bitwise."""
    torch = U.torch_mod()
    w = W.make(cfg, 3000)
    if cfg == "2":
        w.n_steps = 300
    print(f"[case] hipgraph replays cfg={cfg}", flush=True)
    launch = dict(block=256, rays_per_lane=1) if cfg == "2" else dict(block=128, compact_interval=32)
    eager = U.gpu_trace(w, **launch)
    _, _, prog, params = U.program(w)
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    args = dict(integrator=w.integrator, dt=w.dt, n_steps=w.n_steps, h0=w.h0, rtol=w.rtol, atol=w.atol,
                hmin=w.hmin, use_hipgraph=True, **launch)
    if w.budget is not None:
        args["budget"] = U.dev(w.budget.astype(np.int32))
    if w.box_lo is not None:
        args["box"] = (list(w.box_lo), list(w.box_hi))
    out = {"x": torch.empty((3, w.n), dtype=torch.float64, device="cuda"),
           "k": torch.empty((3, w.n), dtype=torch.float64, device="cuda"),
           "t": torch.empty(w.n, dtype=torch.float64, device="cuda"),
           "status": torch.empty(w.n, dtype=torch.int32, device="cuda"),
           "steps": torch.empty(w.n, dtype=torch.int32, device="cuda")}
    d = prog.make_desc(x0, k0, om, [], x_out=out["x"], k_out=out["k"], t_out=out["t"],
                       status_out=out["status"], steps_out=out["steps"], **args)
    y = U.dev(np.concatenate([w.x0[:, :64], w.k0[:, :64]]))
    for rep in range(4):
        for v in out.values():
            v.fill_(-1 if v.dtype == torch.int32 else float("nan"))
        torch.cuda.synchronize()
        prog.trace_desc(d)
        torch.cuda.synchronize()
        for key in ("x", "k", "t", "status", "steps"):
            assert np.array_equal(out[key].cpu().numpy(), eager[key]), (rep, key)
        # eager work of the same program between the replays
        U.gpu_trace(w, **launch)
        prog.eval(y, U.dev(w.omega[:64]))
        torch.cuda.synchronize()
