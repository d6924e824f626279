"""The boundary's caller-owned workspace: the library allocates no device
memory in the trace and adjoint calls; per-call scratch (the Dormand-Prince
refill queue, the per-step forms' per-ray state, the adjoint's segment
buffer and gradient partials) comes from a buffer the caller allocates
(torch) after asking for its size.  The adjoint accepts checkpoints = NULL
and then runs the forward itself inside the call."""
import ctypes as C

import numpy as np
import pytest

from paper_2508_15967_amd import raygraph as rgb
from paper_2508_15967_amd import workloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _desc(prog, w, torch, **kw):
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    n = w.n
    outs = dict(x_out=torch.empty((w.dim, n), dtype=torch.float64, device="cuda"),
                k_out=torch.empty((w.dim, n), dtype=torch.float64, device="cuda"),
                status_out=torch.empty(n, dtype=torch.int32, device="cuda"),
                steps_out=torch.empty(n, dtype=torch.int32, device="cuda"))
    args = dict(integrator=w.integrator, dt=w.dt, n_steps=w.n_steps, h0=w.h0, rtol=w.rtol,
                atol=w.atol, hmin=w.hmin)
    if w.budget is not None:
        args["budget"] = U.dev(w.budget.astype(np.int32))
    if w.box_lo is not None:
        args["box"] = (list(w.box_lo), list(w.box_hi))
    args.update(kw)
    d = prog.make_desc(x0, k0, om, [], **args, **outs)
    d._bufs = (x0, k0, om, outs, args)
    return d, outs


def test_workspace_sizes_and_refusals():
    """Persistent RK4 needs no workspace; the others report a size that
    grows with the ray count; a missing or short workspace is refused with a
    message before any launch."""
    torch = U.torch_mod()
    w1 = W.make("1", 300)
    w1.n_steps = 20
    _, _, prog1, _ = U.program(w1)
    d, _ = _desc(prog1, w1, torch)
    assert prog1.workspace_size(d) == 0
    d, _ = _desc(prog1, w1, torch, mode=rgb.PLAIN)
    assert prog1.workspace_size(d) >= 16 * 300
    w3 = W.make("3", 1000)
    _, _, prog3, _ = U.program(w3)
    d, _ = _desc(prog3, w3, torch, block=256, compact_interval=8)
    assert 8 <= prog3.workspace_size(d) <= 4096
    dp, _ = _desc(prog3, w3, torch, mode=rgb.PLAIN)
    assert prog3.workspace_size(dp) >= 1000 * (16 * 6 + 36)
    for ws, nbytes in ((None, 0), (d._ws, 4)):
        d.workspace, d.workspace_bytes = (None if ws is None else ws.data_ptr()), nbytes
        with pytest.raises(rgb.RayGraphError) as e:
            prog3.trace_desc(d)
        assert e.value.status == rgb.RG_EINVAL and "workspace" in str(e.value)
    # a workspace that overlaps an output is refused as well
    d2, outs = _desc(prog3, w3, torch, block=256, compact_interval=8)
    d2.workspace, d2.workspace_bytes = outs["x_out"].data_ptr(), 8 * 3 * 1000
    with pytest.raises(rgb.RayGraphError) as e:
        prog3.trace_desc(d2)
    assert e.value.status == rgb.RG_EINVAL and "overlaps" in str(e.value)


def test_dopri_traces_on_two_streams_with_own_workspaces():
    """Two Dormand-Prince traces of different rays enqueued on two streams at
    once, each with its own workspace (refill queue): results bitwise equal
    to the same traces run one after the other."""
    torch = U.torch_mod()
    w = W.make("3", 6000)
    wa, wb = w.select(np.arange(0, 3000)), w.select(np.arange(3000, 6000))
    _, _, prog, _ = U.program(w)
    ref = []
    for ww in (wa, wb):
        d, outs = _desc(prog, ww, torch, block=256, compact_interval=8, use_hipgraph=True)
        prog.trace_desc(d)
        torch.cuda.synchronize()
        ref.append({k: v.cpu().numpy() for k, v in outs.items()})
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    da, oa = _desc(prog, wa, torch, block=256, compact_interval=8, use_hipgraph=True)
    db, ob = _desc(prog, wb, torch, block=256, compact_interval=8, use_hipgraph=True)
    torch.cuda.synchronize()
    prog.trace_desc(da, s1)
    prog.trace_desc(db, s2)
    torch.cuda.synchronize()
    for r, o in zip(ref, (oa, ob)):
        for k, v in o.items():
            assert np.array_equal(r[k], v.cpu().numpy()), k


@pytest.mark.parametrize("cfg,n,steps,mode", [("4", 700, 350, rgb.PERSISTENT), ("5", 300, 250, rgb.PERSISTENT),
                                               ("4", 300, 230, rgb.PLAIN)])
def test_adjoint_without_checkpoints_runs_the_forward_itself(cfg, n, steps, mode):
    """fwd->checkpoints = NULL: the adjoint call recomputes the forward into
    its workspace; per-ray gradients bitwise equal to the adjoint on the
    stored checkpoints, parameter gradients up to the summation order, and
    the caller's forward outputs untouched."""
    torch = U.torch_mod()
    w = W.make(cfg, n)
    w.n_steps = steps
    print(f"[case] adjoint without checkpoints cfg={cfg} n={n} steps={steps} mode={mode}", flush=True)
    _, _, prog, params = U.program(w, want_adjoint=True)
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    pt = [U.dev(p) for p in params]
    out = prog.trace(x0, k0, om, pt, dt=w.dt, n_steps=w.n_steps, checkpoint_every=100, mode=mode)
    torch.cuda.synchronize()
    lx = (2.0 * (out["x"] - U.dev(w.targets))).contiguous()
    res = []
    for with_ckpt in (True, False):
        desc = out["_desc"]
        x_before = out["x"].clone()
        if not with_ckpt:
            desc.checkpoints = None
            desc.steps_out = None
            desc._adj_ws = None
            out["x"].fill_(7.0)  # not read and not written by the adjoint
        gx0, gk0 = torch.empty_like(x0), torch.empty_like(k0)
        gp = [torch.empty_like(p) for p in pt]
        prog.adjoint_desc(desc, lx, None, gx0, gk0, gp)
        torch.cuda.synchronize()
        if not with_ckpt:
            assert bool((out["x"] == 7.0).all())
        res.append((gx0.cpu().numpy(), gk0.cpu().numpy(), [g.cpu().numpy() for g in gp]))
    (ax, ak, ap), (bx, bk, bp) = res
    assert np.array_equal(ax, bx) and np.array_equal(ak, bk)
    for p1, p2 in zip(ap, bp):
        assert np.abs(p1 - p2).max() <= 1e-12 * np.abs(p1).max()


def test_adjoint_workspace_refused_when_short():
    torch = U.torch_mod()
    w = W.make("4", 256)
    w.n_steps = 120
    _, _, prog, params = U.program(w, want_adjoint=True)
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    pt = [U.dev(p) for p in params]
    out = prog.trace(x0, k0, om, pt, dt=w.dt, n_steps=w.n_steps, checkpoint_every=100)
    lx = (2.0 * (out["x"] - U.dev(w.targets))).contiguous()
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(rgb.RayGraphError) as e:
        prog.adjoint_desc(out["_desc"], lx, None, torch.empty_like(x0), None, [], workspace=small)
    assert e.value.status == rgb.RG_EINVAL and "workspace" in str(e.value)


def test_adjoint_gradient_buffers_may_not_overlap():
    """A parameter gradient that shares memory with a parameter it is the
    gradient of, or with another gradient output, is refused before any
    launch (it is zeroed before the parameters are read)."""
    torch = U.torch_mod()
    w = W.make("4", 256)
    w.n_steps = 120
    _, _, prog, params = U.program(w, want_adjoint=True)
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    pt = [U.dev(p) for p in params]
    out = prog.trace(x0, k0, om, pt, dt=w.dt, n_steps=w.n_steps, checkpoint_every=100)
    lx = (2.0 * (out["x"] - U.dev(w.targets))).contiguous()
    big = torch.empty(pt[0].numel() + x0.numel(), dtype=torch.float64, device="cuda")
    cases = (([pt[0]], torch.empty_like(x0), "overlaps params[0]"),
             ([big[:pt[0].numel()]], big[:x0.numel()].view(x0.shape), "overlaps dL_dparams[0]"))
    for gp, gx0, msg in cases:
        with pytest.raises(rgb.RayGraphError) as e:
            prog.adjoint_desc(out["_desc"], lx, None, gx0, None, gp)
        assert e.value.status == rgb.RG_EINVAL and msg in str(e.value), str(e.value)
    gx0 = torch.empty_like(x0)
    gp = [torch.empty_like(pt[0])]
    prog.adjoint_desc(out["_desc"], lx, None, gx0, None, gp)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(gp[0]).all()) and bool(torch.isfinite(gx0).all())


def test_descriptor_keeps_its_tensors():
    """A trace whose inputs were temporaries: the descriptor it returns
    holds them, so the adjoint on it, after new allocations of the same
    sizes, reads the launch states and parameters of the trace (bitwise the
    gradients of a trace whose inputs the caller kept)."""
    torch = U.torch_mod()
    w = W.make("5", 256)
    w.n_steps = 60
    _, _, prog, params = U.program(w, want_adjoint=True)
    res = []
    for keep in (True, False):
        x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
        pt = [U.dev(p) for p in params]
        out = prog.trace(x0, k0, om, pt, dt=w.dt, n_steps=w.n_steps, checkpoint_every=10)
        if not keep:
            del x0, k0, om, pt
            # blocks of the same sizes, filled with other values
            junk = [U.dev(np.full(a.shape, 3.0)) for a in (w.x0, w.k0, w.omega, *params)]
        lx = (2.0 * (out["x"] - U.dev(w.targets))).contiguous()
        gx0 = torch.empty((3, w.n), dtype=torch.float64, device="cuda")
        gk0 = torch.empty_like(gx0)
        gp = [torch.empty(p.size, dtype=torch.float64, device="cuda") for p in params]
        prog.adjoint_desc(out["_desc"], lx, None, gx0, gk0, gp)
        torch.cuda.synchronize()
        res.append((gx0.cpu().numpy(), gk0.cpu().numpy(), gp[0].cpu().numpy()))
        if not keep:
            del junk
    for a, b in zip(*res):
        assert np.array_equal(a, b)
