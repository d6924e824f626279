"""rg_trace_rays_noalloc (the entry point for callers that cannot allocate
device memory) against rg_trace_rays on the same inputs: two calls in a row,
the second with fewer rays, for the forms that use scratch (persistent
Dormand-Prince: refill queue; one-launch-per-step RK4: per-ray state) and
for persistent RK4 (no scratch).  Results must be bitwise equal (same
kernels, same launch parameters).  Sizes beyond the static scratch and
missing launch parameters are refused before any launch."""
import numpy as np
import pytest

from paper_2508_15967_amd import raygraph as rgb
from paper_2508_15967_amd import workloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _outs(torch, w):
    n = w.n
    return dict(x_out=torch.empty((w.dim, n), dtype=torch.float64, device="cuda"),
                k_out=torch.empty((w.dim, n), dtype=torch.float64, device="cuda"),
                t_out=torch.empty(n, dtype=torch.float64, device="cuda"),
                status_out=torch.empty(n, dtype=torch.int32, device="cuda"),
                steps_out=torch.empty(n, dtype=torch.int32, device="cuda"))


def _args(w, **kw):
    a = dict(integrator=w.integrator, dt=w.dt, n_steps=w.n_steps, h0=w.h0, rtol=w.rtol, atol=w.atol,
             hmin=w.hmin)
    if w.box_lo is not None:
        a["box"] = (list(w.box_lo), list(w.box_hi))
    a.update(kw)
    return a


@pytest.mark.parametrize("cfg,sizes,launch", [
    ("3", (8192, 3000), dict(block=256, compact_interval=8)),
    ("2", (20000, 5000), dict(mode=rgb.PLAIN, block=256)),
    ("2", (9000, 4100), dict(block=256, rays_per_lane=1)),
])
def test_noalloc_matches_trace(cfg, sizes, launch):
    torch = U.torch_mod()
    w = W.make(cfg, max(sizes))
    if cfg == "2":
        w.n_steps = 300
        w.store_every = 0
    _, _, prog, _ = U.program(w)
    prog.load()
    for n in sizes:
        print(f"[case] noalloc cfg={cfg} n={n} launch={launch}", flush=True)
        ww = w.select(np.arange(n))
        x0, k0, om = U.dev(ww.x0), U.dev(ww.k0), U.dev(ww.omega)
        extra = {}
        if ww.budget is not None:
            extra["budget"] = U.dev(ww.budget.astype(np.int32))
        res = []
        for noalloc in (False, True):
            outs = _outs(torch, ww)
            d = prog.make_desc(x0, k0, om, [], **_args(ww, **launch, **extra), **outs)
            if noalloc:
                d.workspace, d.workspace_bytes = None, 0  # ignored by the no-alloc form
                prog.trace_desc_noalloc(d)
            else:
                prog.trace_desc(d)
            torch.cuda.synchronize()
            res.append({k: v.cpu().numpy() for k, v in outs.items()})
        for k in res[0]:
            assert np.array_equal(res[0][k], res[1][k]), (n, k)


def test_noalloc_refusals():
    torch = U.torch_mod()
    w = W.make("2", 300000)
    w.n_steps = 5
    w.store_every = 0
    _, _, prog, _ = U.program(w)
    prog.load()
    x0, k0, om = U.dev(w.x0), U.dev(w.k0), U.dev(w.omega)
    outs = _outs(torch, w)
    # the plain form's per-ray state (16 bytes per ray) exceeds the 4 MiB array
    d = prog.make_desc(x0, k0, om, [], **_args(w, mode=rgb.PLAIN, block=256), **outs)
    with pytest.raises(rgb.RayGraphError) as e:
        prog.trace_desc_noalloc(d)
    assert e.value.status == rgb.RG_EINVAL and "static" in str(e.value)
    # no autotuning and no hipGraph in the no-alloc form
    for kw in (dict(block=0, rays_per_lane=1), dict(block=256, rays_per_lane=0),
               dict(block=256, rays_per_lane=1, use_hipgraph=True)):
        d = prog.make_desc(x0, k0, om, [], **_args(w, **kw), **outs)
        with pytest.raises(rgb.RayGraphError) as e:
            prog.trace_desc_noalloc(d)
        assert e.value.status == rgb.RG_EINVAL
