"""The GPU kernels on random dispersion relations (the generator of
test_emit_random.py: shared sub-sums, scaled sums, Gaussians, omega and
parameter elements, in two of them the time t with launch times t0 != 0,
in two others square roots, logarithms, integer powers, sines and
quotients;
in 3-D and 2-D, relations small enough for the unrolled stages and large
enough for the rolled stages with the constant table).  The reference is
the same emitted functions built as host C++ (which test_emit_random.py
checks against the graph's own derivatives), driven by a host RK4 loop, a
host discrete RK4 adjoint and a host Dormand-Prince controller written
from the method's definition: right-hand side and D at points to
rounding, endpoints after 200 steps and every 50th state to 1e-11 per ray,
D along the rays, dL/dx0, dL/dk0 per ray and dL/dtheta to 1e-9, the
Dormand-Prince step counts, attempts and statuses exactly, and the Newton
launch conditions against a host Newton over the graph's own derivative.  This covers
the kernels' handling of programs other than the five workload media."""
import ctypes as C
import re
import tempfile

import numpy as np
import pytest

from paper_2508_15967_amd import raygraph as rgb
from paper_2508_15967_amd import workloads as W
from tests import gpu_util as U
from tests.test_emit_host import _host_lib
from tests.test_emit_random import _random_D

pytestmark = pytest.mark.gpu


def _host_rhs(lib, y, om, t, pp, with_D=False):
    n = y.shape[1]
    y, t = np.ascontiguousarray(y), np.ascontiguousarray(t)
    f, D = np.zeros_like(y), np.zeros(n)
    lib.host_eval_t(n, y.shape[0], C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data),
                    C.c_void_p(t.ctypes.data), pp, C.c_void_p(f.ctypes.data), C.c_void_p(D.ctypes.data))
    return (f, D) if with_D else f


def _host_vjp(lib, y, om, t, pp, v, gp):
    y, v, t = np.ascontiguousarray(y), np.ascontiguousarray(v), np.ascontiguousarray(t)
    jv = np.zeros_like(y)
    lib.host_vjp_t(y.shape[1], y.shape[0], C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data),
                   C.c_void_p(t.ctypes.data), pp, C.c_void_p(v.ctypes.data), C.c_void_p(jv.ctypes.data),
                   C.c_void_p(gp.ctypes.data))
    return jv


@pytest.mark.parametrize("seed,n_terms,dim,extra", [(1, 10, 3, ""), (4, 60, 3, ""), (8, 8, 2, ""), (9, 50, 2, ""),
                                                    (10, 12, 3, "t"), (11, 40, 2, "t"), (12, 10, 3, "ops"),
                                                    (15, 20, 2, "ops")])
def test_random_relation_matches_host_build(seed, n_terms, dim, extra):
    torch = U.torch_mod()
    rng = np.random.default_rng(seed)
    g = rgb.Graph(dim)
    with_t = extra == "t"
    D, _, _, _ = _random_D(g, rng, n_terms, dim, with_t, rich=extra == "ops")
    ny = 2 * dim
    print(f"[case] random relation seed={seed} terms={n_terms} dim={dim} {extra}", flush=True)
    prog = g.compile(D, want_adjoint=True)
    src = prog.source()
    ns = int(prog.info()["n_grad_slots"])
    elems = [int(t) for t in re.search(r"rg_grad_elem\[\d+\] = \{([^}]*)\}", src).group(1).split(",")][:ns]
    params = [np.ascontiguousarray(rng.uniform(0.5, 1.5, 4))]
    n, steps, dt = 512, 200, 1e-3
    y0 = np.ascontiguousarray(np.concatenate([rng.uniform(-1.0, 1.0, (dim, n)), rng.uniform(0.5, 1.5, (dim, n))]))
    om = np.full(n, 1.5)
    t0 = rng.uniform(0.0, 3.0, n) if with_t else np.zeros(n)
    target = rng.uniform(-1.0, 1.0, (dim, n))
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, True, tmp)
        pp = (C.c_void_p * 8)(params[0].ctypes.data, *([None] * 7))
        # right-hand side and D at points
        fg, Dg = prog.eval(U.dev(y0), U.dev(om), [U.dev(params[0])], t=U.dev(t0))
        fh = _host_rhs(lib, y0, om, t0, pp)
        scale = np.abs(fh).max(axis=0)
        assert (np.abs(fg.cpu().numpy() - fh).max(axis=0) / scale).max() < 1e-13
        # RK4 forward on the host, every stage state kept for the adjoint,
        # every 50th state and D there kept as snapshots
        Y = np.zeros((steps, 4, ny, n))
        snaps, snaps_D = [], []
        y = y0.copy()
        T = np.zeros((steps + 1, n))  # time of each step's start, as the integrator accumulates it
        T[0] = t0
        for s in range(steps + 1):
            if s % 50 == 0:
                snaps.append(y.copy())
                snaps_D.append(_host_rhs(lib, y, om, T[s], pp, with_D=True)[1])
            if s == steps:
                break
            t, th = T[s], T[s] + 0.5 * dt
            Y[s, 0] = y
            k1 = _host_rhs(lib, y, om, t, pp)
            Y[s, 1] = y + 0.5 * dt * k1
            k2 = _host_rhs(lib, Y[s, 1], om, th, pp)
            Y[s, 2] = y + 0.5 * dt * k2
            k3 = _host_rhs(lib, Y[s, 2], om, th, pp)
            Y[s, 3] = y + dt * k3
            k4 = _host_rhs(lib, Y[s, 3], om, t + dt, pp)
            y = y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
            T[s + 1] = T[s] + dt
        # rays whose host trajectory moves by more than 1e-12 when the last
        # bit of the launch state is flipped are ill-conditioned (rounding
        # differences grow there beyond the tolerances): set aside, at most
        # U.MAX_ILL of them
        yp = np.nextafter(y0, np.inf)
        for s in range(steps):
            t, th = T[s], T[s] + 0.5 * dt
            k1 = _host_rhs(lib, yp, om, t, pp)
            k2 = _host_rhs(lib, yp + 0.5 * dt * k1, om, th, pp)
            k3 = _host_rhs(lib, yp + 0.5 * dt * k2, om, th, pp)
            k4 = _host_rhs(lib, yp + dt * k3, om, t + dt, pp)
            yp = yp + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        ex, ek = U.ray_errors({"x": yp[:dim], "k": yp[dim:]}, {"x": y[:dim], "k": y[dim:]}, om, dim)
        ok = np.maximum(ex, ek) <= 1e-12
        assert (~ok).mean() <= U.MAX_ILL
        # discrete adjoint of that map for L = sum |x_end - target|^2
        lam = np.concatenate([2.0 * (y[:dim] - target), np.zeros((dim, n))])
        gp = np.zeros(64)
        for s in range(steps - 1, -1, -1):
            t, th = T[s], T[s] + 0.5 * dt
            kb4 = dt / 6.0 * lam
            yb4 = _host_vjp(lib, Y[s, 3], om, t + dt, pp, kb4, gp)
            kb3 = dt / 3.0 * lam + dt * yb4
            yb3 = _host_vjp(lib, Y[s, 2], om, th, pp, kb3, gp)
            kb2 = dt / 3.0 * lam + 0.5 * dt * yb3
            yb2 = _host_vjp(lib, Y[s, 1], om, th, pp, kb2, gp)
            kb1 = dt / 6.0 * lam + 0.5 * dt * yb2
            yb1 = _host_vjp(lib, Y[s, 0], om, t, pp, kb1, gp)
            lam = lam + yb1 + yb2 + yb3 + yb4
    x0, k0 = U.dev(y0[:dim]), U.dev(y0[dim:])
    pt = [U.dev(params[0])]
    out = prog.trace(x0, k0, U.dev(om), pt, dt=dt, n_steps=steps, checkpoint_every=10, store=True,
                     store_D=True, store_every=50, t0=U.dev(t0))
    torch.cuda.synchronize()
    assert np.abs(out["t"].cpu().numpy() - T[steps]).max() <= 1e-13 * (1.0 + T[steps].max())
    ex, ek = U.ray_errors({"x": out["x"].cpu().numpy(), "k": out["k"].cpu().numpy()},
                          {"x": y[:dim], "k": y[dim:]}, om, dim)
    assert ex[ok].max() < U.TOL and ek[ok].max() < U.TOL, (ex[ok].max(), ek[ok].max())
    tx, tk = U.traj_errors(out["traj"].cpu().numpy()[:, :, ok], np.stack(snaps)[:, :, ok], om[ok], dim)
    assert tx < U.TOL and tk < U.TOL, (tx, tk)
    dref = np.stack(snaps_D)[:, ok]
    assert np.abs(out["traj_D"].cpu().numpy()[:, ok] - dref).max() < 1e-12 * (1.0 + np.abs(dref).max())
    lx = (2.0 * (out["x"] - U.dev(target))).contiguous()
    gx0, gk0, gps = torch.empty_like(x0), torch.empty_like(k0), [torch.empty_like(pt[0])]
    prog.adjoint_desc(out["_desc"], lx, None, gx0, gk0, gps)
    torch.cuda.synchronize()
    rel = lambda a, b: np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)
    assert rel(gx0.cpu().numpy(), lam[:dim])[ok].max() < 1e-9
    assert rel(gk0.cpu().numpy(), lam[dim:])[ok].max() < 1e-9
    if ns and ok.all():  # (a sum over all rays)
        ref = np.zeros(4)
        ref[elems] = gp[:ns]
        got = gps[0].cpu().numpy()
        assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max(), (got, ref)


def _dp_factor(err, facmax):
    """The step factor of the Dormand-Prince controller: k/32 for the
    largest integer k in [0, 161] with err (5k)^5 <= 144^5 (0.9 err^(-1/5)
    rounded down to a multiple of 1/32), clipped to [0.2, facmax]."""
    ks = np.arange(162, dtype=np.float64)
    with np.errstate(invalid="ignore"):  # inf * 0 for k = 0: not within
        ok = err[:, None] * (5.0 * ks[None, :]) ** 5 <= 144.0 ** 5
    k = np.where(ok.any(axis=1), 161 - np.argmax(ok[:, ::-1], axis=1), 0)
    return np.minimum(np.maximum(k / 32.0, 0.2), facmax)


@pytest.mark.parametrize("seed,n_terms,dim,with_t", [(4, 60, 3, False), (11, 40, 2, True)])
def test_random_relation_dopri_matches_host_build(oracle, seed, n_terms, dim, with_t):
    """Dormand-Prince 5(4) on random relations (its stages take the
    constants as literals; the rolled RK4 stages read them from the table):
    every ray's accepted steps, attempts and status equal to a host
    Dormand-Prince with the same controller over the same emitted
    functions built for the host, and endpoints and end times to 1e-11."""
    torch = U.torch_mod()
    rng = np.random.default_rng(seed)
    g = rgb.Graph(dim)
    D, _, _, _ = _random_D(g, rng, n_terms, dim, with_t)
    ny = 2 * dim
    print(f"[case] random relation Dormand-Prince seed={seed} dim={dim} t={with_t}", flush=True)
    prog = g.compile(D)
    params = [np.ascontiguousarray(rng.uniform(0.5, 1.5, 4))]
    n, budget, h0, tol, hmin = 256, 60, 1e-2, 1e-9, 1e-12
    y0 = np.ascontiguousarray(np.concatenate([rng.uniform(-1.0, 1.0, (dim, n)), rng.uniform(0.5, 1.5, (dim, n))]))
    om = np.full(n, 1.5)
    t0 = rng.uniform(0.0, 3.0, n) if with_t else np.zeros(n)
    c, a, b5, b4 = oracle.dopri_tableau()
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, False, tmp)
        pp = (C.c_void_p * 8)(params[0].ctypes.data, *([None] * 7))
        y, t = y0.copy(), t0.copy()
        h, fm = np.full(n, h0), np.full(n, 5.0)
        acc, att, st = np.zeros(n, np.int64), np.zeros(n, np.int64), np.full(n, -1)
        k1 = _host_rhs(lib, y, om, t, pp)
        while (st < 0).any():
            st[(st < 0) & ((acc >= budget) | (att >= 4 * budget))] = rgb.RAY_BUDGET
            r = np.nonzero(st < 0)[0]
            if r.size == 0:
                break
            hs, yr, tr, omr = h[r], y[:, r], t[r], om[r]
            K = [k1[:, r]]
            for i in range(1, 7):
                Yi = yr + hs * sum(a[i, j] * K[j] for j in range(i))
                K.append(_host_rhs(lib, Yi, omr, tr + c[i] * hs, pp))
            y5 = yr + hs * sum(b5[j] * K[j] for j in range(7))
            e = hs * sum((b5[j] - b4[j]) * K[j] for j in range(7))
            sc = tol + tol * np.maximum(np.abs(yr), np.abs(y5))
            err = np.sqrt(((e / sc) ** 2).sum(axis=0) / ny)
            att[r] += 1
            ok = (err <= 1.0) & np.isfinite(y5).all(axis=0) & np.isfinite(K[6]).all(axis=0)
            fac = _dp_factor(np.where(ok, err, np.where(err > 1.0, err, np.inf)), np.where(ok, fm[r], 1.0))
            h[r] = hs * fac
            ra = r[ok]
            y[:, ra], k1[:, ra] = y5[:, ok], K[6][:, ok]
            t[ra] = t[ra] + hs[ok]
            acc[ra] += 1
            fm[r] = np.where(ok, 5.0, 1.0)
            st[r[h[r] < hmin]] = rgb.RAY_STEP_UNDERFLOW
    out = prog.trace(U.dev(y0[:dim]), U.dev(y0[dim:]), U.dev(om), [U.dev(params[0])], integrator=rgb.DOPRI54,
                     h0=h0, rtol=tol, atol=tol, hmin=hmin, max_steps=budget, t0=U.dev(t0))
    torch.cuda.synchronize()
    assert np.array_equal(out["status"].cpu().numpy(), st)
    assert np.array_equal(out["steps"].cpu().numpy(), acc) and np.array_equal(out["attempts"].cpu().numpy(), att)
    assert (att > acc).any()  # some attempts were rejected
    ex, ek = U.ray_errors({"x": out["x"].cpu().numpy(), "k": out["k"].cpu().numpy()},
                          {"x": y[:dim], "k": y[dim:]}, om, dim)
    assert ex.max() < U.TOL and ek.max() < U.TOL, (ex.max(), ek.max())
    assert np.abs(out["t"].cpu().numpy() - t).max() <= 1e-11 * (1.0 + np.abs(t).max())


@pytest.mark.parametrize("seed,n_terms,dim", [(1, 10, 3), (8, 8, 2), (4, 60, 3)])
def test_random_relation_newton_matches_host(seed, n_terms, dim):
    """Launch conditions on random relations: the GPU Newton solve for k_x
    (rg_solve_k, emitted D and dD/dk) against a host Newton iteration over
    the graph's own D and dD/dk_x, from the same initial guesses: the rays
    the host solves to |D| <= 1e-13 the GPU solves too, to the same root
    (1e-12 relative), with |D| <= 1e-13 reported and the maximum over the
    rays reduced on the GPU.  (Rays the host needs more than 20 iterations
    for sit near a double root, where rounding can move the iterates
    apart; they are left out.)"""
    torch = U.torch_mod()
    rng = np.random.default_rng(seed)
    g = rgb.Graph(dim)
    D, x, k, om = _random_D(g, rng, n_terms, dim)
    dD = D.df(k[0])
    print(f"[case] random relation Newton seed={seed} dim={dim}", flush=True)
    prog = g.compile(D)
    params = [np.ascontiguousarray(rng.uniform(0.5, 1.5, 4))]
    n, tol = 256, 1e-13
    X = rng.uniform(-1.0, 1.0, (dim, n))
    K = np.concatenate([np.ones((1, n)), rng.uniform(0.1, 0.4, (dim - 1, n))])
    root, solved = K[0].copy(), np.zeros(n, bool)
    for r in range(n):
        kv, xv = list(K[:, r]), list(X[:, r])
        for it in range(51):
            Dv = g.eval(D, xv, kv, 1.5, params=params)
            if abs(Dv) <= tol:
                solved[r] = it <= 20  # well-conditioned: quadratic convergence reached the root
                break
            if it == 50:
                break
            kv[0] -= Dv / g.eval(dD, xv, kv, 1.5, params=params)
        root[r] = kv[0]
    assert solved.mean() > 0.8
    kd = U.dev(K)
    it, Dg, mx = prog.solve_k(U.dev(X), kd, U.dev(np.full(n, 1.5)), [U.dev(params[0])], component=0, tol=tol)
    torch.cuda.synchronize()
    it, Dg, kg = it.cpu().numpy(), Dg.cpu().numpy(), kd.cpu().numpy()
    assert (it[solved] >= 0).all() and (np.abs(Dg[solved]) <= tol).all()
    assert np.abs(kg[0, solved] - root[solved]).max() < 1e-12 * np.abs(root[solved]).max()
    assert np.array_equal(kg[1:], K[1:])  # the other components untouched
    fin = np.isfinite(Dg)
    assert float(mx.cpu()[0]) == (np.abs(Dg).max() if fin.all() else np.inf)


def _host_rk4(lib, y0, om, t0, pp, steps, dt):
    """Classic RK4 over the host build: end state and every stage state."""
    Y = np.zeros((steps, 4) + y0.shape)
    y, t = y0.copy(), t0.copy()
    T = np.zeros((steps + 1,) + t0.shape)
    T[0] = t0
    for s in range(steps):
        th = T[s] + 0.5 * dt
        Y[s, 0] = y
        k1 = _host_rhs(lib, y, om, T[s], pp)
        Y[s, 1] = y + 0.5 * dt * k1
        k2 = _host_rhs(lib, Y[s, 1], om, th, pp)
        Y[s, 2] = y + 0.5 * dt * k2
        k3 = _host_rhs(lib, Y[s, 2], om, th, pp)
        Y[s, 3] = y + dt * k3
        k4 = _host_rhs(lib, Y[s, 3], om, T[s] + dt, pp)
        y = y + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        T[s + 1] = T[s] + dt
    return y, Y, T


def _host_rk4_adjoint(lib, Y, T, om, pp, lam, dt):
    """The discrete adjoint of _host_rk4's map, last step first."""
    gp = np.zeros(64)
    for s in range(Y.shape[0] - 1, -1, -1):
        t, th = T[s], T[s] + 0.5 * dt
        kb4 = dt / 6.0 * lam
        yb4 = _host_vjp(lib, Y[s, 3], om, t + dt, pp, kb4, gp)
        kb3 = dt / 3.0 * lam + dt * yb4
        yb3 = _host_vjp(lib, Y[s, 2], om, th, pp, kb3, gp)
        kb2 = dt / 3.0 * lam + 0.5 * dt * yb3
        yb2 = _host_vjp(lib, Y[s, 1], om, th, pp, kb2, gp)
        kb1 = dt / 6.0 * lam + 0.5 * dt * yb2
        yb1 = _host_vjp(lib, Y[s, 0], om, t, pp, kb1, gp)
        lam = lam + yb1 + yb2 + yb3 + yb4
    return lam, gp


@pytest.mark.parametrize("mode,x0", [("O", -5.0), ("X", 12.0)])
def test_coldplasma_adjoint_matches_host_build(oracle, mode, x0):
    """The adjoint of the cold-plasma medium (electrons and hydrogen ions,
    oblique n_z = 0.2, k_x from the oracle's Newton solve; the oracle's
    cold-plasma model is forward only): GPU endpoints and dL/dx0, dL/dk0
    per ray against a host RK4 and discrete adjoint over the host build of
    the emitted functions, whose VJP test_emit_host.py checks against the
    graph's own second derivatives."""
    from paper_2508_15967_amd import media
    torch = U.torch_mod()
    w = W.coldplasma(mode, n_rays=256, x0=x0, direction=1.0, dt=1e-2, n_steps=300, mu=W.MU_H, nz=W.CP_NZ)
    print(f"[case] coldplasma adjoint {mode}", flush=True)
    w.k0, _, _ = oracle.newton_k(w.medium, w.x0, w.k0, w.omega, component=w.solve_k, tol=1e-15, max_iter=60)
    g, D, params = media.build(w.medium)
    prog = g.compile(D, want_adjoint=True)
    y0 = np.ascontiguousarray(np.concatenate([w.x0, w.k0]))
    om, t0 = np.ascontiguousarray(w.omega), np.zeros(w.n)
    target = w.x0 + np.random.default_rng(3).uniform(-1.0, 1.0, w.x0.shape)
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, True, tmp)
        pp = (C.c_void_p * 8)(*([p.ctypes.data for p in params] + [None] * (8 - len(params))))
        y, Y, T = _host_rk4(lib, y0, om, t0, pp, w.n_steps, w.dt)
        yp, _, _ = _host_rk4(lib, np.nextafter(y0, np.inf), om, t0, pp, w.n_steps, w.dt)
        ex, ek = U.ray_errors({"x": yp[:3], "k": yp[3:]}, {"x": y[:3], "k": y[3:]}, om, 3)
        ok = np.maximum(ex, ek) <= 1e-12
        assert (~ok).mean() <= U.MAX_ILL
        lam0, _ = _host_rk4_adjoint(lib, Y, T, om, pp, np.concatenate([2.0 * (y[:3] - target), 0.5 * y[3:]]),
                                    w.dt)
    pt = [U.dev(p) for p in params]
    x0d, k0d = U.dev(w.x0), U.dev(w.k0)
    out = prog.trace(x0d, k0d, U.dev(om), pt, dt=w.dt, n_steps=w.n_steps, checkpoint_every=100)
    torch.cuda.synchronize()
    ex, ek = U.ray_errors({"x": out["x"].cpu().numpy(), "k": out["k"].cpu().numpy()},
                          {"x": y[:3], "k": y[3:]}, om, 3)
    assert ex[ok].max() < U.TOL and ek[ok].max() < U.TOL, (ex[ok].max(), ek[ok].max())
    lx = (2.0 * (out["x"] - U.dev(target))).contiguous()
    lk = (0.5 * out["k"]).contiguous()
    gx0, gk0 = torch.empty_like(x0d), torch.empty_like(k0d)
    prog.adjoint_desc(out["_desc"], lx, lk, gx0, gk0, [torch.empty_like(p) for p in pt])
    torch.cuda.synchronize()
    rel = lambda a, b: np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)
    assert rel(gx0.cpu().numpy(), lam0[:3])[ok].max() < 1e-9
    assert rel(gk0.cpu().numpy(), lam0[3:])[ok].max() < 1e-9
