"""The emission pipeline on random dispersion relations (no GPU, no
oracle): the right-hand side f = (-D_k/D_w, D_x/D_w), D and the
vector-Jacobian product v^T df/dy of the emitted device functions, compiled
as host C++, against the graph front end's own evaluation of the same
symbolic derivatives taken on the unfactored graph.  The random relations
are sums of products over a pool that shares sub-sums, scaled copies of
sums, Gaussians, ray invariants (omega, parameter elements) and, in some,
the time t or square roots, logarithms, integer powers, sines and
quotients of positive expressions, so that the
common-factor, scaled-sum, product and division passes all rewrite them;
a pass that drops a term, flips a sign or mixes up an operand changes the
values far beyond rounding.  The larger relations carry enough constants
for the rolled form with its constant table."""
import ctypes as C
import re
import tempfile

import numpy as np
import pytest

from paper_2508_15967_amd import raygraph as rgb
from tests.test_emit_host import _host_lib


def _random_D(g, rng, n_terms, dim=3, with_t=False, rich=False):
    x = [g.x(i) for i in range(dim)]
    k = [g.k(i) for i in range(dim)]
    om = g.omega
    s = g.param("s", 4)
    base = x + k
    sums = []
    for _ in range(4):
        i, j = rng.choice(2 * dim, 2, replace=False)
        c1, c2 = rng.choice([-2.0, -1.0, -0.5, 0.5, 1.0, 1.5, 2.0], 2)
        lin = c1 * base[i] + c2 * base[j]
        sums.append(lin)
        sums.append((2.0 * c1) * base[i] + (2.0 * c2) * base[j])  # a scaled copy of the same sum
        sums.append(lin + float(rng.uniform(-1.0, 1.0)))
    gauss = []
    for _ in range(3):
        i = int(rng.integers(0, dim))
        c, w = float(rng.uniform(-1.0, 1.0)), float(rng.uniform(1.0, 2.0))
        d = x[i] - c
        gauss.append((d * d * (-1.0 / (w * w))).exp())
    inv = [g.elem(s, j) for j in range(4)] + [om]
    pool = base + sums + gauss
    if with_t:  # time-dependent factors
        pool += [(0.7 * g.t + 0.2).sin(), 0.5 * g.t + 1.0, (x[0] - 0.3 * g.t).cos()]
    if rich:  # square roots, logarithms, integer powers and quotients of positive expressions
        pos = [xi * xi + 1.5 for xi in x] + [(k[0] - 0.2 * x[-1]) ** 2 + 0.5]
        for _ in range(4):
            p1, p2 = pos[int(rng.integers(0, len(pos)))], pos[int(rng.integers(0, len(pos)))]
            pool += [p1.sqrt(), p1.log(), p1 ** int(rng.choice([-2, -1, 2, 3])), base[int(rng.integers(0, 2 * dim))] / p2,
                     (base[int(rng.integers(0, 2 * dim))] * 0.7).sin()]
    D = -(om * om)
    for ki in k:
        D = D + ki * ki
    for _ in range(n_terms):
        nf = int(rng.integers(2, 4))
        fs = [pool[int(rng.integers(0, len(pool)))] for _ in range(nf)]
        if rng.random() < 0.5:
            fs.append(inv[int(rng.integers(0, 4))])  # a parameter element
        if rng.random() < 0.1:
            fs.append(om)
        t = fs[0]
        for f in fs[1:]:
            t = t * f
        D = D + float(rng.uniform(0.02, 0.1)) * float(rng.choice([-1.0, 1.0])) * t
    return D, x, k, om


@pytest.mark.parametrize("seed,n_terms,dim,extra", [
    (0, 6, 3, ""), (1, 10, 3, ""), (2, 14, 3, ""), (3, 40, 3, ""), (4, 60, 3, ""),
    (5, 8, 3, ""), (6, 12, 3, ""), (7, 20, 3, ""), (8, 8, 2, ""), (9, 50, 2, ""),
    (10, 12, 3, "t"), (11, 40, 2, "t"), (12, 10, 3, "ops"), (13, 30, 3, "ops"), (14, 20, 2, "ops")])
def test_emitted_functions_match_graph(seed, n_terms, dim, extra):
    rng = np.random.default_rng(seed)
    g = rgb.Graph(dim)
    with_t = extra == "t"
    D, x, k, om = _random_D(g, rng, n_terms, dim, with_t, rich=extra == "ops")
    ny = 2 * dim
    Dw = D.df(om)
    f_nodes = [-(D.df(ki)) / Dw for ki in k] + [D.df(xi) / Dw for xi in x]
    ys = x + k
    J_nodes = [[fi.df(yj) for yj in ys] for fi in f_nodes]
    prog = g.compile(D, want_adjoint=True, compile_only=True)
    # parameter-gradient slots: slot e holds element rg_grad_elem[e] of the
    # (only) parameter array
    src = prog.source()
    ns = int(prog.info()["n_grad_slots"])
    slots = [int(t) for t in re.search(r"rg_grad_elem\[\d+\] = \{([^}]*)\}", src).group(1).split(",")][:ns]
    assert re.search(r"rg_grad_param\[\d+\] = \{([^}]*)\}", src).group(1).replace(" ", "").strip("0,") == ""
    assert ns == len(set(slots))
    P_nodes = [[fi.df(g.elem(0, j)) for j in slots] for fi in f_nodes]
    params = [np.ascontiguousarray(rng.uniform(0.5, 1.5, 4))]
    n = 64
    y = np.ascontiguousarray(np.concatenate([rng.uniform(-1.0, 1.0, (dim, n)), rng.uniform(0.5, 1.5, (dim, n))]))
    omv = np.full(n, 1.5)
    tv = np.ascontiguousarray(rng.uniform(0.0, 3.0, n) if with_t else np.zeros(n))
    v = np.ascontiguousarray(rng.standard_normal((ny, n)))
    f_ref = np.zeros((ny, n))
    D_ref = np.zeros(n)
    jv_ref = np.zeros((ny, n))
    gp_ref = np.zeros(len(slots))
    for r in range(n):
        xv, kv = list(y[:dim, r]), list(y[dim:, r])
        ev = lambda nd: g.eval(nd, xv, kv, 1.5, t=float(tv[r]), params=params)
        D_ref[r] = ev(D)
        f_ref[:, r] = [ev(fi) for fi in f_nodes]
        J = np.array([[ev(J_nodes[i][j]) for j in range(ny)] for i in range(ny)])
        jv_ref[:, r] = v[:, r] @ J
        gp_ref += v[:, r] @ np.array([[ev(P_nodes[i][e]) for e in range(len(slots))] for i in range(ny)])
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, True, tmp)
        pp = (C.c_void_p * 8)(params[0].ctypes.data, *([None] * 7))
        f = np.zeros((ny, n))
        Dv = np.zeros(n)
        lib.host_eval_t(n, ny, C.c_void_p(y.ctypes.data), C.c_void_p(omv.ctypes.data),
                        C.c_void_p(tv.ctypes.data), pp, C.c_void_p(f.ctypes.data), C.c_void_p(Dv.ctypes.data))
        jv = np.zeros((ny, n))
        gp = np.zeros(64)
        lib.host_vjp_t(n, ny, C.c_void_p(y.ctypes.data), C.c_void_p(omv.ctypes.data),
                       C.c_void_p(tv.ctypes.data), pp, C.c_void_p(v.ctypes.data), C.c_void_p(jv.ctypes.data),
                       C.c_void_p(gp.ctypes.data))
    assert np.abs(Dv - D_ref).max() <= 1e-13 * (1.0 + np.abs(D_ref).max())
    assert (np.abs(f - f_ref).max(axis=0) / np.abs(f_ref).max(axis=0)).max() < 1e-12
    assert (np.abs(jv - jv_ref).max(axis=0) / np.abs(jv_ref).max(axis=0)).max() < 1e-11
    if slots:
        assert np.abs(gp[:len(slots)] - gp_ref).max() < 1e-11 * np.abs(gp_ref).max()
