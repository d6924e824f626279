"""The emitted device functions compiled as host C++ (g++, no contraction)
and evaluated on the CPU: right-hand side, D and the vector-Jacobian
products must match the oracle's hand-derived formulas.  This checks the
graph differentiation (first and second order), reduction, CSE, fma fusion
and the spline gather/scatter emission without a GPU."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2508_15967_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRELUDE = os.path.join(ROOT, "paper_2508_15967_amd", "csrc", "kernels")

HOST_HARNESS = r'''
#include <math.h>
#include <string.h>
#define RG_FN static inline
#define RG_KTAB static const
#define RG_KBASE const double *rg_k = rg_ktab;
#include "rg_prelude.h"
static const double *g_tab[8];
static int g_tab_ny[8];
static double *g_grad[8];
#define RG_SPL_TAB(k) (g_tab[k])
struct rg_GA {
    void add(int k, int x, int y, const double *g) {
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) g_grad[k][(x - 1 + a) * g_tab_ny[k] + (y - 1 + b)] += g[4 * a + b];
    }
};
#include "functions.h"
extern "C" void set_table(int k, const double *t, int ny, double *grad) { g_tab[k] = t; g_tab_ny[k] = ny; g_grad[k] = grad; }
extern "C" void host_eval(int n, int ny, const double *y, const double *om, const double *const *pp,
                          double *f, double *D) {
    rg_P P; memset(&P, 0, sizeof P);
    for (int i = 0; i < 8 && pp; i++) P.p[i] = pp[i];
    for (int r = 0; r < n; r++) {
        double yy[6], ff[6];
        for (int c = 0; c < ny; c++) yy[c] = y[c * n + r];
        rg_rhs(yy, om[r], 0.0, P, ff);
        for (int c = 0; c < ny; c++) f[c * n + r] = ff[c];
        D[r] = rg_D(yy, om[r], 0.0, P);
    }
}
// the same functions with the constants as literals (RG_KL)
extern "C" void host_eval_lit(int n, int ny, const double *y, const double *om, const double *const *pp,
                              double *f, double *D) {
    rg_P P; memset(&P, 0, sizeof P);
    for (int i = 0; i < 8 && pp; i++) P.p[i] = pp[i];
    for (int r = 0; r < n; r++) {
        double yy[6], ff[6];
        for (int c = 0; c < ny; c++) yy[c] = y[c * n + r];
        rg_rhs<true>(yy, om[r], 0.0, P, ff);
        for (int c = 0; c < ny; c++) f[c * n + r] = ff[c];
        D[r] = rg_D<true>(yy, om[r], 0.0, P);
    }
}
// with a time per point (time-dependent relations)
extern "C" void host_eval_t(int n, int ny, const double *y, const double *om, const double *t,
                            const double *const *pp, double *f, double *D) {
    rg_P P; memset(&P, 0, sizeof P);
    for (int i = 0; i < 8 && pp; i++) P.p[i] = pp[i];
    for (int r = 0; r < n; r++) {
        double yy[6], ff[6];
        for (int c = 0; c < ny; c++) yy[c] = y[c * n + r];
        rg_rhs(yy, om[r], t[r], P, ff);
        for (int c = 0; c < ny; c++) f[c * n + r] = ff[c];
        D[r] = rg_D(yy, om[r], t[r], P);
    }
}
#ifdef HAS_F32
extern "C" void host_eval32(int n, int ny, const float *y, const float *om, const double *const *pp,
                            float *f) {
    rg_P P; memset(&P, 0, sizeof P);
    for (int i = 0; i < 8 && pp; i++) P.p[i] = pp[i];
    for (int r = 0; r < n; r++) {
        float yy[6], ff[6];
        for (int c = 0; c < ny; c++) yy[c] = y[c * n + r];
        rg_rhs(yy, om[r], 0.0f, P, ff);
        for (int c = 0; c < ny; c++) f[c * n + r] = ff[c];
    }
}
#endif
#ifdef HAS_VJP
extern "C" void host_vjp(int n, int ny, const double *y, const double *om, const double *const *pp,
                         const double *v, double *jv, double *gp) {
    rg_P P; memset(&P, 0, sizeof P);
    for (int i = 0; i < 8 && pp; i++) P.p[i] = pp[i];
    rg_GA G;
    for (int r = 0; r < n; r++) {
        double yy[6], vv[6], jj[6];
        for (int c = 0; c < ny; c++) { yy[c] = y[c * n + r]; vv[c] = v[c * n + r]; }
        rg_vjp(yy, om[r], 0.0, P, vv, jj, gp, G);
        for (int c = 0; c < ny; c++) jv[c * n + r] = jj[c];
    }
}
extern "C" void host_vjp_t(int n, int ny, const double *y, const double *om, const double *t,
                           const double *const *pp, const double *v, double *jv, double *gp) {
    rg_P P; memset(&P, 0, sizeof P);
    for (int i = 0; i < 8 && pp; i++) P.p[i] = pp[i];
    rg_GA G;
    for (int r = 0; r < n; r++) {
        double yy[6], vv[6], jj[6];
        for (int c = 0; c < ny; c++) { yy[c] = y[c * n + r]; vv[c] = v[c * n + r]; }
        rg_vjp(yy, om[r], t[r], P, vv, jj, gp, G);
        for (int c = 0; c < ny; c++) jv[c * n + r] = jj[c];
    }
}
#endif
'''


def _host_lib(prog, has_vjp, tmp, has_f32=False):
    with open(os.path.join(tmp, "functions.h"), "w") as f:
        f.write(prog.functions())
    src = os.path.join(tmp, "h.cpp")
    with open(src, "w") as f:
        f.write(HOST_HARNESS)
    so = os.path.join(tmp, "h.so")
    cmd = ["g++", "-O1", "-ffp-contract=off", "-fPIC", "-shared", "-I" + PRELUDE, "-I" + tmp, src,
           "-o", so] + (["-DHAS_VJP"] if has_vjp else []) + (["-DHAS_F32"] if has_f32 else [])
    subprocess.run(cmd, check=True, capture_output=True)
    return C.CDLL(so)


def _ptrs(arrs):
    return (C.c_void_p * 8)(*([a.ctypes.data for a in arrs] + [None] * (8 - len(arrs))))


def _points(w, n, rng):
    idx = rng.integers(0, w.n, n)
    y = np.concatenate([w.x0[:, idx] + rng.uniform(-1, 1, (w.dim, n)),
                        w.k0[:, idx] * (1 + 0.05 * rng.uniform(-1, 1, (1, n)))])
    return np.ascontiguousarray(y), np.ascontiguousarray(w.omega[idx])


# cold-plasma media of the tests: electrons only with k perpendicular to B
# (cO, cX), and with a hydrogen ion species and an oblique n_z (cO2, cX2),
# where the M13, M23 and n_z terms of the determinant and the ion terms of
# the species sums (eqs. 6, 8-10) are nonzero
COLD = {"cO": lambda: W.coldplasma("O"), "cX": lambda: W.coldplasma("X", x0=12.0),
        "cO2": lambda: W.coldplasma("O", mu=W.MU_H, nz=W.CP_NZ),
        "cX2": lambda: W.coldplasma("X", x0=12.0, mu=W.MU_H, nz=0.3)}


@pytest.mark.parametrize("cfg", ["1", "2", "3", "4", "5", "cO", "cX", "cO2", "cX2"])
def test_emitted_functions_match_oracle(oracle, cfg):
    from paper_2508_15967_amd import media
    w = COLD.get(cfg, lambda: W.make(cfg, 2048))()
    g, D, params = media.build(w.medium)
    adj = cfg in ("4", "5")
    prog = g.compile(D, want_adjoint=adj, compile_only=True)
    rng = np.random.default_rng(3)
    n = 400
    y, om = _points(w, n, rng)
    ny = 2 * w.dim
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, adj, tmp)
        pp = _ptrs(params)
        grad = np.zeros(params[0].size if params else 1)
        if cfg == "4":
            lib.set_table(0, C.c_void_p(params[0].ctypes.data), 64, C.c_void_p(grad.ctypes.data))
        f = np.zeros((ny, n))
        Dv = np.zeros(n)
        lib.host_eval(n, ny, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), pp,
                      C.c_void_p(f.ctypes.data), C.c_void_p(Dv.ctypes.data))
        fo, Do, J = oracle.eval_points(w.medium, y, om, jac=True)
        scale = np.abs(fo).max(axis=0)
        # the oracle's cold-plasma partials are complex-step derivatives of
        # its own D: agreement to rounding of the two derivative routes
        assert (np.abs(f - fo).max(axis=0) / scale).max() < (1e-12 if cfg.startswith("c") else 1e-13)
        assert np.abs(Dv - Do).max() < 1e-13 * (1 + np.abs(Do).max())
        if adj:
            v = np.ascontiguousarray(rng.standard_normal((ny, n)))
            jv = np.zeros((ny, n))
            gp = np.zeros(64)
            lib.host_vjp(n, ny, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), pp,
                         C.c_void_p(v.ctypes.data), C.c_void_p(jv.ctypes.data), C.c_void_p(gp.ctypes.data))
            jvo = np.einsum("nij,in->jn", J, v)
            assert np.abs(jv - jvo).max() / np.abs(jvo).max() < 1e-12
            go = oracle.param_vjp_points(w.medium, y, om, v)
            got = grad if cfg == "4" else gp[:16]
            assert np.abs(got - go).max() / np.abs(go).max() < 1e-12


@pytest.mark.parametrize("cfg", ["2", "3", "5"])
def test_constant_table_equals_literals(cfg):
    """Programs with many constants (the bumps and the anisotropic medium)
    read their FP64 constants from one table; the same functions with the
    RG_KL flag take them as literals.  Both forms hold the same doubles, so
    the results are bitwise equal; programs with few constants keep
    literals only."""
    from paper_2508_15967_amd import media
    w = W.make(cfg, 2048)
    g, D, params = media.build(w.medium)
    prog = g.compile(D, compile_only=True)
    src = prog.functions()
    rolled = cfg in ("3", "5")
    assert ("rg_ktab[" in src) == rolled and ("RG_KV(" in src) == rolled
    rng = np.random.default_rng(5)
    n = 300
    y, om = _points(w, n, rng)
    ny = 2 * w.dim
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, False, tmp)
        pp = _ptrs(params)
        out = []
        for fn in (lib.host_eval, lib.host_eval_lit):
            f, Dv = np.zeros((ny, n)), np.zeros(n)
            fn(n, ny, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), pp,
               C.c_void_p(f.ctypes.data), C.c_void_p(Dv.ctypes.data))
            out.append((f, Dv))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert np.isfinite(out[0][0]).all()


@pytest.mark.parametrize("cfg", ["1", "2", "3", "5", "cO", "cX", "cO2"])
def test_emitted_fp32_rhs(oracle, cfg):
    """The single precision right-hand side (same graph, float arithmetic)
    against the oracle's FP64 formulas at the same (float-representable)
    points.  Each output is a short expression of the inputs evaluated in
    float: its error is a modest multiple of the unit roundoff 2^-24 (about
    6e-8) relative to the output scale, amplified by the expression's
    conditioning; 5e-6 leaves margin for the cancellation in the cold-plasma
    determinant near its cutoffs.  The cold-plasma determinant itself is a
    sum of products several orders of magnitude larger than its value near
    the cutoffs, and its partials lose correspondingly more: 1e-3 there."""
    from paper_2508_15967_amd import media
    w = COLD.get(cfg, lambda: W.make(cfg, 2048))()
    g, D, params = media.build(w.medium)
    prog = g.compile(D, compile_only=True, fp32=True)
    rng = np.random.default_rng(5)
    n = 400
    y, om = _points(w, n, rng)
    if cfg in ("2", "3"):
        y[2] = rng.uniform(2.0, 18.0, n)  # inside the stratified layer (the launch plane has N = 1)
    y32, om32 = y.astype(np.float32), om.astype(np.float32)
    ny = 2 * w.dim
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, False, tmp, has_f32=True)
        f = np.zeros((ny, n), dtype=np.float32)
        lib.host_eval32(n, ny, C.c_void_p(y32.ctypes.data), C.c_void_p(om32.ctypes.data), _ptrs(params),
                        C.c_void_p(f.ctypes.data))
    fo, _, _ = oracle.eval_points(w.medium, np.ascontiguousarray(y32, dtype=np.float64),
                                  np.ascontiguousarray(om32, dtype=np.float64), jac=False)
    scale = np.abs(fo).max(axis=0)
    err = (np.abs(f.astype(np.float64) - fo).max(axis=0) / scale).max()
    print(cfg, "max relative error", err)
    assert err < (1e-3 if cfg.startswith("c") else 5e-6)
    # and not accidentally double precision
    assert err > 1e-12


def _exp_points(rng, n):
    x = np.concatenate([rng.uniform(-745.0, 709.7, n), rng.uniform(-30.0, 30.0, n),
                        rng.uniform(-1.0, 1.0, n), (rng.random(n) - 0.5) * 1e-3])
    special = np.array([0.0, -0.0, 709.78, 709.79, -745.0, -745.2, -1e5, -1e300, 1e300, 1100.0, 1101.0,
                        -np.inf, np.inf, np.nan])
    return x, special


def _exp_reference(x):
    """e^x correctly rounded to double (60-digit decimal arithmetic)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    out = np.empty_like(x)
    for i, v in enumerate(x):
        out[i] = float(Decimal(float(v)).exp())
    return out


def _exp_ulps(got, ref):
    with np.errstate(invalid="ignore", over="ignore"):
        sp = np.spacing(np.abs(ref))
        sp = np.where(ref == 0.0, 2.0 ** -1074, sp)
        return np.abs(got - ref) / sp


def test_exp_table_matches_generator():
    """The constants in rg_prelude.h are the generator's output."""
    import importlib.util
    path = os.path.join(PRELUDE, "gen_exp_table.py")
    spec = importlib.util.spec_from_file_location("gen_exp_table", path)
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    text = open(os.path.join(PRELUDE, "rg_prelude.h")).read()
    assert gen.block() in text


def _exp_variant_programs(compile_only=True):
    """D = omega e^(x0 e^x1), whose argument can be NaN at finite inputs
    (0 * inf), takes the general rg_exp; D = omega e^x0, whose argument is
    NaN only at a NaN input, the NaN-free variant rg_exp_nn.  At x1 = 0 and
    omega = 1 both are e^x0 (e^0 = 1 exactly)."""
    from paper_2508_15967_amd import raygraph as rgb
    g = rgb.Graph(2)
    gen = g.compile(g.omega * (g.x(0) * g.x(1).exp()).exp(), compile_only=compile_only)
    g2 = rgb.Graph(2)
    nn = g2.compile(g2.omega * g2.x(0).exp(), compile_only=compile_only)
    assert "rg_exp(" in gen.functions() and "rg_exp_n" not in gen.functions().split("rg_exp(", 1)[1].split(";")[0]
    assert "rg_exp_nn(" in nn.functions() and "rg_exp(" not in nn.functions()
    return gen, nn


def _check_exp_values(Dv, x, special, nan_gives_zero):
    ulps = _exp_ulps(Dv[:x.size], _exp_reference(x))
    assert ulps.max() <= 1.5, ulps.max()
    got_sp = Dv[x.size:]
    with np.errstate(over="ignore"):
        ref_sp = np.exp(special)
    if nan_gives_zero:
        ref_sp = np.where(np.isnan(special), 0.0, ref_sp)
    same = (got_sp == ref_sp) | (np.isnan(got_sp) & np.isnan(ref_sp))
    # the finite specials are compared within the same bound
    fin = np.isfinite(ref_sp) & (ref_sp > 0)
    same |= fin & (_exp_ulps(got_sp, ref_sp) <= 1.5)
    assert same.all(), list(zip(special[~same], got_sp[~same], ref_sp[~same]))


def test_exp_host_accuracy():
    """rg_exp (table-driven, host build of the same code) within 1.5 ulp of
    the correctly rounded e^x, and exact special cases: overflow to +inf,
    underflow to 0, e^(+-inf), NaN.  The NaN-free variant gives the same
    doubles everywhere but at a NaN argument, where it gives 0."""
    gen, nn = _exp_variant_programs()
    rng = np.random.default_rng(17)
    x, special = _exp_points(rng, 5000)
    xs = np.concatenate([x, special])
    n = xs.size
    y = np.zeros((4, n))
    y[0] = xs
    y[2] = 1.0
    om = np.ones(n)
    out = []
    for prog in (gen, nn):
        with tempfile.TemporaryDirectory() as tmp:
            lib = _host_lib(prog, False, tmp)
            f = np.zeros((4, n))
            Dv = np.zeros(n)
            lib.host_eval(n, 4, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), _ptrs([]),
                          C.c_void_p(f.ctypes.data), C.c_void_p(Dv.ctypes.data))
        out.append(Dv)
    _check_exp_values(out[0], x, special, nan_gives_zero=False)
    _check_exp_values(out[1], x, special, nan_gives_zero=True)
    num = ~np.isnan(xs)
    assert np.array_equal(out[0][num], out[1][num])


def test_ray_invariant_flops_counted_apart():
    """Work on omega alone is done once per ray: for D = k.k - W(omega) (1 + x/2)
    the right-hand side's per-evaluation flops do not depend on how the
    frequency factor W is written (omega, omega^2, omega^3, omega^2 + 3 omega,
    e^(omega/2)); what W adds is counted apart as ray-invariant."""
    from paper_2508_15967_amd import raygraph as rgb
    counts = []
    for wf in (lambda w: w, lambda w: w * w, lambda w: w * w * w, lambda w: w * w + 3.0 * w,
               lambda w: (0.5 * w).exp()):
        g = rgb.Graph(2)
        D = g.k(0) * g.k(0) + g.k(1) * g.k(1) - wf(g.omega) * (1.0 + 0.5 * g.x(0))
        info = g.compile(D, compile_only=True).info()
        counts.append((info["rhs_flops_alg"], info["rhs_flops_ray_invariant"]))
    assert len({c[0] for c in counts}) == 1, counts
    assert all(c[1] > counts[0][1] for c in counts[1:]), counts


def test_exp_of_nonpositive_argument():
    """The variant of each exponential: an argument that cannot be NaN at
    finite inputs and that the graph proves non-positive (-x0^2,
    -(x0^2 + x1^2)/3) takes rg_exp_np, without the overflow clamp; one that
    cannot be NaN but has no proven sign (x0, x0^2, the Chapman form
    1 + w - e^w) rg_exp_nn; one that can be NaN at finite inputs (x0 e^x1
    and -omega x0^2: 0 * inf, sqrt(x0), 1/x0 - 1/x1: inf - inf) the general
    rg_exp.  rg_exp_np is within 1.5 ulp of the
    correctly rounded e^(-x0^2), exact at 0, underflow and +-inf, and 0 at
    a NaN argument."""
    from paper_2508_15967_amd import raygraph as rgb

    def src(expr_of):
        g = rgb.Graph(2)
        x, y = g.x(0), g.x(1)
        return g.compile(g.omega * expr_of(g, x, y), compile_only=True).functions()

    def variants(s):
        return {v for v in ("rg_exp(", "rg_exp_nn(", "rg_exp_np(") if v in s}

    for f in (lambda g, x, y: (-(x * x)).exp(), lambda g, x, y: (-(x * x + y * y) / 3.0).exp()):
        assert variants(src(f)) == {"rg_exp_np("}
    for f in (lambda g, x, y: x.exp(), lambda g, x, y: (x * x).exp(),
              lambda g, x, y: (1.0 + (-0.5 * x) - (-0.5 * x).exp()).exp()):
        assert variants(src(f)) == {"rg_exp_nn("}, src(f)
    for f in (lambda g, x, y: (x * y.exp()).exp(), lambda g, x, y: x.sqrt().exp(),
              lambda g, x, y: (1.0 / x - 1.0 / y).exp(),
              lambda g, x, y: (-(g.omega * x * x)).exp()):
        assert "rg_exp(" in src(f), src(f)

    g = rgb.Graph(2)
    D = g.omega * (-(g.x(0) * g.x(0))).exp()
    prog = g.compile(D, compile_only=True)
    rng = np.random.default_rng(23)
    x = np.concatenate([rng.uniform(0.0, 28.0, 4000), rng.uniform(0.0, 1.0, 2000),
                        rng.uniform(-5.0, 5.0, 2000)])
    special = np.array([0.0, -0.0, 27.3, 33.4, 40.0, 1e200, np.inf, -np.inf])
    xs = np.concatenate([x, special])
    n = xs.size
    y = np.zeros((4, n))
    y[0] = xs
    y[2] = 1.0
    om = np.ones(n)
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, False, tmp)
        f = np.zeros((4, n))
        Dv = np.zeros(n)
        lib.host_eval(n, 4, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), _ptrs([]),
                      C.c_void_p(f.ctypes.data), C.c_void_p(Dv.ctypes.data))
    with np.errstate(over="ignore", invalid="ignore"):
        arg = -(xs * xs)   # the emitted argument: one rounded product, negated
    ref = _exp_reference(arg[:x.size])
    assert _exp_ulps(Dv[:x.size], ref).max() <= 1.5
    got_sp = Dv[x.size:]
    with np.errstate(over="ignore", invalid="ignore"):
        ref_sp = np.exp(arg[x.size:])
    same = (got_sp == ref_sp) | (np.isnan(got_sp) & np.isnan(ref_sp))
    fin = np.isfinite(ref_sp) & (ref_sp > 0)
    same |= fin & (_exp_ulps(got_sp, ref_sp) <= 1.5)
    assert same.all(), list(zip(special[~same], got_sp[~same], ref_sp[~same]))
    # a NaN argument gives 0 in this variant (its lower clamp is a maximum):
    # the stage state it came from is NaN, and the step through it is
    # rejected as non-finite whatever the exponential returns
    y1 = np.zeros((4, 1))
    y1[0], y1[2] = np.nan, 1.0
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, False, tmp)
        f1, D1 = np.zeros((4, 1)), np.zeros(1)
        lib.host_eval(1, 4, C.c_void_p(y1.ctypes.data), C.c_void_p(np.ones(1).ctypes.data), _ptrs([]),
                      C.c_void_p(f1.ctypes.data), C.c_void_p(D1.ctypes.data))
    assert D1[0] == 0.0


def test_exp_sign_proof_respects_signed_zero_divisors():
    """A quotient's sign is claimed only where its divisor cannot be a zero
    of the other sign: -1/sqrt(x0) at x0 = -0 is 1/(-0) negated, +inf, so
    its exponential keeps the overflow clamp and gives +inf (the variant
    without the clamp would give NaN there).  A proven sign alone does not
    select a variant that maps NaN to 0: -x0^2/e^x1 (inf/inf),
    -x0^2/x1^2 (0/0) and -x0^2 x1^-2 (0 * inf) can be NaN at finite inputs
    and take the general exponential, as do the quotients by square
    roots."""
    from paper_2508_15967_amd import raygraph as rgb

    def build(expr_of):
        g = rgb.Graph(2)
        return g.compile(g.omega * expr_of(g.x(0), g.x(1)), compile_only=True)

    for f in (lambda x, y: (-(x * x) / y.exp()).exp(),
              lambda x, y: (-(x * x) / (y * y)).exp(),
              lambda x, y: (-(x * x) * (y ** -2)).exp(),
              lambda x, y: (-(1.0 / x.sqrt())).exp(),
              lambda x, y: (-(x * x) / y.sqrt()).exp(),
              lambda x, y: (-(y.sqrt() ** -1)).exp()):
        s = build(f).functions()
        # (e^x1 itself, of a NaN-free argument, takes rg_exp_nn)
        assert "rg_exp(" in s and "rg_exp_np(" not in s

    prog = build(lambda x, y: (-(1.0 / x.sqrt())).exp())
    n = 3
    y = np.zeros((4, n))
    y[0] = [-0.0, 0.0, 4.0]
    y[2] = 1.0
    om = np.ones(n)
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, False, tmp)
        f = np.zeros((4, n))
        Dv = np.zeros(n)
        lib.host_eval(n, 4, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), _ptrs([]),
                      C.c_void_p(f.ctypes.data), C.c_void_p(Dv.ctypes.data))
    assert Dv[0] == np.inf and Dv[1] == 0.0, Dv
    assert abs(Dv[2] - np.exp(-0.5)) <= 2e-16 * np.exp(-0.5)


def test_emitted_operation_counts():
    """Guard on the emitter's output size (host compile only, no GPU): the
    per-evaluation flops of the compiled graph for the anisotropic medium
    (right-hand side and VJP; the VJP relies on the common-factor and
    scaled-sum passes sharing (x - c_b).v and M_b k) and for the cold-plasma
    right-hand side (common factors of its determinant), with the flops of
    one adjoint step that the benchmark's roofline counts."""
    from paper_2508_15967_amd import media
    w = W.make("5", 16)
    g, D, _ = media.build(w.medium)
    info = g.compile(D, want_adjoint=True, compile_only=True).info()
    assert info["rhs_flops_alg"] <= 742, info
    assert info["vjp_flops_alg"] <= 1467, info
    assert info["adj_step_flops_alg"] <= 8987, info
    cp = COLD["cO2"]()
    g, D, _ = media.build(cp.medium)
    info = g.compile(D, compile_only=True).info()
    assert info["rhs_flops_alg"] <= 114, info


def test_non_square_spline_matches_oracle(oracle):
    """A B-spline medium whose grid and domain are not square (9 x 14
    coefficients over [-3, 4] x [-5, 2]): the emitted right-hand side, D,
    VJP and coefficient gradient against the oracle, at points inside the
    domain and beyond its edges (where the edge cells' cubics extend).  A
    mix-up of the two axes' sizes or spacings, invisible on the square
    workload grid, fails it."""
    from paper_2508_15967_amd import media
    rng = np.random.default_rng(11)
    nx, ny = 9, 14
    coef = 1.0 + 0.05 * rng.standard_normal((nx, ny))
    med = W.Medium(W.SPLINE2D, 2, coef=coef, lo=np.array([-3.0, -5.0]), hi=np.array([4.0, 2.0]))
    g, D, params = media.build(med)
    prog = g.compile(D, want_adjoint=True, compile_only=True)
    n = 500
    y = np.ascontiguousarray(np.concatenate([
        np.stack([rng.uniform(-3.5, 4.5, n), rng.uniform(-5.5, 2.5, n)]),
        np.stack([rng.uniform(0.5, 1.5, n), rng.uniform(-0.5, 0.5, n)])]))
    om = np.ascontiguousarray(rng.uniform(0.9, 1.1, n))
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, True, tmp)
        pp = _ptrs(params)
        grad = np.zeros(nx * ny)
        lib.set_table(0, C.c_void_p(params[0].ctypes.data), ny, C.c_void_p(grad.ctypes.data))
        f, Dv = np.zeros((4, n)), np.zeros(n)
        lib.host_eval(n, 4, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), pp,
                      C.c_void_p(f.ctypes.data), C.c_void_p(Dv.ctypes.data))
        v = np.ascontiguousarray(rng.standard_normal((4, n)))
        jv = np.zeros((4, n))
        gp = np.zeros(64)
        lib.host_vjp(n, 4, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), pp,
                     C.c_void_p(v.ctypes.data), C.c_void_p(jv.ctypes.data), C.c_void_p(gp.ctypes.data))
    fo, Do, J = oracle.eval_points(med, y, om, jac=True)
    assert (np.abs(f - fo).max(axis=0) / np.abs(fo).max(axis=0)).max() < 1e-13
    assert np.abs(Dv - Do).max() < 1e-13 * (1 + np.abs(Do).max())
    jvo = np.einsum("nij,in->jn", J, v)
    assert np.abs(jv - jvo).max() / np.abs(jvo).max() < 1e-12
    go = oracle.param_vjp_points(med, y, om, v)
    assert np.abs(grad - go).max() / np.abs(go).max() < 1e-12


@pytest.mark.parametrize("cfg", ["cO2", "cX2"])
def test_coldplasma_vjp_matches_graph(cfg):
    """The cold-plasma determinant's VJP (second derivatives of eqs. 5-10;
    the oracle's cold-plasma model is forward only): the emitted VJP, built
    as host C++, against v^T J with J the graph's own symbolic derivatives
    of f = (-D_k/D_w, D_x/D_w) on the unfactored graph, at points near the
    benchmark's rays."""
    from paper_2508_15967_amd import media
    w = COLD[cfg]()
    g, D, params = media.build(w.medium)
    xs = [g.x(i) for i in range(3)]
    ks = [g.k(i) for i in range(3)]
    Dw = D.df(g.omega)
    f_nodes = [-(D.df(ki)) / Dw for ki in ks] + [D.df(xi) / Dw for xi in xs]
    J_nodes = [[fi.df(yj) for yj in xs + ks] for fi in f_nodes]
    prog = g.compile(D, want_adjoint=True, compile_only=True)
    rng = np.random.default_rng(21)
    n = 64
    y, om = _points(w, n, rng)
    v = np.ascontiguousarray(rng.standard_normal((6, n)))
    with tempfile.TemporaryDirectory() as tmp:
        lib = _host_lib(prog, True, tmp)
        jv, gp = np.zeros((6, n)), np.zeros(64)
        lib.host_vjp(n, 6, C.c_void_p(y.ctypes.data), C.c_void_p(om.ctypes.data), _ptrs(params),
                     C.c_void_p(v.ctypes.data), C.c_void_p(jv.ctypes.data), C.c_void_p(gp.ctypes.data))
    jv_ref = np.zeros((6, n))
    for r in range(n):
        ev = lambda nd: g.eval(nd, list(y[:3, r]), list(y[3:, r]), float(om[r]))
        jv_ref[:, r] = v[:, r] @ np.array([[ev(J_nodes[i][j]) for j in range(6)] for i in range(6)])
    assert (np.abs(jv - jv_ref).max(axis=0) / np.abs(jv_ref).max(axis=0)).max() < 1e-11
