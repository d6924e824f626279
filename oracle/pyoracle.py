"""ctypes binding of the FP64 CPU oracle (``oracle.c``).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline call this module.  It imports nothing from the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

RAY_OK, RAY_EXITED_BOX, RAY_BUDGET, RAY_NONFINITE, RAY_STEP_UNDERFLOW = range(5)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Medium(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dim", C.c_int32), ("nb", C.c_int32),
                ("nx", C.c_int32), ("ny", C.c_int32), ("pad", C.c_int32),
                ("p", C.c_double * 8),
                ("centers", C.c_void_p), ("widths", C.c_void_p), ("amps", C.c_void_p),
                ("mats", C.c_void_p), ("scales", C.c_void_p), ("coef", C.c_void_p),
                ("lo", C.c_double * 2), ("hi", C.c_double * 2)]


class _Opts(C.Structure):
    _fields_ = [("integrator", C.c_int32), ("n_steps", C.c_int32), ("dt", C.c_double),
                ("h0", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("hmin", C.c_double), ("budget", C.c_void_p), ("max_steps", C.c_int32),
                ("has_box", C.c_int32), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3), ("t_end", C.c_double),
                ("store_every", C.c_int32), ("n_threads", C.c_int32),
                ("traj", C.c_void_p), ("traj_D", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=False)
        _lib = C.CDLL(LIB)
        _lib.om_trace.restype = C.c_int
        _lib.om_eval_points.restype = C.c_int
        _lib.om_rk4_tangent.restype = C.c_int
        _lib.om_rk4_adjoint.restype = C.c_int
        _lib.om_param_vjp_points.restype = C.c_int
        _lib.om_n_params.restype = C.c_int64
        _lib.om_threads.restype = C.c_int
        _lib.om_dp_factor.restype = C.c_double
        _lib.om_dp_factor.argtypes = [C.c_double, C.c_double]
    return _lib


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Medium:
    """Holds the C struct plus the arrays it points into (kept alive)."""

    def __init__(self, med):
        self._keep = []
        s = _Medium()
        s.kind, s.dim = int(med.kind), int(med.dim)
        p = np.zeros(8)
        if med.p is not None:
            p[: len(med.p)] = med.p
        s.p[:] = list(p)
        for name in ("centers", "widths", "amps", "mats", "scales", "coef"):
            arr = _f64(getattr(med, name))
            if arr is not None:
                self._keep.append(arr)
                setattr(s, name, arr.ctypes.data)
        if med.centers is not None:
            s.nb = int(med.centers.shape[0])
        if med.coef is not None:
            s.nx, s.ny = (int(v) for v in med.coef.shape)
            s.lo[:] = list(med.lo)
            s.hi[:] = list(med.hi)
        self.s = s
        self.dim = s.dim

    def n_params(self) -> int:
        return int(lib().om_n_params(C.byref(self.s)))


def _opts(w, n_threads=0, traj=None, traj_D=None, max_steps=0, t_end=0.0):
    o = _Opts()
    o.integrator = int(w.integrator)
    o.n_steps = int(w.n_steps)
    o.dt = float(w.dt)
    o.h0, o.rtol, o.atol, o.hmin = float(w.h0), float(w.rtol), float(w.atol), float(w.hmin)
    o.max_steps = int(max_steps)
    o.t_end = float(t_end)
    if w.box_lo is not None:
        o.has_box = 1
        lo = np.zeros(3)
        hi = np.zeros(3)
        lo[: w.dim] = w.box_lo
        hi[: w.dim] = w.box_hi
        o.box_lo[:] = list(lo)
        o.box_hi[:] = list(hi)
    o.store_every = int(w.store_every) if traj is not None or traj_D is not None else 0
    o.n_threads = int(n_threads)
    o.traj = None if traj is None else traj.ctypes.data
    o.traj_D = None if traj_D is None else traj_D.ctypes.data
    return o


def n_snapshots(w) -> int:
    return w.n_steps // w.store_every + 1 if w.store_every > 0 else 0


def trace(w, n_threads: int = 0, store: bool = False, store_D: bool = False,
          max_steps: int = 0, t_end: float = 0.0):
    """Trace all rays of workload ``w``.  Returns a dict of numpy arrays."""
    med = Medium(w.medium)
    n, d = w.n, w.dim
    x0, k0, om = _f64(w.x0), _f64(w.k0), _f64(w.omega)
    out = {"x": np.zeros((d, n)), "k": np.zeros((d, n)), "t": np.zeros(n),
           "status": np.zeros(n, np.int32), "steps": np.zeros(n, np.int32),
           "attempts": np.zeros(n, np.int32)}
    traj = trajD = None
    if store and w.store_every > 0:
        traj = np.zeros((n_snapshots(w), 2 * d, n))
        out["traj"] = traj
    if store_D and w.store_every > 0:
        trajD = np.zeros((n_snapshots(w), n))
        out["traj_D"] = trajD
    o = _opts(w, n_threads, traj, trajD, max_steps, t_end)
    budget = None
    if w.budget is not None:
        budget = np.ascontiguousarray(w.budget, dtype=np.int32)
        o.budget = budget.ctypes.data
    rc = lib().om_trace(C.byref(med.s), C.byref(o), C.c_int64(n), _ptr(x0), _ptr(k0), _ptr(om),
                        _ptr(out["x"]), _ptr(out["k"]), _ptr(out["t"]), _ptr(out["status"]),
                        _ptr(out["steps"]), _ptr(out["attempts"]))
    if rc != 0:
        raise RuntimeError(f"om_trace failed ({rc})")
    return out


def eval_points(medium, y, omega, jac: bool = False):
    """Ray right-hand side f (SoA [2d][n]), D [n] and optionally J [n][2d][2d]."""
    med = Medium(medium)
    y = _f64(y)
    n = y.shape[1]
    n2 = y.shape[0]
    om = _f64(np.broadcast_to(omega, (n,)))
    f = np.zeros((n2, n))
    D = np.zeros(n)
    J = np.zeros((n, n2, n2)) if jac else None
    lib().om_eval_points(C.byref(med.s), C.c_int64(n), _ptr(y), _ptr(om), _ptr(f), _ptr(D),
                         _ptr(J))
    return f, D, J


def param_vjp_points(medium, y, omega, v):
    med = Medium(medium)
    y, v = _f64(y), _f64(v)
    n = y.shape[1]
    om = _f64(np.broadcast_to(omega, (n,)))
    g = np.zeros(max(med.n_params(), 1))
    lib().om_param_vjp_points(C.byref(med.s), C.c_int64(n), _ptr(y), _ptr(om), _ptr(v), _ptr(g))
    return g[: med.n_params()]


def tangent(w, dy0, p: int = -1, n_threads: int = 0):
    """Tangent-linear RK4: returns dy_end (SoA [2d][n]) for initial
    perturbation dy0 and unit parameter direction p (p < 0: none)."""
    med = Medium(w.medium)
    dy0 = _f64(dy0)
    out = np.zeros_like(dy0)
    o = _opts(w, n_threads)
    lib().om_rk4_tangent(C.byref(med.s), C.byref(o), C.c_int64(w.n), _ptr(_f64(w.x0)),
                         _ptr(_f64(w.k0)), _ptr(_f64(w.omega)), _ptr(dy0), C.c_int64(p),
                         _ptr(out))
    return out


def adjoint(w, lam_end, n_threads: int = 0):
    """Discrete RK4 adjoint: returns (dL/dy0 SoA [2d][n], dL/dtheta)."""
    med = Medium(w.medium)
    lam_end = _f64(lam_end)
    lam0 = np.zeros_like(lam_end)
    g = np.zeros(max(med.n_params(), 1))
    o = _opts(w, n_threads)
    lib().om_rk4_adjoint(C.byref(med.s), C.byref(o), C.c_int64(w.n), _ptr(_f64(w.x0)),
                         _ptr(_f64(w.k0)), _ptr(_f64(w.omega)), _ptr(lam_end), _ptr(lam0),
                         _ptr(g))
    return lam0, g[: med.n_params()]


def threads() -> int:
    return int(lib().om_threads())


def dp_factor(err: float, facmax: float = 5.0) -> float:
    """The Dormand-Prince step-size factor after an attempt with scaled error err."""
    return float(lib().om_dp_factor(float(err), float(facmax)))


def dopri_attempt(medium, y, omega, h, rtol, atol):
    """One Dormand-Prince attempt of size h from each point y (SoA [2d][n]):
    returns (5th-order solution y5, error vector e = y5 - y4, scaled RMS
    error err)."""
    med = Medium(medium)
    y = _f64(y)
    n = y.shape[1]
    om = _f64(np.broadcast_to(omega, (n,)))
    y5, e, err = np.zeros_like(y), np.zeros_like(y), np.zeros(n)
    lib().om_dopri_attempt(C.byref(med.s), C.c_int64(n), _ptr(y), _ptr(om), C.c_double(h),
                           C.c_double(rtol), C.c_double(atol), _ptr(y5), _ptr(e), _ptr(err))
    return y5, e, err


def dopri_tableau():
    c, a, b5, b4 = np.zeros(7), np.zeros((7, 6)), np.zeros(7), np.zeros(7)
    lib().om_dopri_tableau(_ptr(c), _ptr(a), _ptr(b5), _ptr(b4))
    return c, a, b5, b4


def newton_k(medium, x, k, omega, component=0, tol=1e-15, max_iter=50):
    """Newton solve of D = 0 for k[component]; returns (k, iters, D)."""
    med = Medium(medium)
    x = _f64(x)
    k = np.array(k, dtype=np.float64, copy=True, order="C")
    n = x.shape[1]
    om = _f64(np.broadcast_to(omega, (n,)))
    it = np.zeros(n, np.int32)
    D = np.zeros(n)
    lib().om_newton_k(C.byref(med.s), C.c_int64(n), _ptr(x), _ptr(k), _ptr(om), C.c_int(component),
                      C.c_double(tol), C.c_int(max_iter), _ptr(it), _ptr(D))
    return k, it, D
