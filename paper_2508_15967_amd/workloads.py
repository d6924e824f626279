"""Seeded synthetic workloads for the ray-tracing path.

This module only draws random numbers and lays out arrays.  It holds none of
the ray-tracing arithmetic (no ray equations, no integrator): both the CPU
oracle and the GPU path read the arrays built here.  The one piece of medium
arithmetic it does is placing each launch wavevector on the dispersion shell,
because the launch condition is part of each workload's definition.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) with the seed
equal to the workload number.  Arrays are float64, SoA: ``x0``/``k0`` have shape
``(dim, n_rays)``.  Asking for fewer rays than the full workload returns the
first ``n_rays`` of the full draw, so every subset is a slice of the same rays.

Workloads (the medium is always D = k.A(x).k - omega^2 N(x) or a special case):

1 ``lens2d``   2-D Gaussian lens n = 1 + 0.3 exp(-|x|^2/1.0), N = n^2; 1,024 rays
               from x=-5, y ~ U[-2,2], k = (n(x0), 0); RK4 dt=1e-3 x 1,000 steps,
               every state stored.
1b ``lens2d_long`` same medium, x0=-2, 4,000 steps, so the lens is crossed.
2 ``strat3d``  N = 1 - 0.8 exp(1 - zeta - exp(-zeta)), zeta = (z-10)/2;
               1,048,576 rays from the origin, elevation U[10,80] deg, azimuth
               U[0,360) deg, |k| = n(0); RK4 dt=5e-3 x 10,000 steps, every 100th
               state stored.
3 ``bumps3d``  strat3d + 8 Gaussian bumps on N (amplitude +-0.1, width U[1,3],
               centre U([-20,20]^2 x [2,20])); 4,194,304 rays, (x,y) ~ U[-10,10]^2,
               z=0; Dormand-Prince 5(4), rtol=atol=1e-9; box [-50,50]^2 x [0,40];
               per-ray budget round(2000 exp(0.8 Z)) clipped to [1, 50000].
4 ``spline2d`` N = 64x64 uniform cubic B-spline over [-10,10]^2, coefficients
               1 + 0.05 N(0,1); 65,536 rays from x=-8, y ~ U[-8,8], k=(sqrt N(x0),0);
               RK4 dt=2e-3 x 5,000 steps; targets U[-8,8]^2; checkpoints every 100.
5 ``aniso3d``  A(x) = I + sum_b s_b M_b exp(-|x-c_b|^2/w_b^2), 16 blobs, M_b SPD
               with eigenvalues in (0, 0.2], s_b = 1; 1,048,576 rays from x=-12,
               (y,z) ~ U[-8,8]^2, direction uniform in the 30-degree cap about +x,
               k = d / sqrt(d.A(x0).d); RK4 dt=1e-3 x 20,000 steps; targets
               U[-10,10]^3; checkpoints every 10 (117 GB of checkpoints, so
               that the adjoint's per-lane buffer of recomputed stage states
               is 393 MB instead of 3.9 GB at 100).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Medium kinds.  The integer values are part of the oracle's C interface too.
HOMOG, OLINEAR, LINEARN, LENS2D, STRAT3D, BUMPS3D, SPLINE2D, ANISO3D, COLDPLASMA = range(9)

RK4, DOPRI54 = 0, 1


@dataclasses.dataclass
class Medium:
    kind: int
    dim: int
    # scalar parameters; meaning depends on kind (see ``describe``)
    p: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(8))
    # Gaussian bumps / blobs
    centers: Optional[np.ndarray] = None  # (nb, 3)
    widths: Optional[np.ndarray] = None   # (nb,)
    amps: Optional[np.ndarray] = None     # (nb,)  bump amplitudes on N
    mats: Optional[np.ndarray] = None     # (nb, 6) symmetric xx,xy,xz,yy,yz,zz
    scales: Optional[np.ndarray] = None   # (nb,)  blob scales s_b (differentiable)
    # B-spline
    coef: Optional[np.ndarray] = None     # (nx, ny), row index = x
    lo: Optional[np.ndarray] = None       # (2,)
    hi: Optional[np.ndarray] = None       # (2,)

    def describe(self) -> str:
        names = {HOMOG: "homogeneous N=p0", OLINEAR: "D=|k|^2-w^2+(p0+g.x), g=p1..p3",
                 LINEARN: "N=p0+g.x, g=p1..p3", LENS2D: "n=1+p0 exp(-|x|^2/p1)",
                 STRAT3D: "N=1-p0 exp(1-z'-exp(-z')), z'=(z-p1)/p2",
                 BUMPS3D: "strat3d + sum a_b exp(-|x-c|^2/w^2)",
                 SPLINE2D: "cubic B-spline N", ANISO3D: "k.A.k-w^2",
                 COLDPLASMA: "Det(eps + nn - n^2 I), w_pe^2 = p0 (p1 x + 1), Omega_e = p2, m_i/m_e = p3"}
        return names[self.kind]


@dataclasses.dataclass
class Workload:
    name: str
    cfg: str
    dim: int
    medium: Medium
    x0: np.ndarray          # (dim, n)
    k0: np.ndarray          # (dim, n)
    omega: np.ndarray       # (n,)
    integrator: int = RK4
    dt: float = 0.0
    n_steps: int = 0
    store_every: int = 0    # 0: endpoints only
    # adaptive
    h0: float = 0.0
    rtol: float = 0.0
    atol: float = 0.0
    hmin: float = 0.0
    budget: Optional[np.ndarray] = None   # (n,) int32
    box_lo: Optional[np.ndarray] = None   # (dim,)
    box_hi: Optional[np.ndarray] = None
    # adjoint
    targets: Optional[np.ndarray] = None  # (dim, n)
    ckpt_every: int = 0
    fd_params: Optional[np.ndarray] = None  # parameter indices checked by FD
    # launch by Newton's method: k0[solve_k] is an initial guess (its sign and
    # size select the branch) to be replaced by the root of D = 0 in that
    # component before tracing; -1: k0 is already on the dispersion surface
    solve_k: int = -1

    @property
    def n(self) -> int:
        return int(self.x0.shape[1])

    def select(self, idx) -> "Workload":
        """The rays ``idx`` of this workload (same medium and settings)."""
        idx = np.asarray(idx)
        w = dataclasses.replace(self)
        w.x0 = np.ascontiguousarray(self.x0[:, idx])
        w.k0 = np.ascontiguousarray(self.k0[:, idx])
        w.omega = np.ascontiguousarray(self.omega[idx])
        if self.budget is not None:
            w.budget = np.ascontiguousarray(self.budget[idx])
        if self.targets is not None:
            w.targets = np.ascontiguousarray(self.targets[:, idx])
        return w

    def subset(self, n: int) -> "Workload":
        """First ``n`` rays of this workload (same medium and settings)."""
        n = min(n, self.n)
        w = dataclasses.replace(self)
        w.x0 = np.ascontiguousarray(self.x0[:, :n])
        w.k0 = np.ascontiguousarray(self.k0[:, :n])
        w.omega = np.ascontiguousarray(self.omega[:n])
        if self.budget is not None:
            w.budget = np.ascontiguousarray(self.budget[:n])
        if self.targets is not None:
            w.targets = np.ascontiguousarray(self.targets[:, :n])
        return w


# hydrogen ion to electron mass ratio; n_z of the oblique cold-plasma launches
MU_H = 1836.15267343
CP_NZ = 0.2

FULL_RAYS = {"1": 1024, "1b": 1024, "2": 1048576, "3": 4194304, "4": 65536, "5": 1048576}


def _slice(w: Workload, n_rays: Optional[int]) -> Workload:
    return w if n_rays is None else w.subset(n_rays)


# ---------------------------------------------------------------------------
# launch-shell helpers (medium values at the launch point only)

def _lens_n(x, y, amp=0.3, width=1.0):
    return 1.0 + amp * np.exp(-(x * x + y * y) / width)


def _strat_N(z, amp=0.8, z0=10.0, H=2.0):
    zeta = (z - z0) / H
    return 1.0 - amp * np.exp(1.0 - zeta - np.exp(-zeta))


def _bspline_weights(u):
    """Uniform cubic B-spline weights for local coordinate u in the cell."""
    return np.stack([(1 - u) ** 3 / 6, (3 * u ** 3 - 6 * u ** 2 + 4) / 6,
                     (-3 * u ** 3 + 3 * u ** 2 + 3 * u + 1) / 6, u ** 3 / 6])


def _spline_N(coef, lo, hi, x, y):
    nx, ny = coef.shape
    hx = (hi[0] - lo[0]) / (nx - 3)
    hy = (hi[1] - lo[1]) / (ny - 3)
    sx = (x - lo[0]) / hx + 1.0
    sy = (y - lo[1]) / hy + 1.0
    mx = np.clip(np.floor(sx), 1, nx - 3).astype(np.int64)
    my = np.clip(np.floor(sy), 1, ny - 3).astype(np.int64)
    wx = _bspline_weights(sx - mx)
    wy = _bspline_weights(sy - my)
    out = np.zeros_like(x)
    for a in range(4):
        for b in range(4):
            out += coef[mx - 1 + a, my - 1 + b] * wx[a] * wy[b]
    return out


# ---------------------------------------------------------------------------

def lens2d(n_rays: Optional[int] = None, long: bool = False) -> Workload:
    rng = np.random.default_rng(1)
    n = FULL_RAYS["1"]
    x0v = -2.0 if long else -5.0
    y0 = rng.uniform(-2.0, 2.0, n)
    x0 = np.stack([np.full(n, x0v), y0])
    nn = _lens_n(x0[0], x0[1])
    k0 = np.stack([nn, np.zeros(n)])
    med = Medium(LENS2D, 2, p=np.array([0.3, 1.0, 0, 0, 0, 0, 0, 0.0]))
    w = Workload("lens2d_long" if long else "lens2d", "1b" if long else "1", 2, med,
                 x0, k0, np.ones(n), RK4, dt=1e-3, n_steps=4000 if long else 1000,
                 store_every=1)
    return _slice(w, n_rays)


def _elev_azim(rng, n):
    el = np.deg2rad(rng.uniform(10.0, 80.0, n))
    az = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])


def strat3d(n_rays: Optional[int] = None) -> Workload:
    rng = np.random.default_rng(2)
    n = FULL_RAYS["2"]
    d = _elev_azim(rng, n)
    x0 = np.zeros((3, n))
    k0 = d * np.sqrt(_strat_N(0.0))
    med = Medium(STRAT3D, 3, p=np.array([0.8, 10.0, 2.0, 0, 0, 0, 0, 0.0]))
    w = Workload("strat3d", "2", 3, med, x0, k0, np.ones(n), RK4, dt=5e-3,
                 n_steps=10000, store_every=100)
    return _slice(w, n_rays)


def bumps3d(n_rays: Optional[int] = None) -> Workload:
    rng = np.random.default_rng(3)
    nb = 8
    amps = 0.1 * np.where(rng.random(nb) < 0.5, -1.0, 1.0)
    widths = rng.uniform(1.0, 3.0, nb)
    centers = np.stack([rng.uniform(-20, 20, nb), rng.uniform(-20, 20, nb),
                        rng.uniform(2, 20, nb)], axis=1)
    n = FULL_RAYS["3"]
    xy = rng.uniform(-10.0, 10.0, (2, n))
    x0 = np.concatenate([xy, np.zeros((1, n))])
    d = _elev_azim(rng, n)
    N0 = _strat_N(x0[2]) + sum(
        amps[b] * np.exp(-((x0 - centers[b][:, None]) ** 2).sum(0) / widths[b] ** 2)
        for b in range(nb))
    k0 = d * np.sqrt(N0)
    z = rng.standard_normal(n)
    budget = np.clip(np.round(2000.0 * np.exp(0.8 * z)), 1, 50000).astype(np.int32)
    med = Medium(BUMPS3D, 3, p=np.array([0.8, 10.0, 2.0, 0, 0, 0, 0, 0.0]),
                 centers=centers, widths=widths, amps=amps)
    w = Workload("bumps3d", "3", 3, med, x0, k0, np.ones(n), DOPRI54, h0=1e-2,
                 rtol=1e-9, atol=1e-9, hmin=1e-12, budget=budget,
                 box_lo=np.array([-50.0, -50.0, 0.0]), box_hi=np.array([50.0, 50.0, 40.0]))
    return _slice(w, n_rays)


def spline2d(n_rays: Optional[int] = None) -> Workload:
    rng = np.random.default_rng(4)
    coef = 1.0 + 0.05 * rng.standard_normal((64, 64))
    lo, hi = np.array([-10.0, -10.0]), np.array([10.0, 10.0])
    n = FULL_RAYS["4"]
    y0 = rng.uniform(-8.0, 8.0, n)
    x0 = np.stack([np.full(n, -8.0), y0])
    k0 = np.stack([np.sqrt(_spline_N(coef, lo, hi, x0[0], x0[1])), np.zeros(n)])
    targets = rng.uniform(-8.0, 8.0, (2, n))
    med = Medium(SPLINE2D, 2, coef=coef, lo=lo, hi=hi)
    # Coefficients checked by finite differences: drawn among those whose basis
    # support is crossed by many rays (rows of cells along the launch band).
    fd = _spline_fd_params(rng, coef.shape)
    w = Workload("spline2d", "4", 2, med, x0, k0, np.ones(n), RK4, dt=2e-3,
                 n_steps=5000, targets=targets, ckpt_every=100, fd_params=fd)
    return _slice(w, n_rays)


def _spline_fd_params(rng, shape):
    # x from -8 to about +2 and y in [-8, 8] are swept; coefficient (i, j) has
    # support on nodes X_{i-2}..X_{i+2}; keep i, j well inside that band.
    nx, ny = shape
    h = 20.0 / (nx - 3)
    xi = np.arange(nx) * h - 10.0 - h
    ok_i = np.nonzero((xi > -7.0) & (xi < 0.0))[0]
    ok_j = np.nonzero((xi > -7.0) & (xi < 7.0))[0]
    cand = (ok_i[:, None] * ny + ok_j[None, :]).ravel()
    return np.sort(rng.choice(cand, 32, replace=False)).astype(np.int64)


def _haar_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.diag(r))


def aniso3d(n_rays: Optional[int] = None) -> Workload:
    rng = np.random.default_rng(5)
    nb = 16
    centers = rng.uniform(-10.0, 10.0, (nb, 3))
    widths = rng.uniform(1.0, 3.0, nb)
    mats = np.zeros((nb, 6))
    for b in range(nb):
        q = _haar_rotation(rng)
        lam = 0.2 * (1.0 - rng.random(3))  # in (0, 0.2]
        m = q @ np.diag(lam) @ q.T
        mats[b] = [m[0, 0], m[0, 1], m[0, 2], m[1, 1], m[1, 2], m[2, 2]]
    scales = np.ones(nb)
    n = FULL_RAYS["5"]
    yz = rng.uniform(-8.0, 8.0, (2, n))
    x0 = np.concatenate([np.full((1, n), -12.0), yz])
    cth = rng.uniform(np.cos(np.deg2rad(30.0)), 1.0, n)
    sth = np.sqrt(1.0 - cth * cth)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    d = np.stack([cth, sth * np.cos(ph), sth * np.sin(ph)])
    # d.A(x0).d with A = I + sum_b s_b M_b g_b
    q = (d * d).sum(0)
    for b in range(nb):
        g = np.exp(-((x0 - centers[b][:, None]) ** 2).sum(0) / widths[b] ** 2)
        m = mats[b]
        dmd = (m[0] * d[0] * d[0] + m[3] * d[1] * d[1] + m[5] * d[2] * d[2]
               + 2 * (m[1] * d[0] * d[1] + m[2] * d[0] * d[2] + m[4] * d[1] * d[2]))
        q = q + scales[b] * g * dmd
    k0 = d / np.sqrt(q)
    targets = rng.uniform(-10.0, 10.0, (3, n))
    med = Medium(ANISO3D, 3, centers=centers, widths=widths, mats=mats, scales=scales)
    w = Workload("aniso3d", "5", 3, med, x0, k0, np.ones(n), RK4, dt=1e-3,
                 n_steps=20000, targets=targets, ckpt_every=10,
                 fd_params=np.arange(nb, dtype=np.int64))
    return _slice(w, n_rays)


def make(cfg: str, n_rays: Optional[int] = None) -> Workload:
    cfg = str(cfg)
    if cfg == "1":
        return lens2d(n_rays)
    if cfg == "1b":
        return lens2d(n_rays, long=True)
    if cfg == "2":
        return strat3d(n_rays)
    if cfg == "3":
        return bumps3d(n_rays)
    if cfg == "4":
        return spline2d(n_rays)
    if cfg == "5":
        return aniso3d(n_rays)
    if cfg == "cp":
        # the paper's own physics at its benchmark scale: 1,048,576 O-mode
        # rays in a two-species (electron, hydrogen ion) cold-plasma slab,
        # launched obliquely to B with k_x found by Newton's method, to the
        # plasma cut-off and back
        return coldplasma("O", n_rays if n_rays is not None else 1048576, dt=1e-2, n_steps=4000,
                          mu=MU_H, nz=CP_NZ)
    raise ValueError(f"unknown workload {cfg!r}")


# ---------------------------------------------------------------------------
# small analytic media used by the closed-form checks

def homog(n_rays: int = 64, dim: int = 3, N0: float = 1.7, seed: int = 11) -> Workload:
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-1, 1, (dim, n_rays))
    d = rng.standard_normal((dim, n_rays))
    d /= np.linalg.norm(d, axis=0)
    k0 = d * np.sqrt(N0) * 1.3
    omega = np.full(n_rays, 1.3)
    med = Medium(HOMOG, dim, p=np.array([N0, 0, 0, 0, 0, 0, 0, 0.0]))
    return Workload("homog", "h", dim, med, x0, k0, omega, RK4, dt=1e-2, n_steps=500)


def olinear(n_rays: int = 64, seed: int = 12) -> Workload:
    """O-mode with the linear profile f(x) = 0.1x + 1 for omega_p^2 (eq. 4)."""
    rng = np.random.default_rng(seed)
    x0 = np.stack([rng.uniform(-5, 0, n_rays), rng.uniform(-1, 1, n_rays),
                   rng.uniform(-1, 1, n_rays)])
    omega = np.full(n_rays, 1.2)
    ang = rng.uniform(-0.5, 0.5, (2, n_rays))
    d = np.stack([np.cos(ang[0]) * np.cos(ang[1]), np.sin(ang[0]) * np.cos(ang[1]),
                  np.sin(ang[1])])
    # on the shell: |k|^2 = w^2 - (0.1 x + 1)
    kk = np.sqrt(omega ** 2 - (0.1 * x0[0] + 1.0))
    k0 = d * kk
    med = Medium(OLINEAR, 3, p=np.array([1.0, 0.1, 0.0, 0.0, 0, 0, 0, 0.0]))
    return Workload("olinear", "o", 3, med, x0, k0, omega, RK4, dt=2e-2, n_steps=1500)


def linearn(n_rays: int = 8, seed: int = 13, dt: float = 1e-2, t_end: float = 4.0) -> Workload:
    """Isotropic medium with N = a + g.x (closed form in a ray parameter)."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-0.5, 0.5, (3, n_rays))
    a, g = 2.0, np.array([0.3, -0.2, 0.25])
    N0 = a + g @ x0
    d = rng.standard_normal((3, n_rays))
    d /= np.linalg.norm(d, axis=0)
    omega = np.full(n_rays, 1.1)
    k0 = d * omega * np.sqrt(N0)
    med = Medium(LINEARN, 3, p=np.array([a, g[0], g[1], g[2], 0, 0, 0, 0.0]))
    return Workload("linearn", "l", 3, med, x0, k0, omega, RK4, dt=dt,
                    n_steps=int(round(t_end / dt)))


# ---------------------------------------------------------------------------
# cold plasma (eqs. 5-10) in a slab: B along z, electron density following the
# linear profile f(x) = 0.1 x + 1 of eq. 4; omega, c = 1 units

def _stix(med, x, w):
    """Stix S, D, P at positions x for frequency w (electrons, optional ions)."""
    wpe2 = med.p[0] * (med.p[1] * x + 1.0)
    Xe, Ye = wpe2 / w ** 2, med.p[2] / w
    S = 1.0 - Xe / (1.0 - Ye ** 2)
    Dst = Ye * Xe / (1.0 - Ye ** 2)
    P = 1.0 - Xe
    if med.p[3] > 0:
        Xi, Yi = Xe / med.p[3], -Ye / med.p[3]
        S = S - Xi / (1.0 - Yi ** 2)
        Dst = Dst + Yi * Xi / (1.0 - Yi ** 2)
        P = P - Xi
    return S, Dst, P


def coldplasma(mode: str = "O", n_rays: int = 64, seed: int = 14, x0: float = -5.0,
               direction: float = 1.0, dt: float = 1e-2, n_steps: int = 2000, mu: float = 0.0,
               nz: float = 0.0) -> Workload:
    """Rays launched in the cold-plasma slab on the O- or X-mode branch.
    Profile: X = w_pe^2/w^2 = 0.5 (0.1 x + 1), Omega_e = -0.5 w, so for
    electrons the O cut-off (X = 1) is at x = 10, the upper-hybrid resonance
    (X = 0.75) at x = 5, the R cut-off (X = 0.5) at x = 0 and the L cut-off
    (X = 1.5) at x = 20.

    With mu = 0 and nz = 0 (electrons only, k perpendicular to B) the launch
    wavevector is on the branch's closed-form shell n^2 = P (O) or R L / S
    (X).  With an ion species (mass ratio mu > 0) or an oblique n_z = nz,
    k_z = nz w is fixed and k_x holds an initial guess for Newton's method
    (``solve_k = 0``): the electron-only perpendicular root of the branch,
    whose sign (direction) and size select the root of the full D."""
    rng = np.random.default_rng(seed)
    med = Medium(COLDPLASMA, 3, p=np.array([0.5, 0.1, -0.5, float(mu), 0, 0, 0, 0.0]))
    x = np.stack([np.full(n_rays, x0), rng.uniform(-1, 1, n_rays), np.zeros(n_rays)])
    w = np.ones(n_rays)
    el = Medium(COLDPLASMA, 3, p=np.array([0.5, 0.1, -0.5, 0.0, 0, 0, 0, 0.0]))
    S, Dst, P = _stix(el, x[0], w)
    n2 = P if mode == "O" else (S * S - Dst * Dst) / S   # perpendicular: P or RL/S
    ky = rng.uniform(-0.1, 0.1, n_rays) * np.sqrt(np.abs(n2))
    kz = np.full(n_rays, nz) * w
    kx = direction * np.sqrt(n2 * w ** 2 - ky ** 2 - kz ** 2)
    k = np.stack([kx, ky, kz])
    oblique = mu > 0 or nz != 0
    name = f"coldplasma_{mode}" + ("2" if oblique else "")
    return Workload(name, "c" + mode + ("2" if oblique else ""), 3, med, x, k, w, RK4, dt=dt,
                    n_steps=n_steps, solve_k=0 if oblique else -1)
