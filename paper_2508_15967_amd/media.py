"""Dispersion relations of the workload media, built as expression graphs.

This is the application layer the paper describes ("Impact" section): an
equilibrium/medium expression and a dispersion relation D(x, k, omega) built
from graph nodes; the ray equations are then obtained by the library's
automatic differentiation at compile time.  Medium constants become graph
constants (folded into the generated code); differentiable quantities
(B-spline coefficients, blob scales) are parameter arrays.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import raygraph as rgb
from . import workloads as W


def _sum(nodes):
    out = nodes[0]
    for n in nodes[1:]:
        out = out + n
    return out


def build(med: W.Medium) -> Tuple[rgb.Graph, rgb.Node, List[np.ndarray]]:
    """Return (graph, D, parameter arrays in declaration order)."""
    d = med.dim
    g = rgb.Graph(d)
    x = [g.x(i) for i in range(d)]
    k = [g.k(i) for i in range(d)]
    om = g.omega
    kk = _sum([ki * ki for ki in k])
    w2 = om * om
    params: List[np.ndarray] = []
    p = med.p
    if med.kind == W.HOMOG:
        D = kk - w2 * float(p[0])
    elif med.kind == W.OLINEAR:
        # O-mode, omega_p^2 = a + g.x (eq. 10 with the eq. 4 profile)
        D = kk - w2 + (float(p[0]) + _sum([float(p[1 + i]) * x[i] for i in range(d)]))
    elif med.kind == W.LINEARN:
        D = kk - w2 * (float(p[0]) + _sum([float(p[1 + i]) * x[i] for i in range(d)]))
    elif med.kind == W.LENS2D:
        r2 = _sum([xi * xi for xi in x])
        n = 1.0 + float(p[0]) * (r2 * (-1.0 / float(p[1]))).exp()
        D = kk - w2 * (n * n)
    elif med.kind in (W.STRAT3D, W.BUMPS3D):
        zeta = (x[2] - float(p[1])) * (1.0 / float(p[2]))
        N = 1.0 - float(p[0]) * (1.0 - zeta - (-zeta).exp()).exp()
        if med.kind == W.BUMPS3D:
            for b in range(len(med.amps)):
                c = med.centers[b]
                r2 = _sum([(x[i] - float(c[i])) * (x[i] - float(c[i])) for i in range(3)])
                N = N + float(med.amps[b]) * (r2 * (-1.0 / float(med.widths[b]) ** 2)).exp()
        D = kk - w2 * N
    elif med.kind == W.SPLINE2D:
        nx, ny = med.coef.shape
        pid = g.param("coef", nx * ny)
        params.append(np.ascontiguousarray(med.coef, dtype=np.float64).ravel())
        N = g.bspline2(pid, nx, ny, list(med.lo), list(med.hi), x[0], x[1])
        D = kk - w2 * N
    elif med.kind == W.ANISO3D:
        nb = len(med.scales)
        pid = g.param("s", nb)
        params.append(np.ascontiguousarray(med.scales, dtype=np.float64))
        terms = []
        for b in range(nb):
            c = med.centers[b]
            m = [float(v) for v in med.mats[b]]  # xx xy xz yy yz zz
            r2 = _sum([(x[i] - float(c[i])) * (x[i] - float(c[i])) for i in range(3)])
            gb = (r2 * (-1.0 / float(med.widths[b]) ** 2)).exp()
            # q = k . (M k)
            M = [[m[0], m[1], m[2]], [m[1], m[3], m[4]], [m[2], m[4], m[5]]]
            mk = [_sum([M[i][j] * k[j] for j in range(3)]) for i in range(3)]
            q = _sum([k[i] * mk[i] for i in range(3)])
            terms.append(g.elem(pid, b) * gb * q)
        D = kk - w2 + _sum(terms)
    elif med.kind == W.COLDPLASMA:
        # "Cold Plasma Dispersion Relation": D = Det(eps + n n - n^2 I) (eq. 5)
        # with n = k/omega (eq. 6, c = 1) and the Stix elements of eqs. 8-10;
        # eps_12 = -i G is purely imaginary, so the Hermitian determinant is
        # the real expression M11 M22 M33 - M11 M23^2 - M22 M13^2
        # - (a^2 + G^2) M33 + 2 a M13 M23 with a = n_x n_y.
        X = (float(p[0]) * (float(p[1]) * x[0] + 1.0)) / w2
        Y = float(p[2]) / om
        den = 1.0 - Y * Y
        S = 1.0 - X / den
        G = (Y * X) / den
        P = 1.0 - X
        if p[3] > 0:
            mu = float(p[3])
            Xi, Yi = X * (1.0 / mu), Y * (-1.0 / mu)
            deni = 1.0 - Yi * Yi
            S = S - Xi / deni
            G = G + (Yi * Xi) / deni
            P = P - Xi
        n = [ki / om for ki in k]
        n2 = _sum([ni * ni for ni in n])
        M11 = S + n[0] * n[0] - n2
        M22 = S + n[1] * n[1] - n2
        M33 = P + n[2] * n[2] - n2
        a = n[0] * n[1]
        M13 = n[0] * n[2]
        M23 = n[1] * n[2]
        D = (M11 * M22 * M33 - M11 * (M23 * M23) - M22 * (M13 * M13)
             - (a * a + G * G) * M33 + 2.0 * (a * M13 * M23))
    else:
        raise ValueError(f"unknown medium kind {med.kind}")
    return g, D, params
