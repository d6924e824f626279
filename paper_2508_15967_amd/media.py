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
            q = (m[0] * (k[0] * k[0]) + m[3] * (k[1] * k[1]) + m[5] * (k[2] * k[2])
                 + (2.0 * m[1]) * (k[0] * k[1]) + (2.0 * m[2]) * (k[0] * k[2])
                 + (2.0 * m[4]) * (k[1] * k[2]))
            terms.append(g.elem(pid, b) * gb * q)
        D = kk - w2 + _sum(terms)
    else:
        raise ValueError(f"unknown medium kind {med.kind}")
    return g, D, params
