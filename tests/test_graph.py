"""Expression-graph front end through the C ABI (no GPU): the paper's
Listing 1, the reduce identities, hash-consing, the df leaf rules, the
chain rule against finite differences, and CPU evaluation."""
import math

import numpy as np
import pytest

from paper_2508_15967_amd import raygraph as rgb


def test_listing1_line_and_slope():
    """y = 10 x + 0.5 over a variable; dy/dx reduces to the constant 10 as
    the graph is built (Listing 1 and the discussion of Fig. 1)."""
    g = rgb.Graph(2)
    x = g.x(0)
    y = 10.0 * x + 0.5
    dydx = y.df(x)
    assert dydx.is_const(10.0)
    for v in (-3.0, 0.0, 2.5):
        assert g.eval(y, [v, 0.0], [0.0, 0.0]) == 10.0 * v + 0.5
    # d/dx of a different variable is exactly 0
    assert y.df(g.x(1)).is_const(0.0)


def test_reduce_identities():
    g = rgb.Graph(3)
    x = g.x(0)
    zero, one = g.const(0.0), g.const(1.0)
    assert (x + zero) == x and (zero + x) == x
    assert (x * one) == x and (one * x) == x
    assert (x * zero).is_const(0.0) and (zero * x).is_const(0.0)
    assert (x - zero) == x
    assert (x - x).is_const(0.0)
    assert (x / one) == x
    assert (-(-x)) == x
    assert (g.const(2.0) + g.const(3.0)).is_const(5.0)       # constant folding
    assert g.const(2.0).exp().is_const(math.exp(2.0))
    assert (2.0 * (3.0 * x)) == (6.0 * x)


def test_hash_consing():
    """The same sub-graph built twice is the same node (node cache)."""
    g = rgb.Graph(3)
    a = (g.x(0) * g.k(1) + g.omega).exp()
    n = g.size()
    b = (g.x(0) * g.k(1) + g.omega).exp()
    assert a == b and g.size() == n
    # commutative operands are canonicalised
    assert (g.x(0) + g.x(1)) == (g.x(1) + g.x(0))
    assert (g.k(0) * g.x(2)) == (g.x(2) * g.k(0))


def test_leaf_derivatives():
    g = rgb.Graph(2)
    assert g.const(3.0).df(g.x(0)).is_const(0.0)
    assert g.x(0).df(g.x(0)).is_const(1.0)
    assert g.x(0).df(g.x(1)).is_const(0.0)
    assert g.k(1).df(g.k(1)).is_const(1.0)
    assert g.omega.df(g.omega).is_const(1.0)


def _fd(g, f, wrt_kind, i, x, k, om, h=1e-6):
    def ev(dx):
        xx, kk, oo = list(x), list(k), om
        if wrt_kind == "x":
            xx[i] += dx
        elif wrt_kind == "k":
            kk[i] += dx
        else:
            oo += dx
        return g.eval(f, xx, kk, oo)
    return (ev(h) - ev(-h)) / (2 * h)


@pytest.mark.parametrize("seed", range(4))
def test_chain_rule_vs_finite_differences(seed):
    rng = np.random.default_rng(seed)
    g = rgb.Graph(3)
    x = [g.x(i) for i in range(3)]
    k = [g.k(i) for i in range(3)]
    om = g.omega
    f = ((x[0] * k[1] - x[2] / (1.5 + k[0] * k[0])).exp() * (x[1] * x[1] + 2.0).sqrt()
         + (om * x[2]).sin() - (k[2] + 3.0).log() * (x[0] ** 3) + (x[1] - k[0]).cos() / om)
    xv = rng.uniform(-0.7, 0.7, 3)
    kv = rng.uniform(-0.7, 0.7, 3)
    ov = 1.3
    for kind, nodes in (("x", x), ("k", k), ("w", [om])):
        for i, v in enumerate(nodes):
            d = f.df(v)
            an = g.eval(d, xv, kv, ov)
            fd = _fd(g, f, kind, i, xv, kv, ov)
            assert abs(an - fd) < 1e-7 * (1 + abs(fd)), (kind, i, an, fd)
            # second derivative through df of df
            d2 = d.df(x[0])
            h = 1e-5
            xp, xm = xv.copy(), xv.copy()
            xp[0] += h
            xm[0] -= h
            fd2 = (g.eval(d, xp, kv, ov) - g.eval(d, xm, kv, ov)) / (2 * h)
            assert abs(g.eval(d2, xv, kv, ov) - fd2) < 1e-6 * (1 + abs(fd2))


def test_parameters_and_spline_nodes():
    g = rgb.Graph(2)
    p = g.param("s", 3)
    e = g.elem(p, 2)
    f = e * g.x(0) * g.x(0)
    assert f.df(e) == g.x(0) * g.x(0)
    vals = np.array([0.0, 0.0, 4.0])
    assert g.eval(f, [3.0, 0.0], [0.0, 0.0], params=[vals]) == 36.0
    c = g.param("coef", 8 * 8)
    coef = np.ones(64)
    s = g.bspline2(c, 8, 8, [-1.0, -1.0], [1.0, 1.0], g.x(0), g.x(1))
    # partition of unity: spline of ones is 1, its derivative 0
    assert abs(g.eval(s, [0.3, -0.2], [0, 0], params=[vals, coef]) - 1.0) < 1e-15
    assert abs(g.eval(s.df(g.x(0)), [0.3, -0.2], [0, 0], params=[vals, coef])) < 1e-14
    with pytest.raises(rgb.RayGraphError):
        g.elem(p, 3)  # out of range
    with pytest.raises(rgb.RayGraphError):
        g.bspline2(c, 9, 8, [-1.0, -1.0], [1.0, 1.0], g.x(0), g.x(1))  # too few coefficients


def test_rendering():
    g = rgb.Graph(2)
    s = repr(10.0 * g.x(0) + 0.5)
    assert "x0" in s and "10" in s and "0.5" in s
