"""The C-ABI library loads without a GPU and exports every entry point that
include/raygraph.h declares; host-only error paths return the documented
status codes; hipRTC compiles generated programs for gfx950."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2508_15967_amd import media
from paper_2508_15967_amd import raygraph as rgb
from paper_2508_15967_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "raygraph.h")).read()
    return sorted(set(re.findall(r"\b(rg_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    decl = _declared()
    assert "rg_trace_rays" in decl and "rg_compile" in decl and "rg_create_graph" in decl
    lib = C.CDLL(rgb.LIB_PATH)
    missing = [s for s in decl if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(rgb.SYMBOLS) == decl


def test_host_error_paths():
    lib = rgb._lib
    h = C.c_void_p()
    assert lib.rg_create_graph(C.c_uint32(4), C.byref(h)) == rgb.RG_EINVAL
    assert b"dim" in lib.rg_last_error()
    assert lib.rg_create_graph(C.c_uint32(2), None) == rgb.RG_EINVAL
    g = rgb.Graph(2)
    out = C.c_uint32()
    assert lib.rg_node_var(g.h, rgb.RG_X, C.c_uint32(2), C.byref(out)) == rgb.RG_EINVAL
    assert lib.rg_node_binary(g.h, 99, 0, 0, C.byref(out)) == rgb.RG_EINVAL
    assert lib.rg_node_binary(g.h, rgb.RG_ADD, 0, 10 ** 6, C.byref(out)) == rgb.RG_EINVAL
    assert lib.rg_trace_rays(None, None, None) == rgb.RG_EINVAL
    # a graph without omega dependence cannot give ray equations
    with pytest.raises(rgb.RayGraphError) as e:
        g.compile(g.x(0) * g.k(0), compile_only=True)
    assert e.value.status == rgb.RG_EINVAL


def test_compile_only_program_refuses_to_trace():
    w = W.make("1", 8)
    g, D, _ = media.build(w.medium)
    prog = g.compile(D, compile_only=True)
    d = rgb.TraceDesc()
    d.struct_size = C.sizeof(rgb.TraceDesc)
    assert rgb._lib.rg_trace_rays(prog.h, C.byref(d), None) == rgb.RG_ESTATE
    info = prog.info()
    assert info["dim"] == 2 and info["rhs_flops_alg"] > 0 and info["source_hash"] != 0
    src = prog.source()
    assert "rg_rk4_r1" in src and "rg_dopri_persistent" in src


def test_compile_opts_struct_size_checked():
    """A compile-options struct that is too small is refused before hipRTC runs."""
    o = rgb._CompileOpts(4, 0, 1, 0, None)
    w = W.make("1", 8)
    g, D, _ = media.build(w.medium)
    h = C.c_void_p()
    assert rgb._lib.rg_compile(g.h, D.id, C.byref(o), C.byref(h)) == rgb.RG_EINVAL
    assert b"struct_size" in rgb._lib.rg_last_error()


def test_trace_workspace_sizes_on_the_host():
    """rg_workspace_size needs no GPU for traces: none for persistent RK4, the
    per-ray state of the one-launch-per-step forms (16 B per ray for RK4,
    y, k1, t, h, facmax, status, steps, attempts for Dormand-Prince), 8 B of
    refill queue for persistent Dormand-Prince; zero rays need none."""
    w = W.make("3", 8)
    g, D, _ = media.build(w.medium)
    prog = g.compile(D, compile_only=True)
    ny = 2 * w.dim

    def size(n, integrator, mode):
        d = rgb.TraceDesc()
        d.struct_size = C.sizeof(rgb.TraceDesc)
        d.n_rays, d.integrator, d.mode = n, integrator, mode
        b = C.c_size_t()
        assert rgb._lib.rg_workspace_size(prog.h, C.byref(d), C.byref(b)) == rgb.RG_OK
        return b.value

    n = 1000
    assert size(n, rgb.RK4, rgb.PERSISTENT) == 0
    assert size(0, rgb.RK4, rgb.PLAIN) == 0
    assert 16 * n <= size(n, rgb.RK4, rgb.PLAIN) <= 16 * n + 3 * 256
    assert size(n, rgb.DOPRI54, rgb.PERSISTENT) == 8
    per_ray = 8 * (2 * ny + 3) + 4 * 3
    assert per_ray * n <= size(n, rgb.DOPRI54, rgb.PLAIN) <= per_ray * n + 10 * 256
    small = rgb.TraceDesc()
    small.struct_size = 4
    assert rgb._lib.rg_workspace_size(prog.h, C.byref(small), C.byref(C.c_size_t())) == rgb.RG_EINVAL


def test_graph_api_random_calls():
    """Random sequences of node-builder, df, eval, rendering and compile
    calls, valid and invalid (unknown kinds and operations, node ids out of
    range, parameters of length 0, non-finite constants): every call
    returns a status, the library never crashes, and whatever builds a
    relation in omega compiles (the emitter on arbitrary graphs)."""
    import random
    lib = rgb._lib
    rng = random.Random(0)
    vals = [0.0, -0.0, 1.0, -1.0, 2.0, 0.5, 1e300, -1e300, 1e-310, math.inf, -math.inf, math.nan, 3.7]
    out = C.c_uint32()
    compiled = 0
    for it in range(80):
        g = rgb.Graph(rng.choice([2, 3]))
        nodes = []

        def pick():
            return rng.choice(nodes) if nodes and rng.random() < 0.9 else rng.randint(0, 10 ** 6)
        for i in range(rng.randint(1, 60)):
            r = rng.random()
            if r < 0.2:
                st = lib.rg_node_var(g.h, rng.randint(-1, 4), C.c_uint32(rng.randint(0, 3)), C.byref(out))
            elif r < 0.35:
                st = lib.rg_node_const(g.h, C.c_double(rng.choice(vals)), C.byref(out))
            elif r < 0.55:
                st = lib.rg_node_unary(g.h, rng.randint(-1, 6), C.c_uint32(pick()), C.byref(out))
            elif r < 0.8:
                st = lib.rg_node_binary(g.h, rng.randint(-1, 4), C.c_uint32(pick()), C.c_uint32(pick()),
                                        C.byref(out))
            elif r < 0.88:
                st = lib.rg_node_powi(g.h, C.c_uint32(pick()), C.c_int32(rng.randint(-4, 6)), C.byref(out))
            elif r < 0.95 and nodes:
                st = lib.rg_df(g.h, C.c_uint32(rng.choice(nodes)), C.c_uint32(rng.choice(nodes)), C.byref(out))
            else:
                pidx = C.c_uint32()
                st = lib.rg_node_param(g.h, b"p%d" % i, C.c_uint32(rng.randint(0, 5)), C.byref(pidx))
                if st == rgb.RG_OK:
                    st = lib.rg_node_elem(g.h, pidx, C.c_uint32(rng.randint(0, 6)), C.byref(out))
            assert st in (rgb.RG_OK, rgb.RG_EINVAL), st
            if st == rgb.RG_OK:
                nodes.append(out.value)
        for n in nodes[-3:]:
            x = (C.c_double * 3)(*[rng.uniform(-2, 2) for _ in range(3)])
            k = (C.c_double * 3)(*[rng.uniform(-2, 2) for _ in range(3)])
            res = C.c_double()
            lib.rg_eval(g.h, C.c_uint32(n), x, k, C.c_double(1.3), C.c_double(0.2), None, C.byref(res))
            buf, need = C.create_string_buffer(64), C.c_size_t()
            assert lib.rg_node_to_string(g.h, C.c_uint32(n), buf, C.c_size_t(64), C.byref(need)) == rgb.RG_OK
        if nodes and rng.random() < 0.3:
            try:
                p = g.compile(rgb.Node(g, rng.choice(nodes)), want_adjoint=rng.random() < 0.5, compile_only=True)
                assert p.info()["source_hash"] != 0
                compiled += 1
            except rgb.RayGraphError as e:
                assert e.status in (rgb.RG_EINVAL, rgb.RG_EUNSUPPORTED), e
    assert compiled > 0
