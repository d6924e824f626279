// extern "C" boundary of the library (include/raygraph.h).  Every entry
// point validates its arguments, catches every C++ exception and reports
// failures through a status code plus a thread-local message.
#include <cstring>
#include <exception>
#include <new>
#include <stdexcept>
#include <string>

#include "graph.hpp"
#include "program.hpp"

struct rg_graph {
    explicit rg_graph(uint32_t dim) : g(dim) {}
    rg::Graph g;
};

namespace {
thread_local std::string g_err;
}

namespace rg {
rg_status fail(rg_status code, const std::string &msg) {
    g_err = msg;
    return code;
}
}  // namespace rg

using rg::fail;

#define GUARD_BEGIN try {
#define GUARD_END                                                   \
    }                                                               \
    catch (const std::bad_alloc &) {                                \
        return fail(RG_ENOMEM, "host allocation failed");           \
    }                                                               \
    catch (const std::invalid_argument &e) {                        \
        return fail(RG_EINVAL, e.what());                           \
    }                                                               \
    catch (const std::exception &e) {                               \
        return fail(RG_EINVAL, e.what());                           \
    }                                                               \
    catch (...) {                                                   \
        return fail(RG_EINVAL, "unknown error");                    \
    }

static bool valid_node(const rg_graph *g, rg_node n) { return g && n < g->g.size(); }

extern "C" {

const char *rg_last_error(void) { return g_err.c_str(); }

rg_status rg_create_graph(uint32_t dim, rg_graph **out) {
    if (!out) return fail(RG_EINVAL, "out is NULL");
    if (dim != 2 && dim != 3) return fail(RG_EINVAL, "dim must be 2 or 3");
    GUARD_BEGIN
    *out = new rg_graph(dim);
    return RG_OK;
    GUARD_END
}

rg_status rg_destroy_graph(rg_graph *g) {
    delete g;
    return RG_OK;
}

rg_status rg_node_var(rg_graph *g, int32_t which, uint32_t i, rg_node *out) {
    if (!g || !out) return fail(RG_EINVAL, "NULL argument");
    if (which == RG_X || which == RG_K) {
        if (i >= g->g.dim()) return fail(RG_EINVAL, "component index out of range");
    } else if (which == RG_OMEGA || which == RG_T) {
        if (i != 0) return fail(RG_EINVAL, "omega and t are scalars (i must be 0)");
    } else {
        return fail(RG_EINVAL, "unknown variable kind");
    }
    GUARD_BEGIN
    *out = g->g.var(which, i);
    return RG_OK;
    GUARD_END
}

rg_status rg_node_const(rg_graph *g, double v, rg_node *out) {
    if (!g || !out) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    *out = g->g.constant(v);
    return RG_OK;
    GUARD_END
}

rg_status rg_node_param(rg_graph *g, const char *name, uint32_t len, uint32_t *param_out) {
    if (!g || !param_out) return fail(RG_EINVAL, "NULL argument");
    if (len == 0) return fail(RG_EINVAL, "parameter length must be > 0");
    if (g->g.params().size() >= RG_KMAX_PARAMS) return fail(RG_EUNSUPPORTED, "at most 8 parameter arrays");
    GUARD_BEGIN
    *param_out = g->g.declare_param(name ? name : "p", len);
    return RG_OK;
    GUARD_END
}

rg_status rg_node_elem(rg_graph *g, uint32_t param, uint32_t idx, rg_node *out) {
    if (!g || !out) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    *out = g->g.param_elem(param, idx);
    return RG_OK;
    GUARD_END
}

rg_status rg_node_unary(rg_graph *g, int32_t op, rg_node a, rg_node *out) {
    if (!out || !valid_node(g, a)) return fail(RG_EINVAL, "bad graph or node");
    GUARD_BEGIN
    switch (op) {
    case RG_NEG: *out = g->g.neg(a); break;
    case RG_EXP: *out = g->g.unary(rg::EXP, a); break;
    case RG_LOG: *out = g->g.unary(rg::LOG, a); break;
    case RG_SQRT: *out = g->g.unary(rg::SQRT, a); break;
    case RG_SIN: *out = g->g.unary(rg::SIN, a); break;
    case RG_COS: *out = g->g.unary(rg::COS, a); break;
    default: return fail(RG_EINVAL, "unknown unary op");
    }
    return RG_OK;
    GUARD_END
}

rg_status rg_node_binary(rg_graph *g, int32_t op, rg_node a, rg_node b, rg_node *out) {
    if (!out || !valid_node(g, a) || !valid_node(g, b)) return fail(RG_EINVAL, "bad graph or node");
    GUARD_BEGIN
    switch (op) {
    case RG_ADD: *out = g->g.add(a, b); break;
    case RG_SUB: *out = g->g.sub(a, b); break;
    case RG_MUL: *out = g->g.mul(a, b); break;
    case RG_DIV: *out = g->g.div(a, b); break;
    default: return fail(RG_EINVAL, "unknown binary op");
    }
    return RG_OK;
    GUARD_END
}

rg_status rg_node_powi(rg_graph *g, rg_node a, int32_t n, rg_node *out) {
    if (!out || !valid_node(g, a)) return fail(RG_EINVAL, "bad graph or node");
    if (n < -64 || n > 64) return fail(RG_EINVAL, "|n| must be <= 64");
    GUARD_BEGIN
    *out = g->g.powi(a, n);
    return RG_OK;
    GUARD_END
}

rg_status rg_node_bspline2(rg_graph *g, uint32_t coeff_param, uint32_t nx, uint32_t ny,
                           const double lo[2], const double hi[2], rg_node u, rg_node v,
                           rg_node *out) {
    if (!out || !lo || !hi || !valid_node(g, u) || !valid_node(g, v))
        return fail(RG_EINVAL, "bad argument");
    if (coeff_param >= g->g.params().size()) return fail(RG_EINVAL, "unknown parameter");
    if (nx < 4 || ny < 4) return fail(RG_EINVAL, "a cubic B-spline needs at least 4 coefficients per axis");
    if ((uint64_t)nx * ny > g->g.params()[coeff_param].len)
        return fail(RG_EINVAL, "parameter shorter than nx*ny");
    if (!(hi[0] > lo[0]) || !(hi[1] > lo[1])) return fail(RG_EINVAL, "empty spline domain");
    GUARD_BEGIN
    rg::SplineDef d{coeff_param, nx, ny, {lo[0], lo[1]}, {hi[0], hi[1]}};
    uint32_t def = g->g.declare_spline(d);
    *out = g->g.spline(def, 0, 0, u, v);
    return RG_OK;
    GUARD_END
}

rg_status rg_df(rg_graph *g, rg_node f, rg_node wrt, rg_node *out) {
    if (!out || !valid_node(g, f) || !valid_node(g, wrt)) return fail(RG_EINVAL, "bad graph or node");
    GUARD_BEGIN
    *out = g->g.df(f, wrt);
    return RG_OK;
    GUARD_END
}

rg_status rg_node_get(const rg_graph *g, rg_node n, rg_node_desc *out) {
    if (!out || !valid_node(g, n)) return fail(RG_EINVAL, "bad graph or node");
    const rg::Node &nd = g->g.node(n);
    out->op = nd.op;
    out->aux = nd.aux;
    out->a = nd.a;
    out->b = nd.b;
    out->value = nd.val;
    return RG_OK;
}

rg_status rg_graph_size(const rg_graph *g, uint32_t *n) {
    if (!g || !n) return fail(RG_EINVAL, "NULL argument");
    *n = g->g.size();
    return RG_OK;
}

rg_status rg_eval(const rg_graph *g, rg_node f, const double *x, const double *k, double omega,
                  double t, const double *const *params, double *out) {
    if (!out || !x || !k || !valid_node(g, f)) return fail(RG_EINVAL, "bad argument");
    GUARD_BEGIN
    *out = g->g.eval(f, x, k, omega, t, params);
    return RG_OK;
    GUARD_END
}

rg_status rg_node_to_string(const rg_graph *g, rg_node n, char *buf, size_t cap, size_t *needed) {
    if (!valid_node(g, n)) return fail(RG_EINVAL, "bad graph or node");
    GUARD_BEGIN
    std::string s = g->g.to_string(n);
    if (needed) *needed = s.size() + 1;
    if (buf && cap > 0) {
        size_t m = s.size() < cap - 1 ? s.size() : cap - 1;
        std::memcpy(buf, s.data(), m);
        buf[m] = '\0';
    }
    return RG_OK;
    GUARD_END
}

rg_status rg_compile(rg_graph *g, rg_node D, const rg_compile_opts *opts, rg_program **out) {
    if (!out || !valid_node(g, D)) return fail(RG_EINVAL, "bad graph, node or output");
    rg_compile_opts o{};
    o.struct_size = sizeof o;
    if (opts) {
        if (opts->struct_size < sizeof(rg_compile_opts)) return fail(RG_EINVAL, "rg_compile_opts.struct_size too small");
        o = *opts;
    }
    GUARD_BEGIN
    rg_program *p = new rg_program();
    rg_status st = rg::build_program(g->g, D, o, p);
    if (st != RG_OK) {
        delete p;
        return st;
    }
    *out = p;
    return RG_OK;
    GUARD_END
}

rg_status rg_destroy_program(rg_program *p) {
    GUARD_BEGIN
    delete p;
    return RG_OK;
    GUARD_END
}

rg_status rg_program_info_get(const rg_program *p, rg_program_info *out) {
    if (!p || !out) return fail(RG_EINVAL, "NULL argument");
    if (out->struct_size != 0 && out->struct_size < sizeof(rg_program_info))
        return fail(RG_EINVAL, "rg_program_info.struct_size too small");
    *out = p->info;
    return RG_OK;
}

rg_status rg_program_source(const rg_program *p, const char **src) {
    if (!p || !src) return fail(RG_EINVAL, "NULL argument");
    *src = p->full_src.c_str();
    return RG_OK;
}

rg_status rg_program_functions(const rg_program *p, const char **src) {
    if (!p || !src) return fail(RG_EINVAL, "NULL argument");
    *src = p->functions_src.c_str();
    return RG_OK;
}

rg_status rg_trace_rays(rg_program *p, const rg_trace_desc *d, void *stream) {
    if (!p || !d) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    return rg::trace(p, *d, (hipStream_t)stream);
    GUARD_END
}

rg_status rg_trace_rays_adjoint(rg_program *p, const rg_adjoint_desc *d, void *stream) {
    if (!p || !d) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    return rg::adjoint(p, *d, (hipStream_t)stream);
    GUARD_END
}

rg_status rg_program_load(rg_program *p) {
    if (!p) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    return rg::program_load(p);
    GUARD_END
}

rg_status rg_trace_rays_noalloc(rg_program *p, const rg_trace_desc *d, void *stream) {
    if (!p || !d) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    return rg::trace_noalloc(p, *d, (hipStream_t)stream);
    GUARD_END
}

rg_status rg_workspace_size(rg_program *p, const rg_trace_desc *d, size_t *bytes) {
    if (!p || !d || !bytes) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    return rg::workspace_size(p, *d, bytes);
    GUARD_END
}

rg_status rg_adjoint_workspace_size(rg_program *p, const rg_adjoint_desc *d, size_t *bytes) {
    if (!p || !d || !bytes) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    return rg::adjoint_workspace_size(p, *d, bytes);
    GUARD_END
}

rg_status rg_solve_k(rg_program *p, const rg_solve_desc *d, void *stream) {
    if (!p || !d) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    return rg::solve_k(p, *d, (hipStream_t)stream);
    GUARD_END
}

rg_status rg_eval_rays(rg_program *p, uint32_t n, const double *y, const double *omega,
                       const double *t, const double *const *params, double *f_out,
                       double *D_out, void *stream) {
    if (!p) return fail(RG_EINVAL, "NULL program");
    GUARD_BEGIN
    return rg::eval_points(p, n, y, omega, t, params, f_out, D_out, (hipStream_t)stream);
    GUARD_END
}

rg_status rg_last_launch(const rg_program *p, rg_launch_info *out) {
    if (!p || !out) return fail(RG_EINVAL, "NULL argument");
    *out = p->last;
    out->struct_size = sizeof(rg_launch_info);
    GUARD_BEGIN
    return rg::last_kernel_ms(p, &out->last_kernel_ms);
    GUARD_END
}

rg_status rg_trace_stats(rg_program *p, const rg_trace_desc *d, uint64_t *stats_dev, void *stream) {
    if (!p || !d) return fail(RG_EINVAL, "NULL argument");
    GUARD_BEGIN
    return rg::trace_stats(p, *d, stats_dev, (hipStream_t)stream);
    GUARD_END
}

}  // extern "C"
