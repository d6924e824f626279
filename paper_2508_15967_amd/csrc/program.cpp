// From a dispersion relation D to a gfx950 code object.
//
// Ray equations by implicit differentiation (paper, eqs. 2-3):
//   dx/dt = -(dD/dk) / (dD/domega),   dk/dt = (dD/dx) / (dD/domega)
// built with the graph's df, so reduction and hash-consing apply to the
// derivatives as they are built.  One reciprocal of dD/domega is shared by
// all 2*dim components.  For the adjoint the scalar s = sum_j v_j f_j(y) is
// built with seed variables v_j; df of s with respect to each state
// component, each parameter element and each spline node gives the
// vector-Jacobian products J^T v and (df/dtheta)^T v.
#include <hip/hiprtc.h>

#include <cmath>
#include <algorithm>
#include <cstdlib>

#include <chrono>
#include <cstdio>
#include <thread>
#include <mutex>
#include <map>
#include <fstream>
#include <cstring>
#include <sstream>

#include "emit.hpp"
#include "program.hpp"

#include "_embedded_kernels.inc"

namespace rg {

uint64_t fnv1a(const void *data, size_t n, uint64_t h) {
    const unsigned char *p = (const unsigned char *)data;
    for (size_t i = 0; i < n; i++) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

static std::string int_array(const char *name, const std::vector<int> &v) {
    std::ostringstream os;
    os << "__constant__ int " << name << "[" << (v.empty() ? 1 : v.size()) << "] = {";
    if (v.empty()) os << "0";
    for (size_t i = 0; i < v.size(); i++) os << (i ? ", " : "") << v[i];
    os << "};\n";
    return os.str();
}

// ------------------------------------------------------ code-object cache

static std::mutex g_cache_mu;
static std::map<uint64_t, std::vector<char>> g_code_cache;

static std::string cache_path(uint64_t key) {
    const char *dir = std::getenv("RAYGRAPH_CODE_CACHE");
    if (!dir || !*dir) return std::string();
    char name[40];
    std::snprintf(name, sizeof name, "/%016llx.co", (unsigned long long)key);
    return std::string(dir) + name;
}

static bool code_cache_get(uint64_t key, std::vector<char> *code) {
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto it = g_code_cache.find(key);
        if (it != g_code_cache.end()) {
            *code = it->second;
            return true;
        }
    }
    const std::string path = cache_path(key);
    if (path.empty()) return false;
    std::ifstream in(path, std::ios::binary);
    if (!in) return false;
    std::vector<char> buf((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
    if (buf.size() < 64) return false;  // not a code object
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_code_cache[key] = buf;
    *code = std::move(buf);
    return true;
}

static void code_cache_put(uint64_t key, const std::vector<char> &code) {
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_code_cache[key] = code;
    }
    const std::string path = cache_path(key);
    if (path.empty()) return;
    const std::string tmp = path + ".tmp" + std::to_string((unsigned long long)std::hash<std::thread::id>()(std::this_thread::get_id()));
    {
        std::ofstream out(tmp, std::ios::binary);
        if (!out) return;
        out.write(code.data(), (std::streamsize)code.size());
        if (!out) return;
    }
    std::rename(tmp.c_str(), path.c_str());  // atomic replace; a failure leaves no cache entry
}

// Products of every function are re-associated before emission (shared
// factor pairs formed once; see Graph::factor_products).  With `hoist`, the
// ray-invariant parts of denominators and products are also split off so
// that they are computed once per ray; each such value then stays live in
// registers across the time loop, which the rolled programs (register
// bound already) do not afford.
static void factor_spec(Graph &g, FunctionSpec &spec, bool hoist, const std::vector<int> &table_slot,
                        bool collect_ok) {
    // (the state components fixed along a ray are not used for factoring:
    // grouping products around them measured slower on the cold-plasma
    // medium, 558 against 498 VALU instructions per step, with more values
    // live across the loop; the emitter still counts their work as
    // ray-invariant, as the compiler hoists it)
    const uint32_t inv_state = 0;
    std::vector<uint32_t> roots;
    for (const Output &o : spec.outputs) roots.push_back(o.node);
    for (const SplineSeed &s : spec.spline_seeds) {
        roots.push_back(s.seed);
        roots.push_back(s.spline_node);
    }
    // the roots factored, with common factors taken out of sums in
    // `rounds` rounds (a second round finds the factors that the sharing of
    // scaled sums exposes: 2 x a + 2 y b -> 2 (x a + y b))
    auto factored = [&](int rounds) {
        std::vector<uint32_t> nr = g.hoist_divisions(roots, hoist, inv_state);
        for (int i = 0; i < std::max(rounds, 1); i++) {
            if (rounds > 0) nr = g.collect_factors(nr);
            nr = g.share_scaled_sums(g.factor_products(g.factor_sums(nr), hoist, inv_state));
        }
        FunctionSpec out = spec;
        size_t k = 0;
        for (Output &o : out.outputs) o.node = nr[k++];
        for (SplineSeed &s : out.spline_seeds) {
            s.seed = nr[k++];
            s.spline_node = nr[k++];
        }
        return out;
    };
    // Common factors are taken out of sums (Graph::collect_factors) only
    // where that lowers the emitted operations per evaluation (an fma
    // counting one; the ray-invariant ones only where they are not
    // hoisted), in one round or two.  It shares the directional
    // derivatives of the cold-plasma right-hand side and of the anisotropic
    // VJP.  Not for the right-hand sides of rolled programs (collect_ok
    // false): for the anisotropic medium two rounds save 15 of 491
    // operations but turn M_b k into nine sums over the blobs, and the
    // forward kernel then needs 204 VGPRs (two waves per SIMD) against 119.
    auto cost = [&](FunctionSpec s) {
        s.const_table = nullptr;  // counting only: leave the constant table alone
        Flops f;
        emit_function(g, s, table_slot, &f);
        return (long)f.ops - (hoist ? (long)f.inv_ops : 0L);
    };
    spec = factored(0);
    long best = cost(spec);
    for (int rounds = 1; rounds <= (collect_ok ? 2 : 0); rounds++) {
        FunctionSpec c = factored(rounds);
        const long k = cost(c);
        if (k < best) {
            best = k;
            spec = c;
        }
    }
}

rg_status build_program(Graph &g, uint32_t D, const rg_compile_opts &opts, rg_program *p) {
    auto t0 = std::chrono::steady_clock::now();
    const uint32_t d = g.dim(), ny = 2 * d;
    p->dim = d;
    p->n_params = (uint32_t)g.params().size();
    if (p->n_params > RG_KMAX_PARAMS) return fail(RG_EUNSUPPORTED, "at most 8 parameter arrays");
    for (const ParamDef &pd : g.params()) p->param_len.push_back(pd.len);
    p->has_vjp = opts.want_adjoint != 0;
    p->compile_only = opts.compile_only != 0;

    // ---- ray equations
    std::vector<uint32_t> yv(ny);
    for (uint32_t i = 0; i < d; i++) {
        yv[i] = g.var(VK_X, i);
        yv[d + i] = g.var(VK_K, i);
    }
    const uint32_t om = g.var(VK_OMEGA, 0);
    const uint32_t Dw = g.df(D, om);
    if (g.is_const(Dw, 0.0)) return fail(RG_EINVAL, "dD/domega is identically zero");
    const uint32_t inv = g.div(g.constant(1.0), Dw);
    // a partial of the form c*u is multiplied as (c*inv)*u, so the scaled
    // reciprocal c*inv is one shared node (e.g. dD/dk_i = 2 k_i for all i)
    auto times_inv = [&](uint32_t a) {
        const Node &na = g.node(a);
        if (na.op == MUL && g.is_const(na.a)) return g.mul(g.mul(na.a, inv), na.b);
        return g.mul(a, inv);
    };
    std::vector<uint32_t> f(ny);
    for (uint32_t i = 0; i < d; i++) {
        f[i] = g.neg(times_inv(g.df(D, yv[d + i])));
        f[d + i] = times_inv(g.df(D, yv[i]));
    }
    unsigned zero_mask = 0;  // components whose right-hand side is identically 0
    for (uint32_t i = 0; i < ny; i++)
        if (g.is_const(f[i], 0.0)) zero_mask |= 1u << i;
    // distinct constants of the right-hand side that are not inline operands
    // of FP64 instructions (0, +-0.5, +-1, +-2, +-4); each takes two scalar
    // registers where it is used
    uint32_t n_consts = 0;
    for (uint32_t n : g.reachable(f)) {
        const Node &nd = g.node(n);
        if (nd.op != CONST) continue;
        const double v = std::fabs(nd.val);
        if (v == 0.0 || v == 0.5 || v == 1.0 || v == 2.0 || v == 4.0) continue;
        n_consts++;
    }

    // ---- spline tables used by the program
    std::vector<uint32_t> roots(f.begin(), f.end());
    roots.push_back(D);
    std::vector<int> table_slot(p->n_params, -1);
    for (uint32_t n : g.reachable(roots)) {
        const Node &nd = g.node(n);
        if (nd.op != SPLINE) continue;
        const SplineDef &s = g.splines()[(size_t)nd.val];
        if (table_slot[s.param] >= 0) continue;
        if (g.params()[s.param].len < s.nx * s.ny)
            return fail(RG_EINVAL, "spline parameter shorter than nx*ny");
        table_slot[s.param] = (int)p->spl_param.size();
        p->spl_param.push_back((int)s.param);
        p->spl_off.push_back(p->spl_total);
        p->spl_len.push_back((int)(s.nx * s.ny));
        p->spl_ny.push_back((int)s.ny);
        p->spl_total += (int)(s.nx * s.ny);
    }
    if (p->spl_total > 8192)
        return fail(RG_EUNSUPPORTED, "spline tables larger than 8192 coefficients (LDS staging)");
    // Rolled stage loops (one copy of the right-hand side per kernel loop)
    // for right-hand sides with many constants, unless large spline tables
    // already fill LDS.
    p->rolled = n_consts > 32 && p->spl_total <= 4096;

    // ---- emit rhs and D
    std::ostringstream fs;
    // Rolled programs read their FP64 constants from one table through the
    // scalar cache: a wide load brings several constants where each literal
    // costs two scalar moves per use (about a third of the instructions of
    // a rolled RK4 stage).  Every FP64 function takes a template flag
    // RG_KL that turns the table reads back into literals (the
    // Dormand-Prince attempt, whose seven inlined right-hand sides keep
    // literals in scalar registers across stages).
    std::vector<double> ktab;
    std::vector<double> *kt = p->rolled ? &ktab : nullptr;
    Flops fl_rhs, fl_rhs_dp, fl_D, fl_vjp, fl_rhs_vjp;
    {
        FunctionSpec spec;
        spec.const_table = kt;
        spec.signature =
            "template <bool RG_KL = false>\n"
            "RG_FN void rg_rhs(const double *__restrict__ y, const double om, const double t, "
            "const rg_P &P, double *__restrict__ f) {\n  (void)om; (void)t; (void)P;";
        for (uint32_t i = 0; i < ny; i++) spec.outputs.push_back({f[i], "f[" + std::to_string(i) + "]", false});
        // the integrators keep components with a zero right-hand side fixed,
        // so what depends only on them and on omega is invariant along a ray
        spec.inv_state = zero_mask;
        factor_spec(g, spec, !p->rolled, table_slot, !p->rolled);
        fs << emit_function(g, spec, table_slot, &fl_rhs);
        // the Dormand-Prince attempt updates every component: counted with
        // only omega, parameters and constants as invariant
        spec.inv_state = 0;
        emit_function(g, spec, table_slot, &fl_rhs_dp);
    }
    if (opts.fp32) {
        // the same right-hand side in single precision (an overload of rg_rhs)
        for (uint32_t n : g.reachable(f))
            if (g.node(n).op == SPLINE)
                return fail(RG_EUNSUPPORTED, "single precision right-hand side with spline nodes");
        FunctionSpec spec;
        spec.const_table = kt;
        spec.fp32 = true;
        spec.signature =
            "RG_FN void rg_rhs(const float *__restrict__ y, const float om, const float t, "
            "const rg_P &P, float *__restrict__ f) {\n  (void)om; (void)t; (void)P;";
        for (uint32_t i = 0; i < ny; i++) spec.outputs.push_back({f[i], "f[" + std::to_string(i) + "]", false});
        spec.inv_state = zero_mask;
        Flops fl32;
        factor_spec(g, spec, !p->rolled, table_slot, !p->rolled);
        fs << emit_function(g, spec, table_slot, &fl32);
        p->has_f32 = true;
    }
    {
        FunctionSpec spec;
        spec.const_table = kt;
        spec.signature =
            "template <bool RG_KL = false>\n"
            "RG_FN double rg_D(const double *__restrict__ y, const double om, const double t, "
            "const rg_P &P) {\n  (void)om; (void)t; (void)P; (void)y;";
        spec.outputs.push_back({D, "", false});
        spec.returns_value = true;
        factor_spec(g, spec, !p->rolled, table_slot, !p->rolled);
        fs << emit_function(g, spec, table_slot, &fl_D);
    }
    {
        // D and dD/dk (Newton solve for launch conditions)
        FunctionSpec spec;
        spec.const_table = kt;
        spec.signature =
            "template <bool RG_KL = false>\n"
            "RG_FN void rg_Dk(const double *__restrict__ y, const double om, const double t, "
            "const rg_P &P, double *__restrict__ out) {\n  (void)om; (void)t; (void)P; (void)y;";
        spec.outputs.push_back({D, "out[0]", false});
        for (uint32_t i = 0; i < d; i++)
            spec.outputs.push_back({g.df(D, yv[d + i]), "out[" + std::to_string(i + 1) + "]", false});
        Flops fl_dk;
        factor_spec(g, spec, !p->rolled, table_slot, !p->rolled);
        fs << emit_function(g, spec, table_slot, &fl_dk);
    }
    p->info.n_nodes_rhs = fl_rhs.ops;

    // ---- emit the VJP
    if (p->has_vjp) {
        // reverse mode: adjoints of s = sum_j v_j f_j with respect to the
        // state, the parameter elements and the spline nodes
        std::vector<uint32_t> seeds(ny);
        for (uint32_t j = 0; j < ny; j++) seeds[j] = g.var(VK_SEED, j);
        const std::vector<uint32_t> adj = g.adjoints(f, seeds);
        auto A = [&](uint32_t n) { return adj[n] == NONE ? g.constant(0.0) : adj[n]; };
        FunctionSpec spec;
        spec.const_table = kt;
        spec.signature =
            "template <typename GPT, bool RG_KL = false>\nRG_FN void rg_vjp(const double *__restrict__ y, const double om, const double t, "
            "const rg_P &P, const double *__restrict__ av, double *__restrict__ jv, "
            "GPT gp, rg_GA &G) {\n  (void)om; (void)t; (void)P; (void)gp; (void)G;";
        for (uint32_t j = 0; j < ny; j++) spec.outputs.push_back({A(yv[j]), "jv[" + std::to_string(j) + "]", false});
        std::vector<uint32_t> freach = g.reachable(f);
        for (uint32_t n : freach) {
            const Node &nd = g.node(n);
            if (nd.op == PARAM) {
                int slot = (int)p->grad_param.size();
                p->grad_param.push_back(nd.aux);
                p->grad_elem.push_back((int)nd.val);
                spec.outputs.push_back({A(n), "gp[" + std::to_string(slot) + "]", true});
            }
        }
        for (uint32_t n : freach) {
            const Node &nd = g.node(n);
            if (nd.op == SPLINE) spec.spline_seeds.push_back({n, A(n)});
        }
        // (for the flop count only) the VJP and the right-hand side at the
        // same state as one function: the work the two share counts once
        FunctionSpec both = spec;
        for (uint32_t i = 0; i < ny; i++) both.outputs.push_back({f[i], "f[" + std::to_string(i) + "]", false});
        factor_spec(g, spec, !p->rolled, table_slot, true);
        fs << emit_function(g, spec, table_slot, &fl_vjp);
        p->info.n_nodes_vjp = fl_vjp.ops;
        factor_spec(g, both, !p->rolled, table_slot, true);
        emit_function(g, both, table_slot, &fl_rhs_vjp);
    }
    if (!ktab.empty()) {
        std::ostringstream kd;
        kd << "RG_KTAB double rg_ktab[" << ktab.size() << "] = {";
        for (size_t i = 0; i < ktab.size(); i++) kd << (i ? ", " : "") << hex_double(ktab[i]);
        kd << "};\n";
        p->functions_src = kd.str() + fs.str();
    } else {
        p->functions_src = fs.str();
    }
    // The adjoint recomputes the stage states Y2..Y4 where three right-hand
    // sides cost less than waiting for them from the segment buffer (a few
    // hundred issued flops against a global-memory latency the few waves of
    // a small ray batch cannot hide); otherwise they are stored.
    p->adj_recompute = fl_rhs.issued + fl_rhs.inv_issued < 400.0;
    // Four rays per lane only for cheap right-hand sides (four copies of the
    // state and stages must stay in registers).
    p->has_r4 = !p->rolled && fl_rhs.issued < 200.0;
    // With stored stage states the reverse step is a loop around one large
    // VJP whose registers decide the waves per SIMD: there the per-lane
    // gradient partials of scalar parameters are accumulated in LDS instead
    // of registers (one LDS add each per VJP) and the kernel is bounded to
    // 168 registers (three waves per SIMD), where that LDS and the tables'
    // still leave room for three workgroups per CU.
    {
        const size_t ngrad1 = p->grad_param.empty() ? 1 : p->grad_param.size();
        const size_t lds = ngrad1 * kAdjointBlock * 8 + (size_t)p->spl_total * 16 + 2048 + 8 * ngrad1 * 8;
        p->gp_lds = p->has_vjp && !p->adj_recompute && lds <= 53248;
    }
    // deterministic spline-coefficient gradients: asked for, and there are
    // spline tables whose gradients would otherwise go through shared atomics
    p->det_grad = opts.deterministic && p->has_vjp && p->spl_total > 0;
    {
    }

    // ---- configuration header
    std::ostringstream cs;
    cs << "#pragma once\n#define RG_DIM " << d << "\n#define RG_NY " << ny << "\n#define RG_NPARAM "
       << p->n_params << "\n#define RG_NGRAD " << p->grad_param.size() << "\n#define RG_NSPLTAB "
       << p->spl_param.size() << "\n#define RG_SPL_TOTAL " << (p->spl_total ? p->spl_total : 1)
       << "\n#define RG_HAS_VJP " << (p->has_vjp ? 1 : 0) << "\n#define RG_HAS_F32 " << (p->has_f32 ? 1 : 0)
       << "\n#define RG_HAS_R4 " << (p->has_r4 ? 1 : 0)
       << "\n#define RG_USES_EXP " << (p->functions_src.find("rg_exp") != std::string::npos ? 1 : 0)
       << "\n#define RG_RHS_ZERO " << zero_mask
       << "u\n#define RG_ROLL " << (p->rolled ? 1 : 0) << "\n#define RG_ADJ_RECOMPUTE "
       << (p->adj_recompute ? 1 : 0) << "\n#define RG_GP_LDS " << (p->gp_lds ? 1 : 0)
       << "\n#define RG_DET_GRAD " << (p->det_grad ? 1 : 0)
       << "\n#define RG_ADJ_BLOCK " << kAdjointBlock << "\n";
    cs << int_array("rg_spl_param", p->spl_param) << int_array("rg_spl_off", p->spl_off)
       << int_array("rg_spl_len", p->spl_len) << int_array("rg_spl_ny", p->spl_ny)
       << int_array("rg_grad_param", p->grad_param) << int_array("rg_grad_elem", p->grad_elem);
    p->config_src = cs.str();

    // ---- flop accounting
    rg_program_info &I = p->info;
    I.struct_size = sizeof(rg_program_info);
    I.dim = d;
    I.n_params = p->n_params;
    I.n_grad_slots = (uint32_t)p->grad_param.size();
    I.rhs_flops_alg = fl_rhs.alg;
    I.rhs_flops_issued = fl_rhs.issued;
    I.rhs_flops_ray_invariant = fl_rhs.inv_alg;
    // RK4 update: per component 3 stage fma + fma, fma, add + final fma = 13
    // flops, plus t += dt (the two step constants are computed once per
    // launch).  Components whose right-hand side is identically zero keep
    // their value and cost nothing (rg_rk4_step skips them).
    const double upd = 13.0 * (ny - __builtin_popcount(zero_mask)) + 1.0;
    I.rk4_step_flops_alg = 4 * fl_rhs.alg + upd;
    I.rk4_step_flops_issued = 4 * fl_rhs.issued + upd;
    // DOPRI attempt: 6 new right-hand sides; stage sums 2s+1 flops per
    // component for s = 1..6 (48), error estimate 11 + scale 2 + div 1 +
    // square-accumulate 2 (16), plus sqrt, mean and the step factor.
    const double dp = 64.0 * ny + 8.0;
    const IssuedWeights &w = issued_weights();
    I.dopri_attempt_flops_alg = 6 * fl_rhs_dp.alg + dp;
    // (sqrt and the division by the scale per component counted at their
    // issued weights; the step factor is a single-precision estimate and two
    // exact tests of five FP64 multiplications each: 10)
    I.dopri_attempt_flops_issued = 6 * fl_rhs_dp.issued + dp - 3.0 - ny + w.sqrt + ny * w.div + 10.0;
    if (p->has_vjp) {
        I.vjp_flops_alg = fl_vjp.alg;
        I.vjp_flops_issued = fl_vjp.issued;
        I.vjp_flops_ray_invariant = fl_vjp.inv_alg;
        // reverse of one step: recompute (one RK4 step) [+ 3 stage RHS and
        // 3 stage fma when the stages are recomputed] + 4 VJP + recurrence
        // (per component: 3 fma, 3 add, 1 mul, 1 add = 12 flops).  Three of
        // the four VJPs run at states whose right-hand side the step
        // evaluates: the algorithmic count takes what the two share once,
        // the issued count all of it, since the kernel recomputes the shared
        // part inside the VJP rather than keep it live across the stages.
        const double rec = 12.0 * ny;
        const double st_alg = p->adj_recompute ? 3 * (fl_rhs_vjp.alg - fl_vjp.alg) + 6.0 * ny : 0.0;
        const double st_iss = p->adj_recompute ? 3 * fl_rhs.issued + 6.0 * ny : 0.0;
        I.adj_step_flops_alg = I.rk4_step_flops_alg + st_alg + 4 * fl_vjp.alg + rec;
        I.adj_step_flops_issued = I.rk4_step_flops_issued + st_iss + 4 * fl_vjp.issued + rec;
    }

    // ---- full source: one self-contained translation unit (headers spliced
    // in), compilable by hipRTC or by hipcc
    auto splice = [&](std::string text) {
        const std::pair<const char *, std::string> inc[] = {
            {"#include \"rg_kargs.h\"", RG_SRC_KARGS},
            {"#include \"rg_config.h\"", p->config_src},
            {"#include \"rg_prelude.h\"", RG_SRC_PRELUDE},
            {"#include \"rg_functions.h\"", p->functions_src}};
        for (const auto &kv : inc) {
            size_t pos = text.find(kv.first);
            if (pos != std::string::npos) text.replace(pos, std::strlen(kv.first), kv.second);
        }
        return text;
    };
    p->full_src = std::string("// generated by raygraph\n#ifndef __HIPCC_RTC__\n#include <hip/hip_runtime.h>\n#endif\n") +
                  splice(RG_SRC_KERNELS);
    p->hash = fnv1a(p->full_src.data(), p->full_src.size());
    I.source_hash = p->hash;

    const char *arch = opts.arch ? opts.arch : "gfx950";
    std::string arch_opt = std::string("--offload-arch=") + arch;
    int olvl = opts.opt_level > 0 ? opts.opt_level : 3;
    std::string o_opt = "-O" + std::to_string(olvl);
    // no FP contraction beyond the fma written in the source; no packed FP32
    // With rolled stage loops, machine-level loop-invariant code motion is
    // off: it would hoist every constant's scalar-register materialization
    // out of the stage loop and so keep them all live again.
    const char *copts[] = {arch_opt.c_str(), o_opt.c_str(), "-ffp-contract=off", "-std=c++17",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-mllvm", "-disable-machine-licm"};
    const int ncopts = p->rolled ? 10 : 8;
    // code objects are cached by source and options (in the process, and in
    // the directory RAYGRAPH_CODE_CACHE if set)
    int rtc_major = 0, rtc_minor = 0;
    hiprtcVersion(&rtc_major, &rtc_minor);
    std::string key_text = p->full_src;
    for (int i = 0; i < ncopts; i++) key_text += std::string("\n") + copts[i];
    key_text += "\nhiprtc " + std::to_string(rtc_major) + "." + std::to_string(rtc_minor);
    const uint64_t key = fnv1a(key_text.data(), key_text.size());
    if (code_cache_get(key, &p->code)) {
        I.compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return RG_OK;
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, p->full_src.c_str(), "raygraph_kernels.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return fail(RG_ECOMPILE, "hiprtcCreateProgram failed");
    hiprtcResult rc = hiprtcCompileProgram(prog, ncopts, copts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(RG_ECOMPILE, std::string("hipRTC: ") + hiprtcGetErrorString(rc) + "\n" + log);
    }
    size_t cs_ = 0;
    hiprtcGetCodeSize(prog, &cs_);
    p->code.resize(cs_);
    hiprtcGetCode(prog, p->code.data());
    hiprtcDestroyProgram(&prog);
    code_cache_put(key, p->code);
    I.compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return RG_OK;
}

}  // namespace rg
