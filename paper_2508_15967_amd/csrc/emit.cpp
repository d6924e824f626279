// Straight-line HIP emission from the expression graph (see emit.hpp).
#include "emit.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <sstream>
#include <stdexcept>

namespace rg {

const IssuedWeights &issued_weights() {
    // FP64 flops in the gfx950 instruction sequence of each operation,
    // counted in the AMD assembly of single-operation kernels compiled here
    // (hipcc --offload-arch=gfx950 -O3 -ffp-contract=off): v_fma_f64 and
    // v_div_fmas_f64 = 2; v_add_f64, v_mul_f64, v_rcp_f64, v_rsq_f64 = 1;
    // compares, class tests, ldexp/frexp, rounding, conversions and selects = 0.
    //   exp (rg_exp, table-driven): 6 fma + 2 mul = 14
    //   div: 5 fma + div_fmas + mul + rcp = 14
    //   sqrt: 7 fma + 2 mul + rsq         = 17
    //   log: 14 fma + 43 add + 7 mul + rcp = 79
    //   sin/cos: 24 fma + 56 add + 11 mul = 115
    //   rg_rcp (reciprocal, rcp + two Newton steps): rcp + 4 fma = 9
    static const IssuedWeights w{/*div*/ 14.0, /*exp*/ 14.0, /*log*/ 79.0, /*sqrt*/ 17.0,
                                 /*sincos*/ 115.0, /*rcp*/ 9.0};
    return w;
}

std::string hex_double(double v) {
    char buf[64];
    if (std::isnan(v)) return "(__builtin_nan(\"\"))";
    if (std::isinf(v)) return v > 0 ? "(__builtin_inf())" : "(-__builtin_inf())";
    std::snprintf(buf, sizeof buf, "(%a)", v);
    return buf;
}

// A float literal holding v rounded to single precision.
static std::string hex_float(double v) {
    const float f = (float)v;
    char buf[64];
    if (std::isnan(f)) return "(__builtin_nanf(\"\"))";
    if (std::isinf(f)) return f > 0 ? "(__builtin_inff())" : "(-__builtin_inff())";
    std::snprintf(buf, sizeof buf, "(%af)", (double)f);
    return buf;
}

namespace {

struct Emitter {
    const Graph &g;
    const std::vector<int> &table_slot;
    std::ostringstream os;
    Flops fl;
    std::vector<uint32_t> uses;
    std::vector<char> fused;   // MUL folded into a consuming fma
    std::vector<char> emitted;
    std::map<uint32_t, int> group_of;  // spline node -> group index
    struct Group {
        uint32_t def, u, v;
        std::vector<uint32_t> nodes;
        int maxdu = 0, maxdv = 0;
        bool emitted = false;
        int rows_done = 0;  // bit dv: row sums for order dv in v emitted
    };
    std::vector<Group> groups;
    // Chains of single-use additions/subtractions become accumulations whose
    // terms may be added in any order (see schedule()).
    struct Chain {
        uint32_t root;
        std::vector<std::pair<uint32_t, int>> leaves;  // term node, sign
        bool started = false;
        bool acc_inv = true;  // every term accumulated so far is ray-invariant
    };
    std::vector<Chain> chains;
    std::vector<int> chain_of_root;  // node -> chain index or -1
    std::vector<char> interior;      // node folded into a chain
    std::vector<uint32_t> consumer;  // unique consumer of a single-use node
    bool f32 = false;                // emit single precision (float) code
    std::vector<signed char> sgn;    // 1: value >= 0, -1: <= 0 (or NaN), 0: not known
    // Finite-input analysis (inputs: state, omega, t, parameters): fin, the
    // value is finite whenever the inputs are (no overflow possible); nnan,
    // it is not NaN whenever the inputs are finite.
    std::vector<char> fin, nnan;
    std::vector<char> inv;           // value depends only on constants, parameters, omega
    uint32_t inv_state = 0;          // and these state components (constant along a ray)
    bool cur_inv = false;            // the operation being counted is ray-invariant

    const char *T() const { return f32 ? "float" : "double"; }
    std::vector<double> *ktab = nullptr;  // FunctionSpec::const_table
    // Inline FP64 operands of gfx9 instructions: 0, +-0.5, +-1, +-2, +-4
    // and the integers -16..64 (1/(2 pi) is one too but never a graph constant).
    static bool inline_f64(double v) {
        if (v == 0.5 || v == -0.5 || v == 2.0 || v == -2.0 || v == 4.0 || v == -4.0) return true;
        return v == std::floor(v) && v >= -16.0 && v <= 64.0;
    }
    std::string lit(double v) const {
        if (f32) return hex_float(v);
        if (!ktab || !std::isfinite(v) || inline_f64(v)) return hex_double(v);
        size_t i = 0;
        for (; i < ktab->size(); i++)
            if (std::memcmp(&(*ktab)[i], &v, sizeof v) == 0) break;
        if (i == ktab->size()) ktab->push_back(v);
        return "RG_KV(" + std::to_string(i) + ", " + hex_double(v) + ")";
    }
    std::string fn(const char *base) const { return f32 ? std::string(base) + "f" : std::string(base); }

    Emitter(const Graph &g_, const std::vector<int> &ts) : g(g_), table_slot(ts) {
        uses.assign(g.size(), 0);
        fused.assign(g.size(), 0);
        emitted.assign(g.size(), 0);
        chain_of_root.assign(g.size(), -1);
        interior.assign(g.size(), 0);
        consumer.assign(g.size(), NONE);
    }

    std::string name(uint32_t n) const {
        const Node &nd = g.node(n);
        if (nd.op == CONST) return lit(nd.val);
        if (nd.op == VAR) {
            int kind = nd.aux / 8, i = nd.aux % 8;
            uint32_t d = g.dim();
            switch (kind) {
            case VK_X: return "y[" + std::to_string(i) + "]";
            case VK_K: return "y[" + std::to_string(d + i) + "]";
            case VK_OMEGA: return "om";
            case VK_T: return "t";
            default: return "av[" + std::to_string(i) + "]";
            }
        }
        return "v" + std::to_string(n);
    }

    // Counted into the ray-invariant part while cur_inv is set.
    void tally(double alg, double iss) {
        if (cur_inv) { fl.inv_alg += alg; fl.inv_issued += iss; }
        else { fl.alg += alg; fl.issued += iss; }
    }
    void count(int op, int aux = 0) {
        const IssuedWeights &w = issued_weights();
        fl.ops++;
        if (cur_inv && op != NEG) fl.inv_ops++;
        switch (op) {
        case ADD: case SUB: case MUL: tally(1, 1); break;
        case DIV: tally(1, w.div); break;
        case EXP: tally(1, w.exp); break;
        case LOG: tally(1, w.log); break;
        case SQRT: tally(1, w.sqrt); break;
        case SIN: case COS: tally(1, w.sincos); break;
        case POWI: {
            int n = aux < 0 ? -aux : aux;
            tally(n - 1, n - 1);
            if (aux < 0) tally(1, w.div);
            break;
        }
        case NEG: fl.ops--; break;
        default: break;
        }
    }
    void count_fma(int n = 1) {
        tally(2 * n, 2 * n);
        fl.ops += n;
        if (cur_inv) fl.inv_ops += n;
    }
    void count_plain(double f) { tally(f, f); }

    bool fusable_mul(uint32_t m) const {
        const Node &nd = g.node(m);
        return nd.op == MUL && uses[m] == 1;
    }

    void plan(const std::vector<uint32_t> &order, const std::vector<uint32_t> &roots) {
        // signs the graph fixes (rounding keeps the sign of each of these
        // operations; NaN may appear wherever a sign is claimed).  A zero
        // counts as either sign, but a zero of the other sign in a divisor
        // flips the sign of the quotient (1/-0 = -inf, and sqrt(-0) = -0),
        // so a quotient's sign is claimed only when its divisor cannot be
        // a zero of the wrong sign: an exponential, an even power, a square
        // or a nonzero constant.
        sgn.assign(g.size(), 0);
        auto zero_safe = [&](uint32_t m) {
            const Node &d = g.node(m);
            return d.op == EXP || (d.op == CONST && d.val != 0.0) ||
                   (d.op == POWI && d.aux % 2 == 0) || (d.op == MUL && d.a == d.b);
        };
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            auto S = [&](uint32_t m) { return m == NONE ? 0 : (int)sgn[m]; };
            int s = 0;
            switch (nd.op) {
            case CONST: s = nd.val >= 0.0 ? 1 : nd.val <= 0.0 ? -1 : 0; break;
            case EXP: case SQRT: s = 1; break;
            case NEG: s = -S(nd.a); break;
            case POWI:
                s = nd.aux % 2 == 0 ? 1 : (nd.aux > 0 || zero_safe(nd.a)) ? S(nd.a) : 0;
                break;
            case MUL: s = nd.a == nd.b ? 1 : S(nd.a) * S(nd.b); break;
            case DIV: s = zero_safe(nd.b) ? S(nd.a) * S(nd.b) : 0; break;
            case ADD: s = S(nd.a) == S(nd.b) ? S(nd.a) : 0; break;
            case SUB: s = S(nd.a) == -S(nd.b) ? S(nd.a) : 0; break;
            default: break;
            }
            sgn[n] = (signed char)s;
        }
        // NaN arises only from inf - inf, 0 * inf, 0 / 0, inf / inf, the
        // square root or logarithm of a negative number, or the sine or
        // cosine of an infinity; overflow only from operations that can
        // grow a finite value.  The rules below claim a property only where
        // none of these can happen; everything else is left unclaimed.
        fin.assign(g.size(), 0);
        nnan.assign(g.size(), 0);
        auto is_const = [&](uint32_t m) { return m != NONE && g.node(m).op == CONST; };
        auto cval = [&](uint32_t m) { return g.node(m).val; };
        auto nz_const = [&](uint32_t m) { return is_const(m) && cval(m) != 0.0 && std::isfinite(cval(m)); };
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            auto S = [&](uint32_t m) { return m == NONE ? 0 : (int)sgn[m]; };
            const bool fa = nd.a != NONE && fin[nd.a], fb = nd.b != NONE && fin[nd.b];
            const bool na = nd.a != NONE && nnan[nd.a], nb = nd.b != NONE && nnan[nd.b];
            bool F = false, N = false;
            switch (nd.op) {
            case CONST: F = N = std::isfinite(nd.val); break;
            case VAR: case PARAM: F = N = true; break;
            case NEG: F = fa; N = na; break;
            case ADD: case SUB: {
                // infinities of one direction add without NaN: operands of
                // one proven sign (ADD), of opposite signs (SUB)
                const int sa = S(nd.a), sb = S(nd.b);
                const bool one_dir = sa != 0 && (nd.op == ADD ? sa == sb : sa == -sb);
                N = na && nb && (fa || fb || one_dir);
                // a finite value plus a constant below half an ulp of the
                // largest double rounds to at most that double
                auto small = [&](uint32_t m) { return is_const(m) && std::fabs(cval(m)) <= 0x1p969; };
                F = (fa && small(nd.b)) || (fb && small(nd.a));
                break;
            }
            case MUL:
                // finite * finite may overflow but is not NaN; a nonzero
                // constant times an infinity is an infinity; x * x >= 0
                N = na && nb && ((fa && fb) || nz_const(nd.a) || nz_const(nd.b) || nd.a == nd.b);
                F = (fa && is_const(nd.b) && std::fabs(cval(nd.b)) <= 1.0) ||
                    (fb && is_const(nd.a) && std::fabs(cval(nd.a)) <= 1.0);
                break;
            case DIV:
                // c / x (x = 0: inf, x = inf: 0) and x / c, c a nonzero constant
                N = (nz_const(nd.a) && nb) || (nz_const(nd.b) && na);
                F = fa && nz_const(nd.b) && std::fabs(cval(nd.b)) >= 1.0;
                break;
            case EXP: N = na; F = na && S(nd.a) < 0; break;
            case SQRT: N = na && S(nd.a) > 0; F = N && fa; break;
            case LOG: N = na && S(nd.a) > 0; break;
            case SIN: case COS: F = N = fa; break;
            case POWI: N = na; break;  // x^k, 1/x^k: 0 and inf give 0 or inf
            default: break;            // spline nodes: not claimed
            }
            fin[n] = F;
            nnan[n] = N;
        }
        inv.assign(g.size(), 0);
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            if (nd.op == CONST || nd.op == PARAM) inv[n] = 1;
            else if (nd.op == VAR) inv[n] = g.ray_invariant_var(nd, inv_state);
            else inv[n] = (nd.a == NONE || inv[nd.a]) && (nd.b == NONE || inv[nd.b]);
        }
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            if (nd.a != NONE) uses[nd.a]++;
            if (nd.b != NONE) uses[nd.b]++;
        }
        std::vector<char> is_root(g.size(), 0);
        for (uint32_t r : roots) {
            uses[r]++;
            is_root[r] = 1;
        }
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            if (nd.a != NONE && uses[nd.a] == 1) consumer[nd.a] = n;
            if (nd.b != NONE && uses[nd.b] == 1) consumer[nd.b] = n;
        }
        auto addsub = [&](uint32_t n) { return g.node(n).op == ADD || g.node(n).op == SUB; };
        for (uint32_t n : order)
            if (addsub(n) && uses[n] == 1 && !is_root[n] && consumer[n] != NONE && addsub(consumer[n]))
                interior[n] = 1;
        // chain roots: additions with at least one interior operand
        for (uint32_t n : order) {
            if (!addsub(n) || interior[n]) continue;
            const Node &nd = g.node(n);
            if (!interior[nd.a] && !interior[nd.b]) {
                // plain two-operand addition: fuse one single-use product
                if (fusable_mul(nd.a)) fused[nd.a] = 1;
                else if (fusable_mul(nd.b)) fused[nd.b] = 1;
                continue;
            }
            Chain c;
            c.root = n;
            std::vector<std::pair<uint32_t, int>> stack{{n, 1}};
            while (!stack.empty()) {
                auto [m, sg] = stack.back();
                stack.pop_back();
                const Node &md = g.node(m);
                auto push = [&](uint32_t o, int so) {
                    if (interior[o]) stack.push_back({o, so});
                    else c.leaves.push_back({o, so});
                };
                // right operand first so that leaves come out in left-to-right order
                push(md.b, md.op == SUB ? -sg : sg);
                push(md.a, sg);
            }
            for (auto &lf : c.leaves)
                if (fusable_mul(lf.first)) fused[lf.first] = 1;
            chain_of_root[n] = (int)chains.size();
            chains.push_back(std::move(c));
        }
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            if (nd.op == SPLINE) {
                uint32_t def = (uint32_t)nd.val;
                int gi = -1;
                for (size_t i = 0; i < groups.size(); i++)
                    if (groups[i].def == def && groups[i].u == nd.a && groups[i].v == nd.b) gi = (int)i;
                if (gi < 0) {
                    groups.push_back(Group{def, nd.a, nd.b, {}, 0, 0, false, 0});
                    gi = (int)groups.size() - 1;
                }
                groups[gi].nodes.push_back(n);
                groups[gi].maxdu = std::max(groups[gi].maxdu, nd.aux / 4);
                groups[gi].maxdv = std::max(groups[gi].maxdv, nd.aux % 4);
                group_of[n] = gi;
            }
        }
    }

    void emit_group_head(int gi) {
        Group &gr = groups[gi];
        if (gr.emitted) return;
        gr.emitted = true;
        const SplineDef &s = g.splines()[gr.def];
        std::string G = "s" + std::to_string(gi);
        double ihx = (double)(s.nx - 3) / (s.hi[0] - s.lo[0]);
        double ihy = (double)(s.ny - 3) / (s.hi[1] - s.lo[1]);
        os << "  int " << G << "x, " << G << "y; double " << G << "u, " << G << "v;\n";
        os << "  rg_bs_cell(" << name(gr.u) << ", " << hex_double(s.lo[0]) << ", " << hex_double(ihx)
           << ", " << s.nx << ", " << G << "x, " << G << "u);\n";
        os << "  rg_bs_cell(" << name(gr.v) << ", " << hex_double(s.lo[1]) << ", " << hex_double(ihy)
           << ", " << s.ny << ", " << G << "y, " << G << "v);\n";
        count_plain(8);
        static const double wf[4] = {17, 11, 5, 0};
        for (int o = 0; o <= gr.maxdu; o++) {
            os << "  double " << G << "wx" << o << "[4]; rg_bs_w" << o << "(" << G << "u, " << G << "wx" << o << ");\n";
            count_plain(wf[o]);
        }
        for (int o = 0; o <= gr.maxdv; o++) {
            os << "  double " << G << "wy" << o << "[4]; rg_bs_w" << o << "(" << G << "v, " << G << "wy" << o << ");\n";
            count_plain(wf[o]);
        }
        int slot = table_slot.at(s.param);
        os << "  const double *" << G << "p = RG_SPL_TAB(" << slot << ") + (" << G << "x - 1) * "
           << s.ny << " + (" << G << "y - 1);\n";
        os << "  double " << G << "c[16];\n";
        os << "  for (int a_ = 0; a_ < 4; a_++) for (int b_ = 0; b_ < 4; b_++) " << G
           << "c[4 * a_ + b_] = " << G << "p[a_ * " << s.ny << " + b_];\n";
    }

    std::string spline_scale(uint32_t n) const {
        const Node &nd = g.node(n);
        const SplineDef &s = g.splines()[(size_t)nd.val];
        double ihx = (double)(s.nx - 3) / (s.hi[0] - s.lo[0]);
        double ihy = (double)(s.ny - 3) / (s.hi[1] - s.lo[1]);
        double sc = 1.0;
        for (int i = 0; i < nd.aux / 4; i++) sc *= ihx;
        for (int i = 0; i < nd.aux % 4; i++) sc *= ihy;
        return sc == 1.0 ? "" : hex_double(sc);
    }

    void emit_node(uint32_t n) {
        const Node &nd = g.node(n);
        if (emitted[n]) return;
        emitted[n] = 1;
        cur_inv = inv[n];
        switch (nd.op) {
        case CONST: case VAR:
            return;
        case PARAM:
            os << "  const " << T() << " " << name(n) << " = " << (f32 ? "(float)" : "") << "P.p[" << nd.aux
               << "][" << (size_t)nd.val << "];\n";
            return;
        case SPLINE: {
            int gi = group_of.at(n);
            emit_group_head(gi);
            std::string G = "s" + std::to_string(gi);
            const int dv = nd.aux % 4;
            if (!(groups[gi].rows_done & (1 << dv))) {
                // row sums for this order in v, shared by the group's nodes
                groups[gi].rows_done |= 1 << dv;
                os << "  double " << G << "q" << dv << "[4]; rg_bs_rows(" << G << "c, " << G << "wy" << dv << ", "
                   << G << "q" << dv << ");\n";
                count_plain(28);
            }
            std::string sc = spline_scale(n);
            os << "  const double " << name(n) << " = " << (sc.empty() ? "" : sc + " * ") << "rg_bs_comb(" << G << "q"
               << dv << ", " << G << "wx" << nd.aux / 4 << ");\n";
            count_plain(7 + (sc.empty() ? 0 : 1));
            return;
        }
        default: break;
        }
        if (fused[n] || interior[n] || chain_of_root[n] >= 0) return;  // emitted elsewhere
        std::string A = nd.a != NONE ? name(nd.a) : "", B = nd.b != NONE ? name(nd.b) : "";
        std::string e;
        switch (nd.op) {
        case ADD: case SUB: {
            bool fa = fused[nd.a] && g.node(nd.a).op == MUL;
            bool fb = !fa && fused[nd.b] && g.node(nd.b).op == MUL;
            if (fa) {
                const Node &m = g.node(nd.a);
                e = fn("fma") + "(" + name(m.a) + ", " + name(m.b) + ", " + (nd.op == SUB ? "-" : "") + B + ")";
                count_fma();
            } else if (fb) {
                const Node &m = g.node(nd.b);
                e = fn("fma") + "(" + std::string(nd.op == SUB ? "-" : "") + name(m.a) + ", " + name(m.b) + ", " + A + ")";
                count_fma();
            } else {
                e = A + (nd.op == ADD ? " + " : " - ") + B;
                count(nd.op);
            }
            break;
        }
        case MUL: e = A + " * " + B; count(MUL); break;
        case DIV:
            if (g.is_const(nd.a, 1.0)) {
                e = fn("rg_rcp") + "(" + B + ")";
                tally(1, issued_weights().rcp);
                fl.ops++;
                if (cur_inv) fl.inv_ops++;
            } else {
                e = A + " / " + B;
                count(DIV);
            }
            break;
        case NEG: e = "-" + A; break;
        case EXP:
            // an argument that is not NaN for finite inputs: the variant
            // whose lower clamp is a maximum (NaN -> 0); proven
            // non-positive as well: also without the overflow clamp
            e = (f32 ? "expf(" : !nnan[nd.a] ? "rg_exp(" : sgn[nd.a] < 0 ? "rg_exp_np(" : "rg_exp_nn(") + A + ")";
            count(EXP);
            break;
        case LOG: e = fn("log") + "(" + A + ")"; count(LOG); break;
        case SQRT: e = fn("sqrt") + "(" + A + ")"; count(SQRT); break;
        case SIN: e = fn("sin") + "(" + A + ")"; count(SIN); break;
        case COS: e = fn("cos") + "(" + A + ")"; count(COS); break;
        case POWI: {
            int k = nd.aux < 0 ? -nd.aux : nd.aux;
            std::string p = A;
            for (int i = 1; i < k; i++) p += " * " + A;
            e = nd.aux < 0 ? lit(1.0) + " / (" + p + ")" : p;
            count(POWI, nd.aux);
            break;
        }
        default:
            throw std::logic_error("emit: unexpected node");
        }
        os << "  const " << T() << " " << name(n) << " = " << e << ";\n";
    }

    // One term of a chain: the first defines the accumulator, the others
    // add to it (an fma when the term is a single-use product).
    void emit_acc(int ci, size_t li) {
        Chain &c = chains[ci];
        const uint32_t leaf = c.leaves[li].first;
        const int sg = c.leaves[li].second;
        const std::string R = name(c.root);
        const bool prod = fused[leaf] && g.node(leaf).op == MUL;
        c.acc_inv = c.acc_inv && inv[leaf];
        cur_inv = c.acc_inv;
        if (!c.started) {
            c.started = true;
            std::string t;
            if (prod) {
                const Node &m = g.node(leaf);
                t = std::string(sg < 0 ? "-" : "") + name(m.a) + " * " + name(m.b);
                count(MUL);
            } else {
                t = std::string(sg < 0 ? "-" : "") + name(leaf);
            }
            os << "  " << T() << " " << R << " = " << t << ";\n";
            return;
        }
        if (prod) {
            const Node &m = g.node(leaf);
            os << "  " << R << " = " << fn("fma") << "(" << (sg < 0 ? "-" : "") << name(m.a) << ", " << name(m.b) << ", " << R
               << ");\n";
            count_fma();
        } else {
            os << "  " << R << " = " << R << (sg < 0 ? " - " : " + ") << name(leaf) << ";\n";
            count(ADD);
        }
    }

    // Register-pressure-aware order (greedy list scheduling) over three kinds
    // of units: a node, one term of a chain, and a chain's completion.  Among
    // the units whose inputs are available, take the one that adds the fewest
    // live values: +1 for a new value (a chain's first term creates its
    // accumulator), -1 for every input it is the last user of.  Ties go to the
    // unit that continues the most recently computed value, then to the lower
    // node index.  A sum over many similar terms (16 Gaussian blobs, in a
    // vector-Jacobian product with 6 outputs) is thereby accumulated term by
    // term as its inputs appear, instead of keeping every term's shared
    // values alive until one long chain reaches them.  Only independent
    // operations move; sums are reassociated (deterministically).
    // One output statement ("lhs = v;" or "lhs += v;").
    void emit_output(const Output &o) {
        cur_inv = false;
        if (o.accumulate) {
            if (!g.is_const(o.node, 0.0)) {
                os << "  " << o.lhs << " += " << name(o.node) << ";\n";
                count_plain(1);
            }
        } else {
            os << "  " << o.lhs << " = " << name(o.node) << ";\n";
        }
    }

    // `outs` (may be null) are written as soon as their value is complete,
    // so that a value kept only for an output dies there.
    void schedule_and_emit(const std::vector<uint32_t> &order, const std::vector<uint32_t> &roots,
                           const std::vector<Output> *outs, std::vector<char> *out_done) {
        const size_t N = g.size();
        enum { U_NODE, U_ACC, U_FIN };
        struct Unit {
            int kind;
            uint32_t node;
            int chain;
            size_t leaf;
            std::vector<uint32_t> vals;  // input values
        };
        std::vector<Unit> units;
        std::vector<int> def_unit(N, -1);
        auto inputs = [&](uint32_t m, std::vector<uint32_t> &out) {
            if (m == NONE) return;
            const Node &md = g.node(m);
            if (md.op == CONST || md.op == VAR) return;
            if (fused[m]) {
                for (uint32_t o : {md.a, md.b})
                    if (o != NONE && g.node(o).op != CONST && g.node(o).op != VAR) out.push_back(o);
                return;
            }
            out.push_back(m);
        };
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            if (nd.op == CONST || nd.op == VAR || fused[n] || interior[n]) continue;
            int ci = chain_of_root[n];
            if (ci >= 0) {
                std::vector<int> accs;
                for (size_t li = 0; li < chains[ci].leaves.size(); li++) {
                    Unit u{U_ACC, n, ci, li, {}};
                    uint32_t leaf = chains[ci].leaves[li].first;
                    if (fused[leaf]) inputs(leaf, u.vals);
                    else if (g.node(leaf).op != CONST && g.node(leaf).op != VAR) u.vals.push_back(leaf);
                    accs.push_back((int)units.size());
                    units.push_back(std::move(u));
                }
                Unit f{U_FIN, n, ci, 0, {}};
                def_unit[n] = (int)units.size();
                units.push_back(std::move(f));
                continue;
            }
            Unit u{U_NODE, n, -1, 0, {}};
            inputs(nd.a, u.vals);
            inputs(nd.b, u.vals);
            def_unit[n] = (int)units.size();
            units.push_back(std::move(u));
        }
        const size_t U = units.size();
        std::vector<std::vector<int>> succ(U);
        std::vector<int> unmet(U, 0);
        std::vector<int> remaining(N, 0);
        for (size_t i = 0; i < U; i++) {
            Unit &u = units[i];
            std::sort(u.vals.begin(), u.vals.end());
            u.vals.erase(std::unique(u.vals.begin(), u.vals.end()), u.vals.end());
            for (uint32_t v : u.vals) {
                remaining[v]++;
                succ[def_unit[v]].push_back((int)i);
                unmet[i]++;
            }
        }
        // a chain completes after all its terms
        for (size_t i = 0; i < U; i++)
            if (units[i].kind == U_ACC) {
                succ[i].push_back(def_unit[units[i].node]);
                unmet[def_unit[units[i].node]]++;
            }
        for (uint32_t r : roots)
            if (r != NONE && def_unit.size() > r && def_unit[r] >= 0) remaining[r]++;
        // Phases.  In a sum over many exponentials (Gaussian blobs) most
        // units depend on at most one of them, so the units can run group
        // by group: each unit gets the set of exponentials it depends on and
        // a level, the number of reductions over several groups (a value
        // that depends on two or more) on its longest input path.  Units
        // then run level by level and, within a level, group by group, with
        // the units that need several groups last.  A unit that depends on
        // no exponential runs in the first phase of its consumers, just
        // before its first use.  An exponential of an expression that
        // already holds one (a double exponential) joins the inner one's
        // group.  Phases never fall along an edge, so every phase completes
        // before the next begins.
        std::vector<int> phase(U, 0);
        {
            std::vector<uint64_t> mask(U, 0);
            std::vector<int> lev(U, 0);
            std::vector<std::vector<int>> pred(U);
            for (size_t i = 0; i < U; i++)
                for (int c : succ[i]) pred[c].push_back((int)i);
            auto multi = [](uint64_t m) { return (m & (m - 1)) != 0; };
            int nexp = 0;
            for (size_t i = 0; i < U; i++) {
                for (int v : pred[i]) {
                    if (multi(mask[v])) {
                        lev[i] = std::max(lev[i], lev[v] + 1);
                    } else {
                        lev[i] = std::max(lev[i], lev[v]);
                        mask[i] |= mask[v];
                    }
                }
                if (units[i].kind == U_NODE && g.node(units[i].node).op == EXP && mask[i] == 0) {
                    if (nexp < 64) mask[i] = 1ull << nexp;
                    nexp++;
                }
            }
            if (nexp >= 4 && nexp <= 64) {
                const int per = nexp + 2;
                for (size_t i = U; i-- > 0;) {
                    if (mask[i] == 0) {
                        int ph = 1 << 30;
                        for (int c : succ[i]) ph = std::min(ph, phase[c]);
                        phase[i] = succ[i].empty() ? lev[i] * per : ph;
                    } else if (multi(mask[i])) {
                        phase[i] = lev[i] * per + nexp + 1;
                    } else {
                        phase[i] = lev[i] * per + 1 + __builtin_ctzll(mask[i]);
                    }
                }
                // a unit's phase is at least its inputs'
                for (size_t i = 0; i < U; i++)
                    for (int c : succ[i]) phase[c] = std::max(phase[c], phase[i]);
            }
        }
        std::vector<int> when(N, -1);
        std::vector<char> started(chains.size(), 0);
        std::vector<int> ready;
        for (size_t i = 0; i < U; i++)
            if (unmet[i] == 0) ready.push_back((int)i);
        int step = 0, cur_phase = 0;
        while (!ready.empty()) {
            // stay in the current phase while it has ready units
            int lowest = 1 << 30;
            for (int r : ready) lowest = std::min(lowest, phase[r]);
            cur_phase = std::max(cur_phase, lowest);
            size_t best = 0;
            long best_cost = 1L << 40;
            int best_recent = -2;
            bool have = false;
            for (size_t r = 0; r < ready.size(); r++) {
                if (phase[ready[r]] > cur_phase) continue;
                if (!have) {
                    best = r;
                    have = true;
                }
                const Unit &u = units[ready[r]];
                long cost;
                int recent = -1;  // priority among equal cost: larger is better
                if (u.kind == U_FIN) {
                    cost = -1000;
                } else {
                    cost = (u.kind == U_NODE) ? (remaining[u.node] > 0 ? 1 : 0) : (started[u.chain] ? 0 : 1);
                    for (uint32_t v : u.vals) {
                        if (remaining[v] == 1) cost--;
                        recent = std::max(recent, when[v]);
                    }
                }
                const Unit &b = units[ready[best]];
                if (cost < best_cost || (cost == best_cost && recent > best_recent) ||
                    (cost == best_cost && recent == best_recent && u.node < b.node)) {
                    best = r;
                    best_cost = cost;
                    best_recent = recent;
                }
            }
            const int ui = ready[best];
            ready[best] = ready.back();
            ready.pop_back();
            const Unit &u = units[ui];
            if (u.kind == U_NODE) {
                emit_node(u.node);
                when[u.node] = step++;
            } else if (u.kind == U_ACC) {
                emit_acc(u.chain, u.leaf);
                started[u.chain] = 1;
                when[u.node] = step++;
            } else {
                emitted[u.node] = 1;
            }
            for (uint32_t v : u.vals) --remaining[v];
            if (outs && u.kind != U_ACC && remaining[u.node] > 0)
                for (size_t oi = 0; oi < outs->size(); oi++)
                    if (!(*out_done)[oi] && (*outs)[oi].node == u.node) {
                        emit_output((*outs)[oi]);
                        (*out_done)[oi] = 1;
                        --remaining[u.node];
                    }
            for (int sidx : succ[ui])
                if (--unmet[sidx] == 0) ready.push_back(sidx);
        }
    }

    // Gradient scatter of spline coefficients: for each cell group, the 16
    // coefficient gradients sum_n seed_n * scale_n * wx_du[a] * wy_dv[b].
    void emit_spline_grads(const std::vector<SplineSeed> &seeds) {
        cur_inv = false;
        std::map<int, std::vector<SplineSeed>> by_group;
        for (const SplineSeed &s : seeds) {
            if (g.is_const(s.seed, 0.0)) continue;
            by_group[group_of.at(s.spline_node)].push_back(s);
        }
        for (auto &kv : by_group) {
            int gi = kv.first;
            emit_group_head(gi);
            const Group &gr = groups[gi];
            const SplineDef &sd = g.splines()[gr.def];
            std::string G = "s" + std::to_string(gi);
            // rows per dv order
            std::map<int, std::vector<SplineSeed>> by_dv;
            for (const SplineSeed &s : kv.second) by_dv[g.node(s.spline_node).aux % 4].push_back(s);
            for (auto &dv : by_dv) {
                std::string R = G + "r" + std::to_string(dv.first);
                os << "  double " << R << "[4];\n";
                bool first = true;
                for (const SplineSeed &s : dv.second) {
                    const Node &nd = g.node(s.spline_node);
                    std::string sc = spline_scale(s.spline_node);
                    std::string a = sc.empty() ? name(s.seed) : "(" + sc + " * " + name(s.seed) + ")";
                    if (!sc.empty()) count_plain(1);
                    std::string wx = G + "wx" + std::to_string(nd.aux / 4);
                    for (int i = 0; i < 4; i++) {
                        if (first) {
                            os << "  " << R << "[" << i << "] = " << a << " * " << wx << "[" << i << "];\n";
                            count_plain(1);
                        } else {
                            os << "  " << R << "[" << i << "] = fma(" << a << ", " << wx << "[" << i << "], "
                               << R << "[" << i << "]);\n";
                            count_fma();
                        }
                    }
                    first = false;
                }
            }
            os << "  double " << G << "g[16];\n";
            os << "  for (int a_ = 0; a_ < 4; a_++) for (int b_ = 0; b_ < 4; b_++) {\n";
            bool first = true;
            for (auto &dv : by_dv) {
                std::string R = G + "r" + std::to_string(dv.first);
                std::string wy = G + "wy" + std::to_string(dv.first);
                if (first)
                    os << "    double g_ = " << R << "[a_] * " << wy << "[b_];\n";
                else
                    os << "    g_ = fma(" << R << "[a_], " << wy << "[b_], g_);\n";
                count_plain(first ? 16 : 32);
                first = false;
            }
            os << "    " << G << "g[4 * a_ + b_] = g_;\n  }\n";
            os << "  G.add(" << table_slot.at(sd.param) << ", " << G << "x, " << G << "y, " << G << "g);\n";
        }
    }
};

}  // namespace

std::string emit_function(const Graph &g, const FunctionSpec &spec,
                          const std::vector<int> &param_table_slot, Flops *flops) {
    Emitter em(g, param_table_slot);
    em.f32 = spec.fp32;
    em.inv_state = spec.inv_state;
    em.ktab = spec.fp32 ? nullptr : spec.const_table;
    if (spec.fp32 && !spec.spline_seeds.empty()) throw std::invalid_argument("single precision VJP");
    std::vector<uint32_t> roots;
    for (const Output &o : spec.outputs) roots.push_back(o.node);
    for (const SplineSeed &s : spec.spline_seeds) {
        roots.push_back(s.seed);
        roots.push_back(s.spline_node);
    }
    std::vector<uint32_t> order = g.reachable(roots);
    em.plan(order, roots);
    em.os << spec.signature << "\n";
    if (em.ktab) em.os << "  RG_KBASE\n";
    std::vector<char> out_done(spec.outputs.size(), 0);
    em.schedule_and_emit(order, roots, spec.returns_value ? nullptr : &spec.outputs, &out_done);
    if (!spec.spline_seeds.empty()) em.emit_spline_grads(spec.spline_seeds);
    for (size_t oi = 0; oi < spec.outputs.size(); oi++) {
        const Output &o = spec.outputs[oi];
        if (spec.returns_value) em.os << "  return " << em.name(o.node) << ";\n";
        else if (!out_done[oi]) em.emit_output(o);
    }
    em.os << "}\n";
    if (flops) *flops = em.fl;
    return em.os.str();
}

}  // namespace rg
