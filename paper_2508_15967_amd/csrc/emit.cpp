// Straight-line HIP emission from the expression graph (see emit.hpp).
#include "emit.hpp"

#include <cmath>
#include <cstdio>
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
    //   exp: 13 fma + 1 mul              = 27
    //   div: 5 fma + div_fmas + mul + rcp = 14
    //   sqrt: 7 fma + 2 mul + rsq         = 17
    //   log: 14 fma + 43 add + 7 mul + rcp = 79
    //   sin/cos: 24 fma + 56 add + 11 mul = 115
    //   pow: 42 fma + 70 add + 11 mul + rcp = 166
    //   rg_rcp (reciprocal, rcp + two Newton steps): rcp + 4 fma = 9
    static const IssuedWeights w{/*div*/ 14.0, /*exp*/ 27.0, /*log*/ 79.0, /*sqrt*/ 17.0,
                                 /*sincos*/ 115.0, /*pow*/ 166.0, /*rcp*/ 9.0};
    return w;
}

std::string hex_double(double v) {
    char buf[64];
    if (std::isnan(v)) return "(__builtin_nan(\"\"))";
    if (std::isinf(v)) return v > 0 ? "(__builtin_inf())" : "(-__builtin_inf())";
    std::snprintf(buf, sizeof buf, "(%a)", v);
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
    };
    std::vector<Group> groups;

    Emitter(const Graph &g_, const std::vector<int> &ts) : g(g_), table_slot(ts) {
        uses.assign(g.size(), 0);
        fused.assign(g.size(), 0);
        emitted.assign(g.size(), 0);
    }

    std::string name(uint32_t n) const {
        const Node &nd = g.node(n);
        if (nd.op == CONST) return hex_double(nd.val);
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

    void count(int op, int aux = 0) {
        const IssuedWeights &w = issued_weights();
        fl.ops++;
        switch (op) {
        case ADD: case SUB: case MUL: fl.alg += 1; fl.issued += 1; break;
        case DIV: fl.alg += 1; fl.issued += w.div; break;
        case EXP: fl.alg += 1; fl.issued += w.exp; break;
        case LOG: fl.alg += 1; fl.issued += w.log; break;
        case SQRT: fl.alg += 1; fl.issued += w.sqrt; break;
        case SIN: case COS: fl.alg += 1; fl.issued += w.sincos; break;
        case POWI: {
            int n = aux < 0 ? -aux : aux;
            fl.alg += n - 1; fl.issued += n - 1;
            if (aux < 0) { fl.alg += 1; fl.issued += w.div; }
            break;
        }
        case NEG: fl.ops--; break;
        default: break;
        }
    }
    void count_fma(int n = 1) { fl.alg += 2 * n; fl.issued += 2 * n; fl.ops += n; }
    void count_plain(double f) { fl.alg += f; fl.issued += f; }

    bool fusable_mul(uint32_t m) const {
        const Node &nd = g.node(m);
        return nd.op == MUL && uses[m] == 1;
    }

    void plan(const std::vector<uint32_t> &order, const std::vector<uint32_t> &roots) {
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            if (nd.a != NONE) uses[nd.a]++;
            if (nd.b != NONE) uses[nd.b]++;
        }
        for (uint32_t r : roots) uses[r]++;
        for (uint32_t n : order) {
            const Node &nd = g.node(n);
            if (nd.op == ADD || nd.op == SUB) {
                if (fusable_mul(nd.a) && !fused[nd.a]) fused[nd.a] = 1;
                else if (fusable_mul(nd.b) && !fused[nd.b]) fused[nd.b] = 1;
            }
            if (nd.op == SPLINE) {
                uint32_t def = (uint32_t)nd.val;
                int gi = -1;
                for (size_t i = 0; i < groups.size(); i++)
                    if (groups[i].def == def && groups[i].u == nd.a && groups[i].v == nd.b) gi = (int)i;
                if (gi < 0) {
                    groups.push_back(Group{def, nd.a, nd.b, {}, 0, 0, false});
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
        switch (nd.op) {
        case CONST: case VAR:
            return;
        case PARAM:
            os << "  const double " << name(n) << " = P.p[" << nd.aux << "][" << (size_t)nd.val << "];\n";
            return;
        case SPLINE: {
            int gi = group_of.at(n);
            emit_group_head(gi);
            std::string G = "s" + std::to_string(gi);
            std::string sc = spline_scale(n);
            os << "  const double " << name(n) << " = " << (sc.empty() ? "" : sc + " * ") << "rg_bs_dot("
               << G << "c, " << G << "wx" << nd.aux / 4 << ", " << G << "wy" << nd.aux % 4 << ");\n";
            count_plain(35 + (sc.empty() ? 0 : 1));
            return;
        }
        default: break;
        }
        if (fused[n]) return;  // emitted inside its consumer
        std::string A = nd.a != NONE ? name(nd.a) : "", B = nd.b != NONE ? name(nd.b) : "";
        std::string e;
        switch (nd.op) {
        case ADD: case SUB: {
            bool fa = fused[nd.a] && g.node(nd.a).op == MUL;
            bool fb = !fa && fused[nd.b] && g.node(nd.b).op == MUL;
            if (fa) {
                const Node &m = g.node(nd.a);
                e = "fma(" + name(m.a) + ", " + name(m.b) + ", " + (nd.op == SUB ? "-" : "") + B + ")";
                count_fma();
            } else if (fb) {
                const Node &m = g.node(nd.b);
                e = "fma(" + std::string(nd.op == SUB ? "-" : "") + name(m.a) + ", " + name(m.b) + ", " + A + ")";
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
                e = "rg_rcp(" + B + ")";
                fl.alg += 1; fl.issued += issued_weights().rcp; fl.ops++;
            } else {
                e = A + " / " + B;
                count(DIV);
            }
            break;
        case NEG: e = "-" + A; break;
        case EXP: e = "exp(" + A + ")"; count(EXP); break;
        case LOG: e = "log(" + A + ")"; count(LOG); break;
        case SQRT: e = "sqrt(" + A + ")"; count(SQRT); break;
        case SIN: e = "sin(" + A + ")"; count(SIN); break;
        case COS: e = "cos(" + A + ")"; count(COS); break;
        case POWI: {
            int k = nd.aux < 0 ? -nd.aux : nd.aux;
            std::string p = A;
            for (int i = 1; i < k; i++) p += " * " + A;
            e = nd.aux < 0 ? "1.0 / (" + p + ")" : p;
            count(POWI, nd.aux);
            break;
        }
        default:
            throw std::logic_error("emit: unexpected node");
        }
        os << "  const double " << name(n) << " = " << e << ";\n";
    }

    // Gradient scatter of spline coefficients: for each cell group, the 16
    // coefficient gradients sum_n seed_n * scale_n * wx_du[a] * wy_dv[b].
    void emit_spline_grads(const std::vector<SplineSeed> &seeds) {
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
    std::vector<uint32_t> roots;
    for (const Output &o : spec.outputs) roots.push_back(o.node);
    for (const SplineSeed &s : spec.spline_seeds) {
        roots.push_back(s.seed);
        roots.push_back(s.spline_node);
    }
    std::vector<uint32_t> order = g.reachable(roots);
    em.plan(order, roots);
    em.os << spec.signature << "\n";
    for (uint32_t n : order) em.emit_node(n);
    if (!spec.spline_seeds.empty()) em.emit_spline_grads(spec.spline_seeds);
    for (const Output &o : spec.outputs) {
        if (spec.returns_value) {
            em.os << "  return " << em.name(o.node) << ";\n";
        } else if (o.accumulate) {
            if (!g.is_const(o.node, 0.0)) {
                em.os << "  " << o.lhs << " += " << em.name(o.node) << ";\n";
                em.count_plain(1);
            }
        } else {
            em.os << "  " << o.lhs << " = " << em.name(o.node) << ";\n";
        }
    }
    em.os << "}\n";
    if (flops) *flops = em.fl;
    return em.os.str();
}

}  // namespace rg
