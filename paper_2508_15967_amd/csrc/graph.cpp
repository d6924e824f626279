// Expression graph construction, reduction, differentiation and evaluation.
// Paper, "Graph" subsection and the worked example that follows Listing 1.
#include "graph.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <sstream>
#include <stdexcept>

namespace rg {

static uint64_t dbits(double v) {
    uint64_t b;
    std::memcpy(&b, &v, 8);
    return b;
}

size_t Graph::KeyHash::operator()(const Key &k) const {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t v) {
        h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    };
    mix((uint64_t)(uint32_t)k.op);
    mix((uint64_t)(uint32_t)k.aux);
    mix(k.a);
    mix(k.b);
    mix(k.bits);
    return (size_t)h;
}

Graph::Graph(uint32_t dim) : dim_(dim) {
    nodes_.reserve(1024);
    // pre-declare the kernel inputs: x[dim], k[dim], omega, t
    for (uint32_t i = 0; i < dim; i++) var(VK_X, i);
    for (uint32_t i = 0; i < dim; i++) var(VK_K, i);
    var(VK_OMEGA, 0);
    var(VK_T, 0);
}

uint32_t Graph::intern(int32_t op, int32_t aux, uint32_t a, uint32_t b, double val) {
    // +0.0 and -0.0 are one constant for hashing purposes only if equal bits;
    // keep them distinct (they differ under division).
    Key key{op, aux, a, b, dbits(val)};
    auto it = cache_.find(key);
    if (it != cache_.end()) return it->second;
    uint32_t id = (uint32_t)nodes_.size();
    nodes_.push_back(Node{op, aux, a, b, val});
    cache_.emplace(key, id);
    return id;
}

double Graph::fold(int32_t op, double a, double b, int32_t aux) const {
    switch (op) {
    case ADD: return a + b;
    case SUB: return a - b;
    case MUL: return a * b;
    case DIV: return a / b;
    case NEG: return -a;
    case EXP: return std::exp(a);
    case LOG: return std::log(a);
    case SQRT: return std::sqrt(a);
    case SIN: return std::sin(a);
    case COS: return std::cos(a);
    case POWI: {
        double r = 1.0, base = a;
        int n = aux < 0 ? -aux : aux;
        for (int i = 0; i < n; i++) r *= base;
        return aux < 0 ? 1.0 / r : r;
    }
    }
    return NAN;
}

uint32_t Graph::constant(double v) { return intern(CONST, 0, NONE, NONE, v); }

uint32_t Graph::var(int32_t kind, uint32_t i) { return intern(VAR, kind * 8 + (int32_t)i, NONE, NONE, 0.0); }

uint32_t Graph::param_elem(uint32_t param, uint32_t idx) {
    if (param >= params_.size() || idx >= params_[param].len)
        throw std::invalid_argument("parameter element out of range");
    return intern(PARAM, (int32_t)param, NONE, NONE, (double)idx);
}

uint32_t Graph::declare_param(const std::string &name, uint32_t len) {
    params_.push_back(ParamDef{name, len});
    return (uint32_t)params_.size() - 1;
}

uint32_t Graph::declare_spline(const SplineDef &d) {
    for (size_t i = 0; i < splines_.size(); i++) {
        const SplineDef &s = splines_[i];
        if (s.param == d.param && s.nx == d.nx && s.ny == d.ny && s.lo[0] == d.lo[0] &&
            s.lo[1] == d.lo[1] && s.hi[0] == d.hi[0] && s.hi[1] == d.hi[1])
            return (uint32_t)i;
    }
    splines_.push_back(d);
    return (uint32_t)splines_.size() - 1;
}

// ------------------------------------------------------------ arithmetic ---

uint32_t Graph::add(uint32_t a, uint32_t b) {
    if (is_const(a) && is_const(b)) return constant(nodes_[a].val + nodes_[b].val);
    if (is_const(a, 0.0)) return b;
    if (is_const(b, 0.0)) return a;
    const Node &na = nodes_[a], &nb = nodes_[b];
    if (nb.op == NEG) return sub(a, nb.a);          // a + (-b) -> a - b
    if (na.op == NEG) return sub(b, na.a);          // (-a) + b -> b - a
    if (a == b) return mul(constant(2.0), a);       // x + x -> 2 x
    // canonical operand order: constants first, then by index
    if (is_const(b) || (!is_const(a) && b < a)) std::swap(a, b);
    return intern(ADD, 0, a, b, 0.0);
}

uint32_t Graph::sub(uint32_t a, uint32_t b) {
    if (is_const(a) && is_const(b)) return constant(nodes_[a].val - nodes_[b].val);
    if (is_const(b, 0.0)) return a;
    if (is_const(a, 0.0)) return neg(b);
    if (a == b) return constant(0.0);
    const Node &nb = nodes_[b];
    if (nb.op == NEG) return add(a, nb.a);          // a - (-b) -> a + b
    if (nodes_[a].op == NEG) return neg(add(nodes_[a].a, b));  // -a - b -> -(a + b)
    return intern(SUB, 0, a, b, 0.0);
}

uint32_t Graph::mul(uint32_t a, uint32_t b) {
    if (is_const(b) && !is_const(a)) std::swap(a, b);
    if (is_const(a) && is_const(b)) return constant(nodes_[a].val * nodes_[b].val);
    if (is_const(a, 0.0) || is_const(b, 0.0)) return constant(0.0);  // x*0 -> 0 (as the paper)
    if (is_const(a, 1.0)) return b;
    if (is_const(a, -1.0)) return neg(b);
    const Node &na = nodes_[a], &nb = nodes_[b];
    if (na.op == NEG && nb.op == NEG) return mul(na.a, nb.a);
    if (na.op == NEG) return neg(mul(na.a, b));
    if (nb.op == NEG) return neg(mul(a, nb.a));
    // c1 * (c2 * x) -> (c1 c2) * x
    if (is_const(a) && nb.op == MUL && is_const(nb.a)) return mul(constant(na.val * nodes_[nb.a].val), nb.b);
    if (!is_const(a) && b < a) std::swap(a, b);
    return intern(MUL, 0, a, b, 0.0);
}

uint32_t Graph::div(uint32_t a, uint32_t b) {
    if (is_const(a) && is_const(b)) return constant(nodes_[a].val / nodes_[b].val);
    if (is_const(b, 1.0)) return a;
    if (is_const(b, -1.0)) return neg(a);
    if (is_const(a, 0.0)) return constant(0.0);
    const Node &na = nodes_[a], &nb = nodes_[b];
    if (na.op == NEG) return neg(div(na.a, b));
    if (nb.op == NEG) return neg(div(a, nb.a));
    if (is_const(b)) {
        // division by a power of two is an exact multiplication
        int e;
        double m = std::frexp(nb.val, &e);
        if (m == 0.5 || m == -0.5) return mul(constant(1.0 / nb.val), a);
    }
    return intern(DIV, 0, a, b, 0.0);
}

uint32_t Graph::neg(uint32_t a) {
    if (is_const(a)) return constant(-nodes_[a].val);
    const Node &na = nodes_[a];
    if (na.op == NEG) return na.a;
    if (na.op == MUL && is_const(na.a)) return mul(constant(-nodes_[na.a].val), na.b);
    if (na.op == SUB) return sub(na.b, na.a);
    return intern(NEG, 0, a, NONE, 0.0);
}

uint32_t Graph::unary(int32_t op, uint32_t a) {
    if (op != EXP && op != LOG && op != SQRT && op != SIN && op != COS)
        throw std::invalid_argument("bad unary op");
    if (is_const(a)) return constant(fold(op, nodes_[a].val, 0.0, 0));
    return intern(op, 0, a, NONE, 0.0);
}

uint32_t Graph::powi(uint32_t a, int32_t n) {
    if (n == 0) return constant(1.0);
    if (n == 1) return a;
    if (is_const(a)) return constant(fold(POWI, nodes_[a].val, 0.0, n));
    if (n == -1) return div(constant(1.0), a);
    return intern(POWI, n, a, NONE, 0.0);
}

uint32_t Graph::spline(uint32_t def, int32_t du, int32_t dv, uint32_t u, uint32_t v) {
    if (def >= splines_.size()) throw std::invalid_argument("bad spline definition");
    if (du > 3 || dv > 3) return constant(0.0);  // cubic: 4th derivative vanishes
    return intern(SPLINE, du * 4 + dv, u, v, (double)def);
}

// -------------------------------------------------------------------- df ---

std::vector<uint32_t> Graph::reachable(const std::vector<uint32_t> &roots) const {
    std::vector<char> mark(nodes_.size(), 0);
    std::vector<uint32_t> stack(roots.begin(), roots.end());
    while (!stack.empty()) {
        uint32_t n = stack.back();
        stack.pop_back();
        if (n == NONE || mark[n]) continue;
        mark[n] = 1;
        const Node &nd = nodes_[n];
        if (nd.a != NONE) stack.push_back(nd.a);
        if (nd.b != NONE) stack.push_back(nd.b);
    }
    std::vector<uint32_t> out;
    for (uint32_t i = 0; i < mark.size(); i++)
        if (mark[i]) out.push_back(i);
    return out;
}

uint32_t Graph::df(uint32_t f, uint32_t wrt) {
    // Forward sweep over the nodes f depends on (indices are topological);
    // d[n] = d node_n / d wrt, built with the same reducing factories.
    std::vector<uint32_t> order = reachable({f});
    std::unordered_map<uint32_t, uint32_t> d;
    d.reserve(order.size() * 2);
    const uint32_t zero = constant(0.0), one = constant(1.0);
    for (uint32_t n : order) {
        if (n == wrt) { d[n] = one; continue; }
        const Node nd = nodes_[n];  // copy: factories may grow nodes_
        uint32_t da = nd.a != NONE ? d[nd.a] : zero;
        uint32_t db = nd.b != NONE ? d[nd.b] : zero;
        uint32_t r = zero;
        switch (nd.op) {
        case CONST: case VAR: case PARAM:
            r = zero;
            break;
        case ADD: r = add(da, db); break;
        case SUB: r = sub(da, db); break;
        case MUL: r = add(mul(da, nd.b), mul(nd.a, db)); break;
        case DIV:
            // (a/b)' = (a' - (a/b) b') / b;  (1/b)' = -(1/b)^2 b' needs no division
            if (is_const(db, 0.0)) r = div(da, nd.b);
            else if (is_const(nd.a, 1.0)) r = neg(mul(mul(n, n), db));
            else r = div(sub(da, mul(n, db)), nd.b);
            break;
        case NEG: r = neg(da); break;
        case EXP: r = mul(n, da); break;
        case LOG: r = div(da, nd.a); break;
        case SQRT: r = div(mul(constant(0.5), da), n); break;
        case SIN: r = mul(unary(COS, nd.a), da); break;
        case COS: r = neg(mul(unary(SIN, nd.a), da)); break;
        case POWI:
            r = mul(mul(constant((double)nd.aux), powi(nd.a, nd.aux - 1)), da);
            break;
        case SPLINE: {
            int du = nd.aux / 4, dv = nd.aux % 4;
            uint32_t def = (uint32_t)nd.val;
            r = add(mul(spline(def, du + 1, dv, nd.a, nd.b), da),
                    mul(spline(def, du, dv + 1, nd.a, nd.b), db));
            break;
        }
        }
        d[n] = r;
    }
    return d[f];
}

// Reverse mode: adjoints flow from each node to its operands in decreasing
// index order (a node's consumers all have larger indices, so its adjoint is
// complete when it is reached).  Contributions are summed with the reducing
// factories, so zero terms vanish and shared sub-expressions are reused.
std::vector<uint32_t> Graph::adjoints(const std::vector<uint32_t> &outs,
                                      const std::vector<uint32_t> &seeds) {
    std::vector<uint32_t> order = reachable(outs);
    std::vector<uint32_t> adj(nodes_.size(), NONE);
    auto acc = [&](uint32_t n, uint32_t c) {
        if (n == NONE || is_const(c, 0.0)) return;
        if (adj.size() <= n) adj.resize(nodes_.size(), NONE);
        adj[n] = adj[n] == NONE ? c : add(adj[n], c);
    };
    for (size_t i = 0; i < outs.size(); i++) acc(outs[i], seeds[i]);
    for (size_t oi = order.size(); oi-- > 0;) {
        const uint32_t n = order[oi];
        if (adj.size() < nodes_.size()) adj.resize(nodes_.size(), NONE);
        const uint32_t a = adj[n];
        if (a == NONE) continue;
        const Node nd = nodes_[n];  // copy: factories may grow nodes_
        switch (nd.op) {
        case CONST: case VAR: case PARAM:
            break;
        case ADD: acc(nd.a, a); acc(nd.b, a); break;
        case SUB: acc(nd.a, a); acc(nd.b, neg(a)); break;
        case MUL: acc(nd.a, mul(a, nd.b)); acc(nd.b, mul(a, nd.a)); break;
        case DIV:
            // n = a/b: dn/da = 1/b, dn/db = -n/b;  (1/b): -(1/b)^2
            if (is_const(nd.a, 1.0)) {
                acc(nd.b, neg(mul(a, mul(n, n))));
            } else {
                const uint32_t q = div(a, nd.b);
                acc(nd.a, q);
                acc(nd.b, neg(mul(q, n)));
            }
            break;
        case NEG: acc(nd.a, neg(a)); break;
        case EXP: acc(nd.a, mul(a, n)); break;
        case LOG: acc(nd.a, div(a, nd.a)); break;
        case SQRT: acc(nd.a, div(mul(constant(0.5), a), n)); break;
        case SIN: acc(nd.a, mul(a, unary(COS, nd.a))); break;
        case COS: acc(nd.a, neg(mul(a, unary(SIN, nd.a)))); break;
        case POWI:
            acc(nd.a, mul(a, mul(constant((double)nd.aux), powi(nd.a, nd.aux - 1))));
            break;
        case SPLINE: {
            const int du = nd.aux / 4, dv = nd.aux % 4;
            const uint32_t def = (uint32_t)nd.val;
            acc(nd.a, mul(a, spline(def, du + 1, dv, nd.a, nd.b)));
            acc(nd.b, mul(a, spline(def, du, dv + 1, nd.a, nd.b)));
            break;
        }
        }
    }
    adj.resize(nodes_.size(), NONE);
    return adj;
}

// ------------------------------------------------------ hoist divisions ---

std::vector<uint32_t> Graph::hoist_divisions(const std::vector<uint32_t> &roots, bool split_products,
                                             uint32_t inv_state) {
    const std::vector<uint32_t> order = reachable(roots);
    const size_t N0 = nodes_.size();
    std::vector<char> inv(N0, 0);
    std::vector<uint32_t> nw(N0, NONE);
    for (uint32_t n : order) {
        const Node d = nodes_[n];  // copy: factories may grow nodes_
        if (d.op == CONST || d.op == PARAM) inv[n] = 1;
        else if (d.op == VAR) inv[n] = ray_invariant_var(d, inv_state);
        else inv[n] = (d.a == NONE || inv[d.a]) && (d.b == NONE || inv[d.b]);
        if (d.op == CONST || d.op == VAR || d.op == PARAM) {
            nw[n] = n;
            continue;
        }
        const uint32_t a = d.a != NONE ? nw[d.a] : NONE, b = d.b != NONE ? nw[d.b] : NONE;
        switch (d.op) {
        case ADD: nw[n] = add(a, b); break;
        case SUB: nw[n] = sub(a, b); break;
        case MUL: nw[n] = mul(a, b); break;
        case DIV: {
            if (inv[d.b] || !split_products) {
                nw[n] = inv[d.b] && !inv[d.a] && !is_const(b) && !is_const(a, 1.0) ? mul(a, div(constant(1.0), b)) : div(a, b);
                break;
            }
            // a variant denominator that is a product with invariant factors:
            // a / (I V) = (a / V) (1 / I), the second factor once per ray
            std::vector<uint32_t> fi, fv;
            bool negate = false;
            std::function<void(uint32_t)> walk = [&](uint32_t m) {
                const Node &q = nodes_[m];
                if (q.op == MUL && fi.size() + fv.size() < 32) {
                    walk(q.a);
                    walk(q.b);
                } else if (q.op == NEG) {
                    negate = !negate;
                    walk(q.a);
                } else {
                    (inv[m] ? fi : fv).push_back(nw[m]);
                }
            };
            walk(d.b);
            if (fi.empty() || fv.empty()) {
                nw[n] = div(a, b);
                break;
            }
            uint32_t pv = fv[0], pi = fi[0];
            for (size_t i = 1; i < fv.size(); i++) pv = mul(pv, fv[i]);
            for (size_t i = 1; i < fi.size(); i++) pi = mul(pi, fi[i]);
            if (negate) pi = neg(pi);
            nw[n] = mul(div(a, pv), div(constant(1.0), pi));
            break;
        }
        case NEG: nw[n] = neg(a); break;
        case POWI: nw[n] = powi(a, d.aux); break;
        case SPLINE: nw[n] = spline((uint32_t)d.val, d.aux / 4, d.aux % 4, a, b); break;
        default: nw[n] = unary(d.op, a); break;
        }
    }
    std::vector<uint32_t> out(roots.size(), NONE);
    for (size_t i = 0; i < roots.size(); i++) out[i] = roots[i] == NONE ? NONE : nw[roots[i]];
    return out;
}

// ------------------------------------------------------ factor products ---

std::vector<uint32_t> Graph::factor_products(const std::vector<uint32_t> &roots, bool merge_invariants,
                                             uint32_t inv_state) {
    const std::vector<uint32_t> order = reachable(roots);
    const size_t N0 = nodes_.size();
    auto is_prod = [&](uint32_t n) {
        const Node &d = nodes_[n];
        return d.op == MUL || (d.op == NEG && nodes_[d.a].op == MUL);
    };
    // a product is rebuilt on its own where its value is used by a
    // non-product or is a root; elsewhere it is folded into its consumers
    std::vector<char> top(N0, 0);
    for (uint32_t r : roots)
        if (r != NONE) top[r] = 1;
    for (uint32_t n : order) {
        const Node &d = nodes_[n];
        if (d.op == CONST || d.op == VAR || d.op == PARAM || is_prod(n)) continue;
        if (d.a != NONE) top[d.a] = 1;
        if (d.b != NONE) top[d.b] = 1;
    }
    // flattened factor count (bounded: a product of powers could double at
    // every level)
    const size_t kMaxFactors = 32;
    std::vector<size_t> fsize(N0, 1);
    for (uint32_t n : order) {
        const Node &d = nodes_[n];
        if (d.op == MUL) fsize[n] = std::min(kMaxFactors + 1, fsize[d.a] + fsize[d.b]);
        else if (d.op == NEG && nodes_[d.a].op == MUL) fsize[n] = fsize[d.a];
    }
    struct Prod {
        uint32_t node;
        double c;                   // folded constant factors and sign
        std::vector<uint32_t> sym;  // leaf nodes, or kVirtual | pair index
    };
    const uint32_t kVirtual = 0x80000000u;
    std::vector<Prod> prods;
    std::vector<int> prod_of(N0, -1);
    for (uint32_t n : order) {
        if (!is_prod(n) || !top[n]) continue;
        if (fsize[n] > kMaxFactors) return roots;  // leave such graphs alone
        Prod P{n, 1.0, {}};
        std::vector<uint32_t> stack{n};
        while (!stack.empty()) {
            const uint32_t m = stack.back();
            stack.pop_back();
            const Node &d = nodes_[m];
            if (d.op == MUL) {
                stack.push_back(d.b);
                stack.push_back(d.a);
            } else if (d.op == NEG && nodes_[d.a].op == MUL) {
                P.c = -P.c;
                stack.push_back(d.a);
            } else if (d.op == CONST) {
                P.c *= d.val;
            } else {
                P.sym.push_back(m);
            }
        }
        // a constant factor takes part in the pairing (a scaled common
        // factor such as 2/D_omega is then formed once); a sign stays apart
        // (negation is free as an operand modifier)
        if (P.c != 1.0 && P.c != -1.0) {
            P.sym.push_back(constant(std::fabs(P.c)));
            P.c = P.c < 0 ? -1.0 : 1.0;
        }
        std::sort(P.sym.begin(), P.sym.end());
        prod_of[n] = (int)prods.size();
        prods.push_back(std::move(P));
    }
    // factors are multiplied in order of variability: constants, then what
    // depends only on omega and parameters (invariant along a ray: the
    // compiler hoists that part of the product out of the time loop), then
    // what depends on the state, t or the seeds
    std::vector<int> rank(N0, 0);
    for (uint32_t n : order) {
        const Node &d = nodes_[n];
        if (d.op == VAR) rank[n] = ray_invariant_var(d, inv_state) ? 1 : 2;
        else if (d.op == PARAM) rank[n] = 1;
        else if (d.op != CONST)
            rank[n] = std::max(d.a != NONE ? rank[d.a] : 0, d.b != NONE ? rank[d.b] : 0);
    }
    auto leaf_rank = [&](uint32_t s2) { return s2 < N0 ? rank[s2] : 0; };  // new nodes: folded constants
    // Greedy pairing (most shared pair first, ties to the smaller pair),
    // tried two ways: as is, and with the invariant factors of each product
    // made one factor first.  The second keeps every invariant factor out of
    // the time loop, while the first may share a pair of an invariant and a
    // variant factor between products; the one with fewer multiplications
    // per evaluation is kept.
    struct Pairing {
        std::vector<std::pair<uint32_t, uint32_t>> pairs;
        std::vector<Prod> prods;
    };
    // rank of a symbol of a pairing (a pair ranks as its higher side)
    std::function<int(const Pairing &, uint32_t)> srank_in = [&](const Pairing &R, uint32_t s2) -> int {
        if (s2 & kVirtual) {
            const auto &pr = R.pairs[s2 & ~kVirtual];
            return std::max(srank_in(R, pr.first), srank_in(R, pr.second));
        }
        return leaf_rank(s2);
    };
    auto run_pairing = [&](bool merge) {
        Pairing R{{}, prods};
        std::map<std::pair<uint32_t, uint32_t>, uint32_t> pair_id;
        auto make_pair = [&](uint32_t x, uint32_t y) {
            const std::pair<uint32_t, uint32_t> key{std::min(x, y), std::max(x, y)};
            auto it = pair_id.find(key);
            if (it != pair_id.end()) return it->second;
            const uint32_t v = kVirtual | (uint32_t)R.pairs.size();
            R.pairs.push_back(key);
            pair_id[key] = v;
            return v;
        };
        if (merge)
            for (Prod &P : R.prods) {
                std::vector<uint32_t> iv, vv;
                for (uint32_t s2 : P.sym) (leaf_rank(s2) <= 1 ? iv : vv).push_back(s2);
                if (iv.size() < 2) continue;
                uint32_t acc = iv[0];
                for (size_t i = 1; i < iv.size(); i++) acc = make_pair(acc, iv[i]);
                vv.push_back(acc);
                std::sort(vv.begin(), vv.end());
                P.sym = std::move(vv);
            }
        for (;;) {
            std::map<std::pair<uint32_t, uint32_t>, int> count;
            for (const Prod &P : R.prods) {
                std::set<std::pair<uint32_t, uint32_t>> here;
                for (size_t i = 0; i < P.sym.size(); i++)
                    for (size_t j = i + 1; j < P.sym.size(); j++) here.insert({P.sym[i], P.sym[j]});
                for (const auto &pr : here) count[pr]++;
            }
            std::pair<uint32_t, uint32_t> best{0, 0};
            int bc = 1;
            for (const auto &kv : count)
                if (kv.second > bc) {
                    bc = kv.second;
                    best = kv.first;
                }
            if (bc < 2) break;
            const uint32_t v = make_pair(best.first, best.second);
            for (Prod &P : R.prods) {
                // every disjoint occurrence (x y x y holds the pair twice)
                for (;;) {
                    auto ia = std::find(P.sym.begin(), P.sym.end(), best.first);
                    if (ia == P.sym.end()) break;
                    auto ib = std::find(ia + 1, P.sym.end(), best.second);
                    if (ib == P.sym.end()) break;
                    P.sym.erase(ib);
                    P.sym.erase(ia);
                    P.sym.push_back(v);
                    std::sort(P.sym.begin(), P.sym.end());
                }
            }
        }
        return R;
    };
    // multiplications per evaluation: in a product of m factors, k of them
    // invariant, the k - 1 among the invariant ones are hoisted; a formed
    // pair costs one if either side varies
    auto per_eval_muls = [&](const Pairing &R) {
        auto sr = [&](uint32_t s2) { return srank_in(R, s2); };
        size_t c = 0;
        std::set<uint32_t> used;
        std::function<void(uint32_t)> mark = [&](uint32_t s2) {
            if (!(s2 & kVirtual) || !used.insert(s2).second) return;
            mark(R.pairs[s2 & ~kVirtual].first);
            mark(R.pairs[s2 & ~kVirtual].second);
        };
        for (const Prod &P : R.prods) {
            size_t k = 0;
            for (uint32_t s2 : P.sym) {
                k += sr(s2) <= 1;
                mark(s2);
            }
            if (!P.sym.empty()) c += P.sym.size() - 1 - (k > 0 ? k - 1 : 0);
        }
        for (uint32_t v : used) c += sr(v) > 1;
        return c;
    };
    Pairing plain = run_pairing(false), merged;
    if (merge_invariants) merged = run_pairing(true);
    Pairing &chosen = merge_invariants && per_eval_muls(merged) < per_eval_muls(plain) ? merged : plain;
    std::vector<std::pair<uint32_t, uint32_t>> pairs = std::move(chosen.pairs);
    prods = std::move(chosen.prods);
    std::function<int(uint32_t)> srank = [&](uint32_t s2) -> int {
        if (s2 & kVirtual) {
            const auto &pr = pairs[s2 & ~kVirtual];
            return std::max(srank(pr.first), srank(pr.second));
        }
        return leaf_rank(s2);
    };
    for (Prod &P : prods)
        std::stable_sort(P.sym.begin(), P.sym.end(),
                         [&](uint32_t x, uint32_t y) { return srank(x) < srank(y); });
    // rebuild in topological order
    std::vector<uint32_t> nw(N0, NONE), vnew(pairs.size(), NONE);
    std::function<uint32_t(uint32_t)> get = [&](uint32_t s) -> uint32_t {
        if (!(s & kVirtual)) return nodes_[s].op == CONST ? s : nw[s];  // folded constants may be new
        const uint32_t i = s & ~kVirtual;
        if (vnew[i] == NONE) vnew[i] = mul(get(pairs[i].first), get(pairs[i].second));
        return vnew[i];
    };
    for (uint32_t n : order) {
        const Node d = nodes_[n];  // copy: factories may grow nodes_
        if (d.op == CONST || d.op == VAR || d.op == PARAM) {
            nw[n] = n;
            continue;
        }
        if (is_prod(n)) {
            if (prod_of[n] < 0) continue;  // folded into its consumers
            const Prod &P = prods[prod_of[n]];
            uint32_t acc = NONE;
            for (uint32_t s2 : P.sym) acc = acc == NONE ? get(s2) : mul(acc, get(s2));
            nw[n] = acc == NONE ? constant(P.c) : P.c < 0 ? neg(acc) : acc;
            continue;
        }
        const uint32_t a = d.a != NONE ? nw[d.a] : NONE, b = d.b != NONE ? nw[d.b] : NONE;
        switch (d.op) {
        case ADD: nw[n] = add(a, b); break;
        case SUB: nw[n] = sub(a, b); break;
        case DIV: nw[n] = div(a, b); break;
        case NEG: nw[n] = neg(a); break;
        case POWI: nw[n] = powi(a, d.aux); break;
        case SPLINE: nw[n] = spline((uint32_t)d.val, d.aux / 4, d.aux % 4, a, b); break;
        default: nw[n] = unary(d.op, a); break;
        }
    }
    std::vector<uint32_t> out(roots.size(), NONE);
    for (size_t i = 0; i < roots.size(); i++) out[i] = roots[i] == NONE ? NONE : nw[roots[i]];
    return out;
}

std::vector<uint32_t> Graph::collect_factors(const std::vector<uint32_t> &roots) {
    const std::vector<uint32_t> order = reachable(roots);
    const size_t N0 = nodes_.size();
    auto is_sum = [&](uint32_t n) {
        const Node &d = nodes_[n];
        return d.op == ADD || d.op == SUB ||
               (d.op == NEG && (nodes_[d.a].op == ADD || nodes_[d.a].op == SUB));
    };
    std::vector<char> top(N0, 0);
    for (uint32_t r : roots)
        if (r != NONE) top[r] = 1;
    for (uint32_t n : order) {
        const Node &d = nodes_[n];
        if (d.op == CONST || d.op == VAR || d.op == PARAM || is_sum(n)) continue;
        if (d.a != NONE) top[d.a] = 1;
        if (d.b != NONE) top[d.b] = 1;
    }
    const size_t kMaxTerms = 4096, kMaxFactors = 32;
    struct Term {
        std::vector<uint32_t> f;  // factors, sorted (new nodes)
        int sg;
    };
    // factors of a (new) node through products and negations
    auto factors = [&](uint32_t t, Term &out) {
        std::vector<uint32_t> stack{t};
        while (!stack.empty()) {
            const uint32_t m = stack.back();
            stack.pop_back();
            const Node &d = nodes_[m];
            if (d.op == MUL && out.f.size() + stack.size() < kMaxFactors) {
                stack.push_back(d.b);
                stack.push_back(d.a);
            } else if (d.op == NEG) {
                out.sg = -out.sg;
                stack.push_back(d.a);
            } else {
                out.f.push_back(m);
            }
        }
        std::sort(out.f.begin(), out.f.end());
    };
    auto product = [&](const std::vector<uint32_t> &f) {
        uint32_t p = NONE;
        for (uint32_t x : f) p = p == NONE ? x : mul(p, x);
        return p == NONE ? constant(1.0) : p;
    };
    // sum of terms with common factors taken out; terms in a fixed order
    std::function<uint32_t(std::vector<Term>)> build = [&](std::vector<Term> ts) -> uint32_t {
        for (;;) {
            std::map<uint32_t, int> count;
            for (const Term &t : ts) {
                for (size_t i = 0; i < t.f.size(); i++)
                    if (i == 0 || t.f[i] != t.f[i - 1]) count[t.f[i]]++;
            }
            uint32_t best = NONE;
            int bc = 1;
            for (const auto &kv : count)
                if (kv.second > bc) {
                    bc = kv.second;
                    best = kv.first;
                }
            if (best == NONE) break;
            std::vector<Term> in, rest;
            for (Term &t : ts) {
                auto it = std::find(t.f.begin(), t.f.end(), best);
                if (it == t.f.end()) {
                    rest.push_back(std::move(t));
                } else {
                    t.f.erase(it);
                    in.push_back(std::move(t));
                }
            }
            const uint32_t inner = build(std::move(in));
            Term nt{{best, inner}, 1};
            if (nodes_[inner].op == NEG) {
                nt.f[1] = nodes_[inner].a;
                nt.sg = -1;
            }
            std::sort(nt.f.begin(), nt.f.end());
            rest.push_back(std::move(nt));
            ts = std::move(rest);
        }
        // canonical order: by factor lists
        std::sort(ts.begin(), ts.end(), [](const Term &a, const Term &b) {
            return a.f != b.f ? a.f < b.f : a.sg < b.sg;
        });
        uint32_t acc = NONE;
        for (const Term &t : ts) {
            const uint32_t p = product(t.f);
            if (acc == NONE) acc = t.sg < 0 ? neg(p) : p;
            else acc = t.sg < 0 ? sub(acc, p) : add(acc, p);
        }
        return acc == NONE ? constant(0.0) : acc;
    };
    std::vector<uint32_t> nw(N0, NONE);
    for (uint32_t n : order) {
        const Node d = nodes_[n];
        if (d.op == CONST || d.op == VAR || d.op == PARAM) {
            nw[n] = n;
            continue;
        }
        if (is_sum(n)) {
            if (!top[n]) continue;  // folded into its consumers
            std::vector<Term> ts;
            double c = 0.0;
            std::vector<std::pair<uint32_t, int>> stack{{n, 1}};
            bool too_big = false;
            while (!stack.empty()) {
                const auto [m, sg] = stack.back();
                stack.pop_back();
                const Node &md = nodes_[m];
                if (md.op == ADD || md.op == SUB) {
                    stack.push_back({md.b, md.op == SUB ? -sg : sg});
                    stack.push_back({md.a, sg});
                } else if (md.op == NEG && is_sum(m)) {
                    stack.push_back({md.a, -sg});
                } else if (md.op == CONST) {
                    c += sg * md.val;
                } else {
                    Term t{{}, sg};
                    factors(nw[m], t);
                    ts.push_back(std::move(t));
                    if (ts.size() > kMaxTerms) {
                        too_big = true;
                        break;
                    }
                }
            }
            if (too_big) return roots;  // leave such graphs alone
            uint32_t r = build(std::move(ts));
            if (c != 0.0) r = add(constant(c), r);
            nw[n] = r;
            continue;
        }
        const uint32_t a = d.a != NONE ? nw[d.a] : NONE, b = d.b != NONE ? nw[d.b] : NONE;
        switch (d.op) {
        case MUL: nw[n] = mul(a, b); break;
        case DIV: nw[n] = div(a, b); break;
        case NEG: nw[n] = neg(a); break;
        case POWI: nw[n] = powi(a, d.aux); break;
        case SPLINE: nw[n] = spline((uint32_t)d.val, d.aux / 4, d.aux % 4, a, b); break;
        default: nw[n] = unary(d.op, a); break;
        }
    }
    std::vector<uint32_t> out;
    for (uint32_t r : roots) out.push_back(r == NONE ? NONE : nw[r]);
    return out;
}

std::vector<uint32_t> Graph::share_scaled_sums(const std::vector<uint32_t> &roots) {
    const std::vector<uint32_t> order = reachable(roots);
    const size_t N0 = nodes_.size();
    auto is_sum = [&](uint32_t n) { return nodes_[n].op == ADD || nodes_[n].op == SUB; };
    std::vector<char> top(N0, 0);
    for (uint32_t r : roots)
        if (r != NONE) top[r] = 1;
    for (uint32_t n : order) {
        const Node &d = nodes_[n];
        if (d.op == CONST || d.op == VAR || d.op == PARAM || is_sum(n)) continue;
        if (d.a != NONE) top[d.a] = 1;
        if (d.b != NONE) top[d.b] = 1;
    }
    // key: the terms (value, coefficient) sorted by value, every
    // coefficient divided by the power of two of the first one; entry: the
    // first sum with that key and its power of two
    std::map<std::vector<std::pair<uint32_t, double>>, std::pair<uint32_t, int>> seen;
    std::vector<uint32_t> nw(N0, NONE);
    for (uint32_t n : order) {
        const Node d = nodes_[n];
        if (d.op == CONST || d.op == VAR || d.op == PARAM) {
            nw[n] = n;
            continue;
        }
        const uint32_t a = d.a != NONE ? nw[d.a] : NONE, b = d.b != NONE ? nw[d.b] : NONE;
        uint32_t r;
        switch (d.op) {
        case ADD: r = add(a, b); break;
        case SUB: r = sub(a, b); break;
        case MUL: r = mul(a, b); break;
        case DIV: r = div(a, b); break;
        case NEG: r = neg(a); break;
        case POWI: r = powi(a, d.aux); break;
        case SPLINE: r = spline((uint32_t)d.val, d.aux / 4, d.aux % 4, a, b); break;
        default: r = unary(d.op, a); break;
        }
        nw[n] = r;
        if (!is_sum(n) || !top[n] || !is_sum(r)) continue;
        // the terms of the rebuilt maximal sum
        std::vector<std::pair<uint32_t, double>> terms;
        bool linear = true;
        std::vector<std::pair<uint32_t, double>> stack{{r, 1.0}};
        while (!stack.empty() && linear) {
            const auto [m, sg] = stack.back();
            stack.pop_back();
            const Node &md = nodes_[m];
            if (md.op == ADD || md.op == SUB) {
                stack.push_back({md.b, md.op == SUB ? -sg : sg});
                stack.push_back({md.a, sg});
            } else if (md.op == NEG) {
                stack.push_back({md.a, -sg});
            } else if (md.op == MUL && is_const(md.a) && !is_const(md.b)) {
                terms.push_back({md.b, sg * nodes_[md.a].val});
            } else if (md.op == CONST) {
                linear = false;  // constant terms: not handled
            } else {
                terms.push_back({m, sg});
            }
        }
        if (!linear || terms.size() < 2) continue;
        std::sort(terms.begin(), terms.end());
        if (!std::isfinite(terms[0].second) || terms[0].second == 0.0) continue;
        const int e = std::ilogb(terms[0].second);
        std::vector<std::pair<uint32_t, double>> key;
        for (const auto &t : terms) {
            if (!std::isfinite(t.second) || t.second == 0.0) {
                key.clear();
                break;
            }
            key.push_back({t.first, std::ldexp(t.second, -e)});
            // the scaled coefficient must be exact
            if (std::ldexp(key.back().second, e) != t.second) {
                key.clear();
                break;
            }
        }
        if (key.empty()) continue;
        auto it = seen.find(key);
        if (it == seen.end()) {
            seen[key] = {r, e};
        } else if (it->second.second != e) {
            nw[n] = mul(constant(std::ldexp(1.0, e - it->second.second)), it->second.first);
        } else {
            nw[n] = it->second.first;
        }
    }
    std::vector<uint32_t> out;
    for (uint32_t x : roots) out.push_back(x == NONE ? NONE : nw[x]);
    return out;
}

std::vector<uint32_t> Graph::factor_sums(const std::vector<uint32_t> &roots) {
    const std::vector<uint32_t> order = reachable(roots);
    const size_t N0 = nodes_.size();
    auto is_sum = [&](uint32_t n) {
        const Node &d = nodes_[n];
        return d.op == ADD || d.op == SUB ||
               (d.op == NEG && (nodes_[d.a].op == ADD || nodes_[d.a].op == SUB));
    };
    std::vector<char> top(N0, 0);
    for (uint32_t r : roots)
        if (r != NONE) top[r] = 1;
    for (uint32_t n : order) {
        const Node &d = nodes_[n];
        if (d.op == CONST || d.op == VAR || d.op == PARAM || is_sum(n)) continue;
        if (d.a != NONE) top[d.a] = 1;
        if (d.b != NONE) top[d.b] = 1;
    }
    const size_t kMaxTerms = 4096;  // a sum of shared sums could double at every level
    std::vector<size_t> tsize(N0, 1);
    for (uint32_t n : order) {
        const Node &d = nodes_[n];
        if (d.op == ADD || d.op == SUB) tsize[n] = std::min(kMaxTerms + 1, tsize[d.a] + tsize[d.b]);
        else if (is_sum(n)) tsize[n] = tsize[d.a];
    }
    // a symbol is (node or kVirtual | pair index) * 2 + (1 if negated)
    const uint64_t kVirtual = 0x80000000ull;
    struct Sum {
        uint32_t node;
        double c;                   // folded constant terms
        std::vector<uint64_t> sym;  // signed terms
    };
    std::vector<Sum> sums;
    std::vector<int> sum_of(N0, -1);
    for (uint32_t n : order) {
        if (!is_sum(n) || !top[n]) continue;
        if (tsize[n] > kMaxTerms) return roots;  // leave such graphs alone
        Sum S{n, 0.0, {}};
        std::vector<std::pair<uint32_t, int>> stack{{n, 1}};
        while (!stack.empty()) {
            const auto [m, sg] = stack.back();
            stack.pop_back();
            const Node &d = nodes_[m];
            if (d.op == ADD) {
                stack.push_back({d.b, sg});
                stack.push_back({d.a, sg});
            } else if (d.op == SUB) {
                stack.push_back({d.b, -sg});
                stack.push_back({d.a, sg});
            } else if (d.op == NEG && is_sum(m)) {
                stack.push_back({d.a, -sg});
            } else if (d.op == CONST) {
                S.c += sg * d.val;
            } else {
                S.sym.push_back((uint64_t)m * 2 + (sg < 0 ? 1 : 0));
            }
        }
        std::sort(S.sym.begin(), S.sym.end());
        sum_of[n] = (int)sums.size();
        sums.push_back(std::move(S));
    }
    // greedy pairing of terms; a pair and its negation are the same node
    // (key: first term positive), each occurrence keeps its overall sign
    auto id_of = [](uint64_t s) { return s >> 1; };
    auto neg_of = [](uint64_t s) { return (s & 1) != 0; };
    struct Pair {
        uint64_t a, b;  // a positive
    };
    std::vector<Pair> pairs;
    auto key = [&](uint64_t x, uint64_t y) {
        if (id_of(y) < id_of(x) || (id_of(y) == id_of(x) && y < x)) std::swap(x, y);
        const bool flip = neg_of(x);
        if (flip) {
            x ^= 1;
            y ^= 1;
        }
        return std::make_pair(std::make_pair(x, y), flip);
    };
    for (;;) {
        std::map<std::pair<uint64_t, uint64_t>, int> count;
        for (const Sum &S : sums) {
            std::set<std::pair<uint64_t, uint64_t>> here;
            for (size_t i = 0; i < S.sym.size(); i++)
                for (size_t j = i + 1; j < S.sym.size(); j++) here.insert(key(S.sym[i], S.sym[j]).first);
            for (const auto &pr : here) count[pr]++;
        }
        std::pair<uint64_t, uint64_t> best{0, 0};
        int bc = 1;
        for (const auto &kv : count)
            if (kv.second > bc) {
                bc = kv.second;
                best = kv.first;
            }
        if (bc < 2) break;
        const uint64_t v = (kVirtual | pairs.size()) * 2;
        pairs.push_back(Pair{best.first, best.second});
        for (Sum &S : sums) {
            // every disjoint occurrence (x + y + x + y holds the pair twice)
            for (bool found = true; found;) {
                found = false;
                for (size_t i = 0; i < S.sym.size() && !found; i++)
                    for (size_t j = i + 1; j < S.sym.size() && !found; j++) {
                        const auto k = key(S.sym[i], S.sym[j]);
                        if (k.first != best) continue;
                        S.sym.erase(S.sym.begin() + j);
                        S.sym.erase(S.sym.begin() + i);
                        S.sym.push_back(v | (k.second ? 1 : 0));
                        found = true;
                    }
            }
            std::sort(S.sym.begin(), S.sym.end());
        }
    }
    std::vector<uint32_t> nw(N0, NONE), vnew(pairs.size(), NONE);
    std::function<uint32_t(uint64_t)> get_abs = [&](uint64_t s) -> uint32_t {
        const uint64_t id = id_of(s);
        if (!(id & kVirtual)) return nodes_[id].op == CONST ? (uint32_t)id : nw[id];
        const size_t i = (size_t)(id & ~kVirtual);
        if (vnew[i] == NONE) {
            const Pair &P = pairs[i];
            const uint32_t a = get_abs(P.a), b = get_abs(P.b);
            vnew[i] = neg_of(P.b) ? sub(a, b) : add(a, b);
        }
        return vnew[i];
    };
    for (uint32_t n : order) {
        const Node d = nodes_[n];
        if (d.op == CONST || d.op == VAR || d.op == PARAM) {
            nw[n] = n;
            continue;
        }
        if (is_sum(n)) {
            if (sum_of[n] < 0) continue;  // folded into its consumers
            const Sum &S = sums[sum_of[n]];
            // equal terms are combined first: m x is one scaled term (an fma
            // in an accumulation) instead of m additions
            std::map<uint64_t, long> mult;
            std::vector<uint64_t> ids;
            for (uint64_t s2 : S.sym) {
                const uint64_t id = id_of(s2);
                if (!mult.count(id)) ids.push_back(id);
                mult[id] += neg_of(s2) ? -1 : 1;
            }
            uint32_t acc = NONE;
            for (uint64_t id : ids) {
                const long m = mult[id];
                if (m == 0) continue;
                uint32_t t = get_abs(id << 1);
                const bool ng = m < 0;
                if (m != 1 && m != -1) t = mul(constant((double)(ng ? -m : m)), t);
                if (acc == NONE) acc = ng ? neg(t) : t;
                else acc = ng ? sub(acc, t) : add(acc, t);
            }
            if (S.c != 0.0) acc = acc == NONE ? constant(S.c) : add(constant(S.c), acc);
            nw[n] = acc == NONE ? constant(0.0) : acc;
            continue;
        }
        const uint32_t a = d.a != NONE ? nw[d.a] : NONE, b = d.b != NONE ? nw[d.b] : NONE;
        switch (d.op) {
        case MUL: nw[n] = mul(a, b); break;
        case DIV: nw[n] = div(a, b); break;
        case NEG: nw[n] = neg(a); break;
        case POWI: nw[n] = powi(a, d.aux); break;
        case SPLINE: nw[n] = spline((uint32_t)d.val, d.aux / 4, d.aux % 4, a, b); break;
        default: nw[n] = unary(d.op, a); break;
        }
    }
    std::vector<uint32_t> out(roots.size(), NONE);
    for (size_t i = 0; i < roots.size(); i++) out[i] = roots[i] == NONE ? NONE : nw[roots[i]];
    return out;
}

// -------------------------------------------------------------- evaluate ---

void bspline_weights(int order, double u, double w[4]) {
    double v = 1.0 - u;
    switch (order) {
    case 0:
        w[0] = v * v * v / 6.0;
        w[1] = (3.0 * u * u * u - 6.0 * u * u + 4.0) / 6.0;
        w[2] = (-3.0 * u * u * u + 3.0 * u * u + 3.0 * u + 1.0) / 6.0;
        w[3] = u * u * u / 6.0;
        break;
    case 1:
        w[0] = -v * v / 2.0;
        w[1] = (3.0 * u * u - 4.0 * u) / 2.0;
        w[2] = (-3.0 * u * u + 2.0 * u + 1.0) / 2.0;
        w[3] = u * u / 2.0;
        break;
    case 2:
        w[0] = v; w[1] = 3.0 * u - 2.0; w[2] = 1.0 - 3.0 * u; w[3] = u;
        break;
    default:
        w[0] = -1.0; w[1] = 3.0; w[2] = -3.0; w[3] = 1.0;
        break;
    }
}

void bspline_cell(double x, double lo, double hi, uint32_t n, int *m, double *u, double *invh) {
    *invh = (double)(n - 3) / (hi - lo);
    double s = (x - lo) * *invh + 1.0;
    double fm = std::floor(s);
    fm = std::min(std::max(fm, 1.0), (double)(n - 3));
    *m = (int)fm;
    *u = s - fm;
}

double Graph::eval(uint32_t f, const double *x, const double *k, double omega, double t,
                   const double *const *params, const double *seeds) const {
    std::vector<uint32_t> order = reachable({f});
    std::unordered_map<uint32_t, double> v;
    v.reserve(order.size() * 2);
    for (uint32_t n : order) {
        const Node &nd = nodes_[n];
        double r = 0.0;
        switch (nd.op) {
        case CONST: r = nd.val; break;
        case VAR: {
            int kind = nd.aux / 8, i = nd.aux % 8;
            r = kind == VK_X ? x[i] : kind == VK_K ? k[i] : kind == VK_OMEGA ? omega
                : kind == VK_T ? t : (seeds ? seeds[i] : 0.0);
            break;
        }
        case PARAM: {
            const double *p = params ? params[nd.aux] : nullptr;
            if (!p) throw std::invalid_argument("parameter value missing");
            r = p[(size_t)nd.val];
            break;
        }
        case SPLINE: {
            const SplineDef &s = splines_[(size_t)nd.val];
            const double *c = params ? params[s.param] : nullptr;
            if (!c) throw std::invalid_argument("spline coefficients missing");
            int mx, my;
            double ux, uy, ihx, ihy, wx[4], wy[4];
            bspline_cell(v[nd.a], s.lo[0], s.hi[0], s.nx, &mx, &ux, &ihx);
            bspline_cell(v[nd.b], s.lo[1], s.hi[1], s.ny, &my, &uy, &ihy);
            int du = nd.aux / 4, dv = nd.aux % 4;
            bspline_weights(du, ux, wx);
            bspline_weights(dv, uy, wy);
            double acc = 0.0;
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++)
                    acc += c[(size_t)(mx - 1 + a) * s.ny + (my - 1 + b)] * wx[a] * wy[b];
            for (int i = 0; i < du; i++) acc *= ihx;
            for (int i = 0; i < dv; i++) acc *= ihy;
            r = acc;
            break;
        }
        case POWI: r = fold(POWI, v[nd.a], 0.0, nd.aux); break;
        default:
            r = fold(nd.op, v[nd.a], nd.b != NONE ? v[nd.b] : 0.0, nd.aux);
        }
        v[n] = r;
    }
    return v[f];
}

// ------------------------------------------------------------- rendering ---

std::string Graph::to_string(uint32_t n) const {
    const Node &nd = nodes_[n];
    std::ostringstream os;
    os.precision(17);
    auto s = [this](uint32_t m) { return to_string(m); };
    static const char *vn[] = {"x", "k", "omega", "t", "v"};
    switch (nd.op) {
    case CONST: os << nd.val; break;
    case VAR: {
        int kind = nd.aux / 8, i = nd.aux % 8;
        os << vn[kind];
        if (kind == VK_X || kind == VK_K || kind == VK_SEED) os << i;
        break;
    }
    case PARAM: os << params_[nd.aux].name << "[" << (size_t)nd.val << "]"; break;
    case ADD: os << "(" << s(nd.a) << " + " << s(nd.b) << ")"; break;
    case SUB: os << "(" << s(nd.a) << " - " << s(nd.b) << ")"; break;
    case MUL: os << "(" << s(nd.a) << "*" << s(nd.b) << ")"; break;
    case DIV: os << "(" << s(nd.a) << "/" << s(nd.b) << ")"; break;
    case NEG: os << "(-" << s(nd.a) << ")"; break;
    case EXP: os << "exp(" << s(nd.a) << ")"; break;
    case LOG: os << "log(" << s(nd.a) << ")"; break;
    case SQRT: os << "sqrt(" << s(nd.a) << ")"; break;
    case SIN: os << "sin(" << s(nd.a) << ")"; break;
    case COS: os << "cos(" << s(nd.a) << ")"; break;
    case POWI: os << "(" << s(nd.a) << ")^" << nd.aux; break;
    case SPLINE:
        os << "spline" << (size_t)nd.val << "_d" << nd.aux / 4 << nd.aux % 4 << "(" << s(nd.a)
           << ", " << s(nd.b) << ")";
        break;
    }
    return os.str();
}

}  // namespace rg
