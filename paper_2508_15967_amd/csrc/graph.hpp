// Expression graph: a hash-consed arena of nodes, reduced as it is built.
//
// Paper, "Graph" subsection: nodes are made by factory methods, a node cache
// keyed by a hash of the sub-graph returns an existing node instead of a
// duplicate, every construction is reduced (constant folding by evaluation,
// identities such as x+0 -> x, x*1 -> x, x*0 -> 0), and df applies the chain
// rule node by node.  Here a node is a plain record in a vector (not a
// virtual class); operands always have smaller indices than the node, so the
// index order is a topological order.
#pragma once

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

namespace rg {

enum Op : int32_t {
    CONST = 0, VAR = 1, PARAM = 2, ADD = 3, SUB = 4, MUL = 5, DIV = 6, NEG = 7,
    EXP = 8, LOG = 9, SQRT = 10, SIN = 11, COS = 12, POWI = 13, SPLINE = 14
};

constexpr uint32_t NONE = 0xffffffffu;

// Variable kinds (VAR aux = kind*8 + index).
enum VarKind : int32_t { VK_X = 0, VK_K = 1, VK_OMEGA = 2, VK_T = 3, VK_SEED = 4 };

struct Node {
    int32_t op;
    int32_t aux;    // VAR: kind*8+i; PARAM: param index; POWI: exponent; SPLINE: du*4+dv
    uint32_t a, b;  // operands
    double val;     // CONST value; PARAM element index; SPLINE definition index
};

struct ParamDef {
    std::string name;
    uint32_t len;
};

struct SplineDef {
    uint32_t param, nx, ny;
    double lo[2], hi[2];
};

class Graph {
public:
    explicit Graph(uint32_t dim);

    uint32_t dim() const { return dim_; }
    const Node &node(uint32_t i) const { return nodes_[i]; }
    uint32_t size() const { return (uint32_t)nodes_.size(); }
    const std::vector<ParamDef> &params() const { return params_; }
    const std::vector<SplineDef> &splines() const { return splines_; }

    // factories (all hash-consed and reduced)
    uint32_t constant(double v);
    uint32_t var(int32_t kind, uint32_t i);
    uint32_t param_elem(uint32_t param, uint32_t idx);
    uint32_t add(uint32_t a, uint32_t b);
    uint32_t sub(uint32_t a, uint32_t b);
    uint32_t mul(uint32_t a, uint32_t b);
    uint32_t div(uint32_t a, uint32_t b);
    uint32_t neg(uint32_t a);
    uint32_t unary(int32_t op, uint32_t a);  // EXP LOG SQRT SIN COS
    uint32_t powi(uint32_t a, int32_t n);
    uint32_t spline(uint32_t def, int32_t du, int32_t dv, uint32_t u, uint32_t v);

    uint32_t declare_param(const std::string &name, uint32_t len);
    uint32_t declare_spline(const SplineDef &d);

    // d f / d wrt by the chain rule; wrt may be any node (treated as a leaf).
    uint32_t df(uint32_t f, uint32_t wrt);

    // Reverse-mode derivative of s = sum_i seeds[i] * outs[i]: the adjoint
    // ds/dn of every node n that s depends on (NONE where it is zero),
    // indexed by node.
    std::vector<uint32_t> adjoints(const std::vector<uint32_t> &outs,
                                   const std::vector<uint32_t> &seeds);

    // Products re-associated: every maximal product (a MUL or a negated MUL
    // whose value is used by something other than a product, or a root) is
    // flattened into its factors, constant factors are folded into one, the
    // factor pairs that two or more products share are formed once (greedy,
    // most shared pair first) and each product is rebuilt from them.  Other
    // nodes are rebuilt on the new operands.  Returns the roots' new nodes
    // (the old ones stay valid).  Reassociation changes rounding only.
    // With merge_invariants, a second pairing that first makes the
    // ray-invariant factors of each product one factor is tried, and kept
    // if it needs fewer multiplications per evaluation.
    // inv_state: state components (bit c for y[c]) that count as invariant
    // along a ray besides omega, parameters and constants (components whose
    // right-hand side is identically zero).
    std::vector<uint32_t> factor_products(const std::vector<uint32_t> &roots, bool merge_invariants = true,
                                          uint32_t inv_state = 0);

    // The same for sums: every maximal sum (ADD/SUB chains, negations
    // included) is flattened into signed terms, constant terms folded, term
    // pairs shared by two or more sums formed once, and the sums rebuilt
    // (a sum that reappears as a sub-sum of another is then one node, and
    // x + x reduces to 2x).
    std::vector<uint32_t> factor_sums(const std::vector<uint32_t> &roots);

    // Common factors out of sums: every maximal sum is flattened into
    // signed terms, each term into its factors (through products and
    // negations), and the factor found in most terms (two at least) is
    // taken out of those terms, f a + f b -> f (a + b), recursively inside
    // the new sub-sum and repeatedly over the remaining terms.  Sub-sums are
    // built with their terms in a fixed order, so a sub-sum that several
    // sums share under different factors (a directional derivative that the
    // reverse sweep spreads over several adjoints, say) becomes one node.
    // Returns the roots' new nodes; reassociation changes rounding only.
    std::vector<uint32_t> collect_factors(const std::vector<uint32_t> &roots);

    // A sum whose terms are constants times values (or plain values) and
    // that equals an earlier such sum with every coefficient scaled by one
    // power of two (2 M k next to M k, from differentiating k.M k) becomes
    // that sum times the power of two: the same double, one multiplication
    // instead of the sum.  Returns the roots' new nodes.
    std::vector<uint32_t> share_scaled_sums(const std::vector<uint32_t> &roots);

    // A division whose denominator is invariant along a ray (built from
    // omega, parameters and constants only) and whose numerator is not
    // becomes a product with the reciprocal, which the compiler then
    // computes once per ray instead of once per evaluation; a variant
    // denominator that is a product with invariant factors I keeps only
    // its variant part V: a / (I V) = (a / V) (1 / I) (with split_products).
    std::vector<uint32_t> hoist_divisions(const std::vector<uint32_t> &roots, bool split_products = true,
                                          uint32_t inv_state = 0);

    // A variable that does not change along a ray: omega, or a state
    // component whose bit is set in inv_state.
    bool ray_invariant_var(const Node &d, uint32_t inv_state) const {
        const int kind = d.aux / 8, i = d.aux % 8;
        if (kind == VK_OMEGA) return true;
        if (kind == VK_X) return (inv_state >> i) & 1u;
        if (kind == VK_K) return (inv_state >> (dim() + i)) & 1u;
        return false;
    }

    bool is_const(uint32_t n) const { return nodes_[n].op == CONST; }
    bool is_const(uint32_t n, double v) const {
        return nodes_[n].op == CONST && nodes_[n].val == v;
    }

    // Evaluate at one point.  params[p] is a host array (may be null if unused).
    double eval(uint32_t f, const double *x, const double *k, double omega, double t,
                const double *const *params, const double *seeds = nullptr) const;

    std::string to_string(uint32_t n) const;

    // Nodes reachable from `roots`, in increasing (topological) order.
    std::vector<uint32_t> reachable(const std::vector<uint32_t> &roots) const;

private:
    struct Key {
        int32_t op, aux;
        uint32_t a, b;
        uint64_t bits;
        bool operator==(const Key &o) const {
            return op == o.op && aux == o.aux && a == o.a && b == o.b && bits == o.bits;
        }
    };
    struct KeyHash {
        size_t operator()(const Key &k) const;
    };

    uint32_t intern(int32_t op, int32_t aux, uint32_t a, uint32_t b, double val);
    double fold(int32_t op, double a, double b, int32_t aux) const;

    uint32_t dim_;
    std::vector<Node> nodes_;
    std::unordered_map<Key, uint32_t, KeyHash> cache_;
    std::vector<ParamDef> params_;
    std::vector<SplineDef> splines_;
};

// Uniform cubic B-spline helpers shared by graph evaluation (host).
void bspline_weights(int order, double u, double w[4]);
void bspline_cell(double x, double lo, double hi, uint32_t n, int *m, double *u, double *invh);

}  // namespace rg
