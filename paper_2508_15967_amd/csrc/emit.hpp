// Emission of straight-line HIP device functions from the expression graph.
//
// Paper, "JIT" subsection: the kernel body is produced by a recursive
// traversal of the graph that writes one line per node into its own
// register variable, skipping sub-graphs already emitted, with memory loaded
// once at the start and stored once at the end.  Here the traversal is the
// index order of the hash-consed arena (already topological), a multiply
// used only by one add/subtract becomes an explicit fma, and the nodes of a
// B-spline that share a cell share one gather of the 16 coefficients.
#pragma once

#include <string>
#include <vector>

#include "graph.hpp"

namespace rg {

// Operations on values that depend only on constants, parameters and omega
// are invariant along a ray: the integrator loop computes them once per ray,
// so they are counted apart (inv_*) from the work of one evaluation.
struct Flops {
    double alg = 0.0;     // add/sub/mul/div/sqrt/exp/... = 1, fma = 2
    double issued = 0.0;  // FP64 add/mul/fma flops of the gfx950 expansion
    uint32_t ops = 0;     // emitted operations (ray-invariant ones included)
    uint32_t inv_ops = 0; // the ray-invariant ones among them
    double inv_alg = 0.0, inv_issued = 0.0;  // ray-invariant part, not in alg/issued
};

// Issued FP64 flops of one operation's instruction expansion on gfx950
// (fma counted as 2, add/mul as 1; compares, selects, integer and exponent
// manipulation count 0).
struct IssuedWeights {
    double div, exp, log, sqrt, sincos, rcp;
};
const IssuedWeights &issued_weights();

struct Output {
    uint32_t node;
    std::string lhs;   // e.g. "f[0]"
    bool accumulate;   // "+=" instead of "="
};

// A spline coefficient table whose gradient is scattered: for every spline
// node of the table reachable from the function, `seed` gives d(out)/d(node)
// (a node of the same graph).
struct SplineSeed {
    uint32_t spline_node;
    uint32_t seed;
};

struct FunctionSpec {
    std::string signature;  // full function head, up to and including "{"
    std::vector<Output> outputs;
    std::vector<SplineSeed> spline_seeds;  // VJP only
    bool returns_value = false;            // single output via "return"
    bool fp32 = false;                     // single precision (no spline nodes)
    uint32_t inv_state = 0;                // state components constant along a ray (bit c: y[c])
    // FP64 constants that are not inline operands of the instruction set are
    // entered in this table (shared by the functions of a program) and
    // written RG_KV(i, literal): entry i of the table, or the literal where
    // the function's RG_KL flag is set; null: literals only.
    std::vector<double> *const_table = nullptr;
};

// Emit a function.  `tables` maps a spline-definition's parameter to a table
// slot used by the RG_SPL_TAB(slot) accessor; `grad_tables` is the same for
// the gradient accumulator.
std::string emit_function(const Graph &g, const FunctionSpec &spec,
                          const std::vector<int> &param_table_slot, Flops *flops);

std::string hex_double(double v);

}  // namespace rg
