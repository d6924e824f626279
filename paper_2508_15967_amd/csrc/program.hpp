// Compiled program: generated source, gfx950 code object, kernel handles,
// autotuning results and captured hipGraphs (no device buffers: per-call
// scratch is the caller's workspace).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/raygraph.h"
#include "graph.hpp"
#include "kernels/rg_kargs.h"

// Largest workgroup of the adjoint kernel (its launch bound and the size of
// its per-lane LDS staging).
constexpr int kAdjointBlock = 256;

struct TuneEntry {
    int block = 256, rpl = 1, compact = 64;
    int occ = 0;  // 1: the RK4 kernel variant built for at least 4 waves per SIMD
};

struct GraphEntry {
    std::string key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct rg_program {
    uint32_t dim = 0;
    uint32_t n_params = 0;
    std::vector<uint32_t> param_len;
    bool has_vjp = false;
    bool compile_only = false;
    bool rolled = false;  // RK4 stage loops rolled (RG_ROLL)
    bool has_f32 = false; // single precision RK4 kernel built (RG_HAS_F32)
    bool has_r4 = false;  // four-rays-per-lane RK4 kernel built (RG_HAS_R4)
    bool adj_recompute = false;  // adjoint recomputes stage states (RG_ADJ_RECOMPUTE)
    bool gp_lds = false;  // adjoint gradient partials in LDS, 3 waves per SIMD (RG_GP_LDS)
    bool det_grad = false; // spline-coefficient gradients summed in a fixed order (RG_DET_GRAD)
    // gradient layout
    std::vector<int> grad_param, grad_elem;       // scalar slots
    std::vector<int> spl_param, spl_off, spl_len, spl_ny;
    int spl_total = 0;
    // sources and code
    std::string config_src, functions_src, full_src;
    std::vector<char> code;
    uint64_t hash = 0;
    rg_program_info info{};
    // runtime
    int device = -1;
    int n_cu = 0;
    hipModule_t module = nullptr;
    std::map<std::string, hipFunction_t> kernels;
    std::map<std::string, TuneEntry> tune;
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;
    rg_launch_info last{};
    // events around the last trace or adjoint call's launches (start, stop);
    // ev_state 1: both recorded for that call
    hipEvent_t ev[2] = {nullptr, nullptr};
    int ev_state = 0;

    ~rg_program();
};

namespace rg {
// Thread-local error message handling (capi.cpp).
rg_status fail(rg_status code, const std::string &msg);
// Build sources and compile (program.cpp).
rg_status build_program(Graph &g, uint32_t D, const rg_compile_opts &opts, rg_program *p);
// Runtime (runtime.cpp).
rg_status trace(rg_program *p, const rg_trace_desc &d, hipStream_t s);
rg_status adjoint(rg_program *p, const rg_adjoint_desc &d, hipStream_t s);
rg_status workspace_size(rg_program *p, const rg_trace_desc &d, size_t *bytes);
rg_status program_load(rg_program *p);
rg_status last_kernel_ms(const rg_program *p, double *ms);
rg_status trace_stats(rg_program *p, const rg_trace_desc &d, uint64_t *stats, hipStream_t s);
rg_status trace_noalloc(rg_program *p, const rg_trace_desc &d, hipStream_t s);
rg_status adjoint_workspace_size(rg_program *p, const rg_adjoint_desc &d, size_t *bytes);
rg_status solve_k(rg_program *p, const rg_solve_desc &d, hipStream_t s);
rg_status eval_points(rg_program *p, uint32_t n, const double *y, const double *omega,
                      const double *t, const double *const *params, double *f, double *D,
                      hipStream_t s);
uint64_t fnv1a(const void *data, size_t n, uint64_t h = 1469598103934665603ull);
}  // namespace rg
