/*
 * raygraph: compiled expression graphs for geometric-optics ray tracing on
 * AMD Instinct MI355X (gfx950), FP64.
 *
 * The paper (graph_framework, arXiv 2508.15967) builds an application in
 * three moves: build an expression graph, JIT-compile kernels from it, and
 * run the kernels in a workflow ("Software description").  For ray tracing
 * the graph is a dispersion relation D(x, k, omega); automatic
 * differentiation of D gives the ray equations (eqs. 2-3)
 *
 *     dx/dt = -(dD/dk)/(dD/domega),   dk/dt = (dD/dx)/(dD/domega),
 *
 * and the kernel advances x, k and t of every ray with 4th-order Runge-Kutta
 * ("Impact" section).  This library exposes exactly those moves as a C ABI:
 *
 *   rg_create_graph / rg_node_*      build D (hash-consed, reduced on the fly)
 *   rg_compile                        differentiate, emit HIP, hipRTC -> gfx950
 *   rg_trace_rays                     integrate many rays on the GPU
 *   rg_trace_rays_adjoint             gradients of a loss on ray endpoints
 *
 * Conventions for every entry point
 *   - Every function returns rg_status.  RG_OK is 0; errors are negative and
 *     leave a thread-local message readable with rg_last_error().
 *   - Handles (rg_graph, rg_program) are owned by the library and released
 *     with the matching rg_destroy_* call.  A handle is not thread-safe:
 *     use one per host thread (the paper keeps one workflow manager per
 *     thread/device).
 *   - Device arrays passed to rg_trace_rays* are FP64 (int32 where stated),
 *     contiguous, owned by the caller and resident on the current HIP
 *     device.  The library never frees or retains them past the stream work
 *     of the call.  Ray arrays are structure-of-arrays: component c of ray r
 *     of an array declared [dim][n] is at index c*n + r.
 *   - Trace calls enqueue work on the caller's hipStream_t (passed as void*)
 *     and return without synchronising.  Argument, compile and launch errors
 *     are reported synchronously; device faults surface at the caller's next
 *     synchronisation.  Per-ray numerical trouble (a non-finite state, a step
 *     underflow) is not an API error: it is reported in status_out.
 *   - C++ exceptions never cross this boundary.
 *   - The library must use the same HIP runtime instance as the caller that
 *     owns the streams and memory: load it after that runtime (for PyTorch,
 *     after importing torch, which ships its own libamdhip64).
 */
#ifndef RAYGRAPH_H
#define RAYGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rg_status;
enum {
    RG_OK = 0,
    RG_EINVAL = -1,        /* bad argument (null, out of range, wrong node kind) */
    RG_ENOMEM = -2,        /* host or device allocation failed */
    RG_ECOMPILE = -3,      /* hipRTC rejected the generated source; log in rg_last_error */
    RG_EHIP = -4,          /* a HIP runtime call failed */
    RG_EUNSUPPORTED = -5,  /* valid request this build does not implement */
    RG_ESTATE = -6         /* call out of order (e.g. adjoint without forward data) */
};

typedef struct rg_graph rg_graph;
typedef struct rg_program rg_program;
/* A node is an index into its graph, valid for the graph's lifetime. */
typedef uint32_t rg_node;

/* Variables every ray graph has (kernel inputs, "Impact" section). */
enum { RG_X = 0, RG_K = 1, RG_OMEGA = 2, RG_T = 3 };
/* Operations (graph node kinds built by the factories). */
enum { RG_NEG = 0, RG_EXP = 1, RG_LOG = 2, RG_SQRT = 3, RG_SIN = 4, RG_COS = 5 };
enum { RG_ADD = 0, RG_SUB = 1, RG_MUL = 2, RG_DIV = 3 };
/* Node introspection kinds (rg_node_desc.op). */
enum {
    RG_OP_CONST = 0, RG_OP_VAR = 1, RG_OP_PARAM = 2, RG_OP_ADD = 3, RG_OP_SUB = 4,
    RG_OP_MUL = 5, RG_OP_DIV = 6, RG_OP_NEG = 7, RG_OP_EXP = 8, RG_OP_LOG = 9,
    RG_OP_SQRT = 10, RG_OP_SIN = 11, RG_OP_COS = 12, RG_OP_POWI = 13, RG_OP_SPLINE = 14
};
enum { RG_RK4 = 0, RG_DOPRI54 = 1 };
enum { RG_PERSISTENT = 0, RG_PLAIN = 1 };
enum { RG_FP64 = 0, RG_FP32 = 1 };
/* Per-ray termination status. */
enum {
    RG_RAY_OK = 0,            /* ran all steps (RK4) or reached t_end */
    RG_RAY_EXITED_BOX = 1,    /* first state strictly outside [box_lo, box_hi] */
    RG_RAY_BUDGET = 2,        /* accepted-step budget (or 4x that in attempts) used up */
    RG_RAY_NONFINITE = 3,     /* a step produced a non-finite state; last finite state kept */
    RG_RAY_STEP_UNDERFLOW = 4 /* adaptive step fell below hmin */
};

/* ---------------------------------------------------------------- graph -- */

/* Create a graph for rays in `dim` (2 or 3) space dimensions.  The graph
 * pre-declares the variables x[dim], k[dim], omega and t.  Nodes are built by
 * factories that hash-cons (an identical sub-graph returns the existing node)
 * and reduce on construction (constant folding, x+0, x*1, x*0 ...), as the
 * paper's Graph section describes. */
rg_status rg_create_graph(uint32_t dim, rg_graph **out);
rg_status rg_destroy_graph(rg_graph *g);

/* which = RG_X or RG_K with i < dim, or RG_OMEGA / RG_T with i = 0. */
rg_status rg_node_var(rg_graph *g, int32_t which, uint32_t i, rg_node *out);
rg_status rg_node_const(rg_graph *g, double v, rg_node *out);
/* Declare a differentiable parameter array of `len` doubles (device-resident
 * at trace time, passed in rg_trace_desc.params in declaration order).  *out
 * receives the parameter's index (0, 1, ...), not a node. */
rg_status rg_node_param(rg_graph *g, const char *name, uint32_t len, uint32_t *param_out);
/* Scalar element `idx` of parameter `param` as a node. */
rg_status rg_node_elem(rg_graph *g, uint32_t param, uint32_t idx, rg_node *out);
rg_status rg_node_unary(rg_graph *g, int32_t op, rg_node a, rg_node *out);
rg_status rg_node_binary(rg_graph *g, int32_t op, rg_node a, rg_node b, rg_node *out);
/* a^n for integer n (n = 0 gives 1). */
rg_status rg_node_powi(rg_graph *g, rg_node a, int32_t n, rg_node *out);
/* Piecewise-polynomial node (the paper's piecewise constants used to build
 * spline interpolation): uniform tensor cubic B-spline with nx*ny
 * coefficients taken from parameter `coeff_param` (x index major, length
 * nx*ny, nx, ny >= 4) over [lo[0],hi[0]] x [lo[1],hi[1]], evaluated at
 * (u, v).  Knot spacing h = (hi-lo)/(n-3); coefficient i sits at
 * lo + (i-1) h; outside the domain the edge cell's cubic is extended. */
rg_status rg_node_bspline2(rg_graph *g, uint32_t coeff_param, uint32_t nx, uint32_t ny,
                           const double lo[2], const double hi[2], rg_node u, rg_node v,
                           rg_node *out);

/* Symbolic derivative d f / d wrt (the df method: chain rule per node;
 * constants give 0, a variable gives 1 with respect to itself).  wrt may be
 * a variable, a parameter element or any other node (then treated as a
 * leaf). */
rg_status rg_df(rg_graph *g, rg_node f, rg_node wrt, rg_node *out);

typedef struct {
    int32_t op;          /* RG_OP_* */
    int32_t aux;         /* VAR: which*8+i; PARAM: param index; POWI: exponent;
                            SPLINE: derivative orders du*4+dv */
    rg_node a, b;        /* operands (UINT32_MAX if absent) */
    double value;        /* CONST value; PARAM element index */
} rg_node_desc;
rg_status rg_node_get(const rg_graph *g, rg_node n, rg_node_desc *out);
rg_status rg_graph_size(const rg_graph *g, uint32_t *n_nodes);

/* CPU evaluation of node f at one point (host pointers): x[dim], k[dim],
 * params[p] -> host array of parameter p (may be NULL if unused).  Used by
 * constant folding and by tests; never by the ray kernels. */
rg_status rg_eval(const rg_graph *g, rg_node f, const double *x, const double *k,
                  double omega, double t, const double *const *params, double *out);

/* Infix rendering of a node (debug aid).  Writes at most cap bytes
 * (NUL-terminated) and the full length to *needed. */
rg_status rg_node_to_string(const rg_graph *g, rg_node n, char *buf, size_t cap,
                            size_t *needed);

/* -------------------------------------------------------------- compile -- */

typedef struct {
    uint32_t struct_size;   /* sizeof(rg_compile_opts) */
    int32_t want_adjoint;   /* also build the vector-Jacobian product and adjoint kernels */
    int32_t compile_only;   /* 1: emit + hipRTC compile but do not load a module
                               (works without a GPU) */
    int32_t opt_level;      /* hipRTC -O level, 0 = default (3) */
    const char *arch;       /* NULL = "gfx950" */
    int32_t fp32;           /* 1: also emit a single precision right-hand side and
                               build the RG_FP32 persistent RK4 kernel (graphs
                               without spline nodes; RG_EUNSUPPORTED otherwise) */
    int32_t deterministic;  /* 1: the adjoint sums spline-coefficient gradients in
                               a fixed order, so that they are bitwise the same
                               from run to run for a given launch configuration
                               (each wave accumulates into its own copy of the
                               table in the workspace, the copies summed in wave
                               order; slower and more workspace).  Without it
                               those sums go through shared LDS atomics whose
                               order varies at the rounding level.  Scalar
                               parameter gradients are summed in a fixed order
                               either way. */
} rg_compile_opts;

/* Differentiate D (eqs. 2-3), reduce and CSE, emit the HIP right-hand side
 * (one reciprocal of dD/domega shared by all components, explicit fma), the
 * D residual and, if asked, the VJP; splice them into the integrator
 * kernels and compile for gfx950 with hipRTC.  The graph must outlive
 * nothing: the program keeps its own copy of what it needs.  A failed
 * hipRTC compile returns RG_ECOMPILE with the compiler log in
 * rg_last_error().  Code objects are cached by generated source, compile
 * options and hipRTC version, in the process and, if the environment
 * variable RAYGRAPH_CODE_CACHE names a directory, on disk there. */
rg_status rg_compile(rg_graph *g, rg_node D, const rg_compile_opts *opts, rg_program **out);
rg_status rg_destroy_program(rg_program *p);

typedef struct {
    uint32_t struct_size;
    uint32_t dim;
    uint32_t n_params;          /* declared parameter arrays */
    uint32_t n_grad_slots;      /* scalar parameter elements that receive gradients */
    uint32_t n_nodes_rhs;       /* emitted operations of the right-hand side */
    uint32_t n_nodes_vjp;       /* emitted operations of the VJP (0 without adjoint) */
    /* flops counted from the emitted operations: "alg" counts add, sub, mul,
       div, sqrt, exp, log, sin, cos as 1 and fma as 2; "issued" weights each
       operation by the FP64 add/mul/fma flops of its gfx950 instruction
       expansion */
    double rhs_flops_alg, rhs_flops_issued;       /* one right-hand side */
    double rk4_step_flops_alg, rk4_step_flops_issued; /* one RK4 step (4 RHS + update) */
    double dopri_attempt_flops_alg, dopri_attempt_flops_issued; /* 6 RHS + update/error */
    double vjp_flops_alg, vjp_flops_issued;       /* one VJP */
    double adj_step_flops_alg, adj_step_flops_issued; /* reverse of one RK4 step incl. recompute */
    uint64_t source_hash;
    double compile_ms;
    /* flops ("alg") of operations on values that depend only on constants,
       parameters and omega: invariant along a ray, computed once per ray by
       the integrator loops and excluded from the per-evaluation counts above */
    double rhs_flops_ray_invariant, vjp_flops_ray_invariant;
} rg_program_info;
rg_status rg_program_info_get(const rg_program *p, rg_program_info *out);
/* Borrowed pointer to the full generated HIP source; valid while p lives. */
rg_status rg_program_source(const rg_program *p, const char **src);
/* Borrowed pointer to just the emitted device functions (rhs, D, vjp);
 * they are plain C++ apart from the RG_FN qualifier macro. */
rg_status rg_program_functions(const rg_program *p, const char **src);

/* ---------------------------------------------------------------- trace -- */

typedef struct {
    uint32_t struct_size;       /* sizeof(rg_trace_desc) */
    uint32_t n_rays;
    /* inputs (device) */
    const double *x0, *k0;      /* [dim][n] */
    const double *t0;           /* [n], NULL = 0 */
    const double *omega;        /* [n] */
    const double *const *params;/* host array of n_params device pointers */
    /* integrator */
    int32_t integrator;         /* RG_RK4 | RG_DOPRI54 */
    int32_t n_steps;            /* RK4: number of steps */
    double dt;                  /* RK4: step */
    double h0, rtol, atol, hmin;/* DOPRI54 */
    double t_end;               /* DOPRI54: stop at t_end when > 0 */
    const int32_t *budget;      /* DOPRI54: [n] accepted-step budget, NULL = max_steps */
    int32_t max_steps;          /* DOPRI54 budget when budget == NULL */
    int32_t has_box;            /* terminate on leaving [box_lo, box_hi] */
    double box_lo[3], box_hi[3];
    /* outputs (device) */
    int32_t store_every;        /* RK4: snapshot every this many steps, 0 = none */
    double *traj;               /* [n_snap][2*dim][n], n_snap = n_steps/store_every + 1 */
    double *traj_D;             /* [n_snap][n] D residual at each snapshot, nullable */
    double *x_out, *k_out;      /* [dim][n] */
    double *t_out;              /* [n] nullable */
    int32_t *status_out;        /* [n] nullable */
    int32_t *steps_out;         /* [n] accepted steps, nullable */
    int32_t checkpoint_every;   /* RK4: store states every this many steps for the adjoint */
    double *checkpoints;        /* [n_ckpt][2*dim][n], n_ckpt = ceil(n_steps/checkpoint_every) */
    /* execution */
    int32_t mode;               /* RG_PERSISTENT | RG_PLAIN (one launch per step) */
    int32_t use_hipgraph;       /* replay the launch sequence from a captured hipGraph */
    int32_t block;              /* threads per workgroup, 0 = tuned */
    int32_t rays_per_lane;      /* 1 | 2 | 4 (4: right-hand sides under 200 issued
                                   flops), 0 = tuned */
    int32_t compact_interval;   /* DOPRI54: refill dead lanes every this many attempts,
                                   0 = tuned, -1 = only when a whole wave is dead */
    int32_t *attempts_out;      /* DOPRI54: [n] step attempts incl. rejected ones, nullable */
    int32_t precision;          /* RG_FP64, or RG_FP32: state, stages and right-hand
                                   side in single precision (RK4, RG_PERSISTENT, no
                                   checkpoints, program compiled with fp32 = 1); the
                                   arrays stay double, t and the traj_D residual
                                   are computed in double */
    /* per-call device scratch, owned by the caller (a torch tensor): at least
       the bytes rg_workspace_size reports for this description, 8-byte
       aligned, overlapping no other buffer of the call.  NULL is allowed
       when that size is 0 (persistent RK4 needs none).  Its contents on
       entry do not matter; the call's stream work owns it until it ends. */
    void *workspace;
    size_t workspace_bytes;
    int32_t min_waves_per_simd; /* persistent FP64 RK4, one ray per lane: 4 = the
                                   kernel variant built for at least 4 waves per
                                   SIMD (at most 128 VGPRs; same results);
                                   0 = the autotuner's choice when it tunes,
                                   else the plain kernel */
} rg_trace_desc;

/* Trace n_rays rays.  RK4 runs exactly n_steps steps per ray (fewer if it
 * stops, see status); DOPRI54 runs until the box is left, the budget is used
 * or t_end is reached.  Requires a program compiled without compile_only.
 * n_rays = 0 returns RG_OK without touching any ray buffer (they may then
 * be NULL).  No output buffer may overlap an input buffer or another output
 * (RG_EINVAL): the autotuner's sample runs write the outputs first.
 * The library allocates no device memory here: per-call scratch (the
 * Dormand-Prince refill queue, the per-ray state of the one-launch-per-step
 * forms) comes from d->workspace, so calls on different streams with
 * different workspaces do not share state.  A workspace smaller than
 * rg_workspace_size reports is RG_EINVAL. */
rg_status rg_trace_rays(rg_program *p, const rg_trace_desc *d, void *hip_stream);

/* Loads the program's code object on the current device and prepares the
 * device for rg_trace_rays_noalloc (resolves the address of the library's
 * static scratch array there).  Once per device, before the first
 * rg_trace_rays_noalloc on it; the other entry points load on first use. */
rg_status rg_program_load(rg_program *p);

/* rg_trace_rays for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same trace, inputs and outputs as rg_trace_rays (results bitwise equal),
 * but nothing in the call allocates.  Its per-call scratch (the
 * Dormand-Prince refill queue, the per-ray state of the one-launch-per-step
 * forms) comes from a static device array of RG_NOALLOC_SCRATCH_BYTES = 4 MiB
 * per device, held by the library until the process ends; d->workspace is
 * ignored.  Limits and rules:
 *   - rg_program_load must have run on the current device (RG_ESTATE);
 *   - a trace needing more scratch than the array holds is RG_EINVAL
 *     (rg_workspace_size tells: persistent RK4 needs none, persistent
 *     Dormand-Prince 8 bytes, the plain forms 16 (RK4) or 132
 *     (Dormand-Prince, 3-D) bytes per ray);
 *   - launch parameters must be given (block; rays_per_lane for RK4;
 *     compact_interval for Dormand-Prince): no autotuning (RG_EINVAL);
 *   - use_hipgraph must be 0: the launches are issued directly (RG_EINVAL).
 * Every call on a device shares that device's array and leaves its contents
 * behind (what must start at zero is cleared by a kernel inside the call):
 * calls that overlap in time on one device, on any streams, race and give
 * wrong results. */
rg_status rg_trace_rays_noalloc(rg_program *p, const rg_trace_desc *d, void *hip_stream);

/* Device workspace, in bytes, that rg_trace_rays needs for description d
 * (its workspace fields are ignored).  Depends on the integrator, the mode
 * and n_rays; 0 for persistent RK4.  Loads the program's code object on the
 * current device if it is not loaded yet (so it needs a GPU). */
rg_status rg_workspace_size(rg_program *p, const rg_trace_desc *d, size_t *bytes);

typedef struct {
    uint32_t struct_size;       /* sizeof(rg_adjoint_desc) */
    const rg_trace_desc *fwd;   /* the forward description (RK4 only; its own
                                   workspace fields are not used here).  Its
                                   checkpoints and steps_out hold the results of
                                   rg_trace_rays on the same inputs, or
                                   checkpoints is NULL: the forward is then run
                                   again inside this call (same launch form,
                                   checkpoints every fwd->checkpoint_every steps
                                   into the workspace; the caller's outputs are
                                   not written) */
    const double *dL_dx_end;    /* [dim][n] */
    const double *dL_dk_end;    /* [dim][n], nullable = 0 */
    double *dL_dx0;             /* [dim][n], nullable */
    double *dL_dk0;             /* [dim][n], nullable */
    double *const *dL_dparams;  /* host array of n_params device pointers (entries
                                   nullable); overwritten, not accumulated.
                                   The gradient buffers may overlap no other
                                   buffer of the call (RG_EINVAL) */
    /* per-call device scratch owned by the caller: at least the bytes
       rg_adjoint_workspace_size reports (the segment buffer of stage states
       and the per-workgroup gradient partials; with fwd->checkpoints NULL
       also the internal forward's checkpoints and step counts), 8-byte
       aligned, overlapping no other buffer of the call */
    void *workspace;
    size_t workspace_bytes;
} rg_adjoint_desc;

/* Discrete adjoint of the RK4 trajectory (exact transpose of the step map),
 * reverse sweep segment by segment from the forward checkpoints with the
 * states of each segment recomputed.  Gradients of a loss L whose
 * derivatives at the endpoints are given.  Workgroups hold
 * min(fwd->block, 256) threads (256 when fwd->block is 0).  With
 * fwd->mode == RG_PLAIN the same adjoint runs as one launch per step (the
 * per-step comparator: state and adjoint pass through device memory
 * between launches); results as the persistent form (per-ray gradients
 * bitwise, parameter gradients up to the summation order). */
rg_status rg_trace_rays_adjoint(rg_program *p, const rg_adjoint_desc *d, void *hip_stream);

/* Device workspace, in bytes, that rg_trace_rays_adjoint needs for d (its
 * workspace fields are ignored).  The segment buffer holds, per resident
 * lane of the adjoint launch (not per ray), the states of one checkpoint
 * interval: checkpoint_every x (4 x 2 dim + 1) doubles where the stage
 * states are stored, checkpoint_every x (2 dim + 1) where they are
 * recomputed.  Loads the code object like rg_workspace_size. */
rg_status rg_adjoint_workspace_size(rg_program *p, const rg_adjoint_desc *d, size_t *bytes);

/* Elementwise evaluation of D and the right-hand side at n points (one
 * independent work item per point: inputs -> outputs, no time stepping).
 * y: [2*dim][n], omega: [n], f_out: [2*dim][n] (nullable), D_out: [n]
 * (nullable).  Device pointers. */
rg_status rg_eval_rays(rg_program *p, uint32_t n, const double *y, const double *omega,
                       const double *t, const double *const *params, double *f_out,
                       double *D_out, void *hip_stream);

/* Launch conditions by Newton's method (paper, end of the "Impact" section:
 * omega, x and all but one wavevector component are fixed and the remaining
 * component is found by Newton iteration until |D| < 1e-15; the initial
 * guess selects the branch of the multi-valued dispersion relation).  Each
 * ray iterates k_c <- k_c - D / (dD/dk_c) in its own lane until
 * |D| <= tol or max_iter; the largest final |D| over all rays is reduced
 * into *max_abs_D (the convergence test of the paper's Newton workflow). */
typedef struct {
    uint32_t struct_size;       /* sizeof(rg_solve_desc) */
    uint32_t n_rays;
    const double *x;            /* [dim][n] */
    double *k;                  /* [dim][n]: initial guess in, solution out */
    const double *omega;        /* [n] */
    const double *t;            /* [n], NULL = 0 */
    const double *const *params;/* host array of n_params device pointers */
    int32_t component;          /* index of the k component solved for */
    int32_t max_iter;           /* > 0 */
    double tol;                 /* |D| tolerance, e.g. 1e-15 */
    double *D_out;              /* [n] final D, nullable */
    int32_t *iters_out;         /* [n] iterations used, -1 if not converged, nullable */
    double *max_abs_D;          /* device scalar: max |D| after the solve, nullable */
} rg_solve_desc;
rg_status rg_solve_k(rg_program *p, const rg_solve_desc *d, void *hip_stream);

typedef struct {
    uint32_t struct_size;
    int32_t block, rays_per_lane, compact_interval; /* last configuration used */
    int32_t grid;               /* workgroups launched (persistent) */
    int32_t tuned;              /* 1 if the values came from the autotuner */
    int32_t min_waves_per_simd; /* 4 if the at-least-four-waves RK4 variant ran */
    double last_kernel_ms;      /* device time of the last rg_trace_rays or
                                   rg_trace_rays_adjoint call, from events
                                   recorded around its launches on its stream
                                   (autotuning included on a call that tuned):
                                   -1 while that work has not finished, 0 if
                                   it was not timed (the stream was being
                                   captured, or rg_trace_rays_noalloc) */
} rg_launch_info;
/* Launch configuration and device time of the last call (does not wait). */
rg_status rg_last_launch(const rg_program *p, rg_launch_info *out);

/* Per-trace solver statistics (the diagnostics the paper plots along its
 * rays): reduces a finished trace's per-ray outputs on the GPU into 10
 * caller-owned device counters (uint64) stats_dev:
 *   [0..4] rays ending with each RG_RAY_* status, [5] rays with another
 *   status value, [6] accepted steps summed over rays, [7] attempts summed
 *   (DOPRI54; rejected attempts = [7] - [6]), [8] most accepted steps of one
 *   ray, [9] most attempts of one ray.
 * d is the description the trace ran with; its status_out, steps_out and
 * (DOPRI54) attempts_out are read, NULL ones count as 0.  Enqueued on
 * hip_stream (order it after the trace); the counters are zeroed first. */
rg_status rg_trace_stats(rg_program *p, const rg_trace_desc *d, uint64_t *stats_dev, void *hip_stream);

/* Thread-local message for the last non-OK status on this thread. */
const char *rg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RAYGRAPH_H */
