// Runtime: module loading, argument validation, per-call scratch carved
// from the caller's workspace, launch sequences (persistent or
// one-launch-per-step), hipGraph capture and replay, autotuning, and the
// adjoint pass.  No device memory is allocated here: every buffer a launch
// touches is the caller's.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "noalloc.hpp"
#include "program.hpp"

namespace rg {

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(RG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

#define RGCHK(expr)                  \
    do {                             \
        rg_status s_ = (expr);       \
        if (s_ != RG_OK) return s_;  \
    } while (0)

static const char *const KERNELS[] = {
    "rg_rk4_r1", "rg_rk4_r2", "rg_rk4_r1o4", "rg_rk4_r4", "rg_rk4_plain_init", "rg_rk4_plain_step", "rg_plain_finish",
    "rg_dopri_persistent", "rg_dopri_plain_init", "rg_dopri_plain_step", "rg_fill_f64",
    "rg_eval_points", "rg_rk4_adjoint", "rg_grad_finalize", "rg_newton_k", "rg_rk4_f32",
    "rg_adjp_init", "rg_adjp_seg", "rg_adjp_fwd", "rg_adjp_rev", "rg_adjp_finish", "rg_stats"};

static void drop_graphs(rg_program *p) {
    for (GraphEntry &ge : p->graphs) {
        if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
        if (ge.graph) (void)hipGraphDestroy(ge.graph);
    }
    p->graphs.clear();
}

}  // namespace rg

rg_program::~rg_program() {
    rg::drop_graphs(this);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (module) (void)hipModuleUnload(module);
}

namespace rg {

static rg_status ensure_module(rg_program *p) {
    if (p->compile_only) return fail(RG_ESTATE, "program was compiled with compile_only=1");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (p->module && p->device == dev) return RG_OK;
    if (p->module) {
        drop_graphs(p);
        (void)hipModuleUnload(p->module);
        p->module = nullptr;
        p->kernels.clear();
    }
    HIPCHK(hipModuleLoadData(&p->module, p->code.data()));
    for (const char *k : KERNELS) {
        hipFunction_t f = nullptr;
        if (hipModuleGetFunction(&f, p->module, k) == hipSuccess) p->kernels[k] = f;
    }
    (void)hipGetLastError();
    HIPCHK(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    p->device = dev;
    return RG_OK;
}

static rg_status kernel(rg_program *p, const char *name, hipFunction_t *f) {
    auto it = p->kernels.find(name);
    if (it == p->kernels.end()) return fail(RG_EUNSUPPORTED, std::string("kernel not in module: ") + name);
    *f = it->second;
    return RG_OK;
}

// A device pointer must lie inside one device allocation together with the
// `bytes` that follow it; anything else (host memory, a stale pointer, a
// buffer too small for the rays) is rejected before any launch.
static rg_status check_dev(const void *ptr, size_t bytes, const char *what) {
    if (bytes == 0) return RG_OK;  // never touched (zero rays); may be NULL
    if (!ptr) return fail(RG_EINVAL, std::string(what) + " is NULL");
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof at);
    hipError_t e = hipPointerGetAttributes(&at, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RG_EINVAL, std::string(what) + " is not device memory");
    }
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        return fail(RG_EINVAL, std::string(what) + " is not device memory");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RG_EINVAL, std::string(what) + ": cannot query allocation range");
    }
    const char *b = (const char *)base, *q = (const char *)ptr;
    if (q < b || (size_t)(q - b) + bytes > size)
        return fail(RG_EINVAL, std::string(what) + " is smaller than required (" + std::to_string(bytes) + " bytes)");
    if (((uintptr_t)ptr & 7u) != 0) return fail(RG_EINVAL, std::string(what) + " is not 8-byte aligned");
    return RG_OK;
}

// Sub-buffers of the caller's workspace, each starting 256 bytes past a
// multiple of 256 from the workspace base.  With base == nullptr only the
// total size is computed (the pointers handed out are then not used).
struct Carve {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *r = (T *)(base + off);
        off += count * sizeof(T);
        return r;
    }
};

// The workspace must hold `need` bytes (a size query the caller made with
// rg_workspace_size / rg_adjoint_workspace_size) and be device memory.
static rg_status check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (need == 0) return RG_OK;
    if (!ws || ws_bytes < need)
        return fail(RG_EINVAL, "workspace of " + std::to_string(need) + " bytes needed (" +
                                   std::to_string(ws ? ws_bytes : 0) + " given); query it with the workspace-size call");
    return check_dev(ws, need, "workspace");
}

struct Launch {
    const char *name;
    unsigned grid, block;
    rg_kargs a;
};

static rg_status launch_one(rg_program *p, const Launch &L, hipStream_t s) {
    hipFunction_t f;
    RGCHK(kernel(p, L.name, &f));
    if (L.grid == 0) return RG_OK;
    void *args[] = {(void *)&L.a};
    HIPCHK(hipModuleLaunchKernel(f, L.grid, 1, 1, L.block, 1, 1, 0, s, args, nullptr));
    return RG_OK;
}

static std::string seq_key(const std::vector<Launch> &seq) {
    uint64_t h = 1469598103934665603ull;
    for (const Launch &L : seq) {
        h = fnv1a(L.name, std::strlen(L.name), h);
        h = fnv1a(&L.grid, sizeof L.grid, h);
        h = fnv1a(&L.block, sizeof L.block, h);
        h = fnv1a(&L.a, sizeof L.a, h);
    }
    return std::to_string(h) + ":" + std::to_string(seq.size());
}

// Run a launch sequence directly or through a cached hipGraph.
static rg_status run_seq(rg_program *p, const std::vector<Launch> &seq, bool graph, hipStream_t s) {
    if (!graph) {
        for (const Launch &L : seq) RGCHK(launch_one(p, L, s));
        return RG_OK;
    }
    std::string key = seq_key(seq);
    for (GraphEntry &ge : p->graphs)
        if (ge.key == key) {
            HIPCHK(hipGraphLaunch(ge.exec, s));
            return RG_OK;
        }
    if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    rg_status st = RG_OK;
    for (const Launch &L : seq) {
        st = launch_one(p, L, p->cap_stream);
        if (st != RG_OK) break;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != RG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(RG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(RG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (p->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(p->graphs.front().exec);
        (void)hipGraphDestroy(p->graphs.front().graph);
        p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back(GraphEntry{key, g, ex});
    HIPCHK(hipGraphLaunch(ex, s));
    return RG_OK;
}

static unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// Events around a call's launch sequence on the caller's stream, so that
// rg_last_launch can report its device time once it has run.  Not recorded
// while the stream is being captured (the events would become graph nodes)
// or when timing is off (the no-allocation entry point).
static void time_mark(rg_program *p, hipStream_t s, int which) {
    if (which == 0) p->ev_state = 0;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return;
    }
    if (!p->ev[which] && hipEventCreate(&p->ev[which]) != hipSuccess) {
        (void)hipGetLastError();
        p->ev[which] = nullptr;
        return;
    }
    if (hipEventRecord(p->ev[which], s) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (which == 1 && p->ev_state == 0) p->ev_state = 1;
    if (which == 0) p->ev_state = 0;
}

static rg_status occupancy_grid(rg_program *p, const char *name, int block, long long want, unsigned *grid) {
    hipFunction_t f;
    RGCHK(kernel(p, name, &f));
    int nb = 0;
    HIPCHK(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, block, 0));
    if (nb < 1) nb = 1;
    long long cap = (long long)nb * p->n_cu;
    *grid = (unsigned)std::max<long long>(1, std::min(cap, want));
    return RG_OK;
}

// ------------------------------------------------------------ validation --

// Checks d and fills the launch arguments.  ckpt_optional: checkpoints may
// be NULL (the adjoint then runs the forward itself); ws: the workspace the
// call will use (may not overlap any other buffer), ws_bytes its size.
static rg_status validate(rg_program *p, const rg_trace_desc &d, rg_kargs &a, bool ckpt_optional,
                          const void *ws, size_t ws_bytes) {
    const uint32_t dim = p->dim, ny = 2 * dim;
    const size_t n = d.n_rays;
    if (d.struct_size < sizeof(rg_trace_desc)) return fail(RG_EINVAL, "rg_trace_desc.struct_size too small");
    if (d.integrator != RG_RK4 && d.integrator != RG_DOPRI54) return fail(RG_EINVAL, "unknown integrator");
    if (d.mode != RG_PERSISTENT && d.mode != RG_PLAIN) return fail(RG_EINVAL, "unknown mode");
    if (d.block != 0 && d.block != 64 && d.block != 128 && d.block != 256 && d.block != 512)
        return fail(RG_EINVAL, "block must be 0, 64, 128, 256 or 512");
    if (d.rays_per_lane < 0 || d.rays_per_lane > 4 || d.rays_per_lane == 3)
        return fail(RG_EINVAL, "rays_per_lane must be 0, 1, 2 or 4");
    if (d.rays_per_lane == 4 && !p->has_r4)
        return fail(RG_EUNSUPPORTED, "four rays per lane are built only for right-hand sides under 200 issued flops");
    if (d.min_waves_per_simd != 0 && d.min_waves_per_simd != 4)
        return fail(RG_EINVAL, "min_waves_per_simd must be 0 or 4");
    if (d.min_waves_per_simd == 4 && (d.integrator != RG_RK4 || d.mode != RG_PERSISTENT || d.rays_per_lane > 1 ||
                                      d.precision != RG_FP64))
        return fail(RG_EUNSUPPORTED, "min_waves_per_simd = 4 is built for persistent FP64 RK4, one ray per lane");
    if (d.precision != RG_FP64 && d.precision != RG_FP32) return fail(RG_EINVAL, "unknown precision");
    if (d.precision == RG_FP32) {
        if (!p->has_f32) return fail(RG_ESTATE, "RG_FP32 needs a program compiled with fp32 = 1");
        if (d.integrator != RG_RK4 || d.mode != RG_PERSISTENT)
            return fail(RG_EUNSUPPORTED, "RG_FP32 is implemented for persistent RK4");
        if (d.checkpoint_every != 0) return fail(RG_EUNSUPPORTED, "RG_FP32 traces keep no adjoint checkpoints");
        if (d.rays_per_lane > 1) return fail(RG_EUNSUPPORTED, "RG_FP32 runs one ray per lane");
    }
    std::memset(&a, 0, sizeof a);
    a.n = (long long)n;
    a.n_run = (long long)n;
    RGCHK(check_dev(d.x0, 8 * dim * n, "x0"));
    RGCHK(check_dev(d.k0, 8 * dim * n, "k0"));
    RGCHK(check_dev(d.omega, 8 * n, "omega"));
    RGCHK(check_dev(d.x_out, 8 * dim * n, "x_out"));
    RGCHK(check_dev(d.k_out, 8 * dim * n, "k_out"));
    if (d.t0) RGCHK(check_dev(d.t0, 8 * n, "t0"));
    if (d.t_out) RGCHK(check_dev(d.t_out, 8 * n, "t_out"));
    if (d.status_out) RGCHK(check_dev(d.status_out, 4 * n, "status_out"));
    if (d.steps_out) RGCHK(check_dev(d.steps_out, 4 * n, "steps_out"));
    if (p->n_params > 0 && !d.params) return fail(RG_EINVAL, "params is NULL but the graph has parameters");
    for (uint32_t i = 0; i < p->n_params; i++) {
        RGCHK(check_dev(d.params[i], 8 * (size_t)p->param_len[i], "params[i]"));
        a.params[i] = d.params[i];
    }
    a.x0 = d.x0; a.k0 = d.k0; a.t0 = d.t0; a.omega = d.omega;
    a.x_out = d.x_out; a.k_out = d.k_out; a.t_out = d.t_out;
    a.status_out = d.status_out; a.steps_out = d.steps_out;
    a.has_box = d.has_box ? 1 : 0;
    for (int i = 0; i < 3; i++) { a.box_lo[i] = d.box_lo[i]; a.box_hi[i] = d.box_hi[i]; }
    if (d.integrator == RG_RK4) {
        if (d.n_steps < 0) return fail(RG_EINVAL, "n_steps < 0");
        if (!(d.dt == d.dt) || std::isinf(d.dt)) return fail(RG_EINVAL, "dt is not finite");
        a.dt = d.dt;
        a.n_steps = d.n_steps;
        if (d.store_every < 0 || d.checkpoint_every < 0) return fail(RG_EINVAL, "negative store/checkpoint interval");
        if (d.store_every > 0) {
            size_t ns = (size_t)d.n_steps / d.store_every + 1;
            RGCHK(check_dev(d.traj, 8 * ns * ny * n, "traj"));
            if (d.traj_D) RGCHK(check_dev(d.traj_D, 8 * ns * n, "traj_D"));
            a.store_every = d.store_every;
            a.traj = d.traj;
            a.traj_D = d.traj_D;
        }
        if (d.checkpoint_every > 0) {
            size_t nc = ((size_t)d.n_steps + d.checkpoint_every - 1) / d.checkpoint_every;
            if (d.checkpoints || !ckpt_optional)
                RGCHK(check_dev(d.checkpoints, 8 * nc * (ny + 1) * n, "checkpoints"));
            a.ckpt_every = d.checkpoint_every;
            a.ckpt = d.checkpoints;
        }
    } else {
        if (d.store_every != 0 || d.checkpoint_every != 0)
            return fail(RG_EUNSUPPORTED, "snapshots and checkpoints are RK4-only");
        if (!(d.h0 > 0.0) || !(d.rtol >= 0.0) || !(d.atol >= 0.0) || !(d.rtol + d.atol > 0.0))
            return fail(RG_EINVAL, "DOPRI54 needs h0 > 0 and rtol + atol > 0");
        if (d.budget) RGCHK(check_dev(d.budget, 4 * n, "budget"));
        if (d.attempts_out) RGCHK(check_dev(d.attempts_out, 4 * n, "attempts_out"));
        a.attempts_out = d.attempts_out;
        a.budget = d.budget;
        a.max_steps = d.max_steps;
        a.h0 = d.h0; a.rtol = d.rtol; a.atol = d.atol; a.hmin = d.hmin; a.t_end = d.t_end;
    }
    // No output may overlap an input or another output: the autotuner's
    // sample runs write the outputs before the trace reads its inputs.
    struct Range { const void *p; size_t bytes; const char *name; };
    const size_t ns = (d.integrator == RG_RK4 && d.store_every > 0) ? (size_t)(d.n_steps / d.store_every + 1) : 0;
    const size_t nc = (d.integrator == RG_RK4 && d.checkpoint_every > 0)
                          ? (size_t)((d.n_steps + d.checkpoint_every - 1) / d.checkpoint_every) : 0;
    const Range in[] = {{d.x0, 8 * dim * n, "x0"}, {d.k0, 8 * dim * n, "k0"}, {d.t0, 8 * n, "t0"},
                        {d.omega, 8 * n, "omega"},
                        {d.integrator == RG_DOPRI54 ? d.budget : nullptr, 4 * n, "budget"}};
    const Range out[] = {{d.x_out, 8 * dim * n, "x_out"}, {d.k_out, 8 * dim * n, "k_out"},
                         {d.t_out, 8 * n, "t_out"}, {d.status_out, 4 * n, "status_out"},
                         {d.steps_out, 4 * n, "steps_out"},
                         {d.integrator == RG_DOPRI54 ? d.attempts_out : nullptr, 4 * n, "attempts_out"},
                         {ns ? d.traj : nullptr, 8 * ns * 2 * dim * n, "traj"},
                         {ns ? d.traj_D : nullptr, 8 * ns * n, "traj_D"},
                         {nc ? d.checkpoints : nullptr, 8 * nc * (2 * dim + 1) * n, "checkpoints"},
                         {ws, ws_bytes, "workspace"}};
    auto overlap = [](const Range &u, const Range &v) {
        if (!u.p || !v.p || !u.bytes || !v.bytes) return false;
        const char *a0 = (const char *)u.p, *b0 = (const char *)v.p;
        return a0 < b0 + v.bytes && b0 < a0 + u.bytes;
    };
    const size_t n_out = sizeof out / sizeof out[0];
    for (size_t i = 0; i < n_out; i++) {
        for (const Range &r : in)
            if (overlap(out[i], r))
                return fail(RG_EINVAL, std::string(out[i].name) + " overlaps input " + r.name);
        for (size_t j = i + 1; j < n_out; j++)
            if (overlap(out[i], out[j]))
                return fail(RG_EINVAL, std::string(out[i].name) + " overlaps " + out[j].name);
    }
    return RG_OK;
}

// -------------------------------------------------------------- autotune --

static std::string tune_file() {
    const char *e = std::getenv("RAYGRAPH_TUNE_CACHE");
    return e ? std::string(e) : std::string();
}

static void tune_load(rg_program *p) {
    std::string f = tune_file();
    if (f.empty()) return;
    std::ifstream in(f);
    std::string key;
    TuneEntry t;
    while (in >> key >> t.block >> t.rpl >> t.compact >> t.occ) p->tune[key] = t;
}

static void tune_save(const std::string &key, const TuneEntry &t) {
    std::string f = tune_file();
    if (f.empty()) return;
    std::ofstream out(f, std::ios::app);
    out << key << " " << t.block << " " << t.rpl << " " << t.compact << " " << t.occ << "\n";
}

// Fastest of three timed runs after a warm-up run.
static rg_status time_seq(rg_program *p, const std::vector<Launch> &seq, hipStream_t s, float *ms) {
    hipEvent_t e[4];
    for (hipEvent_t &x : e) HIPCHK(hipEventCreate(&x));
    RGCHK(run_seq(p, seq, false, s));  // warm
    HIPCHK(hipEventRecord(e[0], s));
    for (int rep = 0; rep < 3; rep++) {
        RGCHK(run_seq(p, seq, false, s));
        HIPCHK(hipEventRecord(e[rep + 1], s));
    }
    HIPCHK(hipEventSynchronize(e[3]));
    *ms = 1e30f;
    for (int rep = 0; rep < 3; rep++) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, e[rep], e[rep + 1]));
        *ms = std::min(*ms, t);
    }
    for (hipEvent_t &x : e) (void)hipEventDestroy(x);
    return RG_OK;
}

// A candidate within this factor of the fastest counts as equally fast
// (repeated sample timings agree within about 0.5 %).
static constexpr float kTuneTolerance = 1.015f;

// Keyed by program, integrator, ray count (power of two below it), the
// device's architecture name and CU count, and the hipRTC version.
static std::string tune_key(rg_program *p, const char *what, long long n) {
    int lg = 0;
    while ((1ll << (lg + 1)) <= n) lg++;
    int rtc_major = 0, rtc_minor = 0;
    hiprtcVersion(&rtc_major, &rtc_minor);
    std::string arch = "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');  // drop feature suffixes (":sramecc+:xnack-")
        if (colon != std::string::npos) arch.resize(colon);
    } else {
        (void)hipGetLastError();
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "%016llx|%s|n2^%d|cu%d|%s|hiprtc%d.%d", (unsigned long long)p->hash, what,
                  lg, p->n_cu, arch.c_str(), rtc_major, rtc_minor);
    return buf;
}

static rg_status persistent_rk4_seq(rg_program *p, const rg_kargs &a, int block, int rpl,
                                    std::vector<Launch> &seq, bool fp32 = false, int occ = 0) {
    const char *name = fp32 ? "rg_rk4_f32" : rpl == 4 ? "rg_rk4_r4" : rpl == 2 ? "rg_rk4_r2"
                                                     : occ ? "rg_rk4_r1o4" : "rg_rk4_r1";
    unsigned grid;
    RGCHK(occupancy_grid(p, name, block, (long long)cdiv(a.n_run, (long long)block * rpl), &grid));
    seq.push_back(Launch{name, grid, (unsigned)block, a});
    p->last.grid = (int)grid;
    return RG_OK;
}

// a.queue: the refill counter in the caller's workspace (carve_trace)
static rg_status dopri_seq(rg_program *p, rg_kargs a, int block, int compact, std::vector<Launch> &seq) {
    a.compact = compact;
    rg_kargs f;
    std::memset(&f, 0, sizeof f);
    f.fill_p = (double *)a.queue;
    f.fill_n = 1;
    f.fill_v = 0.0;
    seq.push_back(Launch{"rg_fill_f64", 1, 64, f});
    unsigned grid;
    RGCHK(occupancy_grid(p, "rg_dopri_persistent", block, (long long)cdiv(a.n_run, block), &grid));
    seq.push_back(Launch{"rg_dopri_persistent", grid, (unsigned)block, a});
    p->last.grid = (int)grid;
    return RG_OK;
}

static rg_status tune_rk4(rg_program *p, const rg_kargs &a, hipStream_t s, TuneEntry *out, bool fp32) {
    std::string key = tune_key(p, fp32 ? "rk4f32" : "rk4", a.n);
    if (p->tune.empty()) tune_load(p);
    auto it = p->tune.find(key);
    if (it != p->tune.end()) { *out = it->second; p->last.tuned = 1; return RG_OK; }
    // a shortened run of the real launch, stores included (they write the
    // caller's first snapshots and checkpoints, which the run that follows
    // overwrites): long enough to rank the candidates above timer noise
    // Candidates in order of preference: among those within the tolerance
    // of the fastest (run-to-run noise), the first is taken, so near-equal
    // configurations do not flip from one process to the next.
    rg_kargs t = a;
    t.n_steps = std::min(a.n_steps, std::max(128, std::min(1024, a.n_steps / 16)));
    // (rays per lane, block, at-least-four-waves variant).  The variant
    // comes first where it is more occupancy for free (fewer registers than
    // the plain kernel and no spill), else last, so that it is taken only
    // where it is faster beyond the tolerance.
    struct Cand { int rpl, block, occ; };
    std::vector<Cand> cand = {{1, 256, 0}, {1, 512, 0}, {1, 128, 0}, {2, 256, 0}, {2, 128, 0}, {1, 64, 0},
                              {2, 512, 0}, {2, 64, 0}, {4, 128, 0}, {4, 256, 0}};
    bool occ_free = false;
    if (!fp32) {
        hipFunction_t f1, f4;
        int r1 = 0, r4 = 0, spill = 1;
        if (kernel(p, "rg_rk4_r1", &f1) == RG_OK && kernel(p, "rg_rk4_r1o4", &f4) == RG_OK &&
            hipFuncGetAttribute(&r1, HIP_FUNC_ATTRIBUTE_NUM_REGS, f1) == hipSuccess &&
            hipFuncGetAttribute(&r4, HIP_FUNC_ATTRIBUTE_NUM_REGS, f4) == hipSuccess &&
            hipFuncGetAttribute(&spill, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, f4) == hipSuccess)
            occ_free = r4 < r1 && spill == 0;
        (void)hipGetLastError();
    }
    const std::vector<Cand> o4 = {{1, 256, 1}, {1, 512, 1}};
    cand.insert(occ_free ? cand.begin() : cand.end(), o4.begin(), o4.end());
    std::vector<float> ms_of;
    for (const Cand &c : cand) {
        float ms = 1e30f;
        const bool ok = !(fp32 && (c.rpl > 1 || c.occ)) && !(c.rpl == 4 && !p->has_r4);
        if (ok) {
            std::vector<Launch> seq;
            RGCHK(persistent_rk4_seq(p, t, c.block, c.rpl, seq, fp32, c.occ));
            RGCHK(time_seq(p, seq, s, &ms));
        }
        ms_of.push_back(ms);
    }
    const float best = *std::min_element(ms_of.begin(), ms_of.end());
    TuneEntry bt;
    for (size_t i = 0; i < ms_of.size(); i++)
        if (ms_of[i] <= kTuneTolerance * best) {
            bt.rpl = cand[i].rpl;
            bt.block = cand[i].block;
            bt.occ = cand[i].occ;
            break;
        }
    p->tune[key] = bt;
    tune_save(key, bt);
    *out = bt;
    p->last.tuned = 1;
    return RG_OK;
}

static rg_status tune_dopri(rg_program *p, const rg_kargs &a, hipStream_t s, TuneEntry *out) {
    std::string key = tune_key(p, "dopri", a.n);
    if (p->tune.empty()) tune_load(p);
    auto it = p->tune.find(key);
    if (it != p->tune.end()) { *out = it->second; p->last.tuned = 1; return RG_OK; }
    // The compaction interval pays only where rays finish at different
    // times, which a sample with capped budgets does not show: a problem
    // whose trace is short (one run at block 256, interval 8, under 100 ms)
    // is tuned on itself (its outputs are overwritten by the run that
    // follows); a longer one on a sixteenth of the rays, budgets capped at
    // 400 steps.
    rg_kargs t = a;
    {
        std::vector<Launch> seq;
        RGCHK(dopri_seq(p, a, 256, 8, seq));
        hipEvent_t e[2];
        for (hipEvent_t &x : e) HIPCHK(hipEventCreate(&x));
        HIPCHK(hipEventRecord(e[0], s));
        RGCHK(run_seq(p, seq, false, s));
        HIPCHK(hipEventRecord(e[1], s));
        HIPCHK(hipEventSynchronize(e[1]));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e[0], e[1]));
        for (hipEvent_t &x : e) (void)hipEventDestroy(x);
        if (ms > 100.0f) {
            t.n_run = std::min<long long>(a.n, std::max<long long>(65536, a.n / 16));
            t.budget_cap = 400;
        }
    }
    // (preference order and tolerance as for RK4)
    const std::pair<int, int> cand[] = {{256, 8}, {128, 8}, {64, 8}, {256, 32}, {128, 32}, {64, 32},
                                        {256, 128}, {128, 128}, {64, 128}, {256, -1}, {128, -1}, {64, -1}};
    std::vector<float> ms_of;
    for (const auto &c : cand) {
        std::vector<Launch> seq;
        RGCHK(dopri_seq(p, t, c.first, c.second, seq));
        float ms;
        RGCHK(time_seq(p, seq, s, &ms));
        ms_of.push_back(ms);
    }
    const float best = *std::min_element(ms_of.begin(), ms_of.end());
    TuneEntry bt;
    for (size_t i = 0; i < ms_of.size(); i++)
        if (ms_of[i] <= kTuneTolerance * best) {
            bt.block = cand[i].first;
            bt.compact = cand[i].second;
            break;
        }
    p->tune[key] = bt;
    tune_save(key, bt);
    *out = bt;
    p->last.tuned = 1;
    return RG_OK;
}

// ----------------------------------------------------------------- trace --

// Per-call scratch of each launch form, carved from the workspace: the
// plain RK4 form's per-ray t, status and step count; the Dormand-Prince
// refill queue; the plain Dormand-Prince form's per-ray state.  Persistent
// RK4 keeps everything in registers and needs none.
static void carve_trace(const rg_trace_desc &d, uint32_t ny, rg_kargs &a, Carve &c) {
    const long long n = a.n;
    if (d.integrator == RG_RK4 && d.mode == RG_PERSISTENT) return;
    if (d.integrator == RG_RK4) {
        a.s_t = c.take<double>(n);
        a.s_st = c.take<int>(n);
        a.s_acc = c.take<int>(n);
        return;
    }
    if (d.mode == RG_PERSISTENT) {
        a.queue = c.take<unsigned long long>(1);
        return;
    }
    a.s_y = c.take<double>(ny * n);
    a.s_k1 = c.take<double>(ny * n);
    a.s_t = c.take<double>(n);
    a.s_h = c.take<double>(n);
    a.s_fm = c.take<double>(n);
    a.s_st = c.take<int>(n);
    a.s_acc = c.take<int>(n);
    a.s_att = c.take<int>(n);
    a.counter = c.take<int>(2);
}

static size_t trace_ws_bytes(const rg_program *p, const rg_trace_desc &d) {
    if (d.n_rays == 0) return 0;
    rg_kargs a;
    std::memset(&a, 0, sizeof a);
    a.n = d.n_rays;
    Carve c{nullptr};
    carve_trace(d, 2 * p->dim, a, c);
    return c.off;
}

rg_status workspace_size(rg_program *p, const rg_trace_desc &d, size_t *bytes) {
    if (d.struct_size < sizeof(rg_trace_desc)) return fail(RG_EINVAL, "rg_trace_desc.struct_size too small");
    *bytes = trace_ws_bytes(p, d);
    return RG_OK;
}

// static_ws: d.workspace is the library's static scratch (its size was
// checked by the caller; it is not a runtime allocation to be queried).
static rg_status trace_impl(rg_program *p, const rg_trace_desc &d, hipStream_t s, bool static_ws) {
    RGCHK(ensure_module(p));
    rg_kargs a;
    if (d.struct_size < sizeof(rg_trace_desc)) return fail(RG_EINVAL, "rg_trace_desc.struct_size too small");
    const size_t need = trace_ws_bytes(p, d);
    RGCHK(validate(p, d, a, false, need ? d.workspace : nullptr, need));
    if (d.n_rays == 0) return RG_OK;
    if (!static_ws) RGCHK(check_ws(d.workspace, d.workspace_bytes, need));
    const long long n = a.n;
    const uint32_t ny = 2 * p->dim;
    Carve cw{(char *)d.workspace};
    carve_trace(d, ny, a, cw);
    p->last = rg_launch_info{};
    p->last.struct_size = sizeof(rg_launch_info);
    const bool graph = d.use_hipgraph != 0;

    if (d.integrator == RG_RK4 && d.mode == RG_PERSISTENT) {
        const bool fp32 = d.precision == RG_FP32;
        TuneEntry te;
        if (d.block == 0 || (d.rays_per_lane == 0 && !fp32)) RGCHK(tune_rk4(p, a, s, &te, fp32));
        const bool tuned = d.block == 0 || (d.rays_per_lane == 0 && !fp32);
        int block = d.block ? d.block : te.block;
        int rpl = fp32 ? 1 : d.rays_per_lane ? d.rays_per_lane : te.rpl;
        // the at-least-four-waves variant: chosen by the tuner, or asked for
        const int occ = rpl == 1 && !fp32 && (d.min_waves_per_simd == 4 || (tuned && d.min_waves_per_simd == 0 && te.occ));
        std::vector<Launch> seq;
        RGCHK(persistent_rk4_seq(p, a, block, rpl, seq, fp32, occ));
        p->last.block = block;
        p->last.rays_per_lane = rpl;
        p->last.min_waves_per_simd = occ ? 4 : 0;
        return run_seq(p, seq, graph, s);
    }
    if (d.integrator == RG_RK4) {  // plain: one launch per step
        int block = d.block ? d.block : 256;
        std::vector<Launch> seq;
        unsigned grid = cdiv(n, block);
        seq.push_back(Launch{"rg_rk4_plain_init", grid, (unsigned)block, a});
        for (int st = 0; st < d.n_steps; st++) {
            rg_kargs b = a;
            b.step = st;
            b.snap = (a.store_every > 0 && (st + 1) % a.store_every == 0) ? (st + 1) / a.store_every : -1;
            b.ckpt_idx = (a.ckpt_every > 0 && st % a.ckpt_every == 0) ? st / a.ckpt_every : -1;
            seq.push_back(Launch{"rg_rk4_plain_step", grid, (unsigned)block, b});
        }
        seq.push_back(Launch{"rg_plain_finish", grid, (unsigned)block, a});
        p->last.block = block;
        p->last.rays_per_lane = 1;
        p->last.grid = (int)grid;
        return run_seq(p, seq, graph, s);
    }
    if (d.mode == RG_PERSISTENT) {
        TuneEntry te;
        if (d.block == 0 || d.compact_interval == 0) RGCHK(tune_dopri(p, a, s, &te));
        int block = d.block ? d.block : te.block;
        int C = d.compact_interval ? d.compact_interval : te.compact;
        std::vector<Launch> seq;
        RGCHK(dopri_seq(p, a, block, C, seq));
        p->last.block = block;
        p->last.rays_per_lane = 1;
        p->last.compact_interval = C;
        return run_seq(p, seq, graph, s);
    }
    // plain adaptive: one attempt per launch, alive count read back every 64 launches
    int block = d.block ? d.block : 256;
    unsigned grid = cdiv(n, block);
    RGCHK(launch_one(p, Launch{"rg_dopri_plain_init", grid, (unsigned)block, a}, s));
    long long maxb = d.max_steps;
    if (d.budget) {
        std::vector<int> hb(n);
        HIPCHK(hipMemcpyAsync(hb.data(), d.budget, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        maxb = *std::max_element(hb.begin(), hb.end());
    }
    const long long cap = 4 * std::max<long long>(maxb, 1) + 128;
    for (long long it = 0; it < cap; it++) {
        const bool check = (it % 64) == 63;
        rg_kargs b = a;
        b.count_alive = check ? 1 : 0;
        if (check) {
            rg_kargs f;
            std::memset(&f, 0, sizeof f);
            f.fill_p = (double *)a.counter;
            f.fill_n = 1;
            f.fill_v = 0.0;
            RGCHK(launch_one(p, Launch{"rg_fill_f64", 1, 64, f}, s));
        }
        RGCHK(launch_one(p, Launch{"rg_dopri_plain_step", grid, (unsigned)block, b}, s));
        if (check) {
            int alive = 0;  // pageable host memory: the copy completes before the synchronisation returns
            hipError_t e = hipMemcpyAsync(&alive, a.counter, 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return fail(RG_EHIP, std::string("plain DOPRI readback: ") + hipGetErrorString(e));
            if (alive == 0) break;
        }
    }
    p->last.block = block;
    p->last.rays_per_lane = 1;
    p->last.grid = (int)grid;
    return RG_OK;
}

rg_status trace(rg_program *p, const rg_trace_desc &d, hipStream_t s) {
    RGCHK(ensure_module(p));
    time_mark(p, s, 0);
    rg_status st = trace_impl(p, d, s, false);
    if (st == RG_OK) time_mark(p, s, 1);
    else p->ev_state = 0;
    return st;
}

rg_status last_kernel_ms(const rg_program *p, double *ms) {
    *ms = 0.0;
    if (p->ev_state != 1 || !p->ev[0] || !p->ev[1]) return RG_OK;
    hipError_t e = hipEventQuery(p->ev[1]);
    if (e == hipErrorNotReady) {
        (void)hipGetLastError();
        *ms = -1.0;
        return RG_OK;
    }
    float t = 0.0f;
    if (e != hipSuccess || hipEventElapsedTime(&t, p->ev[0], p->ev[1]) != hipSuccess) {
        (void)hipGetLastError();
        return RG_OK;
    }
    *ms = t;
    return RG_OK;
}

rg_status trace_stats(rg_program *p, const rg_trace_desc &d, uint64_t *stats, hipStream_t s) {
    RGCHK(ensure_module(p));
    if (d.struct_size < sizeof(rg_trace_desc)) return fail(RG_EINVAL, "rg_trace_desc.struct_size too small");
    const size_t n = d.n_rays;
    RGCHK(check_dev(stats, 8 * 10, "stats"));
    if (d.status_out) RGCHK(check_dev(d.status_out, 4 * n, "status_out"));
    if (d.steps_out) RGCHK(check_dev(d.steps_out, 4 * n, "steps_out"));
    if (d.integrator == RG_DOPRI54 && d.attempts_out) RGCHK(check_dev(d.attempts_out, 4 * n, "attempts_out"));
    rg_kargs f;
    std::memset(&f, 0, sizeof f);
    f.fill_p = (double *)stats;
    f.fill_n = 10;
    f.fill_v = 0.0;  // all-zero bits
    RGCHK(launch_one(p, Launch{"rg_fill_f64", 1, 64, f}, s));
    if (n == 0) return RG_OK;
    rg_kargs a;
    std::memset(&a, 0, sizeof a);
    a.n = (long long)n;
    a.n_run = (long long)n;
    a.status_out = d.status_out;
    a.steps_out = d.steps_out;
    a.attempts_out = d.integrator == RG_DOPRI54 ? d.attempts_out : nullptr;
    a.stats = (unsigned long long *)stats;
    unsigned grid;
    RGCHK(occupancy_grid(p, "rg_stats", 256, (long long)cdiv(n, 256), &grid));
    return launch_one(p, Launch{"rg_stats", grid, 256, a}, s);
}

rg_status program_load(rg_program *p) {
    RGCHK(ensure_module(p));
    std::string err;
    if (noalloc_resolve(p->device, &err) != 0) return fail(RG_EHIP, err);
    return RG_OK;
}

// rg_trace_rays with the per-call scratch taken from the static device
// array instead of d.workspace, and nothing else that allocates: the code
// object must already be loaded on the current device (program_load), the
// launch parameters must be given (the autotuner creates events) and the
// launch sequence runs directly (instantiating a hipGraph allocates).
rg_status trace_noalloc(rg_program *p, const rg_trace_desc &d, hipStream_t s) {
    if (d.struct_size < sizeof(rg_trace_desc)) return fail(RG_EINVAL, "rg_trace_desc.struct_size too small");
    if (p->compile_only) return fail(RG_ESTATE, "program was compiled with compile_only=1");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    void *scr = noalloc_address(dev);
    if (!p->module || p->device != dev || !scr)
        return fail(RG_ESTATE, "rg_trace_rays_noalloc: call rg_program_load on this device first");
    if (d.use_hipgraph) return fail(RG_EINVAL, "rg_trace_rays_noalloc: use_hipgraph must be 0");
    const bool persistent = d.mode == RG_PERSISTENT;
    if (persistent && (d.block == 0 || (d.integrator == RG_RK4 && d.precision == RG_FP64 && d.rays_per_lane == 0) ||
                       (d.integrator == RG_DOPRI54 && d.compact_interval == 0)))
        return fail(RG_EINVAL, "rg_trace_rays_noalloc: block, rays_per_lane (RK4) and compact_interval "
                               "(Dormand-Prince) must be given (no autotuning)");
    const size_t need = trace_ws_bytes(p, d);
    if (need > RG_NOALLOC_SCRATCH_BYTES)
        return fail(RG_EINVAL, "rg_trace_rays_noalloc: this trace needs " + std::to_string(need) +
                                   " bytes of scratch, more than the static " +
                                   std::to_string((size_t)RG_NOALLOC_SCRATCH_BYTES));
    rg_trace_desc dd = d;
    dd.workspace = need ? scr : nullptr;
    dd.workspace_bytes = need ? RG_NOALLOC_SCRATCH_BYTES : 0;
    return trace_impl(p, dd, s, true);
}

// --------------------------------------------------------------- adjoint --

// Workspace of the adjoint: [internal forward: checkpoints, endpoints, step
// counts and that trace's own scratch] [segment buffer] [gradient partials].
struct AdjPlan {
    bool internal_fwd = false;  // fwd->checkpoints == NULL: the forward runs inside the call
    int block = 0;
    unsigned grid = 0;          // workgroups of the reverse launch(es)
    long long lanes = 0;        // per-lane segment buffer rows (persistent) or n (plain)
    int stride = 0;             // gradient slots per workgroup partial
    int ns_kept = 0;            // stage states per step in the segment buffer
    long long n_part = 0;       // partial slots: workgroups, or waves (deterministic sums)
};

static rg_status adj_plan(rg_program *p, const rg_trace_desc &d, AdjPlan *pl) {
    const long long n = d.n_rays;
    pl->internal_fwd = d.checkpoints == nullptr;
    pl->block = d.block > 0 && d.block < kAdjointBlock ? d.block : kAdjointBlock;
    pl->stride = (int)(p->grad_param.size() + (size_t)p->spl_total);
    pl->ns_kept = p->adj_recompute ? 1 : 4;
    if (d.mode == RG_PLAIN) {
        pl->grid = cdiv(n, pl->block);
        pl->lanes = n;
    } else {
        RGCHK(occupancy_grid(p, "rg_rk4_adjoint", pl->block, (long long)cdiv(n, pl->block), &pl->grid));
        pl->lanes = (long long)pl->grid * pl->block;
    }
    // one partials slot per workgroup, or per wave for deterministic sums
    pl->n_part = p->det_grad ? (long long)pl->grid * ((pl->block + 63) / 64) : pl->grid;
    return RG_OK;
}

// Carves the adjoint's buffers.  fd receives the internal forward's
// description when the plan has one.
static void carve_adjoint(rg_program *p, const rg_trace_desc &d, const AdjPlan &pl, rg_kargs &a,
                          rg_trace_desc &fd, Carve &c) {
    const long long n = d.n_rays;
    const uint32_t dim = p->dim, ny = 2 * dim;
    if (pl.internal_fwd) {
        fd = d;
        const size_t nc = ((size_t)d.n_steps + d.checkpoint_every - 1) / d.checkpoint_every;
        fd.checkpoints = c.take<double>(nc * (ny + 1) * n);
        fd.x_out = c.take<double>(dim * n);
        fd.k_out = c.take<double>(dim * n);
        fd.steps_out = c.take<int>(n);
        fd.t_out = nullptr;
        fd.status_out = nullptr;
        fd.store_every = 0;
        fd.traj = nullptr;
        fd.traj_D = nullptr;
        fd.use_hipgraph = 0;
        fd.workspace_bytes = trace_ws_bytes(p, fd);
        fd.workspace = fd.workspace_bytes ? c.take<char>(fd.workspace_bytes) : nullptr;
        a.ckpt = fd.checkpoints;
        a.steps_out = fd.steps_out;
    }
    const size_t seg = (size_t)d.checkpoint_every * (pl.ns_kept * ny + 1) * pl.lanes;
    a.scratch = c.take<double>(seg);
    a.scratch_lanes = pl.lanes;
    if (d.mode == RG_PLAIN) {
        a.s_y = c.take<double>(ny * n);
        a.s_lam = c.take<double>(ny * n);
        a.s_t = c.take<double>(n);
    }
    a.gpart = pl.stride > 0 ? c.take<double>((size_t)pl.n_part * pl.stride) : nullptr;
    a.n_part = (int)pl.n_part;
    a.part_stride = pl.stride;
}

static rg_status adj_check(rg_program *p, const rg_adjoint_desc &ad) {
    if (!p->has_vjp) return fail(RG_ESTATE, "program compiled without want_adjoint");
    if (ad.struct_size < sizeof(rg_adjoint_desc)) return fail(RG_EINVAL, "rg_adjoint_desc.struct_size too small");
    if (!ad.fwd) return fail(RG_EINVAL, "adjoint needs the forward description");
    const rg_trace_desc &d = *ad.fwd;
    if (d.struct_size < sizeof(rg_trace_desc)) return fail(RG_EINVAL, "rg_trace_desc.struct_size too small");
    if (d.integrator != RG_RK4) return fail(RG_EUNSUPPORTED, "adjoint is implemented for RK4");
    if (d.precision != RG_FP64) return fail(RG_EUNSUPPORTED, "adjoint is implemented in FP64");
    if (d.checkpoint_every <= 0) return fail(RG_ESTATE, "adjoint needs fwd->checkpoint_every > 0");
    if (d.checkpoints && !d.steps_out)
        return fail(RG_ESTATE, "adjoint on stored checkpoints needs the forward's steps_out");
    return RG_OK;
}

static rg_status adjoint_bytes(rg_program *p, const rg_trace_desc &d, size_t *bytes) {
    *bytes = 0;
    if (d.n_rays == 0) return RG_OK;
    AdjPlan pl;
    RGCHK(adj_plan(p, d, &pl));
    rg_kargs a;
    std::memset(&a, 0, sizeof a);
    rg_trace_desc fd;
    Carve c{nullptr};
    carve_adjoint(p, d, pl, a, fd, c);
    *bytes = c.off;
    return RG_OK;
}

rg_status adjoint_workspace_size(rg_program *p, const rg_adjoint_desc &ad, size_t *bytes) {
    RGCHK(ensure_module(p));
    RGCHK(adj_check(p, ad));
    return adjoint_bytes(p, *ad.fwd, bytes);
}

static rg_status adjoint_impl(rg_program *p, const rg_adjoint_desc &ad, hipStream_t s) {
    RGCHK(ensure_module(p));
    RGCHK(adj_check(p, ad));
    const rg_trace_desc &d = *ad.fwd;
    size_t need = 0;
    RGCHK(adjoint_bytes(p, d, &need));
    rg_kargs a;
    RGCHK(validate(p, d, a, true, need ? ad.workspace : nullptr, need));
    if (d.n_rays == 0) return RG_OK;
    RGCHK(check_ws(ad.workspace, ad.workspace_bytes, need));
    const long long n = a.n;
    const uint32_t dim = p->dim;
    RGCHK(check_dev(ad.dL_dx_end, 8 * dim * n, "dL_dx_end"));
    if (ad.dL_dk_end) RGCHK(check_dev(ad.dL_dk_end, 8 * dim * n, "dL_dk_end"));
    if (ad.dL_dx0) RGCHK(check_dev(ad.dL_dx0, 8 * dim * n, "dL_dx0"));
    if (ad.dL_dk0) RGCHK(check_dev(ad.dL_dk0, 8 * dim * n, "dL_dk0"));
    for (uint32_t i = 0; i < p->n_params; i++)
        if (ad.dL_dparams && ad.dL_dparams[i]) {
            RGCHK(check_dev(ad.dL_dparams[i], 8 * (size_t)p->param_len[i], "dL_dparams[i]"));
            a.dparams[i] = ad.dL_dparams[i];
        }
    // What the call writes (the gradients, the workspace) may overlap
    // nothing it reads and nothing else it writes: the parameter gradients
    // are zeroed and the workspace filled before the seeds, checkpoints and
    // parameters are read.
    {
        struct Buf { const void *p; size_t bytes; std::string name; };
        std::vector<Buf> rd = {{d.x0, 8 * dim * n, "x0"}, {d.k0, 8 * dim * n, "k0"}, {d.omega, 8 * n, "omega"},
                               {d.t0, 8 * n, "t0"}, {ad.dL_dx_end, 8 * dim * n, "dL_dx_end"},
                               {ad.dL_dk_end, 8 * dim * n, "dL_dk_end"}};
        if (d.checkpoints) {
            const size_t nc = ((size_t)d.n_steps + d.checkpoint_every - 1) / d.checkpoint_every;
            rd.push_back({d.checkpoints, 8 * nc * (2 * dim + 1) * n, "checkpoints"});
            rd.push_back({d.steps_out, 4 * n, "steps_out"});
        }
        std::vector<Buf> wr = {{ad.dL_dx0, 8 * dim * n, "dL_dx0"}, {ad.dL_dk0, 8 * dim * n, "dL_dk0"},
                               {ad.workspace, need, "workspace"}};
        for (uint32_t i = 0; i < p->n_params; i++) {
            const std::string k = std::to_string(i);
            rd.push_back({d.params[i], 8 * (size_t)p->param_len[i], "params[" + k + "]"});
            wr.push_back({a.dparams[i], 8 * (size_t)p->param_len[i], "dL_dparams[" + k + "]"});
        }
        auto overlap = [](const Buf &u, const Buf &v) {
            if (!u.p || !v.p || !u.bytes || !v.bytes) return false;
            const char *a0 = (const char *)u.p, *b0 = (const char *)v.p;
            return a0 < b0 + v.bytes && b0 < a0 + u.bytes;
        };
        for (size_t i = 0; i < wr.size(); i++) {
            for (const Buf &r : rd)
                if (overlap(wr[i], r)) return fail(RG_EINVAL, wr[i].name + " overlaps " + r.name);
            for (size_t j = i + 1; j < wr.size(); j++)
                if (overlap(wr[i], wr[j])) return fail(RG_EINVAL, wr[i].name + " overlaps " + wr[j].name);
        }
    }
    a.lam_x = ad.dL_dx_end;
    a.lam_k = ad.dL_dk_end;
    a.gx0 = ad.dL_dx0;
    a.gk0 = ad.dL_dk0;

    AdjPlan pl;
    RGCHK(adj_plan(p, d, &pl));
    rg_trace_desc fd;
    Carve cw{(char *)ad.workspace};
    carve_adjoint(p, d, pl, a, fd, cw);
    if (pl.internal_fwd) RGCHK(trace_impl(p, fd, s, false));  // checkpoints and step counts into the workspace
    const int block = pl.block;
    const unsigned grid = pl.grid;
    const int stride = pl.stride;
    // zero the parameter gradients that will be written
    for (uint32_t i = 0; i < p->n_params; i++)
        if (a.dparams[i]) {
            rg_kargs f;
            std::memset(&f, 0, sizeof f);
            f.fill_p = a.dparams[i];
            f.fill_n = p->param_len[i];
            f.fill_v = 0.0;
            RGCHK(launch_one(p, Launch{"rg_fill_f64", cdiv(f.fill_n, 256), 256, f}, s));
        }

    if (d.mode == RG_PLAIN) {
        // one launch per step, per-ray state and adjoint in the workspace
        std::vector<Launch> seq;
        seq.push_back(Launch{"rg_adjp_init", grid, (unsigned)block, a});
        const int ce = d.checkpoint_every;
        const int nseg = (d.n_steps + ce - 1) / ce;
        for (int sg = nseg - 1; sg >= 0; sg--) {
            const int s0 = sg * ce, s1 = std::min(s0 + ce, d.n_steps);
            rg_kargs b = a;
            b.ckpt_idx = sg;
            b.seg_s0 = s0;
            seq.push_back(Launch{"rg_adjp_seg", grid, (unsigned)block, b});
            for (int j = s0; j < s1; j++) {
                b.step = j;
                seq.push_back(Launch{"rg_adjp_fwd", grid, (unsigned)block, b});
            }
            for (int j = s1 - 1; j >= s0; j--) {
                b.step = j;
                seq.push_back(Launch{"rg_adjp_rev", grid, (unsigned)block, b});
            }
        }
        seq.push_back(Launch{"rg_adjp_finish", grid, (unsigned)block, a});
        if (stride > 0) seq.push_back(Launch{"rg_grad_finalize", cdiv(stride, 256), 256, a});
        RGCHK(run_seq(p, seq, false, s));
        p->last.block = block;
        p->last.grid = (int)grid;
        return RG_OK;
    }

    if (p->det_grad && a.gpart) {  // the per-wave tables are added to from zero
        rg_kargs f;
        std::memset(&f, 0, sizeof f);
        f.fill_p = a.gpart;
        f.fill_n = (long long)pl.n_part * stride;
        f.fill_v = 0.0;
        RGCHK(launch_one(p, Launch{"rg_fill_f64", cdiv(f.fill_n, 256), 256, f}, s));
    }
    RGCHK(launch_one(p, Launch{"rg_rk4_adjoint", grid, (unsigned)block, a}, s));
    if (stride > 0) RGCHK(launch_one(p, Launch{"rg_grad_finalize", cdiv(stride, 256), 256, a}, s));
    p->last.block = block;
    p->last.grid = (int)grid;
    return RG_OK;
}

rg_status adjoint(rg_program *p, const rg_adjoint_desc &ad, hipStream_t s) {
    RGCHK(ensure_module(p));
    time_mark(p, s, 0);
    rg_status st = adjoint_impl(p, ad, s);
    if (st == RG_OK) time_mark(p, s, 1);
    else p->ev_state = 0;
    return st;
}

rg_status solve_k(rg_program *p, const rg_solve_desc &d, hipStream_t s) {
    RGCHK(ensure_module(p));
    if (d.struct_size < sizeof(rg_solve_desc)) return fail(RG_EINVAL, "rg_solve_desc.struct_size too small");
    if (d.component < 0 || d.component >= (int)p->dim) return fail(RG_EINVAL, "component out of range");
    if (d.max_iter <= 0 || d.max_iter > 1000) return fail(RG_EINVAL, "max_iter must be in 1..1000");
    if (!(d.tol >= 0.0)) return fail(RG_EINVAL, "tol must be >= 0");
    const size_t n = d.n_rays;
    if (n == 0) return RG_OK;
    const uint32_t dim = p->dim;
    rg_kargs a;
    std::memset(&a, 0, sizeof a);
    a.n = (long long)n;
    a.n_run = (long long)n;
    RGCHK(check_dev(d.x, 8 * dim * n, "x"));
    RGCHK(check_dev(d.k, 8 * dim * n, "k"));
    RGCHK(check_dev(d.omega, 8 * n, "omega"));
    if (d.t) RGCHK(check_dev(d.t, 8 * n, "t"));
    if (d.D_out) RGCHK(check_dev(d.D_out, 8 * n, "D_out"));
    if (d.iters_out) RGCHK(check_dev(d.iters_out, 4 * n, "iters_out"));
    if (d.max_abs_D) RGCHK(check_dev(d.max_abs_D, 8, "max_abs_D"));
    if (p->n_params > 0 && !d.params) return fail(RG_EINVAL, "params is NULL but the graph has parameters");
    for (uint32_t i = 0; i < p->n_params; i++) {
        RGCHK(check_dev(d.params[i], 8 * (size_t)p->param_len[i], "params[i]"));
        a.params[i] = d.params[i];
    }
    a.x0 = d.x;
    a.k_io = d.k;
    a.omega = d.omega;
    a.t0 = d.t;
    a.D_out = d.D_out;
    a.iters_out = d.iters_out;
    a.max_abs_D = d.max_abs_D;
    a.component = d.component;
    a.max_iter = d.max_iter;
    a.tol = d.tol;
    if (d.max_abs_D) {
        rg_kargs f;
        std::memset(&f, 0, sizeof f);
        f.fill_p = d.max_abs_D;
        f.fill_n = 1;
        f.fill_v = 0.0;
        RGCHK(launch_one(p, Launch{"rg_fill_f64", 1, 64, f}, s));
    }
    return launch_one(p, Launch{"rg_newton_k", cdiv(n, 256), 256, a}, s);
}

rg_status eval_points(rg_program *p, uint32_t n, const double *y, const double *omega,
                      const double *t, const double *const *params, double *f, double *D,
                      hipStream_t s) {
    RGCHK(ensure_module(p));
    if (n == 0) return RG_OK;
    const uint32_t ny = 2 * p->dim;
    rg_kargs a;
    std::memset(&a, 0, sizeof a);
    a.n = n;
    a.n_run = n;
    RGCHK(check_dev(y, 8 * (size_t)ny * n, "y"));
    RGCHK(check_dev(omega, 8 * (size_t)n, "omega"));
    if (t) RGCHK(check_dev(t, 8 * (size_t)n, "t"));
    if (f) RGCHK(check_dev(f, 8 * (size_t)ny * n, "f_out"));
    if (D) RGCHK(check_dev(D, 8 * (size_t)n, "D_out"));
    if (p->n_params > 0 && !params) return fail(RG_EINVAL, "params is NULL but the graph has parameters");
    for (uint32_t i = 0; i < p->n_params; i++) {
        RGCHK(check_dev(params[i], 8 * (size_t)p->param_len[i], "params[i]"));
        a.params[i] = params[i];
    }
    a.x0 = y;
    a.omega = omega;
    a.t0 = t;
    a.x_out = f;
    a.t_out = D;
    return launch_one(p, Launch{"rg_eval_points", cdiv(n, 256), 256, a}, s);
}

}  // namespace rg
