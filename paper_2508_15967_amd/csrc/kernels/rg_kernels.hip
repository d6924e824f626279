// Integrator kernels for gfx950 (wave64), FP64.  This text is compiled at
// run time by hipRTC together with the device functions emitted from the
// expression graph:
//   rg_config.h     RG_DIM, RG_NY, table and gradient-slot layout (generated)
//   rg_prelude.h    B-spline helpers, rg_P
//   rg_functions.h  rg_rhs, rg_D and (with RG_HAS_VJP) rg_vjp (generated)
//
// The paper's kernel takes x, k, t, omega and returns the D residual and
// the RK4 update of x, k, t, with setter maps feeding outputs back to inputs
// for the next step ("Impact" and "JIT" sections).  The persistent kernels
// here keep that loop inside the kernel: each lane holds its ray in
// registers for all steps and touches HBM only for the initial load,
// snapshots/checkpoints and the final store.  The "plain" kernels keep the
// paper's one-launch-per-step structure (state round-trips through HBM) and
// serve as the comparison baseline.
#include "rg_kargs.h"
#include "rg_config.h"
#include "rg_prelude.h"

#define RG_RAY_OK 0
#define RG_RAY_EXITED_BOX 1
#define RG_RAY_BUDGET 2
#define RG_RAY_NONFINITE 3
#define RG_RAY_STEP_UNDERFLOW 4

// ---------------------------------------------------------------- tables --
#if RG_NSPLTAB > 0
__shared__ double rg_spl_lds[RG_SPL_TOTAL];
#define RG_SPL_TAB(k) (rg_spl_lds + rg_spl_off[k])
#endif

// Gradient accumulator for spline coefficient tables (adjoint only): the
// 16 coefficient gradients of the current cell stay in registers while the
// ray stays in that cell and are flushed with atomics when it leaves: to an
// LDS copy of the table shared by the workgroup, or, with
// RG_DET_GRAD (deterministic sums), to the wave's own copy in its slot of
// the per-wave partials (global memory), so that each copy is added to by
// one wave in program order and the partials are then summed in a fixed
// order.
#if RG_HAS_VJP && RG_NSPLTAB > 0
#if !RG_DET_GRAD
__shared__ double rg_spl_grad_lds[RG_SPL_TOTAL];
#endif
struct rg_GA {
    int cx[RG_NSPLTAB], cy[RG_NSPLTAB];
    double acc[RG_NSPLTAB][16];
    double *tab;  // the table copy this lane's flushes go to
    // part: this wave's slot of the partials ([RG_NGRAD scalars][tables])
    __device__ __forceinline__ void init(double *part) {
        for (int k = 0; k < RG_NSPLTAB; k++) { cx[k] = -1; cy[k] = -1; }
#if RG_DET_GRAD
        tab = part + RG_NGRAD;
#else
        (void)part;
        tab = rg_spl_grad_lds;
#endif
    }
    __device__ __forceinline__ void flush(int k) {
        if (cx[k] >= 0) {
            double *base = tab + rg_spl_off[k] + (cx[k] - 1) * rg_spl_ny[k] + (cy[k] - 1);
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) atomicAdd(base + a * rg_spl_ny[k] + b, acc[k][4 * a + b]);
        }
    }
    __device__ __forceinline__ void add(int k, int x, int y, const double *g) {
        if (x != cx[k] || y != cy[k]) {
            flush(k);
            cx[k] = x;
            cy[k] = y;
            for (int i = 0; i < 16; i++) acc[k][i] = g[i];
        } else {
            for (int i = 0; i < 16; i++) acc[k][i] += g[i];
        }
    }
};
#else
struct rg_GA {
    __device__ __forceinline__ void init(double *) {}
    __device__ __forceinline__ void flush(int) {}
    __device__ __forceinline__ void add(int, int, int, const double *) {}
};
#endif

#include "rg_functions.h"

#if RG_USES_EXP
__constant__ double rg_exp_const[RG_EXP_N] = {RG_EXP_TABLE_VALUES};
#endif

// Copies the spline tables and the exponential's table into LDS (every
// thread of the workgroup must call it).
__device__ __forceinline__ void rg_stage_tables(const rg_kargs &a) {
#if RG_NSPLTAB > 0
    for (int k = 0; k < RG_NSPLTAB; k++) {
        const double *src = a.params[rg_spl_param[k]];
        for (int i = threadIdx.x; i < rg_spl_len[k]; i += blockDim.x) rg_spl_lds[rg_spl_off[k] + i] = src[i];
    }
#endif
#if RG_USES_EXP
    for (int i = threadIdx.x; i < RG_EXP_N; i += blockDim.x) rg_exp_lds[i] = rg_exp_const[i];
#endif
#if RG_NSPLTAB > 0 || RG_USES_EXP
    __syncthreads();
#endif
    (void)a;
}

__device__ __forceinline__ rg_P rg_params(const rg_kargs &a) {
    rg_P P;
    for (int i = 0; i < RG_MAX_PARAMS; i++) P.p[i] = a.params[i];
    return P;
}

template <typename T>
__device__ __forceinline__ bool rg_finite(const T *y) {
    bool f = true;
    for (int i = 0; i < RG_NY; i++) f = f && __builtin_isfinite(y[i]);
    return f;
}

// strictly outside the box (a single precision state is compared exactly,
// promoted to double)
template <typename T>
__device__ __forceinline__ bool rg_outside(const rg_kargs &a, const T *y) {
    bool o = false;
    for (int i = 0; i < RG_DIM; i++) o = o || ((double)y[i] < a.box_lo[i]) || ((double)y[i] > a.box_hi[i]);
    return o;
}

// One classic RK4 step (weights 1/6, 1/3, 1/3, 1/6), fused: the stage
// vectors live in registers and the update accumulates as the stages come.
// Components whose right-hand side is identically zero (RG_RHS_ZERO, known
// when the graph is compiled) keep their value through every stage: the
// stage arithmetic would add exact zeros to them.
//
// With RG_ROLL (a right-hand side with many distinct constants) the four
// stages are a loop around one copy of the right-hand side: the constants,
// which live in scalar registers, are then live for one stage only instead
// of across four inlined copies (which overflows the scalar register file
// into vector-register lanes).  The arithmetic is the same in both forms.
#define RG_ZERO(i) ((RG_RHS_ZERO >> (i)) & 1u)

// With st non-null (the adjoint's segment buffer) the stage states Y2, Y3,
// Y4 are also stored, at st[(s RG_NY + c) SL] for stage s = 1..3.
template <typename T>
__device__ __forceinline__ void rg_rk4_step(const T *y, T om, T t, T dt, const rg_P &P, T *yn,
                                            double *st = nullptr, long long SL = 0) {
    const T h2 = T(0.5) * dt, dt6 = dt / T(6.0);
    T K[RG_NY], acc[RG_NY], Y[RG_NY];
#if RG_ROLL
    const T th = t + h2, tf = t + dt;
    for (int i = 0; i < RG_NY; i++) {
        Y[i] = y[i];
        acc[i] = T(0.0);
    }
#pragma unroll 1
    for (int s = 0; s < 4; s++) {
        rg_rhs(Y, om, s == 0 ? t : (s == 3 ? tf : th), P, K);
        if (s == 3) break;
        // the stage's coefficients depend on s only (scalar selects); acc
        // starts at 0, so the first stage adds K1 exactly (1 K1 + 0)
        const T c = s == 2 ? dt : h2, w = s == 0 ? T(1.0) : T(2.0);
        for (int i = 0; i < RG_NY; i++)
            if (!RG_ZERO(i)) {
                acc[i] = fma(w, K[i], acc[i]);
                Y[i] = fma(c, K[i], y[i]);
            }
        if (st)
            for (int i = 0; i < RG_NY; i++) st[(long long)((s + 1) * RG_NY + i) * SL] = Y[i];
    }
#else
    rg_rhs(y, om, t, P, K);
    for (int i = 0; i < RG_NY; i++) { acc[i] = K[i]; Y[i] = RG_ZERO(i) ? y[i] : fma(h2, K[i], y[i]); }
    if (st)
        for (int i = 0; i < RG_NY; i++) st[(long long)(RG_NY + i) * SL] = Y[i];
    rg_rhs(Y, om, t + h2, P, K);
    for (int i = 0; i < RG_NY; i++) {
        if (!RG_ZERO(i)) { acc[i] = fma(T(2.0), K[i], acc[i]); Y[i] = fma(h2, K[i], y[i]); }
    }
    if (st)
        for (int i = 0; i < RG_NY; i++) st[(long long)(2 * RG_NY + i) * SL] = Y[i];
    rg_rhs(Y, om, t + h2, P, K);
    for (int i = 0; i < RG_NY; i++) {
        if (!RG_ZERO(i)) { acc[i] = fma(T(2.0), K[i], acc[i]); Y[i] = fma(dt, K[i], y[i]); }
    }
    if (st)
        for (int i = 0; i < RG_NY; i++) st[(long long)(3 * RG_NY + i) * SL] = Y[i];
    rg_rhs(Y, om, t + dt, P, K);
#endif
    for (int i = 0; i < RG_NY; i++) yn[i] = RG_ZERO(i) ? y[i] : fma(dt6, acc[i] + K[i], y[i]);
}

// ------------------------------------------------------- persistent RK4 --
// Grid-stride over rays; R rays per lane advanced in lock-step so that the
// compiler can interleave their independent right-hand sides.  T is the
// arithmetic type of the state and the stages (double, or float for the
// single precision variant, whose inputs and outputs stay double and whose
// time and D-residual snapshots are computed in double).
template <typename T>
__device__ __forceinline__ double rg_D_mon(const T *y, double om, double t, const rg_P &P) {
    double yd[RG_NY];
    for (int c = 0; c < RG_NY; c++) yd[c] = (double)y[c];
    return rg_D(yd, om, t, P);
}

template <typename T, int R>
__device__ __forceinline__ void rg_rk4_persistent(const rg_kargs &a) {
    rg_stage_tables(a);
    const rg_P P = rg_params(a);
    const long long n = a.n;
    const long long G = (long long)gridDim.x * blockDim.x;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double dtd = a.dt;
    const T dt = (T)dtd;
    const long long nr = a.n_run;
    for (long long base = gid; base < nr; base += G * R) {
        T y[R][RG_NY], om[R];
        double t[R];
        int st[R], ns[R];
        long long rid[R];
        for (int r = 0; r < R; r++) {
            rid[r] = base + (long long)r * G;
            const long long q = rid[r] < nr ? rid[r] : base;  // inactive slot re-reads a valid ray
            for (int i = 0; i < RG_DIM; i++) {
                y[r][i] = (T)a.x0[i * n + q];
                y[r][RG_DIM + i] = (T)a.k0[i * n + q];
            }
            t[r] = a.t0 ? a.t0[q] : 0.0;
            om[r] = (T)a.omega[q];
            st[r] = rid[r] < nr ? RG_RAY_OK : -1;
            ns[r] = 0;
        }
        int snap = 0, snap_cd = a.store_every, ck = 0, ck_cd = 0;
        if (a.store_every > 0) {
            for (int r = 0; r < R; r++)
                if (st[r] >= 0) {
                    for (int c = 0; c < RG_NY; c++) a.traj[(long long)c * n + rid[r]] = y[r][c];
                    if (a.traj_D) a.traj_D[rid[r]] = rg_D_mon(y[r], a.omega[rid[r]], t[r], P);
                }
            snap = 1;
        }
        for (int s = 0; s < a.n_steps; s++) {
            if (a.ckpt_every > 0 && ck_cd == 0) {
                for (int r = 0; r < R; r++)
                    if (st[r] >= 0) {
                        double *cp = a.ckpt + (long long)ck * (RG_NY + 1) * n + rid[r];
                        for (int c = 0; c < RG_NY; c++) cp[(long long)c * n] = y[r][c];
                        cp[(long long)RG_NY * n] = t[r];
                    }
                ck++;
                ck_cd = a.ckpt_every;
            }
            ck_cd--;
            T yn[R][RG_NY];
            for (int r = 0; r < R; r++) rg_rk4_step(y[r], om[r], (T)t[r], dt, P, yn[r]);
            for (int r = 0; r < R; r++) {
                const bool fin = rg_finite(yn[r]);
                const bool live = st[r] == RG_RAY_OK;
                if (live && fin) {
                    for (int c = 0; c < RG_NY; c++) y[r][c] = yn[r][c];
                    t[r] = t[r] + dtd;
                    ns[r]++;
                    if (a.has_box && rg_outside(a, y[r])) st[r] = RG_RAY_EXITED_BOX;
                } else if (live) {
                    st[r] = RG_RAY_NONFINITE;
                }
            }
            if (a.store_every > 0 && --snap_cd == 0) {
                for (int r = 0; r < R; r++)
                    if (st[r] >= 0) {
                        double *tp = a.traj + (long long)snap * RG_NY * n + rid[r];
                        for (int c = 0; c < RG_NY; c++) tp[(long long)c * n] = y[r][c];
                        if (a.traj_D)
                            a.traj_D[(long long)snap * n + rid[r]] = rg_D_mon(y[r], a.omega[rid[r]], t[r], P);
                    }
                snap++;
                snap_cd = a.store_every;
            }
        }
        for (int r = 0; r < R; r++) {
            if (st[r] < 0) continue;
            for (int i = 0; i < RG_DIM; i++) {
                a.x_out[i * n + rid[r]] = y[r][i];
                a.k_out[i * n + rid[r]] = y[r][RG_DIM + i];
            }
            if (a.t_out) a.t_out[rid[r]] = t[r];
            if (a.status_out) a.status_out[rid[r]] = st[r];
            if (a.steps_out) a.steps_out[rid[r]] = ns[r];
        }
    }
}

extern "C" __global__ void __launch_bounds__(512) rg_rk4_r1(rg_kargs a) { rg_rk4_persistent<double, 1>(a); }
extern "C" __global__ void __launch_bounds__(512) rg_rk4_r2(rg_kargs a) { rg_rk4_persistent<double, 2>(a); }
// The same one-ray-per-lane kernel built for at least four waves per SIMD
// (at most 128 VGPRs): where the natural register count is a little above
// that, the extra wave can hide more latency than the spills cost; the
// autotuner takes it only where it measures faster.  Same arithmetic.
extern "C" __global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
rg_rk4_r1o4(rg_kargs a) { rg_rk4_persistent<double, 1>(a); }
#if RG_HAS_R4
extern "C" __global__ void __launch_bounds__(512) rg_rk4_r4(rg_kargs a) { rg_rk4_persistent<double, 4>(a); }
#endif
#if RG_HAS_F32
extern "C" __global__ void __launch_bounds__(512) rg_rk4_f32(rg_kargs a) { rg_rk4_persistent<float, 1>(a); }
#endif

// ------------------------------------------------------------ plain RK4 --
// One step per launch: load state, one step, store state (the paper's
// setter-map loop).  State lives in x_out/k_out/s_t/s_st/s_acc.
extern "C" __global__ void __launch_bounds__(512) rg_rk4_plain_init(rg_kargs a) {
    if (a.traj_D) rg_stage_tables(a);  // uniform condition: every thread reaches the barrier
    const long long n = a.n;
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_run) return;
    double y[RG_NY];
    for (int i = 0; i < RG_DIM; i++) {
        y[i] = a.x0[i * n + r];
        y[RG_DIM + i] = a.k0[i * n + r];
        a.x_out[i * n + r] = y[i];
        a.k_out[i * n + r] = y[RG_DIM + i];
    }
    const double t = a.t0 ? a.t0[r] : 0.0;
    a.s_t[r] = t;
    a.s_st[r] = RG_RAY_OK;
    a.s_acc[r] = 0;
    if (a.store_every > 0) {
        for (int c = 0; c < RG_NY; c++) a.traj[(long long)c * n + r] = y[c];
        if (a.traj_D) a.traj_D[r] = rg_D(y, a.omega[r], t, rg_params(a));
    }
}

extern "C" __global__ void __launch_bounds__(512) rg_rk4_plain_step(rg_kargs a) {
    rg_stage_tables(a);
    const long long n = a.n;
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_run) return;
    const rg_P P = rg_params(a);
    double y[RG_NY], yn[RG_NY];
    for (int i = 0; i < RG_DIM; i++) {
        y[i] = a.x_out[i * n + r];
        y[RG_DIM + i] = a.k_out[i * n + r];
    }
    double t = a.s_t[r];
    int st = a.s_st[r];
    const double om = a.omega[r];
    if (a.ckpt_idx >= 0) {
        double *cp = a.ckpt + (long long)a.ckpt_idx * (RG_NY + 1) * n + r;
        for (int c = 0; c < RG_NY; c++) cp[(long long)c * n] = y[c];
        cp[(long long)RG_NY * n] = t;
    }
    if (st == RG_RAY_OK) {
        rg_rk4_step(y, om, t, a.dt, P, yn);
        if (rg_finite(yn)) {
            for (int c = 0; c < RG_NY; c++) y[c] = yn[c];
            t = t + a.dt;
            a.s_acc[r] += 1;
            if (a.has_box && rg_outside(a, y)) st = RG_RAY_EXITED_BOX;
            for (int i = 0; i < RG_DIM; i++) {
                a.x_out[i * n + r] = y[i];
                a.k_out[i * n + r] = y[RG_DIM + i];
            }
            a.s_t[r] = t;
        } else {
            st = RG_RAY_NONFINITE;
        }
        a.s_st[r] = st;
    }
    if (a.snap >= 0) {
        double *tp = a.traj + (long long)a.snap * RG_NY * n + r;
        for (int c = 0; c < RG_NY; c++) tp[(long long)c * n] = y[c];
        if (a.traj_D) a.traj_D[(long long)a.snap * n + r] = rg_D(y, om, t, P);
    }
}

// Copy the plain-mode state to the optional outputs.
extern "C" __global__ void __launch_bounds__(512) rg_plain_finish(rg_kargs a) {
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_run) return;
    if (a.t_out) a.t_out[r] = a.s_t[r];
    if (a.status_out) a.status_out[r] = a.s_st[r];
    if (a.steps_out) a.steps_out[r] = a.s_acc[r];
}

// ----------------------------------------------------- Dormand-Prince 5(4) --
// Published tableau (Dormand & Prince 1980).
#define DPA21 (1.0 / 5.0)
#define DPA31 (3.0 / 40.0)
#define DPA32 (9.0 / 40.0)
#define DPA41 (44.0 / 45.0)
#define DPA42 (-56.0 / 15.0)
#define DPA43 (32.0 / 9.0)
#define DPA51 (19372.0 / 6561.0)
#define DPA52 (-25360.0 / 2187.0)
#define DPA53 (64448.0 / 6561.0)
#define DPA54 (-212.0 / 729.0)
#define DPA61 (9017.0 / 3168.0)
#define DPA62 (-355.0 / 33.0)
#define DPA63 (46732.0 / 5247.0)
#define DPA64 (49.0 / 176.0)
#define DPA65 (-5103.0 / 18656.0)
#define DPB1 (35.0 / 384.0)
#define DPB3 (500.0 / 1113.0)
#define DPB4 (125.0 / 192.0)
#define DPB5 (-2187.0 / 6784.0)
#define DPB6 (11.0 / 84.0)
// error weights b5 - b4
#define DPE1 (35.0 / 384.0 - 5179.0 / 57600.0)
#define DPE3 (500.0 / 1113.0 - 7571.0 / 16695.0)
#define DPE4 (125.0 / 192.0 - 393.0 / 640.0)
#define DPE5 (-2187.0 / 6784.0 - -92097.0 / 339200.0)
#define DPE6 (11.0 / 84.0 - 187.0 / 2100.0)
#define DPE7 (0.0 - 1.0 / 40.0)

// Step factor 0.9 err^(-1/5) rounded down to a multiple of 1/32 and clipped
// to [0.2, facmax]; the rounding makes the next step an exactly
// reproducible function of err except at the rounding points.
// Step-size factor: 0.9 err^(-1/5) rounded down to a multiple of 1/32 and
// clipped to [0.2, facmax], i.e. k/32 with k the largest integer such that
// err (5k)^5 <= 144^5 (28.8 = 144/5; (5k)^5 and 144^5 are exact in double,
// so the inequality is decided with one rounded product and no
// transcendental).  A single-precision estimate of 28.8 err^(-1/5)
// (hardware log2 and exp2, relative error about 1e-6, so within one of k for
// k <= 161) is corrected by testing the inequality one step up and one step
// down: a few dozen instructions instead of a double-precision pow.
__device__ __forceinline__ bool rg_dp_fac_ok(double err, int k) {
    const double c = 5.0 * k;
    return err * (c * c * c * c * c) <= 61917364224.0;  // 144^5
}
__device__ __forceinline__ double rg_dp_factor(double err, double facmax) {
    const float g = 28.8f * exp2f(-0.2f * log2f((float)err));
    int k = (int)fminf(fmaxf(floorf(g), 0.0f), 161.0f);  // NaN -> 0
    if (k < 161 && rg_dp_fac_ok(err, k + 1)) k++;
    if (k > 0 && !rg_dp_fac_ok(err, k)) k--;
    double fac = k / 32.0;
    if (!(fac >= 0.2)) fac = 0.2;
    if (fac > facmax) fac = facmax;
    return fac;
}

struct rg_dp_ray {
    double y[RG_NY], k1[RG_NY];
    double t, h, fm, om;
    int acc, att, budget, st;  // st < 0: still running
};

// One Dormand-Prince attempt with the termination tests that precede and
// follow it.  Sets r.st >= 0 when the ray is finished.  Its seven right-hand sides
// are inlined one after the other and take their constants as literals
// (rg_rhs<true>), which the compiler keeps in scalar registers across them.
__device__ __forceinline__ void rg_dp_attempt(const rg_kargs &a, const rg_P &P, rg_dp_ray &r) {
    if (r.acc >= r.budget || r.att >= 4 * r.budget) { r.st = RG_RAY_BUDGET; return; }
    if (a.t_end > 0.0 && r.t >= a.t_end) { r.st = RG_RAY_OK; return; }
    double hs = r.h;
    if (a.t_end > 0.0 && r.t + hs > a.t_end) hs = a.t_end - r.t;
    double k2[RG_NY], k3[RG_NY], k4[RG_NY], k5[RG_NY], k6[RG_NY], k7[RG_NY], Y[RG_NY];
    const double *y = r.y, *k1 = r.k1;
    for (int i = 0; i < RG_NY; i++) Y[i] = fma(hs, DPA21 * k1[i], y[i]);
    rg_rhs<true>(Y, r.om, r.t + hs * (1.0 / 5.0), P, k2);
    for (int i = 0; i < RG_NY; i++) Y[i] = fma(hs, fma(DPA32, k2[i], DPA31 * k1[i]), y[i]);
    rg_rhs<true>(Y, r.om, r.t + hs * (3.0 / 10.0), P, k3);
    for (int i = 0; i < RG_NY; i++)
        Y[i] = fma(hs, fma(DPA43, k3[i], fma(DPA42, k2[i], DPA41 * k1[i])), y[i]);
    rg_rhs<true>(Y, r.om, r.t + hs * (4.0 / 5.0), P, k4);
    for (int i = 0; i < RG_NY; i++)
        Y[i] = fma(hs, fma(DPA54, k4[i], fma(DPA53, k3[i], fma(DPA52, k2[i], DPA51 * k1[i]))), y[i]);
    rg_rhs<true>(Y, r.om, r.t + hs * (8.0 / 9.0), P, k5);
    for (int i = 0; i < RG_NY; i++)
        Y[i] = fma(hs, fma(DPA65, k5[i], fma(DPA64, k4[i], fma(DPA63, k3[i], fma(DPA62, k2[i], DPA61 * k1[i])))), y[i]);
    rg_rhs<true>(Y, r.om, r.t + hs, P, k6);
    // 5th-order solution (also the 7th stage point, FSAL)
    double y5[RG_NY];
    for (int i = 0; i < RG_NY; i++)
        y5[i] = fma(hs, fma(DPB6, k6[i], fma(DPB5, k5[i], fma(DPB4, k4[i], fma(DPB3, k3[i], DPB1 * k1[i])))), y[i]);
    rg_rhs<true>(y5, r.om, r.t + hs, P, k7);
    // k2 has weight 0 in both solutions; its 0 * k2 term makes the error
    // estimate NaN when k2 is not finite, so that the attempt is rejected
    // like one whose stage states are not finite (a stage right-hand side
    // may be finite at a non-finite state: NaN-free exponentials map a NaN
    // argument to 0)
    double sum = 0.0;
    for (int i = 0; i < RG_NY; i++) {
        double e = fma(DPE7, k7[i], fma(DPE6, k6[i], fma(DPE5, k5[i], fma(DPE4, k4[i], fma(DPE3, k3[i],
                   fma(0.0, k2[i], DPE1 * k1[i]))))));
        e = hs * e;
        const double ay = fabs(y[i]), ay5 = fabs(y5[i]);
        const double sc = fma(a.rtol, ay > ay5 ? ay : ay5, a.atol);
        const double q = e / sc;
        sum = fma(q, q, sum);
    }
    const double err = sqrt(sum / (double)RG_NY);
    r.att++;
    // one step factor for both outcomes (lanes of a wave take both branches,
    // so a factor computed in each would cost two pow per attempt)
    const bool ok = err <= 1.0 && rg_finite(y5) && rg_finite(k7);
    const double fac = rg_dp_factor(ok ? err : (err > 1.0 ? err : __builtin_inf()), ok ? r.fm : 1.0);
    r.h = hs * fac;
    if (ok) {
        for (int i = 0; i < RG_NY; i++) { r.y[i] = y5[i]; r.k1[i] = k7[i]; }
        r.t = r.t + hs;
        r.acc++;
        r.fm = 5.0;
        if (a.has_box && rg_outside(a, r.y)) { r.st = RG_RAY_EXITED_BOX; return; }
    } else {
        r.fm = 1.0;
    }
    if (r.h < a.hmin) r.st = RG_RAY_STEP_UNDERFLOW;
}

__device__ __forceinline__ void rg_dp_load(const rg_kargs &a, const rg_P &P, long long id, rg_dp_ray &r) {
    const long long n = a.n;
    for (int i = 0; i < RG_DIM; i++) {
        r.y[i] = a.x0[i * n + id];
        r.y[RG_DIM + i] = a.k0[i * n + id];
    }
    r.t = a.t0 ? a.t0[id] : 0.0;
    r.om = a.omega[id];
    r.h = a.h0;
    r.fm = 5.0;
    r.acc = 0;
    r.att = 0;
    r.budget = a.budget ? a.budget[id] : a.max_steps;
    if (a.budget_cap > 0 && r.budget > a.budget_cap) r.budget = a.budget_cap;
    r.st = -1;
}

__device__ __forceinline__ void rg_dp_store(const rg_kargs &a, long long id, rg_dp_ray &r) {
    const long long n = a.n;
    if (!rg_finite(r.y)) r.st = RG_RAY_NONFINITE;
    for (int i = 0; i < RG_DIM; i++) {
        a.x_out[i * n + id] = r.y[i];
        a.k_out[i * n + id] = r.y[RG_DIM + i];
    }
    if (a.t_out) a.t_out[id] = r.t;
    if (a.status_out) a.status_out[id] = r.st;
    if (a.steps_out) a.steps_out[id] = r.acc;
    if (a.attempts_out) a.attempts_out[id] = r.att;
}

// Persistent adaptive kernel with wave-level compaction: every `compact`
// attempts (and whenever the whole wave is idle) the finished lanes of a
// wave are refilled with new rays from a global queue.  One atomic per wave
// reserves as many rays as the wave has free lanes; ballot + popcount give
// each free lane its rank, so the new rays land in the free lanes in order.
extern "C" __global__ void __launch_bounds__(512) rg_dopri_persistent(rg_kargs a) {
    rg_stage_tables(a);
    const rg_P P = rg_params(a);
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    rg_dp_ray r;
    r.st = 0;
    long long id = -1;
    bool alive = false, need_k1 = false, exhausted = false;
    int iter = 0;
    const int C = a.compact;
    for (;;) {
        const unsigned long long live = __ballot(alive);
        const bool due = (live == 0ull) || (C > 0 && iter % C == 0);
        if (!exhausted && due && live != ~0ull) {
            const unsigned long long freem = ~live;
            const int nfree = __popcll(freem);
            const int leader = __ffsll((long long)freem) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)nfree);
            base = __shfl(base, leader);
            if (!alive) {
                const long long cand = (long long)base + __popcll(freem & below);
                if (cand < a.n_run) {
                    id = cand;
                    rg_dp_load(a, P, id, r);
                    alive = true;
                    need_k1 = true;
                }
            }
            if ((long long)base + nfree >= a.n_run) exhausted = true;
        }
        if (__ballot(alive) == 0ull) break;
        iter++;
        if (alive) {
            if (need_k1) {
                rg_rhs<true>(r.y, r.om, r.t, P, r.k1);
                need_k1 = false;
            }
            rg_dp_attempt(a, P, r);
            if (r.st >= 0) {
                rg_dp_store(a, id, r);
                alive = false;
            }
        }
    }
}

// Plain adaptive form: one attempt per launch for every ray, state in HBM.
extern "C" __global__ void __launch_bounds__(512) rg_dopri_plain_init(rg_kargs a) {
    rg_stage_tables(a);
    const long long n = a.n;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= a.n_run) return;
    const rg_P P = rg_params(a);
    rg_dp_ray r;
    rg_dp_load(a, P, id, r);
    rg_rhs<true>(r.y, r.om, r.t, P, r.k1);
    for (int c = 0; c < RG_NY; c++) {
        a.s_y[(long long)c * n + id] = r.y[c];
        a.s_k1[(long long)c * n + id] = r.k1[c];
    }
    a.s_t[id] = r.t;
    a.s_h[id] = r.h;
    a.s_fm[id] = r.fm;
    a.s_acc[id] = 0;
    a.s_att[id] = 0;
    a.s_st[id] = -1;
}

extern "C" __global__ void __launch_bounds__(512) rg_dopri_plain_step(rg_kargs a) {
    rg_stage_tables(a);
    const long long n = a.n;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= a.n_run) return;
    int st = a.s_st[id];
    if (st >= 0) return;
    const rg_P P = rg_params(a);
    rg_dp_ray r;
    for (int c = 0; c < RG_NY; c++) {
        r.y[c] = a.s_y[(long long)c * n + id];
        r.k1[c] = a.s_k1[(long long)c * n + id];
    }
    r.t = a.s_t[id];
    r.h = a.s_h[id];
    r.fm = a.s_fm[id];
    r.om = a.omega[id];
    r.acc = a.s_acc[id];
    r.att = a.s_att[id];
    r.budget = a.budget ? a.budget[id] : a.max_steps;
    if (a.budget_cap > 0 && r.budget > a.budget_cap) r.budget = a.budget_cap;
    r.st = -1;
    rg_dp_attempt(a, P, r);
    for (int c = 0; c < RG_NY; c++) {
        a.s_y[(long long)c * n + id] = r.y[c];
        a.s_k1[(long long)c * n + id] = r.k1[c];
    }
    a.s_t[id] = r.t;
    a.s_h[id] = r.h;
    a.s_fm[id] = r.fm;
    a.s_acc[id] = r.acc;
    a.s_att[id] = r.att;
    a.s_st[id] = r.st;
    if (r.st >= 0) rg_dp_store(a, id, r);
    else if (a.count_alive) atomicAdd(a.counter, 1);
}

// --------------------------------------------------------- Newton solve --
// k_c <- k_c - D/(dD/dk_c) per ray until |D| <= tol; the largest final |D|
// is reduced per wave and folded into a device scalar with one atomic max on
// its bit pattern (non-negative doubles order like their bits).
extern "C" __global__ void __launch_bounds__(512) rg_newton_k(rg_kargs a) {
    rg_stage_tables(a);
    const long long n = a.n;
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double absD = 0.0;
    if (r < a.n_run) {
        const rg_P P = rg_params(a);
        double y[RG_NY], g[RG_DIM + 1];
        for (int i = 0; i < RG_DIM; i++) {
            y[i] = a.x0[i * n + r];
            y[RG_DIM + i] = a.k_io[i * n + r];
        }
        const double om = a.omega[r], t = a.t0 ? a.t0[r] : 0.0;
        const int c = a.component;
        int it = 0, done = 0;
        for (;;) {
            rg_Dk(y, om, t, P, g);
            if (fabs(g[0]) <= a.tol) { done = 1; break; }
            if (it >= a.max_iter || !__builtin_isfinite(g[0])) break;
            double dk = 0.0;
            for (int i = 0; i < RG_DIM; i++) dk = (i == c) ? g[1 + i] : dk;
            double kc = 0.0;
            for (int i = 0; i < RG_DIM; i++) kc = (i == c) ? y[RG_DIM + i] : kc;
            kc = kc - g[0] / dk;
            for (int i = 0; i < RG_DIM; i++) y[RG_DIM + i] = (i == c) ? kc : y[RG_DIM + i];
            it++;
        }
        for (int i = 0; i < RG_DIM; i++) a.k_io[i * n + r] = y[RG_DIM + i];
        if (a.D_out) a.D_out[r] = g[0];
        if (a.iters_out) a.iters_out[r] = done ? it : -1;
        absD = __builtin_isfinite(g[0]) ? fabs(g[0]) : __builtin_inf();
    }
    if (a.max_abs_D) {
        for (int off = 32; off > 0; off >>= 1) absD = fmax(absD, __shfl_xor(absD, off));
        if ((threadIdx.x & 63) == 0)
            atomicMax((unsigned long long *)a.max_abs_D, (unsigned long long)__double_as_longlong(absD));
    }
}

// ------------------------------------------------------ trace statistics --
// Rays per termination status, accepted steps and attempts summed and their
// largest per-ray values, over a finished trace's outputs.  Each lane
// counts a grid-stride share of the rays, the wave sums them by shuffles,
// and lane 0 folds the wave's totals into the counters with one atomic
// each.  stats: [0..4] rays per status, [5] other status values, [6] steps,
// [7] attempts, [8] most steps, [9] most attempts.
#define RG_NSTATS 10
extern "C" __global__ void __launch_bounds__(512) rg_stats(rg_kargs a) {
    unsigned long long c[RG_NSTATS];
    for (int i = 0; i < RG_NSTATS; i++) c[i] = 0;
    const long long G = (long long)gridDim.x * blockDim.x;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < a.n_run; r += G) {
        const int s = a.status_out ? a.status_out[r] : 0;
        for (int k = 0; k < 6; k++) c[k] += ((unsigned)s < 5u ? s : 5) == k;
        const unsigned long long st = a.steps_out ? (unsigned)a.steps_out[r] : 0u;
        const unsigned long long at = a.attempts_out ? (unsigned)a.attempts_out[r] : 0u;
        c[6] += st;
        c[7] += at;
        c[8] = st > c[8] ? st : c[8];
        c[9] = at > c[9] ? at : c[9];
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int i = 0; i < RG_NSTATS; i++) {
            const unsigned long long o = __shfl_xor(c[i], off);
            c[i] = i < 8 ? c[i] + o : (o > c[i] ? o : c[i]);
        }
    if ((threadIdx.x & 63) == 0) {
        for (int i = 0; i < 8; i++)
            if (c[i]) atomicAdd(a.stats + i, c[i]);
        for (int i = 8; i < RG_NSTATS; i++) atomicMax(a.stats + i, c[i]);
    }
}

// ----------------------------------------------------------------- utils --
extern "C" __global__ void __launch_bounds__(512) rg_fill_f64(rg_kargs a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.fill_n) a.fill_p[i] = a.fill_v;
}

extern "C" __global__ void __launch_bounds__(512) rg_eval_points(rg_kargs a) {
    rg_stage_tables(a);
    const long long n = a.n;
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_run) return;
    const rg_P P = rg_params(a);
    double y[RG_NY], f[RG_NY];
    for (int c = 0; c < RG_NY; c++) y[c] = a.x0[(long long)c * n + r];
    const double om = a.omega[r], t = a.t0 ? a.t0[r] : 0.0;
    if (a.x_out) {
        rg_rhs(y, om, t, P, f);
        for (int c = 0; c < RG_NY; c++) a.x_out[(long long)c * n + r] = f[c];
    }
    if (a.t_out) a.t_out[r] = rg_D(y, om, t, P);
}

// --------------------------------------------------------------- adjoint --
#if RG_HAS_VJP
#define RG_NGRAD1 (RG_NGRAD > 0 ? RG_NGRAD : 1)
__shared__ double rg_red_lds[8 * RG_NGRAD1];

// Per-lane gradient partials in LDS, parameter-major ([slot][lane], so a
// wave's adds hit consecutive doubles): gp[i] += v is one LDS add of the
// lane's own slot (an atomic, so that the compiler does not keep the slots
// in registers across the loop; each slot has one writer, so the sum is the
// same sequence of additions as in registers).
struct rg_GPRef {
    double *q;
    __device__ __forceinline__ void operator+=(double v) const {
        __hip_atomic_fetch_add(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ __forceinline__ operator double() const { return *q; }
};
struct rg_GPLds {
    double *p;
    __device__ __forceinline__ rg_GPRef operator[](int i) const { return rg_GPRef{p + i * RG_ADJ_BLOCK}; }
};

// Discrete adjoint of the RK4 map (exact transpose of one step):
//   Kb4 = dt/6 lam,            Yb4 = J(Y4)^T Kb4
//   Kb3 = dt/3 lam + dt Yb4,   Yb3 = J(Y3)^T Kb3
//   Kb2 = dt/3 lam + dt/2 Yb3, Yb2 = J(Y2)^T Kb2
//   Kb1 = dt/6 lam + dt/2 Yb2, Yb1 = J(Y1)^T Kb1
//   lam <- lam + Yb1 + Yb2 + Yb3 + Yb4,  dL/dtheta += sum_i (df/dtheta(Y_i))^T Kb_i
// Segments between forward checkpoints are walked last to first; the states
// of a segment are recomputed from its checkpoint into per-lane scratch
// (coalesced [j][c][lane]) and read back in reverse.
// Reverse of one RK4 step: the discrete adjoint recurrence with one VJP
// per stage, last stage first.  The stage states come from the segment
// buffer sp (stage s component c at sp[(s RG_NY + c) SL], t at
// sp[RG_ADJ_NS RG_NY SL]).
//
// RG_ADJ_RECOMPUTE (a cheap right-hand side): only Y1 is stored; Y2..Y4 are
// recomputed here with three right-hand sides and kept in registers, the
// four VJPs inlined.  Otherwise the segment's forward recomputation stored
// all four states and the stages are a loop around one copy of the VJP
// (four inlined copies of a large VJP cost registers and code and add no
// parallelism, the stages depending on each other), the next stage's state
// loaded before the current VJP runs.  (Measured on the spline workload,
// one wave per SIMD: inlined recomputation 23.6 ms, looped recomputation
// with LDS 27.2 ms, stored states 28.3 ms; on the anisotropic workload the
// stored states are 13 % faster than the recomputation.)
#if RG_ADJ_RECOMPUTE
#define RG_ADJ_NS 1
#else
#define RG_ADJ_NS 4
#endif

template <typename GPT>
__device__ __forceinline__ void rg_adjoint_step(const double *sp, long long SL, double om, double dt,
                                                const rg_P &P, double *lam, GPT gp, rg_GA &G) {
    const double h2 = 0.5 * dt, dt3 = dt / 3.0, dt6 = dt / 6.0;
    const double tj = sp[(long long)RG_ADJ_NS * RG_NY * SL];
    double Kb[RG_NY], Yb[RG_NY], lsum[RG_NY];
#if RG_ADJ_RECOMPUTE
    double Y1[RG_NY], Y2[RG_NY], Y3[RG_NY], Y4[RG_NY], K[RG_NY];
    for (int c = 0; c < RG_NY; c++) Y1[c] = sp[(long long)c * SL];
    rg_rhs(Y1, om, tj, P, K);
    for (int c = 0; c < RG_NY; c++) Y2[c] = fma(h2, K[c], Y1[c]);
    rg_rhs(Y2, om, tj + h2, P, K);
    for (int c = 0; c < RG_NY; c++) Y3[c] = fma(h2, K[c], Y1[c]);
    rg_rhs(Y3, om, tj + h2, P, K);
    for (int c = 0; c < RG_NY; c++) Y4[c] = fma(dt, K[c], Y1[c]);
    // The stage states pass through an empty asm, so the compiler sees them
    // as new values: each VJP recomputes its forward intermediates instead
    // of keeping those of the three right-hand sides above live across the
    // reverse stages (spline workload: 528 AGPR moves per step and the
    // scratch spills gone, the loop 7 % shorter, the adjoint 3 % faster).
    for (int c = 0; c < RG_NY; c++) asm volatile("" : "+v"(Y1[c]), "+v"(Y2[c]), "+v"(Y3[c]));
    for (int c = 0; c < RG_NY; c++) Kb[c] = dt6 * lam[c];
    rg_vjp(Y4, om, tj + dt, P, Kb, Yb, gp, G);
    for (int c = 0; c < RG_NY; c++) { lsum[c] = Yb[c]; Kb[c] = fma(dt, Yb[c], dt3 * lam[c]); }
    rg_vjp(Y3, om, tj + h2, P, Kb, Yb, gp, G);
    for (int c = 0; c < RG_NY; c++) { lsum[c] += Yb[c]; Kb[c] = fma(h2, Yb[c], dt3 * lam[c]); }
    rg_vjp(Y2, om, tj + h2, P, Kb, Yb, gp, G);
    for (int c = 0; c < RG_NY; c++) { lsum[c] += Yb[c]; Kb[c] = fma(h2, Yb[c], dt6 * lam[c]); }
    rg_vjp(Y1, om, tj, P, Kb, Yb, gp, G);
    for (int c = 0; c < RG_NY; c++) lam[c] = lam[c] + (lsum[c] + Yb[c]);
#else
    double Y[RG_NY];
    for (int c = 0; c < RG_NY; c++) Y[c] = sp[(long long)(3 * RG_NY + c) * SL];
    for (int c = 0; c < RG_NY; c++) Kb[c] = dt6 * lam[c];
#pragma unroll 1
    for (int s = 3; s >= 0; s--) {
        double Yn[RG_NY];
        const int sn = s > 0 ? s - 1 : 0;
        for (int c = 0; c < RG_NY; c++) Yn[c] = sp[(long long)(sn * RG_NY + c) * SL];
        rg_vjp(Y, om, s == 0 ? tj : (s == 3 ? tj + dt : tj + h2), P, Kb, Yb, gp, G);
        const double ca = s == 3 ? dt : h2, cb = s == 1 ? dt6 : dt3;
        for (int c = 0; c < RG_NY; c++) {
            lsum[c] = s == 3 ? Yb[c] : lsum[c] + Yb[c];
            Kb[c] = fma(ca, Yb[c], cb * lam[c]);
            Y[c] = Yn[c];
        }
    }
    for (int c = 0; c < RG_NY; c++) lam[c] = lam[c] + lsum[c];
#endif
}

// Parameter-gradient partials of this workgroup: the scalar slots reduced
// in a fixed order (wave shuffles, then waves in order), the spline
// coefficients from the LDS accumulator; written (add = false) or added to
// what the workgroup's earlier launches left (add = true).
// The partials' slot of this workgroup (one per workgroup), or of this
// wave (RG_DET_GRAD: one per wave, the workgroup's scalar sums in the slot
// of its first wave).
__device__ __forceinline__ double *rg_part_slot(const rg_kargs &a) {
    if (!a.gpart) return nullptr;
#if RG_DET_GRAD
    return a.gpart + ((long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * a.part_stride;
#else
    return a.gpart + (long long)blockIdx.x * a.part_stride;
#endif
}

template <typename GPT>
__device__ __forceinline__ void rg_write_partials(const rg_kargs &a, GPT gp, rg_GA &G, bool add) {
#if RG_NSPLTAB > 0
    for (int k = 0; k < RG_NSPLTAB; k++) G.flush(k);
#endif
    (void)G;
    if (!a.gpart) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int s = 0; s < RG_NGRAD; s++) {
        double v = gp[s];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) rg_red_lds[wave * RG_NGRAD1 + s] = v;
    }
    __syncthreads();
#if RG_DET_GRAD
    // scalar sums into the first wave's slot; the spline tables are already
    // in each wave's slot
    double *out = a.gpart + (long long)blockIdx.x * nw * a.part_stride;
#else
    double *out = a.gpart + (long long)blockIdx.x * a.part_stride;
#endif
    for (int s = threadIdx.x; s < RG_NGRAD; s += blockDim.x) {
        double v = 0.0;
        for (int w = 0; w < nw; w++) v += rg_red_lds[w * RG_NGRAD1 + s];
        out[s] = add ? out[s] + v : v;
    }
#if RG_NSPLTAB > 0 && !RG_DET_GRAD
    for (int i = threadIdx.x; i < RG_SPL_TOTAL; i += blockDim.x)
        out[RG_NGRAD + i] = add ? out[RG_NGRAD + i] + rg_spl_grad_lds[i] : rg_spl_grad_lds[i];
#endif
}

#if RG_GP_LDS
__shared__ double rg_gp_lds[RG_NGRAD1 * RG_ADJ_BLOCK];
#define RG_ADJ_OCCUPANCY __attribute__((amdgpu_waves_per_eu(3, 8)))
#else
#define RG_ADJ_OCCUPANCY
#endif
extern "C" __global__ void __launch_bounds__(RG_ADJ_BLOCK) RG_ADJ_OCCUPANCY rg_rk4_adjoint(rg_kargs a) {
    rg_stage_tables(a);
#if RG_NSPLTAB > 0 && !RG_DET_GRAD
    for (int i = threadIdx.x; i < RG_SPL_TOTAL; i += blockDim.x) rg_spl_grad_lds[i] = 0.0;
    __syncthreads();
#endif
    const rg_P P = rg_params(a);
    rg_GA G;
    G.init(rg_part_slot(a));  // (RG_DET_GRAD: the slots were zeroed before the launch)
#if RG_GP_LDS
    for (int i = 0; i < RG_NGRAD1; i++) rg_gp_lds[i * RG_ADJ_BLOCK + threadIdx.x] = 0.0;
    const rg_GPLds gp{rg_gp_lds + threadIdx.x};
#else
    double gp[RG_NGRAD1];
    for (int i = 0; i < RG_NGRAD1; i++) gp[i] = 0.0;
#endif
    const long long n = a.n;
    const long long GL = (long long)gridDim.x * blockDim.x;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double dt = a.dt;
    const int ce = a.ckpt_every;
    const long long SL = a.scratch_lanes;
    for (long long rid = gid; rid < a.n_run; rid += GL) {
        double lam[RG_NY];
        for (int i = 0; i < RG_DIM; i++) {
            lam[i] = a.lam_x[i * n + rid];
            lam[RG_DIM + i] = a.lam_k ? a.lam_k[i * n + rid] : 0.0;
        }
        const int ns = a.steps_out[rid];
        const double om = a.omega[rid];
        const int nseg = (a.n_steps + ce - 1) / ce;
        for (int seg = nseg - 1; seg >= 0; seg--) {
            const int s0 = seg * ce;
            if (s0 >= ns) continue;
            const int s1 = s0 + ce < ns ? s0 + ce : ns;
            double y[RG_NY], t;
            const double *cp = a.ckpt + (long long)seg * (RG_NY + 1) * n + rid;
            for (int c = 0; c < RG_NY; c++) y[c] = cp[(long long)c * n];
            t = cp[(long long)RG_NY * n];
            for (int j = s0; j < s1; j++) {
                double *sp = a.scratch + (long long)(j - s0) * (RG_ADJ_NS * RG_NY + 1) * SL + gid;
                for (int c = 0; c < RG_NY; c++) sp[(long long)c * SL] = y[c];
                sp[(long long)RG_ADJ_NS * RG_NY * SL] = t;
                double yn[RG_NY];
                rg_rk4_step(y, om, t, dt, P, yn, RG_ADJ_NS > 1 ? sp : nullptr, SL);
                for (int c = 0; c < RG_NY; c++) y[c] = yn[c];
                t = t + dt;
            }
            for (int j = s1 - 1; j >= s0; j--)
                rg_adjoint_step(a.scratch + (long long)(j - s0) * (RG_ADJ_NS * RG_NY + 1) * SL + gid, SL, om,
                                dt, P, lam, gp, G);
        }
        for (int i = 0; i < RG_DIM; i++) {
            if (a.gx0) a.gx0[i * n + rid] = lam[i];
            if (a.gk0) a.gk0[i * n + rid] = lam[RG_DIM + i];
        }
    }
    rg_write_partials(a, gp, G, false);
}

// ------------------------------------------------------- plain adjoint --
// One launch per step, state and adjoint in HBM between launches (the
// per-step form of the same checkpointed adjoint): per segment, a launch
// loads the checkpoint, one launch per step recomputes the state and
// stores the stage states (segment buffer [j][RG_ADJ_NS NY + 1][n]), and
// one launch per step runs the reverse step, its workgroup adding its
// gradient partials to its own slot.  Rays stopped before a step skip it.
extern "C" __global__ void __launch_bounds__(512) rg_adjp_init(rg_kargs a) {
    const long long n = a.n, r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a.gpart) {  // this workgroup's slot, or its waves' slots (same grid as rg_adjp_rev)
#if RG_DET_GRAD
        const long long m = (long long)(blockDim.x >> 6) * a.part_stride;
#else
        const long long m = a.part_stride;
#endif
        for (long long s = threadIdx.x; s < m; s += blockDim.x) a.gpart[(long long)blockIdx.x * m + s] = 0.0;
    }
    if (r >= a.n_run) return;
    for (int i = 0; i < RG_DIM; i++) {
        a.s_lam[i * n + r] = a.lam_x[i * n + r];
        a.s_lam[(RG_DIM + i) * n + r] = a.lam_k ? a.lam_k[i * n + r] : 0.0;
    }
}

extern "C" __global__ void __launch_bounds__(512) rg_adjp_seg(rg_kargs a) {
    const long long n = a.n, r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_run) return;
    const double *cp = a.ckpt + (long long)a.ckpt_idx * (RG_NY + 1) * n + r;
    for (int c = 0; c < RG_NY; c++) a.s_y[c * n + r] = cp[(long long)c * n];
    a.s_t[r] = cp[(long long)RG_NY * n];
}

extern "C" __global__ void __launch_bounds__(512) rg_adjp_fwd(rg_kargs a) {
    rg_stage_tables(a);
    const long long n = a.n, r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_run || a.step >= a.steps_out[r]) return;
    const rg_P P = rg_params(a);
    double y[RG_NY], yn[RG_NY];
    for (int c = 0; c < RG_NY; c++) y[c] = a.s_y[c * n + r];
    const double t = a.s_t[r];
    double *sp = a.scratch + (long long)(a.step - a.seg_s0) * (RG_ADJ_NS * RG_NY + 1) * n + r;
    for (int c = 0; c < RG_NY; c++) sp[(long long)c * n] = y[c];
    sp[(long long)RG_ADJ_NS * RG_NY * n] = t;
    rg_rk4_step(y, a.omega[r], t, a.dt, P, yn, RG_ADJ_NS > 1 ? sp : nullptr, n);
    for (int c = 0; c < RG_NY; c++) a.s_y[c * n + r] = yn[c];
    a.s_t[r] = t + a.dt;
}

extern "C" __global__ void __launch_bounds__(RG_ADJ_BLOCK) rg_adjp_rev(rg_kargs a) {
    rg_stage_tables(a);
#if RG_NSPLTAB > 0 && !RG_DET_GRAD
    for (int i = threadIdx.x; i < RG_SPL_TOTAL; i += blockDim.x) rg_spl_grad_lds[i] = 0.0;
    __syncthreads();
#endif
    const rg_P P = rg_params(a);
    rg_GA G;
    G.init(rg_part_slot(a));
    double gp[RG_NGRAD1];
    for (int i = 0; i < RG_NGRAD1; i++) gp[i] = 0.0;
    const long long n = a.n, r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < a.n_run && a.step < a.steps_out[r]) {
        double lam[RG_NY];
        for (int c = 0; c < RG_NY; c++) lam[c] = a.s_lam[c * n + r];
        rg_adjoint_step(a.scratch + (long long)(a.step - a.seg_s0) * (RG_ADJ_NS * RG_NY + 1) * n + r, n,
                        a.omega[r], a.dt, P, lam, gp, G);
        for (int c = 0; c < RG_NY; c++) a.s_lam[c * n + r] = lam[c];
    }
    rg_write_partials(a, gp, G, true);
}

extern "C" __global__ void __launch_bounds__(512) rg_adjp_finish(rg_kargs a) {
    const long long n = a.n, r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_run) return;
    for (int i = 0; i < RG_DIM; i++) {
        if (a.gx0) a.gx0[i * n + r] = a.s_lam[i * n + r];
        if (a.gk0) a.gk0[i * n + r] = a.s_lam[(RG_DIM + i) * n + r];
    }
}

// Sum the per-workgroup partials in workgroup order and scatter them to the
// parameter gradient arrays (already zeroed).
extern "C" __global__ void __launch_bounds__(512) rg_grad_finalize(rg_kargs a) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.part_stride) return;
    double v = 0.0;
    for (int p = 0; p < a.n_part; p++) v += a.gpart[(long long)p * a.part_stride + e];
    if (e < RG_NGRAD) {
#if RG_NGRAD > 0
        double *dst = a.dparams[rg_grad_param[e]];
        if (dst) dst[rg_grad_elem[e]] = v;
#endif
    } else {
#if RG_NSPLTAB > 0
        const long long i = e - RG_NGRAD;
        for (int k = 0; k < RG_NSPLTAB; k++)
            if (i >= rg_spl_off[k] && i < rg_spl_off[k] + rg_spl_len[k]) {
                double *dst = a.dparams[rg_spl_param[k]];
                if (dst) dst[i - rg_spl_off[k]] = v;
            }
#endif
    }
}
#endif
