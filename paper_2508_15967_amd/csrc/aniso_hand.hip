// Hand-derived comparison kernels for the anisotropic medium (see
// include/raygraph_hand.h).  Same RK4 scheme, same checkpointed discrete
// adjoint and same launch structure as the compiled kernels; only the
// right-hand side and its vector-Jacobian product are written by hand:
//
//   f_x = A k / w,  f_k = (1/w) sum_b s_b q_b g_b (x - c_b)/w_b^2,
//   q_b = k.M_b.k,  g_b = exp(-|x - c_b|^2/w_b^2),  A = I + sum_b s_b g_b M_b
//
//   (J^T v)_x = (1/w) sum_b s_b g_b [ -2/w_b^2 (v_x.M_b k + q_b/w_b^2 v_k.dx) dx
//                                      + q_b/w_b^2 v_k ]
//   (J^T v)_k = (1/w) [ v_x + sum_b s_b g_b (M_b v_x + 2/w_b^2 (v_k.dx) M_b k) ]
//   d(v.f)/ds_b = (1/w) g_b (v_x.M_b k + q_b/w_b^2 v_k.dx)
#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>

#include "../../include/raygraph_hand.h"

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string &m) {
    g_err = m;
    return code;
}

struct Args {
    const double *x0, *k0, *omega, *s;
    double *x_out, *k_out, *ckpt;
    const double *lam_x, *lam_k;
    double *gx0, *gk0, *scratch, *gpart;
    double dt;
    long long n, lanes;
    int n_steps, ckpt_every;
};

template <int NB>
__device__ __forceinline__ void hand_rhs(const rg_hand_aniso &m, const double *sv, const double *y,
                                         double winv, double *f) {
    double ak0 = y[3], ak1 = y[4], ak2 = y[5];
    double fk0 = 0.0, fk1 = 0.0, fk2 = 0.0;
    const double k0 = y[3], k1 = y[4], k2 = y[5];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        if (b >= m.nb) break;
        const double dx = y[0] - m.c[b][0], dy = y[1] - m.c[b][1], dz = y[2] - m.c[b][2];
        const double iw = m.inv_w2[b];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double sg = sv[b] * exp(-r2 * iw);
        const double *M = m.m[b];
        const double mk0 = fma(M[2], k2, fma(M[1], k1, M[0] * k0));
        const double mk1 = fma(M[4], k2, fma(M[3], k1, M[1] * k0));
        const double mk2 = fma(M[5], k2, fma(M[4], k1, M[2] * k0));
        const double q = fma(k2, mk2, fma(k1, mk1, k0 * mk0));
        ak0 = fma(sg, mk0, ak0);
        ak1 = fma(sg, mk1, ak1);
        ak2 = fma(sg, mk2, ak2);
        const double tq = sg * q * iw;
        fk0 = fma(tq, dx, fk0);
        fk1 = fma(tq, dy, fk1);
        fk2 = fma(tq, dz, fk2);
    }
    f[0] = ak0 * winv; f[1] = ak1 * winv; f[2] = ak2 * winv;
    f[3] = fk0 * winv; f[4] = fk1 * winv; f[5] = fk2 * winv;
}

template <int NB>
__device__ __forceinline__ void hand_vjp(const rg_hand_aniso &m, const double *sv, const double *y,
                                         double winv, const double *v, double *jv, double *gs) {
    const double k0 = y[3], k1 = y[4], k2 = y[5];
    double jx0 = 0.0, jx1 = 0.0, jx2 = 0.0;
    double jk0 = v[0], jk1 = v[1], jk2 = v[2];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        if (b >= m.nb) break;
        const double dx = y[0] - m.c[b][0], dy = y[1] - m.c[b][1], dz = y[2] - m.c[b][2];
        const double iw = m.inv_w2[b];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const double g = exp(-r2 * iw);
        const double sg = sv[b] * g;
        const double *M = m.m[b];
        const double mk0 = fma(M[2], k2, fma(M[1], k1, M[0] * k0));
        const double mk1 = fma(M[4], k2, fma(M[3], k1, M[1] * k0));
        const double mk2 = fma(M[5], k2, fma(M[4], k1, M[2] * k0));
        const double mv0 = fma(M[2], v[2], fma(M[1], v[1], M[0] * v[0]));
        const double mv1 = fma(M[4], v[2], fma(M[3], v[1], M[1] * v[0]));
        const double mv2 = fma(M[5], v[2], fma(M[4], v[1], M[2] * v[0]));
        const double q = fma(k2, mk2, fma(k1, mk1, k0 * mk0));
        const double vxmk = fma(v[2], mk2, fma(v[1], mk1, v[0] * mk0));
        const double vkdx = fma(v[5], dz, fma(v[4], dy, v[3] * dx));
        const double qi = q * iw;
        const double a = fma(qi, vkdx, vxmk);          // v_x.Mk + q/w^2 v_k.dx
        gs[b] = fma(g * winv, a, gs[b]);
        const double cx = -2.0 * iw * a;
        jx0 = fma(sg, fma(cx, dx, qi * v[3]), jx0);
        jx1 = fma(sg, fma(cx, dy, qi * v[4]), jx1);
        jx2 = fma(sg, fma(cx, dz, qi * v[5]), jx2);
        const double ck = 2.0 * iw * vkdx;
        jk0 = fma(sg, fma(ck, mk0, mv0), jk0);
        jk1 = fma(sg, fma(ck, mk1, mv1), jk1);
        jk2 = fma(sg, fma(ck, mk2, mv2), jk2);
    }
    jv[0] = jx0 * winv; jv[1] = jx1 * winv; jv[2] = jx2 * winv;
    jv[3] = jk0 * winv; jv[4] = jk1 * winv; jv[5] = jk2 * winv;
}

template <int NB>
__device__ __forceinline__ void hand_step(const rg_hand_aniso &m, const double *sv, const double *y,
                                          double winv, double dt, double *yn) {
    const double h2 = 0.5 * dt, dt6 = dt / 6.0;
    double K[6], acc[6], Y[6];
    hand_rhs<NB>(m, sv, y, winv, K);
    for (int i = 0; i < 6; i++) { acc[i] = K[i]; Y[i] = fma(h2, K[i], y[i]); }
    hand_rhs<NB>(m, sv, Y, winv, K);
    for (int i = 0; i < 6; i++) { acc[i] = fma(2.0, K[i], acc[i]); Y[i] = fma(h2, K[i], y[i]); }
    hand_rhs<NB>(m, sv, Y, winv, K);
    for (int i = 0; i < 6; i++) { acc[i] = fma(2.0, K[i], acc[i]); Y[i] = fma(dt, K[i], y[i]); }
    hand_rhs<NB>(m, sv, Y, winv, K);
    for (int i = 0; i < 6; i++) { acc[i] = acc[i] + K[i]; yn[i] = fma(dt6, acc[i], y[i]); }
}

template <int NB>
__global__ void __launch_bounds__(512) hand_trace(rg_hand_aniso m, Args a) {
    const long long n = a.n;
    const long long G = (long long)gridDim.x * blockDim.x;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += G) {
        double y[6];
        for (int i = 0; i < 3; i++) { y[i] = a.x0[i * n + r]; y[3 + i] = a.k0[i * n + r]; }
        const double winv = 1.0 / a.omega[r];
        double t = 0.0;
        int ck = 0, cd = 0;
        for (int s = 0; s < a.n_steps; s++) {
            if (a.ckpt_every > 0 && cd == 0) {
                double *cp = a.ckpt + (long long)ck * 7 * n + r;
                for (int c = 0; c < 6; c++) cp[(long long)c * n] = y[c];
                cp[6 * n] = t;
                ck++;
                cd = a.ckpt_every;
            }
            cd--;
            double yn[6];
            hand_step<NB>(m, a.s, y, winv, a.dt, yn);
            for (int c = 0; c < 6; c++) y[c] = yn[c];
            t = t + a.dt;
        }
        for (int i = 0; i < 3; i++) { a.x_out[i * n + r] = y[i]; a.k_out[i * n + r] = y[3 + i]; }
    }
}

template <int NB>
__global__ void __launch_bounds__(512) hand_adjoint(rg_hand_aniso m, Args a) {
    __shared__ double red[8][NB];
    const long long n = a.n, SL = a.lanes;
    const long long G = (long long)gridDim.x * blockDim.x;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double dt = a.dt, h2 = 0.5 * dt, dt3 = dt / 3.0, dt6 = dt / 6.0;
    const int ce = a.ckpt_every;
    double gs[NB];
    for (int b = 0; b < NB; b++) gs[b] = 0.0;
    for (long long r = gid; r < n; r += G) {
        double lam[6];
        for (int i = 0; i < 3; i++) {
            lam[i] = a.lam_x[i * n + r];
            lam[3 + i] = a.lam_k ? a.lam_k[i * n + r] : 0.0;
        }
        const double winv = 1.0 / a.omega[r];
        const int nseg = (a.n_steps + ce - 1) / ce;
        for (int seg = nseg - 1; seg >= 0; seg--) {
            const int s0 = seg * ce, s1 = s0 + ce < a.n_steps ? s0 + ce : a.n_steps;
            double y[6];
            const double *cp = a.ckpt + (long long)seg * 7 * n + r;
            for (int c = 0; c < 6; c++) y[c] = cp[(long long)c * n];
            for (int j = s0; j < s1; j++) {
                double *sp = a.scratch + (long long)(j - s0) * 6 * SL + gid;
                for (int c = 0; c < 6; c++) sp[(long long)c * SL] = y[c];
                double yn[6];
                hand_step<NB>(m, a.s, y, winv, dt, yn);
                for (int c = 0; c < 6; c++) y[c] = yn[c];
            }
            for (int j = s1 - 1; j >= s0; j--) {
                const double *sp = a.scratch + (long long)(j - s0) * 6 * SL + gid;
                double Y1[6], Y2[6], Y3[6], Y4[6], K[6];
                for (int c = 0; c < 6; c++) Y1[c] = sp[(long long)c * SL];
                hand_rhs<NB>(m, a.s, Y1, winv, K);
                for (int c = 0; c < 6; c++) Y2[c] = fma(h2, K[c], Y1[c]);
                hand_rhs<NB>(m, a.s, Y2, winv, K);
                for (int c = 0; c < 6; c++) Y3[c] = fma(h2, K[c], Y1[c]);
                hand_rhs<NB>(m, a.s, Y3, winv, K);
                for (int c = 0; c < 6; c++) Y4[c] = fma(dt, K[c], Y1[c]);
                double Kb[6], Yb[6], ls[6];
                for (int c = 0; c < 6; c++) Kb[c] = dt6 * lam[c];
                hand_vjp<NB>(m, a.s, Y4, winv, Kb, Yb, gs);
                for (int c = 0; c < 6; c++) { ls[c] = Yb[c]; Kb[c] = fma(dt, Yb[c], dt3 * lam[c]); }
                hand_vjp<NB>(m, a.s, Y3, winv, Kb, Yb, gs);
                for (int c = 0; c < 6; c++) { ls[c] += Yb[c]; Kb[c] = fma(h2, Yb[c], dt3 * lam[c]); }
                hand_vjp<NB>(m, a.s, Y2, winv, Kb, Yb, gs);
                for (int c = 0; c < 6; c++) { ls[c] += Yb[c]; Kb[c] = fma(h2, Yb[c], dt6 * lam[c]); }
                hand_vjp<NB>(m, a.s, Y1, winv, Kb, Yb, gs);
                for (int c = 0; c < 6; c++) lam[c] = lam[c] + (ls[c] + Yb[c]);
            }
        }
        for (int i = 0; i < 3; i++) {
            if (a.gx0) a.gx0[i * n + r] = lam[i];
            if (a.gk0) a.gk0[i * n + r] = lam[3 + i];
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int b = 0; b < NB; b++) {
        double v = gs[b];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][b] = v;
    }
    __syncthreads();
    if (threadIdx.x < NB) {
        double v = 0.0;
        for (int w = 0; w < nw; w++) v += red[w][threadIdx.x];
        a.gpart[(long long)blockIdx.x * NB + threadIdx.x] = v;
    }
}

__global__ void hand_finalize(const double *gpart, int n_part, int nb, int stride, double *out) {
    const int b = threadIdx.x;
    if (b >= nb) return;
    double v = 0.0;
    for (int p = 0; p < n_part; p++) v += gpart[(long long)p * stride + b];
    out[b] = v;
}


template <class K>
int32_t grid_for(K kern, int block, long long n, unsigned *grid) {
    int nb = 0, dev = 0, cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, block, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(-4, "occupancy query failed");
    long long want = (n + block - 1) / block, cap = (long long)(nb > 0 ? nb : 1) * cu;
    *grid = (unsigned)(want < cap ? want : cap);
    if (*grid == 0) *grid = 1;
    return 0;
}

}  // namespace

extern "C" {

const char *rg_hand_last_error(void) { return g_err.c_str(); }

int32_t rg_hand_aniso_trace(const rg_hand_aniso *m, uint32_t n, const double *x0, const double *k0,
                            const double *omega, const double *s, double dt, int32_t n_steps,
                            double *x_out, double *k_out, int32_t ckpt_every, double *ckpt,
                            int32_t block, void *stream) {
    if (!m || !x0 || !k0 || !omega || !s || !x_out || !k_out) return fail(-1, "NULL argument");
    if (m->nb < 0 || m->nb > 16) return fail(-5, "at most 16 blobs in this build");
    if (ckpt_every > 0 && !ckpt) return fail(-1, "checkpoints requested but ckpt is NULL");
    if (n == 0) return 0;
    if (block == 0) block = 256;
    if (block != 64 && block != 128 && block != 256 && block != 512) return fail(-1, "bad block size");
    Args a{};
    a.x0 = x0; a.k0 = k0; a.omega = omega; a.s = s; a.x_out = x_out; a.k_out = k_out;
    a.ckpt = ckpt; a.dt = dt; a.n = n; a.n_steps = n_steps; a.ckpt_every = ckpt_every;
    unsigned grid;
    if (grid_for(hand_trace<16>, block, n, &grid)) return -4;
    hipLaunchKernelGGL(hand_trace<16>, dim3(grid), dim3(block), 0, (hipStream_t)stream, *m, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : fail(-4, hipGetErrorString(e));
}

int32_t rg_hand_aniso_adjoint_workspace_size(uint32_t n, int32_t ckpt_every, int32_t block,
                                             size_t *bytes) {
    if (!bytes) return fail(-1, "NULL argument");
    *bytes = 0;
    if (ckpt_every <= 0) return fail(-1, "ckpt_every must be > 0");
    if (n == 0) return 0;
    if (block == 0) block = 256;
    if (block != 64 && block != 128 && block != 256 && block != 512) return fail(-1, "bad block size");
    unsigned grid;
    if (grid_for(hand_adjoint<16>, block, n, &grid)) return -4;
    const long long lanes = (long long)grid * block;
    const size_t scratch = (size_t)ckpt_every * 6 * lanes, part = (size_t)grid * 16;
    *bytes = ((8 * scratch + 255) & ~(size_t)255) + 8 * part;
    return 0;
}

int32_t rg_hand_aniso_adjoint(const rg_hand_aniso *m, uint32_t n, const double *omega, const double *s,
                              double dt, int32_t n_steps, int32_t ckpt_every, const double *ckpt,
                              const double *dL_dx_end, const double *dL_dk_end, double *dL_dx0,
                              double *dL_dk0, double *dL_ds, int32_t block, void *workspace,
                              size_t workspace_bytes, void *stream) {
    if (!m || !omega || !s || !ckpt || !dL_dx_end) return fail(-1, "NULL argument");
    if (m->nb < 0 || m->nb > 16) return fail(-5, "at most 16 blobs in this build");
    if (ckpt_every <= 0) return fail(-1, "ckpt_every must be > 0");
    if (n == 0) return 0;
    size_t need = 0;
    if (int32_t st = rg_hand_aniso_adjoint_workspace_size(n, ckpt_every, block, &need)) return st;
    if (!workspace || workspace_bytes < need) return fail(-1, "workspace smaller than the size query reports");
    if (block == 0) block = 256;
    unsigned grid;
    if (grid_for(hand_adjoint<16>, block, n, &grid)) return -4;
    const long long lanes = (long long)grid * block;
    const size_t scratch = (size_t)ckpt_every * 6 * lanes;
    Args a{};
    a.omega = omega; a.s = s; a.ckpt = const_cast<double *>(ckpt); a.lam_x = dL_dx_end;
    a.lam_k = dL_dk_end; a.gx0 = dL_dx0; a.gk0 = dL_dk0; a.dt = dt; a.n = n; a.lanes = lanes;
    a.n_steps = n_steps; a.ckpt_every = ckpt_every;
    a.scratch = (double *)workspace;
    a.gpart = (double *)((char *)workspace + ((8 * scratch + 255) & ~(size_t)255));
    hipLaunchKernelGGL(hand_adjoint<16>, dim3(grid), dim3(block), 0, (hipStream_t)stream, *m, a);
    if (dL_ds)
        hipLaunchKernelGGL(hand_finalize, dim3(1), dim3(64), 0, (hipStream_t)stream,
                           (const double *)a.gpart, (int)grid, m->nb, 16, dL_ds);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : fail(-4, hipGetErrorString(e));
}

}  // extern "C"
