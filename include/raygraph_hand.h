/*
 * Hand-derived comparison kernels for the anisotropic medium
 *
 *     D(x, k, omega) = k.A(x).k - omega^2,
 *     A(x) = I + sum_b s_b M_b exp(-|x - c_b|^2 / w_b^2),
 *
 * with every partial derivative written by hand instead of generated from
 * the expression graph.  They integrate the same ray equations (paper,
 * eqs. 2-3: dx/dt = -(dD/dk)/(dD/domega) = A k / omega,
 * dk/dt = (dD/dx)/(dD/domega) = (1/omega) sum_b s_b (k.M_b.k) g_b (x - c_b)/w_b^2)
 * with the same RK4 scheme and the same discrete adjoint, and serve as a
 * second GPU parity source and as the speed reference for the compiled
 * kernels.  Same conventions as raygraph.h: device pointers, SoA [dim][n]
 * ray arrays, asynchronous on the caller's HIP stream, negative status on
 * error with a message from rg_hand_last_error().
 */
#ifndef RAYGRAPH_HAND_H
#define RAYGRAPH_HAND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RG_HAND_MAX_BLOBS 32

/* Medium constants (host struct, passed to the kernels by value). */
typedef struct {
    int32_t nb;                              /* number of blobs, <= 32 */
    double c[RG_HAND_MAX_BLOBS][3];          /* centres */
    double inv_w2[RG_HAND_MAX_BLOBS];        /* 1 / w_b^2 */
    double m[RG_HAND_MAX_BLOBS][6];          /* M_b: xx xy xz yy yz zz */
} rg_hand_aniso;

/* Forward RK4 over n rays (3-D): x0, k0 [3][n], omega [n], s [nb] (device).
 * Writes x_out, k_out [3][n]; if ckpt_every > 0 also the checkpoints
 * [ceil(n_steps/ckpt_every)][7][n] (x, k, t) used by the adjoint.
 * block = 0 picks 256. */
int32_t rg_hand_aniso_trace(const rg_hand_aniso *m, uint32_t n, const double *x0,
                            const double *k0, const double *omega, const double *s, double dt,
                            int32_t n_steps, double *x_out, double *k_out, int32_t ckpt_every,
                            double *ckpt, int32_t block, void *hip_stream);

/* Bytes of device workspace rg_hand_aniso_adjoint needs (per-lane segment
 * states of ckpt_every steps and per-workgroup partial sums). */
int32_t rg_hand_aniso_adjoint_workspace_size(uint32_t n, int32_t ckpt_every, int32_t block,
                                             size_t *bytes);

/* Discrete adjoint of the forward above: seeds dL/dx_end, dL/dk_end
 * (nullable) [3][n]; outputs dL/dx0, dL/dk0 [3][n] (nullable) and dL/ds [nb]
 * (nullable, overwritten).  Needs the checkpoints of the forward call and a
 * caller-owned device workspace of at least the size query's bytes. */
int32_t rg_hand_aniso_adjoint(const rg_hand_aniso *m, uint32_t n, const double *omega,
                              const double *s, double dt, int32_t n_steps, int32_t ckpt_every,
                              const double *ckpt, const double *dL_dx_end,
                              const double *dL_dk_end, double *dL_dx0, double *dL_dk0,
                              double *dL_ds, int32_t block, void *workspace,
                              size_t workspace_bytes, void *hip_stream);

const char *rg_hand_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
