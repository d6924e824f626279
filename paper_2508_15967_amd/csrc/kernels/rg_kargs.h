// Argument block of every integrator kernel, passed by value.  Included by
// the host runtime and by the generated device source, so the layout is the
// same on both sides (LP64, natural alignment).
#pragma once

#define RG_KMAX_PARAMS 8

struct rg_kargs {
    // inputs
    const double *x0, *k0, *t0, *omega;
    const double *params[RG_KMAX_PARAMS];
    const int *budget;
    // outputs
    double *x_out, *k_out, *t_out;
    int *status_out, *steps_out, *attempts_out;
    double *traj, *traj_D, *ckpt;
    // adjoint
    const double *lam_x, *lam_k;
    double *gx0, *gk0;
    double *scratch;          // [ckpt_every][NY+1][scratch_lanes]
    double *gpart;            // [n_part][part_stride]
    double *dparams[RG_KMAX_PARAMS];
    // plain-mode state (SoA over rays) and counters
    double *s_y, *s_k1, *s_t, *s_h, *s_fm;
    double *s_lam;            // plain adjoint: [NY][n]
    int seg_s0;               // plain adjoint: first step of the segment
    int *s_st, *s_acc, *s_att;
    unsigned long long *queue;
    int *counter;
    // scalars
    double dt, h0, rtol, atol, hmin, t_end;
    double box_lo[3], box_hi[3];
    long long n;              // ray count = SoA stride
    long long n_run;          // rays processed (the first n_run; n_run <= n)
    int budget_cap;           // > 0: cap every ray's budget (autotuning samples)
    int n_steps, store_every, ckpt_every, has_box, max_steps, compact;
    int step, snap, ckpt_idx, count_alive;
    long long scratch_lanes;
    int n_part, part_stride;
    // Newton solve
    double *k_io, *D_out, *max_abs_D;
    int *iters_out;
    int component, max_iter;
    double tol;
    long long fill_n;
    double fill_v;
    double *fill_p;
    // per-trace statistics (rg_stats)
    unsigned long long *stats;
};
