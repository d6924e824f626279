/*
 * Plain FP64 CPU oracle for geometric-optics ray tracing.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or constant with the GPU
 * path; the two meet only through the seeded input arrays.
 *
 * What it computes (paper: "Impact" section, eqs. 1-3 and the RK4 kernel
 * description that follows them):
 *   - the dispersion relation D(x, k, omega) of each medium, written out by
 *     hand, and the ray equations obtained from it by implicit differentiation,
 *       dx/dt = -(dD/dk)/(dD/domega),   dk/dt = (dD/dx)/(dD/domega),
 *     with every partial derivative derived by hand (no graph, no autodiff);
 *   - classic fourth-order Runge-Kutta time stepping (one step updates x, k, t);
 *   - Dormand-Prince 5(4) adaptive stepping with the step controller used by
 *     the GPU path (published tableau: Dormand & Prince, J. Comput. Appl. Math.
 *     6 (1980) 19-26; also Hairer, Norsett & Wanner, Solving ODEs I, II.5);
 *   - per-ray termination (box exit, step budget, non-finite state, step
 *     underflow);
 *   - the exact discrete adjoint of the RK4 map (Hager, Numer. Math. 87 (2000))
 *     and, independently, the tangent-linear (forward-mode) derivative, both
 *     from the hand-derived Jacobian.
 * Built with -O2 -fno-fast-math -ffp-contract=off: no contraction, no
 * reassociation.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { HOMOG = 0, OLINEAR = 1, LINEARN = 2, LENS2D = 3, STRAT3D = 4, BUMPS3D = 5,
       SPLINE2D = 6, ANISO3D = 7, COLDPLASMA = 8 };
enum { RAY_OK = 0, RAY_EXITED_BOX = 1, RAY_BUDGET = 2, RAY_NONFINITE = 3,
       RAY_STEP_UNDERFLOW = 4 };

typedef struct {
    int32_t kind, dim, nb, nx, ny, pad;
    double p[8];
    const double *centers; /* nb x 3 */
    const double *widths;  /* nb */
    const double *amps;    /* nb */
    const double *mats;    /* nb x 6: xx xy xz yy yz zz */
    const double *scales;  /* nb */
    const double *coef;    /* nx x ny, x index major */
    double lo[2], hi[2];
} om_medium;

typedef struct {
    int32_t integrator; /* 0 = RK4, 1 = Dormand-Prince 5(4) */
    int32_t n_steps;    /* RK4 step count */
    double dt;          /* RK4 step */
    double h0, rtol, atol, hmin; /* adaptive */
    const int32_t *budget;       /* adaptive: accepted-step cap per ray (nullable) */
    int32_t max_steps;           /* adaptive: cap when budget is NULL */
    int32_t has_box;
    double box_lo[3], box_hi[3];
    double t_end;                /* adaptive: stop at t_end if > 0 */
    int32_t store_every;         /* RK4 snapshots every this many steps (0 = none) */
    int32_t n_threads;           /* 0 = OpenMP default */
    double *traj;                /* [n_snap][2*dim][n] */
    double *traj_D;              /* [n_snap][n] */
} om_opts;

#define MAXD 3
#define MAXY 6

/* ------------------------------------------------------------------------ */
/* isotropic media: D = |k|^2 - omega^2 N(x)                                  */

/* Uniform cubic B-spline weights and their first and second derivatives in
 * the local coordinate u of a cell (de Boor, A Practical Guide to Splines). */
static void bspline_basis(double u, double w[4], double dw[4], double d2w[4])
{
    double v = 1.0 - u;
    w[0] = v * v * v / 6.0;
    w[1] = (3.0 * u * u * u - 6.0 * u * u + 4.0) / 6.0;
    w[2] = (-3.0 * u * u * u + 3.0 * u * u + 3.0 * u + 1.0) / 6.0;
    w[3] = u * u * u / 6.0;
    dw[0] = -v * v / 2.0;
    dw[1] = (3.0 * u * u - 4.0 * u) / 2.0;
    dw[2] = (-3.0 * u * u + 2.0 * u + 1.0) / 2.0;
    dw[3] = u * u / 2.0;
    d2w[0] = 1.0 - u;
    d2w[1] = 3.0 * u - 2.0;
    d2w[2] = 1.0 - 3.0 * u;
    d2w[3] = u;
}

/* Cell of a uniform spline with n coefficients over [lo, hi]: node spacing
 * h = (hi - lo)/(n - 3), coefficient i sits at lo + (i - 1) h.  The cell
 * index is clamped so that outside the domain the edge cell's cubic is
 * extended. */
static int spline_cell(double x, double lo, double hi, int n, double *u, double *h)
{
    *h = (hi - lo) / (double)(n - 3);
    double s = (x - lo) / *h + 1.0;
    double m = floor(s);
    if (m < 1.0) m = 1.0;
    if (m > (double)(n - 3)) m = (double)(n - 3);
    *u = s - m;
    return (int)m;
}

typedef struct {
    int mx, my;             /* cell */
    double hx, hy;
    double wx[4], dwx[4], d2wx[4];
    double wy[4], dwy[4], d2wy[4];
} spline_pt;

static void spline_locate(const om_medium *m, const double *x, spline_pt *sp)
{
    double ux, uy;
    sp->mx = spline_cell(x[0], m->lo[0], m->hi[0], m->nx, &ux, &sp->hx);
    sp->my = spline_cell(x[1], m->lo[1], m->hi[1], m->ny, &uy, &sp->hy);
    bspline_basis(ux, sp->wx, sp->dwx, sp->d2wx);
    bspline_basis(uy, sp->wy, sp->dwy, sp->d2wy);
}

/* N(x), its gradient g and (if H != NULL) its Hessian H (row-major dim x dim). */
static void iso_N(const om_medium *m, const double *x, double *N, double *g, double *H)
{
    int d = m->dim;
    for (int i = 0; i < d; i++) g[i] = 0.0;
    if (H) for (int i = 0; i < d * d; i++) H[i] = 0.0;
    switch (m->kind) {
    case HOMOG:
        *N = m->p[0];
        break;
    case LINEARN: {
        double s = m->p[0];
        for (int i = 0; i < d; i++) { s += m->p[1 + i] * x[i]; g[i] = m->p[1 + i]; }
        *N = s;
        break;
    }
    case LENS2D: {
        /* n = 1 + A e, e = exp(-|x|^2/W), N = n^2 */
        double A = m->p[0], W = m->p[1];
        double r2 = 0.0;
        for (int i = 0; i < d; i++) r2 += x[i] * x[i];
        double e = exp(-r2 / W);
        double n = 1.0 + A * e;
        double gn[MAXD];
        for (int i = 0; i < d; i++) gn[i] = A * e * (-2.0 * x[i] / W);
        *N = n * n;
        for (int i = 0; i < d; i++) g[i] = 2.0 * n * gn[i];
        if (H) {
            for (int i = 0; i < d; i++)
                for (int j = 0; j < d; j++) {
                    double Hn = A * e * (4.0 * x[i] * x[j] / (W * W) - (i == j ? 2.0 / W : 0.0));
                    H[i * d + j] = 2.0 * gn[i] * gn[j] + 2.0 * n * Hn;
                }
        }
        break;
    }
    case STRAT3D:
    case BUMPS3D: {
        /* N = 1 - a E, E = exp(1 - z' - q), q = exp(-z'), z' = (z - z0)/L */
        double a = m->p[0], z0 = m->p[1], L = m->p[2];
        double zeta = (x[2] - z0) / L;
        double q = exp(-zeta);
        double E = exp(1.0 - zeta - q);
        *N = 1.0 - a * E;
        g[2] = a * E * (1.0 - q) / L;
        if (H) H[8] = a * E * (q - (1.0 - q) * (1.0 - q)) / (L * L);
        if (m->kind == BUMPS3D) {
            for (int b = 0; b < m->nb; b++) {
                const double *c = m->centers + 3 * b;
                double w2 = m->widths[b] * m->widths[b];
                double r2 = 0.0, dx[3];
                for (int i = 0; i < 3; i++) { dx[i] = x[i] - c[i]; r2 += dx[i] * dx[i]; }
                double gb = exp(-r2 / w2);
                double ab = m->amps[b];
                *N += ab * gb;
                for (int i = 0; i < 3; i++) g[i] += ab * gb * (-2.0 * dx[i] / w2);
                if (H)
                    for (int i = 0; i < 3; i++)
                        for (int j = 0; j < 3; j++)
                            H[i * 3 + j] += ab * gb * (4.0 * dx[i] * dx[j] / (w2 * w2)
                                                       - (i == j ? 2.0 / w2 : 0.0));
            }
        }
        break;
    }
    case SPLINE2D: {
        spline_pt sp;
        spline_locate(m, x, &sp);
        double v = 0, vx = 0, vy = 0, vxx = 0, vxy = 0, vyy = 0;
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                double c = m->coef[(sp.mx - 1 + a) * m->ny + (sp.my - 1 + b)];
                v += c * sp.wx[a] * sp.wy[b];
                vx += c * sp.dwx[a] * sp.wy[b];
                vy += c * sp.wx[a] * sp.dwy[b];
                vxx += c * sp.d2wx[a] * sp.wy[b];
                vxy += c * sp.dwx[a] * sp.dwy[b];
                vyy += c * sp.wx[a] * sp.d2wy[b];
            }
        *N = v;
        g[0] = vx / sp.hx;
        g[1] = vy / sp.hy;
        if (H) {
            H[0] = vxx / (sp.hx * sp.hx);
            H[1] = H[2] = vxy / (sp.hx * sp.hy);
            H[3] = vyy / (sp.hy * sp.hy);
        }
        break;
    }
    default:
        *N = NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* anisotropic medium: D = k.A(x).k - omega^2, A = I + sum_b s_b M_b g_b(x)  */

static void sym3(const double *m6, double M[9])
{
    M[0] = m6[0]; M[1] = m6[1]; M[2] = m6[2];
    M[3] = m6[1]; M[4] = m6[3]; M[5] = m6[4];
    M[6] = m6[2]; M[7] = m6[4]; M[8] = m6[5];
}

/* ------------------------------------------------------------------------ */
/* cold plasma ("Cold Plasma Dispersion Relation", eqs. 5-10)                */
/* B along z; electron density w_pe^2(x) = p0 (p1 x + 1) (eq. 4 profile);    */
/* electron cyclotron frequency p2 (signed); ions of mass ratio p3 (0: none). */
/* Units omega, c = 1: n = k / omega (eq. 6).                                 */

static double complex cp_D(const om_medium *m, const double complex *x, const double complex *k,
                           double complex w)
{
    /* dielectric tensor elements, eqs. 8-10 (X = w_p^2/w^2, Y = Omega/w) */
    double complex X = m->p[0] * (m->p[1] * x[0] + 1.0) / (w * w);
    double complex Y = m->p[2] / w;
    double complex S = 1.0 - X / (1.0 - Y * Y);        /* eps_11 */
    double complex G = Y * X / (1.0 - Y * Y);          /* eps_12 = -i G */
    double complex P = 1.0 - X;                        /* eps_33 */
    if (m->p[3] > 0.0) {
        double complex Xi = X / m->p[3], Yi = -Y / m->p[3];
        S = S - Xi / (1.0 - Yi * Yi);
        G = G + Yi * Xi / (1.0 - Yi * Yi);
        P = P - Xi;
    }
    /* D = Det(eps + n n - n^2 I), eq. 5; the off-diagonal entries are
       eps_12 + n_x n_y = n_x n_y - i G and its conjugate, the rest real, so
       the determinant of the Hermitian matrix is the real expression
       M11 M22 M33 - M11 M23^2 - M22 M13^2 - (a^2 + G^2) M33 + 2 a M13 M23. */
    double complex nx = k[0] / w, ny = k[1] / w, nz = k[2] / w;
    double complex n2 = nx * nx + ny * ny + nz * nz;
    double complex M11 = S + nx * nx - n2, M22 = S + ny * ny - n2, M33 = P + nz * nz - n2;
    double complex a = nx * ny, M13 = nx * nz, M23 = ny * nz;
    return M11 * M22 * M33 - M11 * M23 * M23 - M22 * M13 * M13 - (a * a + G * G) * M33
           + 2.0 * a * M13 * M23;
}

/* Partial derivatives of the cold-plasma D by complex-step differentiation
 * (Squire & Trapp 1998): dD/dv = Im D(v + i h) / h, exact to rounding for an
 * analytic function, h = 1e-30.  grad = (D_x[3], D_k[3]), Dw = dD/domega. */
static void cp_grad(const om_medium *m, const double *y, double w, double *D, double *grad,
                    double *Dw)
{
    const double h = 1e-30;
    double complex x[3], k[3];
    for (int i = 0; i < 3; i++) { x[i] = y[i]; k[i] = y[3 + i]; }
    *D = creal(cp_D(m, x, k, w));
    for (int j = 0; j < 6; j++) {
        double complex xx[3] = {x[0], x[1], x[2]}, kk[3] = {k[0], k[1], k[2]};
        if (j < 3) xx[j] += I * h; else kk[j - 3] += I * h;
        grad[j] = cimag(cp_D(m, xx, kk, w)) / h;
    }
    *Dw = cimag(cp_D(m, x, k, w + I * h)) / h;
}

/* ------------------------------------------------------------------------ */
/* D, ray right-hand side f = (dx/dt, dk/dt) and its Jacobian J = df/dy      */
/* (y = (x, k), J row-major 2d x 2d).  eqs. (2)-(3).                          */

static double om_D1(const om_medium *m, const double *y, double w)
{
    int d = m->dim;
    const double *x = y, *k = y + d;
    if (m->kind == COLDPLASMA) {
        double D, g[6], Dw;
        cp_grad(m, y, w, &D, g, &Dw);
        return D;
    }
    if (m->kind == ANISO3D) {
        double D = -w * w;
        double kk = 0.0;
        for (int i = 0; i < 3; i++) kk += k[i] * k[i];
        D += kk;
        for (int b = 0; b < m->nb; b++) {
            const double *c = m->centers + 3 * b;
            double w2 = m->widths[b] * m->widths[b], r2 = 0.0;
            for (int i = 0; i < 3; i++) r2 += (x[i] - c[i]) * (x[i] - c[i]);
            double M[9];
            sym3(m->mats + 6 * b, M);
            double q = 0.0;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) q += k[i] * M[i * 3 + j] * k[j];
            D += m->scales[b] * exp(-r2 / w2) * q;
        }
        return D;
    }
    double kk = 0.0;
    for (int i = 0; i < d; i++) kk += k[i] * k[i];
    if (m->kind == OLINEAR) {
        double s = m->p[0];
        for (int i = 0; i < d; i++) s += m->p[1 + i] * x[i];
        return kk - w * w + s;
    }
    double N, g[MAXD];
    iso_N(m, x, &N, g, NULL);
    return kk - w * w * N;
}

static void om_eval(const om_medium *m, const double *y, double w, double *f, double *J)
{
    int d = m->dim, n2 = 2 * d;
    const double *x = y, *k = y + d;
    if (J) for (int i = 0; i < n2 * n2; i++) J[i] = 0.0;
    if (m->kind == COLDPLASMA) {
        /* eqs. 2-3 with the complex-step partials; no Jacobian (forward only) */
        double D, g[6], Dw;
        cp_grad(m, y, w, &D, g, &Dw);
        for (int i = 0; i < 3; i++) {
            f[i] = -g[3 + i] / Dw;
            f[3 + i] = g[i] / Dw;
        }
        if (J) for (int i = 0; i < n2 * n2; i++) J[i] = NAN;
        return;
    }
    if (m->kind == OLINEAR) {
        /* D = |k|^2 - w^2 + (a + g.x): D_k = 2k, D_w = -2w, D_x = g */
        for (int i = 0; i < d; i++) {
            f[i] = k[i] / w;
            f[d + i] = -m->p[1 + i] / (2.0 * w);
            if (J) J[i * n2 + d + i] = 1.0 / w;
        }
        return;
    }
    if (m->kind == ANISO3D) {
        /* D_k = 2 A k, D_w = -2w, D_x = sum_b s_b (k.M_b.k) grad g_b,
         * grad g_b = -2 (x - c_b) g_b / w_b^2.
         * dx/dt = A k / w,  dk/dt = (1/w) sum_b s_b q_b g_b (x - c_b)/w_b^2. */
        double Ak[3] = {k[0], k[1], k[2]};
        double fk[3] = {0, 0, 0};
        double Jxx[9] = {0}, Jxk[9] = {0}, Jkx[9] = {0}, Jkk[9] = {0};
        for (int i = 0; i < 3; i++) Jxk[i * 3 + i] = 1.0;
        for (int b = 0; b < m->nb; b++) {
            const double *c = m->centers + 3 * b;
            double w2 = m->widths[b] * m->widths[b], r2 = 0.0, dx[3];
            for (int i = 0; i < 3; i++) { dx[i] = x[i] - c[i]; r2 += dx[i] * dx[i]; }
            double gb = exp(-r2 / w2);
            double s = m->scales[b];
            double M[9], Mk[3], q = 0.0;
            sym3(m->mats + 6 * b, M);
            for (int i = 0; i < 3; i++) {
                Mk[i] = 0.0;
                for (int j = 0; j < 3; j++) Mk[i] += M[i * 3 + j] * k[j];
                q += k[i] * Mk[i];
            }
            for (int i = 0; i < 3; i++) {
                Ak[i] += s * gb * Mk[i];
                fk[i] += s * q * gb * dx[i] / w2;
            }
            if (J) {
                double gg[3];
                for (int j = 0; j < 3; j++) gg[j] = -2.0 * dx[j] * gb / w2;  /* grad g_b */
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        Jxx[i * 3 + j] += s * Mk[i] * gg[j];
                        Jxk[i * 3 + j] += s * gb * M[i * 3 + j];
                        Jkx[i * 3 + j] += s * q / w2 * (gg[j] * dx[i] + (i == j ? gb : 0.0));
                        Jkk[i * 3 + j] += s * 2.0 * Mk[j] * gb * dx[i] / w2;
                    }
            }
        }
        for (int i = 0; i < 3; i++) { f[i] = Ak[i] / w; f[3 + i] = fk[i] / w; }
        if (J)
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    J[i * 6 + j] = Jxx[i * 3 + j] / w;
                    J[i * 6 + 3 + j] = Jxk[i * 3 + j] / w;
                    J[(3 + i) * 6 + j] = Jkx[i * 3 + j] / w;
                    J[(3 + i) * 6 + 3 + j] = Jkk[i * 3 + j] / w;
                }
        return;
    }
    /* isotropic: D_k = 2k, D_w = -2 w N, D_x = -w^2 grad N
     * dx/dt = k/(w N),  dk/dt = w grad N / (2 N) */
    double N, g[MAXD], H[MAXD * MAXD];
    iso_N(m, x, &N, g, J ? H : NULL);
    for (int i = 0; i < d; i++) {
        f[i] = k[i] / (w * N);
        f[d + i] = w * g[i] / (2.0 * N);
    }
    if (J) {
        for (int i = 0; i < d; i++) {
            J[i * n2 + d + i] = 1.0 / (w * N);
            for (int j = 0; j < d; j++) {
                J[i * n2 + j] = -k[i] * g[j] / (w * N * N);
                J[(d + i) * n2 + j] = w * (H[i * d + j] / (2.0 * N) - g[i] * g[j] / (2.0 * N * N));
            }
        }
    }
}

/* Number of differentiable medium parameters: spline coefficients or blob
 * scales s_b.  Other media have none. */
static int64_t n_params(const om_medium *m)
{
    if (m->kind == SPLINE2D) return (int64_t)m->nx * m->ny;
    if (m->kind == ANISO3D) return m->nb;
    return 0;
}

#define MAXCOLS 64

/* Non-zero columns of df/dtheta at one point: idx[c] is the parameter index,
 * col[c][0..2d-1] the column.  Spline: the 16 coefficients of the cell;
 * anisotropic medium: the blob scales s_b.  Returns the column count. */
static int param_cols(const om_medium *m, const double *y, double w, int64_t *idx,
                      double col[][MAXY])
{
    int d = m->dim;
    const double *x = y, *k = y + d;
    int nc = 0;
    if (m->kind == SPLINE2D) {
        /* df_x/dc = -k phi/(w N^2);  df_k/dc = w (grad phi/(2N) - phi grad N/(2 N^2)) */
        double N, g[2];
        iso_N(m, x, &N, g, NULL);
        spline_pt sp;
        spline_locate(m, x, &sp);
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                double phi = sp.wx[a] * sp.wy[b];
                double gphi[2] = {sp.dwx[a] * sp.wy[b] / sp.hx, sp.wx[a] * sp.dwy[b] / sp.hy};
                idx[nc] = (int64_t)(sp.mx - 1 + a) * m->ny + (sp.my - 1 + b);
                for (int i = 0; i < 2; i++) {
                    col[nc][i] = -k[i] * phi / (w * N * N);
                    col[nc][2 + i] = w * (gphi[i] / (2.0 * N) - phi * g[i] / (2.0 * N * N));
                }
                nc++;
            }
    } else if (m->kind == ANISO3D) {
        /* df_x/ds_b = M_b k g_b / w;  df_k/ds_b = q_b g_b (x - c_b)/(w_b^2 w) */
        for (int b = 0; b < m->nb && b < MAXCOLS; b++) {
            const double *c = m->centers + 3 * b;
            double w2 = m->widths[b] * m->widths[b], r2 = 0.0, dx[3];
            for (int i = 0; i < 3; i++) { dx[i] = x[i] - c[i]; r2 += dx[i] * dx[i]; }
            double gb = exp(-r2 / w2);
            double M[9], Mk[3], q = 0.0;
            sym3(m->mats + 6 * b, M);
            for (int i = 0; i < 3; i++) {
                Mk[i] = 0.0;
                for (int j = 0; j < 3; j++) Mk[i] += M[i * 3 + j] * k[j];
                q += k[i] * Mk[i];
            }
            idx[nc] = b;
            for (int i = 0; i < 3; i++) {
                col[nc][i] = Mk[i] * gb / w;
                col[nc][3 + i] = q * gb * dx[i] / (w2 * w);
            }
            nc++;
        }
    }
    return nc;
}

/* gp[p] += v . df/dtheta_p for every parameter p (parameter VJP). */
static void om_param_vjp(const om_medium *m, const double *y, double w, const double *v, double *gp)
{
    int64_t idx[MAXCOLS];
    double col[MAXCOLS][MAXY];
    int nc = param_cols(m, y, w, idx, col), n2 = 2 * m->dim;
    for (int c = 0; c < nc; c++) {
        double s = 0.0;
        for (int i = 0; i < n2; i++) s += v[i] * col[c][i];
        gp[idx[c]] += s;
    }
}

/* df/dtheta_p for one parameter p (tangent-linear forcing); zero if p < 0. */
static void om_param_jvp(const om_medium *m, const double *y, double w, int64_t p, double *fp)
{
    int n2 = 2 * m->dim;
    for (int i = 0; i < n2; i++) fp[i] = 0.0;
    if (p < 0) return;
    int64_t idx[MAXCOLS];
    double col[MAXCOLS][MAXY];
    int nc = param_cols(m, y, w, idx, col);
    for (int c = 0; c < nc; c++)
        if (idx[c] == p)
            for (int i = 0; i < n2; i++) fp[i] += col[c][i];
}

/* ------------------------------------------------------------------------ */
/* integrators                                                              */

static int all_finite(const double *y, int n)
{
    for (int i = 0; i < n; i++)
        if (!isfinite(y[i])) return 0;
    return 1;
}

static int outside_box(const om_opts *o, const double *x, int d)
{
    if (!o->has_box) return 0;
    for (int i = 0; i < d; i++)
        if (x[i] < o->box_lo[i] || x[i] > o->box_hi[i]) return 1;
    return 0;
}

/* One classic RK4 step (the 1/6, 1/3, 1/3, 1/6 scheme). */
static void rk4_step(const om_medium *m, const double *y, double w, double dt, double *out)
{
    int n2 = 2 * m->dim;
    double K1[MAXY], K2[MAXY], K3[MAXY], K4[MAXY], Y[MAXY];
    om_eval(m, y, w, K1, NULL);
    for (int i = 0; i < n2; i++) Y[i] = y[i] + 0.5 * dt * K1[i];
    om_eval(m, Y, w, K2, NULL);
    for (int i = 0; i < n2; i++) Y[i] = y[i] + 0.5 * dt * K2[i];
    om_eval(m, Y, w, K3, NULL);
    for (int i = 0; i < n2; i++) Y[i] = y[i] + dt * K3[i];
    om_eval(m, Y, w, K4, NULL);
    for (int i = 0; i < n2; i++)
        out[i] = y[i] + dt / 6.0 * (K1[i] + 2.0 * K2[i] + 2.0 * K3[i] + K4[i]);
}

static void store_snapshot(const om_medium *m, const om_opts *o, int64_t n, int64_t r,
                           int64_t snap, const double *y, double w)
{
    int n2 = 2 * m->dim;
    if (o->traj)
        for (int c = 0; c < n2; c++) o->traj[(snap * n2 + c) * n + r] = y[c];
    if (o->traj_D) o->traj_D[snap * n + r] = om_D1(m, y, w);
}

static void trace_rk4_ray(const om_medium *m, const om_opts *o, int64_t n, int64_t r,
                          const double *x0, const double *k0, const double *omega,
                          double *x_out, double *k_out, double *t_out,
                          int32_t *status, int32_t *steps)
{
    int d = m->dim, n2 = 2 * d;
    double y[MAXY], yn[MAXY];
    for (int i = 0; i < d; i++) { y[i] = x0[i * n + r]; y[d + i] = k0[i * n + r]; }
    double w = omega[r], t = 0.0;
    int st = RAY_OK, ns = 0;
    int se = o->store_every;
    if (se > 0) store_snapshot(m, o, n, r, 0, y, w);
    for (int s = 0; s < o->n_steps; s++) {
        if (st == RAY_OK) {
            rk4_step(m, y, w, o->dt, yn);
            if (!all_finite(yn, n2)) {
                st = RAY_NONFINITE;
            } else {
                memcpy(y, yn, sizeof(double) * n2);
                t = t + o->dt;
                ns++;
                if (outside_box(o, y, d)) st = RAY_EXITED_BOX;
            }
        }
        if (se > 0 && (s + 1) % se == 0) store_snapshot(m, o, n, r, (s + 1) / se, y, w);
    }
    for (int i = 0; i < d; i++) { x_out[i * n + r] = y[i]; k_out[i * n + r] = y[d + i]; }
    t_out[r] = t;
    status[r] = st;
    steps[r] = ns;
}

/* Dormand-Prince 5(4) tableau. */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0},
    {1.0 / 5.0},
    {3.0 / 40.0, 9.0 / 40.0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
static const double DP_B5[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                                -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double DP_B4[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

/* Step-size factor after an attempt with scaled error err:
 * 0.9 err^(-1/5), rounded down to a multiple of 1/32, clipped to
 * [0.2, facmax].  That is k/32 with k the largest integer such that
 * k <= 28.8 err^(-1/5), i.e. such that err (5k)^5 <= 144^5 (28.8 = 144/5).
 * The inequality is decided here as written: (5k)^5 and 144^5 are integers
 * below 2^53, exact in double, so the only rounding is the product
 * err * (5k)^5, and no transcendental function takes part; the next step
 * size is an exactly reproducible function of err.  k is found by counting
 * up (k <= 161 is enough: 161/32 exceeds the largest factor, 5). */
static double dp_factor(double err, double facmax)
{
    const double lim = 61917364224.0; /* 144^5 */
    int k = 0;
    while (k < 161) {
        const double c = 5.0 * (k + 1);
        if (!(err * (c * c * c * c * c) <= lim)) break; /* also stops at NaN */
        k++;
    }
    double fac = k / 32.0;
    if (!(fac >= 0.2)) fac = 0.2;
    if (fac > facmax) fac = facmax;
    return fac;
}

/* One Dormand-Prince attempt of size hs from (y, K1 = f(y)): the stage
 * derivatives K[0..6] (K[6] = f(y5), first-same-as-last), the 5th-order
 * solution y5 (propagated), the difference e = y5 - y4 to the embedded
 * 4th-order solution, and the scaled RMS error
 *   err = sqrt(mean_i (e_i / sc_i)^2),  sc_i = atol + rtol max(|y_i|, |y5_i|)
 * over the 2d components of (x, k). */
static double dopri_attempt(const om_medium *m, const double *y, double w, double hs,
                            double rtol, double atol, double K[7][MAXY], double *y5, double *e)
{
    int n2 = 2 * m->dim;
    double Y[MAXY];
    for (int s = 1; s < 7; s++) {
        for (int i = 0; i < n2; i++) {
            double acc_i = 0.0;
            for (int j = 0; j < s; j++) acc_i += DP_A[s][j] * K[j][i];
            Y[i] = y[i] + hs * acc_i;
        }
        om_eval(m, Y, w, K[s], NULL);
    }
    /* the last stage is evaluated at the 5th-order solution (FSAL) */
    for (int i = 0; i < n2; i++) y5[i] = Y[i];
    double sum = 0.0;
    for (int i = 0; i < n2; i++) {
        double ei = 0.0;
        for (int j = 0; j < 7; j++) ei += (DP_B5[j] - DP_B4[j]) * K[j][i];
        ei = hs * ei;
        e[i] = ei;
        double ay = fabs(y[i]), ay5 = fabs(y5[i]);
        double sc = atol + rtol * (ay > ay5 ? ay : ay5);
        sum += (ei / sc) * (ei / sc);
    }
    return sqrt(sum / (double)n2);
}

static void trace_dopri_ray(const om_medium *m, const om_opts *o, int64_t n, int64_t r,
                            const double *x0, const double *k0, const double *omega,
                            double *x_out, double *k_out, double *t_out,
                            int32_t *status, int32_t *steps, int32_t *attempts_out)
{
    int d = m->dim, n2 = 2 * d;
    double y[MAXY], K[7][MAXY], y5[MAXY], e[MAXY];
    for (int i = 0; i < d; i++) { y[i] = x0[i * n + r]; y[d + i] = k0[i * n + r]; }
    double w = omega[r], t = 0.0, h = o->h0, facmax = 5.0;
    int64_t budget = o->budget ? o->budget[r] : o->max_steps;
    int64_t acc = 0, att = 0;
    int st = RAY_OK;
    om_eval(m, y, w, K[0], NULL);
    for (;;) {
        if (acc >= budget || att >= 4 * budget) { st = RAY_BUDGET; break; }
        if (o->t_end > 0.0 && t >= o->t_end) { st = RAY_OK; break; }
        double hs = h;
        if (o->t_end > 0.0 && t + hs > o->t_end) hs = o->t_end - t;
        double err = dopri_attempt(m, y, w, hs, o->rtol, o->atol, K, y5, e);
        att++;
        if (err <= 1.0 && all_finite(y5, n2) && all_finite(K[6], n2)) {
            memcpy(y, y5, sizeof(double) * n2);
            memcpy(K[0], K[6], sizeof(double) * n2);
            t = t + hs;
            acc++;
            h = hs * dp_factor(err, facmax);
            facmax = 5.0;
            if (outside_box(o, y, d)) { st = RAY_EXITED_BOX; break; }
        } else {
            h = hs * dp_factor(err > 1.0 ? err : INFINITY, 1.0);
            facmax = 1.0;
        }
        if (h < o->hmin) { st = RAY_STEP_UNDERFLOW; break; }
    }
    if (!all_finite(y, n2)) st = RAY_NONFINITE;
    for (int i = 0; i < d; i++) { x_out[i * n + r] = y[i]; k_out[i * n + r] = y[d + i]; }
    t_out[r] = t;
    status[r] = st;
    steps[r] = (int32_t)acc;
    if (attempts_out) attempts_out[r] = (int32_t)att;
}

/* One Dormand-Prince attempt of size h from each point (for tests of the
 * error estimate): y SoA [2d][n]; y5 and e SoA [2d][n]; err [n]. */
int om_dopri_attempt(const om_medium *m, int64_t n, const double *y, const double *omega, double h,
                     double rtol, double atol, double *y5, double *e, double *err)
{
    int n2 = 2 * m->dim;
    for (int64_t r = 0; r < n; r++) {
        double yy[MAXY], K[7][MAXY], y5r[MAXY], er[MAXY];
        for (int i = 0; i < n2; i++) yy[i] = y[i * n + r];
        om_eval(m, yy, omega[r], K[0], NULL);
        err[r] = dopri_attempt(m, yy, omega[r], h, rtol, atol, K, y5r, er);
        for (int i = 0; i < n2; i++) { y5[i * n + r] = y5r[i]; e[i * n + r] = er[i]; }
    }
    return 0;
}

static void set_threads(int nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

double om_dp_factor(double err, double facmax) { return dp_factor(err, facmax); }

int om_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Trace n rays.  Returns 0, or -1 on bad arguments. */
int om_trace(const om_medium *m, const om_opts *o, int64_t n, const double *x0,
             const double *k0, const double *omega, double *x_out, double *k_out,
             double *t_out, int32_t *status, int32_t *steps, int32_t *attempts)
{
    if (!m || !o || m->dim < 1 || m->dim > MAXD) return -1;
    if (o->integrator == 1 && (o->traj || o->traj_D)) return -1;
    set_threads(o->n_threads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n; r++) {
        if (o->integrator == 0)
            trace_rk4_ray(m, o, n, r, x0, k0, omega, x_out, k_out, t_out, status, steps);
        else
            trace_dopri_ray(m, o, n, r, x0, k0, omega, x_out, k_out, t_out, status, steps,
                            attempts);
    }
    return 0;
}

/* Point evaluations: y is SoA [2d][n]; f is SoA [2d][n]; D is [n];
 * J (nullable) is [n][2d][2d]. */
int om_eval_points(const om_medium *m, int64_t n, const double *y, const double *omega,
                   double *f, double *D, double *J)
{
    int n2 = 2 * m->dim;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; r++) {
        double yy[MAXY], ff[MAXY];
        for (int i = 0; i < n2; i++) yy[i] = y[i * n + r];
        om_eval(m, yy, omega[r], ff, J ? J + r * n2 * n2 : NULL);
        for (int i = 0; i < n2; i++) f[i * n + r] = ff[i];
        if (D) D[r] = om_D1(m, yy, omega[r]);
    }
    return 0;
}

/* Parameter VJP at points: g[p] += sum_r v_r . df/dtheta_p (y_r). */
int om_param_vjp_points(const om_medium *m, int64_t n, const double *y, const double *omega,
                        const double *v, double *g)
{
    int n2 = 2 * m->dim;
    for (int64_t r = 0; r < n; r++) {
        double yy[MAXY], vv[MAXY];
        for (int i = 0; i < n2; i++) { yy[i] = y[i * n + r]; vv[i] = v[i * n + r]; }
        om_param_vjp(m, yy, omega[r], vv, g);
    }
    return 0;
}

int64_t om_n_params(const om_medium *m) { return n_params(m); }

/* ------------------------------------------------------------------------ */
/* derivatives of the RK4 trajectory                                        */

/* Tangent-linear: integrate (y, dy) with dy' = J(y) dy + df/dtheta_p on the
 * same RK4 scheme, which differentiates the discrete map exactly.  dy0 is SoA
 * [2d][n]; p < 0 means no parameter direction.  Steps after a ray stops (its
 * status) are skipped exactly as in the forward trace. */
int om_rk4_tangent(const om_medium *m, const om_opts *o, int64_t n, const double *x0,
                   const double *k0, const double *omega, const double *dy0, int64_t p,
                   double *dy_out)
{
    int d = m->dim, n2 = 2 * d;
    set_threads(o->n_threads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n; r++) {
        double y[MAXY], dy[MAXY], Y[MAXY], dY[MAXY], yn[MAXY];
        double K[4][MAXY], dK[4][MAXY], J[MAXY * MAXY], fp[MAXY];
        static const double cs[4] = {0.0, 0.5, 0.5, 1.0};
        for (int i = 0; i < d; i++) { y[i] = x0[i * n + r]; y[d + i] = k0[i * n + r]; }
        for (int i = 0; i < n2; i++) dy[i] = dy0[i * n + r];
        double w = omega[r];
        for (int s = 0; s < o->n_steps; s++) {
            rk4_step(m, y, w, o->dt, yn);
            if (!all_finite(yn, n2)) break;
            for (int st = 0; st < 4; st++) {
                for (int i = 0; i < n2; i++) {
                    Y[i] = st ? y[i] + cs[st] * o->dt * K[st - 1][i] : y[i];
                    dY[i] = st ? dy[i] + cs[st] * o->dt * dK[st - 1][i] : dy[i];
                }
                om_eval(m, Y, w, K[st], J);
                om_param_jvp(m, Y, w, p, fp);
                for (int i = 0; i < n2; i++) {
                    double a = fp[i];
                    for (int j = 0; j < n2; j++) a += J[i * n2 + j] * dY[j];
                    dK[st][i] = a;
                }
            }
            for (int i = 0; i < n2; i++)
                dy[i] = dy[i] + o->dt / 6.0 * (dK[0][i] + 2.0 * dK[1][i] + 2.0 * dK[2][i] + dK[3][i]);
            memcpy(y, yn, sizeof(double) * n2);
            if (outside_box(o, y, d)) break;
        }
        for (int i = 0; i < n2; i++) dy_out[i * n + r] = dy[i];
    }
    return 0;
}

/* Discrete adjoint of the RK4 trajectory.  lam_end is SoA [2d][n]
 * (dL/dx_end, dL/dk_end); lam0 receives dL/d(x0, k0); gparam (length
 * om_n_params) receives dL/dtheta summed over rays (overwritten). */
int om_rk4_adjoint(const om_medium *m, const om_opts *o, int64_t n, const double *x0,
                   const double *k0, const double *omega, const double *lam_end,
                   double *lam0, double *gparam)
{
    int d = m->dim, n2 = 2 * d;
    int64_t np = n_params(m);
    if (gparam) memset(gparam, 0, sizeof(double) * (size_t)(np > 0 ? np : 0));
    set_threads(o->n_threads);
#pragma omp parallel
    {
        double *gl = np > 0 ? (double *)calloc((size_t)np, sizeof(double)) : NULL;
        double *traj = (double *)malloc(sizeof(double) * (size_t)n2 * (size_t)(o->n_steps + 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n; r++) {
            double w = omega[r];
            double *yv = traj;
            for (int i = 0; i < d; i++) { yv[i] = x0[i * n + r]; yv[d + i] = k0[i * n + r]; }
            int ns = 0;
            for (int s = 0; s < o->n_steps; s++) {
                double *yc = traj + (size_t)s * n2, *yn = yc + n2;
                rk4_step(m, yc, w, o->dt, yn);
                if (!all_finite(yn, n2)) break;
                ns++;
                if (outside_box(o, yn, d)) break;
            }
            double lam[MAXY];
            for (int i = 0; i < n2; i++) lam[i] = lam_end[i * n + r];
            double dt = o->dt;
            for (int s = ns - 1; s >= 0; s--) {
                const double *y = traj + (size_t)s * n2;
                double Ys[4][MAXY], K[4][MAXY], Kb[4][MAXY], Yb[4][MAXY], J[4][MAXY * MAXY];
                static const double cs[4] = {0.0, 0.5, 0.5, 1.0};
                for (int st = 0; st < 4; st++) {
                    for (int i = 0; i < n2; i++)
                        Ys[st][i] = st ? y[i] + cs[st] * dt * K[st - 1][i] : y[i];
                    om_eval(m, Ys[st], w, K[st], J[st]);
                }
                /* transpose of y+ = y + dt/6 (K1 + 2K2 + 2K3 + K4), Y_i = y + c_i dt K_{i-1} */
                for (int i = 0; i < n2; i++) Kb[3][i] = dt / 6.0 * lam[i];
                for (int st = 3; st >= 0; st--) {
                    for (int j = 0; j < n2; j++) {
                        double a = 0.0;
                        for (int i = 0; i < n2; i++) a += J[st][i * n2 + j] * Kb[st][i];
                        Yb[st][j] = a;
                    }
                    if (st == 3)
                        for (int i = 0; i < n2; i++) Kb[2][i] = dt / 3.0 * lam[i] + dt * Yb[3][i];
                    else if (st == 2)
                        for (int i = 0; i < n2; i++) Kb[1][i] = dt / 3.0 * lam[i] + 0.5 * dt * Yb[2][i];
                    else if (st == 1)
                        for (int i = 0; i < n2; i++) Kb[0][i] = dt / 6.0 * lam[i] + 0.5 * dt * Yb[1][i];
                    if (gl) om_param_vjp(m, Ys[st], w, Kb[st], gl);
                }
                for (int i = 0; i < n2; i++) lam[i] = lam[i] + Yb[0][i] + Yb[1][i] + Yb[2][i] + Yb[3][i];
            }
            for (int i = 0; i < n2; i++) lam0[i * n + r] = lam[i];
        }
        if (gl) {
#pragma omp critical
            for (int64_t p = 0; p < np; p++) gparam[p] += gl[p];
            free(gl);
        }
        free(traj);
    }
    return 0;
}

/* Copy of the Dormand-Prince tableau, so that tests can check its order
 * conditions: c[7], a[7][6] row-major, b5[7], b4[7]. */
void om_dopri_tableau(double *c, double *a, double *b5, double *b4)
{
    for (int i = 0; i < 7; i++) {
        c[i] = DP_C[i];
        b5[i] = DP_B5[i];
        b4[i] = DP_B4[i];
        for (int j = 0; j < 6; j++) a[i * 6 + j] = DP_A[i][j];
    }
}

/* dD/dk: by hand for the isotropic media and the O-mode profile (2k) and
 * the anisotropic medium (2 A k); for the cold plasma the complex-step
 * partials of its D (eqs. 5-10). */
static void om_Dk(const om_medium *m, const double *y, double w, double *Dk)
{
    int d = m->dim;
    const double *x = y, *k = y + d;
    if (m->kind == COLDPLASMA) {
        double D, g[6], Dw;
        cp_grad(m, y, w, &D, g, &Dw);
        for (int i = 0; i < 3; i++) Dk[i] = g[3 + i];
        return;
    }
    if (m->kind != ANISO3D) {
        for (int i = 0; i < d; i++) Dk[i] = 2.0 * k[i];
        return;
    }
    double Ak[3] = {k[0], k[1], k[2]};
    for (int b = 0; b < m->nb; b++) {
        const double *c = m->centers + 3 * b;
        double w2 = m->widths[b] * m->widths[b], r2 = 0.0;
        for (int i = 0; i < 3; i++) r2 += (x[i] - c[i]) * (x[i] - c[i]);
        double gb = exp(-r2 / w2), M[9];
        sym3(m->mats + 6 * b, M);
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) Ak[i] += m->scales[b] * gb * M[i * 3 + j] * k[j];
    }
    for (int i = 0; i < 3; i++) Dk[i] = 2.0 * Ak[i];
}

/* Launch conditions ("Impact" section): Newton's method on k_c with x, omega
 * and the other components fixed, k_c <- k_c - D / (dD/dk_c), until
 * |D| <= tol or max_iter iterations.  k is SoA [dim][n], updated in place;
 * iters_out gets the iteration count (-1 if not converged). */
int om_newton_k(const om_medium *m, int64_t n, const double *x, double *k, const double *omega,
                int c, double tol, int max_iter, int32_t *iters_out, double *D_out)
{
    int d = m->dim;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; r++) {
        double y[MAXY], Dk[MAXD];
        for (int i = 0; i < d; i++) { y[i] = x[i * n + r]; y[d + i] = k[i * n + r]; }
        int it = 0, done = 0;
        double D = om_D1(m, y, omega[r]);
        for (;;) {
            if (fabs(D) <= tol) { done = 1; break; }
            if (it >= max_iter || !isfinite(D)) break;
            om_Dk(m, y, omega[r], Dk);
            y[d + c] = y[d + c] - D / Dk[c];
            it++;
            D = om_D1(m, y, omega[r]);
        }
        for (int i = 0; i < d; i++) k[i * n + r] = y[d + i];
        if (iters_out) iters_out[r] = done ? it : -1;
        if (D_out) D_out[r] = D;
    }
    return 0;
}
