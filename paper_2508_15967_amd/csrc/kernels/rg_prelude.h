// Helpers called by the emitted device functions.  Compiles both as HIP
// device code (RG_FN defaults to __device__ __forceinline__) and as host
// C++ (define RG_FN before including).
#pragma once

#ifndef RG_FN
#define RG_FN __device__ __forceinline__
#endif

#define RG_MAX_PARAMS 8

// Parameter arrays (device pointers, in declaration order).
struct rg_P {
    const double *p[RG_MAX_PARAMS];
};

// 1/d: the hardware reciprocal estimate refined by two Newton steps
// r <- r + r (1 - d r), within one ulp of 1/d for normal finite d (the
// correctly rounded division takes about twice the instructions).  d = 0,
// +-inf and subnormal d give a non-finite result instead of +-inf / 0.
RG_FN double rg_rcp(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(e, r, r);
    e = fma(-d, r, 1.0);
    return fma(e, r, r);
#else
    return 1.0 / d;
#endif
}

// e^x by Tang's table-driven method (P. T. P. Tang, ACM TOMS 15 (1989)
// 144-157): x = (64 m + j) ln2/64 + r with n = 64 m + j = rint(64 x / ln2),
// r = x - n ln2/64 in two pieces (n L1 exact for |n| < 2^21), |r| <= ln2/128;
// e^x = 2^m 2^(j/64) (1 + r p(r)) with p(r) = (e^r - 1)/r by its degree-4
// Taylor polynomial (truncation below 0.32 ulp on that interval) and
// 2^(j/64) from a 64-entry table (gen_exp_table.py).  Within 1.3 ulp over
// the double range; overflow gives +inf, underflow 0 (subnormals on the
// way), e^(-inf) = 0, e^(+inf) = +inf, NaN stays NaN.  About 19
// instructions on gfx950 against about 24 for the library exp, whose
// 11-term polynomial covers |r| <= ln2/2.
// RG_EXP_TABLE begin (written by gen_exp_table.py)
#define RG_EXP_INV_L (0x1.71547652b82fep+6)  /* 64 / ln 2 */
#define RG_EXP_L1 (0x1.62e42ff000000p-7)  /* ln2/64, high 32 bits */
#define RG_EXP_L2 (-0x1.718432a1b0e26p-41)  /* ln2/64 - L1 */
#define RG_EXP_TABLE_VALUES \
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0, \
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0, \
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0, \
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0, \
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0, \
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0, \
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0, \
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0, \
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0, \
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0, \
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0, \
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0, \
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0, \
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0, \
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0, \
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0
// RG_EXP_TABLE end

RG_FN double rg_exp_tab(double x, const double *tab) {
    // below -1100 the result is 0 (a select keeps NaN); above 1100 n stays
    // bounded while r grows with x, so the result overflows to +inf, and a
    // NaN reaches r and the result
    x = x < -1100.0 ? -1100.0 : x;
    const double n = rint(fmin(x, 1100.0) * RG_EXP_INV_L);
    double r = fma(-n, RG_EXP_L1, x);
    r = fma(-n, RG_EXP_L2, r);
    double p = fma(r, 0x1.1111111111111p-7, 0x1.5555555555555p-5);  // 1/120, 1/24
    p = fma(r, p, 0x1.5555555555555p-3);                              // 1/6
    p = fma(r, p, 0.5);
    p = fma(r, p, 1.0);
    const int i = (int)n;
    const double t = tab[i & 63];
    return ldexp(fma(t, r * p, t), i >> 6);
}
#if defined(__HIPCC__) || defined(__HIPCC_RTC__)
// the table lives in LDS; every kernel that calls rg_exp stages it first
__shared__ double rg_exp_lds[64];
RG_FN double rg_exp(double x) { return rg_exp_tab(x, rg_exp_lds); }
#else
static const double rg_exp_host_tab[64] = {RG_EXP_TABLE_VALUES};
RG_FN double rg_exp(double x) { return rg_exp_tab(x, rg_exp_host_tab); }
#endif

// Single precision reciprocal: the hardware estimate and one Newton step
// (about one ulp of 1/d for normal finite d).
RG_FN float rg_rcpf(float d) {
#if defined(__HIP_DEVICE_COMPILE__)
    float r = __builtin_amdgcn_rcpf(d);
    const float e = fmaf(-d, r, 1.0f);
    return fmaf(e, r, r);
#else
    return 1.0f / d;
#endif
}

// Cell of a uniform cubic B-spline with n coefficients: s = (x - lo)/h + 1,
// m = clamp(floor(s), 1, n - 3), u = s - m (u leaves [0,1] outside the
// domain, extending the edge cell's cubic).  4 flops.
RG_FN void rg_bs_cell(double x, double lo, double invh, int n, int &m, double &u) {
    double s = (x - lo) * invh + 1.0;
    double fm = floor(s);
    fm = fmin(fmax(fm, 1.0), (double)(n - 3));
    m = (int)fm;
    u = s - fm;
}

// Basis weights of the cell for derivative order 0..3 in u.
// order 0: (1-u)^3/6, (3u^3-6u^2+4)/6, (-3u^3+3u^2+3u+1)/6, u^3/6   17 flops
RG_FN void rg_bs_w0(double u, double *w) {
    const double v = 1.0 - u;
    const double u2 = u * u, u3 = u2 * u;
    const double v3 = v * v * v;
    w[0] = v3 * (1.0 / 6.0);
    w[3] = u3 * (1.0 / 6.0);
    w[1] = fma(0.5, u3, fma(-1.0, u2, 2.0 / 3.0));
    w[2] = fma(-0.5, u3, fma(0.5, u2, fma(0.5, u, 1.0 / 6.0)));
}
// order 1: -(1-u)^2/2, (3u^2-4u)/2, (-3u^2+2u+1)/2, u^2/2   11 flops
RG_FN void rg_bs_w1(double u, double *w) {
    const double v = 1.0 - u;
    const double u2 = u * u;
    w[0] = -0.5 * (v * v);
    w[3] = 0.5 * u2;
    w[1] = fma(1.5, u2, -2.0 * u);
    w[2] = fma(-1.5, u2, u + 0.5);
}
// order 2: 1-u, 3u-2, 1-3u, u   5 flops
RG_FN void rg_bs_w2(double u, double *w) {
    w[0] = 1.0 - u;
    w[1] = fma(3.0, u, -2.0);
    w[2] = fma(-3.0, u, 1.0);
    w[3] = u;
}
// order 3: -1, 3, -3, 1
RG_FN void rg_bs_w3(double u, double *w) {
    (void)u;
    w[0] = -1.0; w[1] = 3.0; w[2] = -3.0; w[3] = 1.0;
}

// sum_a wx[a] sum_b c[4a+b] wy[b]   35 flops
RG_FN double rg_bs_dot(const double *c, const double *wx, const double *wy) {
    double r[4];
    for (int a = 0; a < 4; a++)
        r[a] = fma(c[4 * a + 3], wy[3], fma(c[4 * a + 2], wy[2], fma(c[4 * a + 1], wy[1], c[4 * a] * wy[0])));
    return fma(r[3], wx[3], fma(r[2], wx[2], fma(r[1], wx[1], r[0] * wx[0])));
}
