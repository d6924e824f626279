// Helpers called by the emitted device functions.  Compiles both as HIP
// device code (RG_FN defaults to __device__ __forceinline__) and as host
// C++ (define RG_FN before including).
#pragma once

#ifndef RG_FN
#define RG_FN __device__ __forceinline__
#endif

#define RG_MAX_PARAMS 8

// Constant table of functions with many FP64 constants: the emitted code
// writes RG_KV(i, literal), entry i of the table rg_ktab unless the
// function's template flag RG_KL asks for the literal.  On the device the
// table is read through the scalar cache, one wide load fetching up to
// eight constants, from a base pointer made opaque at each call so that the
// loads stay in the loop that uses them instead of being hoisted into scalar
// registers for the whole kernel.  Host builds define RG_KTAB and RG_KBASE
// themselves.
#define RG_KV(i, v) (RG_KL ? (v) : rg_k[i])
#ifndef RG_KTAB
#define RG_KTAB __constant__
typedef const __attribute__((address_space(4))) double rg_kd;
#define RG_KBASE                    \
    rg_kd *rg_k = (rg_kd *)rg_ktab; \
    if (!RG_KL) __asm__ volatile("" : "+s"(rg_k));
#endif

// Parameter arrays (device pointers, in declaration order).
struct rg_P {
    const double *p[RG_MAX_PARAMS];
};

// 1/d: the hardware reciprocal estimate refined by two Newton steps
// r <- r + r (1 - d r), within one ulp of 1/d for normal finite d (the
// correctly rounded division takes about twice the instructions).  The
// Newton steps turn the estimate's exact special values into NaN (at d = 0
// the estimate is inf and d r = 0 inf); the division fix-up instruction
// puts back the IEEE result of 1/d for zero, infinite and NaN d and for
// quotients that overflow or underflow, and passes r through otherwise.
RG_FN double rg_rcp(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(e, r, r);
    e = fma(-d, r, 1.0);
    r = fma(e, r, r);
    return __builtin_amdgcn_div_fixup(r, d, 1.0);
#else
    return 1.0 / d;
#endif
}

// e^x by Tang's table-driven method (P. T. P. Tang, ACM TOMS 15 (1989)
// 144-157): x = (N m + j) ln2/N + r with n = N m + j = N x / ln2 rounded,
// N = 256, r = x - n ln2/N in two pieces (n L1 exact for |n| < 2^21),
// |r| <= ln2/512; e^x = 2^m 2^(j/N) (1 + r p(r)) with p(r) = (e^r - 1)/r by
// its degree-3 Taylor polynomial (truncation below 0.35 ulp on that
// interval) and 2^(j/N) from a 256-entry table (gen_exp_table.py).  Within
// 1.5 ulp over the double range; overflow gives +inf, underflow 0
// (subnormals on the way), e^(-inf) = 0, e^(+inf) = +inf, NaN stays NaN.
// About 17 instructions on gfx950 against about 24 for the library exp,
// whose 11-term polynomial covers |r| <= ln2/2.  (A 64-entry table needs a
// degree-4 polynomial for the same bound: one fma more.)
// RG_EXP_TABLE begin (written by gen_exp_table.py)
#define RG_EXP_BITS 8
#define RG_EXP_N 256
#define RG_EXP_INV_L (0x1.71547652b82fep+8)  /* 256 / ln 2 */
#define RG_EXP_L1 (0x1.62e42ff000000p-9)  /* ln2/256, high 32 bits */
#define RG_EXP_L2 (-0x1.718432a1b0e26p-43)  /* ln2/256 - L1 */
#define RG_EXP_TABLE_VALUES \
    0x1.0000000000000p+0, 0x1.00b1afa5abcbfp+0, 0x1.0163da9fb3335p+0, 0x1.02168143b0281p+0, \
    0x1.02c9a3e778061p+0, 0x1.037d42e11bbccp+0, 0x1.04315e86e7f85p+0, 0x1.04e5f72f654b1p+0, \
    0x1.059b0d3158574p+0, 0x1.0650a0e3c1f89p+0, 0x1.0706b29ddf6dep+0, 0x1.07bd42b72a836p+0, \
    0x1.0874518759bc8p+0, 0x1.092bdf66607e0p+0, 0x1.09e3ecac6f383p+0, 0x1.0a9c79b1f3919p+0, \
    0x1.0b5586cf9890fp+0, 0x1.0c0f145e46c85p+0, 0x1.0cc922b7247f7p+0, 0x1.0d83b23395decp+0, \
    0x1.0e3ec32d3d1a2p+0, 0x1.0efa55fdfa9c5p+0, 0x1.0fb66affed31bp+0, 0x1.1073028d7233ep+0, \
    0x1.11301d0125b51p+0, 0x1.11edbab5e2ab6p+0, 0x1.12abdc06c31ccp+0, 0x1.136a814f204abp+0, \
    0x1.1429aaea92de0p+0, 0x1.14e95934f312ep+0, 0x1.15a98c8a58e51p+0, 0x1.166a45471c3c2p+0, \
    0x1.172b83c7d517bp+0, 0x1.17ed48695bbc0p+0, 0x1.18af9388c8deap+0, 0x1.1972658375d2fp+0, \
    0x1.1a35beb6fcb75p+0, 0x1.1af99f8138a1cp+0, 0x1.1bbe084045cd4p+0, 0x1.1c82f95281c6bp+0, \
    0x1.1d4873168b9aap+0, 0x1.1e0e75eb44027p+0, 0x1.1ed5022fcd91dp+0, 0x1.1f9c18438ce4dp+0, \
    0x1.2063b88628cd6p+0, 0x1.212be3578a819p+0, 0x1.21f49917ddc96p+0, 0x1.22bdda27912d1p+0, \
    0x1.2387a6e756238p+0, 0x1.2451ffb82140ap+0, 0x1.251ce4fb2a63fp+0, 0x1.25e85711ece75p+0, \
    0x1.26b4565e27cddp+0, 0x1.2780e341ddf29p+0, 0x1.284dfe1f56381p+0, 0x1.291ba7591bb70p+0, \
    0x1.29e9df51fdee1p+0, 0x1.2ab8a66d10f13p+0, 0x1.2b87fd0dad990p+0, 0x1.2c57e39771b2fp+0, \
    0x1.2d285a6e4030bp+0, 0x1.2df961f641589p+0, 0x1.2ecafa93e2f56p+0, 0x1.2f9d24abd886bp+0, \
    0x1.306fe0a31b715p+0, 0x1.31432edeeb2fdp+0, 0x1.32170fc4cd831p+0, 0x1.32eb83ba8ea32p+0, \
    0x1.33c08b26416ffp+0, 0x1.3496266e3fa2dp+0, 0x1.356c55f929ff1p+0, 0x1.36431a2de883bp+0, \
    0x1.371a7373aa9cbp+0, 0x1.37f26231e754ap+0, 0x1.38cae6d05d866p+0, 0x1.39a401b7140efp+0, \
    0x1.3a7db34e59ff7p+0, 0x1.3b57fbfec6cf4p+0, 0x1.3c32dc313a8e5p+0, 0x1.3d0e544ede173p+0, \
    0x1.3dea64c123422p+0, 0x1.3ec70df1c5175p+0, 0x1.3fa4504ac801cp+0, 0x1.40822c367a024p+0, \
    0x1.4160a21f72e2ap+0, 0x1.423fb2709468ap+0, 0x1.431f5d950a897p+0, 0x1.43ffa3f84b9d4p+0, \
    0x1.44e086061892dp+0, 0x1.45c2042a7d232p+0, 0x1.46a41ed1d0057p+0, 0x1.4786d668b3237p+0, \
    0x1.486a2b5c13cd0p+0, 0x1.494e1e192aed2p+0, 0x1.4a32af0d7d3dep+0, 0x1.4b17dea6db7d7p+0, \
    0x1.4bfdad5362a27p+0, 0x1.4ce41b817c114p+0, 0x1.4dcb299fddd0dp+0, 0x1.4eb2d81d8abffp+0, \
    0x1.4f9b2769d2ca7p+0, 0x1.508417f4531eep+0, 0x1.516daa2cf6642p+0, 0x1.5257de83f4eefp+0, \
    0x1.5342b569d4f82p+0, 0x1.542e2f4f6ad27p+0, 0x1.551a4ca5d920fp+0, 0x1.56070dde910d2p+0, \
    0x1.56f4736b527dap+0, 0x1.57e27dbe2c4cfp+0, 0x1.58d12d497c7fdp+0, 0x1.59c0827ff07ccp+0, \
    0x1.5ab07dd485429p+0, 0x1.5ba11fba87a03p+0, 0x1.5c9268a5946b7p+0, 0x1.5d84590998b93p+0, \
    0x1.5e76f15ad2148p+0, 0x1.5f6a320dceb71p+0, 0x1.605e1b976dc09p+0, 0x1.6152ae6cdf6f4p+0, \
    0x1.6247eb03a5585p+0, 0x1.633dd1d1929fdp+0, 0x1.6434634ccc320p+0, 0x1.652b9febc8fb7p+0, \
    0x1.6623882552225p+0, 0x1.671c1c70833f6p+0, 0x1.68155d44ca973p+0, 0x1.690f4b19e9538p+0, \
    0x1.6a09e667f3bcdp+0, 0x1.6b052fa75173ep+0, 0x1.6c012750bdabfp+0, 0x1.6cfdcddd47645p+0, \
    0x1.6dfb23c651a2fp+0, 0x1.6ef9298593ae5p+0, 0x1.6ff7df9519484p+0, 0x1.70f7466f42e87p+0, \
    0x1.71f75e8ec5f74p+0, 0x1.72f8286ead08ap+0, 0x1.73f9a48a58174p+0, 0x1.74fbd35d7cbfdp+0, \
    0x1.75feb564267c9p+0, 0x1.77024b1ab6e09p+0, 0x1.780694fde5d3fp+0, 0x1.790b938ac1cf6p+0, \
    0x1.7a11473eb0187p+0, 0x1.7b17b0976cfdbp+0, 0x1.7c1ed0130c132p+0, 0x1.7d26a62ff86f0p+0, \
    0x1.7e2f336cf4e62p+0, 0x1.7f3878491c491p+0, 0x1.80427543e1a12p+0, 0x1.814d2add106d9p+0, \
    0x1.82589994cce13p+0, 0x1.8364c1eb941f7p+0, 0x1.8471a4623c7adp+0, 0x1.857f4179f5b21p+0, \
    0x1.868d99b4492edp+0, 0x1.879cad931a436p+0, 0x1.88ac7d98a6699p+0, 0x1.89bd0a478580fp+0, \
    0x1.8ace5422aa0dbp+0, 0x1.8be05bad61778p+0, 0x1.8cf3216b5448cp+0, 0x1.8e06a5e0866d9p+0, \
    0x1.8f1ae99157736p+0, 0x1.902fed0282c8ap+0, 0x1.9145b0b91ffc6p+0, 0x1.925c353aa2fe2p+0, \
    0x1.93737b0cdc5e5p+0, 0x1.948b82b5f98e5p+0, 0x1.95a44cbc8520fp+0, 0x1.96bdd9a7670b3p+0, \
    0x1.97d829fde4e50p+0, 0x1.98f33e47a22a2p+0, 0x1.9a0f170ca07bap+0, 0x1.9b2bb4d53fe0dp+0, \
    0x1.9c49182a3f090p+0, 0x1.9d674194bb8d5p+0, 0x1.9e86319e32323p+0, 0x1.9fa5e8d07f29ep+0, \
    0x1.a0c667b5de565p+0, 0x1.a1e7aed8eb8bbp+0, 0x1.a309bec4a2d33p+0, 0x1.a42c980460ad8p+0, \
    0x1.a5503b23e255dp+0, 0x1.a674a8af46052p+0, 0x1.a799e1330b358p+0, 0x1.a8bfe53c12e59p+0, \
    0x1.a9e6b5579fdbfp+0, 0x1.ab0e521356ebap+0, 0x1.ac36bbfd3f37ap+0, 0x1.ad5ff3a3c2774p+0, \
    0x1.ae89f995ad3adp+0, 0x1.afb4ce622f2ffp+0, 0x1.b0e07298db666p+0, 0x1.b20ce6c9a8952p+0, \
    0x1.b33a2b84f15fbp+0, 0x1.b468415b749b1p+0, 0x1.b59728de5593ap+0, 0x1.b6c6e29f1c52ap+0, \
    0x1.b7f76f2fb5e47p+0, 0x1.b928cf22749e4p+0, 0x1.ba5b030a1064ap+0, 0x1.bb8e0b79a6f1fp+0, \
    0x1.bcc1e904bc1d2p+0, 0x1.bdf69c3f3a207p+0, 0x1.bf2c25bd71e09p+0, 0x1.c06286141b33dp+0, \
    0x1.c199bdd85529cp+0, 0x1.c2d1cd9fa652cp+0, 0x1.c40ab5fffd07ap+0, 0x1.c544778fafb22p+0, \
    0x1.c67f12e57d14bp+0, 0x1.c7ba88988c933p+0, 0x1.c8f6d9406e7b5p+0, 0x1.ca3405751c4dbp+0, \
    0x1.cb720dcef9069p+0, 0x1.ccb0f2e6d1675p+0, 0x1.cdf0b555dc3fap+0, 0x1.cf3155b5bab74p+0, \
    0x1.d072d4a07897cp+0, 0x1.d1b532b08c968p+0, 0x1.d2f87080d89f2p+0, 0x1.d43c8eacaa1d6p+0, \
    0x1.d5818dcfba487p+0, 0x1.d6c76e862e6d3p+0, 0x1.d80e316c98398p+0, 0x1.d955d71ff6075p+0, \
    0x1.da9e603db3285p+0, 0x1.dbe7cd63a8315p+0, 0x1.dd321f301b460p+0, 0x1.de7d5641c0658p+0, \
    0x1.dfc97337b9b5fp+0, 0x1.e11676b197d17p+0, 0x1.e264614f5a129p+0, 0x1.e3b333b16ee12p+0, \
    0x1.e502ee78b3ff6p+0, 0x1.e653924676d76p+0, 0x1.e7a51fbc74c83p+0, 0x1.e8f7977cdb740p+0, \
    0x1.ea4afa2a490dap+0, 0x1.eb9f4867cca6ep+0, 0x1.ecf482d8e67f1p+0, 0x1.ee4aaa2188510p+0, \
    0x1.efa1bee615a27p+0, 0x1.f0f9c1cb6412ap+0, 0x1.f252b376bba97p+0, 0x1.f3ac948dd7274p+0, \
    0x1.f50765b6e4540p+0, 0x1.f6632798844f8p+0, 0x1.f7bfdad9cbe14p+0, 0x1.f91d802243c89p+0, \
    0x1.fa7c1819e90d8p+0, 0x1.fbdba3692d514p+0, 0x1.fd3c22b8f71f1p+0, 0x1.fe9d96b2a23d9p+0
// RG_EXP_TABLE end

// kMode 0 (rg_exp): any argument; a NaN argument gives NaN.
// kMode 1 (rg_exp_nn): the argument is not NaN while the stage state, omega,
// t and the parameters are finite (the emitter proves it from the graph).
// The lower clamp is then a plain maximum, which maps a NaN argument to
// -1100 and so to e^x = 0 (one instruction against a compare and two
// selects).  Such a NaN comes from a non-finite stage state, and a
// non-finite stage state makes the step or attempt through it non-finite
// or its error estimate NaN, so it is rejected with the same outcome
// whatever the exponential returned.
// kMode 2 (rg_exp_np): as 1 and the argument is also proven <= 0, so the
// upper clamp, whose only role is to keep n in range for x > 1100, is left
// out as well.
template <int kMode>
RG_FN double rg_exp_tab(double x, const double *tab) {
    // below -1100 the result is 0 (the general form's select keeps NaN);
    // above 1100 n stays bounded while r grows with x, so the result
    // overflows to +inf, and a NaN reaches r and the result
    x = kMode > 0 ? fmax(x, -1100.0) : (x < -1100.0 ? -1100.0 : x);
    // n = x N/ln2 rounded to nearest (even) by adding 1.5 2^52, whose ulp is
    // 1: the sum holds n in its low 32 bits (two's complement), and
    // subtracting the constant again gives n as a double
    const double s = fma(kMode == 2 ? x : fmin(x, 1100.0), RG_EXP_INV_L, 0x1.8p52);
    const double n = s - 0x1.8p52;
    double r = fma(-n, RG_EXP_L1, x);
    r = fma(-n, RG_EXP_L2, r);
    double p = fma(r, 0x1.5555555555555p-5, 0x1.5555555555555p-3);  // 1/24, 1/6
    p = fma(r, p, 0.5);
    p = fma(r, p, 1.0);
    unsigned long long bits;
    __builtin_memcpy(&bits, &s, sizeof bits);
    const int i = (int)(unsigned)bits;
    const double t = tab[i & (RG_EXP_N - 1)];
    return ldexp(fma(t, r * p, t), i >> RG_EXP_BITS);
}
#if defined(__HIPCC__) || defined(__HIPCC_RTC__)
// the table lives in LDS; every kernel that calls rg_exp stages it first
__shared__ double rg_exp_lds[RG_EXP_N];
RG_FN double rg_exp(double x) { return rg_exp_tab<0>(x, rg_exp_lds); }
RG_FN double rg_exp_nn(double x) { return rg_exp_tab<1>(x, rg_exp_lds); }
RG_FN double rg_exp_np(double x) { return rg_exp_tab<2>(x, rg_exp_lds); }
#else
static const double rg_exp_host_tab[RG_EXP_N] = {RG_EXP_TABLE_VALUES};
RG_FN double rg_exp(double x) { return rg_exp_tab<0>(x, rg_exp_host_tab); }
RG_FN double rg_exp_nn(double x) { return rg_exp_tab<1>(x, rg_exp_host_tab); }
RG_FN double rg_exp_np(double x) { return rg_exp_tab<2>(x, rg_exp_host_tab); }
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

// Tensor-product evaluation sum_a wx[a] sum_b c[4a+b] wy[b] in two parts:
// the row sums r[a] = sum_b c[4a+b] wy[b] (28 flops), shared by every
// derivative with the same order in v, and their combination with the
// weights in u (7 flops).
RG_FN void rg_bs_rows(const double *c, const double *wy, double *r) {
    for (int a = 0; a < 4; a++)
        r[a] = fma(c[4 * a + 3], wy[3], fma(c[4 * a + 2], wy[2], fma(c[4 * a + 1], wy[1], c[4 * a] * wy[0])));
}
RG_FN double rg_bs_comb(const double *r, const double *wx) {
    return fma(r[3], wx[3], fma(r[2], wx[2], fma(r[1], wx[1], r[0] * wx[0])));
}
