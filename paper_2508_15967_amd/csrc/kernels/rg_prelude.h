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
