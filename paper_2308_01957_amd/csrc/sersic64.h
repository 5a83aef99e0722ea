// FP64 Sersic profile (§2.1.1) and its seven parameter derivatives at one point, shared by
// the FP64 render and the adaptive integration.  Same parametrisation as the FP32 kernels:
// I = 2^(A - B t), t = 2^(g log2 R^2 - h) = (R / Re)^(1/n), with the elliptical radius
// floored at R^2 = 1e-12 (the cusp of n > 1 profiles; no radial derivative there).
#pragma once

#include "apx_internal.h"

namespace apx {

// FP64 2^x and log2(x) for the profile, from their series (a few ulp; the profile needs
// FP64-level smoothness in theta, not correctly rounded results).
//   2^x: x = n + f with n the nearest integer (f exact, |f| <= 1/2), 2^f = e^(f ln 2) by its
//   Taylor series to degree 13 (next term < 5e-18), then scaled by 2^n.  Arguments are
//   clamped to [-1100, 1100] first (results underflow to 0 / overflow to inf as they
//   should); NaN propagates.
//   log2(x), x positive and normal: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m =
//   2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...), s = (m - 1) / (m + 1), |s| <= 0.1716, to
//   s^21 (next term < 3e-17 relative); 1/(m + 1) is the hardware reciprocal refined by two
//   Newton steps.
struct Exp2Series {
    double c[14];
    constexpr Exp2Series() : c() {
        c[0] = 1.0;
        for (int k = 1; k < 14; ++k) c[k] = c[k - 1] * 0.6931471805599453094 / k;
    }
};
struct AtanhSeries {
    double q[11];
    constexpr AtanhSeries() : q() {
        for (int k = 0; k < 11; ++k) q[k] = 1.0 / (2 * k + 1);
    }
};

__device__ __forceinline__ double exp2_d(double x) {
    constexpr Exp2Series S;
    x = x < -1100.0 ? -1100.0 : (x > 1100.0 ? 1100.0 : x);
    const double n = rint(x);
    const double f = x - n;
    double p = S.c[13];
#pragma unroll
    for (int k = 12; k >= 0; --k) p = fma(p, f, S.c[k]);
    return ldexp(p, (int)n);
}

__device__ __forceinline__ double log2_d(double x) {
    constexpr AtanhSeries S;
    double m = __builtin_amdgcn_frexp_mant(x);          // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    if (m < 0.70710678118654752440) {
        m += m;
        e -= 1;
    }
    const double d = m + 1.0;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    const double s = (m - 1.0) * r;
    const double z = s * s;
    double q = S.q[10];
#pragma unroll
    for (int k = 9; k >= 0; --k) q = fma(q, z, S.q[k]);
    return fma(2.0 * s * q, 1.4426950408889634074, (double)e);
}

// Table-driven FP64 2^x and log2(x) for the objective render (fewer FP64 operations than
// the series above; same target: a few ulp, smooth in x).  The table (PTAB_N doubles, built
// on the host in extended precision, staged in LDS by the caller) holds
//   [0, 64)    2^(j/64);
//   [64, 128)  r_j = 1/c_j rounded, c_j = 1/2 + (j + 1/2)/128 the centre of the j-th of 64
//              intervals that cut [1/2, 1);
//   [128, 192) -log2(r_j).
//   2^x: n = rint(64 x), f = x - n/64 (exact, |f| <= 1/128), 2^x = 2^(n >> 6) 2^((n & 63)/64)
//   e^(f ln 2), the last by its Taylor series to degree 5 (next term < 4e-17).  With CLAMP, x
//   is first clamped to [-1100, 1100] (results underflow to 0 / overflow to inf) by a max and
//   a min, which map a NaN argument to -1100; the callers' arguments are finite (the
//   profile's constants are checked before any pixel is rendered).  Without it |x| must stay
//   below 2^24 (n fits an int): the argument g log2(R^2) - h of t does, as |g| <= 1/0.72 and
//   |h| < 37 for a valid component and |log2 R^2| <= 1024 (R^2 finite, floored at 1e-12).
//   log2(x) = e + log2(m) for x = m 2^e, m in [1/2, 1): with j the interval of m (the top
//   six mantissa bits), u = m r_j - 1 (one rounding, |u| < 0.0079) and log2(m) = -log2(r_j)
//   + ln(1 + u) log2(e), ln(1 + u) by its series to u^7 (next term < 2e-18).
//
// A VALU instruction reads at most one SGPR operand, and the compiler turns FMAs into the
// two-address v_fmac_f64 with a fresh copy of a constant addend at every node.  The node
// loop's FMAs are therefore written out (fma_vvs, fma_svv: the operand kinds in order) with
// their constants in SGPRs or, where an FMA needs two, in the VGPR copies of Poly64Regs,
// which are made once per component before the loop.  Same operations in the same order as
// the plain fma() calls: the same results.
constexpr double EXP2_C5 = 0.6931471805599453094 * 0.6931471805599453094 * 0.6931471805599453094 *
                           0.6931471805599453094 * 0.6931471805599453094 / 120.0;
constexpr double EXP2_C4 = 0.6931471805599453094 * 0.6931471805599453094 * 0.6931471805599453094 *
                           0.6931471805599453094 / 24.0;
struct Poly64Regs { double e4, l6, h, A; };            // EXP2_C4, -1/6, the component's h and A
__device__ __forceinline__ double vcopy64(double s) {
    double v;
    asm("v_mov_b64 %0, %1" : "=v"(v) : "s"(s));
    return v;
}
__device__ __forceinline__ Poly64Regs poly64_regs(const CompConst& c) {
    return {vcopy64(EXP2_C4), vcopy64(-1.0 / 6.0), vcopy64(c.h_d), vcopy64(c.A_d)};
}
__device__ __forceinline__ double fma_vvs(double a, double b, double cs) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(cs));
    return r;
}
__device__ __forceinline__ double fma_svv(double as, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "s"(as), "v"(b), "v"(c));
    return r;
}

template <bool CLAMP>
__device__ __forceinline__ double exp2_t(double x, const double* __restrict__ tab, const Poly64Regs& rg) {
    constexpr double L = 0.6931471805599453094;
    if constexpr (CLAMP) x = __builtin_fmin(__builtin_fmax(x, -1100.0), 1100.0);
    const double nd = rint(x * 64.0);
    const double f = fma(nd, -0.015625, x);
    const int n = (int)nd;
    double p = fma_svv(EXP2_C5, f, rg.e4);
    p = fma_vvs(p, f, L * L * L / 6.0);
    p = fma_vvs(p, f, L * L / 2.0);
    p = fma_vvs(p, f, L);
    p = fma(p, f, 1.0);
    return ldexp(tab[n & 63] * p, n >> 6);
}

__device__ __forceinline__ double log2_t(double x, const double* __restrict__ tab, const Poly64Regs& rg) {
    const double m = __builtin_amdgcn_frexp_mant(x);          // [1/2, 1)
    const int e = __builtin_amdgcn_frexp_exp(x);
    const int j = (__double2hiint(m) >> 14) & 63;
    const double u = fma(m, tab[64 + j], -1.0);
    double q = fma_svv(1.0 / 7.0, u, rg.l6);
    q = fma_vvs(q, u, 1.0 / 5.0);
    q = fma_vvs(q, u, -1.0 / 4.0);
    q = fma_vvs(q, u, 1.0 / 3.0);
    q = fma(q, u, -0.5);
    q = fma(q, u, 1.0);
    return fma(q * u, 1.4426950408889634074, tab[128 + j] + (double)e);
}

// I at a point given in the component's frame (xp along the major axis, yq = yp / q).
__device__ __forceinline__ double sersic_I64_r(const CompConst& c, double xp, double yq,
                                               const double* __restrict__ tab, const Poly64Regs& rg) {
    const double R2 = fmax(xp * xp + yq * yq, 1e-12);
    const double t = exp2_t<false>(fma(c.g_d, log2_t(R2, tab, rg), -rg.h), tab, rg);
    return exp2_t<true>(fma(-c.B_d, t, rg.A), tab, rg);
}

__device__ __forceinline__ double sersic_I64_t(const CompConst& c, double dx, double dy,
                                               const double* __restrict__ tab) {
    const double xp = dx * c.cs_d + dy * c.sn_d;
    const double yq = (-dx * c.sn_d + dy * c.cs_d) * c.iq_d;
    return sersic_I64_r(c, xp, yq, tab, poly64_regs(c));
}

__device__ __forceinline__ double sersic_I64(const CompConst& c, double dx, double dy) {
    const double xp = dx * c.cs_d + dy * c.sn_d;
    const double yq = (-dx * c.sn_d + dy * c.cs_d) * c.iq_d;
    const double R2 = fmax(xp * xp + yq * yq, 1e-12);
    const double t = exp2_d(c.g_d * log2_d(R2) - c.h_d);
    return exp2_d(c.A_d - c.B_d * t);
}

// Adds wgt * I and wgt * dI/dtheta_k (k = x0, y0, q, PA, n, Re, log10 Ie) into val, acc.
__device__ __forceinline__ void sersic_dI64(const CompConst& c, double dx, double dy, double wgt,
                                            double& val, double acc[7]) {
    const double xp = dx * c.cs_d + dy * c.sn_d;
    const double yp = -dx * c.sn_d + dy * c.cs_d;
    const double iq = c.iq_d;
    const double yq = yp * iq;
    double R2 = xp * xp + yq * yq;
    const bool floored = R2 < 1e-12;
    R2 = floored ? 1e-12 : R2;
    const double lt = c.g_d * log2_d(R2) - c.h_d;
    const double t = exp2_d(lt);
    const double I = exp2_d(c.A_d - c.B_d * t) * wgt;
    const double inv_n = 2.0 * c.g_d;
    const double b = c.B_d * 0.69314718055994531;   // B = b log2 e
    const double G = floored ? 0.0 : -I * b * t * inv_n / R2;   // (dI/dR) / R
    const double dxp = G * xp;
    const double dyp = G * yq * iq;
    val += I;
    acc[0] += -c.cs_d * dxp + c.sn_d * dyp;
    acc[1] += -c.sn_d * dxp - c.cs_d * dyp;
    acc[2] += -G * yq * yq * iq;
    acc[3] += G * xp * yp * (1.0 - iq * iq);
    acc[4] += I * ((double)c.bp * (1.0 - t) + b * t * lt * 0.69314718055994531 * inv_n);
    acc[5] += I * b * t * inv_n / ((double)c.re);
    acc[6] += I * 2.302585092994046;
}

}  // namespace apx
