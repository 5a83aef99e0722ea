// FP64 Sersic profile (§2.1.1) and its seven parameter derivatives at one point, shared by
// the FP64 render and the adaptive integration.  Same parametrisation as the FP32 kernels:
// I = 2^(A - B t), t = 2^(g log2 R^2 - h) = (R / Re)^(1/n), with the elliptical radius
// floored at R^2 = 1e-12 (the cusp of n > 1 profiles; no radial derivative there).
#pragma once

#include "apx_internal.h"

namespace apx {

__device__ __forceinline__ double sersic_I64(const CompConst& c, double dx, double dy) {
    const double xp = dx * c.cs_d + dy * c.sn_d;
    const double yq = (-dx * c.sn_d + dy * c.cs_d) / c.q_d;
    const double R2 = fmax(xp * xp + yq * yq, 1e-12);
    const double t = exp2(c.g_d * log2(R2) - c.h_d);
    return exp2(c.A_d - c.B_d * t);
}

// Adds wgt * I and wgt * dI/dtheta_k (k = x0, y0, q, PA, n, Re, log10 Ie) into val, acc.
__device__ __forceinline__ void sersic_dI64(const CompConst& c, double dx, double dy, double wgt,
                                            double& val, double acc[7]) {
    const double xp = dx * c.cs_d + dy * c.sn_d;
    const double yp = -dx * c.sn_d + dy * c.cs_d;
    const double iq = 1.0 / c.q_d;
    const double yq = yp * iq;
    double R2 = xp * xp + yq * yq;
    const bool floored = R2 < 1e-12;
    R2 = floored ? 1e-12 : R2;
    const double lt = c.g_d * log2(R2) - c.h_d;
    const double t = exp2(lt);
    const double I = exp2(c.A_d - c.B_d * t) * wgt;
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
