// Component evaluation kernels: parameter preparation (b_n on the device), the
// supersampled pre-convolution render, derivative images for the Jacobian and the
// adjoint contraction for the chi^2 gradient.
//
// Profile (Sersic, §2.1.1): I(R) = Ie exp(-b_n ((R/Re)^(1/n) - 1)) with elliptical
// R = sqrt(x'^2 + (y'/q)^2), x' = dx cos PA + dy sin PA, y' = -dx sin PA + dy cos PA.
// It is evaluated as I = 2^(A - B t), t = 2^(g log2 R^2 - h) with A = log2 Ie + b log2 e,
// B = b log2 e, g = 1/(2n), h = log2(Re)/n: three hardware transcendentals (v_log_f32,
// v_exp_f32) per sub-pixel node, the exponent arithmetic in FP64 (full rate on CDNA4)
// so the FP32 result carries only the transcendentals' rounding.
// Pixel integration (§2.1.2): area * sum_k w_k I(node_k) over s x s nodes.
#include "apx_internal.h"
#include "sersic64.h"

namespace apx {

#define LN2F 0.69314718055994531f
#define LN10F 2.3025850929940457f

// ------------------------------------------------------------------------ b_n
// b_n and db_n/dn by cubic Hermite interpolation of the host-built FP64 table (nodes
// every 1/256 in n; interpolation error below 1e-10 relative on [0.36, 10]).
__device__ void sersic_bn_table(const double* tab, double n, double& b, double& bp) {
    const double u = (n - BN_N0) * BN_INV_H;
    int k = (int)floor(u);
    k = k < 0 ? 0 : (k > BN_COUNT - 2 ? BN_COUNT - 2 : k);
    const double t = u - k, h = 1.0 / BN_INV_H;
    const double b0 = tab[2 * k], d0 = tab[2 * k + 1], b1 = tab[2 * k + 2], d1 = tab[2 * k + 3];
    const double t2 = t * t, t3 = t2 * t;
    b = (2 * t3 - 3 * t2 + 1) * b0 + (t3 - 2 * t2 + t) * h * d0 + (-2 * t3 + 3 * t2) * b1 + (t3 - t2) * h * d1;
    bp = (6 * t2 - 6 * t) * BN_INV_H * b0 + (3 * t2 - 4 * t + 1) * d0 + (-6 * t2 + 6 * t) * BN_INV_H * b1 +
         (3 * t2 - 2 * t) * d1;
}

// ------------------------------------------------------------------- re-centring taps
// Weights that move a pixel-sampled image by delta (|delta| <= 1/2) along one axis,
// shifted(i) = sum_t w[t + a] img(i - t), and their derivatives in delta (§2.1.3).
// Bilinear: the two nearest samples (derivative from the right at delta = 0).  Lanczos of
// order a: sinc(t - delta) sinc((t - delta) / a) (normalised sinc), divided by its sum.
__device__ __forceinline__ double nsinc(double x) { return x == 0.0 ? 1.0 : sinpi(x) / (M_PI * x); }
__device__ __forceinline__ double nsinc_d(double x) { return x == 0.0 ? 0.0 : (cospi(x) - nsinc(x)) / x; }

__device__ void shift_taps(int method, int a, double delta, double* w, double* dw) {
    if (method == APX_SHIFT_BILINEAR) {
        const double side = delta >= 0.0 ? 1.0 : -1.0;
        for (int j = 0; j < 3; ++j) {
            const double t = (double)(j - 1);
            w[j] = fmax(0.0, 1.0 - fabs(t - delta));
            dw[j] = (t == 0.0 ? -side : 0.0) + (t == side ? side : 0.0);
        }
        return;
    }
    double N = 0.0, dN = 0.0;
    for (int j = 0; j <= 2 * a; ++j) {
        const double x = (double)(j - a) - delta;
        const bool in = fabs(x) < (double)a;
        const double L = in ? nsinc(x) * nsinc(x / a) : 0.0;
        const double dL = in ? -(nsinc_d(x) * nsinc(x / a) + nsinc(x) * nsinc_d(x / a) / a) : 0.0;
        w[j] = L;
        dw[j] = dL;
        N += L;
        dN += dL;
    }
    for (int j = 0; j <= 2 * a; ++j) {
        dw[j] = (dw[j] * N - w[j] * dN) / (N * N);
        w[j] = w[j] / N;
    }
}

// ------------------------------------------------------------------------- prep
__global__ void k_prep(Plan p, const double* __restrict__ theta, int lm_trial) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n_images) {
        const DImage& im = p.images[i];
        const double sky = im.sky_par >= 0 ? theta[im.sky_par] : im.sky_fixed;
        p.sky_val[i] = sky;
        if (!isfinite(sky)) {
            if (lm_trial) atomicOr(&p.lmf[im.sub].trial_bad, 1);
            else atomicOr(p.sticky, FLAG_NONFINITE);
        }
    }
    if (i >= p.n_comps) return;
    const DComp cp = p.comps[i];
    const DImage& im = p.images[cp.image];
    double v[7];
    bool finite = true;
    for (int k = 0; k < 7; ++k) {
        v[k] = cp.par[k] >= 0 ? theta[cp.par[k]] : cp.fixed[k];
        finite = finite && isfinite(v[k]);
    }
    CompConst c;
    c.x0 = c.y0 = c.cs_d = c.sn_d = c.q_d = c.iq_d = c.kre = c.h_d = c.A_d = c.B_d = c.g_d = 0.0;
    c.cs = c.sn = c.iq = c.g = c.b = c.bp = c.n = c.re = c.q = c.F = 0.f;
    c.pad = 0;
    c.F64 = 0.0;
    bool valid = finite;
    if (cp.type == APX_SERSIC) {
        const double q = v[2], pa = v[3], n = v[4], re = v[5], lie = v[6];
        valid = valid && q >= 0.01 && q <= 1.0 && n >= 0.36 && n <= 10.0 && re >= 0.01 && re <= 1e4;
        if (valid) {
            double b, bp;
            sersic_bn_table(p.bn_tab, n, b, bp);
            const double log2e = 1.4426950408889634;
            c.x0 = v[0];
            c.y0 = v[1];
            c.cs_d = cos(pa);
            c.sn_d = sin(pa);
            c.q_d = q;
            c.iq_d = 1.0 / q;
            c.kre = p.k_re * re;
            c.h_d = log2(re) / n;
            c.A_d = lie * 3.3219280948873622 + b * log2e;
            c.B_d = b * log2e;
            c.g_d = 0.5 / n;
            c.cs = (float)c.cs_d;
            c.sn = (float)c.sn_d;
            c.iq = (float)(1.0 / q);
            c.g = (float)(0.5 / n);
            c.b = (float)b;
            c.bp = (float)bp;
            c.n = (float)n;
            c.re = (float)re;
            c.q = (float)q;
            if (p.shift != APX_SHIFT_NONE) {
                // sample with the centre at the nearest pixel centre n; the taps move the
                // result back by delta = (pixel position) - n
                const double px = im.inv[0] + im.inv[1] * c.x0 + im.inv[2] * c.y0;
                const double py = im.inv[3] + im.inv[4] * c.x0 + im.inv[5] * c.y0;
                const double nx = floor(px + 0.5), ny = floor(py + 0.5);
                c.x0 = im.aff[0] + im.aff[1] * nx + im.aff[2] * ny;
                c.y0 = im.aff[3] + im.aff[4] * nx + im.aff[5] * ny;
                double* tp = p.stap + (long long)i * STAP_STRIDE;
                shift_taps(p.shift, p.shift_a, px - nx, tp, tp + 2 * SHIFT_NT);
                shift_taps(p.shift, p.shift_a, py - ny, tp + SHIFT_NT, tp + 3 * SHIFT_NT);
            }
        }
    } else {
        // point source: sky position -> pixel position of its image
        const double ux = v[0], uy = v[1];
        const double px = im.inv[0] + im.inv[1] * ux + im.inv[2] * uy;
        const double py = im.inv[3] + im.inv[4] * ux + im.inv[5] * uy;
        c.x0 = px;
        c.y0 = py;
        c.F64 = exp(v[2] * 2.302585092994046);
        c.F = (float)c.F64;
    }
    c.valid = valid ? 1 : 0;
    if (cp.type == APX_SERSIC && p.shift != APX_SHIFT_NONE && !valid)
        for (int j = 0; j < STAP_STRIDE; ++j) p.stap[(long long)i * STAP_STRIDE + j] = 0.0;
    p.cc[i] = c;
    if (!valid) {
        if (lm_trial) atomicOr(&p.lmf[cp.sub].trial_bad, 1);
        else atomicOr(p.sticky, FLAG_DOMAIN);
    }
}

// Stamps of every image for this theta: fixed stamps promoted to FP64 (objective
// convolution); live Moffat stamps (§2.1.3, §3.4) rendered at the integer offsets,
// normalised, with d/dn and d/dR_d of the normalised stamp (quotient rule), in FP64 and
// as FP32 copies for the FP32 kernels.  One workgroup per image; the sums are ordered.
__global__ __launch_bounds__(256) void k_psf_prep(Plan p, const double* __restrict__ theta, int lm_trial) {
    __shared__ double red[4][3];
    const int k = blockIdx.x;
    const DImage& im = p.images[k];
    const int P = im.P, c = im.c, P2 = P * P;
    double* K64 = p.psf64 + im.psf_off;
    if (!im.live) {
        for (int e = threadIdx.x; e < P2; e += blockDim.x) K64[e] = (double)p.psf[im.psf_off + e];
        return;
    }
    double n = im.live_par[0] >= 0 ? theta[im.live_par[0]] : im.live_fixed[0];
    double rd = im.live_par[1] >= 0 ? theta[im.live_par[1]] : im.live_fixed[1];
    const bool valid = isfinite(n) && isfinite(rd) && n >= PSF_N_MIN && n <= PSF_N_MAX &&
                       rd >= PSF_RD_MIN && rd <= PSF_RD_MAX;
    if (!valid) {
        if (threadIdx.x == 0) {
            if (lm_trial) atomicOr(&p.lmf[im.sub].trial_bad, 1);
            else atomicOr(p.sticky, FLAG_DOMAIN);
        }
        n = 1.0;                                   // keeps the (unused) stamp finite
        rd = 1.0;
    }
    const double ird2 = 1.0 / (rd * rd);
    double sf = 0.0, sdn = 0.0, sdr = 0.0;
    for (int e = threadIdx.x; e < P2; e += blockDim.x) {
        const double u = (double)(e / P - c), v = (double)(e % P - c);
        const double r2 = u * u + v * v;
        const double x = 1.0 + r2 * ird2;
        const double f = exp(-n * log(x));
        sf += f;
        sdn += -log(x) * f;
        sdr += f * (-n) / x * (-2.0 * r2 * ird2 / rd);
    }
    for (int o = 32; o > 0; o >>= 1) {
        sf += __shfl_xor(sf, o, 64);
        sdn += __shfl_xor(sdn, o, 64);
        sdr += __shfl_xor(sdr, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = sf;
        red[threadIdx.x >> 6][1] = sdn;
        red[threadIdx.x >> 6][2] = sdr;
    }
    __syncthreads();
    const double S = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
    const double Sdn = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
    const double Sdr = ((red[0][2] + red[1][2]) + red[2][2]) + red[3][2];
    const double iS = 1.0 / S;
    float* K32 = p.psf_live + im.live_off;
    for (int e = threadIdx.x; e < P2; e += blockDim.x) {
        const double u = (double)(e / P - c), v = (double)(e % P - c);
        const double r2 = u * u + v * v;
        const double x = 1.0 + r2 * ird2;
        const double f = exp(-n * log(x));
        const double Kv = f * iS;
        const double dn = (-log(x) * f - Kv * Sdn) * iS;
        const double dr = (f * (-n) / x * (-2.0 * r2 * ird2 / rd) - Kv * Sdr) * iS;
        K64[e] = Kv;
        K32[e] = (float)Kv;
        K32[P2 + e] = (float)dn;
        K32[2 * P2 + e] = (float)dr;
    }
}

hipError_t launch_prep(const Plan& p, const double* theta, int lm_trial, hipStream_t st) {
    const int n = p.n_comps > p.n_images ? p.n_comps : p.n_images;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep, dim3((n + 127) / 128), dim3(128), 0, st, p, theta, lm_trial);
    if (p.n_images > 0) hipLaunchKernelGGL(k_psf_prep, dim3(p.n_images), dim3(256), 0, st, p, theta, lm_trial);
    return hipGetLastError();
}

// ------------------------------------------------------------------ samples
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ float sersic_I(const CompConst& c, float dx, float dy) {
    const float xp = fmaf(dx, c.cs, dy * c.sn);
    const float yq = fmaf(dy, c.cs, -dx * c.sn) * c.iq;
    const float R2 = fmaxf(fmaf(xp, xp, yq * yq), 1e-12f);
    const double lt = fma((double)c.g, (double)fast_log2(R2), -c.h_d);
    const float t = fast_exp2((float)lt);
    return fast_exp2((float)fma(-c.B_d, (double)t, c.A_d));
}

// Adds wgt * dI/dtheta_k (k = x0, y0, q, PA, n, Re, log10 Ie) into acc.
// ... at a point given in the component's frame (xp along the major axis, yp across it)
__device__ __forceinline__ void sersic_dI_r(const CompConst& c, float xp, float yp, float wgt, float acc[7]) {
    const float yq = yp * c.iq;
    float R2 = fmaf(xp, xp, yq * yq);
    const bool floored = R2 < 1e-12f;
    R2 = floored ? 1e-12f : R2;
    const float lt = (float)fma((double)c.g, (double)fast_log2(R2), -c.h_d);
    const float t = fast_exp2(lt);
    const float I = fast_exp2((float)fma(-c.B_d, (double)t, c.A_d)) * wgt;
    const float inv_n = 2.f * c.g;
    // dI/dR divided by R (hardware reciprocals, 1 ulp: these derivative images feed the
    // FP32 Jacobian and adjoint, held to 3e-5 of each column's scale)
    const float bt = I * c.b * t * inv_n;
    const float G = floored ? 0.f : -bt * __builtin_amdgcn_rcpf(R2);
    const float dxp = G * xp;                 // dI/dx'
    const float dyp = G * yq * c.iq;          // dI/dy' = G y' / q^2
    acc[0] += -c.cs * dxp + c.sn * dyp;
    acc[1] += -c.sn * dxp - c.cs * dyp;
    acc[2] += -G * yq * yq * c.iq;            // dR/dq = -y'^2 / (q^3 R)
    acc[3] += G * xp * yp * (1.f - c.iq * c.iq);
    acc[4] += I * (c.bp * (1.f - t) + c.b * t * lt * LN2F * inv_n);
    acc[5] += bt * __builtin_amdgcn_rcpf(c.re);
    acc[6] += I * LN10F;
}

__device__ __forceinline__ void sersic_dI(const CompConst& c, float dx, float dy, float wgt,
                                          float acc[7]) {
    sersic_dI_r(c, fmaf(dx, c.cs, dy * c.sn), fmaf(dy, c.cs, -dx * c.sn), wgt, acc);
}

struct NodeSet {
    int s, rule, mode;
    float o[MAX_NODES_1D], w[MAX_NODES_1D];
};

__device__ __forceinline__ bool within_kre(const CompConst& c, double ucx, double ucy) {
    const double dx = ucx - c.x0, dy = ucy - c.y0;
    const double xp = dx * c.cs_d + dy * c.sn_d;
    const double yp = -dx * c.sn_d + dy * c.cs_d;
    const double yq = yp / c.q_d;
    return sqrt(xp * xp + yq * yq) < c.kre;
}

// Pixel value (before the area factor) of a Sersic component.
__device__ __forceinline__ float sersic_pixel(const Plan& p, const CompConst& c, const DImage& im,
                                              double ucx, double ucy) {
    const float dxc = (float)(ucx - c.x0), dyc = (float)(ucy - c.y0);
    if (p.mode == APX_MODE_WITHIN_K_RE && !within_kre(c, ucx, ucy)) return sersic_I(c, dxc, dyc);
    const float a1 = (float)im.aff[1], a2 = (float)im.aff[2], a4 = (float)im.aff[4], a5 = (float)im.aff[5];
    float sum = 0.f;
    for (int ky = 0; ky < p.s; ++ky) {
        const float oy = p.node_o[ky], wy = p.node_w[ky];
        float row = 0.f;
        for (int kx = 0; kx < p.s; ++kx) {
            const float ox = p.node_o[kx];
            row = fmaf(p.node_w[kx], sersic_I(c, dxc + fmaf(a1, ox, a2 * oy), dyc + fmaf(a4, ox, a5 * oy)), row);
        }
        sum = fmaf(wy, row, sum);
    }
    return sum;
}

// Window-pixel index of (y, x) in the adaptive-integration arrays.
__device__ __forceinline__ long long adapt_index(const DComp& cp, int y, int x) {
    return cp.aoff + (long long)(y - cp.box[0]) * (cp.box[3] - cp.box[1]) + (x - cp.box[1]);
}

__device__ __forceinline__ void sersic_pixel_grad(const Plan& p, const CompConst& c, const DImage& im,
                                                  const DComp& cp, int y, int x, double ucx, double ucy,
                                                  float acc[7]) {
    for (int k = 0; k < 7; ++k) acc[k] = 0.f;
    const float dxc = (float)(ucx - c.x0), dyc = (float)(ucy - c.y0);
    if (p.mode == APX_MODE_WITHIN_K_RE && !within_kre(c, ucx, ucy)) {
        sersic_dI(c, dxc, dyc, 1.f, acc);
        return;
    }
    if (p.mode == APX_MODE_ADAPTIVE) {
        // the rule chosen at this theta: centre, 3 x 3 (the s x s nodes below), or refined
        const int code = p.acode[adapt_index(cp, y, x)];
        if (code == 0) {
            sersic_dI(c, dxc, dyc, 1.f, acc);
            return;
        }
        if (code < 0) {
            const long long r = -1LL - code;          // refine entry (always < n_apix)
            const float* dv = p.adval + 7LL * (r < p.n_apix ? r : 0);
            for (int k = 0; k < 7; ++k) acc[k] = r < p.n_apix ? dv[k] : __builtin_nanf("");
            return;
        }
    }
    // the nodes in the component's frame: (xp, yp) = (xp0 + ox ax + oy bx, yp0 + ox ay + oy by)
    // with (ax, ay), (bx, by) the pixel axes mapped and rotated once
    const float a1 = (float)im.aff[1], a2 = (float)im.aff[2], a4 = (float)im.aff[4], a5 = (float)im.aff[5];
    const float xp0 = fmaf(dxc, c.cs, dyc * c.sn), yp0 = fmaf(dyc, c.cs, -dxc * c.sn);
    const float ax = fmaf(a1, c.cs, a4 * c.sn), ay = fmaf(a4, c.cs, -a1 * c.sn);
    const float bx = fmaf(a2, c.cs, a5 * c.sn), by = fmaf(a5, c.cs, -a2 * c.sn);
    for (int ky = 0; ky < p.s; ++ky) {
        const float oy = p.node_o[ky];
        const float xr = fmaf(oy, bx, xp0), yr = fmaf(oy, by, yp0);
        for (int kx = 0; kx < p.s; ++kx) {
            const float ox = p.node_o[kx];
            sersic_dI_r(c, fmaf(ox, ax, xr), fmaf(ox, ay, yr), p.node_w[kx] * p.node_w[ky], acc);
        }
    }
}

__device__ __forceinline__ double point_weight(const CompConst& c, int y, int x) {
    const double wx = fmax(0.0, 1.0 - fabs((double)x - c.x0));
    const double wy = fmax(0.0, 1.0 - fabs((double)y - c.y0));
    return wx * wy;
}

// The same pixel integral in double precision throughout (FP64 log2/exp2), for the
// objective path: chi^2 differences of the LM gain ratio are resolved far below FP32
// rounding.
// tab: the 2^x / log2 table in LDS (PTAB_N doubles)
// The nodes of a pixel in the component's frame: the node at pixel offset (ox, oy) sits at
// (xp, yq) = (xp0 + ox ax + oy bx, yq0 + ox ay + oy by), with (xp0, yq0) the pixel centre's
// rotated and 1/q-scaled offset and (ax, ay), (bx, by) the images of the pixel axes (the
// affine map's columns rotated and scaled the same way): two FMAs per node instead of
// mapping and rotating every node.
__device__ __forceinline__ double sersic_pixel64(const Plan& p, const CompConst& c, const DImage& im,
                                                 double ucx, double ucy, const double* __restrict__ tab) {
    const double dxc = ucx - c.x0, dyc = ucy - c.y0;
    if (p.mode == APX_MODE_WITHIN_K_RE && !within_kre(c, ucx, ucy)) return sersic_I64_t(c, dxc, dyc, tab);
    const double xp0 = dxc * c.cs_d + dyc * c.sn_d;
    const double yq0 = (-dxc * c.sn_d + dyc * c.cs_d) * c.iq_d;
    const double ax = im.aff[1] * c.cs_d + im.aff[4] * c.sn_d;
    const double bx = im.aff[2] * c.cs_d + im.aff[5] * c.sn_d;
    const double ay = (-im.aff[1] * c.sn_d + im.aff[4] * c.cs_d) * c.iq_d;
    const double by = (-im.aff[2] * c.sn_d + im.aff[5] * c.cs_d) * c.iq_d;
    const Poly64Regs rg = poly64_regs(c);
    double sum = 0.0;
    if (p.s == 3) {
        // the usual 3 x 3 rule, unrolled with its nodes and weights loaded once (the same
        // operations in the same order as the loop below)
        const double od[3] = {p.node_od[0], p.node_od[1], p.node_od[2]};
        const double wd[3] = {p.node_wd[0], p.node_wd[1], p.node_wd[2]};
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const double xr = fma(od[ky], bx, xp0), yr = fma(od[ky], by, yq0);
            double row = 0.0;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx)
                row += wd[kx] * sersic_I64_r(c, fma(od[kx], ax, xr), fma(od[kx], ay, yr), tab, rg);
            sum += wd[ky] * row;
        }
        return sum;
    }
    for (int ky = 0; ky < p.s; ++ky) {
        const double oy = p.node_od[ky];
        const double xr = fma(oy, bx, xp0), yr = fma(oy, by, yq0);
        double row = 0.0;
        for (int kx = 0; kx < p.s; ++kx) {
            const double ox = p.node_od[kx];
            row += p.node_wd[kx] * sersic_I64_r(c, fma(ox, ax, xr), fma(ox, ay, yr), tab, rg);
        }
        sum += p.node_wd[ky] * row;
    }
    return sum;
}

// Stage the 2^x / log2 table into LDS (the caller synchronises before use).
__device__ __forceinline__ void stage_ptab(const Plan& p, double* sh) {
    for (int k = (int)threadIdx.x; k < PTAB_N; k += (int)blockDim.x) sh[k] = p.ptab[k];
}

// ------------------------------------------------------------- re-centred tiles
// A re-centred Sersic (§2.1.3) enters the pre-convolution grid as T * S': S' sampled with
// the centre at the nearest pixel centre, T the separable interpolation taps (the shift
// commutes with the PSF convolution).  A workgroup owning an RT_Y x RT_X tile with origin
// (y0, x0) samples S' once over the tile grown by a on every side into LDS (zero outside
// the sampled window sbox), then every pixel sums its (2a+1)^2 taps from LDS.
constexpr int SH_H = RT_Y + 2 * APX_SHIFT_MAX_A, SH_W = RT_X + 2 * APX_SHIFT_MAX_A;

// Stage NPL planes of f(ry, rx, out[NPL]) over the grown tile, sh[q][hy * (RT_X + 2a) + hx],
// and the component's taps into tw (wx, wy, dwx, dwy; SHIFT_NT each).  The caller
// synchronises before reading them.
template <int NPL, typename T, typename F>
__device__ __forceinline__ void stage_halo(const Plan& p, int ci, const DComp& cp, int y0, int x0,
                                           T (*sh)[SH_H * SH_W], T* tw, F&& f) {
    const int a = p.shift_a, HW = RT_X + 2 * a, n = (RT_Y + 2 * a) * HW;
    if (threadIdx.x < STAP_STRIDE) tw[threadIdx.x] = (T)p.stap[(long long)ci * STAP_STRIDE + threadIdx.x];
    for (int e = (int)threadIdx.x; e < n; e += 256) {
        const int hy = e / HW, hx = e - hy * HW;
        const int ry = y0 - a + hy, rx = x0 - a + hx;
        T v[NPL];
        for (int q = 0; q < NPL; ++q) v[q] = (T)0;
        if (ry >= cp.sbox[0] && ry < cp.sbox[2] && rx >= cp.sbox[1] && rx < cp.sbox[3]) f(ry, rx, v);
        for (int q = 0; q < NPL; ++q) sh[q][e] = v[q];
    }
}

// sum_t wy[ty] wx[tx] plane(ly - ty, lx - tx) for the pixel (ly, lx) of the tile (taps in
// LDS, the same for every thread); unrolled per half-width A.
template <int A, typename T>
__device__ __forceinline__ T tap_sum_a(const T* plane, int ly, int lx, const T* wy, const T* wx) {
    constexpr int HW = RT_X + 2 * A;
    const T* base = plane + (ly + 2 * A) * HW + lx + 2 * A;
    T out = (T)0;
#pragma unroll
    for (int jy = 0; jy <= 2 * A; ++jy) {
        const T* row = base - jy * HW;
        T acc = (T)0;
#pragma unroll
        for (int jx = 0; jx <= 2 * A; ++jx) acc = fma(wx[jx], row[-jx], acc);
        out = fma(wy[jy], acc, out);
    }
    return out;
}

template <typename T>
__device__ __forceinline__ T tap_sum(const T* plane, int a, int ly, int lx, const T* wy, const T* wx) {
    switch (a) {
        case 1: return tap_sum_a<1>(plane, ly, lx, wy, wx);
        case 2: return tap_sum_a<2>(plane, ly, lx, wy, wx);
        case 3: return tap_sum_a<3>(plane, ly, lx, wy, wx);
        case 4: return tap_sum_a<4>(plane, ly, lx, wy, wx);
        default: return tap_sum_a<5>(plane, ly, lx, wy, wx);
    }
}

// The 7 pre-convolution derivative values (area included: it is in the staged planes) of
// a re-centred Sersic at pixel (ly, lx) of a tile whose origin is (y0, x0):
// d/d(q, PA, n, Re, log Ie) are T * dS'/dtheta; x0 and y0 move only delta, so
// d/d x0 = inv1 (dT/d delta_x * S') + inv4 (dT/d delta_y * S') (inv2, inv5 for y0), with
// S' = (d/d log Ie plane) / ln 10.  Every thread of the block calls it.
__device__ void shifted_derivs(const Plan& p, int ci, const CompConst& c, const DComp& cp, const DImage& im,
                               int y0, int x0, int ly, int lx, bool want, float (*sh)[SH_H * SH_W],
                               float* tw, float out[7]) {
    stage_halo<5, float>(p, ci, cp, y0, x0, sh, tw, [&](int ry, int rx, float* v) {
        const double ucx = im.aff[0] + im.aff[1] * rx + im.aff[2] * ry;
        const double ucy = im.aff[3] + im.aff[4] * rx + im.aff[5] * ry;
        float acc[7];
        sersic_pixel_grad(p, c, im, cp, ry, rx, ucx, ucy, acc);
        const float area = (float)im.area;
        for (int q = 0; q < 5; ++q) v[q] = acc[q + 2] * area;
    });
    __syncthreads();
    for (int q = 0; q < 7; ++q) out[q] = 0.f;
    if (want) {
        const float *wx = tw, *wy = tw + SHIFT_NT, *dwx = tw + 2 * SHIFT_NT, *dwy = tw + 3 * SHIFT_NT;
        const int a = p.shift_a;
        for (int q = 0; q < 5; ++q) out[q + 2] = tap_sum(sh[q], a, ly, lx, wy, wx);
        const float inv_ln10 = 1.f / LN10F;
        const float mx = tap_sum(sh[4], a, ly, lx, wy, dwx) * inv_ln10;
        const float my = tap_sum(sh[4], a, ly, lx, dwy, wx) * inv_ln10;
        out[0] = (float)im.inv[1] * mx + (float)im.inv[4] * my;
        out[1] = (float)im.inv[2] * mx + (float)im.inv[5] * my;
    }
    __syncthreads();
}

// Pixel value T * S' (area included) of a re-centred Sersic at pixel (ly, lx) of the render
// tile with origin (y0, x0); 0 where !want.  Every thread of the block calls it.
template <typename T>
__device__ T shifted_pixel(const Plan& p, int ci, const CompConst& c, const DComp& cp, const DImage& im, int y0,
                           int x0, int ly, int lx, bool want, T (*sh)[SH_H * SH_W], T* tw,
                           const double* __restrict__ tab = nullptr) {
    stage_halo<1, T>(p, ci, cp, y0, x0, sh, tw, [&](int ry, int rx, T* v) {
        const double rcx = im.aff[0] + im.aff[1] * rx + im.aff[2] * ry;
        const double rcy = im.aff[3] + im.aff[4] * rx + im.aff[5] * ry;
        if constexpr (sizeof(T) == 8) v[0] = sersic_pixel64(p, c, im, rcx, rcy, tab) * im.area;
        else v[0] = (float)((double)sersic_pixel(p, c, im, rcx, rcy) * im.area);
    });
    __syncthreads();
    const T out = want ? tap_sum(sh[0], p.shift_a, ly, lx, tw + SHIFT_NT, tw) : (T)0;
    __syncthreads();
    return out;
}

// ----------------------------------------------------------------------- render
// S (extended grid) = sum of all components whose window holds the pixel.
// SHIFT: the problem re-centres its Sersics (a separate instantiation keeps the plain
// kernels' register and LDS budgets)
template <bool SHIFT>
__global__ __launch_bounds__(256) void k_render(Plan p, int skip_mode, const apx_lm_state* lm) {
    __shared__ float sh[1][SHIFT ? SH_H * SH_W : 1];
    __shared__ float tw[SHIFT ? STAP_STRIDE : 1];
    const RTile t = p.rtiles[blockIdx.x];
    const DImage& im = p.images[t.a];
    if (sub_skipped(p, im.sub, skip_mode, lm)) return;
    const int ly = (int)threadIdx.x / RT_X, lx = (int)threadIdx.x % RT_X;
    const int y = t.y0 + ly, x = t.x0 + lx;
    const bool inside = y < im.H + im.c && x < im.W + im.c;
    const double ucx = im.aff[0] + im.aff[1] * x + im.aff[2] * y;
    const double ucy = im.aff[3] + im.aff[4] * x + im.aff[5] * y;
    double sum = 0.0;
    const int kb = p.rtile_off[blockIdx.x], ke = p.rtile_off[blockIdx.x + 1];
    for (int k = kb; k < ke; ++k) {
        const int ci = p.rtile_comps[k];
        const DComp& cp = p.comps[ci];
        const bool inbox = inside && y >= cp.box[0] && y < cp.box[2] && x >= cp.box[1] && x < cp.box[3];
        const CompConst& c = p.cc[ci];
        if (!c.valid) {
            if (inbox) sum += __builtin_nan("");
            continue;
        }
        if (SHIFT && cp.type == APX_SERSIC) {      // block-uniform
            if constexpr (SHIFT) sum += (double)shifted_pixel<float>(p, ci, c, cp, im, t.y0, t.x0, ly, lx, inbox, sh, tw);
            continue;
        }
        if (!inbox) continue;
        if (cp.type == APX_SERSIC)
            sum += (p.mode == APX_MODE_ADAPTIVE ? p.aval[adapt_index(cp, y, x)]
                                                : (double)sersic_pixel(p, c, im, ucx, ucy)) * im.area;
        else sum += (double)c.F * point_weight(c, y, x);
    }
    if (inside) p.S[im.ext_off + (long long)(y + im.c) * im.EW + (x + im.c)] = (float)sum;
}

hipError_t launch_render_mode(const Plan& p, int skip_mode, const apx_lm_state* lm, hipStream_t st) {
    if (p.n_rtiles == 0) return hipSuccess;
    if (p.shift != APX_SHIFT_NONE)
        hipLaunchKernelGGL(k_render<true>, dim3(p.n_rtiles), dim3(256), 0, st, p, skip_mode, lm);
    else
        hipLaunchKernelGGL(k_render<false>, dim3(p.n_rtiles), dim3(256), 0, st, p, skip_mode, lm);
    return hipGetLastError();
}

// ------------------------------------------------------------- FP64 render
// S64 (extended grid, FP64): the objective path's render.
template <bool SHIFT>
__global__ __launch_bounds__(256) void k_render64(Plan p, int skip_mode, const apx_lm_state* lm) {
    __shared__ double sh[1][SHIFT ? SH_H * SH_W : 1];
    __shared__ double tw[SHIFT ? STAP_STRIDE : 1];
    __shared__ double ptab[PTAB_N];
    const RTile t = p.rtiles[blockIdx.x];
    const DImage& im = p.images[t.a];
    if (sub_skipped(p, im.sub, skip_mode, lm)) return;
    stage_ptab(p, ptab);
    __syncthreads();
    const int ly = (int)threadIdx.x / RT_X, lx = (int)threadIdx.x % RT_X;
    const int y = t.y0 + ly, x = t.x0 + lx;
    const bool inside = y < im.H + im.c && x < im.W + im.c;
    const double ucx = im.aff[0] + im.aff[1] * x + im.aff[2] * y;
    const double ucy = im.aff[3] + im.aff[4] * x + im.aff[5] * y;
    double sum = 0.0;
    const int kb = p.rtile_off[blockIdx.x], ke = p.rtile_off[blockIdx.x + 1];
    for (int k = kb; k < ke; ++k) {
        const int ci = p.rtile_comps[k];
        const DComp& cp = p.comps[ci];
        const bool inbox = inside && y >= cp.box[0] && y < cp.box[2] && x >= cp.box[1] && x < cp.box[3];
        const CompConst& c = p.cc[ci];
        if (!c.valid) {
            if (inbox) sum += __builtin_nan("");
            continue;
        }
        if (SHIFT && cp.type == APX_SERSIC) {      // block-uniform
            if constexpr (SHIFT) sum += shifted_pixel<double>(p, ci, c, cp, im, t.y0, t.x0, ly, lx, inbox, sh, tw, ptab);
            continue;
        }
        if (!inbox) continue;
        if (cp.type == APX_SERSIC)
            sum += (p.mode == APX_MODE_ADAPTIVE ? p.aval[adapt_index(cp, y, x)]
                                                : sersic_pixel64(p, c, im, ucx, ucy, ptab)) * im.area;
        else sum += (double)c.F64 * point_weight(c, y, x);
    }
    if (inside) p.S64[im.ext_off + (long long)(y + im.c) * im.EW + (x + im.c)] = sum;
}

hipError_t launch_render64(const Plan& p, int skip_mode, const apx_lm_state* lm, hipStream_t st) {
    if (p.n_rtiles == 0) return hipSuccess;
    if (p.shift != APX_SHIFT_NONE)
        hipLaunchKernelGGL(k_render64<true>, dim3(p.n_rtiles), dim3(256), 0, st, p, skip_mode, lm);
    else
        hipLaunchKernelGGL(k_render64<false>, dim3(p.n_rtiles), dim3(256), 0, st, p, skip_mode, lm);
    return hipGetLastError();
}

// ------------------------------------------------------------ derivative images
// D[col] over the group's input box: the pixel-integrated derivative of each free
// parameter of each component of the group (pre-convolution).
template <bool SHIFT>
__global__ __launch_bounds__(256) void k_deriv(Plan p, const apx_lm_state* lm) {
    __shared__ float sh[5][SHIFT ? SH_H * SH_W : 1];
    __shared__ float tw[SHIFT ? STAP_STRIDE : 1];
    const RTile t = p.gtiles[blockIdx.x];
    const DGroup& gr = p.groups[t.a];
    if (lm && lm[gr.sub].need_jac == 0) return;
    const DImage& im = p.images[gr.image];
    const int ty = (int)threadIdx.x / RT_X, tx = (int)threadIdx.x % RT_X;
    const int ly = t.y0 + ty, lx = t.x0 + tx;
    const bool inside = ly < gr.ih && lx < gr.iw;
    const int y = gr.iy0 + ly, x = gr.ix0 + lx;
    const double ucx = im.aff[0] + im.aff[1] * x + im.aff[2] * y;
    const double ucy = im.aff[3] + im.aff[4] * x + im.aff[5] * y;
    const long long plane = (long long)gr.ih * gr.iw;
    float* Dg = p.D + gr.d_off + (long long)ly * gr.iw + lx;
    for (int k = gr.comp_begin; k < gr.comp_end; ++k) {
        const int ci = p.group_comps[k];
        const DComp& cp = p.comps[ci];
        const CompConst& c = p.cc[ci];
        if (SHIFT && cp.type == APX_SERSIC) {      // block-uniform
            float acc[7] = {};
            if constexpr (SHIFT)
                shifted_derivs(p, ci, c, cp, im, gr.iy0 + t.y0, gr.ix0 + t.x0, ty, tx, inside, sh, tw, acc);
            if (inside)
                for (int q = 0; q < 7; ++q)
                    if (cp.col[q] >= 0) Dg[cp.col[q] * plane] = acc[q];
            continue;
        }
        if (!inside) continue;
        if (cp.type == APX_SERSIC) {
            float acc[7];
            sersic_pixel_grad(p, c, im, cp, y, x, ucx, ucy, acc);
            const float area = (float)im.area;
            for (int q = 0; q < 7; ++q)
                if (cp.col[q] >= 0) Dg[cp.col[q] * plane] = acc[q] * area;
        } else {
            if (cp.col[2] >= 0) Dg[cp.col[2] * plane] = (float)((double)c.F * point_weight(c, y, x) * 2.302585092994046);
        }
    }
}

hipError_t launch_deriv(const Plan& p, const apx_lm_state* lm, hipStream_t st) {
    if (p.n_gtiles == 0) return hipSuccess;
    if (p.shift != APX_SHIFT_NONE)
        hipLaunchKernelGGL(k_deriv<true>, dim3(p.n_gtiles), dim3(256), 0, st, p, lm);
    else
        hipLaunchKernelGGL(k_deriv<false>, dim3(p.n_gtiles), dim3(256), 0, st, p, lm);
    return hipGetLastError();
}

// ------------------------------------------------------------- adjoint gradient
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// grad_part[col][tile] = sum over the tile of Abar * dS/dtheta_col (recomputed).
template <bool SHIFT>
__global__ __launch_bounds__(256) void k_grad_tiles(Plan p) {
    __shared__ double red[4][7];
    __shared__ float sh[5][SHIFT ? SH_H * SH_W : 1];
    __shared__ float tw[SHIFT ? STAP_STRIDE : 1];
    const RTile t = p.gtiles[blockIdx.x];
    const DGroup& gr = p.groups[t.a];
    const DImage& im = p.images[gr.image];
    const int tile_local = blockIdx.x - gr.tile_begin;
    const int ly = t.y0 + (int)threadIdx.x / RT_X;
    const int lx = t.x0 + (int)threadIdx.x % RT_X;
    const bool inside = ly < gr.ih && lx < gr.iw;
    const int y = gr.iy0 + ly, x = gr.ix0 + lx;
    const double ucx = im.aff[0] + im.aff[1] * x + im.aff[2] * y;
    const double ucy = im.aff[3] + im.aff[4] * x + im.aff[5] * y;
    float abar = 0.f;
    if (inside) abar = p.Abar[im.ext_off + (long long)(y + im.c) * im.EW + (x + im.c)];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = gr.comp_begin; k < gr.comp_end; ++k) {
        const int ci = p.group_comps[k];
        const DComp& cp = p.comps[ci];
        const CompConst& c = p.cc[ci];
        double v[7];
        if (SHIFT && cp.type == APX_SERSIC) {      // block-uniform
            float acc[7] = {};
            if constexpr (SHIFT)
                shifted_derivs(p, ci, c, cp, im, gr.iy0 + t.y0, gr.ix0 + t.x0, ly - t.y0, lx - t.x0, inside, sh, tw,
                               acc);
            for (int q = 0; q < 7; ++q) v[q] = (double)acc[q] * (double)abar;
        } else if (cp.type == APX_SERSIC) {
            float acc[7];
            if (inside) sersic_pixel_grad(p, c, im, cp, y, x, ucx, ucy, acc);
            else for (int q = 0; q < 7; ++q) acc[q] = 0.f;
            for (int q = 0; q < 7; ++q) v[q] = (double)acc[q] * im.area * (double)abar;
        } else {
            for (int q = 0; q < 7; ++q) v[q] = 0.0;
            if (inside) v[2] = (double)c.F * point_weight(c, y, x) * 2.302585092994046 * (double)abar;
        }
        for (int q = 0; q < 7; ++q) {
            if (cp.col[q] < 0) continue;            // uniform across the block
            const double s = wave_sum(v[q]);
            if (lane == 0) red[wv][q] = s;
        }
        __syncthreads();
        if (threadIdx.x < 7 && cp.col[threadIdx.x] >= 0) {
            const int q = threadIdx.x;
            const double s = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
            p.grad_part[gr.gp_off + (long long)cp.col[q] * gr.ntiles + tile_local] = s;
        }
        __syncthreads();
    }
}

hipError_t launch_grad_tiles(const Plan& p, hipStream_t st) {
    if (p.n_gtiles == 0) return hipSuccess;
    if (p.shift != APX_SHIFT_NONE)
        hipLaunchKernelGGL(k_grad_tiles<true>, dim3(p.n_gtiles), dim3(256), 0, st, p);
    else
        hipLaunchKernelGGL(k_grad_tiles<false>, dim3(p.n_gtiles), dim3(256), 0, st, p);
    return hipGetLastError();
}

// -------------------------------------------------------------- flipped PSF
__global__ void k_flip_psf(Plan p) {
    const int k = blockIdx.y;
    const DImage& im = p.images[k];
    const int P = im.P;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < P * P; e += gridDim.x * blockDim.x) {
        const int u = e / P, v = e % P;
        const float* K = im.live ? p.psf_live + im.live_off : p.psf + im.psf_off;
        p.psf_flip[im.psf_off + e] = K[(P - 1 - u) * P + (P - 1 - v)];
    }
}

// -------------------------------------------------------------- seed sums (VJP sky column)
// Block c of image k sums pixels c*256 + t + SEED_BLOCKS*256*m in FP64 (fixed order per
// thread, then waves in order); one wave per image folds the SEED_BLOCKS partials.
constexpr int SEED_BLOCKS = 64;
__global__ __launch_bounds__(256) void k_seed_part(Plan p, const float* __restrict__ seed, double* part) {
    __shared__ double red[4];
    const int k = blockIdx.y, c = blockIdx.x;
    const DImage& im = p.images[k];
    const long long npx = (long long)im.Hc * im.Wc;
    double acc = 0.0;
    for (long long e = (long long)c * 256 + threadIdx.x; e < npx; e += (long long)SEED_BLOCKS * 256)
        acc += (double)seed[im.pix_off + e];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[k * SEED_BLOCKS + c] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void k_seed_fold(Plan p, const double* __restrict__ part) {
    const int k = blockIdx.x;
    double v = part[k * SEED_BLOCKS + threadIdx.x];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x == 0) p.img_sum[3 * k + 1] = -0.5 * v;
}

hipError_t launch_seed_sums(const Plan& p, const float* seed, double* part, hipStream_t st) {
    static_assert(SEED_BLOCKS == 64, "one lane per partial in the fold");
    if (p.n_images == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed_part, dim3(SEED_BLOCKS, p.n_images), dim3(256), 0, st, p, seed, part);
    hipLaunchKernelGGL(k_seed_fold, dim3(p.n_images), dim3(64), 0, st, p, part);
    return hipGetLastError();
}

hipError_t launch_flip_psf(const Plan& p, hipStream_t st) {
    if (p.n_images == 0) return hipSuccess;
    hipLaunchKernelGGL(k_flip_psf, dim3(4, p.n_images), dim3(256), 0, st, p);
    return hipGetLastError();
}

}  // namespace apx
