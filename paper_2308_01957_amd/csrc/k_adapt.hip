// Adaptive sub-pixel integration of the Sersic components (§2.1.2: a first pass at the
// pixel centres sets an error budget from the window flux, a second pass refines only the
// pixels whose integration error would exceed it, with Gauss-Legendre quadrature of
// increasing order over progressively smaller sub-pixels).  Everything here is FP64: the
// choices are taken once per theta, stored per window pixel, and every later kernel (FP64
// and FP32 renders, derivative images, adjoint contraction) reads them, so the model and
// its derivatives always use the same rule (the derivatives are those of the chosen rule).
//
//   k_adapt_flux / k_adapt_fold  centre values of the window (stored), F = area * their
//                                 sum (ordered chunk sums), e = tol F / N
//   k_adapt_pix                  one thread per window pixel: the midpoint error estimate
//                                 area * (|I(x+1) + I(x-1) - 2 I| + |I(y+1) + I(y-1) - 2 I|)
//                                 / 24 against e (neighbours inside the window read from the
//                                 stored centre values, the same numbers); 3 x 3
//                                 Gauss-Legendre if it moves the value by at most e;
//                                 otherwise the pixel joins the refine list
//   k_adapt_refine               one workgroup per listed pixel: its 5 x 5 sub-pixels take
//                                 5 x 5 Gauss-Legendre when within e of their 3 x 3 value,
//                                 the others the mean of their 5 x 5 sub-sub-pixels at 7 x 7
//   k_adapt_refine_grad          the 7 parameter derivatives of the rule each listed pixel
//                                 took (only where derivatives are wanted)
//
// Values and derivatives are stored before the pixel-area factor.  The refine list is
// filled by an atomic counter, so its order varies between runs, but each entry's result
// depends only on its pixel: the output is bitwise reproducible.
#include "apx_internal.h"
#include "sersic64.h"

namespace apx {

constexpr int REFINE_THREADS = 256;
constexpr int N_G3 = 25 * 9, N_G5 = 25 * 25;           // phase-1 nodes: every sub-pixel at 3x3, 5x5
constexpr int N_G7 = 25 * 49;                          // nodes of one sub-pixel refined at 7x7

// pixel coordinates -> sky frame
__device__ __forceinline__ void to_sky(const DImage& im, double px, double py, double& ux, double& uy) {
    ux = im.aff[0] + im.aff[1] * px + im.aff[2] * py;
    uy = im.aff[3] + im.aff[4] * px + im.aff[5] * py;
}

__device__ __forceinline__ double prof_at(const CompConst& c, const DImage& im, double px, double py) {
    double ux, uy;
    to_sky(im, px, py, ux, uy);
    return sersic_I64(c, ux - c.x0, uy - c.y0);
}

// centre offset of sub-pixel i (0..4) along one axis of a unit square
__device__ __forceinline__ double sub_off(int i) { return (i + 0.5) * 0.2 - 0.5; }

__global__ void k_adapt_reset(Plan p) {
    if (threadIdx.x == 0) p.acount[0] = 0;
}

__device__ __forceinline__ bool chunk_active(const Plan& p, const AChunk& ch, int skip_mode, const apx_lm_state* lm) {
    const DComp& cp = p.comps[ch.comp];
    return !sub_skipped(p, cp.sub, skip_mode, lm) && p.cc[ch.comp].valid;
}

// apart[chunk] = sum of the centre values of the chunk's pixels (fixed order).
__global__ __launch_bounds__(ADAPT_CHUNK) void k_adapt_flux(Plan p, int skip_mode, const apx_lm_state* lm) {
    __shared__ double red[ADAPT_CHUNK / 64];
    const AChunk ch = p.achunks[blockIdx.x];
    if (!chunk_active(p, ch, skip_mode, lm)) return;
    const DComp& cp = p.comps[ch.comp];
    const CompConst& c = p.cc[ch.comp];
    const DImage& im = p.images[cp.image];
    const int bw = cp.box[3] - cp.box[1];
    const int npx = (cp.box[2] - cp.box[0]) * bw;
    const int e = ch.start + (int)threadIdx.x;
    double v = 0.0;
    if (e < npx) {
        v = prof_at(c, im, (double)(cp.box[1] + e % bw), (double)(cp.box[0] + e / bw));
        p.av0[cp.aoff + e] = v;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0];
        for (int w = 1; w < ADAPT_CHUNK / 64; ++w) s += red[w];
        p.apart[blockIdx.x] = s;
    }
}

// One wave per component: ae[comp] = tol * area * (sum of its chunk partials) / N.
__global__ __launch_bounds__(64) void k_adapt_fold(Plan p, int skip_mode, const apx_lm_state* lm) {
    const int ci = blockIdx.x;
    const int cb = p.acomp_chunk[ci], ce = p.acomp_chunk[ci + 1];
    if (cb == ce) return;
    if (!chunk_active(p, AChunk{ci, 0}, skip_mode, lm)) return;
    const DComp& cp = p.comps[ci];
    double s = 0.0;
    for (int k = cb + (int)threadIdx.x; k < ce; k += 64) s += p.apart[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) {
        const double N = (double)(cp.box[2] - cp.box[0]) * (double)(cp.box[3] - cp.box[1]);
        const double F = p.images[cp.image].area * s;
        p.ae[ci] = p.k_re * F / N;
    }
}

// One thread per window pixel: centre or 3 x 3 value and its choice, or a refine entry.
__global__ __launch_bounds__(ADAPT_CHUNK) void k_adapt_pix(Plan p, int skip_mode, const apx_lm_state* lm) {
    const AChunk ch = p.achunks[blockIdx.x];
    const DComp& cp = p.comps[ch.comp];
    if (sub_skipped(p, cp.sub, skip_mode, lm)) return;
    const CompConst& c = p.cc[ch.comp];
    const DImage& im = p.images[cp.image];
    const int bw = cp.box[3] - cp.box[1];
    const int npx = (cp.box[2] - cp.box[0]) * bw;
    const int e = ch.start + (int)threadIdx.x;
    if (e >= npx) return;
    if (!c.valid) {                       // outside the domain (reported by k_prep)
        p.aval[cp.aoff + e] = __builtin_nan("");
        p.acode[cp.aoff + e] = 0;
        return;
    }
    const int ix = e % bw, iy = e / bw, bh = cp.box[2] - cp.box[0];
    const double x = (double)(cp.box[1] + ix), y = (double)(cp.box[0] + iy);
    const double area = im.area, budget = p.ae[ch.comp];
    const long long gi = cp.aoff + e;
    const double* c0 = p.av0 + gi;
    const double v0 = c0[0];
    const double xp1 = ix + 1 < bw ? c0[1] : prof_at(c, im, x + 1.0, y);
    const double xm1 = ix > 0 ? c0[-1] : prof_at(c, im, x - 1.0, y);
    const double yp1 = iy + 1 < bh ? c0[bw] : prof_at(c, im, x, y + 1.0);
    const double ym1 = iy > 0 ? c0[-bw] : prof_at(c, im, x, y - 1.0);
    const double est = area * (fabs(xp1 + xm1 - 2.0 * v0) + fabs(yp1 + ym1 - 2.0 * v0)) / 24.0;
    if (est <= budget) {
        p.aval[gi] = v0;
        p.acode[gi] = 0;
        return;
    }
    const double* o3 = p.agl;
    const double* w3 = p.agl + 3;
    double v1 = 0.0;
    for (int ky = 0; ky < 3; ++ky)
        for (int kx = 0; kx < 3; ++kx) v1 += (w3[ky] * w3[kx]) * prof_at(c, im, x + o3[kx], y + o3[ky]);
    if (area * fabs(v1 - v0) <= budget) {
        p.aval[gi] = v1;
        p.acode[gi] = 1;
        return;
    }
    const int r = atomicAdd(p.acount, 1);
    p.aref[r] = ARef{ch.comp, e};
    p.acode[gi] = -1 - r;
}

// Fixed-order sum over the workgroup (result valid in thread 0).
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
    for (int w = 1; w < REFINE_THREADS / 64; ++w) s += red[w];
    return s;
}

// Position (pixel coordinates) of node q of the refined sub-pixels: nq = index into the
// list of 7x7-refined sub-pixels, then sub-sub-pixel m and node (kx, ky).
__device__ __forceinline__ void node7(const Plan& p, const int* need_list, double x, double y, int q,
                                      double& px, double& py, double& wgt) {
    const int j = need_list[q / N_G7], rem = q % N_G7, m = rem / 49, k = rem % 49;
    const double* o7 = p.agl + 16;
    const double* w7 = p.agl + 23;
    px = x + sub_off(j % 5) + 0.2 * sub_off(m % 5) + 0.04 * o7[k % 7];
    py = y + sub_off(j / 5) + 0.2 * sub_off(m / 5) + 0.04 * o7[k / 7];
    wgt = (w7[k % 7] * w7[k / 7]) * 0.04;              // sub-sub-pixel mean over 25
}

__global__ __launch_bounds__(REFINE_THREADS) void k_adapt_refine(Plan p) {
    __shared__ double nv[N_G3 + N_G5];
    __shared__ double g5s[25];
    __shared__ int need_list[25];
    __shared__ int flags[25];
    __shared__ int n_need;
    __shared__ double red[REFINE_THREADS / 64];
    const int t = threadIdx.x;
    const int count = p.acount[0];
    const double* o3 = p.agl;
    const double* w3 = p.agl + 3;
    const double* o5 = p.agl + 6;
    const double* w5 = p.agl + 11;
    for (int r = blockIdx.x; r < count; r += gridDim.x) {
        const ARef ar = p.aref[r];
        const DComp& cp = p.comps[ar.comp];
        const CompConst& c = p.cc[ar.comp];
        const DImage& im = p.images[cp.image];
        const int bw = cp.box[3] - cp.box[1];
        const double x = (double)(cp.box[1] + ar.idx % bw), y = (double)(cp.box[0] + ar.idx / bw);
        const double area = im.area, budget = p.ae[ar.comp];
        // phase 1: every sub-pixel at 3 x 3 and 5 x 5
        for (int n = t; n < N_G3 + N_G5; n += REFINE_THREADS) {
            int j, kx, ky;
            const double *o, *w;
            if (n < N_G3) {
                j = n / 9; kx = (n % 9) % 3; ky = (n % 9) / 3; o = o3; w = w3;
            } else {
                const int m = n - N_G3;
                j = m / 25; kx = (m % 25) % 5; ky = (m % 25) / 5; o = o5; w = w5;
            }
            const double px = x + sub_off(j % 5) + 0.2 * o[kx], py = y + sub_off(j / 5) + 0.2 * o[ky];
            nv[n] = (w[ky] * w[kx]) * prof_at(c, im, px, py);
        }
        __syncthreads();
        if (t < 25) {
            double g3 = 0.0, g5 = 0.0;
            for (int k = 0; k < 9; ++k) g3 += nv[t * 9 + k];
            for (int k = 0; k < 25; ++k) g5 += nv[N_G3 + t * 25 + k];
            g5s[t] = g5;
            flags[t] = area * fabs(g5 - g3) <= budget ? 0 : 1;
        }
        __syncthreads();
        if (t == 0) {
            int k = 0, mask = 0;
            for (int j = 0; j < 25; ++j)
                if (flags[j]) {
                    need_list[k++] = j;
                    mask |= 1 << j;
                }
            n_need = k;
            p.aneed[r] = mask;
        }
        __syncthreads();
        const int T7 = n_need * N_G7;
        // phase 2: value = mean over the sub-pixels of (5 x 5 value or 7 x 7 sub-sub mean)
        double v = 0.0;
        for (int q = t; q < T7; q += REFINE_THREADS) {
            double px, py, wgt;
            node7(p, need_list, x, y, q, px, py, wgt);
            v += wgt * prof_at(c, im, px, py);
        }
        const double s7 = block_sum(v, red);
        if (t == 0) {
            double s5 = 0.0;
            for (int j = 0; j < 25; ++j)
                if (!flags[j]) s5 += g5s[j];
            p.aval[cp.aoff + ar.idx] = (s5 + s7) / 25.0;
        }
        __syncthreads();                    // LDS reuse by the next entry
    }
}

// The derivatives of the rule each listed pixel took: 7 x 7 nodes of its refined
// sub-pixels, 5 x 5 nodes of the others, all in one strided node range.
__global__ __launch_bounds__(REFINE_THREADS) void k_adapt_refine_grad(Plan p) {
    __shared__ int need_list[25], keep_list[25];
    __shared__ int n_need;
    __shared__ double red[REFINE_THREADS / 64][7];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int count = p.acount[0];
    const double* o5 = p.agl + 6;
    const double* w5 = p.agl + 11;
    for (int r = blockIdx.x; r < count; r += gridDim.x) {
        const ARef ar = p.aref[r];
        const DComp& cp = p.comps[ar.comp];
        const CompConst& c = p.cc[ar.comp];
        const DImage& im = p.images[cp.image];
        const int bw = cp.box[3] - cp.box[1];
        const double x = (double)(cp.box[1] + ar.idx % bw), y = (double)(cp.box[0] + ar.idx / bw);
        if (t == 0) {
            const int mask = p.aneed[r];
            int a = 0, b = 0;
            for (int j = 0; j < 25; ++j) {
                if ((mask >> j) & 1) need_list[a++] = j;
                else keep_list[b++] = j;
            }
            n_need = a;
        }
        __syncthreads();
        const int T7 = n_need * N_G7, T = T7 + (25 - n_need) * 25;
        double acc[7] = {0, 0, 0, 0, 0, 0, 0}, vv = 0.0;
        for (int q = t; q < T; q += REFINE_THREADS) {
            double px, py, wgt, ux, uy;
            if (q < T7) {
                node7(p, need_list, x, y, q, px, py, wgt);
            } else {
                const int j = keep_list[(q - T7) / 25], k = (q - T7) % 25;
                px = x + sub_off(j % 5) + 0.2 * o5[k % 5];
                py = y + sub_off(j / 5) + 0.2 * o5[k / 5];
                wgt = w5[k % 5] * w5[k / 5];
            }
            to_sky(im, px, py, ux, uy);
            sersic_dI64(c, ux - c.x0, uy - c.y0, wgt, vv, acc);
        }
        for (int k = 0; k < 7; ++k) {
            double s = acc[k];
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (lane == 0) red[wv][k] = s;
        }
        __syncthreads();
        if (t < 7) {
            double s = red[0][t];
            for (int w = 1; w < REFINE_THREADS / 64; ++w) s += red[w][t];
            p.adval[7LL * r + t] = (float)(s / 25.0);
        }
        __syncthreads();                    // LDS reuse by the next entry
    }
}

hipError_t launch_adapt(const Plan& p, int skip_mode, const apx_lm_state* lm, int want_grad, hipStream_t st) {
    if (p.n_achunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adapt_reset, dim3(1), dim3(64), 0, st, p);
    hipLaunchKernelGGL(k_adapt_flux, dim3(p.n_achunks), dim3(ADAPT_CHUNK), 0, st, p, skip_mode, lm);
    hipLaunchKernelGGL(k_adapt_fold, dim3(p.n_comps), dim3(64), 0, st, p, skip_mode, lm);
    hipLaunchKernelGGL(k_adapt_pix, dim3(p.n_achunks), dim3(ADAPT_CHUNK), 0, st, p, skip_mode, lm);
    const long long g = p.n_apix < 4096 ? p.n_apix : 4096;
    hipLaunchKernelGGL(k_adapt_refine, dim3((unsigned)g), dim3(REFINE_THREADS), 0, st, p);
    if (want_grad) hipLaunchKernelGGL(k_adapt_refine_grad, dim3((unsigned)g), dim3(REFINE_THREADS), 0, st, p);
    return hipGetLastError();
}

}  // namespace apx
