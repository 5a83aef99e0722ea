// Direct-mode PSF convolution (§2.1.3) for gfx950.
//
// out(y, x) = sum_{U,V} K[U][V] * in(y - U + c, x - V + c), in = 0 outside its rectangle.
//
// One workgroup owns a TH x TW output tile (TH * TW / CV_R threads).  The input tile with its
// (P-1) halo is staged once into LDS; each lane then produces CV_R consecutive outputs
// of one row: per PSF row it loads a CV_R + P - 1 register window from LDS (ds_read_b128)
// and runs P x CV_R FMAs whose PSF operand is wave-uniform (scalar loads, then copied to
// a VGPR), so the VALU does useful FMAs at ~CV_R*P per (CV_R+P-1)/4 LDS instructions.  Each PSF row is summed
// into a fresh partial before being added to the accumulator (error ~2P ulp, not P^2).
//
// On an image whose PSF has a higher resolution than its pixels the grid is of sub-pixels,
// and the model and Jacobian epilogues first sum each pixel's sub-pixel outputs.
//
// Epilogues (template KIND):
//   CONV_FWD  model + sky, optional model store, FP32 residual store, FP64 partials of
//             sum w r^2, sum w r, sum w (chi^2 of Eq. chi2, sky gradient, sky-sky entry);
//   CONV_JCOL Jacobian column store, FP64 partials of sum w r J, sum w J (only for jobs
//             without gram_part: the 4 x 4-block Gram kernel forms them for the others);
//   CONV_ADJ  input is -2 w r staged from the residual (the adjoint seed of chi^2), or a
//             given seed (vector-Jacobian product of the render), PSF flipped,
//             output is dchi2/dS on the extended grid.
#pragma once
#include <type_traits>

#include "apx_internal.h"

namespace apx {

// Sum of each run of UU consecutive entries into the first CV_R / UU entries.
template <int UU, typename T>
__device__ __forceinline__ void bin_lane(T (&acc)[CV_R]) {
#pragma unroll
    for (int q = 0; q < CV_R / UU; ++q) {
        T v = acc[q * UU];
#pragma unroll
        for (int i = 1; i < UU; ++i) v += acc[q * UU + i];
        acc[q] = v;
    }
}

__device__ __forceinline__ double conv_wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// T is the arithmetic type of the staged input and the accumulators: float for the
// Jacobian and adjoint passes, double for the FP64 objective.
template <int P, int KIND, typename T, int TH, int TW>
__global__ __launch_bounds__(TH * TW / CV_R) void k_conv(Plan p, const ConvJob* __restrict__ jobs,
                                                         const ConvItem* __restrict__ items, int item_begin,
                                                         ConvIO io) {
    constexpr int c = (P - 1) / 2;
    constexpr int NT = TH * TW / CV_R;              // threads
    constexpr int LPR = TW / CV_R;                  // lanes per output row
    constexpr int NW = NT / 64;                     // waves
    static_assert(NW >= 1 && NT % 64 == 0, "whole waves");
    constexpr int LH = TH + P - 1;
    constexpr int LW0 = TW + P - 1;
    constexpr int LW = (LW0 + 3) & ~3;
    __shared__ __attribute__((aligned(16))) T tile[LH * LW];
    __shared__ double red[NW][3];

    const int item_idx = item_begin + xcd_chunk_item((int)blockIdx.x, (int)gridDim.x);
    const ConvItem it = items[item_idx];
    const ConvJob jb = jobs[it.job];
    const DImage& im = p.images[jb.image];
    if (io.skip_mode == 1) {
        if (p.lmf[im.sub].chol_done == 0 || p.lmf[im.sub].trial_bad != 0) return;
    } else if (io.skip_mode == 2) {
        if (io.lm[im.sub].need_jac == 0) return;
    }
    const int oy0 = jb.out_y0 + it.ty * TH;
    const int ox0 = jb.out_x0 + it.tx * TW;
    const int iy_base = oy0 - c, ix_base = ox0 - c;

    // ---- stage the input tile (zero outside the input rectangle); every load of a thread
    // is issued before its LDS stores so the latencies overlap
    constexpr int NE = (LH * LW0 + NT - 1) / NT;
    T v[NE];
    if constexpr (KIND == CONV_ADJ) {
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = threadIdx.x + NT * q;
            const int ly = e / LW0, lx = e - ly * LW0;
            const int y = iy_base + ly, x = ix_base + lx;
            T val = 0;
            if (e < LH * LW0 && y >= 0 && y < im.H && x >= 0 && x < im.W) {
                // a pixel's seed reaches each of its sub-pixels (the adjoint of their sum)
                const long long pix = im.pix_off + (long long)(y / im.up) * im.Wc + x / im.up;
                val = io.seed ? io.seed[pix] : -2.f * io.weight[pix] * p.rbuf[pix];
            }
            v[q] = val;
        }
    } else {
        const T* __restrict__ in;
        if constexpr (sizeof(T) == 8) in = io.in64 + jb.in_off + (long long)it.ch * jb.in_cs;
        else in = (jb.in_src ? io.in_s : io.in) + jb.in_off + (long long)it.ch * jb.in_cs;
        const int iy1 = jb.in_y0 + jb.in_h, ix1 = jb.in_x0 + jb.in_w;
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = threadIdx.x + NT * q;
            const int ly = e / LW0, lx = e - ly * LW0;
            const int y = iy_base + ly, x = ix_base + lx;
            T val = 0;
            if (e < LH * LW0 && y >= jb.in_y0 && y < iy1 && x >= jb.in_x0 && x < ix1)
                val = in[(long long)(y - jb.in_y0) * jb.in_w + (x - jb.in_x0)];
            v[q] = val;
        }
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = threadIdx.x + NT * q;
        if (e < LH * LW0) {
            const int ly = e / LW0, lx = e - ly * LW0;
            tile[ly * LW + lx] = v[q];
        }
    }
    __syncthreads();

    // ---- register-window convolution
    const int ty = (int)threadIdx.x / LPR, tx = (int)threadIdx.x % LPR;
    // the stamp: FP64 copies for the FP64 objective; the flipped stamp for the adjoint;
    // on a live-PSF image the rendered stamp, or for its PSF columns a derivative stamp
    using KT = typename std::conditional<sizeof(T) == 8, double, float>::type;
    const KT* __restrict__ K;
    if constexpr (sizeof(T) == 8) K = p.psf64 + im.psf_off;
    else if constexpr (KIND == CONV_ADJ) K = p.psf_flip + im.psf_off;
    else K = im.live ? p.psf_live + im.live_off + (long long)jb.kslot[it.ch < 1 ? 0 : 1] * P * P
                     : p.psf + im.psf_off;
    T acc[CV_R];
#pragma unroll
    for (int r = 0; r < CV_R; ++r) acc[r] = 0;
    for (int U = 0; U < P; ++U) {
        const T* row = tile + (ty + P - 1 - U) * LW + tx * CV_R;
        T s[CV_R + P - 1];
#pragma unroll
        for (int k = 0; k < CV_R + P - 1; ++k) s[k] = row[k];
        T part[CV_R];
#pragma unroll
        for (int r = 0; r < CV_R; ++r) part[r] = 0;
#pragma unroll
        for (int V = 0; V < P; ++V) {
            T kv = (T)K[U * P + V];
            // FP32: the PSF value (scalar load) moves from its SGPR into a VGPR, one v_mov
            // per CV_R FMAs: gfx950 issues FMAs of VGPR operands from two waves at once,
            // FMAs that read an SGPR one at a time (measured 124 vs 76 TFLOP/s)
            if constexpr (sizeof(T) == 4) {
                T kvv;
                asm("v_mov_b32 %0, %1" : "=v"(kvv) : "s"(kv));
                kv = kvv;
            }
#pragma unroll
            for (int r = 0; r < CV_R; ++r) part[r] = fma(kv, s[r + P - 1 - V], part[r]);
        }
#pragma unroll
        for (int r = 0; r < CV_R; ++r) acc[r] += part[r];
    }

    // ---- epilogue
    const int y = oy0 + ty;
    const int xb = ox0 + tx * CV_R;
    const int xend = jb.out_x0 + jb.out_w;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // Sub-pixel grids (up = U > 1, a power of two <= CV_R): sum each pixel's U x U outputs,
    // U consecutive ones in a lane, then across the lanes of rows ty ^ 1 .. ty ^ (U - 1)
    // (one wave holds 64 / LPR >= 8 rows; tiles and output boxes are whole pixels).  Lane
    // rows with ty % U == 0 then hold CV_R / U pixel values each.
    const int up = im.up;
    if (KIND != CONV_ADJ && up > 1) {
        if (up == 2) bin_lane<2>(acc);
        else if (up == 4) bin_lane<4>(acc);
        else bin_lane<8>(acc);
        for (int k = 1; k < up; k <<= 1)
#pragma unroll
            for (int r = 0; r < CV_R; ++r) acc[r] += __shfl_xor(acc[r], k * LPR, 64);
    }
    const int nq = KIND == CONV_ADJ ? CV_R : CV_R / up;         // values per lane
    const int sx = KIND == CONV_ADJ ? 1 : up;                   // render-grid step between them
    const bool yok = y < jb.out_y0 + jb.out_h && (KIND == CONV_ADJ || (ty & (up - 1)) == 0);
    const int yc = KIND == CONV_ADJ ? y : y / up;               // image pixel row
    if constexpr (KIND == CONV_FWD) {
        const T sky = (T)p.sky_val[jb.image];
        double c2 = 0.0, swr = 0.0, sw = 0.0;
        if (yok) {
            const long long rowpix = im.pix_off + (long long)yc * im.Wc;
            // the row's weights and data first: their loads overlap instead of following
            // one another
            float wv[CV_R], dv[CV_R];
#pragma unroll
            for (int r = 0; r < CV_R; ++r) {
                const int x = xb + r * sx;
                wv[r] = dv[r] = 0.f;
                if (io.data && r < nq && x < xend) {
                    wv[r] = io.weight[rowpix + x / up];
                    dv[r] = io.data[rowpix + x / up];
                }
            }
#pragma unroll
            for (int r = 0; r < CV_R; ++r) {
                const int x = xb + r * sx;
                if (r < nq && x < xend) {
                    const T m = acc[r] + sky;
                    const long long pix = rowpix + x / up;
                    if (io.out) io.out[pix] = (float)m;
                    if (io.data) {
                        const double w = (double)wv[r];
                        const double rr = (double)dv[r] - (double)m;
                        c2 += w * rr * rr;
                        swr += w * rr;
                        sw += w;
                        p.rbuf[pix] = (float)rr;
                    }
                }
            }
        }
        if (io.data) {
            c2 = conv_wave_sum(c2);
            swr = conv_wave_sum(swr);
            sw = conv_wave_sum(sw);
            if (lane == 0) { red[wv][0] = c2; red[wv][1] = swr; red[wv][2] = sw; }
            __syncthreads();
            if (threadIdx.x < 3) {
                const int q = threadIdx.x;
                double sum = red[0][q];
#pragma unroll
                for (int w = 1; w < NW; ++w) sum += red[w][q];
                io.part[(long long)item_idx * 3 + q] = sum;
            }
        }
    } else if constexpr (KIND == CONV_JCOL) {
        float* __restrict__ out = io.out + jb.out_off + (long long)it.ch * jb.out_cs;
        double s1 = 0.0, s2 = 0.0;
        const bool epart = io.weight && !jb.gram_part;       // sum w r J and sum w J here
        if (yok) {
            // the column's plane is stored on the image pixels of the output box
            const int ow = jb.out_w / up;
            const long long orow = (long long)(yc - jb.out_y0 / up) * ow - jb.out_x0 / up;
            const long long rowpix = im.pix_off + (long long)yc * im.Wc;
            float wv[CV_R], rv[CV_R];                   // loads first, as above
#pragma unroll
            for (int r = 0; r < CV_R; ++r) {
                const int x = xb + r * sx;
                wv[r] = rv[r] = 0.f;
                if (epart && r < nq && x < xend) {
                    wv[r] = io.weight[rowpix + x / up];
                    rv[r] = p.rbuf[rowpix + x / up];
                }
            }
#pragma unroll
            for (int r = 0; r < CV_R; ++r) {
                const int x = xb + r * sx;
                if (r < nq && x < xend) {
                    const int xc = x / up;
                    out[orow + xc] = acc[r];
                    if (epart) {
                        const double wj = (double)wv[r] * (double)acc[r];
                        s1 += wj * (double)rv[r];
                        s2 += wj;
                    }
                }
            }
        }
        if (epart) {
            s1 = conv_wave_sum(s1);
            s2 = conv_wave_sum(s2);
            if (lane == 0) { red[wv][0] = s1; red[wv][1] = s2; }
            __syncthreads();
            if (threadIdx.x < 2) {
                const int q = threadIdx.x;
                double sum = red[0][q];
#pragma unroll
                for (int w = 1; w < NW; ++w) sum += red[w][q];
                io.part[(long long)item_idx * 2 + q] = sum;
            }
        }
    } else {
        float* __restrict__ out = io.out + jb.out_off;
        if (yok) {
            const long long orow = (long long)(y - jb.out_y0) * jb.out_w - jb.out_x0;
#pragma unroll
            for (int r = 0; r < CV_R; ++r) {
                const int x = xb + r;
                if (x < xend) out[orow + x] = acc[r];
            }
        }
    }
}

// Jacobian-column convolution with a rank-one stamp K_UV = a_U b_V (jobs of shape
// SHAPE_SEP) as two 1-D passes over an SEP_TH x SEP_TW output tile, 256 threads: the input
// tile with its P - 1 halo is staged in LDS as for the 2-D kernel; the row pass convolves
// every staged row with b into a second LDS buffer (the tile rows plus the vertical halo);
// the column pass convolves that with a, each lane making CV_R consecutive outputs of one
// column, and the epilogue is that of the 2-D kernel's JCOL (column store, and the FP64
// partials of sum w r J and sum w J per item unless the job's gram_part is set).  2 (P + P (TH + P - 1) / TH) multiply-adds per output
// instead of 2 P^2.
template <int P>
__global__ __launch_bounds__(256) void k_conv_sep(Plan p, const ConvJob* __restrict__ jobs,
                                                  const ConvItem* __restrict__ items, int item_begin,
                                                  ConvIO io) {
    constexpr int TH = SEP_TH, TW = SEP_TW, NT = 256;
    constexpr int c = (P - 1) / 2;
    constexpr int LPR = TW / CV_R;                  // lanes per output row
    constexpr int NW = NT / 64;
    static_assert(TH * TW / CV_R == NT && TH == CV_R * (NT / TW), "one lane per CV_R outputs of a column");
    constexpr int LH = TH + P - 1;
    constexpr int LW0 = TW + P - 1;
    constexpr int LW = (LW0 + 3) & ~3;
    __shared__ __attribute__((aligned(16))) float tile[LH * LW];
    __shared__ __attribute__((aligned(16))) float hb[LH * TW];
    __shared__ double red[NW][2];

    const int item_idx = item_begin + xcd_chunk_item((int)blockIdx.x, (int)gridDim.x);
    const ConvItem it = items[item_idx];
    const ConvJob jb = jobs[it.job];
    const DImage& im = p.images[jb.image];
    if (io.skip_mode == 1) {
        if (p.lmf[im.sub].chol_done == 0 || p.lmf[im.sub].trial_bad != 0) return;
    } else if (io.skip_mode == 2) {
        if (io.lm[im.sub].need_jac == 0) return;
    }
    const int oy0 = jb.out_y0 + it.ty * TH;
    const int ox0 = jb.out_x0 + it.tx * TW;
    const int iy_base = oy0 - c, ix_base = ox0 - c;

    // ---- stage the input tile (zero outside the input rectangle)
    constexpr int NE = (LH * LW0 + NT - 1) / NT;
    {
        const float* __restrict__ in = (jb.in_src ? io.in_s : io.in) + jb.in_off + (long long)it.ch * jb.in_cs;
        const int iy1 = jb.in_y0 + jb.in_h, ix1 = jb.in_x0 + jb.in_w;
        float v[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = threadIdx.x + NT * q;
            const int ly = e / LW0, lx = e - ly * LW0;
            const int y = iy_base + ly, x = ix_base + lx;
            float val = 0.f;
            if (e < LH * LW0 && y >= jb.in_y0 && y < iy1 && x >= jb.in_x0 && x < ix1)
                val = in[(long long)(y - jb.in_y0) * jb.in_w + (x - jb.in_x0)];
            v[q] = val;
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = threadIdx.x + NT * q;
            if (e < LH * LW0) {
                const int ly = e / LW0, lx = e - ly * LW0;
                tile[ly * LW + lx] = v[q];
            }
        }
    }
    __syncthreads();

    const float* __restrict__ fa = p.psf_sep + im.sep_off;       // a_U (rows)
    const float* __restrict__ fb = fa + P;                       // b_V (columns)
    // ---- row pass: hb[r][x] = sum_V b_V tile[r][x + P - 1 - V], r < LH, x < TW
    for (int task = (int)threadIdx.x; task < LH * LPR; task += NT) {
        const int r = task / LPR, g = task - r * LPR;
        const float* row = tile + r * LW + g * CV_R;
        float sw[CV_R + P - 1];
#pragma unroll
        for (int k = 0; k < CV_R + P - 1; ++k) sw[k] = row[k];
        float part[CV_R];
#pragma unroll
        for (int q = 0; q < CV_R; ++q) part[q] = 0.f;
#pragma unroll
        for (int V = 0; V < P; ++V) {
            // the factor (a scalar load) moves into a VGPR, one v_mov per CV_R FMAs, so that
            // the FMAs of two waves issue together (as in the 2-D kernel)
            float kv;
            asm("v_mov_b32 %0, %1" : "=v"(kv) : "s"(fb[V]));
#pragma unroll
            for (int q = 0; q < CV_R; ++q) part[q] = fmaf(kv, sw[q + P - 1 - V], part[q]);
        }
#pragma unroll
        for (int q = 0; q < CV_R; ++q) hb[r * TW + g * CV_R + q] = part[q];
    }
    __syncthreads();

    // ---- column pass: out[y][x] = sum_U a_U hb[y + P - 1 - U][x]; each lane makes CV_R
    // consecutive outputs of one column from a register window down that column (lanes of
    // a wave take consecutive columns: conflict-free LDS reads, coalesced stores)
    const int cx = (int)threadIdx.x % TW, rb = (int)threadIdx.x / TW;      // column, row block
    float acc[CV_R];
    {
        float sw[CV_R + P - 1];
#pragma unroll
        for (int k = 0; k < CV_R + P - 1; ++k) sw[k] = hb[(rb * CV_R + k) * TW + cx];
#pragma unroll
        for (int q = 0; q < CV_R; ++q) acc[q] = 0.f;
#pragma unroll
        for (int U = 0; U < P; ++U) {
            float ka;
            asm("v_mov_b32 %0, %1" : "=v"(ka) : "s"(fa[U]));
#pragma unroll
            for (int q = 0; q < CV_R; ++q) acc[q] = fmaf(ka, sw[q + P - 1 - U], acc[q]);
        }
    }

    // ---- epilogue (the JCOL epilogue of the 2-D kernel on a pixel grid)
    const int x = ox0 + cx;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float* __restrict__ out = io.out + jb.out_off + (long long)it.ch * jb.out_cs;
    double s1 = 0.0, s2 = 0.0;
    const bool epart = io.weight && !jb.gram_part;           // sum w r J and sum w J here
    if (x < jb.out_x0 + jb.out_w) {
        // the column's weights and residuals first: their loads overlap instead of following
        // one another
        float wv[CV_R], rv[CV_R];
#pragma unroll
        for (int q = 0; q < CV_R; ++q) {
            const int y = oy0 + rb * CV_R + q;
            wv[q] = rv[q] = 0.f;
            if (epart && y < jb.out_y0 + jb.out_h) {
                const long long pix = im.pix_off + (long long)y * im.Wc + x;
                wv[q] = io.weight[pix];
                rv[q] = p.rbuf[pix];
            }
        }
#pragma unroll
        for (int q = 0; q < CV_R; ++q) {
            const int y = oy0 + rb * CV_R + q;
            if (y < jb.out_y0 + jb.out_h) {
                out[(long long)(y - jb.out_y0) * jb.out_w + (x - jb.out_x0)] = acc[q];
                if (epart) {
                    const double wj = (double)wv[q] * (double)acc[q];
                    s1 += wj * (double)rv[q];
                    s2 += wj;
                }
            }
        }
    }
    if (epart) {
        s1 = conv_wave_sum(s1);
        s2 = conv_wave_sum(s2);
        if (lane == 0) { red[wv][0] = s1; red[wv][1] = s2; }
        __syncthreads();
        if (threadIdx.x < 2) {
            const int q = threadIdx.x;
            double sum = red[0][q];
#pragma unroll
            for (int w = 1; w < NW; ++w) sum += red[w][q];
            io.part[(long long)item_idx * 2 + q] = sum;
        }
    }
}

#define APX_FOR_EACH_P(X)                                                                     \
    X(1) X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) X(27) X(29)     \
    X(31) X(33) X(35) X(37) X(39) X(41) X(43) X(45) X(47) X(49) X(51) X(53) X(55) X(57)      \
    X(59) X(61) X(63)

template <int KIND, typename T, int TH, int TW>
hipError_t launch_conv_shape(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    dim3 grid(L.item_count), block(TH * TW / CV_R);
    switch (L.P) {
#define APX_CASE(PP)                                                                         \
    case PP:                                                                                 \
        hipLaunchKernelGGL((k_conv<PP, KIND, T, TH, TW>), grid, block, 0, st, p, L.jobs,     \
                           L.items, L.item_begin, io);                                      \
        break;
        APX_FOR_EACH_P(APX_CASE)
#undef APX_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

inline hipError_t launch_conv_sep_impl(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    if (L.item_count <= 0) return hipSuccess;
    dim3 grid(L.item_count), block(256);
    switch (L.P) {
#define APX_CASE(PP)                                                                                   \
    case PP:                                                                                           \
        hipLaunchKernelGGL((k_conv_sep<PP>), grid, block, 0, st, p, L.jobs, L.items, L.item_begin, io); \
        break;
        APX_FOR_EACH_P(APX_CASE)
#undef APX_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KIND, typename T = float>
hipError_t launch_conv_kind(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    if (L.item_count <= 0) return hipSuccess;
    static_assert(N_TILE_SHAPES == 4, "one case per tile shape");
    switch (L.shape) {
        case 0: return launch_conv_shape<KIND, T, tile_th(0), tile_tw(0)>(p, L, io, st);
        case 1: return launch_conv_shape<KIND, T, tile_th(1), tile_tw(1)>(p, L, io, st);
        case 2: return launch_conv_shape<KIND, T, tile_th(2), tile_tw(2)>(p, L, io, st);
        case 3: return launch_conv_shape<KIND, T, tile_th(3), tile_tw(3)>(p, L, io, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace apx
