// FFT-mode PSF convolution (§2.1.3: besides direct convolution the paper offers an FFT mode
// for large PSFs).  Overlap-save on 128 x 128 tiles held in LDS: a workgroup stages a
// 128 x 128 input tile (zero outside the input rectangle), takes its 2-D FFT, multiplies
// by the stamp's spectrum (computed once per stamp and theta), transforms back and keeps
// the (129 - P)^2 outputs that the circular wrap does not touch.  Two output blocks that
// use the same stamp ride in one complex transform (one in the real part, one in the
// imaginary part: the stamp is real, so the two convolutions separate exactly).
//
// The 128-point transforms run as 16 x 8 Cooley-Tukey: a 16-point DFT in registers per
// stride-8 subsequence, the 128th-root twiddles, then an 8-point DFT in registers; rows,
// then columns, with LDS rows padded by one element.  The inverse uses conj(FFT(conj(.))).
// FP32 throughout (the objective's FP64 convolution stays direct); the error is a few ulp
// of the tile's largest values times log2 of the transform size.
//
// Same epilogues as the direct kernel: model + chi^2 partials (FP32 objective), Jacobian
// columns (+ partials unless the job's gram_part is set), adjoint.  Images with a higher-resolution PSF (a sub-pixel render
// grid) are never planned here, so the render grid is the pixel grid.
#include "apx_internal.h"

namespace apx {

constexpr int FT = FFT_T;                 // 128
constexpr int FTP = FT + 1;               // padded LDS row
constexpr int FFT_THREADS = 1024;
constexpr int EPI_B = 4;                  // epilogue elements per thread whose loads go out together
static_assert(FT == 128, "the 16 x 8 decomposition below is for 128-point transforms");

struct cf { float x, y; };
__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// exp(-2 pi i m / 16), m = 0..15
__device__ __forceinline__ cf w16(int m) {
    constexpr float C1 = 0.92387953251128674f, S1 = 0.38268343236508978f, R2 = 0.70710678118654752f;
    const float cs[16] = {1.f, C1, R2, S1, 0.f, -S1, -R2, -C1, -1.f, -C1, -R2, -S1, 0.f, S1, R2, C1};
    const float sn[16] = {0.f, S1, R2, C1, 1.f, C1, R2, S1, 0.f, -S1, -R2, -C1, -1.f, -C1, -R2, -S1};
    return {cs[m & 15], -sn[m & 15]};
}

// a * exp(-2 pi i m / 16).  The quarter turns are a swap and sign changes: a general complex
// product with the constants 1 and 0 would still cost its multiplies by zero, which IEEE
// arithmetic does not let the compiler drop (same values either way, up to the sign of zeros).
// m is a constant once the callers' loops are unrolled, so the branches fold away.
__device__ __forceinline__ cf mul_w16(cf a, int m) {
    m &= 15;
    if (m == 0) return a;
    if (m == 4) return {a.y, -a.x};
    if (m == 8) return {-a.x, -a.y};
    if (m == 12) return {-a.y, a.x};
    return cmul(a, w16(m));
}

__host__ __device__ constexpr int bitrev(int v, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
    return r;
}

// In-register DFT of N = 8 or 16 points, natural order in and out (radix-2, decimation in
// time; every index and twiddle is a compile-time constant after unrolling).
template <int N>
__device__ __forceinline__ void dft_reg(cf (&x)[N]) {
    constexpr int LOG = N == 16 ? 4 : 3;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int j = bitrev(i, LOG);
        if (i < j) { const cf t = x[i]; x[i] = x[j]; x[j] = t; }
    }
#pragma unroll
    for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
        for (int i = 0; i < N; i += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const cf u = x[i + k], v = mul_w16(x[i + k + len / 2], k * (16 / len));
                x[i + k] = cadd(u, v);
                x[i + k + len / 2] = csub(u, v);
            }
        }
    }
}

// 128-point forward FFTs of all 128 lines of the LDS tile; rows (dir 0: element e of line
// l at l * FTP + e) or columns (dir 1: at e * FTP + l).  tw[m] = exp(-2 pi i m / 128).
// Lanes of a wave take 64 consecutive lines at one position: with the odd row pitch FTP the
// 64 addresses of every LDS access fall in distinct banks (two per bank for 8-byte
// elements), for rows and columns alike.
//
// Pass A, in place: thread (line, n2), n2 < 8: 16-point DFT over n1 of x[n2 + 8 n1], times
// W^(n2 k1).
__device__ __forceinline__ void pass_a(cf* sm, const cf* tw, int dir) {
    const int t = threadIdx.x;
    const int ls = dir == 0 ? FTP : 1, es = dir == 0 ? 1 : FTP;
    const int line = t & 127;
    const int n2 = t >> 7;
    cf* base = sm + line * ls;
    cf x[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) x[n1] = base[(n2 + 8 * n1) * es];
    dft_reg<16>(x);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) base[(n2 + 8 * k1) * es] = k1 == 0 ? x[0] : cmul(x[k1], tw[(n2 * k1) & 127]);
}
// Pass B's inputs: thread (line, k1) for two k1 (k1 = t / 128 + 8 h, line = t mod 128); the
// 8-point DFT over n2 of x[h] then gives X[k1 + 16 k2], k2 < 8.
__device__ __forceinline__ void pass_b_load(const cf* sm, int dir, cf (&x)[2][8], int (&line)[2], int (&k1)[2]) {
    const int t = threadIdx.x;
    const int ls = dir == 0 ? FTP : 1, es = dir == 0 ? 1 : FTP;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int u = t + FFT_THREADS * h;                 // 0 .. 2047
        line[h] = u & 127;
        k1[h] = u >> 7;
        const cf* base = sm + line[h] * ls;
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) x[h][n2] = base[(n2 + 8 * k1[h]) * es];
    }
}
__device__ __forceinline__ void fft_lines(cf* sm, const cf* tw, int dir) {
    const int ls = dir == 0 ? FTP : 1, es = dir == 0 ? 1 : FTP;
    pass_a(sm, tw, dir);
    __syncthreads();
    cf x[2][8];
    int line[2], k1[2];
    pass_b_load(sm, dir, x, line, k1);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        dft_reg<8>(x[h]);
        cf* base = sm + line[h] * ls;
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) base[(k1[h] + 16 * k2) * es] = x[h][k2];
    }
    __syncthreads();
}

__device__ __forceinline__ void fft2d(cf* sm, const cf* tw) {
    fft_lines(sm, tw, 0);
    fft_lines(sm, tw, 1);
}

__device__ __forceinline__ void load_twiddles(const Plan& p, cf* tw) {
    if (threadIdx.x < FT) {
        const float2 v = p.fft_tw[threadIdx.x];
        tw[threadIdx.x] = {v.x, v.y};
    }
}

// Spectrum of one stamp slot of one image, zero-padded to 128 x 128 at the origin: K
// (slot 0, the model and Jacobian convolutions) and K flipped (slot 1, the adjoint).  On a
// live-PSF image K is the stamp rendered for the current theta.
__global__ __launch_bounds__(FFT_THREADS) void k_fft_stamp(Plan p, int live_only) {
    __shared__ cf sm[FT * FTP];
    __shared__ cf tw[FT];
    const int k = blockIdx.y, slot = blockIdx.x;
    const DImage& im = p.images[k];
    if (im.fft_off < 0 || (live_only && !im.live)) return;

    load_twiddles(p, tw);
    const int P = im.P;
    const float* K = im.live ? p.psf_live + im.live_off : p.psf + im.psf_off;
    for (int e = threadIdx.x; e < FT * FT; e += FFT_THREADS) {
        const int u = e >> 7, v = e & 127;
        float val = 0.f;
        if (u < P && v < P) val = slot == 1 ? K[(P - 1 - u) * P + (P - 1 - v)] : K[u * P + v];
        sm[u * FTP + v] = {val, 0.f};
    }
    __syncthreads();
    fft2d(sm, tw);
    float2* out = p.fft_spec + im.fft_off + (long long)slot * FT * FT;
    for (int e = threadIdx.x; e < FT * FT; e += FFT_THREADS) {
        const cf v = sm[(e >> 7) * FTP + (e & 127)];
        out[e] = make_float2(v.x, v.y);
    }
}

hipError_t launch_fft_stamps(const Plan& p, int live_only, hipStream_t st) {
    if (p.n_images == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fft_stamp, dim3(2, p.n_images), dim3(FFT_THREADS), 0, st, p, live_only);
    return hipGetLastError();
}

__device__ __forceinline__ double fft_block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        s = red[0];
        for (int w = 1; w < FFT_THREADS / 64; ++w) s += red[w];
    }
    __syncthreads();
    return s;
}

template <int KIND>
__global__ __launch_bounds__(FFT_THREADS) void k_conv_fft(Plan p, const ConvJob* __restrict__ jobs,
                                                          const ConvItem* __restrict__ items,
                                                          const int4* __restrict__ pairs, int pair_begin,
                                                          ConvIO io) {
    __shared__ cf sm[FT * FTP];
    __shared__ cf tw[FT];
    __shared__ double red[FFT_THREADS / 64];
    // the pair carries its sub-problem, so a pair whose sub-problem skips this phase exits
    // after two dependent loads instead of five (items, job, image first)
    const int4 pr = pairs[pair_begin + xcd_chunk_item((int)blockIdx.x, (int)gridDim.x)];
    if (io.skip_mode == 1) {
        if (p.lmf[pr.z].chol_done == 0 || p.lmf[pr.z].trial_bad != 0) return;
    } else if (io.skip_mode == 2) {
        if (io.lm[pr.z].need_jac == 0) return;
    }
    const int half_item[2] = {pr.x, pr.y};
    const ConvJob jb0 = jobs[items[pr.x].job];
    const DImage& im = p.images[jb0.image];
    load_twiddles(p, tw);
    const int P = im.P, c = (P - 1) / 2, V = FT - P + 1;

    // ---- stage both halves: element (ly, lx) = input (oy - c + ly, ox - c + lx).  Every
    // thread issues all its global loads (NPT per half) before its first LDS store, so their
    // latencies overlap instead of following one another.
    constexpr int NPT = FT * FT / FFT_THREADS;
    static_assert(NPT * FFT_THREADS == FT * FT, "whole elements per thread");
    float hv[2][NPT];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int itx = half_item[h];
        const ConvItem it = items[itx < 0 ? pr.x : itx];
        const ConvJob jb = jobs[it.job];
        const int iy_base = jb.out_y0 + it.ty * V - c, ix_base = jb.out_x0 + it.tx * V - c;
        const float* in = nullptr;
        if constexpr (KIND != CONV_ADJ) in = io.in + jb.in_off + (long long)it.ch * jb.in_cs;
        const int iy1 = jb.in_y0 + jb.in_h, ix1 = jb.in_x0 + jb.in_w;
        // offsets within one image or one input plane fit in 32 bits
        if constexpr (KIND == CONV_ADJ) {
            // the seed, or -2 w r, on the image (zero elsewhere)
            const float* wimg = io.weight + im.pix_off;
            const float* rimg = p.rbuf + im.pix_off;
            const float* simg = io.seed ? io.seed + im.pix_off : nullptr;
            float rv[NPT];
            unsigned okm = 0;
#pragma unroll
            for (int q = 0; q < NPT; ++q) {
                const int e = (int)threadIdx.x + FFT_THREADS * q;
                const int y = iy_base + (e >> 7), x = ix_base + (e & 127);
                const bool ok = itx >= 0 && y >= 0 && y < im.H && x >= 0 && x < im.W;
                const int pix = y * im.Wc + x;
                hv[h][q] = 0.f;
                rv[q] = 0.f;
                if (ok) {
                    okm |= 1u << q;
                    if (simg) {
                        hv[h][q] = simg[pix];
                    } else {
                        hv[h][q] = wimg[pix];
                        rv[q] = rimg[pix];
                    }
                }
            }
            if (!simg) {
#pragma unroll
                for (int q = 0; q < NPT; ++q)
                    if ((okm >> q) & 1u) hv[h][q] = -2.f * hv[h][q] * rv[q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < NPT; ++q) {
                const int e = (int)threadIdx.x + FFT_THREADS * q;
                const int y = iy_base + (e >> 7), x = ix_base + (e & 127);
                float val = 0.f;
                if (itx >= 0 && y >= jb.in_y0 && y < iy1 && x >= jb.in_x0 && x < ix1)
                    val = in[(y - jb.in_y0) * jb.in_w + (x - jb.in_x0)];
                hv[h][q] = val;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int e = (int)threadIdx.x + FFT_THREADS * q;
        sm[(e >> 7) * FTP + (e & 127)] = {hv[0][q], hv[1][q]};
    }
    // the stamp spectrum at the elements this thread takes in the last pass of the forward
    // transform (the column pass B: column t mod 128 at rows t / 128 + 8 h + 16 k2), loaded
    // now so that their latency hides behind the transform
    const int slot = KIND == CONV_ADJ ? 1 : 0;
    const float2* Kf = p.fft_spec + im.fft_off + (long long)slot * FT * FT;
    float2 kv[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2)
            kv[h][k2] = Kf[((int)(threadIdx.x >> 7) + 8 * h + 16 * k2) * FT + (int)(threadIdx.x & 127)];
    __syncthreads();

    // ---- forward transform: rows, then columns, whose results are multiplied by the stamp
    // spectrum and conjugated for the inverse as they are stored
    fft_lines(sm, tw, 0);
    {
        pass_a(sm, tw, 1);
        __syncthreads();
        cf x[2][8];
        int line[2], k1[2];
        pass_b_load(sm, 1, x, line, k1);
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            dft_reg<8>(x[h]);
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) {
                const cf m = cmul(x[h][k2], {kv[h][k2].x, kv[h][k2].y});
                sm[(k1[h] + 16 * k2) * FTP + line[h]] = {m.x, -m.y};
            }
        }
        __syncthreads();
    }
    fft2d(sm, tw);
    const float scale = 1.f / (float)(FT * FT);     // real part of the inverse: x / N, imaginary: -y / N

    // ---- epilogues, one half at a time.  A thread takes the block's elements
    // threadIdx.x + k FFT_THREADS in row-major order; it steps their (row, column) by the
    // quotient and remainder of FFT_THREADS by the block width instead of dividing for each.
    const long long pix_off = im.pix_off;
    const int Wc = im.Wc;
    for (int h = 0; h < 2; ++h) {
        const int itx = half_item[h];
        if (itx < 0) break;                          // uniform across the block
        const ConvItem it = items[itx];
        const ConvJob jb = jobs[it.job];
        const int oy = jb.out_y0 + it.ty * V, ox = jb.out_x0 + it.tx * V;
        const int yend = min(oy + V, jb.out_y0 + jb.out_h), xend = min(ox + V, jb.out_x0 + jb.out_w);
        const int bh = yend - oy, bw = xend - ox;
        if (bh <= 0 || bw <= 0) continue;           // uniform; planned blocks are never empty
        const int sq = FFT_THREADS / bw, sr = FFT_THREADS - sq * bw;
        int ey = (int)threadIdx.x / bw, ex = (int)threadIdx.x - ey * bw;
        // offsets within one image or one output plane fit in 32 bits
        const int orow = oy - jb.out_y0, ocol = ox - jb.out_x0;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        if constexpr (KIND == CONV_FWD) {
            const float sky = (float)p.sky_val[jb.image];
            const float* wimg = io.data ? io.weight + pix_off : nullptr;
            const float* dimg = io.data ? io.data + pix_off : nullptr;
            float* oimg = io.out ? io.out + pix_off : nullptr;
            float* rimg = p.rbuf + pix_off;
            while (ey < bh) {
                int yy[EPI_B], xx[EPI_B];
                float wv[EPI_B], dv[EPI_B];
#pragma unroll
                for (int u = 0; u < EPI_B; ++u) {
                    yy[u] = ey;
                    xx[u] = ex;
                    ex += sr;
                    ey += sq;
                    if (ex >= bw) { ex -= bw; ++ey; }
                }
#pragma unroll
                for (int u = 0; u < EPI_B; ++u) {          // the batch's loads first
                    wv[u] = dv[u] = 0.f;
                    if (wimg && yy[u] < bh) {
                        const int pix = (oy + yy[u]) * Wc + ox + xx[u];
                        wv[u] = wimg[pix];
                        dv[u] = dimg[pix];
                    }
                }
#pragma unroll
                for (int u = 0; u < EPI_B; ++u) {
                    if (yy[u] >= bh) break;
                    const cf s = sm[(yy[u] + 2 * c) * FTP + xx[u] + 2 * c];
                    const float m = (h == 0 ? s.x : -s.y) * scale + sky;
                    const int pix = (oy + yy[u]) * Wc + ox + xx[u];
                    if (oimg) oimg[pix] = m;
                    if (wimg) {
                        const double w = (double)wv[u];
                        const double rr = (double)dv[u] - (double)m;
                        a0 += w * rr * rr;
                        a1 += w * rr;
                        a2 += w;
                        rimg[pix] = (float)rr;
                    }
                }
            }
            if (io.data) {
                a0 = fft_block_sum(a0, red);
                a1 = fft_block_sum(a1, red);
                a2 = fft_block_sum(a2, red);
                if (threadIdx.x == 0) {
                    io.part[(long long)itx * 3 + 0] = a0;
                    io.part[(long long)itx * 3 + 1] = a1;
                    io.part[(long long)itx * 3 + 2] = a2;
                }
            }
        } else if constexpr (KIND == CONV_JCOL) {
            float* __restrict__ out = io.out + jb.out_off + (long long)it.ch * jb.out_cs;
            const bool epart = io.weight && !jb.gram_part;   // sum w r J and sum w J here
            const float* wimg = io.weight + pix_off;
            const float* rimg = p.rbuf + pix_off;
            while (ey < bh) {
                int yy[EPI_B], xx[EPI_B];
                float wv[EPI_B], rv[EPI_B];
#pragma unroll
                for (int u = 0; u < EPI_B; ++u) {
                    yy[u] = ey;
                    xx[u] = ex;
                    ex += sr;
                    ey += sq;
                    if (ex >= bw) { ex -= bw; ++ey; }
                }
#pragma unroll
                for (int u = 0; u < EPI_B; ++u) {          // the batch's loads first
                    wv[u] = rv[u] = 0.f;
                    if (epart && yy[u] < bh) {
                        const int pix = (oy + yy[u]) * Wc + ox + xx[u];
                        wv[u] = wimg[pix];
                        rv[u] = rimg[pix];
                    }
                }
#pragma unroll
                for (int u = 0; u < EPI_B; ++u) {
                    if (yy[u] >= bh) break;
                    const cf s = sm[(yy[u] + 2 * c) * FTP + xx[u] + 2 * c];
                    const float v = (h == 0 ? s.x : -s.y) * scale;
                    out[(orow + yy[u]) * jb.out_w + ocol + xx[u]] = v;
                    if (epart) {
                        const double wj = (double)wv[u] * (double)v;
                        a0 += wj * (double)rv[u];
                        a1 += wj;
                    }
                }
            }
            if (epart) {
                a0 = fft_block_sum(a0, red);
                a1 = fft_block_sum(a1, red);
                if (threadIdx.x == 0) {
                    io.part[(long long)itx * 2 + 0] = a0;
                    io.part[(long long)itx * 2 + 1] = a1;
                }
            }
        } else {
            float* __restrict__ out = io.out + jb.out_off;
            while (ey < bh) {
                const cf s = sm[(ey + 2 * c) * FTP + ex + 2 * c];
                out[(orow + ey) * jb.out_w + ocol + ex] = (h == 0 ? s.x : -s.y) * scale;
                ex += sr;
                ey += sq;
                if (ex >= bw) { ex -= bw; ++ey; }
            }
        }
    }
}

template <int KIND>
static hipError_t launch_fft_kind(const Plan& p, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    if (L.pair_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_conv_fft<KIND>, dim3(L.pair_count), dim3(FFT_THREADS), 0, st, p, L.jobs, L.items,
                       L.pairs, L.pair_begin, io);
    return hipGetLastError();
}

hipError_t launch_conv_fft(const Plan& p, int kind, const ConvLaunch& L, const ConvIO& io, hipStream_t st) {
    if (kind == CONV_FWD) return launch_fft_kind<CONV_FWD>(p, L, io, st);
    if (kind == CONV_JCOL) return launch_fft_kind<CONV_JCOL>(p, L, io, st);
    if (kind == CONV_ADJ) return launch_fft_kind<CONV_ADJ>(p, L, io, st);
    return hipErrorInvalidValue;
}

}  // namespace apx
