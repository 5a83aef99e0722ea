// Normal-equation kernels: J^T W J tiles on FP64 MFMA, ordered reductions and the
// assembly of J^T W J, J^T W r, chi^2 and the gradient from their partial sums.
//
// A_pq = sum_i w_i J_ip J_iq (§2.5, the Gauss-Newton Hessian of Eq. chi2).  Columns of
// one group share an output box; the product of two groups runs over the intersection
// of their boxes.  FP32 Jacobian entries are promoted to FP64 (w J_p is exact in FP64),
// staged in LDS and contracted with v_mfma_f64_16x16x4_f64; every tile of every
// K-slice is written to its own slot and summed later in a fixed order, so the result
// does not depend on scheduling.
#include <type_traits>

#include "apx_internal.h"

namespace apx {

typedef double apx_d4 __attribute__((ext_vector_type(4)));

// TM = 64: the tile's 16 x 16 blocks that hold needed entries (a block is skipped when its
// rows or its columns lie past the group's last column, or, on a diagonal tile of a group
// with itself, when it lies wholly below the diagonal) are dealt to the 4 waves in turn,
// at most 4 blocks (MFMA accumulators) each.
// TM = 16: 4 waves share one 16 x 16 tile and split each LDS stage along K.
// Stages of KC = PAIR_KC pixels (one row segment of the box intersection) are software
// pipelined two deep: the global loads of stages s+1 and s+2 are in flight while the
// MFMAs consume s.  Each thread stages the same tile columns and pixel offsets in every
// stage, so its column offsets into J are computed once.
template <int TM>
__global__ __launch_bounds__(256) void k_pair(Plan p, const DPair* __restrict__ pairs,
                                              const PairItem* __restrict__ items,
                                              const float* __restrict__ weight,
                                              const apx_lm_state* lm) {
    constexpr int KC = PAIR_KC;
    constexpr int PER = TM * KC / 256;              // elements of A (and of B) per thread
    constexpr int NB = TM >= 64 ? 2 : 1;            // accumulators: NB x NB per wave
    __shared__ double As[TM][KC + 1];
    __shared__ double Bs[TM][KC + 1];
    // the 64-wide tile pairs of one K-slice (up to 21 for a 350-column group) share its rows
    // of J in one L2 when each XCD takes a contiguous range of items (in runs of 8 they read
    // J 3.3x over from HBM); the narrow ones, of cutouts that may skip, go in runs
    const PairItem it = items[TM >= 64 ? xcd_item((int)blockIdx.x, (int)gridDim.x)
                                       : xcd_chunk_item((int)blockIdx.x, (int)gridDim.x)];
    const DPair pr = pairs[it.pair];
    if (lm && lm[pr.sub].need_jac == 0) return;
    // by value: the fields live in registers for the whole loop (no reloads through the
    // pointers after every store)
    const DGroup G = p.groups[pr.g];
    const DGroup Hh = p.groups[pr.h];
    const long long pix_off = p.images[pr.image].pix_off;
    const int imW = p.images[pr.image].Wc;          // image pixels (output boxes are in pixels)
    const long long gs = (long long)G.oh * G.ow, hs = (long long)Hh.oh * Hh.ow;
    const float* __restrict__ Jg = p.J + G.j_off;
    const float* __restrict__ Jh = p.J + Hh.j_off;
    const int a0 = it.ta * TM, b0 = it.tb * TM;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // TM = 64: this wave's blocks s < nbk, row block (blk >> 4 s) & 3, column block
    // (blk >> (4 s + 2)) & 3
    int blk = 0, nbk = 0;
    if constexpr (TM >= 64) {
        const int rows = G.ncols - a0, cols = Hh.ncols - b0;
        const bool diag = pr.g == pr.h && it.ta == it.tb;
        int k = 0;
        for (int m = 0; m < 4; ++m)
            for (int n = 0; n < 4; ++n) {
                if (16 * m >= rows || 16 * n >= cols || (diag && m > n)) continue;
                if ((k & 3) == wv) {
                    blk |= (m | (n << 2)) << (4 * nbk);
                    ++nbk;
                }
                ++k;
            }
    }
    auto bm = [&](int q) { return (blk >> (4 * q)) & 3; };
    auto bn = [&](int q) { return (blk >> (4 * q + 2)) & 3; };
    apx_d4 acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = (apx_d4){0.0, 0.0, 0.0, 0.0};

    // element q of this thread: tile column i0 + DI q at stage pixel kq, the same in every
    // stage; its offset into J is colA + q * stepA (the step is uniform)
    constexpr int DI = 256 / KC;
    const int i0 = threadIdx.x / KC, kq = threadIdx.x % KC;
    const long long colA = (long long)(a0 + i0) * gs - G.ox0, stepA = (long long)DI * gs;
    const long long colB = (long long)(b0 + i0) * hs - Hh.ox0, stepB = (long long)DI * hs;
    const int nva = G.ncols - a0 - i0, nvb = Hh.ncols - b0 - i0;   // element q valid: DI q < nv
    const long long lastA = (long long)(G.ncols - 1) * gs - G.ox0;   // a column that exists
    const long long lastB = (long long)(Hh.ncols - 1) * hs - Hh.ox0;

    const int nxs = (pr.x1 - pr.x0 + KC - 1) / KC;
    const int n_stage = it.s1 - it.s0;
    // two stages of global loads in flight (register ring): the loads of stage s+2 are
    // issued while the MFMAs consume stages s and s+1
    float ra0[PER], rb0[PER], rw0 = 0.f, ra1[PER], rb1[PER], rw1 = 0.f;
    // every load is issued unconditionally (a lane past the box or past the last column
    // reads a valid entry and zeroes it afterwards), so the 2 PER + 1 loads of a stage go
    // out back to back instead of one branch each
    auto fetch = [&](int st, float (&ra)[PER], float (&rb)[PER], float& rw) {
        const int gs_ = it.s0 + st;
        const int row = pr.y0 + gs_ / nxs;
        const int x = pr.x0 + (gs_ - (gs_ / nxs) * nxs) * KC + kq;
        const bool in = x < pr.x1;
        const int xc = in ? x : pr.x1 - 1;
        const long long grow = (long long)(row - G.oy0) * G.ow + xc;
        const long long hrow = (long long)(row - Hh.oy0) * Hh.ow + xc;
        const float wv = weight[pix_off + (long long)row * imW + xc];
        rw = in ? wv : 0.f;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const bool va = DI * q < nva, vb = DI * q < nvb;
            const float a = Jg[(va ? colA + q * stepA : lastA) + grow];
            const float b = Jh[(vb ? colB + q * stepB : lastB) + hrow];
            ra[q] = (in && va) ? a : 0.f;
            rb[q] = (in && vb) ? b : 0.f;
        }
    };
    auto stage = [&](const float (&ra)[PER], const float (&rb)[PER], float rw) {
        const double wd = (double)rw;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            As[i0 + DI * q][kq] = (double)ra[q] * wd;
            Bs[i0 + DI * q][kq] = (double)rb[q];
        }
    };
    auto compute = [&]() {
        if constexpr (TM >= 64) {
            // one branch per stage on the wave's block count; inside, the LDS reads of a
            // K step are all issued before its MFMAs
            // a wave with fewer than 4 blocks spreads each over 4 / NS accumulators (K steps
            // dealt in turn), so it still has 4 independent MFMA chains
            auto run = [&](auto ns) {
                constexpr int NS = decltype(ns)::value;
                constexpr int R = NS == 1 ? 4 : NS == 2 ? 2 : 1;
#pragma unroll
                for (int kk = 0; kk < KC; kk += 4) {
                    const int rr = (kk / 4) % R;
                    double av[NS], bv[NS];
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        av[q] = As[bm(q) * 16 + (lane & 15)][kk + (lane >> 4)];
                        bv[q] = Bs[bn(q) * 16 + (lane & 15)][kk + (lane >> 4)];
                    }
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        const int c = q * R + rr;
                        acc[c >> 1][c & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc[c >> 1][c & 1], 0, 0, 0);
                    }
                }
            };
            switch (nbk) {
                case 4: run(std::integral_constant<int, 4>{}); break;
                case 3: run(std::integral_constant<int, 3>{}); break;
                case 2: run(std::integral_constant<int, 2>{}); break;
                case 1: run(std::integral_constant<int, 1>{}); break;
                default: break;
            }
        } else {
#pragma unroll
            for (int kk = 8 * wv; kk < 8 * wv + 8; kk += 4) {
                const double av = As[lane & 15][kk + (lane >> 4)];
                const double bv = Bs[lane & 15][kk + (lane >> 4)];
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[0][0], 0, 0, 0);
            }
        }
    };
    if (n_stage > 0) fetch(0, ra0, rb0, rw0);
    if (n_stage > 1) fetch(1, ra1, rb1, rw1);
    for (int st = 0; st < n_stage; st += 2) {
        stage(ra0, rb0, rw0);
        __syncthreads();
        if (st + 2 < n_stage) fetch(st + 2, ra0, rb0, rw0);
        compute();
        __syncthreads();
        if (st + 1 < n_stage) {
            stage(ra1, rb1, rw1);
            __syncthreads();
            if (st + 3 < n_stage) fetch(st + 3, ra1, rb1, rw1);
            compute();
            __syncthreads();
        }
    }

    double* out = p.pair_part + it.out_off;
    if constexpr (TM >= 64) {
        // blocks no wave holds are left unwritten: the assembly reads none of their entries.
        // A block's R accumulators are added in order.
        auto emit = [&](auto ns) {
            constexpr int NS = decltype(ns)::value;
            constexpr int R = NS == 1 ? 4 : NS == 2 ? 2 : 1;
#pragma unroll
            for (int q = 0; q < NS; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double sum = acc[(q * R) >> 1][(q * R) & 1][v];
#pragma unroll
                    for (int r = 1; r < R; ++r) sum += acc[(q * R + r) >> 1][(q * R + r) & 1][v];
                    // v_mfma_f64_16x16x4: D[i][j] sits in lane j + 16 (i % 4), register i / 4
                    const int i = bm(q) * 16 + (lane >> 4) + 4 * v;
                    const int j = bn(q) * 16 + (lane & 15);
                    out[i * TM + j] = sum;
                }
        };
        switch (nbk) {
            case 4: emit(std::integral_constant<int, 4>{}); break;
            case 3: emit(std::integral_constant<int, 3>{}); break;
            case 2: emit(std::integral_constant<int, 2>{}); break;
            case 1: emit(std::integral_constant<int, 1>{}); break;
            default: break;
        }
    } else {
        // reduce the four K-slices in a fixed order
        __shared__ double red[4][256];
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wv][((lane >> 4) + 4 * v) * 16 + (lane & 15)] = acc[0][0][v];
        __syncthreads();
        const int t = threadIdx.x;
        out[t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    }
}

// J^T W J of a narrow group (NT tiles of 4 columns, at most 36 columns) with itself over one
// K-slice, on v_mfma_f64_4x4x4f64: the instruction holds four independent 4 x 4 x 4 products
// (blocks), block b of lanes 16 k + 4 b + i (A[i][k], B[k][j] at lane 16 k + 4 b + j, D[i][j] at
// lane 16 i + 4 b + j; measured on gfx950).  Lane L takes pixel L / 4 of a 16-pixel chunk and
// column L % 4 of a tile, so one instruction contracts 16 pixels of one 4 x 4 tile pair, and
// the tiles are loaded straight from J into registers (each reused by every pair it is in).
// Waves take every fourth 32-pixel stage of the slice; at the end each wave folds its four
// blocks (lanes xor 4, xor 8) and the four waves are added in order.  Against 16 x 16 tiles
// this pads a group of 7k columns to a multiple of 4, not 16.  Each tile is also contracted
// with [r 1 0 0] (the pixel's residual, a one), giving the columns' J^T W r and sum w J (the
// sky row of J^T W J) over the slice in NT more blocks, after the tile pairs.
template <int NT>
__global__ __launch_bounds__(256) void k_gram4(Plan p, const DPair* __restrict__ pairs,
                                               const PairItem* __restrict__ items, int n_items,
                                               const float* __restrict__ weight, const apx_lm_state* lm) {
    constexpr int NP = NT * (NT + 1) / 2;
    constexpr int KC = PAIR_KC;
    const PairItem it = items[xcd_chunk_item((int)blockIdx.x, n_items)];
    const DPair pr = pairs[it.pair];
    if (lm && lm[pr.sub].need_jac == 0) return;
    const DGroup G = p.groups[pr.g];
    const long long pix_off = p.images[pr.image].pix_off;
    const int imW = p.images[pr.image].Wc;
    const long long gs = (long long)G.oh * G.ow;
    const float* __restrict__ Jg = p.J + G.j_off;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 3, pxl = lane >> 2;       // column within a tile, pixel within a chunk
    const long long lastA = (long long)(G.ncols - 1) * gs - G.ox0;
    long long coff[NT];
    bool cval[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int ca = 4 * t + col;
        cval[t] = ca < G.ncols;
        coff[t] = cval[t] ? (long long)ca * gs - G.ox0 : lastA;
    }
    double acc[NP], acx[NT];
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[q] = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) acx[t] = 0.0;
    const int nxs = (pr.x1 - pr.x0 + KC - 1) / KC;
    // the wave's 16-pixel chunks, in order: chunk h of stages it.s0 + wv, + 4, + 8, ...; the
    // loads of the next chunk are issued before the MFMAs of the current one
    constexpr int NH = KC / 16;
    auto fetch = [&](int st, int h, float (&bv)[NT], float& wf, float& rf, bool& in) {
        const int row = pr.y0 + st / nxs;
        const int x = pr.x0 + (st - (st / nxs) * nxs) * KC + 16 * h + pxl;
        in = x < pr.x1;
        const int xc = in ? x : pr.x1 - 1;
        const long long grow = (long long)(row - G.oy0) * G.ow + xc;
        const long long pix = pix_off + (long long)row * imW + xc;
        wf = weight[pix];
        rf = p.rbuf[pix];
#pragma unroll
        for (int t = 0; t < NT; ++t) bv[t] = Jg[coff[t] + grow];
    };
    float bc[NT], wc = 0.f, rc = 0.f;
    bool inc = false;
    int st = it.s0 + wv, h = 0;
    if (st < it.s1) fetch(st, 0, bc, wc, rc, inc);
    while (st < it.s1) {
        int st2 = st, h2 = h + 1;
        if (h2 == NH) {
            h2 = 0;
            st2 += 4;
        }
        float bn[NT], wn = 0.f, rn = 0.f;
        bool inn = false;
        if (st2 < it.s1) fetch(st2, h2, bn, wn, rn, inn);
        const double w = inc ? (double)wc : 0.0;
        const double vx = col == 0 ? (double)rc : (col == 1 ? 1.0 : 0.0);     // [r 1 0 0]
        double b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = (inc && cval[t]) ? (double)bc[t] : 0.0;
        int q = 0;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta) {
            const double a = b[ta] * w;
#pragma unroll
            for (int tb = ta; tb < NT; ++tb, ++q)
                acc[q] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b[tb], acc[q], 0, 0, 0);
            acx[ta] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, vx, acx[ta], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) bc[t] = bn[t];
        wc = wn;
        rc = rn;
        inc = inn;
        st = st2;
        h = h2;
    }
    // fold the four blocks of each wave, then the four waves in order
    __shared__ double red[4][(NP + NT) * 16];
#pragma unroll
    for (int q = 0; q < NP + NT; ++q) {
        double v = q < NP ? acc[q] : acx[q - NP];
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        // lanes with block 0 (lane % 16 < 4) hold D[i][j] at lane 16 i + j
        if ((lane & 12) == 0) red[wv][q * 16 + (lane >> 4) * 4 + (lane & 3)] = v;
    }
    __syncthreads();
    double* out = p.pair_part + it.out_off;
    for (int e = (int)threadIdx.x; e < (NP + NT) * 16; e += 256)
        out[e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

hipError_t launch_gram4(const Plan& p, const PairLaunch& L, const float* weight,
                        const apx_lm_state* lm, hipStream_t st) {
    if (L.n_items <= 0) return hipSuccess;
    dim3 grid(L.n_items), block(256);
    switch (L.tm) {
#define APX_G4(T)                                                                                       \
    case T:                                                                                             \
        hipLaunchKernelGGL(k_gram4<T>, grid, block, 0, st, p, L.pairs, L.items, L.n_items, weight, lm); \
        break;
        APX_G4(1) APX_G4(2) APX_G4(3) APX_G4(4) APX_G4(5) APX_G4(6) APX_G4(7) APX_G4(8) APX_G4(9)
#undef APX_G4
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int pair_blocks_per_cu(int tm) {
    int nb = 0;
    const hipError_t e = tm == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair<64>, 256, 0)
                                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair<16>, 256, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

hipError_t launch_pairs(const Plan& p, const PairLaunch& L, const float* weight,
                        const apx_lm_state* lm, hipStream_t st) {
    if (L.n_items <= 0) return hipSuccess;
    if (L.tm == 64)
        hipLaunchKernelGGL(k_pair<64>, dim3(L.n_items), dim3(256), 0, st, p, L.pairs, L.items, weight, lm);
    else
        hipLaunchKernelGGL(k_pair<16>, dim3(L.n_items), dim3(256), 0, st, p, L.pairs, L.items, weight, lm);
    return hipGetLastError();
}

// out[s*ostride + ocomp] = scale * sum_k wts[k] * src[(idx ? idx[k] : k) * stride + comp],
// k in [seg[s], seg[s+1]).  One wave per segment: lane l sums entries l, l+64, ... in
// order, then a fixed butterfly combines the lanes -- the same order on every run.
// Segments of sub-problems that keep their Jacobian are skipped when lm is given.  With
// ncomp > 1 one launch sums components comp + q into ocomp + q (q < ncomp), one wave per
// (segment, component), each in the same order as a launch of its own.
__global__ __launch_bounds__(256) void k_segsum(SegSum a) {
    const int nc = a.ncomp > 1 ? a.ncomp : 1;
    const int sf = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (sf >= a.n_seg * nc) return;
    const int s = sf / nc, q = sf - s * nc;
    if (a.lm && a.seg_sub && a.lm[a.seg_sub[s]].need_jac == 0) return;
    double acc = 0.0;
    for (int k = a.seg[s] + lane; k < a.seg[s + 1]; k += 64) {
        const long long j = a.idx ? (long long)a.idx[k] : (long long)k;
        const double v = a.src[j * a.stride + a.comp + q];
        acc += a.wts ? a.wts[k] * v : v;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) a.out[(long long)s * a.ostride + a.ocomp + q] = acc * a.scale;
}

hipError_t launch_segsum(const SegSum& a, hipStream_t st) {
    const long long n = (long long)a.n_seg * (a.ncomp > 1 ? a.ncomp : 1);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_segsum, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// J^T W J assembly: every upper entry (sub, a <= b) sums its sources in list order and
// is written to both (a, b) and (b, a) of its sub-problem's row-major block.
__global__ void k_assemble_A(AsmA a) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n_ent) return;
    const int s = a.ent_sub[e];
    if (a.lm && a.lm[s].need_jac == 0) return;
    double acc = 0.0;
    for (long long k = a.ent_off[e]; k < a.ent_off[e + 1]; ++k) acc += a.src[a.ent_src[k]];
    const DSub sb = a.subs[s];
    const int r = a.ent_row[e], c = a.ent_col[e];
    a.out[sb.a_off + (long long)r * sb.n + c] = acc;
    a.out[sb.a_off + (long long)c * sb.n + r] = acc;
}

hipError_t launch_assemble_A(const AsmA& a, hipStream_t st) {
    if (a.n_ent <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_assemble_A, dim3((unsigned)((a.n_ent + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Dense Jacobian for callers that want it: J[k * ldJ + i] = sum of the stored blocks of
// the columns tied to theta index k (in column order) + 1 on the pixels of images whose
// sky is theta index k.
__global__ void k_jscatter(Plan p, const int* __restrict__ par_off, const int* __restrict__ par_cols,
                           const int* __restrict__ par_sky_off, const int* __restrict__ par_sky,
                           float* __restrict__ Jd, long long ldJ) {
    const int k = blockIdx.y;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_pix) return;
    // image of pixel i (binary search on pix_off)
    int lo = 0, hi = p.n_images - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.images[mid].pix_off <= i) lo = mid; else hi = mid - 1;
    }
    const DImage& im = p.images[lo];
    const long long local = i - im.pix_off;
    const int y = (int)(local / im.Wc), x = (int)(local - (long long)y * im.Wc);
    float v = 0.f;
    for (int q = par_off[k]; q < par_off[k + 1]; ++q) {
        const DCol cl = p.cols[par_cols[q]];
        const DGroup& g = p.groups[cl.group];
        if (g.image != lo) continue;
        if (y < g.oy0 || y >= g.oy0 + g.oh || x < g.ox0 || x >= g.ox0 + g.ow) continue;
        const int ci = par_cols[q] - g.col_begin;
        v += p.J[g.j_off + (long long)ci * g.oh * g.ow + (long long)(y - g.oy0) * g.ow + (x - g.ox0)];
    }
    for (int q = par_sky_off[k]; q < par_sky_off[k + 1]; ++q)
        if (par_sky[q] == lo) v += 1.f;
    Jd[(long long)k * ldJ + i] = v;
}

hipError_t launch_jscatter(const Plan& p, const int* par_off, const int* par_cols,
                           const int* par_sky_off, const int* par_sky, float* Jd, long long ldJ,
                           hipStream_t st) {
    if (p.n_par == 0 || p.n_pix == 0) return hipSuccess;
    dim3 grid((unsigned)((p.n_pix + 255) / 256), p.n_par);
    hipLaunchKernelGGL(k_jscatter, grid, dim3(256), 0, st, p, par_off, par_cols, par_sky_off,
                       par_sky, Jd, ldJ);
    return hipGetLastError();
}

__global__ void k_fill_d(double* x, long long n, double v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_fill_f(float* x, long long n, float v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

hipError_t launch_fill_f(float* x, long long n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(k_fill_f, dim3((unsigned)b), dim3(256), 0, st, x, n, v);
    return hipGetLastError();
}

hipError_t launch_fill(double* x, long long n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(k_fill_d, dim3((unsigned)b), dim3(256), 0, st, x, n, v);
    return hipGetLastError();
}

// Sticky non-finite flag from per-sub chi^2 values.
__global__ void k_chi2_check(const double* chi2, int n, int* sticky) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n && !isfinite(chi2[s])) atomicOr(sticky, FLAG_NONFINITE);
}

hipError_t launch_chi2_check(const double* chi2, int n, int* sticky, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chi2_check, dim3((n + 255) / 256), dim3(256), 0, st, chi2, n, sticky);
    return hipGetLastError();
}

}  // namespace apx
