// Levenberg-Marquardt kernels (§2.5): Marquardt-damped normal equations solved by FP64
// Cholesky on the device, with the damping raised and the factorisation retried when a
// pivot is not positive (the step never meets a singular matrix), the trial step, and
// the gain-ratio accept/reject with lambda update.  All control stays on the device so
// an iteration can be captured in a HIP graph; every sub-problem carries its own state.
#include "apx_internal.h"

namespace apx {

__device__ __forceinline__ double lm_wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double lm_wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Start of an iteration: clear the per-iteration flags of both solve copies and decide
// whether a large sub-problem takes the step solved ahead: the same A (its last trial was
// rejected, so no new normal equations) and the lambda that solve started from.
__global__ void k_lm_begin(Plan p, const apx_lm_state* lm) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_sub) return;
    LMFlags f;
    f.chol_done = 0;
    f.chol_fail = 0;
    f.trial_bad = 0;
    f.skip = 0;
    f.subst_fail = 0;
    f.rhs_folded = 0;
    f.adopted = 0;
    p.lmf[p.n_sub + s] = f;
    const LMSpec sp = p.spec[s];
    f.adopted = p.subs[s].large && sp.valid && lm[s].need_jac == 0 && lm[s].lambda == sp.lam_start;
    p.lmf[s] = f;
}

hipError_t launch_lm_begin(const Plan& p, apx_lm_state* lm, hipStream_t st) {
    hipLaunchKernelGGL(k_lm_begin, dim3((p.n_sub + 255) / 256), dim3(256), 0, st, p, lm);
    return hipGetLastError();
}

// k_lm_begin, then adoption, in one launch with one wave per sub-problem (for problems with
// a large sub-problem, whose solves are made ahead): lane 0 sets the flags as k_lm_begin does;
// an adopting sub-problem then takes the step, its predicted decrease, lambda and retry
// count from the solve made ahead (exactly what solving now would give: same A, D, g and
// starting lambda, same kernels), and the record is used up.
__global__ __launch_bounds__(64) void k_lm_begin_adopt(Plan p, apx_lm_state* lm) {
    const int s = blockIdx.x;
    int adopted = 0;
    if (threadIdx.x == 0) {
        LMFlags f;
        f.chol_done = 0;
        f.chol_fail = 0;
        f.trial_bad = 0;
        f.skip = 0;
        f.subst_fail = 0;
        f.rhs_folded = 0;
        f.adopted = 0;
        p.lmf[p.n_sub + s] = f;
        const LMSpec sp = p.spec[s];
        f.adopted = p.subs[s].large && sp.valid && lm[s].need_jac == 0 && lm[s].lambda == sp.lam_start;
        p.lmf[s] = f;
        adopted = f.adopted;
    }
    adopted = __shfl(adopted, 0, 64);
    if (!adopted) return;
    const DSub sb = p.subs[s];
    for (int i = (int)threadIdx.x; i < sb.n; i += 64) p.hvec[sb.p0 + i] = p.hvec[p.n_par + sb.p0 + i];
    if (threadIdx.x == 0) {
        const LMSpec sp = p.spec[s];
        lm[s].pred = sp.pred;
        lm[s].lambda = sp.lam_final;
        lm[s].n_chol_retry += sp.retries;
        p.lmf[s].chol_done = sp.done;
        p.spec[s].valid = 0;
    }
}

hipError_t launch_lm_begin_adopt(const Plan& p, apx_lm_state* lm, hipStream_t st) {
    hipLaunchKernelGGL(k_lm_begin_adopt, dim3(p.n_sub), dim3(64), 0, st, p, lm);
    return hipGetLastError();
}

__global__ void k_lm_init(Plan p, const double* chi2_sub, apx_lm_state* lm) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_sub) return;
    apx_lm_state st;
    st.lambda = APX_LM_LAMBDA0;
    st.chi2 = chi2_sub[s];
    st.chi2_trial = 0.0;
    st.pred = 0.0;
    st.rho = 0.0;
    st.need_jac = 1;
    st.accepted = 0;
    st.n_accept = 0;
    st.n_reject = 0;
    st.n_chol_retry = 0;
    st.status = isfinite(st.chi2) ? APX_OK : APX_E_NONFINITE;
    lm[s] = st;
    p.spec[s].valid = 0;
}

hipError_t launch_lm_init(const Plan& p, const double* chi2_sub, apx_lm_state* lm, hipStream_t st) {
    hipLaunchKernelGGL(k_lm_init, dim3((p.n_sub + 255) / 256), dim3(256), 0, st, p, chi2_sub, lm);
    return hipGetLastError();
}

// -------------------------------------------------------------- small sub-problems
// One wave64 per sub-problem (n <= 64): the damped matrix, its factor and the step
// live in LDS; the retries happen inside the kernel.
__global__ __launch_bounds__(64) void k_chol_small(Plan p, const int* __restrict__ small_subs,
                                                   int nmax, apx_lm_state* lm) {
    extern __shared__ double sm[];
    const int s = small_subs[blockIdx.x];
    const DSub sb = p.subs[s];
    const int n = sb.n, ld = nmax + 1;
    double* M = sm;
    double* y = sm + (long long)nmax * ld;
    const int i = threadIdx.x;
    const double* A = p.A + sb.a_off;
    const double* g = p.gvec + sb.p0;
    if (n == 0) {
        if (i == 0) { p.lmf[s].chol_done = 1; lm[s].pred = 0.0; }
        return;
    }
    const double di = i < n ? A[(long long)i * n + i] : 0.0;
    const double dmax = lm_wave_max(i < n ? di : -1e308);
    const double Di = fmax(di, APX_LM_DAMP_FLOOR * dmax);
    double lam = lm[s].lambda;
    int done = 0, retries = 0;
    for (int att = 0; att < APX_LM_ATTEMPTS; ++att) {
        if (i < n)
            for (int j = 0; j <= i; ++j) M[i * ld + j] = A[(long long)i * n + j] + (i == j ? lam * Di : 0.0);
        __syncthreads();
        bool ok = true;
        for (int k = 0; k < n; ++k) {
            const double piv = M[k * ld + k];
            if (!(piv > 0.0) || !isfinite(piv)) { ok = false; break; }
            const double lkk = sqrt(piv);
            __syncthreads();
            if (i == k) M[k * ld + k] = lkk;
            if (i > k && i < n) M[i * ld + k] = M[i * ld + k] / lkk;
            __syncthreads();
            if (i > k && i < n) {
                const double lik = M[i * ld + k];
                for (int j = k + 1; j <= i; ++j) M[i * ld + j] -= lik * M[j * ld + k];
            }
            __syncthreads();
        }
        __syncthreads();
        if (ok) { done = 1; break; }
        lam = fmin(lam * APX_LM_UP, APX_LM_LAMBDA_MAX);
        ++retries;
    }
    double h = 0.0;
    if (done) {
        if (i < n) y[i] = g[i];
        __syncthreads();
        for (int k = 0; k < n; ++k) {
            if (i == k) y[k] = y[k] / M[k * ld + k];
            __syncthreads();
            if (i > k && i < n) y[i] -= M[i * ld + k] * y[k];
            __syncthreads();
        }
        for (int k = n - 1; k >= 0; --k) {
            if (i == k) y[k] = y[k] / M[k * ld + k];
            __syncthreads();
            if (i < k) y[i] -= M[k * ld + i] * y[k];
            __syncthreads();
        }
        if (i < n) h = y[i];
    }
    const double pr = lm_wave_sum(i < n ? h * (lam * Di * h + g[i]) : 0.0);
    if (i < n) {
        p.hvec[sb.p0 + i] = h;
        p.Ddiag[sb.p0 + i] = Di;
    }
    if (i == 0) {
        lm[s].lambda = lam;
        lm[s].pred = pr;
        lm[s].n_chol_retry += retries;
        p.lmf[s].chol_done = done;
    }
}

hipError_t launch_chol_small(const Plan& p, const int* small_subs, int n_small, int nmax,
                             apx_lm_state* lm, hipStream_t st) {
    if (n_small <= 0) return hipSuccess;
    const size_t lds = (size_t)nmax * (nmax + 1) * sizeof(double) + (size_t)nmax * sizeof(double);
    hipLaunchKernelGGL(k_chol_small, dim3(n_small), dim3(64), lds, st, p, small_subs, nmax, lm);
    return hipGetLastError();
}

// -------------------------------------------------------------- large sub-problems
// Right-looking blocked Cholesky (block CHOL_NB).  The first attempt runs as a sequence
// of launches (panel, trailing update) so the update spreads over the chip; a failed
// attempt is retried (lambda *= UP) by one fallback workgroup that factors the whole
// matrix itself -- the rare path costs one launch that exits at once when unused.

// 1/sqrt(x) for positive normal x: the hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2 (each roughly doubles the correct bits), a short dependent chain
// on the factorisation's critical path.
__device__ __forceinline__ double rsqrt_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}

// Value of v in lane `src` (a compile-time constant after unrolling), to every lane.
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Blocked factorisation of one CHOL_NB x CHOL_NB diagonal block in LDS, by the whole
// 256-thread workgroup (every thread must call it).  The block is taken in four 16-column
// sub-panels.  For each, wave 0 holds one row per lane (16 entries in registers) and runs
// the 16 column steps of a right-looking Cholesky over every row at or below the
// sub-panel -- the 16 x 16 diagonal factor and the solve of the rows below it in one pass:
// the pivot comes from its lane by readlane, 1/sqrt refines the hardware estimate, the
// scaled column goes through LDS and the later entries of the row are updated with
// independent FMAs.  The trailing rows and columns are then updated with the sub-panel
// (a rank-16 update) on FP64 MFMA, its 16 x 16 blocks shared out over the four waves.
// Rows at or beyond the block size must arrive as identity rows.  On return B holds the
// factor (lower triangle, row-major) and invd the reciprocals of its diagonal; the
// return value is false (in every thread) on a non-positive or non-finite pivot.
typedef double chol_d4 __attribute__((ext_vector_type(4)));
constexpr int SUBP = 16;                       // sub-panel width

// D[16 di + r][16 dk + c] -= sum_{k < 16} A[16 ai + r][c0 + k] * Bm[16 bk + c][c0 + k]
// for one 16 x 16 block, by one wave (v_mfma_f64_16x16x4: A row m = lane % 16 and B
// column n = lane % 16 at k = lane / 16; D[i][j] sits in lane j + 16 (i % 4), register i / 4).
__device__ __forceinline__ void rank16_block(double (*D)[CHOL_NB + 1], int di, int dk,
                                             const double (*A)[CHOL_NB + 1], int ai,
                                             const double (*Bm)[CHOL_NB + 1], int bk, int c0, int lane) {
    chol_d4 acc = (chol_d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < SUBP; k0 += 4) {
        const double a = A[SUBP * ai + (lane & 15)][c0 + k0 + (lane >> 4)];
        const double b = Bm[SUBP * bk + (lane & 15)][c0 + k0 + (lane >> 4)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) D[SUBP * di + (lane >> 4) + 4 * v][SUBP * dk + (lane & 15)] -= acc[v];
}

__device__ __forceinline__ bool factor_diag_blocked(double (*B)[CHOL_NB + 1], double* col, double* invd, int* bad) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) *bad = 0;
    __syncthreads();
    for (int p = 0; p < CHOL_NB / SUBP; ++p) {
        const int c0 = SUBP * p;
        if (wv == 0) {
            double f[SUBP];
#pragma unroll
            for (int q = 0; q < SUBP; ++q) f[q] = B[lane][c0 + q];
            bool ok = true;
#pragma unroll
            for (int j = 0; j < SUBP; ++j) {
                const int cj = c0 + j;
                double piv = lane_bcast(f[j], cj);
                // a failed pivot is recorded and replaced by 1 so the (discarded) factor
                // stays finite and the loop has no exit
                if (!(piv > 0.0) || !isfinite(piv)) { ok = false; piv = 1.0; }
                const double rj = rsqrt_f64(piv);
                const double l = lane > cj ? f[j] * rj : 0.0;
                f[j] = lane > cj ? l : (lane == cj ? piv * rj : f[j]);
                if (lane == 0) invd[cj] = rj;
                col[lane] = l;
                __builtin_amdgcn_wave_barrier();
                double cv[SUBP];
#pragma unroll
                for (int q = j + 1; q < SUBP; ++q) cv[q] = col[c0 + q];
#pragma unroll
                for (int q = j + 1; q < SUBP; ++q) f[q] = fma(-l, cv[q], f[q]);
                __builtin_amdgcn_wave_barrier();
            }
            if (lane >= c0) {
#pragma unroll
                for (int q = 0; q < SUBP; ++q) B[lane][c0 + q] = f[q];
            }
            if (!ok && lane == 0) *bad = 1;
        }
        __syncthreads();
        if (*bad) return false;
        // trailing lower-triangular blocks (bi >= bk > p): 6, 3, 1 of them
        const int first = p + 1, nt = CHOL_NB / SUBP - first;
        for (int e = wv; e < nt * (nt + 1) / 2; e += 4) {
            int bi = 0, r = e;
            while (r > bi) { r -= bi + 1; ++bi; }
            rank16_block(B, first + bi, first + r, B, first + bi, B, first + r, c0, lane);
        }
        __syncthreads();
    }
    return true;
}

// x L^T = m for a CHOL_NB-row block X in LDS against the factored diagonal block B (the
// whole workgroup calls it): per 16-column sub-panel, wave 0 solves its columns (one row
// per lane, multiplications by invd, broadcast reads of B), then the later columns of
// every row are updated on FP64 MFMA by the four waves.
__device__ __forceinline__ void trsm_blocked(double (*X)[CHOL_NB + 1], const double (*B)[CHOL_NB + 1],
                             const double* invd) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int p = 0; p < CHOL_NB / SUBP; ++p) {
        const int c0 = SUBP * p;
        if (wv == 0) {
            double x[SUBP];
#pragma unroll
            for (int q = 0; q < SUBP; ++q) x[q] = X[lane][c0 + q];
#pragma unroll
            for (int j = 0; j < SUBP; ++j) {
                double cv[SUBP];
#pragma unroll
                for (int q = j + 1; q < SUBP; ++q) cv[q] = B[c0 + q][c0 + j];
                const double xj = x[j] * invd[c0 + j];
                x[j] = xj;
#pragma unroll
                for (int q = j + 1; q < SUBP; ++q) x[q] = fma(-xj, cv[q], x[q]);
            }
#pragma unroll
            for (int q = 0; q < SUBP; ++q) X[lane][c0 + q] = x[q];
        }
        __syncthreads();
        // X[:, later sub-panels] -= X[:, this sub-panel] L[later rows, this sub-panel]^T
        const int first = p + 1, nt = CHOL_NB / SUBP - first;
        for (int e = wv; e < (CHOL_NB / SUBP) * nt; e += 4)
            rank16_block(X, e / nt, first + e % nt, X, e / nt, B, first + e % nt, c0, lane);
        __syncthreads();
    }
}

// Stage the nr x nc block at (r0, c0) of the n x n row-major matrix into LDS with
// coalesced loads by the whole (256-thread) workgroup, identity-padded to CHOL_NB x CHOL_NB
// when pad_identity, zero-padded otherwise.  All 16 loads of a thread are issued before
// any LDS store so their latencies overlap.  The caller synchronises.
__device__ __forceinline__ void stage_block(const double* Mg, int n, int r0, int c0, int nr, int nc,
                                            double (*B)[CHOL_NB + 1], bool pad_identity) {
    constexpr int PER = CHOL_NB * CHOL_NB / 256;
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int i = e >> 6, j = e & 63;
        v[q] = (i < nr && j < nc) ? Mg[(long long)(r0 + i) * n + c0 + j] : ((pad_identity && i == j) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q;
        B[e >> 6][e & 63] = v[q];
    }
}

__global__ void k_chol_damp(Plan p, int s, apx_lm_state* lm) {
    // one block: damping diagonal D from the diagonal of A and its maximum; clears the
    // flags of copy 0 (and, given lm, of the solve-ahead copy 1).  The LM's large solves
    // form D inside k_chol_fill instead; this kernel serves the covariance factorisation.
    __shared__ double red[4];
    if (lm && p.lmf[s].adopted) return;
    const DSub sb = p.subs[s];
    const int n = sb.n;
    const double* A = p.A + sb.a_off;
    double m = -1e308;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, A[(long long)i * n + i]);
    m = lm_wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    const double dmax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        p.Ddiag[sb.p0 + i] = fmax(A[(long long)i * n + i], APX_LM_DAMP_FLOOR * dmax);
    const int nflag = 2 * ((n + CHOL_NB - 1) / CHOL_NB);
    for (int w = 0; w < (lm ? 2 : 1); ++w) {
        const Plan q = solve_view(p, w);
        for (int i = threadIdx.x; i < nflag; i += blockDim.x) q.sflag[sb.flag_off + i] = 0;
        if (threadIdx.x == 0) {
            q.lmf[s].chol_fail = 0;
            q.lmf[s].subst_fail = 0;
            q.lmf[s].rhs_folded = 0;
        }
    }
}

// M = A + lambda D, and the working right-hand side yvec = J^T W r that the first
// factorisation attempt turns into y = L^-1 g as it goes.
// Copy 0 (blockIdx.y = 0) takes this iteration's lambda, copy 1 the solve-ahead
// lambda' = min(UP lambda, max).  The damping diagonal D (the diagonal of A, floored at
// APX_LM_DAMP_FLOOR times its maximum) is formed by every block from the diagonal of A, the
// same values k_chol_damp stores; block 0 of each copy also stores D (copy 0) and clears
// that copy's flags, which k_chol_damp does for the other solves.
__global__ void k_chol_fill(Plan p, int s, apx_lm_state* lm) {
    __shared__ double red[4];
    if (p.lmf[s].adopted) return;
    const int which = blockIdx.y;
    const Plan q = solve_view(p, which);
    const DSub sb = p.subs[s];
    const int n = sb.n;
    const double* A = p.A + sb.a_off;
    double m = -1e308;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, A[(long long)i * n + i]);
    m = lm_wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    const double dfloor = APX_LM_DAMP_FLOOR * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (blockIdx.x == 0) {
        if (which == 0)
            for (int i = threadIdx.x; i < n; i += blockDim.x)
                p.Ddiag[sb.p0 + i] = fmax(A[(long long)i * n + i], dfloor);
        const int nflag = 2 * ((n + CHOL_NB - 1) / CHOL_NB);
        for (int i = threadIdx.x; i < nflag; i += blockDim.x) q.sflag[sb.flag_off + i] = 0;
        if (threadIdx.x == 0) {
            q.lmf[s].chol_fail = 0;
            q.lmf[s].subst_fail = 0;
            q.lmf[s].rhs_folded = 0;
        }
    }
    const double lam = which ? fmin(lm[s].lambda * APX_LM_UP, APX_LM_LAMBDA_MAX) : lm[s].lambda;
    if (which && blockIdx.x == 0 && threadIdx.x == 0) p.spec[s].lam_start = lam;
    const long long nn = (long long)n * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (long long)i * n);
        double v = A[e];
        if (i == j) {
            v += lam * fmax(v, dfloor);
            q.yvec[sb.p0 + i] = p.gvec[sb.p0 + i];
        }
        q.M[sb.a_off + e] = v;
    }
}

// Block column k: every workgroup factors the diagonal block (redundantly, blocked on
// FP64 MFMA); workgroup 0 stores it and reports a failed pivot, workgroup b > 0 solves row
// block k+b (X L_kk^T = M_rk).  The factored diagonal block goes to the sub-problem's
// chol_diag slot, not into M, because the other workgroups of the launch are still reading
// that block of M (the next step copies it into M).  With fold, workgroup 0 also finishes block k of the forward
// substitution: the trailing updates have already taken sum_{c<k} L_kc y_c off the right-
// hand side, so y_k = L_kk^-1 yvec_k (64 column steps on wave 0, by readlane broadcasts).
__global__ __launch_bounds__(256) void k_chol_panel(Plan p0, int s, int kblk, int fold) {
    if (fold && p0.lmf[s].adopted) return;          // fold: the LM's solve (blockIdx.y = copy)
    const Plan p = solve_view(p0, blockIdx.y);
    __shared__ double L[CHOL_NB][CHOL_NB + 1];
    __shared__ double X[CHOL_NB][CHOL_NB + 1];
    __shared__ double col[CHOL_NB], invd[CHOL_NB];
    __shared__ int bad;
    if (p.lmf[s].chol_fail) return;
    const DSub sb = p.subs[s];
    const int n = sb.n;
    double* Mg = p.M + sb.a_off;
    const int kb = kblk * CHOL_NB;
    const int nb = min(CHOL_NB, n - kb);
    const int t = threadIdx.x;
    const int rb = kb + blockIdx.x * CHOL_NB;
    const int nr = blockIdx.x > 0 ? min(CHOL_NB, n - rb) : 0;
    stage_block(Mg, n, kb, kb, nb, nb, L, true);
    if (nr > 0) stage_block(Mg, n, rb, kb, nr, nb, X, false);
    __syncthreads();
    if (!factor_diag_blocked(L, col, invd, &bad)) {
        if (blockIdx.x == 0 && t == 0) p.lmf[s].chol_fail = 1;
        return;
    }
    if (blockIdx.x == 0) {
        double* DF = p.chol_diag + (long long)sb.diag_idx * CHOL_NB * CHOL_NB;
        for (int e = t; e < nb * nb; e += 256) {
            const int i = e / nb, j = e - (e / nb) * nb;
            if (j <= i) DF[i * CHOL_NB + j] = L[i][j];
        }
        if (fold && t < 64) {
            double* y = p.yvec + sb.p0 + kb;
            double yi = t < nb ? y[t] : 0.0;
#pragma unroll
            for (int j = 0; j < CHOL_NB; ++j) {
                const double yj = lane_bcast(yi, j) * invd[j];
                if (t == j) yi = yj;
                else if (t > j) yi = fma(-L[t][j], yj, yi);
            }
            if (t < nb) y[t] = yi;
        }
        return;
    }
    trsm_blocked(X, L, invd);
    for (int e = t; e < nr * nb; e += 256) {
        const int i = e / nb, j = e - (e / nb) * nb;
        Mg[(long long)(rb + i) * n + kb + j] = X[i][j];
    }
}

// L_ik L_jk^T for one 64 x 64 block pair on FP64 MFMA from the panels staged in LDS: each
// wave accumulates a 32 x 32 quadrant as 2 x 2 tiles of v_mfma_f64_16x16x4 (D[i][j] in
// lane j + 16 (i % 4), register i / 4 of tile [(i % 32) / 16][(j % 32) / 16]).
__device__ __forceinline__ void trail_product(const double (*Li)[CHOL_NB + 1], const double (*Lj)[CHOL_NB + 1],
                                              chol_d4 (&acc)[2][2]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wr = wv >> 1, wc = wv & 1;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[m][q] = (chol_d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < CHOL_NB; k0 += 4) {
        double av[2], bv[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) av[m] = Li[wr * 32 + m * 16 + (lane & 15)][k0 + (lane >> 4)];
#pragma unroll
        for (int q = 0; q < 2; ++q) bv[q] = Lj[wc * 32 + q * 16 + (lane & 15)][k0 + (lane >> 4)];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int q = 0; q < 2; ++q)
                acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bv[q], acc[m][q], 0, 0, 0);
    }
}

// X -= L_ik L_jk^T on the entries i < ni, j < nj (and j <= i when diag) of an LDS block;
// the caller synchronises before and after.
__device__ __forceinline__ void trail_update_lds(double (*X)[CHOL_NB + 1], const double (*Li)[CHOL_NB + 1],
                                                 const double (*Lj)[CHOL_NB + 1], int ni, int nj, bool diag) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wr = wv >> 1, wc = wv & 1;
    chol_d4 acc[2][2];
    trail_product(Li, Lj, acc);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = wr * 32 + m * 16 + (lane >> 4) + 4 * v;
                const int j = wc * 32 + q * 16 + (lane & 15);
                if (i < ni && j < nj && (!diag || j <= i)) X[i][j] -= acc[m][q][v];
            }
}

// Trailing update M_ij -= L_ik L_jk^T of one 64 x 64 block pair in global memory: both
// 64 x 64 panels are staged in LDS and multiplied on FP64 MFMA.
__device__ void chol_update_block(double* Mg, int n, int ri, int rj, int kc, bool diag,
                                  double (*Li)[CHOL_NB + 1], double (*Lj)[CHOL_NB + 1]) {
    const int ni = min(CHOL_NB, n - ri), nj = min(CHOL_NB, n - rj), nk = min(CHOL_NB, n - kc);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    stage_block(Mg, n, ri, kc, ni, nk, Li, false);
    stage_block(Mg, n, rj, kc, nj, nk, Lj, false);
    __syncthreads();
    const int wr = wv >> 1, wc = wv & 1;
    chol_d4 acc[2][2];
    trail_product(Li, Lj, acc);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = wr * 32 + m * 16 + (lane >> 4) + 4 * v;
                const int j = wc * 32 + q * 16 + (lane & 15);
                if (i < ni && j < nj && (!diag || j <= i)) Mg[(long long)(ri + i) * n + rj + j] -= acc[m][q][v];
            }
    __syncthreads();
}

// rhs rows of block i: yvec_i -= L_ik y_k (L_ik staged in Li; 4 threads per row, 16 products
// each, summed in a fixed order).  Every thread calls it.
__device__ __forceinline__ void fold_rhs(const Plan& p, const DSub& sb, int ri, int kc, const double (*Li)[CHOL_NB + 1]) {
    const int n = sb.n, ni = min(CHOL_NB, n - ri), nk = min(CHOL_NB, n - kc);
    const int r = threadIdx.x >> 2, qq = threadIdx.x & 3;
    const double* yk = p.yvec + sb.p0 + kc;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int c = 16 * qq + q;
        if (c < nk) acc = fma(Li[r][c], yk[c], acc);
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (qq == 0 && r < ni) p.yvec[sb.p0 + ri + r] -= acc;
}

// One step of the right-looking factorisation with look-ahead: the trailing update of
// block column k fused with the panel of block column k+1, so that a block of the next
// panel is factored the moment it is up to date instead of after the whole update.
// Workgroup (bi, bj), bj <= bi, owns block (k+1+bi, k+1+bj) and brings it up to date in LDS
// (X = M - L_ik L_jk^T).  Blocks right of column k+1 are written back.  Block (k+1, k+1) is
// factored (and, with fold, y_{k+1} solved); every other block of column k+1 updates its
// own copy of that diagonal block with the same arithmetic, factors it (bitwise the same
// factor), and solves its row block against it (X L_{k+1,k+1}^T = X).  The arithmetic of
// every entry is that of the separate panel and update kernels.  Since the lower blocks read
// block (k+1, k+1) of M while its owner factors it, the factor goes to the chol_diag slot and
// reaches M in the next step (whose workgroups do not read that block), or directly in the
// last step, which has no other workgroup.
__global__ __launch_bounds__(256) void k_chol_step(Plan p0, int s, int kblk, int fold) {
    __shared__ double Li[CHOL_NB][CHOL_NB + 1];     // L_ik, then the diagonal block copy
    __shared__ double Lj[CHOL_NB][CHOL_NB + 1];     // L_jk
    __shared__ double X[CHOL_NB][CHOL_NB + 1];      // the block being brought up to date
    __shared__ double col[CHOL_NB], invd[CHOL_NB];
    __shared__ int bad;
    if (fold && p0.lmf[s].adopted) return;
    const Plan p = solve_view(p0, blockIdx.y);
    if (p.lmf[s].chol_fail) return;
    const DSub sb = p.subs[s];
    const int n = sb.n;
    double* Mg = p.M + sb.a_off;
    int e = blockIdx.x, bi = 0;
    while (e >= bi + 1) { e -= bi + 1; ++bi; }
    const int bj = e;
    const int t = threadIdx.x;
    const int kc = kblk * CHOL_NB, r1 = (kblk + 1) * CHOL_NB;
    const int ri = r1 + bi * CHOL_NB, rj = r1 + bj * CHOL_NB;
    const int ni = min(CHOL_NB, n - ri), nj = min(CHOL_NB, n - rj), nk = min(CHOL_NB, n - kc);
    const bool diag = bi == bj;
    double* DF = p.chol_diag + (long long)sb.diag_idx * CHOL_NB * CHOL_NB;
    if (blockIdx.x == 0)                             // L_kk (factored by the previous launch) into M
        for (int q = t; q < nk * nk; q += 256) {
            const int i = q / nk, j = q - (q / nk) * nk;
            if (j <= i) Mg[(long long)(kc + i) * n + kc + j] = DF[i * CHOL_NB + j];
        }
    stage_block(Mg, n, ri, kc, ni, nk, Li, false);
    stage_block(Mg, n, rj, kc, nj, nk, Lj, false);
    stage_block(Mg, n, ri, rj, ni, nj, X, diag);
    __syncthreads();
    trail_update_lds(X, Li, Lj, ni, nj, diag);
    __syncthreads();
    if (fold && diag) fold_rhs(p, sb, ri, kc, Li);
    if (bj > 0) {                                    // not in the next panel: write back
        for (int q = t; q < ni * nj; q += 256) {
            const int i = q / nj, j = q - (q / nj) * nj;
            if (!diag || j <= i) Mg[(long long)(ri + i) * n + rj + j] = X[i][j];
        }
        return;
    }
    if (bi == 0) {                                   // the next diagonal block itself
        if (!factor_diag_blocked(X, col, invd, &bad)) {
            if (t == 0) p.lmf[s].chol_fail = 1;
            return;
        }
        const bool last = gridDim.x == 1;
        for (int q = t; q < ni * ni; q += 256) {
            const int i = q / ni, j = q - (q / ni) * ni;
            if (j > i) continue;
            if (last) Mg[(long long)(ri + i) * n + ri + j] = X[i][j];
            else DF[i * CHOL_NB + j] = X[i][j];
        }
        if (fold) {
            __syncthreads();                          // the rhs of block k+1 (fold_rhs above)
            if (t < 64) {
                double* y = p.yvec + sb.p0 + ri;
                double yi = t < ni ? y[t] : 0.0;
#pragma unroll
                for (int j = 0; j < CHOL_NB; ++j) {
                    const double yj = lane_bcast(yi, j) * invd[j];
                    if (t == j) yi = yj;
                    else if (t > j) yi = fma(-X[t][j], yj, yi);
                }
                if (t < ni) y[t] = yi;
            }
        }
        return;
    }
    // a lower block of the next panel: its own copy of the up-to-date diagonal block
    // (Lj holds L_{k+1,k} here, since bj = 0)
    stage_block(Mg, n, r1, r1, nj, nj, Li, true);
    __syncthreads();
    trail_update_lds(Li, Lj, Lj, nj, nj, true);
    __syncthreads();
    if (!factor_diag_blocked(Li, col, invd, &bad)) return;
    trsm_blocked(X, Li, invd);
    for (int q = t; q < ni * nj; q += 256) {
        const int i = q / nj, j = q - (q / nj) * nj;
        Mg[(long long)(ri + i) * n + rj + j] = X[i][j];
    }
}

// Retries: if the first attempt failed, raise lambda and refactor with this single
// workgroup (up to APX_LM_ATTEMPTS - 1 more times).  Otherwise mark success and exit.
// blockIdx.y = copy: copy 0 updates the LM state, copy 1 the solve-ahead record.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void k_chol_retry(Plan p0, int s, apx_lm_state* lm) {
    __shared__ double L[CHOL_NB][CHOL_NB + 1];
    __shared__ double X[CHOL_NB][CHOL_NB + 1];
    __shared__ double Li[CHOL_NB][CHOL_NB + 1], Lj[CHOL_NB][CHOL_NB + 1];
    __shared__ double col[CHOL_NB], invd[CHOL_NB];
    __shared__ int bad;
    if (p0.lmf[s].adopted) return;
    const int which = blockIdx.y;
    const Plan p = solve_view(p0, which);
    const int t = threadIdx.x;
    const double lam0 = which ? p0.spec[s].lam_start : lm[s].lambda;
    if (!p.lmf[s].chol_fail) {
        if (t == 0) {
            p.lmf[s].chol_done = 1;
            p.lmf[s].rhs_folded = 1;
            if (which) {
                p0.spec[s].lam_final = lam0;
                p0.spec[s].retries = 0;
            }
        }
        return;
    }
    const DSub sb = p.subs[s];
    const int n = sb.n;
    double* Mg = p.M + sb.a_off;
    const int nblk = (n + CHOL_NB - 1) / CHOL_NB;
    double lam = lam0;
    int done = 0, retries = 1;                      // the failed first attempt
    for (int att = 1; att < APX_LM_ATTEMPTS && !done; ++att) {
        lam = fmin(lam * APX_LM_UP, APX_LM_LAMBDA_MAX);
        const long long nn = (long long)n * n;
        for (long long e = t; e < nn; e += 256) {
            const int i = (int)(e / n), j = (int)(e - (long long)i * n);
            Mg[e] = p.A[sb.a_off + e] + (i == j ? lam * p.Ddiag[sb.p0 + i] : 0.0);
        }
        __syncthreads();
        bool ok = true;
        for (int k = 0; k < nblk && ok; ++k) {
            const int kb = k * CHOL_NB, nb = min(CHOL_NB, n - kb);
            stage_block(Mg, n, kb, kb, nb, nb, L, true);
            __syncthreads();
            if (!factor_diag_blocked(L, col, invd, &bad)) { ok = false; break; }
            for (int e = t; e < nb * nb; e += 256) {
                const int i = e / nb, j = e - (e / nb) * nb;
                if (j <= i) Mg[(long long)(kb + i) * n + kb + j] = L[i][j];
            }
            for (int r = k + 1; r < nblk; ++r) {
                const int rb = r * CHOL_NB, nr = min(CHOL_NB, n - rb);
                stage_block(Mg, n, rb, kb, nr, nb, X, false);
                __syncthreads();
                trsm_blocked(X, L, invd);
                for (int e = t; e < nr * nb; e += 256) {
                    const int i = e / nb, j = e - (e / nb) * nb;
                    Mg[(long long)(rb + i) * n + kb + j] = X[i][j];
                }
                __syncthreads();
            }
            for (int bi = k + 1; bi < nblk; ++bi)
                for (int bj = k + 1; bj <= bi; ++bj)
                    chol_update_block(Mg, n, bi * CHOL_NB, bj * CHOL_NB, kb, bi == bj, Li, Lj);
            __syncthreads();
        }
        ++retries;
        if (ok) done = 1;
    }
    if (t == 0) {
        const double lam_out = done ? lam : fmin(lam * APX_LM_UP, APX_LM_LAMBDA_MAX);
        const int retry_out = done ? retries - 1 : retries;
        if (which) {
            p0.spec[s].lam_final = lam_out;
            p0.spec[s].retries = retry_out;
        } else {
            lm[s].lambda = lam_out;
            lm[s].n_chol_retry += retry_out;
        }
        p.lmf[s].chol_done = done;
    }
}

// Forward and back substitution L y = g, L^T h = y, one workgroup per CHOL_NB block in
// one launch per direction.  Block b needs the solved blocks before it (forward) or after
// it (backward); workgroups are numbered so that those belong to workgroups with lower
// indices, which the hardware dispatches first, so a workgroup only ever waits on
// workgroups that are already running or done.  A finished block is published through a
// flag (release at device scope); a consumer prefetches the matrix block it needs, then
// waits for the flag (acquire) and folds in that block's contribution, in a fixed order.
// The waits are bounded: one that runs out raises FLAG_STALL and marks the iteration's
// step as failed instead of hanging.  y and then h overwrite yvec.
__device__ void subst_wait(Plan& p, int s, const int* f) {
    if (threadIdx.x == 0) {
        const bool never = p.wait_spin_max < 0;
        const int limit = never ? -p.wait_spin_max : p.wait_spin_max;
        int spins = 0;
        while (never || __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            if (++spins > limit) {
                atomicOr(p.sticky, FLAG_STALL);
                p.lmf[s].subst_fail = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// wave 0: make this wave's stores visible at device scope, then raise the flag
__device__ __forceinline__ void subst_publish(int* f, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) __hip_atomic_store(f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Runs only when the factor came from the fallback workgroup (the first attempt folds the
// forward substitution into its panels and updates).
__global__ __launch_bounds__(256) void k_subst_fwd(Plan p0, int s) {
    __shared__ double Lb[CHOL_NB][CHOL_NB + 1];
    __shared__ double rhs[CHOL_NB];
    if (p0.lmf[s].adopted) return;
    Plan p = solve_view(p0, blockIdx.y);
    if (!p.lmf[s].chol_done || p.lmf[s].rhs_folded) return;
    const DSub sb = p.subs[s];
    const int n = sb.n, b = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63;
    const int r0 = b * CHOL_NB, nr = min(CHOL_NB, n - r0);
    const double* L = p.M + sb.a_off;
    double* y = p.yvec + sb.p0;
    int* f = p.sflag + sb.flag_off;
    stage_block(L, n, r0, r0, nr, nr, Lb, true);
    // thread: row il of the block, 16-column quarter kq of every earlier block
    const int il = t >> 2, kq = t & 3;
    const double* Lrow = L + (long long)(r0 + min(il, nr - 1)) * n + 16 * kq;
    double lv[16], ln[16], acc = 0.0;
    if (b > 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) lv[q] = Lrow[q];
    }
    for (int c = 0; c < b; ++c) {
        if (c + 1 < b) {
#pragma unroll
            for (int q = 0; q < 16; ++q) ln[q] = Lrow[CHOL_NB * (c + 1) + q];
        }
        subst_wait(p, s, f + c);
        const double* yc = y + CHOL_NB * c + 16 * kq;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc = fma(lv[q], yc[q], acc);
#pragma unroll
        for (int q = 0; q < 16; ++q) lv[q] = ln[q];
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (kq == 0 && il < nr) rhs[il] = p.gvec[sb.p0 + r0 + il] - acc;
    __syncthreads();
    if (t < 64) {
        double a[CHOL_NB];
#pragma unroll
        for (int q = 0; q < CHOL_NB; ++q) a[q] = Lb[lane][q];
        const double rd = 1.0 / Lb[lane][lane];
        double yi = lane < nr ? rhs[lane] : 0.0;
#pragma unroll
        for (int j = 0; j < CHOL_NB; ++j) {
            const double yj = lane_bcast(yi, j) * lane_bcast(rd, j);
            if (lane == j) yi = yj;
            else if (lane > j) yi = fma(-a[j], yj, yi);
        }
        if (lane < nr) y[r0 + lane] = yi;
        subst_publish(f + b, lane);
    }
}

__global__ __launch_bounds__(256) void k_subst_bwd(Plan p0, int s) {
    __shared__ double Lb[CHOL_NB][CHOL_NB + 1];
    __shared__ double part[4][CHOL_NB];
    if (p0.lmf[s].adopted) return;
    Plan p = solve_view(p0, blockIdx.y);
    if (!p.lmf[s].chol_done) return;
    const DSub sb = p.subs[s];
    const int n = sb.n, nblk = (n + CHOL_NB - 1) / CHOL_NB;
    const int b = nblk - 1 - (int)blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int r0 = b * CHOL_NB, nr = min(CHOL_NB, n - r0);
    const double* L = p.M + sb.a_off;
    double* y = p.yvec + sb.p0;
    int* f = p.sflag + sb.flag_off + nblk;
    stage_block(L, n, r0, r0, nr, nr, Lb, true);
    // thread: column lane of this block, rows 16 wv .. 16 wv + 15 of every later block
    const int col = r0 + min(lane, nr - 1);
    auto load = [&](double (&v)[16], int c) {
        const int rc = CHOL_NB * c + 16 * wv;
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = rc + q < n ? L[(long long)(rc + q) * n + col] : 0.0;
    };
    double lv[16], ln[16], acc = 0.0;
    if (b + 1 < nblk) load(lv, nblk - 1);
    for (int c = nblk - 1; c > b; --c) {
        if (c - 1 > b) load(ln, c - 1);
        subst_wait(p, s, f + c);
        const int rc = CHOL_NB * c + 16 * wv;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (rc + q < n) acc = fma(lv[q], y[rc + q], acc);
#pragma unroll
        for (int q = 0; q < 16; ++q) lv[q] = ln[q];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (t < 64) {
        double c_[CHOL_NB];                         // c_[j] = L[r0 + j][r0 + lane]
#pragma unroll
        for (int q = 0; q < CHOL_NB; ++q) c_[q] = Lb[q][lane];
        const double rd = 1.0 / Lb[lane][lane];
        const double sum = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        double yi = lane < nr ? y[r0 + lane] - sum : 0.0;
#pragma unroll
        for (int j = CHOL_NB - 1; j >= 0; --j) {
            const double hj = lane_bcast(yi, j) * lane_bcast(rd, j);
            if (lane == j) yi = hj;
            else if (lane < j) yi = fma(-c_[j], hj, yi);
        }
        if (lane < nr) y[r0 + lane] = yi;
        subst_publish(f + b, lane);
    }
}

// h = y, pred = h^T (lambda D h + g); zeros when the factorisation or a hand-off failed.
// blockIdx.y = copy: copy 1 fills the solve-ahead record (step in its hvec copy).
__global__ __launch_bounds__(256) void k_subst_finish(Plan p0, int s, apx_lm_state* lm) {
    __shared__ double red[4];
    if (p0.lmf[s].adopted) return;
    const int which = blockIdx.y;
    const Plan p = solve_view(p0, which);
    const DSub sb = p.subs[s];
    const int n = sb.n;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const bool done = p.lmf[s].chol_done != 0 && p.lmf[s].subst_fail == 0;
    const double lam = which ? p0.spec[s].lam_final : lm[s].lambda;
    double v = 0.0;
    for (int i = t; i < n; i += 256) {
        const double h = done ? p.yvec[sb.p0 + i] : 0.0;
        p.hvec[sb.p0 + i] = h;
        v += h * (lam * p.Ddiag[sb.p0 + i] * h + p.gvec[sb.p0 + i]);
    }
    v = lm_wave_sum(v);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (t == 0) {
        const double pred = done ? ((red[0] + red[1]) + red[2]) + red[3] : 0.0;
        if (which) {
            p0.spec[s].pred = pred;
            p0.spec[s].done = done ? 1 : 0;
            p0.spec[s].valid = 1;
        } else {
            lm[s].pred = pred;
        }
        if (!done) p.lmf[s].chol_done = 0;
    }
}

// For the covariance: clear the factorisation flags of sub-problem s, and factor its M
// (filled by the caller) with the blocked kernels, no damping and no retry; a failed pivot
// leaves lmf[s].chol_fail set.
hipError_t launch_chol_reset(const Plan& p, int s, hipStream_t st) {
    hipLaunchKernelGGL(k_chol_damp, dim3(1), dim3(256), 0, st, p, s, nullptr);
    return hipGetLastError();
}

hipError_t launch_chol_blocks(const Plan& p, int s, int n, hipStream_t st) {
    const int nblk = (n + CHOL_NB - 1) / CHOL_NB;
    hipLaunchKernelGGL(k_chol_panel, dim3(nblk), dim3(256), 0, st, p, s, 0, 0);
    for (int k = 0; k + 1 < nblk; ++k) {
        const int T = nblk - k - 1;
        hipLaunchKernelGGL(k_chol_step, dim3(T * (T + 1) / 2), dim3(256), 0, st, p, s, k, 0);
    }
    return hipGetLastError();
}

hipError_t launch_chol_large(const Plan& p, int s, int n, apx_lm_state* lm, hipStream_t st) {
    const int nblk = (n + CHOL_NB - 1) / CHOL_NB;
    const long long nn = (long long)n * n;
    long long fb = (nn + 255) / 256;
    if (fb > 4096) fb = 4096;
    // y = 2 copies: this iteration's lambda and the solve-ahead lambda'
    hipLaunchKernelGGL(k_chol_fill, dim3((unsigned)fb, 2), dim3(256), 0, st, p, s, lm);
    hipLaunchKernelGGL(k_chol_panel, dim3(nblk, 2), dim3(256), 0, st, p, s, 0, 1);
    for (int k = 0; k + 1 < nblk; ++k) {
        const int T = nblk - k - 1;
        hipLaunchKernelGGL(k_chol_step, dim3(T * (T + 1) / 2, 2), dim3(256), 0, st, p, s, k, 1);
    }
    hipLaunchKernelGGL(k_chol_retry, dim3(1, 2), dim3(256), 0, st, p, s, lm);
    hipLaunchKernelGGL(k_subst_fwd, dim3(nblk, 2), dim3(256), 0, st, p, s);
    hipLaunchKernelGGL(k_subst_bwd, dim3(nblk, 2), dim3(256), 0, st, p, s);
    hipLaunchKernelGGL(k_subst_finish, dim3(1, 2), dim3(256), 0, st, p, s, lm);
    return hipGetLastError();
}

// -------------------------------------------------------------------- trial/accept
__global__ void k_lm_trial(Plan p, const double* __restrict__ theta) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= p.n_par) return;
    const int s = p.par_sub[k];
    double v = theta[k];
    if (s >= 0 && p.lmf[s].chol_done) v += p.hvec[k];
    p.theta_trial[k] = v;
}

hipError_t launch_lm_trial(const Plan& p, const double* theta, apx_lm_state* lm, hipStream_t st) {
    (void)lm;
    if (p.n_par == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lm_trial, dim3((p.n_par + 255) / 256), dim3(256), 0, st, p, theta);
    return hipGetLastError();
}

__global__ void k_lm_accept(Plan p, const double* __restrict__ chi2_trial, double* theta,
                            apx_lm_state* lm) {
    __shared__ int acc_flag;
    const int s = blockIdx.x;
    const DSub sb = p.subs[s];
    if (threadIdx.x == 0) {
        apx_lm_state st = lm[s];
        const LMFlags f = p.lmf[s];
        int accept = 0;
        if (!f.chol_done) {
            st.chi2_trial = __builtin_nan("");
            st.rho = __builtin_nan("");
        } else if (f.trial_bad) {
            st.chi2_trial = __builtin_inf();
            st.rho = -__builtin_inf();
            st.lambda = fmin(st.lambda * APX_LM_UP, APX_LM_LAMBDA_MAX);
        } else {
            const double c2t = chi2_trial[s];
            const double rho = st.pred != 0.0 ? (st.chi2 - c2t) / st.pred : __builtin_nan("");
            st.chi2_trial = c2t;
            st.rho = rho;
            if (rho > APX_LM_EPS4) {
                accept = 1;
                st.chi2 = c2t;
                st.lambda = fmax(st.lambda / APX_LM_DOWN, APX_LM_LAMBDA_MIN);
            } else {
                st.lambda = fmin(st.lambda * APX_LM_UP, APX_LM_LAMBDA_MAX);
            }
        }
        st.accepted = accept;
        st.need_jac = accept;
        if (accept) st.n_accept += 1; else st.n_reject += 1;
        lm[s] = st;
        // a step solved ahead stays usable only after a rejection of a solved trial (same A,
        // lambda raised exactly once)
        if (accept || !f.chol_done) p.spec[s].valid = 0;
        acc_flag = accept;
    }
    __syncthreads();
    if (acc_flag)
        for (int k = threadIdx.x; k < sb.n; k += blockDim.x) theta[sb.p0 + k] = p.theta_trial[sb.p0 + k];
}

hipError_t launch_lm_accept(const Plan& p, const double* chi2_trial, double* theta,
                            apx_lm_state* lm, hipStream_t st) {
    hipLaunchKernelGGL(k_lm_accept, dim3(p.n_sub), dim3(64), 0, st, p, chi2_trial, theta, lm);
    return hipGetLastError();
}

}  // namespace apx
