// Parameter covariance at a fit: the inverse of the Gauss-Newton Hessian J^T W J of each
// sub-problem (§2.5: the inverse of the Hessian that the LM approximates gives the
// parameter uncertainties and their full covariance).  FP64 throughout.
//
// Sub-problems of at most SMALL_N parameters: one wave factors the block in LDS and every
// lane solves A x = e_c for its own column c (forward then back substitution, no barriers
// between steps).  Larger ones: the blocked Cholesky of the LM (no damping), then the
// inverse block column by block column -- workgroup j solves L Y = E_j and L^T X = Y for
// the CHOL_NB columns of block j, with the off-diagonal products on FP64 MFMA and the
// triangular 64 x 64 solves one column per lane.  A matrix that is not positive definite
// yields NaN in its whole block.
//
// Factor mode (the mass-matrix factor of the sampler): only the forward solves, Y = L^{-1},
// stored transposed, F = L^{-T}, so that F F^T = L^{-T} L^{-1} = A^{-1}.
#include "apx_internal.h"

namespace apx {

__global__ __launch_bounds__(64) void k_cov_small(Plan p, const int* __restrict__ small_subs, int nmax,
                                                  double* __restrict__ cov, int factor) {
    extern __shared__ double sm[];
    const int s = small_subs[blockIdx.x];
    const DSub sb = p.subs[s];
    const int n = sb.n, ld = nmax + 1;
    double* L = sm;                                  // factor, row-major, ld
    double* Y = sm + (long long)nmax * ld;           // Y[i * ld + c]
    const int c = threadIdx.x;
    const double* A = p.A + sb.a_off;
    double* out = cov + sb.a_off;
    if (n == 0) return;
    if (c < n)
        for (int j = 0; j < n; ++j) L[c * ld + j] = A[(long long)c * n + j];
    __syncthreads();
    bool ok = true;
    for (int k = 0; k < n; ++k) {                    // right-looking, one row per lane
        const double piv = L[k * ld + k];
        if (!(piv > 0.0) || !isfinite(piv)) { ok = false; break; }
        const double lkk = sqrt(piv);
        __syncthreads();
        if (c == k) L[k * ld + k] = lkk;
        if (c > k && c < n) L[c * ld + k] = L[c * ld + k] / lkk;
        __syncthreads();
        if (c > k && c < n) {
            const double lck = L[c * ld + k];
            for (int j = k + 1; j <= c; ++j) L[c * ld + j] -= lck * L[j * ld + k];
        }
        __syncthreads();
    }
    if (!ok) {
        if (c < n)
            for (int i = 0; i < n; ++i) out[(long long)i * n + c] = __builtin_nan("");
        return;
    }
    if (c >= n) return;
    // column c of L^{-1} (zero above row c), then of L^{-T} L^{-1}
    for (int i = 0; i < c; ++i) Y[i * ld + c] = 0.0;
    for (int i = c; i < n; ++i) {
        double t = i == c ? 1.0 : 0.0;
        for (int m = c; m < i; ++m) t -= L[i * ld + m] * Y[m * ld + c];
        Y[i * ld + c] = t / L[i * ld + i];
    }
    if (factor) {                                    // row c of F = L^{-T}
        for (int i = 0; i < n; ++i) out[(long long)c * n + i] = Y[i * ld + c];
        return;
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = Y[i * ld + c];
        for (int m = i + 1; m < n; ++m) t -= L[m * ld + i] * Y[m * ld + c];
        Y[i * ld + c] = t / L[i * ld + i];
    }
    for (int i = 0; i < n; ++i) out[(long long)i * n + c] = Y[i * ld + c];
}

hipError_t launch_cov_small(const Plan& p, const int* small_subs, int n_small, int nmax, double* cov,
                            int factor, hipStream_t st) {
    if (n_small <= 0 || nmax <= 0) return hipSuccess;
    const size_t lds = 2 * (size_t)nmax * (nmax + 1) * sizeof(double);
    hipLaunchKernelGGL(k_cov_small, dim3(n_small), dim3(64), lds, st, p, small_subs, nmax, cov, factor);
    return hipGetLastError();
}

// M = A for the undamped factorisation.
__global__ void k_cov_fill(Plan p, int s) {
    const DSub sb = p.subs[s];
    const long long nn = (long long)sb.n * sb.n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x)
        p.M[sb.a_off + e] = p.A[sb.a_off + e];
}

typedef double cov_d4 __attribute__((ext_vector_type(4)));

// Stage the nr x nc block at (r0, c0) of an n-column row-major matrix into LDS (zeros
// outside), all loads of a thread before its stores.
__device__ __forceinline__ void cov_stage(const double* G, long long ldg, int r0, int c0, int nr, int nc,
                                          double (*B)[CHOL_NB + 1]) {
    constexpr int PER = CHOL_NB * CHOL_NB / 256;
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q, i = e >> 6, j = e & 63;
        v[q] = (i < nr && j < nc) ? G[(long long)(r0 + i) * ldg + c0 + j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q;
        B[e >> 6][e & 63] = v[q];
    }
}

// T -= op(Lb) * Yb over the 64 x 64 blocks in LDS, T accumulated in acc (each wave a
// 32 x 32 quadrant as 2 x 2 MFMA tiles).  op = identity (forward) or transpose (backward).
template <bool TRANS>
__device__ __forceinline__ void cov_gemm(const double (*Lb)[CHOL_NB + 1], const double (*Yb)[CHOL_NB + 1],
                                         cov_d4 (&acc)[2][2], int lane, int wr, int wc) {
#pragma unroll
    for (int k0 = 0; k0 < CHOL_NB; k0 += 4) {
        double a[2], b[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int row = wr * 32 + m * 16 + (lane & 15), kk = k0 + (lane >> 4);
            a[m] = TRANS ? Lb[kk][row] : Lb[row][kk];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) b[q] = Yb[k0 + (lane >> 4)][wc * 32 + q * 16 + (lane & 15)];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[q], acc[m][q], 0, 0, 0);
    }
}

// Workgroup j: block column j of A^{-1}.  Forward L Y = E_j over row blocks b >= j (Y is
// zero above block j), then backward L^T X = Y over every row block from the last; Y and
// then X live in the output block column.
__global__ __launch_bounds__(256) void k_cov_cols(Plan p, int s, double* __restrict__ cov, int forward_only) {
    __shared__ double Lb[CHOL_NB][CHOL_NB + 1];
    __shared__ double Yb[CHOL_NB][CHOL_NB + 1];
    __shared__ double T[CHOL_NB][CHOL_NB + 1];
    const DSub sb = p.subs[s];
    const int n = sb.n, nblk = (n + CHOL_NB - 1) / CHOL_NB;
    const int j = blockIdx.x, c0 = j * CHOL_NB, ncl = min(CHOL_NB, n - c0);
    const double* L = p.M + sb.a_off;
    double* X = cov + sb.a_off;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, wr = wv >> 1, wc = wv & 1;
    if (p.lmf[s].chol_fail) {
        for (long long e = t; e < (long long)n * ncl; e += 256) {
            const long long i = e / ncl;
            X[i * n + c0 + (e - i * ncl)] = __builtin_nan("");
        }
        return;
    }
    auto write_T = [&](const cov_d4 (&acc)[2][2]) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    T[wr * 32 + m * 16 + (lane >> 4) + 4 * v][wc * 32 + q * 16 + (lane & 15)] -= acc[m][q][v];
    };
    for (int dir = 0; dir < (forward_only ? 1 : 2); ++dir) {
        const int b_first = dir == 0 ? j : nblk - 1, b_last = dir == 0 ? nblk : -1, step = dir == 0 ? 1 : -1;
        for (int b = b_first; b != b_last; b += step) {
            const int r0 = b * CHOL_NB, nr = min(CHOL_NB, n - r0);
            // T = right-hand side of this block: E_j (forward) or Y (backward)
            if (dir == 0) {
                for (int e = t; e < CHOL_NB * CHOL_NB; e += 256) {
                    const int i = e >> 6, c = e & 63;
                    T[i][c] = (b == j && i == c) ? 1.0 : 0.0;
                }
            } else {
                cov_stage(X, n, r0, c0, nr, ncl, T);
            }
            __syncthreads();
            // minus the products with the blocks already solved
            cov_d4 acc[2][2];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int q = 0; q < 2; ++q) acc[m][q] = (cov_d4){0.0, 0.0, 0.0, 0.0};
            const int k_first = dir == 0 ? j : b + 1, k_last = dir == 0 ? b : nblk;
            for (int k = k_first; k < k_last; ++k) {
                const int rk = k * CHOL_NB, nk = min(CHOL_NB, n - rk);
                if (dir == 0) cov_stage(L, n, r0, rk, nr, nk, Lb);    // L_bk
                else cov_stage(L, n, rk, r0, nk, nr, Lb);             // L_kb (used transposed)
                cov_stage(X, n, rk, c0, nk, ncl, Yb);
                __syncthreads();
                if (dir == 0) cov_gemm<false>(Lb, Yb, acc, lane, wr, wc);
                else cov_gemm<true>(Lb, Yb, acc, lane, wr, wc);
                __syncthreads();
            }
            write_T(acc);
            cov_stage(L, n, r0, r0, nr, nr, Lb);                      // L_bb
            __syncthreads();
            // triangular solve in place in T, one right-hand-side column per lane of wave 0
            if (wv == 0) {
                if (dir == 0) {
                    for (int m = 0; m < nr; ++m) {
                        const double xm = T[m][lane] / Lb[m][m];
                        T[m][lane] = xm;
                        for (int i = m + 1; i < nr; ++i) T[i][lane] = fma(-Lb[i][m], xm, T[i][lane]);
                    }
                } else {
                    for (int m = nr - 1; m >= 0; --m) {
                        const double xm = T[m][lane] / Lb[m][m];
                        T[m][lane] = xm;
                        for (int i = 0; i < m; ++i) T[i][lane] = fma(-Lb[m][i], xm, T[i][lane]);
                    }
                }
                if (lane < ncl)
                    for (int i = 0; i < nr; ++i) X[(long long)(r0 + i) * n + c0 + lane] = T[i][lane];
            }
            __syncthreads();
        }
        // forward: zero the rows above block j (the lower-triangular inverse is zero there)
        if (dir == 0)
            for (long long e = t; e < (long long)c0 * ncl; e += 256) {
                const long long i = e / ncl;
                X[i * n + c0 + (e - i * ncl)] = 0.0;
            }
        __syncthreads();
        __threadfence_block();
    }
}

hipError_t launch_cov_cols(const Plan& p, int s, int n, double* cov, int forward_only, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cov_cols, dim3((n + CHOL_NB - 1) / CHOL_NB), dim3(256), 0, st, p, s, cov, forward_only);
    return hipGetLastError();
}

// X <- X^T in place for the n x n block of sub-problem s (each pair swapped by one thread).
__global__ void k_cov_transpose(Plan p, int s, double* __restrict__ X) {
    const DSub sb = p.subs[s];
    const long long n = sb.n, nn = n * n;
    double* B = X + sb.a_off;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e / n, j = e - i * n;
        if (i < j) {
            const double a = B[i * n + j], b = B[j * n + i];
            B[i * n + j] = b;
            B[j * n + i] = a;
        }
    }
}

hipError_t launch_cov_transpose(const Plan& p, int s, int n, double* X, hipStream_t st) {
    const long long nn = (long long)n * n;
    long long fb = (nn + 255) / 256;
    if (fb > 4096) fb = 4096;
    if (fb < 1) return hipSuccess;
    hipLaunchKernelGGL(k_cov_transpose, dim3((unsigned)fb), dim3(256), 0, st, p, s, X);
    return hipGetLastError();
}

hipError_t launch_cov_fill(const Plan& p, int s, int n, hipStream_t st) {
    const long long nn = (long long)n * n;
    long long fb = (nn + 255) / 256;
    if (fb > 4096) fb = 4096;
    if (fb < 1) return hipSuccess;
    hipLaunchKernelGGL(k_cov_fill, dim3((unsigned)fb), dim3(256), 0, st, p, s);
    return hipGetLastError();
}

}  // namespace apx
