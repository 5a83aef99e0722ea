// Hamiltonian Monte Carlo on U = chi^2 / 2 per sub-problem (§2.5; §3.5 starts the chain at
// the LM fit with the LM covariance as the inverse mass matrix).  With a factor F of the
// covariance (F F^T = Sigma) the momenta are whitened, r = F^T p, so K = |r|^2 / 2 and the
// leapfrog step is
//     r <- r - (eps/2) F^T grad U,   theta <- theta + eps F r,   r <- r - (eps/2) F^T grad U.
// The gradient passes are the library's adjoint; these kernels are the small per-sub-problem
// vector steps around them.  Each sub-problem is its own chain with its own Metropolis test.
// All sums run in a fixed order (bitwise reproducible).
#include "apx_internal.h"

namespace apx {

// Ft = F^T block by block (so that both products below read their matrix by columns).
__global__ void k_hmc_transpose(Plan p, const double* __restrict__ F, double* __restrict__ Ft) {
    const DSub sb = p.subs[blockIdx.y];
    const long long n = sb.n, nn = n * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
         e += (long long)gridDim.x * blockDim.x) {
        const long long i = e / n, j = e - i * n;
        Ft[sb.a_off + j * n + i] = F[sb.a_off + e];
    }
}

// One thread per theta index j of a sub-problem (local index i): out[j] += coef * sum_k M[k][i] v[k].
// With M = F this is F^T v (the kick), with M = F^T it is F v (the drift).
__global__ void k_hmc_matvec(Plan p, const double* __restrict__ M, const double* __restrict__ v,
                             double* __restrict__ out, double coef) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.n_par) return;
    const int s = p.par_sub[j];
    if (s < 0) return;
    const DSub sb = p.subs[s];
    const int i = j - sb.p0;
    const double* col = M + sb.a_off + i;
    const double* vs = v + sb.p0;
    double acc = 0.0;
    for (int k = 0; k < sb.n; ++k) acc = fma(col[(long long)k * sb.n], vs[k], acc);
    out[j] = fma(coef, acc, out[j]);
}

__device__ __forceinline__ double sub_sq(const double* r, const DSub& sb) {
    double a = 0.0;
    for (int k = (int)threadIdx.x; k < sb.n; k += 64) a = fma(r[sb.p0 + k], r[sb.p0 + k], a);
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    return a;
}

// One wave per sub-problem: r = z_i, theta0 = theta, H0 = chi2 / 2 + |r|^2 / 2, clear the
// domain flag of the trajectory.
__global__ __launch_bounds__(64) void k_hmc_begin(Plan p, HmcIO h, long long i) {
    const int s = blockIdx.x;
    const DSub sb = p.subs[s];
    const double* z = h.z + i * p.n_par;
    for (int k = (int)threadIdx.x; k < sb.n; k += 64) {
        h.r[sb.p0 + k] = z[sb.p0 + k];
        h.theta0[sb.p0 + k] = h.theta[sb.p0 + k];
    }
    const double r2 = sub_sq(z, sb);
    if (threadIdx.x == 0) {
        h.H0[s] = 0.5 * h.chi2_cur[s] + 0.5 * r2;
        p.lmf[s].trial_bad = 0;
    }
}

// One wave per sub-problem: Metropolis test on H1 - H0; accepted -> keep theta and the end
// point's gradient and chi^2, rejected -> restore theta0.  Block n_sub copies the entries of
// theta that belong to no sub-problem.
__global__ __launch_bounds__(64) void k_hmc_accept(Plan p, HmcIO h, long long i) {
    const int s = blockIdx.x;
    double* out = h.samples + i * p.n_par;
    if (s == p.n_sub) {
        for (int j = (int)threadIdx.x; j < p.n_par; j += 64)
            if (p.par_sub[j] < 0) out[j] = h.theta[j];
        return;
    }
    const DSub sb = p.subs[s];
    const double r2 = sub_sq(h.r, sb);
    const double H0 = h.H0[s];
    const double H1 = 0.5 * h.chi2_new[s] + 0.5 * r2;
    const bool ok = p.lmf[s].trial_bad == 0 && isfinite(H1) && log(h.u[i * p.n_sub + s]) < H0 - H1;
    for (int k = (int)threadIdx.x; k < sb.n; k += 64) {
        const int j = sb.p0 + k;
        if (ok) h.grad_cur[j] = h.grad_new[j];
        else h.theta[j] = h.theta0[j];
        out[j] = h.theta[j];
    }
    if (threadIdx.x == 0) {
        if (ok) h.chi2_cur[s] = h.chi2_new[s];
        double* st = h.stats + (i * p.n_sub + s) * 3;
        st[0] = ok ? 1.0 : 0.0;
        st[1] = H0;
        st[2] = H1;
    }
}

hipError_t launch_hmc_transpose(const Plan& p, const double* F, double* Ft, hipStream_t st) {
    if (p.n_sub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hmc_transpose, dim3(16, p.n_sub), dim3(256), 0, st, p, F, Ft);
    return hipGetLastError();
}

hipError_t launch_hmc_matvec(const Plan& p, const double* M, const double* v, double* out, double coef,
                             hipStream_t st) {
    if (p.n_par == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hmc_matvec, dim3((p.n_par + 255) / 256), dim3(256), 0, st, p, M, v, out, coef);
    return hipGetLastError();
}

hipError_t launch_hmc_begin(const Plan& p, const HmcIO& h, long long i, hipStream_t st) {
    hipLaunchKernelGGL(k_hmc_begin, dim3(p.n_sub), dim3(64), 0, st, p, h, i);
    return hipGetLastError();
}

hipError_t launch_hmc_accept(const Plan& p, const HmcIO& h, long long i, hipStream_t st) {
    hipLaunchKernelGGL(k_hmc_accept, dim3(p.n_sub + 1), dim3(64), 0, st, p, h, i);
    return hipGetLastError();
}

}  // namespace apx
