// Hamiltonian Monte Carlo on U = chi^2 / 2 per sub-problem (§2.5; §3.5 starts the chain at
// the LM fit with the LM covariance as the inverse mass matrix).  With a factor F of the
// covariance (F F^T = Sigma) the momenta are whitened, r = F^T p, so K = |r|^2 / 2 and the
// leapfrog step is
//     r <- r - (eps/2) F^T grad U,   theta <- theta + eps F r,   r <- r - (eps/2) F^T grad U.
// The gradient passes are the library's adjoint; these kernels are the small per-sub-problem
// vector steps around them.  Each sub-problem is its own chain with its own Metropolis test.
// The No-U-Turn sampler (the variant the paper's example runs) reuses the kick and drift;
// its tree logic runs on the host between the energy and U-turn reductions below.
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

// NUTS energy of the joint chain: H = sum_s chi2_s / 2 + |r|^2 / 2 over the entries of
// every sub-problem, +inf when any sub-problem's point left the domain (whose flags it
// then clears).  One workgroup, fixed-order sums; the result goes to out[0].
__global__ __launch_bounds__(256) void k_nuts_energy(Plan p, const double* __restrict__ chi2,
                                                     const double* __restrict__ r, double* out) {
    __shared__ double red[4];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    double a = 0.0;
    for (int j = (int)threadIdx.x; j < p.n_par; j += 256)
        if (p.par_sub[j] >= 0) a = fma(r[j], r[j], a);
    for (int s = (int)threadIdx.x; s < p.n_sub; s += 256)
        if (p.lmf[s].trial_bad) atomicOr(&bad, 1);
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double c = 0.0;
        for (int s = 0; s < p.n_sub; ++s) c += chi2[s];
        const double h = 0.5 * c + 0.5 * (((red[0] + red[1]) + red[2]) + red[3]);
        out[0] = bad || !isfinite(h) ? __builtin_inf() : h;
    }
    __syncthreads();
    for (int s = (int)threadIdx.x; s < p.n_sub; s += 256) p.lmf[s].trial_bad = 0;
}

// U-turn products of a trajectory with ends (tm, rm) and (tp, rp): out[0] = (tp - tm) . vm,
// out[1] = (tp - tm) . vp, with the velocities vm = F rm, vp = F rp given.
__global__ __launch_bounds__(256) void k_nuts_uturn(Plan p, const double* __restrict__ tm,
                                                    const double* __restrict__ tp, const double* __restrict__ vm,
                                                    const double* __restrict__ vp, double* out) {
    __shared__ double red[4][2];
    double a = 0.0, b = 0.0;
    for (int j = (int)threadIdx.x; j < p.n_par; j += 256) {
        if (p.par_sub[j] < 0) continue;
        const double d = tp[j] - tm[j];
        a = fma(d, vm[j], a);
        b = fma(d, vp[j], b);
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = a;
        red[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    if (threadIdx.x < 2) out[threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                           red[3][threadIdx.x];
}

__global__ void k_clear_trial_flags(Plan p) {
    for (int s = (int)threadIdx.x; s < p.n_sub; s += blockDim.x) p.lmf[s].trial_bad = 0;
}

hipError_t launch_clear_trial_flags(const Plan& p, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_trial_flags, dim3(1), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_nuts_energy(const Plan& p, const double* chi2, const double* r, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_energy, dim3(1), dim3(256), 0, st, p, chi2, r, out);
    return hipGetLastError();
}

hipError_t launch_nuts_uturn(const Plan& p, const double* tm, const double* tp, const double* vm,
                             const double* vp, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_uturn, dim3(1), dim3(256), 0, st, p, tm, tp, vm, vp, out);
    return hipGetLastError();
}

}  // namespace apx
