// Hamiltonian Monte Carlo on U = chi^2 / 2 per sub-problem (§2.5; §3.5 starts the chain at
// the LM fit with the LM covariance as the inverse mass matrix).  With a factor F of the
// covariance (F F^T = Sigma) the momenta are whitened, r = F^T p, so K = |r|^2 / 2 and the
// leapfrog step is
//     r <- r - (eps/2) F^T grad U,   theta <- theta + eps F r,   r <- r - (eps/2) F^T grad U.
// The gradient passes are the library's adjoint; these kernels are the small per-sub-problem
// vector steps around them.  Each sub-problem is its own chain with its own Metropolis test.
// The No-U-Turn sampler (the variant the paper's example runs) reuses the kick and drift;
// its tree state lives on the device (NutsDev): the host launches every step of a doubling
// and the kernels below take the tree's decisions, so a doubling needs one host read.
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
                             double* __restrict__ out, double coef, const int* skip) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.n_par || (skip && *skip)) return;
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
                             hipStream_t st, const int* skip) {
    if (p.n_par == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hmc_matvec, dim3((p.n_par + 255) / 256), dim3(256), 0, st, p, M, v, out, coef, skip);
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
// every sub-problem, +inf when any sub-problem's point left the domain (whose flags it then
// clears).  Called by all 256 threads of one workgroup; fixed-order sums; the result is
// valid in thread 0.
__device__ double nuts_energy(const Plan& p, const double* __restrict__ chi2, const double* __restrict__ r) {
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
    double h = 0.0;
    if (threadIdx.x == 0) {
        double c = 0.0;
        for (int s = 0; s < p.n_sub; ++s) c += chi2[s];
        h = 0.5 * c + 0.5 * (((red[0] + red[1]) + red[2]) + red[3]);
        if (bad || !isfinite(h)) h = __builtin_inf();
    }
    __syncthreads();
    for (int s = (int)threadIdx.x; s < p.n_sub; s += 256) p.lmf[s].trial_bad = 0;
    return h;
}

__global__ __launch_bounds__(256) void k_nuts_start(Plan p, NutsDev* d, const double* __restrict__ chi2,
                                                    const double* __restrict__ r, const double* __restrict__ u) {
    const double h = nuts_energy(p, chi2, r);
    if (threadIdx.x == 0) {
        d->H0 = h;
        d->log_slice = log(u[0]) - h;
        d->k = 1;
        d->cnt = 1;
        d->steps = 0;
        d->divergent = 0;
        d->alpha = 0.0;
        d->n_alpha = 0;
        d->stop = 0;
        d->one = 1;
        d->take = 0;
        d->accept = 0;
    }
}

__global__ void k_nuts_doubling(NutsDev* d) {
    if (threadIdx.x == 0) {
        d->k += 1;                          // the direction (the host read it from the same slot)
        d->stop = 0;
        d->alpha = 0.0;
        d->n_alpha = 0;
    }
}

__device__ __forceinline__ void nuts_copy_all(const NutsCopy& c, long long n) {
    for (int v = 0; v < c.n; ++v)
        for (long long e = threadIdx.x; e < n; e += blockDim.x) c.dst[v][e] = c.src[v][e];
}

__global__ __launch_bounds__(256) void k_nuts_copy(const int* flag, int want, NutsCopy c, long long n) {
    if (flag && *flag != want) return;
    nuts_copy_all(c, n);
}

// A leaf: point in the slice when log_slice <= -H; the doubling stops (divergent) when
// log_slice >= -H + APX_NUTS_DELTA_MAX.
__global__ __launch_bounds__(256) void k_nuts_leaf(Plan p, NutsDev* d, const double* __restrict__ chi2,
                                                   const double* __restrict__ r) {
    const double h = nuts_energy(p, chi2, r);
    if (threadIdx.x == 0 && !d->stop) {
        d->alpha += isfinite(h) ? fmin(1.0, exp(d->H0 - h)) : 0.0;
        d->n_alpha += 1;
        d->c[0] = d->log_slice <= -h ? 1 : 0;
        if (!(d->log_slice < -h + APX_NUTS_DELTA_MAX)) {
            d->divergent = 1;
            d->stop = 1;
        }
        d->steps += 1;
    }
}

__global__ __launch_bounds__(256) void k_nuts_level(NutsDev* d, int j, const int* entry, NutsCopy c, long long n) {
    const bool in = *entry != 0;
    if (threadIdx.x == 0) {
        if (in) d->c[j] = d->c[j - 1];
        d->gate[j] = d->stop ? 0 : 1;
    }
    if (in) nuts_copy_all(c, n);
}

__global__ __launch_bounds__(256) void k_nuts_merge(NutsDev* d, int j, const double* __restrict__ u, NutsCopy prop,
                                                    NutsCopy outer, long long n) {
    __shared__ int g, t;
    if (threadIdx.x == 0) {
        g = d->gate[j];
        t = 0;
        if (g) {
            const long long n1 = d->c[j], n2 = d->c[j - 1];
            t = u[d->k] * (double)(n1 + n2) < (double)n2 ? 1 : 0;
            d->k += 1;
            d->c[j] = n1 + n2;
        }
        d->take = t;
    }
    __syncthreads();
    if (t) nuts_copy_all(prop, n);
    if (g) nuts_copy_all(outer, n);
}

__global__ __launch_bounds__(256) void k_nuts_top(NutsDev* d, int depth, const double* __restrict__ u, NutsCopy edge,
                                                  NutsCopy sample, long long n) {
    __shared__ int acc;
    nuts_copy_all(edge, n);
    if (threadIdx.x == 0) {
        acc = 0;
        if (!d->stop) {
            acc = u[d->k] * (double)d->cnt < (double)d->c[depth] ? 1 : 0;
            d->k += 1;
        }
        d->cnt += d->c[depth];
        d->accept = acc;
    }
    __syncthreads();
    if (acc) nuts_copy_all(sample, n);
}

__global__ __launch_bounds__(256) void k_nuts_uturn(Plan p, const double* __restrict__ tm,
                                                    const double* __restrict__ tp, const double* __restrict__ vm,
                                                    const double* __restrict__ vp, NutsDev* d, const int* flag,
                                                    int want) {
    __shared__ double red[4][2];
    if (*flag != want) return;                // uniform across the workgroup
    double a = 0.0, b = 0.0;
    for (int j = (int)threadIdx.x; j < p.n_par; j += 256) {
        if (p.par_sub[j] < 0) continue;
        const double dd = tp[j] - tm[j];
        a = fma(dd, vm[j], a);
        b = fma(dd, vp[j], b);
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
    if (threadIdx.x == 0) {
        const double ua = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
        const double ub = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
        if (!(ua >= 0.0 && ub >= 0.0)) d->stop = 1;
    }
}

__global__ void k_clear_trial_flags(Plan p) {
    for (int s = (int)threadIdx.x; s < p.n_sub; s += blockDim.x) p.lmf[s].trial_bad = 0;
}

hipError_t launch_clear_trial_flags(const Plan& p, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_trial_flags, dim3(1), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_nuts_start(const Plan& p, NutsDev* d, const double* chi2, const double* r, const double* u,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_start, dim3(1), dim3(256), 0, st, p, d, chi2, r, u);
    return hipGetLastError();
}

hipError_t launch_nuts_doubling(NutsDev* d, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_doubling, dim3(1), dim3(64), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_nuts_copy(const int* flag, int want, const NutsCopy& c, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_copy, dim3(1), dim3(256), 0, st, flag, want, c, n);
    return hipGetLastError();
}

hipError_t launch_nuts_leaf(const Plan& p, NutsDev* d, const double* chi2, const double* r, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_leaf, dim3(1), dim3(256), 0, st, p, d, chi2, r);
    return hipGetLastError();
}

hipError_t launch_nuts_level(NutsDev* d, int j, const int* entry, const NutsCopy& c, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_level, dim3(1), dim3(256), 0, st, d, j, entry, c, n);
    return hipGetLastError();
}

hipError_t launch_nuts_merge(NutsDev* d, int j, const double* u, const NutsCopy& prop, const NutsCopy& outer,
                             long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_merge, dim3(1), dim3(256), 0, st, d, j, u, prop, outer, n);
    return hipGetLastError();
}

hipError_t launch_nuts_top(NutsDev* d, int depth, const double* u, const NutsCopy& edge, const NutsCopy& sample,
                           long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_top, dim3(1), dim3(256), 0, st, d, depth, u, edge, sample, n);
    return hipGetLastError();
}

hipError_t launch_nuts_uturn(const Plan& p, const double* tm, const double* tp, const double* vm,
                             const double* vp, NutsDev* d, const int* flag, int want, hipStream_t st) {
    hipLaunchKernelGGL(k_nuts_uturn, dim3(1), dim3(256), 0, st, p, tm, tp, vm, vp, d, flag, want);
    return hipGetLastError();
}

}  // namespace apx
