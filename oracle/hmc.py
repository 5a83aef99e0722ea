"""Hamiltonian Monte Carlo on the chi^2 posterior (TEST INFRASTRUCTURE ONLY).

Plain FP64 reference of the sampler the library runs on the GPU.  Only the test suite may
import it.  What it computes, with the passages it follows:

* Target (§2.2, §2.5): with flat priors the negative log posterior of a sub-problem is
  U(theta) = chi^2(theta) / 2 (the paper's Eq. chi2 is -log L); grad U = (d chi^2/d theta) / 2.
* Hamiltonian Monte Carlo (§2.5 and the Bayesian example of §3.5; the method of
  Duane et al. 1987 the paper cites): a momentum drawn afresh per sample, leapfrog
  integration of Hamilton's equations, and a Metropolis test on the change of the total
  energy H = U + K, which keeps detailed balance.
* Mass matrix (§3.5): the LM covariance Sigma = (J^T W J)^-1 at the fit is used
  as the inverse mass matrix, M = Sigma^-1.  With a factor F, F F^T = Sigma, and whitened
  momenta r = F^T p (r ~ N(0, I) exactly when p ~ N(0, M)), the kinetic energy is
  K = |r|^2 / 2 and the leapfrog step of size eps reads
      r <- r - (eps/2) F^T grad U(theta);  theta <- theta + eps F r;  r <- r - (eps/2) F^T grad U(theta).
* Every sub-problem is its own chain (its chi^2 involves only its parameters): its own
  energy, its own accept test, its own uniform draw.  The random numbers are inputs
  (standard normals z for the momenta, uniforms u for the tests).  A trajectory that
  leaves the model domain at any leapfrog step is rejected (its energy is infinite).
"""
from __future__ import annotations

import math

import numpy as np

from .core import chi2_images, images_of_sub, in_domain, jtwj


def covariance_factor(spec, theta, data, weight, sub: int = 0) -> np.ndarray:
    """F = L^-T for J^T W J = L L^T (lower L), so that F F^T = (J^T W J)^-1, the covariance."""
    A, _, _ = jtwj(spec, theta, data, weight, sub)
    L = np.linalg.cholesky(A)
    return np.linalg.inv(L).T


def leapfrog(theta, r, F, grad_U, step: float, n_steps: int):
    """n_steps whitened leapfrog steps (kick, drift, kick) from (theta, r); returns the end
    point and the list of positions after each drift."""
    theta = np.array(theta, dtype=np.float64)
    r = np.array(r, dtype=np.float64)
    g = grad_U(theta)
    path = []
    for _ in range(n_steps):
        r = r - 0.5 * step * (F.T @ g)
        theta = theta + step * (F @ r)
        path.append(theta.copy())
        g = grad_U(theta)
        r = r - 0.5 * step * (F.T @ g)
    return theta, r, path


def _sub_energy(spec, theta, data, weight, sub):
    return 0.5 * chi2_images(spec, theta, data, weight, images_of_sub(spec, sub))


def hmc_chain(spec, theta0, data, weight, F_blocks, step: float, n_leapfrog: int, z, u):
    """n_samples = len(z) HMC transitions from theta0.

    F_blocks[s]: the factor of sub-problem s (n_s x n_s).  z: [n_samples, n_par] standard
    normals (the whitened momenta, entries of each sub-problem's range used), u:
    [n_samples, n_sub] uniforms.  Returns (samples [n_samples, n_par], stats
    [n_samples, n_sub, 3] = accepted (0/1), H0, H1)."""
    z = np.asarray(z, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n_samples = z.shape[0]
    theta = np.array(theta0, dtype=np.float64)
    samples = np.tile(theta, (n_samples, 1))         # parameters outside every sub-problem stay
    stats = np.zeros((n_samples, len(spec["subs"]), 3))
    for s, (p0, npar) in enumerate(spec["subs"]):
        sl = slice(p0, p0 + npar)
        F = np.asarray(F_blocks[s], dtype=np.float64)

        def grad_U(t_sub, s=s, sl=sl):
            t = theta.copy()
            t[sl] = t_sub
            if not in_domain(spec, t, s):
                return np.full(t_sub.size, np.nan)
            _, g, _ = jtwj(spec, t, data, weight, s)
            return -g                                  # (d chi2 / d theta) / 2 = -J^T W r

        for i in range(n_samples):
            r0 = z[i, sl]
            U0 = _sub_energy(spec, theta, data, weight, s)
            H0 = U0 + 0.5 * float(r0 @ r0)
            tL, rL, path = leapfrog(theta[sl], r0, F, grad_U, step, n_leapfrog)
            trial = theta.copy()
            ok_dom = True
            for tp in path:
                trial[sl] = tp
                ok_dom = ok_dom and in_domain(spec, trial, s)
            trial[sl] = tL
            H1 = (_sub_energy(spec, trial, data, weight, s) + 0.5 * float(rL @ rL)) if ok_dom else math.inf
            acc = ok_dom and math.isfinite(H1) and math.log(u[i, s]) < H0 - H1
            if acc:
                theta[sl] = tL
            samples[i, sl] = theta[sl]
            stats[i, s] = (1.0 if acc else 0.0, H0, H1)
    return samples, stats
