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
* No-U-Turn sampling (§2.5, §3.5: the paper's example runs NUTS with the LM covariance
  as mass matrix): the slice-sampling NUTS of Hoffman & Gelman in the same whitened
  coordinates, one joint chain over all sub-problems (`nuts_transition`, `nuts_chain`).
* Every HMC sub-problem is its own chain (its chi^2 involves only its parameters): its own
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


# --------------------------------------------------------------------------- NUTS
NUTS_DELTA_MAX = 1000.0          # energy error that ends a trajectory as divergent


class _Draws:
    """The uniforms of one NUTS transition, taken strictly in the order the algorithm asks
    for them: the slice variable first, then one per doubling direction and one per merge
    of a subtree or of a doubling, as they occur."""

    def __init__(self, u):
        self.u = u
        self.k = 0

    def next(self):
        v = float(self.u[self.k])
        self.k += 1
        return v


def nuts_draws_per_sample(max_depth: int) -> int:
    """Uniforms a transition may consume: slice + directions + at most one per tree node."""
    return 1 + max_depth + (1 << (max_depth + 1))


def nuts_transition(theta0, r0, F, U, grad_U, step, max_depth, u):
    """One No-U-Turn transition (the "efficient" slice-sampling NUTS of Hoffman & Gelman,
    which the paper's Bayesian example (§3.5) runs through an external package) in whitened
    momenta: energy H = U(theta) + |r|^2 / 2, leapfrog as `leapfrog`, velocity F r.

    The trajectory doubles in a random direction per step (v = -1 if the draw < 1/2); a
    point is in the slice when log(slice) <= -H, i.e. log(u0) - H0 <= -H; a subtree stops
    when -H < log(slice) - NUTS_DELTA_MAX (divergence) or when its ends make a U-turn,
    (theta+ - theta-) . F r- < 0 or (theta+ - theta-) . F r+ < 0.  The proposal of a subtree
    is replaced by that of its second half with probability n'' / (n' + n''); that of the
    chain by a new doubling's with probability min(1, n' / n).  Returns (theta, stats) with
    stats = (depth, leapfrog steps, points in the slice, divergent, alpha, n_alpha), where
    alpha sums min(1, exp(H0 - H)) over the leaves of the last doubling and n_alpha counts
    them (the acceptance statistic of the step-size warm-up)."""
    d = _Draws(u)
    theta0 = np.asarray(theta0, dtype=np.float64)
    r0 = np.asarray(r0, dtype=np.float64)

    def H(t, r):
        e = U(t)
        return math.inf if not math.isfinite(e) else e + 0.5 * float(r @ r)

    H0 = H(theta0, r0)
    log_slice = math.log(d.next()) - H0
    counters = {"steps": 0, "divergent": 0, "alpha": 0.0, "n_alpha": 0}

    def step1(t, r, g, v):
        r = r - 0.5 * v * step * (F.T @ g)
        t = t + v * step * (F @ r)
        g = grad_U(t)
        r = r - 0.5 * v * step * (F.T @ g)
        counters["steps"] += 1
        return t, r, g

    def no_uturn(tm, rm, tp, rp):
        dt = tp - tm
        return float(dt @ (F @ rm)) >= 0.0 and float(dt @ (F @ rp)) >= 0.0

    def build(t, r, g, v, j):
        """(t-, r-, g-, t+, r+, g+, proposal, n, s) of a subtree of 2^j leapfrog steps."""
        if j == 0:
            t1, r1, g1 = step1(t, r, g, v)
            h = H(t1, r1)
            counters["alpha"] += min(1.0, math.exp(H0 - h)) if math.isfinite(h) else 0.0
            counters["n_alpha"] += 1
            n = 1 if log_slice <= -h else 0
            s = 1 if log_slice < -h + NUTS_DELTA_MAX else 0
            if not s:
                counters["divergent"] = 1
            return t1, r1, g1, t1, r1, g1, t1, n, s
        tm, rm, gm, tp, rp, gp, prop, n1, s1 = build(t, r, g, v, j - 1)
        if s1:
            if v < 0:
                tm, rm, gm, _, _, _, prop2, n2, s2 = build(tm, rm, gm, v, j - 1)
            else:
                _, _, _, tp, rp, gp, prop2, n2, s2 = build(tp, rp, gp, v, j - 1)
            if d.next() * (n1 + n2) < n2:
                prop = prop2
            s1 = s2 if no_uturn(tm, rm, tp, rp) else 0
            n1 = n1 + n2
        return tm, rm, gm, tp, rp, gp, prop, n1, s1

    g0 = grad_U(theta0)
    tm = tp = theta0
    rm = rp = r0
    gm = gp = g0
    theta = theta0
    n, s, depth = 1, 1, 0
    while s and depth < max_depth:
        v = -1.0 if d.next() < 0.5 else 1.0
        counters["alpha"], counters["n_alpha"] = 0.0, 0
        if v < 0:
            tm, rm, gm, _, _, _, prop, n1, s1 = build(tm, rm, gm, v, depth)
        else:
            _, _, _, tp, rp, gp, prop, n1, s1 = build(tp, rp, gp, v, depth)
        if s1 and d.next() * n < n1:
            theta = prop
        n += n1
        s = s1 if no_uturn(tm, rm, tp, rp) else 0
        depth += 1
    return theta, (depth, counters["steps"], n, counters["divergent"], counters["alpha"], counters["n_alpha"])


def _joint_energy(spec, data, weight):
    """U(theta) = sum of the sub-problems' chi^2 / 2 (+inf outside the domain) and its
    gradient -J^T W r per sub-problem (NaN outside the domain)."""
    from .core import chi2 as chi2_all
    subs = spec["subs"]

    def U(t):
        if not all(in_domain(spec, t, s) for s in range(len(subs))):
            return math.inf
        return 0.5 * float(np.sum(chi2_all(spec, t, data, weight)))

    def grad_U(t):
        if not all(in_domain(spec, t, s) for s in range(len(subs))):
            return np.full(t.size, np.nan)
        g = np.zeros(t.size)
        for s, (p0, npar) in enumerate(subs):
            _, gs, _ = jtwj(spec, t, data, weight, s)
            g[p0:p0 + npar] = -gs
        return g
    return U, grad_U


def nuts_warmup(spec, theta0, data, weight, F, step0: float, max_depth: int, target: float, z, u):
    """The step-size warm-up of the paper's NUTS run (§3.5: warm-up samples select the step)
    on the joint chi^2 posterior: returns (theta, adapted step, steps used)."""
    U, grad_U = _joint_energy(spec, data, weight)
    return nuts_warmup_core(theta0, F, U, grad_U, step0, max_depth, target,
                            np.asarray(z, dtype=np.float64), np.asarray(u, dtype=np.float64))


def nuts_chain(spec, theta0, data, weight, F, step: float, max_depth: int, z, u):
    """NUTS on the joint posterior of every sub-problem (one chain; U = sum chi^2 / 2) with
    the inverse-mass factor F (n_par x n_par, block diagonal per sub-problem).  z:
    [n_samples, n_par] standard normals (the momenta), u: [n_samples,
    nuts_draws_per_sample(max_depth)] uniforms.  Returns (samples, stats [n_samples, 4])."""
    theta = np.array(theta0, dtype=np.float64)
    U, grad_U = _joint_energy(spec, data, weight)
    z = np.asarray(z, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    samples = np.zeros((z.shape[0], theta.size))
    stats = np.zeros((z.shape[0], 4))
    for i in range(z.shape[0]):
        theta, st = nuts_transition(theta, z[i], F, U, grad_U, step, max_depth, u[i])
        samples[i] = theta
        stats[i] = st[:4]
    return samples, stats


# dual-averaging constants of the step-size warm-up (Hoffman & Gelman's defaults)
DA_GAMMA, DA_T0, DA_KAPPA = 0.05, 10.0, 0.75


def dual_averaging(step0: float, target: float):
    """Step sizes of the warm-up by dual averaging: with mu = log(10 step0), after warm-up
    transition m (m = 1, 2, ...) with acceptance statistic a_m = alpha / n_alpha,
    Hbar_m = (1 - 1/(m + t0)) Hbar_{m-1} + (target - a_m) / (m + t0),
    log step_m = mu - sqrt(m) / gamma Hbar_m,
    log stepbar_m = m^-kappa log step_m + (1 - m^-kappa) log stepbar_{m-1}.
    Yields (step_m, stepbar_m) as the statistics arrive (a generator fed by `send`)."""
    mu = math.log(10.0 * step0)
    hbar, log_bar, m = 0.0, 0.0, 0
    a = yield step0, step0
    while True:
        m += 1
        hbar = (1.0 - 1.0 / (m + DA_T0)) * hbar + (target - a) / (m + DA_T0)
        log_step = mu - math.sqrt(m) / DA_GAMMA * hbar
        w = m ** (-DA_KAPPA)
        log_bar = w * log_step + (1.0 - w) * log_bar
        a = yield math.exp(log_step), math.exp(log_bar)


def nuts_warmup_core(theta0, F, U, grad_U, step0, max_depth, target, z, u):
    """len(z) warm-up transitions adapting the step (dual averaging on the acceptance
    statistic of each transition's last doubling); returns (theta, the final averaged
    step, the steps used)."""
    gen = dual_averaging(step0, target)
    step, bar = next(gen)
    theta = np.asarray(theta0, dtype=np.float64)
    used = []
    for i in range(len(z)):
        used.append(step)
        theta, st = nuts_transition(theta, z[i], F, U, grad_U, step, max_depth, u[i])
        a = st[4] / st[5] if st[5] > 0 else 0.0
        step, bar = gen.send(a)
    return theta, bar, used
