"""Pins of the HMC oracle against closed forms (CPU only).

For a quadratic potential U = |phi|^2 / 2 in whitened coordinates the leapfrog step of size
eps is the linear map (phi, r) -> (a phi + eps r, -eps (1 - eps^2/4) phi + a r) with
a = 1 - eps^2/2 (kick-drift-kick solved by hand), so L steps are its L-th power.  A
correlated Gaussian target, a sky-only image fit (chi^2 exactly quadratic in the sky, with
variance 1 / sum w) and the model domain fix what the sampler must do; planted mistakes
(a transposed factor, a missing factor 1/2 in U) must fail them."""
import math

import numpy as np
import pytest

import oracle
import oracle.hmc
from paper_2308_01957_amd import synth


def _osc(eps, L):
    a = 1.0 - 0.5 * eps * eps
    M = np.array([[a, eps], [-eps * (1.0 - 0.25 * eps * eps), a]])
    return np.linalg.matrix_power(M, L)


def test_leapfrog_on_a_correlated_gaussian_is_the_oscillator_map():
    rng = np.random.default_rng(11)
    B = rng.standard_normal((3, 3))
    Sigma = B @ B.T + 0.5 * np.eye(3)
    mu = rng.standard_normal(3)
    P = np.linalg.inv(Sigma)
    F = np.linalg.cholesky(Sigma) @ np.linalg.qr(rng.standard_normal((3, 3)))[0]   # any F F^T = Sigma
    assert np.allclose(F @ F.T, Sigma)
    theta0, r0 = rng.standard_normal(3), rng.standard_normal(3)
    eps, L = 0.37, 9
    tL, rL, _ = oracle.leapfrog(theta0, r0, F, lambda t: P @ (t - mu), eps, L)
    phi0 = np.linalg.solve(F, theta0 - mu)
    M = _osc(eps, L)
    phiL = M[0, 0] * phi0 + M[0, 1] * r0
    rLc = M[1, 0] * phi0 + M[1, 1] * r0
    assert np.allclose(tL, mu + F @ phiL, rtol=0, atol=1e-12)
    assert np.allclose(rL, rLc, rtol=0, atol=1e-12)


def _sky_only(H=14, W=16):
    P = 5
    psf = synth.gaussian_psf(P, 1.0)
    g = [7.3, 8.1, 0.7, 0.5, 1.5, 2.5, 0.8]
    spec = {"name": "hmc_sky", "images": [dict(H=H, W=W, psf=psf, affine=synth.IDENTITY_AFFINE.copy(),
                                               sky_par=0, sky_fixed=0.0, sub=0)],
            "comps": [dict(type=0, image=0, box=synth.full_window(H, W, P), par=[-1] * 7, fixed=g)],
            "subs": [(0, 1)], "sampling": dict(s=3, rule=0, mode=0, k=0.0),
            "theta_true": [0.08], "kinds": [8], "re_of": [1.0]}
    synth._finish(spec)
    m = oracle.model_image(spec, np.array(spec["theta_true"]), 0)
    d, w = synth.make_data(m, np.random.default_rng(5).standard_normal((H, W)))
    spec["data"], spec["weight"] = [d], [w]
    M0 = oracle.model_image(spec, np.array([0.0]), 0)
    dd, ww = d.astype(np.float64), w.astype(np.float64)
    return spec, float(np.sum(ww * (dd - M0)) / np.sum(ww)), 1.0 / math.sqrt(float(np.sum(ww)))


def test_hmc_on_the_sky_only_fit_follows_the_closed_form():
    """U(s) = (s - s*)^2 / (2 sigma^2) + U*: with F = sigma every transition is the
    oscillator map, H1 - H0 is known exactly, and the Metropolis test follows u."""
    spec, s_star, sigma = _sky_only()
    F = oracle.covariance_factor(spec, np.array([0.0]), spec["data"], spec["weight"])
    assert F.shape == (1, 1) and math.isclose(F[0, 0], sigma, rel_tol=1e-10)
    eps, L, n = 1.3, 3, 12
    rng = np.random.default_rng(7)
    z = rng.standard_normal((n, 1))
    u = rng.uniform(size=(n, 1))
    theta0 = np.array([s_star + 2.5 * sigma])
    samples, stats = oracle.hmc_chain(spec, theta0, spec["data"], spec["weight"], [F], eps, L, z, u)
    M = _osc(eps, L)
    s = float(theta0[0])
    n_acc = 0
    for i in range(n):
        phi0, r0 = (s - s_star) / sigma, z[i, 0]
        phiL, rL = M[0, 0] * phi0 + M[0, 1] * r0, M[1, 0] * phi0 + M[1, 1] * r0
        dH = 0.5 * (phiL ** 2 + rL ** 2) - 0.5 * (phi0 ** 2 + r0 ** 2)
        assert math.isclose(stats[i, 0, 2] - stats[i, 0, 1], dH, rel_tol=1e-7, abs_tol=1e-9)
        acc = math.log(u[i, 0]) < -dH
        assert bool(stats[i, 0, 0]) == acc
        if acc:
            s = s_star + sigma * phiL
            n_acc += 1
        assert math.isclose(samples[i, 0], s, rel_tol=0, abs_tol=1e-10 * sigma + 1e-12)
    assert 0 < n_acc < n                 # both outcomes exercised


def test_hmc_rejects_a_trajectory_that_leaves_the_domain():
    """q driven beyond 1 by a large step: the transition is rejected and theta stays."""
    spec = synth.blend(seed_id=120, H=20, W=22, n_sersic=1, n_point=0, P=5, mode=synth.MODE_UNIFORM)
    m = oracle.model_image(spec, np.array(spec["theta_true"]), 0)
    d, w = synth.make_data(m, np.random.default_rng(3).standard_normal((20, 22)))
    spec["data"], spec["weight"] = [d], [w]
    th = np.array(spec["theta_true"])
    n = spec["n_par"]
    F = np.zeros((n, n))
    F[2, 2] = 1.0                        # move only q
    z = np.zeros((1, n))
    z[0, 2] = 5.0
    samples, stats = oracle.hmc_chain(spec, th, spec["data"], spec["weight"], [F], 1.0, 2, z, np.array([[1e-300]]))
    assert stats[0, 0, 0] == 0.0 and math.isinf(stats[0, 0, 2])
    assert np.array_equal(samples[0], th)


def test_planted_transposed_factor_fails_the_oscillator_pin(monkeypatch):
    def transposed_drift(theta, r, F, grad_U, step, n_steps):
        theta = np.array(theta, dtype=np.float64)
        r = np.array(r, dtype=np.float64)
        g = grad_U(theta)
        for _ in range(n_steps):
            r = r - 0.5 * step * (F.T @ g)
            theta = theta + step * (F.T @ r)          # planted: F^T in the drift
            g = grad_U(theta)
            r = r - 0.5 * step * (F.T @ g)
        return theta, r, []
    monkeypatch.setattr(oracle, "leapfrog", transposed_drift)
    with pytest.raises(AssertionError):
        test_leapfrog_on_a_correlated_gaussian_is_the_oscillator_map()


def test_planted_missing_half_in_the_potential_fails_the_sky_pin(monkeypatch):
    """U = chi^2 instead of chi^2 / 2 doubles the force: the sky transitions stop matching."""
    orig = oracle.hmc.jtwj

    def doubled(spec, theta, data, weight, sub=0):
        A, g, c = orig(spec, theta, data, weight, sub)
        return A, 2.0 * g, c
    monkeypatch.setattr(oracle.hmc, "jtwj", doubled)
    with pytest.raises(AssertionError):
        test_hmc_on_the_sky_only_fit_follows_the_closed_form()


# ------------------------------------------------------------------------------ NUTS
def _gauss2(rng=None):
    Sigma = np.array([[2.0, 1.2], [1.2, 1.5]])
    mu = np.array([0.7, -1.3])
    P = np.linalg.inv(Sigma)
    U = lambda t: 0.5 * float((t - mu) @ P @ (t - mu))
    G = lambda t: P @ (t - mu)
    return Sigma, mu, U, G


def _nuts_run(F, U, G, step, n, max_depth=8, seed=3, theta0=None):
    rng = np.random.default_rng(seed)
    th = np.zeros(F.shape[0]) if theta0 is None else np.array(theta0, float)
    nd = oracle.nuts_draws_per_sample(max_depth)
    out, st = [], []
    for _ in range(n):
        th, s = oracle.nuts_transition(th, rng.standard_normal(F.shape[0]), F, U, G, step, max_depth,
                                       rng.uniform(size=nd))
        out.append(th)
        st.append(s)
    return np.array(out), np.array(st)


def test_nuts_samples_a_correlated_gaussian():
    """Stationary mean and covariance of 3000 NUTS draws within 4 standard errors."""
    Sigma, mu, U, G = _gauss2()
    F = np.linalg.cholesky(Sigma)
    x, st = _nuts_run(F, U, G, 0.4, 3000)
    n = x.shape[0]
    se_mean = np.sqrt(np.diag(Sigma) / n)
    assert np.all(np.abs(x.mean(0) - mu) < 4 * se_mean), (x.mean(0), mu)
    C = np.cov(x.T)
    se_cov = np.sqrt((Sigma ** 2 + np.outer(np.diag(Sigma), np.diag(Sigma))) / n)
    assert np.all(np.abs(C - Sigma) < 4 * se_cov), (C, Sigma)
    assert np.all(st[:, 3] == 0)


def test_nuts_tree_sizes_follow_the_half_period():
    """Unit Gaussian, step 0.1: in phase space the leapfrog turns by ~0.1 rad per step, and
    the ends make a U-turn within half a period (pi, ~31 steps), so no tree is deeper than
    6 (63 steps); every doubling but the last is complete."""
    F = np.eye(1)
    x, st = _nuts_run(F, lambda t: 0.5 * float(t @ t), lambda t: t.copy(), 0.1, 300)
    depth, steps = st[:, 0], st[:, 1]
    assert depth.max() == 6 and depth.min() >= 1
    assert np.all(steps >= 2 ** (depth - 1)) and np.all(steps <= 2 ** depth - 1)
    assert np.all(st[:, 2] >= 1)


def test_nuts_divergence_keeps_the_start():
    """A step so large that the energy error passes the divergence threshold: the
    transition stops at once, is flagged divergent and returns its start."""
    F = np.eye(1)
    th0 = np.array([0.3])
    th, st = oracle.nuts_transition(th0, np.array([0.5]), F, lambda t: 0.5 * float(t @ t) * 1e8,
                                    lambda t: 1e8 * t, 1.0, 8, np.full(oracle.nuts_draws_per_sample(8), 0.9))
    assert st[3] == 1 and st[0] == 1 and np.array_equal(th, th0)


def test_planted_inverted_merge_test_fails_the_gaussian_pin(monkeypatch):
    """A merge test that never takes the new half (an inverted comparison) breaks detailed
    balance: the chain stays near its start and the moments pin fails."""
    class Stuck(oracle.hmc._Draws):
        def next(self):
            v = super().next()
            return v if self.k == 1 else 0.999
    monkeypatch.setattr(oracle.hmc, "_Draws", Stuck)
    with pytest.raises(AssertionError):
        test_nuts_samples_a_correlated_gaussian()


def _accept_stat(F, U, G, step, n, seed, max_depth=8):
    rng = np.random.default_rng(seed)
    th = np.zeros(F.shape[0])
    nd = oracle.nuts_draws_per_sample(max_depth)
    a = []
    for _ in range(n):
        th, st = oracle.nuts_transition(th, rng.standard_normal(F.shape[0]), F, U, G, step, max_depth,
                                        rng.uniform(size=nd))
        a.append(st[4] / st[5])
    return float(np.mean(a))


@pytest.mark.parametrize("step0", [0.02, 4.0])
def test_nuts_warmup_reaches_the_target_acceptance(step0):
    """Dual averaging from a far too small or far too large step: 400 warm-up transitions
    give a step whose mean acceptance statistic is near the target 0.8 (within 0.1: the
    averaged step of dual averaging lands close to, not exactly on, the target)."""
    Sigma, mu, U, G = _gauss2()
    F = np.linalg.cholesky(Sigma) * 2.0          # a mass matrix off by a factor: the step must adapt
    rng = np.random.default_rng(17)
    nd = oracle.nuts_draws_per_sample(8)
    _, step, used = oracle.nuts_warmup_core(np.zeros(2), F, U, G, step0, 8, 0.8,
                                            rng.standard_normal((400, 2)), rng.uniform(size=(400, nd)))
    assert used[0] == step0 and 0.05 < step < 2.0
    assert abs(_accept_stat(F, U, G, step, 1500, 23) - 0.8) < 0.1


def test_planted_sign_error_in_dual_averaging_fails(monkeypatch):
    def bad(step0, target):
        mu = math.log(10.0 * step0)
        hbar, log_bar, m = 0.0, 0.0, 0
        a = yield step0, step0
        while True:
            m += 1
            hbar = (1.0 - 1.0 / (m + 10.0)) * hbar - (target - a) / (m + 10.0)     # planted sign
            log_step = mu - math.sqrt(m) / 0.05 * hbar
            w = m ** -0.75
            log_bar = w * log_step + (1.0 - w) * log_bar
            a = yield math.exp(min(log_step, 50.0)), math.exp(min(log_bar, 50.0))
    monkeypatch.setattr(oracle.hmc, "dual_averaging", bad)
    with pytest.raises(AssertionError):
        test_nuts_warmup_reaches_the_target_acceptance(0.02)
