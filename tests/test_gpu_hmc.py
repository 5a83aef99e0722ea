"""The sampler through the C ABI against the FP64 oracle: the covariance factor used as the
inverse mass matrix (one-wave and blocked paths), HMC chains of batched sub-problems
(transitions, energies and Metropolis decisions), the stationary mean and variance of a
sky-only chain against the closed-form posterior, and the rejection of trajectories that
leave the model domain."""
import math

import numpy as np
import pytest

import oracle
from paper_2308_01957_amd import synth
from tests import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def apx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2308_01957_amd import apx as mod
    return mod


def _problem(apx, spec):
    print(f"[case] {spec['name']}", flush=True)
    P = apx.Problem(spec)
    return P, P.pixels(spec["data"]), P.pixels(spec["weight"])


@pytest.mark.parametrize("make", [cases.bright_cutouts, cases.grid_large_sub], ids=["one_wave", "blocked"])
def test_covariance_factor(apx, make):
    """F upper triangular (exact zeros below the diagonal) with F F^T the oracle's
    covariance, per sub-problem."""
    spec = make()
    P, d, w = _problem(apx, spec)
    th = spec["theta_true"]
    F, _ = P.covariance_factor(th, d, w)
    F = F.cpu().numpy()
    for s, (p0, n) in enumerate(spec["subs"]):
        Fs = F[int(P.a_offsets[s]):int(P.a_offsets[s + 1])].reshape(n, n)
        assert np.all(np.tril(Fs, -1) == 0.0)
        assert np.all(np.diag(Fs) > 0)
        Ao, _, _ = oracle.jtwj(spec, th, spec["data"], spec["weight"], s)
        Co = np.linalg.inv(Ao)
        sd = np.sqrt(np.diag(Ao))
        tolc = np.abs(Co) @ (2e-5 * np.outer(sd, sd)) @ np.abs(Co) + 1e-12 * np.abs(Co)
        assert np.all(np.abs(Fs @ Fs.T - Co) <= tolc), s
        Fo = oracle.covariance_factor(spec, th, spec["data"], spec["weight"], s)
        assert np.allclose(Fs, Fo, rtol=0, atol=1e-3 * np.max(np.abs(Fo))), s
    P.check()


def test_hmc_chains_match_the_oracle(apx):
    """Six independent cutout chains, 4 transitions of 5 leapfrog steps from the truth, the
    oracle's covariance factor as the mass matrix: the same Metropolis decisions, the
    energies, and the points within 1e-4 of each parameter's posterior width."""
    spec = cases.bright_cutouts()
    P, d, w = _problem(apx, spec)
    th0 = np.array(spec["theta_true"])
    n_sub, n_par = len(spec["subs"]), spec["n_par"]
    Fb = [oracle.covariance_factor(spec, th0, spec["data"], spec["weight"], s) for s in range(n_sub)]
    Fflat = np.concatenate([f.ravel() for f in Fb])
    rng = np.random.default_rng(2311)
    n_samples, L, eps = 4, 5, 0.45
    z = rng.standard_normal((n_samples, n_par))
    u = rng.uniform(size=(n_samples, n_sub))
    so, sto = oracle.hmc_chain(spec, th0, spec["data"], spec["weight"], Fb, eps, L, z, u)
    import torch
    th = torch.tensor(th0, dtype=torch.float64, device=P.device)
    sg, stg = P.hmc(th, d, w, Fflat, eps, L, z, u)
    P.check()
    sg, stg = sg.cpu().numpy(), stg.cpu().numpy()
    width = np.concatenate([np.sqrt(np.diag(f @ f.T)) for f in Fb])
    margin = np.abs(np.log(u) - (sto[:, :, 1] - sto[:, :, 2]))
    assert np.nanmin(margin) > 1e-3, "a Metropolis test lies within rounding of its threshold"
    assert np.array_equal(stg[:, :, 0], sto[:, :, 0])
    assert 0 < sto[:, :, 0].sum() < sto[:, :, 0].size or sto[:, :, 0].all()
    assert np.all(np.abs(stg[:, :, 1] - sto[:, :, 1]) <= 1e-7 * np.abs(sto[:, :, 1]) + 1e-9)
    fin = np.isfinite(sto[:, :, 2])                 # infinite: the trajectory left the domain
    assert np.all(stg[:, :, 0][~fin] == 0.0)
    dH1 = np.abs(stg[:, :, 2] - sto[:, :, 2])[fin]
    print("H1 diff", dH1.max(), "pos", float(np.max(np.abs(sg - so) / width[None, :])), flush=True)
    assert np.all(dH1 <= 1e-7 * np.abs(sto[:, :, 2][fin]) + 1e-4)
    assert np.all(np.abs(sg - so) <= 1e-4 * width[None, :]), float(np.max(np.abs(sg - so) / width[None, :]))
    assert np.array_equal(th.cpu().numpy(), sg[-1])


def _sky_only():
    H, W, Pz = 40, 44, 7
    psf = synth.gaussian_psf(Pz, 1.2)
    g = [20.3, 21.1, 0.7, 0.5, 1.5, 4.0, 0.8]
    spec = {"name": "hmc_sky", "images": [dict(H=H, W=W, psf=psf, affine=synth.IDENTITY_AFFINE.copy(),
                                               sky_par=0, sky_fixed=0.0, sub=0)],
            "comps": [dict(type=0, image=0, box=synth.full_window(H, W, Pz), par=[-1] * 7, fixed=g)],
            "subs": [(0, 1)], "sampling": dict(s=3, rule=0, mode=0, k=0.0),
            "theta_true": [0.08], "kinds": [8], "re_of": [1.0]}
    synth._finish(spec)
    spec["noise"] = [np.random.default_rng(93).standard_normal((H, W))]
    spec["theta_init"] = np.array([0.08])
    cases.with_data(spec)
    M0 = oracle.model_image(spec, np.array([0.0]), 0)
    dd, ww = spec["data"][0].astype(np.float64), spec["weight"][0].astype(np.float64)
    return spec, float(np.sum(ww * (dd - M0)) / np.sum(ww)), 1.0 / math.sqrt(float(np.sum(ww)))


def test_hmc_sky_only_chain_has_the_closed_form_posterior(apx):
    """chi^2 is quadratic in the sky: the posterior is N(s*, 1 / sum w).  4000 transitions
    of 4 steps of 0.4 (about a quarter period: nearly independent draws) from s* + 3 sigma;
    the mean and variance agree within 4 standard errors."""
    import torch
    spec, s_star, sigma = _sky_only()
    P, d, w = _problem(apx, spec)
    F, _ = P.covariance_factor(np.array([s_star]), d, w)
    assert math.isclose(float(F.cpu()[0]), sigma, rel_tol=1e-5)
    n = 4000
    rng = np.random.default_rng(97)
    th = torch.tensor([s_star + 3 * sigma], dtype=torch.float64, device=P.device)
    samples, stats = P.hmc(th, d, w, F, 0.4, 4, rng.standard_normal((n, 1)), rng.uniform(size=(n, 1)))
    P.check()
    x = samples.cpu().numpy()[100:, 0]
    acc = stats.cpu().numpy()[:, 0, 0].mean()
    assert acc > 0.95
    m, v = x.mean(), x.var()
    assert abs(m - s_star) < 4 * sigma / math.sqrt(x.size), (m, s_star, sigma)
    assert abs(v / sigma ** 2 - 1.0) < 4 * math.sqrt(2.0 / x.size), v / sigma ** 2


def test_hmc_rejects_trajectories_that_leave_the_domain(apx):
    """A step that drives q past 1 is rejected (theta stays) and raises no sticky flag."""
    import torch
    spec = cases.bright_cutouts()
    P, d, w = _problem(apx, spec)
    th0 = np.array(spec["theta_true"])
    n_sub, n_par = len(spec["subs"]), spec["n_par"]
    F = np.zeros(int(P.a_offsets[-1]))
    p0, n = spec["subs"][0]
    F[int(P.a_offsets[0]) + 2 * n + 2] = 1.0          # sub-problem 0: move only its q
    z = np.zeros((1, n_par))
    z[0, p0 + 2] = 5.0
    u = np.full((1, n_sub), 1e-300)
    th = torch.tensor(th0, dtype=torch.float64, device=P.device)
    samples, stats = P.hmc(th, d, w, F, 1.0, 2, z, u)
    P.check()
    st = stats.cpu().numpy()
    assert st[0, 0, 0] == 0.0
    assert np.array_equal(th.cpu().numpy()[p0:p0 + n], th0[p0:p0 + n])
    assert np.all(st[0, 1:, 0] == 1.0)              # the other chains (F = 0: no move) accept
    assert np.array_equal(samples.cpu().numpy()[0], th.cpu().numpy())


def test_hmc_argument_checks(apx):
    import torch
    spec = cases.bright_cutouts()
    P, d, w = _problem(apx, spec)
    th = torch.tensor(spec["theta_true"], dtype=torch.float64, device=P.device)
    F = np.zeros(int(P.a_offsets[-1]))
    z, u = np.zeros((1, spec["n_par"])), np.full((1, len(spec["subs"])), 0.5)
    for step, L in [(0.0, 3), (-1.0, 3), (float("nan"), 3), (0.1, 0)]:
        with pytest.raises(apx.ApxError):
            P.hmc(th, d, w, F, step, L, z, u)


def test_nuts_chain_matches_the_oracle(apx):
    """NUTS over the joint posterior of six cutouts, 3 transitions of step 0.3 from the
    truth with the oracle's covariance factor: the same trees (depth, leapfrog steps, slice
    points, divergences) and the same samples within 1e-4 of each posterior width."""
    import torch
    spec = cases.bright_cutouts()
    P, d, w = _problem(apx, spec)
    th0 = np.array(spec["theta_true"])
    n_sub, n_par = len(spec["subs"]), spec["n_par"]
    Fb = [oracle.covariance_factor(spec, th0, spec["data"], spec["weight"], s) for s in range(n_sub)]
    Fflat = np.concatenate([f.ravel() for f in Fb])
    Fd = np.zeros((n_par, n_par))
    for (p0, n), f in zip(spec["subs"], Fb):
        Fd[p0:p0 + n, p0:p0 + n] = f
    depth, n_samples, eps = 6, 3, 0.3
    rng = np.random.default_rng(4211)
    z = rng.standard_normal((n_samples, n_par))
    u = rng.uniform(size=(n_samples, oracle.nuts_draws_per_sample(depth)))
    so, sto = oracle.nuts_chain(spec, th0, spec["data"], spec["weight"], Fd, eps, depth, z, u)
    th = torch.tensor(th0, dtype=torch.float64, device=P.device)
    sg, stg = P.nuts(th, d, w, Fflat, eps, depth, z, u)
    P.check()
    sg, stg = sg.cpu().numpy(), stg.cpu().numpy()
    print("trees", stg.tolist(), flush=True)
    assert np.array_equal(stg, sto), (stg, sto)
    width = np.sqrt(np.diag(Fd @ Fd.T))
    assert np.all(np.abs(sg - so) <= 1e-4 * width[None, :]), float(np.max(np.abs(sg - so) / width[None, :]))
    assert np.array_equal(th.cpu().numpy(), sg[-1])


def test_nuts_sky_only_chain_has_the_closed_form_posterior(apx):
    """1500 NUTS transitions on the quadratic sky posterior N(s*, 1 / sum w): mean and
    variance within 4 standard errors, no divergences."""
    import torch
    spec, s_star, sigma = _sky_only()
    P, d, w = _problem(apx, spec)
    F, _ = P.covariance_factor(np.array([s_star]), d, w)
    n, depth = 1500, 6
    rng = np.random.default_rng(99)
    th = torch.tensor([s_star + 2 * sigma], dtype=torch.float64, device=P.device)
    samples, stats = P.nuts(th, d, w, F, 0.5, depth, rng.standard_normal((n, 1)),
                            rng.uniform(size=(n, oracle.nuts_draws_per_sample(depth))))
    P.check()
    x = samples.cpu().numpy()[50:, 0]
    st = stats.cpu().numpy()
    assert np.all(st[:, 3] == 0) and np.all(st[:, 0] >= 1)
    m, v = x.mean(), x.var()
    assert abs(m - s_star) < 4 * sigma / math.sqrt(x.size), (m, s_star, sigma)
    assert abs(v / sigma ** 2 - 1.0) < 4 * math.sqrt(2.0 / x.size), v / sigma ** 2


def test_nuts_argument_checks(apx):
    import torch
    spec = cases.bright_cutouts()
    P, d, w = _problem(apx, spec)
    th = torch.tensor(spec["theta_true"], dtype=torch.float64, device=P.device)
    F = np.zeros(int(P.a_offsets[-1]))
    z = np.zeros((1, spec["n_par"]))
    for step, depth in [(0.0, 3), (0.1, 0), (0.1, 11)]:
        u = np.full((1, 1 + depth + (1 << (depth + 1))), 0.5)
        with pytest.raises(apx.ApxError):
            P.nuts(th, d, w, F, step, depth, z, u)


def test_nuts_warmup_matches_the_oracle(apx):
    """30 warm-up transitions on the sky posterior from a step of 2.5 (whitened units):
    the adapted step and the chain's state agree with the oracle's dual averaging."""
    import torch
    spec, s_star, sigma = _sky_only()
    P, d, w = _problem(apx, spec)
    Fo = np.array([[sigma]])
    depth, n = 6, 30
    rng = np.random.default_rng(101)
    z = rng.standard_normal((n, 1))
    u = rng.uniform(size=(n, oracle.nuts_draws_per_sample(depth)))
    th0 = np.array([s_star + sigma])
    to, step_o, _ = oracle.nuts_warmup(spec, th0, spec["data"], spec["weight"], Fo, 2.5, depth, 0.8, z, u)
    th = torch.tensor(th0, dtype=torch.float64, device=P.device)
    step_g = P.nuts_warmup(th, d, w, Fo.ravel(), 2.5, depth, 0.8, z, u)
    P.check()
    print("steps", step_g, step_o, flush=True)
    assert math.isclose(step_g, step_o, rel_tol=1e-6), (step_g, step_o)
    assert abs(float(th.cpu()[0]) - float(to[0])) <= 1e-6 * sigma
