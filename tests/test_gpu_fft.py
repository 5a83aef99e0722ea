"""FFT-mode convolution (§2.1.3) through the C ABI against the FP64 oracle (which convolves
directly: both modes compute the same convolution): Jacobian columns, J^T W J, the chi^2
gradient and the render VJP with the FFT adjoint, the FP32 objective's model on FFT tiles,
the largest stamp (P = 63, 66 x 66 outputs per transform), a live PSF whose spectra follow
theta, and a converged fit."""
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


@pytest.fixture(scope="module")
def spec():
    return cases.fft_blend()


def _problem(apx, spec, **kw):
    print(f"[case] {spec['name']}", flush=True)
    P = apx.Problem(spec, **kw)
    return P, P.pixels(spec["data"]), P.pixels(spec["weight"])


def _jacobian_parity(P, spec, th):
    J = P.jacobian(th).cpu().numpy().T.astype(np.float64)
    Jo = oracle.jacobian(spec, th)
    scale = np.maximum(np.max(np.abs(Jo), axis=0), 1e-30)
    err = np.max(np.abs(J - Jo), axis=0) / scale
    assert np.all(err <= 3e-5), (np.argmax(err), float(np.max(err)))
    return Jo


def test_fft_jobs_are_planned(apx, spec):
    P, _, _ = _problem(apx, spec)
    assert P.tile_shapes(1)[4] >= 1 and P.tile_shapes(2)[4] == 1


def test_fft_jacobian_normal_equations_gradient_vjp(apx, spec):
    P, d, w = _problem(apx, spec)
    th = spec["theta_init"]
    n = spec["n_par"]
    Jo = _jacobian_parity(P, spec, th)
    A, g, _ = P.jtwj(th, d, w)
    A = A.cpu().numpy().reshape(n, n)
    Ao, go, c2o = oracle.jtwj(spec, th, spec["data"], spec["weight"], 0)
    sd = np.sqrt(np.diag(Ao))
    assert np.all(np.abs(A - Ao) <= 1e-4 * np.outer(sd, sd))
    assert np.all(np.abs(g.cpu().numpy() - go) <= 1e-4 * sd * math.sqrt(c2o))
    gr, c2 = P.chi2_grad(th, d, w)
    assert math.isclose(float(c2.cpu()[0]), c2o, rel_tol=1e-6)
    gro = oracle.chi2_grad(spec, th, spec["data"], spec["weight"])
    r, wv = oracle.residual(spec, th, spec["data"], spec["weight"], [0])
    tol = 1e-4 * np.maximum(np.abs(gro), 2.0 * (np.abs(wv * r) @ np.abs(Jo)))
    assert np.all(np.abs(gr.cpu().numpy() - gro) <= tol), float(np.max(np.abs(gr.cpu().numpy() - gro) / tol))
    seed = np.random.default_rng(131).standard_normal(P.n_pix).astype(np.float32)
    v = P.render_vjp(th, seed).cpu().numpy()
    s64 = seed.astype(np.float64)
    vo = s64 @ Jo
    tolv = 1e-4 * np.maximum(np.abs(vo), np.abs(s64) @ np.abs(Jo))
    assert np.all(np.abs(v - vo) <= tolv), float(np.max(np.abs(v - vo) / tolv))
    P.check()


def test_fft_fp32_objective_model(apx, spec):
    """FP32 objective: the model convolution itself runs on FFT tiles."""
    P, d, w = _problem(apx, spec, objective=1)
    assert P.tile_shapes(0)[4] == 1
    th = spec["theta_init"]
    m = P.split(P.render(th))[0].astype(np.float64)
    mo = oracle.model_image(spec, th, 0)
    tol = 1e-5 * np.abs(mo) + 1e-6 * np.max(np.abs(mo))
    assert np.all(np.abs(m - mo) <= tol), float(np.max(np.abs(m - mo) / tol))
    c2 = float(P.chi2(th, d, w).cpu()[0])
    assert math.isclose(c2, float(oracle.chi2(spec, th, spec["data"], spec["weight"])[0]), rel_tol=1e-4)
    P.check()


def test_fft_largest_stamp(apx):
    """P = 63: 66 x 66 outputs per transform over a ragged 100 x 93 image."""
    spec = synth.single(3, H=100, W=93, P=63)
    spec["conv_mode"] = 1
    spec["name"] = "fft_single_P63"
    cases.with_data(spec)
    P, d, w = _problem(apx, spec, objective=1)
    assert P.tile_shapes(1)[4] == 1
    th = spec["theta_init"]
    m = P.split(P.render(th))[0].astype(np.float64)
    mo = oracle.model_image(spec, th, 0)
    tol = 1e-5 * np.abs(mo) + 1e-6 * np.max(np.abs(mo))
    assert np.all(np.abs(m - mo) <= tol), float(np.max(np.abs(m - mo) / tol))
    _jacobian_parity(P, spec, th)
    P.check()


def test_fft_live_psf_follows_theta(apx):
    """Live Moffat PSF in FFT mode: the stamp spectra are recomputed at every theta; the
    Jacobian (main columns on FFT tiles, PSF columns direct) matches at two thetas."""
    spec = cases.live_psf_small()
    spec = dict(spec)
    spec["conv_mode"] = 1
    spec["name"] = "fft_live_psf"
    P, _, _ = _problem(apx, spec)
    assert P.tile_shapes(1)[4] >= 1
    th = np.array(spec["theta_init"])
    _jacobian_parity(P, spec, th)
    th2 = th.copy()
    th2[-1] *= 1.15                         # a wider PSF
    _jacobian_parity(P, spec, th2)
    P.check()


def test_fft_lm_converges_to_the_oracle_fit(apx):
    """The LM with FFT-mode Jacobians reaches the oracle's fit (its objective is the FP64
    direct convolution, so the optimum is the same point)."""
    spec = cases.fft_fit()
    P, d, w = _problem(apx, spec)
    assert P.tile_shapes(1)[4] == 1
    th, st = P.lm_init(spec["theta_init"], d, w)
    P.lm_run(40, d, w, th, st)
    P.check()
    tg = th.cpu().numpy()
    to, _ = oracle.lm_fit(spec, spec["theta_init"], spec["data"], spec["weight"], 40)
    A, g, _ = oracle.jtwj(spec, to, spec["data"], spec["weight"], 0)
    assert float(g @ np.linalg.solve(A, g)) < 1e-6
    cases.assert_fit_parity(spec, tg, to)
