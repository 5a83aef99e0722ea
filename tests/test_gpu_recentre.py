"""Sub-pixel re-centring (§2.1.3: each Sersic sampled at the nearest pixel centre, convolved,
and moved back by bilinear or Lanczos interpolation) through the C ABI against the FP64
oracle, which convolves each re-centred component on its own and shifts afterwards (the
library shifts before its one convolution).  Model, Jacobian, J^T W J, gradient and render
VJP for bilinear, Lanczos-3 and Lanczos-5; two rotated images with tied shapes; the FP32
objective; FFT-mode convolution; a live PSF; a converged fit."""
import math

import numpy as np
import pytest

import oracle
from paper_2308_01957_amd import synth
from tests import cases

pytestmark = pytest.mark.gpu

BIL, LAN = synth.SHIFT_BILINEAR, synth.SHIFT_LANCZOS


@pytest.fixture(scope="module")
def apx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2308_01957_amd import apx as mod
    return mod


def _problem(apx, spec, **kw):
    print(f"[case] {spec['name']} {kw}", flush=True)
    P = apx.Problem(spec, **kw)
    return P, P.pixels(spec["data"]), P.pixels(spec["weight"])


def _model_and_jacobian(P, spec, th, jtol=3e-5):
    for k in range(len(spec["images"])):
        m = P.split(P.render(th))[k].astype(np.float64)
        mo = oracle.model_image(spec, th, k)
        tol = cases.tol_pixels(mo)
        assert np.all(np.abs(m - mo) <= tol), (k, float(np.max(np.abs(m - mo) / tol)))
    J = P.jacobian(th).cpu().numpy().T.astype(np.float64)
    Jo = oracle.jacobian(spec, th)
    scale = np.maximum(np.max(np.abs(Jo), axis=0), 1e-30)
    err = np.max(np.abs(J - Jo), axis=0) / scale
    assert np.all(err <= jtol), (int(np.argmax(err)), float(np.max(err)))
    return Jo


def _gradient(P, spec, th, d, w, Jo):
    gr, _ = P.chi2_grad(th, d, w)
    gro = oracle.chi2_grad(spec, th, spec["data"], spec["weight"])
    ks = range(len(spec["images"]))
    r, wv = oracle.residual(spec, th, spec["data"], spec["weight"], ks)
    tol = 1e-4 * np.maximum(np.abs(gro), 2.0 * (np.abs(wv * r) @ np.abs(Jo)))
    assert np.all(np.abs(gr.cpu().numpy() - gro) <= tol), float(np.max(np.abs(gr.cpu().numpy() - gro) / tol))


@pytest.mark.parametrize("method,a", [(BIL, 1), (LAN, 3), (LAN, 5)], ids=["bilinear", "lanczos3", "lanczos5"])
def test_recentred_model_jacobian_gradient(apx, method, a):
    spec = cases.recentred_blend(method, a)
    P, d, w = _problem(apx, spec)
    th = spec["theta_init"]
    Jo = _model_and_jacobian(P, spec, th)
    n = spec["n_par"]
    A, g, c2 = P.jtwj(th, d, w)
    A = A.cpu().numpy().reshape(n, n)
    Ao, go, c2o = oracle.jtwj(spec, th, spec["data"], spec["weight"], 0)
    sd = np.sqrt(np.diag(Ao))
    assert np.all(np.abs(A - Ao) <= 1e-4 * np.outer(sd, sd))
    assert np.all(np.abs(g.cpu().numpy() - go) <= 1e-4 * sd * math.sqrt(c2o))
    assert math.isclose(float(c2.cpu()[0]), c2o, rel_tol=1e-6)
    _gradient(P, spec, th, d, w, Jo)
    seed = np.random.default_rng(161).standard_normal(P.n_pix).astype(np.float32)
    v = P.render_vjp(th, seed).cpu().numpy()
    s64 = seed.astype(np.float64)
    vo = s64 @ Jo
    tolv = 1e-4 * np.maximum(np.abs(vo), np.abs(s64) @ np.abs(Jo))
    assert np.all(np.abs(v - vo) <= tolv), float(np.max(np.abs(v - vo) / tolv))
    P.check()


def test_recentred_affine_pair(apx):
    spec = cases.recentred_affine_pair()
    P, d, w = _problem(apx, spec)
    th = spec["theta_init"]
    Jo = _model_and_jacobian(P, spec, th)
    _gradient(P, spec, th, d, w, Jo)
    P.check()


def test_recentred_fp32_objective(apx):
    spec = cases.recentred_blend(BIL, 1)
    P, d, w = _problem(apx, spec, objective=1)
    th = spec["theta_init"]
    m = P.split(P.render(th))[0].astype(np.float64)
    mo = oracle.model_image(spec, th, 0)
    tol = 1e-5 * np.abs(mo) + 1e-6 * np.max(np.abs(mo))
    assert np.all(np.abs(m - mo) <= tol), float(np.max(np.abs(m - mo) / tol))
    P.check()


def test_recentred_fft_mode(apx):
    spec = cases.recentred_fft()
    P, d, w = _problem(apx, spec)
    assert P.tile_shapes(1)[4] > 0, "no Jacobian job in FFT mode"
    th = spec["theta_init"]
    Jo = _model_and_jacobian(P, spec, th, jtol=5e-5)
    _gradient(P, spec, th, d, w, Jo)
    P.check()


def test_recentred_live_psf(apx):
    spec = cases.recentred_live_psf()
    P, d, w = _problem(apx, spec)
    th = spec["theta_init"]
    Jo = _model_and_jacobian(P, spec, th)
    _gradient(P, spec, th, d, w, Jo)
    P.check()


def test_recentred_lm_converges_to_the_oracle_fit(apx):
    spec = cases.recentred_fit()
    P, d, w = _problem(apx, spec)
    th, st = P.lm_init(spec["theta_init"], d, w)
    P.lm_run(40, d, w, th, st)
    P.check()
    tg = th.cpu().numpy()
    to, _ = oracle.lm_fit(spec, spec["theta_init"], spec["data"], spec["weight"], 40)
    A, g, _ = oracle.jtwj(spec, to, spec["data"], spec["weight"], 0)
    assert float(g @ np.linalg.solve(A, g)) < 1e-6
    cases.assert_fit_parity(spec, tg, to)
