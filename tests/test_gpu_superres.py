"""Images whose PSF has a higher resolution than their pixels (§2.1.3: the model is sampled
and convolved at the PSF's resolution, then integrated onto the pixels) through the C ABI
against the FP64 oracle: model, Jacobian, J^T W J, gradient and render VJP at U = 2 and
U = 4 (the latter under a rotated, scaled map), an image with sub-pixels beside an ordinary
one in one fit, the FP32 objective, and a converged fit."""
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


def _problem(apx, spec, **kw):
    print(f"[case] {spec['name']}", flush=True)
    P = apx.Problem(spec, **kw)
    return P, P.pixels(spec["data"]), P.pixels(spec["weight"])


def _model_and_jacobian(P, spec, th):
    for k in range(len(spec["images"])):
        m = P.split(P.render(th))[k].astype(np.float64)
        mo = oracle.model_image(spec, th, k)
        tol = cases.tol_pixels(mo)
        assert np.all(np.abs(m - mo) <= tol), (k, float(np.max(np.abs(m - mo) / tol)))
    J = P.jacobian(th).cpu().numpy().T.astype(np.float64)
    Jo = oracle.jacobian(spec, th)
    scale = np.maximum(np.max(np.abs(Jo), axis=0), 1e-30)
    err = np.max(np.abs(J - Jo), axis=0) / scale
    assert np.all(err <= 3e-5), (np.argmax(err), float(np.max(err)))
    return Jo


@pytest.mark.parametrize("U,aff", [(2, None), (4, [0.7, 1.01, -0.18, -0.4, 0.17, 0.99])], ids=["U2", "U4_affine"])
def test_superres_model_jacobian_gradient(apx, U, aff):
    spec = cases.superres(U=U, aff=aff)
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
    gr, _ = P.chi2_grad(th, d, w)
    gro = oracle.chi2_grad(spec, th, spec["data"], spec["weight"])
    r, wv = oracle.residual(spec, th, spec["data"], spec["weight"], [0])
    tol = 1e-4 * np.maximum(np.abs(gro), 2.0 * (np.abs(wv * r) @ np.abs(Jo)))
    assert np.all(np.abs(gr.cpu().numpy() - gro) <= tol), float(np.max(np.abs(gr.cpu().numpy() - gro) / tol))
    seed = np.random.default_rng(141).standard_normal(P.n_pix).astype(np.float32)
    v = P.render_vjp(th, seed).cpu().numpy()
    s64 = seed.astype(np.float64)
    vo = s64 @ Jo
    tolv = 1e-4 * np.maximum(np.abs(vo), np.abs(s64) @ np.abs(Jo))
    assert np.all(np.abs(v - vo) <= tolv), float(np.max(np.abs(v - vo) / tolv))
    P.check()


def test_superres_beside_an_ordinary_image(apx):
    """Two images of one fit: the first with U = 2 sub-pixels, the second at its own
    resolution; the Sersics are shared (tied), each image has its own sky."""
    base = cases.superres(U=2, seed=150)
    H, W = 30, 34
    P2 = 9
    psf2 = synth.moffat_psf(P2, 2.4, 3.0)
    im2 = dict(H=H, W=W, psf=psf2, affine=np.array([1.5, 1.0, 0.0, 2.0, 0.0, 1.0]),
               sky_par=base["n_par"], sky_fixed=0.0, sub=0)
    spec = dict(base)
    spec["images"] = [base["images"][0], im2]
    spec["comps"] = list(base["comps"]) + [dict(type=0, image=1, box=synth.full_window(H, W, P2),
                                                 par=list(range(q * 7, q * 7 + 7)), fixed=[0.0] * 7)
                                            for q in range(2)]
    th = np.concatenate([base["theta_true"], [0.03]])
    spec["theta_true"], spec["kinds"], spec["re_of"] = th, list(base["kinds"]) + [8], list(base["re_of"]) + [1.0]
    spec["subs"] = [(0, len(th))]
    spec["name"] = "superres_pair"
    synth._finish(spec)
    spec["noise"] = [base["noise"][0], np.random.default_rng(151).standard_normal((H, W))]
    spec["theta_init"] = synth.perturb(th, spec["kinds"], spec["re_of"], np.random.default_rng(152))
    cases.with_data(spec)
    P, d, w = _problem(apx, spec)
    _model_and_jacobian(P, spec, spec["theta_init"])
    gr, _ = P.chi2_grad(spec["theta_init"], d, w)
    gro = oracle.chi2_grad(spec, spec["theta_init"], spec["data"], spec["weight"])
    assert np.allclose(gr.cpu().numpy(), gro, rtol=1e-4, atol=1e-4 * np.abs(gro).max())
    P.check()


def test_superres_fp32_objective(apx):
    spec = cases.superres(U=2)
    P, d, w = _problem(apx, spec, objective=1)
    th = spec["theta_init"]
    m = P.split(P.render(th))[0].astype(np.float64)
    mo = oracle.model_image(spec, th, 0)
    tol = 1e-5 * np.abs(mo) + 1e-6 * np.max(np.abs(mo))
    assert np.all(np.abs(m - mo) <= tol), float(np.max(np.abs(m - mo) / tol))
    P.check()


def test_superres_rejects_other_factors(apx):
    spec = cases.superres(U=2)
    spec["images"][0]["up"] = 3
    with pytest.raises(apx.ApxError):
        apx.Problem(spec)


def test_superres_lm_converges_to_the_oracle_fit(apx):
    spec = cases.superres(U=2, fit=True)
    P, d, w = _problem(apx, spec)
    th, st = P.lm_init(spec["theta_init"], d, w)
    P.lm_run(40, d, w, th, st)
    P.check()
    tg = th.cpu().numpy()
    to, _ = oracle.lm_fit(spec, spec["theta_init"], spec["data"], spec["weight"], 40)
    A, g, _ = oracle.jtwj(spec, to, spec["data"], spec["weight"], 0)
    assert float(g @ np.linalg.solve(A, g)) < 1e-6
    cases.assert_fit_parity(spec, tg, to)
