"""Adaptive sub-pixel integration (§2.1.2) through the C ABI against the FP64 oracle: the
model, the Jacobian with the choices held, J^T W J, the chi^2 gradient and the render VJP,
bitwise reproducibility despite the refine list's run-to-run order, two images under
rotated pixel->sky maps, the FP32 objective, and a converged LM fit.

The choices (centre, 3 x 3, refined sub-pixels, 7 x 7 sub-sub-pixels) are taken in FP64 on
both sides; a choice could differ only where an estimate lies within rounding of its
budget, which these seeded inputs do not hit."""
import math

import numpy as np
import pytest

import oracle
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
    return cases.adaptive_small(1e-3)


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


def test_adaptive_model_and_jacobian(apx, spec):
    P, d, w = _problem(apx, spec)
    th = spec["theta_init"]
    m = P.split(P.render(th))[0].astype(np.float64)
    mo = oracle.model_image(spec, th, 0)
    tol = cases.tol_pixels(mo)
    assert np.all(np.abs(m - mo) <= tol), float(np.max(np.abs(m - mo) / tol))
    _jacobian_parity(P, spec, th)
    c2 = float(P.chi2(th, d, w).cpu()[0])
    assert math.isclose(c2, float(oracle.chi2(spec, th, spec["data"], spec["weight"])[0]), rel_tol=1e-6)
    P.check()


def test_adaptive_normal_equations_gradient_vjp(apx, spec):
    P, d, w = _problem(apx, spec)
    th = spec["theta_init"]
    n = spec["n_par"]
    A, g, _ = P.jtwj(th, d, w)
    A = A.cpu().numpy().reshape(n, n)
    Ao, go, c2o = oracle.jtwj(spec, th, spec["data"], spec["weight"], 0)
    sd = np.sqrt(np.diag(Ao))
    assert np.all(np.abs(A - Ao) <= 1e-4 * np.outer(sd, sd))
    assert np.all(np.abs(g.cpu().numpy() - go) <= 1e-4 * sd * math.sqrt(c2o))
    gr, _ = P.chi2_grad(th, d, w)
    gro = oracle.chi2_grad(spec, th, spec["data"], spec["weight"])
    Jo = oracle.jacobian(spec, th)
    r, wv = oracle.residual(spec, th, spec["data"], spec["weight"], [0])
    tol = 1e-4 * np.maximum(np.abs(gro), 2.0 * (np.abs(wv * r) @ np.abs(Jo)))
    assert np.all(np.abs(gr.cpu().numpy() - gro) <= tol), float(np.max(np.abs(gr.cpu().numpy() - gro) / tol))
    seed = np.random.default_rng(83).standard_normal(P.n_pix).astype(np.float32)
    v = P.render_vjp(th, seed).cpu().numpy()
    s64 = seed.astype(np.float64)
    vo = s64 @ Jo
    tolv = 1e-4 * np.maximum(np.abs(vo), np.abs(s64) @ np.abs(Jo))
    assert np.all(np.abs(v - vo) <= tolv), float(np.max(np.abs(v - vo) / tolv))
    P.check()


def test_adaptive_results_are_bitwise_reproducible(apx, spec):
    """The refine list is appended to atomically; the model, Jacobian and gradient still
    come out bit for bit the same on every call."""
    P, d, w = _problem(apx, spec)
    th = spec["theta_init"]
    m1, m2 = P.render(th).cpu().numpy(), P.render(th).cpu().numpy()
    assert np.array_equal(m1.view(np.uint32), m2.view(np.uint32))
    J1, J2 = P.jacobian(th).cpu().numpy(), P.jacobian(th).cpu().numpy()
    assert np.array_equal(J1.view(np.uint32), J2.view(np.uint32))
    g1 = P.chi2_grad(th, d, w)[0].cpu().numpy()
    g2 = P.chi2_grad(th, d, w)[0].cpu().numpy()
    assert np.array_equal(g1.view(np.uint64), g2.view(np.uint64))
    P.check()


def test_adaptive_affine_pair(apx):
    """Two images under rotated / scaled pixel->sky maps, adaptive with tol = 1e-3."""
    spec = cases.affine_pair()
    spec["sampling"] = dict(s=3, rule=0, mode=2, k=1e-3)
    spec["name"] = "affine_pair_adaptive"
    P, _, _ = _problem(apx, spec)
    th = spec["theta_init"]
    ms = P.split(P.render(th))
    for k in range(2):
        mo = oracle.model_image(spec, th, k)
        tol = cases.tol_pixels(mo)
        assert np.all(np.abs(ms[k].astype(np.float64) - mo) <= tol), (k, float(np.max(np.abs(ms[k] - mo) / tol)))
    _jacobian_parity(P, spec, th)
    P.check()


def test_adaptive_fp32_objective(apx, spec):
    """The FP32 objective path (FP32 convolution) over the same FP64 pixel integrals."""
    P, d, w = _problem(apx, spec, objective=1)
    th = spec["theta_init"]
    m = P.split(P.render(th))[0].astype(np.float64)
    mo = oracle.model_image(spec, th, 0)
    tol = 1e-5 * np.abs(mo) + 1e-6 * np.max(np.abs(mo))
    assert np.all(np.abs(m - mo) <= tol), float(np.max(np.abs(m - mo) / tol))
    P.check()


def test_adaptive_lm_converges_to_the_oracle_fit(apx):
    """Both fits converge (oracle Newton decrement < 1e-6) from the perturbed start and
    agree to 1e-6 (|theta| + scale)."""
    spec = cases.adaptive_fit()
    P, d, w = _problem(apx, spec)
    th, st = P.lm_init(spec["theta_init"], d, w)
    P.lm_run(40, d, w, th, st)
    P.check()
    tg = th.cpu().numpy()
    to, _ = oracle.lm_fit(spec, spec["theta_init"], spec["data"], spec["weight"], 40)
    A, g, _ = oracle.jtwj(spec, to, spec["data"], spec["weight"], 0)
    assert float(g @ np.linalg.solve(A, g)) < 1e-6
    cases.assert_fit_parity(spec, tg, to)
