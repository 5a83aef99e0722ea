"""The chi^2 adjoint as a torch.autograd.Function, central finite differences of the FP64
objective against the adjoint gradient, the FP32 objective against the oracle, and the
host-forced give-up path of the damped solve's hand-off waits (all through the C ABI)."""
import numpy as np
import pytest

import oracle
from paper_2308_01957_amd import synth
from tests import cases

pytestmark = pytest.mark.gpu

_CACHE = {}


def get(name):
    if name not in _CACHE:
        _CACHE[name] = getattr(cases, name)()
    return _CACHE[name]


@pytest.fixture(scope="module")
def apx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2308_01957_amd import apx as mod
    return mod


def problem(apx, spec, **kw):
    print(f"[case] {spec['name']} {kw}", flush=True)
    P = apx.Problem(spec, **kw)
    return P, P.pixels(spec["data"]), P.pixels(spec["weight"])


def _grad_tol(spec, th, go):
    """1e-4 of max(|g_k|, the summand scale 2 sum_i |w_i r_i J_ik|) (the sky gradient
    -2 sum w r cancels, so |g_k| alone is no scale for its rounding)."""
    J = oracle.jacobian(spec, th)
    r, wv = oracle.residual(spec, th, spec["data"], spec["weight"], range(len(spec["images"])))
    return 1e-4 * np.maximum(np.abs(go), 2.0 * (np.abs(wv * r) @ np.abs(J)))


def test_chi2_autograd_backward_scales_each_sub_problem(apx):
    """Chi2Fn over six cutouts: forward equals apx_chi2; backward of sum_s c_s chi2_s with
    uneven c_s equals apx_chi2_grad times the c of each parameter's sub-problem (bitwise),
    and the oracle's gradient times c to the gradient tolerance."""
    import torch
    spec = get("few_cutouts")
    assert len(spec["subs"]) >= 2
    P, d, w = problem(apx, spec)
    th = torch.tensor(spec["theta_init"], dtype=torch.float64, device=P.device, requires_grad=True)
    c2 = apx.chi2_autograd(th, P, d, w)
    assert torch.equal(c2.detach(), P.chi2(th.detach(), d, w))
    cs = torch.tensor(np.linspace(0.5, 3.0, len(spec["subs"])) * (-1.0) ** np.arange(len(spec["subs"])),
                      dtype=torch.float64, device=P.device)
    (c2 * cs).sum().backward()
    g, _ = P.chi2_grad(th.detach(), d, w)
    per_par = cs.cpu().numpy()[P.par_sub]
    assert torch.equal(th.grad, g * torch.as_tensor(per_par, device=P.device))
    go = oracle.chi2_grad(spec, spec["theta_init"], spec["data"], spec["weight"]) * per_par
    tol = _grad_tol(spec, spec["theta_init"], go / per_par) * np.abs(per_par)
    gg = th.grad.cpu().numpy()
    assert np.all(np.abs(gg - go) <= tol), float(np.max(np.abs(gg - go) / tol))


def test_chi2_autograd_of_a_scalar_loss_with_torch_ops(apx):
    """A loss built from torch ops on the chi^2 vector (log of the total) backpropagates
    through Chi2Fn: grad = apx_chi2_grad / total chi^2."""
    import torch
    spec = get("few_cutouts")
    P, d, w = problem(apx, spec)
    th = torch.tensor(spec["theta_init"], dtype=torch.float64, device=P.device, requires_grad=True)
    torch.log(apx.chi2_autograd(th, P, d, w).sum()).backward()
    g, c2 = P.chi2_grad(th.detach(), d, w)
    ref = g / c2.sum()
    assert torch.allclose(th.grad, ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("name", ["few_cutouts", "affine_pair", "single64"])
def test_adjoint_gradient_matches_central_differences(apx, name):
    """Central differences of the FP64 objective chi^2 at h = 1e-3 of each parameter's scale
    (its value; Re for a centre coordinate) against the adjoint gradient.  Error model of
    the difference: truncation h^2 f'''/6, estimated from the same difference at h/2
    (their gap is 3/4 of it), plus the rounding of two chi^2 evaluations over 2h, plus the
    adjoint's own 1e-4 gradient tolerance.  These specs sample every pixel with the same
    nodes: under 3 x 3 nodes within 2 Re only, a pixel that crosses the 2 Re isophote
    between theta - h and theta + h switches rule, and the difference quotient measures
    that jump, not the derivative."""
    spec = get(name)
    P, d, w = problem(apx, spec)
    th = np.asarray(spec["theta_init"], np.float64)
    g = P.chi2_grad(th, d, w)[0].cpu().numpy()
    c2 = P.chi2(th, d, w).cpu().numpy()
    gtol = _grad_tol(spec, th, oracle.chi2_grad(spec, th, spec["data"], spec["weight"]))
    worst = (0.0, None)
    for k in range(spec["n_par"]):
        s = int(P.par_sub[k])
        ref = spec["scale"][k] if spec["kinds"][k] in (synth.K_X, synth.K_Y) else max(abs(th[k]), 1e-2)

        def fd(h):
            tp, tm = th.copy(), th.copy()
            tp[k] += h
            tm[k] -= h
            return (float(P.chi2(tp, d, w).cpu()[s]) - float(P.chi2(tm, d, w).cpu()[s])) / (2 * h)
        h = 1e-3 * ref
        f1, f2 = fd(h), fd(h / 2)
        trunc = 4.0 / 3.0 * abs(f1 - f2)
        rnd = 2 * 1e-13 * abs(c2[s]) / h
        tol = 2 * trunc + rnd + gtol[k]
        err = abs(f1 - g[k])
        assert err <= tol, (k, spec["kinds"][k], f1, f2, g[k], trunc, rnd, gtol[k])
        rel = err / max(abs(g[k]), 1e-3 * np.max(np.abs(g)))
        if rel > worst[0]:
            worst = (rel, spec["kinds"][k])
    print(f"[fd] {name}: worst relative FD error {worst[0]:.2e} on parameter kind {worst[1]}", flush=True)


@pytest.mark.parametrize("name", ["small_blend", "affine_pair", "large_sub"])
def test_fp32_objective_render_and_chi2_parity(apx, name):
    """The FP32 objective path (FP32 profiles and convolution, APX_OBJECTIVE_FP32): the model
    within 1e-5 |m| + 1e-7 max|m| of the oracle and chi^2 within the propagated bound."""
    spec = get(name)
    P, d, w = problem(apx, spec, objective=apx.OBJECTIVE_FP32)
    th = spec["theta_init"]
    m = P.split(P.render(th))
    c2 = P.chi2(th, d, w).cpu().numpy()
    P.check()
    bound = np.zeros(len(spec["subs"]))
    worst = 0.0
    for k, im in enumerate(spec["images"]):
        mo = oracle.model_image(spec, th, k)
        t = cases.tol_pixels(mo)
        err = np.abs(m[k].astype(np.float64) - mo)
        worst = max(worst, float(np.max(err / t)))
        assert np.all(err <= t), (k, float(np.max(err / t)))
        r = spec["data"][k].astype(np.float64) - mo
        bound[im["sub"]] += float(np.sum(spec["weight"][k].astype(np.float64) * (2 * np.abs(r) * t + t * t)))
    ref = oracle.chi2(spec, th, spec["data"], spec["weight"])
    assert np.all(np.abs(c2 - ref) <= bound + 1e-12 * np.abs(ref)), (c2, ref, bound)
    print(f"[fp32] {name}: max pixel error / tolerance {worst:.3f}", flush=True)


def test_stalled_hand_off_wait_drops_the_step_and_the_fit_goes_on(apx):
    """The blocked solve's hand-off waits forced to give up from the host (flags taken as
    never raised, 4 polls): every kernel ends, apx_problem_check reports APX_E_HIP, theta
    and lambda are those of a dropped step.  With the default bound restored the fit
    continues exactly as a fresh one does from the same start (bitwise)."""
    import torch
    spec = get("large_sub")
    assert spec["n_par"] > 64
    P, d, w = problem(apx, spec)
    th, st = P.lm_init(spec["theta_init"], d, w)
    th0 = th.clone()
    P.set_wait_limit(-4)
    P.lm_step(d, w, th, st)
    with pytest.raises(apx.ApxError) as e:
        P.check()
    assert e.value.status == apx.APX_E_HIP
    s0 = P.lm_state(st)[0]
    assert torch.equal(th, th0) and s0["n_accept"] == 0 and s0["n_reject"] == 1
    assert s0["lambda"] == oracle.LM_LAMBDA0 and np.isnan(s0["chi2_trial"])
    P.set_wait_limit(0)
    for _ in range(4):
        P.lm_step(d, w, th, st)
    P.check()
    Q, dq, wq = problem(apx, spec)
    tq, sq = Q.lm_init(spec["theta_init"], dq, wq)
    for _ in range(4):
        Q.lm_step(dq, wq, tq, sq)
    Q.check()
    assert torch.equal(th, tq)
    s1, s2 = P.lm_state(st)[0], Q.lm_state(sq)[0]
    assert s1["n_accept"] == s2["n_accept"] and s1["n_reject"] == s2["n_reject"] + 1
    assert s1["lambda"] == s2["lambda"] and s1["chi2"] == s2["chi2"]
