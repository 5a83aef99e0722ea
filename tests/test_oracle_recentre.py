"""Pins of the oracle's sub-pixel re-centring (§2.1.3) against things other than itself
(CPU only): closed forms of the interpolation kernels, the identity at zero offset, the
point-source model the bilinear shift of a point must reproduce, the commutation of the
shift with the convolution, flux conservation, the interpolation accuracy on a smooth
profile and finite differences of the model for the Jacobian."""
import math

import numpy as np
import pytest
import scipy.signal

import oracle
from paper_2308_01957_amd import synth

BIL, LAN = oracle.SHIFT_BILINEAR, oracle.SHIFT_LANCZOS


def _rot_affine(phi, sc, H, W, tx=0.0, ty=0.0):
    a1, a2 = sc * math.cos(phi), -sc * math.sin(phi)
    a4, a5 = sc * math.sin(phi), sc * math.cos(phi)
    pcx, pcy = (W - 1) / 2, (H - 1) / 2
    return np.array([pcx - a1 * pcx - a2 * pcy + tx, a1, a2, pcy - a4 * pcx - a5 * pcy + ty, a4, a5])


def _spec(H, W, K, comps, theta, aff=None, s=3, rule=0, mode=0, k=0.0, shift=None, sky=0.0):
    spec = {
        "images": [dict(H=H, W=W, psf=np.asarray(K, np.float32),
                        affine=synth.IDENTITY_AFFINE.copy() if aff is None else np.asarray(aff),
                        sky_par=-1, sky_fixed=sky, sub=0)],
        "comps": comps, "subs": [(0, len(theta))], "n_par": len(theta),
        "sampling": dict(s=s, rule=rule, mode=mode, k=k),
    }
    if shift is not None:
        spec["recentre"] = {"method": shift[0], "a": shift[1]}
    return spec, np.asarray(theta, np.float64)


def _free_sersic(prm, box):
    """A Sersic whose 7 parameters are theta[0:7]."""
    return dict(type=oracle.SERSIC, image=0, box=box, par=list(range(7)), fixed=[0.0] * 7), list(prm)


def _asym(P, seed):
    return synth.asymmetric_psf(P, np.random.default_rng(seed))


# ----------------------------------------------------------------- kernel closed forms
def test_lanczos_closed_forms():
    # L(0) = 1; zero at the other integers inside the window; sinc(1/2) sinc(1/(2a)) at 1/2
    for a in (2, 3, 4, 5):
        assert oracle.lanczos(0.0, a) == 1.0
        for t in range(1, a):
            assert abs(oracle.lanczos(float(t), a)) < 1e-16
            assert abs(oracle.lanczos(-float(t), a)) < 1e-16
        assert oracle.lanczos(a + 0.25, a) == 0.0 and oracle.lanczos(-a, a) == 0.0
    assert oracle.lanczos(0.5, 3) == pytest.approx(6.0 / math.pi ** 2, rel=1e-15)
    assert oracle.lanczos(0.5, 2) == pytest.approx(4.0 * math.sqrt(2.0) / math.pi ** 2, rel=1e-15)
    assert oracle.lanczos(1.5, 3) == pytest.approx(-4.0 / (3.0 * math.pi ** 2), rel=1e-14)  # sinc(3/2) sinc(1/2)
    # the derivative against central differences of the window itself
    x = np.linspace(-2.9, 2.9, 41)
    h = 1e-6
    fd = (oracle.lanczos(x + h, 3) - oracle.lanczos(x - h, 3)) / (2 * h)
    assert np.max(np.abs(fd - oracle.lanczos_prime(x, 3))) < 1e-8


@pytest.mark.parametrize("delta", [-0.5, -0.31, -1e-9, 0.0, 0.17, 0.4999])
def test_taps(delta):
    w, dw = oracle.shift_taps(delta, BIL, 1)
    assert np.allclose(w, [max(0.0, -delta), 1.0 - abs(delta), max(0.0, delta)], rtol=0, atol=1e-16)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    for a in (2, 3, 5):
        w, dw = oracle.shift_taps(delta, LAN, a)
        t = np.arange(-a, a + 1)
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        # zero shift is the identity (the window vanishes at the other integers)
        if delta == 0.0:
            assert np.allclose(w, (t == 0).astype(float), rtol=0, atol=1e-16)
        if abs(delta) < 0.5:
            h = 1e-7
            fd = (oracle.shift_taps(delta + h, LAN, a)[0] - oracle.shift_taps(delta - h, LAN, a)[0]) / (2 * h)
            assert np.max(np.abs(fd - dw)) < 1e-7


# --------------------------------------------------------------------- model-level pins
@pytest.mark.parametrize("shift", [(BIL, 1), (LAN, 2), (LAN, 3), (LAN, 5)])
def test_centred_component_is_unchanged(shift):
    """A centre exactly on a pixel centre needs no shift: the re-centred model is the plain one."""
    H, W, P = 31, 27, 7
    aff = _rot_affine(0.7, 1.02, H, W, 0.3, -0.2)
    ux, uy = aff[0] + aff[1] * 12 + aff[2] * 15, aff[3] + aff[4] * 12 + aff[5] * 15
    comp, prm = _free_sersic([ux, uy, 0.6, 0.9, 1.5, 3.0, 0.2], synth.full_window(H, W, P))
    plain, th = _spec(H, W, _asym(P, 1), [comp], prm, aff=aff, mode=1, k=2.0)
    rc, _ = _spec(H, W, _asym(P, 1), [comp], prm, aff=aff, mode=1, k=2.0, shift=shift)
    m0 = oracle.model_image(plain, th, 0)
    m1 = oracle.model_image(rc, th, 0)
    assert np.max(np.abs(m1 - m0)) <= 1e-13 * np.max(np.abs(m0))


def test_bilinear_recentred_point_equals_point_source():
    """A Sersic far narrower than a pixel sampled at its pixel centre is a single-pixel
    spike; shifting it back bilinearly must give exactly the point-source model (a bilinear
    splat of the same flux at the same position) through the same asymmetric PSF."""
    H, W, P = 21, 24, 9
    K = _asym(P, 3)
    x0, y0 = 9.37, 11.81
    box = synth.full_window(H, W, P)
    comp, prm = _free_sersic([x0, y0, 1.0, 0.0, 0.5, 0.02, 0.1], box)
    rc, th = _spec(H, W, K, [comp], prm, s=1, shift=(BIL, 1))
    # the spike's value: Ie exp(-b ((R/Re)^(1/n) - 1)) at the floored radius R_MIN, b_0.5 = ln 2
    flux = 10 ** 0.1 * math.exp(-math.log(2.0) * ((oracle.R_MIN / 0.02) ** 2 - 1.0))
    pt = dict(type=oracle.POINT, image=0, box=box, par=[-1] * 7, fixed=[x0, y0, math.log10(flux), 0, 0, 0, 0])
    ps, _ = _spec(H, W, K, [pt], [])
    m_rc = oracle.model_image(rc, th, 0)
    m_pt = oracle.model_image(ps, np.zeros(0), 0)
    assert np.max(np.abs(m_rc - m_pt)) <= 1e-12 * np.max(m_pt)


@pytest.mark.parametrize("shift", [(BIL, 1), (LAN, 3)])
def test_shift_commutes_with_convolution(shift):
    """The paper's order (convolve, then shift) equals shifting the sampled component and
    convolving that (two independent convolutions by scipy), for a window reaching the
    edge of the extended grid."""
    H, W, P = 23, 26, 7
    c = 3
    K = _asym(P, 5)
    comp, prm = _free_sersic([-0.8, 12.3, 0.7, 0.4, 2.2, 6.0, 0.0], synth.full_window(H, W, P))
    spec, th = _spec(H, W, K, [comp], prm, shift=shift)
    a = shift[1]
    m = oracle.model_image(spec, th, 0)
    Sc, (wy, wx, _, _), _ = oracle.recentred_parts(spec, oracle.clipped(comp, spec["images"][0]), th)
    T = np.outer(wy, wx)                                        # T[ty + a, tx + a]
    shifted = scipy.signal.convolve2d(Sc, T, mode="full")       # extended grid grown by a
    full = scipy.signal.convolve2d(shifted, K.astype(np.float64), mode="full")
    # image pixel (i, j) sits at index i + c + a + c of the full result
    ref = full[2 * c + a:2 * c + a + H, 2 * c + a:2 * c + a + W]
    assert np.max(np.abs(m - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("shift", [(BIL, 1), (LAN, 3)])
def test_recentring_keeps_flux(shift):
    H, W, P = 40, 40, 9
    comp, prm = _free_sersic([19.3, 20.6, 0.8, 1.1, 0.5, 2.0, 0.0], synth.full_window(H, W, P))
    spec, th = _spec(H, W, synth.moffat_psf(P, 2.5, 3.0), [comp], prm, shift=shift)
    Sc, _, _ = oracle.recentred_parts(spec, comp, th)
    m = oracle.model_image(spec, th, 0)
    assert m.sum() == pytest.approx(Sc.sum() * float(np.asarray(spec["images"][0]["psf"], np.float64).sum()),
                                    rel=1e-12)


def test_lanczos_recentring_approximates_the_true_position():
    """On a smooth, well-sampled profile the re-centred model approaches the model sampled
    at the true position.  The windowed sinc is not exact even for low-order polynomials
    (its first moment is not delta), so the error falls slowly with the order: on a
    sampled 1-D Gaussian of sigma 4 px moved by 0.3 px, Lanczos-2, -3, -5 leave 4.0e-3,
    2.3e-3, 1.1e-3 of the peak; bilinear is worse than Lanczos-3."""
    H, W, P = 48, 48, 9
    comp, prm = _free_sersic([23.31, 24.77, 0.75, 0.6, 0.5, 6.0, 0.0], synth.full_window(H, W, P))
    K = synth.moffat_psf(P, 3.0, 2.5)
    plain, th = _spec(H, W, K, [comp], prm, s=5, rule=1)
    m0 = oracle.model_image(plain, th, 0)
    errs = {}
    for sh in [(BIL, 1), (LAN, 2), (LAN, 3), (LAN, 5)]:
        spec, _ = _spec(H, W, K, [comp], prm, s=5, rule=1, shift=sh)
        errs[sh] = np.max(np.abs(oracle.model_image(spec, th, 0) - m0)) / np.max(m0)
    assert errs[(LAN, 3)] < 5e-3
    assert errs[(LAN, 3)] < 0.5 * errs[(BIL, 1)]
    assert errs[(LAN, 5)] < errs[(LAN, 3)] < errs[(LAN, 2)]


@pytest.mark.parametrize("shift", [(BIL, 1), (LAN, 3)])
def test_recentred_jacobian_matches_finite_differences(shift):
    """Columns of every parameter of a re-centred Sersic (rotated, scaled pixel map, so the
    centre derivative goes through the inverse map) against central differences of the
    model; the steps stay inside one pixel cell (no change of the nearest centre)."""
    H, W, P = 25, 28, 7
    aff = _rot_affine(0.4, 0.97, H, W, 0.1, 0.35)
    comp, prm = _free_sersic([13.2, 11.9, 0.65, 0.5, 1.8, 3.5, 0.1], synth.full_window(H, W, P))
    spec, th = _spec(H, W, _asym(P, 9), [comp], prm, aff=aff, shift=shift)
    _, d, _ = oracle.recentre_geometry(spec["images"][0], th[0], th[1])
    assert min(abs(d[0]), abs(d[1])) > 0.05 and max(abs(d[0]), abs(d[1])) < 0.45
    J = oracle.jacobian_image(spec, th, 0)
    for k in range(7):
        h = 1e-6 * max(1.0, abs(th[k]))
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = ((oracle.model_image(spec, tp, 0) - oracle.model_image(spec, tm, 0)) / (2 * h)).ravel()
        scale = np.max(np.abs(fd))
        assert np.max(np.abs(J[:, k] - fd)) <= 2e-6 * scale, k
