"""Problem specs and data for the GPU parity tests (inputs from the seeded generator,
noise-free models and expected values from the oracle only)."""
import math

import numpy as np

import oracle
from paper_2308_01957_amd import synth


def with_data(spec, theta=None):
    """Attach data/weight built from the oracle's noise-free model at theta (default truth)."""
    th = spec["theta_true"] if theta is None else theta
    data, weight = [], []
    for k, im in enumerate(spec["images"]):
        m = oracle.model_image(spec, th, k)
        d, w = synth.make_data(m, spec["noise"][k][:im["H"], :im["W"]])
        data.append(d)
        weight.append(w)
    spec["data"], spec["weight"] = data, weight
    return spec


def small_blend():
    """Ragged 75x93 field: full and partial Sersic windows, point sources, sky,
    asymmetric 9x9 PSF, s = 3 within 2 Re and the centre elsewhere."""
    rng = np.random.default_rng(21)
    spec = synth.blend(seed_id=102, H=75, W=93, n_sersic=3, n_point=4, P=9,
                       psf=synth.asymmetric_psf(9, rng))
    # give two of the Sersics partial windows
    spec["comps"][1]["box"] = (5, -4, 60, 70)
    spec["comps"][2]["box"] = (-4, 20, 79, 97)
    return with_data(spec)


def wide_groups():
    """Two Sersic groups wide enough for the 64-column J^T W J tiles on one 70x80 image:
    12 Sersics on the full window (84 columns: a full 64-column block and a ragged one) and
    8 on a shared partial window (56 columns), plus point sources and sky; each wide group
    meets itself and the other one on the 64-column tile path."""
    spec = synth.blend(seed_id=131, H=70, W=80, n_sersic=20, n_point=2, P=7)
    for q in range(12, 20):
        spec["comps"][q]["box"] = (6, 9, 62, 70)
    spec["name"] = "wide_groups70x80"
    return with_data(spec)


def affine_pair():
    """Two images with rotated/scaled/shifted pixel->sky maps, different PSF sizes,
    two Sersics with tied shape parameters and per-image brightness and sky,
    Gauss-Legendre 4 x 4 nodes."""
    rng = np.random.default_rng(5)
    H, W = 70, 66
    affs = []
    for (phi, sc, tx, ty) in [(0.3, 1.01, 0.25, 0.6), (2.1, 0.985, 0.8, 0.1)]:
        a1, a2 = sc * math.cos(phi), -sc * math.sin(phi)
        a4, a5 = sc * math.sin(phi), sc * math.cos(phi)
        pcx, pcy = (W - 1) / 2, (H - 1) / 2
        affs.append(np.array([pcx - a1 * pcx - a2 * pcy + tx, a1, a2, pcy - a4 * pcx - a5 * pcy + ty, a4, a5]))
    psfs = [synth.moffat_psf(7, 2.5, 3.0), synth.asymmetric_psf(11, rng)]
    gals = [[30.2, 35.7, 0.55, 0.8, 1.7, 5.0], [42.1, 25.3, 0.8, 2.0, 0.9, 3.5]]
    theta, kinds, re_of = [], [], []
    for g in gals:
        theta += g + [0.3, 0.1]               # shape + two per-image log10 Ie
        kinds += [0, 1, 2, 3, 4, 5, 6, 6]
        re_of += [g[5]] * 8
    theta += [0.05, 0.07]
    kinds += [8, 8]
    re_of += [1.0, 1.0]
    images, comps = [], []
    for k in range(2):
        images.append(dict(H=H, W=W, psf=psfs[k], affine=affs[k], sky_par=16 + k, sky_fixed=0.0, sub=0))
        for gi, g in enumerate(gals):
            p0 = 8 * gi
            box = synth.ellipse_window(g[0], g[1], g[2], g[3], g[5], 8.0, H, W, psfs[k].shape[0], affs[k])
            comps.append(dict(type=0, image=k, box=box,
                              par=[p0, p0 + 1, p0 + 2, p0 + 3, p0 + 4, p0 + 5, p0 + 6 + k], fixed=[0.0] * 7))
    spec = {"name": "affine_pair", "images": images, "comps": comps, "subs": [(0, 18)],
            "sampling": dict(s=4, rule=1, mode=0, k=0.0), "theta_true": theta, "kinds": kinds,
            "re_of": re_of}
    synth._finish(spec)
    nr = np.random.default_rng(7)
    spec["noise"] = [nr.standard_normal((H, W)) for _ in range(2)]
    spec["theta_init"] = synth.perturb(spec["theta_true"], spec["kinds"], spec["re_of"], np.random.default_rng(8))
    return with_data(spec)


def single64():
    return with_data(synth.single(1))


def few_cutouts():
    return with_data(synth.cutouts(seed_id=104, n_cutouts=6, side_range=(20, 72), p_range=(5, 17), max_comp=3))


def large_sub():
    """One sub-problem above the one-wave solver size (blocked Cholesky path)."""
    return with_data(synth.blend(seed_id=105, H=96, W=110, n_sersic=11, n_point=8, P=11))


def bright_cutouts():
    """Six single-Sersic cutouts bright enough for the fit to converge (batched LM)."""
    return with_data(synth.cutouts(seed_id=104, n_cutouts=6, side_range=(24, 72), p_range=(5, 17),
                                   max_comp=1, logie_range=(0.5, 1.5)))


def bright_large_sub():
    """77-parameter blend (10 Sersic + 6 point sources + sky) that the LM settles."""
    return with_data(synth.blend(seed_id=106, H=120, W=128, n_sersic=10, n_point=6, P=11,
                                 logie_range=(0.5, 1.5)))


def tol_pixels(m_ora):
    return 1e-5 * np.abs(m_ora) + 1e-7 * np.max(np.abs(m_ora))


def grid_large_sub():
    """66 parameters in one sub-problem (blocked Cholesky path): nine bright,
    well-separated Sersics on a 3 x 3 grid, two point sources and the sky."""
    rng = np.random.default_rng(2024)
    H = W = 150
    P = 11
    K = synth.moffat_psf(P, 3.0, 2.5)
    theta, kinds, re_of, comps = [], [], [], []
    for gy in range(3):
        for gx in range(3):
            cx, cy = 25 + 50 * gx + rng.uniform(-2, 2), 25 + 50 * gy + rng.uniform(-2, 2)
            prm = [cx, cy, rng.uniform(0.5, 0.9), rng.uniform(0, math.pi), rng.uniform(0.8, 3.0),
                   rng.uniform(2.5, 4.0), rng.uniform(0.5, 1.5)]
            p0 = len(theta)
            theta += prm
            kinds += [0, 1, 2, 3, 4, 5, 6]
            re_of += [prm[5]] * 7
            comps.append(dict(type=0, image=0, box=synth.full_window(H, W, P), par=list(range(p0, p0 + 7)),
                              fixed=[0.0] * 7))
    for (px, py) in [(50.3, 99.6), (101.7, 48.2)]:
        theta.append(rng.uniform(1.0, 2.0))
        kinds.append(7)
        re_of.append(1.0)
        comps.append(dict(type=1, image=0, box=synth.point_window(px, py, H, W, P),
                          par=[-1, -1, len(theta) - 1, -1, -1, -1, -1], fixed=[px, py, 0, 0, 0, 0, 0]))
    theta.append(0.05)
    kinds.append(8)
    re_of.append(1.0)
    spec = {"name": "grid66", "images": [dict(H=H, W=W, psf=K, affine=synth.IDENTITY_AFFINE.copy(),
                                               sky_par=len(theta) - 1, sky_fixed=0.0, sub=0)],
            "comps": comps, "subs": [(0, len(theta))], "sampling": dict(s=3, rule=0, mode=1, k=2.0),
            "theta_true": theta, "kinds": kinds, "re_of": re_of}
    synth._finish(spec)
    spec["noise"] = [np.random.default_rng(2025).standard_normal((H, W))]
    spec["theta_init"] = synth.perturb(spec["theta_true"], spec["kinds"], spec["re_of"], np.random.default_rng(2026))
    return with_data(spec)


def live_psf_small():
    """Live Moffat PSF (n, R_d free) fitted with 6 bright stars, 2 galaxies and the sky on a
    ragged 70 x 76 image, P = 15."""
    spec = synth.live_psf(seed_id=107, H=70, W=76, n_star=6, n_sersic=2, P=15, psf_n=2.2, psf_rd=2.4,
                          logf_range=(2.0, 3.0), logie_range=(0.5, 1.5))
    return with_data(spec)


def adaptive_small(tol=1e-3):
    """Adaptive integration (tolerance tol) on a ragged 64 x 72 blend: a steep n ~ 5.9
    Sersic at the image edge, two more Sersics (one with a window cut by the extended
    grid), three point sources and the sky; P = 9."""
    spec = synth.blend(seed_id=108, H=64, W=72, n_sersic=3, n_point=3, P=9, mode=synth.MODE_ADAPTIVE,
                       k_re=tol)
    spec["comps"][1]["box"] = (-4, 10, 50, 80)
    spec["name"] = f"adaptive64x72_tol{tol:g}"
    return with_data(spec)


def adaptive_fit():
    """Adaptive integration, tol = 1e-2, on a 56 x 60 blend of two bright Sersics, two point
    sources and the sky that the LM settles from the perturbed start; P = 9."""
    spec = synth.blend(seed_id=110, H=56, W=60, n_sersic=2, n_point=2, P=9, mode=synth.MODE_ADAPTIVE,
                       k_re=1e-2, logie_range=(0.5, 1.5))
    spec["name"] = "adaptive56x60_fit"
    return with_data(spec)


def fft_blend():
    """FFT-mode convolution on a ragged 150 x 170 blend, P = 25: four Sersics (one with a
    window cut by the extended grid) on FFT tiles, five point sources on direct tiles."""
    spec = synth.blend(seed_id=130, H=150, W=170, n_sersic=4, n_point=5, P=25, logie_range=(0.0, 1.0))
    spec["comps"][1]["box"] = (-12, 30, 120, 182)
    spec["conv_mode"] = 1
    spec["name"] = "fft_blend150x170_P25"
    return with_data(spec)


def fft_fit():
    """A 110 x 120 blend (3 bright Sersics, 2 point sources, sky; P = 25) that the LM
    settles, with FFT-mode convolution."""
    spec = synth.blend(seed_id=132, H=110, W=120, n_sersic=3, n_point=2, P=25, logie_range=(0.5, 1.5))
    spec["conv_mode"] = 1
    spec["name"] = "fft_fit110x120_P25"
    return with_data(spec)


def superres(U=2, H=38, W=44, seed=140, aff=None, P=11, fit=False):
    """An image whose PSF has U x U samples per pixel: two Sersics (windows on the fine
    grid, one cut), a point source and the sky; fine asymmetric-ish Moffat stamp P."""
    rng = np.random.default_rng(seed)
    Hf, Wf = U * H, U * W
    psf = synth.moffat_psf(P, 1.2 * U, 2.8)
    a = synth.IDENTITY_AFFINE.copy() if aff is None else np.asarray(aff, dtype=np.float64)
    lie = (0.5, 1.5) if fit else (0.0, 1.0)
    gals = [[0.45 * W + rng.uniform(-1, 1), 0.5 * H + rng.uniform(-1, 1), 0.65, 0.9, 1.6, 4.5, rng.uniform(*lie)],
            [0.7 * W, 0.3 * H, 0.8, 2.1, 1.1, 3.0, rng.uniform(*lie)]]
    theta, kinds, re_of, comps = [], [], [], []
    c = (P - 1) // 2
    boxes = [synth.full_window(Hf, Wf, P), (-c, U * 4, U * H - 3, Wf + c)]
    for gi, g in enumerate(gals):
        p0 = len(theta)
        theta += g
        kinds += [0, 1, 2, 3, 4, 5, 6]
        re_of += [g[5]] * 7
        comps.append(dict(type=0, image=0, box=boxes[gi], par=list(range(p0, p0 + 7)), fixed=[0.0] * 7))
    # point source at sky position (ux, uy); its window on the fine grid
    px, py = 0.25 * W + 0.37, 0.7 * H + 0.21                # image pixel position
    ux, uy = a[0] + a[1] * px + a[2] * py, a[3] + a[4] * px + a[5] * py
    theta.append(1.8 if fit else 1.4)
    kinds.append(7)
    re_of.append(1.0)
    comps.append(dict(type=1, image=0, box=synth.point_window((px + 0.5) * U - 0.5, (py + 0.5) * U - 0.5, Hf, Wf, P),
                      par=[-1, -1, len(theta) - 1, -1, -1, -1, -1], fixed=[ux, uy, 0, 0, 0, 0, 0]))
    theta.append(0.05)
    kinds.append(8)
    re_of.append(1.0)
    spec = {"name": f"superres_U{U}_{H}x{W}", "images": [dict(H=H, W=W, psf=psf, affine=a, sky_par=len(theta) - 1,
                                                               sky_fixed=0.0, sub=0, up=U)],
            "comps": comps, "subs": [(0, len(theta))], "sampling": dict(s=2, rule=0, mode=0, k=0.0),
            "theta_true": theta, "kinds": kinds, "re_of": re_of}
    synth._finish(spec)
    spec["noise"] = [np.random.default_rng(seed + 1).standard_normal((H, W))]
    spec["theta_init"] = synth.perturb(spec["theta_true"], spec["kinds"], spec["re_of"], np.random.default_rng(seed + 2))
    return with_data(spec)


def recentred_blend(method, a=3):
    """The ragged 75 x 93 blend of `small_blend` (partial windows, point sources, asymmetric
    9 x 9 PSF, s = 3 within 2 Re) with sub-pixel re-centring of its Sersics."""
    rng = np.random.default_rng(21)
    spec = synth.blend(seed_id=102, H=75, W=93, n_sersic=3, n_point=4, P=9,
                       psf=synth.asymmetric_psf(9, rng))
    spec["comps"][1]["box"] = (5, -4, 60, 70)
    spec["comps"][2]["box"] = (-4, 20, 79, 97)
    return with_data(synth.with_recentring(spec, method, a))


def recentred_affine_pair(method=synth.SHIFT_LANCZOS, a=3):
    """`affine_pair` (two rotated, scaled images, tied shapes, Gauss-Legendre 4 x 4) with
    re-centring: each image moves each Sersic to its own nearest pixel centre."""
    return with_data(synth.with_recentring(affine_pair(), method, a))


def recentred_fft(method=synth.SHIFT_LANCZOS, a=3):
    """`fft_blend` (P = 25, FFT-mode convolution) with re-centring."""
    return with_data(synth.with_recentring(fft_blend(), method, a))


def recentred_live_psf(method=synth.SHIFT_LANCZOS, a=2):
    """`live_psf_small` (live Moffat PSF with free n, R_d) with re-centring."""
    return with_data(synth.with_recentring(live_psf_small(), method, a))


def recentred_fit(method=synth.SHIFT_LANCZOS, a=3):
    """A 64 x 70 blend of three bright Sersics, two point sources and the sky (P = 9) that
    the LM settles, with re-centring."""
    spec = synth.blend(seed_id=160, H=64, W=70, n_sersic=3, n_point=2, P=9, logie_range=(0.5, 1.5))
    return with_data(synth.with_recentring(spec, method, a))


# Relative rounding of an FP64 chi^2 of many terms (a few ulp of each term, summed): the LM
# decides on chi^2 differences, so two exact LMs stop within sigma_k sqrt(CHI2_REL_RES chi^2)
# of the minimum along parameter k (a step of that size changes chi^2 by about the
# rounding).  RES_MULT: 2 for the two fits stopping on opposite sides of the minimum, and
# a margin of 1.5 for the estimate of the rounding (measured: at most 1.9 of the resolution).
CHI2_REL_RES = 2e-15
RES_MULT = 3.0


def fit_gates(spec, theta):
    """(the benchmark spec, resolution) per parameter at the oracle's optimum theta:
    1e-6 (|theta_k| + scale_k), and sigma_k sqrt(CHI2_REL_RES chi^2_s) with the posterior
    width sigma_k = sqrt((J^T W J)^-1)_kk of sub-problem s."""
    res = np.zeros(spec["n_par"])
    for s, (p0, n) in enumerate(spec["subs"]):
        if n == 0:
            continue
        A, _, c2 = oracle.jtwj(spec, theta, spec["data"], spec["weight"], s)
        res[p0:p0 + n] = np.sqrt(np.abs(np.diag(np.linalg.inv(A)))) * math.sqrt(CHI2_REL_RES * c2)
    return 1e-6 * (np.abs(theta) + spec["scale"]), res


def fit_tolerance(spec, theta):
    """Per-parameter bound for comparing two converged fits at the oracle's optimum theta:
    1e-6 (|theta_k| + scale_k), or RES_MULT times the FP64 chi^2 resolution where that is
    larger (a cutout's sky with sigma 0.15 at chi^2 = 564: resolution 1.6e-7 against a
    spec gate of 1.5e-7).  Where the resolution is the larger, no LM deciding on FP64
    chi^2 differences can be held to the spec gate."""
    ns, res = fit_gates(spec, theta)
    return np.maximum(ns, RES_MULT * res)


def assert_fit_parity(spec, tg, to, label=""):
    """Converged-fit parity: |tg - to| within fit_tolerance.  The ratios to the north-star
    gate and to the chi^2 resolution go into the assertion message, and to the JSON-lines
    file named by APX_FIT_REPORT when that is set."""
    import json
    import os
    ns, res = fit_gates(spec, to)
    d = np.abs(np.asarray(tg, np.float64) - to)
    tol = np.maximum(ns, RES_MULT * res)
    kinds = np.asarray(spec.get("kinds", np.full(len(d), -1)))
    rep = {"case": label or spec.get("name", "?"), "max_over_northstar": float(np.max(d / ns)),
           "worst_kind": int(kinds[int(np.argmax(d / ns))]),
           "max_over_resolution": float(np.max(d / np.maximum(res, 1e-300))),
           "n_over_northstar": int(np.sum(d > ns)), "n_par": int(spec["n_par"])}
    path = os.environ.get("APX_FIT_REPORT")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(rep) + "\n")
    bad = d > tol
    assert not bad.any(), (rep, np.nonzero(bad), np.asarray(tg)[bad], to[bad], tol[bad])
    return rep


def auto_cutouts():
    """Automatic convolution mode on six cutouts of 27-92 px, P = 21-29, 1-3 Sersics each:
    three Jacobian jobs priced cheaper on FFT tiles, one rank-one (Gaussian) stamp on the
    two-pass kernel, two jobs on direct 2-D tiles (windows under 32 px)."""
    spec = synth.cutouts(seed_id=160, n_cutouts=6, side_range=(24, 160), p_range=(21, 31), max_comp=3)
    spec["conv_mode"] = 3
    spec["name"] = "auto_cutouts6"
    return with_data(spec)


def auto_fit():
    """Six bright single-Sersic cutouts of 64-160 px (P = 21-31) that the batched LM settles
    in automatic convolution mode (FFT and two-pass Jacobian jobs)."""
    spec = synth.cutouts(seed_id=171, n_cutouts=6, side_range=(64, 160), p_range=(21, 31), max_comp=1,
                         logie_range=(0.5, 1.5))
    spec["conv_mode"] = 3
    spec["name"] = "auto_fit6"
    return with_data(spec)
