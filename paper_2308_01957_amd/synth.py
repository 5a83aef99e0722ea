"""Seeded synthetic workloads for the chi^2 forward-modelling hot path.

This module only draws inputs: parameter vectors, PSF stamps, component windows and
standard-normal noise fields.  It holds none of the fitting method's arithmetic (no
profile rendering, no convolution, no likelihood); the caller renders the noise-free
model with its own renderer and composes the data with :func:`make_data`.

Workload recipes follow the random-Sersic benchmark of §3.2 (Table 1: uniform priors
on centre, axis ratio, angle, index and radius, initial values perturbed by ~10% and
clipped back into range) with the sizes and priors of the five benchmark fields:

* ``single``   64x64, one Sersic + flat sky, Gaussian PSF 11x11 (sigma 1.5 px).
* ``blend``    512x512, 50 Sersic + 200 point sources + sky, Moffat PSF 25x25.
* ``gradient`` 2048x2048, 500 Sersic + sky, Moffat PSF 51x51, 10 Re windows.
* ``cutouts``  4096 independent cutouts of 32-256 px with 1-5 Sersic + sky each.
* ``multiband`` 6 images (3 bands x 2 epochs) of 2048x2048 with per-image affine
  maps and shared shape parameters (§3.3, per-band brightness).

Every workload is a plain ``dict`` (the *spec*) that both the HIP binding and the
test oracle read.  Conventions shared by both sides:

* pixel (i, j) of an image has its centre at x = j, y = i (pixel frame);
* a per-image affine map ``aff`` sends pixel coordinates to the common (sky) frame:
  ``u_x = aff[0] + aff[1] x + aff[2] y``, ``u_y = aff[3] + aff[4] x + aff[5] y``;
* a component window is a half-open box ``(y0, x0, y1, x1)`` on the image's extended
  (pre-convolution) grid, which spans ``[-c, H + c) x [-c, W + c)`` for a PSF of
  size ``P = 2c + 1``;
* a Sersic component has local parameters ``(x0, y0, q, PA, n, Re, log10 Ie)``
  (centre in the sky frame, PA in radians counter-clockwise from +x, App. C units);
  a point source has ``(x, y, log10 F)`` with a fixed position;
* ``par[k]`` is the index into theta of local parameter k, or -1 when the value is
  held fixed at ``fixed[k]``;
* every sub-problem owns one contiguous range of theta (``subs``).
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

SERSIC = 0
POINT = 1

RULE_MIDPOINT = 0
RULE_GAUSS_LEGENDRE = 1

MODE_UNIFORM = 0
MODE_WITHIN_K_RE = 1
MODE_ADAPTIVE = 2            # two-pass adaptive integration, k = tolerance

# parameter kinds (used for tolerances, perturbation and domain checks)
K_X, K_Y, K_Q, K_PA, K_N, K_RE, K_LOGIE, K_LOGF, K_SKY, K_PSF_N, K_PSF_RD = range(11)

Q_RANGE = (0.4, 0.9)
N_RANGE = (0.8, 4.0)
RE_RANGE = (3.0, 10.0)
LOGIE_RANGE = (-1.0, 1.0)
SKY_RANGE = (0.0, 0.1)
VAR_FLOOR = 0.01 ** 2     # variance = model / gain + 0.01^2, gain = 1


def seeds(config_id: int):
    """(truth, noise, init) seeds of workload ``config_id`` (PCG64)."""
    return 1000 * config_id + 1, 1000 * config_id + 2, 1000 * config_id + 3


# ----------------------------------------------------------------------------- PSFs
def gaussian_psf(P: int, sigma: float) -> np.ndarray:
    """Point-sampled circular Gaussian on integer offsets, unit sum, stored FP32."""
    c = (P - 1) // 2
    v = np.arange(-c, c + 1, dtype=np.float64)
    r2 = v[None, :] ** 2 + v[:, None] ** 2
    k = np.exp(-r2 / (2.0 * sigma * sigma))
    return (k / k.sum()).astype(np.float32)


def moffat_alpha(fwhm: float, beta: float) -> float:
    return fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))


def moffat_psf(P: int, fwhm: float, beta: float) -> np.ndarray:
    """Point-sampled Moffat (1 + r^2/alpha^2)^-beta, unit sum, stored FP32."""
    c = (P - 1) // 2
    a = moffat_alpha(fwhm, beta)
    v = np.arange(-c, c + 1, dtype=np.float64)
    r2 = v[None, :] ** 2 + v[:, None] ** 2
    k = (1.0 + r2 / (a * a)) ** (-beta)
    return (k / k.sum()).astype(np.float32)


def asymmetric_psf(P: int, rng: np.random.Generator) -> np.ndarray:
    """A positive, deliberately lopsided stamp (tells convolution from correlation)."""
    c = (P - 1) // 2
    v = np.arange(-c, c + 1, dtype=np.float64)
    X, Y = np.meshgrid(v, v)
    k = np.exp(-((X - 0.7) ** 2 / 3.0 + (Y + 0.4) ** 2 / 1.5)) + 0.05 * rng.random((P, P))
    return (k / k.sum()).astype(np.float32)


def separable_psf(P: int) -> np.ndarray:
    """A positive, lopsided stamp that is the outer product of two different vectors
    (a_u b_v: rank one, rows and columns distinguishable), unit sum, stored FP32."""
    c = (P - 1) // 2
    v = np.arange(-c, c + 1, dtype=np.float64)
    a = np.exp(-(v - 0.7) ** 2 / (2 * 1.3 ** 2))
    b = np.exp(-(v + 0.4) ** 2 / (2 * 2.1 ** 2)) * (1.0 + 0.1 * v / c)
    k = np.outer(a, b)
    return (k / k.sum()).astype(np.float32)


# -------------------------------------------------------------------------- helpers
IDENTITY_AFFINE = np.array([0.0, 1.0, 0.0, 0.0, 0.0, 1.0])


def full_window(H: int, W: int, P: int):
    c = (P - 1) // 2
    return (-c, -c, H + c, W + c)


def ellipse_window(x0, y0, q, pa, re, factor, H, W, P, aff=IDENTITY_AFFINE):
    """Bounding box (pixel frame, extended grid) of the ellipse of semi-major axis
    ``factor*re`` (sky frame), clipped to the extended grid."""
    c = (P - 1) // 2
    a = factor * re
    b = a * q
    # sky-frame half extents of the rotated ellipse
    hx = math.sqrt((a * math.cos(pa)) ** 2 + (b * math.sin(pa)) ** 2)
    hy = math.sqrt((a * math.sin(pa)) ** 2 + (b * math.cos(pa)) ** 2)
    A = np.array([[aff[1], aff[2]], [aff[4], aff[5]]])
    Ai = np.linalg.inv(A)
    corners = []
    for sx in (-hx, hx):
        for sy in (-hy, hy):
            u = np.array([x0 + sx - aff[0], y0 + sy - aff[3]])
            corners.append(Ai @ u)
    corners = np.array(corners)
    xmin, ymin = corners.min(axis=0)
    xmax, ymax = corners.max(axis=0)
    y0b = max(-c, int(math.floor(ymin)))
    x0b = max(-c, int(math.floor(xmin)))
    y1b = min(H + c, int(math.ceil(ymax)) + 1)
    x1b = min(W + c, int(math.ceil(xmax)) + 1)
    if y1b <= y0b or x1b <= x0b:
        return (0, 0, 0, 0)
    return (y0b, x0b, y1b, x1b)


def point_window(px: float, py: float, H: int, W: int, P: int):
    """The 2x2 bilinear support of a point at pixel position (px, py)."""
    c = (P - 1) // 2
    jx, iy = int(math.floor(px)), int(math.floor(py))
    y0b, x0b = max(-c, iy), max(-c, jx)
    y1b, x1b = min(H + c, iy + 2), min(W + c, jx + 2)
    if y1b <= y0b or x1b <= x0b:
        return (0, 0, 0, 0)
    return (y0b, x0b, y1b, x1b)


def _draw_sersic(rng, cx, cy, logie_range=LOGIE_RANGE):
    q = rng.uniform(*Q_RANGE)
    pa = rng.uniform(0.0, math.pi)
    n = rng.uniform(*N_RANGE)
    re = rng.uniform(*RE_RANGE)
    lie = rng.uniform(*logie_range)
    return [cx, cy, q, pa, n, re, lie]


def perturb(theta: np.ndarray, kinds: np.ndarray, re_of: np.ndarray, rng) -> np.ndarray:
    """Initial values ~10% away from truth in the pattern of Table 1 (§3.2):
    additive on positions (sigma 0.1 Re) and angle (0.1 rad), multiplicative on
    q, n, Re and sky, log-multiplicative on brightness; q and n clipped to range."""
    t = theta.copy()
    z = rng.standard_normal(theta.shape[0])
    for k in range(theta.shape[0]):
        kd = kinds[k]
        if kd in (K_X, K_Y):
            t[k] += 0.1 * re_of[k] * z[k]
        elif kd == K_PA:
            t[k] += 0.1 * z[k]
        elif kd in (K_Q, K_N, K_RE, K_SKY, K_PSF_N, K_PSF_RD):
            t[k] *= 1.0 + 0.1 * z[k]
            if kd == K_Q:
                t[k] = min(max(t[k], Q_RANGE[0]), Q_RANGE[1])
            elif kd == K_N:
                t[k] = min(max(t[k], N_RANGE[0]), N_RANGE[1])
        elif kd in (K_LOGIE, K_LOGF):
            t[k] += math.log10(max(1.0 + 0.1 * z[k], 0.5))
    return t


def param_scale(kinds: np.ndarray, re_of: np.ndarray) -> np.ndarray:
    """Per-parameter scale: Re for centres, 1 for angle/shape/brightness, 0.1 for sky."""
    s = np.ones(kinds.shape[0])
    for k in range(kinds.shape[0]):
        if kinds[k] in (K_X, K_Y):
            s[k] = re_of[k]
        elif kinds[k] == K_SKY:
            s[k] = 0.1
    return s


def make_data(model: np.ndarray, noise: np.ndarray, dtype=np.float32):
    """Noisy data and inverse-variance weight from a noise-free model image.

    variance = model / gain + 0.01^2 with gain 1; data = model + sqrt(var) * z.
    Both are rounded once to ``dtype``; the kernels and the oracle read those values.
    """
    var = np.maximum(model, 0.0) + VAR_FLOOR
    d = model + np.sqrt(var) * noise
    return d.astype(dtype), (1.0 / var).astype(dtype)


def _finish(spec):
    spec["n_par"] = int(len(spec["theta_true"]))
    spec["theta_true"] = np.asarray(spec["theta_true"], dtype=np.float64)
    spec["kinds"] = np.asarray(spec["kinds"], dtype=np.int32)
    spec["re_of"] = np.asarray(spec["re_of"], dtype=np.float64)
    spec["scale"] = param_scale(spec["kinds"], spec["re_of"])
    return spec


# ------------------------------------------------------------------------ workloads
def single(seed_id: int = 1, H: int = 64, W: int = 64, P: int = 11, sigma: float = 1.5,
           s: int = 3, rule: int = RULE_MIDPOINT, psf: np.ndarray | None = None) -> Dict:
    """One Sersic + flat sky on a small image, full-image window, uniform s x s nodes."""
    st, sn, si = seeds(seed_id)
    rng = np.random.Generator(np.random.PCG64(st))
    cx, cy = (W - 1) / 2.0 + rng.uniform(-2, 2), (H - 1) / 2.0 + rng.uniform(-2, 2)
    prm = _draw_sersic(rng, cx, cy)
    sky = rng.uniform(*SKY_RANGE)
    theta = prm + [sky]
    kinds = [K_X, K_Y, K_Q, K_PA, K_N, K_RE, K_LOGIE, K_SKY]
    re_of = [prm[5]] * 7 + [1.0]
    K = gaussian_psf(P, sigma) if psf is None else psf
    spec = {
        "name": f"single{H}x{W}",
        "images": [dict(H=H, W=W, psf=K, affine=IDENTITY_AFFINE.copy(), sky_par=7,
                        sky_fixed=0.0, sub=0)],
        "comps": [dict(type=SERSIC, image=0, box=full_window(H, W, P),
                       par=list(range(7)), fixed=[0.0] * 7)],
        "subs": [(0, 8)],
        "sampling": dict(s=s, rule=rule, mode=MODE_UNIFORM, k=0.0),
        "theta_true": theta, "kinds": kinds, "re_of": re_of,
    }
    _finish(spec)
    rng_n = np.random.Generator(np.random.PCG64(sn))
    spec["noise"] = [rng_n.standard_normal((H, W))]
    rng_i = np.random.Generator(np.random.PCG64(si))
    spec["theta_init"] = perturb(spec["theta_true"], spec["kinds"], spec["re_of"], rng_i)
    return spec


def blend(seed_id: int = 2, H: int = 512, W: int = 512, n_sersic: int = 50,
          n_point: int = 200, P: int = 25, fwhm: float = 3.0, beta: float = 2.5,
          s: int = 3, k_re: float = 2.0, mode: int = MODE_WITHIN_K_RE,
          psf: np.ndarray | None = None, logie_range=LOGIE_RANGE) -> Dict:
    """Blended field: Sersics with full-image windows + fixed-position point sources
    (free log10 flux, uniform in [0, 2]) + sky.  s x s nodes within k_re*Re of each
    Sersic centre, the pixel centre elsewhere."""
    st, sn, si = seeds(seed_id)
    rng = np.random.Generator(np.random.PCG64(st))
    K = moffat_psf(P, fwhm, beta) if psf is None else psf
    theta, kinds, re_of, comps = [], [], [], []
    for g in range(n_sersic):
        cx, cy = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
        prm = _draw_sersic(rng, cx, cy, logie_range)
        p0 = len(theta)
        theta += prm
        kinds += [K_X, K_Y, K_Q, K_PA, K_N, K_RE, K_LOGIE]
        re_of += [prm[5]] * 7
        comps.append(dict(type=SERSIC, image=0, box=full_window(H, W, P),
                          par=list(range(p0, p0 + 7)), fixed=[0.0] * 7))
    for k in range(n_point):
        px, py = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
        lf = rng.uniform(0.0, 2.0)
        p0 = len(theta)
        theta.append(lf)
        kinds.append(K_LOGF)
        re_of.append(1.0)
        comps.append(dict(type=POINT, image=0, box=point_window(px, py, H, W, P),
                          par=[-1, -1, p0, -1, -1, -1, -1],
                          fixed=[px, py, 0.0, 0.0, 0.0, 0.0, 0.0]))
    sky_par = len(theta)
    theta.append(rng.uniform(*SKY_RANGE))
    kinds.append(K_SKY)
    re_of.append(1.0)
    spec = {
        "name": f"blend{H}x{W}_{n_sersic}s{n_point}p_P{P}",
        "images": [dict(H=H, W=W, psf=K, affine=IDENTITY_AFFINE.copy(), sky_par=sky_par,
                        sky_fixed=0.0, sub=0)],
        "comps": comps,
        "subs": [(0, len(theta))],
        "sampling": dict(s=s, rule=RULE_MIDPOINT, mode=mode, k=k_re),
        "theta_true": theta, "kinds": kinds, "re_of": re_of,
    }
    _finish(spec)
    rng_n = np.random.Generator(np.random.PCG64(sn))
    spec["noise"] = [rng_n.standard_normal((H, W))]
    rng_i = np.random.Generator(np.random.PCG64(si))
    spec["theta_init"] = perturb(spec["theta_true"], spec["kinds"], spec["re_of"], rng_i)
    return spec


def field(seed_id: int = 3, H: int = 2048, W: int = 2048, n_sersic: int = 500,
          P: int = 51, fwhm: float = 4.0, beta: float = 3.0, s: int = 3,
          box_re: float = 10.0, psf: np.ndarray | None = None) -> Dict:
    """Large field of windowed Sersics + sky (gradient workload): each window is the
    bounding box of the box_re*Re ellipse, uniform s x s nodes."""
    st, sn, si = seeds(seed_id)
    rng = np.random.Generator(np.random.PCG64(st))
    K = moffat_psf(P, fwhm, beta) if psf is None else psf
    theta, kinds, re_of, comps = [], [], [], []
    for g in range(n_sersic):
        cx, cy = rng.uniform(0, W - 1), rng.uniform(0, H - 1)
        prm = _draw_sersic(rng, cx, cy)
        p0 = len(theta)
        theta += prm
        kinds += [K_X, K_Y, K_Q, K_PA, K_N, K_RE, K_LOGIE]
        re_of += [prm[5]] * 7
        comps.append(dict(type=SERSIC, image=0,
                          box=ellipse_window(cx, cy, prm[2], prm[3], prm[5], box_re, H, W, P),
                          par=list(range(p0, p0 + 7)), fixed=[0.0] * 7))
    sky_par = len(theta)
    theta.append(rng.uniform(*SKY_RANGE))
    kinds.append(K_SKY)
    re_of.append(1.0)
    spec = {
        "name": f"field{H}x{W}_{n_sersic}s_P{P}",
        "images": [dict(H=H, W=W, psf=K, affine=IDENTITY_AFFINE.copy(), sky_par=sky_par,
                        sky_fixed=0.0, sub=0)],
        "comps": comps,
        "subs": [(0, len(theta))],
        "sampling": dict(s=s, rule=RULE_MIDPOINT, mode=MODE_UNIFORM, k=0.0),
        "theta_true": theta, "kinds": kinds, "re_of": re_of,
    }
    _finish(spec)
    rng_n = np.random.Generator(np.random.PCG64(sn))
    spec["noise"] = [rng_n.standard_normal((H, W))]
    rng_i = np.random.Generator(np.random.PCG64(si))
    spec["theta_init"] = perturb(spec["theta_true"], spec["kinds"], spec["re_of"], rng_i)
    return spec


def cutouts(seed_id: int = 4, n_cutouts: int = 4096, side_range=(32, 256),
            p_range=(15, 31), fwhm_range=(2.0, 5.0), max_comp: int = 5, s: int = 3,
            logie_range=LOGIE_RANGE) -> Dict:
    """Many independent cutouts (one sub-problem each): side log-uniform in side_range,
    1..max_comp Sersics (the first centred within 2 px, the rest uniform over the
    central 80%) + sky; per-cutout Gaussian or Moffat (beta 3) PSF of odd size
    uniform in p_range with FWHM uniform in fwhm_range; window = whole cutout."""
    st, sn, si = seeds(seed_id)
    rng = np.random.Generator(np.random.PCG64(st))
    images, comps, subs, theta, kinds, re_of = [], [], [], [], [], []
    for ci in range(n_cutouts):
        side = int(round(math.exp(rng.uniform(math.log(side_range[0]), math.log(side_range[1])))))
        Pc = int(rng.integers((p_range[0] - 1) // 2, (p_range[1] - 1) // 2 + 1)) * 2 + 1
        fw = rng.uniform(*fwhm_range)
        if rng.random() < 0.5:
            K = gaussian_psf(Pc, fw / (2.0 * math.sqrt(2.0 * math.log(2.0))))
        else:
            K = moffat_psf(Pc, fw, 3.0)
        kc = int(rng.integers(1, max_comp + 1))
        p_start = len(theta)
        for g in range(kc):
            if g == 0:
                cx = (side - 1) / 2.0 + rng.uniform(-2, 2)
                cy = (side - 1) / 2.0 + rng.uniform(-2, 2)
            else:
                cx = rng.uniform(0.1 * side, 0.9 * side - 1)
                cy = rng.uniform(0.1 * side, 0.9 * side - 1)
            prm = _draw_sersic(rng, cx, cy, logie_range)
            p0 = len(theta)
            theta += prm
            kinds += [K_X, K_Y, K_Q, K_PA, K_N, K_RE, K_LOGIE]
            re_of += [prm[5]] * 7
            comps.append(dict(type=SERSIC, image=ci, box=full_window(side, side, Pc),
                              par=list(range(p0, p0 + 7)), fixed=[0.0] * 7))
        sky_par = len(theta)
        theta.append(rng.uniform(*SKY_RANGE))
        kinds.append(K_SKY)
        re_of.append(1.0)
        images.append(dict(H=side, W=side, psf=K, affine=IDENTITY_AFFINE.copy(),
                           sky_par=sky_par, sky_fixed=0.0, sub=ci))
        subs.append((p_start, len(theta) - p_start))
    spec = {
        "name": f"cutouts{n_cutouts}",
        "images": images, "comps": comps, "subs": subs,
        "sampling": dict(s=s, rule=RULE_MIDPOINT, mode=MODE_UNIFORM, k=0.0),
        "theta_true": theta, "kinds": kinds, "re_of": re_of,
    }
    _finish(spec)
    rng_n = np.random.Generator(np.random.PCG64(sn))
    spec["noise"] = [rng_n.standard_normal((im["H"], im["W"])) for im in images]
    rng_i = np.random.Generator(np.random.PCG64(si))
    spec["theta_init"] = perturb(spec["theta_true"], spec["kinds"], spec["re_of"], rng_i)
    return spec


def live_psf(seed_id: int = 6, H: int = 512, W: int = 512, n_star: int = 100, n_sersic: int = 20,
             P: int = 25, psf_n: float = 2.5, psf_rd: float = 2.6, s: int = 3,
             logf_range=(1.0, 2.5), logie_range=LOGIE_RANGE) -> Dict:
    """Stars (fixed positions, free log10 flux) and Sersic galaxies on one image whose PSF is
    a live Moffat model with free power n and scale R_d (its stamp in `psf` only sets P)
    + sky; all fitted jointly.  Galaxies have full-image windows, stars PSF-sized ones."""
    st, sn, si = seeds(seed_id)
    rng = np.random.Generator(np.random.PCG64(st))
    theta, kinds, re_of, comps = [], [], [], []
    for _ in range(n_star):
        px, py = rng.uniform(P / 2, W - 1 - P / 2), rng.uniform(P / 2, H - 1 - P / 2)
        theta.append(rng.uniform(*logf_range))
        kinds.append(K_LOGF)
        re_of.append(1.0)
        comps.append(dict(type=POINT, image=0, box=point_window(px, py, H, W, P),
                          par=[-1, -1, len(theta) - 1, -1, -1, -1, -1], fixed=[px, py, 0, 0, 0, 0, 0]))
    for _ in range(n_sersic):
        prm = _draw_sersic(rng, rng.uniform(0.1 * W, 0.9 * W), rng.uniform(0.1 * H, 0.9 * H), logie_range)
        p0 = len(theta)
        theta += prm
        kinds += [K_X, K_Y, K_Q, K_PA, K_N, K_RE, K_LOGIE]
        re_of += [prm[5]] * 7
        comps.append(dict(type=SERSIC, image=0, box=full_window(H, W, P), par=list(range(p0, p0 + 7)),
                          fixed=[0.0] * 7))
    theta.append(rng.uniform(*SKY_RANGE))
    kinds.append(K_SKY)
    re_of.append(1.0)
    sky = len(theta) - 1
    theta += [psf_n, psf_rd]
    kinds += [K_PSF_N, K_PSF_RD]
    re_of += [1.0, 1.0]
    spec = {"name": f"livepsf{H}x{W}_{n_star}st{n_sersic}s_P{P}",
            "images": [dict(H=H, W=W, psf=np.zeros((P, P), dtype=np.float32), affine=IDENTITY_AFFINE.copy(),
                            sky_par=sky, sky_fixed=0.0, sub=0)],
            "comps": comps, "subs": [(0, len(theta))],
            "psf_models": [dict(image=0, par=[len(theta) - 2, len(theta) - 1], fixed=[0.0, 0.0])],
            "sampling": dict(s=s, rule=RULE_MIDPOINT, mode=MODE_UNIFORM, k=0.0),
            "theta_true": theta, "kinds": kinds, "re_of": re_of}
    _finish(spec)
    spec["noise"] = [np.random.Generator(np.random.PCG64(sn)).standard_normal((H, W))]
    spec["theta_init"] = perturb(spec["theta_true"], spec["kinds"], spec["re_of"],
                                 np.random.Generator(np.random.PCG64(si)))
    return spec


def multiband(seed_id: int = 5, H: int = 2048, W: int = 2048, n_gal: int = 300,
              n_band: int = 3, n_epoch: int = 2, P: int = 41, beta: float = 3.0,
              fwhm_range=(3.0, 5.0), s: int = 3, box_re: float = 10.0,
              radius_frac: float = 0.45) -> Dict:
    """Joint multi-band multi-epoch field (§3.3): each image has its own affine
    pixel->sky map (rotation U[0,2pi), sub-pixel shift U[0,1)^2, scale 1 +- 2% about
    the centre), its own Moffat PSF and sky; galaxies share (x0, y0, q, PA, n, Re) in
    the sky frame and carry one log10 Ie per band."""
    st, sn, si = seeds(seed_id)
    rng = np.random.Generator(np.random.PCG64(st))
    n_img = n_band * n_epoch
    affs, psfs = [], []
    pcx, pcy = (W - 1) / 2.0, (H - 1) / 2.0
    for k in range(n_img):
        phi = rng.uniform(0, 2 * math.pi)
        tx, ty = rng.uniform(0, 1), rng.uniform(0, 1)
        sc = rng.uniform(0.98, 1.02)
        a1, a2 = sc * math.cos(phi), -sc * math.sin(phi)
        a4, a5 = sc * math.sin(phi), sc * math.cos(phi)
        a0 = pcx - a1 * pcx - a2 * pcy + tx
        a3 = pcy - a4 * pcx - a5 * pcy + ty
        affs.append(np.array([a0, a1, a2, a3, a4, a5]))
        psfs.append(moffat_psf(P, rng.uniform(*fwhm_range), beta))
    theta, kinds, re_of, gal = [], [], [], []
    for g in range(n_gal):
        r = radius_frac * min(H, W) * math.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * math.pi)
        cx, cy = pcx + r * math.cos(ang), pcy + r * math.sin(ang)
        prm = _draw_sersic(rng, cx, cy)
        p0 = len(theta)
        band_ie = [prm[6] + rng.uniform(-0.3, 0.3) for _ in range(n_band)]
        theta += prm[:6] + band_ie
        kinds += [K_X, K_Y, K_Q, K_PA, K_N, K_RE] + [K_LOGIE] * n_band
        re_of += [prm[5]] * (6 + n_band)
        gal.append((p0, prm))
    images, comps = [], []
    for k in range(n_img):
        band = k // n_epoch
        sky_par = len(theta)
        theta.append(rng.uniform(*SKY_RANGE))
        kinds.append(K_SKY)
        re_of.append(1.0)
        images.append(dict(H=H, W=W, psf=psfs[k], affine=affs[k], sky_par=sky_par,
                           sky_fixed=0.0, sub=0))
        for (p0, prm) in gal:
            box = ellipse_window(prm[0], prm[1], prm[2], prm[3], prm[5], box_re, H, W, P, affs[k])
            comps.append(dict(type=SERSIC, image=k, box=box,
                              par=[p0, p0 + 1, p0 + 2, p0 + 3, p0 + 4, p0 + 5, p0 + 6 + band],
                              fixed=[0.0] * 7))
    spec = {
        "name": f"multiband{n_img}x{H}x{W}_{n_gal}g_P{P}",
        "images": images, "comps": comps, "subs": [(0, len(theta))],
        "sampling": dict(s=s, rule=RULE_MIDPOINT, mode=MODE_UNIFORM, k=0.0),
        "theta_true": theta, "kinds": kinds, "re_of": re_of,
    }
    _finish(spec)
    rng_n = np.random.Generator(np.random.PCG64(sn))
    spec["noise"] = [rng_n.standard_normal((H, W)) for _ in range(n_img)]
    rng_i = np.random.Generator(np.random.PCG64(si))
    spec["theta_init"] = perturb(spec["theta_true"], spec["kinds"], spec["re_of"], rng_i)
    return spec


WORKLOADS = {"single": single, "blend": blend, "field": field, "cutouts": cutouts,
             "multiband": multiband}


def spec_summary(spec: Dict) -> Dict:
    npx = sum(im["H"] * im["W"] for im in spec["images"])
    return dict(name=spec["name"], n_images=len(spec["images"]), n_comps=len(spec["comps"]),
                n_par=spec["n_par"], n_sub=len(spec["subs"]), n_pix=npx)


def stack_images(arrays: List[np.ndarray], dtype=np.float32) -> np.ndarray:
    """Concatenate per-image arrays (row-major, image order) into one flat buffer."""
    return np.concatenate([np.ascontiguousarray(a, dtype=dtype).ravel() for a in arrays])


def sub_spec(spec: Dict, sub: int) -> Dict:
    """The spec of one sub-problem on its own (its images, components and parameters,
    re-indexed from zero) -- a single cutout of a batched workload."""
    p0, n = spec["subs"][sub]
    ks = [k for k, im in enumerate(spec["images"]) if im["sub"] == sub]
    kmap = {k: i for i, k in enumerate(ks)}
    images = []
    for k in ks:
        im = dict(spec["images"][k])
        im["sub"] = 0
        im["sky_par"] = im["sky_par"] - p0 if im["sky_par"] >= 0 else -1
        images.append(im)
    comps = []
    for c in spec["comps"]:
        if c["image"] in kmap:
            c2 = dict(c)
            c2["image"] = kmap[c["image"]]
            c2["par"] = [q - p0 if q >= 0 else -1 for q in c["par"]]
            comps.append(c2)
    out = {"name": f"{spec['name']}_sub{sub}", "images": images, "comps": comps, "subs": [(0, n)],
           "sampling": dict(spec["sampling"]), "theta_true": spec["theta_true"][p0:p0 + n],
           "kinds": spec["kinds"][p0:p0 + n], "re_of": spec["re_of"][p0:p0 + n]}
    _finish(out)
    out["theta_init"] = spec["theta_init"][p0:p0 + n].copy()
    out["noise"] = [spec["noise"][k] for k in ks]
    return out


def with_psf_upsampling(spec: Dict, U: int, P_fine: int, fwhm: float = 3.0, beta: float = 2.5) -> Dict:
    """The same field observed through a PSF sampled U times finer than the pixels: each
    image gets psf_up = U and a P_fine x P_fine Moffat stamp of FWHM `fwhm` pixels (U *
    fwhm sub-pixels); component windows move to the sub-pixel grid (whole-image windows
    stay whole-image, point-source supports follow their sub-pixel positions)."""
    out = dict(spec)
    out["images"], out["comps"] = [], []
    for im in spec["images"]:
        im2 = dict(im)
        im2["up"] = U
        im2["psf"] = moffat_psf(P_fine, fwhm * U, beta)
        out["images"].append(im2)
    for comp in spec["comps"]:
        im = spec["images"][comp["image"]]
        Hf, Wf = U * im["H"], U * im["W"]
        c2 = dict(comp)
        if comp["type"] == SERSIC:
            c2["box"] = full_window(Hf, Wf, P_fine)
        else:
            a = np.asarray(im["affine"], dtype=np.float64)
            A = np.array([[a[1], a[2]], [a[4], a[5]]])
            px, py = np.linalg.solve(A, [comp["fixed"][0] - a[0], comp["fixed"][1] - a[3]])
            c2["box"] = point_window((px + 0.5) * U - 0.5, (py + 0.5) * U - 0.5, Hf, Wf, P_fine)
        out["comps"].append(c2)
    out["name"] = f"{spec['name']}_up{U}_P{P_fine}"
    return out


SHIFT_NONE, SHIFT_BILINEAR, SHIFT_LANCZOS = 0, 1, 2


def with_recentring(spec: Dict, method: int, a: int = 3) -> Dict:
    """The same workload with sub-pixel re-centring of its Sersic components (§2.1.3):
    `method` SHIFT_BILINEAR or SHIFT_LANCZOS of order `a`."""
    out = dict(spec)
    out["recentre"] = {"method": int(method), "a": int(a)}
    out["name"] = f"{spec['name']}_shift{method}a{a}"
    return out
