"""Test oracle for the chi^2 forward-modelling hot path (TEST INFRASTRUCTURE ONLY).

A plain, slow, FP64 CPU implementation of what the HIP path computes, written from the
paper's definitions.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product path never does.  It shares no code with the
HIP library: it reads the same plain-dict workload spec and the same FP32-rounded
arrays, promoted to FP64.

What it computes, with the passage each step follows (section numbers of the paper):

* Sersic profile with elliptical isophotes (the "sersic galaxy model" of §2.1.1;
  parameters x, y, q, PA, n, Re, Ie as listed in §3.5, units of App. C):
  I(R) = Ie exp(-b_n ((R/Re)^(1/n) - 1)), R = sqrt(x'^2 + (y'/q)^2), with b_n the
  root of gamma(2n, b_n) = Gamma(2n)/2 (regularised P(2n, b_n) = 1/2).
* Pixel integration (§2.1.2): the pixel value is the pixel area times the weighted
  mean of the profile over s x s sub-pixel nodes (uniform midpoints, or the product
  Gauss-Legendre rule the paper uses for its second pass); optionally s x s nodes only
  where the pixel centre lies within k Re and the pixel centre alone elsewhere
  (the paper's first-pass midpoint).
* Point source (§2.1.1 "psf star model": a PSF map shifted by bilinear interpolation),
  written as a bilinear splat of the flux onto the four surrounding pixels before the
  convolution, which gives the same image.
* Composite model (§2.1, §2.2): the sum of all components on the pre-convolution
  ("extended") grid, then a true 2-D convolution with the PSF stamp (§2.1.3, direct
  mode), then a flat sky per image.  An image whose PSF has a higher resolution than its
  pixels (§2.1.3) is sampled and convolved on a grid of U x U sub-pixels per pixel and the
  result is integrated (summed) onto its pixels (`render_grid`, `bin_pixels`).
* Sub-pixel re-centring (§2.1.3, optional): a Sersic is sampled with its centre moved to
  the nearest pixel centre, convolved, and the convolved image is shifted back to the
  true position by Lanczos or bilinear interpolation (`shifted_conv`).
* Likelihood (§2.2, Eq. likelihood and Eq. chi2): chi2 = sum_i w_i (d_i - m_i)^2 with
  w = 1/sigma^2.  The paper's Eq. (chi2) carries a factor 1/2 (it is -log L); this
  oracle reports the conventional sum without it.
* Derivatives (§2.3): the exact Jacobian dm/dtheta by the chain rule, J^T W J, J^T W r
  and the gradient d chi2/d theta = -2 J^T W r.
* Levenberg-Marquardt (§2.5): damped normal equations (A + lambda D) h = J^T W r with
  Marquardt scaling D = diag(A), solved by Cholesky; a failed factorisation raises
  lambda and retries, so the step never meets a singular matrix; the gain ratio decides
  acceptance (Gavin's "update 1" form).  The constants are pinned in this module.

Every sub-problem (one contiguous range of theta) is independent: its chi^2, Jacobian
and LM run only over its own images.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np
import scipy.special

SERSIC, POINT = 0, 1
RULE_MIDPOINT, RULE_GAUSS_LEGENDRE = 0, 1
MODE_UNIFORM, MODE_WITHIN_K_RE, MODE_ADAPTIVE = 0, 1, 2

R_MIN = 1e-6                 # floor on the elliptical radius (cusp of n > 1 profiles)
LN10 = math.log(10.0)

# Levenberg-Marquardt constants (§2.5; the paper gives none, these are the readings)
LM_LAMBDA0 = 1e-2
LM_UP = 11.0
LM_DOWN = 9.0
LM_EPS4 = 0.1
LM_LAMBDA_MIN = 1e-9
LM_LAMBDA_MAX = 1e9
LM_ATTEMPTS = 4              # Cholesky attempts per iteration before the step is dropped
LM_DAMP_FLOOR = 1e-12        # D_kk = max(A_kk, floor * max_k A_kk)

# parameter domain; a trial step outside it is rejected
Q_MIN, Q_MAX = 0.01, 1.0
N_MIN, N_MAX = 0.36, 10.0
RE_MIN, RE_MAX = 0.01, 1e4
# live Moffat PSF (power n, scale R_d in pixels)
PSF_N_MIN, PSF_N_MAX = 0.2, 20.0
PSF_RD_MIN, PSF_RD_MAX = 0.05, 1e3


# ----------------------------------------------------------------------------- b_n
def sersic_b(n: float) -> float:
    """b_n solving P(2n, b_n) = 1/2 (half the light inside Re)."""
    return float(scipy.special.gammaincinv(2.0 * n, 0.5))


def sersic_b_prime(n: float, h: float = 1e-5) -> float:
    """db_n/dn by a central difference of the root (truncation ~h^2 b''')."""
    return (sersic_b(n + h) - sersic_b(n - h)) / (2.0 * h)


def sersic_total_flux(q, re, ie, n) -> float:
    """Closed-form total flux of the elliptical Sersic profile (integral over the plane)."""
    b = sersic_b(n)
    return 2.0 * math.pi * q * re * re * ie * n * math.exp(b) * b ** (-2.0 * n) * math.gamma(2.0 * n)


# --------------------------------------------------------------------------- nodes
def nodes_1d(s: int, rule: int):
    """1-D sub-pixel node offsets (pixel units, centred) and weights summing to 1."""
    if rule == RULE_MIDPOINT:
        o = (np.arange(s, dtype=np.float64) + 0.5) / s - 0.5
        w = np.full(s, 1.0 / s)
    else:
        x, wl = np.polynomial.legendre.leggauss(s)
        o, w = x / 2.0, wl / 2.0
    return o, w


def nodes_2d(s: int, rule: int):
    o, w = nodes_1d(s, rule)
    ox = np.tile(o, s)          # x varies fastest
    oy = np.repeat(o, s)
    ww = np.repeat(w, s) * np.tile(w, s)
    return ox, oy, ww


# ---------------------------------------------------------------------- components
def local_params(comp: Dict, theta: np.ndarray) -> List[float]:
    return [float(theta[p]) if p >= 0 else float(f) for p, f in zip(comp["par"], comp["fixed"])]


def _affine(im):
    a = np.asarray(im["affine"], dtype=np.float64)
    return a


def _sky_coords(a, x, y):
    return a[0] + a[1] * x + a[2] * y, a[3] + a[4] * x + a[5] * y


def sersic_profile(ux, uy, prm, b, with_grad=False, bp=0.0):
    """Profile (and its 7 parameter derivatives) at sky-frame points (ux, uy)."""
    x0, y0, q, pa, n, re, lie = prm
    cs, sn = math.cos(pa), math.sin(pa)
    dx, dy = ux - x0, uy - y0
    xp = dx * cs + dy * sn
    yp = -dx * sn + dy * cs
    R_raw = np.sqrt(xp * xp + (yp / q) ** 2)
    floored = R_raw < R_MIN
    R = np.where(floored, R_MIN, R_raw)
    ie = 10.0 ** lie
    t = (R / re) ** (1.0 / n)
    I = ie * np.exp(-b * (t - 1.0))
    if not with_grad:
        return I
    dIdR = -I * b * t / (n * R)
    inv = np.where(floored, 0.0, 1.0 / R)
    dRdxp = xp * inv
    dRdyp = yp / (q * q) * inv
    g = np.empty((7,) + np.shape(I))
    # x0: dx'/dx0 = -cos, dy'/dx0 = +sin ; y0: dx'/dy0 = -sin, dy'/dy0 = -cos
    g[0] = dIdR * (-cs * dRdxp + sn * dRdyp)
    g[1] = dIdR * (-sn * dRdxp - cs * dRdyp)
    g[2] = dIdR * (-(yp * yp) / (q ** 3) * inv)
    g[3] = dIdR * (xp * yp * (1.0 - 1.0 / (q * q)) * inv)
    g[4] = I * (-bp * (t - 1.0) + b * t * np.log(R / re) / (n * n))
    g[5] = I * b * t / (n * re)
    g[6] = I * LN10
    return I, g


def _box_grid(box):
    y0, x0, y1, x1 = box
    yy, xx = np.meshgrid(np.arange(y0, y1, dtype=np.float64),
                         np.arange(x0, x1, dtype=np.float64), indexing="ij")
    return yy, xx


def _square_means(a, prm, b, bp, xc, yc, side, order, with_grad):
    """Means of the profile over the squares of the given side centred at pixel
    coordinates (xc[i], yc[i]) by order x order Gauss-Legendre (and of its 7 derivatives)."""
    o, w = nodes_1d(order, RULE_GAUSS_LEGENDRE)
    ox, oy = np.tile(o, order), np.repeat(o, order)
    wk = np.repeat(w, order) * np.tile(w, order)
    xc, yc = np.atleast_1d(xc)[:, None], np.atleast_1d(yc)[:, None]
    ux, uy = _sky_coords(a, xc + side * ox, yc + side * oy)
    r = sersic_profile(ux, uy, prm, b, with_grad, bp)
    if with_grad:
        return r[0] @ wk, r[1] @ wk                  # [squares], [7, squares]
    return r @ wk


def adaptive_pixels(im, comp, prm, tol, with_grad=False):
    """Adaptive sub-pixel integration of a Sersic over its window (§2.1.2): a first pass
    at the pixel centres gives the window flux F and the per-pixel error budget
    e = tol F / N (N pixels); a pixel whose second differences of the profile at unit
    spacing (the midpoint rule's leading error, sum of |d2/dx2| + |d2/dy2| over 24, times
    the pixel area) stay within e keeps the centre value; the others take 3 x 3
    Gauss-Legendre if that moves the value by at most e; the rest are cut into 5 x 5
    sub-pixels, each taking 5 x 5 Gauss-Legendre if that is within e of its 3 x 3 value
    and otherwise the mean of its own 5 x 5 sub-sub-pixels at 7 x 7 Gauss-Legendre.
    Returns area x value on the window (and the 7 derivative images of that value with
    every choice held fixed)."""
    a = _affine(im)
    area = abs(a[1] * a[5] - a[2] * a[4])
    n = prm[4]
    b = sersic_b(n)
    bp = sersic_b_prime(n) if with_grad else 0.0
    yy, xx = _box_grid(comp["box"])
    ux, uy = _sky_coords(a, xx, yy)
    r0 = sersic_profile(ux, uy, prm, b, with_grad, bp)
    v0 = r0[0] if with_grad else r0
    F = area * float(np.sum(v0))
    e = tol * F / xx.size
    prof = lambda x, y: sersic_profile(*_sky_coords(a, x, y), prm, b)
    est = area * (np.abs(prof(xx + 1, yy) + prof(xx - 1, yy) - 2 * v0) +
                  np.abs(prof(xx, yy + 1) + prof(xx, yy - 1) - 2 * v0)) / 24.0
    val = v0.copy()
    grad = r0[1].copy() if with_grad else None
    sub = (np.arange(5) + 0.5) / 5 - 0.5
    for iy, ix in zip(*np.nonzero(est > e)):
        xc, yc = xx[iy, ix], yy[iy, ix]
        q1 = _square_means(a, prm, b, bp, xc, yc, 1.0, 3, with_grad)
        v1 = float(q1[0][0] if with_grad else q1[0])
        if area * abs(v1 - v0[iy, ix]) <= e:
            val[iy, ix] = v1
            if with_grad:
                grad[:, iy, ix] = q1[1][:, 0]
            continue
        cx, cy = xc + np.tile(sub, 5), yc + np.repeat(sub, 5)         # 25 sub-pixels, x fastest
        g3 = _square_means(a, prm, b, bp, cx, cy, 0.2, 3, False)
        g5 = _square_means(a, prm, b, bp, cx, cy, 0.2, 5, with_grad)
        v5 = g5[0] if with_grad else g5
        tot, gtot = 0.0, np.zeros(7)
        for j in range(25):
            if area * abs(v5[j] - g3[j]) <= e:
                tot += v5[j]
                if with_grad:
                    gtot += g5[1][:, j]
                continue
            g7 = _square_means(a, prm, b, bp, cx[j] + np.tile(sub, 5) / 5, cy[j] + np.repeat(sub, 5) / 5,
                               0.04, 7, with_grad)
            tot += float(np.mean(g7[0] if with_grad else g7))
            if with_grad:
                gtot += g7[1].mean(axis=1)
        val[iy, ix] = tot / 25.0
        if with_grad:
            grad[:, iy, ix] = gtot / 25.0
    val = val * area
    if with_grad:
        return val, grad * area
    return val


def within_k_re(ux, uy, prm, k):
    """Pixels whose centre (sky position ux, uy) lies strictly inside the isophote of
    elliptical radius k Re (§2.1.2: the first, cheap pass at the pixel centre; the fine
    nodes only where the profile is steep)."""
    x0, y0, q, pa = prm[0], prm[1], prm[2], prm[3]
    dx, dy = ux - x0, uy - y0
    xp = dx * math.cos(pa) + dy * math.sin(pa)
    yp = -dx * math.sin(pa) + dy * math.cos(pa)
    return np.sqrt(xp * xp + (yp / q) ** 2) < k * prm[5]


def sersic_pixels(im, comp, prm, sampling, with_grad=False):
    """Pixel-integrated Sersic (area x weighted node mean) over the component window;
    returns the value on the window and, if asked, the 7 derivative images."""
    if sampling["mode"] == MODE_ADAPTIVE:
        return adaptive_pixels(im, comp, prm, sampling["k"], with_grad)
    a = _affine(im)
    area = abs(a[1] * a[5] - a[2] * a[4])
    n = prm[4]
    b = sersic_b(n)
    bp = sersic_b_prime(n) if with_grad else 0.0
    yy, xx = _box_grid(comp["box"])
    s, rule, mode = sampling["s"], sampling["rule"], sampling["mode"]
    ox, oy, ww = nodes_2d(s, rule)
    val = np.zeros_like(xx)
    grad = np.zeros((7,) + xx.shape) if with_grad else None
    for kx, ky, kw in zip(ox, oy, ww):
        ux, uy = _sky_coords(a, xx + kx, yy + ky)
        r = sersic_profile(ux, uy, prm, b, with_grad, bp)
        if with_grad:
            val += kw * r[0]
            grad += kw * r[1]
        else:
            val += kw * r
    if mode == MODE_WITHIN_K_RE:
        # the centre alone outside k Re (pixel-centre elliptical radius, strict <)
        ux, uy = _sky_coords(a, xx, yy)
        inside = within_k_re(ux, uy, prm, sampling["k"])
        r = sersic_profile(ux, uy, prm, b, with_grad, bp)
        if with_grad:
            val = np.where(inside, val, r[0])
            grad = np.where(inside[None], grad, r[1])
        else:
            val = np.where(inside, val, r)
    val *= area
    if with_grad:
        grad *= area
        return val, grad
    return val


def point_pixels(im, comp, prm, with_grad=False):
    """Bilinear splat of a point source of flux 10^lf at sky position (x, y)."""
    a = _affine(im)
    A = np.array([[a[1], a[2]], [a[4], a[5]]])
    px, py = np.linalg.solve(A, np.array([prm[0] - a[0], prm[1] - a[3]]))
    yy, xx = _box_grid(comp["box"])
    wgt = np.maximum(0.0, 1.0 - np.abs(xx - px)) * np.maximum(0.0, 1.0 - np.abs(yy - py))
    F = 10.0 ** prm[2]
    val = F * wgt
    if with_grad:
        g = np.zeros((7,) + xx.shape)
        g[2] = LN10 * val
        return val, g
    return val


# ------------------------------------------------------------ sub-pixel re-centring
# §2.1.3: with re-centring on, a Sersic component is sampled (and pixel-integrated) with its
# centre moved to the centre of the nearest pixel, convolved with the PSF, and the convolved
# image is then moved back to the true sub-pixel position by interpolation (Lanczos or
# bilinear).  Point sources are bilinear splats already and are left as they are.
SHIFT_NONE, SHIFT_BILINEAR, SHIFT_LANCZOS = 0, 1, 2


def shift_setting(spec: Dict):
    """(method, a): the re-centring interpolation and its half-width in pixels (1 for
    bilinear, the order a for Lanczos), or (SHIFT_NONE, 0)."""
    rc = spec.get("recentre")
    if not rc or int(rc["method"]) == SHIFT_NONE:
        return SHIFT_NONE, 0
    m = int(rc["method"])
    return m, (1 if m == SHIFT_BILINEAR else int(rc["a"]))


def lanczos(x, a: int):
    """Lanczos window of order a: sinc(x) sinc(x / a) for |x| < a, else 0 (normalised
    sinc, sin(pi x) / (pi x))."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(np.abs(x) < a, np.sinc(x) * np.sinc(x / a), 0.0)


def lanczos_prime(x, a: int):
    """d/dx of the Lanczos window; sinc'(z) = (cos(pi z) - sinc(z)) / z, 0 at z = 0."""
    x = np.asarray(x, dtype=np.float64)

    def dsinc(z):
        zs = np.where(z == 0.0, 1.0, z)
        return np.where(z == 0.0, 0.0, (np.cos(np.pi * zs) - np.sinc(zs)) / zs)

    return np.where(np.abs(x) < a, dsinc(x) * np.sinc(x / a) + np.sinc(x) * dsinc(x / a) / a, 0.0)


def shift_taps(delta: float, method: int, a: int):
    """Weights w[t + a], t = -a..a, that move a pixel-sampled image by delta pixels
    (|delta| <= 1/2) along one axis, shifted(i) = sum_t w_t img(i - t) (the image read at
    i - delta), and dw/d delta.  Bilinear: the two nearest samples (at delta = 0 the
    derivative is the one from the right, delta -> 0+).  Lanczos: the window at t - delta,
    normalised to unit sum so that the shift keeps the flux."""
    t = np.arange(-a, a + 1, dtype=np.float64)
    if method == SHIFT_BILINEAR:
        w = np.maximum(0.0, 1.0 - np.abs(t - delta))
        side = 1.0 if delta >= 0.0 else -1.0
        dw = np.where(t == 0.0, -side, 0.0) + np.where(t == side, side, 0.0)
        return w, dw
    L = lanczos(t - delta, a)
    dL = -lanczos_prime(t - delta, a)
    N, dN = float(L.sum()), float(dL.sum())
    return L / N, (dL * N - L * dN) / (N * N)


def recentre_geometry(im, x0: float, y0: float):
    """Nearest pixel centre of the sky position (x0, y0) on image im: returns the sky
    position of that pixel centre, the offset delta = (pixel position) - (that centre)
    in pixels (each in [-1/2, 1/2)), and d delta / d (x0, y0) (the inverse of the linear
    part of the pixel -> sky map)."""
    a = _affine(im)
    A = np.array([[a[1], a[2]], [a[4], a[5]]])
    px, py = np.linalg.solve(A, np.array([x0 - a[0], y0 - a[3]]))
    nx, ny = math.floor(px + 0.5), math.floor(py + 0.5)
    ux, uy = _sky_coords(a, float(nx), float(ny))
    return (ux, uy), (px - nx, py - ny), np.linalg.inv(A)


def recentred(spec: Dict, comp: Dict) -> bool:
    return comp["type"] == SERSIC and shift_setting(spec)[0] != SHIFT_NONE


def shifted_conv(Sc: np.ndarray, K: np.ndarray, wy: np.ndarray, wx: np.ndarray, a: int) -> np.ndarray:
    """The paper's order for one re-centred component: the true convolution K * S'
    (S' on the extended grid, zero beyond it) taken on the image grown by a pixels on
    every side, then the interpolation shift back onto the image:
    out(i) = sum_t wy[ty] wx[tx] (K * S')(i - t)."""
    Mp = convolve_valid(np.pad(Sc, a), K)             # image coords -a .. H+a
    H, W = Mp.shape[0] - 2 * a, Mp.shape[1] - 2 * a
    out = np.zeros((H, W))
    for jy in range(2 * a + 1):
        for jx in range(2 * a + 1):
            ty, tx = jy - a, jx - a
            out += wy[jy] * wx[jx] * Mp[a - ty:a - ty + H, a - tx:a - tx + W]
    return out


def recentred_parts(spec: Dict, comp: Dict, theta: np.ndarray, with_grad: bool = False):
    """One re-centred Sersic on the extended grid of its image: S' (sampled with the
    centre at the nearest pixel centre), the x and y taps (and their delta-derivatives)
    and d delta / d (x0, y0); with_grad adds dS'/dtheta_k (k = q, PA, n, Re, Ie; S' does
    not move with x0 and y0, whose derivative comes through the taps alone)."""
    im = render_grid(spec["images"][comp["image"]])
    c = psf_half(im)
    method, a = shift_setting(spec)
    prm = local_params(comp, theta)
    (ux, uy), (dx, dy), dd = recentre_geometry(im, prm[0], prm[1])
    prm_c = [ux, uy] + prm[2:]
    y0, x0, y1, x1 = comp["box"]
    Sc = np.zeros((im["H"] + 2 * c, im["W"] + 2 * c))
    r = sersic_pixels(im, comp, prm_c, spec["sampling"], with_grad)
    wx, dwx = shift_taps(dx, method, a)
    wy, dwy = shift_taps(dy, method, a)
    if not with_grad:
        Sc[y0 + c:y1 + c, x0 + c:x1 + c] = r
        return Sc, (wy, wx, dwy, dwx), dd
    Sc[y0 + c:y1 + c, x0 + c:x1 + c] = r[0]
    G = np.zeros((7,) + Sc.shape)
    G[:, y0 + c:y1 + c, x0 + c:x1 + c] = r[1]
    G[0] = G[1] = 0.0
    return Sc, (wy, wx, dwy, dwx), dd, G


def render_grid(im) -> Dict:
    """The grid an image's model is sampled and convolved on.  An image whose PSF has a
    higher resolution than its pixels (§2.1.3: sampling and convolution then run at the
    PSF's resolution and the result is integrated onto the image pixels) carries
    "up" = U > 1: its render grid has U x U sub-pixels per pixel, fine pixel (yf, xf)
    centred at pixel coordinates ((xf + 1/2)/U - 1/2, (yf + 1/2)/U - 1/2), so its
    pixel -> sky map is the image's composed with that scaling (and its pixel area is the
    image's over U^2); windows of its components and its PSF stamp are in fine pixels."""
    U = int(im.get("up", 1))
    if U == 1:
        return im
    a = np.asarray(im["affine"], dtype=np.float64)
    o = (1.0 - U) / (2.0 * U)
    fine = dict(im)
    fine["H"], fine["W"] = U * im["H"], U * im["W"]
    fine["affine"] = np.array([a[0] + (a[1] + a[2]) * o, a[1] / U, a[2] / U,
                               a[3] + (a[4] + a[5]) * o, a[4] / U, a[5] / U])
    fine["up"] = 1
    return fine


def bin_pixels(M: np.ndarray, U: int) -> np.ndarray:
    """Integrate a render-grid image onto the image pixels: each pixel is the sum of its
    U x U sub-pixels."""
    if U == 1:
        return M
    H, W = M.shape[0] // U, M.shape[1] // U
    return M.reshape(H, U, W, U).sum(axis=(1, 3))


def comp_pixels(spec, comp, theta, with_grad=False):
    im = render_grid(spec["images"][comp["image"]])
    prm = local_params(comp, theta)
    if comp["type"] == SERSIC:
        return sersic_pixels(im, comp, prm, spec["sampling"], with_grad)
    return point_pixels(im, comp, prm, with_grad)


# ------------------------------------------------------------------- image model
def psf_half(im) -> int:
    return (np.asarray(im["psf"]).shape[0] - 1) // 2


def clipped(comp: Dict, im) -> Dict | None:
    """The component with its window cut to the extended grid of its image (pixels
    outside that grid never reach the image through the valid convolution), or None
    when nothing is left."""
    c = psf_half(im)
    y0, x0, y1, x1 = comp["box"]
    y0, x0 = max(y0, -c), max(x0, -c)
    y1, x1 = min(y1, im["H"] + c), min(x1, im["W"] + c)
    if y1 <= y0 or x1 <= x0:
        return None
    out = dict(comp)
    out["box"] = (y0, x0, y1, x1)
    return out


def render_ext(spec: Dict, theta: np.ndarray, k: int) -> np.ndarray:
    """Sum of all components of image k on the extended render grid [-c, H+c) x [-c, W+c)
    (fine pixels for an image with a higher-resolution PSF); re-centred components are
    left out (they are convolved one by one, `model_conv`)."""
    im = render_grid(spec["images"][k])
    c = psf_half(im)
    S = np.zeros((im["H"] + 2 * c, im["W"] + 2 * c))
    for comp in spec["comps"]:
        if comp["image"] != k or recentred(spec, comp):
            continue
        comp = clipped(comp, im)
        if comp is None:
            continue
        y0, x0, y1, x1 = comp["box"]
        S[y0 + c:y1 + c, x0 + c:x1 + c] += comp_pixels(spec, comp, theta)
    return S


def convolve_valid(S_ext: np.ndarray, K: np.ndarray) -> np.ndarray:
    """True 2-D convolution sampled on the image: M[i,j] = sum_uv K[c+u,c+v] S[i-u,j-v],
    S given on the extended grid (index offset c), direct shift-and-add in FP64."""
    K = np.asarray(K, dtype=np.float64)
    P = K.shape[0]
    c = (P - 1) // 2
    H, W = S_ext.shape[0] - 2 * c, S_ext.shape[1] - 2 * c
    M = np.zeros((H, W))
    for U in range(P):
        for V in range(P):
            # S[i-u, j-v] with u = U-c lives at extended index i + c - u = i + 2c - U
            M += K[U, V] * S_ext[2 * c - U:2 * c - U + H, 2 * c - V:2 * c - V + W]
    return M


def sky_value(im, theta) -> float:
    return float(theta[im["sky_par"]]) if im["sky_par"] >= 0 else float(im["sky_fixed"])


# ------------------------------------------------------------------ live PSF
def psf_model_of(spec: Dict, k: int) -> Dict | None:
    """The live PSF model of image k (its parameters fitted with everything else, §2.1.3
    and §3.4), or None when the image has a fixed stamp."""
    for pm in spec.get("psf_models", []):
        if pm["image"] == k:
            return pm
    return None


def psf_params(pm: Dict, theta: np.ndarray):
    return [float(theta[p]) if p >= 0 else float(f) for p, f in zip(pm["par"], pm["fixed"])]


def moffat_stamp(n: float, rd: float, P: int, with_grad: bool = False):
    """Moffat PSF stamp: f = (1 + r^2/R_d^2)^(-n) point-sampled at the integer offsets of
    a P x P grid, normalised to unit sum (the stamp is normalised before convolution,
    §3.4).  With with_grad also d stamp / d n and d stamp / d R_d of the normalised
    stamp (quotient rule: dK = (df - K sum df) / sum f)."""
    c = (P - 1) // 2
    v, u = np.meshgrid(np.arange(-c, c + 1, dtype=np.float64), np.arange(-c, c + 1, dtype=np.float64))
    x = 1.0 + (u * u + v * v) / (rd * rd)
    f = x ** (-n)
    S = f.sum()
    K = f / S
    if not with_grad:
        return K
    df_dn = -np.log(x) * f
    df_drd = f * (-n) / x * (-2.0 * (u * u + v * v) / rd ** 3)
    dK_dn = (df_dn - K * df_dn.sum()) / S
    dK_drd = (df_drd - K * df_drd.sum()) / S
    return K, dK_dn, dK_drd


def psf_of(spec: Dict, theta: np.ndarray, k: int) -> np.ndarray:
    """The stamp image k is convolved with: its fixed stamp (FP32 values in FP64) or the
    live Moffat model at theta."""
    im = spec["images"][k]
    pm = psf_model_of(spec, k)
    if pm is None:
        return np.asarray(im["psf"], dtype=np.float64)
    n, rd = psf_params(pm, theta)
    return moffat_stamp(n, rd, np.asarray(im["psf"]).shape[0])


def recentred_comps(spec: Dict, k: int):
    """The re-centred components of image k, windows cut to its extended grid."""
    im = render_grid(spec["images"][k])
    out = []
    for comp in spec["comps"]:
        if comp["image"] == k and recentred(spec, comp):
            comp = clipped(comp, im)
            if comp is not None:
                out.append(comp)
    return out


def model_conv(spec: Dict, theta: np.ndarray, k: int, K: np.ndarray) -> np.ndarray:
    """Image k's components convolved with the stamp K, on its render grid: the sum of
    the ordinary components convolved at once, plus every re-centred component
    convolved and shifted back on its own (`shifted_conv`)."""
    M = convolve_valid(render_ext(spec, theta, k), K)
    a = shift_setting(spec)[1]
    for comp in recentred_comps(spec, k):
        Sc, (wy, wx, _, _), _ = recentred_parts(spec, comp, theta)
        M += shifted_conv(Sc, K, wy, wx, a)
    return M


def model_image(spec: Dict, theta: np.ndarray, k: int) -> np.ndarray:
    """Convolved model of image k (integrated onto its pixels) plus its flat sky (the sky
    is not convolved)."""
    im = spec["images"][k]
    U = int(im.get("up", 1))
    if U > 1 and shift_setting(spec)[0] != SHIFT_NONE:
        raise ValueError("re-centring is defined on image pixels; a higher-resolution PSF replaces it")
    M = model_conv(spec, theta, k, psf_of(spec, theta, k))
    return bin_pixels(M, U) + sky_value(im, theta)


def images_of_sub(spec: Dict, sub: int) -> List[int]:
    return [k for k, im in enumerate(spec["images"]) if im["sub"] == sub]


def chi2_images(spec, theta, data, weight, ks: Sequence[int]) -> float:
    """sum_i w_i (d_i - m_i)^2 over the pixels of images ks (Eq. chi2 without the 1/2)."""
    tot = 0.0
    for k in ks:
        m = model_image(spec, theta, k)
        r = np.asarray(data[k], dtype=np.float64) - m
        tot += float(np.sum(np.asarray(weight[k], dtype=np.float64) * r * r))
    return tot


def chi2(spec, theta, data, weight) -> np.ndarray:
    """chi^2 of every sub-problem."""
    return np.array([chi2_images(spec, theta, data, weight, images_of_sub(spec, s))
                     for s in range(len(spec["subs"]))])


# ----------------------------------------------------------------------- Jacobian
def jacobian_image(spec, theta, k, cols: Sequence[int] | None = None) -> np.ndarray:
    """dm/dtheta on image k, shape (H*W, n_par) (or only the listed columns):
    each column is the PSF convolution of the derivative of the pre-convolution image;
    the sky column is 1; tied parameters sum their contributions."""
    im0 = spec["images"][k]
    U = int(im0.get("up", 1))
    im = render_grid(im0)
    c = psf_half(im)
    H, W = im["H"], im["W"]
    n_par = spec["n_par"]
    if U > 1 and shift_setting(spec)[0] != SHIFT_NONE:
        raise ValueError("re-centring is defined on image pixels; a higher-resolution PSF replaces it")
    want = set(range(n_par)) if cols is None else set(cols)
    dS = {}
    for comp in spec["comps"]:
        if comp["image"] != k or recentred(spec, comp):
            continue
        comp = clipped(comp, im)
        if comp is None:
            continue
        y0, x0, y1, x1 = comp["box"]
        if not any(p >= 0 and p in want for p in comp["par"]):
            continue
        _, g = comp_pixels(spec, comp, theta, with_grad=True)
        for loc, p in enumerate(comp["par"]):
            if p < 0 or p not in want:
                continue
            if p not in dS:
                dS[p] = np.zeros((H + 2 * c, W + 2 * c))
            dS[p][y0 + c:y1 + c, x0 + c:x1 + c] += g[loc]
    out_cols = list(range(n_par)) if cols is None else list(cols)
    J = np.zeros(((H // U) * (W // U), len(out_cols)))
    K = psf_of(spec, theta, k)
    for ci, p in enumerate(out_cols):
        if p in dS:
            J[:, ci] = bin_pixels(convolve_valid(dS[p], K), U).ravel()
        if im["sky_par"] == p:
            J[:, ci] += 1.0
    # re-centred components: m_c = T(delta) * (K * S'); the shape parameters move S', the
    # centre moves only delta (by d delta / d(x0, y0)), i.e. the taps
    a = shift_setting(spec)[1]
    for comp in recentred_comps(spec, k):
        if not any(p >= 0 and p in want for p in comp["par"]):
            continue
        Sc, (wy, wx, dwy, dwx), dd, G = recentred_parts(spec, comp, theta, with_grad=True)
        for loc, p in enumerate(comp["par"]):
            if p < 0 or p not in want:
                continue
            if loc < 2:
                Mx = shifted_conv(Sc, K, wy, dwx, a)          # d / d delta_x
                My = shifted_conv(Sc, K, dwy, wx, a)          # d / d delta_y
                col = dd[0, loc] * Mx + dd[1, loc] * My
            else:
                col = shifted_conv(G[loc], K, wy, wx, a)
            J[:, out_cols.index(p)] += col.ravel()
    # live PSF: m = K(phi) * S + sky, so dm/dphi = (dK/dphi) * S
    pm = psf_model_of(spec, k)
    if pm is not None and any(p >= 0 and p in want for p in pm["par"]):
        n, rd = psf_params(pm, theta)
        _, dK_dn, dK_drd = moffat_stamp(n, rd, np.asarray(im["psf"]).shape[0], with_grad=True)
        for p, dK in zip(pm["par"], (dK_dn, dK_drd)):
            if p >= 0 and p in want:
                J[:, out_cols.index(p)] += bin_pixels(model_conv(spec, theta, k, dK), U).ravel()
    return J


def jacobian(spec, theta, images: Sequence[int] | None = None,
             cols: Sequence[int] | None = None) -> np.ndarray:
    """Dense Jacobian, rows = pixels of the listed images concatenated in image order."""
    ks = range(len(spec["images"])) if images is None else images
    return np.concatenate([jacobian_image(spec, theta, k, cols) for k in ks], axis=0)


def residual(spec, theta, data, weight, ks):
    r = np.concatenate([(np.asarray(data[k], np.float64) - model_image(spec, theta, k)).ravel()
                        for k in ks])
    w = np.concatenate([np.asarray(weight[k], np.float64).ravel() for k in ks])
    return r, w


def jtwj(spec, theta, data, weight, sub: int = 0):
    """(J^T W J, J^T W r, chi2) of one sub-problem over its own parameter range."""
    p0, npar = spec["subs"][sub]
    ks = images_of_sub(spec, sub)
    cols = list(range(p0, p0 + npar))
    J = jacobian(spec, theta, ks, cols)
    r, w = residual(spec, theta, data, weight, ks)
    A = J.T @ (w[:, None] * J)
    g = J.T @ (w * r)
    return A, g, float(np.sum(w * r * r))


def chi2_grad(spec, theta, data, weight) -> np.ndarray:
    """d chi2 / d theta = -2 J^T W r, from the explicit Jacobian of every sub-problem."""
    grad = np.zeros(spec["n_par"])
    for s, (p0, npar) in enumerate(spec["subs"]):
        _, g, _ = jtwj(spec, theta, data, weight, s)
        grad[p0:p0 + npar] = -2.0 * g
    return grad


def covariance(spec, theta, data, weight, sub: int = 0) -> np.ndarray:
    """Parameter covariance of one sub-problem: the inverse of the Gauss-Newton Hessian
    J^T W J (section 2.5: the inverse of the Hessian the LM approximates gives the
    uncertainties and the full covariance of the parameters)."""
    A, _, _ = jtwj(spec, theta, data, weight, sub)
    return np.linalg.inv(A)


# ------------------------------------------------------------ Levenberg-Marquardt
def in_domain(spec, theta, sub: int) -> bool:
    for comp in spec["comps"]:
        if comp["type"] != SERSIC or spec["images"][comp["image"]]["sub"] != sub:
            continue
        x0, y0, q, pa, n, re, lie = local_params(comp, theta)
        vals = (x0, y0, q, pa, n, re, lie)
        if not all(math.isfinite(v) for v in vals):
            return False
        if not (Q_MIN <= q <= Q_MAX and N_MIN <= n <= N_MAX and RE_MIN <= re <= RE_MAX):
            return False
    for pm in spec.get("psf_models", []):
        if spec["images"][pm["image"]]["sub"] != sub:
            continue
        n, rd = psf_params(pm, theta)
        if not (math.isfinite(n) and math.isfinite(rd) and PSF_N_MIN <= n <= PSF_N_MAX
                and PSF_RD_MIN <= rd <= PSF_RD_MAX):
            return False
    return True


def cholesky_or_none(M: np.ndarray):
    """Lower Cholesky factor, or None when a pivot is not positive (or not finite)."""
    n = M.shape[0]
    L = np.zeros_like(M)
    for j in range(n):
        d = M[j, j] - L[j, :j] @ L[j, :j]
        if not (d > 0.0) or not math.isfinite(d):
            return None
        L[j, j] = math.sqrt(d)
        L[j + 1:, j] = (M[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def lm_predicted_decrease(h, lam, D, g) -> float:
    """chi2 decrease the linearised model predicts for the step h of (A + lam D) h = g:
    2 h.g - h.A.h, which the normal equations turn into h.(lam D h + g)."""
    return float(h @ (lam * D * h + g))


def lm_fit_sub(spec, theta0, data, weight, sub: int, n_iter: int):
    """n_iter LM iterations on one sub-problem; returns (theta, history).

    Per iteration: if the last step was accepted (or at the start) form chi2, A = J^T W J,
    g = J^T W r at theta; try Cholesky of A + lambda D (D = diag(A) floored), raising
    lambda by LM_UP after each failure (LM_ATTEMPTS tries); solve for h; reject an
    out-of-domain trial; otherwise rho = (chi2 - chi2(theta + h)) / h^T (lambda D h + g);
    accept when rho > LM_EPS4 (lambda /= LM_DOWN), else lambda *= LM_UP; lambda is
    kept within [LM_LAMBDA_MIN, LM_LAMBDA_MAX]."""
    theta = np.array(theta0, dtype=np.float64)
    p0, npar = spec["subs"][sub]
    ks = images_of_sub(spec, sub)
    lam = LM_LAMBDA0
    need = True
    hist = []
    A = g = None
    c2 = None
    for it in range(n_iter):
        if need:
            A, g, c2 = jtwj(spec, theta, data, weight, sub)
            need = False
        diagA = np.diag(A).copy()
        D = np.maximum(diagA, LM_DAMP_FLOOR * np.max(diagA))
        L = None
        for attempt in range(LM_ATTEMPTS):
            L = cholesky_or_none(A + lam * np.diag(D))
            if L is not None:
                break
            lam = min(lam * LM_UP, LM_LAMBDA_MAX)
        rec = dict(it=it, chi2=c2, lam=lam, accepted=False, chi2_trial=None, rho=None)
        if L is None:
            hist.append(rec)
            continue
        y = np.linalg.solve(L, g) if npar > 0 else g
        h = np.linalg.solve(L.T, y)
        trial = theta.copy()
        trial[p0:p0 + npar] += h
        pred = lm_predicted_decrease(h, lam, D, g)
        if in_domain(spec, trial, sub):
            c2t = chi2_images(spec, trial, data, weight, ks)
            rho = (c2 - c2t) / pred if pred != 0.0 else float("nan")
        else:
            c2t, rho = float("inf"), -float("inf")
        rec.update(chi2_trial=c2t, rho=rho, pred=pred)
        if rho > LM_EPS4:
            theta = trial
            c2 = c2t
            lam = max(lam / LM_DOWN, LM_LAMBDA_MIN)
            need = True
            rec["accepted"] = True
        else:
            lam = min(lam * LM_UP, LM_LAMBDA_MAX)
        hist.append(rec)
    return theta, hist


def lm_fit(spec, theta0, data, weight, n_iter: int, subs: Sequence[int] | None = None):
    """Independent LM fits of the listed sub-problems (all by default)."""
    theta = np.array(theta0, dtype=np.float64)
    hists = {}
    for s in (range(len(spec["subs"])) if subs is None else subs):
        p0, npar = spec["subs"][s]
        t, h = lm_fit_sub(spec, theta, data, weight, s, n_iter)
        theta[p0:p0 + npar] = t[p0:p0 + npar]
        hists[s] = h
    return theta, hists


def wrap_pa(spec, theta):
    """Position angles reduced to [0, pi) (output convention only)."""
    t = np.array(theta, dtype=np.float64)
    for comp in spec["comps"]:
        if comp["type"] == SERSIC and comp["par"][3] >= 0:
            t[comp["par"][3]] = math.fmod(t[comp["par"][3]], math.pi)
            if t[comp["par"][3]] < 0:
                t[comp["par"][3]] += math.pi
    return t
