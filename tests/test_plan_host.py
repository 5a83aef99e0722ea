"""Host-side descriptor validation and planning through the C ABI (no GPU: a host-only
context plans and sizes problems but never launches)."""
import copy
import os

import numpy as np
import pytest

from paper_2308_01957_amd import synth

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2308_01957_amd", "libapx.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libapx.so not built")


@pytest.fixture(scope="module")
def apx():
    from paper_2308_01957_amd import apx as mod
    return mod


def _small():
    return synth.blend(seed_id=301, H=40, W=52, n_sersic=2, n_point=3, P=7)


def test_plan_sizes_match_the_layout(apx):
    spec = _small()
    p = apx.Plan(spec)
    assert p.n_pix == 40 * 52
    assert p.n_ext == (40 + 6) * (52 + 6)
    # Jacobian entries: 14 Sersic columns on the full image + 3 point columns on their
    # (2+6) x (2+6) output boxes (clipped to the image)
    npt = 0
    for c in spec["comps"]:
        if c["type"] == 1:
            y0, x0, y1, x1 = c["box"]
            oh = min(40, y1 + 3) - max(0, y0 - 3)
            ow = min(52, x1 + 3) - max(0, x0 - 3)
            npt += oh * ow
    assert p.n_jac == 14 * 40 * 52 + npt
    assert p.workspace_bytes > 0


@pytest.mark.parametrize("mutate,status", [
    (lambda s: s["images"][0].__setitem__("psf", np.ones((6, 6), np.float32)), -1),     # even P
    (lambda s: s["images"][0].__setitem__("psf", np.ones((65, 65), np.float32)), -5),   # P > 63
    (lambda s: s["comps"][2]["par"].__setitem__(0, 0), -5),                            # free point position
    (lambda s: s["comps"][0]["par"].__setitem__(2, s["images"][0]["sky_par"]), -1),    # shares the sky index
    (lambda s: s["comps"][0]["par"].__setitem__(3, 10 ** 6), -1),                      # index out of range
    (lambda s: s.__setitem__("subs", [(0, 10), (5, 10)]), -1),                          # overlapping ranges
    (lambda s: s["images"][0].__setitem__("affine", np.array([0, 1.0, 2.0, 0, 0.5, 1.0])), -1),  # singular map
    (lambda s: s["sampling"].__setitem__("s", 9), -5),                                  # too many nodes
    (lambda s: s["comps"][0].__setitem__("type", 7), -1),                               # unknown type
    (lambda s: s.__setitem__("sampling", dict(s=3, rule=0, mode=2, k=0.0)), -1),         # adaptive tol 0
    (lambda s: s.__setitem__("sampling", dict(s=3, rule=0, mode=2, k=float("nan"))), -1),  # adaptive tol NaN
    (lambda s: s.__setitem__("sampling", dict(s=3, rule=0, mode=3, k=1.0)), -1),         # unknown mode
])
def test_invalid_descriptors(apx, mutate, status):
    spec = copy.deepcopy(_small())
    mutate(spec)
    with pytest.raises(apx.ApxError) as e:
        apx.Plan(spec)
    assert e.value.status == status


def test_parameter_outside_its_sub_problem_is_rejected(apx):
    spec = copy.deepcopy(synth.cutouts(seed_id=302, n_cutouts=3, side_range=(20, 30), p_range=(5, 7), max_comp=1))
    # give cutout 1's galaxy a centre parameter that belongs to cutout 0
    spec["comps"][1]["par"][0] = 0
    with pytest.raises(apx.ApxError) as e:
        apx.Plan(spec)
    assert e.value.status == -1


def test_full_scale_plans(apx):
    """Every benchmark workload plans on the host (sizes only, no GPU)."""
    for f in (synth.single, synth.blend, synth.field):
        p = apx.Plan(f())
        assert p.n_jac > 0 and p.workspace_bytes > 0
        p.close()


@pytest.mark.parametrize("shape", range(4))
def test_fixed_tile_policy_gives_every_job_that_shape(apx, shape):
    spec = _small()
    pl = apx.Plan(spec, tiles=apx.TILES_FIXED + shape)
    for kind in range(3):
        counts = pl.tile_shapes(kind)
        assert sum(counts) > 0 and counts[shape] == sum(counts)
    pl.close()


def test_model_tile_policy_prefers_tiles_that_fit_the_output(apx):
    """The operation-count model keeps 32 x 64 tiles on a 512 x 512 image and takes
    narrower tiles where they cut the padding of a 40-pixel-wide window."""
    big = synth.single(1, H=512, W=512, P=11)
    pl = apx.Plan(big, tiles=apx.TILES_MODEL)
    assert pl.tile_shapes(0) == [1, 0, 0, 0, 0, 0]
    pl.close()
    small = synth.single(1, H=40, W=40, P=11)
    pl = apx.Plan(small, tiles=apx.TILES_MODEL)
    assert pl.tile_shapes(0)[0] == 0
    pl.close()


def test_unknown_tile_policy_is_rejected(apx):
    with pytest.raises(apx.ApxError):
        apx.Plan(_small(), tiles=99)


def test_adaptive_mode_sizes_its_per_pixel_arrays(apx):
    """Adaptive integration keeps, per Sersic window pixel, a value, a choice code and room
    for a refine entry and its 7 derivatives: the workspace grows by at least 48 bytes per
    window pixel over the uniform plan of the same problem."""
    spec = _small()
    base = apx.Plan(spec).workspace_bytes
    spec["sampling"] = dict(s=3, rule=0, mode=synth.MODE_ADAPTIVE, k=1e-3)
    ad = apx.Plan(spec).workspace_bytes
    npx = sum((c["box"][2] - c["box"][0]) * (c["box"][3] - c["box"][1])
              for c in spec["comps"] if c["type"] == 0)
    assert npx > 0 and ad - base >= 48 * npx - 16 * 256       # less the empty arrays of the base plan


def test_fft_mode_takes_the_large_outputs_of_large_stamps(apx):
    """conv_mode FFT: on a P = 25 image the Jacobian columns of the full-image windows and
    the adjoint go to FFT tiles, the small point-source windows stay direct, and the model
    convolution stays direct under the FP64 objective but not under the FP32 one."""
    spec = synth.blend(seed_id=302, H=120, W=130, n_sersic=3, n_point=4, P=25)
    spec["conv_mode"] = apx.CONV_FFT
    pl = apx.Plan(spec)
    assert pl.tile_shapes(0)[4] == 0
    assert pl.tile_shapes(1)[4] == 1 and sum(pl.tile_shapes(1)[:4]) == 4
    assert pl.tile_shapes(2)[4] == 1
    pl.close()
    pl = apx.Plan(spec, objective=1)
    assert pl.tile_shapes(0)[4] == 1
    pl.close()
    small = synth.blend(seed_id=303, H=120, W=130, n_sersic=3, n_point=4, P=11)
    small["conv_mode"] = apx.CONV_FFT
    pl = apx.Plan(small)
    assert all(pl.tile_shapes(k)[4] == 0 for k in range(3))       # P below the FFT threshold
    pl.close()


def test_unknown_conv_mode_is_rejected(apx):
    spec = _small()
    spec["conv_mode"] = 7
    with pytest.raises(apx.ApxError):
        apx.Plan(spec)


@pytest.mark.parametrize("rc,up,mode,status", [
    ({"method": 3, "a": 3}, 1, 1, -1),             # unknown re-centring method
    ({"method": 2, "a": 1}, 1, 1, -5),             # Lanczos order below 2
    ({"method": 2, "a": 6}, 1, 1, -5),             # Lanczos order above the table
    ({"method": 1, "a": 0}, 1, 2, -5),             # with adaptive integration
    ({"method": 2, "a": 3}, 2, 1, -5),             # with a higher-resolution PSF
])
def test_recentring_descriptors(apx, rc, up, mode, status):
    spec = copy.deepcopy(_small())
    spec["recentre"] = rc
    spec["sampling"] = dict(s=3, rule=0, mode=mode, k=2.0 if mode == 1 else 0.01)
    if up > 1:
        spec = synth.with_psf_upsampling(spec, up, 9)
    with pytest.raises(apx.ApxError) as e:
        apx.Plan(spec)
    assert e.value.status == status


def test_recentring_grows_windows_by_the_taps(apx):
    """A re-centred Sersic's shifted image reaches a pixels beyond where it is sampled:
    its Jacobian output box grows by a on every side (clipped to the image)."""
    base = _small()
    win = (8, 10, 20, 30)                         # inside the 40 x 52 image, away from edges
    for c in base["comps"]:
        if c["type"] == 0:
            c["box"] = win
    n0 = apx.Plan(base).n_jac
    for rc, a in [({"method": 1, "a": 0}, 1), ({"method": 2, "a": 3}, 3), ({"method": 2, "a": 5}, 5)]:
        spec = copy.deepcopy(base)
        spec["recentre"] = rc
        n = apx.Plan(spec).n_jac
        h, w = win[2] - win[0] + 6, win[3] - win[1] + 6          # output box: window + c
        grown = min(40, win[2] + 3 + a) - max(0, win[0] - 3 - a), min(52, win[3] + 3 + a) - max(0, win[1] - 3 - a)
        assert n - n0 == 14 * (grown[0] * grown[1] - h * w)


def test_tile_cost_table_can_be_set_and_read_back(apx):
    """A host context stores autotuner table entries given to it and rejects bad ones."""
    import ctypes
    lib = apx.load_library()
    ctx = ctypes.c_void_p()
    assert lib.apx_ctx_create(-1, None, ctypes.byref(ctx)) == apx.APX_OK
    try:
        us = (ctypes.c_double * 4)(3.0, 2.5, 2.0, 1.25)
        out = (ctypes.c_double * 4)()
        assert lib.apx_ctx_tile_cost(ctx, 1, 25, out) != apx.APX_OK        # not timed yet
        assert lib.apx_ctx_set_tile_cost(ctx, 1, 25, us) == apx.APX_OK
        assert lib.apx_ctx_tile_cost(ctx, 1, 25, out) == apx.APX_OK
        assert list(out) == [3.0, 2.5, 2.0, 1.25]
        for kernel, P in [(4, 25), (-1, 25), (1, 24), (1, 0), (1, 65)]:
            assert lib.apx_ctx_set_tile_cost(ctx, kernel, P, us) != apx.APX_OK, (kernel, P)
        for bad in (0.0, -1.0, float("nan"), float("inf")):
            b = (ctypes.c_double * 4)(1.0, bad, 1.0, 1.0)
            assert lib.apx_ctx_set_tile_cost(ctx, 1, 25, b) != apx.APX_OK, bad
        assert lib.apx_ctx_tile_cost(ctx, 1, 25, out) == apx.APX_OK and list(out) == [3.0, 2.5, 2.0, 1.25]
    finally:
        lib.apx_ctx_destroy(ctx)


def test_direct_jobs_of_one_psf_size_share_one_tile_shape(apx):
    """A batch of cutouts of 32-256 px at one PSF size: every direct job of a kind takes the
    one shape of least cost summed over the batch (one launch per PSF size), although the
    operation-count model would give the small cutouts narrower tiles one by one."""
    spec = synth.cutouts(seed_id=7, n_cutouts=40, p_range=(21, 21))
    assert len({np.asarray(im["psf"]).shape[0] for im in spec["images"]}) == 1
    pl = apx.Plan(dict(spec, conv_mode=apx.CONV_DIRECT_2D), tiles=apx.TILES_MODEL)
    for kind in range(3):
        counts = pl.tile_shapes(kind)
        assert sum(1 for c in counts[:4] if c > 0) == 1, (kind, counts)
    assert sum(pl.tile_shapes(0)[:4]) == len(spec["images"])
    pl.close()
