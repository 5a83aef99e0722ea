"""Host logic of bench.py (CPU only): the counted HBM traffic is reported only for the tile
shapes and kernel sources it was counted with, and FFT-mode lines carry a direct-equivalent
rate instead of a roofline fraction."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

SUMMARY = os.path.join(ROOT, "profiles", "conv_jcol_blend512_hbm_counters.md")


def _recorded():
    kv = {}
    for line in open(SUMMARY):
        if ":" in line and not line.startswith("|"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_counted_traffic_needs_the_counted_tile_shapes():
    import hashlib
    kv = _recorded()
    tiles = json.loads(kv["jacobian_tiles"])
    h = hashlib.sha256()
    for src in kv["sources"].split():
        h.update(open(os.path.join(ROOT, src), "rb").read())
    got = bench.counted_traffic(kv["kernel"], tiles)
    if h.hexdigest() == kv["sources_sha256"]:
        assert got == float(kv["traffic_bytes_per_launch"])
    else:                                   # kernel sources changed since the counters
        assert got is None
    other = dict(tiles)
    other["16x32"] = other.get("16x32", 0) + 1
    assert bench.counted_traffic(kv["kernel"], other) is None
    assert bench.counted_traffic("k_conv<99,JCOL>", tiles) is None


def test_fft_lines_report_a_direct_equivalent_rate(capsys):
    bench.CONV_MODE[0] = "fft"
    try:
        bench._line({"metric": "m", "config": {"workload": "w"},
                     "roofline": {"kernel": "k", "achieved": 120.0, "peak": 157.3, "frac": 0.76}})
    finally:
        bench.CONV_MODE[0] = "direct"
    rec = json.loads(capsys.readouterr().out)
    assert "roofline" not in rec and rec["direct_equivalent"]["tflops"] == 120.0
    assert rec["config"]["conv"] == "fft"


def test_jacobian_entries_per_cutout_count_every_convolved_column():
    """Cutouts: each free Sersic parameter is one column over the whole cutout (the window
    is the cutout); the sky column is not convolved."""
    from paper_2308_01957_amd import synth
    spec = synth.cutouts(seed_id=104, n_cutouts=5, side_range=(20, 40), p_range=(5, 9), max_comp=3)
    ent, flop = bench.jac_entries_per_sub(spec)
    for s, (p0, n) in enumerate(spec["subs"]):
        im = [im for im in spec["images"] if im["sub"] == s][0]
        P = im["psf"].shape[0]
        assert ent[s] == (n - 1) * im["H"] * im["W"]
        assert flop[s] == ent[s] * 2.0 * P * P


def test_cpu_baseline_runs_the_oracle_on_a_process_pool():
    """The CPU baseline: a pool of single-threaded workers runs oracle LM iterations on a
    sample of cutouts and reports cutout iterations per second with its core count."""
    import oracle
    from paper_2308_01957_amd import synth
    spec = synth.cutouts(seed_id=104, n_cutouts=4, side_range=(20, 28), p_range=(5, 7), max_comp=1)
    data, weight = [], []
    for k, im in enumerate(spec["images"]):
        d, w = synth.make_data(oracle.model_image(spec, spec["theta_true"], k), spec["noise"][k][:im["H"], :im["W"]])
        data.append(d)
        weight.append(w)
    rec = bench.cpu_baseline_cutouts(spec, data, weight, synth, stride=2, n_iter=1)
    assert rec["kind"] == "oracle" and rec["value"] > 0 and 1 <= rec["cores"] <= 16
    assert rec["unit"] == "cutout LM it/s" and "2 of 4 cutouts" in rec["sample"]


def test_rank_one_images_follow_the_library_rule():
    """The bench's copy of the rank-one test: Gaussian and outer-product stamps qualify,
    Moffat and asymmetric ones do not; FFT or 2-D mode and live images never do."""
    import numpy as np
    from paper_2308_01957_amd import synth
    rng = np.random.default_rng(0)
    psfs = [synth.gaussian_psf(15, 2.0), synth.separable_psf(9), synth.moffat_psf(11, 3.0, 2.5),
            synth.asymmetric_psf(9, rng)]
    spec = {"images": [dict(psf=k) for k in psfs], "psf_models": []}
    assert bench.rank_one_images(spec, 0) == {0, 1}
    assert bench.rank_one_images(spec, 1) == set() and bench.rank_one_images(spec, 2) == set()
    spec["psf_models"] = [dict(image=0)]
    assert bench.rank_one_images(spec, 0) == {1}
