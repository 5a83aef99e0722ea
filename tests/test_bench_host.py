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


def test_class_rooflines_count_by_hand():
    """Per-class algorithmic FLOP of a two-component image worked out by hand: windows grown
    by the PSF half-width and cut to the image, J^T W J pairs over the windows' overlap,
    objective and adjoint convolutions per evaluation; FFT mode prices only the pairs."""
    import numpy as np

    class _Prob:
        objective = 0
    K = np.array([[0.0, 1.0, 0.0], [1.0, 2.0, 1.0], [0.0, 1.0, 0.5]])
    spec = {"images": [dict(H=10, W=12, psf=K, sub=0)], "subs": [(0, 5)], "psf_models": [],
            "comps": [dict(image=0, box=(2, 3, 6, 8), par=[0, 1, 2]),
                      dict(image=0, box=(5, 6, 10, 12), par=[3, -1, 4])]}
    assert bench.rank_one_images(spec, 0) == set()
    kt = {"conv_jcol": (2.0, 4), "pairs": (1.0, 4), "conv_fwd": (0.5, 6), "conv_adj": (0.25, 2), "render": (9.0, 6)}
    dom, per = bench.class_rooflines(spec, _Prob(), kt, phases=3, per_call=(2, 1))
    flop = {k: v["achieved"] * 1e12 * v["ms_total"] * 1e-3 for k, v in per.items() if v["unit"] == "TFLOP/s"}
    # windows (1,2,7,9) and (4,5,10,12): 42 pixels each, overlap 3 x 4 = 12; both groups
    # (3 and 2 columns) are narrow, so J^T W r and sum w J come with them: 4 FLOP per entry
    assert np.isclose(flop["conv_jcol"], 3 * (3 * 42 + 2 * 42) * 2 * 9)
    assert np.isclose(per["pairs"]["flop"], 3 * (2 * 42 * 6 + 2 * 42 * 3 + 2 * 12 * 3 * 2 + 4 * 210))
    # J^T W J reads each of the 210 entries, the 84 window weights and the 84 residuals once:
    # 1512 B per phase, 0.57 ns at 8 TB/s against 0.04 ns of FP64 MFMA work: bound by HBM
    assert per["pairs"]["bound"] == "hbm" and np.isclose(per["pairs"]["algorithmic_bytes"], 3 * 4 * (210 + 84 + 84))
    assert np.isclose(per["pairs"]["achieved"] * 1e9 * 1e-3, 3 * 4 * (210 + 84 + 84))
    assert np.isclose(flop["conv_fwd"], 3 * 2 * 9 * 120)       # 6 launches, 2 per evaluation
    assert np.isclose(flop["conv_adj"], 2 * 2 * 9 * 120)
    assert per["conv_fwd"]["peak"] == bench.PEAK_FP64_TFLOPS and per["conv_jcol"]["peak"] == bench.PEAK_FP32_VALU_TFLOPS
    assert dom is per["conv_jcol"] and "render" not in per
    _, per = bench.class_rooflines(spec, _Prob(), kt, phases=3, per_call=(2, 1), n_obj=1)   # 2 launches idle
    assert np.isclose(per["conv_fwd"]["achieved"] * 1e12 * 0.5e-3, 2 * 9 * 120)
    spec["conv_mode"] = 1
    _, per = bench.class_rooflines(spec, _Prob(), kt, phases=3)
    assert set(per) == {"pairs"}


def test_auto_fft_choice_matches_the_library_plan():
    """The bench's copy of the automatic mode's FFT-or-direct rule picks the same number of
    FFT Jacobian jobs as the library's plan (host-only context: no stamp is read back, so
    none counts as rank one), on cutouts of 32-256 px and on the blended field (one wide
    Sersic group, small point-source windows)."""
    from paper_2308_01957_amd import apx, synth
    for spec in (synth.cutouts(seed_id=104, n_cutouts=300), synth.blend()):
        spec = dict(spec, conv_mode=apx.CONV_AUTO)
        plan = apx.Plan(spec)
        n_fft = plan.tile_shapes(1)[4]
        plan.close()
        groups = bench.auto_fft_groups(spec, rank_one=set())
        assert n_fft == len(groups) and n_fft > 0, (n_fft, len(groups))


def test_auto_fft_rule_by_hand():
    """Worked cases of the rule: a 256 x 256 job of 21 columns at P = 31 takes FFT tiles
    (9 blocks of 98^2 per column, 95 transform pairs at 1.0e6 against 21 x 32 tiles of
    32 x 64 at 2.04e6 units); so does a 40 x 40 job of 7 columns at P = 15 (4 pairs against
    7 x 3 tiles of 16 x 64 at 262360 units); a 32 x 32 job of one column at P = 15 stays
    direct (one pair against one 32 x 32 tile at 260568 units)."""
    assert bench.auto_fft_job(31, 256, 256, 21)
    assert bench.auto_fft_job(15, 40, 40, 7)
    assert not bench.auto_fft_job(15, 32, 32, 1)
    P = 15
    assert 4 * bench.AUTO_FFT_PAIR_COST < 7 * 3 * (16 * 64 * (P * P + 10.0) + 8.0 * (16 + P - 1) * (64 + P - 1) + 3000.0)
    assert 1 * bench.AUTO_FFT_PAIR_COST > 32 * 32 * (P * P + 10.0) + 8.0 * (32 + P - 1) * (32 + P - 1) + 3000.0
    P = 31
    direct = 21 * 32 * (32 * 64 * (P * P + 10.0) + 8.0 * (32 + P - 1) * (64 + P - 1) + 3000.0)
    assert ((21 * 9 + 1) // 2) * bench.AUTO_FFT_PAIR_COST < direct


def test_fft_pairs_by_hand():
    """Transform pairs of FFT-tile jobs: on a 200 x 200 image with P = 29 (blocks of 100^2
    outputs) two jobs of 7 columns whose windows grow to 100 x 100 have 7 items each; the
    image's 14 items ride two per transform: 7 pairs (not 4 + 4 job by job).  A 7-column job
    reaching 114 x 78 pixels has 2 blocks per column (14 items); a second image's lone item
    is a pair of its own."""
    import numpy as np
    spec = {"images": [dict(H=200, W=200, psf=np.ones((29, 29)), sub=0), dict(H=60, W=60, psf=np.ones((29, 29)), sub=1),
                       dict(H=200, W=200, psf=np.ones((29, 29)), sub=2)],
            "subs": [(0, 14), (14, 1), (15, 7)]}
    jobs = [(0, (14, 14, 86, 86), 7), (0, (114, 114, 186, 186), 7), (1, (10, 10, 40, 40), 1),
            (2, (100, 20, 200, 70), 7)]
    assert bench.output_window({"box": jobs[0][1]}, spec["images"][0]) == (0, 0, 100, 100)
    assert bench.output_window({"box": jobs[1][1]}, spec["images"][0]) == (100, 100, 200, 200)
    assert bench.output_window({"box": jobs[3][1]}, spec["images"][2]) == (86, 6, 200, 84)
    pairs = bench.fft_pairs_per_sub(spec, jobs)
    assert list(pairs) == [7, 1, 7]
    assert bench.FFT_PAIR_FLOP == 2 * 5 * 16384 * 14 + 6 * 16384


def test_gram_part_groups_follow_the_library_grouping():
    """Groups whose J^T W r comes from the 4 x 4-block Gram kernel: the Sersic components of
    one image with the same box form one group (6 of 7 columns = 42 columns: too wide, its
    partials stay in the convolution epilogues); a lone Sersic (7 columns) and each point
    source (its own group) qualify; a component without free parameters forms none."""
    import numpy as np
    im = dict(H=40, W=40, psf=np.ones((5, 5)), sub=0)
    box = (4, 4, 30, 30)
    comps = [dict(type=0, image=0, box=box, par=list(range(7 * i, 7 * i + 7))) for i in range(6)]
    comps.append(dict(type=0, image=0, box=(1, 1, 12, 12), par=list(range(42, 49))))
    comps.append(dict(type=1, image=0, box=(20, 20, 24, 24), par=[49, 50, 51]))
    comps.append(dict(type=1, image=0, box=(20, 20, 24, 24), par=[52, -1, -1]))
    comps.append(dict(type=0, image=0, box=(2, 2, 8, 8), par=[-1] * 7))
    spec = {"images": [im], "subs": [(0, 53)], "comps": comps}
    got = bench.gram_part_groups(spec)
    assert [(n, w) for _, w, n in got] == [(7, (0, 0, 14, 14)), (3, (18, 18, 26, 26)), (1, (18, 18, 26, 26))]
    # the wide group alone: its Gram only (no J^T W r work counted in the pairs class)
    base = bench.pair_flop_per_sub(dict(spec, comps=comps[:6]))
    assert np.isclose(base[0], 2 * 30 * 30 * (42 * 43 / 2))
    # bytes: every entry, the weights of each distinct window once (the two point sources
    # share theirs), and the residuals of each group whose J^T W r the Gram kernel forms
    ent, _ = bench.jac_entries_per_sub(spec)
    assert np.isclose(bench.pair_bytes_per_sub(spec)[0],
                      4 * (ent[0] + (30 * 30 + 14 * 14 + 8 * 8) + (14 * 14 + 8 * 8 + 8 * 8)))


def test_objective_flop_by_hand():
    """Trial objective work of a one-image sub-problem: a Sersic window (-3, -3, 5, 20) cut
    to the extended grid [-1, 11) x [-1, 13) of a 10 x 12 image with P = 3 holds 6 x 14
    pixels of 9 nodes; a point source adds no render work; the convolution is 2 P^2 per
    image pixel."""
    import numpy as np
    spec = {"images": [dict(H=10, W=12, psf=np.ones((3, 3)), sub=0)], "subs": [(0, 8)],
            "sampling": dict(s=3, rule=0, mode=0, k=0.0),
            "comps": [dict(type=0, image=0, box=(-3, -3, 5, 20), par=[0, 1, 2, 3, 4, 5, 6]),
                      dict(type=1, image=0, box=(2, 2, 6, 6), par=[7, -1, -1])]}
    ren, fwd = bench.objective_flop_per_sub(spec)
    assert ren[0] == 6 * 14 * 9 * bench.RENDER64_FLOP_PER_NODE
    assert fwd[0] == 2 * 9 * 120


def test_cutouts_counted_traffic_follows_the_kernel_sources():
    """The headline's HBM bytes per transform pair of its dominant class come from the
    committed counter summary only while the FFT kernel's sources hash to the recorded
    value."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "conv_fft_cutouts4096_hbm_counters.md")
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("|"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for src in kv["sources"].split():
        h.update(open(os.path.join(ROOT, src), "rb").read())
    got = bench.counted_record("conv_fft_cutouts4096_hbm_counters.md", kv["kernel"])
    if h.hexdigest() == kv["sources_sha256"]:
        assert got is not None and float(got["bytes_per_pair"]) > 0
        assert abs(float(got["bytes_per_pair"]) * float(got["pairs"]) -
                   float(got["read_bytes"]) - float(got["write_bytes"])) < 1e-5 * float(got["read_bytes"])
    else:
        assert got is None
    assert bench.counted_record("conv_fft_cutouts4096_hbm_counters.md", "k_conv_fft<ADJ>") is None