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
