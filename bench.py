#!/usr/bin/env python3
"""Benchmark of the chi^2 forward-modelling hot path on one MI355X.

Headline workload: 4096 independent survey cutouts, sides log-uniform in 32..256 px, each
with 1-5 elliptical Sersic galaxies and a flat sky, its own Gaussian or Moffat PSF of
15-31 px and 3 x 3 sub-pixel nodes everywhere -- the batching of many small models of
§3.2.  Every kernel of an LM iteration runs over all cutouts at once and the iteration is
replayed from one captured HIP graph; each cutout keeps its own damping, accept/reject
and FP64 Cholesky on the device.  One "step" is one such batched LM iteration; the value is
cutout LM iterations per second over the first --steps iterations from the perturbed
start, inputs resident in HBM.  The same iterations run one cutout at a time (the plain
per-galaxy path: one problem per cutout, eager launches) on a sample of cutouts give
`speedup_batched_vs_plain`.  Inputs are seeded and synthetic: parameters drawn from the
priors of the random-Sersic benchmark (§3.2, Table 1 pattern), the noise-free model
rendered by the library itself, Gaussian noise of variance model + 0.01^2.

The dominant kernel class (the Jacobian-column convolutions) is timed live with HIP events
on the library's stream inside the replayed graphs; its roofline fraction is its
algorithmic FLOP rate (2 P^2 FLOP per Jacobian entry of the cutouts that form a Jacobian
in that iteration, for the cutouts whose stamp is not rank one) over the FP32 VALU peak;
rank-one stamps (the Gaussian PSFs) take two 1-D passes, reported beside it, as is the value
with every convolution 2-D.  The CPU baseline is the FP64 test oracle run
on a sample of the cutouts by a process pool, one thread per worker.  The 512 x 512 blend
(50 Sersic + 200 point sources, 551 parameters in one fit) is reported beside it.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X FP32 vector peak: 256 CUs x 4 SIMD x 32 FMA lanes per clock x 2 FLOP x 2.4 GHz.
# Plain (unpacked) v_fmac_f32 reaches it: two waves issue VALU instructions in one cycle
# when the operands are VGPRs (FP64 vector and FP64 MFMA are half of it, 78.6).
PEAK_FP32_VALU_TFLOPS = 256 * 4 * 32 * 2 * 2.4e9 / 1e12    # 157.3
PEAK_FP64_TFLOPS = PEAK_FP32_VALU_TFLOPS / 2             # 78.6, vector and MFMA
PEAK_HBM_GBS = 8000.0


def cpu_baseline_blend(spec, data, weight):
    """The FP64 oracle on a bounded sample of one LM iteration of this workload:
    one full model evaluation (trial), the 7 Jacobian columns of one galaxy, 2
    point-source columns, J^T W J on 64 columns and one Cholesky of the 551 x 551
    system; scaled to 50 galaxies, 200 point sources and 551^2."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = os.cpu_count() or 1
    th = spec["theta_init"]
    n_gal = sum(1 for c in spec["comps"] if c["type"] == 0)
    pt_par = [c["par"][2] for c in spec["comps"] if c["type"] == 1]
    npar = spec["n_par"]
    npix = spec["images"][0]["H"] * spec["images"][0]["W"]
    t0 = time.perf_counter()
    oracle.model_image(spec, th, 0)
    t_model = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.jacobian_image(spec, th, 0, cols=list(range(7)))
    t_gal = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.jacobian_image(spec, th, 0, cols=pt_par[:2])
    t_pt = (time.perf_counter() - t0) / 2
    rng = np.random.default_rng(0)
    Js = rng.standard_normal((npix, 64))
    wv = np.asarray(weight[0], np.float64).ravel()
    t0 = time.perf_counter()
    Js.T @ (wv[:, None] * Js)
    t_ne = (time.perf_counter() - t0) * (npar / 64.0) ** 2
    X = rng.standard_normal((npar, npar))
    A = X @ X.T + npar * np.eye(npar)
    t0 = time.perf_counter()
    oracle.cholesky_or_none(A)
    t_ch = time.perf_counter() - t0
    t_iter = t_model + n_gal * t_gal + len(pt_par) * t_pt + t_ne + t_ch
    sample_s = t_model + t_gal + 2 * t_pt + t_ne * (64.0 / npar) ** 2 + t_ch
    return {
        "value": 1.0 / t_iter, "unit": "LM it/s", "cores": int(blas_threads), "kind": "oracle",
        "sample": (f"one LM iteration extrapolated from {sample_s:.1f} s of oracle work: 1 model "
                   f"({t_model:.2f} s), 7 Jacobian columns of 1 of {n_gal} galaxies ({t_gal:.2f} s), "
                   f"2 of {len(pt_par)} point-source columns, J^T W J on 64 of {npar} columns, 1 "
                   f"Cholesky of {npar}^2; NumPy elementwise work is single-threaded, the BLAS "
                   f"product uses {blas_threads} threads; extrapolated s/it = {t_iter:.1f}"),
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_cutout_iterations(job):
    """Worker: n_iter oracle LM iterations of one cutout (its own spec, data and weight)."""
    import oracle
    sub, d, w, n_iter = job
    t0 = time.perf_counter()
    oracle.lm_fit(sub, sub["theta_init"], [d], [w], n_iter)
    return time.perf_counter() - t0


def cpu_baseline_cutouts(spec, data, weight, synth, stride=16, n_iter=2):
    """The FP64 oracle on every stride-th cutout (the same sizes, PSFs and component counts
    as the whole batch), n_iter LM iterations each, spread over a process pool of one
    worker per host core (at most 16, the host share of one GPU) with one BLAS/OpenMP
    thread each; the rate is cutout iterations per wall-clock second."""
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    jobs = []
    for s_ in range(0, len(spec["subs"]), stride):
        sub = synth.sub_spec(spec, s_)
        ks = [k for k, im in enumerate(spec["images"]) if im["sub"] == s_]
        jobs.append((sub, data[ks[0]], weight[ks[0]], n_iter))
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            pool.map(_oracle_cutout_iterations, jobs[:workers])          # imports, page-in
            t0 = time.perf_counter()
            busy = pool.map(_oracle_cutout_iterations, jobs, chunksize=1)
            wall = time.perf_counter() - t0
    finally:
        for k, v in env.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    n = len(jobs) * n_iter
    return {
        "value": n / wall, "unit": "cutout LM it/s", "cores": workers, "kind": "oracle",
        "cpu": cpu_model(), "host_cpus": os.cpu_count(),
        "sample": (f"{len(jobs)} of {len(spec['subs'])} cutouts (every {stride}th), {n_iter} LM iterations each "
                   f"(Jacobian, normal equations, Cholesky, trial chi^2), {sum(busy):.1f} s of oracle work "
                   f"on {workers} worker processes with one thread each, {wall:.1f} s wall"),
    }


CONV_MODES = {"direct": 0, "fft": 1, "auto": 3}


def _conv(args, spec):
    """The workload spec with the convolution mode asked for on the command line (direct:
    the spec's own)."""
    if args.conv in ("fft", "auto"):
        spec = dict(spec)
        spec["conv_mode"] = CONV_MODES[args.conv]
    return spec


def _data(prob, spec, synth):
    """Noise-free model of the truth rendered by the library, noisy data and weights."""
    m = prob.split(prob.render(spec["theta_true"]))
    prob.check()
    data, weight = [], []
    for k, mk in enumerate(m):
        d, w = synth.make_data(mk.astype(np.float64), spec["noise"][k])
        data.append(d)
        weight.append(w)
    return data, weight


CONV_MODE = ["direct"]                # set from --conv; recorded in every line's config


def _line(rec):
    if isinstance(rec.get("config"), dict):
        rec["config"]["conv"] = CONV_MODE[0]
    if CONV_MODE[0] == "fft" and isinstance(rec.get("roofline"), dict):
        # the FLOP count is the direct convolution's (2 P^2 per output), which the FFT tiles
        # replace with far fewer operations: a rate, not a fraction of any peak
        rf = rec.pop("roofline")
        rec["direct_equivalent"] = {
            "kernel": rf.get("kernel"), "tflops": rf.get("achieved"), "unit": "TFLOP/s",
            "note": "2 P^2 FLOP per output of the direct convolution over the FFT-mode time"}
    print(json.dumps(rec), flush=True)


def _mpix(prob, spec, torch, reps):
    out = torch.empty(prob.n_pix, dtype=torch.float32, device=prob.device)
    th = torch.as_tensor(spec["theta_true"], dtype=torch.float64, device=prob.device)
    prob.render(th, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.render(th, out)
    torch.cuda.synchronize()
    return prob.n_pix * reps / (time.perf_counter() - t0) / 1e6


def calls_per_launch_count(prob, th, dd, ww):
    """Timed launches of the objective convolution per objective evaluation and of the
    adjoint convolution per gradient evaluation (one per (P, tile shape) range), read from
    one timed call of each."""
    prob.set_timing(True, classes=["conv_fwd", "conv_adj"])
    prob.chi2(th, dd, ww)
    n_fwd = prob.timing()["conv_fwd"][1]
    prob.set_timing(True, classes=["conv_fwd", "conv_adj"])
    prob.chi2_grad(th, dd, ww)
    n_adj = prob.timing()["conv_adj"][1]
    prob.set_timing(False)
    return max(1, n_fwd), max(1, n_adj)


def class_rooflines(spec, prob, kt, phases, per_call=(1, 1), n_obj=None):
    """Roofline of each timed kernel class that has an algorithmic count, over a timed
    region with `phases` Jacobian phases (kt: {class: (ms, launches)}; per_call: launches
    per objective and per gradient evaluation, which count the evaluations when every
    launch does its work; n_obj: the objective evaluations that did work, where some
    launches find nothing to do):
    2-D Jacobian convolutions (2 P^2 per Jacobian entry of images whose stamp is not rank
    one, and 2 P^2 per image pixel for each live-PSF parameter column; FP32 vector peak),
    the objective convolution (2 P^2 per image pixel per evaluation; FP64 or FP32 vector
    peak), the adjoint convolution (2 P^2 per image pixel per gradient; FP32 vector peak),
    the J^T W J tiles (2 FLOP per pixel and upper-triangle column pair of each pair of
    column groups that meet; FP64 MFMA peak).  Returns (dominant of those by time, all)."""
    conv_mode = spec.get("conv_mode", 0)
    sep = rank_one_images(spec, conv_mode)
    ent, flop = jac_entries_per_sub(spec, exclude_images=sep)
    fp64 = prob.objective == 0
    img_flop = [2.0 * np.asarray(im["psf"]).shape[0] ** 2 * int(im.get("up", 1)) ** 2 * im["H"] * im["W"]
                for im in spec["images"]]
    fwd = sum(img_flop)
    psf_cols = sum(img_flop[int(m["image"])] * sum(1 for q in m["par"] if q >= 0)
                   for m in spec.get("psf_models", []))
    pair_flop = float(pair_flop_per_sub(spec).sum())
    pair_bytes = float(pair_bytes_per_sub(spec).sum())
    n_fwd = kt.get("conv_fwd", (0.0, 0))[1] / per_call[0] if n_obj is None else n_obj
    n_adj = kt.get("conv_adj", (0.0, 0))[1] / per_call[1]
    models = {}
    if conv_mode == 0:       # the direct-convolution counts do not price an FFT convolution
        models["conv_jcol"] = ((float(flop.sum()) + psf_cols) * phases, PEAK_FP32_VALU_TFLOPS,
                               "k_conv<P,JCOL> (2-D)")
        models["conv_fwd"] = (fwd * n_fwd, PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_VALU_TFLOPS,
                              "k_conv<P,FWD,%s>" % ("double" if fp64 else "float"))
        models["conv_adj"] = (fwd * n_adj, PEAK_FP32_VALU_TFLOPS, "k_conv<P,ADJ>")
    out = {}
    ms_p = kt.get("pairs", (0.0, 0))[0]
    if ms_p > 0 and pair_flop > 0:
        out["pairs"] = dict(pair_roof(pair_flop * phases, pair_bytes * phases, ms_p, "k_pair / k_gram4 (FP64 MFMA)"),
                            ms_total=ms_p, traffic=None)
    for cls, (fl, peak, name) in models.items():
        ms = kt.get(cls, (0.0, 0))[0]
        if ms <= 0 or fl <= 0:
            continue
        ach = fl / (ms * 1e-3) / 1e12
        out[cls] = {"bound": "alu", "kernel": name, "achieved": ach, "peak": peak,
                    "unit": "TFLOP/s", "frac": ach / peak, "ms_total": ms, "traffic": None}
    dom = max(out, key=lambda k: out[k]["ms_total"]) if out else None
    return (out[dom] if dom else None), out


GRAM4_MAX_COLS = 36          # column groups up to this width take the 4 x 4-block Gram kernel


def gram_part_groups(spec):
    """Column groups as the library forms them (the Sersic components of one image with the
    same box share one, each point source has its own) that the 4 x 4-block Gram kernel
    forms with themselves, and which therefore also take their columns' J^T W r and sum w J
    there: (image, output window, columns) of groups of at most GRAM4_MAX_COLS columns."""
    groups, order = {}, []
    for i, c in enumerate(spec["comps"]):
        n = sum(1 for q in c["par"] if q >= 0)
        if n == 0:
            continue
        key = (c["image"], tuple(c["box"])) if int(c.get("type", 0)) == 0 else ("point", i)
        if key not in groups:
            groups[key] = [c["image"], output_window(c, spec["images"][c["image"]]), 0]
            order.append(key)
        groups[key][2] += n
    out = []
    for key in order:
        k, w, n = groups[key]
        if w[2] > w[0] and w[3] > w[1] and n <= GRAM4_MAX_COLS:
            out.append((k, w, n))
    return out


def pair_flop_per_sub(spec):
    """J^T W J work of each sub-problem: 2 FLOP per pixel and column pair of the upper
    triangle, over the overlap of the output windows of every pair of column groups on one
    image (a component's free parameters form a group; the algorithmic count, whatever
    the tiles pad); and, for the groups whose J^T W r and sum w J the Gram kernel forms
    (gram_part_groups), 4 FLOP per Jacobian entry (w J, its product with r and two sums)."""
    groups = []
    for c in spec["comps"]:
        n = sum(1 for q in c["par"] if q >= 0)
        if n:
            groups.append((c["image"], output_window(c, spec["images"][c["image"]]), n))
    out = np.zeros(len(spec["subs"]))
    for a in range(len(groups)):
        for b in range(a, len(groups)):
            (ia, wa, na), (ib, wb, nb) = groups[a], groups[b]
            if ia != ib:
                continue
            npix = max(0, min(wa[2], wb[2]) - max(wa[0], wb[0])) * max(0, min(wa[3], wb[3]) - max(wa[1], wb[1]))
            out[spec["images"][ia]["sub"]] += 2.0 * npix * (na * (na + 1) / 2 if a == b else na * nb)
    for k, w, n in gram_part_groups(spec):
        out[spec["images"][k]["sub"]] += 4.0 * n * (w[2] - w[0]) * (w[3] - w[1])
    return out


def pair_bytes_per_sub(spec):
    """Algorithmic HBM bytes of each sub-problem's J^T W J: every stored Jacobian entry and
    every weight of the output windows read once (4 B each), and the residual of each pixel
    of the windows whose J^T W r the Gram kernel forms."""
    ent, _ = jac_entries_per_sub(spec)
    px = np.zeros(len(spec["subs"]))
    seen = set()
    for c in spec["comps"]:
        im = spec["images"][c["image"]]
        key = (c["image"], output_window(c, im))
        if key in seen or not any(q >= 0 for q in c["par"]):
            continue
        seen.add(key)
        y0, x0, y1, x1 = key[1]
        px[im["sub"]] += max(0, y1 - y0) * max(0, x1 - x0)
    for k, w, n in gram_part_groups(spec):
        px[spec["images"][k]["sub"]] += (w[2] - w[0]) * (w[3] - w[1])
    return 4.0 * (ent + px)


def pair_roof(flop, nbytes, ms, kernel):
    """Roofline of the J^T W J class: bound by whichever of the FP64 MFMA peak and the HBM
    bandwidth its algorithmic FLOP and bytes take longer on; frac against that roof."""
    hbm = nbytes / (PEAK_HBM_GBS * 1e9) > flop / (PEAK_FP64_TFLOPS * 1e12)
    sec = ms * 1e-3
    if hbm:
        ach = nbytes / sec / 1e9 if sec > 0 else 0.0
        return {"bound": "hbm", "kernel": kernel, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "algorithmic_bytes": nbytes, "flop": flop}
    ach = flop / sec / 1e12 if sec > 0 else 0.0
    return {"bound": "mfma", "kernel": kernel, "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP64_TFLOPS, "algorithmic_bytes": nbytes, "flop": flop}


RENDER64_FLOP_PER_NODE = 73.0   # 47 FP64 operations per Sersic node, 26 of them FMAs (2 FLOP)


def objective_flop_per_sub(spec):
    """Per sub-problem, one trial objective evaluation: (FP64 render, FP64 convolution).
    Render: RENDER64_FLOP_PER_NODE per node, s^2 nodes per pixel of each Sersic window on
    the extended grid (uniform sampling); convolution: 2 P^2 per image pixel."""
    smp = spec["sampling"]
    assert int(smp["mode"]) == 0, "node counts are exact for uniform sampling only"
    nodes = int(smp["s"]) ** 2
    ren = np.zeros(len(spec["subs"]))
    fwd = np.zeros(len(spec["subs"]))
    for im in spec["images"]:
        P = np.asarray(im["psf"]).shape[0]
        fwd[im["sub"]] += 2.0 * P * P * im["H"] * im["W"]
    for c in spec["comps"]:
        if int(c["type"]) != 0:
            continue
        im = spec["images"][c["image"]]
        h = (np.asarray(im["psf"]).shape[0] - 1) // 2
        y0, x0, y1, x1 = c["box"]
        npix = max(0, min(y1, im["H"] + h) - max(y0, -h)) * max(0, min(x1, im["W"] + h) - max(x0, -h))
        ren[im["sub"]] += npix * nodes * RENDER64_FLOP_PER_NODE
    return ren, fwd


def output_window(c, im):
    """Output pixels [y0, x0, y1, x1) a component's Jacobian columns reach: its window
    grown by the PSF half-width, cut to the image, in output (coarse) pixels."""
    P = np.asarray(im["psf"]).shape[0]
    up = int(im.get("up", 1))
    h = (P - 1) // 2
    y0, x0, y1, x1 = c["box"]
    oy0, ox0 = max(0, y0 - h) // up, max(0, x0 - h) // up
    oy1, ox1 = min(up * im["H"], y1 + h), min(up * im["W"], x1 + h)
    return oy0, ox0, -(-oy1 // up), -(-ox1 // up)


def jac_entries_per_sub(spec, exclude_images=()):
    """Jacobian entries (output pixels of every convolved column) of each sub-problem:
    a free parameter of a Sersic or point source is one column over the output pixels its
    window reaches (the window grown by the PSF half-width, cut to the image); the sky
    column is 1 and is not convolved.  Returns (entries, 2 P^2 FLOP) per sub-problem."""
    ent = np.zeros(len(spec["subs"]))
    flop = np.zeros(len(spec["subs"]))
    for c in spec["comps"]:
        if c["image"] in exclude_images:
            continue
        im = spec["images"][c["image"]]
        P = np.asarray(im["psf"]).shape[0]
        up = int(im.get("up", 1))
        oy0, ox0, oy1, ox1 = output_window(c, im)
        npix = max(0, oy1 - oy0) * max(0, ox1 - ox0)
        ncol = sum(1 for q in c["par"] if q >= 0)
        ent[im["sub"]] += ncol * npix
        flop[im["sub"]] += ncol * npix * 2.0 * P * P * up * up
    return ent, flop


TILE_HW = [(32, 64), (16, 64), (32, 32), (16, 32)]   # the library's four direct tile shapes
# One FFT-tile item pair: a forward and an inverse 128 x 128 complex transform at the
# conventional 5 N log2 N operations each (N = 128^2), and the spectrum product (6 per element)
FFT_N = 128 * 128
FFT_PAIR_FLOP = 2 * 5 * FFT_N * 14 + 6 * FFT_N


def fft_pairs_per_sub(spec, fft_jobs):
    """Transform pairs of the FFT-tile Jacobian jobs per sub-problem: each job has nch
    channels of ceil(h / (129 - P)) ceil(w / (129 - P)) output blocks, and the items of one
    image ride two per transform (its jobs' items are consecutive in the launch)."""
    items = {}
    for k, box, nch in fft_jobs:
        im = spec["images"][k]
        B = 129 - np.asarray(im["psf"]).shape[0]
        y0, x0, y1, x1 = output_window({"box": box}, im)
        items[k] = items.get(k, 0) + nch * (-(-(y1 - y0) // B)) * (-(-(x1 - x0) // B))
    out = np.zeros(len(spec["subs"]))
    for k, n in items.items():
        out[spec["images"][k]["sub"]] += (n + 1) // 2
    return out
AUTO_FFT_PAIR_COST = 1.0e6                            # APX_AUTO_FFT_PAIR_COST


def auto_fft_job(P, h, w, nch):
    """The library's automatic-mode rule for one job of nch channels with an h x w output:
    FFT tiles when ceil(nch blocks / 2) transform pairs cost less than the cheapest direct
    tiling by the operation-count model."""
    def tile_model(th, tw):
        return th * tw * (P * P + 10.0) + 8.0 * (th + P - 1) * (tw + P - 1) + 3000.0
    direct = min(-(-h // th) * -(-w // tw) * tile_model(th, tw) for th, tw in TILE_HW)
    B = 129 - P
    blocks = -(-h // B) * -(-w // B)
    return ((nch * blocks + 1) // 2) * AUTO_FFT_PAIR_COST < direct * nch


def auto_fft_groups(spec, rank_one, cost=True):
    """Jacobian-column jobs that run on FFT tiles in automatic mode, as (image, box, columns):
    the library's column groups (Sersic components of one image with the same box share one;
    each point source has its own) on images with a fixed stamp of P >= 15 that is not rank
    one (`rank_one`: the images the library found rank one), no sub-pixel grid, an output
    box of at least 32 x 32, and FFT priced below direct (auto_fft_job).  cost=False: every
    such job (the FFT mode's rule; pass no rank-one images there)."""
    live = {int(m["image"]) for m in spec.get("psf_models", [])}
    groups, order = {}, []
    for i, c in enumerate(spec["comps"]):
        n = sum(1 for q in c["par"] if q >= 0)
        if n == 0 or c["box"][2] <= c["box"][0]:
            continue
        key = (c["image"], tuple(c["box"])) if int(c["type"]) == 0 else ("point", i)
        if key not in groups:
            groups[key] = [c["image"], c, 0]
            order.append(key)
        groups[key][2] += n
    out = []
    for key in order:
        k, c, nch = groups[key]
        im = spec["images"][k]
        P = np.asarray(im["psf"]).shape[0]
        if k in live or k in rank_one or int(im.get("up", 1)) != 1 or P < 15:
            continue
        y0, x0, y1, x1 = output_window(c, im)
        h, w = y1 - y0, x1 - x0
        if h >= 32 and w >= 32 and (not cost or auto_fft_job(P, h, w, nch)):
            out.append((k, tuple(c["box"]), nch))
    return out


def rank_one_images(spec, conv_mode):
    """Images whose Jacobian columns the library convolves as two 1-D passes: the stamp is
    a_u b_v to FP32 rounding (the library's own test, repeated here: with the largest entry
    at (u0, v0), a_u = K[u, v0], b_v = K[u0, v] / K[u0, v0], every entry within 4e-7 of
    itself plus 1e-9 of the largest), not live, not sub-pixel, in direct or automatic mode."""
    out = set()
    if conv_mode not in (0, 3):
        return out
    live = {int(m["image"]) for m in spec.get("psf_models", [])}
    for k, im in enumerate(spec["images"]):
        K = np.asarray(im["psf"], np.float32).astype(np.float64)
        if k in live or int(im.get("up", 1)) != 1 or K.shape[0] < 3:
            continue
        u0, v0 = np.unravel_index(int(np.argmax(np.abs(K))), K.shape)
        kmax = abs(K[u0, v0])
        if not kmax > 0:
            continue
        a = K[:, v0]
        b = K[u0, :] / K[u0, v0]
        if np.all(np.abs(K - np.outer(a, b)) <= 4e-7 * np.abs(K) + 1e-9 * kmax):
            out.add(k)
    return out


def run_cutouts(args, torch, apx, synth):
    """4096 independent cutouts: the batched LM (every kernel over all cutouts, one HIP
    graph replay per iteration) against the plain per-cutout path (one problem per
    cutout, eager launches).  Returns the headline record."""
    t0 = time.perf_counter()
    spec = synth.cutouts()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    Ps = [np.asarray(im["psf"]).shape[0] for im in spec["images"]]
    costs = load_tile_costs(args.tile_costs_in) if args.tile_costs_in else None
    prob = apx.Problem(_conv(args, spec), tile_costs=costs)
    t_plan = time.perf_counter() - t0
    if args.tile_costs_out:
        save_tile_costs(prob, Ps, args.tile_costs_out)
    n_sub = len(spec["subs"])
    print(f"[bench] cutouts: {n_sub} sub-problems, {prob.n_pix / 1e6:.1f} Mpix, "
          f"plan {t_plan:.1f} s, workspace {prob.workspace_bytes / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    data, weight = _data(prob, spec, synth)
    dd, ww = prob.pixels(data), prob.pixels(weight)
    ent, flop_sub = jac_entries_per_sub(spec)
    assert int(ent.sum()) == prob.n_jac, (ent.sum(), prob.n_jac)
    # cutouts whose stamp is rank one take the two-pass Jacobian kernel, and in automatic
    # (or FFT) mode some take FFT tiles: the 2-D class's algorithmic work counts only the
    # others (the bench repeats the library's rules and checks it planned the same jobs)
    mode = _conv(args, spec).get("conv_mode", 0)
    sep_img = rank_one_images(spec, mode)
    assert prob.tile_shapes(1)[5] == len(sep_img), (prob.tile_shapes(1), len(sep_img))
    fft_jobs = auto_fft_groups(spec, sep_img, cost=mode == 3) if mode in (1, 3) else []
    assert prob.tile_shapes(1)[4] == len(fft_jobs), (prob.tile_shapes(1), len(fft_jobs))
    sep_sub = np.zeros(n_sub, bool)
    for k in sep_img:
        sep_sub[spec["images"][k]["sub"]] = True
    fft_flop_sub = np.zeros(n_sub)
    for k, box, nch in fft_jobs:
        im = spec["images"][k]
        y0, x0, y1, x1 = output_window({"box": box}, im)
        fft_flop_sub[im["sub"]] += nch * (y1 - y0) * (x1 - x0) * 2.0 * np.asarray(im["psf"]).shape[0] ** 2
    flop_2d_sub = np.where(sep_sub, 0.0, flop_sub - fft_flop_sub)
    fft_pair_sub = fft_pairs_per_sub(spec, fft_jobs)
    ent_sep_sub = np.where(sep_sub, ent, 0.0)

    # eager pass over the same iterations, one at a time: which cutouts form a Jacobian in
    # each iteration (need_jac), for the algorithmic FLOP count of the Jacobian phases
    ren_sub, fwd_sub = objective_flop_per_sub(spec)
    pair_sub = pair_flop_per_sub(spec)
    pbyte_sub = pair_bytes_per_sub(spec)
    th_e, st_e = prob.lm_init(spec["theta_init"], dd, ww)
    flop_jac = ent_sep = flop_fft = flop_ren = flop_fwd = flop_pair = byte_pair = pairs_fft = 0.0
    for _ in range(args.steps):
        need = prob.lm_state(st_e)["need_jac"] != 0
        flop_jac += float(flop_2d_sub[need].sum())
        ent_sep += float(ent_sep_sub[need].sum())
        flop_fft += float(fft_flop_sub[need].sum())
        pairs_fft += float(fft_pair_sub[need].sum())
        flop_pair += float(pair_sub[need].sum())
        byte_pair += float(pbyte_sub[need].sum())
        prob.lm_step(dd, ww, th_e, st_e)
        ev = np.isfinite(prob.lm_state(st_e)["chi2_trial"])     # trials whose objective ran
        flop_ren += float(ren_sub[ev].sum())
        flop_fwd += float(fwd_sub[ev].sum())
    prob.check()
    torch.cuda.synchronize()
    print(f"[bench] eager pass done ({flop_jac / 1e12:.2f} TFLOP of 2-D Jacobian convolutions, "
          f"{ent_sep / 1e9:.2f} G entries by two passes, {len(fft_jobs)} jobs on FFT tiles)",
          file=sys.stderr, flush=True)

    # warm-up: captures the iteration graph with HIP events around the two classes that can
    # be the largest (the trial render, and the FFT-tile or the 2-D Jacobian convolutions);
    # every event mark costs the replay ~12 us, so the other classes are timed in a second
    # graph pass below and their marks stay out of the timed region
    jclasses = ["render", "conv_fft" if mode in (1, 3) else "conv_jcol"]
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    prob.set_timing(True, classes=jclasses)
    prob.lm_run(max(1, args.warmup), dd, ww, th, st, use_graph=True)
    prob.lm_init(spec["theta_init"], dd, ww, theta_out=th, state_out=st)
    prob.timing()
    prob.set_timing(True, classes=jclasses)     # clears the records (the start's objective
    torch.cuda.synchronize()                    # evaluation is not a timed trial), keeps the graph

    # timed region: K batched iterations from the perturbed start, graph replays
    t0 = time.perf_counter()
    prob.lm_run(args.steps, dd, ww, th, st, use_graph=True)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    kt = prob.timing()
    prob.set_timing(False)
    prob.check()
    stt = prob.lm_state(st)
    same = bool(torch.equal(th, th_e))
    batched = n_sub * args.steps / t_graph
    print(f"[bench] {args.steps} batched iterations in {t_graph * 1e3:.1f} ms (graph = eager: {same})",
          file=sys.stderr, flush=True)

    # eager batched, the same iterations
    th2, st2 = prob.lm_init(spec["theta_init"], dd, ww)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.lm_run(args.steps, dd, ww, th2, st2, use_graph=False)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0

    # the other kernel classes, from a second instrumented graph pass over the same
    # iterations (their event marks stay out of the timed replays)
    oclasses = ["conv_fwd", "pairs"] + [c for c in ("conv_jcol", "conv_sep", "conv_fft") if c not in jclasses]
    prob.set_timing(True, classes=oclasses)
    prob.lm_init(spec["theta_init"], dd, ww, theta_out=th2, state_out=st2)
    prob.lm_run(1, dd, ww, th2, st2, use_graph=True)            # captures with the new marks
    prob.lm_init(spec["theta_init"], dd, ww, theta_out=th2, state_out=st2)
    prob.timing()
    prob.set_timing(True, classes=oclasses)     # after lm_init: its evaluation is not a trial
    prob.lm_run(args.steps, dd, ww, th2, st2, use_graph=True)
    ko = prob.timing()
    prob.set_timing(False)
    kk = {c: (kt[c] if c in jclasses else ko[c]) for c in kt}
    jcol_ms, jcol_launches = kk["conv_jcol"]
    sep_ms, _ = kk["conv_sep"]
    fft_ms, _ = kk["conv_fft"]
    achieved = flop_jac / (jcol_ms * 1e-3) / 1e12 if jcol_ms > 0 else 0.0
    if mode == 1:            # FFT mode: the Jacobian runs on FFT tiles (direct-equivalent rate)
        jcol_ms, flop_jac = fft_ms, flop_fft
        achieved = flop_jac / (jcol_ms * 1e-3) / 1e12 if jcol_ms > 0 else 0.0

    def cls_roof(flop, ms, peak, kernel, bound="alu", timed=False):
        ach = flop / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        return {"bound": bound, "kernel": kernel, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "ms_per_step": ms / max(1, args.steps), "traffic": None,
                "timed_region": timed}
    per_class = {
        "conv_jcol": cls_roof(flop_jac, jcol_ms, PEAK_FP32_VALU_TFLOPS,
                              "k_conv<P,JCOL> (2-D Jacobian-column convolutions: all PSF sizes and tile shapes "
                              "of a phase, cutouts whose stamp is not rank one and whose job stays on direct "
                              "tiles)", timed="conv_jcol" in jclasses or mode == 1),
        "render": cls_roof(flop_ren, kt["render"][0], PEAK_FP64_TFLOPS,
                           "k_render64 (FP64 trial render; %g FLOP per Sersic node)" % RENDER64_FLOP_PER_NODE,
                           timed=True),
        "conv_fft": cls_roof(pairs_fft * FFT_PAIR_FLOP, fft_ms, PEAK_FP32_VALU_TFLOPS,
                             "k_conv_fft<JCOL> (FFT-tile Jacobian convolutions; 5 N log2 N per 128^2 "
                             "transform, two transforms and the spectrum product per item pair)",
                             timed="conv_fft" in jclasses),
        "conv_fwd": cls_roof(flop_fwd, ko["conv_fwd"][0], PEAK_FP64_TFLOPS, "k_conv<P,FWD,double> (FP64 objective)"),
        "pairs": dict(pair_roof(flop_pair, byte_pair, ko["pairs"][0], "k_gram4 / k_pair (FP64 MFMA)"),
                      ms_per_step=ko["pairs"][0] / max(1, args.steps), traffic=None, timed_region=False),
    }
    per_class["conv_jcol"].update({"ms_per_phase": jcol_ms / max(1, args.steps),
                                   "flop_per_phase": flop_jac / max(1, args.steps), "launch_groups": jcol_launches})
    per_class["conv_fft"].update({"pairs_per_phase": pairs_fft / max(1, args.steps), "jobs": len(fft_jobs)})
    # the dominant class: the larger of the two timed in the timed region; the record says
    # whether every class timed in the second pass took less time
    dom = max((c for c in ("conv_jcol", "render", "conv_fft") if c in jclasses),
              key=lambda k: per_class[k]["ms_per_step"])
    dom_is_largest = all(v["ms_per_step"] <= per_class[dom]["ms_per_step"] for v in per_class.values())
    if mode == 1:            # FFT mode reports the Jacobian's direct-equivalent rate
        dom = "conv_jcol"

    # context: the same K iterations with every convolution direct (rank-one stamps by two
    # passes, no FFT tiles), and with every convolution 2-D
    context = {}
    if not args.no_2d_context:
        modes = [("all_2d_convolutions", apx.CONV_DIRECT_2D)]
        if mode == apx.CONV_AUTO:
            modes.insert(0, ("direct_mode", apx.CONV_DIRECT))
        elif mode == apx.CONV_DIRECT:
            modes.insert(0, ("auto_mode", apx.CONV_AUTO))
        for name, m in modes:
            q2 = apx.Problem(dict(spec, conv_mode=m))
            t2, s2 = q2.lm_init(spec["theta_init"], dd, ww)
            q2.lm_run(1, dd, ww, t2, s2, use_graph=True)
            q2.lm_init(spec["theta_init"], dd, ww, theta_out=t2, state_out=s2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            q2.lm_run(args.steps, dd, ww, t2, s2, use_graph=True)
            torch.cuda.synchronize()
            context[name] = n_sub * args.steps / (time.perf_counter() - t0)
            q2.check()
            q2.close()
            print(f"[bench] context {name}: {context[name]:.0f} cutout LM it/s", file=sys.stderr, flush=True)

    # plain path on a sample of cutouts: one problem per cutout, K eager iterations with
    # device-side control and one synchronisation at the end; also with a host read of the
    # LM state after every iteration (a host-driven accept/reject loop)
    sample = list(range(0, n_sub, max(1, n_sub // 32)))
    t_plain = t_plain_host = 0.0
    th_all = th.cpu().numpy()
    plain_dev = 0.0
    for s_ in sample:
        sub = synth.sub_spec(spec, s_)
        pp = apx.Problem(_conv(args, sub))
        ks = [k for k, im in enumerate(spec["images"]) if im["sub"] == s_]
        d_s = pp.pixels([data[k] for k in ks])
        w_s = pp.pixels([weight[k] for k in ks])
        ths, sts = pp.lm_init(sub["theta_init"], d_s, w_s)
        pp.lm_step(d_s, w_s, ths, sts)                # warm-up
        pp.lm_init(sub["theta_init"], d_s, w_s, theta_out=ths, state_out=sts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pp.lm_run(args.steps, d_s, w_s, ths, sts)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        p0, n = spec["subs"][s_]
        ref = th_all[p0:p0 + n]
        plain_dev = max(plain_dev, float(np.max(np.abs(ths.cpu().numpy() - ref) / (np.abs(ref) + sub["scale"]))))
        pp.lm_init(sub["theta_init"], d_s, w_s, theta_out=ths, state_out=sts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pp.lm_step(d_s, w_s, ths, sts)
            pp.lm_state(sts)
        t_plain_host += time.perf_counter() - t0
        pp.close()
    plain = len(sample) * args.steps / t_plain
    plain_host = len(sample) * args.steps / t_plain_host

    # parameter covariance of every cutout at the last iterate (one wave per cutout)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.covariance(th, dd, ww)
    torch.cuda.synchronize()
    cov_ms = (time.perf_counter() - t0) * 1e3
    mpix = _mpix(prob, spec, torch, 5)
    kv = counted_record("render64_cutouts4096_hbm_counters.md", "k_render64 (cutouts)")
    if kv is not None:
        per_class["render"]["traffic"] = float(kv["bytes_per_flop"]) * flop_ren / max(1, args.steps)
        per_class["render"]["traffic_unit"] = "bytes/step"
    # HBM bytes of the FFT-tile class: the counted bytes per transform pair of the counter
    # summary (same kernel sources) times this run's pairs per step
    kv = counted_record("conv_fft_cutouts4096_hbm_counters.md", "k_conv_fft<JCOL> (cutouts)")
    if kv is not None and mode == 3:
        per_class["conv_fft"]["traffic"] = float(kv["bytes_per_pair"]) * pairs_fft / max(1, args.steps)
        per_class["conv_fft"]["traffic_unit"] = "bytes/step"
    roof = dict(per_class[dom])
    roof["class"] = dom
    roof["largest_class"] = dom_is_largest
    rec = {
        "metric": "LM iters/s & Mpix/s rendered (fused adjoint+batched vs plain) at oracle rtol",
        "value": batched, "unit": "cutout LM it/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_graph * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 Jacobian / f64 objective+normal equations",
        "data": "synthetic (seeded; noise-free model rendered by the library, Gaussian noise)",
        "config": {"workload": "4096 cutouts, side 32-256 px log-uniform, 1-5 Sersic + sky each, "
                               "Gaussian/Moffat PSF 15-31 px, 3x3 nodes, batched LM with graph replay",
                   "conv": {0: "direct", 1: "fft", 2: "direct_2d", 3: "auto"}[mode],
                   "n_sub": n_sub, "n_par": spec["n_par"], "n_pix": prob.n_pix, "n_jac": prob.n_jac,
                   "plan_s": t_plan, "generate_s": t_gen},
        "batch_it_per_s": args.steps / t_graph,
        "eager_batch_it_per_s": args.steps / t_eager, "graph_equals_eager": same,
        "plain_cutout_it_per_s": plain, "speedup_batched_vs_plain": batched / plain,
        "plain_host_sync_cutout_it_per_s": plain_host, "speedup_batched_vs_plain_host_sync": batched / plain_host,
        "plain_sample_cutouts": len(sample),
        "plain_vs_batched_max_dtheta": plain_dev,
        "mpix_per_s": mpix,
        "roofline": roof,
        "roofline_per_class": per_class,
        "roofline_per_class_note": "classes with timed_region false were timed in a second graph pass over "
                                   "the same iterations",
        "eager_pass_flop_2d": flop_jac, "eager_pass_flop_render": flop_ren,
        "two_pass_jacobian": {"kernel": "k_conv_sep<P> (rank-one stamps)", "ms_per_phase": sep_ms / max(1, args.steps),
                              "entries_per_phase": ent_sep / max(1, args.steps), "images": len(sep_img)},
        "fft_jacobian": {"kernel": "k_conv_fft<JCOL> (128x128 overlap-save tiles)", "jobs": len(fft_jobs),
                         "ms_per_phase": fft_ms / max(1, args.steps),
                         "direct_equivalent_tflops": flop_fft / (fft_ms * 1e-3) / 1e12 if fft_ms > 0 else None,
                         "note": "2 P^2 per Jacobian entry of these jobs over their FFT time: the rate a direct "
                                 "convolution would need to match them"},
        "context_cutout_it_per_s": context,
        "covariance_ms": cov_ms,
        "accepted_mean": float(np.mean(stt["n_accept"])),
        "tile_shapes": tile_choice(prob),
    }
    prob.close()
    return rec, spec, data, weight


def run_field(args, torch, apx, synth):
    """2048 x 2048 field, 500 windowed Sersics + sky, Moffat 51 x 51: chi^2 gradient
    evaluations per second by the adjoint path; checked against central differences of
    the FP64 chi^2 on 32 seeded parameters."""
    spec = synth.field()
    prob = apx.Problem(_conv(args, spec))
    data, weight = _data(prob, spec, synth)
    dd, ww = prob.pixels(data), prob.pixels(weight)
    th = torch.as_tensor(spec["theta_init"], dtype=torch.float64, device=prob.device)
    for _ in range(3):
        prob.chi2_grad(th, dd, ww)
    torch.cuda.synchronize()
    reps = max(args.steps, 1) * 50
    prob.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        g, c2 = prob.chi2_grad(th, dd, ww)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = prob.timing()
    prob.set_timing(False)
    g = g.cpu().numpy()
    rng = np.random.default_rng(33)
    idx = rng.choice(spec["n_par"], 32, replace=False)
    fd_err = []
    base = spec["theta_init"].copy()
    for k in idx:
        # 1e-3 of the parameter's own scale: its value, or Re for a centre coordinate (a
        # step relative to x ~ 2000 px would cross the profile's cusp)
        ref = spec["scale"][k] if spec["kinds"][k] in (synth.K_X, synth.K_Y) else abs(base[k])
        h = 1e-3 * max(ref, 1e-2)
        tp, tm = base.copy(), base.copy()
        tp[k] += h
        tm[k] -= h
        cp = float(prob.chi2(tp, dd, ww).cpu()[0])
        cm = float(prob.chi2(tm, dd, ww).cpu()[0])
        fd = (cp - cm) / (2 * h)
        fd_err.append(abs(fd - g[k]) / max(abs(g[k]), 1e-3 * np.max(np.abs(g))))
    kind_names = ["x0", "y0", "q", "PA", "n", "Re", "log10 Ie", "log10 F", "sky", "psf n", "psf R_d"]
    worst = int(np.argmax(fd_err))
    kw = int(spec["kinds"][idx[worst]])
    comp = [c for c in spec["comps"] if idx[worst] in c["par"]]
    fd_worst = {"kind": kind_names[kw], "rel_err": float(fd_err[worst]),
                "sersic_n": float(base[comp[0]["par"][4]]) if comp and comp[0]["type"] == 0 else None}
    P_psf = spec["images"][0]["psf"].shape[0]
    # the adjoint convolution: direct tiles, or FFT tiles in FFT mode (their own timing class)
    adj_ms = kt["conv_adj"][0] + kt["conv_fft"][0]
    adj_n = kt["conv_adj"][1] + kt["conv_fft"][1]
    flop_adj = 2.0 * P_psf * P_psf * prob.n_ext * adj_n
    achieved = flop_adj / (adj_ms * 1e-3) / 1e12 if adj_ms > 0 else 0.0
    # the FP64 objective convolution (model, residual and chi^2 of each evaluation):
    # 2 P^2 FLOP per image pixel on the FP64 vector units
    fwd_ms, _ = kt["conv_fwd"]
    flop_fwd = 2.0 * P_psf * P_psf * prob.n_pix * reps
    ach_fwd = flop_fwd / (fwd_ms * 1e-3) / 1e12 if fwd_ms > 0 else 0.0
    adj_name = f"k_conv_fft<ADJ> (P = {P_psf}, FP32)" if kt["conv_fft"][1] else f"k_conv<{P_psf},ADJ> (FP32)"
    rf_adj = {"bound": "alu", "kernel": adj_name, "achieved": achieved,
              "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS,
              "ms_per_eval": adj_ms / reps}
    rf_fwd = {"bound": "alu", "kernel": f"k_conv<{P_psf},FWD,double> (FP64)", "achieved": ach_fwd,
              "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach_fwd / PEAK_FP64_TFLOPS,
              "ms_per_eval": fwd_ms / reps}
    dominant, other = (rf_fwd, rf_adj) if fwd_ms >= adj_ms else (rf_adj, rf_fwd)
    _line({
        "metric": "LM iters/s & Mpix/s rendered (fused adjoint+batched vs plain) at oracle rtol",
        "workload": "field", "value": reps / dt, "unit": "gradient evals/s",
        "ms_per_gradient": dt * 1e3 / reps, "n_gpus": 1, "evals": reps,
        "fd_check_32": {"max_rel_err": float(np.max(fd_err)), "median_rel_err": float(np.median(fd_err)),
                        "h": "1e-3 of |theta_k| (of Re for centre coordinates)", "worst": fd_worst},
        "mpix_per_s": _mpix(prob, spec, torch, 10),
        "roofline": dominant, "roofline_other_conv": other,
        "kernel_ms_per_eval": {k: round(v[0] / reps, 4) for k, v in kt.items()},
        "tile_shapes": tile_choice(prob),
        "config": {"workload": "2048x2048 field, 500 Sersic (10 Re windows) + sky, Moffat 51x51 beta 3 "
                               "FWHM 4, 3x3 nodes", "n_par": spec["n_par"], "n_pix": prob.n_pix},
        "dtype": "f32 adjoint / f64 objective", "data": "synthetic"})
    return 0


def run_lm_workload(args, torch, apx, synth, spec, label, desc):
    prob = apx.Problem(_conv(args, spec))
    data, weight = _data(prob, spec, synth)
    dd, ww = prob.pixels(data), prob.pixels(weight)
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    prob.lm_run(args.warmup, dd, ww, th, st)
    torch.cuda.synchronize()
    # eager pass over the same iterations, one at a time: the Jacobian phases (need_jac on
    # entry) and the trials whose objective was evaluated (finite chi2_trial; a failed
    # Cholesky or an out-of-domain trial skips the objective convolution)
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    phases = n_obj = 0
    for _ in range(args.steps):
        phases += int(prob.lm_state(st)["need_jac"][0] != 0)
        prob.lm_step(dd, ww, th, st)
        n_obj += int(np.isfinite(prob.lm_state(st)["chi2_trial"][0]))
    prob.check()
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    torch.cuda.synchronize()
    prob.set_timing(True)
    t0 = time.perf_counter()
    prob.lm_run(args.steps, dd, ww, th, st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = prob.timing()
    prob.set_timing(False)
    stt = prob.lm_state(st)
    dominant, per_class = class_rooflines(_conv(args, spec), prob, kt, phases, n_obj=n_obj)
    top = max(kt, key=lambda k: kt[k][0])
    _line({
        "metric": "LM iters/s & Mpix/s rendered (fused adjoint+batched vs plain) at oracle rtol",
        "workload": label, "value": args.steps / dt, "unit": "LM it/s", "ms_per_step": dt * 1e3 / args.steps,
        "n_gpus": 1, "steps": args.steps, "mpix_per_s": _mpix(prob, spec, torch, 10),
        "accepted": int(stt["n_accept"][0]),
        "roofline": dominant, "roofline_per_class": per_class, "top_class": top,
        "jacobian_phases": phases, "objective_evaluations": n_obj,
        "kernel_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in kt.items()},
        "tile_shapes": tile_choice(prob),
        "config": {"workload": desc, "n_par": spec["n_par"], "n_pix": prob.n_pix},
        "dtype": "f32 Jacobian / f64 objective+normal equations", "data": "synthetic"})
    return 0


def run_multiband(args, torch, apx, synth):
    return run_lm_workload(args, torch, apx, synth, synth.multiband(), "multiband",
                           "3 bands x 2 epochs of 2048x2048, per-image affine and Moffat 41x41, 300 galaxies "
                           "with shared shape and per-band Ie, 2706 params")


def run_single(args, torch, apx, synth):
    return run_lm_workload(args, torch, apx, synth, synth.single(), "single",
                           "64x64, 1 Sersic + sky, Gaussian 11x11 sigma 1.5, 3x3 nodes, 8 params")


def run_livepsf(args, torch, apx, synth):
    return run_lm_workload(args, torch, apx, synth, synth.live_psf(), "livepsf",
                           "512x512, 100 stars + 20 Sersic + sky, live Moffat PSF 25x25 with free power "
                           "and scale, 243 params")


def run_superres(args, torch, apx, synth):
    spec = synth.with_psf_upsampling(synth.blend(seed_id=12, H=256, W=256, n_sersic=20, n_point=50, P=13),
                                     U=2, P_fine=25)
    return run_lm_workload(args, torch, apx, synth, spec, "superres",
                           "256x256 blend (20 Sersic + 50 point sources + sky) through a PSF sampled 2x "
                           "finer: 512x512 sub-pixel render and 25x25 sub-pixel Moffat, summed onto the "
                           "pixels, 191 params")


def run_recentre(args, torch, apx, synth):
    spec = synth.with_recentring(synth.blend(), synth.SHIFT_LANCZOS, 3)
    return run_lm_workload(args, torch, apx, synth, spec, "recentre",
                           "512x512, 50 Sersic + 200 point sources + sky, Moffat 25x25, Sersics sampled at "
                           "the nearest pixel centre and moved back by Lanczos-3 interpolation, 551 params")


def run_adaptive(args, torch, apx, synth):
    spec = synth.blend(mode=synth.MODE_ADAPTIVE, k_re=1e-2)
    return run_lm_workload(args, torch, apx, synth, spec, "adaptive",
                           "512x512, 50 Sersic + 200 point sources + sky, Moffat 25x25, adaptive "
                           "integration with budget 0.01 F / N, 551 params")


def run_hmc(args, torch, apx, synth):
    """The Bayesian mock of the paper's sampling example: one Sersic galaxy, one star and the
    sky under a live Moffat PSF (11 free parameters), fitted by LM, then sampled with the LM
    covariance as the inverse mass matrix: NUTS (20 warm-up transitions adapting the step,
    then `steps` x 25 timed, as the paper's 20 + 250 at the default 10 steps) and plain HMC
    (10 leapfrog steps per transition)."""
    spec = synth.live_psf(seed_id=9, H=128, W=128, n_star=1, n_sersic=1, P=25, logf_range=(2.0, 2.5),
                          logie_range=(0.0, 0.5))
    prob = apx.Problem(_conv(args, spec))
    data, weight = _data(prob, spec, synth)
    dd, ww = prob.pixels(data), prob.pixels(weight)
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    prob.lm_run(60, dd, ww, th, st, use_graph=True)
    F, _ = prob.covariance_factor(th, dd, ww)
    rng = np.random.default_rng(20230801)
    n_warm, n_samp, n_par = 20, 25 * args.steps, spec["n_par"]
    z = torch.tensor(rng.standard_normal((n_warm + n_samp, n_par)), device=prob.device)
    # NUTS: 20 warm-up transitions select the step (dual averaging to acceptance 0.8)
    depth = 8
    nd = 1 + depth + (1 << (depth + 1))
    un = torch.tensor(rng.uniform(size=(n_warm + n_samp, nd)), device=prob.device)
    thn = th.clone()
    t0 = time.perf_counter()
    eps_nuts = prob.nuts_warmup(thn, dd, ww, F, 1.0, depth, 0.8, z[:n_warm], un[:n_warm])
    torch.cuda.synchronize()
    dt_warm = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, nst = prob.nuts(thn, dd, ww, F, eps_nuts, depth, z[n_warm:], un[n_warm:])
    torch.cuda.synchronize()
    dt_nuts = time.perf_counter() - t0
    nst = nst.cpu().numpy()
    # HMC
    n_leap, eps = 10, 0.3
    u = torch.tensor(rng.uniform(size=(n_warm + n_samp, 1)), device=prob.device)
    prob.hmc(th, dd, ww, F, eps, n_leap, z[:n_warm], u[:n_warm])
    torch.cuda.synchronize()
    prob.set_timing(True)
    t0 = time.perf_counter()
    samples, stats = prob.hmc(th, dd, ww, F, eps, n_leap, z[n_warm:], u[n_warm:])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = prob.timing()
    prob.set_timing(False)
    prob.check()
    acc = float(stats[:, 0, 0].mean().cpu())
    dominant, per_class = class_rooflines(_conv(args, spec), prob, kt, 0, calls_per_launch_count(prob, th, dd, ww))
    top = max(kt, key=lambda k: kt[k][0])
    _line({
        "metric": "NUTS transitions/s (LM covariance mass matrix) on the Bayesian mock",
        "workload": "hmc", "value": n_samp / dt_nuts, "unit": "NUTS samples/s", "ms_per_step": dt_nuts * 1e3 / n_samp,
        "n_gpus": 1, "steps": n_samp, "nuts_step": eps_nuts, "nuts_warmup_s": dt_warm,
        "nuts_mean_depth": float(nst[:, 0].mean()),
        "nuts_leapfrog_per_sample": float(nst[:, 1].mean()), "nuts_divergent": int(nst[:, 3].sum()),
        "hmc_samples_per_s": n_samp / dt, "hmc_gradient_passes_per_s": n_samp * n_leap / dt, "hmc_accept_rate": acc,
        "hmc_kernel_ms_per_sample": {k: round(v[0] / n_samp, 4) for k, v in kt.items()},
        "roofline": dominant, "roofline_per_class": per_class, "top_class": top,
        "roofline_note": "classes of the timed plain-HMC transitions (NUTS runs the same kernels)",
        "paper_context": "NUTS, 20 warm-up + 250 samples of a 13-parameter mock in 738.5 s, hardware unstated",
        "config": {"workload": "128x128, 1 Sersic + 1 star + sky, live Moffat PSF 25x25 (n, R_d fitted), "
                               "11 params; NUTS 20 warm-up (dual averaging, target 0.8) + 25 x steps, depth <= 8; "
                               "HMC step 0.3, 10 leapfrog steps",
                   "n_par": spec["n_par"], "n_pix": prob.n_pix},
        "dtype": "f64 objective / f32 adjoint gradient", "data": "synthetic"})
    return 0


OTHER_WORKLOADS = {"field": run_field, "multiband": run_multiband,
                   "single": run_single, "livepsf": run_livepsf, "adaptive": run_adaptive,
                   "hmc": run_hmc, "superres": run_superres, "recentre": run_recentre}


def tile_choice(prob):
    """Convolution jobs per tile shape (rows x cols) as the autotuner chose them."""
    names = ["%dx%d" % t for t in prob_tile_shapes()] + ["fft", "sep"]
    return {kind: dict(zip(names, prob.tile_shapes(k))) for k, kind in enumerate(["model", "jacobian", "adjoint"])}


def prob_tile_shapes():
    from paper_2308_01957_amd import apx
    return apx.TILE_SHAPES


def counted_record(name, kernel, jac_tiles=None):
    """The machine-readable block of the committed rocprofv3 counter summary
    profiles/<name>, or None when there is none, it covers another kernel, the kernel's
    sources changed after the counters were taken, or (jac_tiles given) this run's Jacobian
    jobs took other tile shapes than the counted run's (the halo re-reads, and so the bytes,
    depend on the shape)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("|"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or "sources" not in kv:
        return None
    h = hashlib.sha256()
    for src in kv["sources"].split():
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != kv.get("sources_sha256"):
        return None
    if "jacobian_tiles" not in kv or (jac_tiles is not None and json.loads(kv["jacobian_tiles"]) != jac_tiles):
        return None
    return kv


def counted_traffic(kernel, jac_tiles):
    """HBM bytes per launch of the blend's Jacobian convolution (counter summary of the
    blend), or None (counted_record)."""
    kv = counted_record("conv_jcol_blend512_hbm_counters.md", kernel, jac_tiles)
    return None if kv is None else float(kv["traffic_bytes_per_launch"])


def load_tile_costs(path):
    """Autotuner table written by --tile-costs-out: {(kernel, P): [us per tile]}."""
    return {tuple(int(v) for v in k.split(",")): c for k, c in json.load(open(path)).items()}


def save_tile_costs(prob, Ps, path):
    table = {f"{k},{P}": prob.tile_cost(k, P) for k in range(4) for P in sorted(set(Ps))}
    json.dump({k: v for k, v in table.items() if v is not None}, open(path, "w"))


def copy_calibration(args, torch):
    """Three elementwise copies y = 1 * x of a known size: a profiler's HBM byte counters
    read on them give the factor between counted and moved bytes."""
    if args.copy_calibration <= 0:
        return
    n = args.copy_calibration * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 x {args.copy_calibration} MiB read + write", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--render-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also launch three plain copy kernels of MIB MiB (read MIB, write MIB) "
                         "after the timed region, to calibrate HBM byte counters")
    ap.add_argument("--tile-costs-out", metavar="JSON",
                    help="cutouts or blend: write the autotuner's measured tile costs to JSON")
    ap.add_argument("--tile-costs-in", metavar="JSON",
                    help="cutouts or blend: take the tile costs from JSON instead of timing them (the "
                         "same tile shapes as the run that wrote it, e.g. under a counter profiler)")
    ap.add_argument("--conv", default=None, choices=["direct", "fft", "auto"],
                    help="PSF convolution mode: direct, FFT tiles for P >= 15, or auto (FFT tiles per job "
                         "where the library's cost model prices them below direct); default auto for the "
                         "cutouts headline, direct for the other workloads")
    ap.add_argument("--workload", default="cutouts",
                    choices=["cutouts", "blend", "field", "multiband", "single", "livepsf", "adaptive", "hmc",
                             "superres", "recentre"],
                    help="cutouts (default, the headline line, with the blend beside it); the others print "
                         "their own line")
    ap.add_argument("--no-blend", action="store_true", help="cutouts: leave out the blend beside the headline")
    ap.add_argument("--no-2d-context", action="store_true",
                    help="cutouts: leave out the same iterations in the other convolution modes (automatic, "
                         "every convolution 2-D)")
    args = ap.parse_args()
    if args.conv is None:
        args.conv = "auto" if args.workload == "cutouts" else "direct"
    CONV_MODE[0] = args.conv
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the fit of one field runs on one device); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_2308_01957_amd import apx, synth
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    if args.workload == "blend":
        rec, spec, data, weight = run_blend(args, torch, apx, synth)
        if not args.no_cpu_baseline:
            print("[bench] timing the oracle sample on the host", file=sys.stderr, flush=True)
            rec["cpu_baseline"] = cpu_baseline_blend(spec, data, weight)
        _line(rec)
        copy_calibration(args, torch)
        return 0
    if args.workload != "cutouts":
        rc = OTHER_WORKLOADS[args.workload](args, torch, apx, synth)
        copy_calibration(args, torch)
        return rc

    rec, spec, data, weight = run_cutouts(args, torch, apx, synth)
    if not args.no_blend:
        # the blend beside the headline runs its direct convolutions (the counted kernel)
        b, _, _, _ = run_blend(argparse.Namespace(**dict(vars(args), conv="direct")), torch, apx, synth,
                               with_fft=False)
        rec["blend"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "mpix_per_s", "roofline", "graph_ms_per_step")}
        rec["blend"]["workload"] = b["config"]["workload"]
        rec["blend"]["conv"] = "direct"
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on a sample of cutouts (process pool)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline_cutouts(spec, data, weight, synth)
    _line(rec)
    copy_calibration(args, torch)
    return 0


def run_blend(args, torch, apx, synth, with_fft=True):
    """The blended 512 x 512 field (50 Sersic + 200 point sources + sky, Moffat 25 x 25,
    3 x 3 nodes within 2 Re, 551 parameters in one joint fit): K LM iterations from the
    perturbed start, eager (graph replays of the same iterations timed before them).
    Returns (record, spec, data, weight)."""
    spec = synth.blend()                       # 512x512, 50 Sersic + 200 PS, Moffat 25
    img = spec["images"][0]
    P_psf = img["psf"].shape[0]
    print(f"[bench] workload {spec['name']}: {spec['n_par']} parameters", file=sys.stderr, flush=True)
    costs = None
    if args.tile_costs_in:
        costs = load_tile_costs(args.tile_costs_in)
    prob = apx.Problem(_conv(args, spec), tile_costs=costs)
    if args.tile_costs_out:
        save_tile_costs(prob, [P_psf], args.tile_costs_out)
    m_true = prob.split(prob.render(spec["theta_true"]))[0].astype(np.float64)
    prob.check()
    d, w = synth.make_data(m_true, spec["noise"][0])
    dd, ww = prob.pixels([d]), prob.pixels([w])

    # warm-up (compiles nothing; touches every kernel and page)
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    prob.lm_run(args.warmup, dd, ww, th, st)
    torch.cuda.synchronize()
    print(f"[bench] warm-up {args.warmup} iterations done", file=sys.stderr, flush=True)

    # context, before the timed region (a pass run first is ~4% slower, whatever it is): the
    # same K iterations as replays of one captured HIP graph of the iteration
    th_g, st_g = prob.lm_init(spec["theta_init"], dd, ww)
    prob.lm_run(1, dd, ww, th_g, st_g, use_graph=True)
    prob.lm_init(spec["theta_init"], dd, ww, theta_out=th_g, state_out=st_g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.lm_run(args.steps, dd, ww, th_g, st_g, use_graph=True)
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps

    # timed region: the first K iterations of the fit from the perturbed start, with HIP
    # events around the dominant kernel's launches only (events around every launch class
    # would cost ~8% of the iteration)
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    torch.cuda.synchronize()
    prob.set_timing(True, classes=["conv_jcol"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.lm_run(args.steps, dd, ww, th, st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = prob.timing()
    prob.set_timing(False)
    state = prob.lm_state(st)[0]
    prob.check()
    assert torch.equal(th_g, th), "graph replay and eager iterations differ"
    # the per-class breakdown from a second, fully instrumented pass over the same iterations
    th2, st2 = prob.lm_init(spec["theta_init"], dd, ww)
    prob.set_timing(True)
    prob.lm_run(args.steps, dd, ww, th2, st2)
    kt_all = prob.timing()
    prob.set_timing(False)
    print(f"[bench] {args.steps} LM iterations in {elapsed * 1e3:.1f} ms "
          f"({int(state['n_accept'])} accepted)", file=sys.stderr, flush=True)

    # dominant kernel: Jacobian-column convolutions, one launch per iteration
    # (the launch also runs in iterations that follow a rejected step, where it finds no new
    # Jacobian to compute and exits within ~12 us: those few us are kept in the total and the
    # average is taken over the launches that computed a Jacobian)
    n_jac = prob.n_jac                        # Jacobian entries = output pixels of all columns
    flop_per_phase = 2.0 * P_psf * P_psf * n_jac
    j_phases = 1 + int(state["n_accept"]) - int(state["accepted"])
    jcol_ms, jcol_launches = kt["conv_jcol"]
    avg_ms = jcol_ms / max(1, j_phases)
    achieved = flop_per_phase / (avg_ms * 1e-3) / 1e12 if jcol_ms > 0 else 0.0

    # parameter covariance at the last iterate: (J^T W J)^-1 of the 551-parameter system
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.covariance(th, dd, ww)
    torch.cuda.synchronize()
    cov_ms = (time.perf_counter() - t0) * 1e3

    # the same K iterations with FFT-mode convolution (context: the headline stays direct)
    fft_mode = None
    if args.conv == "direct" and with_fft:
        spec_f = dict(spec)
        spec_f["conv_mode"] = 1
        pf = apx.Problem(spec_f)
        thf, stf = pf.lm_init(spec["theta_init"], dd, ww)
        pf.lm_run(args.warmup, dd, ww, thf, stf)
        thf, stf = pf.lm_init(spec["theta_init"], dd, ww)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pf.lm_run(args.steps, dd, ww, thf, stf)
        torch.cuda.synchronize()
        dtf = time.perf_counter() - t0
        pf.check()
        fft_mode = {"value": args.steps / dtf, "unit": "LM it/s", "ms_per_step": dtf * 1e3 / args.steps,
                    "note": "FFT-mode Jacobian-column convolutions (128x128 overlap-save tiles); objective "
                            "convolution direct; same iterations, accept decisions and parity gates"}
        pf.close()

    # rendered Mpix/s: objective-path model (FP64 render + convolution) at the truth
    prob.set_timing(False)
    out = torch.empty(prob.n_pix, dtype=torch.float32, device=prob.device)
    th_true = torch.as_tensor(spec["theta_true"], dtype=torch.float64, device=prob.device)
    for _ in range(3):
        prob.render(th_true, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.render_reps):
        prob.render(th_true, out)
    torch.cuda.synchronize()
    mpix = prob.n_pix * args.render_reps / (time.perf_counter() - t0) / 1e6

    rec = {
        "metric": "LM iters/s & Mpix/s rendered (fused adjoint+batched vs plain) at oracle rtol",
        "value": args.steps / elapsed,
        "unit": "LM it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 Jacobian / f64 objective+normal equations",
        "data": "synthetic (seeded; noise-free model rendered by the library, Gaussian noise)",
        "tile_shapes": tile_choice(prob),
        "config": {"workload": "blended field 512x512: 50 Sersic + 200 point sources + sky, "
                               "Moffat 25x25 beta 2.5 FWHM 3, 3x3 nodes within 2 Re, 551 params",
                   "n_par": spec["n_par"], "n_pix": prob.n_pix, "psf": P_psf,
                   "lm_accepted": int(state["n_accept"]), "jacobian_phases": j_phases},
        "mpix_per_s": mpix,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     "traffic": counted_traffic(f"k_conv<{P_psf},JCOL>", tile_choice(prob)["jacobian"]),
                     "traffic_unit": "bytes/launch",
                     "kernel": f"k_conv<{P_psf},JCOL>",
                     "avg_launch_ms": avg_ms, "launches_with_work": j_phases,
                     "launches_total": jcol_launches,
                     "flop_per_launch": flop_per_phase},
        "covariance_ms": cov_ms,
        "graph_ms_per_step": graph_ms,
        "fft_mode": fft_mode,
        "kernel_ms": {k: round(v[0], 4) for k, v in kt_all.items()},
        "kernel_ms_note": "per class over the K iterations, from a second fully instrumented pass",
    }
    prob.close()
    return rec, spec, [d], [w]


if __name__ == "__main__":
    sys.exit(main())
