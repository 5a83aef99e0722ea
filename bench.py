#!/usr/bin/env python3
"""Benchmark of the chi^2 forward-modelling hot path on one MI355X.

Workload: the blended 512 x 512 field -- 50 elliptical Sersic galaxies and 200 point
sources (fixed positions, free fluxes) plus a flat sky, Moffat PSF 25 x 25 (beta 2.5,
FWHM 3 px), 3 x 3 sub-pixel nodes within 2 Re of each galaxy and the pixel centre
elsewhere; all 551 parameters are fit jointly by Levenberg-Marquardt with a dense FP64
J^T W J formed on the GPU.  Inputs are seeded and synthetic: parameters drawn from the
priors of the random-Sersic benchmark (§3.2, Table 1 pattern), the noise-free model
rendered by the library itself, Gaussian noise of variance model + 0.01^2.

One "step" is one full LM iteration (normal equations when the last step was accepted,
damped Cholesky with retries, trial render + chi^2, accept/reject).  The timed region
is the first --steps iterations from the perturbed initial parameters, inputs resident
in HBM; the value is iterations per second.  The dominant kernel (the Jacobian-column
convolutions) is timed live with HIP events on the library's stream; the roofline
fraction is its algorithmic FLOP rate (2 P^2 FLOP per Jacobian entry) over the FP32
VALU FMA peak.  The CPU baseline is the FP64 test oracle on a bounded sample of one LM
iteration, extrapolated to a full iteration.
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

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 FLOP (FMA) x 2.4 GHz, unpacked FP32 / FP64
PEAK_FP32_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12    # 78.6
PEAK_HBM_GBS = 8000.0


def cpu_baseline(spec, data, weight):
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--render-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the fit of one field runs on one device); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    from paper_2308_01957_amd import apx, synth
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1

    spec = synth.blend()                       # 512x512, 50 Sersic + 200 PS, Moffat 25
    img = spec["images"][0]
    P_psf = img["psf"].shape[0]
    print(f"[bench] workload {spec['name']}: {spec['n_par']} parameters", file=sys.stderr, flush=True)
    prob = apx.Problem(spec)
    m_true = prob.split(prob.render(spec["theta_true"]))[0].astype(np.float64)
    prob.check()
    d, w = synth.make_data(m_true, spec["noise"][0])
    dd, ww = prob.pixels([d]), prob.pixels([w])

    # warm-up (compiles nothing; touches every kernel and page)
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    prob.lm_run(args.warmup, dd, ww, th, st)
    torch.cuda.synchronize()
    print(f"[bench] warm-up {args.warmup} iterations done", file=sys.stderr, flush=True)

    # timed region: the first K iterations of the fit from the perturbed start
    th, st = prob.lm_init(spec["theta_init"], dd, ww)
    torch.cuda.synchronize()
    prob.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.lm_run(args.steps, dd, ww, th, st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = prob.timing()
    prob.set_timing(False)
    state = prob.lm_state(st)[0]
    prob.check()
    print(f"[bench] {args.steps} LM iterations in {elapsed * 1e3:.1f} ms "
          f"({int(state['n_accept'])} accepted)", file=sys.stderr, flush=True)

    # dominant kernel: Jacobian-column convolutions, one launch per iteration
    n_jac = prob.n_jac                        # Jacobian entries = output pixels of all columns
    flop_per_phase = 2.0 * P_psf * P_psf * n_jac
    j_phases = 1 + int(state["n_accept"]) - int(state["accepted"])
    jcol_ms, jcol_launches = kt["conv_jcol"]
    achieved = flop_per_phase * j_phases / (jcol_ms * 1e-3) / 1e12 if jcol_ms > 0 else 0.0

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
        "config": {"workload": "blended field 512x512: 50 Sersic + 200 point sources + sky, "
                               "Moffat 25x25 beta 2.5 FWHM 3, 3x3 nodes within 2 Re, 551 params",
                   "n_par": spec["n_par"], "n_pix": prob.n_pix, "psf": P_psf,
                   "lm_accepted": int(state["n_accept"]), "jacobian_phases": j_phases},
        "mpix_per_s": mpix,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": None,
                     "kernel": f"k_conv<{P_psf},JCOL>",
                     "avg_launch_ms": jcol_ms / max(1, jcol_launches),
                     "launches": jcol_launches,
                     "flop_per_jacobian": flop_per_phase},
        "kernel_ms": {k: round(v[0], 4) for k, v in kt.items()},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle sample on the host", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(spec, [d], [w])
    print(json.dumps(rec), flush=True)
    prob.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
