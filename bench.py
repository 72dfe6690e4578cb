#!/usr/bin/env python3
"""Benchmark of the polynomial-preconditioned FISTA hot path on one MI355X.

Workload: Cartesian SENSE 256 x 256, 16 coils, Poisson-disc-like mask (R = 6,
24 x 24 centre), noise sigma = 5e-3, 4-level Haar, lambda = 5e-4 (synthetic,
seeded; it stands in for the paper's Cartesian knee data).

One step = one iteration of Algorithm 4 at degree d (default 3): the gradient
normal apply, d Horner normal applies and the fused prox/momentum step, all on
the GPU.  ``value`` = A^H A applies per second over exactly --steps timed
iterations (inputs resident in HBM, graph-replayed loop).  Also reported:

* roofline of the dominant kernel pass, timed live with HIP events on the
  launch stream (pfista_profile_normal);
* time to 1e-4 relative objective error, plain FISTA vs PFISTA d = 1..5 on the
  same GPU (each method against its own converged objective);
* the FP64 oracle timed on the host cores on a bounded sample (cpu_baseline).

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = 2
PEAK_HBM_GBS = 8000.0
# FP32 vector FMA issue rate without packed-FP32 instructions:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def fft_flops(n):
    return 5.0 * n * math.log2(n)


def pass_model(n, coils, slices, kind):
    """Algorithmic flops and bytes of each kernel pass of one normal apply
    (5 N log2 N flops per length-N complex transform, 6 per complex product,
    8 per complex multiply-add; bytes = what the pass must read and write)."""
    img, coil = slices * n * n * 8, slices * coils * n * n * 8
    if kind == "1d":
        fl = slices * coils * n * (2 * fft_flops(n) + 6 * n + 8 * n)
        return [("phase_encode_1d", fl, 2 * img + coil + slices * n)]
    rows = slices * coils * n
    return [
        ("row_forward", rows * (fft_flops(n) + 6 * n), img + 2 * coil),
        ("column_pair", rows * 2 * fft_flops(n), 2 * coil + slices * n * n),
        ("row_inverse_combine", rows * (fft_flops(n) + 8 * n), 2 * coil + img),
    ]


def setup(torch, pf, dev):
    import numpy as np

    from synth import make_inputs
    inp = make_inputs(WORKLOAD)
    n, coils = inp["n"], inp["coils"]
    plan = pf.Plan(n, coils, 1, haar_levels=inp["levels"], mask_kind=pf.MASK_2D, device=dev)
    sens = torch.from_numpy(inp["sens"].astype(np.complex64)).to(dev)
    mask = torch.from_numpy(inp["mask"]).to(dev)
    img = torch.from_numpy(inp["phantom"].astype(np.complex64)).to(dev)
    noise = torch.from_numpy(inp["noise"].astype(np.complex64)).to(dev)
    b = torch.empty((1, coils, n, n), dtype=torch.complex64, device=dev)
    pf.forward(plan, sens, mask, img, b)                      # M F S x on the GPU
    b += noise * mask[:, None, :, :].to(torch.complex64)      # noise on sampled points only
    lam_max = pf.power_iteration(plan, sens, mask, 100)
    return inp, plan, sens, mask, b, 1.0 / (1.01 * lam_max)


def timed_solve(torch, pf, plan, sens, mask, b, lam, coef, iters, inv_l, stream, graph_iters, k0=0,
                x=None, z=None):
    dev = sens.device
    shp = (1, plan.n, plan.n)
    x = torch.empty(shp, dtype=torch.complex64, device=dev) if x is None else x
    z = torch.empty(shp, dtype=torch.complex64, device=dev) if z is None else z
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = pf.solve(plan, sens, mask, b, x, lam, coef=coef, max_iter=iters, inv_l=inv_l,
                   check_every=max(1, min(iters, 4096)), graph_iters=graph_iters, z=z, k0=k0,
                   stream=stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, rep, x, z


def time_to_tolerance(torch, pf, plan, sens, mask, b, lam, inv_l, stream, graph_iters, tol=1e-4,
                      ref_applies=6000, max_hist_applies=3000):
    out = {}
    methods = [("fista", [1.0])] + [(f"pfista_d{d}", pf.poly_coefficients(d)) for d in range(1, 6)]
    for name, coef in methods:
        per = len(coef)
        kref = ref_applies // per
        x = torch.empty((1, plan.n, plan.n), dtype=torch.complex64, device=sens.device)
        rep = pf.solve(plan, sens, mask, b, x, lam, coef=coef, max_iter=kref, inv_l=inv_l,
                       check_every=kref // 2, history=True, graph_iters=graph_iters, stream=stream)
        f_half, f_inf = rep["history"][-2], rep["history"][-1]
        kmax = max_hist_applies // per
        rep = pf.solve(plan, sens, mask, b, x, lam, coef=coef, max_iter=kmax, inv_l=inv_l,
                       check_every=1, history=True, stream=stream)
        err = [(f - f_inf) / f_inf for f in rep["history"]]
        kstar = None
        for k in range(len(err)):
            if all(e <= tol for e in err[k:]):
                kstar = k + 1
                break
        entry = {"f_inf": f_inf, "f_inf_drift": abs(f_half - f_inf) / f_inf, "ref_iters": kref,
                 "applies_per_iter": per}
        if kstar is not None:
            ts = []
            for _ in range(5):
                dt, _, _, _ = timed_solve(torch, pf, plan, sens, mask, b, lam, coef, kstar, inv_l, stream,
                                          graph_iters)
                ts.append(dt)
            ts.sort()
            entry.update({"iters": kstar, "applies": kstar * per, "ms": 1e3 * ts[len(ts) // 2]})
        else:
            entry.update({"iters": None, "applies": None, "ms": None, "note": f"not within {kmax} iterations"})
        out[name] = entry
        log(f"time-to-{tol:g} {name}: {entry.get('iters')} iterations, {entry.get('ms')} ms")
    fista_ms = out["fista"]["ms"]
    best = min((v["ms"], k) for k, v in out.items() if k != "fista" and v["ms"] is not None)
    return {"tol": tol, "methods": out, "best_pfista": best[1],
            "speedup_vs_fista": (fista_ms / best[0]) if fista_ms and best[0] else None}


def cpu_baseline(inp, degree, seconds):
    """The FP64 oracle's PFISTA iterations on the host, for a bounded time."""
    import numpy as np

    import oracle as orc
    sens = inp["sens"].astype(np.complex64).astype(np.complex128)
    img = inp["phantom"]
    b = orc.kspace_data(sens, inp["mask"], img, inp["noise"])
    bn = b / np.linalg.norm(b)
    coef = orc.l2_poly_coefficients(degree)
    inv_l = 1.0 / 1.01
    x = z = None
    k, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        x, z, _ = orc.pfista(sens, inp["mask"], bn, inv_l, inp["lam"], coef, inp["levels"], 1, x0=x, z0=z, k0=k)
        k += 1
    dt = time.perf_counter() - t0
    return {"value": k * (degree + 1) / dt, "unit": "A^H A applies/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} PFISTA iterations (degree {degree}, {k * (degree + 1)} applies) of the "
                      f"256x256 16-coil workload in {dt:.1f} s, complex128 NumPy/SciPy, one thread"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--degree", type=int, default=3)
    ap.add_argument("--graph-iters", type=int, default=10)
    ap.add_argument("--profile-reps", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance comparison")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path has no multi-GPU mode "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2204_10252_amd as pf
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pf.load_library()
    log("building inputs")
    inp, plan, sens, mask, b, inv_l = setup(torch, pf, dev)
    lam, d = inp["lam"], args.degree
    coef = pf.poly_coefficients(d)
    stream = torch.cuda.Stream()

    with torch.cuda.stream(stream):
        log(f"warmup {args.warmup} iterations")
        _, _, x, z = timed_solve(torch, pf, plan, sens, mask, b, lam, coef, args.warmup, inv_l, stream,
                                 args.graph_iters)
        log(f"timing {args.steps} iterations")
        dt, rep, x, z = timed_solve(torch, pf, plan, sens, mask, b, lam, coef, args.steps, inv_l, stream,
                                    args.graph_iters, k0=args.warmup, x=x, z=z)
        applies = args.steps * (d + 1)
        value = applies / dt
        log(f"{value:.0f} applies/s, {1e3 * dt / args.steps:.4f} ms/iteration")

        # dominant kernel pass, timed live with HIP events on the launch stream
        y = torch.empty_like(x)
        pass_ms = pf.profile_normal(plan, sens, mask, x, y, reps=args.profile_reps, stream=stream)
        model = pass_model(plan.n, plan.coils, 1, "2d")
        k = max(range(len(pass_ms)), key=lambda i: pass_ms[i])
        name, flops, nbytes = model[k]
        t_k = pass_ms[k] * 1e-3
        achieved_tf = flops / t_k / 1e12
        roofline = {"bound": "alu", "kernel": name, "achieved": round(achieved_tf, 3),
                    "peak": round(PEAK_FP32_NONPACKED_TFLOPS, 1), "unit": "TFLOP/s",
                    "frac": round(achieved_tf / PEAK_FP32_NONPACKED_TFLOPS, 4), "traffic": None,
                    "avg_launch_us": round(pass_ms[k] * 1e3, 3),
                    "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes,
                    "hbm_frac": round(nbytes / t_k / 1e9 / PEAK_HBM_GBS, 4),
                    "passes_us": {m[0]: round(t * 1e3, 3) for m, t in zip(model, pass_ms)}}
        apply_bytes = 8 * plan.n * plan.n * (plan.coils + 2)
        apply_us = sum(pass_ms) * 1e3
        roofline["normal_apply_us"] = round(apply_us, 3)
        roofline["normal_apply_hbm_frac"] = round(apply_bytes / (apply_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)
        log(f"passes (us): {roofline['passes_us']}")

        ttt = None
        if not args.no_ttt:
            ttt = time_to_tolerance(torch, pf, plan, sens, mask, b, lam, inv_l, stream, args.graph_iters)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline ({args.cpu_seconds:.0f} s)")
        cpu = cpu_baseline(inp, d, args.cpu_seconds)

    out = {
        "metric": "A^H A applies/s (256^2, 16 coils); time to 1e-4 rel. objective vs plain FISTA",
        "value": round(value, 1),
        "unit": "A^H A applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 (complex64), fp64 reductions",
        "data": "synthetic (seeded phantom, coil maps, Poisson-disc-like mask, noise)",
        "config": {"workload": "Cartesian SENSE 256x256, 16 coils, R=6, 4-level Haar, lambda=5e-4",
                   "degree": d, "step": f"1 PFISTA iteration = {d + 1} A^H A applies + prox/momentum",
                   "graph_iters": args.graph_iters},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_tol": ttt,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
