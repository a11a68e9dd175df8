#!/usr/bin/env python3
"""Throughput of the ladder forward + adjoint on one MI355X.

One step = ladder_forward (g tiles, R, E) + ladder_adjoint (D tiles, X) over the
whole synthetic workload, inputs resident in HBM before the timed region.
Prints one JSON line.  Value = nominal dense flops F = 4 v^4 (n + o^2) + 2 o^2 v^2
per step divided by the measured time (TFLOP/s).

The CPU baseline times the FP64 oracle (numpy matrix-product version, all host
threads) on a bounded sample of the same workload: the forward rows of a few
virtual indices a and the adjoint rows of a few p, at the full shape.  Those rows
of the GPU result are compared with it (err_sample_*).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "tiny": (4, 20, 60, 1),
    "medium": (20, 150, 600, 2),
    "retinal": (78, 657, 2200, 3),
    "autograd": (40, 350, 1200, 5),
}
PEAK = {"fp64": 78.6, "bf16": 2516.6}  # dense MFMA TFLOP/s, MI355X


def nominal_flops(o, v, n):
    return 4.0 * v ** 4 * (n + o * o) + 2.0 * o * o * v * v


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="retinal", choices=sorted(WORKLOADS))
    ap.add_argument("--shape", default=None, help="o,v,n override (probe shapes)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "split"])
    ap.add_argument("--slices", type=int, default=0)
    ap.add_argument("--n-abatch", type=int, default=0)
    ap.add_argument("--cpu-rows", type=int, default=1, help="a (and p) rows the CPU baseline computes; 0 = skip")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the ladder runs on one MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2202_02019_amd as P
    from synthetic import gpu as SG

    o, v, n, seed = WORKLOADS[args.workload]
    name = args.workload
    if args.shape:
        o, v, n = (int(x) for x in args.shape.split(","))
        name = "probe"
    big = nominal_flops(o, v, n) > 1e14
    steps = args.steps if args.steps is not None else (1 if big else 10)
    warmup = args.warmup if args.warmup is not None else (1 if big else 2)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    L = SG.draw_L_vv(seed, o, v, n)
    Lov = SG.draw_L_ov(seed, o, v, n)
    eps = SG.draw_eps(seed, o, v)
    tau = P.mp2_amplitudes(Lov, eps, o=o, v=v, n=n)
    del Lov
    tbar = SG.add_noise(seed, o, v, tau)
    R = torch.empty_like(tau)
    X = torch.empty_like(L)
    E = torch.empty((), dtype=torch.float64, device=dev)
    prec = P.FP64 if args.precision == "fp64" else P.SPLIT_BF16
    opts = P.Options(precision=prec, n_slices=args.slices, n_abatch=args.n_abatch)
    ws = torch.empty(P.workspace_size(o, v, n, opts), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    print("bench: %s o=%d v=%d n=%d precision=%s inputs ready in %.1fs, workspace %.2f GiB"
          % (name, o, v, n, args.precision, time.time() - t0, ws.numel() / 2 ** 30), file=sys.stderr, flush=True)

    def step():
        P.forward(L, tau, tbar, o=o, v=v, n=n, R=R, E=E, ws=ws, opts=opts)
        P.adjoint(L, tau, tbar, o=o, v=v, n=n, X=X, ws=ws, opts=opts)

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        print("bench: warmup step %d done" % i, file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    P.profile_start()
    ev0.record(stream)
    wall0 = time.time()
    for i in range(steps):
        step()
        if big:
            torch.cuda.synchronize()
            print("bench: timed step %d done (%.1fs)" % (i, time.time() - wall0), file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    stages = P.profile_stop()
    ms = ev0.elapsed_time(ev1) / steps
    F = nominal_flops(o, v, n)
    value = F / (ms * 1e-3) / 1e12

    dom_name, dom = max(stages.items(), key=lambda kv: kv[1]["total_ms"])
    dtype_peak = "fp64" if args.precision == "fp64" else "bf16"
    achieved = dom["flops"] / dom["launches"] / (dom["avg_ms"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": dom_name, "achieved": achieved, "peak": PEAK[dtype_peak],
                "unit": "TFLOP/s", "frac": achieved / PEAK[dtype_peak], "traffic": None,
                "avg_launch_ms": dom["avg_ms"], "launches_per_step": dom["launches"] / steps}
    if args.precision == "split":
        S = args.slices or 5
        prods = S * (S + 1) // 2
        # BF16 MFMA work actually issued: every slice pair (p, q) with p + q < S
        roofline["slice_products"] = prods
        roofline["executed_bf16_tflops"] = achieved * prods
        roofline["frac_executed"] = achieved * prods / PEAK["bf16"]
    stage_summary = {k: {"ms_per_step": s["total_ms"] / steps, "launches_per_step": s["launches"] / steps,
                         "tflops": (s["flops"] / (s["total_ms"] * 1e-3) / 1e12) if s["total_ms"] > 0 else None}
                     for k, s in stages.items()}

    cpu = None
    errs = {}
    if args.cpu_rows > 0:
        import oracle
        k = min(args.cpu_rows, v)
        Lh, th, wh = L.cpu().numpy(), tau.cpu().numpy(), tbar.cpu().numpy()
        threads = os.cpu_count()
        c0 = time.time()
        Rr, Er = oracle.matrix.forward(o, v, n, Lh, th, wh, a_range=(0, k))
        Xr = oracle.matrix.adjoint(o, v, n, Lh, th, wh, p_range=(0, k))
        cs = time.time() - c0
        fl = k * (2.0 * v ** 3 * n + 2.0 * o * o * v ** 3 + 2.0 * o * o * v) + k * (2.0 * o * o * v ** 3 + 2.0 * v ** 3 * n)
        cpu = {"value": fl / cs / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
               "seconds": cs, "s_per_iter_extrapolated": F / (fl / cs),
               "sample": "forward rows a<%d and adjoint rows p<%d at the full shape (o=%d v=%d n=%d); "
                         "numpy matrix-product FP64 oracle; nominal flops %.3e" % (k, k, o, v, n, fl)}
        Rg = R[:, :, :k, :].cpu().numpy()
        Xg = X[:k].cpu().numpy()
        errs = {"err_sample_R": float(np.abs(Rg - Rr).max() / np.abs(Rr).max()),
                "err_sample_X": float(np.abs(Xg - Xr).max() / np.abs(Xr).max()),
                "err_sample_E_rows": abs(float(np.sum(wh[:, :, :k, :] * Rg)) - Er) / abs(Er)}

    out = {
        "metric": "ladder fwd+adjoint TFLOP/s & s/iter, split-BF16 vs FP64 at <=1e-10 rel err in E",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "s_per_iter": ms / 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "bf16-split/f64",
        "data": "synthetic",
        "config": {"workload": name, "o": o, "v": v, "n_chol": n, "seed": seed, "precision": args.precision,
                   "n_slices": args.slices, "n_abatch": args.n_abatch, "nominal_flops": F},
        "energy": float(E.cpu()),
        "roofline": roofline, "stages": stage_summary, "cpu_baseline": cpu,
        "frac_fp64_peak": value / PEAK["fp64"],
    }
    out.update(errs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
