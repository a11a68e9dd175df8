#!/usr/bin/env python3
"""Throughput of the ladder forward + adjoint on one MI355X.

One step = ladder_forward (g tiles, R, E) + ladder_adjoint (D tiles, X) over the
whole synthetic workload, inputs resident in HBM before the timed region.
Prints one JSON line.  Value = the FP64-equivalent flops the path's GEMMs execute
per step (2 M N K per product; with the default +/- packing about 0.39 of the
dense count at the retinal shape) divided by the measured time, in TFLOP/s; the
dense-equivalent rate F = 4 v^4 (n + o^2) + 2 o^2 v^2 per step over the same time
is reported beside it.

Wall-clock budget (--budget, default 420 s from process start): the first warm-up
step is timed on the wall clock; the comparison legs (the FP64 path and the CPU
oracle) then run on that step's outputs (the path is bitwise deterministic, which
the run checks) and as many timed steps as fit the rest of the budget follow, at
most --steps; `steps` reports the number timed, `steps_requested` the number asked.

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

T_START = time.time()  # the wall-clock budget counts from process start (imports and input generation included)

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "tiny": (4, 20, 60, 1),
    "medium": (20, 150, 600, 2),
    "retinal": (78, 657, 2200, 3),
    "autograd": (40, 350, 1200, 5),
    "batched": (None, None, None, 4),
    # 64 small instances (o in 4..12, v in 20..80, n = 4(o+v)), sizes from seed 8: launch-bound shapes
    "batched_small": (None, None, None, 8),
    # shapes derived from the paper's other molecules (electrons from the formulas,
    # aug-cc-pVDZ functions, the Cholesky counts the paper quotes): thymine, azobenzene
    "thymine": (33, 228, 967, 6),
    "azobenzene": (48, 364, 1444, 7),
}
PEAK = {"fp64": 78.6, "bf16": 2516.6, "int8": 5033.2}  # dense MFMA TFLOP/s (TOP/s for INT8), MI355X
# (forward, adjoint) slice counts per split format: the benchmark's defaults, and the counts the
# committed traffic counters of that format are taken at
DEFAULT_SLICES = {"int8": (6, 5), "bf16": (5, 4)}
PREC_CODE = {"fp64": 0, "bf16": 1, "int8": 2}


TUNED_CACHE = os.path.join(ROOT, "paper_2202_02019_amd", "tuned_mi355x.jsonl")


def tuned_batch(path, o, v, n, precision, slices, flags, slices_adj=None):
    """The batch size a ladder_autotune cache file holds for this shape and options (last line
    wins, as in ladder_autotune_load; a line without n_slices_adjoint has the forward's count), or None."""
    if slices_adj is None:
        slices_adj = slices
    if not path or not os.path.exists(path):
        return None
    found = None
    with open(path) as fh:
        for line in fh:
            try:
                d = json.loads(line)
            except ValueError:
                continue
            key = (d.get("o"), d.get("v"), d.get("n"), d.get("precision"), d.get("n_slices"),
                   d.get("n_slices_adjoint", d.get("n_slices")), d.get("flags"))
            if key == (o, v, n, precision, slices if precision else 0, slices_adj if precision else 0, flags):
                found = d.get("n_abatch")
    return found


def gemm_source_hash():
    """First 16 hex digits of the SHA-256 of the library sources (kernels and the host
    code that shapes their launches: the code the stored HBM-traffic counters were
    taken on)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("csrc/split_bf16.hpp", "csrc/split_i8.hpp", "csrc/gemm_f64.hpp", "csrc/pm_pack.hpp", "csrc/ladder.hip",
              "build.py"):
        with open(os.path.join(ROOT, "paper_2202_02019_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def mfma_ceiling(seconds=0.2):
    """Rate of the register-only MFMA probe (ladder_mfma_probe) for BF16, INT8 and FP64, in
    TFLOP/s (TOP/s for INT8): what the matrix cores sustain on this chip under its clock and
    power limits."""
    import torch

    import paper_2202_02019_amd as P
    out = {}
    blocks = 8 * torch.cuda.get_device_properties(0).multi_processor_count
    for name, kind, rate in (("bf16", P.PROBE_BF16, 2.0e15), ("int8", P.PROBE_INT8, 4.0e15),
                             ("fp64", P.PROBE_FP64, 7.0e13)):
        _, per_iter = P.mfma_probe(kind, 1, blocks)
        iters = max(1, int(seconds * rate / per_iter))
        buf, _ = P.mfma_probe(kind, iters, blocks)          # warm-up at full length
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, fl = P.mfma_probe(kind, iters, blocks, out=buf)
        e1.record()
        torch.cuda.synchronize()
        out[name + "_tflops"] = fl / (e0.elapsed_time(e1) * 1e-3) / 1e12
        out[name + "_frac_of_published"] = out[name + "_tflops"] / PEAK[name]
    return out


def measured_traffic(workload, precision, kernel, n_abatch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary for this workload, or None when there is none, it was taken
    at another virtual-batch size, or the GEMM sources have changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_pm.json" % (workload, precision))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("sources_sha256_16") != gemm_source_hash() or kernel not in rec.get("kernels", {}) or \
            rec.get("n_abatch") != n_abatch:
        return None
    return rec["kernels"][kernel]["bytes"]


def traffic_summary(args):
    """rocprofv3 FETCH_SIZE / WRITE_SIZE counter CSVs (KiB per dispatch) of the default split
    command run with --copy-probe -> HBM bytes per launch of each split GEMM stage.  Each counter
    is scaled by what it reads for the 1 GiB device-to-device copy (its largest copy dispatch),
    which moves 1 GiB each way; the record carries the source hash and the batch size that
    measured_traffic checks before bench.py reports it."""
    import collections
    import csv
    import re

    def load(d):
        per = collections.defaultdict(list)
        with open(os.path.join(d, "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return per

    fetch, write = load(args.traffic_summary[0]), load(args.traffic_summary[1])

    def probe(per):
        return max(max(v) for k, v in per.items() if "copy" in k.lower())

    ff, wf = (1 << 20) / probe(fetch), (1 << 20) / probe(write)
    o, v, n, _ = WORKLOADS[args.workload]
    sf, sa = DEFAULT_SLICES[args.precision]
    nA = args.n_abatch or tuned_batch(args.tuned, o, v, n, PREC_CODE[args.precision], sf, 0, sa)
    stage = {"0": "gemm_b", "1": "gemm_c", "3": "gemm_e", "4": "gemm_f"}
    out = {"sources_sha256_16": gemm_source_hash(), "workload": args.workload, "precision": args.precision,
           "n_abatch": nA, "n_slices": sf, "n_slices_adjoint": sa, "fetch_factor": ff, "write_factor": wf,
           "kernels": {}}
    rows = []
    for k in fetch:
        fk = sum(fetch[k]) / len(fetch[k])
        wk = sum(write.get(k, [0.0])) / max(1, len(write.get(k, [])))
        gb = (fk * ff + wk * wf) * 1024 / 1e9
        rows.append((gb, "| `%s` | %d | %.4g | %.4g | %.2f |" % (k.split("(")[0].replace("void ", ""), len(fetch[k]),
                                                                 fk, wk, gb)))
        m = re.search(r"gemm_(?:split|i8)_kernel<(\d), [^,]+, (\d+)>", k)
        if m and m.group(2) in stage:
            out["kernels"][stage[m.group(2)]] = {"fetch_kib": fk, "write_kib": wk, "bytes": (fk * ff + wk * wf) * 1024,
                                                 "slices": int(m.group(1))}
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_pm.json" % (args.workload, args.precision))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("copy probe: FETCH_SIZE x %.3f, WRITE_SIZE x %.3f; written %s" % (ff, wf, os.path.relpath(path, ROOT)))
    print("| Kernel | Launches | FETCH KiB/launch (raw) | WRITE KiB/launch (raw) | HBM GB/launch (scaled) |")
    print("|---|---|---|---|---|")
    for _, line in sorted(rows, key=lambda x: -x[0])[:14]:
        print(line)


def blas_threads():
    """Threads of the BLAS that numpy's matrix products run on (what the CPU oracle uses)."""
    try:
        import threadpoolctl
        n = [d.get("num_threads", 0) for d in threadpoolctl.threadpool_info() if d.get("user_api") == "blas"]
        if n and max(n) > 0:
            return max(n)
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def nominal_flops(o, v, n):
    return 4.0 * v ** 4 * (n + o * o) + 2.0 * o * o * v * v


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="retinal", choices=sorted(WORKLOADS))
    ap.add_argument("--shape", default=None, help="o,v,n override (probe shapes)")
    ap.add_argument("--precision", default="int8", choices=["int8", "bf16", "fp64"],
                    help="split slices in INT8 (the default) or BF16, or the FP64 MFMA path")
    ap.add_argument("--slices", type=int, default=0,
                    help="slices of the forward GEMMs (0 = the format's benchmark default: 6 INT8, 5 BF16)")
    ap.add_argument("--slices-adjoint", type=int, default=None,
                    help="slices of the adjoint GEMMs (default: 5 INT8 / 4 BF16 with the default forward count, "
                         "else the forward's; they keep X within 1e-8 with margin, the energy needs the forward's)")
    ap.add_argument("--n-abatch", type=int, default=0)
    ap.add_argument("--cpu-rows", type=int, default=1, help="a (and p) rows the CPU baseline computes; 0 = skip")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the untimed FP64 leg that the split path is compared with")
    ap.add_argument("--autotune", default=None, metavar="CACHE",
                    help="choose the virtual-batch size with ladder_autotune before the timed region (within the "
                         "free HBM) and append the choice to CACHE (JSON lines); with --n-abatch 0 the timed "
                         "step then uses it")
    ap.add_argument("--tuned", default=TUNED_CACHE, metavar="CACHE",
                    help="load tuned batch sizes from CACHE (ladder_autotune_load) before running; "
                         "default: the committed MI355X cache; 'none' to skip")
    ap.add_argument("--dense", action="store_true",
                    help="dense contraction instead of the +/- packed one (LADDER_FLAG_DENSE)")
    ap.add_argument("--next-rows", action="store_true",
                    help="also time the transposed ladder (dE/dtau), the metric contraction V, the MO "
                         "back-transformation and the excited-state OV^3 block d_abci once on the same "
                         "inputs, with sampled checks")
    ap.add_argument("--decay", type=float, default=0.0, metavar="ALPHA",
                    help="stress variant of the inputs: Cholesky vectors scaled by exp(-ALPHA J / n) "
                         "(0 = the plain recipe)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy first (reference kernel for the HBM traffic counters)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="no GPU: turn the counter CSVs of two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE) "
                         "of this workload's default command with --copy-probe into "
                         "profiles/traffic_<workload>_<precision>_pm.json and print the per-kernel table")
    ap.add_argument("--fd", type=int, default=200, metavar="K",
                    help="autograd workload: LadderEnergy forward + backward (split) timed, then K central finite "
                         "differences of the FP64 energy (step 1e-6) on random L entries against its dE/dL "
                         "(0 = time the plain forward + adjoint step instead)")
    ap.add_argument("--budget", type=float, default=420.0, metavar="SECONDS",
                    help="wall-clock budget from process start; the timed steps are capped so that the run "
                         "(legs included) ends within it (0 = run exactly --steps and --warmup)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the ladder is measured on one GPU (one MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.traffic_summary:
        return traffic_summary(args)

    import numpy as np
    import torch

    import paper_2202_02019_amd as P
    from synthetic import gpu as SG

    if args.workload in ("batched", "batched_small"):
        return run_batched(args)
    if args.workload == "autograd" and args.fd > 0:
        return run_autograd(args)
    o, v, n, seed = WORKLOADS[args.workload]
    name = args.workload
    if args.shape:
        o, v, n = (int(x) for x in args.shape.split(","))
        name = "probe"
    prec_code = PREC_CODE[args.precision]
    split = args.precision != "fp64"
    # the benchmark's slice counts per format unless given; the library's rule then applies
    # (n_slices 0 means 5 for BF16 and 6 for INT8, n_slices_adjoint 0 means n_slices)
    dfw, dadj = DEFAULT_SLICES.get(args.precision, (5, 4))
    if not args.slices:
        args.slices = dfw
    S_fwd = args.slices
    if args.slices_adjoint is None:
        args.slices_adjoint = dadj if S_fwd == dfw else 0
    S_adj = args.slices_adjoint or S_fwd
    flags = 2 if args.dense else 0
    nA_source = "explicit" if args.n_abatch else "library default"
    tuned = None
    if args.n_abatch == 0 and not args.autotune and args.tuned not in (None, "none"):
        tuned = tuned_batch(args.tuned, o, v, n, prec_code, S_fwd, flags, S_adj)
        if tuned:
            nA_source = "autotune cache " + os.path.relpath(args.tuned, ROOT)
    if args.n_abatch == 0 and tuned is None and not args.autotune and name == "retinal":
        args.n_abatch = 8 if args.precision == "bf16" else 16  # a few large virtual batches fit in 288 GB
        nA_source = "fixed fallback"
    big = nominal_flops(o, v, n) > 1e14
    # a step at retinal scale takes about half a minute: one untimed warm-up step (code objects,
    # clocks and the fresh workspace settle), then the timed steps the budget allows
    steps = args.steps if args.steps is not None else (20 if big else 10)
    warmup = args.warmup if args.warmup is not None else (1 if big else 2)
    if steps < 1 or warmup < 1:
        ap.error("--steps and --warmup must be >= 1")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t0 = time.time()
    L = SG.draw_L_vv(seed, o, v, n)
    Lov = SG.draw_L_ov(seed, o, v, n)
    if args.decay:
        import synthetic
        f = torch.from_numpy(synthetic.decay_factors(n, args.decay)).to(dev)
        L.mul_(f)
        Lov.mul_(f)
    eps = SG.draw_eps(seed, o, v)
    tau = P.mp2_amplitudes(Lov, eps, o=o, v=v, n=n)
    del Lov
    tbar = SG.add_noise(seed, o, v, tau)
    R = torch.empty_like(tau)
    X = torch.empty_like(L)
    E = torch.empty((), dtype=torch.float64, device=dev)
    prec = {"fp64": P.FP64, "bf16": P.SPLIT_BF16, "int8": P.SPLIT_INT8}[args.precision]
    opts = P.Options(precision=prec, n_slices=args.slices if split else 0, n_abatch=args.n_abatch,
                     flags=P.FLAG_DENSE if args.dense else 0, n_slices_adjoint=args.slices_adjoint if split else 0)
    tune_s = None
    if tuned:
        P.autotune_load(args.tuned)
    if args.autotune:
        # the tuner may try any batch size whose workspace fits the free HBM (less a margin)
        free, _ = torch.cuda.mem_get_info()
        wst = torch.empty(max(free - (6 << 30), 1 << 20), dtype=torch.uint8, device=dev)
        c0 = time.time()
        tuned = P.autotune(L, tau, tbar, o=o, v=v, n=n, ws=wst, R=R, X=X, opts=opts, cache_path=args.autotune)
        torch.cuda.synchronize()
        tune_s = time.time() - c0
        nA_source = "ladder_autotune (%.1f s)" % tune_s
        del wst
        torch.cuda.empty_cache()
        print("bench: autotune chose n_abatch = %d in %.1f s" % (tuned, tune_s), file=sys.stderr, flush=True)
    wsb = P.workspace_size(o, v, n, opts)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    print("bench: %s o=%d v=%d n=%d precision=%s inputs ready in %.1fs, workspace %.2f GiB"
          % (name, o, v, n, args.precision, time.time() - t0, ws.numel() / 2 ** 30), file=sys.stderr, flush=True)

    def step():
        P.forward(L, tau, tbar, o=o, v=v, n=n, R=R, E=E, ws=ws, opts=opts)
        P.adjoint(L, tau, tbar, o=o, v=v, n=n, X=X, ws=ws, opts=opts)

    def left():
        """Seconds of the wall-clock budget still free (infinite without a budget)."""
        return args.budget - (time.time() - T_START) if args.budget > 0 else float("inf")

    steps_req, warmup_req = steps, warmup
    stream = torch.cuda.current_stream()
    # warm-up step 0 on the wall clock: code objects, clocks and the fresh workspace settle, and its
    # duration sizes the rest of the run
    w0 = time.time()
    step()
    torch.cuda.synchronize()
    t_step = time.time() - w0
    warm_done = 1
    E_warm = float(E.cpu())
    print("bench: warm-up step 0 done (%.1f s), %.0f s of the budget left" % (t_step, left()), file=sys.stderr,
          flush=True)
    F = nominal_flops(o, v, n)
    skipped = {}

    compare = None
    if split and not args.no_compare:
        # the same step on the FP64 MFMA path (untimed for `value`) on the same device arrays; it takes
        # about 1.5 split steps at the retinal shape, so it runs only if that and one timed step fit
        if left() < 2.0 * t_step + t_step + 20.0:
            skipped["fp64_comparison"] = "wall-clock budget"
        else:
            # the FP64 leg takes its batch size from the tuned table when the cache has one for it
            t64 = tuned_batch(args.tuned if args.tuned not in (None, "none") else None, o, v, n, 0, 0, flags)
            if t64:
                P.autotune_load(args.tuned)
            o64 = P.Options(precision=P.FP64, n_abatch=0 if t64 else (16 if name == "retinal" else 0),
                            flags=P.FLAG_DENSE if args.dense else 0)
            # the FP64 leg gets its own workspace in place of the split one (never both at once),
            # with the tuned batch only if it fits beside R64 and X64
            del ws
            torch.cuda.empty_cache()
            free, _ = torch.cuda.mem_get_info()
            extra = (R.numel() + X.numel()) * 8 + (4 << 30)
            if t64 and P.workspace_size(o, v, n, o64) + extra > free:
                t64 = None
                o64 = P.Options(precision=P.FP64, n_abatch=16 if name == "retinal" else 0,
                                flags=P.FLAG_DENSE if args.dense else 0)
            ws64 = torch.empty(P.workspace_size(o, v, n, o64), dtype=torch.uint8, device=dev)
            R64 = torch.empty_like(R)
            E64 = torch.empty((), dtype=torch.float64, device=dev)
            X64 = torch.empty_like(X)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ev0.record(stream)
            P.forward(L, tau, tbar, o=o, v=v, n=n, R=R64, E=E64, ws=ws64, opts=o64)
            P.adjoint(L, tau, tbar, o=o, v=v, n=n, X=X64, ws=ws64, opts=o64)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms64 = ev0.elapsed_time(ev1)
            e64 = float(E64.cpu())
            del ws64
            torch.cuda.empty_cache()

            def err_max(a, b):  # max|a - b| / max|b|, one leading slice at a time (no full-size temporaries)
                num = max(float((a[i] - b[i]).abs().max()) for i in range(a.shape[0]))
                den = max(float(b[i].abs().max()) for i in range(b.shape[0]))
                return num / den

            compare = {"fp64_ms_per_step": ms64, "fp64_dense_equivalent_tflops": F / (ms64 * 1e-3) / 1e12,
                       "fp64_n_abatch": t64 or o64.n_abatch,
                       "err_E_vs_fp64": abs(E_warm - e64) / abs(e64),
                       "err_R_vs_fp64": err_max(R, R64),
                       "err_X_vs_fp64": err_max(X, X64),
                       "outputs_compared": "split outputs of warm-up step 0 (bitwise equal to the timed steps' when "
                                           "deterministic_vs_warmup is true)"}
            # rows of the FP64 outputs kept for the BF16 leg below: R[:, :, a, :] and X[a] for three a
            rows64 = sorted({0, v // 2, v - 1})
            R64_rows = R64[:, :, rows64, :].clone()
            X64_rows = X64[rows64].clone()
            del R64, X64
            torch.cuda.empty_cache()
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
            print("bench: fp64 comparison step %.1f s, %.0f s of the budget left" % (ms64 / 1e3, left()),
                  file=sys.stderr, flush=True)

    cpu = None
    errs = {}
    if args.cpu_rows > 0:
        import oracle
        k = min(args.cpu_rows, v)
        fl = k * (2.0 * v ** 3 * n + 2.0 * o * o * v ** 3 + 2.0 * o * o * v) + k * (2.0 * o * o * v ** 3 + 2.0 * v ** 3 * n)
        # host copies of L, tau and tbar (one byte-copy pass each) plus the oracle at a rate no host here
        # falls below (0.1 TFLOP/s); it runs only if that and one timed step fit
        est = 8.0 * (L.numel() + tau.numel() + tbar.numel()) / 2e9 + fl / 1e11
        if left() < est + t_step + 20.0:
            skipped["cpu_baseline"] = "wall-clock budget (estimated %.0f s)" % est
        else:
            Lh, th, wh = L.cpu().numpy(), tau.cpu().numpy(), tbar.cpu().numpy()
            threads = blas_threads()
            c0 = time.time()
            Rr, Er = oracle.matrix.forward(o, v, n, Lh, th, wh, a_range=(0, k))
            Xr = oracle.matrix.adjoint(o, v, n, Lh, th, wh, p_range=(0, k))
            cs = time.time() - c0
            cpu = {"value": fl / cs / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
                   "seconds": cs, "s_per_iter_extrapolated": F / (fl / cs),
                   "sample": "forward rows a<%d and adjoint rows p<%d at the full shape (o=%d v=%d n=%d); "
                             "numpy matrix-product FP64 oracle; nominal flops %.3e" % (k, k, o, v, n, fl)}
            Rg = R[:, :, :k, :].cpu().numpy()
            Xg = X[:k].cpu().numpy()
            errs = {"err_sample_R": float(np.abs(Rg - Rr).max() / np.abs(Rr).max()),
                    "err_sample_X": float(np.abs(Xg - Xr).max() / np.abs(Xr).max()),
                    "err_sample_E_rows": abs(math.fsum((wh[:, :, :k, :] * Rg).ravel()) - Er) / abs(Er)}
            del Lh, th, wh
            print("bench: CPU oracle sample %.1f s, %.0f s of the budget left" % (cs, left()), file=sys.stderr,
                  flush=True)

    # the metric's named method beside the INT8 headline: one step of the same path with BF16 slices
    # (5 forward / 4 adjoint, its tuned batch) on the same inputs, timed as it runs (its first
    # launches load their code objects, well under a second), with E against the FP64 leg and the
    # kept FP64 rows of R and X; its outputs go to R and X, which the timed steps overwrite
    bf16 = None
    if args.precision == "int8" and compare is not None and not args.dense:
        if left() < 1.4 * t_step + t_step + 20.0:
            skipped["bf16_comparison"] = "wall-clock budget"
        else:
            tb = tuned_batch(args.tuned if args.tuned not in (None, "none") else None, o, v, n, 1, 5, flags, 4)
            if tb:
                P.autotune_load(args.tuned)
            ob = P.Options(precision=P.SPLIT_BF16, n_slices=5, n_slices_adjoint=4, n_abatch=0 if tb else 16)
            del ws
            torch.cuda.empty_cache()
            wsb16 = torch.empty(P.workspace_size(o, v, n, ob), dtype=torch.uint8, device=dev)
            Eb = torch.empty((), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            ev0.record(stream)
            P.forward(L, tau, tbar, o=o, v=v, n=n, R=R, E=Eb, ws=wsb16, opts=ob)
            P.adjoint(L, tau, tbar, o=o, v=v, n=n, X=X, ws=wsb16, opts=ob)
            ev1.record(stream)
            torch.cuda.synchronize()
            msb = ev0.elapsed_time(ev1)
            del wsb16
            torch.cuda.empty_cache()
            eb = float(Eb.cpu())
            bf16 = {"ms_per_step": msb, "n_slices": 5, "n_slices_adjoint": 4, "n_abatch": tb or 16,
                    "timing": "one step, no warm-up of its own",
                    "err_E_vs_fp64": abs(eb - e64) / abs(e64),
                    "err_R_rows_vs_fp64": float((R[:, :, rows64, :] - R64_rows).abs().max() / R64_rows.abs().max()),
                    "err_X_rows_vs_fp64": float((X[rows64] - X64_rows).abs().max() / X64_rows.abs().max()),
                    "rows": "R[:, :, a, :] and X[a] for a in %s" % rows64,
                    "speedup_vs_fp64": compare["fp64_ms_per_step"] / msb}
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
            print("bench: bf16 comparison step %.1f s, %.0f s of the budget left" % (msb / 1e3, left()),
                  file=sys.stderr, flush=True)

    # timed steps: as many as fit the rest of the budget (at most the number asked, at least one), then
    # further warm-up steps before them if there is still room
    tail = 15.0  # the matrix-core probe, the last checks and the JSON line
    fit = int(max(0.0, left() - tail) // t_step) if args.budget > 0 else steps_req
    steps = max(1, min(steps_req, fit))
    extra = min(warmup_req - 1, int(max(0.0, left() - tail - steps * t_step) // t_step)) if args.budget > 0 \
        else warmup_req - 1
    for i in range(max(0, extra)):
        step()
        torch.cuda.synchronize()
        warm_done += 1
        print("bench: warmup step %d done" % warm_done, file=sys.stderr, flush=True)
    print("bench: timing %d of %d requested steps (%.0f s of the budget left)" % (steps, steps_req, left()),
          file=sys.stderr, flush=True)

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
    E_final = float(E.cpu())

    dom_name, dom = max(stages.items(), key=lambda kv: kv[1]["total_ms"])
    # FP64-equivalent rate of the dominant stage: 2 M N K flops per launch over its mean launch time
    fp64_equiv = dom["flops"] / dom["launches"] / (dom["avg_ms"] * 1e-3) / 1e12
    nA_eff = args.n_abatch or tuned
    default_shape = split and (S_fwd, S_adj) == DEFAULT_SLICES[args.precision] and not args.dense
    traffic = measured_traffic(name, args.precision, dom_name, nA_eff) if default_shape else None
    if split:
        # the split method's unit of work: S(S+1)/2 slice products (BF16 or INT8 MFMA) per
        # FP64-equivalent MAC, each product 2 M N K operations
        S = S_adj if dom_name in ("gemm_e", "gemm_f") else S_fwd
        prods = S * (S + 1) // 2
        achieved, peak = fp64_equiv * prods, PEAK[args.precision]
    else:
        prods, achieved, peak = 1, fp64_equiv, PEAK["fp64"]
    roofline = {"bound": "mfma", "kernel": dom_name, "achieved": achieved, "peak": peak,
                "unit": "TOP/s" if args.precision == "int8" else "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic,
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-kernel scaled)",
                "algorithmic_bytes": dom["bytes"] / dom["launches"],
                "avg_launch_ms": dom["avg_ms"], "launches_per_step": dom["launches"] / steps,
                "slice_products": prods if split else None,
                "fp64_equivalent_tflops": fp64_equiv,
                "fp64_equivalent_frac_of_fp64_peak": fp64_equiv / PEAK["fp64"]}
    ceiling = mfma_ceiling()
    roofline["measured_mfma_ceiling"] = ceiling[("fp64" if not split else args.precision) + "_tflops"]
    roofline["frac_of_measured_ceiling"] = achieved / roofline["measured_mfma_ceiling"]
    stage_summary = {k: {"ms_per_step": s_["total_ms"] / steps, "launches_per_step": s_["launches"] / steps,
                         "tflops": (s_["flops"] / (s_["total_ms"] * 1e-3) / 1e12) if s_["total_ms"] > 0 else None}
                     for k, s_ in stages.items()}
    executed = sum(s_["flops"] for k, s_ in stages.items() if k.startswith("gemm")) / steps
    value = executed / (ms * 1e-3) / 1e12
    if compare is not None:
        compare["fp64_tflops"] = executed / (compare["fp64_ms_per_step"] * 1e-3) / 1e12
        compare["speedup_vs_fp64"] = compare["fp64_ms_per_step"] / ms
        if bf16 is not None:
            # the same GEMM shapes: the FP64-equivalent flops executed per step are the INT8 step's
            bf16["value"] = executed / (bf16["ms_per_step"] * 1e-3) / 1e12
            bf16["unit"] = "TFLOP/s"
            compare["bf16_split"] = bf16

    nxt = None
    if args.next_rows:
        import oracle
        nxt = {}
        # its own workspace (at retinal scale with the batch of 8, so that G fits beside it)
        opts_n = P.Options(precision=prec, n_slices=args.slices, n_abatch=8 if name == "retinal" else args.n_abatch,
                           flags=P.FLAG_DENSE if args.dense else 0)
        del ws
        torch.cuda.empty_cache()
        ws = torch.empty(max(P.tau_gradient_workspace_size(o, v, n, opts_n), P.back_transform_workspace_size(v, n)),
                         dtype=torch.uint8, device=dev)
        # dE/dtau = transposed ladder of tbar; nominal flops as the forward (2 n v^4 + 2 o^2 v^4)
        G = torch.empty_like(R)
        torch.cuda.synchronize()
        ev0.record(stream)
        P.tau_gradient(L, tbar, o=o, v=v, n=n, G=G, ws=ws, opts=opts_n)
        ev1.record(stream)
        torch.cuda.synchronize()
        mst = ev0.elapsed_time(ev1)
        Ft = 2.0 * n * v ** 4 + 2.0 * o * o * v ** 4
        Gr = oracle.matrix.tau_gradient(o, v, n, L.cpu().numpy(), tbar.cpu().numpy(), c_range=(0, 1))
        nxt["tau_gradient"] = {"ms": mst, "nominal_flops": Ft, "tflops": Ft / (mst * 1e-3) / 1e12,
                               "err_sample_row_c0": float(np.abs(G[:, :, :1, :].cpu().numpy() - Gr).max()
                                                          / np.abs(Gr).max())}
        del G
        # V = L^T W with W = X/2 (Z := L): trace V must equal E
        torch.cuda.synchronize()
        ev0.record(stream)
        V = P.metric_contraction(L, X, v=v, n=n, alpha=0.5)
        ev1.record(stream)
        torch.cuda.synchronize()
        msv = ev0.elapsed_time(ev1)
        Fv = 2.0 * n * n * v * v
        nxt["metric_contraction"] = {"ms": msv, "flops": Fv, "tflops": Fv / (msv * 1e-3) / 1e12,
                                     "err_trace_V_vs_E": abs(float(torch.trace(V)) - float(E)) / abs(float(E))}
        del V
        # MO back-transformation of W = X/2 with seeded x, y = 1 + noise
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        xm = torch.eye(v, dtype=torch.float64, device=dev) + 0.1 * torch.randn(
            (v, v), dtype=torch.float64, device=dev, generator=gen) / v ** 0.5
        ym = torch.eye(v, dtype=torch.float64, device=dev) + 0.1 * torch.randn(
            (v, v), dtype=torch.float64, device=dev, generator=gen) / v ** 0.5
        Wmo = torch.empty_like(X)
        torch.cuda.synchronize()
        ev0.record(stream)
        P.back_transform(xm, ym, X, v=v, n=n, Wmo=Wmo, alpha=0.5, ws=ws)
        ev1.record(stream)
        torch.cuda.synchronize()
        msb = ev0.elapsed_time(ev1)
        Fb = 4.0 * v ** 3 * n
        K = n // 2
        Wr = 0.5 * oracle.matrix.back_transform(v, 1, xm.cpu().numpy(), ym.cpu().numpy(), X[:, :, K:K + 1].cpu().numpy())
        nxt["back_transform"] = {"ms": msb, "flops": Fb, "tflops": Fb / (msb * 1e-3) / 1e12,
                                 "err_sample_K": float(np.abs(Wmo[:, :, K:K + 1].cpu().numpy() - Wr).max()
                                                       / np.abs(Wr).max())}
        del Wmo
        # excited-state OV^3 block d_abci = L_ji^ac R_j^b with L_2 := tbar, seeded singles R_1 and
        # Z := (L, seeded Zvo); checks: sampled rows against the oracle and sum Zvv*Wab = sum Zvo*Wci
        del ws
        torch.cuda.empty_cache()
        R1 = torch.randn((o, v), dtype=torch.float64, device=dev, generator=gen) * 0.1
        Zvo = torch.randn((v, o, n), dtype=torch.float64, device=dev, generator=gen) / n ** 0.5
        ws = torch.empty(P.ov3_abci_workspace_size(o, v, n), dtype=torch.uint8, device=dev)
        Wab, Wci = torch.empty_like(X), torch.empty((v, o, n), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        ev0.record(stream)
        P.ov3_abci(tbar, R1, L, Zvo, o=o, v=v, n=n, Wab=Wab, Wci=Wci, ws=ws)
        ev1.record(stream)
        torch.cuda.synchronize()
        mso = ev0.elapsed_time(ev1)
        Fo = 4.0 * o * o * v * v * n + 4.0 * o * v * v * n
        s_ab, s_ci = float((L * Wab).sum()), float((Zvo * Wci).sum())
        th_, R1h, Zvoh = tbar.cpu().numpy(), R1.cpu().numpy(), Zvo.cpu().numpy()
        ab, ci = np.array([[0, 0], [v - 1, v // 2]]), np.array([[v // 3, o - 1]])
        ra = oracle.ov3_abci_wab(o, v, n, th_, R1h, Zvoh, ab)
        rc = oracle.ov3_abci_wci(o, v, n, th_, R1h, L.cpu().numpy(), ci)
        ea = float(np.abs(Wab[ab[:, 0], ab[:, 1]].cpu().numpy() - ra).max() / np.abs(ra).max())
        ec = float(np.abs(Wci[ci[:, 0], ci[:, 1]].cpu().numpy() - rc).max() / np.abs(rc).max())
        nxt["ov3_abci"] = {"ms": mso, "flops": Fo, "tflops": Fo / (mso * 1e-3) / 1e12,
                           "err_sample_Wab": ea, "err_sample_Wci": ec,
                           "identity_rel": abs(s_ab - s_ci) / float((L * Wab).abs().sum())}
        del Wab, Wci, th_
        # excited-state OV^3 block d_abic with L_2 := tbar, t := tau, R_2 := R (the ladder output), seeded
        # singles L_1, R_1 and R_0; check: sum Zvv*Wab = sum Zov*Wic (Zvv := L, Zov := the seeded block)
        del ws
        torch.cuda.empty_cache()
        L1 = torch.randn((o, v), dtype=torch.float64, device=dev, generator=gen) * 0.1
        Zov = Zvo.view(v, o, n).permute(1, 0, 2).contiguous()
        del Zvo
        opts_o = P.Options(precision=prec, n_slices=args.slices)
        ws = torch.empty(P.ov3_abic_workspace_size(o, v, n, opts_o), dtype=torch.uint8, device=dev)
        Wab, Wic = torch.empty_like(X), torch.empty((o, v, n), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        ev0.record(stream)
        P.ov3_abic(0.25, L1, tbar, tau, R1, R, L, Zov, o=o, v=v, n=n, Wab=Wab, Wic=Wic, ws=ws, opts=opts_o)
        ev1.record(stream)
        torch.cuda.synchronize()
        msi = ev0.elapsed_time(ev1)
        # GEMM flops above o v^2 n: V+Y, Yt and S (8 o^3 v^3), X_ab, B_iamn, the S contractions of
        # both sides (4 o v^3 n) and the eight (o v)^2 n contractions of terms (1), (2), (4), (5), (7)
        Fi = (8.0 * o ** 3 * v ** 3 + 2.0 * o ** 2 * v ** 3 + 2.0 * o ** 3 * v ** 2 + 4.0 * o * v ** 3 * n
              + 16.0 * o * o * v * v * n)
        s_ab, s_ic = float((L * Wab).sum()), float((Zov * Wic).sum())
        nxt["ov3_abic"] = {"ms": msi, "flops": Fi, "tflops": Fi / (msi * 1e-3) / 1e12,
                           "precision": args.precision,
                           "identity_rel": abs(s_ab - s_ic) / float((L * Wab).abs().sum())}
        del Wab, Wic, Zov, ws
        torch.cuda.empty_cache()
        print("bench: next rows: tau gradient %.1f s, V %.1f ms, back-transform %.1f ms, OV3 d_abci %.1f ms, "
              "OV3 d_abic %.1f s" % (mst / 1e3, msv, msb, mso, msi / 1e3), file=sys.stderr, flush=True)

    out = {
        "metric": "ladder fwd+adjoint TFLOP/s & s/iter, split-BF16 vs FP64 at <=1e-10 rel err in E",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": steps, "warmup": warm_done,
        "steps_requested": steps_req, "warmup_requested": warmup_req,
        "ms_per_step": ms, "s_per_iter": ms / 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if not split else args.precision + "-split/f64",
        "data": "synthetic",
        "config": {"workload": name, "o": o, "v": v, "n_chol": n, "seed": seed, "precision": args.precision,
                   "n_slices": S_fwd if split else 0,
                   "n_slices_adjoint": S_adj if split else 0, "n_abatch": nA_eff or 0,
                   "n_abatch_source": nA_source, "nominal_flops": F,
                   "path": "dense" if args.dense else "+/- packed",
                   "decay": args.decay},
        "flop_count": "value = the FP64-equivalent GEMM flops the path executes per step (2 M N K per product, "
                      "executed_gemm_flops) over the step time; dense_equivalent_tflops counts the dense "
                      "F = 4 v^4 (n + o^2) + 2 o^2 v^2 instead",
        "executed_gemm_flops": executed,
        "frac_fp64_peak": value / PEAK["fp64"],
        "dense_equivalent_tflops": F / (ms * 1e-3) / 1e12,
        "energy": E_final,
        "deterministic_vs_warmup": E_final == E_warm,
        "budget_s": args.budget, "wall_s_at_print": time.time() - T_START, "warmup_step_s": t_step,
        "skipped": skipped or None,
        "roofline": roofline, "stages": stage_summary, "cpu_baseline": cpu, "mfma_probe": ceiling,
        "fp64_comparison": compare,
        "next_rows": nxt,
    }
    out.update(errs)
    print(json.dumps(out), flush=True)


def run_autograd(args):
    """The differentiation workload (o=40, v=350, n=1200, seed 5): E = LadderEnergy(L, tau, tbar) with the
    split forward (R, E) and the library backward (dE/dL by the adjoint, dE/dtau by the transposed ladder),
    timed per step; then K central differences of the FP64 GPU energy, (E(L + h e_k) - E(L - h e_k)) / 2h with
    h = 1e-6, on random (a, c, J) entries against the backward's dE/dL.  E is quadratic in each entry, so the
    central difference has no truncation error: the deviation is rounding only, about u |E| / h."""
    import numpy as np
    import torch

    import paper_2202_02019_amd as P
    from synthetic import gpu as SG

    o, v, n, seed = WORKLOADS["autograd"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L = SG.draw_L_vv(seed, o, v, n)
    Lov = SG.draw_L_ov(seed, o, v, n)
    tau = P.mp2_amplitudes(Lov, SG.draw_eps(seed, o, v), o=o, v=v, n=n)
    del Lov
    tbar = SG.add_noise(seed, o, v, tau)
    fmt = "bf16" if args.precision == "bf16" else "int8"  # the workload is a split one
    dfw, dadj = DEFAULT_SLICES[fmt]
    S_fwd = args.slices or dfw
    S_adj = args.slices_adjoint if args.slices_adjoint is not None else (dadj if S_fwd == dfw else 0)
    opts = P.Options(precision=P.SPLIT_BF16 if fmt == "bf16" else P.SPLIT_INT8, n_slices=S_fwd, n_slices_adjoint=S_adj)
    Lq = L.clone().requires_grad_(True)
    tq = tau.clone().requires_grad_(True)
    steps = args.steps or 3
    warmup = args.warmup or 1

    def step():
        Lq.grad = None
        tq.grad = None
        E = P.ladder_energy(Lq, tq, tbar, (o, v, n), opts)
        E.backward()
        return E

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    P.profile_start()
    ev0.record(stream)
    for _ in range(steps):
        E = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    stages = P.profile_stop()
    ms = ev0.elapsed_time(ev1) / steps
    executed = sum(s_["flops"] for k, s_ in stages.items() if k.startswith("gemm")) / steps
    X = Lq.grad.detach()
    e_split = float(E.detach())
    print("bench: autograd step %.1f ms, E %.15e" % (ms, e_split), file=sys.stderr, flush=True)

    # central differences of the FP64 energy on K random entries
    o64 = P.Options(precision=P.FP64)
    ws64 = torch.empty(P.workspace_size(o, v, n, o64), dtype=torch.uint8, device=dev)
    R64 = torch.empty_like(tau)
    E64 = torch.empty((), dtype=torch.float64, device=dev)
    P.forward(L, tau, tbar, o=o, v=v, n=n, R=R64, E=E64, ws=ws64, opts=o64)
    e_fp64 = float(E64.cpu())
    rng = np.random.default_rng(seed)
    a_, c_, J_ = rng.integers(v, size=args.fd), rng.integers(v, size=args.fd), rng.integers(n, size=args.fd)
    h = 1e-6
    fd = np.empty(args.fd)
    t0 = time.time()
    for k in range(args.fd):
        a, c, J = int(a_[k]), int(c_[k]), int(J_[k])
        x0 = float(L[a, c, J])
        vals = []
        for sgn in (1.0, -1.0):
            L[a, c, J] = x0 + sgn * h
            P.forward(L, tau, tbar, o=o, v=v, n=n, R=R64, E=E64, ws=ws64, opts=o64)
            vals.append(float(E64.cpu()))
        L[a, c, J] = x0
        fd[k] = (vals[0] - vals[1]) / (2.0 * h)
        if k % 50 == 49:
            print("bench: %d central differences (%.0f s)" % (k + 1, time.time() - t0), file=sys.stderr, flush=True)
    fd_s = time.time() - t0
    got = X[a_, c_, J_].cpu().numpy()
    scale = float(X.abs().max())
    dev_abs = np.abs(fd - got)
    out = {
        "metric": "ladder fwd+adjoint TFLOP/s & s/iter, split-BF16 vs FP64 at <=1e-10 rel err in E",
        "value": executed / (ms * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "s_per_iter": ms / 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": fmt + "-split/f64", "data": "synthetic",
        "config": {"workload": "autograd", "o": o, "v": v, "n_chol": n, "seed": seed, "precision": fmt,
                   "n_slices": S_fwd, "n_slices_adjoint": S_adj or S_fwd,
                   "step": "LadderEnergy forward (split R, E) + backward (adjoint dE/dL, transposed ladder dE/dtau)"},
        "executed_gemm_flops": executed,
        "stages": {k: {"ms_per_step": s_["total_ms"] / steps} for k, s_ in stages.items()},
        "energy_split": e_split, "energy_fp64": e_fp64, "err_E_split_vs_fp64": abs(e_split - e_fp64) / abs(e_fp64),
        "finite_differences": {"count": args.fd, "h": h, "seconds": fd_s,
                               "max_abs_dev": float(dev_abs.max()), "max_abs_dev_over_max_abs_X": float(dev_abs.max()) / scale,
                               "median_rel_dev": float(np.median(dev_abs / np.maximum(np.abs(fd), 1e-300))),
                               "rounding_scale_u_E_over_h": 2.0 ** -53 * abs(e_fp64) / h,
                               "entries": "(a, c, J) uniform, numpy default_rng(5)"},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_batched(args):
    """64 ragged instances: one graph launch of ladder_batched vs 64 sequential calls."""
    import torch

    import paper_2202_02019_amd as P
    import synthetic
    from synthetic import gpu as SG

    small = args.workload == "batched_small"
    sizes = synthetic.batched_sizes(8, 64, (4, 12), (20, 80)) if small else synthetic.batched_sizes(4, 64)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = {"fp64": P.FP64, "bf16": P.SPLIT_BF16, "int8": P.SPLIT_INT8}[args.precision]
    dfw, dadj = DEFAULT_SLICES.get(args.precision, (0, 0))
    S_fwd = args.slices or dfw
    S_adj = args.slices_adjoint if args.slices_adjoint is not None else (dadj if S_fwd == dfw else 0)
    opts = P.Options(precision=prec, n_slices=S_fwd, n_abatch=args.n_abatch, n_slices_adjoint=S_adj,
                     flags=P.FLAG_DENSE if args.dense else 0)
    insts = []
    t0 = time.time()
    for m, (o, v, n) in enumerate(sizes):
        seed = 1000 + m
        L = SG.draw_L_vv(seed, o, v, n)
        Lov = SG.draw_L_ov(seed, o, v, n)
        eps = SG.draw_eps(seed, o, v)
        tau = P.mp2_amplitudes(Lov, eps, o=o, v=v, n=n)
        del Lov
        tbar = SG.add_noise(seed, o, v, tau)
        insts.append(dict(o=o, v=v, n=n, L=L, tau=tau, tbar=tbar, R=torch.empty_like(tau),
                          E=torch.empty((), dtype=torch.float64, device=dev), X=torch.empty_like(L)))
    what = P.DO_FORWARD | P.DO_ADJOINT
    tuned_src = None
    if args.n_abatch == 0 and args.autotune:
        # tune every instance shape once (each on its own data), appending to the cache
        c0 = time.time()
        # each instance's plan must leave room for the graph's branch slots side by side
        free, _ = torch.cuda.mem_get_info()
        wst = torch.empty(max(free // 6, 1 << 20), dtype=torch.uint8, device=dev)
        for d in insts:
            P.autotune(d["L"], d["tau"], d["tbar"], o=d["o"], v=d["v"], n=d["n"], ws=wst, R=d["R"], X=d["X"],
                       opts=opts, cache_path=args.autotune)
        torch.cuda.synchronize()
        del wst
        torch.cuda.empty_cache()
        tuned_src = "ladder_autotune (%.1f s)" % (time.time() - c0)
    elif args.n_abatch == 0 and args.tuned not in (None, "none") and os.path.exists(args.tuned):
        if P.autotune_load(args.tuned) > 0:
            tuned_src = "autotune cache " + os.path.relpath(args.tuned, ROOT)
    ws = torch.empty(P.batched_workspace_size(insts, what, opts), dtype=torch.uint8, device=dev)
    F = sum(nominal_flops(o, v, n) for o, v, n in sizes)
    torch.cuda.synchronize()
    print("bench: batched 64 instances, F=%.3e, inputs ready in %.1fs, workspace %.2f GiB"
          % (F, time.time() - t0, ws.numel() / 2 ** 30), file=sys.stderr, flush=True)
    steps = args.steps if args.steps is not None else 2
    warmup = args.warmup if args.warmup is not None else 1
    stream = torch.cuda.current_stream()
    for _ in range(warmup):  # the first call captures the graph
        P.batched(insts, what, ws=ws, opts=opts)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        P.batched(insts, what, ws=ws, opts=opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    print("bench: graph %.1f ms per batch" % ms, file=sys.stderr, flush=True)
    # the same work as 64 sequential forward + adjoint calls on one stream
    wsq = torch.empty(max(P.workspace_size(d["o"], d["v"], d["n"], opts) for d in insts), dtype=torch.uint8, device=dev)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(insts) + 1)]
    evs[0].record(stream)
    for k, d in enumerate(insts):
        P.forward(d["L"], d["tau"], d["tbar"], o=d["o"], v=d["v"], n=d["n"], R=d["R"], E=d["E"], ws=wsq, opts=opts)
        P.adjoint(d["L"], d["tau"], d["tbar"], o=d["o"], v=d["v"], n=d["n"], X=d["X"], ws=wsq, opts=opts)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    ms_seq = evs[0].elapsed_time(evs[-1])
    per_inst = [{"o": d["o"], "v": d["v"], "n": d["n"], "ms": evs[k].elapsed_time(evs[k + 1]),
                 "tflops": nominal_flops(d["o"], d["v"], d["n"]) / (evs[k].elapsed_time(evs[k + 1]) * 1e-3) / 1e12}
                for k, d in enumerate(insts)]
    out = {
        "metric": "ladder fwd+adjoint TFLOP/s & s/iter, split-BF16 vs FP64 at <=1e-10 rel err in E",
        "value": F / (ms * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "s_per_iter": ms / 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else args.precision + "-split/f64", "data": "synthetic",
        "config": {"workload": args.workload, "instances": 64, "sizes_seed": 8 if small else 4,
                   "o_range": [4, 12] if small else [8, 40], "v_range": [20, 80] if small else [60, 300],
                   "data_seeds": "1000+m",
                   "precision": args.precision, "n_abatch": args.n_abatch,
                   "n_abatch_source": tuned_src or ("explicit" if args.n_abatch else "library default"),
                   "nominal_flops": F},
        "sequential_ms": ms_seq, "sequential_tflops": F / (ms_seq * 1e-3) / 1e12, "graph_speedup": ms_seq / ms,
        "sequential_per_instance": per_inst,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
