"""Benchmark: batched Gumbel-Max sketching on one MI355X.

One step = one FastGM-form sketch of the whole document-like batch already
resident in HBM: 10,000 sparse vectors, n+ ~ lognormal(ln 500, 1) clipped to
[10, 50000] (about 8.3 M entries), indices distinct in [0, 2^20), weights
Exp(1) fp32, k = 256 registers per vector, FP64 keys.

Prints one JSON line: registers/s (sum of k over the batch / step time), plus
vectors/s, the roofline of the FastGM kernel (VALU issue bound) measured with
HIP events on the launch stream, and the CPU oracle timed on a bounded sample
of the same batch.
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

# VALU lane-operation peak of MI355X: 256 CUs x 64 lanes x 2.4 GHz (one
# full-rate VALU instruction per lane per cycle).
PEAK_VALU_OPS = 256 * 64 * 2.4e9
# VALU issue slots of one FastGM arrival as compiled for gfx950 (hash of the
# arrival draw and of the shuffle draw, -ln, the order-statistic fma, the key
# multiply, the Fisher-Yates target); quarter-rate instructions (32-bit
# integer multiplies, f64 reciprocal) count 4 slots.
ARRIVAL_SLOTS = 180
HBM_PEAK = 8.0e12


def harmonic(k: int) -> float:
    return sum(1.0 / m for m in range(1, k + 1))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", choices=["fastgm", "plain"], default="fastgm")
    ap.add_argument("--k", type=int, default=256)
    ap.add_argument("--nvec", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2000,
                    help="vectors of the batch the CPU oracle sketches")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sketch "
              "batch is independent per vector, so N GPUs would each run this line on "
              "their own share.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import build as gmbuild
    from paper_2302_05176_amd import workloads as W

    if not os.path.exists(gmbuild.LIB):
        gmbuild.build(force=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    idx, w, off = W.batch(nvec=args.nvec, seed=1002)
    nnz = int(off[-1])
    k = args.k
    ti = torch.from_numpy(idx).to(dev)
    tw = torch.from_numpy(w).to(dev)
    to = torch.from_numpy(off).to(dev)
    out_i = torch.empty((args.nvec, k), dtype=torch.int32, device=dev)
    out_v = torch.empty((args.nvec, k), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        gm.sketch(ti, tw, to, k, args.seed, form=args.form, out_idx=out_i, out_val=out_v)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        starts[s].record(stream)
        gm.sketch(ti, tw, to, k, args.seed, form=args.form, out_idx=out_i, out_val=out_v)
        ends[s].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    ms_step = wall * 1e3 / args.steps
    avg_kern_s = sum(kern_ms) / len(kern_ms) / 1e3

    regs = args.nvec * k
    value = regs / (ms_step / 1e3)
    nplus = np.diff(off)
    if args.form == "fastgm":
        # expected arrivals of an exact pruned run: k H_k + n+ per vector (Sec. 2.5)
        units = float(args.nvec * k * harmonic(k) + nnz)
    else:
        units = float(k) * nnz
    ops = units * ARRIVAL_SLOTS
    achieved = ops / avg_kern_s
    bytes_alg = 8.0 * nnz + 8.0 * (args.nvec + 1) + 12.0 * regs
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_VALU_OPS / 1e12,
        "unit": "TOPS (VALU lane-ops/s)",
        "frac": achieved / PEAK_VALU_OPS,
        "traffic": None,
        "kernel": "fastgm_kernel" if args.form == "fastgm" else "plain_kernel",
        "kernel_ms": avg_kern_s * 1e3,
        "algorithmic_units": units,
        "unit_name": "arrivals" if args.form == "fastgm" else "keys",
        "slots_per_unit": ARRIVAL_SLOTS,
        "hbm_frac": bytes_alg / avg_kern_s / HBM_PEAK,
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        ncores = min(ncores, 16)
        oracle.set_threads(ncores)
        m = min(args.cpu_sample, args.nvec)
        so = off[: m + 1]
        c0 = time.perf_counter()
        oracle.sketch(idx, w, so, k, args.seed,
                      form=oracle.FORM_STREAM if args.form == "fastgm" else oracle.FORM_PLAIN)
        cdt = time.perf_counter() - c0
        cpu = {"value": m * k / cdt, "unit": "registers/s", "cores": ncores, "kind": "oracle",
               "sample": f"first {m} of the {args.nvec} vectors, "
                         f"{'Algorithm 2 (Stream-FastGM)' if args.form == 'fastgm' else 'plain O(k n+)'}"
                         f", {cdt:.2f} s"}

    line = {
        "metric": f"Gumbel-Max registers/sec (k={k})",
        "value": value,
        "unit": "registers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "vectors_per_s": args.nvec / (ms_step / 1e3),
        "config": {"workload": f"document batch: {args.nvec} sparse vectors, n+ ~ "
                               f"lognormal(ln 500, 1) in [10, 50000] (nnz={nnz}), Exp(1) "
                               f"fp32 weights, k={k}, {args.form} form",
                   "form": args.form, "k": k, "nvec": args.nvec, "nnz": nnz,
                   "mean_nplus": float(nplus.mean())},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
