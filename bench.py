"""Benchmark: Gumbel-Max sketching on one MI355X.

Default (the headline line): one step = one FastGM-form sketch of a
document-like batch already resident in HBM -- 10,000 sparse vectors,
n+ ~ lognormal(ln 500, 1) clipped to [10, 50000] (about 8.1 M entries),
distinct indices in [0, 2^20), Exp(1) fp32 weights, k = 256 registers per
vector, FP64 keys.  The JSON line reports registers/s (sum of k over the
batch / step time) and vectors/s, the roofline of the dominant kernel
(VALU-issue bound, durations from HIP events on its launch stream during
the timed steps), the CPU oracle timed on the host cores, and -- measured
after the timed steps -- the same batch at k = 1024 and the plain O(k n+)
form at both k for the FastGM/plain ratio.

Other workloads (`--workload`), each printing its own line:
  single  one vector, n+ = 1000, Uniform(0,1] weights, k = 128, both forms
  stream  one vector, n+ = 1e7, half Uniform(0,1] / half Pareto(1.5), k = 1024 and 4096
  uneven  uneven batch (Zipf n+, per-vector k in {64,256,1024,4096}, lognormal
          weights), autotuned, replayed from a captured HIP graph
  serve   continuous-batching serving loop, Poisson arrivals, k = 512, p50/p99
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU issue peak of MI355X in f64-rate lane-cycles: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (the FP64 vector rate, 78.6 TFLOP/s counting an FMA as 2).
# On gfx950 FP64 add/mul/fma, 32-bit integer multiplies and 64-bit shifts issue
# at this rate (1 slot), simple 32-bit ALU ops at twice it (0.5 slot), the
# FP64 reciprocal at a quarter of it (4 slots) -- rates measured with
# dependent-free instruction streams on MI355X.
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9
# Slots of one arrival of the draw specification as compiled for gfx950 (two
# splitmix64 hashes, the uniform, -ln with its division, the c_z division, the
# fma, the key multiply, the Fisher-Yates target): 106 VALU instructions,
# 100 slots.  A straight-line loop of arrivals runs at 3.3e11 arrivals/s
# (119 lane-cycles each), 84% of this count at the peak.
ARRIVAL_SLOTS = 100
# One plain key with its register compare (hash, uniform, -ln, multiply,
# lexicographic min): 88 VALU instructions, 81 slots.
PLAIN_KEY_SLOTS = 81
HBM_PEAK = 8.0e12
# The FastGM launch that takes most of a step drains every vector of at most
# 32768 entries of the batch's k range (larger ones are prepared by grid-wide
# passes and walked by another launch); the library names its timing entry
# "fastgm_class_kernel<W, G> [class c]" with c the k range (k <= 256: 0,
# <= 1024: 1, <= 2048: 2, else 3).
SMALL_LIMIT = 32768


def k_class(k: int) -> int:
    return 0 if k <= 256 else (1 if k <= 1024 else (2 if k <= 2048 else 3))


def harmonic(k: int) -> float:
    return sum(1.0 / m for m in range(1, k + 1))


def max_exp_quantile(k: int, p: float) -> float:
    """(1 - p) quantile of the maximum of k Exp(1) variables (Sec. 2.5)."""
    import math
    return -math.log(-math.expm1(math.log1p(-p) / k))


def rate_ceiling(k: int, seed: int = 1) -> float:
    """Arrivals/s of gm_rate_probe at this k: 2^21 lanes, each drawing k
    arrivals of its own element with no memory traffic -- the ceiling of the
    arrival arithmetic as compiled."""
    import torch

    import paper_2302_05176_amd as gm
    lanes = 1 << 21
    out = torch.empty(lanes, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    ms, _ = timed_steps(lambda: gm.rate_probe("arrivals", lanes, k, seed, out=out), 3, 1, stream)
    return lanes * k / (ms / 1e3)


def kernel_roofline(name, ms, units=None, slots=None, unit_name=None, hbm_bytes=None,
                    bound="alu", ceiling=None, traffic=None):
    """Roofline entry of one kernel from its average launch duration (ms):
    ALU-bound entries count algorithmic units x issue slots against the VALU
    peak; HBM-bound ones algorithmic bytes against 8 TB/s."""
    sec = ms / 1e3
    e = {"kernel": name, "kernel_ms": ms, "bound": bound}
    if bound == "alu":
        ach = units * slots / sec
        e.update({"achieved": ach / 1e12, "peak": PEAK_VALU_OPS / 1e12, "unit": "TOP/s",
                  "op": "f64-rate VALU lane-cycle (algorithmic units x slots per unit)",
                  "frac": ach / PEAK_VALU_OPS, "algorithmic_units": units, "unit_name": unit_name,
                  "slots_per_unit": slots})
        if ceiling:
            e["arrivals_per_s"] = units / sec
            e["probe_ceiling_arrivals_per_s"] = ceiling
            e["frac_of_probe"] = units / sec / ceiling
    else:
        e.update({"achieved": hbm_bytes / sec / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                  "frac": hbm_bytes / sec / HBM_PEAK})
    if hbm_bytes is not None:
        e["algorithmic_bytes"] = hbm_bytes
        e["hbm_algorithmic_frac"] = hbm_bytes / sec / HBM_PEAK
    e["traffic"] = traffic
    return e


def per_kernel_ms(timing):
    """{name: average ms per launch} from gm.get_timing()."""
    return {n: t / c for n, (t, c) in timing.items() if c}


# Sources that build the measured sketch kernels or set their launch
# parameters: a change to their code (comments and spacing aside) makes
# committed counters stale.
DIGEST_SOURCES = ["paper_2302_05176_amd/csrc/gm_fastgm.hip", "paper_2302_05176_amd/csrc/gm_plain.hip",
                  "paper_2302_05176_amd/csrc/gm_api.hip", "paper_2302_05176_amd/csrc/gm_common.h",
                  "paper_2302_05176_amd/csrc/gm_draw.h", "include/gm.h"]


def _code_only(text: str) -> str:
    text = re.sub(r"//[^\n]*", "", text)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.sub(r"\s+", " ", text).strip()


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in DIGEST_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(rel.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.all_workloads.txt")


def committed_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    from the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("source_sha256") != source_digest():
        return None
    return ent.get("bytes_per_launch")


def _counter_rows(d):
    import csv
    rows = []
    for dirpath, _, files in os.walk(d):
        for fn in files:
            if fn.endswith("counter_collection.csv"):
                with open(os.path.join(dirpath, fn)) as f:
                    rows += list(csv.DictReader(f))
    return rows


def summarize_pmc(args):
    """Turn two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, both with --copy-bytes) into HBM bytes per launch of every
    kernel, each counter scaled so that the calibration copy reads/writes
    exactly its size."""
    fetch_dir, write_dir = args.summarize_pmc
    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = {}
        for r in _counter_rows(d):
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"]
            per.setdefault(name, []).append(float(r["Counter_Value"]) * 1024.0)
        calib = [v for n, vs in per.items() if "elementwise" in n and "Mul" in n for v in vs]
        if not calib:
            raise SystemExit(f"no calibration copy dispatch found for {counter} in {d}")
        factor = args.copy_bytes / (sum(calib) / len(calib))
        for name, vs in per.items():
            short = name.split("(")[0].replace("void ", "").replace("gm::", "")
            e = out.setdefault(short, {"launches": len(vs)})
            e[counter.lower() + "_raw_bytes"] = sum(vs) / len(vs)
            e[counter.lower() + "_factor"] = factor
            e[counter.lower() + "_bytes"] = sum(vs) / len(vs) * factor
    for e in out.values():
        e["bytes_per_launch"] = e.get("fetch_size_bytes", 0.0) + e.get("write_size_bytes", 0.0)
        e["source_sha256"] = source_digest()
    workload = traffic_key(args)
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    rec[workload] = {n: e for n, e in out.items() if "elementwise" not in n and "__amd" not in n}
    wl = "" if args.workload == "batch" else f" --workload {args.workload}"
    extra = {"batch": " --steps 3 --warmup 1 --no-cpu-baseline --no-extras",
             "stream": " --steps 2 --warmup 1",
             "uneven": " --steps 2 --warmup 1 --no-autotune"}.get(args.workload, " --steps 2 --warmup 1")
    kk = f" --k {args.k}" if args.workload == "batch" else ""
    fdir, wdir = (os.path.relpath(os.path.abspath(d), ROOT) for d in args.summarize_pmc)
    rec.setdefault("_commands", {})
    if isinstance(rec["_commands"], list):
        rec["_commands"] = {}
    rec["_commands"][workload] = [
        f"cd /tmp && timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <repo>/{fdir} -o run -- "
        f"python3 <repo>/bench.py{wl}{kk if args.k != 256 else ''}{extra} --copy-bytes 1073741824",
        f"cd /tmp && timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE --output-format csv -d <repo>/{wdir} -o run -- "
        f"python3 <repo>/bench.py{wl}{kk if args.k != 256 else ''}{extra} --copy-bytes 1073741824",
        f"python bench.py{wl} --summarize-pmc {fdir} {wdir} --copy-bytes 1073741824{kk}",
        "FETCH_SIZE and WRITE_SIZE are KiB per dispatch; each is scaled by copy_bytes / (what it reads for the "
        "calibration elementwise kernel that reads and writes copy_bytes)"]
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(rec[workload], indent=1))


def traffic_key(args) -> str:
    """Key of a workload's entry in the committed traffic record."""
    if args.workload == "batch":
        return f"batch_k{args.k}_{args.form}"
    return args.workload


def calibration_copy(args):
    """Counter calibration: one elementwise kernel that reads and writes
    copy_bytes each (FETCH_SIZE and WRITE_SIZE are scaled by it)."""
    if not args.copy_bytes:
        return
    import torch
    a = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    del a, b


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["batch", "single", "stream", "stream_update", "uneven",
                                           "serve", "rates", "lsh"],
                    default="batch")
    ap.add_argument("--form", choices=["fastgm", "plain"], default="fastgm")
    ap.add_argument("--k", type=int, default=256)
    ap.add_argument("--nvec", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-autotune", action="store_true",
                    help="uneven workload: default schedule options instead of gm_autotune's")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one device copy of this many bytes (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write HBM bytes per launch from two rocprofv3 --pmc output folders")
    return ap.parse_args()


def timed_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall * 1e3 / steps, start.elapsed_time(end) / steps


def cpu_baseline(idx, w, off, k, seed, seconds, form):
    import oracle
    # every core of the affinity mask, but no more than OMP_NUM_THREADS when
    # the environment sets it (a host shared by several GPUs gives each GPU's
    # jobs a share of its cores that way)
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    ncores = affinity
    if os.environ.get("OMP_NUM_THREADS", "").isdigit() and int(os.environ["OMP_NUM_THREADS"]) > 0:
        ncores = min(ncores, int(os.environ["OMP_NUM_THREADS"]))
    ncores = max(1, ncores)
    oracle.set_threads(ncores)
    nvec = len(off) - 1
    f = oracle.FORM_STREAM if form == "fastgm" else oracle.FORM_PLAIN
    sub = off if form == "fastgm" else off[: min(nvec, 200) + 1]
    nv = len(sub) - 1
    done, t0 = 0, time.perf_counter()
    while True:
        oracle.sketch(idx, w, sub, k, seed + done, form=f)
        done += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    what = ("Algorithm 2 (Stream-FastGM)" if form == "fastgm" else "plain O(k n+)")
    return {"value": done * nv * k / dt, "unit": "registers/s", "cores": ncores,
            "affinity_cores": affinity, "kind": "oracle",
            "sample": f"{what} over the first {nv} vectors of the batch, {done} pass(es) with "
                      f"different seeds, {dt:.1f} s wall on {ncores} threads"}


def bench_batch(args):
    import numpy as np
    import torch

    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import workloads as W

    dev = torch.device("cuda:0")
    idx, w, off = W.batch(nvec=args.nvec, seed=1002)
    nnz = int(off[-1])
    nplus = np.diff(off)
    k = args.k
    ti, tw, to = (torch.from_numpy(a).to(dev) for a in (idx, w, off))
    out_i = torch.empty((args.nvec, k), dtype=torch.int32, device=dev)
    out_v = torch.empty((args.nvec, k), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    gm.reset_options()
    calibration_copy(args)
    step = lambda kk=k, form=args.form, oi=out_i, ov=out_v: gm.sketch(
        ti, tw, to, kk, args.seed, form=form, out_idx=oi, out_val=ov)
    # Timed region: HIP events around the sketch kernels only (timing level
    # 2), so that the step time carries two events per launch of the
    # dominant kernel and none around the planning passes.
    gm.set_option("timing", 2)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gm.reset_timing()
    ms_step, ev_ms = timed_steps(step, args.steps, 0, stream)
    kt = gm.get_timing()
    # per-kernel breakdown of a step (every launch timed; not the timed region)
    gm.set_option("timing", 1)
    gm.reset_timing()
    for _ in range(3):
        step()
    breakdown = {n: t / c for n, (t, c) in gm.get_timing().items() if c}
    gm.set_option("timing", 0)
    regs = args.nvec * k
    value = regs / (ms_step / 1e3)
    if args.form == "fastgm":
        key = next(n for n in kt if n.startswith("fastgm_class_kernel")
                   and n.endswith(f"[class {k_class(k)}]"))
        kern = key.split(" [")[0]
        small = nplus <= SMALL_LIMIT
        units = float(small.sum() * k * harmonic(k) + nplus[small].sum())
        slots = ARRIVAL_SLOTS
        unit_name = "arrivals (k H_k + n+ per vector, vectors of the kernel's class)"
        vec_bytes = 8.0 * nplus[small].sum() + 8.0 * (small.sum() + 1) + 12.0 * small.sum() * k
    else:
        kern = "plain_kernel"
        units = float(k) * nnz
        slots = PLAIN_KEY_SLOTS
        unit_name = "keys (k n+)"
        vec_bytes = 8.0 * nnz + 8.0 * (args.nvec + 1) + 12.0 * regs
    tot_ms, launches = kt.get(key if args.form == "fastgm" else kern, (0.0, 0))
    kern_ms = tot_ms / launches if launches else ev_ms
    traffic = committed_traffic(kern, f"batch_k{k}_{args.form}")
    ceiling = rate_ceiling(k, args.seed) if args.form == "fastgm" else None
    roofline = kernel_roofline(kern, kern_ms, units, slots, unit_name, vec_bytes, "alu", ceiling,
                               traffic)
    roofline["kernels_ms_per_step"] = breakdown
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(idx, w, off, k, args.seed, args.cpu_seconds, args.form)
    extras = {}
    if not args.no_extras and args.form == "fastgm":
        # same batch at k = 1024 and the plain form, a few steps each
        o2i = torch.empty((args.nvec, 1024), dtype=torch.int32, device=dev)
        o2v = torch.empty((args.nvec, 1024), dtype=torch.float64, device=dev)
        # (the CPU leg idles the GPU: warm it up again first)
        f1024, _ = timed_steps(lambda: step(1024, "fastgm", o2i, o2v), 10, 5, stream)
        p256, _ = timed_steps(lambda: step(k, "plain", out_i, out_v), 5, 1, stream)
        p1024, _ = timed_steps(lambda: step(1024, "plain", o2i, o2v), 3, 1, stream)
        extras = {"fastgm_k1024_ms": f1024, "fastgm_k1024_registers_per_s": args.nvec * 1024 / (f1024 / 1e3),
                  "plain_k256_ms": p256, "plain_k1024_ms": p1024,
                  f"speedup_vs_plain_k{k}": p256 / ms_step, "speedup_vs_plain_k1024": p1024 / f1024}
    line = {
        "metric": "Gumbel-Max registers/sec (FastGM form, k=256 document batch)" if k == 256
        else f"Gumbel-Max registers/sec (k={k} document batch)",
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
        "config": {"workload": f"document batch: {args.nvec} sparse vectors, n+ ~ lognormal(ln 500, 1) "
                               f"clipped to [10, 50000] (nnz={nnz}), indices in [0, 2^20), Exp(1) fp32 "
                               f"weights, k={k}, {args.form} form",
                   "form": args.form, "k": k, "nvec": args.nvec, "nnz": nnz,
                   "mean_nplus": float(nplus.mean())},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


def bench_single(args):
    import numpy as np
    import torch

    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import workloads as W
    dev = torch.device("cuda:0")
    idx, w, off = W.single(nplus=1000)
    ti, tw, to = (torch.from_numpy(a).to(dev) for a in (idx, w, off))
    stream = torch.cuda.current_stream()
    res = {}
    for form in ("fastgm", "plain"):
        ms, ev = timed_steps(lambda: gm.sketch(ti, tw, to, 128, args.seed, form=form),
                             args.steps, args.warmup, stream)
        res[form] = {"ms_per_sketch": ms, "event_ms": ev}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.set_threads(1)
        for form, f in (("fastgm", oracle.FORM_STREAM), ("plain", oracle.FORM_PLAIN)):
            t0 = time.perf_counter()
            n = 0
            while time.perf_counter() - t0 < 1.0:
                oracle.sketch(idx, w, off, 128, args.seed + n, form=f)
                n += 1
            res[form]["cpu_oracle_ms_1thread"] = (time.perf_counter() - t0) * 1e3 / n
    print(json.dumps({"workload": "single vector n+=1000, Uniform(0,1] weights, k=128",
                      "results": res}), flush=True)


def kernel_traffic(name, workload):
    """Committed HBM bytes per launch of the kernel a timing entry names."""
    return committed_traffic(name.split(" [")[0], workload)


def stream_kernel_rooflines(breakdown, n, k):
    """Roofline entries of the kernels of one stream-vector sketch (n entries,
    one vector of more than 32768 entries): the weight sum (4 bytes per
    entry), the probe (index and weight, 8 bytes per entry: with the
    single-precision rejection it is meant to run at the HBM line) and the
    candidate walk (k H_k arrivals beyond the first ones)."""
    ent = {}
    for name, ms in breakdown.items():
        tr = kernel_traffic(name, "stream")
        if name.startswith("big_sum_kernel"):
            ent[name] = kernel_roofline(name, ms, hbm_bytes=4.0 * n, bound="hbm", traffic=tr)
        elif name.startswith("big_probe_kernel"):
            ent[name] = kernel_roofline(name, ms, hbm_bytes=8.0 * n, bound="hbm", traffic=tr)
        elif name.startswith("fastgm_big_kernel"):
            ent[name] = kernel_roofline(name, ms, k * harmonic(k), ARRIVAL_SLOTS,
                                        "arrivals (k H_k beyond the first arrivals)",
                                        hbm_bytes=12.0 * k, bound="alu", traffic=tr)
            ent[name]["note"] = ("one vector's candidate walk: a few workgroups, each a chain of "
                                 "dependent batches, so its time is latency, far below the VALU line")
    return ent


def bench_stream(args):
    """One vector of 10^7 entries, k = 1024 and 4096.  The headline of the
    line is k = 1024; each k reports its step time (no events inside the
    timed loop), the per-kernel roofline entries (HIP events around every
    launch, on the call's stream, over a second pass of as many steps), the
    cardinality estimator over 100 seeds, and the plain form's time for the
    FastGM/plain ratio."""
    import numpy as np
    import torch

    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import workloads as W
    dev = torch.device("cuda:0")
    idx, w, off = W.stream(nplus=10_000_000)
    n = int(off[-1])
    ti, tw, to = (torch.from_numpy(a).to(dev) for a in (idx, w, off))
    stream = torch.cuda.current_stream()
    S = float(w.astype("float64").sum())
    calibration_copy(args)
    out = {}
    for k in (1024, 4096):
        step = lambda kk=k: gm.sketch(ti, tw, to, kk, args.seed)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ms, _ = timed_steps(step, args.steps, 0, stream)
        # the breakdown in a pass of its own: the events around every launch
        # cost a few microseconds each, a noticeable share of a 0.15 ms step
        gm.set_option("timing", 1)
        gm.reset_timing()
        timed_steps(step, args.steps, 0, stream)
        breakdown = per_kernel_ms(gm.get_timing())
        gm.set_option("timing", 0)
        kern = stream_kernel_rooflines(breakdown, n, k)
        dom = max(kern.values(), key=lambda e: e["kernel_ms"])
        ests = []
        for seed in range(1, 101):
            _, y = gm.sketch(ti, tw, to, k, seed)
            ests.append(float(gm.wcard_est(y).item()))
        r = np.array(ests) / S
        out[f"k{k}"] = {"ms_per_sketch": ms, "registers_per_s": k / (ms / 1e3),
                        "entries_per_s": n / (ms / 1e3), "roofline": dom, "kernels": kern,
                        "kernels_ms_per_step": breakdown,
                        "wcard_mean_ratio": float(r.mean()),
                        "wcard_rel_var_x_(k-2)": float(r.var(ddof=1) * (k - 2))}
    pms, _ = timed_steps(lambda: gm.sketch(ti, tw, to, 1024, args.seed, form="plain"), 3, 1, stream)
    out["plain_k1024_ms"] = pms
    out["plain_k1024_roofline"] = kernel_roofline("plain_kernel", pms, 1024.0 * n, PLAIN_KEY_SLOTS,
                                                  "keys (k n+)", 8.0 * n + 16 + 12 * 1024, "alu")
    out["speedup_vs_plain_k1024"] = pms / out["k1024"]["ms_per_sketch"]
    head = out["k1024"]
    print(json.dumps({"metric": "Gumbel-Max registers/sec (FastGM form, one 10^7-entry vector, k=1024)",
                      "value": head["registers_per_s"], "unit": "registers/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_sketch"],
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                      "data": "synthetic",
                      "config": {"workload": "one stream vector n+=1e7, indices distinct in [0, 2^31-1), "
                                             "half Uniform(0,1], half 1+Pareto(1.5) fp32 weights, "
                                             "k=1024 (k=4096 in results)"},
                      "roofline": head["roofline"], "results": out}), flush=True)


def bench_stream_update(args):
    """Stream-FastGM through the update API: the 10^7-entry stream arrives in
    ten chunks of 10^6 entries (in stream order), each merged into one stored
    sketch; later chunks stop at the stored sketch's y* and get cheaper."""
    import numpy as np
    import torch

    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import workloads as W
    dev = torch.device("cuda:0")
    idx, w, off = W.stream(nplus=10_000_000)
    n = int(off[-1])
    out = {}
    for k in (1024, 4096):
        chunks = []
        for c in range(10):
            a, b = c * n // 10, (c + 1) * n // 10
            chunks.append((torch.from_numpy(idx[a:b]).to(dev), torch.from_numpy(w[a:b]).to(dev),
                           torch.tensor([0, b - a], dtype=torch.int64, device=dev)))
        ms_chunks = []
        for rep in range(2):          # the first pass warms up
            si, sv = gm.empty_sketches(1, k, dev)
            ms_chunks = []
            for ti, tw, to in chunks:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                gm.sketch_update(ti, tw, to, k, args.seed, si, sv)
                e1.record()
                torch.cuda.synchronize()
                ms_chunks.append(e0.elapsed_time(e1))
        ti, tw, to = (torch.from_numpy(a).to(dev) for a in (idx, w, off))
        whole_i, whole_v = gm.sketch(ti, tw, to, k, args.seed)
        same = bool(torch.equal(whole_i, si) and torch.equal(whole_v, sv))
        out[f"k{k}"] = {"chunk_ms": [round(x, 4) for x in ms_chunks], "total_ms": sum(ms_chunks),
                        "entries_per_s": n / (sum(ms_chunks) / 1e3), "equals_whole_sketch": same}
    print(json.dumps({"workload": "stream update: one 10^7-entry vector (half Uniform(0,1], half "
                                  "1+Pareto(1.5)) in ten 10^6-entry chunks", "results": out}),
          flush=True)


def uneven_kernel_rooflines(breakdown, n, kk):
    """Roofline entries of the launches of a mixed-k batch.  A class kernel
    drains the vectors of at most 32768 entries of one k range: k H_k + n+
    arrivals per vector; bytes 8 n+ + 8 + 12 k + 12 (k and output offset).
    Big vectors (more than 32768 entries): the sum pass reads 4 bytes and the
    probe 8 bytes per entry; their walk kernel draws k H_k arrivals per
    vector beyond the first ones."""
    import numpy as np
    kcls = np.where(kk <= 256, 0, np.where(kk <= 1024, 1, np.where(kk <= 2048, 2, 3)))
    hk = {int(k): harmonic(int(k)) for k in np.unique(kk)}
    hv = np.array([hk[int(k)] for k in kk])
    small = n <= SMALL_LIMIT
    ent = {}
    for name, ms in breakdown.items():
        tr = kernel_traffic(name, "uneven")
        if name.startswith("big_sum_kernel"):
            ent[name] = kernel_roofline(name, ms, hbm_bytes=4.0 * n[~small].sum(), bound="hbm",
                                        traffic=tr)
        elif name.startswith("big_probe_kernel"):
            ent[name] = kernel_roofline(name, ms, hbm_bytes=8.0 * n[~small].sum(), bound="hbm",
                                        traffic=tr)
        elif "[class " in name:
            c = int(name.split("class ")[1].rstrip("]"))
            sel = (kcls == c % 4) & (small if c < 4 else ~small)
            if not sel.any():
                continue
            if c < 4:
                units = float((kk[sel] * hv[sel]).sum() + n[sel].sum())
                uname = "arrivals (k H_k + n+ per vector of the class)"
                byt = 8.0 * n[sel].sum() + 8.0 * (sel.sum() + 1) + 12.0 * kk[sel].sum() + 12.0 * sel.sum()
            else:
                units = float((kk[sel] * hv[sel]).sum())
                uname = "arrivals (k H_k per big vector, beyond the first arrivals)"
                byt = 12.0 * kk[sel].sum() + 12.0 * sel.sum()
            ent[name] = kernel_roofline(name, ms, units, ARRIVAL_SLOTS, uname, byt, "alu", traffic=tr)
    return ent


def bench_uneven(args):
    import numpy as np
    import torch

    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import workloads as W
    dev = torch.device("cuda:0")
    nvec = args.nvec if args.nvec != 10000 else 100_000
    t0 = time.perf_counter()
    idx, w, off, kk = W.uneven(nvec=nvec)
    gen_s = time.perf_counter() - t0
    outoff = np.zeros(nvec + 1, np.int64)
    np.cumsum(kk, out=outoff[1:])
    t = lambda a: torch.from_numpy(a).to(dev)
    ti, tw, to, tk, too = t(idx), t(w), t(off), t(kk), t(outoff)
    total = int(outoff[-1])
    oi = torch.empty(total, dtype=torch.int32, device=dev)
    ov = torch.empty(total, dtype=torch.float64, device=dev)
    calibration_copy(args)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        gm.reserve(nvec, stream=s)
        if args.no_autotune:
            gm.reset_options()
            tuned = None
        else:
            tuned = gm.autotune(ti, tw, to, 4096, args.seed, k_per_vec=tk, out_offsets=too,
                                out_idx=oi, out_val=ov, reps=1, stream=s)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gm.sketch_batched(ti, tw, to, tk, too, 4096, args.seed, out_idx=oi, out_val=ov,
                          stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    ms, _ = timed_steps(lambda: g.replay(), max(2, args.steps // 4), 1, torch.cuda.current_stream())
    # Per-kernel durations: the captured graph holds no timing events, so the
    # same call (same options) runs eagerly with HIP events around every
    # launch on its stream.
    gm.set_option("timing", 1)
    gm.reset_timing()
    with torch.cuda.stream(s):
        for _ in range(2):
            gm.sketch_batched(ti, tw, to, tk, too, 4096, args.seed, out_idx=oi, out_val=ov, stream=s)
    s.synchronize()
    breakdown = per_kernel_ms(gm.get_timing())
    gm.set_option("timing", 0)
    gm.reset_options()
    n = np.diff(off)
    kern = uneven_kernel_rooflines(breakdown, n, kk)
    dom = max((e for e in kern.values() if e["bound"] == "alu"), key=lambda e: e["kernel_ms"])
    dom_k = {0: 256, 1: 1024, 2: 2048, 3: 4096}[int(dom["kernel"].split("class ")[1].rstrip("]")) % 4]
    dom["probe_ceiling_arrivals_per_s"] = rate_ceiling(min(dom_k, 4096), args.seed)
    dom["arrivals_per_s"] = dom["algorithmic_units"] / (dom["kernel_ms"] / 1e3)
    dom["frac_of_probe"] = dom["arrivals_per_s"] / dom["probe_ceiling_arrivals_per_s"]
    print(json.dumps({"metric": "Gumbel-Max registers/sec (FastGM form, uneven mixed-k batch)",
                      "value": total / (ms / 1e3), "unit": "registers/s", "n_gpus": 1,
                      "steps": max(2, args.steps // 4), "warmup": 1, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"uneven batch: {nvec} vectors, Zipf(1.2) n+ on [10, 1e5] "
                                             f"(nnz={int(off[-1])}), k from {{64,256,1024,4096}}, "
                                             f"lognormal(0,2) weights, one captured graph"},
                      "vectors_per_s": nvec / (ms / 1e3), "entries_per_s": int(off[-1]) / (ms / 1e3),
                      "roofline": dom, "kernels": kern, "kernels_ms_per_call": breakdown,
                      "autotuned": tuned, "graph": True, "input_gen_s": gen_s}), flush=True)


def bench_rates(args):
    """Issue-rate ceiling of the per-arrival and per-key arithmetic: every lane
    draws a long run of arrivals (or plain keys) of its own element with no
    memory traffic; compared with the slot counts the roofline uses."""
    import torch

    import paper_2302_05176_amd as gm
    dev = torch.device("cuda:0")
    lanes = 1 << 21
    out = torch.empty(lanes, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    res = {}
    for what, slots in (("arrivals", ARRIVAL_SLOTS), ("keys", PLAIN_KEY_SLOTS)):
        for steps in (256, 1024):
            ms, _ = timed_steps(lambda: gm.rate_probe(what, lanes, steps, args.seed, out=out),
                                max(2, args.steps // 4), 1, stream)
            rate = lanes * steps / (ms / 1e3)
            res[f"{what}_k{steps}"] = {"per_s": rate, "lane_cycles_each": PEAK_VALU_OPS / rate,
                                      "slots_each": slots, "frac_of_peak": rate * slots / PEAK_VALU_OPS}
    print(json.dumps({"workload": f"issue-rate probe: {lanes} lanes, one element each, no memory traffic",
                      "peak_slots_per_s": PEAK_VALU_OPS, "results": res}), flush=True)


def bench_serve(args):
    import numpy as np
    import torch

    from paper_2302_05176_amd import serve
    nstore = 1_000_000
    k = 512
    t0 = time.perf_counter()
    store = serve.build_store(nstore, k)
    build_s = time.perf_counter() - t0
    # 8 slots, no batching window: a free slot takes what is pending at once
    cfg = dict(slots=8, max_batch_requests=256, max_wait_us=0.0, device_budget_bytes=4 << 30)
    reqs, hi, hw = serve.make_trace(20_000, rate=20_000.0, nstore=nstore)
    res = serve.run(reqs, hi, hw, store, k, seed=args.seed, **cfg)
    summ = serve.summarize(reqs, res)
    # toward saturation: 2x, 5x and 10x the arrival rate
    sweep = []
    for mult in (2, 5, 10):
        rq, rhi, rhw = serve.make_trace(40_000, rate=20_000.0 * mult, nstore=nstore)
        r2 = serve.run(rq, rhi, rhw, store, k, seed=args.seed, **cfg)
        sweep.append({"rate_req_s": 20_000.0 * mult, **serve.summarize(rq, r2),
                      "batches": r2["stats"]["batches"]})
    print(json.dumps({"workload": "serving: Poisson 20,000 req/s, 1 sketch (k=512, n+ ~ "
                                  "lognormal(ln 2000, 1.5) clipped to [10, 1e6]) per 4 Jaccard "
                                  "queries on 1e6 stored sketches",
                      "requests": len(reqs), "summary": summ, "stats": res["stats"],
                      "config": cfg, "saturation": sweep,
                      "store_build_s": build_s}), flush=True)


def bench_lsh(args):
    """LSH index over 1e6 stored sketches (k = 512, 64 bands x 6 registers):
    build time, query throughput, and recall of each perturbed query's source
    row against the banding curve 1 - (1 - J^6)^64."""
    import numpy as np
    import torch

    import paper_2302_05176_amd as gm
    dev = torch.device("cuda:0")
    nstore, k, n, bands, rows = 1_000_000, 512, 32, 64, 6
    nq_near, nq_far = 10_000, 10_000
    rng = np.random.Generator(np.random.PCG64(1013))
    # stored vectors: n distinct indices in [0, 2^24) (duplicates within a row
    # are rare and harmless), Exp(1) weights
    si = rng.integers(0, 1 << 24, size=(nstore, n), dtype=np.int64).astype(np.int32)
    sw = (rng.exponential(1.0, size=(nstore, n)) + 1e-6).astype(np.float32)
    store = torch.empty((nstore, k), dtype=torch.int32, device=dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(dev)
    for s0 in range(0, nstore, 250_000):
        m = min(250_000, nstore - s0)
        gm.sketch(t(si[s0:s0 + m]), t(sw[s0:s0 + m]), t(np.arange(m + 1, dtype=np.int64) * n), k,
                  args.seed, out_idx=store[s0:s0 + m])
    # near queries: a stored row with 4 of its 32 entries replaced; far: fresh
    src = rng.integers(0, nstore, size=nq_near)
    qi = np.concatenate([si[src], rng.integers(0, 1 << 24, size=(nq_far, n)).astype(np.int32)])
    qw = np.concatenate([sw[src], (rng.exponential(1.0, size=(nq_far, n)) + 1e-6).astype(np.float32)])
    repl = rng.integers(0, n, size=(nq_near, 4))
    for c in range(4):
        qi[np.arange(nq_near), repl[:, c]] = rng.integers(1 << 24, 1 << 25, size=nq_near)
        qw[np.arange(nq_near), repl[:, c]] = (rng.exponential(1.0, size=nq_near) + 1e-6).astype(np.float32)
    nq = nq_near + nq_far
    queries = torch.empty((nq, k), dtype=torch.int32, device=dev)
    gm.sketch(t(qi), t(qw), t(np.arange(nq + 1, dtype=np.int64) * n), k, args.seed, out_idx=queries)
    torch.cuda.synchronize()
    # the probability-Jaccard of a near query with its source (same weights on
    # the kept entries, disjoint replacements): sum kept / (sum of both)
    kept = np.ones((nq_near, n), bool)
    kept[np.arange(nq_near)[:, None], repl] = False
    a = sw[src].astype(np.float64)
    b = qw[:nq_near].astype(np.float64)
    shared = (a * kept).sum(1)
    jp = shared / (a.sum(1) + b.sum(1) - shared)
    expect = 1.0 - (1.0 - jp ** rows) ** bands
    t0 = time.perf_counter()
    ix = gm.LshIndex(store, bands, rows)
    build_ms = (time.perf_counter() - t0) * 1e3
    max_cand = 16
    ms, _ = timed_steps(lambda: ix.query(queries, max_cand), 5, 2, torch.cuda.current_stream())
    cand, count = ix.query(queries, max_cand)
    torch.cuda.synchronize()
    cand, count = cand.cpu().numpy(), count.cpu().numpy()
    found = np.array([src[q] in cand[q, :min(count[q], max_cand)] for q in range(nq_near)])
    # brute force for comparison: the Jaccard estimate of one pair per stored row
    ia = torch.randint(0, nstore, (nstore,), device=dev)
    ib = torch.randint(0, nstore, (nstore,), device=dev)
    jout = torch.empty(nstore, dtype=torch.float64, device=dev)
    scan_ms, _ = timed_steps(lambda: gm.jaccard_est_pairs(store, ia, ib, out=jout), 5, 2,
                             torch.cuda.current_stream())
    ix.close()
    print(json.dumps({
        "workload": "LSH index: 1e6 stored sketches (k=512, 32-entry vectors), 64 bands x 6 "
                    "registers; 1e4 queries = stored vectors with 4 of 32 entries replaced, "
                    "1e4 unrelated",
        "build_ms": build_ms, "queries": nq, "query_ms": ms, "queries_per_s": nq / (ms / 1e3),
        "near_recall": float(found.mean()), "near_recall_expected": float(expect.mean()),
        "near_mean_candidates": float(count[:nq_near].mean()),
        "far_mean_candidates": float(count[nq_near:].mean()),
        "overflowed": int((count < 0).sum()),
        "brute_force_scan_ms_per_query": scan_ms,
        "speedup_vs_scan": scan_ms / (ms / nq)}), flush=True)


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}); vectors are "
              "independent, so N GPUs would each sketch their own share of the batch.",
              file=sys.stderr)
        sys.exit(2)
    from paper_2302_05176_amd import build as gmbuild
    if not os.path.exists(gmbuild.LIB):
        gmbuild.build(force=True)
    import torch
    torch.cuda.set_device(0)
    {"batch": bench_batch, "single": bench_single, "stream": bench_stream,
     "uneven": bench_uneven, "serve": bench_serve, "rates": bench_rates,
     "stream_update": bench_stream_update, "lsh": bench_lsh}[args.workload](args)


if __name__ == "__main__":
    main()
