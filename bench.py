#!/usr/bin/env python3
"""Benchmark of the sketch A_hat = S A on one MI355X.

A step is one full sk_sketch call (device validation, inspector, S tiles +
sparse accumulation, split reduction) on the plain-at-scale workload: A is
CSC FP32, m = 2e6, n = 2000, 10 distinct uniform columns per row (nnz = 2e7),
values U(-1,1); S uniform(-1,1) from Philox4x32-10 (seed 21); d = 4000.
Inputs are resident in HBM before the timed region.

Prints one JSON line: throughput in nnz*d/s, the ALU roofline of the
dominant kernel (timed alone with HIP events on the stream it runs on), and
the CPU oracle timed on a bounded row sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = full-rate 32-bit VALU lane-ops/s
VALU_PEAK = 256 * 64 * 2.4e9
# VALU issue slots (full-rate equivalents) per generator call / per S entry:
# Philox4x32-10 is 10 rounds of two 32x32->64 multiplies (v_mad_u64_u32, which
# issues at full rate on gfx950), four xors and the key bumps: about 60 slots
PHILOX_SLOTS = 60
# transform slots per S entry: uniform = shift, convert, multiply-add; Gaussian
# = half a Box-Muller pair (logarithm, square root, sine/cosine polynomials)
TRANSFORM_SLOTS = {"rademacher": 0.0, "uniform": 4.0, "gaussian": 30.0}
FMA_SLOTS = 1           # one v_fma_f32 per multiply-add (packed FP32 disabled)
# HBM traffic of the sketch kernel on the default workload, from hardware
# counters, valid while the kernel sources are the ones it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sketch_plain_scale_traffic.txt")
KERNEL_SOURCES = ["paper_2310_15419_amd/csrc/sk_sketch.hpp",
                  "paper_2310_15419_amd/csrc/sk_rng.hpp"]


def valu_work(dist: str, calls: float, entries: float, fmas: float) -> float:
    return calls * PHILOX_SLOTS + entries * TRANSFORM_SLOTS[dist] + fmas * FMA_SLOTS


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(workload: str):
    """HBM bytes per launch of the sketch kernel from the committed counter
    summary, or None when it does not apply (other workload, changed kernel)."""
    if workload != "plain_scale" or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sources_sha():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_workload(name: str):
    from paper_2310_15419_amd import inputs
    if name == "plain_scale":
        A = inputs.workload_plain_scale()
        return A, 4000, "uniform", 21, (
            "plain_scale: A CSC FP32 m=2000000 n=2000, 10 uniform columns per row "
            "(nnz=2e7), values U(-1,1); S uniform(-1,1) Philox4x32-10 seed 21; d=4000")
    if name == "plain_small":
        A = inputs.workload_plain_small()
        return A, 400, "rademacher", 1, (
            "plain_small: A CSC FP64 m=100000 n=200, 2e5 uniform positions, N(0,1); "
            "S +-1 seed 1; d=400")
    if name == "skewed":
        A, r0 = inputs.workload_skewed()
        return A, 3000, "gaussian", 31, (
            "skewed: A CSC FP32 m=4000000 n=1000, power-law column nnz (exponent 2, max 5% of "
            f"m) plus a dense 2000-row block at row {r0}; S Gaussian (Box-Muller) seed 31; d=3000")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(A, d, dist, seed, target_s: float):
    """The oracle, untouched, on the first rows of A (all columns)."""
    import oracle
    oracle.build()
    from paper_2310_15419_amd import inputs
    threads = len(os.sched_getaffinity(0))

    def sample(rows):
        keep = A.rowidx < rows
        cols = np.repeat(np.arange(A.n), np.diff(A.colptr))[keep]
        return inputs.from_coo(rows, A.n, A.rowidx[keep], cols, A.vals[keep].astype(np.float64))

    rows = max(1000, min(A.m, 2000))
    S = sample(rows)
    t0 = time.perf_counter()
    oracle.sketch(S.m, S.n, S.colptr, S.rowidx, S.vals, d, dist, seed, threads=threads)
    dt = time.perf_counter() - t0
    rows = int(min(A.m, max(rows, rows * target_s / max(dt, 1e-3))))
    S = sample(rows)
    t0 = time.perf_counter()
    oracle.sketch(S.m, S.n, S.colptr, S.rowidx, S.vals, d, dist, seed, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": S.nnz * d / dt, "unit": "nnz*d/s", "cores": threads, "kind": "oracle",
            "sample": f"first {rows} rows of A (nnz={S.nnz}), full d={d}, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_scale")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--rows-per-block", type=int, default=0)
    ap.add_argument("--splits", type=int, default=0)
    ap.add_argument("--dense-min-pct", type=int, default=0)
    ap.add_argument("--col-split", type=int, default=0, help="0 auto, 1 off, 2 on")
    ap.add_argument("--row-pad", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="launch only a plain 1 GiB device copy (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); no multi-GPU figure is "
              "measured", file=sys.stderr)
        raise SystemExit(2)

    import torch
    from paper_2310_15419_amd import binding as B

    if args.copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": x.numel() * 4, "copies": 3}))
        return

    t_gen = time.perf_counter()
    A, d, dist, seed, desc = make_workload(args.workload)
    print(f"[bench] workload generated in {time.perf_counter() - t_gen:.1f} s "
          f"(m={A.m}, n={A.n}, nnz={A.nnz}, d={d})", file=sys.stderr, flush=True)
    dA = B.DeviceCsc.from_host(A, dtype=np.float32 if A.vals.dtype != np.float64 else None)
    tune = {"variant": args.variant, "rows_per_block": args.rows_per_block,
            "splits": args.splits, "dense_min_pct": args.dense_min_pct,
            "col_split": args.col_split, "row_pad": args.row_pad}
    ws = B.alloc_workspace(B.workspace_bytes(dA, d, dist, tune=tune))
    out = torch.empty((A.n, d), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        B.sketch_into(dA, d, dist, seed, out, ws, tune=tune)
    st = B.sketch_status(ws)
    if st["status"] != 0:
        raise SystemExit(f"sketch failed: {st}")
    R, nb = st["nonempty_rows"], st["row_blocks"]

    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        B.sketch_into(dA, d, dist, seed, out, ws, tune=tune)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1) / args.steps

    # the dominant kernel alone (S tiles + sparse accumulation), same stream,
    # same workspace
    ktune = dict(tune, phases=2)
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    k0.record(stream)
    for _ in range(args.steps):
        B.sketch_into(dA, d, dist, seed, out, ws, tune=ktune)
    k1.record(stream)
    torch.cuda.synchronize()
    kms = k0.elapsed_time(k1) / args.steps

    nnz = A.nnz
    rpc = 128 if dist == "rademacher" else 4
    calls = R * -(-d // rpc)
    entries = R * d
    work = valu_work(dist, calls, entries, nnz * d)
    achieved = work / (kms * 1e-3)
    value = nnz * d / (ms * 1e-3)

    res = {
        "metric": "sketched nnz·d per sec (% of roofline); batched vs plain at fixed error; "
                  "p99 latency",
        "value": value,
        "unit": "nnz*d/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "nnz": nnz, "d": d, "nonempty_rows": R, "row_blocks": nb},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "TOP/s (full-rate VALU lane-ops)", "frac": achieved / VALU_PEAK,
                     "traffic": counter_traffic(args.workload), "kernel": "k_sketch",
                     "kernel_ms": kms},
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(A, d, dist, seed, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
