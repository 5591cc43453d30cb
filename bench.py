#!/usr/bin/env python3
"""Benchmark of the sketch A_hat = S A on one MI355X.

Default (``python bench.py``): the plain-at-scale workload.  A step is one
full sk_sketch call (device validation, inspector, S tiles + sparse
accumulation, split reduction): A is CSC FP32, m = 2e6, n = 2000, 10 distinct
uniform columns per row (nnz = 2e7), values U(-1,1); S uniform(-1,1) from
Philox4x32-10 (seed 21); d = 4000.  Inputs are resident in HBM before the
timed region.  One JSON line carries:
  - throughput in nnz*d/s and the step time;
  - the ALU roofline of the sketch kernel, timed alone with HIP events on the
    stream it runs on, with the generator's cost per call and per S value
    measured in the same run by the generator-throughput probe;
  - the FMA-only bound (the kernel with the junk generator), the inspector
    and reduction times, and the distribution-cost ablation (junk generator,
    integer-scaled (-1,1), S stored in HBM);
  - element-wise parity of the timed output against the CPU oracle, and the
    oracle's own throughput on the host cores (cpu_baseline);
  - ``batched``: 64 items of the batched workload, plain FP32 launches
    against one batched launch (FP32, and +-1 S in BF16 / FP8 on the matrix
    cores), every item checked against the oracle;
  - ``serving``: a Poisson stream of sketch-and-precondition least-squares
    solves at 0.9x capacity, plain (one at a time) against continuous
    batching: p50/p99 latency and solves/s.
``--workload batched`` / ``serving`` / ``skewed`` / ``plain_small`` run the
other workloads on their own (the batched and serving ones at full size);
``table1`` / ``abnormal`` run the S-tile kernel and the Algorithm 3
loop-order kernel on stand-ins for the paper's SpMM matrices.
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
# the generator's cost per call as the cost model of the sketch counts it:
# 10 rounds of two 32x32 -> 64-bit multiply-adds and two three-input xors,
# one issue slot each
PHILOX_SLOTS_MODEL = 40
# HBM traffic of the sketch kernel on the default workload, from hardware
# counters, valid while the kernel sources are the ones it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sketch_plain_scale_traffic.txt")
KERNEL_SOURCES = ["paper_2310_15419_amd/csrc/sk_sketch.hpp",
                  "paper_2310_15419_amd/csrc/sk_rng.hpp"]


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def plan_string(plan: dict) -> str:
    return " ".join(f"{k}={plan[k]}" for k in ("variant", "splits", "tile_rows",
                                              "rows_per_block", "col_split", "balance"))


def counter_traffic(workload: str, plan: dict):
    """HBM bytes per launch of the sketch kernel from the committed counter
    summary, or None when it does not apply (other workload, changed kernel
    sources, or another plan)."""
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
    if vals.get("plan") != plan_string(plan):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_ms(fn, reps: int, stream, warm: bool = True) -> float:
    """Average time of fn() over reps calls, HIP events on `stream`."""
    import torch
    if warm:
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


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


# ---------------------------------------------------------------- generator
def generator_costs(B, dist: str, stream) -> dict:
    """Generator calls/s of the throughput probe, as full-rate VALU issue
    slots per call (Philox and the junk hash), and the transform's slots per
    S value (the probe with the distribution's transform against the raw
    words)."""
    import torch
    blocks, calls = 256 * 8, 512
    sink = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    n_calls = blocks * 256 * calls

    def slots(d, gen):
        ms = timed_ms(lambda: B.rng_throughput(d, gen, calls, blocks, 7, sink, stream), 5, stream)
        return VALU_PEAK * ms * 1e-3 / n_calls

    words = slots("rademacher", 0)
    rec = {"philox_slots_per_call": words, "junk_slots_per_call": slots("rademacher", 1),
           "probe": f"{blocks} x 256 threads x {calls} calls, counters (call, thread)"}
    if dist != "rademacher":
        full = slots(dist, 0)
        rec[f"{dist}_slots_per_call"] = full
        rec["transform_slots_per_value"] = max(0.0, (full - words) / 4.0)
    else:
        rec["transform_slots_per_value"] = 0.0
    return rec


# -------------------------------------------------------------- plain runs
def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, d, dist, seed, target_s: float, threads: int = 0):
    """The oracle, untouched, on the first rows of A (all columns).  Returns
    the baseline record, the oracle's A_hat and the sampled matrix."""
    import oracle
    oracle.build()
    from paper_2310_15419_amd import inputs
    threads = threads or len(os.sched_getaffinity(0))

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
    ref = oracle.sketch(S.m, S.n, S.colptr, S.rowidx, S.vals, d, dist, seed, threads=threads)
    dt = time.perf_counter() - t0
    rec = {"value": S.nnz * d / dt, "unit": "nnz*d/s", "cores": threads, "kind": "oracle",
           "cpu": cpu_model(),
           "sample": f"first {rows} rows of A (nnz={S.nnz}), full d={d}, {dt:.1f} s"}
    return rec, ref, S


def parity_record(got, ref, S, dist, what: str):
    """The oracle's error measures for a GPU result on the oracle's sample."""
    import oracle
    p = oracle.parity(got, ref, S.colptr, S.vals, dist)
    p.update({"compared": what, "elem_bound": oracle.ELEM_TOL, "norm_bound": 1e-5})
    p["pass"] = bool(p["nonfinite"] == 0 and p["normwise"] <= 1e-5 and
                     p["max_elem_scaled"] <= oracle.ELEM_TOL)
    return p


def ablation(B, dA, A, d, dist, seed, tune, stream, steps, entries) -> dict:
    """The sketch kernel with the junk generator (the FMA-only analogue), the
    integer-scaled (-1,1) S and S stored in HBM, on the same input and tiling
    (no dense path here).  h: generator time per S value (product minus
    junk), and the generator's share of the product kernel's time."""
    import torch
    base = {k: v for k, v in tune.items() if v}
    base["dense_min_pct"] = 101
    out = torch.empty((A.n, d), dtype=torch.float32, device="cuda")
    rec = {}
    try:
        ws = B.alloc_workspace(B.workspace_bytes(dA, d, dist, tune=base))
        modes = [("philox", 0), ("junk", 1)] + ([("scaled", 3)] if dist == "uniform" else [])
        for name, mode in modes:
            t = dict(base, rng_mode=mode)
            B.sketch_into(dA, d, dist, seed, out, ws, tune=t)  # inspector for this tuning
            t["phases"] = 2
            rec[f"{name}_kernel_ms"] = timed_ms(
                lambda: B.sketch_into(dA, d, dist, seed, out, ws, tune=t), steps, stream)
        if dist == "uniform":
            # S itself in HBM (d rounded up to 128 rows per column)
            lds = -(-d // 128) * 128
            S = torch.empty((A.m, lds), dtype=torch.float32, device="cuda")
            B.lib().sk_materialize_s(0, d, 0, A.m, 1, seed, S.data_ptr(), lds, B._stream(stream))
            t = dict(base)
            B.sketch_stored_into(dA, S, out, ws, tune=t)
            t["phases"] = 2
            rec["stored_kernel_ms"] = timed_ms(
                lambda: B.sketch_stored_into(dA, S, out, ws, tune=t), steps, stream)
            rec["stored_s_bytes"] = float(S.numel() * 4)
            del S
        del ws
    except (B.SketchError, torch.cuda.OutOfMemoryError) as e:
        rec["error"] = str(e)
        return rec
    gen_ms = rec["philox_kernel_ms"] - rec["junk_kernel_ms"]
    rec["h_ns_per_value"] = gen_ms * 1e6 / entries
    rec["generator_share"] = gen_ms / rec["philox_kernel_ms"]
    return rec


def bench_plain(args, B):
    import torch
    t_gen = time.perf_counter()
    A, d, dist, seed, desc = make_workload(args.workload)
    log(f"workload generated in {time.perf_counter() - t_gen:.1f} s "
        f"(m={A.m}, n={A.n}, nnz={A.nnz}, d={d})")
    dA = B.DeviceCsc.from_host(A, dtype=np.float32 if A.vals.dtype != np.float64 else None)
    tune = {"variant": args.variant, "rows_per_block": args.rows_per_block,
            "splits": args.splits, "dense_min_pct": args.dense_min_pct,
            "col_split": args.col_split, "row_pad": args.row_pad, "tile_rows": args.tile_rows,
            "balance": args.balance}
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
    wall0 = time.perf_counter()
    ms = timed_ms(lambda: B.sketch_into(dA, d, dist, seed, out, ws, tune=tune), args.steps,
                  stream, warm=False)
    wall = time.perf_counter() - wall0
    # the phases alone (same stream, same workspace): the sketch kernel, the
    # validation + inspector, the split reduction
    phase_ms = {}
    for name, mask in (("kernel", 2), ("inspector", 1), ("reduction", 4)):
        t = dict(tune, phases=mask)
        phase_ms[name] = timed_ms(lambda: B.sketch_into(dA, d, dist, seed, out, ws, tune=t),
                                  args.steps, stream, warm=False)
    B.sketch_into(dA, d, dist, seed, out, ws, tune=tune)  # the full result again
    kms = phase_ms["kernel"]

    nnz = A.nnz
    e = 128 if dist == "rademacher" else 4
    calls = R * -(-d // e)
    entries = R * d
    fmas = nnz * d
    gen = generator_costs(B, dist, stream)
    work = calls * gen["philox_slots_per_call"] + entries * gen["transform_slots_per_value"] + fmas
    work_model = calls * PHILOX_SLOTS_MODEL + entries * gen["transform_slots_per_value"] + fmas
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
        "config": {"workload": desc, "nnz": nnz, "d": d, "nonempty_rows": R, "row_blocks": nb,
                   "input_sha256": A.sha256()},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "TOP/s (full-rate VALU lane-ops)", "frac": achieved / VALU_PEAK,
                     "traffic": (counter_traffic(args.workload, B.autotune(dA, d, dist))
                                 if not any(tune.values()) else None),
                     "kernel": "k_sketch",
                     "kernel_ms": kms,
                     "work": {"generator_calls": calls, "s_values": entries, "fma": fmas,
                              "lane_ops": work},
                     "generator": gen,
                     "frac_at_40_slots_per_call": work_model / (kms * 1e-3) / VALU_PEAK,
                     "fma_only_bound_ms": fmas / VALU_PEAK * 1e3},
        "phases_ms": phase_ms,
        "wall_s_timed": wall,
    }
    if not args.no_ablation and args.workload in ("plain_scale", "skewed"):
        res["ablation"] = ablation(B, dA, A, d, dist, seed, tune, stream, args.steps, entries)
        if "junk_kernel_ms" in res["ablation"]:
            res["roofline"]["fma_only_kernel_ms"] = res["ablation"]["junk_kernel_ms"]
    del ws
    if not args.no_cpu_baseline:
        rec, ref, S = cpu_baseline(A, d, dist, seed, args.cpu_seconds)
        if S.m == A.m:
            got = out.t().cpu().numpy()  # the whole workload: the timed output itself
            what = "the timed output, every element"
        else:
            vdt = None if A.vals.dtype == np.float64 else np.float32  # as the timed input
            got = B.sketch(B.DeviceCsc.from_host(S, dtype=vdt), d, dist, seed).cpu().numpy()
            what = f"a GPU sketch of the oracle's sample ({S.m} rows), every element"
        res["parity"] = parity_record(got, ref, S, dist, what)
        del ref, got
        if args.workload == "plain_small":
            # one thread too, beside the paper's sequential tables
            one, _, _ = cpu_baseline(A, d, dist, seed, args.cpu_seconds, threads=1)
            rec["one_thread"] = one
        res["cpu_baseline"] = rec
    return res


# ----------------------------------------------------------------- batched
def bench_batched(B, count: int, steps: int, dense_min_pct: int = 0, workers: int = 0,
                  oracle_all: bool = True) -> dict:
    """The batched workload's first `count` items (m log-uniform in [1e4,
    5e5], n in [50, 500], d in [2n, 4n], density U(0.5%, 5%), values BF16,
    S +-1): plain per-item launches against one batched launch, with S in FP32
    on the sparse kernel and in BF16 / FP8 on the matrix cores; every item (or
    a sample) checked against the FP64 oracle."""
    import torch
    from paper_2310_15419_amd import inputs
    t_gen = time.perf_counter()
    workers = workers or min(16, len(os.sched_getaffinity(0)))
    items = inputs.workload_batched(count, workers=workers)
    log(f"{len(items)} batched items in {time.perf_counter() - t_gen:.1f} s")
    mats, host = [], []
    for it in items:
        vb = torch.from_numpy(it.A.vals).to(torch.bfloat16)
        host.append(inputs.Csc(it.A.m, it.A.n, it.A.colptr, it.A.rowidx,
                               vb.to(torch.float64).numpy()))
        mats.append(B.DeviceCsc(it.A.m, it.A.n, torch.from_numpy(it.A.colptr).cuda(),
                                torch.from_numpy(it.A.rowidx).cuda(), vb.cuda()))
    ds = [it.d for it in items]
    seeds = [it.seed for it in items]
    work = float(sum(h.nnz * d for h, d in zip(host, ds)))
    outs = [torch.empty((A.n, d), dtype=torch.float32, device="cuda") for A, d in zip(mats, ds)]
    if oracle_all:
        checked = list(range(len(items)))
    else:  # the cheapest items and a few mid-size ones
        order = sorted(range(len(items)), key=lambda i: host[i].nnz * ds[i])
        checked = order[:6] + order[len(order) // 2: len(order) // 2 + 2]
    import oracle
    oracle.build()
    t_or = time.perf_counter()
    refs = {i: oracle.sketch(host[i].m, host[i].n, host[i].colptr, host[i].rowidx, host[i].vals,
                             ds[i], "rademacher", seeds[i]) for i in checked}
    log(f"oracle on {len(checked)} items in {time.perf_counter() - t_or:.1f} s")

    def errors():
        worst = {"normwise": 0.0, "max_elem_scaled": 0.0}
        for i in checked:
            got = outs[i].t().cpu().numpy().astype(np.float64)
            p = oracle.parity(got, refs[i], host[i].colptr, host[i].vals, "rademacher")
            worst["normwise"] = max(worst["normwise"], p["normwise"])
            worst["max_elem_scaled"] = max(worst["max_elem_scaled"], p["max_elem_scaled"])
        return worst

    stream = torch.cuda.current_stream()
    modes = {}
    for prec, pname in ((0, "f32"), (1, "bf16"), (2, "fp8")):
        tune = {"dense_min_pct": dense_min_pct} if dense_min_pct and prec else None
        if prec == 0:
            wss = [B.alloc_workspace(B.workspace_bytes(A, d, "rademacher", prec, tune))
                   for A, d in zip(mats, ds)]

            def plain():
                for A, d, sd, o, w in zip(mats, ds, seeds, outs, wss):
                    B.sketch_into(A, d, "rademacher", sd, o, w, prec=prec, tune=tune)
            ms = timed_ms(plain, steps, stream)
            modes["plain_f32"] = {"ms": ms, "nnz_d_per_s": work / (ms * 1e-3), **errors()}
            del wss
        batch = B.Batch(mats, ds, ["rademacher"] * len(mats), seeds,
                        tunes=[tune] * len(mats) if tune else None, prec=prec)
        ws = B.alloc_workspace(batch.workspace_bytes())
        ms = timed_ms(lambda: batch.run(outs, ws), steps, stream)
        st = batch.status(ws)
        assert all(c == 0 for c in st), st
        modes[f"batched_{pname}"] = {"ms": ms, "nnz_d_per_s": work / (ms * 1e-3), **errors(),
                                     "matrix_core_items": sum(p["variant"] == 0
                                                              for p in batch.plan())}
        del ws
    for k, v in modes.items():
        log(f"{k}: {v['ms']:.2f} ms, {v['nnz_d_per_s']:.3e} nnz*d/s, normwise error "
            f"{v['normwise']:.2e}")
    best = max((v["nnz_d_per_s"], k) for k, v in modes.items() if v["normwise"] <= 1e-2)
    return {"workload": f"batched: {len(items)} sketches, m log-uniform [1e4, 5e5], n in "
                        "[50, 500], d in [2n, 4n], density U(0.5%, 5%), A values BF16, "
                        "S +-1 (seeds 40000+b)",
            "items": len(items), "sum_nnz_d": work, "modes": modes,
            "speedup_batched_bf16_vs_plain_f32": modes["plain_f32"]["ms"] /
                                                 modes["batched_bf16"]["ms"],
            "best_within_1e-2": best[1], "oracle_items": len(checked),
            "error_bound": {"f32": 1e-5, "bf16_fp8": 1e-2}}


# ----------------------------------------------------------------- serving
def bench_serving(B, pool: int, count: int, rates, slots: int, m_hi: float, n_hi: int,
                  budget_gb: float) -> dict:
    """A Poisson stream of sketch-and-precondition least-squares requests over
    `pool` distinct matrices (power-law columns with a dense block, m
    log-uniform in [1e5, m_hi], n in [100, n_hi], d = 2n, S +-1, LSQR to
    1e-10): p50/p99 latency and solves/s of continuous batching (`slots`
    requests in flight) against the plain per-request path (one slot), at
    arrival rates that are fractions of the measured single-request capacity."""
    import torch
    from paper_2310_15419_amd import inputs, serving as S
    rng = np.random.default_rng(50)
    mats = []
    t_gen = time.perf_counter()
    for i in range(pool):
        m = int(np.exp(rng.uniform(np.log(1e5), np.log(m_hi))))
        n = int(rng.integers(100, n_hi + 1))
        A, b, _ = inputs.ls_request(500 + i, m, n, dense_rows=2000)
        mats.append((B.DeviceCsc.from_host(A), torch.from_numpy(b).cuda(), m, n, A.nnz))
    log(f"{len(mats)} request matrices in {time.perf_counter() - t_gen:.1f} s")

    def requests(k_count, arrivals, seed):
        r = np.random.default_rng(seed)
        out = []
        for k in range(k_count):
            dA, db, m, n, _ = mats[int(r.integers(0, len(mats)))]
            p = B.sap_params(2 * n, "rademacher", 60000 + k, atol=1e-10, btol=1e-10)
            out.append(S.Request(k, dA, db, p, arrival=float(arrivals[k])))
        return out

    budget = int(budget_gb * (1 << 30))
    S.Server(budget, 1).run(requests(2, np.zeros(2), 1))  # warm-up
    probe = requests(len(mats), np.zeros(len(mats)), 2)
    t0 = time.perf_counter()
    S.Server(budget, 1).run(probe)
    service = (time.perf_counter() - t0) / len(probe)
    capacity = 1.0 / service
    log(f"single-request service {service * 1e3:.2f} ms -> capacity {capacity:.1f}/s")
    points = []
    for frac in rates:
        rate = frac * capacity
        arr = S.poisson_arrivals(count, rate, seed=int(frac * 1000))
        row = {"rate_frac": frac, "rate_per_s": rate}
        for name, k_slots in (("plain", 1), ("batched", slots)):
            srv = S.Server(budget, k_slots, chunk=16)
            reqs = srv.run(requests(count, arr, 7))
            st = S.latency_stats(reqs)
            st["peak_inflight"] = srv.peak_inflight
            st["converged"] = sum(bool(r.info) and r.info["istop"] in (1, 2) for r in reqs)
            row[name] = st
            log(f"rate {frac:.2f}x {name}: p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, "
                f"{st['solves_per_s']:.1f} solves/s")
        points.append(row)
    return {"workload": "serving: Poisson stream of min ||Ax-b||, A from the power-law generator "
                        f"with a dense 2000-row block, m log-uniform in [1e5, {m_hi:.0e}], n in "
                        f"[100, {n_hi}], d = 2n, S +-1, LSQR to 1e-10, {len(mats)} distinct "
                        f"matrices, HBM budget {budget_gb} GiB, {slots} slots",
            "requests_per_point": count, "single_request_ms": service * 1e3,
            "capacity_per_s": capacity, "points": points}


# ------------------------------------------------ SAP: QR and SVD forms
def ls_error_host(As, x, b) -> float:
    """Error(x) = ||A^T (A x - b)|| / (||A||_F ||A x - b||) of Sec. V-E-2 (scipy, FP64)."""
    r = As @ x - b
    fro = float(np.sqrt(As.multiply(As).sum()))
    return float(np.linalg.norm(As.T @ r) / (fro * np.linalg.norm(r)))


def bench_sap(B, reps: int) -> dict:
    """Single sketch-and-precondition solves at the largest serving size: the QR
    form and the SVD form (Sec. V-E-1: singular values below sigma_max / 1e12
    dropped) on a full-rank request (m = 4e6, n = 1000, d = 2n), and both on a
    rank-deficient stand-in (m = 1e6, n = 500, rank 400), where R is singular.
    Setup (sketch + factorisation + preconditioner) and LSQR times (wall clock
    around synchronised calls, best of `reps`), iterations, kept rank, Jacobi
    sweeps and Error(x)."""
    import torch
    from paper_2310_15419_amd import inputs
    cases = []
    t0 = time.perf_counter()
    A, b, _ = inputs.ls_request(77, 4_000_000, 1000, dense_rows=2000)
    cases.append(("full rank", A, b, 1000))
    A2, b2, _ = inputs.ls_request_rank_deficient(78, 1_000_000, 500, 400, dense_rows=2000)
    cases.append(("rank deficient (rank 400)", A2, b2, 400))
    log(f"SAP requests in {time.perf_counter() - t0:.1f} s")
    rows = []
    for name, A, b, rank in cases:
        dA = B.DeviceCsc.from_host(A)
        db = torch.from_numpy(b).cuda()
        As = A.to_scipy()
        for method, mname in ((B.SAP_QR, "qr"), (B.SAP_SVD, "svd")):
            p = B.sap_params(2 * A.n, "rademacher", 91, atol=1e-10, btol=1e-10, method=method)
            best = None
            for _ in range(reps):
                sv = B.SapSolve(dA, db, p)
                torch.cuda.synchronize()
                ta = time.perf_counter()
                sv.begin()
                torch.cuda.synchronize()
                tb = time.perf_counter()
                while True:
                    sv.iterate(16)
                    inf = sv.info()
                    if inf["done"]:
                        break
                x = sv.finish()
                torch.cuda.synchronize()
                tc = time.perf_counter()
                t = ((tb - ta) * 1e3, (tc - tb) * 1e3)
                if best is None or sum(t) < sum(best[0]):
                    best = (t, inf, x)
                del sv
            (setup_ms, lsqr_ms), inf, x = best
            xh = x.cpu().numpy()
            finite = bool(np.all(np.isfinite(xh)))
            row = {"case": name, "m": A.m, "n": A.n, "nnz": A.nnz, "true_rank": rank,
                   "method": mname, "setup_ms": setup_ms, "lsqr_ms": lsqr_ms,
                   "total_ms": setup_ms + lsqr_ms, "iterations": int(inf["iterations"]),
                   "istop": int(inf["istop"]), "kept_rank": int(inf["rank"]),
                   "sweeps": int(inf["sweeps"]), "x_finite": finite,
                   "error": ls_error_host(As, xh, b) if finite else None}
            log(f"SAP {name} {mname}: setup {setup_ms:.1f} ms, LSQR {lsqr_ms:.1f} ms, "
                f"{row['iterations']} it, rank {row['kept_rank']}, sweeps {row['sweeps']}, "
                f"Error {row['error']}")
            rows.append(row)
        del dA, db
    return {"workload": "SAP single solves: power-law columns + dense 2000-row block, b = A x + "
                        "1e-6 noise, d = 2n, S +-1 seed 91, LSQR to 1e-10", "solves": rows}


# ------------------------------------------- the paper's SpMM workloads
def bench_spmm_shapes(B, which: str, steps: int) -> dict:
    """Stand-ins for the paper's SpMM test matrices (Table I shapes, or the
    Table VI patterns), d = 3n, (-1,1) S: the S-tile kernel (the whole
    sk_sketch step) beside the Algorithm 3 loop-order kernel, nnz*d/s each,
    their roofline fractions against each kernel's own ALU work (the tile
    kernel generates each S value once per row block, the kji kernel once per
    nonzero), and their agreement (normwise difference of the two A_hat)."""
    import torch
    from paper_2310_15419_amd import inputs
    stream = torch.cuda.current_stream()
    gen = generator_costs(B, "uniform", stream)
    c_call, c_val = gen["philox_slots_per_call"], gen["transform_slots_per_value"]
    names = list(inputs.TABLE1) if which == "table1" else ["A", "B", "C"]
    rows = []
    for name in names:
        if which == "table1":
            A, d = inputs.table1_standin(name)
        else:
            A = inputs.abnormal(name)
            d = 3 * A.n
        dA = B.DeviceCsc.from_host(A)
        out_t = torch.empty((A.n, d), dtype=torch.float32, device="cuda")
        out_c = torch.empty_like(out_t)
        tile = {"kernel": B.KERNEL_TILE}
        ws = B.alloc_workspace(B.workspace_bytes(dA, d, "uniform", tune=tile))
        wc = B.alloc_workspace(B.colwise_workspace_bytes(dA, d))
        t_ms = timed_ms(lambda: B.sketch_into(dA, d, "uniform", 5, out_t, ws, tune=tile), steps,
                        stream)
        R = B.sketch_status(ws)["nonempty_rows"]
        c_ms = timed_ms(lambda: B.sketch_colwise_into(dA, d, "uniform", 5, out_c, wc), steps,
                        stream)
        diff = float(torch.linalg.norm(out_t - out_c) / torch.linalg.norm(out_c))
        # the library's own choice: the cost model's (no tuning), then the
        # measured tuner's (cached for the shape class, so tune=None runs it)
        B.plan_cache_clear()
        pick = B.plan_info(dA, d, "uniform")["kernel"]
        wa = B.alloc_workspace(B.workspace_bytes(dA, d, "uniform"))
        a_ms = timed_ms(lambda: B.sketch_into(dA, d, "uniform", 5, out_c, wa), steps, stream)
        t0 = time.perf_counter()
        tuned, _ = B.autotune_measure(dA, d, "uniform", 5, out_c)
        tune_s = time.perf_counter() - t0
        wt = B.alloc_workspace(B.workspace_bytes(dA, d, "uniform"))
        u_ms = timed_ms(lambda: B.sketch_into(dA, d, "uniform", 5, out_c, wt), steps, stream)
        B.plan_cache_clear()
        nnzd = A.nnz * d
        work_t = R * -(-d // 4) * c_call + R * d * c_val + nnzd
        work_c = A.nnz * -(-d // 4) * c_call + A.nnz * d * c_val + nnzd
        row = {"matrix": name, "m": A.m, "n": A.n, "nnz": A.nnz, "d": d, "nonempty_rows": R,
               "tile_ms": t_ms, "tile_nnz_d_per_s": nnzd / (t_ms * 1e-3),
               "tile_frac": work_t / (t_ms * 1e-3) / VALU_PEAK,
               "kji_ms": c_ms, "kji_nnz_d_per_s": nnzd / (c_ms * 1e-3),
               "kji_frac": work_c / (c_ms * 1e-3) / VALU_PEAK,
               "kji_over_tile": c_ms / t_ms, "normwise_difference": diff,
               "model_kernel": pick, "model_ms": a_ms, "tuned": tuned, "tuned_ms": u_ms,
               "tuner_seconds": tune_s}
        log(f"{name}: tile {t_ms:.2f} ms ({row['tile_nnz_d_per_s']:.3e} nnz*d/s), kji "
            f"{c_ms:.2f} ms ({row['kji_nnz_d_per_s']:.3e}), difference {diff:.1e}; model "
            f"kernel {pick} {a_ms:.2f} ms, tuned {u_ms:.2f} ms {tuned}")
        rows.append(row)
        del ws, wc, wa, wt, out_t, out_c
    return {"workload": ("Table I stand-ins" if which == "table1" else "Table VI patterns") +
                        ": shapes and nonzero counts of the paper's matrices, uniform random "
                        "columns (Table I) or the exotic patterns (m=1e5, n=1e4, density 1e-3), "
                        "d = 3n, S (-1,1) Philox4x32-10 seed 5",
            "generator": gen, "matrices": rows}


def bench_tuner(B, names, steps: int) -> dict:
    """The measured tuner against an exhaustive sweep of the same space
    (Algorithm 3 kernel; every S-tile kernel shape x splits 1..64 x rows in
    order or balanced row blocks) timed
    the bench's way (event-timed average of `steps` calls), per workload."""
    import torch
    stream = torch.cuda.current_stream()
    res = []
    for name in names:
        A, d, dist, seed, _ = make_workload(name)
        dA = B.DeviceCsc.from_host(A)
        out = torch.empty((A.n, d), dtype=torch.float32, device="cuda")
        B.plan_cache_clear()

        def run(tune):
            ws = B.alloc_workspace(B.workspace_bytes(dA, d, dist, tune=tune))
            ms = timed_ms(lambda: B.sketch_into(dA, d, dist, seed, out, ws, tune=tune), steps,
                          stream)
            del ws
            return ms
        model_ms = run(None)
        model = B.autotune(dA, d, dist)
        t0 = time.perf_counter()
        tuned, tuner_ms = B.autotune_measure(dA, d, dist, seed, out)
        tune_s = time.perf_counter() - t0
        tuned_ms = run(tuned)
        sweep = [{"kernel": 2, "ms": run({"kernel": 2})}]
        for v in range(1, B.variant_count() + 1):
            for sp in (1, 2, 4, 6, 8, 12, 16, 20, 24, 32, 48, 64):
                for bal in (1, 2):  # rows in order, balanced row blocks
                    t = {"kernel": 1, "variant": v, "splits": sp, "balance": bal}
                    if bal == 2 and B.plan_info(dA, d, dist, tune=t)["balance_sb"] == 0:
                        continue  # (the plan has no balanced form)
                    try:
                        ms = run(t)
                    except (B.SketchError, RuntimeError) as e:  # too many partial slices, ...
                        log(f"{name}: sweep point {t} skipped: {e}")
                        continue
                    sweep.append(dict(t, ms=ms))
            log(f"{name}: swept variant {v}")
        best = min(sweep, key=lambda r: r["ms"])
        row = {"workload": name, "d": d, "dist": dist, "model_tuning": model,
               "model_ms": model_ms, "tuned": tuned, "tuner_own_ms": tuner_ms,
               "tuned_ms": tuned_ms, "tuner_seconds": tune_s, "best_swept": best,
               "tuned_over_best": tuned_ms / best["ms"], "model_over_best": model_ms / best["ms"],
               "sweep_points": len(sweep),
               "sweep": sorted(sweep, key=lambda r: r["ms"])[:12]}
        log(f"{name}: model {model_ms:.3f} ms, tuned {tuned} {tuned_ms:.3f} ms, best swept "
            f"{best} -> tuned/best {row['tuned_over_best']:.3f}")
        res.append(row)
        B.plan_cache_clear()
        del dA, out
    return {"workloads": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_scale",
                    help="plain_scale (default), plain_small, skewed, batched, serving, "
                         "table1, abnormal, tuner, sap")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: leave out the batched and serving sub-objects")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--rows-per-block", type=int, default=0)
    ap.add_argument("--splits", type=int, default=0)
    ap.add_argument("--dense-min-pct", type=int, default=0)
    ap.add_argument("--col-split", type=int, default=0, help="0 auto, 1 off, 2 on")
    ap.add_argument("--row-pad", type=int, default=0)
    ap.add_argument("--balance", type=int, default=0,
                    help="row blocks: 0 auto, 1 rows in order, 2 balanced")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--workers", type=int, default=0,
                    help="processes generating the batched items (0: up to 16)")
    ap.add_argument("--serve-pool", type=int, default=24)
    ap.add_argument("--serve-requests", type=int, default=150)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-m-hi", type=float, default=4e6)
    ap.add_argument("--serve-n-hi", type=int, default=1000)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-rates", type=float, nargs="+", default=[0.5, 0.9, 1.2])
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

    if args.workload == "serving":
        sv = bench_serving(B, args.serve_pool, args.serve_requests, args.serve_rates,
                           args.serve_slots, args.serve_m_hi, args.serve_n_hi,
                           args.serve_budget_gb)
        head = next((p for p in sv["points"] if abs(p["rate_frac"] - 0.9) < 1e-9),
                    sv["points"][-1])
        print(json.dumps({
            "metric": "p99 latency of served sketch-and-precondition least-squares solves",
            "value": head["batched"]["p99_ms"], "unit": "ms", "n_gpus": 1,
            "steps": args.serve_requests, "warmup": 2, "ms_per_step": head["batched"]["mean_ms"],
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64 (sketch f32)", "data": "synthetic", "config": sv}), flush=True)
        return
    if args.workload == "sap":
        sp = bench_sap(B, max(1, args.steps))
        svd = [r for r in sp["solves"] if r["method"] == "svd"]
        print(json.dumps({
            "metric": "sketch-and-precondition solve time, QR and SVD forms",
            "value": svd[0]["total_ms"], "unit": "ms (SVD form, full-rank m=4e6 n=1000)",
            "n_gpus": 1, "steps": max(1, args.steps), "warmup": 0,
            "ms_per_step": svd[0]["total_ms"], "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64 (sketch f32 for QR, f64 for SVD)",
            "data": "synthetic", "config": sp}), flush=True)
        return
    if args.workload == "tuner":
        tr = bench_tuner(B, ["plain_scale", "skewed"], args.steps)
        worst = max(r["tuned_over_best"] for r in tr["workloads"])
        print(json.dumps({
            "metric": "measured-tuner pick over the best point of an exhaustive sweep",
            "value": worst, "unit": "ratio (worst workload)", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": tr}), flush=True)
        return
    if args.workload in ("table1", "abnormal"):
        sp = bench_spmm_shapes(B, args.workload, args.steps)
        tot = sum(r["nnz"] * r["d"] for r in sp["matrices"])
        t_ms = sum(r["tuned_ms"] for r in sp["matrices"])
        print(json.dumps({
            "metric": "sketched nnz·d per sec on stand-ins for the paper's SpMM matrices "
                      "(measured-tuner plans)",
            "value": tot / (t_ms * 1e-3), "unit": "nnz*d/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": t_ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": sp}), flush=True)
        return
    if args.workload == "batched":
        bt = bench_batched(B, args.batch_count, args.steps, args.dense_min_pct, args.workers,
                           oracle_all=True)
        print(json.dumps({
            "metric": f"batched vs plain at fixed error ({args.batch_count} sketches)",
            "value": bt["modes"]["batched_bf16"]["nnz_d_per_s"], "unit": "nnz*d/s",
            "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": bt["modes"]["batched_bf16"]["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16 operands, f32 accumulate",
            "data": "synthetic", "config": bt}), flush=True)
        return

    res = bench_plain(args, B)
    if args.workload == "plain_scale" and not args.no_extras:
        res["batched"] = bench_batched(B, 64, max(2, args.steps // 2), workers=args.workers)
        res["serving"] = bench_serving(B, pool=6, count=60, rates=[0.9], slots=8, m_hi=1e6,
                                       n_hi=500, budget_gb=64.0)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
