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


def bench_serving(args):
    """Config 5: a Poisson stream of sketch-and-precondition least-squares
    requests; p50/p99 latency and solves/s of continuous batching (several
    slots) against the plain per-request path (one slot), at arrival rates
    that are fractions of the measured single-request capacity."""
    import torch
    from paper_2310_15419_amd import binding as B, inputs, serving as S
    rng = np.random.default_rng(50)
    pool = []
    t_gen = time.perf_counter()
    for i in range(args.serve_pool):
        m = int(np.exp(rng.uniform(np.log(1e5), np.log(args.serve_m_hi))))
        n = int(rng.integers(100, args.serve_n_hi + 1))
        A, b, _ = inputs.ls_request(500 + i, m, n, dense_rows=2000)
        pool.append((B.DeviceCsc.from_host(A), torch.from_numpy(b).cuda(), m, n, A.nnz))
    print(f"[bench] {len(pool)} request matrices in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)

    def requests(count, arrivals, seed):
        r = np.random.default_rng(seed)
        out = []
        for k in range(count):
            dA, db, m, n, _ = pool[int(r.integers(0, len(pool)))]
            p = B.sap_params(2 * n, "rademacher", 60000 + k, atol=1e-10, btol=1e-10)
            out.append(S.Request(k, dA, db, p, arrival=float(arrivals[k])))
        return out

    budget = int(args.serve_budget_gb * (1 << 30))
    # warm-up, then the single-request service time (one slot, all queued)
    S.Server(budget, 1).run(requests(2, np.zeros(2), 1))
    probe = requests(len(pool), np.zeros(len(pool)), 2)
    t0 = time.perf_counter()
    S.Server(budget, 1).run(probe)
    service = (time.perf_counter() - t0) / len(probe)
    capacity = 1.0 / service
    print(f"[bench] single-request service {service * 1e3:.2f} ms -> capacity {capacity:.1f}/s",
          file=sys.stderr, flush=True)
    points = []
    for frac in args.serve_rates:
        rate = frac * capacity
        arr = S.poisson_arrivals(args.serve_requests, rate, seed=int(frac * 1000))
        row = {"rate_frac": frac, "rate_per_s": rate}
        for name, slots in (("plain", 1), ("batched", args.serve_slots)):
            srv = S.Server(budget, slots, chunk=16)
            reqs = srv.run(requests(args.serve_requests, arr, 7))
            st = S.latency_stats(reqs)
            st["peak_inflight"] = srv.peak_inflight
            st["converged"] = sum(bool(r.info) and r.info["istop"] in (1, 2) for r in reqs)
            row[name] = st
            print(f"[bench] rate {frac:.2f}x {name}: p50 {st['p50_ms']:.1f} ms, p99 "
                  f"{st['p99_ms']:.1f} ms, {st['solves_per_s']:.1f} solves/s",
                  file=sys.stderr, flush=True)
        points.append(row)
    head = next((p for p in points if abs(p["rate_frac"] - 0.9) < 1e-9), points[-1])
    res = {
        "metric": "p99 latency of served sketch-and-precondition least-squares solves",
        "value": head["batched"]["p99_ms"], "unit": "ms", "n_gpus": 1,
        "steps": args.serve_requests, "warmup": 2,
        "ms_per_step": head["batched"]["mean_ms"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 (sketch f32)",
        "data": "synthetic",
        "config": {"workload": "serving: Poisson stream of min ||Ax-b||, A from the power-law "
                               f"generator with a dense 2000-row block, m log-uniform in [1e5, "
                               f"{args.serve_m_hi:.0e}], n in [100, {args.serve_n_hi}], d = 2n, "
                               "S +-1, LSQR to 1e-10, "
                               f"{len(pool)} distinct matrices, HBM budget "
                               f"{args.serve_budget_gb} GiB, {args.serve_slots} slots",
                   "single_request_ms": service * 1e3, "capacity_per_s": capacity,
                   "points": points},
    }
    print(json.dumps(res), flush=True)


def bench_batched(args):
    """Config 4: 512 uneven +-1 sketches, A values BF16; plain launches (one
    sk_sketch per item) against one batched launch, with S in FP32 on the
    sparse kernel and in BF16 / FP8 on the matrix cores, each checked against
    the FP64 oracle on a sample of items."""
    import torch
    from paper_2310_15419_amd import binding as B, inputs
    t_gen = time.perf_counter()
    # a process pool generates the items (one process under a profiler:
    # --workers 1)
    workers = args.workers or min(16, len(os.sched_getaffinity(0)))
    items = inputs.workload_batched(args.batch_count, workers=workers)
    print(f"[bench] {len(items)} items in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr,
          flush=True)
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
    # oracle sample: the cheapest items and a few mid-size ones
    order = sorted(range(len(items)), key=lambda i: host[i].nnz * ds[i])
    sample = order[:6] + order[len(order) // 2: len(order) // 2 + 2]
    import oracle
    oracle.build()
    refs = {i: oracle.sketch(host[i].m, host[i].n, host[i].colptr, host[i].rowidx, host[i].vals,
                             ds[i], "rademacher", seeds[i]) for i in sample}

    def err():
        e = 0.0
        for i in sample:
            got = outs[i].t().cpu().numpy().astype(np.float64)
            e = max(e, float(np.linalg.norm(got - refs[i]) / np.linalg.norm(refs[i])))
        return e

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        best = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best.append(e0.elapsed_time(e1))
        return float(np.median(best))

    modes = {}
    # --dense-min-pct: the density (percent) from which items run on the
    # matrix cores in the BF16/FP8 modes (0: the library's measured threshold)
    for prec, pname in ((0, "f32"), (1, "bf16"), (2, "fp8")):
        tune = {"dense_min_pct": args.dense_min_pct} if args.dense_min_pct and prec else None
        wss = [B.alloc_workspace(B.workspace_bytes(A, d, "rademacher", prec, tune))
               for A, d in zip(mats, ds)]

        def plain():
            for A, d, sd, o, w in zip(mats, ds, seeds, outs, wss):
                B.sketch_into(A, d, "rademacher", sd, o, w, prec=prec, tune=tune)
        ms = timed(plain, args.steps)
        modes[f"plain_{pname}"] = {"ms": ms, "nnz_d_per_s": work / (ms * 1e-3), "error": err()}
        del wss
        batch = B.Batch(mats, ds, ["rademacher"] * len(mats), seeds,
                        tunes=[tune] * len(mats) if tune else None, prec=prec)
        ws = B.alloc_workspace(batch.workspace_bytes())
        ms = timed(lambda: batch.run(outs, ws), args.steps)
        st = batch.status(ws)
        assert all(c == 0 for c in st), st
        modes[f"batched_{pname}"] = {"ms": ms, "nnz_d_per_s": work / (ms * 1e-3), "error": err(),
                                     "matrix_core_items": sum(p["variant"] == 0
                                                              for p in batch.plan())}
        del ws
        for k in (f"plain_{pname}", f"batched_{pname}"):
            print(f"[bench] {k}: {modes[k]['ms']:.2f} ms, {modes[k]['nnz_d_per_s']:.3e} nnz*d/s, "
                  f"max rel error {modes[k]['error']:.2e}", file=sys.stderr, flush=True)
    best = max((v["nnz_d_per_s"], k) for k, v in modes.items() if v["error"] <= 1e-2)
    res = {
        "metric": "batched vs plain at fixed error (512 sketches)",
        "value": modes["batched_bf16"]["nnz_d_per_s"], "unit": "nnz*d/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": modes["batched_bf16"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 operands, f32 accumulate", "data": "synthetic",
        "config": {"workload": f"batched: {len(items)} sketches, m log-uniform [1e4, 5e5], n in "
                               "[50, 500], d in [2n, 4n], density U(0.5%, 5%), A values BF16, "
                               "S +-1 (seeds 40000+b)",
                   "sum_nnz_d": work, "modes": modes, "best_within_1e-2": best[1],
                   "oracle_sample_items": len(sample)},
    }
    print(json.dumps(res), flush=True)


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
        bench_serving(args)
        return
    if args.workload == "batched":
        bench_batched(args)
        return

    t_gen = time.perf_counter()
    A, d, dist, seed, desc = make_workload(args.workload)
    print(f"[bench] workload generated in {time.perf_counter() - t_gen:.1f} s "
          f"(m={A.m}, n={A.n}, nnz={A.nnz}, d={d})", file=sys.stderr, flush=True)
    dA = B.DeviceCsc.from_host(A, dtype=np.float32 if A.vals.dtype != np.float64 else None)
    tune = {"variant": args.variant, "rows_per_block": args.rows_per_block,
            "splits": args.splits, "dense_min_pct": args.dense_min_pct,
            "col_split": args.col_split, "row_pad": args.row_pad, "tile_rows": args.tile_rows}
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
    res["config"]["input_sha256"] = A.sha256()
    if not args.no_cpu_baseline:
        rec, ref, S = cpu_baseline(A, d, dist, seed, args.cpu_seconds)
        if S.m == A.m:
            # the whole workload: the timed output itself
            got = out.t().cpu().numpy()
            what = "the timed output, every element"
        else:
            # a row sample: the same call on the sampled rows
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
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
