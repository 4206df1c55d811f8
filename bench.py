#!/usr/bin/env python3
"""Benchmark of the FastID overloaded-GEMM comparison on one MI355X.

Default workload: 2,048 mixture queries x 20,000,000 references x 2,048 SNP
loci (one bit per locus, ~5.1 GB packed database resident in HBM), per-query
top-32 (count, reference index) plus full counts of 64 seeded 256x256 tiles.
One step = one pass of the hot path over that batch: query staging, the
seed/scan/merge top-k pipeline and the tile counts.  The database is built
once before timing (ingest); queries are packed before timing.

Prints one JSON line.  ``value`` is query-ref-locus comparisons per second
(N_Q * N_R * L per step).  ``roofline`` describes the dominant kernel (the
top-k scan), timed live with HIP events on the stream it runs on;
``cpu_baseline`` times the oracle (all cores and one thread) and the packed
x86 baseline on bounded, labelled samples on the host cores; ``serving``
serves 2,000 Poisson requests at 50/s after 200 warm-up on the same resident
database, with continuous batching and with FIFO per-request passes.

``--workload full-64x20K`` times the 64 x 20,000 x 2,048 full count matrix
per call; ``--workload large-panel`` runs 256 x 2M x 32768 loci (threshold +
top-32 from one scan);
``--workload serving`` serves a Poisson request stream (continuous batching
and FIFO per-call); ``--workload ragged-400`` runs the ragged-batch workload: 400
independent top-32 jobs (1-512 queries, 10k-2M reference slices, panels of
1024-16384 loci, mixed modes) as one persistent launch, eagerly and as a HIP
graph, against the same jobs issued as per-job top-k calls.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# MI355X (gfx950): 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz of 32-bit VALU issue.
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
# The popcount path issues 2 VALU ops (AND/XOR, then BCNT with fused add) per
# 32-locus word pair, i.e. 1/16 op per comparison.
OPS_PER_COMPARISON = 2.0 / 32.0
# The matrix-core path: one int8 multiply-accumulate (2 ops) per comparison,
# against MI355X's dense int8 MFMA peak.
MFMA_INT8_OPS_PER_S = 5.0e15
MFMA_FP4_OPS_PER_S = 10.1e15
MFMA_OPS_PER_COMPARISON = 2.0
METRIC = "query-ref-locus comparisons/s at 2048x20Mx2048 loci; served p50/p99 latency"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixture-2048x20Mx2048-top32")
    ap.add_argument("--n-refs", type=int, default=None, help="override the reference count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-refs", type=int, default=262144)
    ap.add_argument("--cpu-sample-queries", type=int, default=256)
    ap.add_argument("--backend", choices=("auto", "popcount", "mfma", "mfma_fp4"), default="auto")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy, to scale HBM byte counters")
    ap.add_argument("--block-refs", type=int, default=2_000_000,
                    help="streamed: references per host-to-device block")
    ap.add_argument("--pageable", action="store_true",
                    help="streamed: keep the rows in pageable instead of pinned host memory")
    ap.add_argument("--jobs", type=int, default=400, help="ragged-400: number of jobs")
    ap.add_argument("--tune", action="store_true",
                    help="ragged-400: run the autotuner first (writes gpurun_out/tune_table.json)")
    ap.add_argument("--no-per-call", action="store_true",
                    help="ragged-400: skip the per-job call baseline")
    ap.add_argument("--serve-requests", type=int, default=2200,
                    help="requests of each serving phase (the first 200 are warm-up)")
    ap.add_argument("--cpu-packed-refs", type=int, default=2_000_000,
                    help="references of the packed x86 baseline's sample (all queries)")
    ap.add_argument("--serve-rate", type=float, default=50.0, help="Poisson arrivals per second")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving phase")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the on-device peak probes (roofline peak_measured)")
    ap.add_argument("--serve-policies", default="continuous,fifo",
                    help="serving workload: policies to run (continuous, fifo)")
    ap.add_argument("--serve-chunks", type=int, default=8, help="continuous policy: database chunks")
    ap.add_argument("--tick-chunks", type=int, default=0,
                    help="continuous policy: chunks per tick (0: the whole database)")
    ap.add_argument("--serve-stress-rate", type=float, default=250.0,
                    help="serving workload: a second, heavier arrival rate (0 to skip)")
    return ap.parse_args()


BACKEND_NAMES = {1: "popcount", 2: "mfma", 3: "mfma_fp4"}
DTYPES = {"popcount": "u32 (exact integer counts)",
          "mfma": "i8 0/1 operands, i32 accumulate (exact integer counts)",
          "mfma_fp4": "fp4-e2m1 0/1-coded operands, f32 accumulate (exact integer counts: every sum is an "
                      "integer below 2^18)"}


def roofline_for(backend: str, comps: float, kernel_s: float) -> dict:
    """Roofline object of the top-k scan kernel of one backend."""
    if backend == "mfma":
        achieved = comps * MFMA_OPS_PER_COMPARISON / kernel_s / 1e12
        peak = MFMA_INT8_OPS_PER_S / 1e12
        r = {"bound": "mfma", "unit": "TOP/s (int8 MFMA)", "kernel": "mfma_scan_kernel (top-k epilogue)"}
    elif backend == "mfma_fp4":
        achieved = comps * MFMA_OPS_PER_COMPARISON / kernel_s / 1e12
        peak = MFMA_FP4_OPS_PER_S / 1e12
        r = {"bound": "mfma", "unit": "TFLOP/s (fp4 MFMA)", "kernel": "fp4_scan_kernel (top-k epilogue)"}
    else:
        achieved = comps * OPS_PER_COMPARISON / kernel_s / 1e12
        peak = VALU_LANE_OPS_PER_S / 1e12
        r = {"bound": "alu", "unit": "Tops/s (32-bit VALU lane-ops)", "kernel": "scan_kernel (top-k epilogue)"}
    r.update({"achieved": round(achieved, 3), "peak": round(peak, 3),
              "frac": round(achieved / peak, 4), "traffic": None,
              "kernel_ms": round(kernel_s * 1e3, 3)})
    return r


def measure_peaks(ctx) -> dict:
    """Sustained rates of the bounding units on this device (fid_peak_probe),
    in the roofline units: fp4 / int8 MFMA in T(FL)OP/s (2 ops per MAC),
    VALU in T lane-ops/s, HBM copy in GB/s."""
    import torch
    from paper_1707_00516_amd import (FID_PROBE_HBM_COPY, FID_PROBE_MFMA_FP4, FID_PROBE_MFMA_I8,
                                      FID_PROBE_VALU, fid_peak_probe)
    buf = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")  # 2 GiB copied each way
    out = {}
    for name, probe, scale in (("mfma_fp4", FID_PROBE_MFMA_FP4, 2e-12), ("mfma", FID_PROBE_MFMA_I8, 2e-12),
                               ("popcount", FID_PROBE_VALU, 1e-12), ("hbm", FID_PROBE_HBM_COPY, 1e-9)):
        rate, ms = fid_peak_probe(ctx.handle, probe, buf.data_ptr(), buf.numel())
        out[name] = round(rate * scale, 3)
        log(f"peak probe {name}: {out[name]} ({ms:.3f} ms per launch)")
    del buf
    return out


def add_measured_peak(roof: dict, backend: str, peaks: dict | None) -> dict:
    """The roofline against the rate the same unit sustains on this device."""
    if peaks:
        roof["peak_measured"] = peaks[backend]
        roof["frac_of_measured"] = round(roof["achieved"] / peaks[backend], 4)
    return roof


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (profiles/scan_traffic.json: FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB
    copy's readings), or None when there are none or a source they depend on
    (the kernel's, and for a batch its plan and tuning table) has changed
    since they were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "scan_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel)
    if not rec:
        return None
    sources = rec.get("sources") or {rec["source"]: rec["source_sha256"]}
    for src, digest in sources.items():
        with open(os.path.join(here, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    kib = 1024.0
    reads = rec["fetch_kib"] * kib * rec["copy_bytes_each"] / (rec["copy_fetch_kib"] * kib)
    writes = rec["write_kib"] * kib * rec["copy_bytes_each"] / (rec["copy_write_kib"] * kib)
    return round(reads + writes)


def tile_origins(seed: int, n_tiles: int, n_q: int, n_refs: int, size: int = 256):
    import gen
    u = gen.u64s(seed, 5, 0, 2 * n_tiles)
    nq_t = max(1, n_q // size)
    nr_t = max(1, n_refs // size)
    return [(int(u[2 * i] % nq_t) * size, int(u[2 * i + 1] % nr_t) * size) for i in range(n_tiles)]


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n: int) -> None:
    """Thread count of later OpenMP regions of this thread (the libgomp the
    oracle and the packed baseline share)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def cpu_baseline(w, n_q: int, n_refs: int, packed_refs: int):
    """CPU baselines on the host cores: the oracle (byte loop + full sort), as
    it stands, on bounded samples with all cores and with one thread; and the
    packed x86 baseline (u64 popcount, OpenMP) on every query against a
    labelled share of the database."""
    import numpy as np

    import gen
    import oracle
    import oracle.packed as cpu_packed
    thr = gen.maf_thresholds(w.seed, w.n_loci, w.maf_lo)
    refs = gen.ref_bytes(w.seed, thr, 0, n_refs)
    Q = gen.mixtures(w.seed, thr, 0, w.n_refs, 0, max(n_q, 64), w.nc_lo, w.nc_hi, w.flip)[0]
    orc = oracle.default()
    cores = orc.num_threads()
    t0 = time.perf_counter()
    orc.topk(orc.counts(refs, Q[:n_q], w.mode), w.k)
    dt = time.perf_counter() - t0
    comps = n_q * n_refs * w.n_loci
    # one thread: 64 queries x a quarter of the references
    n1, r1 = 64, n_refs // 4
    _omp_threads(1)
    try:
        t1 = time.perf_counter()
        orc.topk(orc.counts(refs[:r1], Q[:n1], w.mode), w.k)
        dt1 = time.perf_counter() - t1
    finally:
        _omp_threads(cores)
    del refs
    out = {"value": comps / dt, "unit": "comparisons/s", "cores": cores,
           "kind": "oracle", "seconds": round(dt, 3),
           "sample": f"{n_q} queries x {n_refs} references x {w.n_loci} loci of the same "
                     f"workload (counts + top-{w.k} by full sort)",
           "one_thread": {"value": n1 * r1 * w.n_loci / dt1, "seconds": round(dt1, 3),
                          "sample": f"{n1} queries x {r1} references x {w.n_loci} loci"},
           "nproc": os.cpu_count(), "cpu_model": _cpu_model()}
    # the packed baseline: every query against the first packed_refs references
    if packed_refs > 0:
        words = np.empty((packed_refs, cpu_packed.words(w.n_loci)), np.uint64)
        chunk = 1 << 18
        for r0 in range(0, packed_refs, chunk):
            n = min(chunk, packed_refs - r0)
            cpu_packed.pack(gen.ref_bytes(w.seed, thr, r0, n), out=words[r0:r0 + n])
        M = gen.mixtures(w.seed, thr, 0, w.n_refs, 0, w.n_q, w.nc_lo, w.nc_hi, w.flip)[0]
        qp = cpu_packed.pack(M)
        t2 = time.perf_counter()
        cpu_packed.topk(words, qp, w.n_loci, w.mode, w.k)
        dt2 = time.perf_counter() - t2
        out["cpu_packed"] = {
            "value": w.n_q * packed_refs * w.n_loci / dt2, "unit": "comparisons/s", "seconds": round(dt2, 3),
            "cores": cpu_packed.num_threads(), "isa": cpu_packed.isa(),
            "kind": "packed x86 baseline (u64 popcount, OpenMP)",
            "sample": f"all {w.n_q} queries x the first {packed_refs} references "
                      f"({100.0 * packed_refs / w.n_refs:.0f}% of the database) x {w.n_loci} loci, top-{w.k}"}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the reference-sharded multi-GPU design is documented, not built)", flush=True)
        sys.exit(2)
    if args.workload == "ragged-400":
        return bench_ragged(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "large-panel":
        return bench_large_panel(args)
    if args.workload == "streamed":
        return bench_streamed(args)
    if args.workload == "streamed-full":
        return bench_streamed_full(args)
    if args.workload in ("full-64x20K", "mixture-64x20000x2048-full"):
        return bench_full_small(args)
    return bench_headline(args)


def bench_headline(args):
    import numpy as np
    import torch

    import gen
    from gen.workloads import BY_NAME
    from paper_1707_00516_amd import (FID_BACKEND_AUTO, FID_BACKEND_MFMA, FID_BACKEND_MFMA_FP4,
                                      FID_BACKEND_POPCOUNT,
                                      fid_ctx_enable_timing, fid_ctx_scan_time,
                                      fid_ctx_set_backend)
    from paper_1707_00516_amd.torch_api import Context

    w = BY_NAME[args.workload]
    n_refs = args.n_refs or w.n_refs
    L = w.n_loci
    torch.cuda.init()
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    backend = {"auto": FID_BACKEND_AUTO, "popcount": FID_BACKEND_POPCOUNT,
               "mfma": FID_BACKEND_MFMA, "mfma_fp4": FID_BACKEND_MFMA_FP4}[args.backend]
    fid_ctx_set_backend(ctx.handle, backend)

    # ---------------------------------------------------------------- inputs
    t0 = time.perf_counter()
    thr = gen.maf_thresholds(w.seed, L, w.maf_lo)
    thr_dev = torch.from_numpy(thr.astype(np.uint32)).cuda()
    from paper_1707_00516_amd import fid_row_words
    rows = torch.empty((n_refs, fid_row_words(L)), dtype=torch.int64, device="cuda")
    chunk = 1 << 20
    buf = torch.empty((min(chunk, n_refs), L), dtype=torch.uint8, device="cuda")
    for r0 in range(0, n_refs, chunk):
        n = min(chunk, n_refs - r0)
        gen.ref_bytes_gpu(w.seed, thr_dev.data_ptr(), L, r0, n, buf.data_ptr(), L,
                          stream.cuda_stream)
        ctx.pack(buf[:n], L, out=rows[r0:r0 + n])
    del buf
    t_build = time.perf_counter()
    db = ctx.build_db(rows, L)
    ctx.sync()
    t_build = time.perf_counter() - t_build
    del rows
    torch.cuda.empty_cache()
    M, contrib, ncon, F = gen.mixtures(w.seed, thr, 0, n_refs, 0, w.n_q, w.nc_lo, w.nc_hi, w.flip)
    q_rows = ctx.pack(torch.from_numpy(M).cuda())
    tiles = tile_origins(w.seed, 64, w.n_q, n_refs)
    ws = ctx.topk_workspace(db, w.n_q, w.k)
    ctx.sync()
    log(f"setup {time.perf_counter() - t0:.1f}s (db build {t_build * 1e3:.1f} ms)")

    if args.copy_calibration:
        # A plain copy kernel of known size: 1 GiB read + 1 GiB written (an
        # elementwise kernel, so it shows up in the counters; a same-dtype
        # copy_ may go to a DMA engine instead).  Its FETCH_SIZE / WRITE_SIZE
        # readings calibrate the counters of the scan.
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.bitwise_xor(src, 0, out=dst)
        torch.cuda.synchronize()
        log("copy calibration: 1073741824 bytes read and written by an elementwise kernel")
        del src, dst

    def step():
        cnt, idx = ctx.compare_topk(db, q_rows, w.mode, w.k, ws=ws)
        tl = ctx.compare_tiles(db, q_rows, w.mode, tiles, 256, 256)
        return cnt, idx, tl

    fid_ctx_enable_timing(ctx.handle, True)
    for i in range(args.warmup):
        step()
        ctx.sync()
        log(f"warmup {i + 1}/{args.warmup} done")
    fid_ctx_scan_time(ctx.handle, reset=True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for i in range(args.steps):
        out = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    scan_ms, launches = fid_ctx_scan_time(ctx.handle, reset=True)
    log(f"timed {args.steps} steps: {total_ms:.1f} ms; scan kernel {scan_ms:.1f} ms over "
        f"{launches} launches")

    comps = w.n_q * n_refs * L
    ms_per_step = total_ms / args.steps
    value = comps / (ms_per_step / 1e3)
    scan_avg_s = scan_ms / max(launches, 1) / 1e3
    from paper_1707_00516_amd import fid_backend_for
    used = BACKEND_NAMES[fid_backend_for(ctx.handle, db.handle, w.n_q)]
    roofline = roofline_for(used, comps, scan_avg_s)
    if used == "mfma_fp4" and n_refs == w.n_refs:
        roofline["traffic"] = recorded_traffic("fp4_scan_kernel<0, 1>")
    add_measured_peak(roofline, used, None if args.no_peaks else measure_peaks(ctx))

    serving = None
    if not args.no_serve:
        serving = {}
        warm = min(200, args.serve_requests // 5)
        for name, policy in (("continuous", 0), ("fifo", 1)):
            log(f"serving ({name}) ...")
            serving[name] = serve_run(ctx, db, w, thr, args.serve_requests, warm, args.serve_rate, policy,
                                      n_chunks=args.serve_chunks, tick_chunks=args.tick_chunks)
            log(f"serving {name}: {serving[name]}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        cpu = cpu_baseline(w, args.cpu_sample_queries, args.cpu_sample_refs,
                           min(args.cpu_packed_refs, n_refs))

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "comparisons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[used],
        "data": "synthetic (seeded generator shaped like the paper's workload)",
        "config": {"workload": w.name, "n_queries": w.n_q, "n_refs": n_refs, "n_loci": L,
                   "k": w.k, "tiles": "64 x 256x256", "mode": "mixture (R AND NOT M)",
                   "backend": used,
                   "db_build_ms": round(t_build * 1e3, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)
    db.close()
    ctx.close()


# ----------------------------------------------------------------------------- full matrix, small
def bench_full_small(args):
    """64 mixture queries x 20,000 references x 2,048 loci, the full int32
    count matrix (5.12 MB) per call: a launch-latency-bound size, reported as
    absolute time per call (HIP events over many back-to-back calls) beside
    the kernel's own time and roofline fraction."""
    import numpy as np
    import torch

    import gen
    from gen.workloads import MIX_64x20K as w
    from paper_1707_00516_amd import (fid_backend_for, fid_ctx_enable_timing, fid_ctx_scan_time)
    from paper_1707_00516_amd.torch_api import Context
    torch.cuda.init()
    ctx = Context(0)
    thr = gen.maf_thresholds(w.seed, w.n_loci, w.maf_lo)
    refs = gen.ref_bytes(w.seed, thr, 0, w.n_refs)
    db = ctx.build_db(ctx.pack(torch.from_numpy(refs).cuda()), w.n_loci)
    M = gen.mixtures(w.seed, thr, 0, w.n_refs, 0, w.n_q, w.nc_lo, w.nc_hi, w.flip)[0]
    q = ctx.pack(torch.from_numpy(M).cuda())
    out = torch.empty((w.n_q, w.n_refs), dtype=torch.int32, device="cuda")
    ctx.sync()
    calls = max(1, args.steps) * 100
    for _ in range(max(1, args.warmup) * 20):
        ctx.compare_full(db, q, w.mode, out=out)
    ctx.sync()
    fid_ctx_enable_timing(ctx.handle, True)
    fid_ctx_scan_time(ctx.handle, reset=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(ctx.stream)
    for _ in range(calls):
        ctx.compare_full(db, q, w.mode, out=out)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / calls
    scan_ms, launches = fid_ctx_scan_time(ctx.handle, reset=True)
    fid_ctx_enable_timing(ctx.handle, False)
    import oracle
    exact = bool(np.array_equal(out.cpu().numpy(), oracle.counts(refs, M, w.mode)))
    used = BACKEND_NAMES[fid_backend_for(ctx.handle, db.handle, w.n_q)]
    comps = w.n_q * w.n_refs * w.n_loci
    roof = roofline_for(used, comps, scan_ms / max(launches, 1) / 1e3)
    roof["kernel"] = roof["kernel"].split(" (")[0] + " (full-matrix epilogue)"
    line = {
        "metric": "time per call (ms): 64x20000x2048 full int32 count matrix",
        "value": ms,
        "unit": "ms per call",
        "n_gpus": 1, "steps": calls, "warmup": max(1, args.warmup) * 20,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[used],
        "data": "synthetic (seeded generator shaped like the paper's workload)",
        "config": {"workload": w.name, "n_queries": w.n_q, "n_refs": w.n_refs, "n_loci": w.n_loci,
                   "output": "full int32 matrix (5.12 MB)", "backend": used},
        "comparisons_per_s": comps / (ms / 1e3),
        "equals_oracle": exact,
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    db.close()
    ctx.close()


# ----------------------------------------------------------------------------- serving
SERVE_SEED_STREAM_ROW = 1 << 30  # generator rows of the request table (stream 4)


def serving_requests(seed: int, n: int, rate: float, q_max: int = 256):
    """Seeded open-loop request table: Poisson arrival offsets (ns), query
    counts uniform in 1..q_max, modes 50/50."""
    import math

    import gen
    t, out = 0.0, []
    for i in range(n):
        u = gen.u64s(seed, 4, SERVE_SEED_STREAM_ROW + i, 3)
        t += -math.log(1.0 - (int(u[0]) >> 11) / 9007199254740992.0) / rate
        out.append((int(t * 1e9), 1 + int(u[1] % q_max), int(u[2] % 2)))
    return out


def serve_run(ctx, db, w, thr, n_req: int, warm: int, rate: float, policy: int, k: int = 32,
              budget: int = 16 << 30, max_queries: int = 4096, n_chunks: int = 8, tick_chunks: int = 0):
    """Open-loop serving of a seeded request stream; latency is measured from
    each request's scheduled arrival to its completion on the server."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import gen
    from paper_1707_00516_amd.torch_api import Server
    table = serving_requests(w.seed, n_req, rate)

    def make(i):
        _, nq, mode = table[i]
        row0 = (SERVE_SEED_STREAM_ROW >> 4) + (i << 9)
        if mode == 0:
            return gen.mixtures(w.seed, thr, 0, db.n_refs, row0, nq, w.nc_lo, w.nc_hi, w.flip)[0]
        return gen.identity(w.seed, thr, 0, db.n_refs, row0, nq, w.flip)[0]
    with ThreadPoolExecutor(16) as ex:
        Qs = list(ex.map(make, range(n_req)))
    qs = [ctx.pack(torch.from_numpy(Q).cuda()) for Q in Qs]
    del Qs
    ctx.sync()
    srv = Server(ctx, db, budget, max_queries, k, n_chunks, policy, tick_chunks)
    # warm the server's kernels and scratch once outside the schedule
    srv.wait(srv.submit(qs[0], table[0][2]))
    t0 = time.monotonic_ns() + 20_000_000
    sched = [t0 + off for off, _, _ in table]
    done = {}
    outstanding = {}
    i = 0
    while i < n_req or outstanding:
        now = time.monotonic_ns()
        while i < n_req and sched[i] <= now:
            outstanding[srv.submit(qs[i], table[i][2])] = i
            i += 1
        for t in list(outstanding):
            r = srv.poll(t)
            if r is not None:
                done[outstanding.pop(t)] = r[2][2]
        if i < n_req and not outstanding:
            time.sleep(max(0.0, (sched[i] - time.monotonic_ns()) / 1e9 - 0.0002))
    st = srv.stats()
    srv.close()
    lat = np.array([(done[j] - sched[j]) / 1e6 for j in range(warm, n_req)])
    comps = sum(table[j][1] for j in range(warm, n_req)) * db.n_refs * db.n_loci
    span = (max(done[j] for j in range(warm, n_req)) - sched[warm]) / 1e9
    return {"policy": "continuous" if policy == 0 else "fifo", "rate_per_s": rate,
            "requests": n_req - warm, "warmup_requests": warm, "k": k,
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "served_comparisons_per_s": comps / span,
            "n_chunks": n_chunks if policy == 0 else 1,
            "tick_chunks": ("whole database" if tick_chunks == 0 else tick_chunks) if policy == 0 else 1,
            "ticks": st["ticks"],
            "mean_tick_ms": round(st["tick_ms_total"] / max(st["ticks"], 1), 4),
            "mean_queries_per_tick": round(st["tick_queries_total"] / max(st["ticks"], 1), 1),
            "peak_queries_in_flight": st["peak_queries_in_flight"]}


def bench_serving(args):
    """Serving on the resident 20M x 2048 database: continuous batching and
    FIFO per-call serving of the same seeded request stream."""
    import torch

    import gen
    from gen.workloads import MIX_2048x20M as w
    from paper_1707_00516_amd.torch_api import Context
    n_refs = args.n_refs or w.n_refs
    torch.cuda.init()
    ctx = Context(0)
    thr = gen.maf_thresholds(w.seed, w.n_loci, w.maf_lo)
    db = gpu_panel_db(ctx, w.seed, thr, n_refs)
    n, warm = args.serve_requests, min(200, args.serve_requests // 5)
    res, stress = {}, {}
    for name in args.serve_policies.split(","):
        policy = {"continuous": 0, "fifo": 1}[name]
        res[policy] = serve_run(ctx, db, w, thr, n, warm, args.serve_rate, policy,
                                n_chunks=args.serve_chunks, tick_chunks=args.tick_chunks)
        log(f"serving policy {policy}: {res[policy]}")
    if args.serve_stress_rate > 0:
        ns = min(n, 800)
        for name in args.serve_policies.split(","):
            policy = {"continuous": 0, "fifo": 1}[name]
            stress[name] = serve_run(ctx, db, w, thr, ns, min(100, ns // 5), args.serve_stress_rate,
                                     policy, n_chunks=args.serve_chunks, tick_chunks=args.tick_chunks)
            log(f"serving policy {policy} at {args.serve_stress_rate}/s: {stress[name]}")
    c = res.get(0) or res[1]
    line = {
        "metric": "served p50/p99 latency (ms) and served comparisons/s, 20Mx2048 resident",
        "value": c["p99_ms"],
        "unit": "ms (p99)",
        "n_gpus": 1,
        "steps": n - warm,
        "warmup": warm,
        "ms_per_step": c["mean_ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed (per-call backend)",
        "data": "synthetic (seeded generator shaped like the paper's workload)",
        "config": {"workload": "serving-20Mx2048-poisson", "n_refs": n_refs, "n_loci": w.n_loci,
                   "rate_per_s": args.serve_rate, "queries_per_request": "U{1..256}",
                   "modes": "identity/mixture 50/50", "k": 32},
        "continuous": res.get(0),
        "fifo": res.get(1),
        "stress": stress or None,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    db.close()
    ctx.close()


# ----------------------------------------------------------------------------- large panel
def bench_large_panel(args):
    """256 mixtures x 2M references x 32768 loci: per-query threshold hits
    (count <= floor(2 L / 100)) plus top-32, one step = both outputs."""
    import numpy as np
    import torch

    import gen
    from gen.workloads import MIX_256x2Mx32K as w, threshold_2pct
    from paper_1707_00516_amd import (fid_backend_for, fid_ctx_enable_timing, fid_ctx_scan_time)
    from paper_1707_00516_amd.torch_api import Context
    n_refs = args.n_refs or w.n_refs
    torch.cuda.init()
    ctx = Context(0)
    t0 = time.perf_counter()
    thr = gen.maf_thresholds(w.seed, w.n_loci, w.maf_lo)
    db = gpu_panel_db(ctx, w.seed, thr, n_refs)
    M, contrib, ncon, F = gen.mixtures(w.seed, thr, 0, n_refs, 0, w.n_q, w.nc_lo, w.nc_hi, w.flip)
    q = ctx.pack(torch.from_numpy(M).cuda())
    T = threshold_2pct(w.n_loci)
    thr_q = torch.full((w.n_q,), T, dtype=torch.int32, device="cuda")
    ws = ctx.topk_workspace(db, w.n_q, w.k)
    ctx.sync()
    log(f"setup {time.perf_counter() - t0:.1f}s")
    cap = [1 << 16]

    from paper_1707_00516_amd import fid_threshold_topk_workspace_bytes
    ws_both = [torch.empty(fid_threshold_topk_workspace_bytes(ctx.handle, db.handle, w.n_q, w.k, cap[0]),
                           dtype=torch.uint8, device="cuda")]

    def step():
        # one pass: threshold hits and top-32 from the same scan
        offs, idx, cnt, c, i = ctx.compare_threshold_topk(db, q, w.mode, thr_q, w.k, cap=cap[0], ws=ws_both[0])
        if idx.numel() > cap[0]:
            cap[0] = int(idx.numel())
            ws_both[0] = torch.empty(fid_threshold_topk_workspace_bytes(ctx.handle, db.handle, w.n_q, w.k, cap[0]),
                                     dtype=torch.uint8, device="cuda")
        return offs, idx, cnt, c, i

    def two_calls():
        offs, idx, cnt = ctx.compare_threshold(db, q, w.mode, thr_q, cap=cap[0])
        c, i = ctx.compare_topk(db, q, w.mode, w.k, ws=ws)
        return offs, idx, cnt, c, i

    for _ in range(args.warmup):
        step()
    ctx.sync()
    fid_ctx_enable_timing(ctx.handle, True)
    fid_ctx_scan_time(ctx.handle, reset=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(ctx.stream)
    for _ in range(args.steps):
        out = step()
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    scan_ms, launches = fid_ctx_scan_time(ctx.handle, reset=True)
    fid_ctx_enable_timing(ctx.handle, False)
    # the same outputs from two calls (a threshold scan, then a top-k scan)
    two = two_calls()
    same = all(bool(torch.equal(a, b)) for a, b in zip(two, out))
    torch.cuda.synchronize()
    ev0.record(ctx.stream)
    for _ in range(args.steps):
        two_calls()
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    two_ms = ev0.elapsed_time(ev1) / args.steps
    log(f"two calls: {two_ms:.2f} ms per step; one-pass output equals theirs: {same}")
    offs, idx, cnt, c, i = [t.cpu().numpy() for t in out]
    # planted contributors: found among the hits and the top-32 (statistical check)
    found_hit = found_top = total = 0
    for qi in range(w.n_q):
        hits = set(idx[offs[qi]:offs[qi + 1]].tolist())
        top = set(i[qi].tolist())
        for r in contrib[qi][:ncon[qi]]:
            total += 1
            found_hit += int(r) in hits
            found_top += int(r) in top
    comps = w.n_q * n_refs * w.n_loci
    ms = total_ms / args.steps
    used = BACKEND_NAMES[fid_backend_for(ctx.handle, db.handle, w.n_q)]
    # one scan per step carries both epilogues
    roof = roofline_for(used, comps, scan_ms / max(launches, 1) / 1e3)
    roof["kernel"] = roof["kernel"].split(" (")[0] + " (threshold + top-k epilogue in one scan, chunked rows)"
    roof["launches_per_step"] = launches / args.steps
    add_measured_peak(roof, used, None if args.no_peaks else measure_peaks(ctx))
    line = {
        "metric": "query-ref-locus comparisons/s at 256x2Mx32768 loci (threshold + top-32)",
        "value": comps / (ms / 1e3),
        "unit": "comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[used],
        "data": "synthetic (seeded generator shaped like the paper's workload)",
        "config": {"workload": w.name, "n_queries": w.n_q, "n_refs": n_refs, "n_loci": w.n_loci,
                   "threshold": T, "k": w.k, "backend": used},
        "hits_total": int(offs[-1]),
        "two_call_ms_per_step": round(two_ms, 3),
        "one_pass_equals_two_calls": same,
        "contributors_in_hits": f"{found_hit}/{total}",
        "contributors_in_top32": f"{found_top}/{total}",
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    db.close()
    ctx.close()


# ----------------------------------------------------------------------------- ragged batches
def gpu_panel_db(ctx, seed: int, thr, n_refs: int, chunk_bytes: int = 1 << 31):
    """Reference rows 0..n_refs-1 of one panel generated on the device,
    packed by libfastid and built into a resident database."""
    import numpy as np
    import torch

    import gen
    from paper_1707_00516_amd import fid_row_words
    L = thr.size
    stream = torch.cuda.current_stream()
    thr_dev = torch.from_numpy(thr.astype(np.uint32)).cuda()
    rows = torch.empty((n_refs, fid_row_words(L)), dtype=torch.int64, device="cuda")
    chunk = max(1, min(n_refs, chunk_bytes // L))
    buf = torch.empty((chunk, L), dtype=torch.uint8, device="cuda")
    for r0 in range(0, n_refs, chunk):
        n = min(chunk, n_refs - r0)
        gen.ref_bytes_gpu(seed, thr_dev.data_ptr(), L, r0, n, buf.data_ptr(), L, stream.cuda_stream)
        ctx.pack(buf[:n], L, out=rows[r0:r0 + n])
    del buf
    db = ctx.build_db(rows, L)
    ctx.sync()
    del rows
    torch.cuda.empty_cache()
    return db


def bench_streamed(args):
    """The headline top-32 (2048 x 20M x 2048, mixture) with the database in
    pinned host memory, streamed through the device a block at a time (the
    paper's host driver); PCIe-inclusive, beside the same call on the
    resident database."""
    import numpy as np
    import torch

    import gen
    from gen.workloads import MIX_2048x20M as w
    from paper_1707_00516_amd import (fid_backend_for, fid_ctx_enable_timing, fid_ctx_scan_time, fid_row_words,
                                      fid_stream_workspace_bytes)
    from paper_1707_00516_amd.torch_api import Context

    n_refs = args.n_refs or w.n_refs
    L = w.n_loci
    torch.cuda.init()
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    thr = gen.maf_thresholds(w.seed, L, w.maf_lo)
    thr_dev = torch.from_numpy(thr.astype(np.uint32)).cuda()
    rw = fid_row_words(L)
    rows_host = torch.empty((n_refs, rw), dtype=torch.int64, pin_memory=not args.pageable)
    chunk = 1 << 20
    buf = torch.empty((min(chunk, n_refs), L), dtype=torch.uint8, device="cuda")
    rows = torch.empty((min(chunk, n_refs), rw), dtype=torch.int64, device="cuda")
    for r0 in range(0, n_refs, chunk):
        n = min(chunk, n_refs - r0)
        gen.ref_bytes_gpu(w.seed, thr_dev.data_ptr(), L, r0, n, buf.data_ptr(), L, stream.cuda_stream)
        ctx.pack(buf[:n], L, out=rows[:n])
        rows_host[r0:r0 + n].copy_(rows[:n])
    del buf, rows
    M = gen.mixtures(w.seed, thr, 0, n_refs, 0, w.n_q, w.nc_lo, w.nc_hi, w.flip)[0]
    q = ctx.pack(torch.from_numpy(M).cuda())
    ws = torch.empty(fid_stream_workspace_bytes(ctx.handle, n_refs, L, args.block_refs, w.n_q, w.k),
                     dtype=torch.uint8, device="cuda")
    ctx.sync()
    log(f"streamed: {n_refs} rows ({rows_host.numel() * 8 / 1e9:.2f} GB {'pageable' if args.pageable else 'pinned'}), "
        f"blocks of {args.block_refs}")
    for i in range(args.warmup):
        ctx.compare_topk_streamed(rows_host, L, args.block_refs, q, w.mode, w.k, ws=ws)
        log(f"warmup {i + 1}/{args.warmup} done")
    fid_ctx_enable_timing(ctx.handle, True)
    fid_ctx_scan_time(ctx.handle, reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cnt, idx = ctx.compare_topk_streamed(rows_host, L, args.block_refs, q, w.mode, w.k, ws=ws)
    ms = (time.perf_counter() - t0) * 1e3 / args.steps  # each call synchronises
    scan_ms, launches = fid_ctx_scan_time(ctx.handle, reset=True)
    fid_ctx_enable_timing(ctx.handle, False)
    log(f"timed {args.steps} streamed calls: {ms:.1f} ms each; scan kernels {scan_ms:.1f} ms over {launches}")
    # the same rows resident, for the check and the comparison
    rows_dev = rows_host.cuda()
    db = ctx.build_db(rows_dev, L)
    ctx.sync()
    del rows_dev
    rc, ri = ctx.compare_topk(db, q, w.mode, w.k)
    same = bool(torch.equal(rc, cnt) and torch.equal(ri, idx))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.compare_topk(db, q, w.mode, w.k)
    ev1.record(stream)
    torch.cuda.synchronize()
    resident_ms = ev0.elapsed_time(ev1) / args.steps
    log(f"resident database: {resident_ms:.1f} ms per call; streamed == resident: {same}")
    comps = w.n_q * n_refs * L
    used = BACKEND_NAMES[fid_backend_for(ctx.handle, db.handle, w.n_q)]
    h2d_bytes = rows_host.numel() * 8
    n_blocks = -(-n_refs // args.block_refs)
    scan_s = scan_ms / max(launches, 1) / 1e3
    roof = roofline_for(used, w.n_q * min(args.block_refs, n_refs) * L, scan_s)
    roof["kernel"] += f", one {min(args.block_refs, n_refs)}-reference block"
    line = {
        "metric": "query-ref-locus comparisons/s at 2048x20Mx2048 loci, database streamed from host memory",
        "value": comps / (ms / 1e3),
        "unit": "comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[used],
        "data": "synthetic (seeded generator shaped like the paper's workload)",
        "config": {"workload": "mixture-2048x20Mx2048-top32-streamed" + ("-pageable" if args.pageable else ""),
                   "n_queries": w.n_q, "n_refs": n_refs,
                   "n_loci": L, "k": w.k, "block_refs": args.block_refs, "blocks": n_blocks,
                   "host_memory": "pageable" if args.pageable else "pinned", "backend": used},
        "h2d": {"bytes": h2d_bytes, "GB_per_s": round(h2d_bytes / (ms / 1e3) / 1e9, 2)},
        "resident_ms_per_step": round(resident_ms, 3),
        "streamed_equals_resident": same,
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    db.close()
    ctx.close()


def bench_streamed_full(args):
    """The paper's own pipeline (Section III-C): 2048 queries x 1M references
    x 2048 loci, references streamed in from pinned host memory and the full
    int32 count matrix (8.19 GB) streamed back out to pinned host memory."""
    import numpy as np
    import torch

    import gen
    from gen.workloads import MIX_2048x20M as w
    from paper_1707_00516_amd import fid_full_stream_workspace_bytes, fid_row_words
    from paper_1707_00516_amd.torch_api import Context

    n_refs = args.n_refs or 1_000_000
    block = min(args.block_refs, 131_072)
    L = w.n_loci
    torch.cuda.init()
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    thr = gen.maf_thresholds(w.seed, L, w.maf_lo)
    thr_dev = torch.from_numpy(thr.astype(np.uint32)).cuda()
    rw = fid_row_words(L)
    buf = torch.empty((n_refs, L), dtype=torch.uint8, device="cuda")
    gen.ref_bytes_gpu(w.seed, thr_dev.data_ptr(), L, 0, n_refs, buf.data_ptr(), L, stream.cuda_stream)
    rows = torch.empty((n_refs, rw), dtype=torch.int64, device="cuda")
    ctx.pack(buf, L, out=rows)
    rows_host = torch.empty((n_refs, rw), dtype=torch.int64, pin_memory=True)
    rows_host.copy_(rows)
    del buf
    M = gen.mixtures(w.seed, thr, 0, n_refs, 0, w.n_q, w.nc_lo, w.nc_hi, w.flip)[0]
    q = ctx.pack(torch.from_numpy(M).cuda())
    out = torch.empty((w.n_q, n_refs), dtype=torch.int32, pin_memory=True)
    ws = torch.empty(fid_full_stream_workspace_bytes(ctx.handle, n_refs, L, block, w.n_q), dtype=torch.uint8,
                     device="cuda")
    ctx.sync()
    log(f"streamed full: {n_refs} rows in, {out.numel() * 4 / 1e9:.2f} GB of counts out, blocks of {block}")
    for _ in range(args.warmup):
        ctx.compare_full_streamed(rows_host, L, block, q, w.mode, out=out, ws=ws)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.compare_full_streamed(rows_host, L, block, q, w.mode, out=out, ws=ws)
    ms = (time.perf_counter() - t0) * 1e3 / args.steps  # each call synchronises
    # resident comparison: the same matrix computed into device memory
    db = ctx.build_db(rows, L)
    dev = torch.empty((w.n_q, n_refs), dtype=torch.int32, device="cuda")
    ctx.compare_full(db, q, w.mode, out=dev)
    ctx.sync()
    same = bool(torch.equal(dev.cpu(), out))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.compare_full(db, q, w.mode, out=dev)
    ev1.record(stream)
    torch.cuda.synchronize()
    resident_ms = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} calls: {ms:.1f} ms each; resident full matrix {resident_ms:.1f} ms; equal: {same}")
    comps = w.n_q * n_refs * L
    d2h = out.numel() * 4
    h2d = rows_host.numel() * 8
    line = {
        "metric": "query-ref-locus comparisons/s at 2048x1Mx2048 loci, full matrix, streamed in and out of host memory",
        "value": comps / (ms / 1e3),
        "unit": "comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed (per-call backend)",
        "data": "synthetic (seeded generator shaped like the paper's workload)",
        "config": {"workload": "mixture-2048x1Mx2048-full-streamed", "n_queries": w.n_q, "n_refs": n_refs,
                   "n_loci": L, "block_refs": block, "host_memory": "pinned"},
        "h2d_bytes": h2d, "d2h_bytes": d2h,
        "pcie_GB_per_s": round((h2d + d2h) / (ms / 1e3) / 1e9, 2),
        "resident_ms_per_step": round(resident_ms, 3),
        "streamed_equals_resident": same,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    db.close()
    ctx.close()


def bench_ragged(args):
    from concurrent.futures import ThreadPoolExecutor

    import torch

    import gen
    from gen.workloads import RAGGED_SEED, ragged_jobs, ragged_panel_seed, ragged_queries
    from paper_1707_00516_amd import autotune, fid_ctx_enable_timing, fid_ctx_scan_time
    from paper_1707_00516_amd.torch_api import Batch, Context

    k = 32
    pool = args.n_refs or 2_000_000
    jobs = ragged_jobs(args.jobs, pool=pool)
    comps = sum(j.comparisons for j in jobs)
    torch.cuda.init()
    ctx = Context(0)
    t0 = time.perf_counter()
    panels, thrs = {}, {}
    for L in sorted({j.n_loci for j in jobs}):
        ps = ragged_panel_seed(RAGGED_SEED, L)
        thrs[L] = gen.maf_thresholds(ps, L, 0.05)
        panels[L] = gpu_panel_db(ctx, ps, thrs[L], pool)
        log(f"panel L={L}: {pool} references resident")
    with ThreadPoolExecutor(16) as ex:
        Qs = list(ex.map(lambda j: ragged_queries(j, thrs[j.n_loci]), jobs))
    q_rows = [ctx.pack(torch.from_numpy(Q).cuda()) for Q in Qs]
    del Qs
    ctx.sync()
    log(f"setup {time.perf_counter() - t0:.1f}s: {len(jobs)} jobs, {comps:.3e} comparisons")

    if args.tune:
        def queries_for(L, r_lo, r_hi, n_q, mode, row0):
            ps = ragged_panel_seed(RAGGED_SEED, L)
            if mode == 0:
                Q = gen.mixtures(ps, thrs[L], r_lo, r_hi - r_lo, row0, n_q, 1, 4, 0.005)[0]
            else:
                Q = gen.identity(ps, thrs[L], r_lo, r_hi - r_lo, row0, n_q, 0.005)[0]
            return ctx.pack(torch.from_numpy(Q).cuda())
        table, report = autotune.tune(ctx, panels, queries_for, k=k, log=log)
        log(f"tuned table (sample batches): {table}")
        spec0 = [(panels[j.n_loci], j.r_lo, j.r_hi, q_rows[i], j.mode) for i, j in enumerate(jobs)]
        table, report2 = autotune.refine_fp4_on_batch(ctx, spec0, k, table, log=log)
        report.update(report2)
        os.makedirs("gpurun_out", exist_ok=True)
        autotune.save_table(table, {"report_ms": report}, os.path.join("gpurun_out", "tune_table.json"))
        log(f"tuned table: {table}")
    else:
        table = autotune.load_table()
    spec = [(panels[j.n_loci], j.r_lo, j.r_hi, q_rows[i], j.mode) for i, j in enumerate(jobs)]
    b = Batch(ctx, spec, k, table)
    n_items, n_lists, grid, n_routed = b.info()
    log(f"batch: {n_items} items, {n_lists} lists, {grid} persistent workgroups, "
        f"{n_routed} jobs on the matrix cores (batched fp4 passes)")

    def timed(fn, steps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(ctx.stream)
        for _ in range(steps):
            fn()
        ev1.record(ctx.stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    for _ in range(args.warmup):
        b.run()
    ctx.sync()
    batch_ms = timed(b.run, args.steps)
    log(f"batch eager: {batch_ms:.2f} ms per run")
    # each persistent pass alone, timed with the library's events: the
    # popcount pass (the jobs the plan keeps on the popcount scan) and the
    # batched fp4 top-k pass (the matrix-core jobs; those no longer than the
    # 16,384-reference seed prefix are counted in the seed pass instead)
    def pass_time(idx):
        bp = Batch(ctx, [spec[i] for i in idx], k, table)
        bp.run()
        ctx.sync()
        fid_ctx_enable_timing(ctx.handle, True)
        fid_ctx_scan_time(ctx.handle, reset=True)
        for _ in range(max(1, args.steps)):
            bp.run()
        ctx.sync()
        ms_, n_ = fid_ctx_scan_time(ctx.handle, reset=True)
        fid_ctx_enable_timing(ctx.handle, False)
        bp.close()
        return ms_ / max(n_, 1) / 1e3
    small = [i for i in range(len(jobs)) if not b.routed(i)]
    mc = [i for i in range(len(jobs)) if b.routed(i)]
    persistent_comps = sum(jobs[i].comparisons for i in small)
    fp4_comps = sum(jobs[i].comparisons for i in mc if jobs[i].r_hi - jobs[i].r_lo > 16384)
    scan_s = pass_time(small) if small else None
    fp4_s = pass_time(mc) if mc else None
    if scan_s:
        log(f"persistent popcount pass: {len(small)} jobs, {persistent_comps:.3e} comparisons, "
            f"{scan_s * 1e3:.2f} ms")
    if fp4_s:
        log(f"batched fp4 top-k pass: {len(mc)} jobs, {fp4_comps:.3e} comparisons, {fp4_s * 1e3:.2f} ms")
    b.run(use_graph=True)
    graph_ms = timed(lambda: b.run(use_graph=True), args.steps)
    log(f"batch graph: {graph_ms:.2f} ms per run")

    per_call_ms, parity = None, None
    if not args.no_per_call:
        ws_bytes = max(ctx.topk_range_workspace(d, lo, hi, q.shape[0], k).numel()
                       for d, lo, hi, q, m in spec)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        outs = [(torch.empty((q.shape[0], k), dtype=torch.int32, device="cuda"),
                 torch.empty((q.shape[0], k), dtype=torch.int64, device="cuda"))
                for d, lo, hi, q, m in spec]

        def per_call():
            for (d, lo, hi, q, m), o in zip(spec, outs):
                ctx.compare_topk_range(d, lo, hi, q, m, k, ws=ws, out=o)
        per_call()
        per_call_ms = timed(per_call, max(1, args.steps // 2))
        parity = all(torch.equal(o[0], c) and torch.equal(o[1], i)
                     for o, c, i in zip(outs, b.cnt, b.idx))
        log(f"per-job calls: {per_call_ms:.2f} ms per pass; batch == per-call: {parity}")

    roof = None
    if fp4_s:
        roof = roofline_for("mfma_fp4", fp4_comps, fp4_s)
        roof["kernel"] = (f"fp4_batch_kernel<top-k> (persistent, the {len(mc)} matrix-core jobs, "
                          f"{fp4_comps:.3e} comparisons)")
        if len(jobs) == 400 and pool == 2_000_000 and not args.tune:
            roof["traffic"] = recorded_traffic("fp4_batch_kernel<1>")
    popcount_pass = None
    if scan_s:
        popcount_pass = roofline_for("popcount", persistent_comps, scan_s)
        popcount_pass["kernel"] = (f"batch_scan_kernel (persistent, the {len(small)} jobs kept on the "
                                   f"popcount scan, {persistent_comps:.3e} comparisons)")
    line = {
        "metric": "ragged-batch top-32 comparisons/s (400 jobs in one batch run)",
        "value": comps / (batch_ms / 1e3),
        "unit": "comparisons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(batch_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("u32 (persistent popcount) + " if small else "")
                 + "fp4-e2m1 0/1-coded, f32 accumulate (batched matrix-core passes); exact integer counts",
        "data": "synthetic (seeded generator shaped like the paper's workload)",
        "config": {"workload": "ragged-400", "jobs": len(jobs), "comparisons": comps,
                   "k": k, "pool_refs": pool, "panels": sorted(panels), "tune": table,
                   "items": n_items, "jobs_routed_to_matrix_cores": n_routed},
        "graph_ms_per_step": round(graph_ms, 3),
        "per_call_ms_per_pass": None if per_call_ms is None else round(per_call_ms, 3),
        "speedup_vs_per_call": None if per_call_ms is None else round(per_call_ms / batch_ms, 3),
        "parity_vs_per_call": parity,
        "roofline": roof,
        "popcount_pass": popcount_pass,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    b.close()
    for d in panels.values():
        d.close()
    ctx.close()


if __name__ == "__main__":
    main()
