"""Work-item autotuner for ragged batches.

For every loci panel it times whole batches of seeded synthetic jobs of that
panel over a grid of item shapes and keeps the fastest: the popcount items
(queries per item x 64-reference blocks per item) with the popcount backend
forced on the context, and the fp4 items (512-reference tiles per item) with
the fp4 backend, which AUTO gives every job.  The resulting table (a list of
``(n_loci, q_per_item, blocks_per_item, fp4_tiles)`` rows, the ``fid_tune``
records of the C ABI) is stored as JSON beside this module and passed to
``fid_batch_create``.

Timing uses HIP events on the context's stream around whole batch runs; the
jobs are cheap to plan, so each candidate is planned afresh.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")

Q_CANDIDATES = (8, 16, 32)
BLOCK_CANDIDATES = (32, 128, 512)
FP4_TILE_CANDIDATES = (32, 64, 128, 256, 512)


def load_table(path: str = TABLE_PATH):
    """The stored table, or None if there is none."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rows = json.load(f)["table"]
    return [tuple(int(v) for v in r) for r in rows]


def save_table(table, meta: dict, path: str = TABLE_PATH) -> None:
    with open(path, "w") as f:
        json.dump({"table": [list(r) for r in table], "meta": meta}, f, indent=1)
        f.write("\n")


def _time_batch(ctx, jobs, k, tune, reps, backend):
    from . import fid_ctx_set_backend
    from .torch_api import Batch
    fid_ctx_set_backend(ctx.handle, backend)   # the plan keeps its routing
    try:
        b = Batch(ctx, jobs, k, tune)
    finally:
        fid_ctx_set_backend(ctx.handle, 0)
    b.run()
    ctx.sync()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(ctx.stream)
    for _ in range(reps):
        b.run()
    ev1.record(ctx.stream)
    ev1.synchronize()
    b.close()
    return ev0.elapsed_time(ev1) / reps


def tune(ctx, panels: dict, queries_for, k: int = 32, n_jobs: int = 12, reps: int = 2,
         seed: int = 17, q_candidates=Q_CANDIDATES, block_candidates=BLOCK_CANDIDATES,
         fp4_tile_candidates=FP4_TILE_CANDIDATES, max_refs: int = 2_000_000, log=print):
    """Tune every panel.  ``panels`` maps n_loci -> Database; ``queries_for(L,
    r_lo, r_hi, n_q, mode, row0)`` returns packed device query rows drawn from
    that slice.  The popcount item shape (queries x blocks) is tuned first,
    then, with it, the fp4 item length (512-reference tiles per item).
    Returns (table, report): rows (n_loci, q_per_item, blocks_per_item,
    fp4_tiles)."""
    import gen
    table, report = [], {}
    for L, db in sorted(panels.items()):
        n = min(db.n_refs, max_refs)
        u = gen.u64s(seed + L, 4, 1 << 20, 4 * n_jobs)
        jobs = []
        for j in range(n_jobs):
            n_q = 1 + int(u[4 * j] % 512)
            n_r = max(1000, int(u[4 * j + 1] % n) + 1)
            r_lo = int(u[4 * j + 2] % (db.n_refs - n_r + 1))
            mode = int(u[4 * j + 3] % 2)
            q = queries_for(L, r_lo, r_lo + n_r, n_q, mode, (1 << 20) + j * 1024)
            jobs.append((db, r_lo, r_lo + n_r, q, mode))
        comps = sum(j[3].shape[0] * (j[2] - j[1]) for j in jobs) * L
        best = None
        for qpi in q_candidates:
            for bpi in block_candidates:
                ms = _time_batch(ctx, jobs, k, [(L, qpi, bpi, 0)], reps, backend=1)
                report[f"{L}/{qpi}/{bpi}"] = ms
                log(f"tune L={L} q_per_item={qpi} blocks_per_item={bpi}: {ms:.3f} ms "
                    f"({comps * 1e3 / ms:.3e} comps/s)")
                if best is None or ms < best[0]:
                    best = (ms, qpi, bpi)
        best_t = None
        for t in fp4_tile_candidates:
            ms = _time_batch(ctx, jobs, k, [(L, best[1], best[2], t)], reps, backend=3)
            report[f"{L}/{best[1]}/{best[2]}/fp4:{t}"] = ms
            log(f"tune L={L} fp4_tiles={t}: {ms:.3f} ms ({comps * 1e3 / ms:.3e} comps/s)")
            if best_t is None or ms < best_t[0]:
                best_t = (ms, t)
        table.append((L, best[1], best[2], best_t[1]))
    return table, report


def refine_fp4_on_batch(ctx, jobs, k, table, candidates=FP4_TILE_CANDIDATES, reps: int = 2, log=print):
    """The fp4 item length of every panel re-tuned on the whole batch it will
    serve (``jobs``: the batch's job tuples): one panel at a time, the others
    held at their current entries, keeping the length that runs the whole
    batch fastest.  Small sample batches favour short items (finer load
    balance), which a batch of hundreds of jobs does not need.  Returns the
    refined table and a report."""
    table = [tuple(r) + (0,) * (4 - len(r)) for r in table]
    report = {}
    for i, row in enumerate(table):
        best = None
        for t in candidates:
            trial = list(table)
            trial[i] = (row[0], row[1], row[2], t)
            ms = _time_batch(ctx, jobs, k, trial, reps, backend=0)
            report[f"batch/{row[0]}/fp4:{t}"] = ms
            log(f"refine L={row[0]} fp4_tiles={t}: whole batch {ms:.3f} ms")
            if best is None or ms < best[0]:
                best = (ms, t)
        table[i] = (row[0], row[1], row[2], best[1])
    return table, report

