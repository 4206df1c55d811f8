"""Ragged batch at the workload's scale, against the CPU checkers.

The jobs come from the 400-job ragged table itself (1-512 queries, slices of
10k-2M references of a 2M-reference pool per panel, panels 1024-16384 loci,
modes 50/50): its 20 smallest jobs plus 4 seeded jobs of every panel, run as
one batch exactly as the benchmark plans it (autotuned item shapes,
matrix-core routing), eagerly and replayed from a HIP graph.

* the 20 smallest jobs: the byte oracle's top-k of every query's full row;
* every job: the packed x86 baseline's top-k over the job's slice (pinned
  to the byte oracle in tests/test_cpu_packed.py);
* every returned (count, index) pair of every job: the byte oracle's count.
"""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
import oracle.packed as cpu_packed
from gen.workloads import RAGGED_PANELS, RAGGED_SEED, ragged_jobs, ragged_panel_seed, ragged_queries
from gpu_harness import gpu_generated_db, log, pack_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

POOL = 2_000_000
K = 32


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1707_00516_amd.torch_api import Context
    c = Context(0)
    yield c
    c.sync()
    c.close()


def _subset():
    jobs = ragged_jobs(400, pool=POOL)
    smallest = sorted(jobs, key=lambda j: j.comparisons)[:20]
    chosen = {j.index for j in smallest}
    for L in RAGGED_PANELS:
        cand = [j for j in jobs if j.n_loci == L and j.index not in chosen]
        u = gen.u64s(RAGGED_SEED, 5, 11 + L, 8)
        picked = []
        for x in u:
            j = cand[int(x % len(cand))]
            if j.index not in chosen and len(picked) < 4:
                picked.append(j)
                chosen.add(j.index)
    return [j for j in jobs if j.index in chosen], {j.index for j in smallest}


def _oracle_rows(seed, thr, r_lo, r_hi, Q, mode, max_bytes=1 << 30):
    """The byte oracle's counts of queries Q against references [r_lo, r_hi)
    (regenerated on the CPU in chunks), one oracle pair per (query, ref)."""
    L, nq = thr.size, Q.shape[0]
    rows = np.empty((nq, r_hi - r_lo), np.int32)
    chunk = max(1, max_bytes // L)
    for a in range(r_lo, r_hi, chunk):
        n = min(chunk, r_hi - a)
        b = gen.ref_bytes(seed, thr, a, n)
        got = oracle.count_pairs(b, Q, np.tile(np.arange(n), nq), np.repeat(np.arange(nq), n), mode)
        rows[:, a - r_lo:a - r_lo + n] = got.reshape(nq, n)
    return rows


def _packed_pool(seed, thr, n, chunk_bytes=1 << 30):
    L = thr.size
    out = np.empty((n, cpu_packed.words(L)), np.uint64)
    chunk = max(1, chunk_bytes // L)
    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        cpu_packed.pack(gen.ref_bytes(seed, thr, a, m), out=out[a:a + m])
    return out


@pytest.mark.timeout(1200)
def test_ragged_subset_at_scale_matches_cpu_checkers(ctx):
    from paper_1707_00516_amd import autotune
    from paper_1707_00516_amd.torch_api import Batch
    jobs, smallest = _subset()
    assert {j.n_loci for j in jobs} == set(RAGGED_PANELS) and len(jobs) == 40
    log(f"ragged at scale: {len(jobs)} jobs, {sum(j.comparisons for j in jobs):.3e} comparisons")
    thrs, dbs = {}, {}
    for L in RAGGED_PANELS:
        ps = ragged_panel_seed(RAGGED_SEED, L)
        thrs[L] = gen.maf_thresholds(ps, L, 0.05)
        dbs[L] = gpu_generated_db(ctx, ps, thrs[L], POOL)
    Qs = [ragged_queries(j, thrs[j.n_loci]) for j in jobs]
    spec = [(dbs[j.n_loci], j.r_lo, j.r_hi, pack_rows(ctx, Q), j.mode) for j, Q in zip(jobs, Qs)]
    b = Batch(ctx, spec, K, autotune.load_table())
    n_routed = b.info()[3]
    b.run()
    ctx.sync()
    eager = [(c.cpu().numpy(), i.cpu().numpy()) for c, i in zip(b.cnt, b.idx)]
    for rep in range(2):
        for c, i in zip(b.cnt, b.idx):
            c.fill_(-7)
            i.fill_(-7)
        b.run(use_graph=True)
        ctx.sync()
        for j, (c, i) in enumerate(zip(b.cnt, b.idx)):
            assert np.array_equal(c.cpu().numpy(), eager[j][0]) and np.array_equal(i.cpu().numpy(), eager[j][1])
    b.close()
    log(f"ragged at scale: batch run ({n_routed} routed jobs); two graph replays equal the eager run")

    # every returned pair against the byte oracle
    for j, (c, i) in zip(jobs, eager):
        ps = ragged_panel_seed(RAGGED_SEED, j.n_loci)
        Q = Qs[jobs.index(j)]
        assert np.all((i >= j.r_lo) & (i < j.r_hi)) or (j.r_hi - j.r_lo) < K
        real = i >= 0
        rows = gen.ref_rows(ps, thrs[j.n_loci], i[real])
        want = oracle.count_pairs(rows, Q, np.arange(rows.shape[0]), np.nonzero(real)[0], j.mode)
        assert np.array_equal(c[real], want), j.index
        keys = c.astype(np.int64) * (1 << 40) + i
        assert np.all(np.diff(keys, axis=1) > 0), j.index
    log("ragged at scale: every returned pair equals the byte oracle's count")

    # the 20 smallest jobs: full oracle rows
    for j, (c, i) in zip(jobs, eager):
        if j.index not in smallest:
            continue
        ps = ragged_panel_seed(RAGGED_SEED, j.n_loci)
        rows = _oracle_rows(ps, thrs[j.n_loci], j.r_lo, j.r_hi, Qs[jobs.index(j)], j.mode)
        wc, wi = oracle.topk(rows, K)
        assert np.array_equal(c, wc), j.index
        assert np.array_equal(i, np.where(wi >= 0, wi + j.r_lo, -1)), j.index
    log("ragged at scale: the 20 smallest jobs equal the oracle's top-32 of their full rows")

    # every job: the packed baseline over the job's slice
    for L in RAGGED_PANELS:
        ps = ragged_panel_seed(RAGGED_SEED, L)
        pool = _packed_pool(ps, thrs[L], POOL)
        for j, (c, i) in zip(jobs, eager):
            if j.n_loci != L:
                continue
            pc, pi = cpu_packed.topk(pool[j.r_lo:j.r_hi], cpu_packed.pack(Qs[jobs.index(j)]), L, j.mode, K)
            assert np.array_equal(c, pc), j.index
            assert np.array_equal(i, np.where(pi >= 0, pi + j.r_lo, -1)), j.index
        del pool
        log(f"ragged at scale: panel {L} jobs equal the packed baseline")
    for db in dbs.values():
        db.close()
