"""Parity at the full workload sizes, in the launch configuration the
benchmark times.

* Every returned (count, index) pair of every query is recomputed by the
  byte oracle from the reference rows the CPU generator produces for those
  indices; the ordering, range and uniqueness of the keys are checked.
* For a seeded sample of queries the byte oracle computes the whole count
  row over every reference (the database regenerated on the CPU chunk by
  chunk) and its top-k / threshold CSR must equal the GPU's.
* The packed x86 baseline (oracle/packed, pinned to the byte oracle) gives
  the top-k of every query over the whole database: it must equal the GPU's.
* Every true contributor of a sampled mixture (generator bookkeeping) is
  among the results, and sampled 256 x 256 tiles equal the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
import oracle.packed as cpu_packed
from gen.workloads import MIX_2048x20M, MIX_256x2Mx32K, threshold_2pct
from gpu_harness import gpu_generated_db, log, pack_rows, to_dev, workload_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1707_00516_amd.torch_api import Context
    c = Context(0)
    yield c
    c.sync()
    c.close()


def _sample(seed: int, n: int, count: int) -> list[int]:
    u = gen.u64s(seed, 5, 7, count)
    return sorted({int(x % n) for x in u})


def _check_keys(cnt_q, idx_q, refs_rows, q_bytes, mode, n_refs):
    """Each returned pair: index in range, unique, ascending (count, index),
    and the count the oracle gives for that (reference, query)."""
    valid = idx_q >= 0
    assert valid.all()
    assert np.all((idx_q >= 0) & (idx_q < n_refs))
    assert np.unique(idx_q).size == idx_q.size
    keys = cnt_q.astype(np.int64) * (1 << 40) + idx_q
    assert np.all(np.diff(keys) > 0)
    want = oracle.counts(refs_rows, q_bytes[None, :], mode)[0]
    assert np.array_equal(cnt_q, want)


def _check_all_pairs(cnt, idx, seed, thr, M, mode, n_refs):
    """Every returned pair: in range, unique and ascending per query, and
    its count equal to the oracle's for that (reference, query)."""
    n_q, k = cnt.shape
    valid = idx >= 0
    assert valid.all()
    assert np.all(idx < n_refs)
    for qi in range(n_q):
        assert np.unique(idx[qi]).size == k
    keys = cnt.astype(np.int64) * (1 << 40) + idx
    assert np.all(np.diff(keys, axis=1) > 0)
    rows = gen.ref_rows(seed, thr, idx.ravel())
    want = oracle.count_pairs(rows, M, np.arange(idx.size), np.repeat(np.arange(n_q), k), mode)
    assert np.array_equal(cnt.ravel(), want)


def _full_rows_and_packed(seed, thr, n_refs, Q, mode, chunk):
    """The oracle's counts of queries Q against every reference (rows
    regenerated chunk by chunk on the CPU), and the same references packed
    by the packed baseline."""
    L = thr.size
    nq = Q.shape[0]
    rows = np.empty((nq, n_refs), np.int32)
    packed = np.empty((n_refs, cpu_packed.words(L)), np.uint64)
    for r0 in range(0, n_refs, chunk):
        n = min(chunk, n_refs - r0)
        b = gen.ref_bytes(seed, thr, r0, n)
        # one oracle pair per (query, reference) of the chunk, so that every
        # core has work whatever the number of queries
        got = oracle.count_pairs(b, Q, np.tile(np.arange(n), nq), np.repeat(np.arange(nq), n), mode)
        rows[:, r0:r0 + n] = got.reshape(nq, n)
        cpu_packed.pack(b, out=packed[r0:r0 + n])
        if (r0 // chunk) % 8 == 0:
            log(f"  full rows: {r0 + n} of {n_refs} references")
    return rows, packed


def _oracle_topk_rows(rows, k):
    """oracle.topk of each full row, rows in parallel threads (each call
    sorts one whole row)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(lambda i: oracle.topk(rows[i:i + 1], k), range(rows.shape[0])))
    return np.concatenate([c for c, _ in res]), np.concatenate([i for _, i in res])


def _backend(ctx, name):
    from paper_1707_00516_amd import (FID_BACKEND_AUTO, FID_BACKEND_MFMA_FP4,
                                      FID_BACKEND_POPCOUNT, fid_ctx_set_backend)
    fid_ctx_set_backend(ctx.handle, {"auto": FID_BACKEND_AUTO, "fp4": FID_BACKEND_MFMA_FP4,
                                     "popcount": FID_BACKEND_POPCOUNT}[name])


@pytest.mark.timeout(900)
def test_headline_2048x20Mx2048_top32(ctx):
    w = MIX_2048x20M
    k = w.k
    log(f"headline {w.n_q} x {w.n_refs} x {w.n_loci}: inputs")
    thr, M, contrib, ncon, F = workload_inputs(w)
    db = gpu_generated_db(ctx, w.seed, thr, w.n_refs)
    q = pack_rows(ctx, M)
    _backend(ctx, "auto")
    log("headline: top-32 of all queries (the benchmark's call)")
    cnt, idx = ctx.compare_topk(db, q, w.mode, k)
    cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()

    _check_all_pairs(cnt, idx, w.seed, thr, M, w.mode, w.n_refs)
    log(f"headline: all {cnt.size} returned pairs equal the oracle's counts")
    for qi in _sample(w.seed, w.n_q, 12):
        members = set(idx[qi].tolist())
        for r in contrib[qi][:ncon[qi]]:
            assert int(r) in members, (qi, int(r))
    log("headline: sampled contributors are in the top-32")

    # the whole database regenerated on the CPU: full oracle rows of 16
    # sampled queries, and the packed baseline's top-32 of every query
    sample = _sample(w.seed + 2, w.n_q, 16)
    rows, packed = _full_rows_and_packed(w.seed, thr, w.n_refs, M[sample], w.mode, 1 << 19)
    wc, wi = _oracle_topk_rows(rows, k)
    assert np.array_equal(cnt[sample], wc) and np.array_equal(idx[sample], wi)
    log(f"headline: {len(sample)} queries equal the oracle's top-32 of their full rows")
    del rows
    pc, pi = cpu_packed.topk(packed, cpu_packed.pack(M), w.n_loci, w.mode, k)
    del packed
    assert np.array_equal(cnt, pc) and np.array_equal(idx, pi)
    log(f"headline: all {w.n_q} queries equal the packed CPU baseline's top-32")

    # the k-th boundary: a second kernel family over all 20M references
    sub = _sample(w.seed + 1, w.n_q, 40)
    _backend(ctx, "popcount")
    pc_cnt, pc_idx = ctx.compare_topk(db, q[sub].contiguous(), w.mode, k)
    _backend(ctx, "auto")
    assert np.array_equal(pc_cnt.cpu().numpy(), cnt[sub])
    assert np.array_equal(pc_idx.cpu().numpy(), idx[sub])
    log(f"headline: {len(sub)} queries equal the popcount scan's top-32")

    # the 64 verification tiles the benchmark requests, every one
    u = gen.u64s(w.seed, 5, 0, 128)
    tiles = [(int(u[2 * i] % (w.n_q // 256)) * 256, int(u[2 * i + 1] % (w.n_refs // 256)) * 256)
             for i in range(64)]
    got = ctx.compare_tiles(db, q, w.mode, tiles, 256, 256).cpu().numpy()
    for t, (q0, r0) in enumerate(tiles):
        refs = gen.ref_bytes(w.seed, thr, r0, 256)
        assert np.array_equal(got[t], oracle.counts(refs, M[q0:q0 + 256], w.mode)), t
    log("headline: all 64 tiles match the oracle")
    db.close()


@pytest.mark.timeout(900)
def test_large_panel_256x2Mx32768_threshold_top32(ctx):
    w = MIX_256x2Mx32K
    k = w.k
    T = threshold_2pct(w.n_loci)
    log(f"large panel {w.n_q} x {w.n_refs} x {w.n_loci}: inputs")
    thr, M, contrib, ncon, F = workload_inputs(w)
    db = gpu_generated_db(ctx, w.seed, thr, w.n_refs)
    q = pack_rows(ctx, M)
    _backend(ctx, "auto")
    offs, hidx, hcnt = ctx.compare_threshold(db, q, w.mode, T)
    offs, hidx, hcnt = offs.cpu().numpy(), hidx.cpu().numpy(), hcnt.cpu().numpy()
    cnt, idx = ctx.compare_topk(db, q, w.mode, k)
    cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()
    log("large panel: threshold and top-32 done")
    # the benchmark's one-pass call gives the same outputs (both are checked
    # against the oracle below)
    f_offs, f_hidx, f_hcnt, f_cnt, f_idx = ctx.compare_threshold_topk(db, q, w.mode, T, k)
    assert np.array_equal(f_offs.cpu().numpy(), offs) and np.array_equal(f_hidx.cpu().numpy(), hidx)
    assert np.array_equal(f_hcnt.cpu().numpy(), hcnt)
    assert np.array_equal(f_cnt.cpu().numpy(), cnt) and np.array_equal(f_idx.cpu().numpy(), idx)
    log("large panel: the one-pass threshold + top-32 equals the two calls")

    _check_all_pairs(cnt, idx, w.seed, thr, M, w.mode, w.n_refs)
    assert np.all(np.diff(offs) >= 0) and offs[0] == 0 and offs[-1] == hidx.size
    for qi in range(w.n_q):
        hi = hidx[offs[qi]:offs[qi + 1]]
        assert np.all(np.diff(hi) > 0) and np.all(hcnt[offs[qi]:offs[qi + 1]] <= T)
    hq = np.repeat(np.arange(w.n_q), np.diff(offs))
    want = oracle.count_pairs(gen.ref_rows(w.seed, thr, hidx), M, np.arange(hidx.size), hq, w.mode)
    assert np.array_equal(hcnt, want)
    for qi in _sample(w.seed, w.n_q, 6):
        for r in contrib[qi][:ncon[qi]]:
            assert int(r) in set(hidx[offs[qi]:offs[qi + 1]].tolist()), (qi, int(r))
    log(f"large panel: all {cnt.size} top-32 pairs and {hidx.size} hits equal the oracle's counts")

    # full oracle rows of 2 sampled queries over all 2M references: their
    # threshold CSR and top-32; the packed baseline's top-32 of every query
    sample = _sample(w.seed + 3, w.n_q, 2)
    rows, packed = _full_rows_and_packed(w.seed, thr, w.n_refs, M[sample], w.mode, 1 << 15)
    o_offs, o_idx, o_cnt = oracle.threshold(rows, T)
    for j, qi in enumerate(sample):
        assert np.array_equal(hidx[offs[qi]:offs[qi + 1]], o_idx[o_offs[j]:o_offs[j + 1]]), qi
        assert np.array_equal(hcnt[offs[qi]:offs[qi + 1]], o_cnt[o_offs[j]:o_offs[j + 1]]), qi
    wc, wi = _oracle_topk_rows(rows, k)
    assert np.array_equal(cnt[sample], wc) and np.array_equal(idx[sample], wi)
    del rows
    log(f"large panel: {len(sample)} queries equal the oracle's hits and top-32 of their full rows")
    pc, pi = cpu_packed.topk(packed, cpu_packed.pack(M), w.n_loci, w.mode, k)
    del packed
    assert np.array_equal(cnt, pc) and np.array_equal(idx, pi)
    log(f"large panel: all {w.n_q} queries equal the packed CPU baseline's top-32")

    sub = _sample(w.seed + 1, w.n_q, 10)
    _backend(ctx, "popcount")
    p_offs, p_idx, p_cnt = ctx.compare_threshold(db, q[sub].contiguous(), w.mode, T)
    pc_cnt, pc_idx = ctx.compare_topk(db, q[sub].contiguous(), w.mode, k)
    _backend(ctx, "auto")
    p_offs, p_idx, p_cnt = p_offs.cpu().numpy(), p_idx.cpu().numpy(), p_cnt.cpu().numpy()
    for j, qi in enumerate(sub):
        assert np.array_equal(p_idx[p_offs[j]:p_offs[j + 1]], hidx[offs[qi]:offs[qi + 1]]), qi
        assert np.array_equal(p_cnt[p_offs[j]:p_offs[j + 1]], hcnt[offs[qi]:offs[qi + 1]]), qi
    assert np.array_equal(pc_cnt.cpu().numpy(), cnt[sub])
    assert np.array_equal(pc_idx.cpu().numpy(), idx[sub])
    log(f"large panel: {len(sub)} queries equal the popcount scan's hits and top-32")
    db.close()


@pytest.mark.parametrize("L", [2560, 4608])
def test_chunked_rows_many_tiles_per_workgroup(ctx, L):
    """fp4 rows longer than one LDS chunk, with enough references that every
    workgroup scans several tiles (the query chunks are restaged for every
    tile; L = 2560 and 4608 end in a partial chunk) and a partial query tile
    (zero rows).  Top-k and threshold equal the popcount scan's over all
    600,000 references, every returned pair equals the oracle's count, and
    sampled tiles equal the oracle."""
    n_refs, n_q, k, seed = 600_000, 100, 16, gen.MASTER_SEED + 7000 + L
    thr = gen.maf_thresholds(seed, L, 0.05)
    log(f"chunked rows L={L}: database of {n_refs} references")
    db = gpu_generated_db(ctx, seed, thr, n_refs)
    M = gen.mixtures(seed, thr, 0, n_refs, 0, n_q, 1, 4, 0.005)[0]
    q = pack_rows(ctx, M)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        _backend(ctx, "fp4")
        cnt, idx = ctx.compare_topk(db, q, mode, k)
        T = int(np.sort(cnt.cpu().numpy()[:, 5])[n_q // 2])
        thr_q = to_dev(np.full(n_q, T, dtype=np.int32))
        offs, hidx, hcnt = ctx.compare_threshold(db, q, mode, thr_q, cap=1 << 22)
        _backend(ctx, "popcount")
        pc_cnt, pc_idx = ctx.compare_topk(db, q, mode, k)
        p_offs, p_idx, p_cnt = ctx.compare_threshold(db, q, mode, thr_q, cap=1 << 22)
        _backend(ctx, "auto")
        cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()
        assert np.array_equal(cnt, pc_cnt.cpu().numpy()) and np.array_equal(idx, pc_idx.cpu().numpy()), mode
        assert np.array_equal(offs.cpu().numpy(), p_offs.cpu().numpy()), mode
        assert np.array_equal(hidx.cpu().numpy(), p_idx.cpu().numpy()), mode
        assert np.array_equal(hcnt.cpu().numpy(), p_cnt.cpu().numpy()), mode
        for qi in _sample(seed, n_q, 6):
            _check_keys(cnt[qi], idx[qi], gen.ref_rows(seed, thr, idx[qi]), M[qi], mode, n_refs)
        log(f"chunked rows L={L} mode={mode}: top-k and threshold equal the popcount scan and the oracle")
    _backend(ctx, "fp4")
    u = gen.u64s(seed, 5, 0, 4)
    tiles = [(0, int(u[0] % (n_refs // 256)) * 256), (0, int(u[1] % (n_refs // 256)) * 256)]
    got = ctx.compare_tiles(db, q, oracle.MIXTURE, tiles, 64, 256).cpu().numpy()
    _backend(ctx, "auto")
    for t, (q0, r0) in enumerate(tiles):
        refs = gen.ref_bytes(seed, thr, r0, 256)
        assert np.array_equal(got[t], oracle.counts(refs, M[q0:q0 + 64], oracle.MIXTURE)), t
    db.close()
