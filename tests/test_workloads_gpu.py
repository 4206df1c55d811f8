"""Parity at the full workload sizes, in the launch configuration the
benchmark times, on outputs the oracle can compute one by one.

The oracle cannot scan 20 million references per query in a test, so:
every returned (count, index) pair is recomputed by the oracle from the
reference rows the CPU generator produces for those indices; the ordering,
range and uniqueness of the keys are checked; every true contributor of a
sampled mixture (known from the generator's bookkeeping) must be among the
results with the oracle's count; sampled 256 x 256 verification tiles equal
the oracle; and the k-th boundary is checked against a second, independent
kernel family (the popcount scan) over the whole database for a query sample.
"""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
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


def _backend(ctx, name):
    from paper_1707_00516_amd import (FID_BACKEND_AUTO, FID_BACKEND_MFMA_FP4,
                                      FID_BACKEND_POPCOUNT, fid_ctx_set_backend)
    fid_ctx_set_backend(ctx.handle, {"auto": FID_BACKEND_AUTO, "fp4": FID_BACKEND_MFMA_FP4,
                                     "popcount": FID_BACKEND_POPCOUNT}[name])


def test_headline_2048x20Mx2048_top32_sampled(ctx):
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

    for qi in _sample(w.seed, w.n_q, 12):
        rows = gen.ref_rows(w.seed, thr, idx[qi])
        _check_keys(cnt[qi], idx[qi], rows, M[qi], w.mode, w.n_refs)
        members = set(idx[qi].tolist())
        for r in contrib[qi][:ncon[qi]]:
            assert int(r) in members, (qi, int(r))
    log("headline: sampled keys and contributors match the oracle")

    # the k-th boundary: a second kernel family over all 20M references
    sub = _sample(w.seed + 1, w.n_q, 40)
    _backend(ctx, "popcount")
    pc_cnt, pc_idx = ctx.compare_topk(db, q[sub].contiguous(), w.mode, k)
    _backend(ctx, "auto")
    assert np.array_equal(pc_cnt.cpu().numpy(), cnt[sub])
    assert np.array_equal(pc_idx.cpu().numpy(), idx[sub])
    log(f"headline: {len(sub)} queries equal the popcount scan's top-32")

    # verification tiles, as the benchmark requests them
    u = gen.u64s(w.seed, 5, 0, 8)
    tiles = [(int(u[2 * i] % (w.n_q // 256)) * 256, int(u[2 * i + 1] % (w.n_refs // 256)) * 256)
             for i in range(4)]
    got = ctx.compare_tiles(db, q, w.mode, tiles, 256, 256).cpu().numpy()
    for t, (q0, r0) in enumerate(tiles[:2]):
        refs = gen.ref_bytes(w.seed, thr, r0, 256)
        assert np.array_equal(got[t], oracle.counts(refs, M[q0:q0 + 256], w.mode)), t
    log("headline: tiles match the oracle")
    db.close()


def test_large_panel_256x2Mx32768_threshold_top32_sampled(ctx):
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

    for qi in _sample(w.seed, w.n_q, 6):
        hi, hc = hidx[offs[qi]:offs[qi + 1]], hcnt[offs[qi]:offs[qi + 1]]
        assert np.all(np.diff(hi) > 0) and np.all(hc <= T)
        if hi.size:
            want = oracle.counts(gen.ref_rows(w.seed, thr, hi), M[qi][None, :], w.mode)[0]
            assert np.array_equal(hc, want)
        for r in contrib[qi][:ncon[qi]]:
            assert int(r) in set(hi.tolist()), (qi, int(r))
        _check_keys(cnt[qi], idx[qi], gen.ref_rows(w.seed, thr, idx[qi]), M[qi], w.mode, w.n_refs)
    log("large panel: sampled hits, contributors and keys match the oracle")

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
