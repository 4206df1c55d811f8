"""Streamed database (rows held in host memory, passed through the device a
block at a time): top-k and threshold hits equal fid_compare_topk /
fid_compare_threshold over the same rows held resident, and top-k, threshold
hits and the full matrix (counts shipped back to host memory) equal the
oracle on small cases, including the degenerate block shapes (one block,
one-row blocks, a partial last block, k past the rows, overflow)."""
from __future__ import annotations

import numpy as np
import pytest

import gen
import oracle
from gpu_harness import gen_row_words, log, pack_rows, to_dev

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


def _rows_on_device(ctx, seed, thr, n_refs):
    """Packed rows of references 0..n_refs-1 from the GPU generator."""
    L = thr.size
    thr_dev = to_dev(thr.astype(np.uint32))
    buf = torch.empty((n_refs, L), dtype=torch.uint8, device="cuda")
    gen.ref_bytes_gpu(seed, thr_dev.data_ptr(), L, 0, n_refs, buf.data_ptr(), L,
                      torch.cuda.current_stream().cuda_stream)
    rows = torch.empty((n_refs, gen_row_words(L)), dtype=torch.int64, device="cuda")
    ctx.pack(buf, L, out=rows)
    ctx.sync()
    return rows


@pytest.mark.parametrize("L,n_q", [(1000, 40), (1000, 200), (2500, 150)])
def test_streamed_equals_resident(ctx, L, n_q):
    n_refs, block, k = 300_000, 65_536, 32
    seed = gen.MASTER_SEED + 8000 + L + n_q
    thr = gen.maf_thresholds(seed, L, 0.05)
    log(f"streamed L={L} n_q={n_q}: {n_refs} references in blocks of {block}")
    rows = _rows_on_device(ctx, seed, thr, n_refs)
    rows_host = rows.cpu().pin_memory()
    db = ctx.build_db(rows, L)
    M = gen.mixtures(seed, thr, 0, n_refs, 0, n_q, 1, 4, 0.005)[0]
    q = pack_rows(ctx, M)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        cnt, idx = ctx.compare_topk_streamed(rows_host, L, block, q, mode, k)
        want_c, want_i = ctx.compare_topk(db, q, mode, k)
        assert np.array_equal(cnt.cpu().numpy(), want_c.cpu().numpy()), mode
        assert np.array_equal(idx.cpu().numpy(), want_i.cpu().numpy()), mode
        # sampled rows against the oracle, from the generator's rows
        ic = idx.cpu().numpy()
        cc = cnt.cpu().numpy()
        for qi in (0, n_q // 2, n_q - 1):
            refs = gen.ref_rows(seed, thr, ic[qi])
            assert np.array_equal(cc[qi], oracle.counts(refs, M[qi][None, :], mode)[0]), (mode, qi)
        log(f"streamed L={L} n_q={n_q} mode={mode}: equal to the resident database")
    db.close()


@pytest.mark.parametrize("n_refs,block,k", [(50, 1000, 64), (10, 1, 4), (700, 128, 16)])
def test_streamed_small_against_oracle(ctx, n_refs, block, k):
    """One block (and k past the rows), one-row blocks, a partial last block."""
    L = 300
    rng = np.random.default_rng(n_refs + block + k)
    refs = (rng.random((n_refs, L)) < 0.3).astype(np.uint8)
    Q = (rng.random((6, L)) < 0.4).astype(np.uint8)
    log(f"streamed small n_refs={n_refs} block={block} k={k}")
    rows_host = pack_rows(ctx, refs).cpu().pin_memory()
    q = pack_rows(ctx, Q)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        cnt, idx = ctx.compare_topk_streamed(rows_host, L, block, q, mode, k)
        wc, wi = oracle.topk(oracle.counts(refs, Q, mode), k)
        assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi), mode


def test_streamed_rejects_bad_arguments(ctx):
    from paper_1707_00516_amd import (FID_EINVAL, FID_ENOMEM, FidError, fid_compare_topk_streamed,
                                      fid_stream_workspace_bytes)
    L, n_refs = 100, 64
    rows_host = torch.zeros((n_refs, gen_row_words(L)), dtype=torch.int64).pin_memory()
    q = torch.zeros((2, gen_row_words(L)), dtype=torch.int64, device="cuda")
    cnt = torch.empty((2, 4), dtype=torch.int32, device="cuda")
    idx = torch.empty((2, 4), dtype=torch.int64, device="cuda")
    need = fid_stream_workspace_bytes(ctx.handle, n_refs, L, 16, 2, 4)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    for block, mode, k, nbytes, status in [(0, 0, 4, need, FID_EINVAL), (16, 5, 4, need, FID_EINVAL),
                                           (16, 0, 0, need, FID_EINVAL), (16, 0, 4, need - 256, FID_ENOMEM)]:
        with pytest.raises(FidError) as e:
            fid_compare_topk_streamed(ctx.handle, rows_host.data_ptr(), n_refs, L, block, q.data_ptr(), 2, mode,
                                      k, ws.data_ptr(), nbytes, cnt.data_ptr(), idx.data_ptr())
        assert e.value.status == status, (block, mode, k, nbytes)


@pytest.mark.parametrize("L,block,pad", [(300, 1024, 0), (2500, 1024, 3), (700, 5000, 0), (64, 1, 0)])
def test_full_streamed_against_oracle(ctx, L, block, pad):
    """The full matrix of a streamed database (rows in, counts out, both in
    host memory): every count equals the oracle's, with a padded leading
    dimension, a partial last block, one block, and one-row blocks."""
    n_refs = 5000 if block > 1 else 9
    n_q = 7
    rng = np.random.default_rng(L + block + pad)
    refs = (rng.random((n_refs, L)) < 0.3).astype(np.uint8)
    Q = (rng.random((n_q, L)) < 0.4).astype(np.uint8)
    log(f"full streamed n_refs={n_refs} L={L} block={block} ld=n_refs+{pad}")
    rows_host = pack_rows(ctx, refs).cpu().pin_memory()
    q = pack_rows(ctx, Q)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        out = torch.full((n_q, n_refs + pad), -5, dtype=torch.int32).pin_memory()
        ctx.compare_full_streamed(rows_host, L, block, q, mode, out=out)
        got = out.numpy()
        assert np.array_equal(got[:, :n_refs], oracle.counts(refs, Q, mode)), mode
        assert np.all(got[:, n_refs:] == -5), mode  # the padding columns are left alone


def test_full_streamed_rejects_bad_arguments(ctx):
    from paper_1707_00516_amd import (FID_EINVAL, FID_ENOMEM, FidError, fid_compare_full_streamed,
                                      fid_full_stream_workspace_bytes)
    L, n_refs = 100, 64
    rows_host = torch.zeros((n_refs, gen_row_words(L)), dtype=torch.int64).pin_memory()
    q = torch.zeros((2, gen_row_words(L)), dtype=torch.int64, device="cuda")
    out = torch.empty((2, n_refs), dtype=torch.int32).pin_memory()
    need = fid_full_stream_workspace_bytes(ctx.handle, n_refs, L, 16, 2)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    for block, mode, ld, nbytes, status in [(16, 0, n_refs - 1, need, FID_EINVAL), (0, 0, n_refs, need, FID_EINVAL),
                                            (16, 4, n_refs, need, FID_EINVAL), (16, 0, n_refs, need - 256, FID_ENOMEM)]:
        with pytest.raises(FidError) as e:
            fid_compare_full_streamed(ctx.handle, rows_host.data_ptr(), n_refs, L, block, q.data_ptr(), 2, mode,
                                      ws.data_ptr(), nbytes, out.data_ptr(), ld)
        assert e.value.status == status, (block, mode, ld, nbytes)


@pytest.mark.parametrize("L,n_q,block", [(1000, 40, 65_536), (1000, 200, 65_536), (2500, 150, 100_000)])
def test_threshold_streamed_equals_resident(ctx, L, n_q, block):
    """Threshold hits of a streamed database equal fid_compare_threshold's over
    the same rows held resident (both kernel families by query count, a
    chunked fp4 row length, a partial last block)."""
    n_refs = 300_000
    seed = gen.MASTER_SEED + 9000 + L + n_q
    thr = gen.maf_thresholds(seed, L, 0.05)
    log(f"threshold streamed L={L} n_q={n_q} block={block}")
    rows = _rows_on_device(ctx, seed, thr, n_refs)
    rows_host = rows.cpu().pin_memory()
    db = ctx.build_db(rows, L)
    M = gen.mixtures(seed, thr, 0, n_refs, 0, n_q, 1, 4, 0.005)[0]
    q = pack_rows(ctx, M)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        cnt, _ = ctx.compare_topk(db, q, mode, 9)
        T = to_dev(cnt[:, 8].cpu().numpy().astype(np.int32))  # about 9 hits per query
        so, si, sc = ctx.compare_threshold_streamed(rows_host, L, block, q, mode, T, cap=1 << 16)
        ro, ri, rc = ctx.compare_threshold(db, q, mode, T, cap=1 << 16)
        assert np.array_equal(so.cpu().numpy(), ro.cpu().numpy()), mode
        assert np.array_equal(si.cpu().numpy(), ri.cpu().numpy()), mode
        assert np.array_equal(sc.cpu().numpy(), rc.cpu().numpy()), mode
        assert si.numel() >= 9 * n_q
    db.close()


@pytest.mark.parametrize("n_refs,block", [(700, 128), (50, 1000), (9, 1)])
def test_threshold_streamed_small_against_oracle(ctx, n_refs, block):
    L = 300
    rng = np.random.default_rng(n_refs + block)
    refs = (rng.random((n_refs, L)) < 0.3).astype(np.uint8)
    Q = (rng.random((5, L)) < 0.4).astype(np.uint8)
    rows_host = pack_rows(ctx, refs).cpu().pin_memory()
    q = pack_rows(ctx, Q)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        want = oracle.counts(refs, Q, mode)
        thr = np.sort(want, axis=1)[:, min(5, n_refs - 1)].astype(np.int32)
        offs, idx, cnt = ctx.compare_threshold_streamed(rows_host, L, block, q, mode, to_dev(thr), cap=4096)
        wo, wi, wc = oracle.threshold(want, thr)
        assert np.array_equal(offs.cpu().numpy(), wo) and np.array_equal(idx.cpu().numpy(), wi), mode
        assert np.array_equal(cnt.cpu().numpy(), wc), mode


def test_threshold_streamed_overflow_reports_total(ctx):
    from paper_1707_00516_amd import FID_EOVERFLOW, FidError
    L, n_refs = 200, 3000
    rng = np.random.default_rng(77)
    refs = (rng.random((n_refs, L)) < 0.3).astype(np.uint8)
    Q = (rng.random((3, L)) < 0.4).astype(np.uint8)
    rows_host = pack_rows(ctx, refs).cpu().pin_memory()
    want = oracle.counts(refs, Q, oracle.MIXTURE)
    thr = np.full(3, L, dtype=np.int32)  # every reference is a hit
    with pytest.raises(FidError) as e:
        ctx.compare_threshold_streamed(rows_host, L, 512, pack_rows(ctx, Q), oracle.MIXTURE, to_dev(thr), cap=100)
    assert e.value.status == FID_EOVERFLOW
    assert str(3 * n_refs) in str(e.value)
    assert want.size == 3 * n_refs
