"""fid_compare_topk_noalloc (the top-k entry point for callers that cannot
allocate): through the C ABI, bit-identical to fid_compare_topk on the same
inputs, on two calls in a row (the second smaller, so it runs over what the
first left in the fixed scratch), with no change in the device's free memory;
oversized problems are refused before anything is enqueued."""
import numpy as np
import pytest

import gen
import oracle
from gpu_harness import db_from_bytes, log, pack_rows

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


def _inputs(seed, n_refs, n_q, L):
    thr = gen.maf_thresholds(seed, L, 0.05)
    refs = gen.ref_bytes(seed, thr, 0, n_refs)
    M = gen.mixtures(seed, thr, 0, n_refs, 0, n_q, 1, 4, 0.005)[0]
    return refs, M


def _noalloc(ctx, db, q, mode, k):
    from paper_1707_00516_amd import fid_compare_topk_noalloc
    nq = q.shape[0]
    cnt = torch.full((nq, k), -7, dtype=torch.int32, device="cuda")
    idx = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    fid_compare_topk_noalloc(ctx.handle, db.handle, q.data_ptr(), nq, mode, k, cnt.data_ptr(), idx.data_ptr())
    ctx.sync()
    free1 = torch.cuda.mem_get_info()[0]
    return cnt.cpu().numpy(), idx.cpu().numpy(), free0, free1


def _plain(ctx, db, q, mode, k):
    cnt, idx = ctx.compare_topk(db, q, mode, k)
    ctx.sync()
    return cnt.cpu().numpy(), idx.cpu().numpy()


def test_noalloc_matches_compare_topk_twice(ctx):
    # call 1: 300 queries (fp4 matrix cores, seeded scan over 200,000
    # references, several query tiles); call 2: 20 queries against 40,000
    # references at another row length (the popcount family, smaller
    # workspace written over the first call's)
    cases = [(7101, 200_000, 300, 2048, oracle.MIXTURE, 32), (7102, 40_000, 20, 1000, oracle.IDENTITY, 17)]
    for seed, n_refs, n_q, L, mode, k in cases:
        log(f"noalloc: {n_q} x {n_refs} x {L} mode={mode} k={k}")
        refs, M = _inputs(seed, n_refs, n_q, L)
        db = db_from_bytes(ctx, refs)
        q = pack_rows(ctx, M)
        want_c, want_i = _plain(ctx, db, q, mode, k)
        got_c, got_i, free0, free1 = _noalloc(ctx, db, q, mode, k)
        assert np.array_equal(got_c, want_c) and np.array_equal(got_i, want_i)
        assert free1 == free0, (free0, free1)
        if n_q <= 32:
            oc, oi = oracle.topk(oracle.counts(refs, M, mode), k)
            assert np.array_equal(got_c, oc) and np.array_equal(got_i, oi)
        db.close()


def test_noalloc_refuses_oversized_problem(ctx):
    from paper_1707_00516_amd import FID_ENOMEM, FidError, fid_compare_topk_noalloc
    refs, M = _inputs(7103, 30_000, 512, 256)
    db = db_from_bytes(ctx, refs)
    q = pack_rows(ctx, M)
    cnt = torch.empty((512, 1024), dtype=torch.int32, device="cuda")
    idx = torch.empty((512, 1024), dtype=torch.int64, device="cuda")
    with pytest.raises(FidError) as e:
        fid_compare_topk_noalloc(ctx.handle, db.handle, q.data_ptr(), 512, oracle.MIXTURE, 1024, cnt.data_ptr(),
                                 idx.data_ptr())
    assert e.value.status == FID_ENOMEM
    assert "fixed scratch" in str(e.value)
    db.close()
