"""GPU parity of the bounded top-k (fid_compare_topk_bounded) against the
oracle, and the device-side check of per-query modes.

A caller bound of 0xFFFFFFFF ("none yet": the state of a running top-k that
holds fewer than k keys) over a range larger than the seed prefix, with the
seed pass skipped, is the path a serving tick takes after admitting a
request on a chunk shorter than k; it must give the exact top-k.  Other
bounds are checked against the contract: entries below the bound exact,
entries at or above it correct pairs or padding."""
import numpy as np
import pytest

import gen
import oracle
from gpu_harness import db_from_bytes, log, pack_rows, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BACKENDS = {"auto": 0, "popcount": 1, "mfma_fp4": 3}
NONE = np.uint32(0xFFFFFFFF)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1707_00516_amd.torch_api import Context
    c = Context(0)
    yield c
    c.sync()
    c.close()


def use_backend(ctx, name):
    from paper_1707_00516_amd import fid_ctx_set_backend
    fid_ctx_set_backend(ctx.handle, BACKENDS[name])


def _world(seed, n_refs, n_q, L):
    thr = gen.maf_thresholds(seed, L, 0.05)
    refs = gen.ref_bytes(seed, thr, 0, n_refs)
    u = gen.u64s(seed, 4, 0, n_q)
    modes = (u % 2).astype(np.int32)
    M = gen.mixtures(seed, thr, 0, n_refs, 0, n_q, 1, 4, 0.005)[0]
    I = gen.identity(seed, thr, 0, n_refs, 1 << 12, n_q, 0.005)[0]
    Q = np.where(modes[:, None] == oracle.MIXTURE, M, I)
    return refs, Q, modes


def _oracle_rows(refs, Q, modes, r_lo, r_hi):
    c = np.empty((Q.shape[0], r_hi - r_lo), np.int32)
    for m in (oracle.MIXTURE, oracle.IDENTITY):
        sel = np.nonzero(modes == m)[0]
        if sel.size:
            c[sel] = oracle.counts(refs[r_lo:r_hi], Q[sel], m)
    return c


def _check_contract(cnt, idx, rows, r_lo, bound, k):
    """rows: oracle counts of the range; bound: uint32 per query."""
    wc, wi = oracle.topk(rows, k)
    wi = np.where(wi >= 0, wi + r_lo, -1)
    for q in range(rows.shape[0]):
        b = int(bound[q])
        below = int(np.sum(wc[q] < b)) if b < (1 << 31) else k
        below = min(below, int(np.sum(wc[q] != np.iinfo(np.int32).max)))
        assert np.array_equal(cnt[q, :below], wc[q, :below]), q
        assert np.array_equal(idx[q, :below], wi[q, :below]), q
        rest_i, rest_c = idx[q, below:], cnt[q, below:]
        pad = rest_i < 0
        # padding only after every real entry
        assert np.all(np.diff(pad.astype(np.int8)) >= 0), q
        assert np.all(rest_c[pad] == np.iinfo(np.int32).max), q
        real = ~pad
        assert np.all(rest_c[real] >= b), q
        assert np.array_equal(rest_c[real], rows[q, rest_i[real] - r_lo]), q
        keys = cnt[q][idx[q] >= 0].astype(np.int64) * (1 << 40) + idx[q][idx[q] >= 0]
        assert np.all(np.diff(keys) > 0), q


@pytest.mark.parametrize("L", [256, 2048, 3000])
@pytest.mark.parametrize("backend", sorted(BACKENDS))
@pytest.mark.parametrize("use_seed", [False, True])
def test_bounded_without_a_bound_is_the_exact_topk(ctx, L, backend, use_seed):
    """bound = 0xFFFFFFFF over 70,000 references (past the seed prefix)."""
    n_refs, n_q, k = 70_000, 150, 32
    log(f"bounded none L={L} backend={backend} seed={use_seed}")
    refs, Q, modes = _world(8100 + L, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    use_backend(ctx, backend)
    r_lo, r_hi = 513, n_refs - 7
    bound = to_dev(np.full(n_q, NONE, np.uint32).view(np.int32))
    cnt, idx = ctx.compare_topk_bounded(db, r_lo, r_hi, pack_rows(ctx, Q), to_dev(modes), k, bound, use_seed)
    use_backend(ctx, "auto")
    rows = _oracle_rows(refs, Q, modes, r_lo, r_hi)
    wc, wi = oracle.topk(rows, k)
    assert np.array_equal(cnt.cpu().numpy(), wc)
    assert np.array_equal(idx.cpu().numpy(), np.where(wi >= 0, wi + r_lo, -1))
    db.close()


@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_bounded_with_bounds_keeps_every_entry_below(ctx, backend):
    """Bounds from 0 to above L, including the exact k-th count + 1, a
    bound between the first and k-th count, and none."""
    n_refs, n_q, k, L = 60_000, 140, 24, 2048
    log(f"bounded contract backend={backend}")
    refs, Q, modes = _world(8200, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    rows = _oracle_rows(refs, Q, modes, 0, n_refs)
    wc, _ = oracle.topk(rows, k)
    choice = gen.u64s(8200, 5, 1, n_q) % 6
    bound = np.empty(n_q, np.uint32)
    for q in range(n_q):
        bound[q] = [0, wc[q, 0], wc[q, k // 2], wc[q, k - 1] + 1, L + 1, NONE][int(choice[q])]
    use_backend(ctx, backend)
    for use_seed in (False, True):
        cnt, idx = ctx.compare_topk_bounded(db, 0, n_refs, pack_rows(ctx, Q), to_dev(modes), k,
                                            to_dev(bound.view(np.int32)), use_seed)
        _check_contract(cnt.cpu().numpy(), idx.cpu().numpy(), rows, 0, bound, k)
    use_backend(ctx, "auto")
    db.close()


def test_bounded_short_range_is_direct_and_exact(ctx):
    """A range under the seed prefix and under k: counted directly; the bound
    cannot drop entries there, the padding is (INT32_MAX, -1)."""
    n_refs, n_q, k, L = 3000, 20, 32, 500
    refs, Q, modes = _world(8300, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    bound = to_dev(np.full(n_q, NONE, np.uint32).view(np.int32))
    cnt, idx = ctx.compare_topk_bounded(db, 100, 120, pack_rows(ctx, Q), to_dev(modes), k, bound, False)
    rows = _oracle_rows(refs, Q, modes, 100, 120)
    wc, wi = oracle.topk(rows, k)
    assert np.array_equal(cnt.cpu().numpy(), wc)
    assert np.array_equal(idx.cpu().numpy(), np.where(wi >= 0, wi + 100, -1))
    db.close()


def test_modes_outside_the_enum_are_refused(ctx):
    from paper_1707_00516_amd import FID_EINVAL, FidError
    n_refs, n_q, k, L = 20_000, 10, 8, 300
    refs, Q, modes = _world(8400, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    q = pack_rows(ctx, Q)
    bound = to_dev(np.full(n_q, NONE, np.uint32).view(np.int32))
    for bad in (2, -1, 7):
        m = modes.copy()
        m[n_q // 2] = bad
        with pytest.raises(FidError) as e:
            ctx.compare_topk_mixed(db, 0, n_refs, q, to_dev(m), k)
        assert e.value.status == FID_EINVAL
        with pytest.raises(FidError) as e:
            ctx.compare_topk_bounded(db, 0, n_refs, q, to_dev(m), k, bound, True)
        assert e.value.status == FID_EINVAL
    # the good modes still work afterwards
    cnt, idx = ctx.compare_topk_mixed(db, 0, n_refs, q, to_dev(modes), k)
    wc, wi = oracle.topk(_oracle_rows(refs, Q, modes, 0, n_refs), k)
    assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
    db.close()
