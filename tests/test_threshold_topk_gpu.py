"""GPU parity of the one-pass threshold + top-k (fid_compare_threshold_topk)
against the oracle: the threshold CSR and the top-k of the same queries,
bit-exact, on every kernel family (fp4 fuses both epilogues into one scan;
the others run two scans), past the seed prefix and on the direct path, on
chunked long rows, with per-query thresholds from -1 to above L, and with a
hit capacity that overflows."""
import numpy as np
import pytest

import gen
import oracle
from gpu_harness import db_from_bytes, log, pack_rows, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BACKENDS = {"auto": 0, "popcount": 1, "mfma": 2, "mfma_fp4": 3}


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


def _thresholds(seed, rows, L):
    """Per query: -1, 0, the 3rd / 40th smallest count, 2% of L, or L."""
    s = np.sort(rows, axis=1)
    u = gen.u64s(seed, 5, 9, rows.shape[0]) % 6
    choice = [lambda q: -1, lambda q: 0, lambda q: s[q, 2], lambda q: s[q, min(39, s.shape[1] - 1)],
              lambda q: (2 * L) // 100, lambda q: L]
    return np.array([choice[int(u[q])](q) for q in range(rows.shape[0])], np.int32)


@pytest.mark.parametrize("n_refs,L,k", [(70_000, 2048, 32), (70_000, 1000, 16), (40_000, 4100, 32),
                                         (3_000, 700, 32), (20_000, 65, 64)])
@pytest.mark.parametrize("mode", [oracle.MIXTURE, oracle.IDENTITY])
@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_threshold_topk_matches_oracle(ctx, n_refs, L, k, mode, backend):
    n_q = 200 if backend != "popcount" else 40
    seed = 9100 + L + n_refs
    log(f"threshold+topk refs={n_refs} L={L} k={k} mode={mode} backend={backend}")
    thr = gen.maf_thresholds(seed, L, 0.05)
    refs = gen.ref_bytes(seed, thr, 0, n_refs)
    if mode == oracle.MIXTURE:
        Q = gen.mixtures(seed, thr, 0, n_refs, 0, n_q, 1, 4, 0.005)[0]
    else:
        Q = gen.identity(seed, thr, 0, n_refs, 0, n_q, 0.005)[0]
    rows = oracle.counts(refs, Q, mode)
    T = _thresholds(seed, rows, L)
    db = db_from_bytes(ctx, refs)
    use_backend(ctx, backend)
    offs, hidx, hcnt, cnt, idx = ctx.compare_threshold_topk(db, pack_rows(ctx, Q), mode, to_dev(T), k, cap=1 << 10)
    use_backend(ctx, "auto")
    o_offs, o_idx, o_cnt = oracle.threshold(rows, T)
    assert np.array_equal(offs.cpu().numpy(), o_offs)
    assert np.array_equal(hidx.cpu().numpy(), o_idx)
    assert np.array_equal(hcnt.cpu().numpy(), o_cnt)
    wc, wi = oracle.topk(rows, k)
    assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
    db.close()


def test_threshold_topk_overflow_keeps_topk(ctx):
    """A capacity below the hit total: FID_EOVERFLOW with the exact total, and
    the top-k output complete."""
    from paper_1707_00516_amd import (FID_EOVERFLOW, FidError, fid_compare_threshold_topk,
                                      fid_threshold_topk_workspace_bytes)
    n_refs, L, n_q, k = 60_000, 2048, 150, 32
    seed = 9300
    thr = gen.maf_thresholds(seed, L, 0.05)
    refs = gen.ref_bytes(seed, thr, 0, n_refs)
    Q = gen.mixtures(seed, thr, 0, n_refs, 0, n_q, 1, 4, 0.005)[0]
    rows = oracle.counts(refs, Q, oracle.MIXTURE)
    T = np.full(n_q, 200, np.int32)
    want_total = int((rows <= T[:, None]).sum())
    assert want_total > 100
    db = db_from_bytes(ctx, refs)
    q = pack_rows(ctx, Q)
    for backend in ("mfma_fp4", "popcount"):
        use_backend(ctx, backend)
        cap = want_total // 2
        ws = torch.empty(fid_threshold_topk_workspace_bytes(ctx.handle, db.handle, n_q, k, cap), dtype=torch.uint8,
                         device="cuda")
        offs = torch.empty(n_q + 1, dtype=torch.int64, device="cuda")
        hidx = torch.empty(cap, dtype=torch.int64, device="cuda")
        hcnt = torch.empty(cap, dtype=torch.int32, device="cuda")
        cnt = torch.empty((n_q, k), dtype=torch.int32, device="cuda")
        idx = torch.empty((n_q, k), dtype=torch.int64, device="cuda")
        with pytest.raises(FidError) as e:
            fid_compare_threshold_topk(ctx.handle, db.handle, q.data_ptr(), n_q, oracle.MIXTURE,
                                       to_dev(T).data_ptr(), k, ws.data_ptr(), ws.numel(), cap, offs.data_ptr(),
                                       hidx.data_ptr(), hcnt.data_ptr(), cnt.data_ptr(), idx.data_ptr())
        assert e.value.status == FID_EOVERFLOW and e.value.needed == want_total
        ctx.sync()
        wc, wi = oracle.topk(rows, k)
        assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi), backend
    use_backend(ctx, "auto")
    db.close()
