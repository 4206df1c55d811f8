"""GPU parity: libfastid (through its C ABI) against the oracle, bit-exact.

Inputs come from the shared seeded generator; expected values from the
oracle only.  Sizes here span several 64-reference blocks and workers, ragged
tails in loci and references, every register-chunk width and the chunked
(long-panel) path."""
import numpy as np
import pytest

import gen
import oracle
from gen.workloads import MIX_64x20K
from gpu_harness import db_from_bytes, log, pack_rows, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODES = {"mixture": oracle.MIXTURE, "identity": oracle.IDENTITY}
BACKENDS = {"popcount": 1, "mfma": 2, "mfma_fp4": 3}


def use_backend(ctx, name):
    from paper_1707_00516_amd import fid_ctx_set_backend
    fid_ctx_set_backend(ctx.handle, BACKENDS[name])


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1707_00516_amd.torch_api import Context
    c = Context(0)
    yield c
    c.sync()
    c.close()


def _profiles(seed, n_refs, n_q, L, p_lo=0.05):
    thr = gen.maf_thresholds(seed, L, p_lo)
    refs = gen.ref_bytes(seed, thr, 0, n_refs)
    M, contrib, ncon, F = gen.mixtures(seed, thr, 0, n_refs, 0, n_q, 1, 4, 0.005)
    return refs, M


@pytest.mark.parametrize("L", [1, 31, 32, 33, 63, 64, 65, 127, 1000, 2048, 4100, 9000])
def test_pack_matches_numpy_packbits(ctx, L):
    log(f"pack L={L}")
    rng = np.random.default_rng(L)
    b = (rng.random((37, L)) < 0.4).astype(np.uint8)
    got = pack_rows(ctx, b).cpu().numpy().view(np.uint8)
    want = np.packbits(b, axis=1, bitorder="little")
    assert np.array_equal(got[:, :want.shape[1]], want)
    assert np.all(got[:, want.shape[1]:] == 0)


def test_pack_rejects_non_binary(ctx):
    from paper_1707_00516_amd import FID_EINVAL, FidError
    b = np.zeros((3, 100), np.uint8)
    b[1, 50] = 2
    with pytest.raises(FidError) as e:
        pack_rows(ctx, b)
    assert e.value.status == FID_EINVAL


@pytest.mark.parametrize("L", [1, 33, 127, 500, 1000, 2048, 2304, 3000, 4096, 5000, 9000])
@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_full_matches_oracle(ctx, L, mode, backend):
    n_refs, n_q = 1000 + 37, 37 + (0 if backend == "popcount" else 64 * (1 + (backend == "mfma_fp4")))
    log(f"full L={L} mode={mode} backend={backend} refs={n_refs} q={n_q}")
    use_backend(ctx, backend)
    refs, Q = _profiles(1000 + L, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    assert np.array_equal(db.popcounts().cpu().numpy(), refs.sum(axis=1))
    got = ctx.compare_full(db, pack_rows(ctx, Q), MODES[mode]).cpu().numpy()
    want = oracle.counts(refs, Q, MODES[mode])
    assert np.array_equal(got, want)
    db.close()


@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_full_mixture_64x20000x2048(ctx, backend):
    w = MIX_64x20K
    log(f"full {w.name} backend={backend}")
    use_backend(ctx, backend)
    thr = gen.maf_thresholds(w.seed, w.n_loci, w.maf_lo)
    refs = gen.ref_bytes(w.seed, thr, 0, w.n_refs)
    Q, contrib, ncon, F = gen.mixtures(w.seed, thr, 0, w.n_refs, 0, w.n_q, w.nc_lo, w.nc_hi, w.flip)
    db = db_from_bytes(ctx, refs)
    got = ctx.compare_full(db, pack_rows(ctx, Q), w.mode).cpu().numpy()
    want = oracle.counts(refs, Q, w.mode)
    assert np.array_equal(got, want)
    db.close()


@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_tiles_match_oracle(ctx, backend):
    L, n_refs, n_q = 2048, 5000, 300
    log(f"tiles backend={backend}")
    use_backend(ctx, backend)
    refs, Q = _profiles(77, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    rng = np.random.default_rng(5)
    th, tw = 40, 130
    tiles = [(int(rng.integers(0, n_q - th + 1)), int(rng.integers(0, n_refs - tw + 1)))
             for _ in range(9)] + [(0, 0), (n_q - th, n_refs - tw)]
    for mode in MODES.values():
        got = ctx.compare_tiles(db, pack_rows(ctx, Q), mode, tiles, th, tw).cpu().numpy()
        for t, (q0, r0) in enumerate(tiles):
            want = oracle.counts(refs[r0:r0 + tw], Q[q0:q0 + th], mode)
            assert np.array_equal(got[t], want), (mode, t)
    db.close()


@pytest.mark.parametrize("n_refs,L,k", [(50, 300, 64), (3000, 2048, 32), (50000, 2048, 32),
                                         (40000, 1000, 100), (30000, 5000, 5), (20000, 128, 1)])
@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_topk_matches_oracle(ctx, n_refs, L, k, mode, backend):
    n_q = 19 if backend == "popcount" else 83
    log(f"topk refs={n_refs} L={L} k={k} mode={mode} backend={backend}")
    use_backend(ctx, backend)
    refs, Q = _profiles(n_refs + L + k, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    cnt, idx = ctx.compare_topk(db, pack_rows(ctx, Q), MODES[mode], k)
    wc, wi = oracle.topk(oracle.counts(refs, Q, MODES[mode]), k)
    assert np.array_equal(cnt.cpu().numpy(), wc)
    assert np.array_equal(idx.cpu().numpy(), wi)
    db.close()


@pytest.mark.parametrize("n_refs", [500, 30000])
@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_topk_ties_go_to_lowest_index(ctx, n_refs, backend):
    """All-zero references: every mixture count is 0, so the top-k are the k
    lowest indices; duplicated rows tie in every mode."""
    log(f"topk ties refs={n_refs} backend={backend}")
    use_backend(ctx, backend)
    L, k = 256, 40
    refs = np.zeros((n_refs, L), np.uint8)
    rng = np.random.default_rng(1)
    Q = (rng.random((7, L)) < 0.5).astype(np.uint8)
    db = db_from_bytes(ctx, refs)
    for mode in MODES.values():
        cnt, idx = ctx.compare_topk(db, pack_rows(ctx, Q), mode, k)
        wc, wi = oracle.topk(oracle.counts(refs, Q, mode), k)
        assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
    db.close()
    dup = np.repeat((rng.random((n_refs // 10, L)) < 0.3).astype(np.uint8), 10, axis=0)
    db = db_from_bytes(ctx, dup)
    cnt, idx = ctx.compare_topk(db, pack_rows(ctx, dup[::997][:9]), oracle.IDENTITY, k)
    wc, wi = oracle.topk(oracle.counts(dup, dup[::997][:9], oracle.IDENTITY), k)
    assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
    db.close()


@pytest.mark.parametrize("backend", ["mfma", "mfma_fp4"])
def test_topk_every_pair_a_candidate_full_tiles(ctx, backend):
    """Identical references: every count of a query ties, so every pair stays
    below the filter bound for the whole scan (a full list's bound is its worst
    count plus one) and each tile's candidate queue overflows many times over;
    200 queries fill one 128-query tile and part of a second."""
    log(f"topk all candidates backend={backend}")
    use_backend(ctx, backend)
    n_refs, L, k = 40000, 256, 40
    rng = np.random.default_rng(11)
    row = (rng.random(L) < 0.3).astype(np.uint8)
    refs = np.repeat(row[None, :], n_refs, axis=0)
    Q = (rng.random((200, L)) < 0.5).astype(np.uint8)
    db = db_from_bytes(ctx, refs)
    for mode in MODES.values():
        cnt, idx = ctx.compare_topk(db, pack_rows(ctx, Q), mode, k)
        wc, wi = oracle.topk(oracle.counts(refs, Q, mode), k)
        assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
    db.close()


@pytest.mark.parametrize("n_refs,L", [(3000, 2048), (20000, 700), (7000, 9000)])
@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_threshold_matches_oracle(ctx, n_refs, L, backend):
    n_q = 23 if backend == "popcount" else 70
    log(f"threshold refs={n_refs} L={L} backend={backend}")
    use_backend(ctx, backend)
    refs, Q = _profiles(n_refs * 7 + L, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    rng = np.random.default_rng(3)
    for mode in MODES.values():
        want_counts = oracle.counts(refs, Q, mode)
        thr = np.array([np.sort(want_counts[q])[int(rng.integers(0, 60))] for q in range(n_q)],
                       np.int32)
        offs, idx, cnt = ctx.compare_threshold(db, pack_rows(ctx, Q), mode, to_dev(thr), cap=64)
        wo, wi, wc = oracle.threshold(want_counts, thr)
        assert np.array_equal(offs.cpu().numpy(), wo)
        assert np.array_equal(idx.cpu().numpy(), wi)
        assert np.array_equal(cnt.cpu().numpy(), wc)
    db.close()


def test_threshold_overflow_reports_needed(ctx):
    from paper_1707_00516_amd import FID_EOVERFLOW, FidError, fid_compare_threshold, \
        fid_threshold_workspace_bytes
    log("threshold overflow")
    use_backend(ctx, "popcount")
    refs, Q = _profiles(5, 2000, 4, 256)
    db = db_from_bytes(ctx, refs)
    want = oracle.threshold(oracle.counts(refs, Q, oracle.MIXTURE), [300] * 4)[0][-1]
    q = pack_rows(ctx, Q)
    thr = to_dev(np.full(4, 300, np.int32))
    cap = 10
    ws = torch.empty(fid_threshold_workspace_bytes(db.handle, 4, cap), dtype=torch.uint8,
                     device="cuda")
    offs = torch.empty(5, dtype=torch.int64, device="cuda")
    idx = torch.empty(cap, dtype=torch.int64, device="cuda")
    cnt = torch.empty(cap, dtype=torch.int32, device="cuda")
    with pytest.raises(FidError) as e:
        fid_compare_threshold(ctx.handle, db.handle, q.data_ptr(), 4, oracle.MIXTURE,
                              thr.data_ptr(), ws.data_ptr(), ws.numel(), cap, offs.data_ptr(),
                              idx.data_ptr(), cnt.data_ptr())
    assert e.value.status == FID_EOVERFLOW and e.value.needed == want
    db.close()


def test_gpu_generator_matches_cpu(ctx):
    log("generator gpu vs cpu")
    seed, L = 12345, 777
    thr = gen.maf_thresholds(seed, L, 0.05)
    out = torch.empty((50, 800), dtype=torch.uint8, device="cuda")
    gen.ref_bytes_gpu(seed, to_dev(thr).data_ptr(), L, 1_000_000, 50, out.data_ptr(), 800,
                      torch.cuda.current_stream().cuda_stream)
    got = out.cpu().numpy()[:, :L]
    assert np.array_equal(got, gen.ref_bytes(seed, thr, 1_000_000, 50))


@pytest.mark.parametrize("r_lo,r_hi,L,k", [(0, 50000, 2048, 32), (1000, 1050, 700, 64),
                                           (12345, 47000, 2048, 32), (63, 40100, 1000, 100),
                                           (29990, 30000, 300, 5)])
@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_topk_range_matches_oracle(ctx, r_lo, r_hi, L, k, backend):
    """Top-k over a reference slice: database-row indices, padding past the slice."""
    n_refs, n_q = 50000, 70
    log(f"topk range [{r_lo},{r_hi}) L={L} k={k} backend={backend}")
    use_backend(ctx, backend)
    refs, Q = _profiles(r_lo + L + k, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    for mode in MODES.values():
        cnt, idx = ctx.compare_topk_range(db, r_lo, r_hi, pack_rows(ctx, Q), mode, k)
        wc, wi = oracle.topk(oracle.counts(refs[r_lo:r_hi], Q, mode), k)
        assert np.array_equal(cnt.cpu().numpy(), wc)
        assert np.array_equal(idx.cpu().numpy(), np.where(wi >= 0, wi + r_lo, -1))
    db.close()


def test_topk_range_rejects_bad_ranges(ctx):
    from paper_1707_00516_amd import FID_EINVAL, FidError
    refs, Q = _profiles(3, 500, 4, 100)
    db = db_from_bytes(ctx, refs)
    q = pack_rows(ctx, Q)
    for r_lo, r_hi in [(-1, 10), (10, 10), (0, 501), (400, 300)]:
        with pytest.raises(FidError) as e:
            ctx.compare_topk_range(db, r_lo, r_hi, q, 0, 4, ws=torch.empty(1 << 20, dtype=torch.uint8,
                                                                             device="cuda"))
        assert e.value.status == FID_EINVAL
    db.close()


@pytest.mark.parametrize("n_refs,r_lo,r_hi,L,k", [(3000, 0, 3000, 2048, 32), (60000, 0, 60000, 2048, 32),
                                                  (60000, 999, 51000, 1000, 16), (20000, 5, 20000, 5000, 8)])
@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_topk_mixed_modes_match_oracle(ctx, n_refs, r_lo, r_hi, L, k, backend):
    """Identity and mixture queries in one call: each query's top-k equals the
    oracle's under its own mode."""
    log(f"topk mixed n_refs={n_refs} [{r_lo},{r_hi}) L={L} k={k} backend={backend}")
    use_backend(ctx, backend)
    n_q = 150
    refs, Q = _profiles(n_refs + L + 3 * k, n_refs, n_q, L)
    modes = (gen.u64s(17, 5, L, n_q) % 2).astype(np.int32)
    db = db_from_bytes(ctx, refs)
    cnt, idx = ctx.compare_topk_mixed(db, r_lo, r_hi, pack_rows(ctx, Q), to_dev(modes), k)
    cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()
    for mode in MODES.values():
        sel = np.nonzero(modes == mode)[0]
        wc, wi = oracle.topk(oracle.counts(refs[r_lo:r_hi], Q[sel], mode), k)
        assert np.array_equal(cnt[sel], wc), mode
        assert np.array_equal(idx[sel], np.where(wi >= 0, wi + r_lo, -1)), mode
    db.close()


def test_topk_many_query_tiles_with_witness_levels(ctx):
    """Three 128-query tiles (the last one partial) over 150,000 references:
    the seed block covers 16,384 of them, so each query's witness levels
    collect their k witnesses during the scan; every query's top-k (mixed
    modes) equals the oracle's."""
    L, n_refs, n_q, k = 128, 150000, 300, 32
    log(f"topk {n_q} queries x {n_refs} refs, witness levels")
    use_backend(ctx, "mfma_fp4")
    refs, Q = _profiles(909, n_refs, n_q, L)
    modes = (gen.u64s(23, 5, L, n_q) % 2).astype(np.int32)
    db = db_from_bytes(ctx, refs)
    cnt, idx = ctx.compare_topk_mixed(db, 0, n_refs, pack_rows(ctx, Q), to_dev(modes), k)
    cnt, idx = cnt.cpu().numpy(), idx.cpu().numpy()
    for mode in MODES.values():
        sel = np.nonzero(modes == mode)[0]
        wc, wi = oracle.topk(oracle.counts(refs, Q[sel], mode), k)
        assert np.array_equal(cnt[sel], wc), mode
        assert np.array_equal(idx[sel], wi), mode
    db.close()


@pytest.mark.parametrize("backend", ["mfma_fp4", "popcount"])
def test_long_rows_match_oracle(ctx, backend):
    """Rows far beyond one LDS chunk of the fp4 scan (restaged per chunk):
    full counts, top-k and threshold against the oracle."""
    L, n_refs, n_q = 20000, 2500, 40
    log(f"long rows L={L} backend={backend}")
    use_backend(ctx, backend)
    refs, Q = _profiles(4321, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    q = pack_rows(ctx, Q)
    for mode in MODES.values():
        want = oracle.counts(refs, Q, mode)
        assert np.array_equal(ctx.compare_full(db, q, mode).cpu().numpy(), want)
        cnt, idx = ctx.compare_topk(db, q, mode, 10)
        wc, wi = oracle.topk(want, 10)
        assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
        thr = np.sort(want, axis=1)[:, 7].astype(np.int32)
        offs, hidx, hcnt = ctx.compare_threshold(db, q, mode, to_dev(thr), cap=4096)
        wo, whi, whc = oracle.threshold(want, thr)
        assert np.array_equal(offs.cpu().numpy(), wo) and np.array_equal(hidx.cpu().numpy(), whi)
        assert np.array_equal(hcnt.cpu().numpy(), whc)
    db.close()


@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_degenerate_sizes(ctx, backend):
    """One reference, one query, one locus, every bit pair (k past the
    database: the tail is padding), and the largest k over a small
    database."""
    log(f"degenerate sizes backend={backend}")
    use_backend(ctx, backend)
    for bit_r in (0, 1):
        for bit_q in (0, 1):
            refs = np.array([[bit_r]], np.uint8)
            Q = np.array([[bit_q]], np.uint8)
            db = db_from_bytes(ctx, refs)
            q = pack_rows(ctx, Q)
            for mode in MODES.values():
                want = oracle.counts(refs, Q, mode)
                assert np.array_equal(ctx.compare_full(db, q, mode).cpu().numpy(), want)
                cnt, idx = ctx.compare_topk(db, q, mode, 3)
                wc, wi = oracle.topk(want, 3)
                assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
            db.close()
    refs, Q = _profiles(99, 3000, 5, 500)
    db = db_from_bytes(ctx, refs)
    for mode in MODES.values():
        cnt, idx = ctx.compare_topk(db, pack_rows(ctx, Q), mode, 1024)
        wc, wi = oracle.topk(oracle.counts(refs, Q, mode), 1024)
        assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
    db.close()


@pytest.mark.parametrize("backend", ["mfma_fp4", "popcount"])
def test_longest_rows(ctx, backend):
    """L = 65535, the largest row the library takes: full counts, top-k and
    threshold against the oracle."""
    L, n_refs, n_q = 65535, 300, 3
    log(f"longest rows L={L} backend={backend}")
    use_backend(ctx, backend)
    refs, Q = _profiles(65535, n_refs, n_q, L)
    db = db_from_bytes(ctx, refs)
    q = pack_rows(ctx, Q)
    for mode in MODES.values():
        want = oracle.counts(refs, Q, mode)
        assert np.array_equal(ctx.compare_full(db, q, mode).cpu().numpy(), want)
        cnt, idx = ctx.compare_topk(db, q, mode, 7)
        wc, wi = oracle.topk(want, 7)
        assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi)
        thr = np.sort(want, axis=1)[:, 4].astype(np.int32)
        offs, hidx, hcnt = ctx.compare_threshold(db, q, mode, to_dev(thr))
        wo, whi, whc = oracle.threshold(want, thr)
        assert np.array_equal(offs.cpu().numpy(), wo) and np.array_equal(hidx.cpu().numpy(), whi)
        assert np.array_equal(hcnt.cpu().numpy(), whc)
    db.close()


def test_empty_and_out_of_range_arguments(ctx):
    """No queries, k = 0, k past the limit and an unknown mode are refused
    before any work is enqueued."""
    from paper_1707_00516_amd import FID_EINVAL, FidError, fid_compare_topk
    refs, Q = _profiles(5, 200, 2, 100)
    db = db_from_bytes(ctx, refs)
    q = pack_rows(ctx, Q)
    ws = torch.empty(1 << 22, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(4096, dtype=torch.int32, device="cuda")
    idx = torch.empty(4096, dtype=torch.int64, device="cuda")
    for n_q, mode, k in [(0, 0, 4), (2, 0, 0), (2, 0, 1025), (2, 7, 4)]:
        with pytest.raises(FidError) as e:
            fid_compare_topk(ctx.handle, db.handle, q.data_ptr(), n_q, mode, k, ws.data_ptr(), ws.numel(),
                             cnt.data_ptr(), idx.data_ptr())
        assert e.value.status == FID_EINVAL, (n_q, mode, k)
    db.close()
