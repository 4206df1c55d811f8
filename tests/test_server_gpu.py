"""GPU parity of the serving loop (fid_server_*): every request's top-k
equals the oracle's, and the same request gives the same bytes alone and in
a mix with others (continuous batching, admission by budget, FIFO)."""
import numpy as np
import pytest

import gen
import oracle
from gpu_harness import db_from_bytes, log, pack_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_REFS, L = 30000, 2048
MB = 1 << 20


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1707_00516_amd.torch_api import Context
    c = Context(0)
    yield c
    c.sync()
    c.close()


@pytest.fixture(scope="module")
def world(ctx):
    seed = 5150
    thr = gen.maf_thresholds(seed, L, 0.05)
    refs = gen.ref_bytes(seed, thr, 0, N_REFS)
    db = db_from_bytes(ctx, refs)
    yield seed, thr, refs, db
    db.close()


def requests(ctx, world, n, seed):
    """Seeded requests: 1-40 queries, identity or mixture at 50/50."""
    s, thr, refs, db = world
    u = gen.u64s(seed, 4, 0, 2 * n)
    out = []
    for i in range(n):
        nq = 1 + int(u[2 * i] % 40)
        mode = int(u[2 * i + 1] % 2)
        if mode == oracle.MIXTURE:
            Q = gen.mixtures(s, thr, 0, N_REFS, (seed << 12) + 64 * i, nq, 1, 4, 0.005)[0]
        else:
            Q = gen.identity(s, thr, 0, N_REFS, (seed << 12) + 64 * i, nq, 0.005)[0]
        out.append((Q, pack_rows(ctx, Q), mode))
    return out


def oracle_topk(refs, Q, mode, k):
    return oracle.topk(oracle.counts(refs, Q, mode), k)


def make_server(ctx, world, k=32, budget=256 * MB, max_queries=4096, n_chunks=5, policy=0, tick_chunks=0):
    from paper_1707_00516_amd.torch_api import Server
    return Server(ctx, world[3], budget, max_queries, k, n_chunks, policy, tick_chunks)


# tick_chunks 0: whole-database ticks (a burst shares one pass); 1: one chunk
# per tick (requests join mid-pass and fold their running top-k)
@pytest.mark.parametrize("tick_chunks", [0, 1])
def test_server_mixed_requests_match_oracle(ctx, world, tick_chunks):
    log(f"server: 12 mixed requests at once, tick_chunks {tick_chunks}")
    refs = world[2]
    reqs = requests(ctx, world, 12, seed=1)
    srv = make_server(ctx, world, tick_chunks=tick_chunks)
    assert srv.n_chunks == 5
    tickets = [srv.submit(q, mode) for Q, q, mode in reqs]
    for (Q, q, mode), t in zip(reqs, tickets):
        cnt, idx, times = srv.wait(t, timeout_us=60_000_000)
        wc, wi = oracle_topk(refs, Q, mode, 32)
        assert np.array_equal(cnt, wc) and np.array_equal(idx, wi)
        assert times[0] <= times[1] <= times[2]
    st = srv.stats()
    assert st["completed"] == 12 and st["peak_queries_in_flight"] > 40  # shared ticks
    srv.close()


@pytest.mark.parametrize("tick_chunks", [0, 1])
def test_server_alone_equals_in_mix(ctx, world, tick_chunks):
    log(f"server: alone vs in the mix, tick_chunks {tick_chunks}")
    reqs = requests(ctx, world, 8, seed=2)
    srv = make_server(ctx, world, n_chunks=7, tick_chunks=tick_chunks)
    alone = []
    for Q, q, mode in reqs:
        alone.append(srv.wait(srv.submit(q, mode), timeout_us=60_000_000)[:2])
    tickets = [srv.submit(q, mode) for Q, q, mode in reqs]
    for (c0, i0), t in zip(alone, tickets):
        c1, i1, _ = srv.wait(t, timeout_us=60_000_000)
        assert np.array_equal(c0, c1) and np.array_equal(i0, i1)
    srv.close()


def test_server_admission_by_budget_and_smaller_k(ctx, world):
    """A budget of few slots forces queueing; results stay exact, k per request
    may be below the server's, oversize requests are refused."""
    from paper_1707_00516_amd import FID_EBUDGET, FidError
    log("server: budget admission")
    refs = world[2]
    reqs = requests(ctx, world, 10, seed=3)
    srv = make_server(ctx, world, max_queries=45, n_chunks=3)
    assert srv.slots == 45
    tickets = [srv.submit(q, mode, k=10 + i) for i, (Q, q, mode) in enumerate(reqs)]
    for i, ((Q, q, mode), t) in enumerate(zip(reqs, tickets)):
        cnt, idx, _ = srv.wait(t, timeout_us=60_000_000)
        wc, wi = oracle_topk(refs, Q, mode, 10 + i)
        assert np.array_equal(cnt, wc) and np.array_equal(idx, wi)
    assert srv.stats()["peak_queries_in_flight"] <= 45
    big = pack_rows(ctx, refs[:46])
    with pytest.raises(FidError) as e:
        srv.submit(big, 0)
    assert e.value.status == FID_EBUDGET
    srv.close()
    with pytest.raises(FidError) as e:
        make_server(ctx, world, budget=1024)
    assert e.value.status == FID_EBUDGET


def test_server_fifo_matches_continuous(ctx, world):
    from paper_1707_00516_amd import FID_SERVE_FIFO
    log("server: FIFO policy")
    refs = world[2]
    reqs = requests(ctx, world, 6, seed=4)
    srv = make_server(ctx, world, policy=FID_SERVE_FIFO)
    tickets = [srv.submit(q, mode) for Q, q, mode in reqs]
    for (Q, q, mode), t in zip(reqs, tickets):
        cnt, idx, _ = srv.wait(t, timeout_us=60_000_000)
        wc, wi = oracle_topk(refs, Q, mode, 32)
        assert np.array_equal(cnt, wc) and np.array_equal(idx, wi)
    srv.close()


# ---------------------------------------------------------------------------
# Chunks larger than the top-k seed prefix (16,384 references): ticks without
# an admission filter by the running k-th count alone (the bounded scan, with
# per-query modes), and a tick that admits requests runs the seed pass for
# everyone in flight.  These are the paths the 20M-reference serving runs.
SEED_PREFIX = 16384


def _big_world(ctx, seed, n_refs, L):
    thr = gen.maf_thresholds(seed, L, 0.05)
    refs = gen.ref_bytes(seed, thr, 0, n_refs)
    return thr, refs, db_from_bytes(ctx, refs)


def _requests(ctx, seed, thr, n_refs, n, q_max):
    u = gen.u64s(seed, 4, 0, 2 * n)
    out = []
    for i in range(n):
        nq = 1 + int(u[2 * i] % q_max)
        mode = int(u[2 * i + 1] % 2)
        if mode == oracle.MIXTURE:
            Q = gen.mixtures(seed, thr, 0, n_refs, (seed << 12) + 512 * i, nq, 1, 4, 0.005)[0]
        else:
            Q = gen.identity(seed, thr, 0, n_refs, (seed << 12) + 512 * i, nq, 0.005)[0]
        out.append((Q, pack_rows(ctx, Q), mode))
    return out


def _server_on(ctx, db, backend, **kw):
    """A server whose worker context runs `backend` (the server copies the
    creating context's backend)."""
    from paper_1707_00516_amd import fid_ctx_set_backend
    from paper_1707_00516_amd.torch_api import Server
    fid_ctx_set_backend(ctx.handle, backend)
    try:
        return Server(ctx, db, kw.get("budget", 512 * MB), kw.get("max_queries", 4096), kw.get("k", 32),
                      kw["n_chunks"], 0, kw.get("tick_chunks", 0))
    finally:
        fid_ctx_set_backend(ctx.handle, 0)


def _staggered(srv, reqs, seed, k=32):
    """Submit with seeded gaps of 0-3 ms (so that some ticks admit requests
    and others do not), then collect every result."""
    import time
    gaps = gen.u64s(seed, 5, 3, len(reqs)) % 3000
    tickets = []
    for (Q, q, mode), g in zip(reqs, gaps):
        tickets.append(srv.submit(q, mode, k=k))
        time.sleep(int(g) * 1e-6)
    return [srv.wait(t, timeout_us=120_000_000)[:2] for t in tickets]


@pytest.mark.parametrize("backend,tick_chunks", [(0, 1), (3, 1), (0, 0)])  # AUTO / fp4 forced; spans
def test_server_chunks_past_seed_prefix_match_oracle(ctx, backend, tick_chunks):
    """200,000 x 2048 references in 4 chunks of ~50,000: staggered mixed
    requests, each equal to the oracle and to the same request served alone."""
    n_refs, L = 200_000, 2048
    log(f"server: 4 chunks of {n_refs // 4} references, backend {backend}, tick_chunks {tick_chunks}")
    thr, refs, db = _big_world(ctx, 6100, n_refs, L)
    srv = _server_on(ctx, db, backend, n_chunks=4, tick_chunks=tick_chunks)
    assert srv.n_chunks == 4
    assert n_refs // srv.n_chunks > SEED_PREFIX
    reqs = _requests(ctx, 6100, thr, n_refs, 14, 90)
    mixed = _staggered(srv, reqs, 6100)
    alone = [srv.wait(srv.submit(q, mode), timeout_us=120_000_000)[:2] for Q, q, mode in reqs]
    st = srv.stats()
    srv.close()
    for (Q, q, mode), (c1, i1), (c0, i0) in zip(reqs, mixed, alone):
        wc, wi = oracle_topk(refs, Q, mode, 32)
        assert np.array_equal(c1, wc) and np.array_equal(i1, wi)
        assert np.array_equal(c0, c1) and np.array_equal(i0, i1)
    log(f"server: {st['ticks']} ticks, peak {st['peak_queries_in_flight']} queries in flight")
    db.close()


@pytest.mark.parametrize("backend", [0, 3, 1])  # AUTO, fp4 forced, popcount forced
def test_server_tail_chunk_shorter_than_k(ctx, backend):
    """20 chunks of 17,408 references and a last chunk of 20 (< k = 32): a
    request admitted on the last chunk holds fewer than k keys after its
    first tick, so its next, admission-free tick runs with no bound yet
    (0xFFFFFFFF).  Requests are submitted around the last chunk's tick and
    at seeded random gaps; every one must equal the oracle."""
    import time
    L, chunk, C = 256, 17408, 20
    n_refs = (C - 1) * chunk + 20
    log(f"server: tail chunk of 20 references, backend {backend}")
    thr, refs, db = _big_world(ctx, 6200, n_refs, L)
    srv = _server_on(ctx, db, backend, n_chunks=C, tick_chunks=1)
    assert srv.n_chunks == C
    reqs = _requests(ctx, 6200 + backend, thr, n_refs, 36, 70)
    tickets = []
    # half of the requests: submitted just after the second-to-last chunk's
    # tick starts (a keep-alive request keeps the ticks going), so they are
    # admitted on the 20-reference chunk unless a tick boundary slips past
    keep = reqs[0]
    tail_tries = 0
    for Q, q, mode in reqs[1:19]:
        tickets.append(srv.submit(keep[1], keep[2]))
        t_end = time.monotonic() + 5.0
        while time.monotonic() < t_end:
            if srv.stats()["ticks"] % C == C - 2:
                break
        tickets.append(srv.submit(q, mode))
        tail_tries += 1
        srv.wait(tickets[-2], timeout_us=120_000_000)
    rest = _staggered(srv, reqs[19:], 6200)
    # the aimed requests (the keep-alive ones, at even positions, were collected above)
    got = [srv.wait(t, timeout_us=120_000_000)[:2] for t in tickets[1::2]]
    srv.close()
    checked = list(zip(reqs[1:19], got)) + list(zip(reqs[19:], rest))
    for (Q, q, mode), (c, i) in checked:
        wc, wi = oracle_topk(refs, Q, mode, 32)
        assert np.array_equal(c, wc) and np.array_equal(i, wi)
    log(f"server: {len(checked)} requests equal the oracle ({tail_tries} aimed at the 20-reference chunk)")
    db.close()


# ---------------------------------------------------------------------------
# Per-request threshold hits, tick spans, FIFO.
def _server_cfg(ctx, db, **kw):
    from paper_1707_00516_amd.torch_api import Server
    return Server(ctx, db, kw.get("budget", 512 * MB), kw.get("max_queries", 4096), kw.get("k", 32),
                  kw.get("n_chunks", 4), kw.get("policy", 0), kw.get("tick_chunks", 0),
                  kw.get("hits_per_query", 0))


def _thresholds_for(seed, refs, Q, mode, L):
    """Per query: -1, the smallest count, the 5th, 1% of L, or a value with
    hundreds of hits."""
    rows = oracle.counts(refs, Q, mode)
    s = np.sort(rows, axis=1)
    u = gen.u64s(seed, 5, 21, Q.shape[0]) % 5
    pick = [lambda q: -1, lambda q: s[q, 0], lambda q: s[q, 4], lambda q: L // 100, lambda q: s[q, 300]]
    return rows, np.array([pick[int(u[q])](q) for q in range(Q.shape[0])], np.int32)


@pytest.mark.parametrize("policy,tick_chunks", [(0, 0), (0, 1), (0, 2), (1, 0)])
def test_server_threshold_requests_match_oracle(ctx, policy, tick_chunks):
    """Requests with and without thresholds, both modes, submitted at
    staggered times: top-k and hit CSR equal the oracle's for each request."""
    import time
    n_refs, L = 200_000, 2048
    log(f"server thresholds: policy {policy}, tick_chunks {tick_chunks}")
    thr, refs, db = _big_world(ctx, 6300, n_refs, L)
    srv = _server_cfg(ctx, db, n_chunks=4, policy=policy, tick_chunks=tick_chunks)
    reqs = _requests(ctx, 6300, thr, n_refs, 12, 60)
    want = []
    tickets = []
    gaps = gen.u64s(6300, 5, 4, len(reqs)) % 2000
    for i, ((Q, q, mode), g) in enumerate(zip(reqs, gaps)):
        rows, T = _thresholds_for(6300 + i, refs, Q, mode, L)
        with_thr = i % 3 != 2
        want.append((oracle.topk(rows, 32), oracle.threshold(rows, T) if with_thr else None))
        tickets.append(srv.submit(q, mode, thr=T if with_thr else None, hit_cap=1 << 16))
        time.sleep(int(g) * 1e-6)
    for t, ((wc, wi), wt) in zip(tickets, want):
        res = srv.wait(t, timeout_us=120_000_000)
        assert np.array_equal(res[0], wc) and np.array_equal(res[1], wi)
        if wt is None:
            assert len(res) == 3
            continue
        offs, hidx, hcnt = res[3]
        assert np.array_equal(offs, wt[0])
        assert np.array_equal(hidx, wt[1]) and np.array_equal(hcnt, wt[2])
    log(f"server thresholds: {srv.stats()['ticks']} ticks")
    srv.close()
    db.close()


def test_server_threshold_overflow(ctx, world):
    """More hits than the request's capacity: FID_EOVERFLOW with the hits
    needed in offs[-1]; the top-k is still written and exact."""
    s, thr, refs, db = world
    Q = gen.mixtures(s, thr, 0, N_REFS, 9000, 6, 1, 4, 0.005)[0]
    rows = oracle.counts(refs, Q, oracle.MIXTURE)
    T = np.full(6, 250, np.int32)
    need = int((rows <= 250).sum())
    assert need > 50
    for policy in (0, 1):
        srv = _server_cfg(ctx, db, n_chunks=3, policy=policy)
        res = srv.wait(srv.submit(pack_rows(ctx, Q), oracle.MIXTURE, thr=T, hit_cap=need - 1),
                       timeout_us=60_000_000)
        wc, wi = oracle.topk(rows, 32)
        assert np.array_equal(res[0], wc) and np.array_equal(res[1], wi)
        offs, hidx, hcnt = res[3]
        assert hidx is None and int(offs[-1]) == need
        # the server keeps serving afterwards
        res = srv.wait(srv.submit(pack_rows(ctx, Q), oracle.MIXTURE, thr=T, hit_cap=need), timeout_us=60_000_000)
        o_offs, o_idx, o_cnt = oracle.threshold(rows, T)
        assert np.array_equal(res[3][0], o_offs) and np.array_equal(res[3][1], o_idx)
        srv.close()


def test_server_whole_pass_ticks_and_spans(ctx, world):
    """A lone request takes one tick with whole-database ticks (tick_chunks =
    0), one tick per chunk with tick_chunks = 1, ceil(5 / 2) with 2; all exact."""
    s, thr, refs, db = world
    Q = gen.identity(s, thr, 0, N_REFS, 9500, 9, 0.005)[0]
    wc, wi = oracle.topk(oracle.counts(refs, Q, oracle.IDENTITY), 32)
    for tick_chunks, ticks in ((0, 1), (1, 5), (2, 3)):
        srv = _server_cfg(ctx, db, n_chunks=5, tick_chunks=tick_chunks)
        assert srv.n_chunks == 5
        c, i, _ = srv.wait(srv.submit(pack_rows(ctx, Q), oracle.IDENTITY), timeout_us=60_000_000)
        assert np.array_equal(c, wc) and np.array_equal(i, wi)
        assert srv.stats()["ticks"] == ticks, tick_chunks
        srv.close()
