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


def make_server(ctx, world, k=32, budget=256 * MB, max_queries=4096, n_chunks=5, policy=0):
    from paper_1707_00516_amd.torch_api import Server
    return Server(ctx, world[3], budget, max_queries, k, n_chunks, policy)


def test_server_mixed_requests_match_oracle(ctx, world):
    log("server: 12 mixed requests at once")
    refs = world[2]
    reqs = requests(ctx, world, 12, seed=1)
    srv = make_server(ctx, world)
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


def test_server_alone_equals_in_mix(ctx, world):
    log("server: alone vs in the mix")
    reqs = requests(ctx, world, 8, seed=2)
    srv = make_server(ctx, world, n_chunks=7)
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
