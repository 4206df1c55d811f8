"""GPU parity of ragged batches (fid_batch_*): every job of one persistent
launch against the oracle's top-k of that job alone, bit-exact, eagerly and
through repeated HIP-graph replays."""
import numpy as np
import pytest

import gen
import oracle
from gpu_harness import db_from_bytes, log, pack_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PANELS = {1000: 9000, 2048: 7000, 3100: 5000}  # loci -> database size


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
def panels(ctx):
    out = {}
    for L, n in PANELS.items():
        seed = 4242 + L
        thr = gen.maf_thresholds(seed, L, 0.05)
        refs = gen.ref_bytes(seed, thr, 0, n)
        out[L] = (seed, thr, refs, db_from_bytes(ctx, refs))
    yield out
    for v in out.values():
        v[3].close()


def make_jobs(ctx, panels, n_jobs, seed):
    """Seeded ragged jobs: random panel, slice, query count and mode."""
    u = gen.u64s(seed, 4, 0, 6 * n_jobs)
    specs = []
    for j in range(n_jobs):
        L = sorted(PANELS)[int(u[6 * j] % len(PANELS))]
        s, thr, refs, db = panels[L]
        n = refs.shape[0]
        r_lo = int(u[6 * j + 1] % (n // 2))
        r_hi = min(n, r_lo + 1 + int(u[6 * j + 2] % n))
        if j == 0:
            r_lo, r_hi = 0, n            # whole database
        if j == 1:
            r_lo, r_hi = 77, 77 + 20     # fewer references than k: padded tail
        nq = 1 + int(u[6 * j + 3] % 23)
        mode = int(u[6 * j + 4] % 2)
        if mode == oracle.MIXTURE:
            Q = gen.mixtures(s, thr, r_lo, r_hi - r_lo, 1000 * j, nq, 1, 4, 0.005)[0]
        else:
            Q = gen.identity(s, thr, r_lo, r_hi - r_lo, 1000 * j, nq, 0.005)[0]
        specs.append((L, r_lo, r_hi, Q, mode))
    jobs = [(panels[L][3], r_lo, r_hi, pack_rows(ctx, Q), mode) for L, r_lo, r_hi, Q, mode in specs]
    return specs, jobs


def expected(panels, specs, k):
    out = []
    for L, r_lo, r_hi, Q, mode in specs:
        refs = panels[L][2][r_lo:r_hi]
        c, i = oracle.topk(oracle.counts(refs, Q, mode), k)
        out.append((c, np.where(i >= 0, i + r_lo, -1)))
    return out


BACKENDS = {"auto": 0, "popcount": 1, "int8": 2, "fp4": 3}


def batch_on(ctx, backend, jobs, k, tune=None):
    """A batch planned with `backend` forced on the context (the plan keeps
    its routing; the context goes back to AUTO)."""
    from paper_1707_00516_amd import fid_ctx_set_backend
    from paper_1707_00516_amd.torch_api import Batch
    fid_ctx_set_backend(ctx.handle, BACKENDS[backend])
    try:
        return Batch(ctx, jobs, k, tune)
    finally:
        fid_ctx_set_backend(ctx.handle, 0)


def check(batch, want):
    for j, (wc, wi) in enumerate(want):
        assert np.array_equal(batch.cnt[j].cpu().numpy(), wc), f"job {j} counts"
        assert np.array_equal(batch.idx[j].cpu().numpy(), wi), f"job {j} indices"


# AUTO runs every job on the batched fp4 passes; the popcount backend runs
# them all on the persistent popcount launch, whose item shapes the tuning
# entries (panel, queries per item, blocks per item) set.
@pytest.mark.parametrize("backend", ["auto", "popcount"])
@pytest.mark.parametrize("tune", [None, [(0, 1, 1)], [(0, 5, 3), (2048, 16, 64)],
                                  [(1000, 7, 2), (3100, 2, 9)], [(0, 32, 7)]])
def test_batch_matches_oracle(ctx, panels, tune, backend):
    k = 32
    log(f"batch tune={tune} backend={backend}")
    specs, jobs = make_jobs(ctx, panels, 14, seed=99)
    b = batch_on(ctx, backend, jobs, k, tune)
    assert b.info()[3] == (14 if backend == "auto" else 0)
    b.run()
    ctx.sync()
    check(b, expected(panels, specs, k))
    b.close()


@pytest.mark.parametrize("backend", ["auto", "popcount"])
def test_batch_graph_replays(ctx, panels, backend):
    """Captured once, replayed several times with eager work between the
    replays; every replay must equal the oracle."""
    k = 17
    log(f"batch graph replays, backend={backend}")
    specs, jobs = make_jobs(ctx, panels, 9, seed=7)
    want = expected(panels, specs, k)
    b = batch_on(ctx, backend, jobs, k, [(0, 4, 5)])
    for rep in range(3):
        for c, i in zip(b.cnt, b.idx):
            c.fill_(-7)
            i.fill_(-7)
        b.run(use_graph=True)
        ctx.sync()
        check(b, want)
        b.run(use_graph=False)  # eager run between replays
        ctx.sync()
        check(b, want)
    b.close()


def test_batch_alone_equals_in_batch(ctx, panels):
    """A job's result is the same run alone, in a batch, and through the
    per-call top-k entry point."""
    from paper_1707_00516_amd.torch_api import Batch
    k = 32
    specs, jobs = make_jobs(ctx, panels, 6, seed=1234)
    b = Batch(ctx, jobs, k)
    b.run()
    ctx.sync()
    for j, job in enumerate(jobs):
        alone = Batch(ctx, [job], k)
        alone.run()
        ctx.sync()
        assert torch.equal(alone.cnt[0], b.cnt[j]) and torch.equal(alone.idx[0], b.idx[j])
        alone.close()
        db, r_lo, r_hi, q, mode = job
        if r_lo == 0 and r_hi == db.n_refs:
            c, i = ctx.compare_topk(db, q, mode, k)
            assert torch.equal(c, b.cnt[j]) and torch.equal(i, b.idx[j])
    b.close()


def test_batch_rejects_bad_jobs(ctx, panels):
    from paper_1707_00516_amd import FID_EINVAL, FidError
    from paper_1707_00516_amd.torch_api import Batch
    s, thr, refs, db = panels[1000]
    q = pack_rows(ctx, refs[:3])
    for bad in [(db, 5, 5, q, 0), (db, 0, refs.shape[0] + 1, q, 0), (db, 0, 10, q, 2)]:
        with pytest.raises(FidError) as e:
            Batch(ctx, [bad], 8)
        assert e.value.status == FID_EINVAL
    with pytest.raises(FidError):
        Batch(ctx, [(db, 0, 10, q, 0)], 129)
    with pytest.raises(FidError):
        Batch(ctx, [(db, 0, 10, q, 0)], 8, tune=[(0, 33, 1)])


@pytest.mark.parametrize("backend,routed", [("auto", [True, True, True, True]),
                                            ("int8", [True, False, True, True]),
                                            ("popcount", [False, False, False, False])])
def test_batch_routes_jobs_by_family(ctx, panels, backend, routed):
    """AUTO sends every job, 3-query jobs included, to the batched fp4
    passes; with int8 forced, jobs whose rows the int8 kernel holds (at most
    2304 loci) run as per-call int8 top-k inside the batch and the 3100-locus
    job stays on the persistent popcount launch; with popcount forced all
    share that launch.  Eagerly and in the graph, all equal the oracle."""
    k = 32
    log(f"batch routing, backend={backend}")
    specs = []
    for L, nq, mode in [(2048, 150, 0), (3100, 200, 1), (1000, 5, 1), (2048, 3, 0)]:
        s, thr, refs, db = panels[L]
        n = refs.shape[0]
        if mode == oracle.MIXTURE:
            Q = gen.mixtures(s, thr, 100, n - 300, 7000 + L, nq, 1, 4, 0.005)[0]
        else:
            Q = gen.identity(s, thr, 100, n - 300, 7000 + L, nq, 0.005)[0]
        specs.append((L, 100, n - 200, Q, mode))
    jobs = [(panels[L][3], lo, hi, pack_rows(ctx, Q), m) for L, lo, hi, Q, m in specs]
    b = batch_on(ctx, backend, jobs, k)
    assert b.info()[3] == sum(routed)
    assert [b.routed(j) for j in range(4)] == routed
    from paper_1707_00516_amd import FidError
    with pytest.raises(FidError):
        b.routed(4)
    want = expected(panels, specs, k)
    for use_graph in (False, True, True):
        for c, i in zip(b.cnt, b.idx):
            c.fill_(-7)
            i.fill_(-7)
        b.run(use_graph=use_graph)
        ctx.sync()
        check(b, want)
    b.close()


def test_context_close_releases_its_batches(panels):
    """Closing a context first releases the batches made on it (a batch
    outliving its context would otherwise be destroyed on a freed one)."""
    from paper_1707_00516_amd.torch_api import Batch, Context
    log("batch released with its context")
    own = Context(0)
    s, thr, refs, db = panels[1000]
    Q = gen.mixtures(s, thr, 0, refs.shape[0], 9100, 3, 1, 4, 0.005)[0]
    b = Batch(own, [(db, 0, refs.shape[0], pack_rows(own, Q), oracle.MIXTURE)], 8)
    b.run()
    own.sync()
    own.close()
    assert b.handle == 0
    b.close()


@pytest.mark.parametrize("tune", [None, [(0, 16, 64, 1)], [(0, 16, 64, 3), (2048, 8, 32, 2)]])
def test_batch_all_jobs_on_batched_fp4(ctx, panels, tune):
    """The fp4 backend forced on the context: every job -- 1-query jobs,
    slices shorter than k and than the seed prefix (counted directly),
    whole panels past the seed prefix, chunked rows (3100 loci) -- runs in
    the batched fp4 passes; small item sizes give many reference runs per
    query tile.  Eagerly and replayed from a graph, every job equals the
    oracle."""
    from paper_1707_00516_amd import fid_ctx_set_backend
    from paper_1707_00516_amd.torch_api import Batch
    k = 32
    log(f"batch on the batched fp4 passes, tune={tune}")
    specs, jobs = make_jobs(ctx, panels, 12, seed=4321)
    fid_ctx_set_backend(ctx.handle, 3)
    try:
        b = Batch(ctx, jobs, k, tune)
    finally:
        fid_ctx_set_backend(ctx.handle, 0)
    assert b.info()[3] == 12 and all(b.routed(j) for j in range(12))
    want = expected(panels, specs, k)
    for use_graph in (False, True, True):
        for c, i in zip(b.cnt, b.idx):
            c.fill_(-7)
            i.fill_(-7)
        b.run(use_graph=use_graph)
        ctx.sync()
        check(b, want)
    b.close()


def test_batch_fp4_jobs_past_the_seed_prefix(ctx):
    """Batched fp4 jobs whose slices exceed the seed prefix (so the seed
    pass, seed selection, witness levels, the top-k pass and the merge all
    run), on two panels, both modes, with partial query tiles."""
    from paper_1707_00516_amd.torch_api import Batch
    k = 32
    specs = []
    worlds = {}
    for L in (1000, 2600):
        seed = 4600 + L
        thr = gen.maf_thresholds(seed, L, 0.05)
        refs = gen.ref_bytes(seed, thr, 0, 90_000)
        worlds[L] = (seed, thr, refs, db_from_bytes(ctx, refs))
    for j, (L, r_lo, r_hi, nq, mode) in enumerate([(1000, 0, 90_000, 150, 0), (2600, 5_000, 88_000, 200, 1),
                                                    (1000, 17, 70_017, 130, 1), (2600, 0, 40_000, 300, 0)]):
        s, thr, refs, db = worlds[L]
        if mode == oracle.MIXTURE:
            Q = gen.mixtures(s, thr, r_lo, r_hi - r_lo, 100 * j, nq, 1, 4, 0.005)[0]
        else:
            Q = gen.identity(s, thr, r_lo, r_hi - r_lo, 100 * j, nq, 0.005)[0]
        specs.append((L, r_lo, r_hi, Q, mode))
    jobs = [(worlds[L][3], lo, hi, pack_rows(ctx, Q), m) for L, lo, hi, Q, m in specs]
    b = Batch(ctx, jobs, k, [(0, 16, 64, 8)])
    assert b.info()[3] == 4
    for use_graph in (False, True):
        b.run(use_graph=use_graph)
        ctx.sync()
        for j, (L, r_lo, r_hi, Q, mode) in enumerate(specs):
            refs = worlds[L][2][r_lo:r_hi]
            wc, wi = oracle.topk(oracle.counts(refs, Q, mode), k)
            assert np.array_equal(b.cnt[j].cpu().numpy(), wc), j
            assert np.array_equal(b.idx[j].cpu().numpy(), np.where(wi >= 0, wi + r_lo, -1)), j
    b.close()
    for w in worlds.values():
        w[3].close()
