"""Genotype profiles (0, 1 or 2 minor alleles per locus) packed on the device
into two 1-bit planes per locus, then compared by the ordinary kernels:
allele-level counts equal the genotype oracle, bit-exact."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import genotype as G
from gpu_harness import log, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BACKENDS = {"popcount": 1, "mfma_fp4": 3}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1707_00516_amd.torch_api import Context
    c = Context(0)
    yield c
    c.sync()
    c.close()


def _genotypes(seed, n, L):
    """Hardy-Weinberg genotypes: two independent minor-allele draws per locus."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.05, 0.5, size=L)
    return ((rng.random((n, L)) < p).astype(np.uint8) + (rng.random((n, L)) < p).astype(np.uint8))


@pytest.mark.parametrize("L", [1, 333, 1000, 3000])
@pytest.mark.parametrize("backend", sorted(BACKENDS))
def test_genotype_counts_match_oracle(ctx, L, backend):
    from paper_1707_00516_amd import fid_ctx_set_backend
    n_refs, n_q, k = 3000, 37, 16
    log(f"genotypes L={L} backend={backend}")
    fid_ctx_set_backend(ctx.handle, BACKENDS[backend])
    R = _genotypes(L, n_refs, L)
    Q = np.concatenate([R[[5, 900, 2999]], _genotypes(L + 1, n_q - 3, L)])  # three exact matches
    rows = ctx.pack_genotypes(to_dev(R))
    db = ctx.build_db(rows, 2 * L)
    q = ctx.pack_genotypes(to_dev(Q))
    for mode in (G.MIXTURE, G.IDENTITY):
        want = G.counts(R, Q, mode)
        assert np.array_equal(ctx.compare_full(db, q, mode).cpu().numpy(), want), mode
        cnt, idx = ctx.compare_topk(db, q, mode, k)
        wc, wi = oracle.topk(want, k)
        assert np.array_equal(cnt.cpu().numpy(), wc) and np.array_equal(idx.cpu().numpy(), wi), mode
    db.close()
    fid_ctx_set_backend(ctx.handle, 0)


def test_genotype_pack_rejects_three(ctx):
    from paper_1707_00516_amd import FID_EINVAL, FidError
    g = np.zeros((4, 70), np.uint8)
    g[2, 69] = 3
    with pytest.raises(FidError) as e:
        ctx.pack_genotypes(to_dev(g))
    assert e.value.status == FID_EINVAL
