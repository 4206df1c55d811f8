"""Pins of the packed x86 baseline (oracle/packed, ``cpu_packed``) to the byte
oracle: the full count matrix of the 64 x 20,000 x 2,048 mixture workload,
random profiles at every word-tail length, both modes, and top-k with ties,
duplicated rows and k above the reference count.  The two CPU programs share
no code (the byte oracle never sees a packed word), so agreement pins the
packed one before it is used as a full-size cross-check of the GPU."""
import numpy as np
import pytest

import gen
import oracle
import oracle.packed as cp
from gen.workloads import MIX_64x20K


def test_config1_full_matrix_equals_byte_oracle():
    w = MIX_64x20K
    thr = gen.maf_thresholds(w.seed, w.n_loci, w.maf_lo)
    refs = gen.ref_bytes(w.seed, thr, 0, w.n_refs)
    Q = gen.mixtures(w.seed, thr, 0, w.n_refs, 0, w.n_q, w.nc_lo, w.nc_hi, w.flip)[0]
    R, P = cp.pack(refs), cp.pack(Q)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        assert np.array_equal(cp.counts(R, P, w.n_loci, mode), oracle.counts(refs, Q, mode)), mode


@pytest.mark.parametrize("L", [1, 2, 63, 64, 65, 127, 128, 511, 512, 513, 1000, 3000])
def test_random_profiles_all_tails(L):
    rng = np.random.default_rng(L + 17)
    refs = (rng.random((1203, L)) < rng.uniform(0.05, 0.6)).astype(np.uint8)
    Q = (rng.random((13, L)) < 0.4).astype(np.uint8)
    R, P = cp.pack(refs), cp.pack(Q)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        want = oracle.counts(refs, Q, mode)
        assert np.array_equal(cp.counts(R, P, L, mode), want), mode
        for k in (1, 7, 32):
            c, i = cp.topk(R, P, L, mode, k)
            wc, wi = oracle.topk(want, k)
            assert np.array_equal(c, wc) and np.array_equal(i, wi), (mode, k)


def test_topk_ties_duplicates_and_padding():
    L = 200
    rng = np.random.default_rng(3)
    base = (rng.random((40, L)) < 0.3).astype(np.uint8)
    refs = np.concatenate([base, base, base[::-1]])  # every row three times
    Q = base[:5]
    R, P = cp.pack(refs), cp.pack(Q)
    for mode in (oracle.MIXTURE, oracle.IDENTITY):
        for k in (5, 120, 200):  # 200 > 120 references: padded
            c, i = cp.topk(R, P, L, mode, k)
            wc, wi = oracle.topk(oracle.counts(refs, Q, mode), k)
            assert np.array_equal(c, wc) and np.array_equal(i, wi), (mode, k)
    zero = np.zeros((300, 64), np.uint8)
    c, i = cp.topk(cp.pack(zero), cp.pack(zero[:2]), 64, oracle.MIXTURE, 10)
    assert np.all(c == 0) and np.array_equal(i, np.tile(np.arange(10), (2, 1)))


def test_pack_layout_and_rejection():
    b = np.zeros((2, 70), np.uint8)
    b[0, 0] = b[0, 63] = b[1, 64] = b[1, 69] = 1
    p = cp.pack(b)
    assert p.shape == (2, 2)
    assert p[0, 0] == (1 | (1 << 63)) and p[0, 1] == 0
    assert p[1, 0] == 0 and p[1, 1] == (1 | (1 << 5))
    b[1, 3] = 2
    with pytest.raises(ValueError):
        cp.pack(b)
