"""Pins of the oracle to facts that do not come from the oracle itself.

Each ``pin_*`` function takes an ``oracle.Oracle`` (the real library or a
mutant built by test_oracle_mutants.py) and raises AssertionError when the
oracle disagrees with:

* the worked encoding example printed in Section II-A (tests/golden/),
* the per-locus truth table of Eq. 1 and of the XOR identity comparison,
* set algebra on every pair of tiny profiles (exhaustive, L <= 4),
* closed forms through independent library routes: NumPy integer matmul for
  the 0/1 dot product and ``np.bitwise_count`` on ``np.packbits`` words,
* invariants (symmetry, self-distance, complement, triangle inequality,
  bounds, the mixture/XOR partition identity),
* the noisy-contributor identity from the generator's own bookkeeping,
* hand-worked selection cases and a brute-force selection by Python sorting.
"""
from __future__ import annotations

import os

import numpy as np

import gen
from oracle import IDENTITY, MIXTURE

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name: str) -> dict:
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(None, 1)
            vals[key] = val
    return vals


def _rand_bits(rng, shape, p):
    return (rng.random(shape) < p).astype(np.uint8)


def pin_truth_table(orc):
    # Eq. 1 per locus: counted iff the reference has the minor allele and the
    # query does not.  XOR: counted iff the two differ.
    r = np.array([[0], [0], [1], [1]], dtype=np.uint8)
    q = np.array([[0], [1], [0], [1]], dtype=np.uint8)
    mix = [int(orc.counts(r[i:i + 1], q[i:i + 1], MIXTURE)[0, 0]) for i in range(4)]
    xor = [int(orc.counts(r[i:i + 1], q[i:i + 1], IDENTITY)[0, 0]) for i in range(4)]
    assert mix == [0, 0, 1, 0], mix
    assert xor == [0, 1, 1, 0], xor


def worked_example_bits():
    g = read_golden("worked_example_encoding.txt")
    binary = g["binary"].replace(" ", "")
    assert len(binary) == 32
    assert int(binary, 2) == int(g["hex"], 16) == int(g["decimal"])
    return np.array([[int(c) for c in binary]], dtype=np.uint8), binary


def pin_worked_example(orc):
    ex, binary = worked_example_bits()
    ones = binary.count("1")
    zero = np.zeros_like(ex)
    assert ones == 5
    assert int(orc.counts(ex, zero, MIXTURE)[0, 0]) == ones
    assert int(orc.counts(ex, zero, IDENTITY)[0, 0]) == ones
    assert int(orc.counts(ex, ex, MIXTURE)[0, 0]) == 0
    assert int(orc.counts(ex, ex, IDENTITY)[0, 0]) == 0
    assert int(orc.counts(zero, ex, MIXTURE)[0, 0]) == 0
    assert int(orc.counts(zero, ex, IDENTITY)[0, 0]) == ones
    assert int(orc.counts(ex, 1 - ex, MIXTURE)[0, 0]) == ones
    assert int(orc.counts(ex, 1 - ex, IDENTITY)[0, 0]) == 32
    # 512 SNPs <-> 16 unsigned 32-bit words: one bit per SNP.
    g = read_golden("worked_example_encoding.txt")
    assert int(g["snps_per_profile"]) == 32 * int(g["words_u32"])


def pin_bruteforce_sets(orc):
    for L in range(1, 5):
        pats = np.array([[(v >> k) & 1 for k in range(L)] for v in range(1 << L)], dtype=np.uint8)
        mix = orc.counts(pats, pats, MIXTURE)  # [q][r]
        xor = orc.counts(pats, pats, IDENTITY)
        for qi in range(1 << L):
            qs = {k for k in range(L) if pats[qi, k]}
            for ri in range(1 << L):
                rs = {k for k in range(L) if pats[ri, k]}
                assert mix[qi, ri] == len(rs - qs), (L, qi, ri)
                assert xor[qi, ri] == len(rs ^ qs), (L, qi, ri)


TAIL_LENGTHS = (1, 31, 32, 33, 63, 64, 65, 127, 1000)


def pin_closed_forms_matmul(orc, seed=11):
    rng = np.random.default_rng(seed)
    for L in TAIL_LENGTHS:
        R = _rand_bits(rng, (13, L), rng.uniform(0.05, 0.95))
        Q = _rand_bits(rng, (7, L), rng.uniform(0.05, 0.95))
        dot = Q.astype(np.int64) @ R.astype(np.int64).T      # pc(R AND Q), [q][r]
        pr = R.sum(axis=1, dtype=np.int64)[None, :]
        pq = Q.sum(axis=1, dtype=np.int64)[:, None]
        assert np.array_equal(orc.counts(R, Q, MIXTURE), pr - dot), L
        assert np.array_equal(orc.counts(R, Q, IDENTITY), pr + pq - 2 * dot), L


def pin_packed_popcount(orc, seed=12):
    rng = np.random.default_rng(seed)
    for L in TAIL_LENGTHS:
        R = _rand_bits(rng, (9, L), 0.3)
        Q = _rand_bits(rng, (5, L), 0.6)
        Rp = np.packbits(R, axis=1, bitorder="little")
        Qp = np.packbits(Q, axis=1, bitorder="little")
        xor = np.bitwise_count(Rp[None, :, :] ^ Qp[:, None, :]).sum(axis=2, dtype=np.int64)
        mix = np.bitwise_count(Rp[None, :, :] & ~Qp[:, None, :]).sum(axis=2, dtype=np.int64)
        assert np.array_equal(orc.counts(R, Q, IDENTITY), xor), L
        assert np.array_equal(orc.counts(R, Q, MIXTURE), mix), L


def pin_invariants(orc, seed=13):
    rng = np.random.default_rng(seed)
    for L in (5, 64, 257):
        A = _rand_bits(rng, (11, L), 0.4)
        B = _rand_bits(rng, (6, L), 0.2)
        pa = A.sum(axis=1).astype(np.int64)
        xab = orc.counts(A, B, IDENTITY)
        xba = orc.counts(B, A, IDENTITY)
        assert np.array_equal(xab, xba.T)                           # symmetric
        xaa = orc.counts(A, A, IDENTITY)
        assert np.all(np.diag(xaa) == 0)                            # zero on self
        assert np.all(np.diag(orc.counts(A, 1 - A, IDENTITY)) == L)  # complement
        for i in range(A.shape[0]):                                 # triangle inequality
            assert np.all(xaa[i][:, None] <= xaa[i][None, :] + xaa)
        mab = orc.counts(A, B, MIXTURE)
        mba = orc.counts(B, A, MIXTURE)
        assert np.all(np.diag(orc.counts(A, A, MIXTURE)) == 0)       # MIX(R, R) = 0
        ones = np.ones((1, L), dtype=np.uint8)
        zeros = np.zeros((1, L), dtype=np.uint8)
        assert np.all(orc.counts(A, ones, MIXTURE) == 0)             # all present -> 0
        assert np.array_equal(orc.counts(A, zeros, MIXTURE)[0], pa)  # none present -> pc(R)
        assert np.all((mab >= 0) & (mab <= pa[None, :]))             # 0 <= MIX <= pc(R)
        assert np.array_equal(mab + mba.T, xab)                      # R&~Q, Q&~R split R^Q


def pin_contributors(orc, seed=14):
    """A mixture M = OR(contributors) XOR F: for a contributor R, MIX(R, M) =
    pc(R AND F); without flips it is 0."""
    thr = gen.maf_thresholds(seed, 600, 0.05)
    pool = 40
    refs = gen.ref_bytes(seed, thr, 0, pool)
    for flip in (0.0, 0.05):
        M, contrib, ncon, F = gen.mixtures(seed, thr, 0, pool, 0, 12, 1, 4, flip)
        c = orc.counts(refs, M, MIXTURE)
        for q in range(M.shape[0]):
            for j in range(ncon[q]):
                r = int(contrib[q, j])
                want = int((refs[r] & F[q]).sum())
                assert c[q, r] == want, (flip, q, r)
                if flip == 0.0:
                    assert c[q, r] == 0


def pin_topk_cases(orc, seed=15):
    c = np.array([[5, 3, 3, 7, 0]], dtype=np.int32)
    cnt, idx = orc.topk(c, 3)
    assert cnt.tolist() == [[0, 3, 3]] and idx.tolist() == [[4, 1, 2]]
    cnt, idx = orc.topk(c, 7)                                       # k > N_R: padding
    assert cnt.tolist() == [[0, 3, 3, 5, 7, 2**31 - 1, 2**31 - 1]]
    assert idx.tolist() == [[4, 1, 2, 0, 3, -1, -1]]
    z = np.zeros((2, 50), dtype=np.int32)                           # all ties -> lowest idx
    cnt, idx = orc.topk(z, 32)
    assert np.all(cnt == 0) and np.all(idx == np.arange(32)[None, :])
    rng = np.random.default_rng(seed)
    for k in (1, 5, 32):
        m = rng.integers(0, 6, size=(4, 40)).astype(np.int32)
        cnt, idx = orc.topk(m, k)
        for q in range(4):
            want = sorted((int(m[q, r]), r) for r in range(40))[:k]
            assert [(int(a), int(b)) for a, b in zip(cnt[q], idx[q])] == want


def pin_threshold_cases(orc, seed=16):
    c = np.array([[5, 3, 3, 7, 0], [9, 9, 9, 9, 9]], dtype=np.int32)
    offs, idx, cnt = orc.threshold(c, [3, 8])
    assert offs.tolist() == [0, 3, 3]
    assert idx.tolist() == [1, 2, 4] and cnt.tolist() == [3, 3, 0]
    rng = np.random.default_rng(seed)
    m = rng.integers(0, 20, size=(6, 70)).astype(np.int32)
    t = rng.integers(0, 20, size=6).astype(np.int32)
    offs, idx, cnt = orc.threshold(m, t)
    for q in range(6):
        want = [r for r in range(70) if m[q, r] <= t[q]]
        assert idx[offs[q]:offs[q + 1]].tolist() == want
        assert cnt[offs[q]:offs[q + 1]].tolist() == [int(m[q, r]) for r in want]


def pin_count_pairs(orc, seed=17):
    rng = np.random.default_rng(seed)
    R = _rand_bits(rng, (20, 77), 0.3)
    Q = _rand_bits(rng, (9, 77), 0.5)
    rr = rng.integers(0, 20, size=50)
    qq = rng.integers(0, 9, size=50)
    for mode in (MIXTURE, IDENTITY):
        full = orc.counts(R, Q, mode)
        assert np.array_equal(orc.count_pairs(R, Q, rr, qq, mode), full[qq, rr])


ALL_PINS = (pin_truth_table, pin_worked_example, pin_bruteforce_sets, pin_closed_forms_matmul,
            pin_packed_popcount, pin_invariants, pin_contributors, pin_topk_cases,
            pin_threshold_cases, pin_count_pairs)
