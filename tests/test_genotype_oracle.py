"""Pins of the genotype-level oracle (oracle/genotype.py) to facts that do
not come from it: the per-locus allele tables (tests/golden), the pinned
1-bit oracle on the two-plane expansion, the 0/1 special case (Eq. 1) and
invariants of the allele distance."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import genotype as G
from oracle_pins import read_golden


def _table(text):
    return np.array([[int(x) for x in row.split(",")] for row in text.split(";")], dtype=np.int32)


def test_per_locus_tables():
    gold = read_golden("genotype_locus_tables.txt")
    g = np.array([[0], [1], [2]], dtype=np.uint8)
    for mode, name in ((G.IDENTITY, "identity"), (G.MIXTURE, "mixture")):
        # counts()[q][r]: the golden table is [r][q]
        assert np.array_equal(G.counts(g, g, mode).T, _table(gold[name])), name


@pytest.mark.parametrize("L", [1, 7, 64, 333])
def test_equals_one_bit_oracle_on_planes(L):
    rng = np.random.default_rng(L)
    R = rng.integers(0, 3, size=(40, L), dtype=np.uint8)
    Q = rng.integers(0, 3, size=(9, L), dtype=np.uint8)
    for mode in (G.MIXTURE, G.IDENTITY):
        want = oracle.counts(G.planes(R), G.planes(Q), mode)
        assert np.array_equal(G.counts(R, Q, mode), want), mode


def test_zero_one_profiles_reduce_to_eq1():
    rng = np.random.default_rng(5)
    R = (rng.random((30, 100)) < 0.4).astype(np.uint8)
    Q = (rng.random((6, 100)) < 0.4).astype(np.uint8)
    for mode in (G.MIXTURE, G.IDENTITY):
        assert np.array_equal(G.counts(R, Q, mode), oracle.counts(R, Q, mode)), mode


def test_invariants():
    rng = np.random.default_rng(6)
    A = rng.integers(0, 3, size=(12, 90), dtype=np.uint8)
    I = G.counts(A, A, G.IDENTITY)
    M = G.counts(A, A, G.MIXTURE)
    assert np.array_equal(I, I.T) and not np.diag(I).any() and not np.diag(M).any()
    assert np.array_equal(M + M.T, I)  # excess one way plus the other is the distance
    for a in range(12):
        for b in range(12):
            assert np.all(I[a, b] <= I[a, :] + I[:, b])  # triangle inequality
    assert np.all(I <= 2 * 90)


def test_rejects_genotype_three():
    with pytest.raises(ValueError):
        G.counts(np.array([[3]], np.uint8), np.array([[0]], np.uint8), G.IDENTITY)
