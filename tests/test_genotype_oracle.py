"""Pins of the genotype-level oracle (oracle/genotype.py) to facts that do
not come from it: a brute force over the alleles themselves (each locus of
an individual is an ordered pair of alleles, major M or minor m -- the four
genotypes MM, Mm, mM, mm of Section II-A), the pinned 1-bit oracle on the
two-plane expansion, the 0/1 special case (Eq. 1) and invariants of the
allele distance."""
from __future__ import annotations

import itertools
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle import genotype as G

GENOTYPES = [("M", "M"), ("M", "m"), ("m", "M"), ("m", "m")]


def _allele_identity(r, q):
    """Alleles that differ under the best pairing of the two individuals'
    alleles (allele order within a genotype carries no information)."""
    return min(sum(a != b for a, b in zip(r, perm)) for perm in itertools.permutations(q))


def _allele_mixture(r, q):
    """Minor-allele copies of the reference left over once each of the
    query's minor-allele copies accounts for one of them."""
    return sum((Counter(a for a in r if a == "m") - Counter(a for a in q if a == "m")).values())


def test_allele_brute_force_per_locus():
    """Every pair of the four genotypes at one locus, then every pair of
    two-locus profiles (16 x 16), counted allele by allele."""
    dosage = lambda g: sum(a == "m" for a in g)  # noqa: E731
    for L in (1, 2):
        profiles = list(itertools.product(GENOTYPES, repeat=L))
        g = np.array([[dosage(x) for x in p] for p in profiles], dtype=np.uint8)
        ident = G.counts(g, g, G.IDENTITY)  # [q][r]
        mix = G.counts(g, g, G.MIXTURE)
        for qi, qp in enumerate(profiles):
            for ri, rp in enumerate(profiles):
                assert ident[qi, ri] == sum(_allele_identity(r, q) for r, q in zip(rp, qp)), (qp, rp)
                assert mix[qi, ri] == sum(_allele_mixture(r, q) for r, q in zip(rp, qp)), (qp, rp)


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
