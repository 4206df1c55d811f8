"""Genotype-level counts -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section II-A describes each SNP of an individual as one of the genotypes
MM, Mm, mM, mm (major / minor alleles), i.e. 0, 1 or 2 copies of the minor
allele, and notes that comparing genotypes allele by allele is 2N
comparisons for N loci; the 1-bit encoding the rest of the paper uses keeps
only "minor allele present".  This module is the plain definition of the
allele-level counts for genotype profiles g in {0, 1, 2} per locus (the
reading is recorded with the design notes):

  identity : C[q][r] = sum over loci of |g_r - g_q|
             (minor alleles by which the two genotypes differ)
  mixture  : C[q][r] = sum over loci of max(0, g_r - g_q)
             (minor-allele copies of the reference beyond the query's; for
             a 0/1 profile this is Eq. 1)

Plain NumPy integer arithmetic, one query at a time, no packing.
Pins: tests/test_genotype_oracle.py (a brute force over the alleles of every
pair of genotypes -- best pairing of the alleles for identity, left-over
minor-allele copies for mixtures -- and equality with the 1-bit oracle
applied to the two-plane expansion).
"""
from __future__ import annotations

import numpy as np

MIXTURE = 0
IDENTITY = 1


def _genotypes(a, name):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.ndim != 2:
        raise ValueError(f"{name} must be 2-D [n, loci]")
    if a.size and int(a.max()) > 2:
        raise ValueError(f"{name}: genotypes must be 0, 1 or 2")
    return a


def counts(refs, qrys, mode):
    """int32 [n_q][n_r] allele-level counts of genotype profiles."""
    R = _genotypes(refs, "refs").astype(np.int32)
    Q = _genotypes(qrys, "qrys").astype(np.int32)
    if R.shape[1] != Q.shape[1]:
        raise ValueError("refs and qrys need the same number of loci")
    out = np.empty((Q.shape[0], R.shape[0]), dtype=np.int32)
    for q in range(Q.shape[0]):
        d = R - Q[q][None, :]
        out[q] = (np.abs(d) if mode == IDENTITY else np.maximum(d, 0)).sum(axis=1)
    return out


def planes(g):
    """The two 0/1 planes of each locus (at least one minor allele, two minor
    alleles), interleaved: locus k -> bits 2k and 2k + 1."""
    g = _genotypes(g, "g")
    out = np.empty((g.shape[0], 2 * g.shape[1]), dtype=np.uint8)
    out[:, 0::2] = g >= 1
    out[:, 1::2] = g >= 2
    return out
