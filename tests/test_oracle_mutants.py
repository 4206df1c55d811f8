"""Plant plausible mistakes in the oracle source and check that a pin catches each.

Each mutant is a copy of oracle/fastid_oracle.c with one textual change,
compiled to a temporary library on the CPU; at least one pin must fail on it.
"""
import os

import pytest

import oracle
import oracle_pins

MUTANTS = {
    "and-with-query": ("a = (uint8_t)(a & ref[k]);", "a = (uint8_t)(a & qry[k]);"),
    "or-for-xor": ("(uint8_t)(ref[k] ^ qry[k]);", "(uint8_t)(ref[k] | qry[k]);"),
    "drop-last-locus": ("for (int32_t k = 0; k < n_loci; ++k) {\n        uint8_t a",
                        "for (int32_t k = 0; k + 1 < n_loci; ++k) {\n        uint8_t a"),
    "swap-ref-and-query": (
        "oracle_count_pair(refs + r * (int64_t)n_loci, qrys + q * (int64_t)n_loci,",
        "oracle_count_pair(qrys + q * (int64_t)n_loci, refs + r * (int64_t)n_loci,"),
    "mode-inverted": ("if (mode == ORACLE_MIXTURE) a =", "if (mode != ORACLE_MIXTURE) a ="),
    "or-accumulate": ("p += a;", "p |= a;"),
    "ties-highest-index": ("return x->idx < y->idx ? -1 : 1;", "return x->idx < y->idx ? 1 : -1;"),
    "topk-descending": ("return x->count < y->count ? -1 : 1;",
                        "return x->count < y->count ? 1 : -1;"),
    "threshold-strict": ("counts[q * n_refs + r] <= thr[q]", "counts[q * n_refs + r] < thr[q]"),
    "padding-index-zero": ("out_idx[q * k + j] = -1;", "out_idx[q * k + j] = 0;"),
    "threshold-stores-query": ("idx[n] = r;", "idx[n] = q;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(oracle.SOURCE).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_oracle(str(path), str(tmp_path / "libmutant.so"))
    orc = oracle.Oracle(lib)
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(orc)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin catches mutant {name}"
