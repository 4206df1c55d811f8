"""FastID oracle -- TEST INFRASTRUCTURE ONLY.

A plain CPU implementation (fastid_oracle.c, a loop over unpacked 0/1 locus
bytes) of what the GPU library computes, used to prove the library's results.
Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the library itself never does, and shares no code
with it.

Functions follow arXiv 1707.00516: Section II-A Eq. 1 (mixture mode),
Section II-A's XOR identity comparison, Algorithm 2 (all pairs) and
Section II-B (the overloaded product C = AB, stored here query-major).
Top-k and threshold selection are the per-query reductions Section IV
proposes moving onto the GPU, defined here by a full sort of each row.

Pins (tests/test_oracle_pins.py): the worked encoding example of Section II-A,
per-locus truth tables, exhaustive brute force on tiny profiles by set
algebra, closed forms through NumPy integer matmul and ``np.bitwise_count``,
invariants, the noisy-contributor identity, and mutation tests that plant
plausible mistakes in this file and check that a pin catches each one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

MIXTURE = 0
IDENTITY = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "fastid_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def compile_oracle(source: str = SOURCE, out: str = LIB) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", out, source]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle build failed: {' '.join(cmd)}\n{r.stderr}")
    return out


def build(verbose: bool = False) -> None:
    compile_oracle()
    if verbose:
        print("built", LIB)


def _bytes2d(a, name):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.ndim != 2:
        raise ValueError(f"{name} must be 2-D (rows, loci)")
    if a.size and a.max() > 1:
        raise ValueError(f"{name} must hold 0/1 bytes")
    return a


class Oracle:
    """ctypes view of one compiled oracle library (the real one, or a mutant
    built by the mutation tests)."""

    def __init__(self, path: str = LIB):
        if path == LIB and not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(path)
        lib.oracle_count_pair.restype = ctypes.c_int32
        lib.oracle_count_pair.argtypes = [_u8p, _u8p, ctypes.c_int32, ctypes.c_int]
        lib.oracle_counts.restype = ctypes.c_int
        lib.oracle_counts.argtypes = [_u8p, ctypes.c_int64, _u8p, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_int, _i32p]
        lib.oracle_count_pairs.restype = ctypes.c_int
        lib.oracle_count_pairs.argtypes = [_u8p, _u8p, ctypes.c_int32, ctypes.c_int,
                                           _i64p, _i64p, ctypes.c_int64, _i32p]
        lib.oracle_topk.restype = ctypes.c_int
        lib.oracle_topk.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                    _i32p, _i64p]
        lib.oracle_threshold.restype = ctypes.c_int64
        lib.oracle_threshold.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int64, _i32p,
                                         ctypes.c_int64, _i64p, _i64p, _i32p]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        self.lib = lib

    def counts(self, refs, qrys, mode: int) -> np.ndarray:
        """C[q, r] for all query rows q and reference rows r (Algorithm 2)."""
        refs = _bytes2d(refs, "refs")
        qrys = _bytes2d(qrys, "qrys")
        if refs.shape[1] != qrys.shape[1]:
            raise ValueError("refs and queries must have the same number of loci")
        out = np.empty((qrys.shape[0], refs.shape[0]), dtype=np.int32)
        rc = self.lib.oracle_counts(refs.ctypes.data_as(_u8p), refs.shape[0],
                                    qrys.ctypes.data_as(_u8p), qrys.shape[0],
                                    refs.shape[1], mode, out.ctypes.data_as(_i32p))
        if rc != 0:
            raise ValueError("oracle_counts rejected its arguments")
        return out

    def count_pairs(self, refs, qrys, ref_rows, qry_rows, mode: int) -> np.ndarray:
        refs = _bytes2d(refs, "refs")
        qrys = _bytes2d(qrys, "qrys")
        rr = np.ascontiguousarray(ref_rows, dtype=np.int64)
        qq = np.ascontiguousarray(qry_rows, dtype=np.int64)
        if rr.shape != qq.shape:
            raise ValueError("row lists differ in length")
        if rr.size and (rr.min() < 0 or rr.max() >= refs.shape[0] or qq.min() < 0
                        or qq.max() >= qrys.shape[0]):
            raise IndexError("row index out of range")
        out = np.empty(rr.size, dtype=np.int32)
        self.lib.oracle_count_pairs(refs.ctypes.data_as(_u8p), qrys.ctypes.data_as(_u8p),
                                    refs.shape[1], mode, rr.ctypes.data_as(_i64p),
                                    qq.ctypes.data_as(_i64p), rr.size,
                                    out.ctypes.data_as(_i32p))
        return out

    def topk(self, counts, k: int):
        """k smallest (count, index) pairs of each row; (INT32_MAX, -1) padding."""
        c = np.ascontiguousarray(counts, dtype=np.int32)
        nq, nr = c.shape
        cnt = np.empty((nq, k), dtype=np.int32)
        idx = np.empty((nq, k), dtype=np.int64)
        rc = self.lib.oracle_topk(c.ctypes.data_as(_i32p), nq, nr, k,
                                  cnt.ctypes.data_as(_i32p), idx.ctypes.data_as(_i64p))
        if rc != 0:
            raise ValueError("oracle_topk rejected its arguments")
        return cnt, idx

    def threshold(self, counts, thr):
        """CSR of hits count <= thr[q]: (offs[nq+1], idx ascending per row, cnt)."""
        c = np.ascontiguousarray(counts, dtype=np.int32)
        nq, nr = c.shape
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(thr, dtype=np.int32), (nq,)))
        offs = np.empty(nq + 1, dtype=np.int64)
        n = self.lib.oracle_threshold(c.ctypes.data_as(_i32p), nq, nr, t.ctypes.data_as(_i32p),
                                      0, offs.ctypes.data_as(_i64p), None, None)
        idx = np.empty(max(n, 1), dtype=np.int64)
        cnt = np.empty(max(n, 1), dtype=np.int32)
        n2 = self.lib.oracle_threshold(c.ctypes.data_as(_i32p), nq, nr, t.ctypes.data_as(_i32p),
                                       n, offs.ctypes.data_as(_i64p), idx.ctypes.data_as(_i64p),
                                       cnt.ctypes.data_as(_i32p))
        if n2 != n:
            raise RuntimeError("oracle_threshold count changed between passes")
        return offs, idx[:n], cnt[:n]

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def counts(refs, qrys, mode):
    return default().counts(refs, qrys, mode)


def count_pairs(refs, qrys, ref_rows, qry_rows, mode):
    return default().count_pairs(refs, qrys, ref_rows, qry_rows, mode)


def topk(c, k):
    return default().topk(c, k)


def threshold(c, thr):
    return default().threshold(c, thr)


def num_threads():
    return default().num_threads()
