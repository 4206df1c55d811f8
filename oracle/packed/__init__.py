"""FastID on x86 (``cpu_packed``) -- TEST AND MEASUREMENT INFRASTRUCTURE ONLY.

A packed CPU implementation of the comparison (fastid_packed.c): profiles
packed one bit per locus into 64-bit words, Eq. 1 (mixture) or XOR
(identity) per word with a population count (Section II-A, Algorithm 2),
OpenMP threads over blocks of references, AVX-512 vpopcntq where the CPU
has it.  It is the x86 FastID-style baseline the benchmark reports and a
fast cross-check of GPU top-k results at full size.  It shares no code with
the byte oracle or the GPU library, packs its own words from 0/1 bytes, and
is pinned to the byte oracle by tests/test_cpu_packed.py.  Only the test
suite and the benchmark's CPU-baseline leg load it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "fastid_packed.c")
LIB = os.path.join(_HERE, "libfastid_packed.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build() -> None:
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", LIB, SOURCE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"cpu_packed build failed: {' '.join(cmd)}\n{r.stderr}")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.cp_words.restype = ctypes.c_int32
        L.cp_words.argtypes = [ctypes.c_int32]
        L.cp_pack.restype = ctypes.c_int
        L.cp_pack.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _u64p]
        L.cp_counts.restype = ctypes.c_int
        L.cp_counts.argtypes = [_u64p, ctypes.c_int64, _u64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                _i32p]
        L.cp_topk.restype = ctypes.c_int
        L.cp_topk.argtypes = [_u64p, ctypes.c_int64, _u64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                              ctypes.c_int32, _i32p, _i64p]
        L.cp_isa.restype = ctypes.c_int
        L.cp_isa.argtypes = []
        L.cp_num_threads.restype = ctypes.c_int
        L.cp_num_threads.argtypes = []
        _lib = L
    return _lib


def words(n_loci: int) -> int:
    return int(lib().cp_words(n_loci))


def pack(bytes_u8, out=None) -> np.ndarray:
    """0/1 bytes (n, L) -> packed rows (n, words(L)) uint64."""
    b = np.ascontiguousarray(bytes_u8, dtype=np.uint8)
    n, L = b.shape
    if out is None:
        out = np.empty((n, words(L)), dtype=np.uint64)
    assert out.flags.c_contiguous and out.shape == (n, words(L)) and out.dtype == np.uint64
    if n and lib().cp_pack(b.ctypes.data_as(_u8p), n, L, L, out.ctypes.data_as(_u64p)) != 0:
        raise ValueError("profile bytes must be 0 or 1")
    return out


def counts(refs_packed, qrys_packed, n_loci: int, mode: int) -> np.ndarray:
    r = np.ascontiguousarray(refs_packed, dtype=np.uint64)
    q = np.ascontiguousarray(qrys_packed, dtype=np.uint64)
    out = np.empty((q.shape[0], r.shape[0]), dtype=np.int32)
    if lib().cp_counts(r.ctypes.data_as(_u64p), r.shape[0], q.ctypes.data_as(_u64p), q.shape[0], n_loci, mode,
                       out.ctypes.data_as(_i32p)) != 0:
        raise ValueError("cp_counts rejected its arguments")
    return out


def topk(refs_packed, qrys_packed, n_loci: int, mode: int, k: int):
    r = np.ascontiguousarray(refs_packed, dtype=np.uint64)
    q = np.ascontiguousarray(qrys_packed, dtype=np.uint64)
    cnt = np.empty((q.shape[0], k), dtype=np.int32)
    idx = np.empty((q.shape[0], k), dtype=np.int64)
    if lib().cp_topk(r.ctypes.data_as(_u64p), r.shape[0], q.ctypes.data_as(_u64p), q.shape[0], n_loci, mode, k,
                     cnt.ctypes.data_as(_i32p), idx.ctypes.data_as(_i64p)) != 0:
        raise ValueError("cp_topk rejected its arguments")
    return cnt, idx


def isa() -> str:
    return {2: "avx512-vpopcntq", 1: "popcnt", 0: "c"}[int(lib().cp_isa())]


def num_threads() -> int:
    return int(lib().cp_num_threads())
