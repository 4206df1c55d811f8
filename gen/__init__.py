"""Seeded synthetic SNP profiles shared by the oracle side and the GPU side.

This module only synthesises inputs: per-locus minor-allele frequencies,
Bernoulli reference profiles, mixtures (OR of contributor profiles plus random
bit flips) and single-source queries.  It holds none of the comparison
arithmetic.  All draws are counter-based (splitmix64 of a key built from seed,
stream, row and column; see fidgen.c), so any row can be regenerated alone,
and the CPU library, the GPU kernel and the NumPy twin below agree bit for bit.

The paper's profiles are not available; these generators stand in for them
with the sizes and value distributions of its workloads (see workloads.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
CPU_LIB = os.path.join(_HERE, "libfidgen_cpu.so")
GPU_LIB = os.path.join(_HERE, "libfidgen_gpu.so")

MASTER_SEED = 1707005160

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(verbose: bool = False) -> None:
    """Compile the CPU generator (gcc) and the GPU generator (hipcc, gfx950)."""
    cmds = [
        ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", CPU_LIB, os.path.join(_HERE, "fidgen.c")],
        ["hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-o", GPU_LIB, os.path.join(_HERE, "fidgen_gpu.hip")],
    ]
    for c in cmds:
        r = subprocess.run(c, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"generator build failed: {' '.join(c)}\n{r.stderr}")
        if verbose:
            print(" ".join(c))


_cpu = None
_gpu = None


def _ptr(a, t):
    return a.ctypes.data_as(t)


def cpu_lib():
    global _cpu
    if _cpu is None:
        if not os.path.exists(CPU_LIB):
            build()
        lib = ctypes.CDLL(CPU_LIB)
        lib.fg_mix.restype = ctypes.c_uint64
        lib.fg_mix.argtypes = [ctypes.c_uint64]
        lib.fg_key.restype = ctypes.c_uint64
        lib.fg_key.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
        lib.fg_prob_threshold.restype = ctypes.c_uint32
        lib.fg_prob_threshold.argtypes = [ctypes.c_double]
        lib.fg_maf_thresholds.restype = None
        lib.fg_maf_thresholds.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_double, _u32p]
        lib.fg_ref_bytes.restype = None
        lib.fg_ref_bytes.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int32, ctypes.c_int64,
                                     ctypes.c_int64, _u8p]
        lib.fg_ref_rows.restype = None
        lib.fg_ref_rows.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int32, _i64p, ctypes.c_int64, _u8p]
        lib.fg_mixtures.restype = ctypes.c_int
        lib.fg_mixtures.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                    _u8p, _i64p, _i32p, _u8p]
        lib.fg_identity.restype = ctypes.c_int
        lib.fg_identity.argtypes = [ctypes.c_uint64, _u32p, ctypes.c_int32, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_uint32, _u8p, _i64p]
        lib.fg_u64s.restype = None
        lib.fg_u64s.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.c_uint32, ctypes.c_int64, _u64p]
        _cpu = lib
    return _cpu


def gpu_lib():
    global _gpu
    if _gpu is None:
        if not os.path.exists(GPU_LIB):
            raise RuntimeError(f"GPU generator not built: {GPU_LIB} (run __graft_entry__.build())")
        lib = ctypes.CDLL(GPU_LIB)
        lib.fg_gpu_ref_bytes.restype = ctypes.c_int
        lib.fg_gpu_ref_bytes.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p]
        _gpu = lib
    return _gpu


# ----------------------------------------------------------------------------- CPU API

def prob_threshold(p: float) -> int:
    return int(cpu_lib().fg_prob_threshold(float(p)))


def maf_thresholds(seed: int, n_loci: int, lo: float, hi: float = 0.5) -> np.ndarray:
    thr = np.empty(n_loci, dtype=np.uint32)
    cpu_lib().fg_maf_thresholds(seed, n_loci, lo, hi, _ptr(thr, _u32p))
    return thr


def ref_bytes(seed: int, thr: np.ndarray, r0: int, n: int) -> np.ndarray:
    """Reference rows r0 .. r0+n-1 as 0/1 bytes, shape (n, L)."""
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    out = np.empty((n, thr.size), dtype=np.uint8)
    if n:
        cpu_lib().fg_ref_bytes(seed, _ptr(thr, _u32p), thr.size, r0, n, _ptr(out, _u8p))
    return out


def ref_rows(seed: int, thr: np.ndarray, rows) -> np.ndarray:
    """Arbitrary reference rows (any order) as 0/1 bytes, shape (len(rows), L)."""
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).ravel())
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    out = np.empty((rows.size, thr.size), dtype=np.uint8)
    if rows.size:
        if rows.min() < 0:
            raise ValueError("row numbers must be non-negative")
        cpu_lib().fg_ref_rows(seed, _ptr(thr, _u32p), thr.size, _ptr(rows, _i64p), rows.size, _ptr(out, _u8p))
    return out


def mixtures(seed: int, thr: np.ndarray, pool_base: int, pool_size: int, q0: int, nq: int,
             nc_lo: int, nc_hi: int, flip: float):
    """Mixture queries.  Returns (bytes (nq, L), contributors (nq, nc_hi) -1 padded,
    n_contributors (nq,), flip mask (nq, L))."""
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    L = thr.size
    out = np.empty((nq, L), dtype=np.uint8)
    contrib = np.empty((nq, nc_hi), dtype=np.int64)
    ncon = np.empty(nq, dtype=np.int32)
    flips = np.empty((nq, L), dtype=np.uint8)
    rc = cpu_lib().fg_mixtures(seed, _ptr(thr, _u32p), L, pool_base, pool_size, q0, nq,
                               nc_lo, nc_hi, prob_threshold(flip), _ptr(out, _u8p),
                               _ptr(contrib, _i64p), _ptr(ncon, _i32p), _ptr(flips, _u8p))
    if rc != 0:
        raise ValueError("bad mixture parameters")
    return out, contrib, ncon, flips


def identity(seed: int, thr: np.ndarray, pool_base: int, pool_size: int, q0: int, nq: int,
             flip: float):
    """Single-source queries.  Returns (bytes (nq, L), source row (nq,))."""
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    L = thr.size
    out = np.empty((nq, L), dtype=np.uint8)
    src = np.empty(nq, dtype=np.int64)
    rc = cpu_lib().fg_identity(seed, _ptr(thr, _u32p), L, pool_base, pool_size, q0, nq,
                               prob_threshold(flip), _ptr(out, _u8p), _ptr(src, _i64p))
    if rc != 0:
        raise ValueError("bad identity parameters")
    return out, src


def u64s(seed: int, stream: int, row: int, n: int, col0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    if n:
        cpu_lib().fg_u64s(seed, stream, row, col0, n, _ptr(out, _u64p))
    return out


# ----------------------------------------------------------------------------- GPU API

def ref_bytes_gpu(seed: int, thr_dev_ptr: int, n_loci: int, r0: int, n: int,
                  out_dev_ptr: int, ld: int, stream_ptr: int) -> None:
    """Write reference rows r0 .. r0+n-1 as 0/1 bytes into device memory
    (row stride ld bytes) on the given HIP stream."""
    rc = gpu_lib().fg_gpu_ref_bytes(seed, thr_dev_ptr, n_loci, r0, n, out_dev_ptr, ld,
                                    stream_ptr)
    if rc != 0:
        raise RuntimeError(f"fg_gpu_ref_bytes failed ({rc})")


# ----------------------------------------------------------------------------- NumPy twin

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def np_mix(x: np.ndarray) -> np.ndarray:
    """splitmix64 output function in NumPy uint64 arithmetic (wraps mod 2^64)."""
    with np.errstate(over="ignore"):
        z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def np_key(seed: int, stream: int, row, col) -> np.ndarray:
    row = np.asarray(row, dtype=np.uint64)
    col = np.asarray(col, dtype=np.uint64)
    return (np.uint64(seed) ^ (np.uint64(stream) << np.uint64(56)) ^ (row << np.uint64(16)) ^ col)


def maf_thresholds_np(seed: int, n_loci: int, lo: float, hi: float = 0.5) -> np.ndarray:
    u = (np_mix(np_key(seed, 0, 0, np.arange(n_loci))) >> np.uint64(11)).astype(np.float64)
    p = lo + (hi - lo) * (u * (1.0 / 9007199254740992.0))
    return np.floor(p * 4294967296.0).astype(np.uint32)


def ref_bytes_np(seed: int, thr: np.ndarray, r0: int, n: int) -> np.ndarray:
    rows = np.arange(r0, r0 + n, dtype=np.uint64)[:, None]
    cols = np.arange(thr.size, dtype=np.uint64)[None, :]
    u = (np_mix(np_key(seed, 1, rows, cols)) >> np.uint64(32)).astype(np.uint32)
    return (u < thr[None, :]).astype(np.uint8)
