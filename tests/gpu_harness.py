"""Helpers for the GPU tests: move generated profiles onto the device and into
libfastid databases.  Inputs come only from the shared generator (gen/);
expected values come only from the oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import gen
from gen.workloads import Workload


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pack_rows(ctx, bytes_u8: np.ndarray) -> torch.Tensor:
    return ctx.pack(to_dev(bytes_u8))


def db_from_bytes(ctx, refs_u8: np.ndarray):
    rows = pack_rows(ctx, refs_u8)
    db = ctx.build_db(rows, refs_u8.shape[1])
    ctx.sync()
    return db


def gpu_generated_db(ctx, seed: int, thr: np.ndarray, n_refs: int, chunk: int = 1 << 20):
    """Reference rows 0..n_refs-1 generated on the device in chunks, packed by
    libfastid (fid_pack) and built into a database."""
    L = thr.size
    thr_dev = to_dev(thr.astype(np.uint32))
    rows = torch.empty((n_refs, gen_row_words(L)), dtype=torch.int64, device="cuda")
    buf = torch.empty((min(chunk, n_refs), L), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for r0 in range(0, n_refs, chunk):
        n = min(chunk, n_refs - r0)
        gen.ref_bytes_gpu(seed, thr_dev.data_ptr(), L, r0, n, buf.data_ptr(), L, stream)
        ctx.pack(buf[:n], L, out=rows[r0:r0 + n])
    db = ctx.build_db(rows, L)
    ctx.sync()
    del rows, buf
    return db


def gen_row_words(L: int) -> int:
    from paper_1707_00516_amd import fid_row_words
    return fid_row_words(L)


def workload_inputs(w: Workload, n_refs: int | None = None, n_q: int | None = None):
    """CPU-side inputs of a workload: MAF thresholds, mixture queries and bookkeeping."""
    n_refs = n_refs or w.n_refs
    n_q = n_q or w.n_q
    thr = gen.maf_thresholds(w.seed, w.n_loci, w.maf_lo)
    M, contrib, ncon, F = gen.mixtures(w.seed, thr, 0, n_refs, 0, n_q, w.nc_lo, w.nc_hi, w.flip)
    return thr, M, contrib, ncon, F
