"""Python binding of libfastid (include/fastid.h), argument marshalling only.

Every function has the name of the C entry point it wraps and takes device
pointers as integers (e.g. ``tensor.data_ptr()``) and HIP streams as integers
(``torch.cuda.current_stream().cuda_stream``).  A non-zero status raises
:class:`FidError` carrying the library's message.  All comparison work runs
in the HIP kernels of libfastid.so; there is no CPU fallback -- importing this
module without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# FASTID_LIBRARY selects another build of the same ABI (e.g. a tuning variant).
LIB_PATH = os.environ.get("FASTID_LIBRARY") or os.path.join(_HERE, "libfastid.so")

FID_MODE_MIXTURE = 0
FID_MODE_IDENTITY = 1

FID_BACKEND_AUTO = 0
FID_BACKEND_POPCOUNT = 1
FID_BACKEND_MFMA = 2
FID_BACKEND_MFMA_FP4 = 3

FID_PROBE_MFMA_FP4 = 0
FID_PROBE_MFMA_I8 = 1
FID_PROBE_VALU = 2
FID_PROBE_HBM_COPY = 3

FID_SERVE_CONTINUOUS = 0
FID_SERVE_FIFO = 1
FID_OK = 0
FID_EINVAL = -1
FID_ENOMEM = -2
FID_EHIP = -3
FID_EOVERFLOW = -4
FID_EBUDGET = -5
FID_ETIMEOUT = -6
FID_ENOTREADY = -7
FID_ENODEV = -8

# Every symbol include/fastid.h declares.
EXPORTS = (
    "fid_status_str", "fid_last_error", "fid_version", "fid_ctx_create", "fid_ctx_destroy",
    "fid_ctx_set_backend", "fid_backend_for", "fid_ctx_set_stream", "fid_sync", "fid_ctx_enable_timing", "fid_ctx_scan_time",
    "fid_peak_probe", "fid_stream_workspace_bytes", "fid_compare_topk_streamed",
    "fid_pack_genotypes", "fid_full_stream_workspace_bytes", "fid_compare_full_streamed",
    "fid_threshold_stream_workspace_bytes", "fid_compare_threshold_streamed",
    "fid_row_words", "fid_pack", "fid_pack_host", "fid_db_bytes",
    "fid_db_build", "fid_db_destroy", "fid_db_info", "fid_db_popcounts", "fid_compare_full",
    "fid_compare_tiles", "fid_topk_workspace_bytes", "fid_compare_topk",
    "fid_topk_range_workspace_bytes", "fid_compare_topk_range", "fid_compare_topk_noalloc",
    "fid_topk_mixed_workspace_bytes", "fid_compare_topk_mixed", "fid_compare_topk_bounded",
    "fid_threshold_workspace_bytes", "fid_compare_threshold",
    "fid_threshold_topk_workspace_bytes", "fid_compare_threshold_topk",
    "fid_batch_workspace_bytes", "fid_batch_create", "fid_batch_run", "fid_batch_info", "fid_batch_job_routed",
    "fid_batch_destroy", "fid_server_create", "fid_server_info", "fid_server_submit",
    "fid_server_poll", "fid_server_wait", "fid_server_stats", "fid_server_destroy",
)


class FidError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} [{status}]")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libfastid.so is not built at {LIB_PATH}; run __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t


def _sig(name, restype, *argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = list(argtypes)
    return f


_sig("fid_status_str", ctypes.c_char_p, ctypes.c_int)
_sig("fid_last_error", ctypes.c_char_p)
_sig("fid_version", ctypes.c_int)
_sig("fid_ctx_create", ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int, _vp)
_sig("fid_ctx_destroy", ctypes.c_int, _vp)
_sig("fid_ctx_set_backend", ctypes.c_int, _vp, ctypes.c_int)
_sig("fid_backend_for", ctypes.c_int, _vp, _vp, _i32, ctypes.POINTER(ctypes.c_int))
_sig("fid_ctx_set_stream", ctypes.c_int, _vp, _vp)
_sig("fid_sync", ctypes.c_int, _vp)
_sig("fid_ctx_enable_timing", ctypes.c_int, _vp, ctypes.c_int)
_sig("fid_ctx_scan_time", ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double),
     ctypes.POINTER(_i64), ctypes.c_int)
_sig("fid_peak_probe", ctypes.c_int, _vp, ctypes.c_int, _vp, _sz, ctypes.POINTER(ctypes.c_double),
     ctypes.POINTER(ctypes.c_double))
_sig("fid_stream_workspace_bytes", ctypes.c_int, _vp, _i64, _i32, _i64, _i32, _i32, ctypes.POINTER(_sz))
_sig("fid_compare_topk_streamed", ctypes.c_int, _vp, _vp, _i64, _i32, _i64, _vp, _i32, ctypes.c_int, _i32, _vp,
     _sz, _vp, _vp)
_sig("fid_pack_genotypes", ctypes.c_int, _vp, _vp, _i64, _i32, _i64, _vp)
_sig("fid_full_stream_workspace_bytes", ctypes.c_int, _vp, _i64, _i32, _i64, _i32, ctypes.POINTER(_sz))
_sig("fid_compare_full_streamed", ctypes.c_int, _vp, _vp, _i64, _i32, _i64, _vp, _i32, ctypes.c_int, _vp, _sz,
     _vp, _i64)
_sig("fid_threshold_stream_workspace_bytes", ctypes.c_int, _vp, _i64, _i32, _i64, _i32, _i64, ctypes.POINTER(_sz))
_sig("fid_compare_threshold_streamed", ctypes.c_int, _vp, _vp, _i64, _i32, _i64, _vp, _i32, ctypes.c_int, _vp, _vp,
     _sz, _i64, _vp, _vp, _vp, ctypes.POINTER(_i64))
_sig("fid_row_words", _i64, _i32)
_sig("fid_pack", ctypes.c_int, _vp, _vp, _i64, _i32, _i64, _vp)
_sig("fid_pack_host", ctypes.c_int, _vp, _i64, _i32, _i64, _vp)
_sig("fid_db_bytes", ctypes.c_int, _i64, _i32, ctypes.POINTER(_sz))
_sig("fid_db_build", ctypes.c_int, _vp, _vp, _i64, _i32, _vp, _sz, ctypes.POINTER(_vp))
_sig("fid_db_destroy", ctypes.c_int, _vp)
_sig("fid_db_info", ctypes.c_int, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32))
_sig("fid_db_popcounts", ctypes.c_int, _vp, ctypes.POINTER(_vp))
_sig("fid_compare_full", ctypes.c_int, _vp, _vp, _vp, _i32, ctypes.c_int, _vp, _i64)
_sig("fid_compare_tiles", ctypes.c_int, _vp, _vp, _vp, _i32, ctypes.c_int,
     ctypes.POINTER(_i64), _i32, _i32, _i32, _vp)
_sig("fid_topk_workspace_bytes", ctypes.c_int, _vp, _vp, _i32, _i32, ctypes.POINTER(_sz))
_sig("fid_compare_topk", ctypes.c_int, _vp, _vp, _vp, _i32, ctypes.c_int, _i32, _vp, _sz, _vp,
     _vp)
_sig("fid_compare_topk_noalloc", ctypes.c_int, _vp, _vp, _vp, _i32, ctypes.c_int, _i32, _vp, _vp)
_sig("fid_topk_range_workspace_bytes", ctypes.c_int, _vp, _vp, _i64, _i64, _i32, _i32,
     ctypes.POINTER(_sz))
_sig("fid_compare_topk_range", ctypes.c_int, _vp, _vp, _i64, _i64, _vp, _i32, ctypes.c_int, _i32,
     _vp, _sz, _vp, _vp)
_sig("fid_topk_mixed_workspace_bytes", ctypes.c_int, _vp, _vp, _i64, _i64, _i32, _i32,
     ctypes.POINTER(_sz))
_sig("fid_compare_topk_mixed", ctypes.c_int, _vp, _vp, _i64, _i64, _vp, _vp, _i32, _i32, _vp, _sz,
     _vp, _vp)
_sig("fid_compare_topk_bounded", ctypes.c_int, _vp, _vp, _i64, _i64, _vp, _vp, _i32, _i32, _vp, ctypes.c_int,
     _vp, _sz, _vp, _vp)
_sig("fid_threshold_workspace_bytes", ctypes.c_int, _vp, _i32, _i64, ctypes.POINTER(_sz))
_sig("fid_threshold_topk_workspace_bytes", ctypes.c_int, _vp, _vp, _i32, _i32, _i64, ctypes.POINTER(_sz))
_sig("fid_compare_threshold_topk", ctypes.c_int, _vp, _vp, _vp, _i32, ctypes.c_int, _vp, _i32, _vp, _sz, _i64,
     _vp, _vp, _vp, ctypes.POINTER(_i64), _vp, _vp)
_sig("fid_compare_threshold", ctypes.c_int, _vp, _vp, _vp, _i32, ctypes.c_int, _vp, _vp, _sz,
     _i64, _vp, _vp, _vp, ctypes.POINTER(_i64))


class FidJob(ctypes.Structure):
    """One job of a ragged batch (mirrors ``fid_job``)."""
    _fields_ = [("db", _vp), ("r_lo", _i64), ("r_hi", _i64), ("q_dev", _vp), ("n_q", _i32),
                ("mode", _i32), ("cnt_dev", _vp), ("idx_dev", _vp)]


class FidTune(ctypes.Structure):
    """One autotuner row (mirrors ``fid_tune``)."""
    _fields_ = [("n_loci", _i32), ("q_per_item", _i32), ("blocks_per_item", _i32), ("fp4_tiles", _i32)]


_sig("fid_batch_workspace_bytes", ctypes.c_int, _vp, ctypes.POINTER(FidJob), _i32, _i32,
     ctypes.POINTER(FidTune), _i32, ctypes.POINTER(_sz))
_sig("fid_batch_create", ctypes.c_int, _vp, ctypes.POINTER(FidJob), _i32, _i32,
     ctypes.POINTER(FidTune), _i32, _vp, _sz, ctypes.POINTER(_vp))
_sig("fid_batch_run", ctypes.c_int, _vp, ctypes.c_int)
_sig("fid_batch_info", ctypes.c_int, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
     ctypes.POINTER(_i32), ctypes.POINTER(_i32))
_sig("fid_batch_job_routed", ctypes.c_int, _vp, _i32, ctypes.POINTER(_i32))
_sig("fid_batch_destroy", ctypes.c_int, _vp)


class FidServerConfig(ctypes.Structure):
    """Mirrors ``fid_server_config``."""
    _fields_ = [("hbm_budget", _sz), ("max_queries", _i32), ("k", _i32), ("n_chunks", _i32),
                ("policy", _i32), ("tick_chunks", _i32), ("hits_per_query", _i32)]


class FidRequest(ctypes.Structure):
    """Mirrors ``fid_request``."""
    _fields_ = [("q_dev", _vp), ("n_q", _i32), ("mode", _i32), ("k", _i32), ("reserved", _i32),
                ("cnt_host", _vp), ("idx_host", _vp), ("thr_host", _vp), ("hit_cap", _i64),
                ("hit_offs_host", _vp), ("hit_idx_host", _vp), ("hit_cnt_host", _vp)]


_sig("fid_server_create", ctypes.c_int, _vp, _vp, ctypes.POINTER(FidServerConfig),
     ctypes.POINTER(_vp))
_sig("fid_server_info", ctypes.c_int, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
     ctypes.POINTER(_sz))
_sig("fid_server_submit", ctypes.c_int, _vp, ctypes.POINTER(FidRequest),
     ctypes.POINTER(ctypes.c_uint64))
_sig("fid_server_poll", ctypes.c_int, _vp, ctypes.c_uint64, ctypes.POINTER(_i64))
_sig("fid_server_wait", ctypes.c_int, _vp, ctypes.c_uint64, _i64, ctypes.POINTER(_i64))
_sig("fid_server_stats", ctypes.c_int, _vp, ctypes.POINTER(_i64))
_sig("fid_server_destroy", ctypes.c_int, _vp)


def _check(st: int) -> None:
    if st != FID_OK:
        raise FidError(st, _lib.fid_last_error().decode() or fid_status_str(st))


def fid_status_str(status: int) -> str:
    return _lib.fid_status_str(status).decode()


def fid_last_error() -> str:
    return _lib.fid_last_error().decode()


def fid_version() -> int:
    return _lib.fid_version()


def fid_ctx_create(device: int = 0, stream: int = 0) -> int:
    out = _vp()
    _check(_lib.fid_ctx_create(ctypes.byref(out), device, stream))
    return out.value


def fid_ctx_destroy(ctx: int) -> None:
    _check(_lib.fid_ctx_destroy(ctx))


def fid_ctx_set_backend(ctx: int, backend: int) -> None:
    _check(_lib.fid_ctx_set_backend(ctx, backend))


def fid_backend_for(ctx: int, db: int, n_q: int) -> int:
    out = ctypes.c_int()
    _check(_lib.fid_backend_for(ctx, db, n_q, ctypes.byref(out)))
    return out.value


def fid_ctx_set_stream(ctx: int, stream: int) -> None:
    _check(_lib.fid_ctx_set_stream(ctx, stream))


def fid_sync(ctx: int) -> None:
    _check(_lib.fid_sync(ctx))


def fid_ctx_enable_timing(ctx: int, enable: bool) -> None:
    _check(_lib.fid_ctx_enable_timing(ctx, 1 if enable else 0))


def fid_ctx_scan_time(ctx: int, reset: bool = True) -> tuple[float, int]:
    """(summed milliseconds, number of timed scan launches) since the last reset."""
    ms = ctypes.c_double()
    n = _i64()
    _check(_lib.fid_ctx_scan_time(ctx, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def fid_peak_probe(ctx: int, probe: int, buf_ptr: int, buf_bytes: int) -> tuple[float, float]:
    """(sustained rate, ms per launch) of one peak probe (FID_PROBE_*)."""
    rate = ctypes.c_double()
    ms = ctypes.c_double()
    _check(_lib.fid_peak_probe(ctx, probe, buf_ptr, buf_bytes, ctypes.byref(rate), ctypes.byref(ms)))
    return rate.value, ms.value


def fid_stream_workspace_bytes(ctx: int, n_refs: int, n_loci: int, block_refs: int, n_q: int, k: int) -> int:
    out = _sz()
    _check(_lib.fid_stream_workspace_bytes(ctx, n_refs, n_loci, block_refs, n_q, k, ctypes.byref(out)))
    return out.value


def fid_compare_topk_streamed(ctx: int, rows_host: int, n_refs: int, n_loci: int, block_refs: int, q: int,
                              n_q: int, mode: int, k: int, ws: int, ws_bytes: int, cnt: int, idx: int) -> None:
    _check(_lib.fid_compare_topk_streamed(ctx, rows_host, n_refs, n_loci, block_refs, q, n_q, mode, k, ws,
                                          ws_bytes, cnt, idx))


def fid_pack_genotypes(ctx: int, geno: int, n_rows: int, n_loci: int, ld_bytes: int, rows: int) -> None:
    _check(_lib.fid_pack_genotypes(ctx, geno, n_rows, n_loci, ld_bytes, rows))


def fid_full_stream_workspace_bytes(ctx: int, n_refs: int, n_loci: int, block_refs: int, n_q: int) -> int:
    out = _sz()
    _check(_lib.fid_full_stream_workspace_bytes(ctx, n_refs, n_loci, block_refs, n_q, ctypes.byref(out)))
    return out.value


def fid_compare_full_streamed(ctx: int, rows_host: int, n_refs: int, n_loci: int, block_refs: int, q: int,
                              n_q: int, mode: int, ws: int, ws_bytes: int, counts_host: int, ld: int) -> None:
    _check(_lib.fid_compare_full_streamed(ctx, rows_host, n_refs, n_loci, block_refs, q, n_q, mode, ws, ws_bytes,
                                          counts_host, ld))


def fid_threshold_stream_workspace_bytes(ctx: int, n_refs: int, n_loci: int, block_refs: int, n_q: int,
                                         cap: int) -> int:
    out = _sz()
    _check(_lib.fid_threshold_stream_workspace_bytes(ctx, n_refs, n_loci, block_refs, n_q, cap, ctypes.byref(out)))
    return out.value


def fid_compare_threshold_streamed(ctx: int, rows_host: int, n_refs: int, n_loci: int, block_refs: int, q: int,
                                   n_q: int, mode: int, thr: int, ws: int, ws_bytes: int, cap: int, offs: int,
                                   idx: int, cnt: int) -> int:
    """Returns the number of hits; raises FidError (FID_EOVERFLOW) when they exceed cap."""
    total = _i64()
    st = _lib.fid_compare_threshold_streamed(ctx, rows_host, n_refs, n_loci, block_refs, q, n_q, mode, thr, ws,
                                             ws_bytes, cap, offs, idx, cnt, ctypes.byref(total))
    if st == FID_EOVERFLOW:
        raise FidError(st, f"{total.value} threshold hits exceed capacity {cap}")
    _check(st)
    return total.value


def fid_row_words(n_loci: int) -> int:
    return int(_lib.fid_row_words(n_loci))


def fid_pack(ctx: int, bytes_dev: int, n_rows: int, n_loci: int, ld_bytes: int,
             rows_dev: int) -> None:
    _check(_lib.fid_pack(ctx, bytes_dev, n_rows, n_loci, ld_bytes, rows_dev))


def fid_pack_host(bytes_host: int, n_rows: int, n_loci: int, ld_bytes: int, rows_host: int) -> None:
    _check(_lib.fid_pack_host(bytes_host, n_rows, n_loci, ld_bytes, rows_host))


def fid_db_bytes(n_refs: int, n_loci: int) -> int:
    out = _sz()
    _check(_lib.fid_db_bytes(n_refs, n_loci, ctypes.byref(out)))
    return out.value


def fid_db_build(ctx: int, rows_dev: int, n_refs: int, n_loci: int, db_mem_dev: int,
                 db_bytes: int) -> int:
    out = _vp()
    _check(_lib.fid_db_build(ctx, rows_dev, n_refs, n_loci, db_mem_dev, db_bytes,
                             ctypes.byref(out)))
    return out.value


def fid_db_destroy(db: int) -> None:
    _check(_lib.fid_db_destroy(db))


def fid_db_info(db: int) -> tuple[int, int]:
    nr = _i64()
    nl = _i32()
    _check(_lib.fid_db_info(db, ctypes.byref(nr), ctypes.byref(nl)))
    return nr.value, nl.value


def fid_db_popcounts(db: int) -> int:
    out = _vp()
    _check(_lib.fid_db_popcounts(db, ctypes.byref(out)))
    return out.value


def fid_compare_full(ctx: int, db: int, q_dev: int, n_q: int, mode: int, counts_dev: int,
                     ld: int) -> None:
    _check(_lib.fid_compare_full(ctx, db, q_dev, n_q, mode, counts_dev, ld))


def fid_compare_tiles(ctx: int, db: int, q_dev: int, n_q: int, mode: int, tiles, th: int,
                      tw: int, out_dev: int) -> None:
    flat = [int(v) for t in tiles for v in t]
    arr = (_i64 * max(len(flat), 1))(*flat)
    _check(_lib.fid_compare_tiles(ctx, db, q_dev, n_q, mode, arr, len(flat) // 2, th, tw,
                                  out_dev))


def fid_topk_workspace_bytes(ctx: int, db: int, n_q: int, k: int) -> int:
    out = _sz()
    _check(_lib.fid_topk_workspace_bytes(ctx, db, n_q, k, ctypes.byref(out)))
    return out.value


def fid_compare_topk(ctx: int, db: int, q_dev: int, n_q: int, mode: int, k: int, ws_dev: int,
                     ws_bytes: int, cnt_dev: int, idx_dev: int) -> None:
    _check(_lib.fid_compare_topk(ctx, db, q_dev, n_q, mode, k, ws_dev, ws_bytes, cnt_dev,
                                 idx_dev))


def fid_compare_topk_noalloc(ctx: int, db: int, q_dev: int, n_q: int, mode: int, k: int, cnt_dev: int,
                             idx_dev: int) -> None:
    _check(_lib.fid_compare_topk_noalloc(ctx, db, q_dev, n_q, mode, k, cnt_dev, idx_dev))


def fid_topk_range_workspace_bytes(ctx: int, db: int, r_lo: int, r_hi: int, n_q: int,
                                   k: int) -> int:
    out = _sz()
    _check(_lib.fid_topk_range_workspace_bytes(ctx, db, r_lo, r_hi, n_q, k, ctypes.byref(out)))
    return out.value


def fid_compare_topk_range(ctx: int, db: int, r_lo: int, r_hi: int, q_dev: int, n_q: int,
                           mode: int, k: int, ws_dev: int, ws_bytes: int, cnt_dev: int,
                           idx_dev: int) -> None:
    _check(_lib.fid_compare_topk_range(ctx, db, r_lo, r_hi, q_dev, n_q, mode, k, ws_dev,
                                       ws_bytes, cnt_dev, idx_dev))


def fid_topk_mixed_workspace_bytes(ctx: int, db: int, r_lo: int, r_hi: int, n_q: int,
                                   k: int) -> int:
    out = _sz()
    _check(_lib.fid_topk_mixed_workspace_bytes(ctx, db, r_lo, r_hi, n_q, k, ctypes.byref(out)))
    return out.value


def fid_compare_topk_mixed(ctx: int, db: int, r_lo: int, r_hi: int, q_dev: int, modes_dev: int,
                           n_q: int, k: int, ws_dev: int, ws_bytes: int, cnt_dev: int,
                           idx_dev: int) -> None:
    _check(_lib.fid_compare_topk_mixed(ctx, db, r_lo, r_hi, q_dev, modes_dev, n_q, k, ws_dev,
                                       ws_bytes, cnt_dev, idx_dev))


def fid_compare_topk_bounded(ctx: int, db: int, r_lo: int, r_hi: int, q_dev: int, modes_dev: int,
                             n_q: int, k: int, bound_dev: int, use_seed: bool, ws_dev: int, ws_bytes: int,
                             cnt_dev: int, idx_dev: int) -> None:
    _check(_lib.fid_compare_topk_bounded(ctx, db, r_lo, r_hi, q_dev, modes_dev, n_q, k, bound_dev,
                                         1 if use_seed else 0, ws_dev, ws_bytes, cnt_dev, idx_dev))


def fid_threshold_workspace_bytes(db: int, n_q: int, cap: int) -> int:
    out = _sz()
    _check(_lib.fid_threshold_workspace_bytes(db, n_q, cap, ctypes.byref(out)))
    return out.value


def fid_compare_threshold(ctx: int, db: int, q_dev: int, n_q: int, mode: int, thr_dev: int,
                          ws_dev: int, ws_bytes: int, cap: int, offs_dev: int, idx_dev: int,
                          cnt_dev: int) -> int:
    """Returns the hit total.  Raises FidError(FID_EOVERFLOW) with ``.needed``
    set when the hits exceed ``cap``."""
    total = _i64()
    st = _lib.fid_compare_threshold(ctx, db, q_dev, n_q, mode, thr_dev, ws_dev, ws_bytes, cap,
                                    offs_dev, idx_dev, cnt_dev, ctypes.byref(total))
    if st == FID_EOVERFLOW:
        err = FidError(st, fid_last_error())
        err.needed = total.value
        raise err
    _check(st)
    return total.value


def fid_threshold_topk_workspace_bytes(ctx: int, db: int, n_q: int, k: int, cap: int) -> int:
    out = _sz()
    _check(_lib.fid_threshold_topk_workspace_bytes(ctx, db, n_q, k, cap, ctypes.byref(out)))
    return out.value


def fid_compare_threshold_topk(ctx: int, db: int, q_dev: int, n_q: int, mode: int, thr_dev: int, k: int,
                               ws_dev: int, ws_bytes: int, cap: int, offs_dev: int, hidx_dev: int,
                               hcnt_dev: int, cnt_dev: int, idx_dev: int) -> int:
    """Returns the hit total.  Raises FidError(FID_EOVERFLOW) with ``.needed``
    set when the hits exceed ``cap`` (the top-k output is complete then)."""
    total = _i64()
    st = _lib.fid_compare_threshold_topk(ctx, db, q_dev, n_q, mode, thr_dev, k, ws_dev, ws_bytes, cap, offs_dev,
                                         hidx_dev, hcnt_dev, ctypes.byref(total), cnt_dev, idx_dev)
    if st == FID_EOVERFLOW:
        err = FidError(st, fid_last_error())
        err.needed = total.value
        raise err
    _check(st)
    return total.value


def _jobs_array(jobs):
    arr = (FidJob * max(len(jobs), 1))()
    for i, j in enumerate(jobs):
        arr[i] = FidJob(*j) if not isinstance(j, FidJob) else j
    return arr


def _tune_array(tune):
    if not tune:
        return None, 0
    arr = (FidTune * len(tune))()
    for i, t in enumerate(tune):
        arr[i] = FidTune(*t) if not isinstance(t, FidTune) else t
    return arr, len(tune)


def fid_batch_workspace_bytes(ctx: int, jobs, k: int, tune=None) -> int:
    """``jobs``: sequence of FidJob or (db, r_lo, r_hi, q_dev, n_q, mode, cnt_dev, idx_dev);
    ``tune``: sequence of FidTune or (n_loci, q_per_item, blocks_per_item)."""
    ja = _jobs_array(jobs)
    ta, nt = _tune_array(tune)
    out = _sz()
    _check(_lib.fid_batch_workspace_bytes(ctx, ja, len(jobs), k, ta, nt, ctypes.byref(out)))
    return out.value


def fid_batch_create(ctx: int, jobs, k: int, tune, ws_dev: int, ws_bytes: int) -> int:
    ja = _jobs_array(jobs)
    ta, nt = _tune_array(tune)
    out = _vp()
    _check(_lib.fid_batch_create(ctx, ja, len(jobs), k, ta, nt, ws_dev, ws_bytes,
                                 ctypes.byref(out)))
    return out.value


def fid_batch_run(batch: int, use_graph: bool = False) -> None:
    _check(_lib.fid_batch_run(batch, 1 if use_graph else 0))


def fid_batch_info(batch: int) -> tuple[int, int, int, int]:
    """(work items, item lists, persistent workgroups, jobs routed to per-call top-k)."""
    a, b, c, d = _i64(), _i64(), _i32(), _i32()
    _check(_lib.fid_batch_info(batch, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                               ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


def fid_batch_job_routed(batch: int, job: int) -> bool:
    """True when the plan runs job `job` as a per-call matrix-core top-k."""
    out = _i32()
    _check(_lib.fid_batch_job_routed(batch, job, ctypes.byref(out)))
    return bool(out.value)


def fid_batch_destroy(batch: int) -> None:
    _check(_lib.fid_batch_destroy(batch))


def fid_server_create(ctx: int, db: int, hbm_budget: int, max_queries: int, k: int,
                      n_chunks: int = 0, policy: int = 0, tick_chunks: int = 0, hits_per_query: int = 0) -> int:
    cfg = FidServerConfig(hbm_budget, max_queries, k, n_chunks, policy, tick_chunks, hits_per_query)
    out = _vp()
    _check(_lib.fid_server_create(ctx, db, ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def fid_server_info(server: int) -> tuple[int, int, int]:
    """(query slots, chunks per pass, device bytes)."""
    a, b, c = _i32(), _i32(), _sz()
    _check(_lib.fid_server_info(server, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def fid_server_submit(server: int, q_dev: int, n_q: int, mode: int, k: int, cnt_host: int,
                      idx_host: int, thr_host: int = 0, hit_cap: int = 0, hit_offs_host: int = 0,
                      hit_idx_host: int = 0, hit_cnt_host: int = 0) -> int:
    req = FidRequest(q_dev, n_q, mode, k, 0, cnt_host, idx_host, thr_host, hit_cap, hit_offs_host,
                     hit_idx_host, hit_cnt_host)
    t = ctypes.c_uint64()
    _check(_lib.fid_server_submit(server, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def _check_request(st: int, times) -> None:
    """A completed request's status; FID_EOVERFLOW (threshold hits past the
    request's capacity) raises with ``.times`` set, as the outputs exist."""
    if st != FID_OK:
        err = FidError(st, _lib.fid_last_error().decode() or fid_status_str(st))
        if st == FID_EOVERFLOW:
            err.times = tuple(times)
        raise err


def fid_server_poll(server: int, ticket: int):
    """None while in flight, else (submit_ns, admit_ns, done_ns)."""
    times = (_i64 * 3)()
    st = _lib.fid_server_poll(server, ticket, times)
    if st == FID_ENOTREADY:
        return None
    _check_request(st, times)
    return tuple(times)


def fid_server_wait(server: int, ticket: int, timeout_us: int = -1):
    times = (_i64 * 3)()
    _check_request(_lib.fid_server_wait(server, ticket, timeout_us, times), times)
    return tuple(times)


def fid_server_stats(server: int) -> dict:
    a = (_i64 * 5)()
    _check(_lib.fid_server_stats(server, a))
    return {"ticks": a[0], "completed": a[1], "peak_queries_in_flight": a[2],
            "tick_ms_total": a[3] / 1e6, "tick_queries_total": a[4]}


def fid_server_destroy(server: int) -> None:
    _check(_lib.fid_server_destroy(server))
