"""PyTorch plumbing over the libfastid binding: torch allocates device memory
and provides the HIP stream; every step of the comparison runs in libfastid's
kernels.  Tensors holding packed 64-bit words use dtype int64 (same bits)."""
from __future__ import annotations

import weakref

import torch

from . import (FID_MODE_IDENTITY, FID_MODE_MIXTURE, FidJob, fid_batch_create, fid_batch_destroy,
               fid_batch_info, fid_batch_job_routed, fid_batch_run, fid_batch_workspace_bytes, fid_compare_full,
               fid_compare_threshold, fid_compare_topk_range, fid_compare_topk_streamed, fid_pack_genotypes,
               fid_compare_full_streamed, fid_full_stream_workspace_bytes,
               fid_compare_threshold_streamed, fid_threshold_stream_workspace_bytes,
               fid_stream_workspace_bytes, fid_topk_range_workspace_bytes,
               fid_compare_topk_mixed, fid_topk_mixed_workspace_bytes, fid_compare_topk_bounded,
               fid_compare_threshold_topk, fid_threshold_topk_workspace_bytes,
               fid_compare_tiles, fid_compare_topk, fid_ctx_create, fid_ctx_destroy,
               fid_db_build, fid_db_bytes, fid_db_destroy, fid_db_popcounts, fid_pack,
               fid_row_words, fid_sync, fid_threshold_workspace_bytes, fid_topk_workspace_bytes,
               FidError)

__all__ = ["Batch", "Server", "Context", "Database", "FID_MODE_MIXTURE", "FID_MODE_IDENTITY", "FidError",
           "row_words"]


def row_words(n_loci: int) -> int:
    return fid_row_words(n_loci)


class Database:
    """A resident reference database: device memory owned by torch, handle by libfastid."""

    def __init__(self, handle: int, mem: torch.Tensor, n_refs: int, n_loci: int):
        self.handle = handle
        self.mem = mem
        self.n_refs = n_refs
        self.n_loci = n_loci

    def popcounts(self) -> torch.Tensor:
        """Per-reference minor-allele totals (a copy)."""
        ptr = fid_db_popcounts(self.handle)
        off = ptr - self.mem.data_ptr()
        return self.mem[off:off + 4 * self.n_refs].view(torch.int32).clone()

    def close(self) -> None:
        if self.handle:
            fid_db_destroy(self.handle)
            self.handle = 0
            self.mem = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = fid_ctx_create(device, self.stream.cuda_stream)
        # batches and servers made on this context: released before it
        self._children = weakref.WeakSet()

    def close(self) -> None:
        if self.handle:
            for child in list(self._children):
                child.close()
            fid_ctx_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self) -> None:
        fid_sync(self.handle)

    # ------------------------------------------------------------ ingest
    def pack(self, bytes_u8: torch.Tensor, n_loci: int | None = None,
             out: torch.Tensor | None = None) -> torch.Tensor:
        """0/1 locus bytes [n, >= L] (device) -> packed rows [n, row_words] int64."""
        assert bytes_u8.is_cuda and bytes_u8.dtype == torch.uint8 and bytes_u8.dim() == 2
        assert bytes_u8.stride(1) == 1
        n, ld = bytes_u8.shape[0], bytes_u8.stride(0)
        L = bytes_u8.shape[1] if n_loci is None else n_loci
        rw = row_words(L)
        if out is None:
            out = torch.empty((n, rw), dtype=torch.int64, device=bytes_u8.device)
        fid_pack(self.handle, bytes_u8.data_ptr(), n, L, ld, out.data_ptr())
        return out

    def pack_genotypes(self, geno_u8: torch.Tensor) -> torch.Tensor:
        """Genotypes 0/1/2 [n, L] (device) -> packed rows of 2 L loci [n, row_words(2 L)] int64."""
        assert geno_u8.is_cuda and geno_u8.dtype == torch.uint8 and geno_u8.dim() == 2
        assert geno_u8.stride(1) == 1
        n, L = geno_u8.shape
        out = torch.empty((n, row_words(2 * L)), dtype=torch.int64, device=geno_u8.device)
        fid_pack_genotypes(self.handle, geno_u8.data_ptr(), n, L, geno_u8.stride(0), out.data_ptr())
        return out

    def build_db(self, rows: torch.Tensor, n_loci: int) -> Database:
        n = rows.shape[0]
        assert rows.is_cuda and rows.dtype == torch.int64 and rows.is_contiguous()
        assert rows.shape[1] == row_words(n_loci)
        nbytes = fid_db_bytes(n, n_loci)
        mem = torch.empty(nbytes, dtype=torch.uint8, device=rows.device)
        h = fid_db_build(self.handle, rows.data_ptr(), n, n_loci, mem.data_ptr(), nbytes)
        return Database(h, mem, n, n_loci)

    # ------------------------------------------------------------ comparisons
    def compare_full(self, db: Database, q_rows: torch.Tensor, mode: int,
                     out: torch.Tensor | None = None) -> torch.Tensor:
        nq = q_rows.shape[0]
        if out is None:
            out = torch.empty((nq, db.n_refs), dtype=torch.int32, device=q_rows.device)
        fid_compare_full(self.handle, db.handle, q_rows.data_ptr(), nq, mode, out.data_ptr(),
                         out.stride(0))
        return out

    def compare_tiles(self, db: Database, q_rows: torch.Tensor, mode: int, tiles, th: int,
                      tw: int) -> torch.Tensor:
        out = torch.empty((len(tiles), th, tw), dtype=torch.int32, device=q_rows.device)
        fid_compare_tiles(self.handle, db.handle, q_rows.data_ptr(), q_rows.shape[0], mode,
                          tiles, th, tw, out.data_ptr())
        return out

    def topk_workspace(self, db: Database, n_q: int, k: int) -> torch.Tensor:
        nbytes = fid_topk_workspace_bytes(self.handle, db.handle, n_q, k)
        return torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)

    def compare_topk(self, db: Database, q_rows: torch.Tensor, mode: int, k: int,
                     ws: torch.Tensor | None = None):
        nq = q_rows.shape[0]
        if ws is None:
            ws = self.topk_workspace(db, nq, k)
        cnt = torch.empty((nq, k), dtype=torch.int32, device=q_rows.device)
        idx = torch.empty((nq, k), dtype=torch.int64, device=q_rows.device)
        fid_compare_topk(self.handle, db.handle, q_rows.data_ptr(), nq, mode, k, ws.data_ptr(),
                         ws.numel(), cnt.data_ptr(), idx.data_ptr())
        return cnt, idx

    def compare_topk_streamed(self, rows_host: torch.Tensor, n_loci: int, block_refs: int,
                              q_rows: torch.Tensor, mode: int, k: int, ws: torch.Tensor | None = None):
        """Top-k against packed rows held in host memory (pinned for overlap),
        streamed through the device block_refs rows at a time.  Synchronous."""
        assert not rows_host.is_cuda and rows_host.is_contiguous()
        n_refs = rows_host.shape[0]
        nq = q_rows.shape[0]
        if ws is None:
            nbytes = fid_stream_workspace_bytes(self.handle, n_refs, n_loci, block_refs, nq, k)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        cnt = torch.empty((nq, k), dtype=torch.int32, device=q_rows.device)
        idx = torch.empty((nq, k), dtype=torch.int64, device=q_rows.device)
        fid_compare_topk_streamed(self.handle, rows_host.data_ptr(), n_refs, n_loci, block_refs,
                                  q_rows.data_ptr(), nq, mode, k, ws.data_ptr(), ws.numel(), cnt.data_ptr(),
                                  idx.data_ptr())
        return cnt, idx

    def compare_full_streamed(self, rows_host: torch.Tensor, n_loci: int, block_refs: int,
                              q_rows: torch.Tensor, mode: int, out: torch.Tensor | None = None,
                              ws: torch.Tensor | None = None) -> torch.Tensor:
        """Full counts [nq, n_refs] (host, pinned) of packed rows held in host
        memory, streamed through the device block_refs rows at a time."""
        assert not rows_host.is_cuda and rows_host.is_contiguous()
        n_refs = rows_host.shape[0]
        nq = q_rows.shape[0]
        if out is None:
            out = torch.empty((nq, n_refs), dtype=torch.int32, pin_memory=True)
        assert not out.is_cuda and out.stride(1) == 1
        if ws is None:
            nbytes = fid_full_stream_workspace_bytes(self.handle, n_refs, n_loci, block_refs, nq)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        fid_compare_full_streamed(self.handle, rows_host.data_ptr(), n_refs, n_loci, block_refs,
                                  q_rows.data_ptr(), nq, mode, ws.data_ptr(), ws.numel(), out.data_ptr(),
                                  out.stride(0))
        return out

    def compare_threshold_streamed(self, rows_host: torch.Tensor, n_loci: int, block_refs: int,
                                   q_rows: torch.Tensor, mode: int, thr: torch.Tensor, cap: int = 1 << 16):
        """(offs [nq+1], idx [total], cnt [total]) of a streamed database."""
        assert not rows_host.is_cuda and rows_host.is_contiguous()
        n_refs = rows_host.shape[0]
        nq = q_rows.shape[0]
        nbytes = fid_threshold_stream_workspace_bytes(self.handle, n_refs, n_loci, block_refs, nq, cap)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        offs = torch.empty(nq + 1, dtype=torch.int64, device=self.device)
        idx = torch.empty(max(cap, 1), dtype=torch.int64, device=self.device)
        cnt = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        total = fid_compare_threshold_streamed(self.handle, rows_host.data_ptr(), n_refs, n_loci, block_refs,
                                               q_rows.data_ptr(), nq, mode, thr.data_ptr(), ws.data_ptr(),
                                               ws.numel(), cap, offs.data_ptr(), idx.data_ptr(), cnt.data_ptr())
        self.sync()
        return offs, idx[:total], cnt[:total]

    def topk_range_workspace(self, db: Database, r_lo: int, r_hi: int, n_q: int,
                             k: int) -> torch.Tensor:
        nbytes = fid_topk_range_workspace_bytes(self.handle, db.handle, r_lo, r_hi, n_q, k)
        return torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)

    def compare_topk_range(self, db: Database, r_lo: int, r_hi: int, q_rows: torch.Tensor,
                           mode: int, k: int, ws: torch.Tensor | None = None, out=None):
        nq = q_rows.shape[0]
        if ws is None:
            ws = self.topk_range_workspace(db, r_lo, r_hi, nq, k)
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=q_rows.device),
                   torch.empty((nq, k), dtype=torch.int64, device=q_rows.device))
        cnt, idx = out
        fid_compare_topk_range(self.handle, db.handle, r_lo, r_hi, q_rows.data_ptr(), nq, mode, k,
                               ws.data_ptr(), ws.numel(), cnt.data_ptr(), idx.data_ptr())
        return cnt, idx

    def compare_topk_mixed(self, db: Database, r_lo: int, r_hi: int, q_rows: torch.Tensor,
                           modes: torch.Tensor, k: int, ws: torch.Tensor | None = None, out=None):
        """Top-k over [r_lo, r_hi) with a per-query mode (int32 device tensor)."""
        nq = q_rows.shape[0]
        assert modes.is_cuda and modes.dtype == torch.int32 and modes.numel() == nq
        if ws is None:
            nbytes = fid_topk_mixed_workspace_bytes(self.handle, db.handle, r_lo, r_hi, nq, k)
            ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)
        if out is None:
            out = (torch.empty((nq, k), dtype=torch.int32, device=q_rows.device),
                   torch.empty((nq, k), dtype=torch.int64, device=q_rows.device))
        cnt, idx = out
        fid_compare_topk_mixed(self.handle, db.handle, r_lo, r_hi, q_rows.data_ptr(),
                               modes.data_ptr(), nq, k, ws.data_ptr(), ws.numel(), cnt.data_ptr(),
                               idx.data_ptr())
        return cnt, idx

    def compare_topk_bounded(self, db: Database, r_lo: int, r_hi: int, q_rows: torch.Tensor,
                             modes: torch.Tensor, k: int, bound: torch.Tensor, use_seed: bool,
                             ws: torch.Tensor | None = None):
        """Top-k over [r_lo, r_hi) with per-query modes and a caller bound
        (int32 device tensors; bound holds uint32 bit patterns)."""
        nq = q_rows.shape[0]
        assert modes.is_cuda and modes.dtype == torch.int32 and modes.numel() == nq
        assert bound.is_cuda and bound.dtype == torch.int32 and bound.numel() == nq
        if ws is None:
            nbytes = fid_topk_mixed_workspace_bytes(self.handle, db.handle, r_lo, r_hi, nq, k)
            ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=self.device)
        cnt = torch.empty((nq, k), dtype=torch.int32, device=q_rows.device)
        idx = torch.empty((nq, k), dtype=torch.int64, device=q_rows.device)
        fid_compare_topk_bounded(self.handle, db.handle, r_lo, r_hi, q_rows.data_ptr(), modes.data_ptr(), nq, k,
                                 bound.data_ptr(), use_seed, ws.data_ptr(), ws.numel(), cnt.data_ptr(),
                                 idx.data_ptr())
        return cnt, idx

    def compare_threshold(self, db: Database, q_rows: torch.Tensor, mode: int, thr,
                          cap: int = 1 << 16):
        """Returns (offs [nq+1], idx [total], cnt [total]); grows the output once
        if the first capacity overflows."""
        nq = q_rows.shape[0]
        if not torch.is_tensor(thr):
            thr = torch.full((nq,), int(thr), dtype=torch.int32, device=q_rows.device)
        offs = torch.empty(nq + 1, dtype=torch.int64, device=q_rows.device)
        for _ in range(2):
            ws = torch.empty(fid_threshold_workspace_bytes(db.handle, nq, cap), dtype=torch.uint8,
                             device=q_rows.device)
            idx = torch.empty(max(cap, 1), dtype=torch.int64, device=q_rows.device)
            cnt = torch.empty(max(cap, 1), dtype=torch.int32, device=q_rows.device)
            try:
                total = fid_compare_threshold(self.handle, db.handle, q_rows.data_ptr(), nq, mode,
                                              thr.data_ptr(), ws.data_ptr(), ws.numel(), cap,
                                              offs.data_ptr(), idx.data_ptr(), cnt.data_ptr())
                return offs, idx[:total], cnt[:total]
            except FidError as e:
                if getattr(e, "needed", None) is None:
                    raise
                cap = e.needed
        raise RuntimeError("threshold capacity did not converge")


    def compare_threshold_topk(self, db: Database, q_rows: torch.Tensor, mode: int, thr, k: int,
                               cap: int = 1 << 16, ws: torch.Tensor | None = None):
        """One pass: (offs [nq+1], hit idx [total], hit cnt [total], top-k cnt
        [nq, k], top-k idx [nq, k]); grows the hit capacity once if needed."""
        nq = q_rows.shape[0]
        if not torch.is_tensor(thr):
            thr = torch.full((nq,), int(thr), dtype=torch.int32, device=q_rows.device)
        offs = torch.empty(nq + 1, dtype=torch.int64, device=q_rows.device)
        cnt = torch.empty((nq, k), dtype=torch.int32, device=q_rows.device)
        idx = torch.empty((nq, k), dtype=torch.int64, device=q_rows.device)
        for _ in range(2):
            need = fid_threshold_topk_workspace_bytes(self.handle, db.handle, nq, k, cap)
            if ws is None or ws.numel() < need:
                ws = torch.empty(need, dtype=torch.uint8, device=q_rows.device)
            hidx = torch.empty(max(cap, 1), dtype=torch.int64, device=q_rows.device)
            hcnt = torch.empty(max(cap, 1), dtype=torch.int32, device=q_rows.device)
            try:
                total = fid_compare_threshold_topk(self.handle, db.handle, q_rows.data_ptr(), nq, mode,
                                                   thr.data_ptr(), k, ws.data_ptr(), ws.numel(), cap,
                                                   offs.data_ptr(), hidx.data_ptr(), hcnt.data_ptr(),
                                                   cnt.data_ptr(), idx.data_ptr())
                return offs, hidx[:total], hcnt[:total], cnt, idx
            except FidError as e:
                if getattr(e, "needed", None) is None:
                    raise
                cap = e.needed
        raise RuntimeError("threshold capacity did not converge")


class Batch:
    """A planned ragged batch of top-k jobs (fid_batch_*).  ``jobs`` is a list
    of (db, r_lo, r_hi, q_rows, mode); torch owns the outputs and workspace."""

    def __init__(self, ctx: Context, jobs, k: int, tune=None):
        self.ctx = ctx
        self.k = k
        self.q_rows = [j[3] for j in jobs]
        self.cnt = [torch.empty((j[3].shape[0], k), dtype=torch.int32, device=ctx.device)
                    for j in jobs]
        self.idx = [torch.empty((j[3].shape[0], k), dtype=torch.int64, device=ctx.device)
                    for j in jobs]
        self.jobs = [FidJob(j[0].handle, j[1], j[2], j[3].data_ptr(), j[3].shape[0], j[4],
                            c.data_ptr(), i.data_ptr())
                     for j, c, i in zip(jobs, self.cnt, self.idx)]
        nbytes = fid_batch_workspace_bytes(ctx.handle, self.jobs, k, tune)
        self.ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=ctx.device)
        self.handle = fid_batch_create(ctx.handle, self.jobs, k, tune, self.ws.data_ptr(),
                                       self.ws.numel())
        ctx._children.add(self)

    def run(self, use_graph: bool = False) -> None:
        fid_batch_run(self.handle, use_graph)

    def info(self):
        return fid_batch_info(self.handle)

    def routed(self, job: int) -> bool:
        """True when job `job` runs as a per-call matrix-core top-k."""
        return fid_batch_job_routed(self.handle, job)

    def close(self) -> None:
        if self.handle:
            fid_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A serving loop over one resident database (fid_server_*).  Requests
    carry device query rows; results land in host (numpy) arrays."""

    def __init__(self, ctx: Context, db: Database, hbm_budget: int, max_queries: int, k: int,
                 n_chunks: int = 0, policy: int = 0, tick_chunks: int = 0, hits_per_query: int = 0):
        from . import fid_server_create, fid_server_info
        self.ctx = ctx
        self.db = db
        self.k = k
        self.handle = fid_server_create(ctx.handle, db.handle, hbm_budget, max_queries, k,
                                        n_chunks, policy, tick_chunks, hits_per_query)
        ctx._children.add(self)
        self.slots, self.n_chunks, self.device_bytes = fid_server_info(self.handle)
        self._live = {}

    def submit(self, q_rows: torch.Tensor, mode: int, k: int | None = None, thr=None,
               hit_cap: int = 1 << 12) -> int:
        """Queue a request; the query tensor must stay alive until it completes
        (the server keeps a reference).  thr (per-query ints, host) asks for
        threshold hits as well."""
        import numpy as np
        from . import fid_server_submit
        k = k or self.k
        n = q_rows.shape[0]
        cnt = np.empty((n, k), dtype=np.int32)
        idx = np.empty((n, k), dtype=np.int64)
        hits = None
        args = ()
        if thr is not None:
            thr = np.ascontiguousarray(np.broadcast_to(np.asarray(thr, dtype=np.int32), (n,)))
            hits = (thr, np.empty(n + 1, np.int64), np.empty(max(hit_cap, 1), np.int64),
                    np.empty(max(hit_cap, 1), np.int32))
            args = (thr.ctypes.data, hit_cap, hits[1].ctypes.data, hits[2].ctypes.data, hits[3].ctypes.data)
        t = fid_server_submit(self.handle, q_rows.data_ptr(), n, mode, k, cnt.ctypes.data,
                              idx.ctypes.data, *args)
        self._live[t] = (q_rows, cnt, idx, hits)
        return t

    def _result(self, ticket, times, overflow=False):
        q, cnt, idx, hits = self._live.pop(ticket)
        if hits is None:
            return cnt, idx, times
        thr, offs, hidx, hcnt = hits
        if overflow:
            return cnt, idx, times, (offs, None, None)
        total = int(offs[-1])
        return cnt, idx, times, (offs, hidx[:total], hcnt[:total])

    def poll(self, ticket: int):
        """None while in flight, else (cnt, idx, (submit_ns, admit_ns, done_ns)),
        plus (offs, hit idx, hit cnt) for a threshold request (hit arrays None
        when they overflowed its capacity; offs[-1] then holds the hits needed,
        or -1)."""
        from . import FID_EOVERFLOW, fid_server_poll
        try:
            times = fid_server_poll(self.handle, ticket)
        except FidError as e:
            if e.status != FID_EOVERFLOW:
                raise
            return self._result(ticket, e.times, overflow=True)
        if times is None:
            return None
        return self._result(ticket, times)

    def wait(self, ticket: int, timeout_us: int = -1):
        from . import FID_EOVERFLOW, fid_server_wait
        try:
            times = fid_server_wait(self.handle, ticket, timeout_us)
        except FidError as e:
            if e.status != FID_EOVERFLOW:
                raise
            return self._result(ticket, e.times, overflow=True)
        return self._result(ticket, times)

    def stats(self):
        from . import fid_server_stats
        return fid_server_stats(self.handle)

    def close(self) -> None:
        if self.handle:
            from . import fid_server_destroy
            fid_server_destroy(self.handle)
            self.handle = 0
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
