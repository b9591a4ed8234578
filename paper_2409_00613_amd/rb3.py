"""Thin Python binding of librb3.so (the C ABI of include/rb3.h).

Argument marshalling only: every step of the computation runs in the HIP
library. The binding refuses to work without the built library; there is no
CPU fallback. Names follow the C ABI (rb3_build, rb3_merge, rb3_count,
rb3_smem, ...); ``Index`` wraps the opaque handle.

Strings are passed as one concatenated uint8 buffer plus int64 lengths. The
buffer may be a numpy array (host memory) or a torch tensor on the GPU
(device memory, RB3_MEM_DEVICE); lengths are always host arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librb3.so")

RB3_OK, RB3_EINVAL, RB3_ENOMEM, RB3_EDEVICE, RB3_ENOSPC, RB3_ELIMIT, RB3_EAGAIN = 0, -1, -2, -3, -4, -5, -6
RB3_MEM_HOST, RB3_MEM_DEVICE = 0, 1

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Opts(ctypes.Structure):
    _fields_ = [("both_strands", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("dev_alloc", _ALLOC_FN), ("dev_free", _FREE_FN),
                ("alloc_ctx", ctypes.c_void_p), ("chunk_len", ctypes.c_int64),
                ("launch_per_string", ctypes.c_int32), ("ssa_rate", ctypes.c_int32),
                ("occ_interval", ctypes.c_int32), ("smem_segment", ctypes.c_int32)]


class SmemRec(ctypes.Structure):
    _fields_ = [("start", ctypes.c_int64), ("end", ctypes.c_int64), ("occ", ctypes.c_int64),
                ("k", ctypes.c_int64), ("krc", ctypes.c_int64), ("qid", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


SMEM_DTYPE = np.dtype([("start", np.int64), ("end", np.int64), ("occ", np.int64), ("k", np.int64),
                       ("krc", np.int64), ("qid", np.int32), ("pad", np.int32)])
assert SMEM_DTYPE.itemsize == ctypes.sizeof(SmemRec) == 48


class HaplOpts(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32), ("gap_open", ctypes.c_int32),
                ("gap_ext", ctypes.c_int32), ("band", ctypes.c_int32), ("max_cells", ctypes.c_int32),
                ("device_tables", ctypes.c_int32)]


class HaplRec(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("krc", ctypes.c_int64), ("s", ctypes.c_int64),
                ("score", ctypes.c_int32), ("qid", ctypes.c_int32)]


HAPL_DTYPE = np.dtype([("k", np.int64), ("krc", np.int64), ("s", np.int64), ("score", np.int32),
                       ("qid", np.int32)])
assert HAPL_DTYPE.itemsize == ctypes.sizeof(HaplRec) == 32

# Every function declared in include/rb3.h.
EXPORTS = ["rb3_opts_init", "rb3_build", "rb3_merge", "rb3_count", "rb3_count_noalloc", "rb3_smem", "rb3_last_smem_stats",
           "rb3_locate", "rb3_locate1", "rb3_ssa_info", "rb3_last_locate_stats", "rb3_info",
           "rb3_export", "rb3_import", "rb3_clone", "rb3_index_free", "rb3_strerror",
           "rb3_prof_enable", "rb3_prof_reset", "rb3_prof_read", "rb3_merge_stats", "rb3_test_fail_merge_after",
           "rb3_tune_merge", "rb3_tune_smem", "rb3_hapl_opts_init", "rb3_hapl", "rb3_last_hapl_stats",
           "rb3_rle_build", "rb3_rle_load", "rb3_rle_info", "rb3_rle_image", "rb3_rle_export", "rb3_rle_count",
           "rb3_rle_smem", "rb3_rle_hapl", "rb3_rle_free",
           "rb3_server_opts_init", "rb3_server_create", "rb3_server_submit", "rb3_server_poll",
           "rb3_server_stats", "rb3_server_replay", "rb3_server_free"]

RB3_REQ_COUNT, RB3_REQ_SMEM = 0, 1


class ServerOpts(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("pad", ctypes.c_int32), ("max_batch_queries", ctypes.c_int64),
                ("max_batch_bases", ctypes.c_int64), ("mem_budget", ctypes.c_int64), ("max_queued", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("kind", ctypes.c_int32), ("status", ctypes.c_int32),
                ("lo", ctypes.c_int64), ("hi", ctypes.c_int64), ("smem_off", ctypes.c_int64),
                ("n_smem", ctypes.c_int64)]

_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_i64p = ctypes.POINTER(ctypes.c_int64)


class RB3Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rb3 error {code}: {msg}")
        self.code = code


def lib():
    """Load librb3.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2409_00613_amd.build` (hipcc, gfx950)")
    # torch carries its own HIP runtime under the same soname; load it first
    # so that the library binds to that one copy and shares its device
    # memory and streams (two runtimes in one process do not see each other)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    L.rb3_opts_init.argtypes = [ctypes.POINTER(Opts)]
    L.rb3_opts_init.restype = None
    L.rb3_build.argtypes = [ctypes.POINTER(Opts), _vp, _i64p, _i64, _i32, ctypes.POINTER(_vp)]
    L.rb3_merge.argtypes = [_vp, _vp, _i64p, _i64, _i32]
    L.rb3_count.argtypes = [_vp, _vp, _i64p, _i64, _i32, _i64p, _i64p]
    L.rb3_count_noalloc.argtypes = [_vp, _vp, _i64p, _i64, _i32, _i64p, _i64p]
    L.rb3_smem.argtypes = [_vp, _vp, _i64p, _i64, _i32, _i32, _i64, ctypes.POINTER(SmemRec), _i64, _i64p]
    L.rb3_info.argtypes = [_vp, _i64p, _i64p, _i64p]
    L.rb3_hapl_opts_init.argtypes = [ctypes.POINTER(HaplOpts)]
    L.rb3_hapl_opts_init.restype = None
    L.rb3_hapl.argtypes = [_vp, ctypes.POINTER(HaplOpts), _vp, _i64p, _i64, _i32, ctypes.POINTER(HaplRec), _i64,
                           _i64p]
    L.rb3_hapl.restype = ctypes.c_int
    L.rb3_last_hapl_stats.argtypes = [_i64p, _i64p, _i64p, _i64p]
    L.rb3_last_hapl_stats.restype = ctypes.c_int
    L.rb3_last_smem_stats.argtypes = [_i64p, _i64p]
    L.rb3_locate.argtypes = [_vp, _vp, _i64, _i32, _i64p, _i64p]
    L.rb3_locate1.argtypes = [_vp, _vp, _vp, _i64, _i32, _i64p, _i64p]
    L.rb3_ssa_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), _i64p]
    L.rb3_last_locate_stats.argtypes = [_i64p]
    L.rb3_export.argtypes = [_vp, _vp]
    L.rb3_import.argtypes = [ctypes.POINTER(Opts), _vp, _i64, _i64p, _i64, _i32, ctypes.POINTER(_vp)]
    L.rb3_clone.argtypes = [_vp, ctypes.POINTER(_vp)]
    L.rb3_index_free.argtypes = [_vp]
    L.rb3_index_free.restype = None
    L.rb3_strerror.argtypes = [ctypes.c_int]
    L.rb3_strerror.restype = ctypes.c_char_p
    L.rb3_prof_enable.argtypes = [ctypes.c_int]
    L.rb3_prof_reset.argtypes = []
    L.rb3_prof_read.argtypes = [ctypes.c_char_p, _i64p, ctypes.POINTER(ctypes.c_double), _i64, _i64p]
    L.rb3_merge_stats.argtypes = [_vp, ctypes.c_char_p, _i64p, _i64, _i64p]
    L.rb3_test_fail_merge_after.argtypes = [_i32]
    _dp0 = ctypes.POINTER(ctypes.c_double)
    L.rb3_tune_merge.argtypes = [_vp, _vp, _i64p, _i64, _i32, _i64p, _i64p, _dp0, _i64, _i64p]
    L.rb3_tune_smem.argtypes = [_vp, _vp, _i64p, _i64, _i32, _i32, _i64, _i64p, _i64p, _dp0, _i64, _i64p]
    _u64p_ = ctypes.POINTER(ctypes.c_uint64)
    _u16p_ = ctypes.POINTER(ctypes.c_uint16)
    L.rb3_rle_build.argtypes = [_vp, _i32, ctypes.POINTER(_vp)]
    L.rb3_rle_load.argtypes = [ctypes.POINTER(Opts), _u64p_, _i64, _i64p, _u16p_, _i64, _i32, _i32,
                               ctypes.POINTER(_vp)]
    L.rb3_rle_info.argtypes = [_vp, _i64p, _i64p, _i64p, _i64p, ctypes.POINTER(ctypes.c_int32), _i64p]
    L.rb3_rle_image.argtypes = [_vp, _u64p_, _i64p, _u16p_]
    L.rb3_rle_export.argtypes = [_vp, _vp]
    L.rb3_rle_count.argtypes = [_vp, _vp, _i64p, _i64, _i32, _i64p, _i64p]
    L.rb3_rle_smem.argtypes = [_vp, _vp, _i64p, _i64, _i32, _i32, _i64, ctypes.POINTER(SmemRec), _i64, _i64p]
    L.rb3_rle_hapl.argtypes = [_vp, ctypes.POINTER(HaplOpts), _vp, _i64p, _i64, _i32, ctypes.POINTER(HaplRec),
                               _i64, _i64p]
    L.rb3_rle_free.argtypes = [_vp]
    L.rb3_rle_free.restype = None
    for name in ("rb3_rle_build", "rb3_rle_load", "rb3_rle_info", "rb3_rle_image", "rb3_rle_export",
                 "rb3_rle_count", "rb3_rle_smem", "rb3_rle_hapl"):
        getattr(L, name).restype = ctypes.c_int
    L.rb3_server_opts_init.argtypes = [ctypes.POINTER(ServerOpts)]
    L.rb3_server_opts_init.restype = None
    L.rb3_server_create.argtypes = [_vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)]
    L.rb3_server_submit.argtypes = [_vp, _i32, _vp, _i64, _i32, _i64, ctypes.POINTER(ctypes.c_uint64)]
    L.rb3_server_poll.argtypes = [_vp, _i32, ctypes.POINTER(Result), _i64, ctypes.POINTER(SmemRec), _i64,
                                  _i64p, _i64p]
    L.rb3_server_stats.argtypes = [_vp, _i64p, _i64p, _i64p, _i64p, _i64p, _i64p, _i64p]
    _dp = ctypes.POINTER(ctypes.c_double)
    L.rb3_server_replay.argtypes = [_vp, _i32, _vp, _i64p, _i64, _i32, _i64, _dp, _dp, _dp]
    L.rb3_server_free.argtypes = [_vp]
    L.rb3_server_free.restype = None
    for name in ("rb3_server_create", "rb3_server_submit", "rb3_server_poll", "rb3_server_stats",
                 "rb3_server_replay"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("rb3_build", "rb3_merge", "rb3_count", "rb3_count_noalloc", "rb3_smem", "rb3_last_smem_stats", "rb3_locate",
                 "rb3_locate1", "rb3_ssa_info", "rb3_last_locate_stats", "rb3_info", "rb3_export",
                 "rb3_import", "rb3_clone", "rb3_prof_enable", "rb3_prof_reset", "rb3_prof_read",
                 "rb3_merge_stats", "rb3_test_fail_merge_after", "rb3_tune_merge", "rb3_tune_smem"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != RB3_OK:
        raise RB3Error(rc, lib().rb3_strerror(rc).decode())


def _buffer(x):
    """(pointer, nbytes, mem, keepalive) of a uint8 host array or GPU tensor."""
    if hasattr(x, "is_cuda") and hasattr(x, "data_ptr"):
        if x.is_cuda:
            if x.element_size() != 1 or not x.is_contiguous():
                raise ValueError("device buffer must be a contiguous uint8 tensor")
            # the library may run on its own stream: make the producer's
            # writes visible first
            import torch
            torch.cuda.current_stream(x.device).synchronize()
            return x.data_ptr(), x.numel(), RB3_MEM_DEVICE, x
        x = x.numpy()
    if isinstance(x, (bytes, bytearray)):
        x = np.frombuffer(x, dtype=np.uint8)
    a = np.ascontiguousarray(x, dtype=np.uint8)
    return (a.ctypes.data if a.size else None), a.size, RB3_MEM_HOST, a


def _i64buf(x):
    """(pointer, count, mem, keepalive) of an int64 host array or GPU tensor."""
    if hasattr(x, "is_cuda") and hasattr(x, "data_ptr") and x.is_cuda:
        import torch
        if x.dtype != torch.int64 or not x.is_contiguous():
            raise ValueError("device rows must be a contiguous int64 tensor")
        torch.cuda.current_stream(x.device).synchronize()
        return x.data_ptr(), x.numel(), RB3_MEM_DEVICE, x
    if hasattr(x, "numpy"):
        x = x.numpy()
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
    return (a.ctypes.data if a.size else None), a.size, RB3_MEM_HOST, a


def _lens(lens):
    a = np.ascontiguousarray(np.asarray(lens, dtype=np.int64))
    return a, a.ctypes.data_as(_i64p)


class TorchAllocator:
    """Device allocator hooks backed by torch's caching allocator."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:
                return None

        delete = torch.cuda.caching_allocator_delete

        def _free(ptr, ctx):
            # an index freed while the interpreter shuts down may outlive
            # torch's allocator: the memory goes with the process then
            if ptr:
                try:
                    delete(ptr)
                except Exception:
                    pass

        self.alloc_fn = _ALLOC_FN(_alloc)
        self.free_fn = _FREE_FN(_free)


def make_opts(both_strands: bool = True, device: int = 0, stream=None, allocator: TorchAllocator | None = None,
              chunk_len: int = 0, launch_per_string: bool = False, ssa_rate: int = 0, occ_interval: int = 0,
              smem_segment: int = 0) -> Opts:
    o = Opts()
    lib().rb3_opts_init(ctypes.byref(o))
    o.both_strands = 1 if both_strands else 0
    o.device = device
    if stream is not None:
        o.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    elif allocator is not None:
        o.stream = allocator.stream.cuda_stream
    if allocator is not None:
        o.dev_alloc = allocator.alloc_fn
        o.dev_free = allocator.free_fn
    o.chunk_len = int(chunk_len)
    o.launch_per_string = 1 if launch_per_string else 0
    o.ssa_rate = int(ssa_rate)
    o.occ_interval = int(occ_interval)
    o.smem_segment = int(smem_segment)
    return o


class Index:
    """An rb3_index handle (device-resident BWT)."""

    def __init__(self, handle, keep=()):
        self._h = ctypes.c_void_p(handle)
        self._keep = list(keep)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            lib().rb3_index_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # --- calls ---------------------------------------------------------------
    def merge(self, seq, lens):
        return rb3_merge(self, seq, lens)

    def count(self, q, qlens):
        return rb3_count(self, q, qlens)

    def smem(self, q, qlens, min_len: int, min_occ: int = 1, cap: int | None = None):
        return rb3_smem(self, q, qlens, min_len, min_occ, cap)

    def hapl(self, q, qlens, **kw):
        return rb3_hapl(self, q, qlens, **kw)

    def info(self):
        return rb3_info(self)

    def locate(self, rows):
        return rb3_locate(self, rows)

    def locate1(self, lo, hi):
        return rb3_locate1(self, lo, hi)

    def ssa_info(self):
        return rb3_ssa_info(self)

    def export(self) -> np.ndarray:
        return rb3_export(self)

    def clone(self) -> "Index":
        return rb3_clone(self)

    def merge_stats(self) -> dict:
        return rb3_merge_stats(self)


def rb3_build(seq, lens, both_strands: bool = True, device: int = 0, stream=None,
              allocator: TorchAllocator | None = None, chunk_len: int = 0,
              launch_per_string: bool = False, ssa_rate: int = 0, occ_interval: int = 0,
              smem_segment: int = 0) -> Index:
    o = make_opts(both_strands, device, stream, allocator, chunk_len, launch_per_string, ssa_rate, occ_interval,
                  smem_segment)
    ptr, _, mem, keep = _buffer(seq)
    la, lp = _lens(lens)
    h = ctypes.c_void_p()
    _check(lib().rb3_build(ctypes.byref(o), ptr, lp, la.shape[0], mem, ctypes.byref(h)))
    return Index(h.value, keep=[o, allocator])


def rb3_merge(idx: Index, seq, lens) -> None:
    ptr, _, mem, keep = _buffer(seq)
    la, lp = _lens(lens)
    _check(lib().rb3_merge(idx.handle, ptr, lp, la.shape[0], mem))


def rb3_count(idx: Index, q, qlens):
    ptr, _, mem, keep = _buffer(q)
    la, lp = _lens(qlens)
    n = la.shape[0]
    lo = np.zeros(max(n, 1), np.int64)
    hi = np.zeros(max(n, 1), np.int64)
    _check(lib().rb3_count(idx.handle, ptr, lp, n, mem, lo.ctypes.data_as(_i64p), hi.ctypes.data_as(_i64p)))
    return lo[:n], hi[:n]


def rb3_count_noalloc(idx: Index, q, qlens):
    """rb3_count without device allocation: (lo, hi) as numpy arrays for host
    queries, device tensors for device queries."""
    ptr, _, mem, keep = _buffer(q)
    la, lp = _lens(qlens)
    n = la.shape[0]
    lo, hi, plo, phi = _i64out(n, mem, keep)
    _check(lib().rb3_count_noalloc(idx.handle, ptr, lp, n, mem, plo, phi))
    return lo[:n], hi[:n]


def rb3_smem(idx: Index, q, qlens, min_len: int, min_occ: int = 1, cap: int | None = None):
    """Returns (records, offsets): records is a structured array (SMEM_DTYPE);
    query i owns records[offsets[i]:offsets[i+1]]."""
    ptr, _, mem, keep = _buffer(q)
    la, lp = _lens(qlens)
    n = la.shape[0]
    if cap is None:
        # about one SMEM per 100 bases on reads with 1% differences; a call
        # that needs more is repeated with the exact size
        cap = max(1024, int(la.sum()) // 48 + 16 * n)
    while True:
        out = np.zeros(max(cap, 1), dtype=SMEM_DTYPE)
        off = np.zeros(n + 1, np.int64)
        rc = lib().rb3_smem(idx.handle, ptr, lp, n, mem, int(min_len), int(min_occ),
                            out.ctypes.data_as(ctypes.POINTER(SmemRec)), cap, off.ctypes.data_as(_i64p))
        if rc == RB3_ENOSPC:
            cap = int(off[-1])
            continue
        _check(rc)
        return out[:off[-1]], off


def hapl_opts(match: int = 1, mismatch: int = 4, gap_open: int = 6, gap_ext: int = 1, band: int = 25,
              max_cells: int = 0, device_tables: bool = False) -> HaplOpts:
    o = HaplOpts()
    lib().rb3_hapl_opts_init(ctypes.byref(o))
    o.match, o.mismatch, o.gap_open, o.gap_ext = int(match), int(mismatch), int(gap_open), int(gap_ext)
    o.band, o.max_cells, o.device_tables = int(band), int(max_cells), int(bool(device_tables))
    return o


def _hapl_call(fn, handle, q, qlens, cap, kw):
    ptr, _, mem, keep = _buffer(q)
    la, lp = _lens(qlens)
    n = la.shape[0]
    o = hapl_opts(**kw)
    if cap is None:
        # a query keeps at most `band` results; without a band, a guess
        # (a call that needs more is repeated with the exact size)
        per = o.band if 0 < o.band <= 64 else 64
        cap = min(max(1024, per * n), 1 << 24)
    while True:
        out = np.zeros(max(cap, 1), dtype=HAPL_DTYPE)
        off = np.zeros(n + 1, np.int64)
        rc = fn(handle, ctypes.byref(o), ptr, lp, n, mem, out.ctypes.data_as(ctypes.POINTER(HaplRec)), cap,
                off.ctypes.data_as(_i64p))
        if rc == RB3_ENOSPC:
            cap = int(off[-1])
            continue
        _check(rc)
        return out[:off[-1]], off


def rb3_hapl(idx: Index, q, qlens, cap: int | None = None, **kw):
    """Local haplotype enumeration. Keyword options: match, mismatch,
    gap_open, gap_ext, band, max_cells. Returns (records, offsets): records
    is a structured array (HAPL_DTYPE); query i owns
    records[offsets[i]:offsets[i+1]]."""
    return _hapl_call(lib().rb3_hapl, idx.handle, q, qlens, cap, kw)


def rb3_last_hapl_stats() -> dict:
    """Work of this thread's last haplotype-enumeration call: node extensions,
    index blocks they read, cells held summed over query positions, and
    queries moved from LDS to device-memory tables."""
    e, b, c, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().rb3_last_hapl_stats(ctypes.byref(e), ctypes.byref(b), ctypes.byref(c), ctypes.byref(m)))
    return {"extensions": e.value, "blocks": b.value, "cells": c.value, "moved": m.value}


class Rle:
    """An rb3_rle handle: the run-length static index (counts and SMEMs like
    Index, no merges)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h and self._h.value:
            lib().rb3_rle_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self) -> dict:
        n, m, runs, blocks, nbytes = (ctypes.c_int64() for _ in range(5))
        q = ctypes.c_int32()
        _check(lib().rb3_rle_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(runs),
                                  ctypes.byref(blocks), ctypes.byref(q), ctypes.byref(nbytes)))
        return {"n": n.value, "m": m.value, "runs": runs.value, "blocks": blocks.value, "row_shift": q.value,
                "bytes": nbytes.value}

    def image(self):
        """(blocks [nblocks, 16] uint64, segs [nseg + 1, 8] int64, row uint16)."""
        i = self.info()
        n, q = i["n"], i["row_shift"]
        blocks = np.zeros((i["blocks"], 16), np.uint64)
        segs = np.zeros((((n + (1 << 20) - 1) >> 20) + 1, 8), np.int64)
        row = np.zeros(((n - 1) >> q) + 1, np.uint16)
        _check(lib().rb3_rle_image(self._h, blocks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                   segs.ctypes.data_as(_i64p), row.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))))
        return blocks, segs, row

    def export(self) -> np.ndarray:
        n = self.info()["n"]
        out = np.zeros(n, np.uint8)
        _check(lib().rb3_rle_export(self._h, out.ctypes.data))
        return out

    def count(self, q, qlens):
        ptr, _, mem, keep = _buffer(q)
        la, lp = _lens(qlens)
        n = la.shape[0]
        lo = np.zeros(max(n, 1), np.int64)
        hi = np.zeros(max(n, 1), np.int64)
        _check(lib().rb3_rle_count(self._h, ptr, lp, n, mem, lo.ctypes.data_as(_i64p), hi.ctypes.data_as(_i64p)))
        return lo[:n], hi[:n]

    def smem(self, q, qlens, min_len: int, min_occ: int = 1, cap: int | None = None):
        ptr, _, mem, keep = _buffer(q)
        la, lp = _lens(qlens)
        n = la.shape[0]
        if cap is None:
            cap = max(1024, int(la.sum()) // 48 + 16 * n)
        while True:
            out = np.zeros(max(cap, 1), dtype=SMEM_DTYPE)
            off = np.zeros(n + 1, np.int64)
            rc = lib().rb3_rle_smem(self._h, ptr, lp, n, mem, int(min_len), int(min_occ),
                                    out.ctypes.data_as(ctypes.POINTER(SmemRec)), cap, off.ctypes.data_as(_i64p))
            if rc == RB3_ENOSPC:
                cap = int(off[-1])
                continue
            _check(rc)
            return out[:off[-1]], off

    def hapl(self, q, qlens, cap: int | None = None, **kw):
        return _hapl_call(lib().rb3_rle_hapl, self._h, q, qlens, cap, kw)


def rb3_rle_build(idx: Index, row_shift: int = 0) -> Rle:
    h = _vp()
    _check(lib().rb3_rle_build(idx.handle, int(row_shift), ctypes.byref(h)))
    return Rle(h.value)


def rb3_rle_load(blocks, segs, row, n: int, row_shift: int, both_strands: bool = True, device: int = 0) -> Rle:
    blocks = np.ascontiguousarray(blocks, dtype=np.uint64)
    segs = np.ascontiguousarray(segs, dtype=np.int64)
    row = np.ascontiguousarray(row, dtype=np.uint16)
    o = make_opts(both_strands=both_strands, device=device)
    h = _vp()
    _check(lib().rb3_rle_load(ctypes.byref(o), blocks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                              blocks.shape[0], segs.ctypes.data_as(_i64p),
                              row.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)), int(n), int(row_shift),
                              1 if both_strands else 0, ctypes.byref(h)))
    return Rle(h.value)


def _i64out(n, mem, like):
    """Two int64 output arrays of n entries in the inputs' memory: numpy
    arrays for host inputs, tensors on the same device for device inputs."""
    if mem == RB3_MEM_DEVICE:
        import torch
        a = torch.empty(max(n, 1), dtype=torch.int64, device=like.device)
        b = torch.empty(max(n, 1), dtype=torch.int64, device=like.device)
        return a, b, ctypes.cast(a.data_ptr(), _i64p), ctypes.cast(b.data_ptr(), _i64p)
    a = np.zeros(max(n, 1), np.int64)
    b = np.zeros(max(n, 1), np.int64)
    return a, b, a.ctypes.data_as(_i64p), b.ctypes.data_as(_i64p)


def rb3_locate(idx: Index, rows):
    """(strand, offset): the position of the suffix at each row; numpy arrays
    for host rows, device tensors for device rows."""
    ptr, n, mem, keep = _i64buf(rows)
    st, off, pst, poff = _i64out(n, mem, keep)
    _check(lib().rb3_locate(idx.handle, ptr, n, mem, pst, poff))
    return st[:n], off[:n]


def rb3_locate1(idx: Index, lo, hi):
    """(strand, offset): one occurrence in each SA interval [lo, hi); numpy
    arrays for host inputs, device tensors for device inputs."""
    plo, n, mem, k1 = _i64buf(lo)
    phi, n2, mem2, k2 = _i64buf(hi)
    if n != n2 or mem != mem2:
        raise ValueError("lo and hi must have the same length and memory kind")
    st, off, pst, poff = _i64out(n, mem, k1)
    _check(lib().rb3_locate1(idx.handle, plo, phi, n, mem, pst, poff))
    return st[:n], off[:n]


def rb3_ssa_info(idx: Index):
    """(sampling distance, number of samples)."""
    r = ctypes.c_int32()
    k = ctypes.c_int64()
    _check(lib().rb3_ssa_info(idx.handle, ctypes.byref(r), ctypes.byref(k)))
    return r.value, k.value


def rb3_last_locate_stats() -> dict:
    """Work of this thread's last rb3_locate / rb3_locate1 call."""
    e = ctypes.c_int64()
    _check(lib().rb3_last_locate_stats(ctypes.byref(e)))
    return {"lf_steps": e.value}


def rb3_last_smem_stats() -> dict:
    """Work of this thread's last rb3_smem call: bi-interval extensions and
    the distinct index blocks they read."""
    e = ctypes.c_int64()
    b = ctypes.c_int64()
    _check(lib().rb3_last_smem_stats(ctypes.byref(e), ctypes.byref(b)))
    return {"extensions": e.value, "blocks": b.value}


def rb3_info(idx: Index):
    n = ctypes.c_int64()
    m = ctypes.c_int64()
    C = (ctypes.c_int64 * 6)()
    _check(lib().rb3_info(idx.handle, ctypes.byref(n), ctypes.byref(m), C))
    return n.value, m.value, list(C)


def rb3_export(idx: Index) -> np.ndarray:
    n, _, _ = rb3_info(idx)
    out = np.zeros(max(n, 1), np.uint8)
    _check(lib().rb3_export(idx.handle, out.ctypes.data))
    return out[:n]


def rb3_import(codes, lens, both_strands: bool = True, device: int = 0, stream=None,
               allocator: TorchAllocator | None = None, occ_interval: int = 0, smem_segment: int = 0) -> Index:
    """Index from BWT codes of the strands whose lengths are ``lens`` (the
    strand list the BWT was built from, both strands counted)."""
    o = make_opts(both_strands, device, stream, allocator, occ_interval=occ_interval, smem_segment=smem_segment)
    ptr, nbytes, mem, keep = _buffer(codes)
    la, lp = _lens(lens)
    h = ctypes.c_void_p()
    _check(lib().rb3_import(ctypes.byref(o), ptr, nbytes, lp, la.shape[0], mem, ctypes.byref(h)))
    return Index(h.value, keep=[o, allocator])


def rb3_clone(idx: Index) -> Index:
    h = ctypes.c_void_p()
    _check(lib().rb3_clone(idx.handle, ctypes.byref(h)))
    return Index(h.value, keep=list(idx._keep))


def rb3_merge_stats(idx: Index) -> dict:
    cap = 64
    keys = ctypes.create_string_buffer(32 * cap)
    vals = np.zeros(cap, np.int64)
    n = ctypes.c_int64()
    _check(lib().rb3_merge_stats(idx.handle, keys, vals.ctypes.data_as(_i64p), cap, ctypes.byref(n)))
    raw = keys.raw
    return {raw[i * 32:(i + 1) * 32].split(b"\0")[0].decode(): int(vals[i]) for i in range(min(n.value, cap))}


def rb3_tune_merge(idx: Index, seq, lens) -> dict:
    """Autotune the merge chunk length on this batch (idx unchanged)."""
    ptr, _, mem, keep = _buffer(seq)
    la, lp = _lens(lens)
    best = ctypes.c_int64()
    cand = np.zeros(16, np.int64)
    ms = np.zeros(16, np.float64)
    n = ctypes.c_int64()
    _check(lib().rb3_tune_merge(idx.handle, ptr, lp, la.shape[0], mem, ctypes.byref(best),
                                cand.ctypes.data_as(_i64p), ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                16, ctypes.byref(n)))
    return {"chunk_len": best.value, "trials": {int(c): round(float(t), 3) for c, t in zip(cand[:n.value], ms[:n.value])}}


def rb3_tune_smem(idx: Index, q, qlens, min_len: int, min_occ: int = 1) -> dict:
    """Autotune the SMEM segment length on these queries (-1: the automatic rule)."""
    ptr, _, mem, keep = _buffer(q)
    la, lp = _lens(qlens)
    best = ctypes.c_int64()
    cand = np.zeros(16, np.int64)
    ms = np.zeros(16, np.float64)
    n = ctypes.c_int64()
    _check(lib().rb3_tune_smem(idx.handle, ptr, lp, la.shape[0], mem, int(min_len), int(min_occ),
                               ctypes.byref(best), cand.ctypes.data_as(_i64p),
                               ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 16, ctypes.byref(n)))
    return {"segment": best.value, "trials": {int(c): round(float(t), 3) for c, t in zip(cand[:n.value], ms[:n.value])}}


def rb3_test_fail_merge_after(stage: int):
    """Test hook: merges stop with RB3_EDEVICE after this stage (0: off)."""
    _check(lib().rb3_test_fail_merge_after(int(stage)))


class CountingAllocator(TorchAllocator):
    """Torch's caching allocator behind a counter: allocation number
    ``fail_at`` (1-based, counted from the last reset) returns NULL, as a
    device out of memory would. For tests of failure handling."""

    def __init__(self, device: int = 0, stream=None):
        super().__init__(device, stream)
        self.calls = 0
        self.fail_at = 0
        inner = self.alloc_fn

        def _alloc(nbytes, ctx):
            self.calls += 1
            if self.fail_at and self.calls == self.fail_at:
                return None
            return inner(nbytes, ctx)

        self._inner = inner
        self.alloc_fn = _ALLOC_FN(_alloc)

    def reset(self, fail_at: int = 0):
        self.calls = 0
        self.fail_at = fail_at


def rb3_prof_enable(on: bool = True):
    _check(lib().rb3_prof_enable(1 if on else 0))


def rb3_prof_reset():
    _check(lib().rb3_prof_reset())


def rb3_prof_read() -> dict:
    """{kernel name: (launches, total ms)} since the last reset."""
    cap = 256
    names = ctypes.create_string_buffer(32 * cap)
    launches = np.zeros(cap, np.int64)
    ms = np.zeros(cap, np.float64)
    n = ctypes.c_int64()
    _check(lib().rb3_prof_read(names, launches.ctypes.data_as(_i64p),
                               ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap, ctypes.byref(n)))
    raw = names.raw
    return {raw[i * 32:(i + 1) * 32].split(b"\0")[0].decode(): (int(launches[i]), float(ms[i]))
            for i in range(min(n.value, cap))}


class Server:
    """rb3_server: continuous-batching count / SMEM service over an Index."""

    def __init__(self, idx: Index, workers: int = 4, max_batch_queries: int = 4096,
                 max_batch_bases: int = 8 << 20, mem_budget: int = 0, max_queued: int = 1 << 16):
        L = lib()
        so = ServerOpts()
        L.rb3_server_opts_init(ctypes.byref(so))
        so.workers = workers
        so.max_batch_queries = max_batch_queries
        so.max_batch_bases = max_batch_bases
        so.mem_budget = mem_budget
        so.max_queued = max_queued
        h = ctypes.c_void_p()
        _check(L.rb3_server_create(idx.handle, ctypes.byref(so), ctypes.byref(h)))
        self._h = h
        self._idx = idx  # keep the index alive
        self._res = (Result * 4096)()
        self._cap = 1 << 16
        self._recs = np.zeros(self._cap, dtype=SMEM_DTYPE)

    def submit(self, kind: int, q: bytes, min_len: int = 0, min_occ: int = 1) -> int:
        t = ctypes.c_uint64()
        buf = np.frombuffer(q, dtype=np.uint8) if len(q) else np.zeros(1, np.uint8)
        _check(lib().rb3_server_submit(self._h, kind, buf.ctypes.data, len(q), int(min_len), int(min_occ),
                                       ctypes.byref(t)))
        return t.value

    def poll(self, wait_ms: int = 0) -> list:
        """Finished results: dicts with ticket, kind, status, and lo/hi
        (count) or records (SMEM, structured array)."""
        out = []
        while True:
            nr = ctypes.c_int64()
            nk = ctypes.c_int64()
            rc = lib().rb3_server_poll(self._h, int(wait_ms), self._res, len(self._res),
                                       self._recs.ctypes.data_as(ctypes.POINTER(SmemRec)), self._cap,
                                       ctypes.byref(nr), ctypes.byref(nk))
            if rc == RB3_ENOSPC:
                self._cap = max(2 * self._cap, int(nk.value))
                self._recs = np.zeros(self._cap, dtype=SMEM_DTYPE)
                continue
            _check(rc)
            for i in range(nr.value):
                r = self._res[i]
                d = {"ticket": int(r.ticket), "kind": int(r.kind), "status": int(r.status)}
                if r.kind == RB3_REQ_COUNT:
                    d["lo"], d["hi"] = int(r.lo), int(r.hi)
                else:
                    d["records"] = self._recs[r.smem_off:r.smem_off + r.n_smem].copy()
                out.append(d)
            if nr.value < len(self._res):
                return out
            wait_ms = 0

    def replay(self, kind: int, data, lens, arrival_s, min_len: int = 0, min_occ: int = 1):
        """Open-loop run: query i is submitted at arrival_s[i]; returns
        (latencies in seconds, wall time)."""
        d = np.ascontiguousarray(data, dtype=np.uint8)
        la, lp = _lens(lens)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        lat = np.zeros(max(1, la.shape[0]), np.float64)
        wall = ctypes.c_double()
        _dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().rb3_server_replay(self._h, kind, d.ctypes.data if d.size else None, lp, la.shape[0],
                                       int(min_len), int(min_occ), arr.ctypes.data_as(_dp),
                                       lat.ctypes.data_as(_dp), ctypes.byref(wall)))
        return lat[:la.shape[0]], wall.value

    def stats(self) -> dict:
        v = [ctypes.c_int64() for _ in range(7)]
        _check(lib().rb3_server_stats(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(["queued", "inflight", "batches", "served", "max_batch", "busy_us", "mem_budget"],
                        [x.value for x in v]))

    def close(self):
        if self._h and self._h.value:
            lib().rb3_server_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
