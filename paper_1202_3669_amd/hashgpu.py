"""ctypes binding of ``libhashgpu.so``, the C ABI declared in
``include/hashgpu.h``.

The ``hg_*`` functions mirror the C entry points one to one (same names,
same arguments, raw pointers and integers).  ``Context`` adds torch-tensor
marshalling on top: it passes ``tensor.data_ptr()`` and the current torch
stream and allocates result tensors; every hashing step runs in the
library's kernels.  Importing this module raises ImportError when the library
has not been built (``python -m paper_1202_3669_amd.build``); there is no
other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import functools
import inspect
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhashgpu.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_1202_3669_amd.build`")
_lib = ctypes.CDLL(_LIB_PATH)

HG_MD5, HG_SHA1 = 0, 1
HG_OK, HG_EINVAL, HG_ENOMEM, HG_EDEVICE, HG_ETRUNC, HG_EBUSY = 0, -1, -2, -3, -4, -5
HG_IN_DEVICE, HG_OUT_DEVICE, HG_ASYNC, HG_LEN_ENDS, HG_BACKGROUND, HG_COUNT_HOST = 1, 2, 4, 8, 16, 32
HG_HOST_ROOTS = 64
HG_IN_READY = 128
HG_MAX_WINDOW = 4096
DIGEST_SIZE = {HG_MD5: 16, HG_SHA1: 20}

_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_int = ctypes.c_int
_p_u64 = ctypes.POINTER(ctypes.c_uint64)


class hg_chunk_params(ctypes.Structure):
    _fields_ = [("window", _u32), ("stride", _u32), ("mask", _u32), ("target", _u32),
                ("min_chunk", _u64), ("max_chunk", _u64),
                ("window_digest", ctypes.c_int32), ("chunk_digest", ctypes.c_int32),
                ("chunk_segment", _u64)]


class hg_block_job(ctypes.Structure):
    _fields_ = [("in_", _vp), ("len", _u64), ("block_size", _u64), ("leaf_out", _vp),
                ("root_out", _vp), ("digest", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class hg_batch_params(ctypes.Structure):
    _fields_ = [("block_size", _u64), ("block_digest", ctypes.c_int32), ("roots", ctypes.c_int32),
                ("chunk", hg_chunk_params), ("max_candidates", _u64)]


class hg_batch_out(ctypes.Structure):
    _fields_ = [("leaf_digests", _vp), ("roots", _vp), ("chunk_ends", _vp), ("chunk_digests", _vp),
                ("chunk_off", _vp), ("status", _vp)]


HG_REQ_BLOCK, HG_REQ_CHUNK = 0, 1
HG_REQ_FAIL_INJECT = 1 << 8


class hg_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("flags", _u32), ("payload", _vp), ("len", _u64),
                ("block_size", _u64), ("digest", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("leaf_out", _vp), ("root_out", _vp), ("chunk", hg_chunk_params),
                ("chunk_ends", _vp), ("capacity", _u64), ("n_chunks", _vp), ("chunk_digests", _vp)]


class hg_server_cfg(ctypes.Structure):
    _fields_ = [("slots", _u32), ("max_requests", _u32), ("device_budget", _u64),
                ("max_group_bytes", _u64), ("flags", _u32), ("reserved", _u32)]


class hg_server_stats(ctypes.Structure):
    _fields_ = [("submitted", _u64), ("completed", _u64), ("failed", _u64), ("bytes", _u64),
                ("groups", _u64), ("queued", _u64), ("in_flight", _u32), ("max_in_flight", _u32),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double)]


class hg_ctx_stats(ctypes.Structure):
    _fields_ = [("device_pool_bytes", _u64), ("device_pool_used", _u64), ("pinned_pool_bytes", _u64),
                ("pinned_pool_used", _u64), ("device_allocs", _u64), ("pinned_allocs", _u64),
                ("host_blocks", _u64)]


HG_SERVER_CB = ctypes.CFUNCTYPE(None, _u64, ctypes.c_int, _vp)


def _declare(name, restype, argtypes):
    fn = getattr(_lib, name)
    fn.restype = restype
    fn.argtypes = argtypes
    return fn


hg_create = _declare("hg_create", _int, [_int, ctypes.c_size_t, ctypes.c_size_t, ctypes.POINTER(_vp)])
hg_destroy = _declare("hg_destroy", None, [_vp])
hg_strerror = _declare("hg_strerror", ctypes.c_char_p, [_int])
hg_last_error = _declare("hg_last_error", _int, [_vp, ctypes.c_char_p, ctypes.c_size_t])
hg_digest_size = _declare("hg_digest_size", _int, [_int])
hg_host_hash = _declare("hg_host_hash", _int, [_int, _vp, _u64, _vp])
hg_ctx_stats_read = _declare("hg_ctx_stats_read", _int, [_vp, ctypes.POINTER(hg_ctx_stats)])
hg_window_scan_noalloc = _declare("hg_window_scan_noalloc", _int,
                                  [_vp, _vp, _u64, _u32, _u32, _u32, _u32, _int, _vp, _u64, _vp, _vp])
HG_NOALLOC_SCRATCH_BYTES = 32 << 20
hg_host_alloc = _declare("hg_host_alloc", _int, [_vp, ctypes.c_size_t, ctypes.POINTER(_vp)])
hg_host_free = _declare("hg_host_free", _int, [_vp, _vp])
hg_block_hash = _declare("hg_block_hash", _int, [_vp, _vp, _u64, _u64, _int, _vp, _vp, _u32, _vp])
hg_window_scan = _declare("hg_window_scan", _int,
                          [_vp, _vp, _u64, _u32, _u32, _u32, _u32, _int, _vp, _u64, _vp, _u32, _vp])
hg_chunk = _declare("hg_chunk", _int,
                    [_vp, _vp, _u64, ctypes.POINTER(hg_chunk_params), _vp, _u64, _vp, _vp, _u32, _vp])
hg_similarity = _declare("hg_similarity", _int,
                         [_vp, _vp, _u64, _vp, _vp, _u64, _int, _vp, _vp, _u32, _vp])
hg_chunk_select = _declare("hg_chunk_select", _int,
                           [_vp, _vp, _vp, _u64, _u64, _u32, _u64, _u64, _vp, _u64, _vp, _u32, _vp])
hg_chunk_digests = _declare("hg_chunk_digests", _int,
                            [_vp, _vp, _u64, _vp, _vp, _u64, _int, _u64, _vp, _u32, _vp])
hg_similarity_n = _declare("hg_similarity_n", _int,
                           [_vp, _vp, _u64, _vp, _vp, _vp, _u64, _int, _vp, _vp, _u32, _vp])
hg_leaves_batch = _declare("hg_leaves_batch", _int, [_vp, _vp, _u32, _u32, _vp])
hg_roots_batch = _declare("hg_roots_batch", _int, [_vp, _vp, _u32, _u32, _vp])
hg_block_hash_batch = _declare("hg_block_hash_batch", _int, [_vp, _vp, _u32, _u32, _vp])
hg_batch_create = _declare("hg_batch_create", _int,
                           [_vp, _vp, _vp, _u32, ctypes.POINTER(hg_batch_params), ctypes.POINTER(_vp)])
hg_batch_destroy = _declare("hg_batch_destroy", None, [_vp])
hg_batch_layout = _declare("hg_batch_layout", _int, [_vp, _vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64)])
hg_batch_run = _declare("hg_batch_run", _int, [_vp, _vp, ctypes.POINTER(hg_batch_out), _vp])
hg_batch_capture = _declare("hg_batch_capture", _int, [_vp, _vp, ctypes.POINTER(hg_batch_out), _vp])
hg_batch_replay = _declare("hg_batch_replay", _int, [_vp, _vp])
hg_batch_tune = _declare("hg_batch_tune", _int,
                         [_vp, _vp, ctypes.POINTER(hg_batch_out), _vp, ctypes.c_char_p, ctypes.c_size_t])
hg_timing_enable = _declare("hg_timing_enable", _int, [_vp, _int])
hg_timing_read = _declare("hg_timing_read", _int,
                          [_vp, _int, ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_double)])
hg_timing_reset = _declare("hg_timing_reset", _int, [_vp])
hg_timing_origin = _declare("hg_timing_origin", _int, [_vp, _vp])
hg_chunker_create = _declare("hg_chunker_create", _int, [_vp, ctypes.POINTER(hg_chunk_params), ctypes.POINTER(_vp)])
hg_chunker_destroy = _declare("hg_chunker_destroy", None, [_vp])
hg_chunker_bound = _declare("hg_chunker_bound", _int, [_vp, _u64, ctypes.POINTER(_u64)])
hg_chunker_feed = _declare("hg_chunker_feed", _int, [_vp, _vp, _u64, _u32, _vp, _u64, _vp, _vp, _vp])
hg_chunker_finish = _declare("hg_chunker_finish", _int, [_vp, _u32, _vp, _u64, _vp, _vp, _vp])
hg_chunker_reset = _declare("hg_chunker_reset", _int, [_vp])
hg_blockmap_create = _declare("hg_blockmap_create", _int, [_vp, _int, _u64, ctypes.POINTER(_vp)])
hg_blockmap_destroy = _declare("hg_blockmap_destroy", None, [_vp])
hg_blockmap_size = _declare("hg_blockmap_size", _int, [_vp, ctypes.POINTER(_u64)])
hg_blockmap_write = _declare("hg_blockmap_write", _int, [_vp, _vp, _vp, _u64, _u32, _vp, ctypes.POINTER(_u64),
                                                         ctypes.POINTER(_u64), _vp])
hg_probe_alu = _declare("hg_probe_alu", _int, [_vp, ctypes.POINTER(ctypes.c_double), _vp])
hg_probe_read = _declare("hg_probe_read", _int, [_vp, _vp, _u64, ctypes.POINTER(ctypes.c_double), _vp])
hg_block_hash_dual = _declare("hg_block_hash_dual", _int, [_vp, _vp, _u64, _u64, _vp, _vp, _vp, _vp, _u32, _vp])
hg_timing_intervals = _declare("hg_timing_intervals", _int, [_vp, _int, _vp, _vp, _u64, ctypes.POINTER(_u64)])
hg_server_start = _declare("hg_server_start", _int, [_int, ctypes.POINTER(hg_server_cfg), ctypes.POINTER(_vp)])
hg_submit = _declare("hg_submit", _int,
                     [_vp, ctypes.POINTER(hg_request), HG_SERVER_CB, _vp, ctypes.POINTER(_u64)])
hg_wait = _declare("hg_wait", _int, [_vp, _u64, _int, ctypes.POINTER(_int)])
hg_server_play = _declare("hg_server_play", _int, [_vp, _vp, _vp, _u64, _vp, _vp])
hg_server_stats_read = _declare("hg_server_stats_read", _int, [_vp, ctypes.POINTER(hg_server_stats)])
hg_server_stats_reset = _declare("hg_server_stats_reset", _int, [_vp])
hg_server_stop = _declare("hg_server_stop", _int, [_vp])

HG_K = {"leaves": 0, "root": 1, "window_tiles": 2, "window_emit": 3, "chunk_select": 4,
        "chunk_digests": 5, "similarity": 6, "leaves_batch": 7, "roots_batch": 8}

EXPORTED = ["hg_create", "hg_destroy", "hg_strerror", "hg_last_error", "hg_digest_size",
            "hg_host_alloc", "hg_host_free", "hg_block_hash", "hg_window_scan", "hg_chunk",
            "hg_similarity", "hg_leaves_batch", "hg_roots_batch", "hg_block_hash_batch",
            "hg_timing_enable", "hg_timing_read", "hg_timing_reset", "hg_batch_create",
            "hg_batch_destroy", "hg_batch_layout", "hg_batch_run", "hg_batch_capture",
            "hg_batch_replay", "hg_batch_tune", "hg_server_start", "hg_submit", "hg_wait",
            "hg_server_play", "hg_server_stats_read", "hg_server_stats_reset", "hg_server_stop",
            "hg_timing_origin", "hg_timing_intervals", "hg_probe_alu", "hg_probe_read",
            "hg_block_hash_dual", "hg_chunker_create", "hg_chunker_destroy", "hg_chunker_bound",
            "hg_chunker_feed", "hg_chunker_finish", "hg_chunker_reset", "hg_blockmap_create",
            "hg_blockmap_destroy", "hg_blockmap_size", "hg_blockmap_write", "hg_chunk_select",
            "hg_chunk_digests", "hg_similarity_n", "hg_host_hash", "hg_ctx_stats_read",
            "hg_window_scan_noalloc"]


def host_hash(digest: int, data) -> bytes:
    """The library's host-side standard digest of a bytes-like object or
    uint8 numpy array (hg_host_hash; no context, no GPU)."""
    import numpy as np
    buf = np.frombuffer(bytes(data), dtype=np.uint8) if isinstance(data, (bytes, bytearray, memoryview)) \
        else np.ascontiguousarray(data, dtype=np.uint8).reshape(-1)
    out = (ctypes.c_uint8 * 20)()
    st = hg_host_hash(digest, buf.ctypes.data if buf.size else None, buf.size, ctypes.addressof(out))
    if st != HG_OK:
        raise HashGpuError(st, "hg_host_hash failed")
    return bytes(out)[:hg_digest_size(digest)]


class HashGpuError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{hg_strerror(status).decode()} ({status}): {message}")
        self.status = status


def library_path() -> str:
    return _LIB_PATH


def _torch():
    import torch  # torch provides device memory and streams only
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _on_stream(fn):
    """Runs a method with its `stream` argument (a torch stream, if given)
    as torch's current stream, so that the output tensors it allocates, and
    the fills that zero them, are ordered on the stream the library writes
    them on (and their memory is only reused after that stream's work)."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def run(*args, **kwargs):
        stream = sig.bind_partial(*args, **kwargs).arguments.get("stream")
        if stream is None:
            return fn(*args, **kwargs)
        with _torch().cuda.stream(stream):
            return fn(*args, **kwargs)
    return run


class Context:
    """One hg_ctx on one device, used from one stream at a time."""

    def __init__(self, device: int = 0, device_pool: int = 0, pinned_pool: int = 0):
        """device_pool / pinned_pool: sizes of the pools hg_create allocates
        (0: none; see hg_create)."""
        h = _vp()
        st = hg_create(device, device_pool, pinned_pool, ctypes.byref(h))
        if st != HG_OK:
            raise HashGpuError(st, f"hg_create({device}) failed")
        self.handle = h
        self.device = device

    def stats(self) -> dict:
        """Pool use and allocation counts (hg_ctx_stats_read)."""
        out = hg_ctx_stats()
        self._check(hg_ctx_stats_read(self.handle, ctypes.byref(out)))
        return {f[0]: int(getattr(out, f[0])) for f in hg_ctx_stats._fields_}

    def host_alloc(self, nbytes: int):
        """A pinned host block from the context (hg_host_alloc): (pointer,
        uint8 numpy view of it)."""
        import numpy as np
        p = _vp()
        self._check(hg_host_alloc(self.handle, nbytes, ctypes.byref(p)))
        view = np.ctypeslib.as_array((ctypes.c_uint8 * nbytes).from_address(p.value))
        return p.value, view

    def host_free(self, ptr) -> None:
        self._check(hg_host_free(self.handle, ptr))

    def close(self):
        if self.handle:
            hg_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow_trunc=False):
        if st == HG_OK or (allow_trunc and st == HG_ETRUNC):
            return st
        buf = ctypes.create_string_buffer(512)
        hg_last_error(self.handle, buf, 512)
        raise HashGpuError(st, buf.value.decode(errors="replace"))

    # ------------------------------------------------------------ direct --
    @_on_stream
    def block_hash(self, data, block_size: int, digest: int, leaves: bool = True,
                   root: bool = True, stream=None, flags_extra: int = 0):
        """Segment digests (n, d) uint8 and/or root (d,) uint8 of a uint8
        tensor.  A CUDA tensor is hashed in place; a CPU tensor is streamed
        through the context's pinned staging (host-to-device included)."""
        torch = _torch()
        d = DIGEST_SIZE[digest]
        n = (data.numel() + block_size - 1) // block_size if data.numel() else 0
        dev = torch.device("cuda", self.device)
        lv = torch.empty((n, d), dtype=torch.uint8, device=dev) if leaves else None
        rt = torch.empty((d,), dtype=torch.uint8, device=dev) if root else None
        flags = HG_OUT_DEVICE | (HG_IN_DEVICE if data.is_cuda else 0) | flags_extra
        st = hg_block_hash(self.handle, data.data_ptr() if data.numel() else None, data.numel(),
                           block_size, digest, lv.data_ptr() if lv is not None and n else None,
                           rt.data_ptr() if rt is not None else None, flags,
                           _stream_handle(stream))
        self._check(st)
        return lv, rt

    @_on_stream
    def block_hash_dual(self, data, block_size: int, leaves: bool = True, root: bool = True, stream=None,
                        flags_extra: int = 0):
        """(md5 leaves, md5 root, sha1 leaves, sha1 root) of a uint8 tensor in
        one pass (CUDA tensors; None where not asked for)."""
        torch = _torch()
        n = (data.numel() + block_size - 1) // block_size if data.numel() else 0
        dev = torch.device("cuda", self.device)
        lm = torch.empty((n, 16), dtype=torch.uint8, device=dev) if leaves else None
        ls = torch.empty((n, 20), dtype=torch.uint8, device=dev) if leaves else None
        rm = torch.empty(16, dtype=torch.uint8, device=dev) if root else None
        rs = torch.empty(20, dtype=torch.uint8, device=dev) if root else None
        flags = HG_OUT_DEVICE | (HG_IN_DEVICE if data.is_cuda else 0) | flags_extra
        ptr = lambda t: t.data_ptr() if t is not None and t.numel() else None
        self._check(hg_block_hash_dual(self.handle, data.data_ptr() if data.numel() else None, data.numel(),
                                       block_size, ptr(lm), ptr(rm), ptr(ls), ptr(rs), flags,
                                       _stream_handle(stream)))
        return lm, rm, ls, rs

    def probe_alu(self, stream=None) -> float:
        """Measured int32 VALU rate (Tops/s)."""
        v = ctypes.c_double(0.0)
        self._check(hg_probe_alu(self.handle, ctypes.byref(v), _stream_handle(stream)))
        return v.value

    @_on_stream
    def probe_read(self, data, stream=None) -> float:
        """Measured HBM read rate (GB/s) over a CUDA tensor."""
        v = ctypes.c_double(0.0)
        self._check(hg_probe_read(self.handle, data.data_ptr(), data.numel() * data.element_size(),
                                  ctypes.byref(v), _stream_handle(stream)))
        return v.value

    # ----------------------------------------------------- sliding window --
    @_on_stream
    def window_scan(self, data, window: int, stride: int, mask: int, target: int,
                    digest: int = HG_MD5, capacity: int | None = None, stream=None, out=None):
        """Ascending candidate start offsets (int64 CUDA tensor).  With
        out = (starts, count) preallocated CUDA int64 tensors the scan is
        only enqueued (HG_ASYNC): count[0] gets the total found, starts the
        first len(starts) of them; returns out."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        n = data.numel()
        if out is not None:
            starts, cnt = out
            st = hg_window_scan(self.handle, data.data_ptr() if n else None, n, window, stride, mask, target,
                                digest, starts.data_ptr(), starts.numel(), cnt.data_ptr(),
                                HG_IN_DEVICE | HG_OUT_DEVICE | HG_ASYNC, _stream_handle(stream))
            self._check(st)
            return out
        nwin = (n - window) // stride + 1 if n >= window else 0
        if capacity is None:
            capacity = min(nwin, 4096 + nwin // 1024)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        for _ in range(2):
            out = torch.empty(max(capacity, 1), dtype=torch.int64, device=dev)
            flags = HG_OUT_DEVICE | (HG_IN_DEVICE if data.is_cuda else 0)
            st = hg_window_scan(self.handle, data.data_ptr() if n else None, n, window, stride,
                                mask, target, digest, out.data_ptr(), capacity, cnt.data_ptr(),
                                flags, _stream_handle(stream))
            self._check(st, allow_trunc=True)
            total = int(cnt.item())
            if total <= capacity:
                return out[:total]
            capacity = total
        raise HashGpuError(HG_ETRUNC, "candidate count changed between calls")

    @_on_stream
    def chunk(self, data, window: int, stride: int, mask: int, target: int, min_chunk: int,
              window_digest: int = HG_MD5, chunk_digest: int = HG_SHA1, digests: bool = True,
              capacity: int | None = None, stream=None, out=None, asynchronous: bool = False,
              max_chunk: int = 0, chunk_segment: int = 0):
        """(ends int64, digests (n, d) uint8) CUDA tensors of the chunks.
        With out = (ends, digests) preallocated CUDA tensors (capacity =
        len(ends)) the results are written there and views returned; with
        asynchronous=True as well, the call returns once the chunk digests
        are enqueued (the views are valid when `stream` has completed).
        chunk_segment > 0 selects two-level chunk digests (segments of that
        many bytes)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        n = data.numel()
        p = hg_chunk_params(window, stride, mask, target, min_chunk, max_chunk, window_digest, chunk_digest,
                            chunk_segment)
        d = DIGEST_SIZE[chunk_digest]
        total = _u64(0)
        if out is not None:
            ends, dig = out
            flags = HG_OUT_DEVICE | HG_COUNT_HOST | (HG_IN_DEVICE if data.is_cuda else 0)
            if asynchronous:
                flags |= HG_ASYNC
            st = hg_chunk(self.handle, data.data_ptr() if n else None, n, ctypes.byref(p),
                          ends.data_ptr(), ends.numel(), ctypes.addressof(total),
                          dig.data_ptr() if digests else None, flags, _stream_handle(stream))
            self._check(st)
            k = int(total.value)
            return ends[:k], (dig[:k] if digests else None)
        if capacity is None:
            nwin = (n - window) // stride + 1 if n >= window else 0
            capacity = 1 + min(nwin, 4096 + nwin // 1024)
            if min_chunk:
                capacity = min(capacity, n // min_chunk + 1)
            if max_chunk:
                capacity += n // max_chunk + 1
        for _ in range(2):
            ends = torch.empty(max(capacity, 1), dtype=torch.int64, device=dev)
            dig = torch.empty((max(capacity, 1), d), dtype=torch.uint8, device=dev) if digests else None
            flags = HG_OUT_DEVICE | HG_COUNT_HOST | (HG_IN_DEVICE if data.is_cuda else 0)
            st = hg_chunk(self.handle, data.data_ptr() if n else None, n, ctypes.byref(p),
                          ends.data_ptr(), capacity, ctypes.addressof(total),
                          dig.data_ptr() if dig is not None else None, flags,
                          _stream_handle(stream))
            self._check(st, allow_trunc=True)
            k = int(total.value)
            if k <= capacity:
                return ends[:k], (dig[:k] if dig is not None else None)
            capacity = k
        raise HashGpuError(HG_ETRUNC, "chunk count changed between calls")

    # ------------------------------------------------- chunking stages --
    @_on_stream
    def chunk_select(self, starts, n_starts, length: int, window: int, min_chunk: int, max_chunk: int = 0,
                     out=None, asynchronous: bool = False, stream=None):
        """hg_chunk_select on CUDA tensors: starts (int64, room for
        len(starts) candidates) and n_starts (int64, one count).  Returns
        (ends, n) CUDA tensors; without asynchronous, ends[:n]."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        m = starts.numel()
        bound = m + 1 + (length // max_chunk + 1 if max_chunk else 0)
        if out is None:
            out = (torch.empty(bound, dtype=torch.int64, device=dev), torch.zeros(1, dtype=torch.int64, device=dev))
        ends, n = out
        flags = HG_IN_DEVICE | HG_OUT_DEVICE | (HG_ASYNC if asynchronous else 0)
        self._check(hg_chunk_select(self.handle, starts.data_ptr() if m else None, n_starts.data_ptr(), m, length,
                                    window, min_chunk, max_chunk, ends.data_ptr(), ends.numel(), n.data_ptr(),
                                    flags, _stream_handle(stream)))
        if asynchronous:
            return ends, n
        return ends[:int(n.item())], n

    @_on_stream
    def chunk_digests(self, data, ends, n_chunks, digest: int = HG_SHA1, chunk_segment: int = 0, out=None,
                      asynchronous: bool = False, stream=None):
        """hg_chunk_digests on CUDA tensors: ends (int64, room for len(ends)
        chunks), n_chunks (int64, one count).  Returns the (len(ends), d)
        digest tensor (the first n_chunks rows are the digests)."""
        torch = _torch()
        m = ends.numel()
        d = DIGEST_SIZE[digest]
        if out is None:
            out = torch.empty((max(m, 1), d), dtype=torch.uint8, device=torch.device("cuda", self.device))
        flags = HG_IN_DEVICE | HG_OUT_DEVICE | (HG_ASYNC if asynchronous else 0)
        n = data.numel()
        self._check(hg_chunk_digests(self.handle, data.data_ptr() if n else None, n, ends.data_ptr() if m else None,
                                     n_chunks.data_ptr(), m, digest, chunk_segment, out.data_ptr(), flags,
                                     _stream_handle(stream)))
        return out

    @_on_stream
    def similarity_n(self, dig_a, dig_b, n_b, ends_b=None, len_b=None, digest: int = HG_SHA1, out=None,
                     asynchronous: bool = False, stream=None):
        """hg_similarity_n: B's count n_b is a CUDA int64 tensor read when
        the work runs.  Returns (matched, matched_bytes), or with
        asynchronous=True leaves them in `out` (int64 CUDA tensor of 2)."""
        torch = _torch()
        d = DIGEST_SIZE[digest]
        a = dig_a.reshape(-1, d)
        b = dig_b.reshape(-1, d)
        res = torch.zeros(2, dtype=torch.int64, device=torch.device("cuda", self.device)) if out is None else out
        lens = ends_b if ends_b is not None else len_b
        flags = HG_IN_DEVICE | HG_OUT_DEVICE | (HG_LEN_ENDS if ends_b is not None else 0)
        if asynchronous:
            flags |= HG_ASYNC
        self._check(hg_similarity_n(self.handle, a.data_ptr() if a.numel() else None, a.shape[0],
                                    b.data_ptr() if b.numel() else None,
                                    lens.data_ptr() if lens is not None and lens.numel() else None,
                                    n_b.data_ptr(), b.shape[0], digest, res.data_ptr(), res[1:].data_ptr(), flags,
                                    _stream_handle(stream)))
        if asynchronous:
            return None
        r = res.cpu()
        return int(r[0]), int(r[1])

    # ------------------------------------------------------------- timing --
    def timing(self, enable: bool = True):
        self._check(hg_timing_enable(self.handle, 1 if enable else 0))

    def timing_reset(self):
        self._check(hg_timing_reset(self.handle))

    def timing_origin(self, event):
        """Time axis for timing_intervals: a recorded torch.cuda.Event with
        timing (kept alive by the caller), or None."""
        self._check(hg_timing_origin(self.handle, event.cuda_event if event is not None else None))

    def timing_intervals(self, name: str):
        """(start_ms, end_ms) numpy arrays of the class's launches after the
        origin event."""
        import numpy as np
        k = HG_K[name]
        n = _u64(0)
        self._check(hg_timing_intervals(self.handle, k, None, None, 0, ctypes.byref(n)), allow_trunc=True)
        a = np.zeros(max(int(n.value), 1))
        b = np.zeros_like(a)
        self._check(hg_timing_intervals(self.handle, k, a.ctypes.data, b.ctypes.data, a.size, ctypes.byref(n)))
        return a[:int(n.value)], b[:int(n.value)]

    def timing_read(self, name: str):
        """(launches, total_ms) of a kernel class since the last reset."""
        n = _u64(0)
        ms = ctypes.c_double(0.0)
        self._check(hg_timing_read(self.handle, HG_K[name], ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    # ------------------------------------------------------------ batches --
    def batch_outputs(self, specs, roots: bool = True):
        """Allocate outputs for [(data_tensor, block_size, digest), ...] and
        return (records, leaf tensors, root tensors)."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        recs = (hg_block_job * len(specs))()
        leaves, rts = [], []
        for i, (data, block, digest) in enumerate(specs):
            d = DIGEST_SIZE[digest]
            n = (data.numel() + block - 1) // block if data.numel() else 0
            lv = torch.empty((n, d), dtype=torch.uint8, device=dev)
            rt = torch.empty((d,), dtype=torch.uint8, device=dev) if roots else None
            recs[i] = hg_block_job(data.data_ptr() if data.numel() else None, data.numel(), block,
                                   lv.data_ptr() if n else None,
                                   rt.data_ptr() if rt is not None else None, digest, 0)
            leaves.append(lv)
            rts.append(rt)
        # The records hold raw pointers: they keep the tensors they point at
        # (inputs and outputs) alive for as long as they exist.
        recs._hg_keep = (leaves, rts, [s[0] for s in specs])
        return recs, leaves, rts

    @staticmethod
    def device_job_table(recs):
        """Copy hg_block_job records into a CUDA byte tensor (for
        HG_IN_DEVICE / HG_ASYNC use)."""
        torch = _torch()
        raw = bytes(memoryview(recs).cast("B"))
        table = torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()
        table._hg_keep = recs  # and through them the tensors they point at
        return table

    @_on_stream
    def block_hash_batch(self, specs, roots: bool = True, stream=None):
        """Direct hash of many jobs: specs = [(data, block_size, digest)].
        Returns (leaf tensors, root tensors) in spec order."""
        recs, leaves, rts = self.batch_outputs(specs, roots)
        fn = hg_block_hash_batch if roots else hg_leaves_batch
        st = fn(self.handle, ctypes.addressof(recs), len(specs), HG_OUT_DEVICE,
                _stream_handle(stream))
        self._check(st)
        return leaves, rts

    @_on_stream
    def run_batch(self, table, n_jobs: int, which: str = "both", asynchronous: bool = True,
                  stream=None, background: bool = False, host_roots: bool = False):
        """Run a job table: a device table (from device_job_table) or the
        host records themselves (from batch_outputs); which in {"leaves",
        "roots", "both"}.  host_roots (host table only): the second levels
        on the host's cores (HG_HOST_ROOTS)."""
        fn = {"leaves": hg_leaves_batch, "roots": hg_roots_batch,
              "both": hg_block_hash_batch}[which]
        on_dev = hasattr(table, "data_ptr")
        flags = (HG_IN_DEVICE if on_dev else 0) | HG_OUT_DEVICE | (HG_ASYNC if asynchronous else 0)
        if background:
            flags |= HG_BACKGROUND
        if host_roots:
            flags |= HG_HOST_ROOTS
        ptr = table.data_ptr() if on_dev else ctypes.addressof(table)
        self._check(fn(self.handle, ptr, n_jobs, flags, _stream_handle(stream)))

    @_on_stream
    def similarity(self, dig_a, dig_b, len_b=None, digest: int = HG_SHA1, stream=None,
                   ends_b=None, out=None, asynchronous: bool = False):
        """(matched, matched_bytes) of B's chunk digests against A's.  Chunk
        sizes come from len_b (lengths) or ends_b (hg_chunk end offsets).
        With `out` (int64 CUDA tensor of 2) and asynchronous=True the counts
        are left in `out` and nothing is returned."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        d = DIGEST_SIZE[digest]
        a = dig_a.reshape(-1, d)
        b = dig_b.reshape(-1, d)
        res = torch.zeros(2, dtype=torch.int64, device=dev) if out is None else out
        lens = ends_b if ends_b is not None else len_b
        flags = HG_IN_DEVICE | HG_OUT_DEVICE | (HG_LEN_ENDS if ends_b is not None else 0)
        if asynchronous:
            flags |= HG_ASYNC
        st = hg_similarity(self.handle, a.data_ptr() if a.numel() else None, a.shape[0],
                           b.data_ptr() if b.numel() else None,
                           lens.data_ptr() if lens is not None and lens.numel() else None,
                           b.shape[0], digest, res.data_ptr(), res[1:].data_ptr(), flags,
                           _stream_handle(stream))
        self._check(st)
        if asynchronous:
            return None
        r = res.cpu()
        return int(r[0]), int(r[1])


class Batch:
    """A planned hg_batch over files of one arena, with its output tensors.

    offsets/lengths: host integer sequences (bytes within the arena).  The
    outputs live in CUDA tensors: ``leaves`` (n_leaves, d), ``roots`` (n, d),
    ``chunk_ends`` (max_chunks,) int64, ``chunk_digests`` (max_chunks, d2),
    ``chunk_off`` (n + 1,) int64, ``status`` (4,) int64.
    """

    def __init__(self, ctx: Context, offsets, lengths, block_size: int = 64 * 1024,
                 block_digest: int = HG_SHA1, roots: bool = True, window: int = 20, stride: int = 1,
                 mask: int = 0xFFF, target: int = 0, min_chunk: int = 2048,
                 window_digest: int = HG_MD5, chunk_digest: int = HG_SHA1,
                 max_candidates: int = 0, max_chunk: int = 0, chunk_segment: int = 0):
        torch = _torch()
        import numpy as np
        self.ctx = ctx
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        ln = np.ascontiguousarray(lengths, dtype=np.uint64)
        self.n = int(off.size)
        p = hg_batch_params(block_size, block_digest, 1 if roots else 0,
                            hg_chunk_params(window, stride, mask, target, min_chunk, max_chunk, window_digest,
                                            chunk_digest, chunk_segment), max_candidates)
        h = _vp()
        ctx._check(hg_batch_create(ctx.handle, off.ctypes.data if self.n else None,
                                   ln.ctypes.data if self.n else None, self.n, ctypes.byref(p),
                                   ctypes.byref(h)))
        self.handle = h
        lf = np.zeros(self.n + 1, dtype=np.uint64)
        nl, mc = _u64(0), _u64(0)
        hg_batch_layout(h, lf.ctypes.data, ctypes.byref(nl), ctypes.byref(mc))
        self.leaf_first = lf
        self.n_leaves, self.max_chunks = int(nl.value), int(mc.value)
        dev = torch.device("cuda", ctx.device)
        d1, d2 = DIGEST_SIZE[block_digest], DIGEST_SIZE[chunk_digest]
        self.leaves = torch.zeros((max(self.n_leaves, 1), d1), dtype=torch.uint8, device=dev)
        self.roots = torch.zeros((max(self.n, 1), d1), dtype=torch.uint8, device=dev)
        self.chunk_ends = torch.zeros(max(self.max_chunks, 1), dtype=torch.int64, device=dev)
        self.chunk_digests = torch.zeros((max(self.max_chunks, 1), d2), dtype=torch.uint8, device=dev)
        self.chunk_off = torch.zeros(self.n + 1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(4, dtype=torch.int64, device=dev)
        # the batch may run on another stream: the zero fills end first
        torch.cuda.current_stream(dev).synchronize()
        self._out = hg_batch_out(self.leaves.data_ptr(), self.roots.data_ptr() if roots else None,
                                 self.chunk_ends.data_ptr(), self.chunk_digests.data_ptr(),
                                 self.chunk_off.data_ptr(), self.status.data_ptr())

    def close(self):
        if self.handle:
            hg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, arena, stream=None):
        self.ctx._check(hg_batch_run(self.handle, arena.data_ptr(), ctypes.byref(self._out),
                                     _stream_handle(stream)))

    def capture(self, arena, stream):
        self.ctx._check(hg_batch_capture(self.handle, arena.data_ptr(), ctypes.byref(self._out),
                                         _stream_handle(stream)))

    def replay(self, stream=None):
        self.ctx._check(hg_batch_replay(self.handle, _stream_handle(stream)))

    def tune(self, arena, stream=None) -> str:
        buf = ctypes.create_string_buffer(2048)
        self.ctx._check(hg_batch_tune(self.handle, arena.data_ptr(), ctypes.byref(self._out),
                                      _stream_handle(stream), buf, 2048))
        return buf.value.decode()


class Server:
    """An hg_server (continuous-batching serving loop) on one device."""

    def __init__(self, device: int = 0, slots: int = 3, max_requests: int = 1024,
                 device_budget: int = 1 << 30, max_group_bytes: int = 512 << 20,
                 background: bool = False):
        cfg = hg_server_cfg(slots, max_requests, device_budget, max_group_bytes,
                            HG_BACKGROUND if background else 0, 0)
        h = _vp()
        st = hg_server_start(device, ctypes.byref(cfg), ctypes.byref(h))
        if st != HG_OK:
            raise HashGpuError(st, "hg_server_start failed")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            hg_server_stop(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, req: "hg_request") -> int:
        rid = _u64(0)
        st = hg_submit(self.handle, ctypes.byref(req), HG_SERVER_CB(), None, ctypes.byref(rid))
        if st != HG_OK:
            raise HashGpuError(st, "hg_submit failed")
        return int(rid.value)

    def wait(self, rid: int, timeout_ms: int = -1) -> int:
        out = _int(0)
        st = hg_wait(self.handle, rid, timeout_ms, ctypes.byref(out))
        if st != HG_OK:
            raise HashGpuError(st, "hg_wait failed")
        return int(out.value)

    def play(self, requests: "RequestSet", arrival_s):
        """Replays requests.reqs at the given arrival times; returns
        (latency_ms, status) arrays."""
        import numpy as np
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        n = len(requests)
        assert arr.size == n
        lat = np.zeros(n, dtype=np.float64)
        sts = np.zeros(n, dtype=np.int32)
        st = hg_server_play(self.handle, ctypes.addressof(requests.reqs) if n else None,
                            arr.ctypes.data if n else None, n, lat.ctypes.data if n else None,
                            sts.ctypes.data if n else None)
        if st != HG_OK:
            raise HashGpuError(st, "hg_server_play failed")
        return lat, sts

    def stats(self) -> dict:
        s = hg_server_stats()
        hg_server_stats_read(self.handle, ctypes.byref(s))
        return {k: getattr(s, k) for k, _ in hg_server_stats._fields_}

    def reset_stats(self):
        hg_server_stats_reset(self.handle)


class RequestSet:
    """Serving requests over slices of one payload pool, with host outputs.

    pool_ptr: address of the pool (device memory when in_device, else host
    memory, preferably pinned).  specs: sequence of (kind, offset, length),
    kind 0 = block SHA-1, 1 = block MD5, 2 = chunking (the mix labels of the
    serving workload).  Block requests use `block_size` and ask for segment
    digests and the second level; chunk requests use the chunk parameters
    and a capacity of len // max(min_chunk, 1) + 1 chunks (an upper bound).
    Outputs: ``leaves[i]``, ``root[i]``, ``ends[i]``/``digests[i]`` (first
    ``n_chunks[i]`` entries) as numpy views.
    """

    def __init__(self, pool_ptr: int, in_device: bool, specs, block_size: int = 64 * 1024,
                 window: int = 20, stride: int = 1, mask: int = 0xFFF, target: int = 0,
                 min_chunk: int = 2048, window_digest: int = HG_MD5, chunk_digest: int = HG_SHA1,
                 fail=(), max_chunk: int = 0, chunk_segment: int = 0):
        import numpy as np
        specs = [(int(k), int(o), int(n)) for k, o, n in specs]
        self.specs = specs
        n = len(specs)
        self.reqs = (hg_request * max(n, 1))()
        cp = hg_chunk_params(window, stride, mask, target, min_chunk, max_chunk, window_digest, chunk_digest,
                             chunk_segment)
        self.chunk_params = cp
        dc = DIGEST_SIZE[chunk_digest]
        leaf_n, cap = [], []
        for k, o, ln in specs:
            leaf_n.append((ln + block_size - 1) // block_size if k != 2 else 0)
            cap.append(ln // max(min_chunk, 1) + 1 + (ln // max_chunk if max_chunk else 0) if k == 2 else 0)
        self._leaf_buf = np.zeros(max(sum(leaf_n) * 20, 1), dtype=np.uint8)
        self._root_buf = np.zeros((max(n, 1), 20), dtype=np.uint8)
        self._end_buf = np.zeros(max(sum(cap), 1), dtype=np.uint64)
        self._dig_buf = np.zeros((max(sum(cap), 1), dc), dtype=np.uint8)
        self.n_chunks = np.zeros(max(n, 1), dtype=np.uint64)
        self.leaves, self.root, self.ends, self.digests = [], [], [], []
        lo = eo = 0
        fail = set(fail)
        for i, (k, o, ln) in enumerate(specs):
            r = self.reqs[i]
            r.flags = (HG_IN_DEVICE if in_device else 0) | (HG_REQ_FAIL_INJECT if i in fail else 0)
            r.payload = pool_ptr + o
            r.len = ln
            if k in (0, 1):
                d = 20 if k == 0 else 16
                r.kind = HG_REQ_BLOCK
                r.block_size = block_size
                r.digest = HG_SHA1 if k == 0 else HG_MD5
                lv = self._leaf_buf[lo:lo + leaf_n[i] * d].reshape(leaf_n[i], d)
                lo += leaf_n[i] * 20
                r.leaf_out = lv.ctypes.data if leaf_n[i] else self._leaf_buf.ctypes.data
                r.root_out = self._root_buf[i].ctypes.data
                self.leaves.append(lv)
                self.root.append(self._root_buf[i, :d])
                self.ends.append(None)
                self.digests.append(None)
            else:
                r.kind = HG_REQ_CHUNK
                r.chunk = cp
                c = cap[i]
                r.chunk_ends = self._end_buf[eo:eo + c].ctypes.data
                r.capacity = c
                r.n_chunks = self.n_chunks[i:i + 1].ctypes.data
                r.chunk_digests = self._dig_buf[eo:eo + c].ctypes.data
                self.ends.append(self._end_buf[eo:eo + c])
                self.digests.append(self._dig_buf[eo:eo + c])
                eo += c
                self.leaves.append(None)
                self.root.append(None)

    def __len__(self):
        return len(self.specs)

    def result(self, i: int):
        """('block', leaves, root) or ('chunk', ends, digests), copies."""
        k = self.specs[i][0]
        if k in (0, 1):
            return ("block", self.leaves[i].copy(), bytes(self.root[i]))
        m = int(self.n_chunks[i])
        return ("chunk", self.ends[i][:m].copy(), self.digests[i][:m].copy())


class Chunker:
    """A streaming content-based chunker (hg_chunker) on a Context.

    feed(piece) takes a uint8 CUDA or CPU tensor or numpy array and returns
    (ends, digests) numpy arrays of the chunks decided so far (absolute
    stream offsets); finish() returns the rest.  With asynchronous=True
    both return (ends, digests, count) CUDA tensors instead, written in
    stream order (valid after the stream synchronizes; the first count[0]
    rows hold the chunks), and the call returns once the cuts are decided.
    """

    def __init__(self, ctx: Context, window: int = 20, stride: int = 1, mask: int = 0xFFF, target: int = 0,
                 min_chunk: int = 2048, max_chunk: int = 0, window_digest: int = HG_MD5,
                 chunk_digest: int = HG_SHA1, chunk_segment: int = 0):
        self.ctx = ctx
        self.d = DIGEST_SIZE[chunk_digest]
        p = hg_chunk_params(window, stride, mask, target, min_chunk, max_chunk, window_digest, chunk_digest,
                            chunk_segment)
        h = _vp()
        ctx._check(hg_chunker_create(ctx.handle, ctypes.byref(p), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            hg_chunker_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _host_view(data):
        # a CPU torch tensor is passed as the numpy array over its memory
        if data is not None and hasattr(data, "is_cuda") and not data.is_cuda:
            return data.contiguous().numpy()
        return data

    def _call(self, fn, data, stream, ready=False):
        import numpy as np
        data = self._host_view(data)
        n = 0 if data is None else (data.numel() if hasattr(data, "numel") else data.size)
        b = _u64(0)
        self.ctx._check(hg_chunker_bound(self.handle, n, ctypes.byref(b)))
        cap = int(b.value)
        is_dev = hasattr(data, "is_cuda") and data.is_cuda
        if fn == "feed" and n and not is_dev and not (data.flags["C_CONTIGUOUS"] and data.dtype == np.uint8):
            raise ValueError("host input must be a contiguous uint8 array")
        ends = np.zeros(cap, dtype=np.uint64)
        dig = np.zeros((cap, self.d), dtype=np.uint8)
        cnt = _u64(0)
        if fn == "feed":
            ptr = (data.data_ptr() if is_dev else data.ctypes.data) if n else None
            fl = (HG_IN_DEVICE | (HG_IN_READY if ready else 0)) if is_dev else 0
            st = hg_chunker_feed(self.handle, ptr, n, fl, ends.ctypes.data, cap,
                                 ctypes.byref(cnt), dig.ctypes.data, _stream_handle(stream))
        else:
            st = hg_chunker_finish(self.handle, 0, ends.ctypes.data, cap, ctypes.byref(cnt), dig.ctypes.data,
                                   _stream_handle(stream))
        self.ctx._check(st)
        k = int(cnt.value)
        return ends[:k].copy(), dig[:k].copy()

    def _call_async(self, fn, data, stream, ready=False):
        import torch
        data = self._host_view(data)
        n = 0 if data is None else (data.numel() if hasattr(data, "numel") else data.size)
        b = _u64(0)
        self.ctx._check(hg_chunker_bound(self.handle, n, ctypes.byref(b)))
        cap = int(b.value)
        dev = torch.device("cuda", self.ctx.device)
        ends = torch.empty(cap, dtype=torch.int64, device=dev)
        dig = torch.empty((cap, self.d), dtype=torch.uint8, device=dev)
        cnt = torch.empty(1, dtype=torch.int64, device=dev)
        flags = HG_OUT_DEVICE | HG_ASYNC
        if fn == "feed":
            is_dev = hasattr(data, "is_cuda") and data.is_cuda
            if n and not is_dev and not (data.flags["C_CONTIGUOUS"] and data.dtype.itemsize == 1):
                raise ValueError("host input must be a contiguous uint8 array")
            ptr = (data.data_ptr() if is_dev else data.ctypes.data) if n else None
            fl = flags | ((HG_IN_DEVICE | (HG_IN_READY if ready else 0)) if is_dev else 0)
            st = hg_chunker_feed(self.handle, ptr, n, fl, ends.data_ptr(), cap,
                                 cnt.data_ptr(), dig.data_ptr(), _stream_handle(stream))
        else:
            st = hg_chunker_finish(self.handle, flags, ends.data_ptr(), cap, cnt.data_ptr(), dig.data_ptr(),
                                   _stream_handle(stream))
        self.ctx._check(st)
        return ends, dig, cnt

    @_on_stream
    def feed(self, data, stream=None, asynchronous=False, ready=False):
        """ready: a CUDA tensor whose bytes are complete now (HG_IN_READY: the
        feed need not wait for work pending on the stream before reading it)."""
        if asynchronous:
            return self._call_async("feed", data, stream, ready)
        return self._call("feed", data, stream, ready)

    @_on_stream
    def finish(self, stream=None, asynchronous=False):
        return self._call_async("finish", None, stream) if asynchronous else self._call("finish", None, stream)

    def reset(self):
        self.ctx._check(hg_chunker_reset(self.handle))


class BlockMap:
    """A persistent block-map (hg_blockmap) on a Context."""

    def __init__(self, ctx: Context, digest: int = HG_SHA1, capacity: int = 1 << 22):
        self.ctx = ctx
        h = _vp()
        ctx._check(hg_blockmap_create(ctx.handle, digest, capacity, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            hg_blockmap_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def size(self) -> int:
        n = _u64(0)
        self.ctx._check(hg_blockmap_size(self.handle, ctypes.byref(n)))
        return int(n.value)

    @_on_stream
    def write(self, digests, ends=None, lengths=None, stream=None):
        """Writes a version's chunk digests ((n, d) uint8 CUDA tensor or
        numpy array); ends (chunk end offsets) or lengths, same placement.
        Returns (is_dup numpy bool array, duplicate chunks, duplicate bytes)."""
        import numpy as np
        is_dev = hasattr(digests, "is_cuda") and digests.is_cuda
        n = int(digests.shape[0])
        lens = ends if ends is not None else lengths
        flags = (HG_IN_DEVICE if is_dev else 0) | (HG_LEN_ENDS if ends is not None else 0)
        ptr = (lambda a: (a.data_ptr() if is_dev else a.ctypes.data) if a is not None and n else None)
        if lens is not None and not is_dev:
            lens = np.ascontiguousarray(lens, dtype=np.uint64)
        if not is_dev:
            digests = np.ascontiguousarray(digests)
        dup = np.zeros(max(n, 1), dtype=np.uint8)
        c, b = _u64(0), _u64(0)
        self.ctx._check(hg_blockmap_write(self.handle, ptr(digests), ptr(lens), n, flags, dup.ctypes.data,
                                          ctypes.byref(c), ctypes.byref(b), _stream_handle(stream)))
        return dup[:n].astype(bool), int(c.value), int(b.value)
