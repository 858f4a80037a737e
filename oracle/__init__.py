"""CPU oracle for the HashGPU hashing path (test infrastructure).

This package is a plain, single-threaded C implementation (``oracle.c``) of
what the GPU library computes, wrapped with ctypes.  It is NOT part of the
product: only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it, and it shares no code with the GPU library.

Every routine follows a passage of "GPUs as Storage System Accelerators":

* ``hash``            MD5 (RFC 1321) / SHA-1 (FIPS 180-4), the sequential
                      building block of Sec. 3.2.2 ("Direct Hashing").
* ``leaves``/``root`` parallel Merkle-Damgard direct hash, Sec. 3.2.2: segment
                      digests in one buffer, then the hash of that buffer.
* ``window_scan``     sliding-window hashing with a boundary predicate,
                      Sec. 2.1 ("Content-based chunking") and Sec. 3.2.2.
* ``chunk_select``    boundary decision with a minimum chunk size (Sec. 3.2.2
                      last stage; min/max chunk sizes of Sec. 4.3).
* ``chunk_digests``   digest of each chunk (Fig. 3 legend, Sec. 3.2.4): the
                      standard digest of its bytes, or its two-level direct
                      hash (Sec. 3.2.2) with a segment size.
* ``similarity``      block-map lookup of Sec. 3.2.1 (similarity % of Sec. 4.3).
* ``BlockMap``        the block-map of a content-addressable store across
                      writes (Sec. 3.2.1): per chunk of a write, whether its
                      digest is already held, and the digests held after it.

``map_ranges`` shards independent units (segments, windows) over threads and
concatenates the per-range results in order; the result is identical to the
single call by construction.  It exists so that full-size checks and the CPU
baseline can use the host's cores.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

MD5 = 0
SHA1 = 1
DIGEST_SIZE = {MD5: 16, SHA1: 20}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_int = ctypes.c_int
_vp = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (plain C11, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _bind(path: str):
    lib = ctypes.CDLL(path)
    lib.oracle_init.argtypes = []
    lib.oracle_init.restype = None
    lib.oracle_digest_size.argtypes = [_int]
    lib.oracle_digest_size.restype = _int
    lib.oracle_hash.argtypes = [_int, _vp, _u64, _vp]
    lib.oracle_hash.restype = _int
    lib.oracle_leaf_count.argtypes = [_u64, _u64]
    lib.oracle_leaf_count.restype = _u64
    lib.oracle_leaves_range.argtypes = [_int, _vp, _u64, _u64, _u64, _u64, _vp]
    lib.oracle_leaves_range.restype = _int
    lib.oracle_root.argtypes = [_int, _vp, _u64, _vp]
    lib.oracle_root.restype = _int
    lib.oracle_window_count.argtypes = [_u64, _u64, _u64]
    lib.oracle_window_count.restype = _u64
    lib.oracle_window_scan_range.argtypes = [_int, _vp, _u64, _u64, _u64, _u32, _u32,
                                             _u64, _u64, _vp, _u64]
    lib.oracle_window_scan_range.restype = _u64
    lib.oracle_chunk_select.argtypes = [_vp, _u64, _u64, _u64, _u64, _vp, _u64]
    lib.oracle_chunk_select.restype = _u64
    lib.oracle_chunk_select_max.argtypes = [_vp, _u64, _u64, _u64, _u64, _u64, _vp, _u64]
    lib.oracle_chunk_select_max.restype = _u64
    lib.oracle_chunk_digests.argtypes = [_int, _vp, _vp, _u64, _vp]
    lib.oracle_chunk_digests.restype = _int
    lib.oracle_similarity.argtypes = [_int, _vp, _u64, _vp, _vp, _u64, _vp]
    lib.oracle_similarity.restype = _u64
    lib.oracle_blockmap_create.argtypes = [_int, _u64]
    lib.oracle_blockmap_create.restype = _vp
    lib.oracle_blockmap_destroy.argtypes = [_vp]
    lib.oracle_blockmap_destroy.restype = None
    lib.oracle_blockmap_size.argtypes = [_vp]
    lib.oracle_blockmap_size.restype = _u64
    lib.oracle_blockmap_write.argtypes = [_vp, _vp, _vp, _u64, _vp, _vp, _vp]
    lib.oracle_blockmap_write.restype = _int
    lib.oracle_init()  # fill the constant tables once, before any threads
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _bind(_LIB)
    return _lib


def _swap_library(path: str | None):
    """Bind the wrappers to another build of the oracle (``None`` restores the
    default).  Used only by the tests that plant a mistake in a copy of
    ``oracle.c`` and check that the pins catch it."""
    global _lib
    _lib = None if path is None else _bind(path)


def _bytes_view(data) -> np.ndarray:
    if isinstance(data, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(data), dtype=np.uint8)
    arr = np.ascontiguousarray(data, dtype=np.uint8).reshape(-1)
    return arr


def _ptr(arr: np.ndarray) -> int:
    return arr.ctypes.data if arr.size else 0


def digest_size(kind: int) -> int:
    return DIGEST_SIZE[kind]


def hash(kind: int, data) -> bytes:  # noqa: A001 - mirrors the paper's "hash"
    """Standard MD5 or SHA-1 digest of ``data``."""
    lib = _load()
    buf = _bytes_view(data)
    out = np.zeros(DIGEST_SIZE[kind], dtype=np.uint8)
    if lib.oracle_hash(kind, _ptr(buf), buf.size, _ptr(out)) != 0:
        raise ValueError("unknown digest kind")
    return out.tobytes()


def leaf_count(length: int, block: int) -> int:
    return int(_load().oracle_leaf_count(length, block))


def leaves(kind: int, data, block: int, k0: int = 0, k1: int | None = None) -> np.ndarray:
    """Segment digests (n x d uint8) of segments [k0, k1) (Sec. 3.2.2)."""
    lib = _load()
    buf = _bytes_view(data)
    n = leaf_count(buf.size, block)
    k1 = n if k1 is None else min(k1, n)
    d = DIGEST_SIZE[kind]
    out = np.zeros((max(k1 - k0, 0), d), dtype=np.uint8)
    if k1 > k0:
        if lib.oracle_leaves_range(kind, _ptr(buf), buf.size, block, k0, k1, _ptr(out)) != 0:
            raise ValueError("bad arguments")
    return out


def root(kind: int, leaf_digests: np.ndarray) -> bytes:
    """Second level of the direct hash: hash of the concatenated digests."""
    lib = _load()
    arr = np.ascontiguousarray(leaf_digests, dtype=np.uint8).reshape(-1)
    d = DIGEST_SIZE[kind]
    out = np.zeros(d, dtype=np.uint8)
    lib.oracle_root(kind, _ptr(arr), arr.size // d, _ptr(out))
    return out.tobytes()


def direct_hash(kind: int, data, block: int):
    lv = leaves(kind, data, block)
    return lv, root(kind, lv)


def window_count(length: int, window: int, stride: int) -> int:
    return int(_load().oracle_window_count(length, window, stride))


def window_scan(kind: int, data, window: int, stride: int, mask: int, target: int,
                k0: int = 0, k1: int | None = None) -> np.ndarray:
    """Ascending uint64 start offsets of candidate windows k in [k0, k1)."""
    lib = _load()
    buf = _bytes_view(data)
    nwin = window_count(buf.size, window, stride)
    k1 = nwin if k1 is None else min(k1, nwin)
    if k1 <= k0:
        return np.zeros(0, dtype=np.uint64)
    cap = min(k1 - k0, 4096 + (k1 - k0) // 256)
    out = np.zeros(cap, dtype=np.uint64)
    total = lib.oracle_window_scan_range(kind, _ptr(buf), buf.size, window, stride, mask,
                                         target, k0, k1, _ptr(out), cap)
    if total > cap:  # denser than expected: scan again with room for all
        out = np.zeros(total, dtype=np.uint64)
        lib.oracle_window_scan_range(kind, _ptr(buf), buf.size, window, stride, mask, target,
                                     k0, k1, _ptr(out), total)
    return out[:total].copy()


def chunk_select(starts: np.ndarray, window: int, length: int, min_chunk: int,
                 max_chunk: int = 0) -> np.ndarray:
    """Chunk end offsets (uint64, last == length) from ascending candidates;
    with max_chunk > 0, forced cuts keep every chunk at most that long."""
    lib = _load()
    st = np.ascontiguousarray(starts, dtype=np.uint64)
    if max_chunk == 0:
        cap = st.size + 1
        out = np.zeros(cap, dtype=np.uint64)
        m = lib.oracle_chunk_select(_ptr(st), st.size, window, length, min_chunk, _ptr(out), cap)
        return out[:m].copy()
    cap = st.size + 2 + length // max_chunk
    out = np.zeros(cap, dtype=np.uint64)
    m = lib.oracle_chunk_select_max(_ptr(st), st.size, window, length, min_chunk, max_chunk, _ptr(out), cap)
    if m == (1 << 64) - 1:
        raise ValueError("max_chunk must be 0 or at least max(min_chunk, 1)")
    assert m <= cap
    return out[:m].copy()


def chunk_digests(kind: int, data, ends: np.ndarray, segment: int = 0) -> np.ndarray:
    """Digest of each chunk [ends[j-1], ends[j]).  segment = 0: the standard
    digest of the chunk's bytes.  segment = S > 0: the chunk direct-hashed by
    the parallel construction of Sec. 3.2.2 (as Sec. 3.2.4 hashes every
    detected chunk): its S-byte segment digests, then the digest of those."""
    lib = _load()
    buf = _bytes_view(data)
    e = np.ascontiguousarray(ends, dtype=np.uint64)
    d = DIGEST_SIZE[kind]
    out = np.zeros((e.size, d), dtype=np.uint8)
    if e.size and segment == 0:
        lib.oracle_chunk_digests(kind, _ptr(buf), _ptr(e), e.size, _ptr(out))
    prev = 0
    for j in range(e.size if segment else 0):
        _, r = direct_hash(kind, buf[prev:int(e[j])], segment)
        out[j] = np.frombuffer(r, dtype=np.uint8)
        prev = int(e[j])
    return out


def similarity(kind: int, dig_a: np.ndarray, dig_b: np.ndarray, len_b=None):
    """(matched, matched_bytes): B chunks, with multiplicity, found in A."""
    lib = _load()
    d = DIGEST_SIZE[kind]
    a = np.ascontiguousarray(dig_a, dtype=np.uint8).reshape(-1, d)
    b = np.ascontiguousarray(dig_b, dtype=np.uint8).reshape(-1, d)
    lb = None if len_b is None else np.ascontiguousarray(len_b, dtype=np.uint64)
    mb = ctypes.c_uint64(0)
    m = lib.oracle_similarity(kind, _ptr(a), a.shape[0], _ptr(b),
                              None if lb is None else _ptr(lb), b.shape[0],
                              ctypes.addressof(mb))
    return int(m), int(mb.value)


def chunk(kind_window: int, kind_chunk: int, data, window: int, stride: int, mask: int,
          target: int, min_chunk: int, threads: int = 1, max_chunk: int = 0, segment: int = 0):
    """Whole content-based chunking path: candidates, ends, chunk digests."""
    buf = _bytes_view(data)
    starts = window_scan_sharded(kind_window, buf, window, stride, mask, target, threads)
    ends = chunk_select(starts, window, buf.size, min_chunk, max_chunk)
    return starts, ends, chunk_digests_sharded(kind_chunk, buf, ends, segment, threads)


def chunk_digests_sharded(kind, data, ends, segment=0, threads=1):
    """chunk_digests over contiguous ranges of chunks on several threads
    (chunks are independent: range [j0, j1) is the same call on the bytes
    from ends[j0-1] with its ends shifted by that offset)."""
    buf = _bytes_view(data)
    e = np.ascontiguousarray(ends, dtype=np.uint64)
    if threads <= 1 or e.size < 64:
        return chunk_digests(kind, buf, e, segment)

    def part(j0, j1):
        s0 = int(e[j0 - 1]) if j0 else 0
        return chunk_digests(kind, buf[s0:int(e[j1 - 1])], e[j0:j1] - np.uint64(s0), segment)
    parts = map_ranges(part, e.size, threads, 16)
    return np.concatenate(parts)


def map_ranges(fn, n: int, threads: int, min_per_range: int = 1):
    """Run ``fn(k0, k1)`` over ``threads`` contiguous ranges of [0, n) and
    return the per-range results in order (independent units only)."""
    threads = max(1, int(threads))
    parts = max(1, min(threads * 4, n // max(min_per_range, 1) or 1))
    bounds = [n * i // parts for i in range(parts + 1)]
    ranges = [(bounds[i], bounds[i + 1]) for i in range(parts) if bounds[i + 1] > bounds[i]]
    if threads == 1 or len(ranges) <= 1:
        return [fn(a, b) for a, b in ranges]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda r: fn(*r), ranges))


def window_scan_sharded(kind, data, window, stride, mask, target, threads=1):
    buf = _bytes_view(data)
    nwin = window_count(buf.size, window, stride)
    parts = map_ranges(lambda a, b: window_scan(kind, buf, window, stride, mask, target, a, b),
                       nwin, threads, 4096)
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)


def leaves_sharded(kind, data, block, threads=1):
    buf = _bytes_view(data)
    n = leaf_count(buf.size, block)
    parts = map_ranges(lambda a, b: leaves(kind, buf, block, a, b), n, threads)
    d = DIGEST_SIZE[kind]
    return np.concatenate(parts) if parts else np.zeros((0, d), dtype=np.uint8)


class BlockMap:
    """The store's block-map across writes (Sec. 3.2.1).  ``write`` takes one
    write's chunk digests in order and returns (is_dup, dup_chunks,
    dup_bytes): a chunk is a duplicate iff its digest is held when its turn
    comes (stored by an earlier write, or equal to an earlier chunk of this
    write); the others are stored.  ``lengths`` (or ``ends``, chunk end
    offsets) give the bytes.  A write that could exceed ``capacity`` raises
    ``OverflowError`` and changes nothing."""

    def __init__(self, kind: int, capacity: int = 1 << 62):
        self._lib = _load()
        self.kind, self.d = kind, DIGEST_SIZE[kind]
        self._h = self._lib.oracle_blockmap_create(kind, capacity)
        if not self._h:
            raise MemoryError("oracle_blockmap_create failed")

    def write(self, digests, lengths=None, ends=None):
        dig = np.ascontiguousarray(digests, dtype=np.uint8).reshape(-1, self.d)
        n = dig.shape[0]
        if ends is not None:
            lengths = np.diff(np.ascontiguousarray(ends, dtype=np.uint64), prepend=np.uint64(0))
        ln = None if lengths is None else np.ascontiguousarray(lengths, dtype=np.uint64)
        if ln is not None and ln.size != n:
            raise ValueError("one length per digest")
        dup = np.zeros(n, dtype=np.uint8)
        c, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
        r = self._lib.oracle_blockmap_write(self._h, _ptr(dig), None if ln is None else _ptr(ln), n,
                                            _ptr(dup), ctypes.addressof(c), ctypes.addressof(b))
        if r == -5:
            raise OverflowError("block-map capacity")
        if r != 0:
            raise ValueError("oracle_blockmap_write failed")
        return dup.astype(bool), int(c.value), int(b.value)

    def size(self) -> int:
        return int(self._lib.oracle_blockmap_size(self._h))

    def close(self):
        if self._h:
            self._lib.oracle_blockmap_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
