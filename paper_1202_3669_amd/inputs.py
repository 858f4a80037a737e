"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no hashing arithmetic: it only draws bytes, edit scripts,
file sizes and request streams from numpy's PCG64 generator
(``numpy.random.default_rng(seed)``), so that the GPU path and the CPU oracle
see identical inputs.

The workloads stand in for the paper's evaluation data (Sec. 4.3): uniform
random bytes for the "different" workload, the same buffer twice for the
"similar" workload, and seeded edits of a base version for successive
versions of a file (the BLAST checkpoint images of Sec. 4.3 are not
available; edited synthetic versions take their place).
"""
from __future__ import annotations

import numpy as np

KiB = 1 << 10
MiB = 1 << 20
GiB = 1 << 30


def uniform_bytes(seed: int, n: int) -> np.ndarray:
    """``n`` uniform random bytes from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, size=n, dtype=np.uint8)


def edited_version(base: np.ndarray, seed: int, n_edits: int, size_lo: int = 1 * KiB,
                   size_hi: int = 4 * KiB):
    """Derive a new version of ``base`` by ``n_edits`` seeded edits.

    Edit positions are uniform over ``[0, len(base))`` and sorted; each edit is
    an insert, a delete or an overwrite (uniform) of ``size`` bytes, size
    uniform in ``[size_lo, size_hi]``; new bytes come from the same generator.
    The new version is built in one left-to-right pass; an edit that starts
    inside the region consumed by the previous edit is moved to the end of
    that region.  Returns ``(new_bytes, edits)`` where ``edits`` lists
    ``(kind, position_in_base, size)`` with kind in {"insert", "delete",
    "overwrite"}.
    """
    rng = np.random.default_rng(seed)
    length = int(base.size)
    pos = np.sort(rng.integers(0, max(length, 1), size=n_edits))
    kinds = rng.integers(0, 3, size=n_edits)
    sizes = rng.integers(size_lo, size_hi + 1, size=n_edits)
    pieces = []
    edits = []
    cursor = 0
    for p, k, sz in zip(pos.tolist(), kinds.tolist(), sizes.tolist()):
        p = max(p, cursor)
        if p > length:
            p = length
        pieces.append(base[cursor:p])
        if k == 0:
            pieces.append(rng.integers(0, 256, size=sz, dtype=np.uint8))
            cursor = p
            edits.append(("insert", p, sz))
        elif k == 1:
            cursor = min(p + sz, length)
            edits.append(("delete", p, cursor - p))
        else:
            n = min(sz, length - p)
            pieces.append(rng.integers(0, 256, size=n, dtype=np.uint8))
            cursor = p + n
            edits.append(("overwrite", p, n))
    pieces.append(base[cursor:])
    return np.concatenate(pieces) if pieces else base.copy(), edits


def lognormal_sizes(seed: int, n: int, median: int, sigma: float, lo: int, hi: int,
                    rng: np.random.Generator | None = None) -> np.ndarray:
    """``clip(round(exp(N(ln median, sigma))), lo, hi)`` as int64."""
    rng = np.random.default_rng(seed) if rng is None else rng
    x = np.exp(rng.normal(np.log(median), sigma, size=n))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def file_batch(seed: int, n_files: int, median: int = 256 * KiB, sigma: float = 1.5,
               cap: int = 64 * MiB, align: int = 1):
    """Many files of log-normal sizes packed into one arena.

    Returns ``(arena, offsets, lengths)``: file ``j`` occupies
    ``arena[offsets[j] : offsets[j] + lengths[j]]``.  With ``align > 1`` each
    file starts at a multiple of ``align`` (gap bytes are random too).
    Sizes and contents come from one generator seeded with ``seed``.
    """
    rng = np.random.default_rng(seed)
    lengths = lognormal_sizes(seed, n_files, median, sigma, 1, cap, rng=rng)
    offsets = np.zeros(n_files, dtype=np.int64)
    pos = 0
    for j in range(n_files):
        pos = (pos + align - 1) // align * align
        offsets[j] = pos
        pos += int(lengths[j])
    arena = rng.integers(0, 256, size=pos, dtype=np.uint8)
    return arena, offsets.astype(np.uint64), lengths.astype(np.uint64)


def request_stream(seed: int, n: int, rate_per_s: float, median: int = 1 * MiB,
                   sigma: float = 1.85, lo: int = 4 * KiB, hi: int = 256 * MiB,
                   mix=(0.5, 0.3, 0.2)):
    """Poisson arrivals of hash requests.

    Returns ``(arrival_s, sizes, kinds)``: exponential inter-arrival times at
    ``rate_per_s``; log-normal sizes clipped to ``[lo, hi]``; kinds 0 = block
    SHA-1, 1 = block MD5, 2 = content-based chunking, drawn with ``mix``.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    arrival = np.cumsum(gaps) - gaps[0]
    sizes = lognormal_sizes(seed, n, median, sigma, lo, hi, rng=rng)
    kinds = rng.choice(3, size=n, p=np.asarray(mix, dtype=np.float64))
    return arrival, sizes, kinds.astype(np.int64)
