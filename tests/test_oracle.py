"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself:

* MD5 / SHA-1 against Python's ``hashlib`` (OpenSSL, an independent
  implementation) on every length 0..1100, on the padding edges and on large
  messages.  The RFC 1321 / FIPS 180 known-answer documents are not available
  here, so ``hashlib`` on the standards' short example messages stands in.
* The direct hash against its closed form written with ``hashlib``
  (segment k = data[kB:(k+1)B], root = H(concat(digests))), including the
  single-segment special case root = H(H(data)).
* The window scan against per-offset ``hashlib`` brute force, the window count
  against its closed form (mask 0 makes every window a candidate), and the
  candidate density against its binomial expectation on random bytes.
* The greedy chunk selection against the properties that characterise it
  (partition, minimum size, ends are candidate ends, no skipped eligible
  candidate), and its degenerate cases; with a maximum chunk size, against
  the step-by-step characterisation of each cut (the first eligible
  candidate end within reach, else a forced cut exactly max past the
  previous one), the closed form without candidates, and the reduction to
  no maximum when no chunk can reach it.
* Chunk digests against ``hashlib`` per chunk; similarity against constructed
  digest sets with a known overlap.
* The block-map write (Sec. 3.2.1: a chunk whose digest the store already
  holds is not stored again) against a Python ``set`` walked chunk by chunk
  over successive writes with planted repeats within and across writes, and
  against closed forms: one digest written k times, a write repeated, a
  write of an old version's digests followed by a new version's (duplicates
  = the similarity count), the capacity refusal that changes nothing.
"""
import hashlib
import math

import numpy as np
import pytest

import oracle
from paper_1202_3669_amd import inputs

H = {oracle.MD5: hashlib.md5, oracle.SHA1: hashlib.sha1}
KINDS = [oracle.MD5, oracle.SHA1]


def _rand(seed, n):
    return inputs.uniform_bytes(seed, n)


# ----------------------------------------------------------------- hashes --
@pytest.mark.parametrize("kind", KINDS)
def test_hash_all_lengths_vs_hashlib(kind):
    data = _rand(11, 1101).tobytes()
    for n in range(0, 1101):
        assert oracle.hash(kind, data[:n]) == H[kind](data[:n]).digest(), n


@pytest.mark.parametrize("kind", KINDS)
def test_hash_padding_edges_and_large(kind):
    data = _rand(12, (1 << 20) + 200).tobytes()
    for n in [55, 56, 57, 63, 64, 65, 119, 120, 121, 127, 128, 129, 4095, 4096, 4097,
              65536, (1 << 20) + 13]:
        assert oracle.hash(kind, data[:n]) == H[kind](data[:n]).digest(), n
    million_a = b"a" * 1_000_000
    assert oracle.hash(kind, million_a) == H[kind](million_a).digest()


@pytest.mark.parametrize("kind", KINDS)
def test_hash_standard_example_messages(kind):
    alnum = bytes(range(ord("A"), ord("Z") + 1)) + bytes(range(ord("a"), ord("z") + 1)) + \
        bytes(range(ord("0"), ord("9") + 1))
    msgs = [b"", b"a", b"abc", b"message digest", bytes(range(ord("a"), ord("z") + 1)), alnum,
            b"1234567890" * 8]
    for m in msgs:
        assert oracle.hash(kind, m) == H[kind](m).digest()


def test_digest_sizes():
    assert oracle.digest_size(oracle.MD5) == 16
    assert oracle.digest_size(oracle.SHA1) == 20


# ------------------------------------------------------------ direct hash --
CASES = [(0, 64), (1, 64), (63, 64), (64, 64), (65, 64), (1000, 1), (1000, 7), (4096, 4096),
         (5000, 4096), (3 * 4096 + 1, 4096), (100_000, 1000), (65536 * 3 + 17, 65536),
         (12345, 100000)]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("length,block", CASES)
def test_leaves_and_root_closed_form(kind, length, block):
    data = _rand(13, length).tobytes()
    lv, rt = oracle.direct_hash(kind, data, block)
    n = math.ceil(length / block) if length else 0
    expect = [H[kind](data[k * block:(k + 1) * block]).digest() for k in range(n)]
    assert lv.shape == (n, oracle.digest_size(kind))
    assert [bytes(r) for r in lv] == expect
    assert rt == H[kind](b"".join(expect)).digest()


@pytest.mark.parametrize("kind", KINDS)
def test_root_single_segment_is_hash_of_hash(kind):
    data = _rand(14, 5000).tobytes()
    lv, rt = oracle.direct_hash(kind, data, 8192)
    assert lv.shape[0] == 1
    assert rt == H[kind](H[kind](data).digest()).digest()
    assert rt != H[kind](data).digest()


@pytest.mark.parametrize("kind", KINDS)
def test_leaf_ranges_concatenate(kind):
    data = _rand(15, 70_001)
    full = oracle.leaves(kind, data, 1000)
    parts = np.concatenate([oracle.leaves(kind, data, 1000, a, b)
                            for a, b in [(0, 13), (13, 14), (14, 71)]])
    assert np.array_equal(full, parts)
    assert np.array_equal(full, oracle.leaves_sharded(kind, data, 1000, threads=4))


# ----------------------------------------------------------- window scan --
def _brute(kind, data, w, s, mask, target):
    out = []
    i = 0
    while i + w <= len(data):
        v = int.from_bytes(H[kind](data[i:i + w]).digest()[:4], "little")
        if (v & mask) == target:
            out.append(i)
        i += s
    return out


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("w", [1, 20, 55, 56, 64, 100])
def test_window_scan_vs_bruteforce(kind, w):
    data = _rand(16 + w, 700).tobytes()
    for s in range(1, 8):
        for mask, target in [(0, 0), (1, 0), (3, 1), (0xF, 0x5), (0xFF, 0x3C)]:
            got = oracle.window_scan(kind, data, w, s, mask, target)
            assert got.tolist() == _brute(kind, data, w, s, mask, target), (w, s, mask)


@pytest.mark.parametrize("length,w,s", [(0, 20, 1), (19, 20, 1), (20, 20, 1), (21, 20, 4),
                                        (1000, 20, 1), (1000, 20, 4), (1001, 7, 3),
                                        (64, 64, 5)])
def test_window_count_closed_form(length, w, s):
    data = _rand(17, length)
    expect = (length - w) // s + 1 if length >= w else 0
    assert oracle.window_count(length, w, s) == expect
    got = oracle.window_scan(oracle.MD5, data, w, s, 0, 0)
    assert got.tolist() == [k * s for k in range(expect)]


def test_predicate_reads_low_bits_of_first_word():
    # Candidate iff the little-endian integer of digest bytes 0..3, masked,
    # equals the target: check against the digest computed by hashlib.
    data = _rand(18, 3000).tobytes()
    for i in range(0, 200):
        d = hashlib.md5(data[i:i + 20]).digest()
        low = d[0] & 0xF
        got = oracle.window_scan(oracle.MD5, data[i:i + 20], 20, 1, 0xF, low)
        assert got.tolist() == [0]


def test_candidate_density_matches_2_pow_minus_12():
    # Small workload: 4 MiB of seed-1 bytes, w = 20, s = 1, low 12 bits == 0.
    data = inputs.uniform_bytes(1, 4 << 20)
    n = oracle.window_count(data.size, 20, 1)
    got = oracle.window_scan_sharded(oracle.MD5, data, 20, 1, 0xFFF, 0, threads=8)
    mean = n / 4096
    sd = math.sqrt(n * (1 / 4096) * (1 - 1 / 4096))
    assert abs(got.size - mean) < 5 * sd
    assert np.all(np.diff(got.astype(np.int64)) > 0)


def test_window_ranges_concatenate():
    data = _rand(19, 50_000)
    full = oracle.window_scan(oracle.MD5, data, 20, 3, 0x1F, 7)
    nwin = oracle.window_count(data.size, 20, 3)
    parts = np.concatenate([oracle.window_scan(oracle.MD5, data, 20, 3, 0x1F, 7, a, b)
                            for a, b in [(0, 1000), (1000, 1001), (1001, nwin)]])
    assert np.array_equal(full, parts)
    assert np.array_equal(full, oracle.window_scan_sharded(oracle.MD5, data, 20, 3, 0x1F, 7, 4))


# ----------------------------------------------------------- chunk select --
def _check_greedy(starts, w, length, min_chunk, ends):
    ends = [int(e) for e in ends]
    if length == 0:
        assert ends == []
        return
    cand_ends = sorted({int(s) + w for s in starts})
    assert ends[-1] == length
    assert all(b > a for a, b in zip([0] + ends, ends)), "ends strictly increase"
    last = 0
    for e in ends[:-1]:
        assert e in cand_ends, "every cut is a candidate end"
        assert e - last >= min_chunk, "every chunk but the last is >= min"
        assert e < length
        # no eligible candidate was skipped between the previous cut and e
        assert not [c for c in cand_ends if c < e and c - last >= min_chunk and c > last]
        last = e
    # nothing eligible after the last cut
    assert not [c for c in cand_ends if c < length and c - last >= min_chunk and c > last]


@pytest.mark.parametrize("seed", range(8))
def test_chunk_select_properties(seed):
    rng = np.random.default_rng(100 + seed)
    length = int(rng.integers(1, 200_000))
    w = int(rng.integers(1, 64))
    n = int(rng.integers(0, 400))
    starts = np.unique(rng.integers(0, max(length - w + 1, 1), size=n)).astype(np.uint64)
    for min_chunk in [0, 1, 100, 2048, 10_000, length + 1]:
        ends = oracle.chunk_select(starts, w, length, min_chunk)
        _check_greedy(starts, w, length, min_chunk, ends)


def test_chunk_select_degenerate():
    assert oracle.chunk_select(np.zeros(0, np.uint64), 20, 0, 2048).tolist() == []
    assert oracle.chunk_select(np.zeros(0, np.uint64), 20, 500, 2048).tolist() == [500]
    st = np.array([0, 5, 9, 30], dtype=np.uint64)
    # min 0: every candidate end below len is a cut
    assert oracle.chunk_select(st, 4, 100, 0).tolist() == [4, 9, 13, 34, 100]
    # a candidate ending exactly at len is not a separate cut
    assert oracle.chunk_select(st, 70, 100, 0).tolist() == [70, 75, 79, 100]
    # min larger than the block: one chunk
    assert oracle.chunk_select(st, 4, 100, 1000).tolist() == [100]


def _check_greedy_max(starts, w, length, min_chunk, max_chunk, ends):
    """Every cut is the unique choice of the rule with a maximum: from the
    previous cut p, the first candidate end c with p + step <= c < length if
    it lies within p + max, else the forced cut p + max (step = max(min, 1))."""
    ends = [int(e) for e in ends]
    if length == 0:
        assert ends == []
        return
    step = max(min_chunk, 1)
    cand_ends = sorted({int(s) + w for s in starts})
    assert ends[-1] == length
    assert all(b > a for a, b in zip([0] + ends, ends)), "ends strictly increase"
    assert all(b - a <= max_chunk for a, b in zip([0] + ends, ends)), "no chunk longer than max"
    p = 0
    for e in ends[:-1]:
        eligible = [c for c in cand_ends if p + step <= c < length]
        first = eligible[0] if eligible else None
        if first is not None and first - p <= max_chunk:
            assert e == first, "the first eligible candidate end within reach is the cut"
        else:
            assert e == p + max_chunk, "forced cut exactly max past the previous cut"
        p = e
    eligible = [c for c in cand_ends if p + step <= c < length]
    assert not (eligible and eligible[0] - p <= max_chunk), "a natural cut after the last one was missed"
    assert length - p <= max_chunk


@pytest.mark.parametrize("seed", range(8))
def test_chunk_select_max_properties(seed):
    rng = np.random.default_rng(300 + seed)
    length = int(rng.integers(1, 100_000))
    w = int(rng.integers(1, 64))
    n = int(rng.integers(0, 300))
    starts = np.unique(rng.integers(0, max(length - w + 1, 1), size=n)).astype(np.uint64)
    for min_chunk in [0, 1, 100, 2048]:
        for max_chunk in [max(min_chunk, 1), 2 * max(min_chunk, 1) + 7, 5000, 40_000]:
            ends = oracle.chunk_select(starts, w, length, min_chunk, max_chunk)
            _check_greedy_max(starts, w, length, min_chunk, max_chunk, ends)


def test_chunk_select_max_reductions():
    rng = np.random.default_rng(399)
    for _ in range(20):
        length = int(rng.integers(1, 50_000))
        starts = np.unique(rng.integers(0, length, size=int(rng.integers(0, 200)))).astype(np.uint64)
        starts = starts[starts + 20 <= length] if length >= 20 else starts[:0]
        for mn in [0, 64, 3000]:
            base = oracle.chunk_select(starts, 20, length, mn)
            # a maximum no chunk can reach changes nothing
            assert np.array_equal(oracle.chunk_select(starts, 20, length, mn, max(length + 1, mn)), base)
    # no candidates: forced cuts every max bytes (closed form)
    L, M = 100_001, 7_000
    assert oracle.chunk_select(np.zeros(0, np.uint64), 20, L, 0, M).tolist() == \
        list(range(M, L, M)) + [L]
    # max < min is rejected
    with pytest.raises(ValueError):
        oracle.chunk_select(np.zeros(0, np.uint64), 20, 1000, 100, 50)


# --------------------------------------------------------- chunk digests --
@pytest.mark.parametrize("kind", KINDS)
def test_chunk_digests_vs_hashlib(kind):
    data = _rand(20, 30_000).tobytes()
    ends = np.array([1, 2, 64, 1000, 1055, 29_999, 30_000], dtype=np.uint64)
    dig = oracle.chunk_digests(kind, data, ends)
    prev = 0
    for j, e in enumerate(ends.tolist()):
        assert bytes(dig[j]) == H[kind](data[prev:e]).digest()
        prev = e


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("segment", [1, 7, 64, 1000, 4096])
def test_chunk_digests_two_level_vs_hashlib(kind, segment):
    # Each chunk direct-hashed (Sec. 3.2.2 applied per chunk, Sec. 3.2.4):
    # closed form with hashlib -- the digest of the concatenated digests of
    # the chunk's segment-size pieces, the last piece shorter.
    data = _rand(22, 12_000).tobytes()
    ends = np.array([1, 2, 64, 65, 1000, 1056, 5000, 11_999, 12_000], dtype=np.uint64)
    dig = oracle.chunk_digests(kind, data, ends, segment)
    prev = 0
    for j, e in enumerate(ends.tolist()):
        c = data[prev:e]
        leaves = b"".join(H[kind](c[k:k + segment]).digest() for k in range(0, len(c), segment))
        assert bytes(dig[j]) == H[kind](leaves).digest()
        if segment >= len(c):  # one segment: the digest of the chunk's digest
            assert bytes(dig[j]) == H[kind](H[kind](c).digest()).digest()
        prev = e


def test_chunk_pipeline_partitions_input():
    data = _rand(21, 300_000)
    starts, ends, dig = oracle.chunk(oracle.MD5, oracle.SHA1, data, 20, 1, 0xFF, 0, 2048, 4)
    _check_greedy(starts, 20, data.size, 2048, ends)
    assert dig.shape == (ends.size, 20)


# ------------------------------------------------------------ similarity --
@pytest.mark.parametrize("kind", KINDS)
def test_similarity_constructed_overlap(kind):
    d = oracle.digest_size(kind)
    rng = np.random.default_rng(22)
    a = rng.integers(0, 256, size=(500, d), dtype=np.uint8)
    b = a[rng.permutation(500)[:300]].copy()
    changed = rng.choice(300, size=37, replace=False)
    b[changed, 0] ^= 0xFF  # these no longer occur in A (w.h.p.; checked below)
    a_set = {bytes(r) for r in a}
    assert sum(bytes(b[j]) in a_set for j in changed) == 0
    lens = rng.integers(1, 10_000, size=300).astype(np.uint64)
    m, mb = oracle.similarity(kind, a, b, lens)
    keep = np.ones(300, bool)
    keep[changed] = False
    assert m == 263
    assert mb == int(lens[keep].sum())


def test_similarity_multiplicity_and_identity():
    rng = np.random.default_rng(23)
    a = rng.integers(0, 256, size=(50, 20), dtype=np.uint8)
    b = np.concatenate([a, a[:10], a[:10]])  # duplicates count each time
    assert oracle.similarity(oracle.SHA1, a, b)[0] == 70
    assert oracle.similarity(oracle.SHA1, a, a)[0] == 50
    assert oracle.similarity(oracle.SHA1, a[:0], a)[0] == 0
    assert oracle.similarity(oracle.SHA1, a, a[:0])[0] == 0


def test_edited_versions_are_mostly_similar_at_stride_1():
    # Expected behaviour, not a pin: content-defined chunks survive edits.
    base = inputs.uniform_bytes(3, 1 << 20)
    newv, edits = inputs.edited_version(base, 4, 4)
    assert len(edits) == 4
    _, ea, da = oracle.chunk(oracle.MD5, oracle.SHA1, base, 20, 1, 0xFF, 0, 2048, 8)
    _, eb, db = oracle.chunk(oracle.MD5, oracle.SHA1, newv, 20, 1, 0xFF, 0, 2048, 8)
    m, _ = oracle.similarity(oracle.SHA1, da, db)
    assert m / len(db) > 0.8


# ------------------------------------------------------------- block map --
def _planted_writes(seed, d, plan):
    """Digests of successive writes: random rows, with repeats planted inside
    a write and copies of rows written before; lengths random."""
    rng = np.random.default_rng(seed)
    written, out = [], []
    for n, inner, cross in plan:
        dig = rng.integers(0, 256, size=(n, d), dtype=np.uint8)
        for _ in range(inner if n > 1 else 0):
            i, j = sorted(rng.choice(n, size=2, replace=False).tolist())
            dig[j] = dig[i]
        if written and n:
            pool = np.concatenate(written)
            for j in rng.choice(n, size=min(cross, n), replace=False).tolist():
                dig[j] = pool[int(rng.integers(0, len(pool)))]
        lens = rng.integers(1, 100_000, size=n).astype(np.uint64)
        out.append((dig, lens))
        if n:
            written.append(dig)
    return out


@pytest.mark.parametrize("kind", KINDS)
def test_blockmap_writes_vs_python_set(kind):
    d = oracle.digest_size(kind)
    plan = [(3000, 40, 0), (5000, 300, 400), (1, 0, 1), (0, 0, 0), (2, 0, 2), (8000, 800, 2000)]
    bm = oracle.BlockMap(kind)
    held = set()
    for w, (dig, lens) in enumerate(_planted_writes(31 + kind, d, plan)):
        exp = np.zeros(len(dig), dtype=bool)
        for i, row in enumerate(dig):  # the store, one chunk at a time
            key = row.tobytes()
            exp[i] = key in held
            held.add(key)
        dup, c, b = bm.write(dig, lengths=lens)
        assert np.array_equal(dup, exp), f"write {w}"
        assert c == int(exp.sum()) and b == int(lens[exp].sum()), f"write {w}"
        assert bm.size() == len(held), f"write {w}"
    bm.close()


def test_blockmap_closed_forms():
    rng = np.random.default_rng(32)
    one = rng.integers(0, 256, size=(1, 20), dtype=np.uint8)
    lens = np.arange(1, 8, dtype=np.uint64)
    bm = oracle.BlockMap(oracle.SHA1)
    # one digest written 7 times: the first is stored, the rest are duplicates
    dup, c, b = bm.write(np.repeat(one, 7, axis=0), lengths=lens)
    assert dup.tolist() == [False] + [True] * 6 and (c, b) == (6, 27) and bm.size() == 1
    # a write repeated: every chunk a duplicate, nothing added
    a = rng.integers(0, 256, size=(400, 20), dtype=np.uint8)
    la = rng.integers(1, 5000, size=400).astype(np.uint64)
    dup, c, b = bm.write(a, lengths=la)
    assert not dup.any() and bm.size() == 401
    dup, c, b = bm.write(a, lengths=la)
    assert dup.all() and (c, b) == (400, int(la.sum())) and bm.size() == 401
    # ends instead of lengths
    ends = np.cumsum(la)
    assert bm.write(a, ends=ends)[2] == int(la.sum())
    # an empty write changes nothing
    assert bm.write(a[:0])[1:] == (0, 0) and bm.size() == 401
    bm.close()


def test_blockmap_new_version_duplicates_equal_similarity():
    # Old version's chunks (all distinct) stored, then a new version with no
    # repeats of its own: its duplicates are exactly the chunks the
    # similarity lookup finds, by count and by bytes.
    rng = np.random.default_rng(33)
    a = rng.integers(0, 256, size=(600, 16), dtype=np.uint8)
    b = rng.integers(0, 256, size=(500, 16), dtype=np.uint8)
    pick = rng.choice(500, size=220, replace=False)
    b[pick] = a[rng.choice(600, size=220, replace=False)]
    lb = rng.integers(1, 9000, size=500).astype(np.uint64)
    bm = oracle.BlockMap(oracle.MD5)
    bm.write(a)
    dup, c, by = bm.write(b, lengths=lb)
    assert (c, by) == oracle.similarity(oracle.MD5, a, b, lb) == (220, int(lb[pick].sum()))
    assert bm.size() == 600 + 280
    bm.close()


def test_blockmap_capacity_refusal_changes_nothing():
    rng = np.random.default_rng(34)
    a = rng.integers(0, 256, size=(60, 20), dtype=np.uint8)
    bm = oracle.BlockMap(oracle.SHA1, capacity=100)
    bm.write(a)
    with pytest.raises(OverflowError):
        bm.write(rng.integers(0, 256, size=(41, 20), dtype=np.uint8))
    assert bm.size() == 60
    dup, c, _ = bm.write(a[:40])  # size + n == capacity is accepted
    assert dup.all() and c == 40 and bm.size() == 60
    bm.close()
