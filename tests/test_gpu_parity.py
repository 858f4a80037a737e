"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Everything here is integer and byte work, so every comparison is bit-exact.
Inputs are seeded synthetic bytes with the shapes of the paper's workloads:
  * small: 4 MiB uniform bytes (seed 1), 64 KiB segments, w = 20, stride 1,
    boundary when the low 12 bits of the window digest are 0;
  * large: 1 GiB uniform bytes (seed 2), segments of 4 KiB / 64 KiB / 1 MiB;
  * similarity: 256 MiB version A (seed 3), version B from seeded edits
    (seed 4, 1-4 KiB insert/delete/overwrite, one per MiB), stride 1 and 4,
    minimum chunk 2 KiB, SHA-1 chunk digests;
plus edge cases: empty and tiny inputs, ragged tails, odd segment sizes,
unaligned base pointers, dense boundary masks (the overflow path), window
sizes that need one and several MD5 blocks, and truncated outputs.
"""
import ctypes
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1202_3669_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
THREADS = max(1, min(16, os.cpu_count() or 1))
KINDS = [0, 1]  # MD5, SHA-1 in both numberings
MiB = 1 << 20


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hg():
    from paper_1202_3669_amd import hashgpu
    return hashgpu


@pytest.fixture(scope="module")
def ctx(hg):
    c = hg.Context(0)
    yield c
    c.close()


def dev(arr: np.ndarray, offset: int = 0):
    """Device copy of a uint8 array whose first byte sits `offset` bytes past
    a 256-byte aligned allocation (offset != 0 gives an unaligned base)."""
    t = torch.zeros(arr.size + offset + 16, dtype=torch.uint8, device="cuda")
    if arr.size:
        t[offset:offset + arr.size] = torch.from_numpy(arr).cuda()
    return t[offset:offset + arr.size]


def host(t):
    return t.cpu().numpy()


# ------------------------------------------------------------ direct hash --
@pytest.mark.parametrize("kind", KINDS)
def test_block_hash_small_workload(ctx, kind):
    data = inputs.uniform_bytes(1, 4 * MiB)
    note(f"block_hash small kind={kind}")
    lv, rt = ctx.block_hash(dev(data), 64 * 1024, kind)
    torch.cuda.synchronize()
    exp_lv = oracle.leaves(kind, data, 64 * 1024)
    assert lv.shape == (64, oracle.digest_size(kind))
    assert np.array_equal(host(lv), exp_lv)
    assert bytes(host(rt)) == oracle.root(kind, exp_lv)


EDGE = [(0, 64, 0), (1, 64, 0), (55, 64, 0), (56, 64, 0), (63, 64, 0), (64, 64, 0), (65, 64, 0),
        (119, 64, 0), (120, 64, 0), (1000, 1, 0), (1000, 7, 3), (5000, 100, 1), (4097, 4096, 0),
        (65536 * 3 + 17, 65536, 2), (100_000, 1000, 1), (12345, 1 << 20, 0),
        ((1 << 20) + 13, 4096, 0), ((1 << 20) + 13, 4096, 5), (300_001, 64 * 3, 7)]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("length,block,offset", EDGE)
def test_block_hash_edge_cases(ctx, kind, length, block, offset):
    data = inputs.uniform_bytes(100 + length % 97, length)
    note(f"block_hash edge kind={kind} len={length} B={block} off={offset}")
    lv, rt = ctx.block_hash(dev(data, offset), block, kind)
    torch.cuda.synchronize()
    exp_lv = oracle.leaves(kind, data, block)
    assert np.array_equal(host(lv), exp_lv)
    assert bytes(host(rt)) == oracle.root(kind, exp_lv)


# Many segments: MD5 goes through the LDS-staged kernel (whole lines per
# load instruction); ragged last segments, partial last waves, unaligned
# bases and segment sizes that are not whole line pairs.
MANY = [(65536 * 256 + 77, 256, 3), (70000 * 320 + 5, 320, 1), (65536 * 4096 - 1000, 4096, 0),
        (65600 * 200, 200, 0), (65537 * 1000 + 999, 1000, 7)]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("length,block,offset", MANY)
def test_block_hash_many_segments(ctx, kind, length, block, offset):
    data = inputs.uniform_bytes(300 + length % 83, length)
    note(f"block_hash many kind={kind} len={length} B={block} off={offset}")
    lv, rt = ctx.block_hash(dev(data, offset), block, kind)
    torch.cuda.synchronize()
    exp_lv = oracle.leaves_sharded(kind, data, block, THREADS)
    assert np.array_equal(host(lv), exp_lv)
    assert bytes(host(rt)) == oracle.root(kind, exp_lv)


@pytest.mark.parametrize("length,block,offset", EDGE)
def test_block_hash_dual_edge_cases(ctx, length, block, offset):
    data = inputs.uniform_bytes(200 + length % 89, length)
    note(f"block_hash_dual edge len={length} B={block} off={offset}")
    lm, rm, ls, rs = ctx.block_hash_dual(dev(data, offset), block)
    torch.cuda.synchronize()
    for kind, lv, rt in ((oracle.MD5, lm, rm), (oracle.SHA1, ls, rs)):
        exp_lv = oracle.leaves(kind, data, block)
        assert np.array_equal(host(lv), exp_lv)
        assert bytes(host(rt)) == oracle.root(kind, exp_lv)


def test_block_hash_dual_streams_host_input(ctx):
    # Host input in pinned staging pieces (two 64 MiB pieces and a tail),
    # root-only outputs for MD5 and leaves-only for SHA-1.
    data = inputs.uniform_bytes(211, 130 * MiB + 4097)
    note("block_hash_dual host input")
    rm = np.zeros(16, dtype=np.uint8)
    ls = np.zeros(((data.size + 65535) // 65536, 20), dtype=np.uint8)
    from paper_1202_3669_amd import hashgpu as hgm
    st = hgm.hg_block_hash_dual(ctx.handle, data.ctypes.data, data.size, 65536, None, rm.ctypes.data,
                                ls.ctypes.data, None, 0, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    exp_m = oracle.leaves_sharded(oracle.MD5, data, 65536, THREADS)
    assert bytes(rm) == oracle.root(oracle.MD5, exp_m)
    assert np.array_equal(ls, oracle.leaves_sharded(oracle.SHA1, data, 65536, THREADS))


@pytest.mark.parametrize("kind", KINDS)
def test_block_hash_root_only_and_leaves_only(ctx, kind):
    data = inputs.uniform_bytes(7, 300_000)
    note(f"block_hash root-only kind={kind}")
    d = dev(data)
    lv, rt = ctx.block_hash(d, 4096, kind, leaves=False)
    assert lv is None
    exp_lv = oracle.leaves(kind, data, 4096)
    assert bytes(host(rt)) == oracle.root(kind, exp_lv)
    lv, rt = ctx.block_hash(d, 4096, kind, root=False)
    assert rt is None and np.array_equal(host(lv), exp_lv)


@pytest.mark.parametrize("pinned", [False, True])
def test_block_hash_streams_host_input(ctx, pinned):
    # Larger than two 64 MiB staging pieces, with a ragged tail.
    data = inputs.uniform_bytes(8, 150 * MiB + 1234)
    note(f"block_hash host input pinned={pinned}")
    t = torch.from_numpy(data)
    if pinned:
        t = t.pin_memory()
    lv, rt = ctx.block_hash(t, 64 * 1024, 0)
    torch.cuda.synchronize()
    exp_lv = oracle.leaves_sharded(0, data, 64 * 1024, THREADS)
    assert np.array_equal(host(lv), exp_lv)
    assert bytes(host(rt)) == oracle.root(0, exp_lv)


# ----------------------------------------------------------- window scan --
def test_window_scan_small_workload(ctx):
    data = inputs.uniform_bytes(1, 4 * MiB)
    note("window_scan small w=20 s=1 mask=0xfff")
    got = host(ctx.window_scan(dev(data), 20, 1, 0xFFF, 0))
    exp = oracle.window_scan_sharded(0, data, 20, 1, 0xFFF, 0, THREADS)
    assert got.dtype == np.int64
    assert np.array_equal(got.astype(np.uint64), exp)


WS_CASES = []
for _w in [1, 20, 55, 56, 64, 100]:
    for _s in [1, 2, 3, 4, 7]:
        WS_CASES.append((_w, _s, 0xF, 3))
WS_CASES += [(20, 1, 0xFF, 0), (20, 4, 0xFF, 0x11), (20, 1, 0, 0), (20, 4, 0, 0), (33, 5, 1, 1),
             (4096, 1, 0x3, 0), (4096, 4096, 0, 0), (200, 1000, 0, 0)]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("w,s,mask,target", WS_CASES)
def test_window_scan_cases(ctx, kind, w, s, mask, target):
    length = 20_000 + 7 * w + s
    data = inputs.uniform_bytes(200 + w + s, length)
    for off in (0, 3):
        note(f"window_scan kind={kind} w={w} s={s} mask={mask:#x} off={off}")
        got = host(ctx.window_scan(dev(data, off), w, s, mask, target, kind))
        exp = oracle.window_scan(kind, data, w, s, mask, target)
        assert np.array_equal(got.astype(np.uint64), exp)


@pytest.mark.parametrize("length", [0, 1, 19, 20, 21, 4095, 4096 * 16 + 3, 65537])
def test_window_scan_short_and_ragged(ctx, length):
    data = inputs.uniform_bytes(300, length)
    for s in (1, 4):
        note(f"window_scan ragged len={length} s={s}")
        got = host(ctx.window_scan(dev(data), 20, s, 0x7, 0))
        exp = oracle.window_scan(0, data, 20, s, 0x7, 0)
        assert np.array_equal(got.astype(np.uint64), exp)


@pytest.mark.parametrize("s", [1, 4])
def test_window_scan_dense_mask_uses_overflow_path(ctx, s):
    # mask 0: every window is a candidate, far beyond the per-tile bucket.
    data = inputs.uniform_bytes(301, 300_000)
    note(f"window_scan dense s={s}")
    got = host(ctx.window_scan(dev(data), 20, s, 0, 0))
    n = oracle.window_count(data.size, 20, s)
    assert np.array_equal(got, np.arange(n, dtype=np.int64) * s)
    # Mixed density: some tiles overflow, others use their bucket.
    got = host(ctx.window_scan(dev(data), 20, s, 0x3, 2))
    exp = oracle.window_scan(0, data, 20, s, 0x3, 2)
    assert np.array_equal(got.astype(np.uint64), exp)


def test_window_scan_truncation_reports_full_count(ctx, hg):
    data = inputs.uniform_bytes(302, 200_000)
    exp = oracle.window_scan(0, data, 20, 1, 0xFF, 0)
    assert exp.size > 10
    note("window_scan truncation")
    d = dev(data)
    out = torch.zeros(10, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = hg.hg_window_scan(ctx.handle, d.data_ptr(), d.numel(), 20, 1, 0xFF, 0, hg.HG_MD5,
                           out.data_ptr(), 10, cnt.data_ptr(), hg.HG_IN_DEVICE | hg.HG_OUT_DEVICE,
                           torch.cuda.current_stream().cuda_stream)
    assert st == hg.HG_ETRUNC
    assert int(cnt.item()) == exp.size
    assert np.array_equal(host(out).astype(np.uint64), exp[:10])
    # Host outputs: the same status, count and prefix.
    out_h = (ctypes.c_uint64 * 10)()
    cnt_h = ctypes.c_uint64(0)
    st = hg.hg_window_scan(ctx.handle, d.data_ptr(), d.numel(), 20, 1, 0xFF, 0, hg.HG_MD5,
                           ctypes.addressof(out_h), 10, ctypes.addressof(cnt_h), hg.HG_IN_DEVICE,
                           torch.cuda.current_stream().cuda_stream)
    assert st == hg.HG_ETRUNC and cnt_h.value == exp.size
    assert list(out_h) == exp[:10].tolist()


# ---------------------------------------------------------------- chunks --
def _oracle_chunks(data, w, s, mask, target, min_chunk, wk=0, ck=1):
    starts = oracle.window_scan_sharded(wk, data, w, s, mask, target, THREADS)
    ends = oracle.chunk_select(starts, w, data.size, min_chunk)
    return ends, oracle.chunk_digests(ck, data, ends)


def test_chunk_small_workload(ctx):
    data = inputs.uniform_bytes(1, 4 * MiB)
    note("chunk small")
    ends, dig = ctx.chunk(dev(data), 20, 1, 0xFFF, 0, 2048)
    exp_ends, exp_dig = _oracle_chunks(data, 20, 1, 0xFFF, 0, 2048)
    assert np.array_equal(host(ends).astype(np.uint64), exp_ends)
    assert np.array_equal(host(dig), exp_dig)


CHUNK_CASES = [(0, 20, 1, 0xFF, 0, 2048, 0, 1), (10, 20, 1, 0xFF, 0, 2048, 0, 1),
               (5000, 20, 1, 0x3F, 0, 0, 0, 1), (5000, 20, 1, 0, 0, 0, 0, 1),
               (70_000, 20, 4, 0x3F, 1, 300, 0, 0), (70_000, 48, 3, 0x1F, 2, 500, 1, 1),
               (200_003, 20, 1, 0xFF, 0, 2048, 0, 1), (200_003, 64, 1, 0x7F, 5, 1000, 0, 1),
               (100_000, 20, 1, 0xFF, 0, 10 ** 9, 0, 1),
               # many superblocks (4096 candidates each); chains that skip
               # whole blocks and superblocks; every window a candidate
               (1_000_000, 20, 1, 0x3F, 0, 100_000, 0, 1), (1_000_000, 20, 1, 0xF, 0, 3000, 0, 1),
               (1_000_000, 20, 1, 0x3, 1, 700_000, 0, 1), (2_000_003, 20, 1, 0, 0, 0, 0, 1),
               (2_000_003, 20, 1, 0, 0, 5000, 0, 0), (2_000_003, 20, 4, 0, 0, 33, 0, 1)]


@pytest.mark.parametrize("case", CHUNK_CASES)
def test_chunk_cases(ctx, case):
    length, w, s, mask, target, mn, wk, ck = case
    data = inputs.uniform_bytes(400 + length % 101, length)
    for off in (0, 1):
        note(f"chunk case={case} off={off}")
        ends, dig = ctx.chunk(dev(data, off), w, s, mask, target, mn, wk, ck)
        exp_ends, exp_dig = _oracle_chunks(data, w, s, mask, target, mn, wk, ck)
        assert np.array_equal(host(ends).astype(np.uint64), exp_ends)
        assert np.array_equal(host(dig), exp_dig)


# Maximum chunk size (forced cuts): (length, w, s, mask, target, min, max).
MAX_CASES = [(0, 20, 1, 0xFF, 0, 2048, 4096), (100, 20, 1, 0xFF, 0, 0, 7),
             (200_003, 20, 1, 0xFFF, 0, 2048, 8192), (200_003, 20, 1, 0xFF, 0, 2048, 2048),
             (300_000, 20, 1, 0xFFFFF, 0, 0, 1000),          # almost no candidates: forced runs
             (1_000_000, 20, 1, 0x3F, 0, 100, 150),          # dense candidates, tight max
             (1_000_000, 20, 4, 0x7FF, 3, 3000, 5000), (2_000_003, 20, 1, 0xFFF, 0, 2048, 65536),
             (777_777, 33, 2, 0x1FF, 1, 1, 1)]               # max = step = 1: every byte a chunk


@pytest.mark.parametrize("case", MAX_CASES)
def test_chunk_with_max(ctx, case):
    length, w, s, mask, target, mn, mx = case
    if mn == 1 and mx == 1:
        length = 5000  # one chunk per byte: keep it small
    data = inputs.uniform_bytes(450 + length % 97, length)
    starts = oracle.window_scan_sharded(0, data, w, s, mask, target, THREADS)
    exp_ends = oracle.chunk_select(starts, w, data.size, mn, mx)
    exp_dig = oracle.chunk_digests(1, data, exp_ends)
    for off in (0, 3):
        note(f"chunk max case={case} off={off}")
        ends, dig = ctx.chunk(dev(data, off), w, s, mask, target, mn, max_chunk=mx)
        assert np.array_equal(host(ends).astype(np.uint64), exp_ends)
        assert np.array_equal(host(dig), exp_dig)


TWO_LEVEL_CASES = [  # (length, mask, min, max, segment)
    (3 * 2**20 + 5, 0xFFF, 2048, 0, 4096),           # ~6 KiB chunks: one or two segments each
    (8 * 2**20 + 3, 0xFFFFF, 256 * 1024, 4 * 2**20, 4096),  # ~1.3 MB chunks, forced cuts
    (2**20 + 1, 0xFFF, 2048, 0, 64),                 # one padded block per segment
    (300_000, 0xFF, 0, 0, 1),                        # one-byte segments
    (2 * 2**20, 0xFFF, 2048, 0, 1 << 40),            # one segment per chunk: H(H(chunk))
    (777, 0xF, 10, 0, 100),
    (0, 0xFFF, 2048, 0, 4096),
]


@pytest.mark.parametrize("case", TWO_LEVEL_CASES)
@pytest.mark.parametrize("kind", [0, 1])
def test_chunk_two_level_digests(ctx, case, kind):
    length, mask, mn, mx, seg = case
    data = inputs.uniform_bytes(480 + length % 89, length)
    starts = oracle.window_scan_sharded(0, data, 20, 1, mask, 0, THREADS)
    exp_ends = oracle.chunk_select(starts, 20, data.size, mn, mx)
    exp_dig = oracle.chunk_digests(kind, data, exp_ends, seg)
    for off in (0, 3):
        note(f"two-level chunk digests case={case} kind={kind} off={off}")
        ends, dig = ctx.chunk(dev(data, off), 20, 1, mask, 0, mn, chunk_digest=kind, max_chunk=mx,
                              chunk_segment=seg)
        assert np.array_equal(host(ends).astype(np.uint64), exp_ends)
        assert np.array_equal(host(dig), exp_dig)


def test_chunk_two_level_host_input_and_small_capacity(ctx, hg):
    data = inputs.uniform_bytes(489, 5 * 2**20 + 17)
    starts = oracle.window_scan_sharded(0, data, 20, 1, 0xFFF, 0, THREADS)
    exp_ends = oracle.chunk_select(starts, 20, data.size, 2048)
    exp_dig = oracle.chunk_digests(1, data, exp_ends, 4096)
    note("two-level chunk digests, host input")
    ends, dig = ctx.chunk(torch.from_numpy(data), 20, 1, 0xFFF, 0, 2048, chunk_segment=4096)
    assert np.array_equal(host(ends).astype(np.uint64), exp_ends)
    assert np.array_equal(host(dig), exp_dig)
    note("two-level chunk digests, capacity below the chunk count")
    e = torch.zeros(10, dtype=torch.int64, device="cuda")
    d = torch.zeros((10, 20), dtype=torch.uint8, device="cuda")
    with pytest.raises(hg.HashGpuError):
        ctx.chunk(dev(data), 20, 1, 0xFFF, 0, 2048, out=(e, d), chunk_segment=4096)
    assert np.array_equal(host(e).astype(np.uint64), exp_ends[:10])
    assert np.array_equal(host(d), exp_dig[:10])


def test_chunk_max_rejects_max_below_min(ctx, hg):
    d = dev(inputs.uniform_bytes(451, 1000))
    with pytest.raises(hg.HashGpuError):
        ctx.chunk(d, 20, 1, 0xF, 0, 100, max_chunk=50)


def test_chunk_truncation(ctx, hg):
    data = inputs.uniform_bytes(402, 300_000)
    exp_ends, exp_dig = _oracle_chunks(data, 20, 1, 0xFF, 0, 1024)
    assert exp_ends.size > 5
    note("chunk truncation")
    ends, dig = ctx.chunk(dev(data), 20, 1, 0xFF, 0, 1024, capacity=5)  # retried with the full size
    assert np.array_equal(host(ends).astype(np.uint64), exp_ends)
    d = dev(data)
    p = hg.hg_chunk_params(20, 1, 0xFF, 0, 1024, 0, 0, 1)
    e = torch.zeros(5, dtype=torch.int64, device="cuda")
    dg = torch.zeros((5, 20), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = hg.hg_chunk(ctx.handle, d.data_ptr(), d.numel(), ctypes.byref(p), e.data_ptr(), 5,
                     cnt.data_ptr(), dg.data_ptr(), hg.HG_IN_DEVICE | hg.HG_OUT_DEVICE,
                     torch.cuda.current_stream().cuda_stream)
    assert st == hg.HG_ETRUNC and int(cnt.item()) == exp_ends.size
    assert np.array_equal(host(e).astype(np.uint64), exp_ends[:5])
    assert np.array_equal(host(dg), exp_dig[:5])


def test_chunk_async_with_host_count(ctx, hg):
    data = inputs.uniform_bytes(403, 3 * MiB + 77)
    exp_ends, exp_dig = _oracle_chunks(data, 20, 1, 0xFFF, 0, 2048)
    d = dev(data)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    ends = torch.zeros(4096, dtype=torch.int64, device="cuda")
    dig = torch.zeros((4096, 20), dtype=torch.uint8, device="cuda")
    note("chunk async, host count")
    e, g = ctx.chunk(d, 20, 1, 0xFFF, 0, 2048, stream=s, out=(ends, dig), asynchronous=True)
    s.synchronize()
    assert np.array_equal(host(e).astype(np.uint64), exp_ends)
    assert np.array_equal(host(g), exp_dig)
    n = ctypes.c_uint64(0)
    p = hg.hg_chunk_params(20, 1, 0xFFF, 0, 2048, 0, 0, 1)
    # HG_ASYNC needs device outputs.
    assert hg.hg_chunk(ctx.handle, d.data_ptr(), d.numel(), ctypes.byref(p), ends.data_ptr(), 4096,
                       ctypes.addressof(n), None, hg.HG_IN_DEVICE | hg.HG_ASYNC | hg.HG_COUNT_HOST,
                       s.cuda_stream) == hg.HG_EINVAL


# ------------------------------------------------------------ similarity --
@pytest.mark.parametrize("kind", KINDS)
def test_similarity_constructed(ctx, kind):
    d = oracle.digest_size(kind)
    rng = np.random.default_rng(500 + kind)
    a = rng.integers(0, 256, size=(3000, d), dtype=np.uint8)
    b = np.concatenate([a[rng.permutation(3000)[:1500]], a[:100],
                        rng.integers(0, 256, size=(700, d), dtype=np.uint8)])
    lens = rng.integers(1, 100_000, size=b.shape[0]).astype(np.int64)
    note(f"similarity constructed kind={kind}")
    m, mb = ctx.similarity(dev(a.reshape(-1)), dev(b.reshape(-1)),
                           torch.from_numpy(lens).cuda(), kind)
    em, emb = oracle.similarity(kind, a, b, lens.astype(np.uint64))
    assert (m, mb) == (em, emb)
    assert ctx.similarity(dev(a.reshape(-1)), dev(a.reshape(-1)), None, kind)[0] == 3000
    assert ctx.similarity(dev(a[:0].reshape(-1)), dev(b.reshape(-1)), None, kind)[0] == 0


def _versions(size, n_edits):
    a = inputs.uniform_bytes(3, size)
    b, _ = inputs.edited_version(a, 4, n_edits)
    return a, b


@pytest.mark.parametrize("stride", [1, 4])
def test_similarity_of_versions_small(ctx, stride):
    a, b = _versions(16 * MiB, 16)
    note(f"similarity versions 16MiB s={stride}")
    ea, da = ctx.chunk(dev(a), 20, stride, 0xFFF, 0, 2048)
    eb, db = ctx.chunk(dev(b), 20, stride, 0xFFF, 0, 2048)
    lb = torch.diff(eb, prepend=torch.zeros(1, dtype=torch.int64, device="cuda"))
    m, mb = ctx.similarity(da, db, lb, 1)
    xa, xda = _oracle_chunks(a, 20, stride, 0xFFF, 0, 2048)
    xb, xdb = _oracle_chunks(b, 20, stride, 0xFFF, 0, 2048)
    assert np.array_equal(host(ea).astype(np.uint64), xa)
    assert np.array_equal(host(eb).astype(np.uint64), xb)
    assert np.array_equal(host(db), xdb)
    xlb = np.diff(xb, prepend=np.uint64(0))
    assert (m, mb) == oracle.similarity(1, xda, xdb, xlb)
    # Chunk sizes taken from the end offsets inside the kernel.
    assert ctx.similarity(da, db, ends_b=eb) == (m, mb)


# ------------------------------------------------------ full-size checks --
@pytest.mark.parametrize("block", [4096, 64 * 1024, 1 << 20])
def test_block_hash_large_workload(ctx, block):
    data = _large()
    d = _large_dev()
    for kind in KINDS:
        note(f"block_hash 1GiB kind={kind} B={block}")
        lv, rt = ctx.block_hash(d, block, kind)
        torch.cuda.synchronize()
        exp_lv = oracle.leaves_sharded(kind, data, block, THREADS)
        assert np.array_equal(host(lv), exp_lv)
        assert bytes(host(rt)) == oracle.root(kind, exp_lv)
        _LARGE[(kind, block)] = (exp_lv, oracle.root(kind, exp_lv))
    # Fused: both digests in one pass equal the oracle's.
    note(f"block_hash_dual 1GiB B={block}")
    lm, rm, ls, rs = ctx.block_hash_dual(d, block)
    torch.cuda.synchronize()
    for kind, lv, rt in ((oracle.MD5, lm, rm), (oracle.SHA1, ls, rs)):
        exp_lv, exp_rt = _LARGE[(kind, block)]
        assert np.array_equal(host(lv), exp_lv)
        assert bytes(host(rt)) == exp_rt
    del lm, rm, ls, rs
    # Host input: the 1 GiB streamed from pinned and from pageable memory
    # (pieces copied while earlier pieces hash), each digest and both at once.
    if "pinned" not in _LARGE:
        _LARGE["pinned"] = torch.from_numpy(data).pin_memory()
    for where, src in (("pinned", _LARGE["pinned"]), ("pageable", torch.from_numpy(data))):
        for kind in KINDS:
            note(f"block_hash 1GiB host input {where} kind={kind} B={block}")
            lv, rt = ctx.block_hash(src, block, kind)
            torch.cuda.synchronize()
            exp_lv, exp_rt = _LARGE[(kind, block)]
            assert np.array_equal(host(lv), exp_lv)
            assert bytes(host(rt)) == exp_rt
        note(f"block_hash_dual 1GiB host input {where} B={block}")
        lm, rm, ls, rs = ctx.block_hash_dual(src, block)
        torch.cuda.synchronize()
        for kind, lv, rt in ((oracle.MD5, lm, rm), (oracle.SHA1, ls, rs)):
            exp_lv, exp_rt = _LARGE[(kind, block)]
            assert np.array_equal(host(lv), exp_lv)
            assert bytes(host(rt)) == exp_rt
    for kind in KINDS:
        _LARGE.pop((kind, block))


_LARGE = {}


def _large():
    if "h" not in _LARGE:
        _LARGE["h"] = inputs.uniform_bytes(2, 1 << 30)
    return _LARGE["h"]


def _large_dev():
    if "d" not in _LARGE:
        _LARGE["d"] = torch.from_numpy(_large()).cuda()
    return _LARGE["d"]


@pytest.mark.parametrize("stride", [1, 4])
def test_similarity_workload_full_size(ctx, stride):
    _LARGE.clear()
    a, b = _versions(256 * MiB, 256)
    note(f"similarity 256MiB s={stride}")
    ea, da = ctx.chunk(dev(a), 20, stride, 0xFFF, 0, 2048)
    eb, db = ctx.chunk(dev(b), 20, stride, 0xFFF, 0, 2048)
    lb = torch.diff(eb, prepend=torch.zeros(1, dtype=torch.int64, device="cuda"))
    m, mb = ctx.similarity(da, db, lb, 1)
    xa, xda = _oracle_chunks(a, 20, stride, 0xFFF, 0, 2048)
    xb, xdb = _oracle_chunks(b, 20, stride, 0xFFF, 0, 2048)
    assert np.array_equal(host(ea).astype(np.uint64), xa)
    assert np.array_equal(host(da), xda)
    assert np.array_equal(host(eb).astype(np.uint64), xb)
    assert np.array_equal(host(db), xdb)
    xlb = np.diff(xb, prepend=np.uint64(0))
    assert (m, mb) == oracle.similarity(1, xda, xdb, xlb)
    note(f"similarity s={stride}: {m}/{xb.size} chunks, {mb}/{b.size} bytes")


# ------------------------------------------------------- misc behaviour --
def test_results_are_deterministic(ctx):
    data = inputs.uniform_bytes(600, 3 * MiB + 5)
    d = dev(data, 1)
    note("determinism")
    r1 = [host(x) for x in ctx.chunk(d, 20, 1, 0x3FF, 0, 1024)]
    r2 = [host(x) for x in ctx.chunk(d, 20, 1, 0x3FF, 0, 1024)]
    assert all(np.array_equal(x, y) for x, y in zip(r1, r2))


def test_invalid_arguments(ctx, hg):
    d = dev(inputs.uniform_bytes(601, 1000))
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    fl = hg.HG_IN_DEVICE | hg.HG_OUT_DEVICE
    note("invalid arguments")
    assert hg.hg_block_hash(ctx.handle, d.data_ptr(), 1000, 0, 0, cnt.data_ptr(), None, fl, s) == hg.HG_EINVAL
    assert hg.hg_block_hash(ctx.handle, d.data_ptr(), 1000, 64, 9, cnt.data_ptr(), None, fl, s) == hg.HG_EINVAL
    assert hg.hg_block_hash(ctx.handle, d.data_ptr(), 1000, 64, 0, None, None, fl, s) == hg.HG_EINVAL
    for w, st_ in [(0, 1), (hg.HG_MAX_WINDOW + 1, 1), (20, 0)]:
        assert hg.hg_window_scan(ctx.handle, d.data_ptr(), 1000, w, st_, 0, 0, 0, None, 0,
                                 cnt.data_ptr(), fl, s) == hg.HG_EINVAL
    assert hg.hg_window_scan(ctx.handle, d.data_ptr(), 1000, 20, 1, 0, 0, 0, None, 0, None, fl,
                             s) == hg.HG_EINVAL
    assert hg.hg_window_scan(ctx.handle, d.data_ptr(), 1000, 20, 1, 0, 0, 0, None, 0,
                             cnt.data_ptr(), hg.HG_ASYNC, s) == hg.HG_EINVAL
    p = hg.hg_chunk_params(20, 1, 0, 0, 100, 50, 0, 1)  # max_chunk below min_chunk
    assert hg.hg_chunk(ctx.handle, d.data_ptr(), 1000, ctypes.byref(p), None, 0, cnt.data_ptr(),
                       None, fl, s) == hg.HG_EINVAL
    buf = ctypes.create_string_buffer(256)
    assert hg.hg_last_error(ctx.handle, buf, 256) == hg.HG_EINVAL
    assert b"max_chunk" in buf.value
    h = ctypes.c_void_p()
    assert hg.hg_create(99, 0, 0, ctypes.byref(h)) == hg.HG_EDEVICE


# ---------------------------------------------------------------- batches --
def test_block_hash_batch_mixed_jobs(ctx, hg):
    rng = np.random.default_rng(700)
    specs, arrays = [], []
    for i in range(40):
        length = int(rng.choice([0, 1, 63, 64, 100, 5000, 70_000, 300_001, 2 * MiB + 7]))
        block = int(rng.choice([1, 64, 100, 4096, 65536, 1 << 20]))
        if length > 20_000 and block == 1:
            block = 64
        kind = int(rng.integers(0, 2))
        data = inputs.uniform_bytes(710 + i, length)
        arrays.append((data, block, kind))
        specs.append((dev(data, int(rng.integers(0, 4))), block, kind))
    note("block_hash_batch 40 mixed jobs")
    leaves, roots = ctx.block_hash_batch(specs)
    torch.cuda.synchronize()
    for (data, block, kind), lv, rt in zip(arrays, leaves, roots):
        exp = oracle.leaves(kind, data, block)
        assert np.array_equal(host(lv), exp), (data.size, block, kind)
        assert bytes(host(rt)) == oracle.root(kind, exp)


def test_leaves_and_roots_batches_from_device_table(ctx, hg):
    data = inputs.uniform_bytes(720, 8 * MiB + 3)
    d = dev(data)
    specs = [(d, 1 << 20, 1), (d, 1 << 20, 0), (d, 4096, 1), (d, 4096, 0), (d, 65536, 1),
             (d, 65536, 0)]
    recs, leaves, roots = ctx.batch_outputs(specs)
    table = ctx.device_job_table(recs)
    note("leaves/roots batch, device table, async")
    s = torch.cuda.current_stream()
    ctx.run_batch(table, len(specs), "leaves", stream=s)
    ctx.run_batch(table, len(specs), "roots", stream=s)
    torch.cuda.synchronize()
    for (_, block, kind), lv, rt in zip(specs, leaves, roots):
        exp = oracle.leaves(kind, data, block)
        assert np.array_equal(host(lv), exp)
        assert bytes(host(rt)) == oracle.root(kind, exp)


def test_leaves_batch_odd_block_counts(ctx, hg):
    # Segments of odd and even numbers of 64-byte blocks, with and without a
    # partial last block, in one launch: lanes of a wavefront leave the
    # two-block loop with 0, 1 or more full blocks left, at different times.
    data = inputs.uniform_bytes(722, 3 * MiB + 777)
    d = dev(data, 5)
    blocks = [192, 320, 448, 4160, 8256, 65600, 200, 130, 65535, 129 * 64 + 1]
    specs = [(d, b, k) for b in blocks for k in (0, 1)]
    recs, leaves, _ = ctx.batch_outputs(specs, roots=False)
    table = ctx.device_job_table(recs)
    note("leaves batch, odd block counts")
    ctx.run_batch(table, len(specs), "leaves", asynchronous=False)
    for (_, block, kind), lv in zip(specs, leaves):
        assert np.array_equal(host(lv), oracle.leaves(kind, data, block)), (block, kind)


def test_job_table_keeps_its_tensors(ctx, hg):
    # Job records hold raw pointers: the records and a device table made
    # from them keep the tensors they point at alive, so that dropping the
    # caller's references cannot let a later allocation take their memory
    # while the batch writes to it.
    data = inputs.uniform_bytes(723, 2 * MiB + 11)
    d = dev(data)
    specs = [(d, 4096, 0), (d, 65536, 1)]
    recs, leaves, _ = ctx.batch_outputs(specs, roots=False)
    ptrs = [lv.data_ptr() for lv in leaves]
    del leaves
    table = ctx.device_job_table(recs)
    del recs
    junk = [torch.zeros(n, dtype=torch.uint8, device="cuda") for n in (512, 40960, 196608, 655360)]
    note("leaves batch from a table whose records' outputs the caller dropped")
    ctx.run_batch(table, len(specs), "leaves", asynchronous=False)
    kept = table._hg_keep._hg_keep[0]
    assert [lv.data_ptr() for lv in kept] == ptrs
    for (_, block, kind), lv in zip(specs, kept):
        assert np.array_equal(host(lv), oracle.leaves(kind, data, block)), (block, kind)
    assert all(int(j.sum()) == 0 for j in junk)


# ------------------------------------------------------------------ probes --
def test_probes_report_plausible_ceilings(ctx, hg):
    note("ALU and HBM probes")
    tops = ctx.probe_alu()
    assert 1.0 < tops < 60.0, tops  # data sheet: 39.32 Tops/s int32
    buf = torch.zeros(256 * MiB, dtype=torch.uint8, device="cuda")
    gbps = ctx.probe_read(buf)
    assert 100.0 < gbps < 12000.0, gbps  # data sheet: 8 TB/s
    v = ctypes.c_double(0.0)
    assert hg.hg_probe_read(ctx.handle, None, 0, ctypes.byref(v), None) == hg.HG_EINVAL
