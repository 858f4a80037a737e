"""GPU tests of the streaming chunker (hg_chunker_*): a stream fed in pieces
-- random sizes, pieces shorter than a window, empty pieces, pieces that end
on a cut, host and device memory -- gives exactly the chunks of the oracle's
one-shot chunking of the whole stream (bit-exact ends and digests), for
several window/stride/minimum/maximum settings.  Inputs: seeded uniform
bytes, and bytes with long runs of zeros (no candidates for long stretches,
so the carry grows and forced cuts happen)."""
import hashlib
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1202_3669_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
THREADS = max(1, min(16, os.cpu_count() or 1))
KiB, MiB = 1 << 10, 1 << 20


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


def one_shot(data, w, s, mask, target, mn, mx, seg=0):
    starts = oracle.window_scan_sharded(oracle.MD5, data, w, s, mask, target, THREADS)
    ends = oracle.chunk_select(starts, w, data.size, mn, mx)
    return ends, oracle.chunk_digests(oracle.SHA1, data, ends, seg)


def pieces(rng, n, cuts=()):
    """Random split points of [0, n), including empty and tiny pieces and the
    given offsets."""
    pts = set(int(x) for x in rng.integers(0, n + 1, size=int(rng.integers(1, 12))))
    pts |= {int(c) for c in cuts if 0 <= c <= n}
    pts |= {min(n, 5), min(n, 5)}  # an early tiny piece and an empty one
    pts = sorted(pts | {0, n})
    out = [(a, b) for a, b in zip(pts[:-1], pts[1:])] or [(0, 0)]
    out.insert(min(2, len(out)), (0, 0))  # an empty piece
    return out


CASES = [  # (length, w, s, mask, target, min, max)
    (3 * MiB + 11, 20, 1, 0xFFF, 0, 2048, 0),
    (1 * MiB + 5, 20, 1, 0xFF, 0, 0, 0),        # min below w: windows straddling a cut matter
    (1 * MiB + 7, 48, 4, 0x1FF, 3, 100, 0),     # stride 4 on the absolute grid
    (2 * MiB + 1, 20, 1, 0xFFF, 0, 2048, 8192),
    (1 * MiB, 33, 3, 0x3F, 1, 10, 50),          # dense candidates, tight maximum
    (0, 20, 1, 0xFFF, 0, 2048, 0),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("device_input", [True, False])
def test_stream_equals_one_shot(ctx, hg, case, device_input):
    length, w, s, mask, target, mn, mx = case
    data = inputs.uniform_bytes(500 + length % 89, length)
    exp_ends, exp_dig = one_shot(data, w, s, mask, target, mn, mx)
    rng = np.random.default_rng(501 + length % 13)
    # include split points exactly at some cuts and just after them
    cuts = exp_ends[:: max(1, exp_ends.size // 5)].tolist()
    splits = pieces(rng, length, cuts + [c + 1 for c in cuts])
    note(f"stream case={case} device={device_input} pieces={len(splits)}")
    ch = hg.Chunker(ctx, w, s, mask, target, mn, mx)
    dev = torch.from_numpy(data).cuda() if device_input else None
    got_e, got_d = [], []
    for a, b in splits:
        piece = dev[a:b] if device_input else data[a:b]
        e, d = ch.feed(piece)
        got_e.append(e)
        got_d.append(d)
    e, d = ch.finish()
    got_e.append(e)
    got_d.append(d)
    ends = np.concatenate(got_e)
    dig = np.concatenate(got_d).reshape(-1, 20)
    assert np.array_equal(ends, exp_ends)
    assert np.array_equal(dig, exp_dig)
    # reuse after reset: one piece
    ch.reset()
    e1, d1 = ch.feed(data)
    e2, d2 = ch.finish()
    assert np.array_equal(np.concatenate([e1, e2]), exp_ends)
    ch.close()


def test_stream_long_runs_without_candidates(ctx, hg):
    # Zero runs: with a target that the all-zero window does not hit, no
    # candidates for 3 MiB stretches; without a maximum the carry grows to
    # the whole run, with one the cuts are forced.
    zeros = np.zeros(64, dtype=np.uint8)
    hit = {int(x) for x in range(4096) if oracle.window_scan(oracle.MD5, zeros, 20, 1, 0xFFF, x).size}
    target = next(t for t in range(4096) if t not in hit)
    rnd = inputs.uniform_bytes(510, 2 * MiB)
    data = np.concatenate([rnd[:MiB], np.zeros(3 * MiB, np.uint8), rnd[MiB:]])
    for mx in (0, 65536):
        exp_ends, exp_dig = one_shot(data, 20, 1, 0xFFF, target, 2048, mx)
        ch = hg.Chunker(ctx, 20, 1, 0xFFF, target, 2048, mx)
        note(f"zero runs max={mx}")
        out_e, out_d = [], []
        for a in range(0, data.size, 700_001):
            e, d = ch.feed(data[a:a + 700_001])
            out_e.append(e)
            out_d.append(d)
        e, d = ch.finish()
        out_e.append(e)
        out_d.append(d)
        assert np.array_equal(np.concatenate(out_e), exp_ends)
        assert np.array_equal(np.concatenate(out_d).reshape(-1, 20), exp_dig)
        ch.close()


@pytest.mark.parametrize("device_input", [True, False])
def test_stream_two_level_digests(ctx, hg, device_input):
    data = inputs.uniform_bytes(515, 3 * MiB + 9)
    for mx, seg in ((0, 4096), (65536, 1000)):
        exp_ends, exp_dig = one_shot(data, 20, 1, 0xFFF, 0, 2048, mx, seg)
        ch = hg.Chunker(ctx, 20, 1, 0xFFF, 0, 2048, mx, chunk_segment=seg)
        note(f"stream two-level max={mx} segment={seg} device={device_input}")
        src = torch.from_numpy(data).cuda() if device_input else data
        out_e, out_d = [], []
        for a in range(0, data.size, 500_001):
            e, d = ch.feed(src[a:a + 500_001])
            out_e.append(e)
            out_d.append(d)
        e, d = ch.finish()
        out_e.append(e)
        out_d.append(d)
        ch.close()
        assert np.array_equal(np.concatenate(out_e), exp_ends)
        assert np.array_equal(np.concatenate(out_d).reshape(-1, 20), exp_dig)


def test_stream_rejects_small_capacity_and_use_after_finish(ctx, hg):
    import ctypes
    ch = hg.Chunker(ctx)
    data = inputs.uniform_bytes(520, 100_000)
    ends = np.zeros(4, dtype=np.uint64)
    n = ctypes.c_uint64(0)
    assert hg.hg_chunker_feed(ch.handle, data.ctypes.data, data.size, 0, ends.ctypes.data, 4,
                              ctypes.byref(n), None, None) == hg.HG_EINVAL
    ch.feed(data)
    ch.finish()
    with pytest.raises(hg.HashGpuError):
        ch.feed(data)
    ch.close()


ASYNC_CASES = [  # (length, w, s, mask, target, min, max, segment)
    (3 * MiB + 11, 20, 1, 0xFFF, 0, 2048, 0, 0),
    (1 * MiB + 5, 20, 1, 0xFF, 0, 0, 0, 0),
    (2 * MiB + 1, 20, 1, 0xFFF, 0, 2048, 8192, 0),
    (2 * MiB + 3, 20, 1, 0xFFF, 0, 2048, 0, 4096),
]


@pytest.mark.parametrize("case", ASYNC_CASES)
@pytest.mark.parametrize("where", ["device", "device_ready", "pinned", "pageable", "torch_pinned"])
def test_stream_async_feeds(ctx, hg, case, where):
    # HG_ASYNC: every feed returns once its cuts are decided, its digests
    # still running; host input comes through ONE staging array that is
    # overwritten with the next piece as soon as a feed returns.
    length, w, s, mask, target, mn, mx, seg = case
    data = inputs.uniform_bytes(530 + length % 71, length)
    exp_ends, exp_dig = one_shot(data, w, s, mask, target, mn, mx, seg)
    rng = np.random.default_rng(531 + length % 17)
    cuts = exp_ends[:: max(1, exp_ends.size // 5)].tolist()
    splits = pieces(rng, length, cuts + [c + 1 for c in cuts])
    note(f"async stream case={case} input={where} pieces={len(splits)}")
    big = max(b - a for a, b in splits)
    if where in ("pinned", "torch_pinned"):
        stage_t = torch.empty(max(big, 1), dtype=torch.uint8, pin_memory=True)
        stage = stage_t.numpy()
    else:
        stage = np.empty(max(big, 1), dtype=np.uint8)
    dev = torch.from_numpy(data).cuda() if where.startswith("device") else None
    ch = hg.Chunker(ctx, w, s, mask, target, mn, mx, chunk_segment=seg)
    outs = []
    for a, b in splits:
        if where.startswith("device"):
            piece = dev[a:b]
        else:
            stage[:b - a] = data[a:b]
            piece = stage_t[:b - a] if where == "torch_pinned" else stage[:b - a]  # CPU tensor or array
        # device_ready: HG_IN_READY, the feed reads its input without waiting
        # for the previous feed's digests on the stream
        outs.append(ch.feed(piece, asynchronous=True, ready=where == "device_ready"))
        if not where.startswith("device"):
            stage[:] = 0xA5  # the call has read its input
    outs.append(ch.finish(asynchronous=True))
    torch.cuda.synchronize()
    got_e = [e[:int(c.item())].cpu().numpy().astype(np.uint64) for e, _, c in outs]
    got_d = [d[:int(c.item())].cpu().numpy() for _, d, c in outs]
    ch.close()
    assert np.array_equal(np.concatenate(got_e), exp_ends)
    assert np.array_equal(np.concatenate(got_d).reshape(-1, 20), exp_dig)


@pytest.mark.parametrize("mode", ["sync", "async", "async_ready"])
def test_stream_large_device_feeds_produced_on_the_stream(ctx, hg, mode):
    # Device feeds of 20-27 MiB (several window-tile launch ranges' worth),
    # each produced on the stream just before the feed: without HG_IN_READY
    # the feed's copy must wait for that work.
    length = 56 * MiB + 13
    data = inputs.uniform_bytes(560, length)
    exp_ends, exp_dig = one_shot(data, 20, 1, 0xFFF, 0, 2048, 0)
    splits = [(0, 20 * MiB + 3), (20 * MiB + 3, 20 * MiB + 3), (20 * MiB + 3, 47 * MiB + 1), (47 * MiB + 1, length)]
    note(f"device feeds of up to {27 * MiB} bytes, mode={mode}")
    src = torch.from_numpy(data).cuda()
    ch = hg.Chunker(ctx, 20, 1, 0xFFF, 0, 2048, 0)
    got_e, got_d, outs, keep = [], [], [], []
    for a, b in splits:
        piece = torch.empty(b - a, dtype=torch.uint8, device="cuda")
        piece.copy_(src[a:b], non_blocking=True)  # produced on the stream the feed runs on
        keep.append(piece)
        if mode == "async_ready":
            torch.cuda.synchronize()  # HG_IN_READY: the input is complete when the feed is made
        if mode == "sync":
            e, d = ch.feed(piece)
            got_e.append(e)
            got_d.append(d)
        else:
            outs.append(ch.feed(piece, asynchronous=True, ready=mode == "async_ready"))
    if mode == "sync":
        e, d = ch.finish()
        got_e.append(e)
        got_d.append(d)
    else:
        outs.append(ch.finish(asynchronous=True))
        torch.cuda.synchronize()
        got_e = [e[:int(c.item())].cpu().numpy().astype(np.uint64) for e, _, c in outs]
        got_d = [d[:int(c.item())].cpu().numpy() for _, d, c in outs]
    ch.close()
    assert np.array_equal(np.concatenate(got_e), exp_ends)
    assert np.array_equal(np.concatenate(got_d).reshape(-1, 20), exp_dig)


def test_stream_async_needs_device_outputs(ctx, hg):
    import ctypes
    ch = hg.Chunker(ctx)
    data = inputs.uniform_bytes(540, 10_000)
    ends = np.zeros(64, dtype=np.uint64)
    n = ctypes.c_uint64(0)
    note("async feed with host outputs")
    assert hg.hg_chunker_feed(ch.handle, data.ctypes.data, data.size, hg.HG_ASYNC, ends.ctypes.data, 64,
                              ctypes.byref(n), None, None) == hg.HG_EINVAL
    e, d = ch.feed(data)  # the rejected call left the stream untouched
    e2, d2 = ch.finish()
    exp_ends, exp_dig = one_shot(data, 20, 1, 0xFFF, 0, 2048, 0)
    assert np.array_equal(np.concatenate([e, e2]), exp_ends)
    ch.close()


def test_stream_async_reset_with_digests_pending(ctx, hg):
    # Two streams through one chunker, the second started by reset() while
    # the first one's last digests may still run, with host-count feeds
    # (HG_COUNT_HOST) in the second: both outputs equal the one-shot result.
    import ctypes
    data = inputs.uniform_bytes(550, 3 * MiB + 17)
    exp_ends, exp_dig = one_shot(data, 20, 1, 0xFFF, 0, 2048, 0)
    note("async feeds across a reset")
    ch = hg.Chunker(ctx)
    first = [ch.feed(data[a:a + MiB], asynchronous=True) for a in range(0, data.size, MiB)]
    first.append(ch.finish(asynchronous=True))
    ch.reset()
    outs = []
    for a in range(0, data.size + 1, 777_777):
        piece = data[a:a + 777_777]
        b = ctypes.c_uint64(0)
        assert hg.hg_chunker_bound(ch.handle, piece.size, ctypes.byref(b)) == hg.HG_OK
        ends = torch.empty(int(b.value), dtype=torch.int64, device="cuda")
        dig = torch.empty((int(b.value), 20), dtype=torch.uint8, device="cuda")
        n = ctypes.c_uint64(0)
        st = hg.hg_chunker_feed(ch.handle, piece.ctypes.data if piece.size else None, piece.size,
                                hg.HG_OUT_DEVICE | hg.HG_ASYNC | hg.HG_COUNT_HOST, ends.data_ptr(), int(b.value),
                                ctypes.byref(n), dig.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert st == hg.HG_OK
        outs.append((ends, dig, int(n.value)))  # the host count is final when the call returns
    e, d, c = ch.finish(asynchronous=True)
    torch.cuda.synchronize()
    outs.append((e, d, int(c.item())))
    ch.close()
    got1_e = np.concatenate([e[:int(c.item())].cpu().numpy().astype(np.uint64) for e, _, c in first])
    got1_d = np.concatenate([d[:int(c.item())].cpu().numpy() for _, d, c in first])
    assert np.array_equal(got1_e, exp_ends) and np.array_equal(got1_d, exp_dig)
    got2_e = np.concatenate([e[:k].cpu().numpy().astype(np.uint64) for e, _, k in outs])
    got2_d = np.concatenate([d[:k].cpu().numpy() for _, d, k in outs])
    assert np.array_equal(got2_e, exp_ends) and np.array_equal(got2_d, exp_dig)


def _candidate_window(seed):
    # a 20-byte window whose MD5 has its low 12 bits (first word, little
    # endian) zero: the boundary predicate holds for it
    rng = np.random.default_rng(seed)
    while True:
        w = rng.integers(0, 256, 20, dtype=np.uint8).tobytes()
        d = hashlib.md5(w).digest()
        if int.from_bytes(d[:4], "little") & 0xFFF == 0:
            return np.frombuffer(w, dtype=np.uint8)


@pytest.mark.parametrize("where", ["device", "pinned"])
def test_stream_dense_candidates_redo(ctx, hg, where):
    # A candidate window repeated: every 20th window is a candidate, far
    # more than the room a feed sets aside for a 12-bit mask on random
    # bytes, so each feed redoes its decision with exact room.  The stream
    # still equals the one-shot result.
    w0 = _candidate_window(560)
    data = np.tile(w0, (3 * MiB) // 20 + 1)[:3 * MiB + 7].copy()
    data[-7:] = 1
    exp_ends, exp_dig = one_shot(data, 20, 1, 0xFFF, 0, 2048, 0)
    assert exp_ends.size > 1000
    note(f"dense candidates, {where} input")
    src = torch.from_numpy(data).cuda() if where == "device" else torch.from_numpy(data).pin_memory()
    ch = hg.Chunker(ctx)
    outs = []
    for a in range(0, data.size, MiB):
        piece = src[a:a + MiB] if where == "device" else src[a:a + MiB].numpy()
        outs.append(ch.feed(piece, asynchronous=True))
    outs.append(ch.finish(asynchronous=True))
    torch.cuda.synchronize()
    got_e = np.concatenate([e[:int(c.item())].cpu().numpy().astype(np.uint64) for e, _, c in outs])
    got_d = np.concatenate([d[:int(c.item())].cpu().numpy() for _, d, c in outs])
    ch.close()
    assert np.array_equal(got_e, exp_ends)
    assert np.array_equal(got_d, exp_dig)


def _candidate_window_w(seed, w):
    # a w-byte window whose MD5 has its low 12 bits (first word, little
    # endian) zero
    rng = np.random.default_rng(seed)
    while True:
        x = rng.integers(0, 256, w, dtype=np.uint8).tobytes()
        if int.from_bytes(hashlib.md5(x).digest()[:4], "little") & 0xFFF == 0:
            return np.frombuffer(x, dtype=np.uint8)


SPLIT_CASES = {  # name: (w, s, mask, target, min, max)
    # a candidate window tiled: every 11th window of the stride-3 grid is a
    # candidate, far above the room set aside for a 12-bit mask (redo)
    "dense_w33_s3": (33, 3, 0xFFF, 0, 2048, 0),
    # minimum below the window: the boundary decision walks
    "min_below_w_s3": (33, 3, 0x3F, 1, 10, 0),
    "max_chunk": (20, 1, 0xFFF, 0, 2048, 8192),
}


@pytest.mark.parametrize("ready", [False, True])
@pytest.mark.parametrize("case", sorted(SPLIT_CASES))
def test_stream_large_device_feeds_stride_dense_max(ctx, hg, case, ready):
    # Device pieces of 16 MiB and more (several window-tile launch ranges),
    # with a carry into the second large piece and none into the first,
    # around a tiny and an empty piece, at stride 3 with a 33-byte window,
    # with dense candidates, a minimum below the window and a maximum; the
    # pieces produced on the stream or declared ready: the stream equals the
    # one-shot result.
    w, s, mask, target, mn, mx = SPLIT_CASES[case]
    length = 40 * MiB + 11
    if case == "dense_w33_s3":
        w0 = _candidate_window_w(570, 33)
        data = np.tile(w0, length // 33 + 1)[:length].copy()
        data[-11:] = 1
    else:
        data = inputs.uniform_bytes(571, length)
    exp_ends, exp_dig = one_shot(data, w, s, mask, target, mn, mx)
    cuts = [0, 16 * MiB, 16 * MiB + 3, 16 * MiB + 3, 33 * MiB + 1, length]
    note(f"large device feeds: {case}, ready={ready}")
    src = torch.from_numpy(data).cuda()
    ch = hg.Chunker(ctx, w, s, mask, target, mn, mx)
    outs, keep = [], []
    for a, b in zip(cuts[:-1], cuts[1:]):
        piece = torch.empty(b - a, dtype=torch.uint8, device="cuda")
        piece.copy_(src[a:b], non_blocking=True)
        keep.append(piece)
        if ready:
            torch.cuda.synchronize()
        outs.append(ch.feed(piece, asynchronous=True, ready=ready))
    outs.append(ch.finish(asynchronous=True))
    torch.cuda.synchronize()
    got_e = np.concatenate([e[:int(c.item())].cpu().numpy().astype(np.uint64) for e, _, c in outs])
    got_d = np.concatenate([d[:int(c.item())].cpu().numpy() for _, d, c in outs])
    ch.close()
    assert got_e.size > 1000
    assert np.array_equal(got_e, exp_ends)
    assert np.array_equal(got_d.reshape(-1, 20), exp_dig)
