"""GPU parity of the chunking stages as separate calls (hg_window_scan with
HG_ASYNC, hg_chunk_select, hg_chunk_digests, hg_similarity_n): a pipeline
with every count left on the device gives the oracle's candidates, chunk
ends, digests and similarity exactly, and the same as hg_chunk.  Also: the
host-memory forms of each call, an incomplete candidate list (UINT64_MAX
count, HG_ETRUNC when waiting), counts above the room given, ends past the
buffer, and argument errors."""
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


CASES = [  # (length, w, s, mask, target, min, max, segment)
    (3 * MiB + 5, 20, 1, 0xFFF, 0, 2048, 0, 0),
    (2 * MiB + 7, 20, 1, 0xFFF, 0, 2048, 8192, 0),
    (1 * MiB + 3, 20, 4, 0x3FF, 1, 100, 0, 4096),
    (1 * MiB, 48, 1, 0xFF, 0, 10, 0, 0),            # min below the window
    (777_777, 33, 3, 0x1FF, 2, 0, 3000, 1000),
    (100, 20, 1, 0xF, 0, 10, 0, 0),
    (0, 20, 1, 0xFFF, 0, 2048, 0, 0),
]


@pytest.mark.parametrize("case", CASES)
def test_device_pipeline_equals_oracle_and_hg_chunk(ctx, hg, case):
    length, w, s, mask, target, mn, mx, seg = case
    data = inputs.uniform_bytes(600 + length % 97, length)
    prev, _ = inputs.edited_version(data, 601, 8, 100, 400) if length > 10_000 else (data, None)
    exp_starts = oracle.window_scan_sharded(oracle.MD5, data, w, s, mask, target, THREADS)
    exp_ends = oracle.chunk_select(exp_starts, w, length, mn, mx)
    exp_dig = oracle.chunk_digests(oracle.SHA1, data, exp_ends, seg)
    p_starts = oracle.window_scan_sharded(oracle.MD5, prev, w, s, mask, target, THREADS)
    p_ends = oracle.chunk_select(p_starts, w, prev.size, mn, mx)
    p_dig = oracle.chunk_digests(oracle.SHA1, prev, p_ends, seg)
    exp_sim = oracle.similarity(oracle.SHA1, p_dig, exp_dig, np.diff(exp_ends, prepend=np.uint64(0)))
    note(f"stages case={case}")
    d = torch.from_numpy(data).cuda()
    cap = exp_starts.size + 5
    starts = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ctx.window_scan(d, w, s, mask, target, out=(starts, cnt), stream=st)
        ends, n = ctx.chunk_select(starts, cnt, length, w, mn, mx, asynchronous=True, stream=st)
        dig = ctx.chunk_digests(d, ends, n, chunk_segment=seg, asynchronous=True, stream=st)
        res = torch.zeros(2, dtype=torch.int64, device="cuda")
        ctx.similarity_n(torch.from_numpy(p_dig).cuda(), dig, n, ends_b=ends, out=res, asynchronous=True, stream=st)
    st.synchronize()
    k = int(n.item())
    assert int(cnt.item()) == exp_starts.size
    assert np.array_equal(starts[:exp_starts.size].cpu().numpy().astype(np.uint64), exp_starts)
    assert k == exp_ends.size
    assert np.array_equal(ends[:k].cpu().numpy().astype(np.uint64), exp_ends)
    assert np.array_equal(dig[:k].cpu().numpy(), exp_dig)
    assert tuple(res.cpu().tolist()) == exp_sim
    # and the one-call path agrees
    e2, d2 = ctx.chunk(d, w, s, mask, target, mn, max_chunk=mx, chunk_segment=seg)
    assert np.array_equal(e2.cpu().numpy().astype(np.uint64), exp_ends)
    assert np.array_equal(d2.cpu().numpy(), exp_dig)


def test_incomplete_candidate_list(ctx, hg):
    data = inputs.uniform_bytes(610, 2 * MiB)
    exp_starts = oracle.window_scan_sharded(oracle.MD5, data, 20, 1, 0xFF, 0, THREADS)
    assert exp_starts.size > 100
    d = torch.from_numpy(data).cuda()
    starts = torch.empty(100, dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    note("incomplete candidate list")
    ctx.window_scan(d, 20, 1, 0xFF, 0, out=(starts, cnt))
    torch.cuda.synchronize()
    assert int(cnt.item()) == exp_starts.size
    assert np.array_equal(starts.cpu().numpy().astype(np.uint64), exp_starts[:100])
    ends, n = ctx.chunk_select(starts, cnt, data.size, 20, 1024, asynchronous=True)
    torch.cuda.synchronize()
    assert int(n.item()) == -1  # UINT64_MAX
    with pytest.raises(hg.HashGpuError) as e:
        ctx.chunk_select(starts, cnt, data.size, 20, 1024)
    assert e.value.status == hg.HG_ETRUNC
    # exactly at the room: complete
    cnt100 = torch.tensor([100], dtype=torch.int64, device="cuda")
    ends, n = ctx.chunk_select(starts, cnt100, data.size, 20, 1024)
    assert np.array_equal(ends.cpu().numpy().astype(np.uint64),
                          oracle.chunk_select(exp_starts[:100], 20, data.size, 1024))


def test_host_memory_forms(ctx, hg):
    data = inputs.uniform_bytes(620, 1 * MiB + 11)
    starts = oracle.window_scan(oracle.MD5, data, 20, 1, 0xFFF, 0)
    exp_ends = oracle.chunk_select(starts, 20, data.size, 2048, 65536)
    note("host forms of the stages")
    cap = starts.size + 2 + data.size // 65536
    ends = np.zeros(cap, dtype=np.uint64)
    n = ctypes.c_uint64(0)
    ns = ctypes.c_uint64(starts.size)
    st = hg.hg_chunk_select(ctx.handle, starts.ctypes.data, ctypes.byref(ns), starts.size, data.size, 20, 2048,
                            65536, ends.ctypes.data, cap, ctypes.byref(n), 0, None)
    assert st == hg.HG_OK
    assert np.array_equal(ends[:n.value], exp_ends)
    for seg in (0, 512):
        dig = np.zeros((exp_ends.size, 20), dtype=np.uint8)
        nn = ctypes.c_uint64(exp_ends.size)
        st = hg.hg_chunk_digests(ctx.handle, data.ctypes.data, data.size, exp_ends.ctypes.data, ctypes.byref(nn),
                                 exp_ends.size, hg.HG_SHA1, seg, dig.ctypes.data, 0, None)
        assert st == hg.HG_OK
        assert np.array_equal(dig, oracle.chunk_digests(oracle.SHA1, data, exp_ends, seg))
    # similarity with a host count below the room
    dig = oracle.chunk_digests(oracle.SHA1, data, exp_ends)
    m, mb = ctypes.c_uint64(0), ctypes.c_uint64(0)
    nb = ctypes.c_uint64(5)
    st = hg.hg_similarity_n(ctx.handle, dig.ctypes.data, dig.shape[0], dig.ctypes.data, exp_ends.ctypes.data,
                            ctypes.byref(nb), dig.shape[0], hg.HG_SHA1, ctypes.byref(m), ctypes.byref(mb),
                            hg.HG_LEN_ENDS, None)
    assert st == hg.HG_OK
    lens = np.diff(exp_ends[:5], prepend=np.uint64(0))
    assert (m.value, mb.value) == oracle.similarity(oracle.SHA1, dig, dig[:5], lens)


def test_digest_counts_and_ends_are_clamped(ctx, hg):
    data = inputs.uniform_bytes(630, 300_000)
    ends = np.array([1000, 5000, 4000, 400_000, 299_999, 1 << 62], dtype=np.uint64)  # decreasing, past len
    note("chunk digests of clamped ends")
    d = torch.from_numpy(data).cuda()
    e = torch.from_numpy(ends.astype(np.int64)).cuda()
    for count in (6, 100):  # a count above the room computes the room
        n = torch.tensor([count], dtype=torch.int64, device="cuda")
        dig = ctx.chunk_digests(d, e, n).cpu().numpy()
        prev = 0
        for j, x in enumerate(ends.tolist()):
            a = min(prev, data.size)
            b = max(min(x, data.size), a)
            assert bytes(dig[j]) == oracle.hash(oracle.SHA1, data[a:b]), f"chunk {j}"
            prev = x
    n = torch.tensor([3], dtype=torch.int64, device="cuda")
    dig = ctx.chunk_digests(d, e, n, chunk_segment=700).cpu().numpy()
    exp = oracle.chunk_digests(oracle.SHA1, data, np.array([1000, 5000, 5000], np.uint64), 700)
    assert np.array_equal(dig[:3], exp)


def test_argument_errors(ctx, hg):
    note("stage argument errors")
    n = ctypes.c_uint64(0)
    ends = np.zeros(4, dtype=np.uint64)
    ns = ctypes.c_uint64(0)
    starts = np.zeros(10, dtype=np.uint64)
    # capacity below max_starts + 1
    assert hg.hg_chunk_select(ctx.handle, starts.ctypes.data, ctypes.byref(ns), 10, 1000, 20, 0, 0,
                              ends.ctypes.data, 4, ctypes.byref(n), 0, None) == hg.HG_EINVAL
    # max below min, window 0, NULL starts with room
    big = np.zeros(64, dtype=np.uint64)
    assert hg.hg_chunk_select(ctx.handle, starts.ctypes.data, ctypes.byref(ns), 10, 1000, 20, 100, 50,
                              big.ctypes.data, 64, ctypes.byref(n), 0, None) == hg.HG_EINVAL
    assert hg.hg_chunk_select(ctx.handle, starts.ctypes.data, ctypes.byref(ns), 10, 1000, 0, 0, 0,
                              big.ctypes.data, 64, ctypes.byref(n), 0, None) == hg.HG_EINVAL
    assert hg.hg_chunk_select(ctx.handle, None, ctypes.byref(ns), 10, 1000, 20, 0, 0,
                              big.ctypes.data, 64, ctypes.byref(n), 0, None) == hg.HG_EINVAL
    dig = np.zeros((4, 20), dtype=np.uint8)
    assert hg.hg_chunk_digests(ctx.handle, None, 10, ends.ctypes.data, ctypes.byref(n), 4, hg.HG_SHA1, 0,
                               dig.ctypes.data, 0, None) == hg.HG_EINVAL
    assert hg.hg_chunk_digests(ctx.handle, dig.ctypes.data, 10, ends.ctypes.data, ctypes.byref(n), 4, 7, 0,
                               dig.ctypes.data, 0, None) == hg.HG_EINVAL
    m = ctypes.c_uint64(0)
    assert hg.hg_similarity_n(ctx.handle, dig.ctypes.data, 4, dig.ctypes.data, None, None, 4, hg.HG_SHA1,
                              ctypes.byref(m), None, 0, None) == hg.HG_EINVAL


def test_side_stream_argument(ctx, hg):
    # Calls given a side stream while torch's current stream is busy: the
    # outputs they allocate and the fills that zero them are ordered on the
    # side stream, so nothing lands after the library's writes.
    data = inputs.uniform_bytes(640, 2 * MiB + 3)
    exp_starts = oracle.window_scan_sharded(oracle.MD5, data, 20, 1, 0xFFF, 0, THREADS)
    exp_ends = oracle.chunk_select(exp_starts, 20, data.size, 2048)
    exp_dig = oracle.chunk_digests(oracle.SHA1, data, exp_ends)
    lens = np.diff(exp_ends, prepend=np.uint64(0))
    exp_sim = oracle.similarity(oracle.SHA1, exp_dig, exp_dig[::2], lens[::2])
    d = torch.from_numpy(data).cuda()
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    note("stage calls on a side stream, current stream busy")
    a = torch.randn(2048, 2048, device="cuda")
    for _ in range(200):  # fp32 products: tens of ms on torch's current stream
        a = a @ a
        a = a / a.norm()
    starts = ctx.window_scan(d, 20, 1, 0xFFF, 0, stream=st)
    with torch.cuda.stream(st):
        cnt = torch.full((1,), starts.numel(), dtype=torch.int64, device="cuda")
    ends, n = ctx.chunk_select(starts, cnt, data.size, 20, 2048, asynchronous=True, stream=st)
    dig = ctx.chunk_digests(d, ends, n, asynchronous=True, stream=st)
    st.synchronize()
    k = int(n.item())
    assert np.array_equal(starts.cpu().numpy().astype(np.uint64), exp_starts)
    assert k == exp_ends.size
    assert np.array_equal(ends[:k].cpu().numpy().astype(np.uint64), exp_ends)
    assert np.array_equal(dig[:k].cpu().numpy(), exp_dig)
    for _ in range(100):
        a = a @ a
        a = a / a.norm()
    dd = torch.from_numpy(exp_dig).cuda()
    torch.cuda.synchronize()
    for _ in range(100):
        a = a @ a
        a = a / a.norm()
    with torch.cuda.stream(st):
        nb = torch.full((1,), exp_dig[::2].shape[0], dtype=torch.int64, device="cuda")
        db = dd[::2].contiguous()
        lb = torch.from_numpy(lens[::2].astype(np.int64)).cuda()
    got = ctx.similarity_n(dd, db, nb, len_b=lb, stream=st)
    assert tuple(got) == exp_sim
    # an asynchronous streaming chunker on the side stream
    ch = hg.Chunker(ctx)
    outs = [ch.feed(d[x:x + 700_000], stream=st, asynchronous=True) for x in range(0, data.size, 700_000)]
    outs.append(ch.finish(stream=st, asynchronous=True))
    st.synchronize()
    ch.close()
    got_e = np.concatenate([e[:int(c.item())].cpu().numpy().astype(np.uint64) for e, _, c in outs])
    got_d = np.concatenate([g[:int(c.item())].cpu().numpy() for _, g, c in outs])
    assert np.array_equal(got_e, exp_ends)
    assert np.array_equal(got_d, exp_dig)
    torch.cuda.synchronize()
