"""GPU parity of standard chunk digests when chunks are long: hg_chunk
hashes the longest chunks on the host (one sequential chain each) while the
GPU hashes the rest, and every digest must equal the oracle's.  Cases: the
block-size sweep's content-based configurations on the 256 MiB version of
the similarity workload (MD5 w=20, stride 1, mask of log2(B) bits, min B/4,
max 4B, for B = 1 MiB and 4 MiB), from device memory and from pinned and
pageable host memory; MD5 chunk digests; an input whose long zero run has
no candidate (one chunk of tens of MiB); stride 4 with hundreds of chunks
above 64 KiB; truncated output and HG_ASYNC.
Inputs: seeded uniform bytes (seed 3) and zero runs."""
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


@pytest.fixture(scope="module")
def version_a():
    return inputs.uniform_bytes(3, 256 * MiB)


def _expect(data, mask, mn, mx, kind_chunk=oracle.SHA1):
    _, ends, dig = oracle.chunk(oracle.MD5, kind_chunk, data, 20, 1, mask, 0, mn, THREADS, max_chunk=mx)
    return ends, dig


@pytest.mark.parametrize("size", [MiB, 4 * MiB])
def test_sweep_configuration_device_and_host_input(ctx, version_a, size):
    bits = size.bit_length() - 1
    mask, mn, mx = (1 << bits) - 1, size // 4, 4 * size
    xe, xd = _expect(version_a, mask, mn, mx)
    assert np.diff(xe, prepend=np.uint64(0)).max() >= 64 * KiB  # long chunks present
    d = torch.from_numpy(version_a).cuda()
    pinned = torch.from_numpy(version_a).pin_memory()
    for where, src in (("device", d), ("pinned", pinned), ("pageable", torch.from_numpy(version_a))):
        note(f"long chunks B={size // KiB}k from {where}")
        ends, dig = ctx.chunk(src, 20, 1, mask, 0, mn, max_chunk=mx)
        torch.cuda.synchronize()
        assert np.array_equal(ends.cpu().numpy().astype(np.uint64), xe), where
        assert np.array_equal(dig.cpu().numpy(), xd), where


def test_many_medium_long_chunks_at_stride_4(ctx, version_a):
    # Stride 4 with the similarity workload's parameters (low 12 bits, min
    # 2 KiB): chunks of 18 KiB on average and a few hundred above 64 KiB,
    # so the host takes many chunks at once (packed on the device and copied
    # back in groups); from device and from pageable host memory.
    _, xe, xd = oracle.chunk(oracle.MD5, oracle.SHA1, version_a, 20, 4, 0xFFF, 0, 2 * KiB, THREADS)
    lens = np.diff(xe, prepend=np.uint64(0))
    assert (lens >= 64 * KiB).sum() > 100
    for where, src in (("device", torch.from_numpy(version_a).cuda()), ("pageable", torch.from_numpy(version_a))):
        note(f"stride 4, {int((lens >= 64 * KiB).sum())} chunks of 64 KiB and more, from {where}")
        ends, dig = ctx.chunk(src, 20, 4, 0xFFF, 0, 2 * KiB)
        torch.cuda.synchronize()
        assert np.array_equal(ends.cpu().numpy().astype(np.uint64), xe), where
        assert np.array_equal(dig.cpu().numpy(), xd), where


def test_md5_chunk_digests(ctx, hg, version_a):
    data = version_a[:64 * MiB]
    xe, xd = _expect(data, 0xFFFFF, 256 * KiB, 0, kind_chunk=oracle.MD5)
    note("long chunks, MD5 chunk digests")
    ends, dig = ctx.chunk(torch.from_numpy(data).cuda(), 20, 1, 0xFFFFF, 0, 256 * KiB, chunk_digest=hg.HG_MD5)
    assert np.array_equal(ends.cpu().numpy().astype(np.uint64), xe)
    assert np.array_equal(dig.cpu().numpy(), xd)


def test_giant_chunk_of_zeros(ctx):
    # 48 MiB: random, a 30 MiB zero run (the all-zero window is not a
    # candidate: one chunk spans it), random again; min 2 KiB.
    data = inputs.uniform_bytes(41, 48 * MiB)
    data[9 * MiB:39 * MiB] = 0
    xe, xd = _expect(data, 0xFFF, 2 * KiB, 0)
    assert np.diff(xe, prepend=np.uint64(0)).max() > 29 * MiB
    note("giant chunk over a zero run")
    for src in (torch.from_numpy(data).cuda(), torch.from_numpy(data)):
        ends, dig = ctx.chunk(src, 20, 1, 0xFFF, 0, 2 * KiB)
        assert np.array_equal(ends.cpu().numpy().astype(np.uint64), xe)
        assert np.array_equal(dig.cpu().numpy(), xd)


def test_truncated_and_async(ctx, hg, version_a):
    data = version_a[:96 * MiB]
    mask, mn, mx = 0xFFFFF, 256 * KiB, 4 * MiB
    xe, xd = _expect(data, mask, mn, mx)
    d = torch.from_numpy(data).cuda()
    note("long chunks, capacity below the chunk count")
    cap = xe.size // 2
    p = hg.hg_chunk_params(20, 1, mask, 0, mn, mx, hg.HG_MD5, hg.HG_SHA1, 0)
    ends = np.zeros(cap, dtype=np.uint64)
    dig = np.zeros((cap, 20), dtype=np.uint8)
    n = np.zeros(1, dtype=np.uint64)
    st = hg.hg_chunk(ctx.handle, d.data_ptr(), data.size, hg.ctypes.byref(p), ends.ctypes.data, cap,
                     n.ctypes.data, dig.ctypes.data, hg.HG_IN_DEVICE, torch.cuda.current_stream().cuda_stream)
    assert st == hg.HG_ETRUNC and int(n[0]) == xe.size
    assert np.array_equal(ends, xe[:cap]) and np.array_equal(dig, xd[:cap])
    note("long chunks, HG_ASYNC device outputs")
    e2 = torch.zeros(xe.size + 8, dtype=torch.int64, device="cuda")
    g2 = torch.zeros((xe.size + 8, 20), dtype=torch.uint8, device="cuda")
    n2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = hg.hg_chunk(ctx.handle, d.data_ptr(), data.size, hg.ctypes.byref(p), e2.data_ptr(), xe.size + 8,
                     n2.data_ptr(), g2.data_ptr(), hg.HG_IN_DEVICE | hg.HG_OUT_DEVICE | hg.HG_ASYNC,
                     torch.cuda.current_stream().cuda_stream)
    assert st == hg.HG_OK
    torch.cuda.synchronize()
    assert int(n2.item()) == xe.size
    assert np.array_equal(e2[:xe.size].cpu().numpy().astype(np.uint64), xe)
    assert np.array_equal(g2[:xe.size].cpu().numpy(), xd)
