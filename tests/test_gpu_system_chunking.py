"""GPU parity at the storage system's own chunking parameters (Sec. 4.3):
content-based chunks of about 1.2 MB on average, at least 256 KB and at most
4 MB.  Reading: MD5 windows of 20 bytes at stride 1 with a 20-bit boundary
mask (expected chunk length = minimum + 2^20 bytes, cut short by the
maximum), SHA-1 chunk digests.

The input (seeded uniform bytes with a 12 MiB run of zeros spliced in, whose
all-zero window is not a boundary under this mask) has both candidate-driven
cuts and a run of forced cuts at the maximum.  The single call, the
streaming chunker fed in 8 MiB pieces and a file batch must each give the
oracle's chunk ends and digests exactly."""
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
W, S, MASK, TARGET, MIN, MAX = 20, 1, 0xFFFFF, 0, 256 * KiB, 4 * MiB


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
def case():
    rnd = inputs.uniform_bytes(470, 28 * MiB + 12345)
    data = np.concatenate([rnd[:10 * MiB], np.zeros(12 * MiB, np.uint8), rnd[10 * MiB:]])
    starts = oracle.window_scan_sharded(oracle.MD5, data, W, S, MASK, TARGET, THREADS)
    ends = oracle.chunk_select(starts, W, data.size, MIN, MAX)
    dig = oracle.chunk_digests(oracle.SHA1, data, ends)
    lens = np.diff(ends, prepend=np.uint64(0))
    # the input is meant to exercise both kinds of cut
    assert int((lens == MAX).sum()) >= 2 and int((lens < MAX).sum()) >= 5
    return data, ends, dig


def test_single_call(ctx, case):
    data, ends, dig = case
    note(f"system parameters, single call, {data.size} bytes")
    got_e, got_d = ctx.chunk(torch.from_numpy(data).cuda(), W, S, MASK, TARGET, MIN, max_chunk=MAX)
    assert np.array_equal(got_e.cpu().numpy().astype(np.uint64), ends)
    assert np.array_equal(got_d.cpu().numpy(), dig)


@pytest.mark.parametrize("device_input", [True, False])
def test_streaming(ctx, hg, case, device_input):
    data, ends, dig = case
    note(f"system parameters, streamed in 8 MiB pieces, device={device_input}")
    src = torch.from_numpy(data).cuda() if device_input else data
    ch = hg.Chunker(ctx, W, S, MASK, TARGET, MIN, MAX)
    out_e, out_d = [], []
    for a in range(0, data.size, 8 * MiB):
        e, d = ch.feed(src[a:a + 8 * MiB])
        out_e.append(e)
        out_d.append(d)
    e, d = ch.finish()
    out_e.append(e)
    out_d.append(d)
    ch.close()
    assert np.array_equal(np.concatenate(out_e), ends)
    assert np.array_equal(np.concatenate(out_d).reshape(-1, 20), dig)


@pytest.mark.parametrize("seg", [0, 4096])
def test_file_batch(ctx, hg, case, seg):
    data, ends, dig = case
    if seg:
        dig = oracle.chunk_digests(oracle.SHA1, data, ends, seg)
    # three files: the whole input, its first 5 MiB + 3 bytes, its last 9 MiB
    off = np.array([0, data.size, data.size + 5 * MiB + 3], dtype=np.uint64)
    ln = np.array([data.size, 5 * MiB + 3, 9 * MiB], dtype=np.uint64)
    arena = np.concatenate([data, data[:5 * MiB + 3], data[-9 * MiB:]])
    note(f"system parameters, file batch of 3, chunk segment {seg}")
    b = hg.Batch(ctx, off, ln, mask=MASK, min_chunk=MIN, max_chunk=MAX, chunk_segment=seg)
    d = torch.from_numpy(arena).cuda()
    b.run(d)
    torch.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert st[2] == 0
    co = b.chunk_off.cpu().numpy()
    ce = b.chunk_ends.cpu().numpy().astype(np.uint64)
    cd = b.chunk_digests.cpu().numpy()
    for j in range(3):
        f = arena[int(off[j]):int(off[j]) + int(ln[j])]
        if j == 0:
            exp_e, exp_d = ends, dig
        else:
            s_ = oracle.window_scan_sharded(oracle.MD5, f, W, S, MASK, TARGET, THREADS)
            exp_e = oracle.chunk_select(s_, W, f.size, MIN, MAX)
            exp_d = oracle.chunk_digests(oracle.SHA1, f, exp_e, seg)
        assert np.array_equal(ce[co[j]:co[j + 1]], exp_e), f"file {j} ends"
        assert np.array_equal(cd[co[j]:co[j + 1]], exp_d), f"file {j} digests"
    b.close()
