"""GPU test of hg_window_scan_noalloc, the window scan for callers that
cannot allocate: through the C ABI, its candidates and count equal those
of hg_window_scan on the same device input, on two calls in a row (the
second with a smaller input, so that the fixed scratch still holds the
first call's larger bookkeeping), for the register kernel (w = 20, stride
1) and the LDS kernel (w = 33, stride 3); a scan that needs more scratch
than the fixed array is refused before any launch; the calls make no
device or pinned allocation on the context.  Inputs: seeded uniform
bytes."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1202_3669_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
MiB = 1 << 20


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hg():
    from paper_1202_3669_amd import hashgpu
    return hashgpu


def _noalloc(hg, ctx, d, n, w, s, mask, cap):
    starts = torch.full((max(cap, 1),), -1, dtype=torch.int64, device="cuda")
    count = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = hg.hg_window_scan_noalloc(ctx.handle, d.data_ptr() if n else None, n, w, s, mask, 0, 0,
                                   starts.data_ptr() if cap else None, cap, count.data_ptr(), stream)
    assert st == hg.HG_OK, st
    torch.cuda.synchronize()
    total = int(count.item())
    return starts[:min(total, cap)].cpu().numpy().astype(np.uint64), total


@pytest.mark.parametrize("w,s,mask,sizes", [(20, 1, 0xFFF, (256 * MiB + 77, 3 * MiB + 5)),
                                            (33, 3, 0x3FF, (96 * MiB + 1, 1 * MiB - 7))])
def test_noalloc_equals_window_scan_on_two_calls(hg, w, s, mask, sizes):
    ctx = hg.Context(0)
    data = inputs.uniform_bytes(1300 + w, sizes[0])
    d_all = torch.from_numpy(data).cuda()
    before = None
    for k, n in enumerate(sizes):
        note(f"noalloc window scan w={w} s={s} call {k}: {n} bytes")
        d = d_all[:n]
        ref = ctx.window_scan(d, w, s, mask, 0).cpu().numpy().astype(np.uint64)
        if before is None:
            before = ctx.stats()
        got, total = _noalloc(hg, ctx, d, n, w, s, mask, cap=ref.size + 16)
        assert total == ref.size
        assert np.array_equal(got, ref)
        if k == 1:  # the small input checked against the oracle as well
            assert np.array_equal(got, oracle.window_scan(0, data[:n], w, s, mask, 0))
    # truncated output: count still the full number, the first entries written
    got, total = _noalloc(hg, ctx, d_all[:sizes[1]], sizes[1], w, s, mask, cap=5)
    assert total == ref.size and np.array_equal(got, ref[:5])
    after = ctx.stats()
    assert after["device_allocs"] == before["device_allocs"]
    assert after["pinned_allocs"] == before["pinned_allocs"]
    ctx.close()


def test_noalloc_refuses_scans_larger_than_its_scratch(hg):
    ctx = hg.Context(0)
    big = torch.empty(3 << 30, dtype=torch.uint8, device="cuda")  # not read: refused on the host
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = hg.hg_window_scan_noalloc(ctx.handle, big.data_ptr(), big.numel(), 20, 1, 0xFFF, 0, 0, None, 0,
                                   count.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == hg.HG_EINVAL
    buf = ctypes.create_string_buffer(256)
    hg.hg_last_error(ctx.handle, buf, 256)
    assert b"scratch" in buf.value
    del big
    ctx.close()
