"""GPU tests of second levels computed on the host (Sec. 3.2.2: the CPU
hashes the buffer of segment digests into the final value).  hg_block_hash
and hg_block_hash_dual move the second level to the host from a 16 KiB
digest buffer on; hg_roots_batch / hg_block_hash_batch do with
HG_HOST_ROOTS.  Every root is compared with the oracle's, on both sides of
the threshold (MD5: 1023 / 1024 / 1025 segments; SHA-1: 819 / 820 / 821),
with device and host outputs, synchronous and HG_ASYNC, and for batches of
mixed digests and lengths including empty jobs.  Inputs: seeded uniform
bytes."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1202_3669_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


SIDES = [(0, 1023), (0, 1024), (0, 1025), (1, 819), (1, 820), (1, 821)]


@pytest.mark.parametrize("kind,segments", SIDES)
@pytest.mark.parametrize("mode", ["sync", "async"])
def test_root_both_sides_of_threshold_device_outputs(ctx, hg, kind, segments, mode):
    block = 512
    data = inputs.uniform_bytes(900 + segments, segments * block - 77)
    note(f"host root kind={kind} segments={segments} mode={mode}")
    d = torch.from_numpy(data).cuda()
    extra = hg.HG_ASYNC if mode == "async" else 0
    lv, rt = ctx.block_hash(d, block, kind, flags_extra=extra)
    torch.cuda.synchronize()
    exp = oracle.leaves(kind, data, block)
    assert np.array_equal(lv.cpu().numpy(), exp)
    assert bytes(rt.cpu().numpy()) == oracle.root(kind, exp)
    # root only (the digests never leave the device but for the host step)
    _, rt2 = ctx.block_hash(d, block, kind, leaves=False, flags_extra=extra)
    torch.cuda.synchronize()
    assert bytes(rt2.cpu().numpy()) == oracle.root(kind, exp)


@pytest.mark.parametrize("kind,segments", [(0, 1023), (0, 5000), (1, 819), (1, 5000)])
def test_root_host_outputs(ctx, hg, kind, segments):
    block = 256
    data = inputs.uniform_bytes(950 + segments, segments * block)
    note(f"host root, host outputs kind={kind} segments={segments}")
    d = torch.from_numpy(data).cuda()
    dsz = oracle.digest_size(kind)
    leaves = np.zeros((segments, dsz), dtype=np.uint8)
    root = np.zeros(dsz, dtype=np.uint8)
    s = torch.cuda.current_stream().cuda_stream
    # host leaves and root
    assert hg.hg_block_hash(ctx.handle, d.data_ptr(), data.size, block, kind, leaves.ctypes.data,
                            root.ctypes.data, hg.HG_IN_DEVICE, s) == 0
    exp = oracle.leaves(kind, data, block)
    assert np.array_equal(leaves, exp)
    assert bytes(root) == oracle.root(kind, exp)
    # host root only, host input
    root[:] = 0
    assert hg.hg_block_hash(ctx.handle, data.ctypes.data, data.size, block, kind, None,
                            root.ctypes.data, 0, s) == 0
    assert bytes(root) == oracle.root(kind, exp)


@pytest.mark.parametrize("segments", [100, 1024, 20000])
def test_dual_roots(ctx, hg, segments):
    block = 1024
    data = inputs.uniform_bytes(970 + segments, segments * block + 33)
    note(f"dual roots segments={segments}")
    d = torch.from_numpy(data).cuda()
    lm, rm, ls, rs = ctx.block_hash_dual(d, block)
    torch.cuda.synchronize()
    for kind, lv, rt in ((0, lm, rm), (1, ls, rs)):
        exp = oracle.leaves(kind, data, block)
        assert np.array_equal(lv.cpu().numpy(), exp)
        assert bytes(rt.cpu().numpy()) == oracle.root(kind, exp)
    # roots only, asynchronous
    _, rm2, _, rs2 = ctx.block_hash_dual(d, block, leaves=False, flags_extra=hg.HG_ASYNC)
    torch.cuda.synchronize()
    assert bytes(rm2.cpu().numpy()) == bytes(rm.cpu().numpy())
    assert bytes(rs2.cpu().numpy()) == bytes(rs.cpu().numpy())


@pytest.mark.parametrize("asynchronous", [False, True])
def test_batch_host_roots(ctx, hg, asynchronous):
    rng = np.random.default_rng(990)
    pool = inputs.uniform_bytes(991, 64 << 20)
    dpool = torch.from_numpy(pool).cuda()
    specs, ref = [], []
    for i in range(40):
        ln = 0 if i % 13 == 0 else int(rng.integers(1, 8 << 20))
        off = int(rng.integers(0, pool.size - ln + 1))
        block = int(rng.choice([64, 4096, 65536, 1 << 20]))
        kind = int(i % 2)
        specs.append((dpool[off:off + ln], block, kind))
        ref.append((pool[off:off + ln], block, kind))
    note(f"batch host roots async={asynchronous}")
    recs, leaves, roots = ctx.batch_outputs(specs)
    ctx.run_batch(recs, len(specs), "both", asynchronous=asynchronous, host_roots=True)
    torch.cuda.synchronize()
    for i, (data, block, kind) in enumerate(ref):
        exp = oracle.leaves(kind, data, block)
        assert np.array_equal(leaves[i].cpu().numpy(), exp), i
        assert bytes(roots[i].cpu().numpy()) == oracle.root(kind, exp), i
    # the same second levels again on GPU lanes from the digests just made
    gl = [torch.zeros_like(r) for r in roots]
    for i in range(len(specs)):
        recs[i].root_out = gl[i].data_ptr()
    ctx.run_batch(recs, len(specs), "roots", asynchronous=False)
    for i in range(len(specs)):
        assert torch.equal(gl[i], roots[i]), i


def test_host_roots_flag_errors(ctx, hg):
    data = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    recs, leaves, _ = ctx.batch_outputs([(data, 64, 0)])  # leaves: referenced while the records point at it
    table = ctx.device_job_table(recs)
    with pytest.raises(hg.HashGpuError) as e:
        ctx.run_batch(table, 1, "roots", host_roots=True)
    assert e.value.status == hg.HG_EINVAL
    with pytest.raises(hg.HashGpuError) as e:
        ctx.run_batch(recs, 1, "leaves", host_roots=True)
    assert e.value.status == hg.HG_EINVAL
