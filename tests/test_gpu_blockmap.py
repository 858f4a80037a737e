"""GPU tests of the persistent block-map (hg_blockmap_*) against the
oracle's block-map (Sec. 3.2.1: a chunk whose digest the store already
holds is not stored again; within one write, a repeat of an earlier chunk
is a duplicate too).  Every expected flag, count, byte sum and map size
comes from ``oracle.BlockMap`` fed with the same digests.

Inputs: seeded random digests with planted repeats within and across
writes (five writes, including an empty one and a one-chunk one, host and
device input); the two-version similarity workload at 4 MiB; and the write
path the benchmark times: eight versions of a 256 MiB file (seed 7, each
next version 256 seeded 1-4 KiB edits of the previous, seeds 8 ...),
chunked by the GPU and by the oracle (MD5 w=20, stride 1, low 12 bits,
min 2 KiB, SHA-1 chunk digests), every version written to both maps."""
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


def planted(seed, n, d, repeats, pool=None):
    rng = np.random.default_rng(seed)
    dig = rng.integers(0, 256, size=(n, d), dtype=np.uint8)
    for _ in range(repeats if n > 1 else 0):
        i, j = sorted(rng.choice(n, size=2, replace=False).tolist())
        dig[j] = dig[i]
    if pool is not None and n:  # repeats of digests written before
        for j in rng.choice(n, size=min(repeats, n), replace=False).tolist():
            dig[j] = pool[int(rng.integers(0, len(pool)))]
    lens = rng.integers(1, 10_000, size=n).astype(np.uint64)
    return dig, lens


@pytest.mark.parametrize("d,kind", [(20, 1), (16, 0)])
def test_writes_match_oracle_store(ctx, hg, d, kind):
    bm = hg.BlockMap(ctx, kind, capacity=1 << 20)
    ref = oracle.BlockMap(kind, capacity=1 << 20)
    prev = None
    for w, (n, rep) in enumerate([(50_000, 500), (80_000, 2000), (1, 0), (0, 0), (200_000, 5000)]):
        dig, lens = planted(700 + w, n, d, rep, prev)
        note(f"blockmap write {w}: n={n} d={d}")
        exp_dup, exp_c, exp_b = ref.write(dig, lengths=lens)
        src = torch.from_numpy(dig).cuda() if w % 2 else dig
        ln = torch.from_numpy(lens.view(np.int64)).cuda() if w % 2 else lens
        dup, c, b = bm.write(src, lengths=ln)
        assert np.array_equal(dup, exp_dup), f"write {w}"
        assert (c, b) == (exp_c, exp_b), f"write {w}"
        assert bm.size() == ref.size(), f"write {w}"
        prev = dig if n else prev
    bm.close()
    ref.close()


def test_versions_duplicate_bytes_equal_similarity(ctx, hg):
    a = inputs.uniform_bytes(710, 4 << 20)
    b, _ = inputs.edited_version(a, 711, 16)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    ea, ga = ctx.chunk(da, 20, 1, 0xFFF, 0, 2048)
    eb, gb = ctx.chunk(db, 20, 1, 0xFFF, 0, 2048)
    bm = hg.BlockMap(ctx, hg.HG_SHA1, capacity=1 << 16)
    ref = oracle.BlockMap(oracle.SHA1)
    note("blockmap versions")
    _, xea, xga = oracle.chunk(oracle.MD5, oracle.SHA1, a, 20, 1, 0xFFF, 0, 2048, THREADS)
    _, xeb, xgb = oracle.chunk(oracle.MD5, oracle.SHA1, b, 20, 1, 0xFFF, 0, 2048, THREADS)
    assert np.array_equal(gb.cpu().numpy(), xgb)
    for gpu_in, ends, xg, xe in ((ga, ea, xga, xea), (gb, eb, xgb, xeb)):
        dup, c, by = bm.write(gpu_in, ends=ends)
        xdup, xc, xby = ref.write(xg, ends=xe)
        assert np.array_equal(dup, xdup) and (c, by) == (xc, xby)
        assert bm.size() == ref.size()
    # the same count by the similarity lookup (B has no repeats of its own)
    m, mb = oracle.similarity(oracle.SHA1, xga, xgb, np.diff(xeb, prepend=np.uint64(0)))
    assert (c, by) == (m, mb)
    bm.close()
    ref.close()


def test_eight_version_write_path(ctx, hg):
    """The benchmark's write path, version by version, against the oracle."""
    bm = hg.BlockMap(ctx, hg.HG_SHA1, capacity=1 << 24)
    ref = oracle.BlockMap(oracle.SHA1)
    v = inputs.uniform_bytes(7, 256 * MiB)
    for k in range(8):
        note(f"write path version {k}")
        d = torch.from_numpy(v).cuda()
        ends, dig = ctx.chunk(d, 20, 1, 0xFFF, 0, 2 * KiB)
        dup, c, by = bm.write(dig, ends=ends)
        _, xe, xg = oracle.chunk(oracle.MD5, oracle.SHA1, v, 20, 1, 0xFFF, 0, 2 * KiB, THREADS)
        assert np.array_equal(ends.cpu().numpy().astype(np.uint64), xe), f"version {k} ends"
        assert np.array_equal(dig.cpu().numpy(), xg), f"version {k} digests"
        xdup, xc, xby = ref.write(xg, ends=xe)
        assert np.array_equal(dup, xdup), f"version {k} flags"
        assert (c, by) == (xc, xby), f"version {k} counts"
        assert bm.size() == ref.size(), f"version {k} size"
        if k == 0:
            assert c == 0
        else:
            assert c > 0.9 * len(xe)  # 256 edits per 256 MiB: most chunks repeat
        del d
        if k + 1 < 8:
            v, _ = inputs.edited_version(v, 8 + k, 256)
    bm.close()
    ref.close()


def test_capacity_is_enforced_without_change(ctx, hg):
    bm = hg.BlockMap(ctx, hg.HG_SHA1, capacity=100)
    ref = oracle.BlockMap(oracle.SHA1, capacity=100)
    dig, lens = planted(720, 60, 20, 0)
    bm.write(dig, lengths=lens)
    ref.write(dig, lengths=lens)
    more, _ = planted(721, 50, 20, 0)
    with pytest.raises(hg.HashGpuError) as e:
        bm.write(more)
    assert e.value.status == hg.HG_EBUSY
    with pytest.raises(OverflowError):
        ref.write(more)
    assert bm.size() == ref.size() == 60
    dup, c, _ = bm.write(dig[:40])
    xdup, xc, _ = ref.write(dig[:40])
    assert np.array_equal(dup, xdup) and c == xc == 40 and bm.size() == 60
    bm.close()
    ref.close()
