"""GPU tests of the persistent block-map (hg_blockmap_*): each write marks
exactly the chunks a sequential store would not store again -- digest
already stored, or equal to an earlier chunk of the same write -- against a
Python set walked in order (an independent reference), and the duplicate
bytes of an edited version equal the oracle's byte-weighted similarity.
Inputs: seeded random digests with planted repeats within and across
writes; the two-version similarity workload at 4 MiB."""
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


def planted(seed, n, d, repeats, pool=None):
    rng = np.random.default_rng(seed)
    dig = rng.integers(0, 256, size=(n, d), dtype=np.uint8)
    for _ in range(repeats):
        i, j = sorted(rng.choice(n, size=2, replace=False).tolist())
        dig[j] = dig[i]
    if pool is not None:  # repeats of digests written before
        for j in rng.choice(n, size=repeats, replace=False).tolist():
            dig[j] = pool[int(rng.integers(0, len(pool)))]
    lens = rng.integers(1, 10_000, size=n).astype(np.uint64)
    return dig, lens


def reference(seen, dig, lens):
    dup = np.zeros(len(dig), dtype=bool)
    for i, row in enumerate(dig):
        key = row.tobytes()
        dup[i] = key in seen
        seen.add(key)
    return dup, int(dup.sum()), int(lens[dup].sum())


@pytest.mark.parametrize("d,kind", [(20, 1), (16, 0)])
def test_writes_match_sequential_store(ctx, hg, d, kind):
    bm = hg.BlockMap(ctx, kind, capacity=1 << 20)
    seen = set()
    prev = None
    for w, (n, rep) in enumerate([(50_000, 500), (80_000, 2000), (1, 0), (0, 0), (200_000, 5000)]):
        dig, lens = planted(700 + w, n, d, rep, prev)
        note(f"blockmap write {w}: n={n} d={d}")
        exp_dup, exp_c, exp_b = reference(seen, dig, lens)
        src = torch.from_numpy(dig).cuda() if w % 2 else dig
        ln = torch.from_numpy(lens.view(np.int64)).cuda() if w % 2 else lens
        dup, c, b = bm.write(src, lengths=ln)
        assert np.array_equal(dup, exp_dup), f"write {w}"
        assert (c, b) == (exp_c, exp_b)
        assert bm.size() == len(seen)
        prev = dig if n else prev
    bm.close()


def test_versions_duplicate_bytes_equal_similarity(ctx, hg):
    a = inputs.uniform_bytes(710, 4 << 20)
    b, _ = inputs.edited_version(a, 711, 16)
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    ea, ga = ctx.chunk(da, 20, 1, 0xFFF, 0, 2048)
    eb, gb = ctx.chunk(db, 20, 1, 0xFFF, 0, 2048)
    bm = hg.BlockMap(ctx, hg.HG_SHA1, capacity=1 << 16)
    note("blockmap versions")
    dup_a, ca, ba = bm.write(ga, ends=ea)
    # version A: random data, no chunk repeats itself
    assert ca == 0 and not dup_a.any()
    dup_b, cb, bb = bm.write(gb, ends=eb)
    _, xea, xga = oracle.chunk(oracle.MD5, oracle.SHA1, a, 20, 1, 0xFFF, 0, 2048)
    _, xeb, xgb = oracle.chunk(oracle.MD5, oracle.SHA1, b, 20, 1, 0xFFF, 0, 2048)
    m, mb = oracle.similarity(oracle.SHA1, xga, xgb, np.diff(xeb, prepend=np.uint64(0)))
    assert (cb, bb) == (m, mb)
    assert bm.size() == xga.shape[0] + (xgb.shape[0] - m)
    bm.close()


def test_capacity_is_enforced_without_change(ctx, hg):
    bm = hg.BlockMap(ctx, hg.HG_SHA1, capacity=100)
    dig, lens = planted(720, 60, 20, 0)
    bm.write(dig, lengths=lens)
    more, _ = planted(721, 50, 20, 0)
    with pytest.raises(hg.HashGpuError) as e:
        bm.write(more)
    assert e.value.status == hg.HG_EBUSY
    assert bm.size() == 60
    dup, c, _ = bm.write(dig[:40])
    assert dup.all() and c == 40 and bm.size() == 60
    bm.close()
