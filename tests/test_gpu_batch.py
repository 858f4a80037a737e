"""GPU parity of file batches (hg_batch_*): many files in one arena get the
direct hash (64 KiB SHA-1 segments + second level) and content-based
chunking (MD5 w = 20, stride 1, low 12 bits, min 2 KiB, SHA-1 chunk
digests), and every file's results equal the oracle's (bit-exact).

Inputs: seeded log-normal file sizes (the batched workload: median 256 KiB,
sigma 1.5, capped at 64 MiB, 4096 files; smaller variants for the quick
cases), plus empty files and files shorter than a window, packed without
alignment.
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


def small_batch(seed, n, median=64 * KiB, cap=4 * MiB, extra_tiny=True):
    arena, off, ln = inputs.file_batch(seed, n, median=median, sigma=1.5, cap=cap, align=1)
    off, ln = off.astype(np.int64).tolist(), ln.astype(np.int64).tolist()
    if extra_tiny:
        # empty files and files shorter than a window, pointing into the arena
        off += [0, 5, 17, 100]
        ln += [0, 0, 19, 20]
    return arena, np.array(off, dtype=np.uint64), np.array(ln, dtype=np.uint64)


def check_file(b, j, data, kind_block=1, block=64 * KiB, w=20, s=1, mask=0xFFF, min_chunk=2048):
    lv = b.leaves.cpu().numpy() if not hasattr(b, "_lv") else b._lv
    exp_leaves = oracle.leaves_sharded(kind_block, data, block, THREADS)
    lf = b.leaf_first
    got = lv[int(lf[j]):int(lf[j + 1])]
    assert np.array_equal(got, exp_leaves), f"file {j} leaves"
    assert bytes(b._rt[j]) == oracle.root(kind_block, exp_leaves), f"file {j} root"
    starts = oracle.window_scan_sharded(oracle.MD5, data, w, s, mask, 0, THREADS)
    ends = oracle.chunk_select(starts, w, data.size, min_chunk)
    dig = oracle.chunk_digests(oracle.SHA1, data, ends)
    c0, c1 = int(b._co[j]), int(b._co[j + 1])
    assert np.array_equal(b._ce[c0:c1].astype(np.uint64), ends), f"file {j} chunk ends"
    assert np.array_equal(b._cd[c0:c1], dig), f"file {j} chunk digests"


def fetch(b):
    torch.cuda.synchronize()
    b._lv = b.leaves.cpu().numpy()
    b._rt = b.roots.cpu().numpy()
    b._ce = b.chunk_ends.cpu().numpy()
    b._cd = b.chunk_digests.cpu().numpy()
    b._co = b.chunk_off.cpu().numpy()
    b._st = b.status.cpu().numpy()


def test_batch_matches_oracle_per_file(ctx, hg):
    arena, off, ln = small_batch(900, 60)
    d = torch.from_numpy(arena).cuda()
    note(f"batch {len(off)} files, {arena.size} bytes")
    b = hg.Batch(ctx, off, ln)
    b.run(d)
    fetch(b)
    assert b._st[2] == 0, "candidate capacity exceeded"
    for j in range(len(off)):
        data = arena[int(off[j]):int(off[j]) + int(ln[j])]
        check_file(b, j, data)
    b.close()


def test_batch_equals_single_calls(ctx, hg):
    arena, off, ln = small_batch(901, 40)
    d = torch.from_numpy(arena).cuda()
    note("batch vs single calls")
    b = hg.Batch(ctx, off, ln)
    b.run(d)
    fetch(b)
    for j in range(len(off)):
        o, n = int(off[j]), int(ln[j])
        view = d[o:o + n]
        lv, rt = ctx.block_hash(view, 64 * KiB, hg.HG_SHA1)
        assert np.array_equal(b._lv[int(b.leaf_first[j]):int(b.leaf_first[j + 1])], lv.cpu().numpy())
        assert bytes(b._rt[j]) == bytes(rt.cpu().numpy())
        ends, dig = ctx.chunk(view, 20, 1, 0xFFF, 0, 2048)
        c0, c1 = int(b._co[j]), int(b._co[j + 1])
        assert np.array_equal(b._ce[c0:c1], ends.cpu().numpy())
        assert np.array_equal(b._cd[c0:c1], dig.cpu().numpy())
    b.close()


def test_batch_graph_replays_match_eager(ctx, hg):
    arena, off, ln = small_batch(902, 50)
    d = torch.from_numpy(arena).cuda()
    note("batch graph capture and replays")
    b = hg.Batch(ctx, off, ln)
    b.run(d)
    fetch(b)
    ref = {k: getattr(b, k).copy() for k in ("_lv", "_rt", "_ce", "_cd", "_co", "_st")}
    s = torch.cuda.Stream()
    b.capture(d, s)
    for r in range(3):
        for t in (b.leaves, b.roots, b.chunk_ends, b.chunk_digests, b.chunk_off, b.status):
            t.zero_()  # eager work between replays, and proof the replay rewrites
        torch.cuda.synchronize()
        b.replay(s)
        s.synchronize()
        fetch(b)
        for k, v in ref.items():
            assert np.array_equal(getattr(b, k), v), f"replay {r}: {k} differs"
    b.close()


def test_batch_with_max_chunk(ctx, hg):
    arena, off, ln = small_batch(906, 40)
    d = torch.from_numpy(arena).cuda()
    note("batch with a maximum chunk size")
    b = hg.Batch(ctx, off, ln, max_chunk=3000)
    b.run(d)
    fetch(b)
    assert b._st[2] == 0
    for j in range(len(off)):
        data = arena[int(off[j]):int(off[j]) + int(ln[j])]
        starts = oracle.window_scan(oracle.MD5, data, 20, 1, 0xFFF, 0)
        ends = oracle.chunk_select(starts, 20, data.size, 2048, 3000)
        c0, c1 = int(b._co[j]), int(b._co[j + 1])
        assert np.array_equal(b._ce[c0:c1].astype(np.uint64), ends), f"file {j} chunk ends"
        assert np.array_equal(b._cd[c0:c1], oracle.chunk_digests(oracle.SHA1, data, ends)), f"file {j} digests"
    b.close()


@pytest.mark.parametrize("seg", [1000, 4096])
def test_batch_two_level_chunk_digests(ctx, hg, seg):
    arena, off, ln = small_batch(907, 40)
    d = torch.from_numpy(arena).cuda()
    note(f"batch with two-level chunk digests, segment {seg}")
    b = hg.Batch(ctx, off, ln, chunk_segment=seg, max_chunk=3000 if seg == 1000 else 0)
    mx = 3000 if seg == 1000 else 0
    b.run(d)
    fetch(b)
    assert b._st[2] == 0
    ref = b._cd.copy()
    for j in range(len(off)):
        data = arena[int(off[j]):int(off[j]) + int(ln[j])]
        starts = oracle.window_scan(oracle.MD5, data, 20, 1, 0xFFF, 0)
        ends = oracle.chunk_select(starts, 20, data.size, 2048, mx)
        c0, c1 = int(b._co[j]), int(b._co[j + 1])
        assert np.array_equal(b._ce[c0:c1].astype(np.uint64), ends), f"file {j} chunk ends"
        assert np.array_equal(b._cd[c0:c1], oracle.chunk_digests(oracle.SHA1, data, ends, seg)), f"file {j}"
    # captured into a graph: every replay rewrites the same digests
    s = torch.cuda.Stream()
    b.capture(d, s)
    for r in range(3):
        b.chunk_digests.zero_()
        torch.cuda.synchronize()
        b.replay(s)
        s.synchronize()
        fetch(b)
        n = int(b._co[-1])
        assert np.array_equal(b._cd[:n], ref[:n]), f"replay {r}"
    b.close()


def test_batch_reports_candidate_overflow(ctx, hg):
    arena, off, ln = small_batch(903, 20, extra_tiny=False)
    d = torch.from_numpy(arena).cuda()
    note("batch overflow flag")
    b = hg.Batch(ctx, off, ln, max_candidates=5)
    b.run(d)
    fetch(b)
    assert b._st[0] > 5 and b._st[2] != 0
    b.close()


def test_batch_tuner_keeps_results(ctx, hg):
    arena, off, ln = small_batch(904, 80)
    d = torch.from_numpy(arena).cuda()
    note("batch tuner")
    b = hg.Batch(ctx, off, ln)
    b.run(d)
    fetch(b)
    ref = (b._lv.copy(), b._rt.copy())
    b.leaves.zero_()
    b.roots.zero_()
    torch.cuda.synchronize()
    report = b.tune(d)
    assert "->" in report, report
    # every candidate was timed: both file orders, 64-, 128- and 256-lane
    # workgroups, 1024-8192 wavefronts
    for order in ("longest", "given"):
        for g in (1024, 2048, 4096, 8192):
            for lanes in (64, 128, 256):
                assert f"{order}/{g}x{lanes}:" in report, report
    # the outputs of the last candidate timed (given order, 8192 wavefronts
    # in 256-lane workgroups), then of the chosen schedule
    torch.cuda.synchronize()
    fetch(b)
    assert np.array_equal(b._lv, ref[0]) and np.array_equal(b._rt, ref[1])
    b.run(d)
    fetch(b)
    assert np.array_equal(b._lv, ref[0]) and np.array_equal(b._rt, ref[1])
    b.close()


def _oracle_file(data, threads):
    """The oracle's results for one file: 64 KiB SHA-1 segment digests, the
    second level, chunk ends and SHA-1 chunk digests (MD5 w=20, stride 1,
    low 12 bits, min 2 KiB)."""
    lv = oracle.leaves_sharded(oracle.SHA1, data, 64 * KiB, threads)
    starts = oracle.window_scan_sharded(oracle.MD5, data, 20, 1, 0xFFF, 0, threads)
    ends = oracle.chunk_select(starts, 20, data.size, 2048)
    dig = oracle.chunk_digests_sharded(oracle.SHA1, data, ends, 0, threads)
    return lv, oracle.root(oracle.SHA1, lv), ends, dig


def test_batched_workload_4096_files(ctx, hg):
    # The batched configuration as the benchmark runs it: 4096 files,
    # log-normal sizes (median 256 KiB, sigma 1.5, cap 64 MiB), seed 5
    # (about 3.3 GB), schedule from the autotuner, captured into a graph and
    # replayed.  Every file's segment digests, second level, chunk ends and
    # chunk digests are compared with the oracle's (large files sharded over
    # the host threads, the rest one file per thread).
    from concurrent.futures import ThreadPoolExecutor
    arena, off, ln = inputs.file_batch(5, 4096)
    d = torch.from_numpy(arena).cuda()
    note(f"batched workload: {arena.size / 2**30:.2f} GiB, tune + capture + replay")
    b = hg.Batch(ctx, off, ln)
    s = torch.cuda.Stream()
    b.tune(d, s)
    b.capture(d, s)
    s.synchronize()
    for t in (b.leaves, b.roots, b.chunk_ends, b.chunk_digests, b.chunk_off):
        t.zero_()  # what is compared below comes from the replays
    torch.cuda.synchronize()
    for _ in range(3):
        b.replay(s)
    s.synchronize()
    fetch(b)
    assert b._st[2] == 0
    lf, co = b.leaf_first, b._co
    note("batched workload: oracle over every file")

    def check(j, threads):
        data = arena[int(off[j]):int(off[j]) + int(ln[j])]
        lv, rt, ends, dig = _oracle_file(data, threads)
        assert np.array_equal(b._lv[int(lf[j]):int(lf[j + 1])], lv), f"file {j} leaves"
        assert bytes(b._rt[j]) == rt, f"file {j} root"
        c0, c1 = int(co[j]), int(co[j + 1])
        assert np.array_equal(b._ce[c0:c1].astype(np.uint64), ends), f"file {j} chunk ends"
        assert np.array_equal(b._cd[c0:c1], dig), f"file {j} chunk digests"
        return j

    order = np.argsort(-ln.astype(np.int64), kind="stable").tolist()
    big = [j for j in order if int(ln[j]) >= 8 * MiB]
    small = [j for j in order if int(ln[j]) < 8 * MiB]
    for j in big:
        check(j, THREADS)
    with ThreadPoolExecutor(THREADS) as ex:
        done = list(ex.map(lambda j: check(j, 1), small))
    assert len(big) + len(done) == 4096
    note(f"batched workload: {len(big)} large and {len(done)} other files equal the oracle")
    b.close()
