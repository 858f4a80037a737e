"""GPU tests of the serving loop (hg_server_*): every request's outputs in a
mix of concurrently served requests equal the outputs of the same request
run alone through the single-call entry points (bit-exact), and a seeded
sample equals the oracle.  Also: host payloads admitted through a small
staging budget, requests larger than a group, groups whose candidate count
exceeds their capacity, truncation, injected failures, callbacks.

Inputs: the serving workload's request stream (seed 6: log-normal sizes,
mix 50% block SHA-1 / 30% block MD5 / 20% chunking), with sizes clipped to
a few MiB so that the alone runs and the oracle stay quick; payloads are
slices of one seeded random pool at seeded offsets (unaligned).
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
KiB, MiB = 1 << 10, 1 << 20
THREADS = max(1, min(16, os.cpu_count() or 1))


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
def pool():
    host = inputs.uniform_bytes(61, 32 * MiB)
    return host, torch.from_numpy(host).cuda()


def stream_specs(seed, n, pool_len, hi=4 * MiB):
    _, sizes, kinds = inputs.request_stream(seed, n, 1000.0, lo=0, hi=hi)
    rng = np.random.default_rng(seed + 1000)
    offs = [int(rng.integers(0, pool_len - int(s) + 1)) for s in sizes]
    return [(int(k), o, int(s)) for k, o, s in zip(kinds, offs, sizes)]


def alone(ctx, hg, dev_pool, spec, rs):
    """The single-call result of one request (on the device-resident pool)."""
    k, o, n = spec
    view = dev_pool[o:o + n]
    if k in (0, 1):
        lv, rt = ctx.block_hash(view, 64 * KiB, hg.HG_SHA1 if k == 0 else hg.HG_MD5)
        return ("block", lv.cpu().numpy(), bytes(rt.cpu().numpy()))
    ends, dig = ctx.chunk(view, 20, 1, 0xFFF, 0, 2048)
    return ("chunk", ends.cpu().numpy().astype(np.uint64), dig.cpu().numpy())


def same(a, b):
    return a[0] == b[0] and np.array_equal(a[1], b[1]) and (
        a[2] == b[2] if a[0] == "block" else np.array_equal(a[2], b[2]))


def oracle_result(host_pool, spec):
    k, o, n = spec
    data = host_pool[o:o + n]
    if k in (0, 1):
        kind = oracle.SHA1 if k == 0 else oracle.MD5
        lv = oracle.leaves_sharded(kind, data, 64 * KiB, THREADS)
        return ("block", lv, oracle.root(kind, lv))
    _, ends, dig = oracle.chunk(oracle.MD5, oracle.SHA1, data, 20, 1, 0xFFF, 0, 2048, THREADS)
    return ("chunk", ends, dig)


def check_all(ctx, hg, pool, rs, sts, sample=8, seed=0):
    host, dev = pool
    assert np.all(sts == hg.HG_OK), np.unique(sts, return_counts=True)
    for i, spec in enumerate(rs.specs):
        got = rs.result(i)
        assert same(got, alone(ctx, hg, dev, spec, rs)), f"request {i} {spec} differs from alone"
    rng = np.random.default_rng(seed)
    for i in rng.choice(len(rs), size=min(sample, len(rs)), replace=False):
        assert same(rs.result(int(i)), oracle_result(host, rs.specs[int(i)])), f"request {i} vs oracle"


def test_mix_equals_alone_device_payloads(ctx, hg, pool):
    host, dev = pool
    specs = stream_specs(6, 160, dev.numel())
    specs[3] = (0, 7, 0)       # empty block request
    specs[4] = (2, 9, 0)       # empty chunk request
    specs[5] = (2, 11, 19)     # shorter than a window
    rs = hg.RequestSet(dev.data_ptr(), True, specs)
    note(f"mix of {len(specs)} requests, burst arrival, device payloads")
    with hg.Server(0, slots=3, max_requests=64, device_budget=64 * MiB, max_group_bytes=64 * MiB) as srv:
        lat, sts = srv.play(rs, np.zeros(len(specs)))
        st = srv.stats()
    assert st["completed"] == len(specs) and st["failed"] == 0
    assert st["groups"] < len(specs), "requests were not batched"
    assert np.all(lat >= 0)
    check_all(ctx, hg, pool, rs, sts)


def test_mix_equals_alone_poisson_host_payloads(ctx, hg, pool):
    # Host payloads (pinned), Poisson arrivals, and a staging budget smaller
    # than the requests in flight: admission must wait for returned bytes.
    host, dev = pool
    pinned = torch.from_numpy(host).pin_memory()
    arrival, _, _ = inputs.request_stream(7, 120, 2000.0)
    specs = stream_specs(7, 120, dev.numel())
    rs = hg.RequestSet(pinned.data_ptr(), False, specs)
    note(f"mix of {len(specs)} requests, Poisson arrivals, pinned host payloads, 8 MiB staging")
    with hg.Server(0, slots=3, max_requests=32, device_budget=8 * MiB, max_group_bytes=8 * MiB) as srv:
        lat, sts = srv.play(rs, arrival)
        st = srv.stats()
    assert st["completed"] == len(specs) and st["in_flight"] == 0
    check_all(ctx, hg, pool, rs, sts, seed=1)


def test_oversized_request_runs_alone(ctx, hg, pool):
    host, dev = pool
    specs = [(0, 3, 5 * MiB + 17), (2, 1000, 3 * MiB + 5), (1, 77, 2 * MiB), (0, 5, 100)]
    rs = hg.RequestSet(dev.data_ptr(), True, specs)
    note("requests larger than a group")
    with hg.Server(0, slots=2, max_requests=4, device_budget=16 * MiB, max_group_bytes=1 * MiB) as srv:
        _, sts = srv.play(rs, np.zeros(len(specs)))
    check_all(ctx, hg, pool, rs, sts, sample=2)


def test_dense_candidates_fall_back_to_alone(ctx, hg):
    # Zero bytes with the target set to the low 12 bits of the all-zero
    # window's digest: every window is a candidate, far beyond the group's
    # candidate capacity, so the group serves its chunk requests alone.
    zeros = np.zeros(64, dtype=np.uint8)
    target = next(t for t in range(4096) if oracle.window_scan(oracle.MD5, zeros, 20, 1, 0xFFF, t).size)
    dev = torch.zeros(4 * MiB, dtype=torch.uint8, device="cuda")
    specs = [(2, 0, 1 * MiB), (2, 13, 1 * MiB), (0, 0, 1 * MiB), (2, 100, 2 * MiB - 100)]
    rs = hg.RequestSet(dev.data_ptr(), True, specs, target=target)
    note(f"dense candidates (target {target:#x})")
    with hg.Server(0, slots=1, max_requests=8, device_budget=8 * MiB, max_group_bytes=4 * MiB) as srv:
        _, sts = srv.play(rs, np.zeros(len(specs)))
    assert np.all(sts == hg.HG_OK)
    for i, (k, o, n) in enumerate(specs):
        got = rs.result(i)
        if k == 2:
            ends, dig = ctx.chunk(dev[o:o + n], 20, 1, 0xFFF, target, 2048)
            assert np.array_equal(got[1], ends.cpu().numpy().astype(np.uint64))
            assert np.array_equal(got[2], dig.cpu().numpy())
            data = np.zeros(n, dtype=np.uint8)
            exp = oracle.chunk_select(oracle.window_scan(oracle.MD5, data, 20, 1, 0xFFF, target), 20, n, 2048)
            assert np.array_equal(got[1], exp)
        else:
            lv, rt = ctx.block_hash(dev[o:o + n], 64 * KiB, hg.HG_SHA1)
            assert bytes(rt.cpu().numpy()) == got[2]


def test_chunk_requests_with_max_chunk(ctx, hg, pool):
    host, dev = pool
    specs = [(2, 0, 1 * MiB), (0, 5, 300 * KiB), (2, 50, 2 * MiB + 3), (2, 77, 10)]
    rs = hg.RequestSet(dev.data_ptr(), True, specs, max_chunk=4096)
    note("chunk requests with a maximum chunk size")
    with hg.Server(0, slots=2, max_requests=8, device_budget=8 * MiB, max_group_bytes=8 * MiB) as srv:
        _, sts = srv.play(rs, np.zeros(len(specs)))
    assert np.all(sts == hg.HG_OK)
    for i, (k, o, n) in enumerate(specs):
        got = rs.result(i)
        if k == 2:
            data = host[o:o + n]
            starts = oracle.window_scan(oracle.MD5, data, 20, 1, 0xFFF, 0)
            ends = oracle.chunk_select(starts, 20, n, 2048, 4096)
            assert np.array_equal(got[1], ends)
            assert np.array_equal(got[2], oracle.chunk_digests(oracle.SHA1, data, ends))


def test_chunk_requests_with_two_level_digests(ctx, hg, pool):
    host, dev = pool
    specs = [(2, 0, 1 * MiB), (0, 5, 300 * KiB), (2, 50, 2 * MiB + 3), (2, 77, 10)]
    rs = hg.RequestSet(dev.data_ptr(), True, specs, chunk_segment=1024)
    note("chunk requests with two-level chunk digests")
    with hg.Server(0, slots=2, max_requests=8, device_budget=8 * MiB, max_group_bytes=8 * MiB) as srv:
        _, sts = srv.play(rs, np.zeros(len(specs)))
    assert np.all(sts == hg.HG_OK)
    for i, (k, o, n) in enumerate(specs):
        got = rs.result(i)
        if k == 2:
            data = host[o:o + n]
            starts = oracle.window_scan(oracle.MD5, data, 20, 1, 0xFFF, 0)
            ends = oracle.chunk_select(starts, 20, n, 2048)
            assert np.array_equal(got[1], ends)
            assert np.array_equal(got[2], oracle.chunk_digests(oracle.SHA1, data, ends, 1024))


def test_grouped_chunk_requests_with_two_level_digests(ctx, hg, pool):
    host, dev = pool
    specs = [(2, 1000 * i + 3, 300 * KiB + 777 * i) for i in range(12)] + [(0, 5, 300 * KiB)]
    rs = hg.RequestSet(dev.data_ptr(), True, specs, chunk_segment=4096)
    note("grouped chunk requests with two-level chunk digests (4 KiB segments)")
    with hg.Server(0, slots=1, max_requests=16, device_budget=8 * MiB, max_group_bytes=8 * MiB) as srv:
        _, sts = srv.play(rs, np.zeros(len(specs)))
        st = srv.stats()
    assert np.all(sts == hg.HG_OK)
    assert st["groups"] < 12  # served together, not one by one
    for i, (k, o, n) in enumerate(specs):
        if k != 2:
            continue
        got = rs.result(i)
        data = host[o:o + n]
        starts = oracle.window_scan(oracle.MD5, data, 20, 1, 0xFFF, 0)
        ends = oracle.chunk_select(starts, 20, n, 2048)
        assert np.array_equal(got[1], ends)
        assert np.array_equal(got[2], oracle.chunk_digests(oracle.SHA1, data, ends, 4096))


def test_truncation_and_injected_failure(ctx, hg, pool):
    host, dev = pool
    specs = [(2, 0, 1 * MiB), (0, 5, 300 * KiB), (2, 50, 2 * MiB), (1, 9, 1 * MiB)]
    rs = hg.RequestSet(dev.data_ptr(), True, specs, fail={1})
    rs.reqs[2].capacity = 3  # far fewer than the chunks of 2 MiB
    note("truncation and injected failure")
    with hg.Server(0, slots=2, max_requests=8, device_budget=8 * MiB, max_group_bytes=8 * MiB) as srv:
        _, sts = srv.play(rs, np.zeros(len(specs)))
        st = srv.stats()
    assert sts.tolist() == [hg.HG_OK, hg.HG_EDEVICE, hg.HG_ETRUNC, hg.HG_OK]
    assert st["failed"] == 1
    full = alone(ctx, hg, dev, specs[2], rs)
    assert int(rs.n_chunks[2]) == full[1].size > 3
    assert np.array_equal(rs.ends[2][:3], full[1][:3])
    assert np.array_equal(rs.digests[2][:3], full[2][:3])
    for i in (0, 3):
        assert same(rs.result(i), alone(ctx, hg, dev, specs[i], rs))


def test_submit_wait_and_callbacks(ctx, hg, pool):
    host, dev = pool
    specs = stream_specs(8, 24, dev.numel(), hi=1 * MiB)
    rs = hg.RequestSet(dev.data_ptr(), True, specs)
    seen = {}

    @hg.HG_SERVER_CB
    def cb(rid, status, user):
        seen[int(rid)] = int(status)

    note("submit with hg_wait and with callbacks")
    with hg.Server(0, slots=2, max_requests=16, device_budget=16 * MiB, max_group_bytes=16 * MiB) as srv:
        ids = [srv.submit(rs.reqs[i]) for i in range(0, len(specs), 2)]
        cb_ids = []
        for i in range(1, len(specs), 2):
            rid = ctypes.c_uint64(0)
            assert hg.hg_submit(srv.handle, ctypes.byref(rs.reqs[i]), cb, None, ctypes.byref(rid)) == 0
            cb_ids.append(int(rid.value))
        assert all(srv.wait(r) == hg.HG_OK for r in ids)
        with pytest.raises(hg.HashGpuError):
            srv.wait(ids[0], 0)  # released by the first wait
        bad = hg.hg_request()
        bad.kind = 7
        with pytest.raises(hg.HashGpuError):
            srv.submit(bad)
    # hg_server_stop served every queued request before returning.
    assert sorted(seen) == sorted(cb_ids) and all(v == hg.HG_OK for v in seen.values())
    check_all(ctx, hg, pool, rs, np.zeros(len(specs), dtype=np.int32), sample=3, seed=2)


def test_host_payload_larger_than_budget_is_rejected(hg, pool):
    host, _ = pool
    specs = [(0, 0, 2 * MiB)]
    rs = hg.RequestSet(host.ctypes.data, False, specs)
    with hg.Server(0, slots=1, max_requests=4, device_budget=1 * MiB, max_group_bytes=1 * MiB) as srv:
        with pytest.raises(hg.HashGpuError) as e:
            srv.submit(rs.reqs[0])
        assert e.value.status == hg.HG_EBUSY
