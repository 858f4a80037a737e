"""GPU parity of the serving loop at the serving workload's full sizes: the
request stream the benchmark serves (seed 6: 2000 requests, log-normal
sizes 4 KiB-256 MiB with median 1 MiB and sigma 1.85, mix 50% block SHA-1 /
30% block MD5 with 64 KiB segments and second levels / 20% chunking with
MD5 w=20, stride 1, low 12 bits, min 2 KiB, SHA-1 chunk digests), payloads
sliced from the 1 GiB input (seed 2) at the benchmark's seeded offsets,
through a server configured as the benchmark's (6 workers, 2048 requests
and 2 GiB per group, 4 GiB of staging).  Every request's outputs equal the
same request run alone through the single-call entry points, bit for bit,
with device payloads in a burst and with pinned host payloads at Poisson
arrivals; the oracle checks a seeded sample that includes the largest
request of each kind."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1202_3669_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30
THREADS = max(1, min(16, os.cpu_count() or 1))
N_REQ = 2000


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hg():
    from paper_1202_3669_amd import hashgpu
    return hashgpu


@pytest.fixture(scope="module")
def workload():
    host = inputs.uniform_bytes(2, GiB)
    arr1, sizes, kinds = inputs.request_stream(6, N_REQ, 1.0)
    rng = np.random.default_rng(6 + 1000)
    offs = np.array([int(rng.integers(0, host.size - int(z) + 1)) for z in sizes])
    specs = list(zip(kinds.tolist(), offs.tolist(), sizes.tolist()))
    return host, torch.from_numpy(host).cuda(), arr1, specs


def _alone(ctx, hg, dev, spec):
    k, o, n = spec
    view = dev[o:o + n]
    if k in (0, 1):
        lv, rt = ctx.block_hash(view, 64 * KiB, hg.HG_SHA1 if k == 0 else hg.HG_MD5)
        return ("block", lv.cpu().numpy(), bytes(rt.cpu().numpy()))
    ends, dig = ctx.chunk(view, 20, 1, 0xFFF, 0, 2048)
    return ("chunk", ends.cpu().numpy().astype(np.uint64), dig.cpu().numpy())


def _oracle(host, spec):
    k, o, n = spec
    data = host[o:o + n]
    if k in (0, 1):
        kind = oracle.SHA1 if k == 0 else oracle.MD5
        lv = oracle.leaves_sharded(kind, data, 64 * KiB, THREADS)
        return ("block", lv, oracle.root(kind, lv))
    _, ends, dig = oracle.chunk(oracle.MD5, oracle.SHA1, data, 20, 1, 0xFFF, 0, 2048, THREADS)
    return ("chunk", ends, dig)


def _same(a, b):
    return a[0] == b[0] and np.array_equal(a[1], b[1]) and (
        a[2] == b[2] if a[0] == "block" else np.array_equal(a[2], b[2]))


def _check(hg, host, dev, rs, sts, idx, seed):
    assert np.all(sts == hg.HG_OK), np.unique(sts, return_counts=True)
    with hg.Context(0) as ctx:
        for i in range(len(rs)):
            assert _same(rs.result(i), _alone(ctx, hg, dev, rs.specs[i])), f"request {idx[i]} differs from alone"
    # oracle: the largest request of each kind and a seeded sample
    sample = set()
    for k in (0, 1, 2):
        ks = [i for i, s in enumerate(rs.specs) if s[0] == k]
        if ks:
            sample.add(max(ks, key=lambda i: rs.specs[i][2]))
    rng = np.random.default_rng(seed)
    sample |= set(rng.choice(len(rs), size=min(6, len(rs)), replace=False).tolist())
    for i in sorted(sample):
        note(f"oracle check of request {idx[i]} {rs.specs[i]}")
        assert _same(rs.result(i), _oracle(host, rs.specs[i])), f"request {idx[i]} vs oracle"


def test_full_stream_device_payloads_burst(hg, workload):
    host, dev, _, specs = workload
    sizes = [s[2] for s in specs]
    assert min(sizes) == 4 * KiB and max(sizes) == 256 * MiB  # the stream spans the whole size range
    rs = hg.RequestSet(dev.data_ptr(), True, specs)
    note(f"serving {len(specs)} requests ({sum(sizes) / 1e9:.2f} GB), burst, device payloads")
    with hg.Server(0, slots=6, max_requests=2048, device_budget=4 * GiB, max_group_bytes=2 * GiB) as srv:
        lat, sts = srv.play(rs, np.zeros(len(specs)))
        st = srv.stats()
    assert st["completed"] == len(specs) and st["failed"] == 0
    assert st["groups"] < len(specs) // 10, "requests were not batched"
    _check(hg, host, dev, rs, sts, list(range(len(specs))), 1)


def test_stream_slice_pinned_host_payloads_poisson(hg, workload):
    host, dev, arr1, specs = workload
    # a slice of the stream that holds its largest request
    big = max(range(len(specs)), key=lambda i: specs[i][2])
    lo = max(0, min(big - 150, len(specs) - 400))
    idx = list(range(lo, lo + 400))
    sub = [specs[i] for i in idx]
    pinned = torch.from_numpy(host).pin_memory()
    rs = hg.RequestSet(pinned.data_ptr(), False, sub)
    # arrivals at about half the rate the copy link allows (~25 GB/s)
    total = sum(s[2] for s in sub)
    arr = (arr1[lo:lo + 400] - arr1[lo]) * (total / len(sub)) / 25e9
    note(f"serving {len(sub)} requests with host payloads, Poisson arrivals over {arr[-1]:.2f} s")
    with hg.Server(0, slots=6, max_requests=2048, device_budget=4 * GiB, max_group_bytes=2 * GiB) as srv:
        lat, sts = srv.play(rs, arr)
        st = srv.stats()
    assert st["completed"] == len(sub) and st["failed"] == 0
    _check(hg, host, dev, rs, sts, idx, 2)
    del pinned
