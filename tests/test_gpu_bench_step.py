"""GPU parity of the timed step itself: bench.py's pipeline (the 1 GiB
input, seed 2, resident in HBM; six direct hashes through the persistent
job tables, the 1 MiB segments in a launch of their own per step, the
second levels on the host's cores, chunking round-robin over its chunking
streams, similarity against the previous version's digests) run for more
steps than its ring of output slots holds, in both chunking modes.  Every
slot's segment digests and second levels, the chunk ends and digests of
each chunking stream and every step's similarity equal the oracle's,
computed from the same seeded input on the host cores."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1202_3669_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

THREADS = max(1, min(16, os.cpu_count() or 1))
KiB, GiB = 1 << 10, 1 << 30


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hg():
    from paper_1202_3669_amd import hashgpu
    return hashgpu


@pytest.fixture(scope="module")
def workload():
    note("oracle: the step's expected outputs on the 1 GiB workload")
    data = inputs.uniform_bytes(2, GiB)
    prev, _ = inputs.edited_version(data, 3, 1024)
    _, _, prev_dig = oracle.chunk(oracle.MD5, oracle.SHA1, prev, 20, 1, 0xFFF, 0, 2 * KiB, THREADS)
    del prev
    _, ends, dig = oracle.chunk(oracle.MD5, oracle.SHA1, data, 20, 1, 0xFFF, 0, 2 * KiB, THREADS)
    sim = oracle.similarity(oracle.SHA1, prev_dig, dig, np.diff(ends, prepend=np.uint64(0)))
    leaves, roots = [], []
    for k, b in bench.BLOCK_JOBS:
        lv = oracle.leaves_sharded(k, data, b, THREADS)
        leaves.append(lv)
        roots.append(oracle.root(k, lv))
    return data, prev_dig, ends, dig, sim, leaves, roots


@pytest.mark.parametrize("mode,slots,steps", [("single", 10, 23), ("stages", 4, 11)])
def test_pipeline_step_outputs(hg, workload, monkeypatch, mode, slots, steps):
    data_np, prev_dig, ends, dig, sim, leaves, roots = workload
    monkeypatch.setattr(bench, "CHUNK_CALLS", mode)
    note(f"bench pipeline mode={mode} slots={slots} steps={steps}")
    data = torch.from_numpy(data_np).cuda()
    pipe = bench.Pipeline(torch, hg, data, torch.from_numpy(prev_dig).cuda(), slots)
    pipe.sim.fill_(-1)
    torch.cuda.synchronize()
    pipe.run(0, steps)
    torch.cuda.synchronize()
    assert steps > pipe.slots  # the ring of output slots is reused
    try:
        for slot in range(pipe.slots):
            _, lv, rt = pipe.recs[slot]
            for j, (k, b) in enumerate(bench.BLOCK_JOBS):
                assert np.array_equal(lv[j].cpu().numpy(), leaves[j]), f"slot {slot} job {(k, b)} segments"
                assert bytes(rt[j].cpu().numpy()) == roots[j], f"slot {slot} job {(k, b)} second level"
            assert tuple(pipe.sim[slot].tolist()) == sim, f"slot {slot} similarity"
        counts = [int(c.item()) for c in pipe.nch] if mode == "stages" else [pipe.nchunks] * pipe.NA
        for p in range(pipe.NA):
            assert counts[p] == ends.size, f"stream {p} chunk count"
            assert np.array_equal(pipe.ends[p][:ends.size].cpu().numpy().astype(np.uint64), ends), f"stream {p}"
            assert np.array_equal(pipe.digs[p][:ends.size].cpu().numpy(), dig), f"stream {p} digests"
    finally:
        pipe.close()
