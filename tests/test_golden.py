"""Stored expected values of the small workload (tests/golden/, written by
tests/golden/make_golden.py from the oracle after a hashlib cross-check):
the oracle must keep reproducing them, and the GPU path must match them."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1202_3669_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_4MiB_seed1.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def data():
    return inputs.uniform_bytes(1, 4 << 20)


def test_oracle_reproduces_golden(gold, data):
    B = gold["segment"]
    for kind, name in ((oracle.MD5, "md5"), (oracle.SHA1, "sha1")):
        lv = oracle.leaves(kind, data, B)
        assert [bytes(x).hex() for x in lv] == gold[f"{name}_leaves"]
        assert oracle.root(kind, lv).hex() == gold[f"{name}_root"]
    starts = oracle.window_scan(oracle.MD5, data, gold["window"], gold["stride"], gold["mask"], gold["target"])
    assert starts.tolist() == gold["window_starts"]
    ends = oracle.chunk_select(starts, gold["window"], data.size, gold["min_chunk"])
    assert ends.tolist() == gold["chunk_ends"]
    dig = oracle.chunk_digests(oracle.SHA1, data, ends)
    assert [bytes(x).hex() for x in dig] == gold["chunk_sha1"]


@pytest.mark.gpu
def test_gpu_path_matches_golden(gold, data):
    torch = pytest.importorskip("torch")
    from paper_1202_3669_amd import hashgpu as hg
    d = torch.from_numpy(data).cuda()
    with hg.Context(0) as ctx:
        for kind, name in ((hg.HG_MD5, "md5"), (hg.HG_SHA1, "sha1")):
            lv, rt = ctx.block_hash(d, gold["segment"], kind)
            assert [bytes(x).hex() for x in lv.cpu().numpy()] == gold[f"{name}_leaves"]
            assert bytes(rt.cpu().numpy()).hex() == gold[f"{name}_root"]
        starts = ctx.window_scan(d, gold["window"], gold["stride"], gold["mask"], gold["target"])
        assert starts.cpu().numpy().tolist() == gold["window_starts"]
        ends, dig = ctx.chunk(d, gold["window"], gold["stride"], gold["mask"], gold["target"], gold["min_chunk"])
        assert ends.cpu().numpy().tolist() == gold["chunk_ends"]
        assert [bytes(x).hex() for x in dig.cpu().numpy()] == gold["chunk_sha1"]
