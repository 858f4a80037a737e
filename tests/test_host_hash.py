"""The library's host-side MD5 / SHA-1 (hg_host_hash, no GPU): the routine
that computes the last step of direct hashing on the host (Sec. 3.2.2).
Pinned against Python's hashlib (OpenSSL, an independent implementation)
on every length 0-1100, the padding edges and large messages, for SHA-1 on
both the SHA-extension path and the portable path (the latter selected by
HG_HOST_SHA1_PORTABLE in a child process)."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1202_3669_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
H = {0: hashlib.md5, 1: hashlib.sha1}
LENGTHS = list(range(0, 1101)) + [4095, 4096, 4097, 65536, 65537, (1 << 20) + 13]


def _check_all(hg):
    data = inputs.uniform_bytes(41, (1 << 20) + 64).tobytes()
    for kind in (0, 1):
        for n in LENGTHS:
            assert hg.host_hash(kind, data[:n]) == H[kind](data[:n]).digest(), (kind, n)
        a = b"a" * 1_000_000
        assert hg.host_hash(kind, a) == H[kind](a).digest()


def test_host_hash_vs_hashlib():
    from paper_1202_3669_amd import hashgpu as hg
    _check_all(hg)


def test_host_hash_portable_sha1_vs_hashlib():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from tests import test_host_hash as t\n"
            "from paper_1202_3669_amd import hashgpu as hg\n"
            "t._check_all(hg)\nprint('ok')\n") % ROOT
    env = dict(os.environ, HG_HOST_SHA1_PORTABLE="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]


def test_host_hash_rejects_bad_arguments():
    from paper_1202_3669_amd import hashgpu as hg
    out = (hg.ctypes.c_uint8 * 20)()
    assert hg.hg_host_hash(2, None, 0, hg.ctypes.addressof(out)) == hg.HG_EINVAL
    assert hg.hg_host_hash(0, None, 5, hg.ctypes.addressof(out)) == hg.HG_EINVAL
    assert hg.hg_host_hash(1, None, 0, None) == hg.HG_EINVAL
    assert hg.hg_host_hash(1, None, 0, hg.ctypes.addressof(out)) == hg.HG_OK
    assert bytes(out) == hashlib.sha1(b"").digest()
