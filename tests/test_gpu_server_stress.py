"""Multi-threaded stress of the serving loop through the C ABI alone: the
driver tests/stress/server_stress.cpp (four submitter threads, callbacks
and waiters mixed, injected failures, a concurrent statistics reader, a stop
with requests still queued) checks every served result against the single
call on its own context.  The driver is built with hipcc and cached under
tests/stress/_build, keyed by a hash of the sources (tests/stress/build_stress.py;
__graft_entry__.build() builds it too).

(Built with ThreadSanitizer on the host side, the HIP runtime does not
initialise on these machines -- the sanitizer's address-space layout and the
runtime's reservations collide -- so the driver runs uninstrumented.)"""
import os
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "stress"))
from build_stress import build  # noqa: E402

pytestmark = pytest.mark.gpu


def test_server_under_concurrent_submitters():
    exe = build()
    print("[case] server stress driver", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "server stress ok" in r.stdout
