"""Group formation of the serving loop (no GPU).

``server.cpp`` built over the stub device layer (``tests/sanitize/stub``)
with AddressSanitizer and UndefinedBehaviorSanitizer, under a driver that
holds the one worker inside a request served alone while seven more queue
behind it, then checks the groups from the order of the callbacks: a group
takes the head's kind (block or chunk); device requests of the other kind
and a chunk request served alone for its size stay queued for the next
group; a host payload of the group's kind joins it.  Strict arrival order
(the group closed at the first request that does not join) gives another
order, which the driver reports as wrong.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1202_3669_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
GXX = shutil.which("g++")


@pytest.mark.skipif(GXX is None, reason="g++ needed")
def test_groups_hold_one_kind_and_pass_over_requests_served_alone(tmp_path):
    exe = tmp_path / "formation"
    subprocess.run([GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(SAN, "stub"), "-I",
                    os.path.join(ROOT, "include"), "-I", CSRC, "-o", str(exe),
                    os.path.join(SAN, "server_formation_driver.cpp"), os.path.join(SAN, "server_stub_device.cpp"),
                    os.path.join(CSRC, "server.cpp"), os.path.join(CSRC, "host_hash.cpp"), "-pthread"],
                   check=True)
    r = subprocess.run([str(exe)], env=dict(os.environ, ASAN_OPTIONS="abort_on_error=1"), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "order: 0 1 3 5 7 2 6 4" in r.stdout
    assert "groups: 4" in r.stdout
    assert "server formation driver: ok" in r.stdout
