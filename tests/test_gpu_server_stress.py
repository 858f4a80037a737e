"""Multi-threaded stress of the serving loop through the C ABI alone: the
driver tests/stress/server_stress.cpp (four submitter threads, callbacks
and waiters mixed, injected failures, a concurrent statistics reader, a stop
with requests still queued) checks every served result against the single
call on its own context.  The driver is built with hipcc and cached under
tests/stress/_build, keyed by a hash of the sources.

(Built with ThreadSanitizer on the host side, the HIP runtime does not
initialise on these machines -- the sanitizer's address-space layout and the
runtime's reservations collide -- so the driver runs uninstrumented.)"""
import glob
import hashlib
import os
import shutil
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "stress")
BUILD = os.path.join(HERE, "_build")
EXE = os.path.join(BUILD, "server_stress")


def sources():
    csrc = os.path.join(ROOT, "paper_1202_3669_amd", "csrc")
    return sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.cpp")) +
                  glob.glob(os.path.join(csrc, "*.hpp")) + [os.path.join(ROOT, "include", "hashgpu.h"),
                                                            os.path.join(HERE, "server_stress.cpp")])


def source_hash():
    h = hashlib.sha256()
    for p in sources():
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def build():
    """Builds the driver unless the cached one matches the sources."""
    stamp = os.path.join(BUILD, "sources.sha256")
    want = source_hash()
    if os.path.exists(EXE) and os.path.exists(stamp) and open(stamp).read().strip() == want:
        return EXE
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    sys.path.insert(0, os.path.join(ROOT, "paper_1202_3669_amd"))
    import build as hgbuild
    os.makedirs(BUILD, exist_ok=True)
    units = [p for p in sources() if p.endswith((".hip", ".cpp"))]
    r = subprocess.run([hipcc, *hgbuild.HIPFLAGS, "-o", EXE + ".tmp", *units], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    os.replace(EXE + ".tmp", EXE)
    with open(stamp, "w") as f:
        f.write(want + "\n")
    return EXE


def test_server_under_concurrent_submitters():
    exe = build()
    print("[case] server stress driver", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "server stress ok" in r.stdout
