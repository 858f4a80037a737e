"""Thread-sanitizer run of the serving loop's host code on the GPU: the
stress driver tests/tsan/server_stress.cpp (four submitter threads,
callbacks and waiters, injected failures, a concurrent statistics reader, a
stop with requests queued; every result checked against the single call) is
built with -fsanitize=thread on the host side only and must finish with no
report.  The build is cached under tests/tsan/_build, keyed by a hash of the
sources."""
import hashlib
import glob
import os
import shutil
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TSAN = os.path.join(ROOT, "tests", "tsan")
BUILD = os.path.join(TSAN, "_build")
EXE = os.path.join(BUILD, "server_stress")


def sources():
    csrc = os.path.join(ROOT, "paper_1202_3669_amd", "csrc")
    return sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.cpp")) +
                  glob.glob(os.path.join(csrc, "*.hpp")) + [os.path.join(ROOT, "include", "hashgpu.h"),
                                                            os.path.join(TSAN, "server_stress.cpp")])


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
    cmd = [hipcc, *hgbuild.HIPFLAGS, "-g", "-Xarch_host", "-fsanitize=thread", "-o", EXE + ".tmp", *units]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    os.replace(EXE + ".tmp", EXE)
    with open(stamp, "w") as f:
        f.write(want + "\n")
    return EXE


def test_server_host_code_is_race_free():
    exe = build()
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = ("halt_on_error=1:exitcode=66:second_deadlock_stack=1:"
                           f"suppressions={os.path.join(TSAN, 'suppressions.txt')}")
    print("[case] tsan server stress", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert "server stress ok" in r.stdout
