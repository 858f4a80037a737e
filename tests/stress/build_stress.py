"""Builds the serving-loop stress driver (server_stress.cpp plus the
library sources, with hipcc for gfx950) into tests/stress/_build, unless
the cached binary matches a hash of the sources."""
import glob
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
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


def build(force=False):
    """Returns the driver's path, building it if needed (or if force)."""
    stamp = os.path.join(BUILD, "sources.sha256")
    want = source_hash()
    if not force and os.path.exists(EXE) and os.path.exists(stamp) and open(stamp).read().strip() == want:
        return EXE
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    sys.path.insert(0, os.path.join(ROOT, "paper_1202_3669_amd"))
    import build as hgbuild
    os.makedirs(BUILD, exist_ok=True)
    units = [p for p in sources() if p.endswith((".hip", ".cpp"))]
    r = subprocess.run([hipcc, *hgbuild.HIPFLAGS, "-o", EXE + ".tmp", *units], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for the stress driver:\n" + r.stderr[-4000:])
    os.replace(EXE + ".tmp", EXE)
    with open(stamp, "w") as f:
        f.write(want + "\n")
    return EXE
