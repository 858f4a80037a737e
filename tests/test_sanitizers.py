"""Sanitizer runs of host code (no GPU).

* The oracle (``oracle/oracle.c``) built with AddressSanitizer and
  UndefinedBehaviorSanitizer (every report fatal) runs its whole pin suite
  in a child Python process with the ASan runtime preloaded.
* The library's host hashing and host thread pool (``host_hash.cpp``, the
  host side of the second level) built with ASan + UBSan, and with
  ThreadSanitizer, under a driver that prints digests of every length
  0-1100 and large ones (checked here against ``hashlib``, on both SHA-1
  paths) and runs the pool from eight caller threads at once.
* The serving loop's host logic (``server.cpp``: queue, staging admission,
  group formation, worker hand-off, waits, callbacks, statistics, stop)
  built over a stub device layer (``tests/sanitize/stub``, device memory =
  host memory) with TSan, and with ASan + UBSan, under a driver with several
  submitter threads; each request's status and outputs are checked.
"""
import hashlib
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1202_3669_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_hash_driver.cpp")
GXX = shutil.which("g++")
GCC = shutil.which("gcc")


def _runtime(name):
    p = subprocess.run([GCC, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(GCC is None or _runtime("libasan.so") is None, reason="gcc with ASan runtime needed")
def test_oracle_pin_suite_under_asan_ubsan(tmp_path):
    so = tmp_path / "liboracle_asan.so"
    subprocess.run([GCC, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-shared", "-fPIC", "-o", str(so),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import oracle\n"
            "oracle._swap_library(%r)\n"
            "from tests import test_oracle_mutations as m\n"
            "m._pin_suite()\n"
            "print('pins ok')\n") % (ROOT, str(so))
    env = dict(os.environ, LD_PRELOAD=_runtime("libasan.so"),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, cwd=ROOT,
                       timeout=900)
    assert r.returncode == 0 and "pins ok" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr


def _build_driver(tmp_path, name, flags):
    exe = tmp_path / name
    subprocess.run([GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-I", CSRC, "-o", str(exe),
                    DRIVER, os.path.join(CSRC, "host_hash.cpp"), "-pthread"], check=True)
    return exe


def _check_digests(stdout):
    data = bytearray()
    x = 12345
    for _ in range((1 << 20) + 64):
        x ^= (x << 13) & 0xFFFFFFFF
        x ^= x >> 17
        x ^= (x << 5) & 0xFFFFFFFF
        data.append(x & 0xFF)
    data = bytes(data)
    n_lines = 0
    for line in stdout.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[0] in ("0", "1"):
            kind, n, hexd = int(parts[0]), int(parts[1]), parts[2]
            ref = (hashlib.md5 if kind == 0 else hashlib.sha1)(data[:n]).hexdigest()
            assert hexd == ref, (kind, n)
            n_lines += 1
    assert n_lines == 2 * (1101 + 5)
    assert "pool ok" in stdout


@pytest.mark.skipif(GXX is None or _runtime("libasan.so") is None, reason="g++ with ASan runtime needed")
@pytest.mark.parametrize("portable", [False, True])
def test_host_hash_under_asan_ubsan(tmp_path, portable):
    exe = _build_driver(tmp_path, "hh_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    if portable:
        env["HG_HOST_SHA1_PORTABLE"] = "1"
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    _check_digests(r.stdout)


@pytest.mark.skipif(GXX is None or _runtime("libtsan.so") is None, reason="g++ with TSan runtime needed")
def test_host_pool_under_tsan(tmp_path):
    exe = _build_driver(tmp_path, "hh_tsan", ["-fsanitize=thread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    _check_digests(r.stdout)


def _build_server_driver(tmp_path, name, flags):
    exe = tmp_path / name
    stub = os.path.join(ROOT, "tests", "sanitize")
    subprocess.run([GXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags,
                    "-I", os.path.join(stub, "stub"), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    "-o", str(exe), os.path.join(stub, "server_tsan_driver.cpp"),
                    os.path.join(stub, "server_stub_device.cpp"), os.path.join(CSRC, "server.cpp"),
                    os.path.join(CSRC, "host_hash.cpp"), "-pthread"],
                   check=True)
    return exe


@pytest.mark.skipif(GXX is None or _runtime("libtsan.so") is None, reason="g++ with TSan runtime needed")
def test_server_host_logic_under_tsan(tmp_path):
    # The serving loop (server.cpp) over a stub device layer: submitters,
    # waiters, callbacks, a load replay, a statistics reader, injected
    # failures, staging admission and a stop with requests queued.
    exe = _build_server_driver(tmp_path, "srv_tsan", ["-fsanitize=thread"])
    r = subprocess.run([str(exe)], env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"), capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0 and "WARNING: ThreadSanitizer" not in r.stderr, (r.stdout + r.stderr)[-4000:]
    assert "server tsan driver: ok" in r.stdout


@pytest.mark.skipif(GXX is None or _runtime("libasan.so") is None, reason="g++ with ASan runtime needed")
def test_server_host_logic_under_asan_ubsan(tmp_path):
    exe = _build_server_driver(tmp_path, "srv_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    r = subprocess.run([str(exe)], env=dict(os.environ, ASAN_OPTIONS="abort_on_error=1"), capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "server tsan driver: ok" in r.stdout
