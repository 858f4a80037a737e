"""C-ABI checks that need no GPU: the library loads, exports every function
``include/hashgpu.h`` declares, and reports missing devices and bad handles
with the documented status codes."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hashgpu.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ["hg_create", "hg_destroy", "hg_block_hash", "hg_window_scan", "hg_chunk",
                     "hg_similarity"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1202_3669_amd import hashgpu
    out = subprocess.run(["nm", "-D", "--defined-only", hashgpu.library_path()],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(hg_\w+)", out))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing
    assert sorted(hashgpu.EXPORTED) == sorted(_declared_functions())


def test_struct_layouts_match_the_header(tmp_path):
    # The ctypes mirrors of the header's structs: every field at the offset
    # and every struct of the size a C compiler gives them.
    from paper_1202_3669_amd import hashgpu as hg
    structs = [hg.hg_chunk_params, hg.hg_block_job, hg.hg_batch_params, hg.hg_batch_out, hg.hg_request,
               hg.hg_server_cfg, hg.hg_server_stats, hg.hg_ctx_stats]
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    expect = []
    for cls in structs:
        c = cls.__name__
        lines.append(f'printf("%zu\\n", sizeof({c}));')
        expect.append(ctypes.sizeof(cls))
        for f in cls._fields_:
            name = "in" if f[0] == "in_" else f[0]
            lines.append(f'printf("%zu\\n", offsetof({c}, {name}));')
            expect.append(getattr(cls, f[0]).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect


def test_status_text_and_digest_sizes():
    from paper_1202_3669_amd import hashgpu as hg
    assert hg.hg_strerror(hg.HG_OK) == b"ok"
    assert hg.hg_strerror(hg.HG_ETRUNC) == b"output truncated"
    assert hg.hg_digest_size(hg.HG_MD5) == 16
    assert hg.hg_digest_size(hg.HG_SHA1) == 20
    assert hg.hg_digest_size(7) == hg.HG_EINVAL


def test_null_context_is_rejected():
    from paper_1202_3669_amd import hashgpu as hg
    cnt = ctypes.c_uint64(0)
    assert hg.hg_block_hash(None, None, 0, 64, hg.HG_MD5, None, None, 0, None) == hg.HG_EINVAL
    assert hg.hg_window_scan(None, None, 0, 20, 1, 0, 0, hg.HG_MD5, None, 0,
                             ctypes.addressof(cnt), 0, None) == hg.HG_EINVAL
    assert hg.hg_last_error(None, None, 0) == hg.HG_EINVAL
    p = hg.hg_chunk_params(20, 1, 0xFFF, 0, 2048, 0, hg.HG_MD5, hg.HG_SHA1, 0)
    assert hg.hg_chunk(None, None, 0, ctypes.byref(p), None, 0, ctypes.addressof(cnt), None, 0,
                       None) == hg.HG_EINVAL
    assert hg.hg_similarity(None, None, 0, None, None, 0, hg.HG_SHA1, ctypes.addressof(cnt), None, 0,
                            None) == hg.HG_EINVAL
    assert hg.hg_similarity_n(None, None, 0, None, None, ctypes.addressof(cnt), 0, hg.HG_SHA1,
                              ctypes.addressof(cnt), None, 0, None) == hg.HG_EINVAL
    assert hg.hg_chunk_select(None, None, ctypes.addressof(cnt), 0, 0, 20, 0, 0, None, 1,
                              ctypes.addressof(cnt), 0, None) == hg.HG_EINVAL
    assert hg.hg_chunk_digests(None, None, 0, None, ctypes.addressof(cnt), 0, hg.HG_SHA1, 0, None, 0,
                               None) == hg.HG_EINVAL
    assert hg.hg_block_hash_dual(None, None, 0, 64, None, None, None, None, 0, None) == hg.HG_EINVAL
    h = ctypes.c_void_p()
    assert hg.hg_chunker_create(None, ctypes.byref(p), ctypes.byref(h)) == hg.HG_EINVAL
    assert hg.hg_blockmap_create(None, hg.HG_SHA1, 16, ctypes.byref(h)) == hg.HG_EINVAL
    hg.hg_destroy(None)  # no-op


def test_create_without_gpu_reports_edevice():
    # Runs in a child so that the HIP runtime of this process stays untouched.
    code = (
        "import ctypes, sys\n"
        "from paper_1202_3669_amd import hashgpu as hg\n"
        "import torch\n"
        "if torch.cuda.device_count() > 0: sys.exit(3)\n"
        "h = ctypes.c_void_p()\n"
        "sys.exit(0 if hg.hg_create(0, 0, 0, ctypes.byref(h)) == hg.HG_EDEVICE else 1)\n"
    )
    r = subprocess.run(["python", "-c", code], cwd=ROOT, capture_output=True, text=True)
    if r.returncode == 3:
        pytest.skip("a GPU is present")
    assert r.returncode == 0, r.stderr


def test_server_argument_checks():
    from paper_1202_3669_amd import hashgpu as hg
    h = ctypes.c_void_p()
    assert hg.hg_server_start(0, None, ctypes.byref(h)) == hg.HG_EINVAL
    for bad in (hg.hg_server_cfg(0, 16, 1 << 20, 1 << 20, 0, 0),        # no workers
                hg.hg_server_cfg(2, 0, 1 << 20, 1 << 20, 0, 0),        # no requests per group
                hg.hg_server_cfg(2, 16, 0, 1 << 20, 0, 0),             # no staging budget
                hg.hg_server_cfg(2, 16, 1 << 20, 1 << 19, 0, 0),       # group under 1 MiB
                hg.hg_server_cfg(2, 16, 1 << 20, 1 << 20, 1, 0)):      # unknown flag
        assert hg.hg_server_start(0, ctypes.byref(bad), ctypes.byref(h)) == hg.HG_EINVAL
    rid = ctypes.c_uint64(0)
    req = hg.hg_request()
    assert hg.hg_submit(None, ctypes.byref(req), hg.HG_SERVER_CB(), None, ctypes.byref(rid)) == hg.HG_EINVAL
    assert hg.hg_wait(None, 1, 0, None) == hg.HG_EINVAL
    assert hg.hg_server_play(None, None, None, 0, None, None) == hg.HG_EINVAL
    assert hg.hg_server_stats_read(None, None) == hg.HG_EINVAL
    assert hg.hg_server_stats_reset(None) == hg.HG_EINVAL
    assert hg.hg_server_stop(None) == hg.HG_EINVAL


def test_server_start_without_gpu_reports_edevice():
    code = (
        "import ctypes, sys\n"
        "from paper_1202_3669_amd import hashgpu as hg\n"
        "import torch\n"
        "if torch.cuda.device_count() > 0: sys.exit(3)\n"
        "h = ctypes.c_void_p()\n"
        "cfg = hg.hg_server_cfg(2, 16, 1 << 20, 1 << 20, 0, 0)\n"
        "sys.exit(0 if hg.hg_server_start(0, ctypes.byref(cfg), ctypes.byref(h)) == hg.HG_EDEVICE else 1)\n"
    )
    r = subprocess.run(["python", "-c", code], cwd=ROOT, capture_output=True, text=True)
    if r.returncode == 3:
        pytest.skip("a GPU is present")
    assert r.returncode == 0, r.stderr
