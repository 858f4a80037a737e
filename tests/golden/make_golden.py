"""Writes the stored expected values of the small workload (4 MiB of
default_rng(1) bytes) from the oracle, after checking every value against an
independent reference (Python's hashlib for the digests, a per-offset
hashlib scan for the window candidates).

Run from the repository root:  python tests/golden/make_golden.py
Output: tests/golden/small_4MiB_seed1.json

What is stored (the direct hash of Sec. 3.2.2 and the window scan of the
content-based chunking of Sec. 2.1 / Fig. 3, in the readings the oracle
documents):
  - MD5 and SHA-1 segment digests and second-level digests at 64 KiB
    segments;
  - window-start offsets of MD5 windows, w = 20, stride 1, whose first four
    digest bytes read little-endian have low 12 bits 0;
  - chunk ends and SHA-1 chunk digests with a 2 KiB minimum chunk.
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1202_3669_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_4MiB_seed1.json")
B, W, S, MASK, MIN = 64 * 1024, 20, 1, 0xFFF, 2048


def main():
    data = inputs.uniform_bytes(1, 4 << 20)
    raw = data.tobytes()
    rec = {"workload": "default_rng(1).integers(0, 256, 4 MiB, uint8)", "segment": B, "window": W,
           "stride": S, "mask": MASK, "target": 0, "min_chunk": MIN}
    for kind, name, h in ((oracle.MD5, "md5", hashlib.md5), (oracle.SHA1, "sha1", hashlib.sha1)):
        lv = oracle.leaves(kind, data, B)
        ref = [h(raw[k * B:(k + 1) * B]).digest() for k in range((len(raw) + B - 1) // B)]
        assert [bytes(x) for x in lv] == ref, name
        root = oracle.root(kind, lv)
        assert root == h(b"".join(ref)).digest(), name
        rec[f"{name}_leaves"] = [x.hex() for x in ref]
        rec[f"{name}_root"] = root.hex()
    starts = oracle.window_scan(oracle.MD5, data, W, S, MASK, 0)
    ref = [i for i in range(0, len(raw) - W + 1, S)
           if int.from_bytes(hashlib.md5(raw[i:i + W]).digest()[:4], "little") & MASK == 0]
    assert starts.tolist() == ref
    rec["window_starts"] = ref
    ends = oracle.chunk_select(starts, W, len(raw), MIN)
    last, ref_ends = 0, []
    for i in ref:
        e = i + W
        if e < len(raw) and e - last >= MIN:
            ref_ends.append(e)
            last = e
    ref_ends.append(len(raw))
    assert ends.tolist() == ref_ends
    dig = oracle.chunk_digests(oracle.SHA1, data, ends)
    prev = 0
    ref_dig = []
    for e in ref_ends:
        ref_dig.append(hashlib.sha1(raw[prev:e]).digest())
        prev = e
    assert [bytes(x) for x in dig] == ref_dig
    rec["chunk_ends"] = ref_ends
    rec["chunk_sha1"] = [x.hex() for x in ref_dig]
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=0)
        f.write("\n")
    print(f"wrote {OUT}: {len(rec['window_starts'])} window starts, {len(ref_ends)} chunks")


if __name__ == "__main__":
    main()
