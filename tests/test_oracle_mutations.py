"""The oracle's pins catch plausible mistakes (no GPU).

Each case copies ``oracle/oracle.c``, plants one mistake (a wrong index, a
dropped term, a swapped byte order, an off-by-one), builds the copy with gcc
into a temporary library, binds the oracle wrappers to it and runs the pin
checks of ``test_oracle``: at least one of them must fail.  The unmodified
source must pass the same checks.
"""
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTATIONS = {
    "md5_round2_index": ("k = (1 + 5 * i) % 16;", "k = (5 * i) % 16;"),
    "md5_rotation": ("{5, 9, 14, 20}", "{5, 9, 14, 21}"),
    "md5_I_function": ("f = c ^ (b | ~d);", "f = c ^ (b | d);"),
    "md5_sine_index": ("sin((double)(i + 1))", "sin((double)i)"),
    "md5_length_byte_order": ("if (kind == ORACLE_MD5) lenp[j] = (uint8_t)(bits >> (8 * j));",
                              "if (kind == ORACLE_MD5) lenp[7 - j] = (uint8_t)(bits >> (8 * j));"),
    "sha1_schedule_rotate": ("W[t - 14] ^ W[t - 16], 1);", "W[t - 14] ^ W[t - 16], 0);"),
    "sha1_maj_as_parity": ("f = (b & c) ^ (b & d) ^ (c & d);", "f = b ^ c ^ d;"),
    "sha1_rotl30": ("c = rotl32(b, 30);", "c = rotl32(b, 2);"),
    "sha1_constant": ("{2.0, 3.0, 5.0, 10.0}", "{2.0, 3.0, 5.0, 7.0}"),
    "padding_threshold": ("int nblk = rem < 56 ? 1 : 2;", "int nblk = rem < 55 ? 1 : 2;"),
    "leaf_count_drops_tail": ("return (len + block - 1) / block;", "return len / block;"),
    "root_short_digests": ("return oracle_hash(kind, leaves, n * (uint64_t)d, out);",
                           "return oracle_hash(kind, leaves, n * (uint64_t)(d - 1), out);"),
    "window_predicate_big_endian": ("if ((load_le32(D) & mask) == target) {",
                                    "if ((load_be32(D) & mask) == target) {"),
    "window_count_off_by_one": ("return (len - w) / s + 1;", "return (len - w) / s;"),
    "greedy_strict_min": ("if (e > last && e - last >= min_chunk && e < len) {",
                          "if (e > last && e - last > min_chunk && e < len) {"),
    "greedy_cut_at_len": ("if (e > last && e - last >= min_chunk && e < len) {",
                          "if (e > last && e - last >= min_chunk && e <= len) {"),
    "greedy_last_not_updated": ("            last = e;\n", "\n"),
    "chunk_start_off_by_one": ("        start = ends[j];\n", "        start = ends[j] - 1;\n"),
    "forced_cut_long": ("            last += max_chunk;\n", "            last += max_chunk + 1;\n"),
    "forced_cut_ignores_min": ("        while (j < n && starts[j] + w < last + step) j++;",
                               "        while (j < n && starts[j] + w <= last) j++;"),
    "max_checked_with_ge": ("if (max_chunk != 0 && next - last > max_chunk) {",
                            "if (max_chunk != 0 && next - last >= max_chunk) {"),
    "similarity_bytes_wrong_index": ("if (len_b) bytes += len_b[j];",
                                     "if (len_b) bytes += len_b[0];"),
    "blockmap_repeat_in_write_missed": (
        "const int repeat = k > 0 && memcmp(r[k - 1].dig, r[k].dig, (size_t)d) == 0;",
        "const int repeat = 0;"),
    "blockmap_held_not_checked": ("const int held = m->n && bsearch(", "const int held = 0 && bsearch("),
    "blockmap_first_copy_marked": ("return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);",
                                   "return a->idx > b->idx ? -1 : (a->idx < b->idx ? 1 : 0);"),
    "blockmap_bytes_of_sorted_position": ("if (len) bytes += len[i];", "if (len) bytes += len[r[i].idx];"),
}


def _pin_suite():
    for kind in pins.KINDS:
        pins.test_hash_all_lengths_vs_hashlib(kind)
        pins.test_hash_standard_example_messages(kind)
        for length, block in pins.CASES:
            pins.test_leaves_and_root_closed_form(kind, length, block)
        pins.test_root_single_segment_is_hash_of_hash(kind)
        pins.test_chunk_digests_vs_hashlib(kind)
        pins.test_similarity_constructed_overlap(kind)
        for w in [1, 20]:
            pins.test_window_scan_vs_bruteforce(kind, w)
    for case in [(0, 20, 1), (20, 20, 1), (1000, 20, 4), (1001, 7, 3)]:
        pins.test_window_count_closed_form(*case)
    pins.test_predicate_reads_low_bits_of_first_word()
    for seed in range(4):
        pins.test_chunk_select_properties(seed)
    pins.test_chunk_select_degenerate()
    for seed in range(3):
        pins.test_chunk_select_max_properties(seed)
    pins.test_chunk_select_max_reductions()
    pins.test_similarity_multiplicity_and_identity()
    for kind in pins.KINDS:
        pins.test_blockmap_writes_vs_python_set(kind)
    pins.test_blockmap_closed_forms()
    pins.test_blockmap_new_version_duplicates_equal_similarity()
    pins.test_blockmap_capacity_refusal_changes_nothing()


def _build_variant(src_text, tmpdir, name):
    c_path = os.path.join(tmpdir, name + ".c")
    so_path = os.path.join(tmpdir, name + ".so")
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", so_path, c_path, "-lm"],
                   check=True)
    return so_path


def test_unmodified_oracle_passes_pin_suite():
    with open(SRC) as f:
        text = f.read()
    with tempfile.TemporaryDirectory() as tmp:
        oracle._swap_library(_build_variant(text, tmp, "unmodified"))
        try:
            _pin_suite()
        finally:
            oracle._swap_library(None)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    old, new = MUTATIONS[name]
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) >= 1, "mutation anchor missing from oracle.c"
    with tempfile.TemporaryDirectory() as tmp:
        oracle._swap_library(_build_variant(text.replace(old, new, 1), tmp, name))
        try:
            with pytest.raises(AssertionError):
                _pin_suite()
        finally:
            oracle._swap_library(None)
