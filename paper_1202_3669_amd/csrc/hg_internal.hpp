// hg_internal.hpp -- declarations shared by the C-ABI runtime (hashgpu.cpp)
// and the kernel translation units.  Every launcher enqueues work on the
// given stream and returns the launch status; none of them synchronizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hashgpu.h"

namespace hg {

// A dispatch holds fewer than 2^32 work-items per dimension.  Kernels with
// one lane per unit are launched over at most LAUNCH_LANES units at a time
// (segments, window tiles are split into several launches); the public calls
// reject work that would need more than MAX_LANES lanes in one launch of a
// kernel that cannot be split (candidates, chunks, digests).
constexpr uint64_t LAUNCH_LANES = 1ull << 30;
constexpr uint64_t MAX_LANES = 1ull << 31;

// ----------------------------------------------------------- block hash --
// Segment (leaf) digests: leaf k = H(in[k*block, min((k+1)*block, len))),
// written to out + k*digest_size.  n_leaves = ceil(len / block).
hipError_t launch_leaves(int kind, const uint8_t *in, uint64_t len, uint64_t block,
                         uint64_t n_leaves, uint8_t *out, hipStream_t s);

// MD5 and SHA-1 segment digests in one pass over the input (16-byte and
// 20-byte records, segment order).
hipError_t launch_leaves_dual(const uint8_t *in, uint64_t len, uint64_t block, uint64_t n_leaves,
                              uint8_t *out_md5, uint8_t *out_sha1, hipStream_t s);

// One digest of a whole device byte range (used for the second level of the
// direct hash, whose input is the leaf-digest buffer).
hipError_t launch_hash_one(int kind, const uint8_t *in, uint64_t len, uint8_t *out, hipStream_t s);

// ---------------------------------------------------------- window scan --
constexpr int WS_TPB = 256;  // lanes per workgroup (4 waves)
constexpr int WS_CAP = 16;   // per-tile bucket entries before the overflow path

// Plan of a window scan: how windows are tiled over workgroups, and which
// kernel variant runs.  Produced on the host by plan_window_scan().
struct WsPlan {
    int variant;          // 0 = generic LDS path, 1 = w20/s1 registers, 2 = w20/s4 registers
    int kind;             // window digest
    uint64_t nwin;        // number of windows
    uint64_t tile_windows;  // windows per workgroup tile
    uint64_t n_tiles;
    uint32_t lds_bytes;   // dynamic LDS per workgroup (generic path)
};

// Many files in one arena: tile t covers windows [tiles[t].k0, +tile_windows)
// of file tiles[t].file; a tile never spans two files.
struct FileTile {
    uint32_t file;
    uint32_t pad;
    uint64_t k0;
};
struct WsFiles {
    const uint8_t *arena;
    const uint64_t *off, *len;
    const FileTile *tiles;
};

WsPlan plan_window_scan(const uint8_t *in, uint64_t len, uint32_t w, uint32_t s, int kind);
WsPlan plan_window_scan_files(uint64_t n_tiles, uint64_t total_windows, uint32_t w, uint32_t s, int kind);
// Windows per tile for these parameters (the tile map of files uses it).
uint64_t window_scan_tile_windows(uint32_t w, uint32_t s, int kind);

// Scratch needed by a window scan plan, in bytes (256-byte aligned pieces).
size_t window_scan_scratch_bytes(const WsPlan &p);
// The per-tile first-candidate offsets inside that scratch (valid after
// the prefix pass).
const uint64_t *window_scan_tile_offsets(const WsPlan &p, const void *scratch);

// Pass 1: hash every window, count candidates per tile, keep up to WS_CAP
// tile-local candidate indices per tile.  With `files`, in/len are unused
// and the windows come from the files' tile map.
hipError_t launch_window_scan_tiles(const WsPlan &p, const uint8_t *in, uint64_t len, uint32_t w,
                                    uint32_t s, uint32_t mask, uint32_t target, void *scratch,
                                    hipStream_t st, const WsFiles *files = nullptr);
// Pass 1 for tiles [t0, t1) only (single buffer): a caller whose input
// arrives in pieces runs the tiles whose windows have landed.
hipError_t launch_window_scan_tile_range(const WsPlan &p, const uint8_t *in, uint64_t len, uint32_t w, uint32_t s,
                                         uint32_t mask, uint32_t target, void *scratch, uint64_t t0, uint64_t t1,
                                         hipStream_t st);

// Pass 2: exclusive scan of the tile counts, total to *total_dev, list of
// overflowed tiles.
hipError_t launch_window_scan_prefix(const WsPlan &p, void *scratch, uint64_t *total_dev,
                                     hipStream_t st);

// Pass 3: write the first `cap` candidate start offsets, ascending (per
// file and file-relative with `files`), to out (device).  Uses the scratch
// filled by the two passes above.
hipError_t launch_window_scan_emit(const WsPlan &p, const uint8_t *in, uint64_t len, uint32_t w,
                                   uint32_t s, uint32_t mask, uint32_t target, void *scratch,
                                   uint64_t *out, uint64_t cap, hipStream_t st,
                                   const WsFiles *files = nullptr);

// --------------------------------------------------------------- chunks --
// Greedy selection over ascending candidate starts: end e = start + w is a
// cut iff e >= last + max(min_chunk, 1) and e < len; the final end is len.
// *n_starts_dev holds the candidate count, n_starts (host) the same count
// for sizing the grids; scratch is chunk_select_scratch_bytes(n_starts).
// Writes up to cap ends and *n_chunks_dev.
size_t chunk_select_scratch_bytes(uint64_t n_starts);
// The same decision with a maximum chunk size (forced cuts), by one
// wavefront; cap >= n_starts + 2 + len / max_chunk holds every cut.
hipError_t launch_chunk_select_max(const uint64_t *starts, const uint64_t *n_starts_dev, uint32_t w, uint64_t len,
                                   uint64_t min_chunk, uint64_t max_chunk, uint64_t *ends, uint64_t cap,
                                   uint64_t *n_chunks_dev, hipStream_t s);
hipError_t launch_chunk_select(const uint64_t *starts, const uint64_t *n_starts_dev, uint64_t n_starts,
                               uint32_t w, uint64_t len, uint64_t min_chunk, void *scratch, uint64_t *ends,
                               uint64_t cap, uint64_t *n_chunks_dev, hipStream_t s);

// Digest of every segment j < *n_dev <= max_n, into out + j*digest_size.
// Segment j is [starts[j], ends[j]) when starts is given, else
// [ends[j-1], ends[j]) with ends[-1] = 0 (offsets relative to in, taken
// modulo 2^64).  Without starts, reads stay below in + len; with starts,
// each segment reads only its own bytes (len is then unused).  Scratch is
// segment_digest_scratch_bytes(max_n).
size_t segment_digest_scratch_bytes(uint64_t max_n);
// out[0] = the longest of the segments [ends[j-1], ends[j]) of a buffer of
// len bytes, j < *n_dev <= max_n (0 when there are none).
hipError_t launch_max_gap(const uint64_t *ends, uint64_t len, const uint64_t *n_dev, uint64_t max_n, uint64_t *out,
                          hipStream_t s);
// Packs k byte ranges of src into dst: range r is tab[3r + 1] bytes from
// src + tab[3r] to dst + tab[3r + 2], where dst + tab[3r + 2] and
// src + tab[3r] are equal modulo 16 and dst is 16-byte aligned (one
// workgroup per range at a time: the caller cuts long ranges into slices).
hipError_t launch_gather_ranges(const uint8_t *src, const uint64_t *tab, uint64_t k, uint8_t *dst, hipStream_t s);
// Record k (d bytes) of src to out + idx[k] * d, k < n.
hipError_t launch_digest_scatter(const uint64_t *idx, const uint8_t *src, uint64_t n, int d, uint8_t *out,
                                 hipStream_t s);
hipError_t launch_segment_digests(int kind, const uint8_t *in, uint64_t len, const uint64_t *starts,
                                  const uint64_t *ends, const uint64_t *n_dev, uint64_t max_n, uint8_t *out,
                                  void *scratch, hipStream_t s);

// Two-level chunk digests (each chunk direct-hashed with segments of S
// bytes): chunk j is [ends[j-1], ends[j]) of in (ends[-1] = 0, *n_dev <=
// max_n chunks, reads below in + len).  leaves is scratch of
// two_level_slots(len, max_n, S) * digest bytes; out gets n digests.
uint64_t two_level_slots(uint64_t len, uint64_t max_n, uint64_t S);
hipError_t launch_chunk_digests_two_level(int kind, const uint8_t *in, uint64_t len, const uint64_t *ends,
                                          const uint64_t *n_dev, uint64_t max_n, uint64_t S, uint8_t *leaves,
                                          uint8_t *out, hipStream_t s);

// Two-level chunk digests of chunks [starts[j], ends[j]) of an arena
// (*n_dev <= max_n of them, in any arena order): scratch of
// two_level_arena_scratch_bytes(max_n), n_slots >= sum of ceil(len / S)
// segment-digest slots in `leaves`.
size_t two_level_arena_scratch_bytes(uint64_t max_n);
hipError_t launch_chunk_digests_two_level_arena(int kind, const uint8_t *arena, const uint64_t *starts,
                                                const uint64_t *ends, const uint64_t *n_dev, uint64_t max_n,
                                                uint64_t S, void *scratch, uint8_t *leaves, uint64_t n_slots,
                                                uint8_t *out, hipStream_t s);

// Streaming boundary decision over a carried buffer of len bytes whose
// first chunk starts at last0: candidate starts cand[i] + add (ascending,
// *n_dev of them).  Writes the cuts it can decide (relative to last0) to
// ends (up to cap) and state[0] = their number, state[1] = the last cut;
// with `final` the chunk ending at len is included.
hipError_t launch_stream_walk(const uint64_t *cand, const uint64_t *n_dev, uint64_t add, uint32_t w, uint64_t len,
                              uint64_t last0, uint64_t min_chunk, uint64_t max_chunk, bool final, uint64_t *ends,
                              uint64_t cap, uint64_t *state, hipStream_t s);

// Streaming without a maximum: words[0] = candidates whose end lies below
// limit (a prefix), words[1] = the rest; stream_shift writes the rest as
// starts relative to last0 (cand + add - last0); stream_tail turns a parallel
// selection's count and ends (relative to last0) into state[0] = decided
// chunks (the last one dropped unless final), state[1] = the last decided
// end (last0 + ...; last0 when none).
hipError_t launch_stream_drop(const uint64_t *cand, const uint64_t *n_dev, uint64_t add, uint32_t w, uint64_t limit,
                              uint64_t *words, hipStream_t s);
hipError_t launch_stream_shift(const uint64_t *cand, const uint64_t *words, uint64_t max_m, uint64_t add,
                               uint64_t last0, uint64_t *out, hipStream_t s);
hipError_t launch_stream_tail(const uint64_t *n_chunks, const uint64_t *ends, bool final, uint64_t last0,
                              uint64_t *state, hipStream_t s);

// ---------------------------------------------------------------- files --
// Content-based chunking of many files (see files.hip).  cand: candidate
// starts (file-relative, files in order) with capacity cap_cand; the tile
// offsets and the total come from the window scan's prefix pass.
struct FilesChunk {
    const uint64_t *off, *len;        // per file
    const uint64_t *first_tile;       // n_files + 1
    const uint64_t *tile_off;         // per tile: first candidate
    uint64_t n_tiles;
    const uint64_t *cand;             // candidate starts
    uint64_t cap_cand;
    uint64_t *slots;                  // cap_cand + n_files chunk ends
    uint32_t *cnt;                    // chunks per file
    uint64_t *seg_start, *seg_end;    // absolute arena offsets, cap_cand + n_files
    uint32_t n_files;
    uint64_t max_chunk;               // 0: no maximum chunk size
    const uint64_t *extra;            // with max_chunk: extra slots before file f (forced cuts), else null
};
// status[0] = candidates (written by the prefix pass), status[1] = chunks,
// status[2] = nonzero when the candidate capacity was exceeded.
hipError_t launch_files_select(const FilesChunk &fc, uint32_t w, uint64_t min_chunk, uint64_t *status,
                               hipStream_t s);
hipError_t launch_files_compact(const FilesChunk &fc, uint64_t *chunk_off, uint64_t *chunk_ends,
                                uint64_t max_chunks, uint64_t *status, hipStream_t s);
// Job records of the direct hash of every file (order[i] = file of record i).
hipError_t launch_files_jobs(const uint8_t *arena, const uint64_t *off, const uint64_t *len,
                             const uint64_t *leaf_first, const uint32_t *order, uint32_t n_files,
                             uint64_t block, int digest, uint8_t *leaf_out, uint8_t *roots, hg_block_job *jobs,
                             hipStream_t s);

// ---------------------------------------------------------------- batch --
// Jobs are hg_block_job records in device memory.  The plan (scratch of
// batch_plan_bytes(n_jobs)) is written by launch_batch_plan and read by the
// two launchers that follow it on the same stream.
size_t batch_plan_bytes(uint32_t n_jobs);
hipError_t launch_batch_plan(const hg_block_job *jobs, uint32_t n_jobs, void *plan, hipStream_t s);
// A persistent grid of `waves` wavefronts (rounded up to whole workgroups)
// in workgroups of wg_waves (1, 2 or 4) wavefronts.  boost: waves on long
// chains raise their issue priority.
hipError_t launch_leaves_batch(const hg_block_job *jobs, uint32_t n_jobs, void *plan, uint32_t waves,
                               uint32_t wg_waves, bool boost, hipStream_t s);
hipError_t launch_roots_batch(const hg_block_job *jobs, uint32_t n_jobs, void *plan, bool boost, hipStream_t s);
// Copies root j (20-byte records of `roots`, by job index) to jobs[j].root_out
// for every job with a root_out (second levels computed on the host).
hipError_t launch_roots_scatter(const hg_block_job *jobs, uint32_t n_jobs, const uint8_t *roots, hipStream_t s);

// ----------------------------------------------------------- similarity --
// Open-addressing set of A's digests (table of 2^log2_slots uint32 slots),
// then a probe of every B digest; matched count and matched byte sum land in
// counters[0], counters[1] (cleared by the launcher).
// len_b holds lengths, or chunk end offsets when len_is_ends is set.  With
// n_b_dev, B has min(*n_b_dev, n_b) digests (read when the kernel runs).
hipError_t launch_similarity(int kind, const uint8_t *dig_a, uint64_t n_a, const uint8_t *dig_b,
                             const uint64_t *len_b, int len_is_ends, uint64_t n_b, const uint64_t *n_b_dev,
                             uint32_t *table, int log2_slots, unsigned long long *counters, hipStream_t s);

// ---------------------------------------------------------------- probes --
// int32 VALU issue-rate and HBM read-rate microbenchmarks (out: a 4-byte
// device word that the kernels may write).
uint64_t alu_probe_ops(uint32_t blocks, uint32_t steps);
hipError_t launch_alu_probe(uint32_t blocks, uint32_t steps, uint32_t *out, hipStream_t s);
hipError_t launch_read_probe(const uint8_t *p, uint64_t len, uint32_t *out, hipStream_t s);

// -------------------------------------------------------------- block map --
// The store's digests (capacity * digest size bytes), the open-addressing
// table over them (slot_mask + 1 slots of uint32: 0 empty, k + 1 = stored
// digest k) and the device count of stored digests.
struct BlockMapView {
    uint8_t *store;
    uint32_t *table;
    uint64_t slot_mask;
    unsigned long long *size;
};
// One write of n chunk digests: is_dup[i] (optional) = 1 iff digest i was
// stored before or equals that of a chunk j < i; counters[0] = duplicates,
// counters[1] = their bytes (len: lengths, or ends with len_is_ends; may be
// null).  Scratch: state (n bytes), slot_of (n x 4), pos_of (n x 8).  The
// caller guarantees room for n more digests.
hipError_t launch_blockmap_write(int kind, const BlockMapView &m, const uint8_t *dig, uint64_t n, const uint64_t *len,
                                 int len_is_ends, uint8_t *state, uint32_t *slot_of, uint64_t *pos_of,
                                 uint8_t *is_dup, unsigned long long *counters, hipStream_t s);

// dst[i] = src[i] + add for i < *n_dev (<= max_n, which sizes the grid).
hipError_t launch_add_u64(uint64_t *dst, const uint64_t *src, const uint64_t *n_dev, uint64_t max_n, uint64_t add,
                          hipStream_t s);

// out[0] = min(*n, max) and out[1] = 1 if *n > max, else 0 (one kernel);
// then *n_out = ~0 where *flag is set.
hipError_t launch_count_clamp(const uint64_t *n, uint64_t max, uint64_t *out, hipStream_t s);
hipError_t launch_count_invalidate(const uint64_t *flag, uint64_t *n_out, hipStream_t s);

// Fill n 32-bit words with v (a kernel, so that captured graphs hold no
// memset nodes).
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);

}  // namespace hg
