// hg_internal.hpp -- declarations shared by the C-ABI runtime (hashgpu.cpp)
// and the kernel translation units.  Every launcher enqueues work on the
// given stream and returns the launch status; none of them synchronizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hashgpu.h"

namespace hg {

// ----------------------------------------------------------- block hash --
// Segment (leaf) digests: leaf k = H(in[k*block, min((k+1)*block, len))),
// written to out + k*digest_size.  n_leaves = ceil(len / block).
hipError_t launch_leaves(int kind, const uint8_t *in, uint64_t len, uint64_t block,
                         uint64_t n_leaves, uint8_t *out, hipStream_t s);

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

WsPlan plan_window_scan(const uint8_t *in, uint64_t len, uint32_t w, uint32_t s, int kind);

// Scratch needed by a window scan plan, in bytes (256-byte aligned pieces).
size_t window_scan_scratch_bytes(const WsPlan &p);

// Pass 1: hash every window, count candidates per tile, keep up to WS_CAP
// tile-local candidate indices per tile.
hipError_t launch_window_scan_tiles(const WsPlan &p, const uint8_t *in, uint64_t len, uint32_t w,
                                    uint32_t s, uint32_t mask, uint32_t target, void *scratch,
                                    hipStream_t st);
// Pass 2: exclusive scan of the tile counts, total to *total_dev, list of
// overflowed tiles.
hipError_t launch_window_scan_prefix(const WsPlan &p, void *scratch, uint64_t *total_dev,
                                     hipStream_t st);

// Pass 3: write the first `cap` candidate start offsets, ascending, to out
// (device).  Uses the scratch filled by the two passes above.
hipError_t launch_window_scan_emit(const WsPlan &p, const uint8_t *in, uint64_t len, uint32_t w,
                                   uint32_t s, uint32_t mask, uint32_t target, void *scratch,
                                   uint64_t *out, uint64_t cap, hipStream_t st);

// --------------------------------------------------------------- chunks --
// Greedy selection over ascending candidate starts: end e = start + w is a
// cut iff e >= last + max(min_chunk, 1) and e < len; the final end is len.
// *n_starts_dev holds the candidate count, n_starts (host) the same count
// for sizing the grids; scratch is chunk_select_scratch_bytes(n_starts).
// Writes up to cap ends and *n_chunks_dev.
size_t chunk_select_scratch_bytes(uint64_t n_starts);
hipError_t launch_chunk_select(const uint64_t *starts, const uint64_t *n_starts_dev, uint64_t n_starts,
                               uint32_t w, uint64_t len, uint64_t min_chunk, void *scratch, uint64_t *ends,
                               uint64_t cap, uint64_t *n_chunks_dev, hipStream_t s);

// Digest of every segment [ends[j-1], ends[j]) (ends[-1] = 0) for
// j < *n_dev <= max_n, into out + j*digest_size.  Scratch is
// segment_digest_scratch_bytes(max_n).
size_t segment_digest_scratch_bytes(uint64_t max_n);
hipError_t launch_segment_digests(int kind, const uint8_t *in, uint64_t len, const uint64_t *ends,
                                  const uint64_t *n_dev, uint64_t max_n, uint8_t *out, void *scratch,
                                  hipStream_t s);

// ---------------------------------------------------------------- batch --
// Jobs are hg_block_job records in device memory.  The plan (scratch of
// batch_plan_bytes(n_jobs)) is written by launch_batch_plan and read by the
// two launchers that follow it on the same stream.
size_t batch_plan_bytes(uint32_t n_jobs);
hipError_t launch_batch_plan(const hg_block_job *jobs, uint32_t n_jobs, void *plan, hipStream_t s);
// boost: waves on long chains raise their issue priority.
hipError_t launch_leaves_batch(const hg_block_job *jobs, uint32_t n_jobs, void *plan, uint32_t grid,
                               bool boost, hipStream_t s);
hipError_t launch_roots_batch(const hg_block_job *jobs, uint32_t n_jobs, void *plan, bool boost, hipStream_t s);

// ----------------------------------------------------------- similarity --
// Open-addressing set of A's digests (table of 2^log2_slots uint32 slots),
// then a probe of every B digest; matched count and matched byte sum land in
// counters[0], counters[1] (cleared by the launcher).
// len_b holds lengths, or chunk end offsets when len_is_ends is set.
hipError_t launch_similarity(int kind, const uint8_t *dig_a, uint64_t n_a, const uint8_t *dig_b,
                             const uint64_t *len_b, int len_is_ends, uint64_t n_b, uint32_t *table,
                             int log2_slots, unsigned long long *counters, hipStream_t s);

// Fill n 32-bit words with v (a kernel, so that captured graphs hold no
// memset nodes).
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);

}  // namespace hg
