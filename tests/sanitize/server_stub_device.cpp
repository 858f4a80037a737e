// Stub device layer for the serving loop's sanitizer builds and its
// group-formation test: the
// library calls server.cpp makes, with outputs that identify the request
// they belong to.  A block job's segment digests are filled with the byte
// (len * 7 + block_size) & 0xff and, when it runs alone, its root with
// (len * 13) & 0xff; chunk
// requests find no candidates (each is one chunk ending at its length when
// run alone, none in a group, which the driver accounts for).
#include <hip/hip_runtime.h>

#include <atomic>
#include <thread>

#include "hashgpu.h"
#include "hg_internal.hpp"

namespace {
int db(int d) { return d == HG_MD5 ? 16 : 20; }
}  // namespace

// Test hook of the group-formation driver: a single chunk call on a payload
// of exactly hold_len bytes waits, once it has set `entered`, until
// `released` is set (0: no call waits).
namespace stubhook {
std::atomic<uint64_t> hold_len{0};
std::atomic<int> entered{0}, released{0};
}  // namespace stubhook

namespace {
uint8_t leaf_byte(uint64_t len, uint64_t block) { return (uint8_t)((len * 7 + block) & 0xff); }
uint8_t root_byte(uint64_t len) { return (uint8_t)((len * 13) & 0xff); }
}  // namespace

namespace hg {
size_t window_scan_scratch_bytes(const WsPlan &p) { return 256 + p.n_tiles * 8; }
uint64_t window_scan_tile_windows(uint32_t, uint32_t, int) { return 4096; }
WsPlan plan_window_scan_files(uint64_t n_tiles, uint64_t total_windows, uint32_t, uint32_t, int kind) {
    WsPlan p{};
    p.kind = kind;
    p.nwin = total_windows;
    p.tile_windows = 4096;
    p.n_tiles = n_tiles;
    return p;
}
const uint64_t *window_scan_tile_offsets(const WsPlan &, const void *scratch) { return (const uint64_t *)scratch; }
size_t segment_digest_scratch_bytes(uint64_t) { return 256; }
size_t two_level_arena_scratch_bytes(uint64_t) { return 256; }
size_t batch_plan_bytes(uint32_t) { return 256; }
hipError_t launch_batch_plan(const hg_block_job *, uint32_t, void *, hipStream_t) { return hipSuccess; }
hipError_t launch_leaves_batch(const hg_block_job *jobs, uint32_t n, void *, uint32_t, uint32_t, bool, hipStream_t) {
    for (uint32_t i = 0; i < n; i++) {
        const hg_block_job &j = jobs[i];
        const uint64_t nl = j.len ? (j.len + j.block_size - 1) / j.block_size : 0;
        if (nl) memset(j.leaf_out, leaf_byte(j.len, j.block_size), nl * db(j.digest));
    }
    return hipSuccess;
}
hipError_t launch_roots_batch(const hg_block_job *jobs, uint32_t n, void *, bool, hipStream_t) {
    for (uint32_t i = 0; i < n; i++)
        if (jobs[i].root_out) memset(jobs[i].root_out, root_byte(jobs[i].len), db(jobs[i].digest));
    return hipSuccess;
}
hipError_t launch_window_scan_tiles(const WsPlan &, const uint8_t *, uint64_t, uint32_t, uint32_t, uint32_t,
                                    uint32_t, void *, hipStream_t, const WsFiles *) {
    return hipSuccess;
}
hipError_t launch_window_scan_prefix(const WsPlan &, void *, uint64_t *total_dev, hipStream_t) {
    *total_dev = 0;
    return hipSuccess;
}
hipError_t launch_window_scan_emit(const WsPlan &, const uint8_t *, uint64_t, uint32_t, uint32_t, uint32_t,
                                   uint32_t, void *, uint64_t *, uint64_t, hipStream_t, const WsFiles *) {
    return hipSuccess;
}
hipError_t launch_files_select(const FilesChunk &, uint32_t, uint64_t, uint64_t *, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_files_compact(const FilesChunk &fc, uint64_t *chunk_off, uint64_t *, uint64_t, uint64_t *status,
                                hipStream_t) {
    for (uint32_t f = 0; f <= fc.n_files; f++) chunk_off[f] = 0;
    status[1] = 0;
    return hipSuccess;
}
hipError_t launch_segment_digests(int, const uint8_t *, uint64_t, const uint64_t *, const uint64_t *,
                                  const uint64_t *, uint64_t, uint8_t *, void *, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_chunk_digests_two_level_arena(int, const uint8_t *, const uint64_t *, const uint64_t *,
                                                const uint64_t *, uint64_t, uint64_t, void *, uint8_t *, uint64_t,
                                                uint8_t *, hipStream_t) {
    return hipSuccess;
}
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t) {
    for (uint64_t i = 0; i < n; i++) p[i] = v;
    return hipSuccess;
}
}  // namespace hg

struct hg_ctx {
    int device;
};

extern "C" {
int hg_create(int device, size_t, size_t, hg_ctx **out) {
    *out = new hg_ctx{device};
    return HG_OK;
}
void hg_destroy(hg_ctx *c) { delete c; }
int hg_block_hash(hg_ctx *, const void *, uint64_t len, uint64_t block_size, int digest, void *leaf_out,
                  void *root_out, uint32_t, void *) {
    const uint64_t nl = len ? (len + block_size - 1) / block_size : 0;
    if (leaf_out && nl) memset(leaf_out, leaf_byte(len, block_size), nl * db(digest));
    if (root_out) memset(root_out, root_byte(len), db(digest));
    return HG_OK;
}
int hg_chunk(hg_ctx *, const void *, uint64_t len, const hg_chunk_params *, uint64_t *ends, uint64_t capacity,
             uint64_t *n_chunks, void *, uint32_t, void *) {
    if (len && len == stubhook::hold_len.load()) {
        stubhook::entered.store(1);
        while (!stubhook::released.load()) std::this_thread::yield();
    }
    *n_chunks = len ? 1 : 0;
    if (len && capacity) ends[0] = len;
    return len && !capacity ? HG_ETRUNC : HG_OK;
}
}
