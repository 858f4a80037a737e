// server.cpp -- continuous-batching serving loop for hash requests (the
// CrystalGPU job lifecycle of Sec. 3.2.3: an outstanding queue, buffers
// allocated once and reused, completion by callback; the batching and
// transfer/work overlap of Sec. 3.1).
//
// Workers and groups.  Each of `slots` workers owns one pre-allocated group:
// a main and a helper stream, device tables and scratch for up to
// max_requests requests and max_group_bytes payload bytes, and one pinned
// host buffer for uploads and results.  An idle worker takes requests from
// the head of the queue, in arrival order, while they fit its group and the
// staging region, and enqueues the whole group.  A group holds one kind of
// request: block requests, whose groups are bound by their chains, or chunk
// requests, whose groups are window scans; requests in device memory of the
// other kind stay queued for the next idle worker, so that the two kinds
// run side by side in different groups instead of the chains holding up a
// mixed group after its scans are done.
//   - host payloads are copied into the staging region (device-memory
//     admission: a request waits at the head until its bytes fit);
//   - block requests: one job table and one persistent segment-digest
//     launch for all of them (MD5 and SHA-1 mixed) on the helper stream
//     (a group of host payloads may hold both kinds);
//     their segment digests come back whole and the worker computes the
//     second levels on the host pool (Sec. 3.2.2);
//   - chunk requests (same parameters within a group): one tile map over
//     all payloads, the window scan, per-file boundary selection, compaction
//     and the chunk digests -- on the main stream;
//   - one copy of the results back to the pinned buffer.
// While a worker waits for its group, the other workers form and launch
// theirs, so requests that arrive meanwhile overlap on the device with the
// groups in flight.  A request that does not fit an empty group (or a chunk
// request of more than SOLO_CHUNK_BYTES) runs alone
// through the single-call entry points on the worker's context; such a chunk
// request in device memory does not close the group being formed (it waits
// at its place for the next idle worker, and later requests that fit join).
//
// Payload addressing in a group: chunk payloads are described as offsets
// from the staging region's base taken modulo 2^64, so that payloads in the
// caller's device memory and in the staging region share one table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hashgpu.h"
#include "hg_internal.hpp"
#include "hg_ranges.hpp"
#include "host_hash.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t id = 0;
    hg_request r{};
    void (*cb)(uint64_t, int, void *) = nullptr;
    void *user = nullptr;
    int status = HG_OK;
    bool done = false;
    bool waitable = true;        // released by hg_wait (else after completion)
    double *lat_out = nullptr;   // load replay: where latency and status go
    int32_t *st_out = nullptr;
    std::atomic<uint64_t> *remaining = nullptr;
    uint64_t stage_off = 0, stage_bytes = 0;
    const uint8_t *dev_in = nullptr;  // payload in device memory once admitted
    Clock::time_point t_arrival;
};


constexpr uint64_t STAGE_ALIGN = 256;
constexpr size_t LAT_WINDOW = 1u << 20;  // completions the latency statistics cover
// Two-level chunk digests are grouped for segments of at least this many
// bytes (a group's segment-digest slots are sized for it); smaller segments
// run alone.
constexpr uint64_t TL_MIN_SEGMENT = 4096;
// Chunk requests longer than this are served alone: a group decides each
// file's boundaries with one wavefront walking its candidates cut by cut
// (~0.1 us a cut: ~5 ms for 256 MiB at the configured parameters, on the
// group's critical path), while the single call's parallel speculative
// selection takes well under a millisecond.
constexpr uint64_t SOLO_CHUNK_BYTES = 32ull << 20;

int dbytes(int d) { return d == HG_MD5 ? 16 : (d == HG_SHA1 ? 20 : -1); }
uint64_t up256(uint64_t x) { return (x + 255) & ~255ull; }
uint64_t n_leaves(const hg_request &r) { return r.len ? (r.len + r.block_size - 1) / r.block_size : 0; }

bool same_chunk_params(const hg_chunk_params &a, const hg_chunk_params &b) {
    return a.window == b.window && a.stride == b.stride && a.mask == b.mask && a.target == b.target &&
           a.min_chunk == b.min_chunk && a.max_chunk == b.max_chunk && a.window_digest == b.window_digest &&
           a.chunk_digest == b.chunk_digest && a.chunk_segment == b.chunk_segment;
}

// A request's footprint inside a group.
struct Need {
    uint64_t leaf_bytes = 0, tiles = 0, windows = 0, cand = 0;
};

Need need_of(const hg_request &r) {
    Need n;
    if (r.kind == HG_REQ_BLOCK) {
        n.leaf_bytes = n_leaves(r) * (uint64_t)dbytes(r.digest);
    } else {
        const hg_chunk_params &c = r.chunk;
        n.windows = r.len >= c.window ? (r.len - c.window) / c.stride + 1 : 0;
        const uint64_t tw = hg::window_scan_tile_windows(c.window, c.stride, c.window_digest);
        n.tiles = (n.windows + tw - 1) / tw;
        // Twice the expectation for random data plus slack per file (the
        // rule of planned file batches); a group whose real count exceeds
        // its capacity serves its chunk requests alone.
        n.cand = (uint64_t)(2.0 * std::ldexp(1.0, -__builtin_popcount(c.mask)) * (double)n.windows) + 64;
    }
    return n;
}

}  // namespace

struct hg_server;

namespace {

struct Group {
    hg_server *srv = nullptr;
    hg_ctx *ctx = nullptr;  // for requests that run alone
    hipStream_t st = nullptr, aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::thread th;
    // capacities
    uint32_t R = 0;
    uint64_t leaf_cap = 0, tile_cap = 0, cand_cap = 0, max_chunks = 0, ws_bytes = 0;
    // device
    std::vector<void *> dev_allocs;
    hg_block_job *d_jobs = nullptr;
    void *d_plan = nullptr, *d_ws = nullptr, *d_seg = nullptr;
    uint8_t *d_leaves = nullptr, *d_cdig = nullptr;
    uint64_t *d_off = nullptr, *d_len = nullptr, *d_first_tile = nullptr;
    hg::FileTile *d_tiles = nullptr;
    uint64_t *d_cand = nullptr, *d_slots = nullptr, *d_seg_start = nullptr, *d_seg_end = nullptr;
    uint64_t *d_ends = nullptr, *d_chunk_off = nullptr, *d_status = nullptr;
    uint32_t *d_cnt = nullptr;
    void *d_tl = nullptr;              // two-level digests: prefix scratch
    uint8_t *d_tl_leaves = nullptr;    // and segment-digest slots
    uint64_t tl_cap = 0;
    // pinned host (one allocation, carved)
    uint8_t *h = nullptr;
    hg_block_job *h_jobs = nullptr;
    uint64_t *h_off = nullptr, *h_len = nullptr, *h_first_tile = nullptr;
    hg::FileTile *h_tiles = nullptr;
    uint64_t *h_status = nullptr, *h_chunk_off = nullptr, *h_ends = nullptr;
    uint8_t *h_leaves = nullptr, *h_cdig = nullptr;
    // the group being served
    std::vector<Req *> blocks, chunks, failed;
    Req *solo = nullptr;
    uint64_t bytes = 0, leaf_used = 0, tiles = 0, windows = 0, cand = 0;
    hg_chunk_params cp{};
    void clear() {
        blocks.clear();
        chunks.clear();
        failed.clear();
        solo = nullptr;
        bytes = leaf_used = tiles = windows = cand = 0;
    }
    bool empty() const { return blocks.empty() && chunks.empty() && !solo; }
    size_t members() const { return blocks.size() + chunks.size(); }
};

}  // namespace

struct hg_server {
    int device = 0;
    hg_server_cfg cfg{};
    uint8_t *stage = nullptr;
    hg::Ranges ranges;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> pending;
    std::unordered_map<uint64_t, Req *> reqs;  // waitable requests until hg_wait
    uint64_t next_id = 1;
    bool stopping = false;
    std::vector<Group> groups;
    // statistics
    uint64_t submitted = 0, completed = 0, failed = 0, bytes = 0, n_groups = 0;
    uint32_t in_flight = 0, max_in_flight = 0;
    // Latencies of the last LAT_WINDOW completions (a ring), so that a
    // long-running server's statistics use bounded memory.
    std::vector<double> lat_ms;
    uint64_t lat_next = 0;
};

namespace {

int validate(const hg_request *r) {
    if (!r) return HG_EINVAL;
    if (r->len && !r->payload) return HG_EINVAL;
    if (r->flags & ~(uint32_t)(HG_IN_DEVICE | HG_REQ_FAIL_INJECT)) return HG_EINVAL;
    if (r->kind == HG_REQ_BLOCK) {
        if (dbytes(r->digest) < 0 || r->block_size == 0 || r->reserved) return HG_EINVAL;
        if (!r->leaf_out && !r->root_out) return HG_EINVAL;
    } else if (r->kind == HG_REQ_CHUNK) {
        const hg_chunk_params &c = r->chunk;
        if (dbytes(c.window_digest) < 0 || dbytes(c.chunk_digest) < 0) return HG_EINVAL;
        if (c.window == 0 || c.window > HG_MAX_WINDOW || c.stride == 0) return HG_EINVAL;
        if (c.max_chunk != 0 && c.max_chunk < (c.min_chunk ? c.min_chunk : 1)) return HG_EINVAL;
        if (!r->n_chunks || (r->capacity && !r->chunk_ends)) return HG_EINVAL;
    } else {
        return HG_EINVAL;
    }
    return HG_OK;
}

// ------------------------------------------------------------ allocation --

int group_alloc(Group &g, size_t bytes, void **out) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
        (void)hipGetLastError();
        return HG_ENOMEM;
    }
    g.dev_allocs.push_back(p);
    *out = p;
    return HG_OK;
}

void group_free(Group &g) {
    if (g.st) (void)hipStreamSynchronize(g.st);
    if (g.aux) (void)hipStreamSynchronize(g.aux);
    for (void *p : g.dev_allocs) (void)hipFree(p);
    g.dev_allocs.clear();
    if (g.h) (void)hipHostFree(g.h);
    g.h = nullptr;
    if (g.fork) (void)hipEventDestroy(g.fork);
    if (g.join) (void)hipEventDestroy(g.join);
    if (g.st) (void)hipStreamDestroy(g.st);
    if (g.aux) (void)hipStreamDestroy(g.aux);
    g.fork = g.join = nullptr;
    g.st = g.aux = nullptr;
    hg_destroy(g.ctx);
    g.ctx = nullptr;
}

int group_init(Group &g, int device, const hg_server_cfg &cfg) {
    int st;
    if ((st = hg_create(device, 0, 0, &g.ctx)) != HG_OK) return st;
    if (hipStreamCreateWithFlags(&g.st, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&g.aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g.join, hipEventDisableTiming) != hipSuccess)
        return HG_EDEVICE;
    const uint64_t M = cfg.max_group_bytes;
    g.R = cfg.max_requests;
    // Capacities: segment digests of 1 KiB segments over the whole group;
    // tiles of the smallest tile (2 KiB of windows) plus one per file;
    // candidates four times the expectation of a 12-bit mask at stride 1.
    g.leaf_cap = M / 1024 * 20 + (uint64_t)g.R * 20;
    g.tile_cap = M / 2048 + g.R + 1;
    g.cand_cap = M / 1024 + 64ull * g.R + 4096;
    g.max_chunks = g.cand_cap + g.R;
    g.ws_bytes = hg::window_scan_scratch_bytes(hg::plan_window_scan_files(g.tile_cap, M, 20, 1, HG_MD5));
    void *p;
#define GA(field, type, bytes)                                      \
    do {                                                            \
        if ((st = group_alloc(g, (bytes), &p)) != HG_OK) return st; \
        g.field = (type)p;                                          \
    } while (0)
    GA(d_jobs, hg_block_job *, (size_t)g.R * sizeof(hg_block_job));
    GA(d_plan, void *, hg::batch_plan_bytes(g.R));
    GA(d_leaves, uint8_t *, g.leaf_cap);
    GA(d_off, uint64_t *, (size_t)g.R * 8);
    GA(d_len, uint64_t *, (size_t)g.R * 8);
    GA(d_first_tile, uint64_t *, (size_t)(g.R + 1) * 8);
    GA(d_tiles, hg::FileTile *, g.tile_cap * sizeof(hg::FileTile));
    GA(d_ws, void *, g.ws_bytes);
    GA(d_cand, uint64_t *, g.cand_cap * 8);
    GA(d_slots, uint64_t *, g.max_chunks * 8);
    GA(d_seg_start, uint64_t *, g.max_chunks * 8);
    GA(d_seg_end, uint64_t *, g.max_chunks * 8);
    GA(d_ends, uint64_t *, g.max_chunks * 8);
    GA(d_cdig, uint8_t *, g.max_chunks * 20);
    GA(d_cnt, uint32_t *, (size_t)g.R * 4);
    GA(d_seg, void *, hg::segment_digest_scratch_bytes(g.max_chunks));
    g.tl_cap = M / TL_MIN_SEGMENT + g.max_chunks + 1;
    GA(d_tl, void *, hg::two_level_arena_scratch_bytes(g.max_chunks));
    GA(d_tl_leaves, uint8_t *, g.tl_cap * 20);
    GA(d_chunk_off, uint64_t *, (size_t)(g.R + 1) * 8);
    GA(d_status, uint64_t *, 64);
#undef GA
    // Pinned host buffer, carved in 256-byte aligned pieces.
    const uint64_t sizes[10] = {(uint64_t)g.R * sizeof(hg_block_job),
                                (uint64_t)g.R * 8,
                                (uint64_t)g.R * 8,
                                (uint64_t)(g.R + 1) * 8,
                                g.tile_cap * sizeof(hg::FileTile),
                                64,
                                (uint64_t)(g.R + 1) * 8,
                                g.leaf_cap,
                                g.max_chunks * 8,
                                g.max_chunks * 20};
    uint64_t total = 0;
    for (uint64_t s : sizes) total += up256(s);
    if (hipHostMalloc((void **)&g.h, total, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        g.h = nullptr;
        return HG_ENOMEM;
    }
    uint8_t *piece[10];
    uint8_t *q = g.h;
    for (int i = 0; i < 10; i++) {
        piece[i] = q;
        q += up256(sizes[i]);
    }
    g.h_jobs = (hg_block_job *)piece[0];
    g.h_off = (uint64_t *)piece[1];
    g.h_len = (uint64_t *)piece[2];
    g.h_first_tile = (uint64_t *)piece[3];
    g.h_tiles = (hg::FileTile *)piece[4];
    g.h_status = (uint64_t *)piece[5];
    g.h_chunk_off = (uint64_t *)piece[6];
    g.h_leaves = piece[7];
    g.h_ends = (uint64_t *)piece[8];
    g.h_cdig = piece[9];
    return HG_OK;
}

// ------------------------------------------------------- group formation --

// Whether request q joins group g as it stands.
bool fits(const Group &g, const hg_server_cfg &cfg, const Req *q) {
    const hg_request &r = q->r;
    if (g.members() >= g.R) return false;
    if (g.bytes + r.len > cfg.max_group_bytes) return false;
    const Need n = need_of(r);
    if (r.kind == HG_REQ_BLOCK) return g.leaf_used + n.leaf_bytes <= g.leaf_cap;
    // A maximum chunk size needs per-file room for forced cuts, and two-level
    // chunk digests with short segments more slots than a group holds: such
    // requests are served alone.
    if (r.chunk.max_chunk != 0 || (r.chunk.chunk_segment != 0 && r.chunk.chunk_segment < TL_MIN_SEGMENT) ||
        r.len > SOLO_CHUNK_BYTES)
        return false;
    if (!g.chunks.empty() && !same_chunk_params(g.cp, r.chunk)) return false;
    return g.tiles + n.tiles <= g.tile_cap && g.cand + n.cand <= g.cand_cap;
}

void add(Group &g, Req *q) {
    const Need n = need_of(q->r);
    g.bytes += q->r.len;
    if (q->r.kind == HG_REQ_BLOCK) {
        g.leaf_used += n.leaf_bytes;
        g.blocks.push_back(q);
    } else {
        if (g.chunks.empty()) g.cp = q->r.chunk;
        g.tiles += n.tiles;
        g.windows += n.windows;
        g.cand += n.cand;
        g.chunks.push_back(q);
    }
}

// Chunk requests served alone by their parameters or size (whatever the
// group holds).
bool solo_chunk(const hg_request &r) {
    return r.kind != HG_REQ_BLOCK &&
           (r.chunk.max_chunk != 0 || (r.chunk.chunk_segment != 0 && r.chunk.chunk_segment < TL_MIN_SEGMENT) ||
            r.len > SOLO_CHUNK_BYTES);
}

bool admissible(const hg_server *s, const Req *q) {
    return (q->r.flags & HG_REQ_FAIL_INJECT) || q->stage_bytes == 0 || s->ranges.fits(q->stage_bytes);
}

// Takes requests from the head of the queue into g (lock held).
void form(hg_server *s, Group &g) {
    g.clear();
    auto it = s->pending.begin();
    while (it != s->pending.end()) {
        Req *q = *it;
        if (q->r.flags & HG_REQ_FAIL_INJECT) {
            it = s->pending.erase(it);
            g.failed.push_back(q);
            continue;
        }
        bool alone = false;
        // One kind per group: a request in device memory of the other kind
        // stays queued for the next idle worker.
        if (!g.empty() && !q->stage_bytes && (q->r.kind == HG_REQ_BLOCK) != !g.blocks.empty()) {
            ++it;
            continue;
        }
        if (!fits(g, s->cfg, q)) {
            if (!g.empty()) {
                // A chunk request that is served alone anyway stays queued
                // for the next idle worker; the requests behind it that fit
                // still join this group.
                if (solo_chunk(q->r) && !q->stage_bytes) {
                    ++it;
                    continue;
                }
                break;
            }
            alone = true;  // does not fit even an empty group
        }
        if (q->stage_bytes && !s->ranges.take(q->stage_bytes, &q->stage_off)) break;
        it = s->pending.erase(it);
        q->dev_in = q->stage_bytes ? s->stage + q->stage_off : (const uint8_t *)q->r.payload;
        if (alone) {
            g.solo = q;
            break;
        }
        add(g, q);
    }
    const uint32_t admitted = (uint32_t)(g.members() + (g.solo ? 1 : 0));
    s->in_flight += admitted;
    s->max_in_flight = std::max(s->max_in_flight, s->in_flight);
    if (admitted) s->n_groups++;
}

// -------------------------------------------------------------- execution --

#define SV_HIP(expr)                 \
    do {                             \
        if ((expr) != hipSuccess) {  \
            (void)hipGetLastError(); \
            return HG_EDEVICE;       \
        }                            \
    } while (0)

int stage_in(Group &g, const Req *q) {
    if (!q->stage_bytes || !q->r.len) return HG_OK;
    SV_HIP(hipMemcpyAsync((void *)q->dev_in, q->r.payload, q->r.len, hipMemcpyHostToDevice, g.st));
    return HG_OK;
}

// The segment digests of every block request of the group (helper stream),
// laid out in member order and copied back whole; the second levels are
// computed on the host from that copy once the group is done (Sec. 3.2.2
// places that step on the CPU; a core runs the chain far faster than a GPU
// lane, and the worker waits for the group anyway).  The job table lists
// the members longest first, so that the persistent workers start on the
// longest chains.
int enqueue_blocks(Group &g, bool boost) {
    const uint32_t n = (uint32_t)g.blocks.size();
    std::vector<uint64_t> lofs(n);
    uint64_t leaf_off = 0, total_leaves = 0;
    for (uint32_t i = 0; i < n; i++) {
        const hg_request &r = g.blocks[i]->r;
        lofs[i] = leaf_off;
        leaf_off += n_leaves(r) * (uint64_t)dbytes(r.digest);
        total_leaves += n_leaves(r);
    }
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return g.blocks[a]->r.len > g.blocks[b]->r.len; });
    for (uint32_t k = 0; k < n; k++) {
        const uint32_t i = order[k];
        const Req *q = g.blocks[i];
        hg_block_job &j = g.h_jobs[k];
        j.in = q->dev_in;
        j.len = q->r.len;
        j.block_size = q->r.block_size;
        j.leaf_out = g.d_leaves + lofs[i];
        j.root_out = nullptr;
        j.digest = q->r.digest;
        j.reserved = 0;
    }
    hipStream_t st = g.aux;
    SV_HIP(hipMemcpyAsync(g.d_jobs, g.h_jobs, (size_t)n * sizeof(hg_block_job), hipMemcpyHostToDevice, st));
    SV_HIP(hg::launch_batch_plan(g.d_jobs, n, g.d_plan, st));
    const uint32_t grid = (uint32_t)std::max<uint64_t>(2, std::min<uint64_t>(8192, (total_leaves + 63) / 64 + 1));
    SV_HIP(hg::launch_leaves_batch(g.d_jobs, n, g.d_plan, grid, 2, boost, st));
    if (leaf_off) SV_HIP(hipMemcpyAsync(g.h_leaves, g.d_leaves, leaf_off, hipMemcpyDeviceToHost, st));
    return HG_OK;
}

// Content-based chunking of every chunk request of the group (main stream).
int enqueue_chunks(Group &g, const uint8_t *arena, bool want_dig) {
    const uint32_t n = (uint32_t)g.chunks.size();
    const hg_chunk_params &c = g.cp;
    const uint64_t tw = hg::window_scan_tile_windows(c.window, c.stride, c.window_digest);
    if (g.tiles > g.tile_cap) return HG_EINVAL;  // excluded by group formation
    uint64_t nt = 0;
    for (uint32_t f = 0; f < n; f++) {
        const Req *q = g.chunks[f];
        g.h_off[f] = (uint64_t)((uintptr_t)q->dev_in - (uintptr_t)arena);  // modulo 2^64
        g.h_len[f] = q->r.len;
        g.h_first_tile[f] = nt;
        const uint64_t nw = q->r.len >= c.window ? (q->r.len - c.window) / c.stride + 1 : 0;
        for (uint64_t k0 = 0; k0 < nw; k0 += tw) g.h_tiles[nt++] = hg::FileTile{f, 0, k0};
    }
    g.h_first_tile[n] = nt;
    const hg::WsPlan wsp = hg::plan_window_scan_files(nt, g.windows, c.window, c.stride, c.window_digest);
    if (hg::window_scan_scratch_bytes(wsp) > g.ws_bytes) return HG_EINVAL;  // excluded by group formation
    hipStream_t st = g.st;
    SV_HIP(hg::launch_fill_u32((uint32_t *)g.d_status, 8, 0, st));
    SV_HIP(hipMemcpyAsync(g.d_off, g.h_off, (size_t)n * 8, hipMemcpyHostToDevice, st));
    SV_HIP(hipMemcpyAsync(g.d_len, g.h_len, (size_t)n * 8, hipMemcpyHostToDevice, st));
    SV_HIP(hipMemcpyAsync(g.d_first_tile, g.h_first_tile, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, st));
    if (nt) SV_HIP(hipMemcpyAsync(g.d_tiles, g.h_tiles, nt * sizeof(hg::FileTile), hipMemcpyHostToDevice, st));
    hg::WsFiles files{arena, g.d_off, g.d_len, g.d_tiles};
    SV_HIP(hg::launch_window_scan_tiles(wsp, nullptr, 0, c.window, c.stride, c.mask, c.target, g.d_ws, st, &files));
    SV_HIP(hg::launch_window_scan_prefix(wsp, g.d_ws, &g.d_status[0], st));
    SV_HIP(hg::launch_window_scan_emit(wsp, nullptr, 0, c.window, c.stride, c.mask, c.target, g.d_ws, g.d_cand,
                                       g.cand_cap, st, &files));
    hg::FilesChunk fc{g.d_off, g.d_len, g.d_first_tile, hg::window_scan_tile_offsets(wsp, g.d_ws),
                      wsp.n_tiles, g.d_cand, g.cand_cap, g.d_slots, g.d_cnt, g.d_seg_start, g.d_seg_end, n,
                      0, nullptr};
    SV_HIP(hg::launch_files_select(fc, c.window, c.min_chunk, g.d_status, st));
    SV_HIP(hg::launch_files_compact(fc, g.d_chunk_off, g.d_ends, g.max_chunks, g.d_status, st));
    if (want_dig && c.chunk_segment) {
        // Segment digests of the group's chunks: at most bytes / S plus one
        // partial segment per chunk.
        const uint64_t slots = std::min(g.tl_cap, g.bytes / c.chunk_segment + g.max_chunks + 1);
        SV_HIP(hg::launch_chunk_digests_two_level_arena(c.chunk_digest, arena, g.d_seg_start, g.d_seg_end,
                                                        &g.d_status[1], g.max_chunks, c.chunk_segment, g.d_tl,
                                                        g.d_tl_leaves, slots, g.d_cdig, st));
    } else if (want_dig) {
        SV_HIP(hg::launch_segment_digests(c.chunk_digest, arena, 0, g.d_seg_start, g.d_seg_end, &g.d_status[1],
                                          g.max_chunks, g.d_cdig, g.d_seg, st));
    }
    SV_HIP(hipMemcpyAsync(g.h_chunk_off, g.d_chunk_off, (size_t)(n + 1) * 8, hipMemcpyDeviceToHost, st));
    SV_HIP(hipMemcpyAsync(g.h_status, g.d_status, 32, hipMemcpyDeviceToHost, st));
    return HG_OK;
}

// Runs a request alone through the single-call entry points.
int run_alone(Group &g, const Req *q) {
    const hg_request &r = q->r;
    if (r.kind == HG_REQ_BLOCK)
        return hg_block_hash(g.ctx, q->dev_in, r.len, r.block_size, r.digest, r.leaf_out, r.root_out, HG_IN_DEVICE,
                             g.st);
    return hg_chunk(g.ctx, q->dev_in, r.len, &r.chunk, r.chunk_ends, r.capacity, r.n_chunks, r.chunk_digests,
                    HG_IN_DEVICE, g.st);
}

// Enqueues the group, waits for it and writes every member's outputs and
// status.
void execute(Group &g, bool boost) {
    hg_server *s = g.srv;
    std::vector<Req *> all(g.blocks);
    all.insert(all.end(), g.chunks.begin(), g.chunks.end());
    if (g.solo) all.push_back(g.solo);
    int st = HG_OK;
    for (const Req *q : all)
        if (st == HG_OK) st = stage_in(g, q);
    if (st == HG_OK && g.solo) {
        g.solo->status = run_alone(g, g.solo);
        return;
    }
    bool want_dig = false;
    for (const Req *q : g.chunks) want_dig |= q->r.chunk_digests != nullptr;
    if (st == HG_OK && !g.blocks.empty()) {
        // Block work on the helper stream, after the payload copies.
        if (hipEventRecord(g.fork, g.st) != hipSuccess || hipStreamWaitEvent(g.aux, g.fork, 0) != hipSuccess)
            st = HG_EDEVICE;
        if (st == HG_OK) st = enqueue_blocks(g, boost);
        if (st == HG_OK &&
            (hipEventRecord(g.join, g.aux) != hipSuccess || hipStreamWaitEvent(g.st, g.join, 0) != hipSuccess))
            st = HG_EDEVICE;
    }
    if (st == HG_OK && !g.chunks.empty()) st = enqueue_chunks(g, s->stage, want_dig);
    // Wait for whatever was enqueued, also after a failure.
    if (hipStreamSynchronize(g.aux) != hipSuccess) st = HG_EDEVICE;
    if (hipStreamSynchronize(g.st) != hipSuccess) st = HG_EDEVICE;
    if (st != HG_OK) {
        (void)hipGetLastError();
        for (Req *q : all) q->status = st;
        return;
    }
    // Block results, in member order; the second levels on the host pool,
    // longest first.
    std::vector<uint64_t> lofs(g.blocks.size());
    uint64_t leaf_off = 0;
    for (size_t i = 0; i < g.blocks.size(); i++) {
        Req *q = g.blocks[i];
        const hg_request &r = q->r;
        const uint64_t lb = n_leaves(r) * (uint64_t)dbytes(r.digest);
        lofs[i] = leaf_off;
        if (r.leaf_out && lb) memcpy(r.leaf_out, g.h_leaves + leaf_off, lb);
        leaf_off += lb;
        q->status = HG_OK;
    }
    std::vector<size_t> by_len(g.blocks.size());
    std::iota(by_len.begin(), by_len.end(), (size_t)0);
    std::stable_sort(by_len.begin(), by_len.end(),
                     [&](size_t a, size_t b) { return g.blocks[a]->r.len > g.blocks[b]->r.len; });
    hg::host::parallel_for(by_len.size(), [&](uint64_t t) {
        const hg_request &r = g.blocks[by_len[t]]->r;
        if (r.root_out)
            hg::host::digest(r.digest, g.h_leaves + lofs[by_len[t]], n_leaves(r) * (uint64_t)dbytes(r.digest),
                             (uint8_t *)r.root_out);
    });
    if (g.chunks.empty()) return;
    const uint64_t total = g.h_chunk_off[g.chunks.size()];
    if (g.h_status[2] != 0 || total > g.max_chunks) {
        // More candidates than the group holds: serve these requests alone.
        for (Req *q : g.chunks) q->status = run_alone(g, q);
        return;
    }
    const int dc = dbytes(g.cp.chunk_digest);
    int cst = HG_OK;
    if (total) {
        if (hipMemcpyAsync(g.h_ends, g.d_ends, total * 8, hipMemcpyDeviceToHost, g.st) != hipSuccess)
            cst = HG_EDEVICE;
        if (cst == HG_OK && want_dig &&
            hipMemcpyAsync(g.h_cdig, g.d_cdig, total * (uint64_t)dc, hipMemcpyDeviceToHost, g.st) != hipSuccess)
            cst = HG_EDEVICE;
        if (hipStreamSynchronize(g.st) != hipSuccess) cst = HG_EDEVICE;
        if (cst != HG_OK) (void)hipGetLastError();
    }
    for (size_t f = 0; f < g.chunks.size(); f++) {
        Req *q = g.chunks[f];
        if (cst != HG_OK) {
            q->status = cst;
            continue;
        }
        const hg_request &r = q->r;
        const uint64_t c0 = g.h_chunk_off[f], cnt = g.h_chunk_off[f + 1] - c0;
        const uint64_t k = std::min(cnt, r.capacity);
        if (k) memcpy(r.chunk_ends, g.h_ends + c0, k * 8);
        if (k && r.chunk_digests) memcpy(r.chunk_digests, g.h_cdig + c0 * dc, k * (uint64_t)dc);
        *r.n_chunks = cnt;
        q->status = cnt > r.capacity ? HG_ETRUNC : HG_OK;
    }
}

// What the worker still needs of a completed request once the lock is
// released (a waitable request may be freed by hg_wait at any moment after).
struct Completion {
    void (*cb)(uint64_t, int, void *);
    void *user;
    uint64_t id;
    int status;
    std::atomic<uint64_t> *remaining;
    Req *release;
};

Completion finish_locked(hg_server *s, Req *q, Clock::time_point now, bool admitted) {
    if (q->stage_bytes && admitted) s->ranges.give(q->stage_off, q->stage_bytes);
    if (admitted) s->in_flight--;
    s->completed++;
    if (q->status != HG_OK && q->status != HG_ETRUNC) s->failed++;
    s->bytes += q->r.len;
    const double ms = std::chrono::duration<double, std::milli>(now - q->t_arrival).count();
    if (s->lat_ms.size() < LAT_WINDOW) s->lat_ms.push_back(ms);
    else s->lat_ms[s->lat_next % LAT_WINDOW] = ms;
    s->lat_next++;
    if (q->lat_out) *q->lat_out = ms;
    if (q->st_out) *q->st_out = q->status;
    Completion c{q->cb, q->user, q->id, q->status, q->remaining, q->waitable ? nullptr : q};
    q->done = true;
    return c;
}

void worker(Group *gp) {
    Group &g = *gp;
    hg_server *s = g.srv;
    const bool boost = !(s->cfg.flags & HG_BACKGROUND);
    (void)hipSetDevice(s->device);
    while (true) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                if (s->pending.empty()) return s->stopping;
                return admissible(s, s->pending.front());
            });
            if (s->pending.empty()) return;  // stopping and drained
            form(s, g);
        }
        s->cv_work.notify_all();  // the new head may suit another idle worker
        for (Req *q : g.failed) q->status = HG_EDEVICE;
        if (!g.empty()) execute(g, boost);
        std::vector<Req *> done(g.blocks);
        done.insert(done.end(), g.chunks.begin(), g.chunks.end());
        if (g.solo) done.push_back(g.solo);
        const size_t n_admitted = done.size();
        done.insert(done.end(), g.failed.begin(), g.failed.end());
        std::vector<Completion> comp;
        comp.reserve(done.size());
        {
            std::lock_guard<std::mutex> lk(s->mu);
            const Clock::time_point now = Clock::now();
            for (size_t i = 0; i < done.size(); i++) comp.push_back(finish_locked(s, done[i], now, i < n_admitted));
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();  // returned staging bytes may admit the head
        for (const Completion &c : comp) {
            if (c.cb) c.cb(c.id, c.status, c.user);
            if (c.remaining) c.remaining->fetch_sub(1);
            delete c.release;
        }
        {
            // Pairs with the waiter's predicate check under the lock.
            std::lock_guard<std::mutex> lk(s->mu);
        }
        s->cv_done.notify_all();
    }
}

// Nearest-rank percentile.
double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t rank = (size_t)std::ceil(p / 100.0 * (double)v.size());
    rank = std::min(std::max<size_t>(rank, 1), v.size());
    return v[rank - 1];
}

int make_req(hg_server *s, const hg_request *r, Req **out) {
    int st = validate(r);
    if (st != HG_OK) return st;
    const uint64_t need = (r->flags & HG_IN_DEVICE) ? 0 : (r->len + STAGE_ALIGN - 1) / STAGE_ALIGN * STAGE_ALIGN;
    if (need > s->cfg.device_budget) return HG_EBUSY;  // could never be admitted
    Req *q = new Req();
    q->r = *r;
    q->stage_bytes = need;
    *out = q;
    return HG_OK;
}

// Queues q; the id is assigned before any worker can see it.
int enqueue(hg_server *s, Req *q, uint64_t *id) {
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return HG_EBUSY;
        q->id = s->next_id++;
        if (id) *id = q->id;
        if (q->waitable) s->reqs[q->id] = q;
        s->pending.push_back(q);
        s->submitted++;
    }
    s->cv_work.notify_all();
    return HG_OK;
}

}  // namespace

extern "C" {

int hg_server_start(int device, const hg_server_cfg *cfg, hg_server **out) {
    if (!cfg || !out) return HG_EINVAL;
    *out = nullptr;
    if (cfg->slots == 0 || cfg->slots > 64 || cfg->max_requests == 0 || cfg->device_budget == 0 ||
        cfg->max_group_bytes < (1ull << 20) || (cfg->flags & ~(uint32_t)HG_BACKGROUND))
        return HG_EINVAL;
    hg_server *s = new hg_server();
    s->device = device;
    s->cfg = *cfg;
    int st = HG_OK;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        st = HG_EDEVICE;
    }
    if (st == HG_OK && hipMalloc((void **)&s->stage, cfg->device_budget) != hipSuccess) {
        (void)hipGetLastError();
        s->stage = nullptr;
        st = HG_ENOMEM;
    }
    if (st == HG_OK) {
        s->ranges.init(cfg->device_budget);
        s->groups.resize(cfg->slots);
        for (auto &g : s->groups) {
            g.srv = s;
            if ((st = group_init(g, device, *cfg)) != HG_OK) break;
        }
    }
    if (st != HG_OK) {
        for (auto &g : s->groups) group_free(g);
        if (s->stage) (void)hipFree(s->stage);
        delete s;
        return st;
    }
    for (auto &g : s->groups) g.th = std::thread(worker, &g);
    *out = s;
    return HG_OK;
}

int hg_submit(hg_server *s, const hg_request *req, void (*cb)(uint64_t id, int status, void *user), void *user,
              uint64_t *id) {
    if (!s || !id) return HG_EINVAL;
    Req *q;
    int st = make_req(s, req, &q);
    if (st != HG_OK) return st;
    q->cb = cb;
    q->user = user;
    q->waitable = cb == nullptr;
    q->t_arrival = Clock::now();
    if ((st = enqueue(s, q, id)) != HG_OK) delete q;
    return st;
}

int hg_wait(hg_server *s, uint64_t id, int timeout_ms, int *status) {
    if (!s) return HG_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return HG_EINVAL;
    Req *q = it->second;
    auto pred = [&] { return q->done; };
    if (timeout_ms < 0) s->cv_done.wait(lk, pred);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) return HG_EBUSY;
    if (status) *status = q->status;
    s->reqs.erase(it);
    delete q;
    return HG_OK;
}

int hg_server_play(hg_server *s, const hg_request *req, const double *arrival_s, uint64_t n, double *latency_ms,
                   int32_t *status) {
    if (!s || (n && (!req || !arrival_s || !latency_ms || !status))) return HG_EINVAL;
    for (uint64_t i = 1; i < n; i++)
        if (!(arrival_s[i] >= arrival_s[i - 1])) return HG_EINVAL;
    std::atomic<uint64_t> remaining{0};
    const Clock::time_point t0 = Clock::now();
    for (uint64_t i = 0; i < n; i++) {
        const Clock::time_point at =
            t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
        // Sleep most of the gap, spin the last 200 microseconds.
        const Clock::time_point spin_from = at - std::chrono::microseconds(200);
        if (Clock::now() < spin_from) std::this_thread::sleep_until(spin_from);
        while (Clock::now() < at) {
        }
        Req *q;
        int st = make_req(s, &req[i], &q);
        if (st == HG_OK) {
            q->waitable = false;
            q->lat_out = &latency_ms[i];
            q->st_out = &status[i];
            q->remaining = &remaining;
            q->t_arrival = at;
            remaining.fetch_add(1);
            if ((st = enqueue(s, q, nullptr)) != HG_OK) {
                remaining.fetch_sub(1);
                delete q;
            }
        }
        if (st != HG_OK) {
            latency_ms[i] = 0.0;
            status[i] = st;
        }
    }
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return remaining.load() == 0; });
    return HG_OK;
}

int hg_server_stats_read(hg_server *s, hg_server_stats *out) {
    if (!s || !out) return HG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof *out);
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->bytes = s->bytes;
    out->groups = s->n_groups;
    out->queued = s->pending.size();
    out->in_flight = s->in_flight;
    out->max_in_flight = s->max_in_flight;
    out->p50_ms = percentile(s->lat_ms, 50);
    out->p99_ms = percentile(s->lat_ms, 99);
    double sum = 0, mx = 0;
    for (double x : s->lat_ms) {
        sum += x;
        mx = std::max(mx, x);
    }
    out->mean_ms = s->lat_ms.empty() ? 0.0 : sum / (double)s->lat_ms.size();
    out->max_ms = mx;
    return HG_OK;
}

int hg_server_stats_reset(hg_server *s) {
    if (!s) return HG_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->failed = s->bytes = s->n_groups = 0;
    s->max_in_flight = s->in_flight;
    s->lat_ms.clear();
    s->lat_next = 0;
    return HG_OK;
}

int hg_server_stop(hg_server *s) {
    if (!s) return HG_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto &g : s->groups)
        if (g.th.joinable()) g.th.join();
    (void)hipSetDevice(s->device);
    for (auto &g : s->groups) group_free(g);
    if (s->stage) (void)hipFree(s->stage);
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
    return HG_OK;
}

}  // extern "C"
