// hashgpu.cpp -- the C ABI (include/hashgpu.h): argument checks, context
// resources, host<->device staging and the enqueueing of the kernels.
//
// Resource model (the paper's CrystalGPU concerns, Sec. 3.1 and 3.2.3):
//   - device scratch lives in per-purpose slots that grow on demand and are
//     reused by later calls, so steady-state calls allocate nothing;
//   - host input that is not already device-resident is streamed in pieces
//     through a ring of two pinned buffers allocated once per context: the
//     host copy into one buffer, the DMA of the other and the kernels of
//     the previous piece overlap;
//   - pinned memory for callers comes from hg_host_alloc.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "hashgpu.h"
#include "hg_internal.hpp"
#include "hg_ranges.hpp"
#include "host_hash.hpp"

namespace {

enum Slot {
    SLOT_IN = 0,   // device copy of host input (or of dig_a)
    SLOT_IN2,      // device copy of dig_b
    SLOT_IN3,      // device copy of len_b
    SLOT_LEAVES,   // segment digests
    SLOT_LEAVES2,  // second digest's segment digests (fused direct hash)
    SLOT_WS,       // window-scan tile bookkeeping
    SLOT_CAND,     // candidate starts
    SLOT_ENDS,     // chunk ends
    SLOT_DIG,      // chunk digests
    SLOT_TABLE,    // similarity hash set
    SLOT_OUT,      // staging of host outputs
    SLOT_SEL,      // chunk-selection bookkeeping
    SLOT_SEG,      // chunk-digest ordering
    SLOT_JOBS,     // device copy of a host job table
    SLOT_PLAN,     // batch plan
    SLOT_SMALL,    // counts and counters
    SLOT_AUX,      // shifted candidate starts (streaming chunker)
    SLOT_TLEAF,    // segment digests of two-level chunk digests
    SLOT_ROOTS,    // second levels computed on the host, on their way to root_out
    SLOT_SPLIT,    // chunk digests split with the host: starts, indices, host digests
    N_SLOTS
};

constexpr size_t STAGE_PIECE = 64ull << 20;  // bytes per pinned staging buffer
// Host-to-device pieces for window scans: small enough that the tiles of a
// piece hash while the next piece is copied.  (Segment digests keep whole
// staging buffers: each piece's launch lasts as long as a segment's chain,
// so fewer, larger pieces are faster there.)
constexpr size_t SCAN_PIECE = 16ull << 20;
// Segment-digest bytes from which the second level of hg_block_hash runs on
// the host (Sec. 3.2.2 computes it there): one sequential chain, which a
// CPU core runs 10-40x faster than one GPU lane.  Below this, a lane is
// about as quick and the call needs no host wait for it.
constexpr uint64_t HOST_ROOT_MIN = 16u << 10;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Scratch of hg_window_scan_noalloc: a fixed array on every GPU the library
// runs on, held until the process ends.  Host code never uses its name as an
// address (that is a host-side stand-in): hg_create looks up its device
// address once per device, and the calls pass that address to the kernels.
constexpr size_t NOALLOC_SCRATCH = (size_t)HG_NOALLOC_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH];
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

struct TimedLaunch {
    int klass = -1;
    hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

struct hg_ctx {
    int device = 0;
    int last_status = HG_OK;
    std::string last_error;
    DevBuf slot[N_SLOTS];
    uint64_t *host_small = nullptr;  // pinned, 4 KiB
    void *stage[2] = {nullptr, nullptr};
    hipEvent_t stage_free[2] = {nullptr, nullptr};
    hipEvent_t piece_ready = nullptr;
    hipStream_t copy_stream = nullptr;
    std::unordered_set<void *> host_allocs;  // hg_host_alloc blocks without a pinned pool
    // Pools given at hg_create: a device region that every scratch slot is
    // carved from, and a pinned region for hg_host_alloc.
    uint8_t *dpool = nullptr;
    uint64_t dpool_bytes = 0, dpool_used = 0;
    hg::Ranges dranges;
    uint8_t *ppool = nullptr;
    uint64_t ppool_bytes = 0, ppool_used = 0;
    hg::Ranges pranges;
    std::unordered_map<void *, uint64_t> pool_blocks;  // pinned-pool block -> its carved size
    uint64_t n_device_allocs = 0, n_pinned_allocs = 0;
    // Second levels computed on the host: pinned memory for the segment
    // digests copied back and for the roots sent to device outputs, and an
    // event after the last copy out of it.
    uint8_t *hstep = nullptr;
    size_t hstep_bytes = 0;
    hipEvent_t hstep_free = nullptr;
    // Chunk digests split with the host: the input is ready, and one event
    // per group of long chunks copied back.
    hipEvent_t split_ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> split_groups;
    // Kernel timing (hg_timing_*).
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<TimedLaunch> pending;
    uint64_t t_launches[HG_K_COUNT] = {};
    double t_ms[HG_K_COUNT] = {};
    // With an origin event: every launch's [start, end) in ms after it.
    hipEvent_t t_origin = nullptr;
    std::vector<double> t_start[HG_K_COUNT], t_end[HG_K_COUNT];
};

namespace {

int fail(hg_ctx *ctx, int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) {
        ctx->last_status = status;
        ctx->last_error = buf;
    }
    return status;
}

#define HG_HIP(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((ctx), HG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define HG_TRY(expr)            \
    do {                        \
        int r_ = (expr);        \
        if (r_ != HG_OK) return r_; \
    } while (0)

int digest_bytes(int d) { return d == HG_MD5 ? 16 : (d == HG_SHA1 ? 20 : -1); }

// ------------------------------------------------------------ timing --
int take_event(hg_ctx *ctx, hipEvent_t *e) {
    if (!ctx->ev_pool.empty()) {
        *e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return HG_OK;
    }
    HG_HIP(ctx, hipEventCreate(e));
    return HG_OK;
}

int resolve_timing(hg_ctx *ctx) {
    for (TimedLaunch &t : ctx->pending) {
        HG_HIP(ctx, hipEventSynchronize(t.b));
        float ms = 0.f;
        HG_HIP(ctx, hipEventElapsedTime(&ms, t.a, t.b));
        ctx->t_launches[t.klass] += 1;
        ctx->t_ms[t.klass] += ms;
        if (ctx->t_origin) {
            float a = 0.f, b = 0.f;
            HG_HIP(ctx, hipEventElapsedTime(&a, ctx->t_origin, t.a));
            HG_HIP(ctx, hipEventElapsedTime(&b, ctx->t_origin, t.b));
            ctx->t_start[t.klass].push_back(a);
            ctx->t_end[t.klass].push_back(b);
        }
        ctx->ev_pool.push_back(t.a);
        ctx->ev_pool.push_back(t.b);
    }
    ctx->pending.clear();
    return HG_OK;
}

int timed_begin(hg_ctx *ctx, int klass, hipStream_t st, TimedLaunch *t) {
    if (!ctx->timing) return HG_OK;
    if (ctx->pending.size() >= 8192) HG_TRY(resolve_timing(ctx));
    t->klass = klass;
    HG_TRY(take_event(ctx, &t->a));
    HG_TRY(take_event(ctx, &t->b));
    HG_HIP(ctx, hipEventRecord(t->a, st));
    return HG_OK;
}

int timed_end(hg_ctx *ctx, TimedLaunch *t, hipStream_t st) {
    if (t->klass < 0) return HG_OK;
    HG_HIP(ctx, hipEventRecord(t->b, st));
    ctx->pending.push_back(*t);
    return HG_OK;
}

// Launch `expr` (a hipError_t expression) with optional event timing.
#define HG_LAUNCH(ctx, klass, st, expr)                       \
    do {                                                      \
        TimedLaunch tl_;                                      \
        HG_TRY(timed_begin((ctx), (klass), (st), &tl_));      \
        HG_HIP((ctx), (expr));                                \
        HG_TRY(timed_end((ctx), &tl_, (st)));                 \
    } while (0)

int ensure(hg_ctx *ctx, Slot s, size_t bytes, hipStream_t st, void **out) {
    DevBuf &b = ctx->slot[s];
    if (bytes == 0) bytes = 256;
    if (b.bytes < bytes) {
        // The old buffer may still be read by work queued on this stream.
        HG_HIP(ctx, hipStreamSynchronize(st));
        if (ctx->dpool) {
            // Carved from the device pool (64 KiB units); nothing allocated.
            if (b.p) {
                ctx->dranges.give((uint64_t)((uint8_t *)b.p - ctx->dpool), b.bytes);
                ctx->dpool_used -= b.bytes;
            }
            b.p = nullptr;
            b.bytes = 0;
            const size_t want = (bytes + ((64u << 10) - 1)) & ~(size_t)((64u << 10) - 1);
            uint64_t off;
            if (!ctx->dranges.take(want, &off))
                return fail(ctx, HG_ENOMEM, "device pool: no free range of %zu bytes (%llu of %llu in use)", want,
                            (unsigned long long)ctx->dpool_used, (unsigned long long)ctx->dpool_bytes);
            b.p = ctx->dpool + off;
            b.bytes = want;
            ctx->dpool_used += want;
        } else {
            if (b.p) HG_HIP(ctx, hipFree(b.p));
            b.p = nullptr;
            b.bytes = 0;
            size_t want = std::max(bytes, (size_t)1 << 20);
            want = (want + ((1u << 20) - 1)) & ~(size_t)((1u << 20) - 1);
            hipError_t e = hipMalloc(&b.p, want);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                b.p = nullptr;
                return fail(ctx, HG_ENOMEM, "device allocation of %zu bytes failed: %s", want,
                            hipGetErrorString(e));
            }
            ctx->n_device_allocs++;
            b.bytes = want;
        }
    }
    *out = b.p;
    return HG_OK;
}

bool is_pinned_host(const void *p) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeHost;
}

// The copy stream exists only in contexts that stream host input: every
// extra stream shares the device's few hardware queues.
int ensure_copy_stream(hg_ctx *ctx) {
    if (!ctx->copy_stream) HG_HIP(ctx, hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking));
    return HG_OK;
}

int ensure_stage(hg_ctx *ctx) {
    HG_TRY(ensure_copy_stream(ctx));
    if (ctx->stage[0]) return HG_OK;
    for (int i = 0; i < 2; i++) {
        hipError_t e = hipHostMalloc(&ctx->stage[i], STAGE_PIECE, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, HG_ENOMEM, "pinned staging allocation failed: %s", hipGetErrorString(e));
        }
        ctx->n_pinned_allocs++;
        HG_HIP(ctx, hipEventCreateWithFlags(&ctx->stage_free[i], hipEventDisableTiming));
        HG_HIP(ctx, hipEventRecord(ctx->stage_free[i], ctx->copy_stream));
    }
    return HG_OK;
}

// Copies host [src, src+n) to device dst in pieces on the copy stream; after
// each piece `on_piece(off, n_piece)` may enqueue work on `st` that reads
// it.  Pinned sources are DMA'd directly; pageable ones go through the two
// pinned staging buffers.  `align` keeps piece boundaries on multiples of
// the caller's unit (e.g. the segment size).
template <class F>
int stream_in(hg_ctx *ctx, uint8_t *dst, const uint8_t *src, uint64_t n, uint64_t align,
              hipStream_t st, F on_piece, uint64_t piece = STAGE_PIECE, bool after_stream = true,
              bool taper = false) {
    if (n == 0) return HG_OK;
    HG_TRY(ensure_copy_stream(ctx));
    const bool pinned = is_pinned_host(src);
    if (!pinned) HG_TRY(ensure_stage(ctx));
    if (align > 1) piece = std::max<uint64_t>(align, piece - piece % align);
    // Pieces larger than a staging buffer cannot go through it: copy those
    // in one synchronous step.
    if (!pinned && piece > STAGE_PIECE) {
        HG_HIP(ctx, hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st));
        return on_piece(0, n);
    }
    // The copy stream must not overwrite memory still read by earlier work
    // (unless the caller knows that no pending work on st touches dst).
    if (after_stream) {
        HG_HIP(ctx, hipEventRecord(ctx->piece_ready, st));
        HG_HIP(ctx, hipStreamWaitEvent(ctx->copy_stream, ctx->piece_ready, 0));
    }
    // taper (with align 1): the last piece's bytes go in quarters, so that
    // the work left after the last byte lands -- the last piece's share --
    // is short.
    int k = 0;
    uint64_t len = 0;
    for (uint64_t off = 0; off < n; off += len, k ^= 1) {
        len = std::min(piece, n - off);
        if (taper && align == 1 && n - off <= piece && piece >= 4) len = std::min(n - off, piece / 4);
        if (pinned) {
            HG_HIP(ctx, hipMemcpyAsync(dst + off, src + off, len, hipMemcpyHostToDevice, ctx->copy_stream));
        } else {
            HG_HIP(ctx, hipEventSynchronize(ctx->stage_free[k]));
            memcpy(ctx->stage[k], src + off, len);
            HG_HIP(ctx, hipMemcpyAsync(dst + off, ctx->stage[k], len, hipMemcpyHostToDevice,
                                       ctx->copy_stream));
            HG_HIP(ctx, hipEventRecord(ctx->stage_free[k], ctx->copy_stream));
        }
        HG_HIP(ctx, hipEventRecord(ctx->piece_ready, ctx->copy_stream));
        HG_HIP(ctx, hipStreamWaitEvent(st, ctx->piece_ready, 0));
        HG_TRY(on_piece(off, len));
    }
    return HG_OK;
}

// Pieces of host input whose segments one launch takes.  A launch lasts
// as long as one segment's chain (one lane per segment), and launches on one
// stream run one after another, so with long segments per-piece launches
// queue: a 1 MiB SHA-1 segment takes ~19 ms against ~1.3 ms to copy a
// 64 MiB piece.  The group size is chosen by simulating the schedule --
// group k starts when its last piece has landed and group k-1 has ended,
// and takes one chain -- and taking the earliest finish (the smallest group
// on a tie).  Estimates: one 64-byte block per lane every ~0.6 us (MD5) /
// ~1.15 us (SHA-1) / ~1.75 us (both), ~50 GB/s of host-to-device copy.
uint64_t pieces_per_launch(uint64_t len, uint64_t block_size, double us_per_block, uint64_t piece) {
    const double chain = (double)((block_size + 63) / 64) * us_per_block * 1e-6;
    const double copy = (double)piece / 50e9;
    const uint64_t n = std::max<uint64_t>(1, (len + piece - 1) / piece);
    if (n > 4096) return 1;  // far more copy than any chain: per piece
    uint64_t best_g = 1;
    double best = 0;
    for (uint64_t g = 1; g <= n; g++) {
        double end = 0;
        for (uint64_t last = g; ; last = std::min(n, last + g)) {
            end = std::max(end, (double)last * copy) + chain;
            if (last == n) break;
        }
        if (g == 1 || end < best * (1 - 1e-9)) {
            best = end;
            best_g = g;
        }
    }
    return best_g;
}

// Device view of an input argument: the pointer itself, or a device copy.
int device_input(hg_ctx *ctx, Slot s, const void *p, uint64_t n, bool on_device, hipStream_t st,
                 const uint8_t **out) {
    if (on_device || n == 0) {
        *out = (const uint8_t *)p;
        return HG_OK;
    }
    void *d;
    HG_TRY(ensure(ctx, s, n, st, &d));
    HG_TRY(stream_in(ctx, (uint8_t *)d, (const uint8_t *)p, n, 1, st,
                     [](uint64_t, uint64_t) { return (int)HG_OK; }));
    *out = (const uint8_t *)d;
    return HG_OK;
}

// Window scan pass 1 over an input that is on the device or in host memory.
// Host input is streamed into SLOT_IN in pieces; after each piece, the tiles
// whose windows lie entirely in the bytes that have landed are launched, so
// the copy of later pieces overlaps the hashing of earlier ones.
int scan_tiles_from(hg_ctx *ctx, const void *in, uint64_t len, bool in_dev, uint32_t w, uint32_t s, uint32_t mask,
                    uint32_t target, int kind, hipStream_t st, const uint8_t **din_out, hg::WsPlan *plan_out,
                    void **ws_out) {
    const uint8_t *din = (const uint8_t *)in;
    if (!in_dev && len) {
        void *p;
        HG_TRY(ensure(ctx, SLOT_IN, len, st, &p));
        din = (const uint8_t *)p;
    }
    const hg::WsPlan plan = hg::plan_window_scan(din, len, w, s, kind);
    void *ws;
    HG_TRY(ensure(ctx, SLOT_WS, hg::window_scan_scratch_bytes(plan), st, &ws));
    if (in_dev || len == 0) {
        HG_LAUNCH(ctx, HG_K_WINDOW_TILES, st, hg::launch_window_scan_tiles(plan, din, len, w, s, mask, target, ws, st));
    } else {
        uint64_t t_done = 0;
        HG_TRY(stream_in(ctx, (uint8_t *)din, (const uint8_t *)in, len, 1, st,
                         [&](uint64_t off, uint64_t plen) -> int {
                             const uint64_t avail = off + plen;
                             uint64_t t_end = plan.n_tiles;
                             if (avail < len) {
                                 const uint64_t nw = avail >= w ? (avail - w) / s + 1 : 0;
                                 t_end = std::min<uint64_t>(nw / plan.tile_windows, plan.n_tiles);
                             }
                             if (t_end > t_done) {
                                 HG_LAUNCH(ctx, HG_K_WINDOW_TILES, st,
                                           hg::launch_window_scan_tile_range(plan, din, len, w, s, mask, target, ws,
                                                                             t_done, t_end, st));
                                 t_done = t_end;
                             }
                             return HG_OK;
                         },
                         SCAN_PIECE, true, true));
    }
    *din_out = din;
    *plan_out = plan;
    *ws_out = ws;
    return HG_OK;
}

int check_flags(hg_ctx *ctx, uint32_t flags, bool async_ok) {
    if (flags & ~(uint32_t)(HG_IN_DEVICE | HG_OUT_DEVICE | HG_ASYNC))
        return fail(ctx, HG_EINVAL, "unknown flag bits 0x%x", flags);
    if (flags & HG_ASYNC) {
        if (!async_ok) return fail(ctx, HG_EINVAL, "HG_ASYNC is not accepted by this call");
        if ((flags & (HG_IN_DEVICE | HG_OUT_DEVICE)) != (HG_IN_DEVICE | HG_OUT_DEVICE))
            return fail(ctx, HG_EINVAL, "HG_ASYNC requires HG_IN_DEVICE and HG_OUT_DEVICE");
    }
    return HG_OK;
}

// Small device words (counts, counters) live in SLOT_SMALL.
int small_words(hg_ctx *ctx, hipStream_t st, uint64_t **out) {
    void *p;
    HG_TRY(ensure(ctx, SLOT_SMALL, 4096, st, &p));
    *out = (uint64_t *)p;
    return HG_OK;
}

// Reads one device uint64 (synchronizes the stream); with words = 2 the
// next word too, left in host_small[1].
int read_u64(hg_ctx *ctx, const uint64_t *dev, hipStream_t st, uint64_t *v, int words = 1) {
    HG_HIP(ctx, hipMemcpyAsync(ctx->host_small, dev, 8 * (size_t)words, hipMemcpyDeviceToHost, st));
    HG_HIP(ctx, hipStreamSynchronize(st));
    *v = ctx->host_small[0];
    return HG_OK;
}

int copy_out(hg_ctx *ctx, void *dst, const void *src, size_t n, bool dst_device, hipStream_t st) {
    if (n == 0) return HG_OK;
    HG_HIP(ctx, hipMemcpyAsync(dst, src, n, dst_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    return HG_OK;
}

// Pinned memory for the host's second levels: `roots` bytes for root
// outputs followed by `digests` bytes of segment digests.  Waits until the
// copies out of it that earlier calls enqueued have finished.
int host_step_buffer(hg_ctx *ctx, size_t roots, size_t digests, uint8_t **r, uint8_t **dg) {
    roots = (roots + 255) & ~(size_t)255;
    const size_t want = roots + digests;
    if (!ctx->hstep_free) HG_HIP(ctx, hipEventCreateWithFlags(&ctx->hstep_free, hipEventDisableTiming));
    else HG_HIP(ctx, hipEventSynchronize(ctx->hstep_free));
    if (ctx->hstep_bytes < want) {
        if (ctx->hstep) HG_HIP(ctx, hipHostFree(ctx->hstep));
        ctx->hstep = nullptr;
        ctx->hstep_bytes = 0;
        size_t sz = std::max(want, (size_t)1 << 20);
        sz = (sz + ((1u << 20) - 1)) & ~(size_t)((1u << 20) - 1);
        hipError_t e = hipHostMalloc((void **)&ctx->hstep, sz, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ctx->hstep = nullptr;
            return fail(ctx, HG_ENOMEM, "pinned allocation of %zu bytes failed: %s", sz, hipGetErrorString(e));
        }
        ctx->n_pinned_allocs++;
        ctx->hstep_bytes = sz;
    }
    *r = ctx->hstep;
    *dg = ctx->hstep + roots;
    return HG_OK;
}

// One second level computed on the host.
struct HostRoot {
    int kind;
    const uint8_t *digests;  // device pointer, or host pointer when on_host
    uint64_t bytes;
    bool on_host;
    uint8_t *out;            // host: d bytes
};

// The second levels of `roots` on the host's cores (Sec. 3.2.2): device
// digest buffers are copied back into `stage` (room for all of them) on st,
// the stream is synchronized, and the pool hashes the buffers, longest first.
int host_roots(hg_ctx *ctx, HostRoot *roots, size_t n, uint8_t *stage, hipStream_t st) {
    uint64_t off = 0;
    for (size_t i = 0; i < n; i++) {
        if (roots[i].on_host || roots[i].bytes == 0) continue;
        HG_HIP(ctx, hipMemcpyAsync(stage + off, roots[i].digests, roots[i].bytes, hipMemcpyDeviceToHost, st));
        roots[i].digests = stage + off;
        roots[i].on_host = true;
        off += roots[i].bytes;
    }
    HG_HIP(ctx, hipStreamSynchronize(st));
    std::vector<size_t> order(n);
    std::iota(order.begin(), order.end(), (size_t)0);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return roots[a].bytes > roots[b].bytes; });
    hg::host::parallel_for(n, [&](uint64_t k) {
        const HostRoot &r = roots[order[k]];
        hg::host::digest(r.kind, r.digests, r.bytes, r.out);
    });
    return HG_OK;
}

// Longest chunk from which hg_chunk considers hashing chunks on the host.
constexpr uint64_t HOST_CHUNK_MIN = 64u << 10;

// Standard chunk digests with the longest chunks hashed on the host: each
// digest is one sequential chain, which one GPU lane runs at ~55 MB/s
// (SHA-1) and a CPU core at 0.5-2 GB/s.  The host reads the nc chunk ends,
// picks the k longest chunks by a cost model (the host's copy and hash time
// against the GPU's longest remaining chain), and hashes them on the host
// pool -- from the caller's host input if there is one, else from a copy
// made on the copy stream -- while the GPU hashes the others (the long ones
// get an empty range there); a scatter then puts the host digests in place.
// *split = false when the model keeps everything on the GPU (nothing done).
int chunk_digests_split(hg_ctx *ctx, int kind, const uint8_t *din, const uint8_t *hin, uint64_t len,
                        const uint64_t *dends, const uint64_t *n_dev, uint64_t nc, uint8_t *ddig, hipStream_t st,
                        bool *split) {
    *split = false;
    if (nc == 0) return HG_OK;
    std::vector<uint64_t> ends(nc);
    HG_HIP(ctx, hipMemcpyAsync(ends.data(), dends, nc * 8, hipMemcpyDeviceToHost, st));
    HG_HIP(ctx, hipStreamSynchronize(st));
    std::vector<uint64_t> lens(nc), order;
    for (uint64_t j = 0; j < nc; j++) lens[j] = ends[j] - (j ? ends[j - 1] : 0);
    const double lane = kind == HG_MD5 ? 110e6 : 55e6;
    const double core = kind == HG_MD5 ? 0.5e9 : (hg::host::sha1_accelerated() ? 1.5e9 : 0.5e9);
    const double cores = (double)hg::host::pool_threads() + 1;
    const double copy = hin ? 0.0 : 1.0 / 40e9;
    const uint64_t kmax = std::min<uint64_t>(nc, 1u << 16);
    // Chunks longest first (ties by position).  The cost model below only
    // walks the head of that order -- the host's time never falls as it
    // takes more chunks, so the walk ends once that time alone reaches the
    // best split so far -- so only a prefix is selected and sorted (a full
    // sort of tens of thousands of chunks costs milliseconds), and widened
    // if the walk runs past it.
    std::vector<std::pair<uint64_t, uint64_t>> key(nc);
    for (uint64_t j = 0; j < nc; j++) key[j] = {lens[j], j};
    const auto longer = [](const std::pair<uint64_t, uint64_t> &a, const std::pair<uint64_t, uint64_t> &b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;
    };
    uint64_t best_k = 0;
    double best = 0;
    for (uint64_t m = std::min<uint64_t>(nc, 2048);; m = std::min<uint64_t>(nc, m * 8)) {
        std::nth_element(key.begin(), key.begin() + (m - 1), key.end(), longer);
        std::sort(key.begin(), key.begin() + m, longer);
        best_k = 0;
        best = (double)key[0].first / lane;
        uint64_t bytes = 0;
        bool done = false;
        // k chunks on the host needs the (k+1)-th longest for the GPU's time.
        const uint64_t kend = std::min<uint64_t>(kmax, m == nc ? nc : m - 1);
        for (uint64_t k = 1; k <= kend; k++) {
            bytes += key[k - 1].first;
            // The copy (in groups of ~16 MiB) and the hashing overlap: the
            // host is done after the whole copy and the last group's
            // hashing, or after the first group's copy and all the hashing
            // (the longest chunk on one core), whichever is later.
            const double group = std::min<double>((double)bytes, (double)(16u << 20));
            const double hash_all = std::max((double)key[0].first / core, (double)bytes / (core * cores));
            const double host_t =
                std::max((double)bytes * copy + group / (core * cores), group * copy + hash_all);
            const double gpu_t = k < nc ? (double)key[k].first / lane : 0.0;
            const double t = std::max(host_t, gpu_t);
            if (t < best) {
                best = t;
                best_k = k;
            }
            // Past the best for good, or the rest are short: nothing more
            // to gain.
            if (host_t >= best || gpu_t < 1e-4) {
                done = true;
                break;
            }
        }
        if (done || m == nc || kend == kmax) break;
    }
    if (best_k == 0) return HG_OK;
    order.resize(best_k);
    for (uint64_t i = 0; i < best_k; i++) order[i] = key[i].second;
    const uint64_t k = best_k;
    std::vector<uint8_t> is_long(nc, 0);
    uint64_t host_bytes = 0;
    for (uint64_t i = 0; i < k; i++) {
        is_long[order[i]] = 1;
        host_bytes += lens[order[i]];
    }
    // Long chunks in position order, and the contiguous runs they form.
    std::vector<uint64_t> idx;
    idx.reserve(k);
    for (uint64_t j = 0; j < nc; j++)
        if (is_long[j]) idx.push_back(j);
    const int d = digest_bytes(kind);
    // Device and pinned host alike: indices (k), host digests (k * 20),
    // GPU-side starts (nc), and for device input the gather table (k
    // records: source offset, length, packed offset); then, pinned only,
    // the long chunks' bytes (and on the device, packed the same way).
    // Device input: slices of GATHER_SLICE bytes, and up to 15 bytes of
    // padding per chunk so that each packed chunk keeps its source's address
    // modulo 16.
    constexpr uint64_t GATHER_SLICE = 64u << 10;
    uint64_t n_slices = 0;
    if (!hin)
        for (uint64_t i = 0; i < k; i++) n_slices += (lens[idx[i]] + GATHER_SLICE - 1) / GATHER_SLICE;
    const size_t ibytes = (k * 8 + 255) & ~(size_t)255, gbytes = (k * 20 + 255) & ~(size_t)255,
                 sbytes = (nc * 8 + 255) & ~(size_t)255, tbytes = hin ? 0 : (n_slices * 24 + 255) & ~(size_t)255;
    const size_t pbytes = hin ? 0 : host_bytes + 16 * k;
    void *dsplit;
    HG_TRY(ensure(ctx, SLOT_SPLIT, ibytes + gbytes + sbytes + tbytes + pbytes, st, &dsplit));
    uint64_t *didx = (uint64_t *)dsplit;
    uint8_t *ddg = (uint8_t *)dsplit + ibytes;
    uint64_t *dstarts = (uint64_t *)(ddg + gbytes);
    uint64_t *dtab = (uint64_t *)((uint8_t *)dstarts + sbytes);
    uint8_t *dpacked = (uint8_t *)dtab + tbytes;
    uint8_t *hr, *hbytes;
    HG_TRY(host_step_buffer(ctx, ibytes + gbytes + sbytes + tbytes, pbytes, &hr, &hbytes));
    memcpy(hr, idx.data(), k * 8);
    uint8_t *hdig = hr + ibytes;
    uint64_t *hstarts = (uint64_t *)(hdig + gbytes);
    uint64_t *htab = (uint64_t *)((uint8_t *)hstarts + sbytes);
    for (uint64_t j = 0; j < nc; j++) hstarts[j] = is_long[j] ? ends[j] : (j ? ends[j - 1] : 0);
    for (int i = 0; i < 2; i++)
        if (!ctx->split_ev[i]) HG_HIP(ctx, hipEventCreateWithFlags(&ctx->split_ev[i], hipEventDisableTiming));
    // Host order: longest first (the longest chain sets the host's time).
    std::vector<uint64_t> by_len(k);
    std::iota(by_len.begin(), by_len.end(), (uint64_t)0);
    std::stable_sort(by_len.begin(), by_len.end(),
                     [&](uint64_t a, uint64_t b) { return lens[idx[a]] > lens[idx[b]]; });
    std::vector<const uint8_t *> src(k);
    std::vector<uint32_t> group(k, 0);
    uint32_t n_groups = 0;
    if (!hin) {
        // The long chunks' bytes come back on the copy stream (the input is
        // complete on st): packed on the device in host order by one
        // kernel, then copied in groups of ~16 MiB with an event each, so
        // that hashing starts as soon as the first group has landed and
        // overlaps the rest of the copy -- and the GPU's share runs
        // meanwhile.  (One copy per chunk costs far more: each small copy
        // has a fixed cost of its own.)
        HG_TRY(ensure_copy_stream(ctx));
        uint64_t off = 0, ns = 0;
        for (uint64_t t = 0; t < k; t++) {
            const uint64_t i = by_len[t], j = idx[i], a = j ? ends[j - 1] : 0;
            off += (((uintptr_t)(din + a) & 15) - off) & 15;  // same address modulo 16
            src[i] = hbytes + off;
            for (uint64_t q = 0; q < lens[j]; q += GATHER_SLICE, ns++) {
                htab[3 * ns] = a + q;
                htab[3 * ns + 1] = std::min<uint64_t>(GATHER_SLICE, lens[j] - q);
                htab[3 * ns + 2] = off + q;
            }
            off += lens[j];
        }
        HG_HIP(ctx, hipEventRecord(ctx->split_ev[0], st));
        HG_HIP(ctx, hipStreamWaitEvent(ctx->copy_stream, ctx->split_ev[0], 0));
        HG_HIP(ctx, hipMemcpyAsync(dtab, htab, ns * 24, hipMemcpyHostToDevice, ctx->copy_stream));
        HG_HIP(ctx, hg::launch_gather_ranges(din, dtab, ns, dpacked, ctx->copy_stream));
        uint64_t g0 = 0, in_group = 0;
        for (uint64_t t = 0; t < k; t++) {
            const uint64_t i = by_len[t];
            group[i] = n_groups;
            in_group += lens[idx[i]];
            if (in_group >= (16u << 20) || t + 1 == k) {
                const uint64_t g1 = (uint64_t)(src[i] - hbytes) + lens[idx[i]];
                HG_HIP(ctx, hipMemcpyAsync(hbytes + g0, dpacked + g0, g1 - g0, hipMemcpyDeviceToHost,
                                           ctx->copy_stream));
                if (ctx->split_groups.size() <= n_groups) {
                    hipEvent_t e;
                    HG_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
                    ctx->split_groups.push_back(e);
                }
                HG_HIP(ctx, hipEventRecord(ctx->split_groups[n_groups], ctx->copy_stream));
                n_groups++;
                in_group = 0;
                g0 = g1;
            }
        }
    } else {
        for (uint64_t i = 0; i < k; i++) src[i] = hin + (idx[i] ? ends[idx[i] - 1] : 0);
    }
    // The GPU's share: the long chunks are empty ranges there.
    HG_HIP(ctx, hipMemcpyAsync(dstarts, hstarts, sbytes, hipMemcpyHostToDevice, st));
    void *segs;
    HG_TRY(ensure(ctx, SLOT_SEG, hg::segment_digest_scratch_bytes(nc), st, &segs));
    HG_LAUNCH(ctx, HG_K_CHUNK_DIGESTS, st,
              hg::launch_segment_digests(kind, din, len, dstarts, dends, n_dev, nc, ddig, segs, st));
    // The host's share, longest first, each chunk once its group has landed.
    std::atomic<int> copy_err{0};
    hg::host::parallel_for(k, [&](uint64_t t) {
        const uint64_t i = by_len[t];
        if (!hin && hipEventSynchronize(ctx->split_groups[group[i]]) != hipSuccess) {
            copy_err.store(1);
            return;
        }
        hg::host::digest(kind, src[i], lens[idx[i]], hdig + i * (uint64_t)d);
    });
    if (copy_err.load()) return fail(ctx, HG_EDEVICE, "copy of long chunks to the host failed");
    HG_HIP(ctx, hipMemcpyAsync(didx, hr, ibytes + k * 20, hipMemcpyHostToDevice, st));
    HG_HIP(ctx, hipEventRecord(ctx->hstep_free, st));
    HG_LAUNCH(ctx, HG_K_CHUNK_DIGESTS, st, hg::launch_digest_scatter(didx, ddg, k, d, ddig, st));
    *split = true;
    return HG_OK;
}

// Digests of the chunks [ends[j-1], ends[j]) of in[0, len) (*n_dev <= max_n
// of them): the standard digest of each chunk's bytes, or with chunk_segment
// the two-level direct hash of each chunk.
int chunk_digests_of(hg_ctx *ctx, const hg_chunk_params &p, const uint8_t *in, uint64_t len, const uint64_t *ends,
                     const uint64_t *n_dev, uint64_t max_n, uint8_t *out, hipStream_t st) {
    if (max_n == 0) return HG_OK;
    if (p.chunk_segment) {
        void *leaves;
        const uint64_t slots = hg::two_level_slots(len, max_n, p.chunk_segment);
        if (slots >= hg::MAX_LANES)
            return fail(ctx, HG_EINVAL, "%llu segments (limit 2^31 per call): use a larger chunk_segment",
                        (unsigned long long)slots);
        HG_TRY(ensure(ctx, SLOT_TLEAF, slots * (uint64_t)digest_bytes(p.chunk_digest), st, &leaves));
        HG_LAUNCH(ctx, HG_K_CHUNK_DIGESTS, st,
                  hg::launch_chunk_digests_two_level(p.chunk_digest, in, len, ends, n_dev, max_n, p.chunk_segment,
                                                     (uint8_t *)leaves, out, st));
        return HG_OK;
    }
    void *segs;
    HG_TRY(ensure(ctx, SLOT_SEG, hg::segment_digest_scratch_bytes(max_n), st, &segs));
    HG_LAUNCH(ctx, HG_K_CHUNK_DIGESTS, st,
              hg::launch_segment_digests(p.chunk_digest, in, len, nullptr, ends, n_dev, max_n, out, segs, st));
    return HG_OK;
}

int enter(hg_ctx *ctx) {
    if (!ctx) return HG_EINVAL;
    ctx->last_status = HG_OK;
    ctx->last_error.clear();
    HG_HIP(ctx, hipSetDevice(ctx->device));
    return HG_OK;
}

}  // namespace

// ======================================================================= ABI

extern "C" {

const char *hg_strerror(int status) {
    switch (status) {
        case HG_OK: return "ok";
        case HG_EINVAL: return "invalid argument";
        case HG_ENOMEM: return "out of memory";
        case HG_EDEVICE: return "device error";
        case HG_ETRUNC: return "output truncated";
        case HG_EBUSY: return "busy";
        default: return "unknown status";
    }
}

int hg_host_hash(int digest, const void *in, uint64_t len, void *out) {
    if (digest_bytes(digest) < 0 || !out || (len && !in)) return HG_EINVAL;
    hg::host::digest(digest, (const uint8_t *)in, len, (uint8_t *)out);
    return HG_OK;
}

int hg_digest_size(int digest) {
    int d = digest_bytes(digest);
    return d < 0 ? HG_EINVAL : d;
}

int hg_last_error(const hg_ctx *ctx, char *buf, size_t n) {
    if (!ctx) return HG_EINVAL;
    if (buf && n) {
        size_t k = std::min(n - 1, ctx->last_error.size());
        memcpy(buf, ctx->last_error.data(), k);
        buf[k] = 0;
    }
    return ctx->last_status;
}

int hg_create(int device, size_t device_pool_bytes, size_t pinned_pool_bytes, hg_ctx **out) {
    if (!out) return HG_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return HG_EDEVICE;
    }
    if (device < 0 || device >= n) return HG_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HG_EDEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HG_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return HG_EDEVICE;
    hg_ctx *ctx = new hg_ctx();
    ctx->device = device;
    if (hipHostMalloc((void **)&ctx->host_small, 4096, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->piece_ready, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        hg_destroy(ctx);
        return HG_EDEVICE;
    }
    ctx->n_pinned_allocs++;
    if (device_pool_bytes) {
        const uint64_t sz = (device_pool_bytes + ((64u << 10) - 1)) & ~(uint64_t)((64u << 10) - 1);
        if (hipMalloc((void **)&ctx->dpool, sz) != hipSuccess) {
            (void)hipGetLastError();
            ctx->dpool = nullptr;
            hg_destroy(ctx);
            return HG_ENOMEM;
        }
        ctx->n_device_allocs++;
        ctx->dpool_bytes = sz;
        ctx->dranges.init(sz);
    }
    if (device >= MAX_DEVICES) {
        hg_destroy(ctx);
        return HG_EDEVICE;
    }
    {
        // Device address of this GPU's copy of the fixed scratch array, looked
        // up once per device with the device current.
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) {
                (void)hipGetLastError();
                hg_destroy(ctx);
                return HG_EDEVICE;
            }
            g_scratch_ptr[device] = ptr;
        }
    }
    if (pinned_pool_bytes) {
        const uint64_t sz = (pinned_pool_bytes + 255) & ~(uint64_t)255;
        if (hipHostMalloc((void **)&ctx->ppool, sz, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            ctx->ppool = nullptr;
            hg_destroy(ctx);
            return HG_ENOMEM;
        }
        ctx->n_pinned_allocs++;
        ctx->ppool_bytes = sz;
        ctx->pranges.init(sz);
    }
    *out = ctx;
    return HG_OK;
}

void hg_destroy(hg_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (!ctx->dpool)
        for (auto &b : ctx->slot)
            if (b.p) (void)hipFree(b.p);
    if (ctx->dpool) (void)hipFree(ctx->dpool);
    if (ctx->ppool) (void)hipHostFree(ctx->ppool);
    for (int i = 0; i < 2; i++) {
        if (ctx->stage[i]) (void)hipHostFree(ctx->stage[i]);
        if (ctx->stage_free[i]) (void)hipEventDestroy(ctx->stage_free[i]);
    }
    for (void *p : ctx->host_allocs) (void)hipHostFree(p);
    for (TimedLaunch &t : ctx->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->host_small) (void)hipHostFree(ctx->host_small);
    if (ctx->hstep) (void)hipHostFree(ctx->hstep);
    if (ctx->hstep_free) (void)hipEventDestroy(ctx->hstep_free);
    for (hipEvent_t e : ctx->split_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->split_groups) (void)hipEventDestroy(e);
    if (ctx->piece_ready) (void)hipEventDestroy(ctx->piece_ready);
    if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
    delete ctx;
}

int hg_ctx_stats_read(const hg_ctx *ctx, hg_ctx_stats *out) {
    if (!ctx || !out) return HG_EINVAL;
    out->device_pool_bytes = ctx->dpool_bytes;
    out->device_pool_used = ctx->dpool_used;
    out->pinned_pool_bytes = ctx->ppool_bytes;
    out->pinned_pool_used = ctx->ppool_used;
    out->device_allocs = ctx->n_device_allocs;
    out->pinned_allocs = ctx->n_pinned_allocs;
    out->host_blocks = ctx->ppool ? ctx->pool_blocks.size() : ctx->host_allocs.size();
    return HG_OK;
}

int hg_host_alloc(hg_ctx *ctx, size_t bytes, void **out) {
    HG_TRY(enter(ctx));
    if (!out || bytes == 0) return fail(ctx, HG_EINVAL, "hg_host_alloc: NULL out or zero size");
    *out = nullptr;
    if (ctx->ppool) {
        // First fit in 256-byte units from the pinned pool.
        const uint64_t want = ((uint64_t)bytes + 255) & ~(uint64_t)255;
        uint64_t off;
        if (want < bytes || !ctx->pranges.take(want, &off))
            return fail(ctx, HG_ENOMEM, "pinned pool: no free range of %zu bytes (%llu of %llu in use)", bytes,
                        (unsigned long long)ctx->ppool_used, (unsigned long long)ctx->ppool_bytes);
        void *p = ctx->ppool + off;
        ctx->pool_blocks[p] = want;
        ctx->ppool_used += want;
        *out = p;
        return HG_OK;
    }
    void *p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, HG_ENOMEM, "pinned allocation of %zu bytes failed: %s", bytes,
                    hipGetErrorString(e));
    }
    ctx->n_pinned_allocs++;
    ctx->host_allocs.insert(p);
    *out = p;
    return HG_OK;
}

int hg_host_free(hg_ctx *ctx, void *p) {
    HG_TRY(enter(ctx));
    if (!p) return HG_OK;
    if (ctx->ppool) {
        auto it = ctx->pool_blocks.find(p);
        if (it == ctx->pool_blocks.end())
            return fail(ctx, HG_EINVAL, "pointer is not a live block of this context's pinned pool");
        ctx->pranges.give((uint64_t)((uint8_t *)p - ctx->ppool), it->second);
        ctx->ppool_used -= it->second;
        ctx->pool_blocks.erase(it);
        return HG_OK;
    }
    auto it = ctx->host_allocs.find(p);
    if (it == ctx->host_allocs.end()) return fail(ctx, HG_EINVAL, "pointer not from hg_host_alloc");
    ctx->host_allocs.erase(it);
    HG_HIP(ctx, hipHostFree(p));
    return HG_OK;
}

int hg_block_hash(hg_ctx *ctx, const void *in, uint64_t len, uint64_t block_size, int digest,
                  void *leaf_out, void *root_out, uint32_t flags, void *stream) {
    HG_TRY(enter(ctx));
    HG_TRY(check_flags(ctx, flags, true));
    const int d = digest_bytes(digest);
    if (d < 0) return fail(ctx, HG_EINVAL, "unknown digest %d", digest);
    if (block_size == 0) return fail(ctx, HG_EINVAL, "block_size must be >= 1");
    if (!leaf_out && !root_out) return fail(ctx, HG_EINVAL, "leaf_out and root_out are both NULL");
    if (len && !in) return fail(ctx, HG_EINVAL, "in is NULL");
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    const uint64_t n = len ? (len + block_size - 1) / block_size : 0;

    uint8_t *leaves;
    if (leaf_out && out_dev) {
        leaves = (uint8_t *)leaf_out;
    } else {
        void *p;
        HG_TRY(ensure(ctx, SLOT_LEAVES, n * (uint64_t)d, st, &p));
        leaves = (uint8_t *)p;
    }
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    uint8_t *root = (root_out && out_dev) ? (uint8_t *)root_out : (uint8_t *)small;

    if (in_dev || len == 0) {
        HG_LAUNCH(ctx, HG_K_LEAVES, st, hg::launch_leaves(digest, (const uint8_t *)in, len, block_size, n, leaves, st));
    } else {
        void *dp;
        HG_TRY(ensure(ctx, SLOT_IN, len, st, &dp));
        uint8_t *din = (uint8_t *)dp;
        // Pieces hold whole segments; the segments of a group of pieces are
        // hashed as soon as the group has landed.
        const uint64_t group = pieces_per_launch(len, block_size, digest == HG_MD5 ? 0.6 : 1.15, STAGE_PIECE);
        uint64_t from = 0, npieces = 0;
        HG_TRY(stream_in(ctx, din, (const uint8_t *)in, len, block_size, st,
                         [&](uint64_t off, uint64_t plen) -> int {
                             if (++npieces % group != 0 && off + plen < len) return HG_OK;
                             const uint64_t k0 = from / block_size;
                             const uint64_t k1 = (off + plen + block_size - 1) / block_size;
                             HG_LAUNCH(ctx, HG_K_LEAVES, st,
                                       hg::launch_leaves(digest, din + from, off + plen - from, block_size, k1 - k0,
                                                         leaves + k0 * (uint64_t)d, st));
                             from = off + plen;
                             return HG_OK;
                         }));
    }
    const uint64_t dbytes = n * (uint64_t)d;
    if (leaf_out && !out_dev) HG_TRY(copy_out(ctx, leaf_out, leaves, dbytes, false, st));
    if (root_out && dbytes >= HOST_ROOT_MIN) {
        // The second level on the host: it waits for the segment digests.
        uint8_t *hr, *hd;
        HG_TRY(host_step_buffer(ctx, 64, leaf_out && !out_dev ? 0 : dbytes, &hr, &hd));
        const bool have = leaf_out && !out_dev;
        HostRoot r{digest, have ? (const uint8_t *)leaf_out : leaves, dbytes, have, out_dev ? hr : (uint8_t *)root_out};
        HG_TRY(host_roots(ctx, &r, 1, hd, st));
        if (out_dev) {
            HG_HIP(ctx, hipMemcpyAsync(root_out, hr, (size_t)d, hipMemcpyHostToDevice, st));
            HG_HIP(ctx, hipEventRecord(ctx->hstep_free, st));
        }
    } else if (root_out) {
        HG_LAUNCH(ctx, HG_K_ROOT, st, hg::launch_hash_one(digest, leaves, dbytes, root, st));
        if (!out_dev) HG_TRY(copy_out(ctx, root_out, root, (size_t)d, false, st));
    }
    if (!(flags & HG_ASYNC)) HG_HIP(ctx, hipStreamSynchronize(st));
    return HG_OK;
}

int hg_block_hash_dual(hg_ctx *ctx, const void *in, uint64_t len, uint64_t block_size, void *md5_leaf_out,
                       void *md5_root_out, void *sha1_leaf_out, void *sha1_root_out, uint32_t flags,
                       void *stream) {
    HG_TRY(enter(ctx));
    HG_TRY(check_flags(ctx, flags, true));
    if (block_size == 0) return fail(ctx, HG_EINVAL, "block_size must be >= 1");
    if (!md5_leaf_out && !md5_root_out && !sha1_leaf_out && !sha1_root_out)
        return fail(ctx, HG_EINVAL, "all outputs are NULL");
    if (len && !in) return fail(ctx, HG_EINVAL, "in is NULL");
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    const uint64_t n = len ? (len + block_size - 1) / block_size : 0;
    uint8_t *lm, *ls;
    void *p;
    if (md5_leaf_out && out_dev) {
        lm = (uint8_t *)md5_leaf_out;
    } else {
        HG_TRY(ensure(ctx, SLOT_LEAVES, n * 16, st, &p));
        lm = (uint8_t *)p;
    }
    if (sha1_leaf_out && out_dev) {
        ls = (uint8_t *)sha1_leaf_out;
    } else {
        HG_TRY(ensure(ctx, SLOT_LEAVES2, n * 20, st, &p));
        ls = (uint8_t *)p;
    }
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    uint8_t *rm = (md5_root_out && out_dev) ? (uint8_t *)md5_root_out : (uint8_t *)small;
    uint8_t *rs = (sha1_root_out && out_dev) ? (uint8_t *)sha1_root_out : (uint8_t *)(small + 4);
    if (in_dev || len == 0) {
        HG_LAUNCH(ctx, HG_K_LEAVES, st, hg::launch_leaves_dual((const uint8_t *)in, len, block_size, n, lm, ls, st));
    } else {
        HG_TRY(ensure(ctx, SLOT_IN, len, st, &p));
        uint8_t *din = (uint8_t *)p;
        const uint64_t group = pieces_per_launch(len, block_size, 1.75, STAGE_PIECE);
        uint64_t from = 0, npieces = 0;
        HG_TRY(stream_in(ctx, din, (const uint8_t *)in, len, block_size, st,
                         [&](uint64_t off, uint64_t plen) -> int {
                             if (++npieces % group != 0 && off + plen < len) return HG_OK;
                             const uint64_t k0 = from / block_size;
                             const uint64_t k1 = (off + plen + block_size - 1) / block_size;
                             HG_LAUNCH(ctx, HG_K_LEAVES, st,
                                       hg::launch_leaves_dual(din + from, off + plen - from, block_size, k1 - k0,
                                                              lm + k0 * 16, ls + k0 * 20, st));
                             from = off + plen;
                             return HG_OK;
                         }));
    }
    if (md5_leaf_out && !out_dev) HG_TRY(copy_out(ctx, md5_leaf_out, lm, n * 16, false, st));
    if (sha1_leaf_out && !out_dev) HG_TRY(copy_out(ctx, sha1_leaf_out, ls, n * 20, false, st));
    // Second levels: on the host (both at once on the pool) when the digest
    // buffers are large, else one GPU lane each.
    void *const rout[2] = {md5_root_out, sha1_root_out};
    void *const lout[2] = {md5_leaf_out, sha1_leaf_out};
    const uint8_t *const lv[2] = {lm, ls};
    uint8_t *const rdev[2] = {rm, rs};
    HostRoot hr_[2];
    size_t nh = 0, stage_bytes = 0;
    for (int k = 0; k < 2; k++) {
        if (!rout[k]) continue;
        const int dk = k ? 20 : 16;
        const uint64_t db = n * (uint64_t)dk;
        if (db >= HOST_ROOT_MIN) {
            const bool have = lout[k] && !out_dev;
            hr_[nh++] = HostRoot{k ? HG_SHA1 : HG_MD5, have ? (const uint8_t *)lout[k] : lv[k], db, have,
                                 (uint8_t *)rout[k]};
            if (!have) stage_bytes += db;
        } else {
            HG_LAUNCH(ctx, HG_K_ROOT, st, hg::launch_hash_one(k ? HG_SHA1 : HG_MD5, lv[k], db, rdev[k], st));
            if (!out_dev) HG_TRY(copy_out(ctx, rout[k], rdev[k], (size_t)dk, false, st));
        }
    }
    if (nh) {
        uint8_t *hr, *hd;
        HG_TRY(host_step_buffer(ctx, 64, stage_bytes, &hr, &hd));
        uint8_t *dst[2];
        for (size_t i = 0; i < nh; i++) {
            dst[i] = hr_[i].out;
            if (out_dev) hr_[i].out = hr + 32 * i;
        }
        HG_TRY(host_roots(ctx, hr_, nh, hd, st));
        if (out_dev) {
            for (size_t i = 0; i < nh; i++)
                HG_HIP(ctx, hipMemcpyAsync(dst[i], hr + 32 * i, (size_t)digest_bytes(hr_[i].kind),
                                           hipMemcpyHostToDevice, st));
            HG_HIP(ctx, hipEventRecord(ctx->hstep_free, st));
        }
    }
    if (!(flags & HG_ASYNC)) HG_HIP(ctx, hipStreamSynchronize(st));
    return HG_OK;
}

}  // extern "C"

namespace {

// Shared body of the three batch entry points.
int batch_call(hg_ctx *ctx, const hg_block_job *jobs, uint32_t n_jobs, uint32_t flags, void *stream,
               bool leaves, bool roots) {
    HG_TRY(enter(ctx));
    if (flags & ~(uint32_t)(HG_IN_DEVICE | HG_OUT_DEVICE | HG_ASYNC | HG_BACKGROUND | HG_HOST_ROOTS))
        return fail(ctx, HG_EINVAL, "unknown flag bits 0x%x", flags);
    const bool boost = !(flags & HG_BACKGROUND);
    const bool on_host = flags & HG_HOST_ROOTS;
    if (on_host && !roots) return fail(ctx, HG_EINVAL, "HG_HOST_ROOTS applies to calls with second levels");
    if (on_host && (flags & HG_IN_DEVICE)) return fail(ctx, HG_EINVAL, "HG_HOST_ROOTS needs a host job table");
    if ((flags & HG_ASYNC) && !(flags & HG_IN_DEVICE) && !on_host)
        return fail(ctx, HG_EINVAL, "HG_ASYNC requires a device job table (HG_IN_DEVICE) or HG_HOST_ROOTS");
    if (n_jobs == 0) return HG_OK;
    if (!jobs) return fail(ctx, HG_EINVAL, "jobs is NULL");
    hipStream_t st = (hipStream_t)stream;
    const hg_block_job *djobs = jobs;
    uint64_t total_leaves = 0;
    const bool host_table = !(flags & HG_IN_DEVICE);
    if (host_table) {
        for (uint32_t i = 0; i < n_jobs; i++) {
            const hg_block_job &j = jobs[i];
            if (digest_bytes(j.digest) < 0) return fail(ctx, HG_EINVAL, "job %u: unknown digest", i);
            if (j.block_size == 0) return fail(ctx, HG_EINVAL, "job %u: block_size must be >= 1", i);
            if (j.len && (!j.in || !j.leaf_out)) return fail(ctx, HG_EINVAL, "job %u: NULL in or leaf_out", i);
            if (j.reserved) return fail(ctx, HG_EINVAL, "job %u: reserved must be 0", i);
            total_leaves += j.len ? (j.len + j.block_size - 1) / j.block_size : 0;
        }
        void *d;
        HG_TRY(ensure(ctx, SLOT_JOBS, (size_t)n_jobs * sizeof(hg_block_job), st, &d));
        HG_HIP(ctx, hipMemcpyAsync(d, jobs, (size_t)n_jobs * sizeof(hg_block_job), hipMemcpyHostToDevice, st));
        djobs = (const hg_block_job *)d;
    }
    void *plan = nullptr;
    if (leaves || !on_host) {
        HG_TRY(ensure(ctx, SLOT_PLAN, hg::batch_plan_bytes(n_jobs), st, &plan));
        HG_HIP(ctx, hg::launch_batch_plan(djobs, n_jobs, plan, st));
    }
    if (leaves) {
        // A persistent grid of up to 8192 wavefronts (8 per CU) in 128-lane
        // workgroups; fewer when the host knows there are fewer segments.
        // Two wavefronts per workgroup: beside the window scan on other
        // streams, a pipelined step of every primitive ran about 3% faster
        // with 128-lane workgroups than with 64-lane ones (256-lane ones
        // were as fast on average but varied twice as much from run to run).
        uint32_t grid = 8192;
        if (host_table) grid = (uint32_t)std::max<uint64_t>(2, std::min<uint64_t>(grid, (total_leaves + 63) / 64 + 1));
        HG_LAUNCH(ctx, HG_K_LEAVES_BATCH, st, hg::launch_leaves_batch(djobs, n_jobs, plan, grid, 2, boost, st));
    }
    if (roots && on_host) {
        // The second levels on the host's cores (Sec. 3.2.2): the digest
        // buffers come back, the pool hashes them, longest first, and the
        // roots go to their root_out pointers through one copy and a scatter.
        std::vector<HostRoot> hr;
        uint64_t stage_bytes = 0;
        for (uint32_t i = 0; i < n_jobs; i++) {
            const hg_block_job &j = jobs[i];
            if (!j.root_out) continue;
            const uint64_t bytes = (j.len ? (j.len + j.block_size - 1) / j.block_size : 0) *
                                   (uint64_t)digest_bytes(j.digest);
            hr.push_back(HostRoot{j.digest, (const uint8_t *)j.leaf_out, bytes, false, nullptr});
            stage_bytes += bytes;
        }
        if (!hr.empty()) {
            uint8_t *hroots, *hd;
            HG_TRY(host_step_buffer(ctx, (size_t)n_jobs * 20, stage_bytes, &hroots, &hd));
            for (uint32_t i = 0, k = 0; i < n_jobs; i++)
                if (jobs[i].root_out) hr[k++].out = hroots + 20ull * i;
            HG_TRY(host_roots(ctx, hr.data(), hr.size(), hd, st));
            void *droots;
            HG_TRY(ensure(ctx, SLOT_ROOTS, (size_t)n_jobs * 20, st, &droots));
            HG_HIP(ctx, hipMemcpyAsync(droots, hroots, (size_t)n_jobs * 20, hipMemcpyHostToDevice, st));
            HG_HIP(ctx, hipEventRecord(ctx->hstep_free, st));
            HG_LAUNCH(ctx, HG_K_ROOTS_BATCH, st, hg::launch_roots_scatter(djobs, n_jobs, (const uint8_t *)droots, st));
        }
    } else if (roots) {
        HG_LAUNCH(ctx, HG_K_ROOTS_BATCH, st, hg::launch_roots_batch(djobs, n_jobs, plan, boost, st));
    }
    if (!(flags & HG_ASYNC)) HG_HIP(ctx, hipStreamSynchronize(st));
    return HG_OK;
}

}  // namespace

extern "C" {

int hg_leaves_batch(hg_ctx *ctx, const hg_block_job *jobs, uint32_t n_jobs, uint32_t flags, void *stream) {
    return batch_call(ctx, jobs, n_jobs, flags, stream, true, false);
}

int hg_roots_batch(hg_ctx *ctx, const hg_block_job *jobs, uint32_t n_jobs, uint32_t flags, void *stream) {
    return batch_call(ctx, jobs, n_jobs, flags, stream, false, true);
}

int hg_block_hash_batch(hg_ctx *ctx, const hg_block_job *jobs, uint32_t n_jobs, uint32_t flags,
                        void *stream) {
    return batch_call(ctx, jobs, n_jobs, flags, stream, true, true);
}

int hg_window_scan(hg_ctx *ctx, const void *in, uint64_t len, uint32_t window, uint32_t stride,
                   uint32_t mask, uint32_t target, int digest, uint64_t *starts, uint64_t capacity,
                   uint64_t *count, uint32_t flags, void *stream) {
    HG_TRY(enter(ctx));
    HG_TRY(check_flags(ctx, flags, true));
    if (digest_bytes(digest) < 0) return fail(ctx, HG_EINVAL, "unknown digest %d", digest);
    if (window == 0 || window > HG_MAX_WINDOW)
        return fail(ctx, HG_EINVAL, "window must be in [1, %d]", (int)HG_MAX_WINDOW);
    if (stride == 0) return fail(ctx, HG_EINVAL, "stride must be >= 1");
    if (!count) return fail(ctx, HG_EINVAL, "count is NULL");
    if (capacity && !starts) return fail(ctx, HG_EINVAL, "starts is NULL with capacity > 0");
    if (len && !in) return fail(ctx, HG_EINVAL, "in is NULL");
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;

    const uint8_t *din;
    hg::WsPlan plan;
    void *ws;
    HG_TRY(scan_tiles_from(ctx, in, len, in_dev, window, stride, mask, target, digest, st, &din, &plan, &ws));
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    uint64_t *total_dev = out_dev ? count : small;
    HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, st, hg::launch_window_scan_prefix(plan, ws, total_dev, st));
    if (out_dev) {
        HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, st,
                  hg::launch_window_scan_emit(plan, din, len, window, stride, mask, target, ws, starts,
                                              capacity, st));
        if (flags & HG_ASYNC) return HG_OK;
        uint64_t total;
        HG_TRY(read_u64(ctx, total_dev, st, &total));
        return total > capacity ? fail(ctx, HG_ETRUNC, "%llu candidates, capacity %llu",
                                       (unsigned long long)total, (unsigned long long)capacity)
                                : HG_OK;
    }
    uint64_t total;
    HG_TRY(read_u64(ctx, total_dev, st, &total));
    const uint64_t k = std::min(total, capacity);
    if (k) {
        void *o;
        HG_TRY(ensure(ctx, SLOT_OUT, k * 8, st, &o));
        HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, st,
                  hg::launch_window_scan_emit(plan, din, len, window, stride, mask, target, ws,
                                              (uint64_t *)o, k, st));
        HG_TRY(copy_out(ctx, starts, o, k * 8, false, st));
        HG_HIP(ctx, hipStreamSynchronize(st));
    }
    *count = total;
    return total > capacity ? fail(ctx, HG_ETRUNC, "%llu candidates, capacity %llu",
                                   (unsigned long long)total, (unsigned long long)capacity)
                            : HG_OK;
}

int hg_window_scan_noalloc(hg_ctx *ctx, const void *in, uint64_t len, uint32_t window, uint32_t stride,
                           uint32_t mask, uint32_t target, int digest, uint64_t *starts, uint64_t capacity,
                           uint64_t *count, void *stream) {
    HG_TRY(enter(ctx));
    if (digest_bytes(digest) < 0) return fail(ctx, HG_EINVAL, "unknown digest %d", digest);
    if (window == 0 || window > HG_MAX_WINDOW)
        return fail(ctx, HG_EINVAL, "window must be in [1, %d]", (int)HG_MAX_WINDOW);
    if (stride == 0) return fail(ctx, HG_EINVAL, "stride must be >= 1");
    if (!count) return fail(ctx, HG_EINVAL, "count is NULL");
    if (capacity && !starts) return fail(ctx, HG_EINVAL, "starts is NULL with capacity > 0");
    if (len && !in) return fail(ctx, HG_EINVAL, "in is NULL");
    void *ws;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        ws = g_scratch_ptr[ctx->device];
    }
    if (!ws) return fail(ctx, HG_EDEVICE, "no scratch address for device %d", ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const hg::WsPlan plan = hg::plan_window_scan((const uint8_t *)in, len, window, stride, digest);
    const size_t need = hg::window_scan_scratch_bytes(plan);
    if (need > NOALLOC_SCRATCH)
        return fail(ctx, HG_EINVAL, "scan needs %zu bytes of scratch, more than the %zu of hg_window_scan_noalloc",
                    need, NOALLOC_SCRATCH);
    // The same kernels as hg_window_scan (device input and outputs); every
    // scratch word they read is written first in this call, so nothing
    // needs clearing.
    const uint8_t *din = (const uint8_t *)in;
    HG_HIP(ctx, hg::launch_window_scan_tiles(plan, din, len, window, stride, mask, target, ws, st));
    HG_HIP(ctx, hg::launch_window_scan_prefix(plan, ws, count, st));
    HG_HIP(ctx, hg::launch_window_scan_emit(plan, din, len, window, stride, mask, target, ws, starts, capacity, st));
    return HG_OK;
}

int hg_chunk(hg_ctx *ctx, const void *in, uint64_t len, const hg_chunk_params *pr, uint64_t *ends,
             uint64_t capacity, uint64_t *n_chunks, void *chunk_digests, uint32_t flags, void *stream) {
    HG_TRY(enter(ctx));
    const bool count_host = flags & HG_COUNT_HOST;
    flags &= ~(uint32_t)HG_COUNT_HOST;
    HG_TRY(check_flags(ctx, flags, true));
    if (!pr) return fail(ctx, HG_EINVAL, "params is NULL");
    if (digest_bytes(pr->window_digest) < 0 || digest_bytes(pr->chunk_digest) < 0)
        return fail(ctx, HG_EINVAL, "unknown digest");
    if (pr->window == 0 || pr->window > HG_MAX_WINDOW)
        return fail(ctx, HG_EINVAL, "window must be in [1, %d]", (int)HG_MAX_WINDOW);
    if (pr->stride == 0) return fail(ctx, HG_EINVAL, "stride must be >= 1");
    const uint64_t step = pr->min_chunk ? pr->min_chunk : 1;
    if (pr->max_chunk != 0 && pr->max_chunk < step)
        return fail(ctx, HG_EINVAL, "max_chunk must be 0 or at least max(min_chunk, 1)");
    if (!n_chunks) return fail(ctx, HG_EINVAL, "n_chunks is NULL");
    if (capacity && !ends) return fail(ctx, HG_EINVAL, "ends is NULL with capacity > 0");
    if (len && !in) return fail(ctx, HG_EINVAL, "in is NULL");
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    const int dd = digest_bytes(pr->chunk_digest);

    const uint8_t *din;
    hg::WsPlan plan;
    void *ws;
    HG_TRY(scan_tiles_from(ctx, in, len, in_dev, pr->window, pr->stride, pr->mask, pr->target, pr->window_digest, st,
                           &din, &plan, &ws));
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    // small[0]: candidate total, small[1]: chunk count.
    HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, st, hg::launch_window_scan_prefix(plan, ws, &small[0], st));
    uint64_t n_cand;
    HG_TRY(read_u64(ctx, &small[0], st, &n_cand));
    // Chunks <= candidates + 1 (+ len / max_chunk forced cuts): the boundary
    // decision writes straight into the caller's device buffer when it is
    // that large.
    const uint64_t bound = n_cand + 1 + (pr->max_chunk ? 1 + len / pr->max_chunk : 0);
    if (bound >= hg::MAX_LANES)
        return fail(ctx, HG_EINVAL, "%llu candidates (limit 2^31 per call): split the input or use a wider mask",
                    (unsigned long long)n_cand);
    const bool ends_direct = out_dev && capacity >= bound;
    void *cand, *dends = ends;
    HG_TRY(ensure(ctx, SLOT_CAND, n_cand * 8, st, &cand));
    if (!ends_direct) HG_TRY(ensure(ctx, SLOT_ENDS, bound * 8, st, &dends));
    HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, st,
              hg::launch_window_scan_emit(plan, din, len, pr->window, pr->stride, pr->mask, pr->target, ws,
                                          (uint64_t *)cand, n_cand, st));
    if (pr->max_chunk) {
        HG_LAUNCH(ctx, HG_K_CHUNK_SELECT, st,
                  hg::launch_chunk_select_max((const uint64_t *)cand, &small[0], pr->window, len, pr->min_chunk,
                                              pr->max_chunk, (uint64_t *)dends, bound, &small[1], st));
    } else {
        void *sel;
        HG_TRY(ensure(ctx, SLOT_SEL, hg::chunk_select_scratch_bytes(n_cand), st, &sel));
        HG_LAUNCH(ctx, HG_K_CHUNK_SELECT, st,
                  hg::launch_chunk_select((const uint64_t *)cand, &small[0], n_cand, pr->window, len,
                                          pr->min_chunk, sel, (uint64_t *)dends, n_cand + 1, &small[1], st));
    }
    // The chunk count sizes the outputs; the digests are enqueued after it.
    // With standard chunk digests the longest chunk comes back with it: long
    // chunks are hashed on the host (chunk_digests_split).
    const bool may_split = chunk_digests && pr->chunk_segment == 0 && len >= HOST_CHUNK_MIN;
    if (may_split) HG_HIP(ctx, hg::launch_max_gap((const uint64_t *)dends, len, &small[1], bound, &small[2], st));
    uint64_t nc, longest = 0;
    HG_TRY(read_u64(ctx, &small[1], st, &nc, may_split ? 2 : 1));
    if (may_split) longest = ctx->host_small[1];
    const uint64_t k = std::min(nc, capacity);
    if (!ends_direct) HG_TRY(copy_out(ctx, ends, dends, k * 8, out_dev, st));
    if (chunk_digests) {
        // Straight into the caller's device buffer when it holds them all.
        const bool direct = out_dev && capacity >= nc;
        void *ddig = chunk_digests;
        if (!direct) HG_TRY(ensure(ctx, SLOT_DIG, (nc + 1) * (uint64_t)dd, st, &ddig));
        bool split = false;
        if (longest >= HOST_CHUNK_MIN)
            HG_TRY(chunk_digests_split(ctx, pr->chunk_digest, din, in_dev ? nullptr : (const uint8_t *)in, len,
                                       (const uint64_t *)dends, &small[1], nc, (uint8_t *)ddig, st, &split));
        if (!split)
            HG_TRY(chunk_digests_of(ctx, *pr, din, len, (const uint64_t *)dends, &small[1], nc, (uint8_t *)ddig, st));
        if (!direct) HG_TRY(copy_out(ctx, chunk_digests, ddig, k * (uint64_t)dd, out_dev, st));
    }
    if (out_dev && !count_host) HG_TRY(copy_out(ctx, n_chunks, &small[1], 8, true, st));
    else *n_chunks = nc;
    if (!(flags & HG_ASYNC)) HG_HIP(ctx, hipStreamSynchronize(st));
    return nc > capacity ? fail(ctx, HG_ETRUNC, "%llu chunks, capacity %llu", (unsigned long long)nc,
                                (unsigned long long)capacity)
                         : HG_OK;
}

// B has n_b digests, or with n_b_dev (device or host per HG_IN_DEVICE)
// min(*n_b_dev, n_b) of them, read when the work runs.
static int similarity_impl(hg_ctx *ctx, const void *dig_a, uint64_t n_a, const void *dig_b, const uint64_t *len_b,
                           uint64_t n_b, const uint64_t *n_b_dev, int digest, uint64_t *matched,
                           uint64_t *matched_bytes, uint32_t flags, void *stream) {
    HG_TRY(enter(ctx));
    const bool len_ends = flags & HG_LEN_ENDS;
    flags &= ~(uint32_t)HG_LEN_ENDS;
    HG_TRY(check_flags(ctx, flags, true));
    const int d = digest_bytes(digest);
    if (d < 0) return fail(ctx, HG_EINVAL, "unknown digest %d", digest);
    if (!matched) return fail(ctx, HG_EINVAL, "matched is NULL");
    if ((n_a && !dig_a) || (n_b && !dig_b)) return fail(ctx, HG_EINVAL, "NULL digest array");
    if (n_a >= hg::MAX_LANES || n_b >= hg::MAX_LANES)
        return fail(ctx, HG_EINVAL, "n_a and n_b must be below 2^31");
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    if (n_b_dev && !in_dev) {
        // A host count: B is simply that long.
        n_b = std::min(*n_b_dev, n_b);
        n_b_dev = nullptr;
    }
    const uint8_t *da, *db, *dl = nullptr;
    HG_TRY(device_input(ctx, SLOT_IN, dig_a, n_a * (uint64_t)d, in_dev, st, &da));
    HG_TRY(device_input(ctx, SLOT_IN2, dig_b, n_b * (uint64_t)d, in_dev, st, &db));
    if (len_b) HG_TRY(device_input(ctx, SLOT_IN3, len_b, n_b * 8, in_dev, st, &dl));
    int log2_slots = 6;
    while ((1ull << log2_slots) < 2 * n_a) log2_slots++;
    void *table;
    HG_TRY(ensure(ctx, SLOT_TABLE, (1ull << log2_slots) * 4, st, &table));
    unsigned long long *counters = (unsigned long long *)&small[4];
    HG_LAUNCH(ctx, HG_K_SIMILARITY, st,
              hg::launch_similarity(digest, da, n_a, db, (const uint64_t *)dl, len_ends ? 1 : 0, n_b, n_b_dev,
                                    (uint32_t *)table, log2_slots, counters, st));
    HG_TRY(copy_out(ctx, matched, &counters[0], 8, out_dev, st));
    if (matched_bytes) HG_TRY(copy_out(ctx, matched_bytes, &counters[1], 8, out_dev, st));
    if (!(flags & HG_ASYNC)) HG_HIP(ctx, hipStreamSynchronize(st));
    return HG_OK;
}

int hg_similarity(hg_ctx *ctx, const void *dig_a, uint64_t n_a, const void *dig_b, const uint64_t *len_b,
                  uint64_t n_b, int digest, uint64_t *matched, uint64_t *matched_bytes, uint32_t flags,
                  void *stream) {
    return similarity_impl(ctx, dig_a, n_a, dig_b, len_b, n_b, nullptr, digest, matched, matched_bytes, flags,
                           stream);
}

int hg_similarity_n(hg_ctx *ctx, const void *dig_a, uint64_t n_a, const void *dig_b, const uint64_t *len_b,
                    const uint64_t *n_b, uint64_t max_b, int digest, uint64_t *matched, uint64_t *matched_bytes,
                    uint32_t flags, void *stream) {
    if (ctx && !n_b) return fail(ctx, HG_EINVAL, "n_b is NULL");
    return similarity_impl(ctx, dig_a, n_a, dig_b, len_b, max_b, n_b, digest, matched, matched_bytes, flags,
                           stream);
}

int hg_chunk_select(hg_ctx *ctx, const uint64_t *starts, const uint64_t *n_starts, uint64_t max_starts,
                    uint64_t len, uint32_t window, uint64_t min_chunk, uint64_t max_chunk, uint64_t *ends,
                    uint64_t capacity, uint64_t *n_chunks, uint32_t flags, void *stream) {
    HG_TRY(enter(ctx));
    HG_TRY(check_flags(ctx, flags, true));
    if (window == 0 || window > HG_MAX_WINDOW)
        return fail(ctx, HG_EINVAL, "window must be in [1, %d]", (int)HG_MAX_WINDOW);
    const uint64_t step = min_chunk ? min_chunk : 1;
    if (max_chunk != 0 && max_chunk < step)
        return fail(ctx, HG_EINVAL, "max_chunk must be 0 or at least max(min_chunk, 1)");
    if (!n_starts || !n_chunks || !ends) return fail(ctx, HG_EINVAL, "n_starts, n_chunks or ends is NULL");
    if (max_starts && !starts) return fail(ctx, HG_EINVAL, "starts is NULL with max_starts > 0");
    const uint64_t bound = max_starts + 1 + (max_chunk ? 1 + len / max_chunk : 0);
    if (bound >= hg::MAX_LANES)
        return fail(ctx, HG_EINVAL, "max_starts %llu above the limit of 2^31 per call", (unsigned long long)max_starts);
    if (capacity < bound)
        return fail(ctx, HG_EINVAL, "capacity %llu below the bound %llu (max_starts + 1, plus len / max_chunk + 1)",
                    (unsigned long long)capacity, (unsigned long long)bound);
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    // small[8]: candidates used, small[9]: the list was incomplete,
    // small[10]: chunk count when the output is host memory.
    const uint64_t *dstarts = starts;
    if (in_dev) {
        HG_HIP(ctx, hg::launch_count_clamp(n_starts, max_starts, &small[8], st));
    } else {
        const uint64_t k = std::min(*n_starts, max_starts);
        ctx->host_small[0] = k;
        ctx->host_small[1] = *n_starts > max_starts ? 1 : 0;
        HG_HIP(ctx, hipMemcpyAsync(&small[8], ctx->host_small, 16, hipMemcpyHostToDevice, st));
        const uint8_t *p;
        HG_TRY(device_input(ctx, SLOT_CAND, starts, k * 8, false, st, &p));
        dstarts = (const uint64_t *)p;
        HG_HIP(ctx, hipStreamSynchronize(st));  // host_small is reused below
    }
    void *dends = ends;
    if (!out_dev) HG_TRY(ensure(ctx, SLOT_ENDS, bound * 8, st, &dends));
    uint64_t *dn = out_dev ? n_chunks : &small[10];
    if (max_chunk) {
        HG_LAUNCH(ctx, HG_K_CHUNK_SELECT, st,
                  hg::launch_chunk_select_max(dstarts, &small[8], window, len, min_chunk, max_chunk,
                                              (uint64_t *)dends, bound, dn, st));
    } else {
        void *sel;
        HG_TRY(ensure(ctx, SLOT_SEL, hg::chunk_select_scratch_bytes(max_starts), st, &sel));
        HG_LAUNCH(ctx, HG_K_CHUNK_SELECT, st,
                  hg::launch_chunk_select(dstarts, &small[8], max_starts, window, len, min_chunk, sel,
                                          (uint64_t *)dends, bound, dn, st));
    }
    HG_HIP(ctx, hg::launch_count_invalidate(&small[9], dn, st));
    if (out_dev) {
        if (flags & HG_ASYNC) return HG_OK;
        uint64_t nc;
        HG_TRY(read_u64(ctx, dn, st, &nc));
        return nc == ~0ull ? fail(ctx, HG_ETRUNC, "the candidate list is incomplete (*n_starts > max_starts)")
                           : HG_OK;
    }
    uint64_t nc;
    HG_TRY(read_u64(ctx, dn, st, &nc));
    *n_chunks = nc;
    if (nc == ~0ull) return fail(ctx, HG_ETRUNC, "the candidate list is incomplete (*n_starts > max_starts)");
    HG_TRY(copy_out(ctx, ends, dends, nc * 8, false, st));
    HG_HIP(ctx, hipStreamSynchronize(st));
    return HG_OK;
}

int hg_chunk_digests(hg_ctx *ctx, const void *in, uint64_t len, const uint64_t *ends, const uint64_t *n_chunks,
                     uint64_t max_chunks, int digest, uint64_t chunk_segment, void *digests, uint32_t flags,
                     void *stream) {
    HG_TRY(enter(ctx));
    HG_TRY(check_flags(ctx, flags, true));
    const int d = digest_bytes(digest);
    if (d < 0) return fail(ctx, HG_EINVAL, "unknown digest %d", digest);
    if (!n_chunks || !digests) return fail(ctx, HG_EINVAL, "n_chunks or digests is NULL");
    if (max_chunks && !ends) return fail(ctx, HG_EINVAL, "ends is NULL with max_chunks > 0");
    if (len && !in) return fail(ctx, HG_EINVAL, "in is NULL");
    if (max_chunks >= hg::MAX_LANES) return fail(ctx, HG_EINVAL, "max_chunks must be below 2^31");
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    const uint8_t *din = (const uint8_t *)in;
    const uint64_t *dends = ends, *dn = n_chunks;
    uint64_t k = max_chunks;
    if (!in_dev) {
        k = std::min(*n_chunks, max_chunks);
        const uint8_t *p;
        HG_TRY(device_input(ctx, SLOT_IN, in, len, false, st, &din));
        HG_TRY(device_input(ctx, SLOT_CAND, ends, k * 8, false, st, &p));
        dends = (const uint64_t *)p;
        ctx->host_small[0] = k;
        HG_HIP(ctx, hipMemcpyAsync(&small[11], ctx->host_small, 8, hipMemcpyHostToDevice, st));
        HG_HIP(ctx, hipStreamSynchronize(st));
        dn = &small[11];
    }
    void *dout = digests;
    if (!out_dev) HG_TRY(ensure(ctx, SLOT_DIG, std::max<uint64_t>(k, 1) * d, st, &dout));
    hg_chunk_params p{};
    p.chunk_digest = digest;
    p.chunk_segment = chunk_segment;
    HG_TRY(chunk_digests_of(ctx, p, din, len, dends, dn, k, (uint8_t *)dout, st));
    if (!out_dev) {
        HG_TRY(copy_out(ctx, digests, dout, k * (uint64_t)d, false, st));
        HG_HIP(ctx, hipStreamSynchronize(st));
    } else if (!(flags & HG_ASYNC)) {
        HG_HIP(ctx, hipStreamSynchronize(st));
    }
    return HG_OK;
}

int hg_timing_enable(hg_ctx *ctx, int enable) {
    if (!ctx) return HG_EINVAL;
    ctx->timing = enable != 0;
    return HG_OK;
}

int hg_timing_read(hg_ctx *ctx, int kernel_class, uint64_t *launches, double *total_ms) {
    if (!ctx) return HG_EINVAL;
    if (kernel_class < 0 || kernel_class >= HG_K_COUNT)
        return fail(ctx, HG_EINVAL, "unknown kernel class %d", kernel_class);
    HG_TRY(resolve_timing(ctx));
    if (launches) *launches = ctx->t_launches[kernel_class];
    if (total_ms) *total_ms = ctx->t_ms[kernel_class];
    return HG_OK;
}

int hg_timing_reset(hg_ctx *ctx) {
    if (!ctx) return HG_EINVAL;
    HG_TRY(resolve_timing(ctx));
    for (int k = 0; k < HG_K_COUNT; k++) {
        ctx->t_launches[k] = 0;
        ctx->t_ms[k] = 0.0;
        ctx->t_start[k].clear();
        ctx->t_end[k].clear();
    }
    return HG_OK;
}

int hg_probe_alu(hg_ctx *ctx, double *tops, void *stream) {
    HG_TRY(enter(ctx));
    if (!tops) return fail(ctx, HG_EINVAL, "tops is NULL");
    hipStream_t st = (hipStream_t)stream;
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    // Eight waves per SIMD, about 5 ms at the data-sheet rate.
    const uint32_t blocks = 2048, steps = 1000;
    hipEvent_t a, b;
    HG_HIP(ctx, hipEventCreate(&a));
    HG_HIP(ctx, hipEventCreate(&b));
    float best = 1e30f;
    int st_ = HG_OK;
    for (int r = 0; r < 4 && st_ == HG_OK; r++) {
        if (hipEventRecord(a, st) != hipSuccess ||
            hg::launch_alu_probe(blocks, steps, (uint32_t *)small, st) != hipSuccess ||
            hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
            st_ = fail(ctx, HG_EDEVICE, "ALU probe failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (r > 0) best = std::min(best, ms);  // the first run warms up
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st_ != HG_OK) return st_;
    *tops = (double)hg::alu_probe_ops(blocks, steps) / (best * 1e-3) / 1e12;
    return HG_OK;
}

int hg_probe_read(hg_ctx *ctx, const void *buf, uint64_t len, double *gbps, void *stream) {
    HG_TRY(enter(ctx));
    if (!gbps || !buf || len < 16) return fail(ctx, HG_EINVAL, "need a device buffer of at least 16 bytes");
    hipStream_t st = (hipStream_t)stream;
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    hipEvent_t a, b;
    HG_HIP(ctx, hipEventCreate(&a));
    HG_HIP(ctx, hipEventCreate(&b));
    float best = 1e30f;
    int st_ = HG_OK;
    for (int r = 0; r < 4 && st_ == HG_OK; r++) {
        if (hipEventRecord(a, st) != hipSuccess ||
            hg::launch_read_probe((const uint8_t *)buf, len, (uint32_t *)small, st) != hipSuccess ||
            hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess) {
            st_ = fail(ctx, HG_EDEVICE, "read probe failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (r > 0) best = std::min(best, ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st_ != HG_OK) return st_;
    *gbps = (double)(len / 16 * 16) / (best * 1e-3) / 1e9;
    return HG_OK;
}

int hg_timing_origin(hg_ctx *ctx, void *event) {
    if (!ctx) return HG_EINVAL;
    HG_TRY(resolve_timing(ctx));
    ctx->t_origin = (hipEvent_t)event;
    return HG_OK;
}

int hg_timing_intervals(hg_ctx *ctx, int kernel_class, double *start_ms, double *end_ms, uint64_t capacity,
                        uint64_t *count) {
    if (!ctx) return HG_EINVAL;
    if (kernel_class < 0 || kernel_class >= HG_K_COUNT)
        return fail(ctx, HG_EINVAL, "unknown kernel class %d", kernel_class);
    if (!count || (capacity && (!start_ms || !end_ms))) return fail(ctx, HG_EINVAL, "NULL output");
    HG_TRY(resolve_timing(ctx));
    const std::vector<double> &a = ctx->t_start[kernel_class], &b = ctx->t_end[kernel_class];
    *count = a.size();
    const size_t k = std::min<size_t>(a.size(), capacity);
    for (size_t i = 0; i < k; i++) {
        start_ms[i] = a[i];
        end_ms[i] = b[i];
    }
    return a.size() > capacity ? fail(ctx, HG_ETRUNC, "%zu intervals", a.size()) : HG_OK;
}

}  // extern "C"

// ================================================================ file batches

struct hg_batch {
    hg_ctx *ctx = nullptr;
    uint32_t n = 0;
    hg_batch_params p{};
    int d_block = 0, d_chunk = 0;
    bool do_hash = false, do_chunk = false;
    std::vector<uint64_t> off, len, leaf_first;
    std::vector<uint32_t> order_desc, order_given;
    uint64_t n_leaves = 0, total_windows = 0, n_tiles = 0, cap_cand = 0, max_chunks = 0;
    hg::WsPlan wsp{};
    std::vector<void *> allocs;
    // device tables
    uint64_t *d_off = nullptr, *d_len = nullptr, *d_leaf_first = nullptr, *d_first_tile = nullptr;
    uint64_t *d_extra = nullptr;  // with a maximum chunk size: forced-cut slots before each file
    hg::FileTile *d_tiles = nullptr;
    uint32_t *d_order = nullptr;
    hg_block_job *d_jobs = nullptr;
    void *d_plan = nullptr, *d_ws = nullptr, *d_seg = nullptr;
    uint64_t *d_cand = nullptr, *d_slots = nullptr, *d_seg_start = nullptr, *d_seg_end = nullptr;
    uint32_t *d_cnt = nullptr;
    // two-level chunk digests: prefix scratch and segment-digest slots
    void *d_tl = nullptr;
    uint8_t *d_tl_leaves = nullptr;
    uint64_t tl_slots = 0;
    // schedule (set by hg_batch_tune): wavefronts of the persistent grid,
    // wavefronts per workgroup, file order
    uint32_t grid = 8192;
    uint32_t wg_waves = 4;
    bool longest_first = true;
    // concurrency and graph
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int batch_alloc(hg_batch *b, size_t bytes, void **out) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(b->ctx, HG_ENOMEM, "batch allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    b->allocs.push_back(p);
    *out = p;
    return HG_OK;
}

template <class T>
int batch_upload(hg_batch *b, const std::vector<T> &v, T **out) {
    void *p;
    HG_TRY(batch_alloc(b, v.size() * sizeof(T), &p));
    if (!v.empty()) HG_HIP(b->ctx, hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = (T *)p;
    return HG_OK;
}

void batch_free(hg_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    for (void *p : b->allocs) (void)hipFree(p);
    b->allocs.clear();
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->aux) (void)hipStreamDestroy(b->aux);
}

// The direct hash of every file: job records, plan, segments, roots.
int batch_hash(hg_batch *b, const uint8_t *arena, const hg_batch_out *out, hipStream_t st) {
    HG_HIP(b->ctx, hg::launch_files_jobs(arena, b->d_off, b->d_len, b->d_leaf_first, b->d_order, b->n,
                                         b->p.block_size, b->p.block_digest, (uint8_t *)out->leaf_digests,
                                         b->p.roots ? (uint8_t *)out->roots : nullptr, b->d_jobs, st));
    HG_HIP(b->ctx, hg::launch_batch_plan(b->d_jobs, b->n, b->d_plan, st));
    HG_HIP(b->ctx, hg::launch_leaves_batch(b->d_jobs, b->n, b->d_plan, b->grid, b->wg_waves, true, st));
    if (b->p.roots) HG_HIP(b->ctx, hg::launch_roots_batch(b->d_jobs, b->n, b->d_plan, true, st));
    return HG_OK;
}

int batch_chunk(hg_batch *b, const uint8_t *arena, const hg_batch_out *out, hipStream_t st) {
    const hg_chunk_params &c = b->p.chunk;
    hg::WsFiles files{arena, b->d_off, b->d_len, b->d_tiles};
    HG_HIP(b->ctx, hg::launch_window_scan_tiles(b->wsp, nullptr, 0, c.window, c.stride, c.mask, c.target, b->d_ws,
                                                st, &files));
    HG_HIP(b->ctx, hg::launch_window_scan_prefix(b->wsp, b->d_ws, &out->status[0], st));
    HG_HIP(b->ctx, hg::launch_window_scan_emit(b->wsp, nullptr, 0, c.window, c.stride, c.mask, c.target, b->d_ws,
                                               b->d_cand, b->cap_cand, st, &files));
    hg::FilesChunk fc{b->d_off, b->d_len, b->d_first_tile,
                      hg::window_scan_tile_offsets(b->wsp, b->d_ws),
                      b->wsp.n_tiles, b->d_cand, b->cap_cand, b->d_slots, b->d_cnt, b->d_seg_start,
                      b->d_seg_end, b->n, c.max_chunk, b->d_extra};
    HG_HIP(b->ctx, hg::launch_files_select(fc, c.window, c.min_chunk, out->status, st));
    HG_HIP(b->ctx, hg::launch_files_compact(fc, out->chunk_off, out->chunk_ends, b->max_chunks, out->status, st));
    if (out->chunk_digests && c.chunk_segment)
        HG_HIP(b->ctx, hg::launch_chunk_digests_two_level_arena(
                           c.chunk_digest, arena, b->d_seg_start, b->d_seg_end, &out->status[1], b->max_chunks,
                           c.chunk_segment, b->d_tl, b->d_tl_leaves, b->tl_slots, (uint8_t *)out->chunk_digests, st));
    else if (out->chunk_digests)
        HG_HIP(b->ctx, hg::launch_segment_digests(c.chunk_digest, arena, 0, b->d_seg_start, b->d_seg_end,
                                                  &out->status[1], b->max_chunks, (uint8_t *)out->chunk_digests,
                                                  b->d_seg, st));
    return HG_OK;
}

int batch_enqueue(hg_batch *b, const void *arena, const hg_batch_out *out, hipStream_t st) {
    HG_HIP(b->ctx, hg::launch_fill_u32((uint32_t *)out->status, 8, 0, st));
    if (b->do_hash && b->do_chunk) {
        // Two branches: the direct hash on the helper stream, chunking here.
        HG_HIP(b->ctx, hipEventRecord(b->fork, st));
        HG_HIP(b->ctx, hipStreamWaitEvent(b->aux, b->fork, 0));
        HG_TRY(batch_hash(b, (const uint8_t *)arena, out, b->aux));
        HG_TRY(batch_chunk(b, (const uint8_t *)arena, out, st));
        HG_HIP(b->ctx, hipEventRecord(b->join, b->aux));
        HG_HIP(b->ctx, hipStreamWaitEvent(st, b->join, 0));
    } else if (b->do_hash) {
        HG_TRY(batch_hash(b, (const uint8_t *)arena, out, st));
    } else if (b->do_chunk) {
        HG_TRY(batch_chunk(b, (const uint8_t *)arena, out, st));
    }
    return HG_OK;
}

int check_batch_out(hg_batch *b, const void *arena, const hg_batch_out *out) {
    if (!out || !out->status) return fail(b->ctx, HG_EINVAL, "out or out->status is NULL");
    if (!arena && b->n) return fail(b->ctx, HG_EINVAL, "arena is NULL");
    if (b->do_hash && b->n_leaves && !out->leaf_digests) return fail(b->ctx, HG_EINVAL, "leaf_digests is NULL");
    if (b->do_hash && b->p.roots && !out->roots) return fail(b->ctx, HG_EINVAL, "roots is NULL");
    if (b->do_chunk && (!out->chunk_ends || !out->chunk_off))
        return fail(b->ctx, HG_EINVAL, "chunk_ends or chunk_off is NULL");
    return HG_OK;
}

}  // namespace

extern "C" {

int hg_batch_create(hg_ctx *ctx, const uint64_t *file_off, const uint64_t *file_len, uint32_t n_files,
                    const hg_batch_params *params, hg_batch **out) {
    HG_TRY(enter(ctx));
    if (!out || !params) return fail(ctx, HG_EINVAL, "out or params is NULL");
    *out = nullptr;
    if (n_files && (!file_off || !file_len)) return fail(ctx, HG_EINVAL, "file_off or file_len is NULL");
    const hg_batch_params &p = *params;
    const bool do_hash = p.block_size != 0, do_chunk = p.chunk.window != 0;
    if (do_hash && digest_bytes(p.block_digest) < 0) return fail(ctx, HG_EINVAL, "unknown block digest");
    if (do_chunk) {
        if (digest_bytes(p.chunk.window_digest) < 0 || digest_bytes(p.chunk.chunk_digest) < 0)
            return fail(ctx, HG_EINVAL, "unknown chunk digest");
        if (p.chunk.window > HG_MAX_WINDOW) return fail(ctx, HG_EINVAL, "window must be in [1, %d]", (int)HG_MAX_WINDOW);
        if (p.chunk.stride == 0) return fail(ctx, HG_EINVAL, "stride must be >= 1");
        if (p.chunk.max_chunk != 0 && p.chunk.max_chunk < std::max<uint64_t>(p.chunk.min_chunk, 1))
            return fail(ctx, HG_EINVAL, "max_chunk must be 0 or at least max(min_chunk, 1)");
    }
    hg_batch *b = new hg_batch();
    b->ctx = ctx;
    b->n = n_files;
    b->p = p;
    b->do_hash = do_hash;
    b->do_chunk = do_chunk;
    b->d_block = do_hash ? digest_bytes(p.block_digest) : 0;
    b->d_chunk = do_chunk ? digest_bytes(p.chunk.chunk_digest) : 0;
    b->off.assign(file_off, file_off + n_files);
    b->len.assign(file_len, file_len + n_files);
    int st = HG_OK;
    do {
        // Direct-hash layout and the longest-first file order.
        b->leaf_first.assign(n_files + 1, 0);
        for (uint32_t f = 0; f < n_files; f++)
            b->leaf_first[f + 1] = b->leaf_first[f] + (do_hash && b->len[f] ? (b->len[f] + p.block_size - 1) / p.block_size : 0);
        b->n_leaves = b->leaf_first[n_files];
        b->order_given.resize(n_files);
        std::iota(b->order_given.begin(), b->order_given.end(), 0u);
        b->order_desc = b->order_given;
        std::stable_sort(b->order_desc.begin(), b->order_desc.end(),
                         [&](uint32_t x, uint32_t y) { return b->len[x] > b->len[y]; });
        if ((st = batch_upload(b, b->off, &b->d_off)) != HG_OK) break;
        if ((st = batch_upload(b, b->len, &b->d_len)) != HG_OK) break;
        if ((st = batch_upload(b, b->leaf_first, &b->d_leaf_first)) != HG_OK) break;
        if ((st = batch_upload(b, b->order_desc, &b->d_order)) != HG_OK) break;
        void *q;
        if ((st = batch_alloc(b, (size_t)std::max<uint32_t>(n_files, 1) * sizeof(hg_block_job), &q)) != HG_OK) break;
        b->d_jobs = (hg_block_job *)q;
        if ((st = batch_alloc(b, hg::batch_plan_bytes(std::max<uint32_t>(n_files, 1)), &b->d_plan)) != HG_OK) break;
        // Chunking layout: tiles that never span a file.
        std::vector<uint64_t> first_tile(n_files + 1, 0);
        std::vector<hg::FileTile> tiles;
        if (do_chunk) {
            const uint32_t w = p.chunk.window, s = p.chunk.stride;
            const uint64_t tw = hg::window_scan_tile_windows(w, s, p.chunk.window_digest);
            for (uint32_t f = 0; f < n_files; f++) {
                first_tile[f] = tiles.size();
                const uint64_t nw = b->len[f] >= w ? (b->len[f] - w) / s + 1 : 0;
                b->total_windows += nw;
                for (uint64_t k0 = 0; k0 < nw; k0 += tw) tiles.push_back(hg::FileTile{f, 0, k0});
            }
            first_tile[n_files] = tiles.size();
            b->n_tiles = tiles.size();
            b->wsp = hg::plan_window_scan_files(b->n_tiles, b->total_windows, w, s, p.chunk.window_digest);
            // Candidate capacity: twice the expectation for random data
            // (each window matches with probability 2^-popcount(mask)) plus
            // slack per file, unless given.
            const double prob = std::ldexp(1.0, -__builtin_popcount(p.chunk.mask));
            b->cap_cand = p.max_candidates ? p.max_candidates
                                           : (uint64_t)(2.0 * prob * (double)b->total_windows) + 64ull * n_files + 4096;
            b->cap_cand = std::min<uint64_t>(b->cap_cand, b->total_windows);
            b->max_chunks = b->cap_cand + n_files;
            if (p.chunk.max_chunk) {
                // Each file also gets room for its forced cuts (at most
                // len / max_chunk of them).
                std::vector<uint64_t> extra(std::max<uint32_t>(n_files, 1), 0);
                uint64_t acc = 0;
                for (uint32_t f = 0; f < n_files; f++) {
                    extra[f] = acc;
                    acc += b->len[f] / p.chunk.max_chunk;
                }
                b->max_chunks += acc;
                if ((st = batch_upload(b, extra, &b->d_extra)) != HG_OK) break;
            }
            if (b->max_chunks >= hg::MAX_LANES) {
                st = fail(ctx, HG_EINVAL, "%llu chunks possible in one batch (limit 2^31): split the files",
                          (unsigned long long)b->max_chunks);
                break;
            }
            if ((st = batch_upload(b, first_tile, &b->d_first_tile)) != HG_OK) break;
            if ((st = batch_upload(b, tiles, &b->d_tiles)) != HG_OK) break;
            if ((st = batch_alloc(b, hg::window_scan_scratch_bytes(b->wsp), &b->d_ws)) != HG_OK) break;
            if ((st = batch_alloc(b, b->cap_cand * 8, &q)) != HG_OK) break;
            b->d_cand = (uint64_t *)q;
            if ((st = batch_alloc(b, b->max_chunks * 8, &q)) != HG_OK) break;
            b->d_slots = (uint64_t *)q;
            if ((st = batch_alloc(b, b->max_chunks * 8, &q)) != HG_OK) break;
            b->d_seg_start = (uint64_t *)q;
            if ((st = batch_alloc(b, b->max_chunks * 8, &q)) != HG_OK) break;
            b->d_seg_end = (uint64_t *)q;
            if ((st = batch_alloc(b, (size_t)std::max<uint32_t>(n_files, 1) * 4, &q)) != HG_OK) break;
            b->d_cnt = (uint32_t *)q;
            if ((st = batch_alloc(b, hg::segment_digest_scratch_bytes(b->max_chunks), &b->d_seg)) != HG_OK) break;
            if (p.chunk.chunk_segment) {
                // Segment digests: at most sum(len / S) + one partial segment
                // per chunk.
                uint64_t slots = b->max_chunks + 1;
                for (uint32_t f = 0; f < n_files; f++) slots += b->len[f] / p.chunk.chunk_segment;
                if (slots >= hg::MAX_LANES) {
                    st = fail(ctx, HG_EINVAL, "%llu chunk segments (limit 2^31): use a larger chunk_segment",
                              (unsigned long long)slots);
                    break;
                }
                b->tl_slots = slots;
                if ((st = batch_alloc(b, hg::two_level_arena_scratch_bytes(b->max_chunks), &b->d_tl)) != HG_OK)
                    break;
                if ((st = batch_alloc(b, slots * (uint64_t)b->d_chunk, &q)) != HG_OK) break;
                b->d_tl_leaves = (uint8_t *)q;
            }
        }
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming)) != hipSuccess) {
            st = fail(ctx, HG_EDEVICE, "batch stream/event creation failed: %s", hipGetErrorString(e));
            break;
        }
    } while (0);
    if (st != HG_OK) {
        batch_free(b);
        delete b;
        return st;
    }
    *out = b;
    return HG_OK;
}

void hg_batch_destroy(hg_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipDeviceSynchronize();
    batch_free(b);
    delete b;
}

int hg_batch_layout(const hg_batch *b, uint64_t *leaf_first, uint64_t *n_leaves_total, uint64_t *max_chunks) {
    if (!b) return HG_EINVAL;
    if (leaf_first) memcpy(leaf_first, b->leaf_first.data(), (b->n + 1) * sizeof(uint64_t));
    if (n_leaves_total) *n_leaves_total = b->n_leaves;
    if (max_chunks) *max_chunks = b->max_chunks;
    return HG_OK;
}

int hg_batch_run(hg_batch *b, const void *arena, const hg_batch_out *out, void *stream) {
    if (!b) return HG_EINVAL;
    HG_TRY(enter(b->ctx));
    HG_TRY(check_batch_out(b, arena, out));
    return batch_enqueue(b, arena, out, (hipStream_t)stream);
}

int hg_batch_capture(hg_batch *b, const void *arena, const hg_batch_out *out, void *stream) {
    if (!b) return HG_EINVAL;
    HG_TRY(enter(b->ctx));
    HG_TRY(check_batch_out(b, arena, out));
    hipStream_t st = (hipStream_t)stream;
    if (!st) return fail(b->ctx, HG_EINVAL, "capture needs a non-default stream");
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    HG_HIP(b->ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int r = batch_enqueue(b, arena, out, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (r != HG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return fail(b->ctx, HG_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    b->graph = g;
    HG_HIP(b->ctx, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return HG_OK;
}

int hg_batch_replay(hg_batch *b, void *stream) {
    if (!b) return HG_EINVAL;
    HG_TRY(enter(b->ctx));
    if (!b->exec) return fail(b->ctx, HG_EINVAL, "no captured graph");
    HG_HIP(b->ctx, hipGraphLaunch(b->exec, (hipStream_t)stream));
    return HG_OK;
}

int hg_batch_tune(hg_batch *b, const void *arena, const hg_batch_out *out, void *stream, char *report,
                  size_t report_len) {
    if (!b) return HG_EINVAL;
    HG_TRY(enter(b->ctx));
    HG_TRY(check_batch_out(b, arena, out));
    hipStream_t st = (hipStream_t)stream;
    std::string rep;
    if (!b->do_hash || b->n == 0) {
        rep = "nothing to tune";
    } else {
        hipEvent_t e0, e1;
        HG_HIP(b->ctx, hipEventCreate(&e0));
        HG_HIP(b->ctx, hipEventCreate(&e1));
        float best = 1e30f;
        uint32_t best_grid = b->grid, best_wg = b->wg_waves;
        bool best_order = b->longest_first;
        const uint32_t grids[] = {1024, 2048, 4096, 8192};
        const uint32_t wgs[] = {1, 2, 4};
        for (int lf = 1; lf >= 0; lf--) {
            const std::vector<uint32_t> &ord = lf ? b->order_desc : b->order_given;
            HG_HIP(b->ctx, hipMemcpy(b->d_order, ord.data(), ord.size() * 4, hipMemcpyHostToDevice));
            for (uint32_t wg : wgs)
            for (uint32_t g : grids) {
                b->grid = g;
                b->wg_waves = wg;
                float t = 1e30f;
                for (int rep_i = 0; rep_i < 3; rep_i++) {
                    HG_HIP(b->ctx, hipEventRecord(e0, st));
                    HG_TRY(batch_hash(b, (const uint8_t *)arena, out, st));
                    HG_HIP(b->ctx, hipEventRecord(e1, st));
                    HG_HIP(b->ctx, hipEventSynchronize(e1));
                    float ms = 0.f;
                    HG_HIP(b->ctx, hipEventElapsedTime(&ms, e0, e1));
                    if (rep_i > 0) t = std::min(t, ms);  // first run warms up
                }
                char buf[96];
                snprintf(buf, sizeof buf, "%s/%ux%u:%.3fms ", lf ? "longest" : "given", g, 64 * wg, t);
                rep += buf;
                if (t < best) {
                    best = t;
                    best_grid = g;
                    best_wg = wg;
                    best_order = lf;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->grid = best_grid;
        b->wg_waves = best_wg;
        b->longest_first = best_order;
        const std::vector<uint32_t> &ord = best_order ? b->order_desc : b->order_given;
        HG_HIP(b->ctx, hipMemcpy(b->d_order, ord.data(), ord.size() * 4, hipMemcpyHostToDevice));
        char buf[128];
        snprintf(buf, sizeof buf, "-> %s order, %u wavefronts in workgroups of %u lanes",
                 best_order ? "longest-first" : "given", best_grid, 64 * best_wg);
        rep += buf;
        // A graph captured before holds the old schedule.
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    if (report && report_len) {
        size_t k = std::min(report_len - 1, rep.size());
        memcpy(report, rep.data(), k);
        report[k] = 0;
    }
    return HG_OK;
}

}  // extern "C"

// ============================================================ streaming chunker

// Content-based chunking of a stream fed in pieces (Sec. 3.2.4: the written
// data is buffered, each full buffer is chunked on the GPU, and the bytes
// after the last boundary carry into the next buffer).  The device holds
// only the carry -- the bytes from the last decided cut (and w - 1 before
// it, for windows that straddle it) to the end of the data fed so far --
// plus the new piece.  Each feed scans that buffer's windows on the stream's
// absolute stride grid, decides every cut the known bytes determine, hashes
// the completed chunks, and keeps the rest.
struct hg_chunker {
    hg_ctx *ctx = nullptr;
    hg_chunk_params p{};
    uint64_t pos = 0;       // bytes fed so far
    uint64_t last = 0;      // last decided cut (absolute)
    uint64_t base = 0;      // absolute offset of the first carried byte
    uint8_t *buf[2] = {nullptr, nullptr};
    uint64_t cap[2] = {0, 0};
    int cur = 0;            // buffer holding [cur_start, pos)
    uint64_t cur_start = 0; // absolute offset of buf[cur][0]
    bool finished = false;
    // A feed's front half (copy, window scan, boundary decision) runs on the
    // chunker's own stream and ends with one host wait; its back half (ends,
    // chunk digests, counts) on the caller's stream, so that it overlaps
    // the next feed's front half.  Per buffer b: the cut list (rel[b]), the
    // device words of the decision (state + 8 * b), and an event after the
    // back half that last read buffer b.
    hipStream_t front = nullptr;
    hipEvent_t ev_entry = nullptr, ev_front = nullptr, ev_dig[2] = {nullptr, nullptr};
    uint64_t *rel[2] = {nullptr, nullptr};
    uint64_t relcap[2] = {0, 0};
    uint64_t *state = nullptr;  // 32 device words
};

namespace {

// Grows chunker buffer `i` (the working bytes, or with `ends` its cut list)
// to `bytes`: both streams are drained first, since the front stream writes
// it and the caller's stream may still read it.
int chunker_grow(hg_chunker *c, int i, uint64_t bytes, hipStream_t st, bool ends = false) {
    uint64_t &cap = ends ? c->relcap[i] : c->cap[i];
    if (cap >= bytes) return HG_OK;
    const uint64_t want = std::max<uint64_t>(bytes + bytes / 4, 1 << 20);
    HG_HIP(c->ctx, hipStreamSynchronize(st));
    HG_HIP(c->ctx, hipStreamSynchronize(c->front));
    void *&ptr = ends ? (void *&)c->rel[i] : (void *&)c->buf[i];
    if (ptr) HG_HIP(c->ctx, hipFree(ptr));
    ptr = nullptr;
    cap = 0;
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c->ctx, HG_ENOMEM, "chunker buffer of %llu bytes", (unsigned long long)want);
    }
    c->ctx->n_device_allocs++;
    ptr = p;
    cap = want;
    return HG_OK;
}

// Cuts one call can emit for `len` new bytes.
uint64_t chunker_bound(const hg_chunker *c, uint64_t len) {
    const uint64_t span = (c->pos - c->last) + len;
    const uint64_t step = c->p.min_chunk ? c->p.min_chunk : 1;
    return span / step + 2 + (c->p.max_chunk ? span / c->p.max_chunk + 1 : 0);
}

// Room for a feed's candidates before it learns their number: twice the
// expectation for random bytes (mask bits) plus slack, at most one per
// window; a feed that finds more is redone with exact room.
uint64_t chunker_cand_room(const hg_chunk_params &p, uint64_t nwin) {
    const int bits = __builtin_popcount(p.mask);
    const uint64_t expect = bits >= 63 ? 0 : (nwin >> bits);
    return std::min<uint64_t>(nwin, 2 * expect + 4096);
}

int chunker_step(hg_chunker *c, const void *data, uint64_t len, uint32_t flags, uint64_t *ends, uint64_t capacity,
                 uint64_t *n_out, void *digests, void *stream, bool final) {
    hg_ctx *ctx = c->ctx;
    HG_TRY(enter(ctx));
    const bool count_host = flags & HG_COUNT_HOST;
    const bool async = flags & HG_ASYNC;
    const bool ready = flags & HG_IN_READY;
    flags &= ~(uint32_t)(HG_COUNT_HOST | HG_ASYNC | HG_IN_READY);
    HG_TRY(check_flags(ctx, flags, false));
    if (async && !(flags & HG_OUT_DEVICE)) return fail(ctx, HG_EINVAL, "HG_ASYNC requires HG_OUT_DEVICE");
    if (c->finished) return fail(ctx, HG_EINVAL, "the stream is finished (hg_chunker_reset starts a new one)");
    if (len && !data) return fail(ctx, HG_EINVAL, "data is NULL");
    if (!n_out) return fail(ctx, HG_EINVAL, "n_chunks is NULL");
    const uint64_t bound = chunker_bound(c, len);
    if (capacity < bound)
        return fail(ctx, HG_EINVAL, "capacity %llu below the bound %llu (hg_chunker_bound)",
                    (unsigned long long)capacity, (unsigned long long)bound);
    if (!ends) return fail(ctx, HG_EINVAL, "ends is NULL");
    hipStream_t st = (hipStream_t)stream, F = c->front;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    const hg_chunk_params &p = c->p;
    // The working buffer: carry [base, pos) then the new bytes.
    const uint64_t carry = c->pos - c->base, wlen = carry + len;
    const int nxt = 1 - c->cur;
    HG_TRY(chunker_grow(c, nxt, wlen, st));
    HG_TRY(chunker_grow(c, nxt, bound * 8, st, true));
    uint8_t *W = c->buf[nxt];
    uint64_t *rel = c->rel[nxt], *sw = c->state + 8 * nxt;
    // Buffer nxt, its cut list and its state words were last read by the
    // back half of the feed before the previous one.
    HG_HIP(ctx, hipStreamWaitEvent(F, c->ev_dig[nxt], 0));
    // Device input may be written by work still pending on the caller's
    // stream, unless the caller declares it ready.
    const bool host_in = len && !in_dev;
    if (len && in_dev && !ready) {
        HG_HIP(ctx, hipEventRecord(c->ev_entry, st));
        HG_HIP(ctx, hipStreamWaitEvent(F, c->ev_entry, 0));
    }
    if (carry) HG_HIP(ctx, hipMemcpyAsync(W, c->buf[c->cur] + (c->base - c->cur_start), carry,
                                           hipMemcpyDeviceToDevice, F));
    if (len && in_dev) HG_HIP(ctx, hipMemcpyAsync(W + carry, data, len, hipMemcpyDeviceToDevice, F));
    const uint64_t a0 = c->base, last0 = c->last - a0;
    // Windows on the stream's stride grid: the first at an absolute multiple
    // of the stride at or after a0.
    const uint64_t s_ = p.stride, b0 = (s_ - a0 % s_) % s_;
    const uint64_t step = p.min_chunk ? p.min_chunk : 1;
    const bool has_windows = wlen >= b0 + p.window;
    const bool parallel = p.max_chunk == 0 && (step >= p.window || last0 == 0);
    hg::WsPlan plan{};
    void *ws = nullptr, *cand = nullptr;
    if (has_windows) {
        plan = hg::plan_window_scan(W + b0, wlen - b0, p.window, s_, p.window_digest);
        HG_TRY(ensure(ctx, SLOT_WS, hg::window_scan_scratch_bytes(plan), F, &ws));
        if (host_in) {
            // Host bytes arrive in pieces on the copy stream (after the back
            // half that last read this buffer); the tiles whose windows have
            // landed run while later pieces are copied.
            HG_TRY(ensure_copy_stream(ctx));
            HG_HIP(ctx, hipStreamWaitEvent(ctx->copy_stream, c->ev_dig[nxt], 0));
            uint64_t t_done = 0;
            HG_TRY(stream_in(ctx, W + carry, (const uint8_t *)data, len, 1, F,
                             [&](uint64_t off, uint64_t plen) -> int {
                                 const uint64_t avail = carry + off + plen;
                                 uint64_t t_end = plan.n_tiles;
                                 if (avail < wlen) {
                                     const uint64_t have = avail > b0 ? avail - b0 : 0;
                                     const uint64_t nw = have >= p.window ? (have - p.window) / s_ + 1 : 0;
                                     t_end = std::min<uint64_t>(nw / plan.tile_windows, plan.n_tiles);
                                 }
                                 if (t_end > t_done) {
                                     HG_LAUNCH(ctx, HG_K_WINDOW_TILES, F,
                                               hg::launch_window_scan_tile_range(plan, W + b0, wlen - b0, p.window,
                                                                                 s_, p.mask, p.target, ws, t_done,
                                                                                 t_end, F));
                                     t_done = t_end;
                                 }
                                 return HG_OK;
                             },
                             SCAN_PIECE, false, true));
        } else {
            HG_LAUNCH(ctx, HG_K_WINDOW_TILES, F,
                      hg::launch_window_scan_tiles(plan, W + b0, wlen - b0, p.window, s_, p.mask, p.target, ws, F));
        }
        HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, F, hg::launch_window_scan_prefix(plan, ws, &sw[0], F));
    } else {
        if (host_in) {
            HG_TRY(ensure_copy_stream(ctx));
            HG_HIP(ctx, hipStreamWaitEvent(ctx->copy_stream, c->ev_dig[nxt], 0));
            HG_TRY(stream_in(ctx, W + carry, (const uint8_t *)data, len, 1, F,
                             [](uint64_t, uint64_t) { return (int)HG_OK; }, SCAN_PIECE, false));
        }
        HG_HIP(ctx, hg::launch_fill_u32((uint32_t *)&sw[0], 2, 0, F));
    }
    // The rest of the front half with candidate room from the expectation
    // (counts stay on the device); one host wait at the end reads the
    // candidate total and the decision.  With more candidates than room the
    // decision is redone with exact room.
    uint64_t room = has_windows ? chunker_cand_room(p, plan.nwin) : 0;
    uint64_t k = 0, last_w = 0;
    for (int attempt = 0; attempt < 2; attempt++) {
        HG_TRY(ensure(ctx, SLOT_CAND, std::max<uint64_t>(room, 1) * 8, F, &cand));
        if (has_windows)
            HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, F,
                      hg::launch_window_scan_emit(plan, W + b0, wlen - b0, p.window, s_, p.mask, p.target, ws,
                                                  (uint64_t *)cand, room, F));
        // sw[6] = min(total, room), sw[7] = total > room
        HG_HIP(ctx, hg::launch_count_clamp(&sw[0], room, &sw[6], F));
        if (parallel) {
            // The parallel boundary decision, on the candidates that can
            // still be cuts, shifted so that the carried cut is offset 0;
            // its final chunk is provisional unless the stream ends here.
            // (With step >= w no window that starts before the carried cut
            // can still be a cut, so the shifted starts stay non-negative;
            // otherwise the walk below decides.)
            HG_HIP(ctx, hg::launch_stream_drop((const uint64_t *)cand, &sw[6], b0, p.window, last0 + step, &sw[4], F));
            void *shifted, *sel;
            HG_TRY(ensure(ctx, SLOT_AUX, std::max<uint64_t>(room, 1) * 8, F, &shifted));
            HG_HIP(ctx, hg::launch_stream_shift((const uint64_t *)cand, &sw[4], room, b0, last0, (uint64_t *)shifted,
                                                F));
            HG_TRY(ensure(ctx, SLOT_SEL, hg::chunk_select_scratch_bytes(room), F, &sel));
            HG_LAUNCH(ctx, HG_K_CHUNK_SELECT, F,
                      hg::launch_chunk_select((const uint64_t *)shifted, &sw[5], room, p.window, wlen - last0,
                                              p.min_chunk, sel, rel, bound, &sw[1], F));
            HG_HIP(ctx, hg::launch_stream_tail(&sw[1], rel, final, last0, &sw[2], F));
        } else {
            HG_LAUNCH(ctx, HG_K_CHUNK_SELECT, F,
                      hg::launch_stream_walk((const uint64_t *)cand, &sw[6], b0, p.window, wlen, last0, p.min_chunk,
                                             p.max_chunk, final, rel, bound, &sw[2], F));
        }
        HG_HIP(ctx, hipMemcpyAsync(ctx->host_small, sw, 32, hipMemcpyDeviceToHost, F));
        HG_HIP(ctx, hipStreamSynchronize(F));
        const uint64_t total = ctx->host_small[0];
        k = ctx->host_small[2];
        last_w = ctx->host_small[3];
        if (total >= hg::MAX_LANES)
            return fail(ctx, HG_EINVAL, "%llu candidates in one feed (limit 2^31): feed smaller pieces",
                        (unsigned long long)total);
        if (total <= room) break;
        room = total;  // more candidates than expected: once more with exact room
    }
    if (k > bound) return fail(ctx, HG_EDEVICE, "internal: %llu cuts above the bound", (unsigned long long)k);
    // Back half on the caller's stream: absolute ends, digests of the
    // completed chunks, the count.
    HG_HIP(ctx, hipEventRecord(c->ev_front, F));
    HG_HIP(ctx, hipStreamWaitEvent(st, c->ev_front, 0));
    const uint64_t abs_add = a0 + last0;
    if (k) {
        if (out_dev) {
            HG_HIP(ctx, hg::launch_add_u64(ends, rel, &sw[2], bound, abs_add, st));
        } else {
            HG_HIP(ctx, hipMemcpyAsync(ends, rel, k * 8, hipMemcpyDeviceToHost, st));
        }
        if (digests) {
            const int dd = digest_bytes(p.chunk_digest);
            void *ddig = digests;
            if (!out_dev) HG_TRY(ensure(ctx, SLOT_DIG, k * (uint64_t)dd, st, &ddig));
            HG_TRY(chunk_digests_of(ctx, p, W + last0, wlen - last0, rel, &sw[2], k, (uint8_t *)ddig, st));
            if (!out_dev) HG_HIP(ctx, hipMemcpyAsync(digests, ddig, k * (uint64_t)dd, hipMemcpyDeviceToHost, st));
        }
    }
    if (out_dev && !count_host) HG_HIP(ctx, hipMemcpyAsync(n_out, &sw[2], 8, hipMemcpyDeviceToDevice, st));
    else *n_out = k;
    HG_HIP(ctx, hipEventRecord(c->ev_dig[nxt], st));
    if (!async) HG_HIP(ctx, hipStreamSynchronize(st));
    if (!out_dev)
        for (uint64_t i = 0; i < k; i++) ends[i] += abs_add;
    // New carry: from w - 1 bytes before the last cut (windows straddling it).
    c->cur = nxt;
    c->cur_start = a0;
    c->pos += len;
    c->last = a0 + last_w;
    const uint64_t pre = std::min<uint64_t>(p.window - 1, c->last);
    c->base = c->last - pre;
    if (final) c->finished = true;
    return HG_OK;
}

}  // namespace

extern "C" {

int hg_chunker_create(hg_ctx *ctx, const hg_chunk_params *params, hg_chunker **out) {
    HG_TRY(enter(ctx));
    if (!params || !out) return fail(ctx, HG_EINVAL, "params or out is NULL");
    *out = nullptr;
    const hg_chunk_params &p = *params;
    if (digest_bytes(p.window_digest) < 0 || digest_bytes(p.chunk_digest) < 0)
        return fail(ctx, HG_EINVAL, "unknown digest");
    if (p.window == 0 || p.window > HG_MAX_WINDOW)
        return fail(ctx, HG_EINVAL, "window must be in [1, %d]", (int)HG_MAX_WINDOW);
    if (p.stride == 0) return fail(ctx, HG_EINVAL, "stride must be >= 1");
    if (p.max_chunk != 0 && p.max_chunk < std::max<uint64_t>(p.min_chunk, 1))
        return fail(ctx, HG_EINVAL, "max_chunk must be 0 or at least max(min_chunk, 1)");
    hg_chunker *c = new hg_chunker();
    c->ctx = ctx;
    c->p = p;
    bool ok = hipStreamCreateWithFlags(&c->front, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_entry, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_front, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_dig[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_dig[1], hipEventDisableTiming) == hipSuccess &&
              hipMalloc((void **)&c->state, 32 * 8) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        hg_chunker_destroy(c);
        return fail(ctx, HG_EDEVICE, "chunker stream, events or state could not be created");
    }
    ctx->n_device_allocs++;
    // Both buffers start "read": the first waits on them are immediate.
    for (hipEvent_t e : c->ev_dig) HG_HIP(ctx, hipEventRecord(e, c->front));
    *out = c;
    return HG_OK;
}

int hg_chunker_bound(const hg_chunker *c, uint64_t len, uint64_t *bound) {
    if (!c || !bound) return HG_EINVAL;
    *bound = chunker_bound(c, len);
    return HG_OK;
}

int hg_chunker_feed(hg_chunker *c, const void *data, uint64_t len, uint32_t flags, uint64_t *ends,
                    uint64_t capacity, uint64_t *n_chunks, void *chunk_digests, void *stream) {
    if (!c) return HG_EINVAL;
    return chunker_step(c, data, len, flags, ends, capacity, n_chunks, chunk_digests, stream, false);
}

int hg_chunker_finish(hg_chunker *c, uint32_t flags, uint64_t *ends, uint64_t capacity, uint64_t *n_chunks,
                      void *chunk_digests, void *stream) {
    if (!c) return HG_EINVAL;
    return chunker_step(c, nullptr, 0, flags | HG_IN_DEVICE, ends, capacity, n_chunks, chunk_digests, stream, true);
}

int hg_chunker_reset(hg_chunker *c) {
    if (!c) return HG_EINVAL;
    c->pos = c->last = c->base = c->cur_start = 0;
    c->finished = false;
    return HG_OK;
}

void hg_chunker_destroy(hg_chunker *c) {
    if (!c) return;
    (void)hipSetDevice(c->ctx->device);
    (void)hipDeviceSynchronize();
    for (int i = 0; i < 2; i++) {
        if (c->buf[i]) (void)hipFree(c->buf[i]);
        if (c->rel[i]) (void)hipFree(c->rel[i]);
        if (c->ev_dig[i]) (void)hipEventDestroy(c->ev_dig[i]);
    }
    if (c->state) (void)hipFree(c->state);
    if (c->ev_entry) (void)hipEventDestroy(c->ev_entry);
    if (c->ev_front) (void)hipEventDestroy(c->ev_front);
    if (c->front) (void)hipStreamDestroy(c->front);
    delete c;
}

}  // extern "C"

// ============================================================ block map

struct hg_blockmap {
    hg_ctx *ctx = nullptr;
    int kind = 0, d = 0;
    uint64_t capacity = 0, slots = 0, size = 0;
    uint8_t *store = nullptr;
    uint32_t *table = nullptr;
    unsigned long long *words = nullptr;  // [0] stored digests, [1..2] counters of a write
    // per-write scratch, grown on demand
    uint64_t scratch_n = 0;
    uint8_t *state = nullptr, *dup = nullptr, *dig_in = nullptr;
    uint32_t *slot_of = nullptr;
    uint64_t *pos_of = nullptr, *len_in = nullptr;
};

namespace {

void blockmap_free_scratch(hg_blockmap *m) {
    for (void *p : {(void *)m->state, (void *)m->dup, (void *)m->dig_in, (void *)m->slot_of, (void *)m->pos_of,
                    (void *)m->len_in})
        if (p) (void)hipFree(p);
    m->state = m->dup = m->dig_in = nullptr;
    m->slot_of = nullptr;
    m->pos_of = m->len_in = nullptr;
    m->scratch_n = 0;
}

int blockmap_scratch(hg_blockmap *m, uint64_t n, hipStream_t st) {
    if (m->scratch_n >= n) return HG_OK;
    HG_HIP(m->ctx, hipStreamSynchronize(st));
    blockmap_free_scratch(m);
    const uint64_t k = std::max<uint64_t>(n + n / 4, 4096);
    void *p[6] = {};
    const size_t bytes[6] = {k, k, k * (size_t)m->d, k * 4, k * 8, k * 8};
    for (int i = 0; i < 6; i++) {
        if (hipMalloc(&p[i], bytes[i]) != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < i; j++) (void)hipFree(p[j]);
            return fail(m->ctx, HG_ENOMEM, "block-map scratch for %llu chunks", (unsigned long long)n);
        }
    }
    m->state = (uint8_t *)p[0];
    m->dup = (uint8_t *)p[1];
    m->dig_in = (uint8_t *)p[2];
    m->slot_of = (uint32_t *)p[3];
    m->pos_of = (uint64_t *)p[4];
    m->len_in = (uint64_t *)p[5];
    m->scratch_n = k;
    return HG_OK;
}

}  // namespace

extern "C" {

int hg_blockmap_create(hg_ctx *ctx, int digest, uint64_t capacity, hg_blockmap **out) {
    HG_TRY(enter(ctx));
    if (!out) return fail(ctx, HG_EINVAL, "out is NULL");
    *out = nullptr;
    const int d = digest_bytes(digest);
    if (d < 0) return fail(ctx, HG_EINVAL, "unknown digest %d", digest);
    if (capacity == 0 || capacity > (1ull << 30)) return fail(ctx, HG_EINVAL, "capacity must be in [1, 2^30]");
    hg_blockmap *m = new hg_blockmap();
    m->ctx = ctx;
    m->kind = digest;
    m->d = d;
    m->capacity = capacity;
    m->slots = 1;
    while (m->slots < 2 * capacity) m->slots <<= 1;  // load factor <= 1/2
    void *a = nullptr, *b = nullptr, *c = nullptr;
    if (hipMalloc(&a, capacity * (size_t)d) != hipSuccess || hipMalloc(&b, m->slots * 4) != hipSuccess ||
        hipMalloc(&c, 64) != hipSuccess) {
        (void)hipGetLastError();
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        delete m;
        return fail(ctx, HG_ENOMEM, "block map of %llu digests", (unsigned long long)capacity);
    }
    m->store = (uint8_t *)a;
    m->table = (uint32_t *)b;
    m->words = (unsigned long long *)c;
    int st = HG_OK;
    if (hg::launch_fill_u32(m->table, m->slots, 0, nullptr) != hipSuccess ||
        hg::launch_fill_u32((uint32_t *)m->words, 16, 0, nullptr) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess)
        st = fail(ctx, HG_EDEVICE, "block map initialisation failed");
    if (st != HG_OK) {
        (void)hipFree(a);
        (void)hipFree(b);
        (void)hipFree(c);
        delete m;
        return st;
    }
    *out = m;
    return HG_OK;
}

void hg_blockmap_destroy(hg_blockmap *m) {
    if (!m) return;
    (void)hipSetDevice(m->ctx->device);
    (void)hipDeviceSynchronize();
    blockmap_free_scratch(m);
    (void)hipFree(m->store);
    (void)hipFree(m->table);
    (void)hipFree(m->words);
    delete m;
}

int hg_blockmap_size(const hg_blockmap *m, uint64_t *n) {
    if (!m || !n) return HG_EINVAL;
    *n = m->size;
    return HG_OK;
}

int hg_blockmap_write(hg_blockmap *m, const void *digests, const uint64_t *len_b, uint64_t n, uint32_t flags,
                      uint8_t *is_dup, uint64_t *dup_chunks, uint64_t *dup_bytes, void *stream) {
    if (!m) return HG_EINVAL;
    hg_ctx *ctx = m->ctx;
    HG_TRY(enter(ctx));
    const int len_is_ends = (flags & HG_LEN_ENDS) ? 1 : 0;
    if (flags & ~(uint32_t)(HG_IN_DEVICE | HG_OUT_DEVICE | HG_LEN_ENDS))
        return fail(ctx, HG_EINVAL, "unknown flag bits 0x%x", flags);
    if (n && !digests) return fail(ctx, HG_EINVAL, "digests is NULL");
    if (m->size + n > m->capacity)
        return fail(ctx, HG_EBUSY, "block map holds %llu of %llu digests; %llu more may not fit",
                    (unsigned long long)m->size, (unsigned long long)m->capacity, (unsigned long long)n);
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    HG_TRY(blockmap_scratch(m, std::max<uint64_t>(n, 1), st));
    const uint8_t *dig = (const uint8_t *)digests;
    const uint64_t *len = len_b;
    if (!in_dev && n) {
        HG_HIP(ctx, hipMemcpyAsync(m->dig_in, digests, n * (size_t)m->d, hipMemcpyHostToDevice, st));
        dig = m->dig_in;
        if (len_b) {
            HG_HIP(ctx, hipMemcpyAsync(m->len_in, len_b, n * 8, hipMemcpyHostToDevice, st));
            len = m->len_in;
        }
    }
    uint8_t *dup_dev = is_dup ? (out_dev ? is_dup : m->dup) : nullptr;
    hg::BlockMapView v{m->store, m->table, m->slots - 1, &m->words[0]};
    HG_HIP(ctx, hg::launch_blockmap_write(m->kind, v, dig, n, len, len_is_ends, m->state, m->slot_of, m->pos_of,
                                          dup_dev, &m->words[2], st));
    if (is_dup && !out_dev && n) HG_HIP(ctx, hipMemcpyAsync(is_dup, m->dup, n, hipMemcpyDeviceToHost, st));
    HG_HIP(ctx, hipMemcpyAsync(ctx->host_small, m->words, 32, hipMemcpyDeviceToHost, st));
    HG_HIP(ctx, hipStreamSynchronize(st));
    m->size = ctx->host_small[0];
    if (dup_chunks) *dup_chunks = ctx->host_small[2];
    if (dup_bytes) *dup_bytes = ctx->host_small[3];
    return HG_OK;
}

}  // extern "C"
