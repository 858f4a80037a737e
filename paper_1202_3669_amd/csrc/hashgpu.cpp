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
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "hashgpu.h"
#include "hg_internal.hpp"

namespace {

enum Slot {
    SLOT_IN = 0,   // device copy of host input (or of dig_a)
    SLOT_IN2,      // device copy of dig_b
    SLOT_IN3,      // device copy of len_b
    SLOT_LEAVES,   // segment digests
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
    N_SLOTS
};

constexpr size_t STAGE_PIECE = 64ull << 20;  // bytes per pinned staging buffer

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

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
    std::unordered_set<void *> host_allocs;
    // Kernel timing (hg_timing_*).
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<TimedLaunch> pending;
    uint64_t t_launches[HG_K_COUNT] = {};
    double t_ms[HG_K_COUNT] = {};
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
        b.bytes = want;
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
              hipStream_t st, F on_piece) {
    if (n == 0) return HG_OK;
    HG_TRY(ensure_copy_stream(ctx));
    const bool pinned = is_pinned_host(src);
    if (!pinned) HG_TRY(ensure_stage(ctx));
    uint64_t piece = STAGE_PIECE;
    if (align > 1) piece = std::max<uint64_t>(align, piece - piece % align);
    // Pieces larger than a staging buffer cannot go through it: copy those
    // in one synchronous step.
    if (!pinned && piece > STAGE_PIECE) {
        HG_HIP(ctx, hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st));
        return on_piece(0, n);
    }
    // The copy stream must not overwrite memory still read by earlier work.
    HG_HIP(ctx, hipEventRecord(ctx->piece_ready, st));
    HG_HIP(ctx, hipStreamWaitEvent(ctx->copy_stream, ctx->piece_ready, 0));
    int k = 0;
    for (uint64_t off = 0; off < n; off += piece, k ^= 1) {
        const uint64_t len = std::min(piece, n - off);
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

// Reads one device uint64 (synchronizes the stream).
int read_u64(hg_ctx *ctx, const uint64_t *dev, hipStream_t st, uint64_t *v) {
    HG_HIP(ctx, hipMemcpyAsync(ctx->host_small, dev, 8, hipMemcpyDeviceToHost, st));
    HG_HIP(ctx, hipStreamSynchronize(st));
    *v = ctx->host_small[0];
    return HG_OK;
}

int copy_out(hg_ctx *ctx, void *dst, const void *src, size_t n, bool dst_device, hipStream_t st) {
    if (n == 0) return HG_OK;
    HG_HIP(ctx, hipMemcpyAsync(dst, src, n, dst_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
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

int hg_create(int device, hg_ctx **out) {
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
        hg_destroy(ctx);
        return HG_EDEVICE;
    }
    *out = ctx;
    return HG_OK;
}

void hg_destroy(hg_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &b : ctx->slot)
        if (b.p) (void)hipFree(b.p);
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
    if (ctx->piece_ready) (void)hipEventDestroy(ctx->piece_ready);
    if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
    delete ctx;
}

int hg_host_alloc(hg_ctx *ctx, size_t bytes, void **out) {
    HG_TRY(enter(ctx));
    if (!out || bytes == 0) return fail(ctx, HG_EINVAL, "hg_host_alloc: NULL out or zero size");
    void *p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, HG_ENOMEM, "pinned allocation of %zu bytes failed: %s", bytes,
                    hipGetErrorString(e));
    }
    ctx->host_allocs.insert(p);
    *out = p;
    return HG_OK;
}

int hg_host_free(hg_ctx *ctx, void *p) {
    HG_TRY(enter(ctx));
    if (!p) return HG_OK;
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
        // Pieces hold whole segments; each piece's segments are hashed as
        // soon as the piece has landed.
        HG_TRY(stream_in(ctx, din, (const uint8_t *)in, len, block_size, st,
                         [&](uint64_t off, uint64_t plen) -> int {
                             const uint64_t k0 = off / block_size;
                             const uint64_t k1 = (off + plen + block_size - 1) / block_size;
                             HG_LAUNCH(ctx, HG_K_LEAVES, st,
                                       hg::launch_leaves(digest, din + off, plen, block_size, k1 - k0,
                                                         leaves + k0 * (uint64_t)d, st));
                             return HG_OK;
                         }));
    }
    if (root_out) HG_LAUNCH(ctx, HG_K_ROOT, st, hg::launch_hash_one(digest, leaves, n * (uint64_t)d, root, st));
    if (leaf_out && !out_dev) HG_TRY(copy_out(ctx, leaf_out, leaves, n * (uint64_t)d, false, st));
    if (root_out && !out_dev) HG_TRY(copy_out(ctx, root_out, root, (size_t)d, false, st));
    if (!(flags & HG_ASYNC)) HG_HIP(ctx, hipStreamSynchronize(st));
    return HG_OK;
}

}  // extern "C"

namespace {

// Shared body of the three batch entry points.
int batch_call(hg_ctx *ctx, const hg_block_job *jobs, uint32_t n_jobs, uint32_t flags, void *stream,
               bool leaves, bool roots) {
    HG_TRY(enter(ctx));
    if (flags & ~(uint32_t)(HG_IN_DEVICE | HG_OUT_DEVICE | HG_ASYNC | HG_BACKGROUND))
        return fail(ctx, HG_EINVAL, "unknown flag bits 0x%x", flags);
    const bool boost = !(flags & HG_BACKGROUND);
    if ((flags & HG_ASYNC) && !(flags & HG_IN_DEVICE))
        return fail(ctx, HG_EINVAL, "HG_ASYNC requires a device job table (HG_IN_DEVICE)");
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
    void *plan;
    HG_TRY(ensure(ctx, SLOT_PLAN, hg::batch_plan_bytes(n_jobs), st, &plan));
    HG_HIP(ctx, hg::launch_batch_plan(djobs, n_jobs, plan, st));
    if (leaves) {
        // A persistent grid of up to 8192 one-wavefront workgroups (8 waves
        // per CU); fewer when the host knows there are fewer segments.
        uint32_t grid = 8192;
        if (host_table) grid = (uint32_t)std::max<uint64_t>(2, std::min<uint64_t>(grid, (total_leaves + 63) / 64 + 1));
        HG_LAUNCH(ctx, HG_K_LEAVES_BATCH, st, hg::launch_leaves_batch(djobs, n_jobs, plan, grid, boost, st));
    }
    if (roots) HG_LAUNCH(ctx, HG_K_ROOTS_BATCH, st, hg::launch_roots_batch(djobs, n_jobs, plan, boost, st));
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
    HG_TRY(device_input(ctx, SLOT_IN, in, len, in_dev, st, &din));
    const hg::WsPlan plan = hg::plan_window_scan(din, len, window, stride, digest);
    void *ws;
    HG_TRY(ensure(ctx, SLOT_WS, hg::window_scan_scratch_bytes(plan), st, &ws));
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    uint64_t *total_dev = out_dev ? count : small;
    HG_LAUNCH(ctx, HG_K_WINDOW_TILES, st,
              hg::launch_window_scan_tiles(plan, din, len, window, stride, mask, target, ws, st));
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

int hg_chunk(hg_ctx *ctx, const void *in, uint64_t len, const hg_chunk_params *pr, uint64_t *ends,
             uint64_t capacity, uint64_t *n_chunks, void *chunk_digests, uint32_t flags, void *stream) {
    HG_TRY(enter(ctx));
    HG_TRY(check_flags(ctx, flags, false));
    if (!pr) return fail(ctx, HG_EINVAL, "params is NULL");
    if (digest_bytes(pr->window_digest) < 0 || digest_bytes(pr->chunk_digest) < 0)
        return fail(ctx, HG_EINVAL, "unknown digest");
    if (pr->window == 0 || pr->window > HG_MAX_WINDOW)
        return fail(ctx, HG_EINVAL, "window must be in [1, %d]", (int)HG_MAX_WINDOW);
    if (pr->stride == 0) return fail(ctx, HG_EINVAL, "stride must be >= 1");
    if (pr->max_chunk != 0) return fail(ctx, HG_EINVAL, "max_chunk must be 0");
    if (!n_chunks) return fail(ctx, HG_EINVAL, "n_chunks is NULL");
    if (capacity && !ends) return fail(ctx, HG_EINVAL, "ends is NULL with capacity > 0");
    if (len && !in) return fail(ctx, HG_EINVAL, "in is NULL");
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    const int dd = digest_bytes(pr->chunk_digest);

    const uint8_t *din;
    HG_TRY(device_input(ctx, SLOT_IN, in, len, in_dev, st, &din));
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    // small[0]: candidate total, small[1]: chunk count.
    const hg::WsPlan plan = hg::plan_window_scan(din, len, pr->window, pr->stride, pr->window_digest);
    void *ws;
    HG_TRY(ensure(ctx, SLOT_WS, hg::window_scan_scratch_bytes(plan), st, &ws));
    HG_LAUNCH(ctx, HG_K_WINDOW_TILES, st,
              hg::launch_window_scan_tiles(plan, din, len, pr->window, pr->stride, pr->mask, pr->target,
                                           ws, st));
    HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, st, hg::launch_window_scan_prefix(plan, ws, &small[0], st));
    uint64_t n_cand;
    HG_TRY(read_u64(ctx, &small[0], st, &n_cand));
    void *cand, *dends, *ddig = nullptr;
    HG_TRY(ensure(ctx, SLOT_CAND, n_cand * 8, st, &cand));
    HG_TRY(ensure(ctx, SLOT_ENDS, (n_cand + 1) * 8, st, &dends));
    if (chunk_digests) HG_TRY(ensure(ctx, SLOT_DIG, (n_cand + 1) * (uint64_t)dd, st, &ddig));
    HG_LAUNCH(ctx, HG_K_WINDOW_EMIT, st,
              hg::launch_window_scan_emit(plan, din, len, pr->window, pr->stride, pr->mask, pr->target, ws,
                                          (uint64_t *)cand, n_cand, st));
    void *sel;
    HG_TRY(ensure(ctx, SLOT_SEL, hg::chunk_select_scratch_bytes(n_cand), st, &sel));
    HG_LAUNCH(ctx, HG_K_CHUNK_SELECT, st,
              hg::launch_chunk_select((const uint64_t *)cand, &small[0], n_cand, pr->window, len,
                                      pr->min_chunk, sel, (uint64_t *)dends, n_cand + 1, &small[1], st));
    if (chunk_digests) {
        void *segs;
        HG_TRY(ensure(ctx, SLOT_SEG, hg::segment_digest_scratch_bytes(n_cand + 1), st, &segs));
        HG_LAUNCH(ctx, HG_K_CHUNK_DIGESTS, st,
                  hg::launch_segment_digests(pr->chunk_digest, din, len, (const uint64_t *)dends, &small[1],
                                             n_cand + 1, (uint8_t *)ddig, segs, st));
    }
    uint64_t nc;
    HG_TRY(read_u64(ctx, &small[1], st, &nc));
    const uint64_t k = std::min(nc, capacity);
    HG_TRY(copy_out(ctx, ends, dends, k * 8, out_dev, st));
    if (chunk_digests) HG_TRY(copy_out(ctx, chunk_digests, ddig, k * (uint64_t)dd, out_dev, st));
    if (out_dev) HG_TRY(copy_out(ctx, n_chunks, &small[1], 8, true, st));
    HG_HIP(ctx, hipStreamSynchronize(st));
    if (!out_dev) *n_chunks = nc;
    return nc > capacity ? fail(ctx, HG_ETRUNC, "%llu chunks, capacity %llu", (unsigned long long)nc,
                                (unsigned long long)capacity)
                         : HG_OK;
}

int hg_similarity(hg_ctx *ctx, const void *dig_a, uint64_t n_a, const void *dig_b, const uint64_t *len_b,
                  uint64_t n_b, int digest, uint64_t *matched, uint64_t *matched_bytes, uint32_t flags,
                  void *stream) {
    HG_TRY(enter(ctx));
    const bool len_ends = flags & HG_LEN_ENDS;
    flags &= ~(uint32_t)HG_LEN_ENDS;
    HG_TRY(check_flags(ctx, flags, true));
    const int d = digest_bytes(digest);
    if (d < 0) return fail(ctx, HG_EINVAL, "unknown digest %d", digest);
    if (!matched) return fail(ctx, HG_EINVAL, "matched is NULL");
    if ((n_a && !dig_a) || (n_b && !dig_b)) return fail(ctx, HG_EINVAL, "NULL digest array");
    if (n_a >= (1ull << 31)) return fail(ctx, HG_EINVAL, "n_a too large");
    hipStream_t st = (hipStream_t)stream;
    const bool in_dev = flags & HG_IN_DEVICE, out_dev = flags & HG_OUT_DEVICE;
    const uint8_t *da, *db, *dl = nullptr;
    HG_TRY(device_input(ctx, SLOT_IN, dig_a, n_a * (uint64_t)d, in_dev, st, &da));
    HG_TRY(device_input(ctx, SLOT_IN2, dig_b, n_b * (uint64_t)d, in_dev, st, &db));
    if (len_b) HG_TRY(device_input(ctx, SLOT_IN3, len_b, n_b * 8, in_dev, st, &dl));
    int log2_slots = 6;
    while ((1ull << log2_slots) < 2 * n_a) log2_slots++;
    void *table;
    HG_TRY(ensure(ctx, SLOT_TABLE, (1ull << log2_slots) * 4, st, &table));
    uint64_t *small;
    HG_TRY(small_words(ctx, st, &small));
    unsigned long long *counters = (unsigned long long *)&small[4];
    HG_LAUNCH(ctx, HG_K_SIMILARITY, st,
              hg::launch_similarity(digest, da, n_a, db, (const uint64_t *)dl, len_ends ? 1 : 0, n_b,
                                    (uint32_t *)table, log2_slots, counters, st));
    HG_TRY(copy_out(ctx, matched, &counters[0], 8, out_dev, st));
    if (matched_bytes) HG_TRY(copy_out(ctx, matched_bytes, &counters[1], 8, out_dev, st));
    if (!(flags & HG_ASYNC)) HG_HIP(ctx, hipStreamSynchronize(st));
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
    }
    return HG_OK;
}

}  // extern "C"
