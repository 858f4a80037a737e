// window_scan.hip -- sliding-window hashing for content-based chunking
// (paper Sec. 2.1 "Content-based chunking" and Sec. 3.2.2): every window of
// w bytes that starts at a multiple of the stride is hashed with the
// standard hash, and a window whose digest matches the predefined value
// ((u32le(D[0..3]) & mask) == target) is a boundary candidate.
//
// gfx950 design.  The paper's GPU kept every window hash in one output
// buffer and let the CPU scan it; here the test runs in the kernel and only
// candidates leave the chip, in ascending order, through three passes:
//   1. count: each 256-lane workgroup owns a tile of consecutive windows;
//      lanes hash their windows, a wavefront scan (DPP/ds_bpermute
//      shuffles) plus an LDS combine ranks the candidates, the tile count is
//      stored and up to WS_CAP tile-local indices go to a per-tile bucket;
//   2. scan: tile counts become tile offsets and a total (chunk sums, a
//      scan of the chunk sums, chunk rescans), and tiles whose count
//      exceeded WS_CAP are listed;
//   3. emit: buckets are copied to their offsets; listed (dense) tiles are
//      hashed again and written directly.
// Two window-loading variants:
//   * registers (w = 20, stride 1 or 4): a lane owns 16 consecutive windows
//     and loads the bytes they span once with 16-byte vector loads; the 16
//     windows are cut out of those registers with v_alignbyte_b32.  The
//     message words past the window are compile-time constants, so their
//     steps fold to a single add of a constant.
//   * LDS (any w up to 4096, any stride, MD5 or SHA-1): the tile's bytes are
//     staged once in LDS and each lane reads its windows from there.
#include "hg_device.hpp"
#include "hg_internal.hpp"

namespace hg {

constexpr int WS_G = 16;                  // windows per lane in the register variants
constexpr uint32_t WS_LDS_MAX = 48 * 1024;  // LDS budget of the generic variant

// -------------------------------------------------------- block ranking --
// Exclusive prefix of v over the workgroup and the workgroup total.  Must be
// reached by every lane of the workgroup.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t &total) {
    __shared__ uint32_t wave_sum[WS_TPB / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
    // Most waves of a window scan have no candidate: their inclusive scan
    // is all zeros, so the shuffle steps run only where some lane has v > 0.
    if (__ballot(v != 0)) {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
    }
    if (lane == 63) wave_sum[wid] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < WS_TPB / 64; i++) {
        uint32_t c = wave_sum[i];
        base += i < wid ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

// ---------------------------------------------- register variant (w=20) --
// Message word j of the single padded MD5 block of the window that starts
// `off` bytes into the lane's dword array dw (all indices compile-time).
template <int W, int ND>
__device__ __forceinline__ uint32_t win_word(const uint32_t (&dw)[ND], const int off, const int j) {
    if (4 * j < W) {
        const int o = off + 4 * j, q = o >> 2, sh = o & 3;
        const int valid = W - 4 * j < 4 ? W - 4 * j : 4;
        uint32_t lo = dw[q];
        uint32_t hi = (q + 1 < ND) ? dw[q + 1] : 0u;
        uint32_t v = sh ? __builtin_amdgcn_alignbyte(hi, lo, sh) : lo;
        if (valid < 4) v = (v & ((1u << (8 * valid)) - 1u)) | (0x80u << (8 * valid));
        return v;
    }
    if (4 * j == W) return 0x80u;
    if (j == 14) return (uint32_t)W * 8u;
    return 0u;
}

// Where a tile's windows come from: one buffer cut into tiles of
// consecutive windows, or files of an arena through a tile map (a tile never
// spans two files, so window indices and offsets stay file-relative).
struct TileView {
    const uint8_t *in;  // the buffer (file) the windows lie in
    uint64_t len;       // its length
    uint64_t nwin;      // its number of windows
    uint64_t k0;        // first window of the tile
};

struct SingleSrc {
    const uint8_t *in;
    uint64_t len, nwin, tile_windows;
    uint64_t t0;  // first tile of the launch (a launch may cover a range of tiles)
    __device__ TileView view(uint64_t t) const { return {in, len, nwin, (t0 + t) * tile_windows}; }
};

struct FileSrc {
    const uint8_t *arena;
    const uint64_t *off, *flen;
    const FileTile *tiles;
    uint32_t w, s;
    __device__ TileView view(uint64_t t) const {
        const FileTile ft = tiles[t];
        const uint64_t L = flen[ft.file];
        return {arena + off[ft.file], L, L >= w ? (L - w) / s + 1 : 0, ft.k0};
    }
};

// Candidate bits of the lane's WS_G windows (bit g = window k0 + g) of a
// tile view.
template <int W, int S>
__device__ __forceinline__ uint32_t ws_reg_bits(const TileView v, uint32_t mask, uint32_t target) {
    constexpr int SPAN = (WS_G - 1) * S + W;
    constexpr int ND = (SPAN + 3) / 4;
    const uint64_t k0 = v.k0 + (uint64_t)threadIdx.x * WS_G;
    if (k0 >= v.nwin) return 0;
    const uint64_t b0 = k0 * S;
    const uint8_t *in = v.in;
    const uint64_t len = v.len;
    uint32_t dw[ND];
    if (b0 + 4 * ND <= len) {
        __builtin_memcpy(dw, in + b0, 4 * ND);
    } else {
        // Last lanes of a buffer: whole dwords while they fit, then single
        // bytes, so nothing at or past len is read.  Bytes past len only
        // feed windows k >= nwin.
#pragma unroll
        for (int j = 0; j < ND; j++) {
            uint32_t x = 0;
            const uint64_t o = b0 + 4 * j;
            if (o + 4 <= len) {
                __builtin_memcpy(&x, in + o, 4);
            } else {
#pragma unroll
                for (int b = 0; b < 3; b++)
                    if (o + b < len) x |= (uint32_t)in[o + b] << (8 * b);
            }
            dw[j] = x;
        }
    }
    const uint32_t st[4] = {MD5_IV0, MD5_IV1, MD5_IV2, MD5_IV3};
    // Candidates are rare (one window in 2^popcount(mask)): per window the
    // test is one 3-input logic op, t = (word0 & mask) ^ target (zero for a
    // candidate), and a running minimum; the lane bits are formed only in
    // waves where some lane saw t = 0.  Windows at or past nwin (the lane's
    // last group may run over) are cleared there.
    uint32_t t[WS_G];
    uint32_t z = 0xFFFFFFFFu;
#pragma unroll
    for (int g = 0; g < WS_G; g++) {
        uint32_t X[16];
#pragma unroll
        for (int j = 0; j < 16; j++) X[j] = win_word<W, ND>(dw, g * S, j);
        t[g] = (md5_compress_word0(st, X) & mask) ^ target;
        z = z < t[g] ? z : t[g];
    }
    uint32_t bits = 0;
    if (__ballot(z == 0)) {
#pragma unroll
        for (int g = 0; g < WS_G; g++) bits |= (uint32_t)(t[g] == 0) << g;
        const uint64_t left = v.nwin - k0;  // >= 1 here
        if (left < WS_G) bits &= (1u << left) - 1u;
    }
    return bits;
}

template <int W, int S, class Src>
__global__ __launch_bounds__(WS_TPB) void ws_reg_count(Src src, uint32_t mask, uint32_t target,
                                                       uint32_t *__restrict__ tile_count,
                                                       uint32_t *__restrict__ bucket) {
    const uint64_t tile = blockIdx.x;
    uint32_t bits = ws_reg_bits<W, S>(src.view(tile), mask, target);
    uint32_t total;
    uint32_t pre = block_exclusive(__popc(bits), total);
    if (threadIdx.x == 0) tile_count[tile] = total;
    if (total <= WS_CAP) {
        uint32_t *bk = bucket + tile * WS_CAP + pre;
        while (bits) {
            int g = __ffs(bits) - 1;
            bits &= bits - 1;
            *bk++ = threadIdx.x * WS_G + g;
        }
    }
}

template <int W, int S, class Src>
__global__ __launch_bounds__(WS_TPB) void ws_reg_direct(Src src, uint32_t mask, uint32_t target,
                                                        const uint32_t *__restrict__ ovf_list,
                                                        const uint32_t *__restrict__ ovf_count,
                                                        const uint64_t *__restrict__ tile_off,
                                                        uint64_t *__restrict__ out, uint64_t cap) {
    const uint32_t n_ovf = *ovf_count;
    for (uint32_t i = blockIdx.x; i < n_ovf; i += gridDim.x) {
        const uint64_t tile = ovf_list[i];
        const TileView v = src.view(tile);
        uint32_t bits = ws_reg_bits<W, S>(v, mask, target);
        uint32_t total;
        uint32_t pre = block_exclusive(__popc(bits), total);
        uint64_t pos = tile_off[tile] + pre;
        const uint64_t k0 = v.k0 + (uint64_t)threadIdx.x * WS_G;
        while (bits) {
            int g = __ffs(bits) - 1;
            bits &= bits - 1;
            if (pos < cap) out[pos] = (k0 + g) * S;
            pos++;
        }
    }
}

// ------------------------------------------------------ generic variant --
// Reads the 32-bit little-endian word at byte offset o of the LDS tile.
__device__ __forceinline__ uint32_t lds_word(const uint32_t *lds, uint32_t o) {
    const uint32_t q = o >> 2, sh = o & 3;
    return __builtin_amdgcn_alignbyte(lds[q + 1], lds[q], sh);
}

// Digest bytes 0..3 (little-endian) of the standard hash of the w bytes at
// LDS byte offset o.
template <int KIND>
__device__ __forceinline__ uint32_t lds_hash_word0(const uint32_t *lds, uint32_t o, uint32_t w) {
    uint32_t st[5];
    Hash<KIND>::init(st);
    uint32_t X[16];
    const uint32_t full = w >> 6;
    for (uint32_t b = 0; b < full; b++) {
#pragma unroll
        for (int j = 0; j < 16; j++) X[j] = lds_word(lds, o + 64 * b + 4 * j);
        Hash<KIND>::block(st, X);
    }
    const int rem = (int)(w & 63);
    const uint32_t ot = o + 64 * full;
#pragma unroll
    for (int j = 0; j < 16; j++) X[j] = (4 * j < rem) ? lds_word(lds, ot + 4 * j) : 0u;
    finish_tail<KIND>(st, X, rem, w);
    return Hash<KIND>::word0(st);
}

// One tile: stage its bytes in LDS, hash its windows in rounds of WS_TPB
// consecutive windows (lane i takes window round*WS_TPB + i), rank
// candidates in window order.  EMIT = false: count + bucket; EMIT = true:
// write offsets at tile_off[tile] onward.
template <int KIND, bool EMIT>
__device__ __forceinline__ void ws_gen_tile(const TileView v, uint64_t tile_windows, uint32_t w, uint32_t s,
                                            uint32_t mask, uint32_t target, uint64_t tile, uint32_t *lds,
                                            uint32_t *tile_count, uint32_t *bucket,
                                            const uint64_t *tile_off, uint64_t *out, uint64_t cap) {
    const uint64_t kf = v.k0;
    const uint64_t ke = kf + tile_windows < v.nwin ? kf + tile_windows : v.nwin;
    const uint8_t *src = v.in + kf * s;
    const uintptr_t base = (uintptr_t)src & ~(uintptr_t)3;
    const uint32_t delta = (uint32_t)((uintptr_t)src - base);
    const uint64_t nbytes = ke > kf ? (ke - 1) * s + w - kf * s + delta : 0;
    const uint32_t ndw = (uint32_t)((nbytes + 3) >> 2);
    const uintptr_t first = (uintptr_t)v.in, end = (uintptr_t)(v.in + v.len);
    for (uint32_t i = threadIdx.x; i <= ndw; i += WS_TPB) {
        const uintptr_t addr = base + 4ull * i;
        uint32_t x = 0;
        if (i < ndw) {
            if (addr >= first && addr + 4 <= end) {
                x = *(const uint32_t *)addr;
            } else {
                // Edge dwords: only the bytes inside the buffer.
                for (int b = 0; b < 4; b++)
                    if (addr + b >= first && addr + b < end) x |= (uint32_t)(*(const uint8_t *)(addr + b)) << (8 * b);
            }
        }
        lds[i] = x;  // the pad dword at index ndw is zero
    }
    __syncthreads();
    uint32_t done = 0;
    const uint64_t pos0 = EMIT ? tile_off[tile] : 0;
    for (uint64_t r0 = 0; r0 < ke - kf; r0 += WS_TPB) {
        const uint64_t k = kf + r0 + threadIdx.x;
        bool hit = false;
        if (k < ke) {
            const uint32_t o = delta + (uint32_t)((r0 + threadIdx.x) * s);
            hit = (lds_hash_word0<KIND>(lds, o, w) & mask) == target;
        }
        uint32_t total;
        const uint32_t pre = block_exclusive(hit ? 1u : 0u, total);
        if (hit) {
            const uint32_t rank = done + pre;
            if (EMIT) {
                if (pos0 + rank < cap) out[pos0 + rank] = k * s;
            } else if (rank < (uint32_t)WS_CAP) {
                bucket[tile * WS_CAP + rank] = (uint32_t)(r0 + threadIdx.x);
            }
        }
        done += total;
    }
    if (!EMIT && threadIdx.x == 0) tile_count[tile] = done;
    __syncthreads();  // the LDS tile may be restaged by the next tile
}

template <int KIND, class Src>
__global__ __launch_bounds__(WS_TPB) void ws_gen_count(Src src, uint64_t tile_windows, uint32_t w, uint32_t s,
                                                       uint32_t mask, uint32_t target,
                                                       uint32_t *__restrict__ tile_count,
                                                       uint32_t *__restrict__ bucket) {
    extern __shared__ uint32_t lds[];
    ws_gen_tile<KIND, false>(src.view(blockIdx.x), tile_windows, w, s, mask, target, blockIdx.x, lds,
                             tile_count, bucket, nullptr, nullptr, 0);
}

template <int KIND, class Src>
__global__ __launch_bounds__(WS_TPB) void ws_gen_direct(Src src, uint64_t tile_windows, uint32_t w, uint32_t s,
                                                        uint32_t mask, uint32_t target,
                                                        const uint32_t *__restrict__ ovf_list,
                                                        const uint32_t *__restrict__ ovf_count,
                                                        const uint64_t *__restrict__ tile_off,
                                                        uint64_t *__restrict__ out, uint64_t cap) {
    extern __shared__ uint32_t lds[];
    const uint32_t n_ovf = *ovf_count;
    for (uint32_t i = blockIdx.x; i < n_ovf; i += gridDim.x) {
        const uint64_t tile = ovf_list[i];
        ws_gen_tile<KIND, true>(src.view(tile), tile_windows, w, s, mask, target, tile, lds, nullptr, nullptr,
                                tile_off, out, cap);
    }
}

// ------------------------------------------------- scan and emit passes --
// Tile counts -> exclusive tile offsets in three passes: per-chunk sums of
// SCAN_CHUNK tiles, one workgroup scanning the chunk sums (and writing the
// total), per-chunk rescans writing the offsets and listing overflowed
// tiles.
constexpr int SCAN_TPB = 1024;
constexpr int SCAN_PER_THREAD = 16;
constexpr uint64_t SCAN_CHUNK = 256 * SCAN_PER_THREAD;

__device__ __forceinline__ unsigned long long block_exclusive64(unsigned long long v, unsigned long long &total) {
    __shared__ unsigned long long ws[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned long long x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) ws[wid] = x;
    __syncthreads();
    unsigned long long base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        base += i < wid ? ws[i] : 0;
        tot += ws[i];
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

__global__ __launch_bounds__(256) void ws_chunk_sums(const uint32_t *__restrict__ tile_count, uint64_t n_tiles,
                                                     unsigned long long *__restrict__ chunk_sum) {
    const uint64_t lo = (uint64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_PER_THREAD;
    unsigned long long sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER_THREAD; i++)
        if (lo + i < n_tiles) sum += tile_count[lo + i];
    unsigned long long total;
    block_exclusive64(sum, total);
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_TPB) void ws_chunk_scan(unsigned long long *__restrict__ chunk_sum, uint64_t n_chunks,
                                                          uint64_t *__restrict__ total_out,
                                                          uint32_t *__restrict__ ovf_count) {
    __shared__ unsigned long long v[SCAN_TPB];
    const uint32_t t = threadIdx.x;
    if (t == 0) *ovf_count = 0;
    unsigned long long carry = 0;
    for (uint64_t c0 = 0; c0 < n_chunks; c0 += SCAN_TPB) {
        const unsigned long long x = c0 + t < n_chunks ? chunk_sum[c0 + t] : 0;
        v[t] = x;
        __syncthreads();
        for (int off = 1; off < SCAN_TPB; off <<= 1) {
            const unsigned long long y = t >= (uint32_t)off ? v[t - off] : 0;
            __syncthreads();
            v[t] += y;
            __syncthreads();
        }
        if (c0 + t < n_chunks) chunk_sum[c0 + t] = carry + v[t] - x;  // exclusive
        carry += v[SCAN_TPB - 1];
        __syncthreads();
    }
    if (t == 0) *total_out = carry;
}

__global__ __launch_bounds__(256) void ws_tile_offsets(const uint32_t *__restrict__ tile_count, uint64_t n_tiles,
                                                       const unsigned long long *__restrict__ chunk_off,
                                                       uint64_t *__restrict__ tile_off,
                                                       uint32_t *__restrict__ ovf_list,
                                                       uint32_t *__restrict__ ovf_count) {
    const uint64_t lo = (uint64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * SCAN_PER_THREAD;
    uint32_t c[SCAN_PER_THREAD];
    unsigned long long sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER_THREAD; i++) {
        c[i] = lo + i < n_tiles ? tile_count[lo + i] : 0;
        sum += c[i];
    }
    unsigned long long total;
    unsigned long long off = chunk_off[blockIdx.x] + block_exclusive64(sum, total);
#pragma unroll
    for (int i = 0; i < SCAN_PER_THREAD; i++) {
        if (lo + i < n_tiles) {
            tile_off[lo + i] = off;
            if (c[i] > (uint32_t)WS_CAP) ovf_list[atomicAdd(ovf_count, 1u)] = (uint32_t)(lo + i);
        }
        off += c[i];
    }
}

template <class Src>
__global__ __launch_bounds__(256) void ws_gather(Src src, const uint32_t *__restrict__ tile_count,
                                                 const uint32_t *__restrict__ bucket,
                                                 const uint64_t *__restrict__ tile_off, uint64_t n_tiles,
                                                 uint32_t s, uint64_t *__restrict__ out, uint64_t cap) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t c = tile_count[t];
    if (c == 0 || c > (uint32_t)WS_CAP) return;
    const uint64_t off = tile_off[t];
    const uint64_t k0 = src.view(t).k0;
    for (uint32_t i = 0; i < c; i++) {
        if (off + i < cap) out[off + i] = (k0 + bucket[t * WS_CAP + i]) * s;
    }
}

__global__ void ws_zero_u64(uint64_t *p) { *p = 0; }

// ----------------------------------------------------------------- host --
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsScratch {
    uint32_t *tile_count, *bucket, *ovf_list, *ovf_count;
    uint64_t *tile_off;
    unsigned long long *chunk_sum;
};

static WsScratch carve(const WsPlan &p, void *scratch) {
    uint8_t *q = (uint8_t *)scratch;
    WsScratch s;
    s.tile_off = (uint64_t *)q;  q += align256(p.n_tiles * 8);
    s.tile_count = (uint32_t *)q; q += align256(p.n_tiles * 4);
    s.bucket = (uint32_t *)q;    q += align256(p.n_tiles * 4 * WS_CAP);
    s.ovf_list = (uint32_t *)q;  q += align256(p.n_tiles * 4);
    s.ovf_count = (uint32_t *)q; q += 256;
    s.chunk_sum = (unsigned long long *)q;
    return s;
}

const uint64_t *window_scan_tile_offsets(const WsPlan &p, const void *scratch) {
    return carve(p, (void *)scratch).tile_off;
}

size_t window_scan_scratch_bytes(const WsPlan &p) {
    const uint64_t n_chunks = (p.n_tiles + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return align256(p.n_tiles * 8) + align256(p.n_tiles * 4) + align256(p.n_tiles * 4 * WS_CAP) +
           align256(p.n_tiles * 4) + 256 + align256(n_chunks * 8);
}

uint64_t window_scan_tile_windows(uint32_t w, uint32_t s, int kind) {
    if (kind == KIND_MD5 && w == 20 && (s == 1 || s == 4)) return (uint64_t)WS_TPB * WS_G;
    // Largest tile whose bytes fit the LDS budget, capped at 2048 windows and
    // rounded to whole rounds of WS_TPB windows when possible.
    uint64_t t = ((uint64_t)WS_LDS_MAX - w - 8) / s + 1;
    if (t > 2048) t = 2048;
    if (t >= WS_TPB) t -= t % WS_TPB;
    if (t == 0) t = 1;
    return t;
}

static WsPlan plan_common(uint32_t w, uint32_t s, int kind) {
    WsPlan p{};
    p.kind = kind;
    p.tile_windows = window_scan_tile_windows(w, s, kind);
    if (kind == KIND_MD5 && w == 20 && (s == 1 || s == 4)) {
        p.variant = s == 1 ? 1 : 2;
        p.lds_bytes = 0;
    } else {
        p.variant = 0;
        p.lds_bytes = (uint32_t)((((p.tile_windows - 1) * s + w + 3 + 3) / 4 + 1) * 4);
    }
    return p;
}

WsPlan plan_window_scan(const uint8_t *in, uint64_t len, uint32_t w, uint32_t s, int kind) {
    (void)in;
    WsPlan p = plan_common(w, s, kind);
    p.nwin = (w == 0 || s == 0 || len < w) ? 0 : (len - w) / s + 1;
    p.n_tiles = p.nwin ? (p.nwin + p.tile_windows - 1) / p.tile_windows : 0;
    return p;
}

WsPlan plan_window_scan_files(uint64_t n_tiles, uint64_t total_windows, uint32_t w, uint32_t s, int kind) {
    WsPlan p = plan_common(w, s, kind);
    p.nwin = total_windows;
    p.n_tiles = n_tiles;
    return p;
}

template <class Src>
static hipError_t launch_tiles(const WsPlan &p, Src src, uint32_t w, uint32_t s, uint32_t mask, uint32_t target,
                               const WsScratch &sc, uint64_t n_tiles, hipStream_t st) {
    const dim3 grid((unsigned)n_tiles), blk(WS_TPB);
    if (p.variant == 1) {
        ws_reg_count<20, 1, Src><<<grid, blk, 0, st>>>(src, mask, target, sc.tile_count, sc.bucket);
    } else if (p.variant == 2) {
        ws_reg_count<20, 4, Src><<<grid, blk, 0, st>>>(src, mask, target, sc.tile_count, sc.bucket);
    } else if (p.kind == KIND_MD5) {
        ws_gen_count<KIND_MD5, Src><<<grid, blk, p.lds_bytes, st>>>(src, p.tile_windows, w, s, mask, target,
                                                                   sc.tile_count, sc.bucket);
    } else {
        ws_gen_count<KIND_SHA1, Src><<<grid, blk, p.lds_bytes, st>>>(src, p.tile_windows, w, s, mask, target,
                                                                    sc.tile_count, sc.bucket);
    }
    return hipGetLastError();
}

hipError_t launch_window_scan_tile_range(const WsPlan &p, const uint8_t *in, uint64_t len, uint32_t w, uint32_t s,
                                         uint32_t mask, uint32_t target, void *scratch, uint64_t t0, uint64_t t1,
                                         hipStream_t st) {
    if (t1 > p.n_tiles) t1 = p.n_tiles;
    // At most LAUNCH_LANES / WS_TPB tiles per launch.
    constexpr uint64_t MAX_TILES = LAUNCH_LANES / WS_TPB;
    for (; t0 < t1; t0 += MAX_TILES) {
        const uint64_t n = t1 - t0 < MAX_TILES ? t1 - t0 : MAX_TILES;
        WsScratch sc = carve(p, scratch);
        // The kernels index their outputs by the launch's own tile number.
        sc.tile_count += t0;
        sc.bucket += t0 * WS_CAP;
        const hipError_t e =
            launch_tiles(p, SingleSrc{in, len, p.nwin, p.tile_windows, t0}, w, s, mask, target, sc, n, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_window_scan_tiles(const WsPlan &p, const uint8_t *in, uint64_t len, uint32_t w,
                                    uint32_t s, uint32_t mask, uint32_t target, void *scratch,
                                    hipStream_t st, const WsFiles *files) {
    if (p.n_tiles == 0) return hipSuccess;
    if (!files) return launch_window_scan_tile_range(p, in, len, w, s, mask, target, scratch, 0, p.n_tiles, st);
    constexpr uint64_t MAX_TILES = LAUNCH_LANES / WS_TPB;
    for (uint64_t t0 = 0; t0 < p.n_tiles; t0 += MAX_TILES) {
        const uint64_t n = p.n_tiles - t0 < MAX_TILES ? p.n_tiles - t0 : MAX_TILES;
        WsScratch sc = carve(p, scratch);
        sc.tile_count += t0;
        sc.bucket += t0 * WS_CAP;
        const hipError_t e = launch_tiles(p, FileSrc{files->arena, files->off, files->len, files->tiles + t0, w, s},
                                          w, s, mask, target, sc, n, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_window_scan_prefix(const WsPlan &p, void *scratch, uint64_t *total_dev, hipStream_t st) {
    if (p.n_tiles == 0) {
        ws_zero_u64<<<1, 1, 0, st>>>(total_dev);
        return hipGetLastError();
    }
    WsScratch sc = carve(p, scratch);
    const uint64_t n_chunks = (p.n_tiles + SCAN_CHUNK - 1) / SCAN_CHUNK;
    ws_chunk_sums<<<(unsigned)n_chunks, 256, 0, st>>>(sc.tile_count, p.n_tiles, sc.chunk_sum);
    ws_chunk_scan<<<1, SCAN_TPB, 0, st>>>(sc.chunk_sum, n_chunks, total_dev, sc.ovf_count);
    ws_tile_offsets<<<(unsigned)n_chunks, 256, 0, st>>>(sc.tile_count, p.n_tiles, sc.chunk_sum, sc.tile_off,
                                                        sc.ovf_list, sc.ovf_count);
    return hipGetLastError();
}

template <class Src>
static hipError_t launch_emit(const WsPlan &p, Src src, uint32_t w, uint32_t s, uint32_t mask, uint32_t target,
                              const WsScratch &sc, uint64_t *out, uint64_t cap, hipStream_t st) {
    ws_gather<Src><<<dim3((unsigned)((p.n_tiles + 255) / 256)), dim3(256), 0, st>>>(
        src, sc.tile_count, sc.bucket, sc.tile_off, p.n_tiles, s, out, cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned dgrid = (unsigned)(p.n_tiles < 1024 ? p.n_tiles : 1024);
    if (p.variant == 1) {
        ws_reg_direct<20, 1, Src><<<dgrid, WS_TPB, 0, st>>>(src, mask, target, sc.ovf_list, sc.ovf_count,
                                                           sc.tile_off, out, cap);
    } else if (p.variant == 2) {
        ws_reg_direct<20, 4, Src><<<dgrid, WS_TPB, 0, st>>>(src, mask, target, sc.ovf_list, sc.ovf_count,
                                                           sc.tile_off, out, cap);
    } else if (p.kind == KIND_MD5) {
        ws_gen_direct<KIND_MD5, Src><<<dgrid, WS_TPB, p.lds_bytes, st>>>(
            src, p.tile_windows, w, s, mask, target, sc.ovf_list, sc.ovf_count, sc.tile_off, out, cap);
    } else {
        ws_gen_direct<KIND_SHA1, Src><<<dgrid, WS_TPB, p.lds_bytes, st>>>(
            src, p.tile_windows, w, s, mask, target, sc.ovf_list, sc.ovf_count, sc.tile_off, out, cap);
    }
    return hipGetLastError();
}

hipError_t launch_window_scan_emit(const WsPlan &p, const uint8_t *in, uint64_t len, uint32_t w,
                                   uint32_t s, uint32_t mask, uint32_t target, void *scratch,
                                   uint64_t *out, uint64_t cap, hipStream_t st, const WsFiles *files) {
    if (p.n_tiles == 0 || cap == 0 || out == nullptr) return hipSuccess;
    WsScratch sc = carve(p, scratch);
    if (files) return launch_emit(p, FileSrc{files->arena, files->off, files->len, files->tiles, w, s}, w, s,
                                  mask, target, sc, out, cap, st);
    return launch_emit(p, SingleSrc{in, len, p.nwin, p.tile_windows, 0}, w, s, mask, target, sc, out, cap, st);
}

}  // namespace hg
