// chunk.hip -- boundary decision and chunk digests (paper Sec. 3.2.2: the
// last stage decides block boundaries from the window hashes; Fig. 3 legend
// and Sec. 3.2.4: each detected block is then direct-hashed).
//
// Boundary decision: greedy over ascending candidates with a minimum chunk
// size (the system's min/max chunk sizes are given in Sec. 4.3).  The rule
// is sequential; below it is evaluated with speculative per-block chains and
// a short fix-up walk (see cs_spec / cs_fix).
//
// Chunk digests: one lane per chunk, chunks handed out longest-first (see
// segment_digest_kernel).
#include "hg_device.hpp"
#include "hg_internal.hpp"

#include <algorithm>

namespace hg {

// The sequential greedy rule, computed in parallel.  next(j) is the first
// candidate whose end is >= e_j + step; the cuts are the chain first,
// next(first), next(next(first)), ...  Chains that start at different
// candidates merge within a few steps (each step jumps to the first end at
// least `step` further on), which the passes below exploit twice:
//   cs_spec   one wavefront per block of 64 candidates: every lane finds
//             next(j) by a galloping search, and the block walks the chain
//             that would enter it at its first candidate (a 64-bit member
//             mask and the chain's exit);
//   cs_super  one wavefront per superblock of 64 blocks walks the chain that
//             would enter the superblock at its first candidate, block by
//             block, taking each block's speculative mask as soon as it
//             meets it; the result is a member mask per block and an exit
//             per superblock;
//   cs_fix    one wavefront follows the real chain superblock by superblock:
//             from the real entry it walks until it meets the superblock's
//             chain (usually within a block), then keeps the rest; blocks
//             the real chain does not reach are cleared;
//   cs_scan   block offsets (exclusive popcount scan), total, final end;
//   cs_emit   every member writes its end at its offset.
// Each walk falls back to next() until chains meet, so the result is exact
// for any input.
struct SelScratch {
    uint32_t *next;
    unsigned long long *spec_mask, *final_mask, *block_off;
    uint32_t *spec_exit, *super_exit;
};

__device__ __forceinline__ uint64_t usable_count(const uint64_t *starts, uint64_t n, uint32_t w, uint64_t len) {
    // Starts ascend and every window fits, so only the last candidate can end
    // at len; a cut at len is not a separate chunk.
    return (n > 0 && starts[n - 1] + w >= len) ? n - 1 : n;
}

// First index k in [lo, n) with starts[k] + w >= target, or n.
__device__ __forceinline__ uint64_t gallop(const uint64_t *starts, uint64_t lo, uint64_t n, uint32_t w,
                                           uint64_t target) {
    uint64_t step = 1, hi = lo;
    while (hi < n && starts[hi] + w < target) {
        lo = hi + 1;
        hi = lo + step;
        step <<= 1;
    }
    if (hi > n) hi = n;
    while (lo < hi) {  // starts[lo-1] + w < target; answer in [lo, hi]
        const uint64_t mid = (lo + hi) >> 1;
        if (starts[mid] + w < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t rl32(uint32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ unsigned long long rl64(unsigned long long v, int l) {
    return ((unsigned long long)rl32((uint32_t)(v >> 32), l) << 32) | rl32((uint32_t)v, l);
}

// The real chain inside block b from member lane l: its member mask and the
// first member after the block.  Uses the block's speculative chain (sm, se)
// as soon as the walk meets it, next() before that.  Wave-uniform.
__device__ __forceinline__ unsigned long long block_walk(const SelScratch &sc, uint64_t b, int l,
                                                         unsigned long long sm, uint32_t se, uint64_t nu,
                                                         uint64_t &exit) {
    if ((sm >> l) & 1ull) {
        exit = se;
        return sm & (~0ull << l);
    }
    const uint64_t q = b * 64 + (threadIdx.x & 63);
    const uint32_t nx_l = q < nu ? sc.next[q] : (uint32_t)nu;
    unsigned long long m = 0;
    while (true) {
        m |= 1ull << l;
        const uint32_t to = rl32(nx_l, l);
        if (to >= b * 64 + 64 || to >= nu) {
            exit = to;
            return m;
        }
        l = (int)(to - b * 64);
        if ((sm >> l) & 1ull) {
            exit = se;
            return m | (sm & (~0ull << l));
        }
    }
}

__global__ __launch_bounds__(256) void cs_spec(const uint64_t *__restrict__ starts, const uint64_t *__restrict__ n_dev,
                                               uint32_t w, uint64_t len, uint64_t step, SelScratch sc) {
    const uint64_t n = *n_dev;
    const uint64_t nu = usable_count(starts, n, w, len);
    const int lane = threadIdx.x & 63;
    const uint64_t b = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t j = b * 64 + lane;
    const uint64_t nb = (n + 63) / 64;
    if (b >= nb) return;  // whole wavefront
    uint32_t nx = (uint32_t)nu;
    if (j < nu) {
        const uint64_t e = starts[j] + w;
        nx = (uint32_t)gallop(starts, j + 1, nu, w, e + step);
        sc.next[j] = nx;
    }
    unsigned long long mask = 0;
    uint32_t exit = (uint32_t)nu;
    if (b * 64 < nu) {
        int cur = 0;
        while (true) {
            mask |= 1ull << cur;
            const uint32_t to = rl32(nx, cur);
            if (to >= b * 64 + 64 || to >= nu) {
                exit = to;
                break;
            }
            cur = (int)(to - b * 64);
        }
    }
    if (lane == 0) {
        sc.spec_mask[b] = mask;
        sc.spec_exit[b] = exit;
        sc.final_mask[b] = 0;
    }
}

__global__ __launch_bounds__(256) void cs_super(const uint64_t *__restrict__ starts,
                                                const uint64_t *__restrict__ n_dev, uint32_t w, uint64_t len,
                                                SelScratch sc) {
    const uint64_t nu = usable_count(starts, *n_dev, w, len);
    const int lane = threadIdx.x & 63;
    const uint64_t S = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nb = (nu + 63) / 64;
    const uint64_t b0 = S * 64;
    if (b0 >= nb) return;
    const uint64_t q = b0 + lane;
    const unsigned long long sm_l = q < nb ? sc.spec_mask[q] : 0;
    const uint32_t se_l = q < nb ? sc.spec_exit[q] : (uint32_t)nu;
    uint64_t cur = b0 * 64;
    while (cur < nu && (cur >> 6) < b0 + 64) {
        const uint64_t b = cur >> 6;
        const int bl = (int)(b - b0);
        uint64_t exit;
        const unsigned long long m = block_walk(sc, b, (int)(cur & 63), rl64(sm_l, bl), rl32(se_l, bl), nu, exit);
        if (lane == 0) sc.final_mask[b] = m;
        cur = exit;
    }
    if (lane == 0) sc.super_exit[S] = (uint32_t)cur;
}

// Clears the member masks of blocks [lo, hi) (all lanes store).
__device__ __forceinline__ void clear_blocks(const SelScratch &sc, uint64_t lo, uint64_t hi) {
    for (uint64_t q = lo + (threadIdx.x & 63); q < hi; q += 64) sc.final_mask[q] = 0;
}

__global__ __launch_bounds__(64) void cs_fix(const uint64_t *__restrict__ starts, const uint64_t *__restrict__ n_dev,
                                             uint32_t w, uint64_t len, uint64_t step, SelScratch sc) {
    const int lane = threadIdx.x;
    if (len == 0) return;
    const uint64_t n = *n_dev;
    const uint64_t nu = usable_count(starts, n, w, len);
    const uint64_t nb = (nu + 63) / 64;
    uint64_t cur = gallop(starts, 0, nu, w, step);  // first cut (last = 0)
    uint64_t done_b = 0;  // blocks below this index hold their final masks
    while (cur < nu) {
        const uint64_t S = cur >> 12, b0 = S * 64, b_end = b0 + 64 < nb ? b0 + 64 : nb;
        const uint64_t q = b0 + lane;
        const unsigned long long sm_l = q < nb ? sc.spec_mask[q] : 0;
        const uint32_t se_l = q < nb ? sc.spec_exit[q] : (uint32_t)nu;
        const unsigned long long l1_l = q < nb ? sc.final_mask[q] : 0;
        const uint32_t sx = sc.super_exit[S];
        // Nothing of the real chain lies between the last finished block and
        // the entry block.
        clear_blocks(sc, done_b, cur >> 6);
        while (true) {
            const uint64_t b = cur >> 6;
            const int bl = (int)(b - b0), l = (int)(cur & 63);
            const unsigned long long l1 = rl64(l1_l, bl);
            if ((l1 >> l) & 1ull) {
                // On the superblock's chain: the rest of the superblock is right.
                if (lane == 0) sc.final_mask[b] = l1 & (~0ull << l);
                cur = sx;
                done_b = b_end;
                break;
            }
            uint64_t exit;
            const unsigned long long m = block_walk(sc, b, l, rl64(sm_l, bl), rl32(se_l, bl), nu, exit);
            if (lane == 0) sc.final_mask[b] = m;
            if (m & l1) {  // met the superblock's chain inside block b
                cur = sx;
                done_b = b_end;
                break;
            }
            cur = exit;
            done_b = b + 1;
            if (cur >= nu || (cur >> 6) >= b_end) break;  // left the superblock
            clear_blocks(sc, done_b, cur >> 6);            // blocks the chain jumped over
        }
    }
    clear_blocks(sc, done_b, nb);
}

// One workgroup: block offsets = exclusive scan of member counts; the final
// end and the chunk count.
__global__ __launch_bounds__(1024) void cs_scan(const uint64_t *__restrict__ starts, const uint64_t *__restrict__ n_dev,
                                                uint32_t w, uint64_t len, SelScratch sc, uint64_t *__restrict__ ends,
                                                uint64_t cap, uint64_t *__restrict__ n_chunks_dev) {
    __shared__ unsigned long long v[1024];
    const uint32_t t = threadIdx.x;
    if (len == 0) {
        if (t == 0) *n_chunks_dev = 0;
        return;
    }
    const uint64_t nu = usable_count(starts, *n_dev, w, len);
    const uint64_t nb = (nu + 63) / 64;
    unsigned long long carry = 0;
    for (uint64_t c0 = 0; c0 < nb; c0 += 1024) {
        const unsigned long long x = c0 + t < nb ? __builtin_popcountll(sc.final_mask[c0 + t]) : 0;
        v[t] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const unsigned long long y = t >= (uint32_t)off ? v[t - off] : 0;
            __syncthreads();
            v[t] += y;
            __syncthreads();
        }
        if (c0 + t < nb) sc.block_off[c0 + t] = carry + v[t] - x;
        carry += v[1023];
        __syncthreads();
    }
    if (t == 0) {
        if (carry < cap) ends[carry] = len;
        *n_chunks_dev = carry + 1;
    }
}

__global__ __launch_bounds__(256) void cs_emit(const uint64_t *__restrict__ starts, const uint64_t *__restrict__ n_dev,
                                               uint32_t w, uint64_t len, SelScratch sc, uint64_t *__restrict__ ends,
                                               uint64_t cap) {
    const int lane = threadIdx.x & 63;
    const uint64_t b = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nb = (usable_count(starts, *n_dev, w, len) + 63) / 64;
    if (b >= nb) return;
    const unsigned long long m = sc.final_mask[b];
    if (!((m >> lane) & 1ull)) return;
    const uint64_t pos = sc.block_off[b] + __builtin_popcountll(m & ((1ull << lane) - 1ull));
    if (pos < cap) ends[pos] = starts[b * 64 + lane] + w;
}

static inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t chunk_select_scratch_bytes(uint64_t n_starts) {
    const uint64_t nb = (n_starts + 63) / 64 + 1;
    return a256(n_starts * 4 + 4) + 3 * a256(nb * 8) + a256(nb * 4) + a256((nb / 64 + 1) * 4);
}

hipError_t launch_chunk_select(const uint64_t *starts, const uint64_t *n_starts_dev, uint64_t n_starts,
                               uint32_t w, uint64_t len, uint64_t min_chunk, void *scratch, uint64_t *ends,
                               uint64_t cap, uint64_t *n_chunks_dev, hipStream_t s) {
    // n_starts bounds *n_starts_dev (grids and scratch are sized by it).
    const uint64_t nb = (n_starts + 63) / 64 + 1;
    uint8_t *q = (uint8_t *)scratch;
    SelScratch sc;
    sc.next = (uint32_t *)q;                 q += a256(n_starts * 4 + 4);
    sc.spec_mask = (unsigned long long *)q;  q += a256(nb * 8);
    sc.final_mask = (unsigned long long *)q; q += a256(nb * 8);
    sc.block_off = (unsigned long long *)q;  q += a256(nb * 8);
    sc.spec_exit = (uint32_t *)q;            q += a256(nb * 4);
    sc.super_exit = (uint32_t *)q;
    const uint64_t step = min_chunk ? min_chunk : 1;
    hipError_t e;
    if (n_starts) {
        const uint64_t nbl = (n_starts + 63) / 64;
        cs_spec<<<(unsigned)((nbl + 3) / 4), 256, 0, s>>>(starts, n_starts_dev, w, len, step, sc);
        const uint64_t nsb = (nbl + 63) / 64;
        cs_super<<<(unsigned)((nsb + 3) / 4), 256, 0, s>>>(starts, n_starts_dev, w, len, sc);
        cs_fix<<<1, 64, 0, s>>>(starts, n_starts_dev, w, len, step, sc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    cs_scan<<<1, 1024, 0, s>>>(starts, n_starts_dev, w, len, sc, ends, cap, n_chunks_dev);
    if ((e = hipGetLastError()) != hipSuccess || n_starts == 0) return e;
    const uint64_t nbl = (n_starts + 63) / 64;
    cs_emit<<<(unsigned)((nbl + 3) / 4), 256, 0, s>>>(starts, n_starts_dev, w, len, sc, ends, cap);
    return hipGetLastError();
}

// ------------------------------------------------------- segment digests --
// Chunk j is [ends[j-1], ends[j]).  Lengths are uneven (the gaps between
// boundaries are roughly exponential), and a wavefront lasts as long as its
// longest lane, so chunks are first ordered longest-first by a length class
// (log2 with four sub-steps, i.e. classes 19% apart): a histogram, an
// exclusive scan in descending class order and a scatter.  Lane t then
// hashes chunk order[t]: each wavefront gets chunks of nearly equal length,
// and the longest sequential chains start first.  The order inside a class
// depends on atomics, but each digest is written at its chunk's index, so
// the output does not.
constexpr int SEG_CLASSES = 256;

__device__ __forceinline__ uint32_t len_class(uint64_t n) {
    if (n < 4) return (uint32_t)n;
    const int msb = 63 - __builtin_clzll(n);
    return (uint32_t)(msb * 4 + ((n >> (msb - 2)) & 3));
}

// Segment j is [starts[j], ends[j]) (segments the library laid out), or
// without starts [ends[j-1], ends[j]) of a buffer of len bytes, each end
// clamped to len and a decreasing end read as an empty segment, so that ends
// from the caller never lead outside the buffer.
struct Seg {
    uint64_t s, e;
};
__device__ __forceinline__ Seg seg_of(const uint64_t *starts, const uint64_t *ends, uint64_t len, uint64_t j) {
    if (starts) return {starts[j], ends[j]};
    const uint64_t a = j ? (ends[j - 1] < len ? ends[j - 1] : len) : 0;
    const uint64_t b = ends[j] < len ? ends[j] : len;
    return {a, b > a ? b : a};
}
__device__ __forceinline__ uint64_t seg_len(const uint64_t *starts, const uint64_t *ends, uint64_t len, uint64_t j) {
    const Seg g = seg_of(starts, ends, len, j);
    return g.e - g.s;
}
// The number of segments: *n_dev, at most max_n (the bound grids and
// scratch were sized for).
__device__ __forceinline__ uint64_t seg_count(const uint64_t *n_dev, uint64_t max_n) {
    const uint64_t n = *n_dev;
    return n < max_n ? n : max_n;
}

__global__ __launch_bounds__(256) void seg_hist(const uint64_t *__restrict__ starts, const uint64_t *__restrict__ ends,
                                                uint64_t len, const uint64_t *__restrict__ n_dev, uint64_t max_n,
                                                uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[SEG_CLASSES];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t n = seg_count(n_dev, max_n);
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[len_class(seg_len(starts, ends, len, t))], 1u);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(SEG_CLASSES) void seg_offsets(uint32_t *__restrict__ hist) {
    // In place: hist[c] becomes the first position of class c, classes in
    // descending order (longest first).
    __shared__ uint32_t v[SEG_CLASSES];
    const int t = threadIdx.x;
    v[t] = hist[SEG_CLASSES - 1 - t];
    __syncthreads();
    for (int off = 1; off < SEG_CLASSES; off <<= 1) {
        const uint32_t x = t >= off ? v[t - off] : 0;
        __syncthreads();
        v[t] += x;
        __syncthreads();
    }
    const uint32_t incl = v[t];
    hist[SEG_CLASSES - 1 - t] = incl - hist[SEG_CLASSES - 1 - t];
}

// Each workgroup takes a contiguous range of chunks, counts its classes in
// LDS, reserves one range per class with a single global atomic, and then
// places its chunks inside those ranges with LDS atomics.
constexpr uint32_t SCATTER_PER_WG = 2048;

__global__ __launch_bounds__(256) void seg_scatter(const uint64_t *__restrict__ starts, const uint64_t *__restrict__ ends,
                                                   uint64_t len, const uint64_t *__restrict__ n_dev, uint64_t max_n,
                                                   uint32_t *__restrict__ cursor, uint32_t *__restrict__ order) {
    __shared__ uint32_t cnt[SEG_CLASSES], base[SEG_CLASSES];
    const uint32_t t = threadIdx.x;
    const uint64_t n = seg_count(n_dev, max_n);
    const uint64_t lo = (uint64_t)blockIdx.x * SCATTER_PER_WG;
    const uint64_t hi = lo + SCATTER_PER_WG < n ? lo + SCATTER_PER_WG : n;
    cnt[t] = 0;
    __syncthreads();
    for (uint64_t i = lo + t; i < hi; i += 256) atomicAdd(&cnt[len_class(seg_len(starts, ends, len, i))], 1u);
    __syncthreads();
    base[t] = cnt[t] ? atomicAdd(&cursor[t], cnt[t]) : 0;
    cnt[t] = 0;
    __syncthreads();
    for (uint64_t i = lo + t; i < hi; i += 256) {
        const uint32_t c = len_class(seg_len(starts, ends, len, i));
        order[base[c] + atomicAdd(&cnt[c], 1u)] = (uint32_t)i;
    }
}

template <int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void segment_digest_kernel(const uint8_t *__restrict__ in, uint64_t len,
                                                             const uint64_t *__restrict__ starts,
                                                             const uint64_t *__restrict__ ends,
                                                             const uint64_t *__restrict__ n_dev, uint64_t max_n,
                                                             const uint32_t *__restrict__ order,
                                                             uint8_t *__restrict__ out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= seg_count(n_dev, max_n)) return;
    const uint64_t j = order[t];
    const Seg g = seg_of(starts, ends, len, j);
    // Without explicit starts the segments tile [0, len) of one buffer and a
    // tail may be loaded as a whole block below in + len; with explicit
    // starts (files of an arena) only the segment's own bytes are read.
    const uint8_t *buf_end = starts ? in + g.e : in + len;
    uint32_t st[5];
    hash_range<KIND>(in + g.s, g.e - g.s, buf_end, st);
    store_digest<KIND>(out + j * (uint64_t)Hash<KIND>::DIGEST, st);
}

// The longest of the segments [ends[j-1], ends[j]), j < *n_dev <= max_n, to
// *out (which the launcher clears first).
__global__ __launch_bounds__(256) void max_gap_kernel(const uint64_t *__restrict__ ends, uint64_t len,
                                                      const uint64_t *__restrict__ n_dev, uint64_t max_n,
                                                      unsigned long long *__restrict__ out) {
    const uint64_t n = seg_count(n_dev, max_n);
    uint64_t m = 0;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t l = seg_len(nullptr, ends, len, t);
        m = l > m ? l : m;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m) atomicMax(out, (unsigned long long)m);
}

hipError_t launch_max_gap(const uint64_t *ends, uint64_t len, const uint64_t *n_dev, uint64_t max_n, uint64_t *out,
                          hipStream_t s) {
    hipError_t e = launch_fill_u32((uint32_t *)out, 2, 0, s);
    if (e != hipSuccess || max_n == 0) return e;
    const unsigned grid = (unsigned)std::min<uint64_t>((max_n + 255) / 256, 1024);
    max_gap_kernel<<<grid, 256, 0, s>>>(ends, len, n_dev, max_n, (unsigned long long *)out);
    return hipGetLastError();
}

// Chunks hashed on the host leave the device as one packed buffer.  Each
// table record is a slice of at most a few tens of KiB (so that long chunks
// spread over many workgroups) whose destination has its source's address
// modulo 16: the head bytes up to a 16-byte boundary go one by one, the
// body in 16-byte words, then the tail.
__global__ __launch_bounds__(256) void gather_ranges_kernel(const uint8_t *__restrict__ src,
                                                            const uint64_t *__restrict__ tab, uint64_t k,
                                                            uint8_t *__restrict__ dst) {
    for (uint64_t r = blockIdx.x; r < k; r += gridDim.x) {
        const uint8_t *a = src + tab[3 * r];
        const uint64_t n = tab[3 * r + 1];
        uint8_t *b = dst + tab[3 * r + 2];
        const uint64_t mis = (uint64_t)((uintptr_t)a & 15);
        const uint64_t head = n < ((16 - mis) & 15) ? n : ((16 - mis) & 15);
        const uint64_t nv = (n - head) / 16;
        if (threadIdx.x < head) b[threadIdx.x] = a[threadIdx.x];
        const uint4 *av = (const uint4 *)(a + head);
        uint4 *bv = (uint4 *)(b + head);
        for (uint64_t i = threadIdx.x; i < nv; i += blockDim.x) bv[i] = av[i];
        for (uint64_t i = head + nv * 16 + threadIdx.x; i < n; i += blockDim.x) b[i] = a[i];
    }
}

hipError_t launch_gather_ranges(const uint8_t *src, const uint64_t *tab, uint64_t k, uint8_t *dst, hipStream_t s) {
    if (k == 0) return hipSuccess;
    gather_ranges_kernel<<<(unsigned)std::min<uint64_t>(k, 8192), 256, 0, s>>>(src, tab, k, dst);
    return hipGetLastError();
}

// Digests computed elsewhere (on the host): record k of `src` (d bytes) goes
// to out + idx[k] * d.
__global__ __launch_bounds__(256) void digest_scatter_kernel(const uint64_t *__restrict__ idx,
                                                             const uint8_t *__restrict__ src, uint64_t n, int d,
                                                             uint8_t *__restrict__ out) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint8_t *o = out + idx[k] * (uint64_t)d;
    for (int b = 0; b < d; b++) o[b] = src[k * (uint64_t)d + b];
}

hipError_t launch_digest_scatter(const uint64_t *idx, const uint8_t *src, uint64_t n, int d, uint8_t *out,
                                 hipStream_t s) {
    if (n == 0) return hipSuccess;
    digest_scatter_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(idx, src, n, d, out);
    return hipGetLastError();
}

size_t segment_digest_scratch_bytes(uint64_t max_n) {
    return SEG_CLASSES * 4 + ((max_n * 4 + 255) & ~(uint64_t)255) + 256;
}

hipError_t launch_segment_digests(int kind, const uint8_t *in, uint64_t len, const uint64_t *starts,
                                  const uint64_t *ends, const uint64_t *n_dev, uint64_t max_n, uint8_t *out,
                                  void *scratch, hipStream_t s) {
    if (max_n == 0) return hipSuccess;
    uint32_t *hist = (uint32_t *)scratch;
    uint32_t *order = hist + SEG_CLASSES;
    hipError_t e = launch_fill_u32(hist, SEG_CLASSES, 0, s);
    if (e != hipSuccess) return e;
    const unsigned sgrid = (unsigned)std::min<uint64_t>((max_n + 255) / 256, 1024);
    seg_hist<<<sgrid, 256, 0, s>>>(starts, ends, len, n_dev, max_n, hist);
    seg_offsets<<<1, SEG_CLASSES, 0, s>>>(hist);
    seg_scatter<<<(unsigned)((max_n + SCATTER_PER_WG - 1) / SCATTER_PER_WG), 256, 0, s>>>(starts, ends, len, n_dev,
                                                                                           max_n, hist, order);
    const unsigned grid = (unsigned)((max_n + 255) / 256);
    if (kind == KIND_MD5)
        segment_digest_kernel<KIND_MD5><<<grid, 256, 0, s>>>(in, len, starts, ends, n_dev, max_n, order, out);
    else
        segment_digest_kernel<KIND_SHA1><<<grid, 256, 0, s>>>(in, len, starts, ends, n_dev, max_n, order, out);
    return hipGetLastError();
}

// ------------------------------------------------- two-level chunk digests --
// Each chunk direct-hashed by the parallel construction (Sec. 3.2.2, applied
// to every detected chunk as Sec. 3.2.4 describes): the chunk is cut into
// segments of S bytes (the last one shorter), the segment digests are laid
// out in one buffer, and the chunk digest is the digest of that buffer.
//
// Layout without a prefix sum: chunk j's segment digests occupy the slots
// first_j = floor(start_j / S) + j onward.  With start_j = aS + r and length
// len_j, first_{j+1} - first_j = floor((r + len_j) / S) + 1 >= ceil(len_j / S),
// so consecutive chunks never share a slot, and the slot count is at most
// floor(len / S) + n + 1.

__device__ __forceinline__ uint64_t tl_first(const uint64_t *ends, uint64_t len, uint64_t j, uint64_t S) {
    return seg_of(nullptr, ends, len, j).s / S + j;
}

// One lane per slot p: the chunk whose range of slots holds p (the largest j
// with first_j <= p, by binary search), then that chunk's segment.
template <int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void tl_leaf_kernel(
    const uint8_t *__restrict__ in, uint64_t len, const uint64_t *__restrict__ ends,
    const uint64_t *__restrict__ n_dev, uint64_t max_n, uint64_t S, uint64_t n_slots, uint8_t *__restrict__ leaves) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n = seg_count(n_dev, max_n);
    if (p >= n_slots || n == 0) return;
    uint64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint64_t mid = hi - ((hi - lo) >> 1);
        if (tl_first(ends, len, mid, S) <= p) lo = mid;
        else hi = mid - 1;
    }
    const Seg g = seg_of(nullptr, ends, len, lo);
    const uint64_t start = g.s, clen = g.e - g.s;
    const uint64_t k = p - tl_first(ends, len, lo, S);
    if (k >= (clen + S - 1) / S) return;  // a slot between two chunks' ranges
    const uint64_t s0 = start + k * S;
    const uint64_t sl = clen - k * S < S ? clen - k * S : S;
    uint32_t st[5];
    hash_range<KIND>(in + s0, sl, in + len, st);
    store_digest<KIND>(leaves + p * (uint64_t)Hash<KIND>::DIGEST, st);
}

// One lane per chunk: the digest of its ceil(len_j / S) segment digests.
template <int KIND>
__global__ __launch_bounds__(256) void tl_root_kernel(const uint8_t *__restrict__ leaves, uint64_t n_slots,
                                                      uint64_t len, const uint64_t *__restrict__ ends,
                                                      const uint64_t *__restrict__ n_dev, uint64_t max_n, uint64_t S,
                                                      uint8_t *__restrict__ out) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= seg_count(n_dev, max_n)) return;
    constexpr uint64_t D = Hash<KIND>::DIGEST;
    const Seg g = seg_of(nullptr, ends, len, j);
    const uint64_t clen = g.e - g.s;
    // first + ceil(clen / S) <= floor(e / S) + 1 + j < n_slots for clamped
    // ends: the digests read lie inside the slots.
    const uint8_t *p = leaves + tl_first(ends, len, j, S) * D;
    uint32_t st[5];
    hash_range<KIND>(p, (clen + S - 1) / S * D, leaves + n_slots * D, st);
    store_digest<KIND>(out + j * D, st);
}

uint64_t two_level_slots(uint64_t len, uint64_t max_n, uint64_t S) { return len / S + max_n + 1; }

hipError_t launch_chunk_digests_two_level(int kind, const uint8_t *in, uint64_t len, const uint64_t *ends,
                                          const uint64_t *n_dev, uint64_t max_n, uint64_t S, uint8_t *leaves,
                                          uint8_t *out, hipStream_t s) {
    if (max_n == 0) return hipSuccess;
    const uint64_t slots = two_level_slots(len, max_n, S);
    const unsigned lgrid = (unsigned)((slots + 255) / 256), rgrid = (unsigned)((max_n + 255) / 256);
    if (kind == KIND_MD5) {
        tl_leaf_kernel<KIND_MD5><<<lgrid, 256, 0, s>>>(in, len, ends, n_dev, max_n, S, slots, leaves);
        tl_root_kernel<KIND_MD5><<<rgrid, 256, 0, s>>>(leaves, slots, len, ends, n_dev, max_n, S, out);
    } else {
        tl_leaf_kernel<KIND_SHA1><<<lgrid, 256, 0, s>>>(in, len, ends, n_dev, max_n, S, slots, leaves);
        tl_root_kernel<KIND_SHA1><<<rgrid, 256, 0, s>>>(leaves, slots, len, ends, n_dev, max_n, S, out);
    }
    return hipGetLastError();
}

// Two-level digests of chunks given as (start, end) pairs of an arena (file
// batches: chunks of different files need not be in arena order).  Chunk j's
// segment digests occupy slots first[j] .. first[j+1] - 1, first being the
// exclusive prefix sum of ceil(len_j / S), computed in three passes: local
// scans of 1024 chunks per workgroup with their sums, one workgroup scanning
// the sums, and the sums added back.
constexpr int TLS_TPB = 256, TLS_PER = 4, TLS_BLOCK = TLS_TPB * TLS_PER;

__device__ __forceinline__ uint64_t tl_nseg(const uint64_t *starts, const uint64_t *ends, uint64_t j, uint64_t S) {
    const uint64_t len = ends[j] - starts[j];
    return (len + S - 1) / S;
}

// Exclusive scan of v over the workgroup (TLS_TPB lanes); *total gets the sum.
__device__ __forceinline__ unsigned long long wg_exclusive(unsigned long long v, unsigned long long *total) {
    __shared__ unsigned long long wsum[TLS_TPB / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned long long x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    unsigned long long base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < TLS_TPB / 64; i++) {
        base += i < wid ? wsum[i] : 0;
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

__global__ __launch_bounds__(TLS_TPB) void tl_scan_local(const uint64_t *__restrict__ starts,
                                                         const uint64_t *__restrict__ ends,
                                                         const uint64_t *__restrict__ n_dev, uint64_t max_n,
                                                         uint64_t S, uint64_t *__restrict__ first,
                                                         uint64_t *__restrict__ bsum) {
    const uint64_t n = seg_count(n_dev, max_n);
    const uint64_t i0 = (uint64_t)blockIdx.x * TLS_BLOCK + (uint64_t)threadIdx.x * TLS_PER;
    uint64_t c[TLS_PER], t = 0;
#pragma unroll
    for (int q = 0; q < TLS_PER; q++) {
        c[q] = i0 + q < n ? tl_nseg(starts, ends, i0 + q, S) : 0;
        t += c[q];
    }
    unsigned long long total;
    uint64_t run = wg_exclusive(t, &total);
#pragma unroll
    for (int q = 0; q < TLS_PER; q++) {
        if (i0 + q < n) first[i0 + q] = run;
        run += c[q];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the nb block sums in place; bsum[nb] gets
// the total.
__global__ __launch_bounds__(TLS_TPB) void tl_scan_sums(uint64_t *__restrict__ bsum, uint64_t nb) {
    unsigned long long carry = 0;
    for (uint64_t c0 = 0; c0 < nb; c0 += TLS_TPB) {
        const uint64_t i = c0 + threadIdx.x;
        const unsigned long long v = i < nb ? bsum[i] : 0;
        unsigned long long total;
        const unsigned long long ex = wg_exclusive(v, &total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(TLS_TPB) void tl_scan_add(const uint64_t *__restrict__ n_dev, uint64_t max_n,
                                                       uint64_t *__restrict__ first,
                                                       const uint64_t *__restrict__ bsum, uint64_t nb) {
    const uint64_t n = seg_count(n_dev, max_n);
    const uint64_t i0 = (uint64_t)blockIdx.x * TLS_BLOCK + (uint64_t)threadIdx.x * TLS_PER;
    const uint64_t add = bsum[blockIdx.x];
#pragma unroll
    for (int q = 0; q < TLS_PER; q++)
        if (i0 + q < n) first[i0 + q] += add;
    if (blockIdx.x == 0 && threadIdx.x == 0) first[n] = bsum[nb];
}

template <int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void tl_leaf_arena(
    const uint8_t *__restrict__ in, const uint64_t *__restrict__ starts, const uint64_t *__restrict__ ends,
    const uint64_t *__restrict__ n_dev, uint64_t max_n, uint64_t S, const uint64_t *__restrict__ first,
    uint64_t n_slots, uint8_t *__restrict__ leaves) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n = seg_count(n_dev, max_n);
    if (n == 0 || p >= n_slots || p >= first[n]) return;
    uint64_t lo = 0, hi = n - 1;  // the last chunk whose range starts at or before p
    while (lo < hi) {
        const uint64_t mid = hi - ((hi - lo) >> 1);
        if (first[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    const uint64_t k = p - first[lo], clen = ends[lo] - starts[lo];
    const uint64_t s0 = starts[lo] + k * S, sl = clen - k * S < S ? clen - k * S : S;
    uint32_t st[5];
    hash_range<KIND>(in + s0, sl, in + ends[lo], st);
    store_digest<KIND>(leaves + p * (uint64_t)Hash<KIND>::DIGEST, st);
}

template <int KIND>
__global__ __launch_bounds__(256) void tl_root_arena(const uint8_t *__restrict__ leaves, uint64_t n_slots,
                                                     const uint64_t *__restrict__ first,
                                                     const uint64_t *__restrict__ n_dev, uint64_t max_n,
                                                     uint8_t *__restrict__ out) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= seg_count(n_dev, max_n)) return;
    constexpr uint64_t D = Hash<KIND>::DIGEST;
    const uint64_t a = first[j] < n_slots ? first[j] : n_slots;
    const uint64_t b = first[j + 1] < n_slots ? first[j + 1] : n_slots;
    uint32_t st[5];
    hash_range<KIND>(leaves + a * D, (b > a ? b - a : 0) * D, leaves + n_slots * D, st);
    store_digest<KIND>(out + j * D, st);
}

size_t two_level_arena_scratch_bytes(uint64_t max_n) {
    const uint64_t nb = (max_n + TLS_BLOCK - 1) / TLS_BLOCK;
    return ((max_n + 1) * 8 + 255) / 256 * 256 + (nb + 1) * 8;
}

hipError_t launch_chunk_digests_two_level_arena(int kind, const uint8_t *arena, const uint64_t *starts,
                                                const uint64_t *ends, const uint64_t *n_dev, uint64_t max_n,
                                                uint64_t S, void *scratch, uint8_t *leaves, uint64_t n_slots,
                                                uint8_t *out, hipStream_t s) {
    if (max_n == 0) return hipSuccess;
    const uint64_t nb = (max_n + TLS_BLOCK - 1) / TLS_BLOCK;
    uint64_t *first = (uint64_t *)scratch;
    uint64_t *bsum = (uint64_t *)((uint8_t *)scratch + ((max_n + 1) * 8 + 255) / 256 * 256);
    tl_scan_local<<<(unsigned)nb, TLS_TPB, 0, s>>>(starts, ends, n_dev, max_n, S, first, bsum);
    tl_scan_sums<<<1, TLS_TPB, 0, s>>>(bsum, nb);
    tl_scan_add<<<(unsigned)nb, TLS_TPB, 0, s>>>(n_dev, max_n, first, bsum, nb);
    const unsigned lgrid = (unsigned)((n_slots + 255) / 256), rgrid = (unsigned)((max_n + 255) / 256);
    if (kind == KIND_MD5) {
        tl_leaf_arena<KIND_MD5><<<lgrid, 256, 0, s>>>(arena, starts, ends, n_dev, max_n, S, first, n_slots, leaves);
        tl_root_arena<KIND_MD5><<<rgrid, 256, 0, s>>>(leaves, n_slots, first, n_dev, max_n, out);
    } else {
        tl_leaf_arena<KIND_SHA1><<<lgrid, 256, 0, s>>>(arena, starts, ends, n_dev, max_n, S, first, n_slots, leaves);
        tl_root_arena<KIND_SHA1><<<rgrid, 256, 0, s>>>(leaves, n_slots, first, n_dev, max_n, out);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ similarity --
// Digest keys and comparison: dig_hash / dig_equal (hg_device.hpp).

template <int D>
__global__ __launch_bounds__(256) void set_insert(const uint8_t *__restrict__ dig_a, uint64_t n_a,
                                                  uint32_t *__restrict__ table, uint64_t slot_mask) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_a) return;
    const uint8_t *d = dig_a + i * D;
    uint64_t slot = dig_hash<D>(d) & slot_mask;
    // Linear probing; a slot holds (index + 1) of an A digest, 0 = empty.
    for (uint64_t probe = 0; probe <= slot_mask; probe++) {
        const uint32_t prev = atomicCAS(&table[slot], 0u, (uint32_t)(i + 1));
        if (prev == 0) return;
        if (dig_equal<D>(dig_a + (uint64_t)(prev - 1) * D, d)) return;  // already present
        slot = (slot + 1) & slot_mask;
    }
}

template <int D>
__global__ __launch_bounds__(256) void set_probe(const uint8_t *__restrict__ dig_a,
                                                 const uint8_t *__restrict__ dig_b,
                                                 const uint64_t *__restrict__ len_b, int len_is_ends,
                                                 uint64_t n_b, const uint64_t *__restrict__ n_b_dev,
                                                 const uint32_t *__restrict__ table,
                                                 uint64_t slot_mask, unsigned long long *__restrict__ counters) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // With a device count, n_b is its bound.
    const uint64_t nb = n_b_dev && *n_b_dev < n_b ? *n_b_dev : n_b;
    bool hit = false;
    uint64_t bytes = 0;
    if (i < nb) {
        const uint8_t *d = dig_b + i * D;
        uint64_t slot = dig_hash<D>(d) & slot_mask;
        for (uint64_t probe = 0; probe <= slot_mask; probe++) {
            const uint32_t v = table[slot];
            if (v == 0) break;
            if (dig_equal<D>(dig_a + (uint64_t)(v - 1) * D, d)) {
                hit = true;
                break;
            }
            slot = (slot + 1) & slot_mask;
        }
        if (hit && len_b) bytes = len_is_ends ? len_b[i] - (i ? len_b[i - 1] : 0) : len_b[i];
    }
    // Wave reduction, then one atomic per wave.
    const unsigned long long hits = __builtin_popcountll(__ballot(hit));
    unsigned long long b = bytes;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) b += __shfl_xor(b, off, 64);
    if ((threadIdx.x & 63) == 0 && hits) {
        atomicAdd(&counters[0], hits);
        atomicAdd(&counters[1], b);
    }
}

// out[0] = min(*n, max), out[1] = (*n > max).
__global__ void count_clamp_kernel(const uint64_t *__restrict__ n, uint64_t max, uint64_t *__restrict__ out) {
    if (threadIdx.x == 0) {
        const uint64_t v = *n;
        out[0] = v < max ? v : max;
        out[1] = v > max ? 1 : 0;
    }
}

hipError_t launch_count_clamp(const uint64_t *n, uint64_t max, uint64_t *out, hipStream_t s) {
    count_clamp_kernel<<<1, 64, 0, s>>>(n, max, out);
    return hipGetLastError();
}

__global__ void count_invalidate_kernel(const uint64_t *__restrict__ flag, uint64_t *__restrict__ n) {
    if (threadIdx.x == 0 && *flag) *n = ~0ull;
}

hipError_t launch_count_invalidate(const uint64_t *flag, uint64_t *n, hipStream_t s) {
    count_invalidate_kernel<<<1, 64, 0, s>>>(flag, n);
    return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    fill_u32_kernel<<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

__global__ void add_u64_kernel(uint64_t *__restrict__ dst, const uint64_t *__restrict__ src,
                               const uint64_t *__restrict__ n_dev, uint64_t max_n, uint64_t add) {
    const uint64_t n = *n_dev < max_n ? *n_dev : max_n;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] + add;
}

hipError_t launch_add_u64(uint64_t *dst, const uint64_t *src, const uint64_t *n_dev, uint64_t max_n, uint64_t add,
                          hipStream_t s) {
    if (max_n == 0) return hipSuccess;
    uint64_t blocks = (max_n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    add_u64_kernel<<<(unsigned)blocks, 256, 0, s>>>(dst, src, n_dev, max_n, add);
    return hipGetLastError();
}

hipError_t launch_similarity(int kind, const uint8_t *dig_a, uint64_t n_a, const uint8_t *dig_b,
                             const uint64_t *len_b, int len_is_ends, uint64_t n_b, const uint64_t *n_b_dev,
                             uint32_t *table, int log2_slots, unsigned long long *counters, hipStream_t s) {
    const uint64_t slots = 1ull << log2_slots;
    hipError_t e = launch_fill_u32(table, slots, 0, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u32((uint32_t *)counters, 4, 0, s);
    if (e != hipSuccess) return e;
    const uint64_t mask = slots - 1;
    if (n_a) {
        const unsigned g = (unsigned)((n_a + 255) / 256);
        if (kind == KIND_MD5) set_insert<16><<<g, 256, 0, s>>>(dig_a, n_a, table, mask);
        else set_insert<20><<<g, 256, 0, s>>>(dig_a, n_a, table, mask);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (n_b) {
        const unsigned g = (unsigned)((n_b + 255) / 256);
        if (kind == KIND_MD5)
            set_probe<16><<<g, 256, 0, s>>>(dig_a, dig_b, len_b, len_is_ends, n_b, n_b_dev, table, mask, counters);
        else
            set_probe<20><<<g, 256, 0, s>>>(dig_a, dig_b, len_b, len_is_ends, n_b, n_b_dev, table, mask, counters);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hg
