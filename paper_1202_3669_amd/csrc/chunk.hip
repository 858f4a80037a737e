// chunk.hip -- boundary decision and chunk digests (paper Sec. 3.2.2: the
// last stage decides block boundaries from the window hashes; Fig. 3 legend
// and Sec. 3.2.4: each detected block is then direct-hashed).
//
// Boundary decision: greedy over ascending candidates with a minimum chunk
// size (the system's min/max chunk sizes are given in Sec. 4.3).  It is a
// sequential scan; one wavefront runs it, 64 candidates at a time: a ballot
// finds the first candidate end at or beyond last + max(min, 1), a readlane
// moves `last` there, and the chosen lanes are compacted with a popcount.
//
// Chunk digests: segments have uneven lengths, so a fixed lane-per-segment
// mapping leaves most lanes idle behind the longest segment of each wave.
// Here every lane loops over 64-byte message blocks; a lane that finishes a
// segment stores its digest and takes the next segment index from a global
// counter (one atomic per wave per refill), so all lanes stay busy until the
// segment list runs out.
#include "hg_device.hpp"
#include "hg_internal.hpp"

namespace hg {

__global__ __launch_bounds__(64) void chunk_select_kernel(const uint64_t *__restrict__ starts,
                                                          const uint64_t *__restrict__ n_starts_dev,
                                                          uint32_t w, uint64_t len, uint64_t min_chunk,
                                                          uint64_t *__restrict__ ends, uint64_t cap,
                                                          uint64_t *__restrict__ n_chunks_dev) {
    const int lane = threadIdx.x;
    const uint64_t n = *n_starts_dev;
    const uint64_t step = min_chunk ? min_chunk : 1;
    uint64_t last = 0, m = 0;
    if (len == 0) {
        if (lane == 0) *n_chunks_dev = 0;
        return;
    }
    for (uint64_t base = 0; base < n; base += 64) {
        const uint64_t j = base + lane;
        const bool valid = j < n;
        const uint64_t e = valid ? starts[j] + w : ~0ull;
        const bool usable = valid && e < len;
        uint64_t sel = 0;
        while (true) {
            const uint64_t thr = last + step < last ? ~0ull : last + step;  // saturate
            const uint64_t elig = __ballot(usable && e >= thr);
            if (elig == 0) break;
            const int l = __builtin_ctzll(elig);
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)e, l);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(e >> 32), l);
            last = ((uint64_t)hi << 32) | lo;
            sel |= 1ull << l;
        }
        if ((sel >> lane) & 1ull) {
            const uint64_t pos = m + __builtin_popcountll(sel & ((1ull << lane) - 1ull));
            if (pos < cap) ends[pos] = e;
        }
        m += __builtin_popcountll(sel);
    }
    if (lane == 0) {
        if (m < cap) ends[m] = len;
        *n_chunks_dev = m + 1;
    }
}

hipError_t launch_chunk_select(const uint64_t *starts, const uint64_t *n_starts_dev, uint32_t w,
                               uint64_t len, uint64_t min_chunk, uint64_t *ends, uint64_t cap,
                               uint64_t *n_chunks_dev, hipStream_t s) {
    chunk_select_kernel<<<1, 64, 0, s>>>(starts, n_starts_dev, w, len, min_chunk, ends, cap, n_chunks_dev);
    return hipGetLastError();
}

// ------------------------------------------------------- segment digests --
// Per-lane state of the refill loop.
struct SegLane {
    const uint8_t *p;   // segment start
    uint64_t n;         // segment length
    uint64_t done;      // bytes consumed
    uint64_t id;        // segment index
    int phase;          // 0: data blocks, 1: length-only block pending, 2: idle
};

template <int KIND>
__global__ __launch_bounds__(256) void segment_digest_kernel(const uint8_t *__restrict__ in, uint64_t len,
                                                             const uint64_t *__restrict__ ends,
                                                             const uint64_t *__restrict__ n_dev,
                                                             uint8_t *__restrict__ out,
                                                             uint32_t *__restrict__ counter) {
    const uint64_t nseg = *n_dev;
    const uint8_t *buf_end = in + len;
    const int lane = threadIdx.x & 63;
    SegLane L{nullptr, 0, 0, 0, 2};
    uint32_t st[5] = {0, 0, 0, 0, 0};
    while (true) {
        // Refill idle lanes: one atomic per wave hands out consecutive ids.
        const uint64_t idle = __ballot(L.phase == 2);
        if (idle) {
            const uint32_t want = __builtin_popcountll(idle);
            uint32_t first = 0;
            const int leader = __builtin_ctzll(idle);
            if (lane == leader) first = atomicAdd(counter, want);
            first = __builtin_amdgcn_readlane(first, leader);
            if (L.phase == 2) {
                const uint64_t id = first + __builtin_popcountll(idle & ((1ull << lane) - 1ull));
                if (id < nseg) {
                    const uint64_t s0 = id ? ends[id - 1] : 0;
                    L.p = in + s0;
                    L.n = ends[id] - s0;
                    L.done = 0;
                    L.id = id;
                    L.phase = 0;
                    Hash<KIND>::init(st);
                } else {
                    L.phase = 3;  // no work left for this lane
                }
            }
        }
        if (__ballot(L.phase < 2) == 0) break;
        if (L.phase < 2) {
            uint32_t X[16];
            bool last_block = false;
            if (L.phase == 1) {
#pragma unroll
                for (int j = 0; j < 16; j++) X[j] = 0;
                Hash<KIND>::length_words(X, L.n * 8u);
                last_block = true;
            } else if (L.n - L.done >= 64) {
                load_block(L.p + L.done, X);
                L.done += 64;
            } else {
                const int rem = (int)(L.n - L.done);
                load_tail(L.p + L.done, rem, buf_end, X);
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    int valid = rem - 4 * j;
                    valid = valid < 0 ? 0 : (valid > 4 ? 4 : valid);
                    uint32_t v = X[j] & low_bytes_mask(valid);
                    if (j == (rem >> 2)) v |= 0x80u << (8 * (rem & 3));
                    X[j] = v;
                }
                if (rem < 56) {
                    Hash<KIND>::length_words(X, L.n * 8u);
                    last_block = true;
                } else {
                    L.phase = 1;
                }
                L.done = L.n;
            }
            Hash<KIND>::block(st, X);
            if (last_block) {
                store_digest<KIND>(out + L.id * (uint64_t)Hash<KIND>::DIGEST, st);
                L.phase = 2;
            }
        }
    }
}

__global__ void zero_u32_kernel(uint32_t *p) { *p = 0; }

hipError_t launch_segment_digests(int kind, const uint8_t *in, uint64_t len, const uint64_t *ends,
                                  const uint64_t *n_dev, uint64_t max_n, uint8_t *out,
                                  uint32_t *counter, hipStream_t s) {
    if (max_n == 0) return hipSuccess;
    zero_u32_kernel<<<1, 1, 0, s>>>(counter);
    // Enough lanes to cover the chip a few times over, never more than
    // segments (rounded up to whole workgroups).
    uint64_t lanes = max_n < 256ull * 1024 ? max_n : 256ull * 1024;
    const unsigned grid = (unsigned)((lanes + 255) / 256);
    if (kind == KIND_MD5)
        segment_digest_kernel<KIND_MD5><<<grid, 256, 0, s>>>(in, len, ends, n_dev, out, counter);
    else
        segment_digest_kernel<KIND_SHA1><<<grid, 256, 0, s>>>(in, len, ends, n_dev, out, counter);
    return hipGetLastError();
}

// ------------------------------------------------------------ similarity --
// Digests are uniformly distributed, so their first 8 bytes serve as the
// slot hash directly.
template <int D>
__device__ __forceinline__ uint64_t dig_hash(const uint8_t *d) {
    uint64_t h;
    __builtin_memcpy(&h, d, 8);
    return h;
}

template <int D>
__device__ __forceinline__ bool dig_equal(const uint8_t *x, const uint8_t *y) {
    uint32_t a[D / 4], b[D / 4];
    __builtin_memcpy(a, x, D);
    __builtin_memcpy(b, y, D);
    uint32_t diff = 0;
#pragma unroll
    for (int i = 0; i < D / 4; i++) diff |= a[i] ^ b[i];
    return diff == 0;
}

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
                                                 const uint64_t *__restrict__ len_b, uint64_t n_b,
                                                 const uint32_t *__restrict__ table, uint64_t slot_mask,
                                                 unsigned long long *__restrict__ counters) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool hit = false;
    uint64_t bytes = 0;
    if (i < n_b) {
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
        if (hit && len_b) bytes = len_b[i];
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

hipError_t launch_similarity(int kind, const uint8_t *dig_a, uint64_t n_a, const uint8_t *dig_b,
                             const uint64_t *len_b, uint64_t n_b, uint32_t *table, int log2_slots,
                             unsigned long long *counters, hipStream_t s) {
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
        if (kind == KIND_MD5) set_probe<16><<<g, 256, 0, s>>>(dig_a, dig_b, len_b, n_b, table, mask, counters);
        else set_probe<20><<<g, 256, 0, s>>>(dig_a, dig_b, len_b, n_b, table, mask, counters);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace hg
