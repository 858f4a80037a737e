// block_hash.hip -- direct hashing with the parallel Merkle-Damgard
// construction (paper Sec. 3.2.2, "Direct Hashing"): the block is split into
// fixed-size segments, every segment is hashed by its own lane with the
// sequential hash, the digests land in one buffer in segment order, and that
// buffer is hashed again for the final value.
//
// Mapping on gfx950: one lane per segment, 256 lanes per workgroup.  A lane
// walks its segment 128 bytes (one line, two blocks) at a time with 16-byte
// vector loads, double buffered, and keeps the chaining state in VGPRs; the
// register budget is held to four waves per SIMD, enough to fill the chip
// with one lane per 4 KiB segment of 1 GiB.  The second level is one lane
// over the digest buffer.
#include "hg_device.hpp"
#include "hg_internal.hpp"

namespace hg {

template <int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void leaf_kernel(const uint8_t *__restrict__ in, uint64_t len,
                                                   uint64_t block, uint64_t n_leaves,
                                                   uint8_t *__restrict__ out) {
    uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_leaves) return;
    uint64_t start = k * block;
    uint64_t n = len - start < block ? len - start : block;
    uint32_t st[5];
    hash_range<KIND>(in + start, n, in + len, st);
    store_digest<KIND>(out + k * (uint64_t)Hash<KIND>::DIGEST, st);
}

// Segments read through LDS.  With one lane per segment, a 16-byte load
// instruction of a wave touches 64 lines (one per lane).  Here the wave loads
// its segments' next 128-byte lines together: in load instruction j, lane l
// reads 16-byte piece (l & 7) of segment 8j + (l >> 3) of a group of 64, so
// each instruction reads 8 whole lines; the pieces go to an LDS tile (one
// 144-byte row per segment: 16 bytes of padding make both the row writes and
// the per-lane row reads conflict-free) and every lane then reads its own
// row.  The next line pair is loaded while the current one is compressed.
//
// Segments of one size start at multiples of that size, so lanes that all
// read pair q of their segments hit addresses equal modulo the segment size,
// which HBM serves at about three quarters of its streaming rate.  Each lane
// therefore runs two chains, segments k0 + lane (group A) and k0 + 64 + lane
// (group B), with B half a segment behind A: the wave reads two offsets at a
// time.  The work is the same; the first and last half of the pairs have
// one chain per lane instead of two.  Each lane finishes the rest of its two
// segments (beyond the pairs all segments of the wave have) on its own.
constexpr int LDS_ROW = 9;  // 16-byte units per row: 8 of data, 1 of padding

// 16 bytes at offset `off` of segment `seg`.  Past the last segment (only in
// the last wave, which then holds that segment, so `off` lies inside it) the
// last segment is read instead: the row belongs to an inactive lane and is
// not used.  The input is read once: nontemporal loads (measured: 5% faster
// over 1 GiB of 4 KiB segments than ordinary ones).
typedef uint32_t lds_u32x4 __attribute__((ext_vector_type(4), aligned(1)));

__device__ __forceinline__ uint4 lds_piece(const uint8_t *in, uint64_t block, uint64_t n_leaves, uint64_t seg,
                                           uint64_t off) {
    const uint64_t s = seg < n_leaves ? seg : n_leaves - 1;
    const lds_u32x4 w = __builtin_nontemporal_load((const lds_u32x4 *)(in + s * block + off));
    uint4 v;
    v.x = w.x;
    v.y = w.y;
    v.z = w.z;
    v.w = w.w;
    return v;
}

template <int KIND>
__device__ __forceinline__ void lds_pair(const uint4 *tile, int lane, uint32_t st[5]) {
    uint32_t X[32];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint4 v = tile[lane * LDS_ROW + i];
        X[4 * i] = v.x;
        X[4 * i + 1] = v.y;
        X[4 * i + 2] = v.z;
        X[4 * i + 3] = v.w;
    }
    Hash<KIND>::block(st, X);
    Hash<KIND>::block(st, X + 16);
}

template <int KIND>
__global__ __launch_bounds__(64) void leaf_lds_kernel(const uint8_t *__restrict__ in, uint64_t len, uint64_t block,
                                                      uint64_t n_leaves, uint8_t *__restrict__ out) {
    __shared__ uint4 tile[2][64 * LDS_ROW];
    const int lane = threadIdx.x;
    const uint64_t k0 = (uint64_t)blockIdx.x * 128, ka = k0 + lane, kb = k0 + 64 + lane;
    const bool act_a = ka < n_leaves, act_b = kb < n_leaves;
    const uint64_t na = act_a ? (len - ka * block < block ? len - ka * block : block) : 0;
    const uint64_t nb = act_b ? (len - kb * block < block ? len - kb * block : block) : 0;
    // Pairs of blocks that every active segment of the wave has.
    uint64_t m = act_a ? na >> 7 : ~0ull;
    if (act_b && (nb >> 7) < m) m = nb >> 7;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(m, off, 64);
        m = o < m ? o : m;
    }
    const uint64_t P = m / 2;  // group B runs pair i - P in step i
    const int piece = lane & 7, row0 = lane >> 3;
    uint4 RA[8], RB[8];
    uint32_t sa[5], sb[5];
    Hash<KIND>::init(sa);
    Hash<KIND>::init(sb);
    if (m > 0) {
#pragma unroll
        for (int j = 0; j < 8; j++) RA[j] = lds_piece(in, block, n_leaves, k0 + 8 * j + row0, piece * 16);
#pragma unroll
        for (int j = 0; j < 8; j++) tile[0][(8 * j + row0) * LDS_ROW + piece] = RA[j];
        if (P == 0) {
#pragma unroll
            for (int j = 0; j < 8; j++) RB[j] = lds_piece(in, block, n_leaves, k0 + 64 + 8 * j + row0, piece * 16);
#pragma unroll
            for (int j = 0; j < 8; j++) tile[1][(8 * j + row0) * LDS_ROW + piece] = RB[j];
        }
        __syncthreads();
    }
    for (uint64_t i = 0; i < m + P; i++) {
        const bool a_now = i < m, b_now = i >= P;
        const bool a_next = i + 1 < m, b_next = i + 1 >= P && i + 1 < m + P;
        // Next lines of both groups in flight while the current ones are
        // compressed.
        if (a_next) {
            const uint64_t off = (i + 1) * 128 + piece * 16;
#pragma unroll
            for (int j = 0; j < 8; j++) RA[j] = lds_piece(in, block, n_leaves, k0 + 8 * j + row0, off);
        }
        if (b_next) {
            const uint64_t off = (i + 1 - P) * 128 + piece * 16;
#pragma unroll
            for (int j = 0; j < 8; j++) RB[j] = lds_piece(in, block, n_leaves, k0 + 64 + 8 * j + row0, off);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (a_now) lds_pair<KIND>(tile[0], lane, sa);
        if (b_now) lds_pair<KIND>(tile[1], lane, sb);
        // The tile writes wait for the loads: keep them after the rounds
        // (the compiler would otherwise merge them into the load branches).
        asm volatile("" : "+v"(sa[0]), "+v"(sa[1]), "+v"(sa[2]), "+v"(sa[3]), "+v"(sb[0]), "+v"(sb[1]),
                     "+v"(sb[2]), "+v"(sb[3]) : : "memory");
        __syncthreads();  // every row read before the tiles are refilled
        if (a_next) {
#pragma unroll
            for (int j = 0; j < 8; j++) tile[0][(8 * j + row0) * LDS_ROW + piece] = RA[j];
        }
        if (b_next) {
#pragma unroll
            for (int j = 0; j < 8; j++) tile[1][(8 * j + row0) * LDS_ROW + piece] = RB[j];
        }
        __syncthreads();
    }
    const uint64_t done = m * 128;
    if (act_a) {
        hash_rest<KIND>(in + ka * block + done, na - done, na, in + len, sa);
        store_digest<KIND>(out + ka * (uint64_t)Hash<KIND>::DIGEST, sa);
    }
    if (act_b) {
        hash_rest<KIND>(in + kb * block + done, nb - done, nb, in + len, sb);
        store_digest<KIND>(out + kb * (uint64_t)Hash<KIND>::DIGEST, sb);
    }
}

// Both digests of every segment in one pass over the input.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void leaf_dual_kernel(
    const uint8_t *__restrict__ in, uint64_t len, uint64_t block, uint64_t n_leaves, uint8_t *__restrict__ out_md5,
    uint8_t *__restrict__ out_sha1) {
    uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_leaves) return;
    uint64_t start = k * block;
    uint64_t n = len - start < block ? len - start : block;
    uint32_t sm[5], ss[5];
    hash_range_dual(in + start, n, in + len, sm, ss);
    store_digest<KIND_MD5>(out_md5 + k * 16, sm);
    store_digest<KIND_SHA1>(out_sha1 + k * 20, ss);
}

// Segment ranges of at most LAUNCH_LANES segments: segments [k0, k1) of
// the whole are segments [0, k1 - k0) of in + k0 * block; every range but
// the last holds whole segments only, so its reads stay inside it.
template <class F>
static hipError_t by_ranges(const uint8_t *in, uint64_t len, uint64_t block, uint64_t n_leaves, F launch) {
    for (uint64_t k0 = 0; k0 < n_leaves; k0 += LAUNCH_LANES) {
        const uint64_t k1 = n_leaves - k0 > LAUNCH_LANES ? k0 + LAUNCH_LANES : n_leaves;
        const uint64_t off = k0 * block, sub = k1 < n_leaves ? (k1 - k0) * block : len - off;
        const hipError_t e = launch(in + off, sub, k0, k1 - k0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_leaves_dual(const uint8_t *in, uint64_t len, uint64_t block, uint64_t n_leaves,
                              uint8_t *out_md5, uint8_t *out_sha1, hipStream_t s) {
    if (n_leaves == 0) return hipSuccess;
    if (n_leaves > LAUNCH_LANES)
        return by_ranges(in, len, block, n_leaves, [&](const uint8_t *p, uint64_t l, uint64_t k0, uint64_t n) {
            return launch_leaves_dual(p, l, block, n, out_md5 + k0 * 16, out_sha1 + k0 * 20, s);
        });
    unsigned tpb = n_leaves < 256ull * 1024 ? 64u : 256u;
    uint64_t grid = (n_leaves + tpb - 1) / tpb;
    leaf_dual_kernel<<<dim3((unsigned)grid), dim3(tpb), 0, s>>>(in, len, block, n_leaves, out_md5, out_sha1);
    return hipGetLastError();
}

hipError_t launch_leaves(int kind, const uint8_t *in, uint64_t len, uint64_t block,
                         uint64_t n_leaves, uint8_t *out, hipStream_t s) {
    if (n_leaves == 0) return hipSuccess;
    if (n_leaves > LAUNCH_LANES) {
        const uint64_t d = kind == KIND_MD5 ? 16 : 20;
        return by_ranges(in, len, block, n_leaves, [&](const uint8_t *p, uint64_t l, uint64_t k0, uint64_t n) {
            return launch_leaves(kind, p, l, block, n, out + k0 * d, s);
        });
    }
    if (kind == KIND_MD5 && block >= 256 && n_leaves >= 64 * 1024) {
        // MD5 needs more bytes per op than HBM delivers with one line per
        // lane per load: read whole lines per instruction through LDS.
        const uint64_t grid = (n_leaves + 127) / 128;  // 128 segments per wave
        leaf_lds_kernel<KIND_MD5><<<dim3((unsigned)grid), dim3(64), 0, s>>>(in, len, block, n_leaves, out);
        return hipGetLastError();
    }
    // Few long segments: 64-lane workgroups spread the chains over more CUs.
    unsigned tpb = n_leaves < 256ull * 1024 ? 64u : 256u;
    uint64_t grid = (n_leaves + tpb - 1) / tpb;
    if (kind == KIND_MD5)
        leaf_kernel<KIND_MD5><<<dim3((unsigned)grid), dim3(tpb), 0, s>>>(in, len, block, n_leaves, out);
    else
        leaf_kernel<KIND_SHA1><<<dim3((unsigned)grid), dim3(tpb), 0, s>>>(in, len, block, n_leaves, out);
    return hipGetLastError();
}

hipError_t launch_hash_one(int kind, const uint8_t *in, uint64_t len, uint8_t *out, hipStream_t s) {
    // A single segment covering the whole range (block = max(len, 1)).
    uint64_t block = len ? len : 1;
    if (kind == KIND_MD5)
        leaf_kernel<KIND_MD5><<<dim3(1), dim3(64), 0, s>>>(in, len, block, 1, out);
    else
        leaf_kernel<KIND_SHA1><<<dim3(1), dim3(64), 0, s>>>(in, len, block, 1, out);
    return hipGetLastError();
}

}  // namespace hg
