// blockmap.hip -- the block-map of a content-addressable store (Sec. 3.2.1:
// written data is split into chunks, each chunk is identified by its
// digest, and only chunks whose digest the store does not hold yet are
// stored).  The map keeps the digest of every chunk stored so far on the
// device between writes: an open-addressing table of 32-bit slots (0 =
// empty, k + 1 = the k-th stored digest) over a digest array.
//
// A write of one version's chunks, in four passes:
//   bm_lookup   chunks whose digest is stored already are duplicates;
//   bm_insert   the others enter the table as this write's entries (tagged
//               slot values TMP | index + 1); for equal digests the slot keeps
//               the smallest chunk index (atomicMin);
//   bm_commit   the chunk a slot keeps is new: it gets a place in the digest
//               array; the others with that digest repeat an earlier chunk of
//               the same write and are duplicates;
//   bm_settle   the kept slots become stored entries (k + 1).
// So chunk i is a duplicate iff its digest was stored before the write or
// belongs to a chunk j < i of the same write -- the sequential store's rule.
#include "hg_device.hpp"
#include "hg_internal.hpp"

namespace hg {

constexpr uint32_t BM_TMP = 0x80000000u;

// state: 0 new (stored by this write), 1 repeats an earlier chunk of this
// write, 2 stored before.
template <int D>
__global__ __launch_bounds__(256) void bm_lookup(BlockMapView m, const uint8_t *__restrict__ dig, uint64_t n,
                                                 uint8_t *__restrict__ state) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint8_t *d = dig + i * D;
    uint64_t slot = dig_hash<D>(d) & m.slot_mask;
    uint8_t st = 0;
    for (uint64_t probe = 0; probe <= m.slot_mask; probe++) {
        const uint32_t v = m.table[slot];
        if (v == 0) break;
        if (!(v & BM_TMP) && dig_equal<D>(m.store + (uint64_t)(v - 1) * D, d)) {
            st = 2;
            break;
        }
        slot = (slot + 1) & m.slot_mask;
    }
    state[i] = st;
}

template <int D>
__global__ __launch_bounds__(256) void bm_insert(BlockMapView m, const uint8_t *__restrict__ dig, uint64_t n,
                                                 const uint8_t *__restrict__ state, uint32_t *__restrict__ slot_of) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || state[i] != 0) return;
    const uint8_t *d = dig + i * D;
    const uint32_t mine = BM_TMP | (uint32_t)(i + 1);
    uint64_t slot = dig_hash<D>(d) & m.slot_mask;
    for (uint64_t probe = 0; probe <= m.slot_mask; probe++) {
        uint32_t v = m.table[slot];
        if (v == 0) {
            v = atomicCAS(&m.table[slot], 0u, mine);
            if (v == 0) {
                slot_of[i] = (uint32_t)slot;
                return;
            }
        }
        // Stored entries differ from d (bm_lookup); entries of this write
        // with the same digest share one slot.
        if ((v & BM_TMP) && dig_equal<D>(dig + (uint64_t)((v & ~BM_TMP) - 1) * D, d)) {
            atomicMin(&m.table[slot], mine);
            slot_of[i] = (uint32_t)slot;
            return;
        }
        slot = (slot + 1) & m.slot_mask;
    }
}

template <int D>
__global__ __launch_bounds__(256) void bm_commit(BlockMapView m, const uint8_t *__restrict__ dig, uint64_t n,
                                                 uint8_t *__restrict__ state, const uint32_t *__restrict__ slot_of,
                                                 uint64_t *__restrict__ pos_of) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || state[i] != 0) return;
    const uint32_t v = m.table[slot_of[i]];
    if ((uint64_t)((v & ~BM_TMP) - 1) != i) {
        state[i] = 1;
        return;
    }
    const uint64_t p = atomicAdd(m.size, 1ull);
    __builtin_memcpy(m.store + p * D, dig + i * D, D);
    pos_of[i] = p;
}

__global__ __launch_bounds__(256) void bm_settle(BlockMapView m, uint64_t n, const uint8_t *__restrict__ state,
                                                 const uint32_t *__restrict__ slot_of,
                                                 const uint64_t *__restrict__ pos_of,
                                                 const uint64_t *__restrict__ len, int len_is_ends,
                                                 uint8_t *__restrict__ is_dup, unsigned long long *__restrict__ counters) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool dup = false;
    uint64_t bytes = 0;
    if (i < n) {
        const uint8_t st = state[i];
        if (st == 0) m.table[slot_of[i]] = (uint32_t)(pos_of[i] + 1);
        dup = st != 0;
        if (is_dup) is_dup[i] = dup ? 1 : 0;
        if (dup && len) bytes = len_is_ends ? len[i] - (i ? len[i - 1] : 0) : len[i];
    }
    const unsigned long long c = __builtin_popcountll(__ballot(dup));
    unsigned long long b = bytes;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) b += __shfl_xor(b, off, 64);
    if ((threadIdx.x & 63) == 0 && c) {
        atomicAdd(&counters[0], c);
        atomicAdd(&counters[1], b);
    }
}

hipError_t launch_blockmap_write(int kind, const BlockMapView &m, const uint8_t *dig, uint64_t n, const uint64_t *len,
                                 int len_is_ends, uint8_t *state, uint32_t *slot_of, uint64_t *pos_of,
                                 uint8_t *is_dup, unsigned long long *counters, hipStream_t s) {
    hipError_t e = launch_fill_u32((uint32_t *)counters, 4, 0, s);
    if (e != hipSuccess || n == 0) return e;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (kind == KIND_MD5) {
        bm_lookup<16><<<grid, 256, 0, s>>>(m, dig, n, state);
        bm_insert<16><<<grid, 256, 0, s>>>(m, dig, n, state, slot_of);
        bm_commit<16><<<grid, 256, 0, s>>>(m, dig, n, state, slot_of, pos_of);
    } else {
        bm_lookup<20><<<grid, 256, 0, s>>>(m, dig, n, state);
        bm_insert<20><<<grid, 256, 0, s>>>(m, dig, n, state, slot_of);
        bm_commit<20><<<grid, 256, 0, s>>>(m, dig, n, state, slot_of, pos_of);
    }
    bm_settle<<<grid, 256, 0, s>>>(m, n, state, slot_of, pos_of, len, len_is_ends, is_dup, counters);
    return hipGetLastError();
}

}  // namespace hg
