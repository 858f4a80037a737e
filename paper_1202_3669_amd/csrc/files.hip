// files.hip -- content-based chunking and direct hashing of many files at
// once (batch-oriented computation, paper Sec. 3.1 and Sec. 3.2.4).
//
// The files sit in one arena; every file is chunked on its own (windows,
// boundaries and chunks never cross a file edge).  The window scan runs over
// all files through a tile map and leaves the candidates of all files in one
// ascending array, file after file.  Then:
//   files_select   one wavefront per file applies the greedy boundary rule
//                  to that file's candidates (ballot: the first candidate end
//                  at or beyond last + max(min, 1); readlane moves `last`);
//                  a file has at most (its candidates + 1) chunks, so its
//                  ends go to slots starting at (first candidate + file);
//   files_scan     chunk counts become per-file chunk offsets and a total;
//   files_compact  one wavefront per file copies its ends to their final
//                  place and writes each chunk's absolute arena range for
//                  the digest pass.
// Direct hashing of every file reuses the batch kernels; files_jobs writes
// their job records on the device so that a captured graph can be replayed.
#include "hg_device.hpp"
#include "hg_internal.hpp"

namespace hg {

__device__ __forceinline__ void file_cand_range(const FilesChunk &fc, uint64_t total, uint32_t f, uint64_t &c0,
                                                uint64_t &c1) {
    const uint64_t t0 = fc.first_tile[f], t1 = fc.first_tile[f + 1];
    c0 = t0 < fc.n_tiles ? fc.tile_off[t0] : total;
    c1 = t1 < fc.n_tiles ? fc.tile_off[t1] : total;
}

// The builtin returns int: each half goes through uint32_t, so that a low
// word with bit 31 set is not sign-extended into the high word.
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    return ((uint64_t)hi << 32) | lo;
}

// One wavefront: the cuts of a block of length L from its ascending
// candidate starts cand[c0, c1) (each shifted by `add`), starting after a
// cut at `last0`, with the minimum step and a maximum chunk size maxc
// (0 = none; forced cuts, see hg_chunk).  From the previous cut `last`, a
// ballot finds the first candidate end e >= last + step below L; while it
// lies more than maxc past `last`, cuts are forced at last + maxc.  A run of
// f forced cuts ends when e comes within maxc (then e is the next cut) or
// falls below last + step (then later candidates are looked at), so f is
// known in closed form and the lanes write the run together.  With `final`
// the remaining forced cuts before L and the end L itself follow; without
// it the walk stops at the last cut it can decide below L.  Cut i is written
// as (cut - last0) to out[i] for i < cap; returns the number of cuts and
// leaves the last cut in *last_out.
__device__ uint64_t walk_cuts(const uint64_t *__restrict__ cand, uint64_t c0, uint64_t c1, uint64_t add,
                              uint32_t w, uint64_t L, uint64_t last0, uint64_t step, uint64_t maxc, bool final,
                              uint64_t *__restrict__ out, uint64_t cap, uint64_t *last_out) {
    const int lane = threadIdx.x & 63;
    uint64_t last = last0, m = 0;
    for (uint64_t base = c0; base < c1; base += 64) {
        const uint64_t j = base + lane;
        const bool valid = j < c1;
        const uint64_t e = valid ? cand[j] + add + w : ~0ull;
        const bool usable = valid && e < L;
        while (true) {
            const uint64_t thr = last + step;  // last < L and step <= L: no overflow
            const uint64_t elig = __ballot(usable && e >= thr);
            if (elig == 0) break;
            const uint64_t en = readlane64(e, __builtin_ctzll(elig));
            const uint64_t d = en - last;
            if (maxc && d > maxc) {
                const uint64_t fa = (d - 1) / maxc;         // until en - last <= maxc
                const uint64_t fb = (d - step) / maxc + 1;  // until en < last + step
                const uint64_t f = fa < fb ? fa : fb;
                for (uint64_t i = lane; i < f; i += 64)
                    if (m + i < cap) out[m + i] = last + (i + 1) * maxc - last0;
                m += f;
                last += f * maxc;
                continue;
            }
            if (lane == 0 && m < cap) out[m] = en - last0;
            m++;
            last = en;
        }
    }
    // Forced cuts before L: with `final` up to the end; otherwise only those
    // that lie below L (the bytes up to L are known).
    if (maxc && L > last && L - last > maxc) {
        const uint64_t f = (L - last - 1) / maxc;
        for (uint64_t i = lane; i < f; i += 64)
            if (m + i < cap) out[m + i] = last + (i + 1) * maxc - last0;
        m += f;
        last += f * maxc;
    }
    if (final && L > last0) {
        if (lane == 0 && m < cap) out[m] = L - last0;
        m++;
        last = L;
    }
    *last_out = last;
    return m;
}

__device__ __forceinline__ uint64_t walk_cuts_max(const uint64_t *__restrict__ cand, uint64_t c0, uint64_t c1,
                                                  uint32_t w, uint64_t L, uint64_t step, uint64_t maxc,
                                                  uint64_t *__restrict__ out, uint64_t cap) {
    uint64_t last;
    return walk_cuts(cand, c0, c1, 0, w, L, 0, step, maxc, true, out, cap, &last);
}

// Streaming: cuts of a carried buffer whose first chunk starts at last0,
// candidates at cand + add.  out_state[0] = number of cuts, [1] = last cut.
__global__ __launch_bounds__(64) void stream_walk_kernel(const uint64_t *__restrict__ cand,
                                                        const uint64_t *__restrict__ n_dev, uint64_t add, uint32_t w,
                                                        uint64_t L, uint64_t last0, uint64_t step, uint64_t maxc,
                                                        int final, uint64_t *__restrict__ out, uint64_t cap,
                                                        uint64_t *__restrict__ out_state) {
    uint64_t last;
    const uint64_t m = walk_cuts(cand, 0, *n_dev, add, w, L, last0, step, maxc, final != 0, out, cap, &last);
    if (threadIdx.x == 0) {
        out_state[0] = m;
        out_state[1] = last;
    }
}

__global__ __launch_bounds__(64) void select_max_kernel(const uint64_t *__restrict__ cand,
                                                       const uint64_t *__restrict__ n_dev, uint32_t w, uint64_t L,
                                                       uint64_t step, uint64_t maxc, uint64_t *__restrict__ ends,
                                                       uint64_t cap, uint64_t *__restrict__ n_chunks) {
    const uint64_t m = walk_cuts_max(cand, 0, *n_dev, w, L, step, maxc, ends, cap);
    if (threadIdx.x == 0) *n_chunks = m;
}

__global__ __launch_bounds__(64) void files_select(FilesChunk fc, uint32_t w, uint64_t step,
                                                  uint64_t *__restrict__ status) {
    const uint32_t f = blockIdx.x;
    const int lane = threadIdx.x;
    const uint64_t total = status[0];
    uint64_t c0, c1;
    file_cand_range(fc, total, f, c0, c1);
    if (c1 > fc.cap_cand) {
        // Candidates past the capacity were not stored: the result of this
        // run is incomplete, and says so.
        if (lane == 0) atomicOr((unsigned long long *)&status[2], 1ull);
        c1 = fc.cap_cand;
        if (c0 > c1) c0 = c1;
    }
    const uint64_t L = fc.len[f];
    uint64_t *out = fc.slots + c0 + f + (fc.extra ? fc.extra[f] : 0);
    if (fc.max_chunk) {
        const uint64_t m = walk_cuts_max(fc.cand, c0, c1, w, L, step, fc.max_chunk, out, ~0ull);
        if (lane == 0) fc.cnt[f] = (uint32_t)m;
        return;
    }
    uint64_t last = 0, m = 0;
    for (uint64_t base = c0; base < c1; base += 64) {
        const uint64_t j = base + lane;
        const bool valid = j < c1;
        const uint64_t e = valid ? fc.cand[j] + w : ~0ull;
        const bool usable = valid && e < L;
        uint64_t sel = 0;
        while (true) {
            const uint64_t thr = last + step < last ? ~0ull : last + step;
            const uint64_t elig = __ballot(usable && e >= thr);
            if (elig == 0) break;
            const int l = __builtin_ctzll(elig);
            last = readlane64(e, l);
            sel |= 1ull << l;
        }
        if ((sel >> lane) & 1ull) out[m + __builtin_popcountll(sel & ((1ull << lane) - 1ull))] = e;
        m += __builtin_popcountll(sel);
    }
    if (lane == 0) {
        if (L > 0) out[m++] = L;
        fc.cnt[f] = (uint32_t)m;
    }
}

// One workgroup: chunk offsets per file and the total.
__global__ __launch_bounds__(1024) void files_scan(const uint32_t *__restrict__ cnt, uint32_t n,
                                                   uint64_t *__restrict__ chunk_off, uint64_t *__restrict__ status) {
    __shared__ unsigned long long v[1024];
    const uint32_t t = threadIdx.x;
    unsigned long long carry = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += 1024) {
        const unsigned long long x = c0 + t < n ? cnt[c0 + t] : 0;
        v[t] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const unsigned long long y = t >= (uint32_t)off ? v[t - off] : 0;
            __syncthreads();
            v[t] += y;
            __syncthreads();
        }
        if (c0 + t < n) chunk_off[c0 + t] = carry + v[t] - x;
        carry += v[1023];
        __syncthreads();
    }
    if (t == 0) {
        chunk_off[n] = carry;
        status[1] = carry;
    }
}

__global__ __launch_bounds__(64) void files_compact(FilesChunk fc, const uint64_t *__restrict__ chunk_off,
                                                   uint64_t *__restrict__ chunk_ends, uint64_t max_chunks,
                                                   const uint64_t *__restrict__ status) {
    const uint32_t f = blockIdx.x;
    const uint64_t total = status[0];
    uint64_t c0, c1;
    file_cand_range(fc, total, f, c0, c1);
    if (c0 > fc.cap_cand) c0 = fc.cap_cand;
    const uint64_t *src = fc.slots + c0 + f + (fc.extra ? fc.extra[f] : 0);
    const uint64_t o = chunk_off[f], n = fc.cnt[f], base = fc.off[f];
    for (uint64_t j = threadIdx.x; j < n; j += 64) {
        const uint64_t e = src[j], b = j ? src[j - 1] : 0;
        if (o + j < max_chunks) {
            chunk_ends[o + j] = e;
            fc.seg_start[o + j] = base + b;
            fc.seg_end[o + j] = base + e;
        }
    }
}

__global__ __launch_bounds__(256) void files_jobs(const uint8_t *arena, const uint64_t *__restrict__ off,
                                                  const uint64_t *__restrict__ len,
                                                  const uint64_t *__restrict__ leaf_first,
                                                  const uint32_t *__restrict__ order, uint32_t n, uint64_t block,
                                                  int digest, uint8_t *leaf_out, uint8_t *roots,
                                                  hg_block_job *__restrict__ jobs) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t f = order[i];
    const int d = digest == HG_SHA1 ? 20 : 16;
    hg_block_job j;
    j.in = arena + off[f];
    j.len = len[f];
    j.block_size = block;
    j.leaf_out = leaf_out + leaf_first[f] * d;
    j.root_out = roots ? roots + (uint64_t)f * d : nullptr;
    j.digest = digest;
    j.reserved = 0;
    jobs[i] = j;
}

hipError_t launch_files_select(const FilesChunk &fc, uint32_t w, uint64_t min_chunk, uint64_t *status,
                               hipStream_t s) {
    if (fc.n_files == 0) return hipSuccess;
    files_select<<<fc.n_files, 64, 0, s>>>(fc, w, min_chunk ? min_chunk : 1, status);
    return hipGetLastError();
}

hipError_t launch_chunk_select_max(const uint64_t *starts, const uint64_t *n_starts_dev, uint32_t w, uint64_t len,
                                   uint64_t min_chunk, uint64_t max_chunk, uint64_t *ends, uint64_t cap,
                                   uint64_t *n_chunks_dev, hipStream_t s) {
    select_max_kernel<<<1, 64, 0, s>>>(starts, n_starts_dev, w, len, min_chunk ? min_chunk : 1, max_chunk, ends, cap,
                                       n_chunks_dev);
    return hipGetLastError();
}

// Streaming without a maximum: the candidates whose cut can never be taken
// after last0 (end below last0 + step) form a prefix; the rest, shifted so
// that last0 becomes 0, go to the parallel boundary decision.
__global__ void stream_drop_kernel(const uint64_t *__restrict__ cand, const uint64_t *__restrict__ n_dev, uint64_t add,
                                   uint32_t w, uint64_t limit, uint64_t *__restrict__ out_words) {
    // One lane: binary search for the first candidate end >= limit.
    const uint64_t n = *n_dev;
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) / 2;
        if (cand[mid] + add + w < limit) lo = mid + 1;
        else hi = mid;
    }
    out_words[0] = lo;      // dropped
    out_words[1] = n - lo;  // kept
}

__global__ void stream_shift_kernel(const uint64_t *__restrict__ cand, const uint64_t *__restrict__ words,
                                    uint64_t add, uint64_t last0, uint64_t *__restrict__ out) {
    const uint64_t k = words[0], m = words[1];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = cand[k + i] + add - last0;
}

// The decided part of a parallel selection: the chunk count minus the
// provisional final chunk (unless final), and the last decided end.
__global__ void stream_tail_kernel(const uint64_t *__restrict__ n_chunks, const uint64_t *__restrict__ ends, int final,
                                   uint64_t last0, uint64_t *__restrict__ state) {
    const uint64_t nc = *n_chunks;
    const uint64_t k = final ? nc : (nc ? nc - 1 : 0);
    state[0] = k;
    state[1] = last0 + (k ? ends[k - 1] : 0);
}

hipError_t launch_stream_drop(const uint64_t *cand, const uint64_t *n_dev, uint64_t add, uint32_t w, uint64_t limit,
                              uint64_t *words, hipStream_t s) {
    stream_drop_kernel<<<1, 1, 0, s>>>(cand, n_dev, add, w, limit, words);
    return hipGetLastError();
}

hipError_t launch_stream_shift(const uint64_t *cand, const uint64_t *words, uint64_t max_m, uint64_t add,
                               uint64_t last0, uint64_t *out, hipStream_t s) {
    if (max_m == 0) return hipSuccess;
    uint64_t blocks = (max_m + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    stream_shift_kernel<<<(unsigned)blocks, 256, 0, s>>>(cand, words, add, last0, out);
    return hipGetLastError();
}

hipError_t launch_stream_tail(const uint64_t *n_chunks, const uint64_t *ends, bool final, uint64_t last0,
                              uint64_t *state, hipStream_t s) {
    stream_tail_kernel<<<1, 1, 0, s>>>(n_chunks, ends, final ? 1 : 0, last0, state);
    return hipGetLastError();
}

hipError_t launch_stream_walk(const uint64_t *cand, const uint64_t *n_dev, uint64_t add, uint32_t w, uint64_t len,
                              uint64_t last0, uint64_t min_chunk, uint64_t max_chunk, bool final, uint64_t *ends,
                              uint64_t cap, uint64_t *state, hipStream_t s) {
    stream_walk_kernel<<<1, 64, 0, s>>>(cand, n_dev, add, w, len, last0, min_chunk ? min_chunk : 1, max_chunk,
                                        final ? 1 : 0, ends, cap, state);
    return hipGetLastError();
}

hipError_t launch_files_compact(const FilesChunk &fc, uint64_t *chunk_off, uint64_t *chunk_ends,
                                uint64_t max_chunks, uint64_t *status, hipStream_t s) {
    files_scan<<<1, 1024, 0, s>>>(fc.cnt, fc.n_files, chunk_off, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || fc.n_files == 0) return e;
    files_compact<<<fc.n_files, 64, 0, s>>>(fc, chunk_off, chunk_ends, max_chunks, status);
    return hipGetLastError();
}

hipError_t launch_files_jobs(const uint8_t *arena, const uint64_t *off, const uint64_t *len,
                             const uint64_t *leaf_first, const uint32_t *order, uint32_t n_files,
                             uint64_t block, int digest, uint8_t *leaf_out, uint8_t *roots, hg_block_job *jobs,
                             hipStream_t s) {
    if (n_files == 0) return hipSuccess;
    files_jobs<<<(n_files + 255) / 256, 256, 0, s>>>(arena, off, len, leaf_first, order, n_files, block, digest,
                                                     leaf_out, roots, jobs);
    return hipGetLastError();
}

}  // namespace hg
