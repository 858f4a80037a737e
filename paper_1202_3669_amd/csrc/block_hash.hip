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

hipError_t launch_leaves_dual(const uint8_t *in, uint64_t len, uint64_t block, uint64_t n_leaves,
                              uint8_t *out_md5, uint8_t *out_sha1, hipStream_t s) {
    if (n_leaves == 0) return hipSuccess;
    unsigned tpb = n_leaves < 256ull * 1024 ? 64u : 256u;
    uint64_t grid = (n_leaves + tpb - 1) / tpb;
    leaf_dual_kernel<<<dim3((unsigned)grid), dim3(tpb), 0, s>>>(in, len, block, n_leaves, out_md5, out_sha1);
    return hipGetLastError();
}

hipError_t launch_leaves(int kind, const uint8_t *in, uint64_t len, uint64_t block,
                         uint64_t n_leaves, uint8_t *out, hipStream_t s) {
    if (n_leaves == 0) return hipSuccess;
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
