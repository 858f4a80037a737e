// probe.hip -- microbenchmarks of the two ceilings the hashing kernels are
// measured against: the int32 VALU issue rate and the HBM read rate.  They
// give the achievable peaks beside the data-sheet ones (int32 VALU 39.32
// Tops/s from 256 CUs x 4 SIMD16 x 2.4 GHz; HBM3E 8 TB/s).
#include "hg_device.hpp"
#include "hg_internal.hpp"

namespace hg {

constexpr int PROBE_CHAINS = 8;

// Each lane runs PROBE_CHAINS independent chains of a rotate, an add and a
// three-input logic op (the instruction mix of the hash rounds), so issue,
// not latency, bounds the rate.  3 ops per chain per step.
__global__ __launch_bounds__(256) void alu_probe_kernel(uint32_t seed, uint32_t steps, uint32_t *out) {
    uint32_t x[PROBE_CHAINS];
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; c++) x[c] = seed ^ (t * 0x9e3779b9u) ^ (uint32_t)c;
    const uint32_t y = seed * 3u + 1u, z = seed ^ 0x5bd1e995u;
    for (uint32_t i = 0; i < steps; i++) {
#pragma unroll 16
        for (int r = 0; r < 16; r++) {
#pragma unroll
            for (int c = 0; c < PROBE_CHAINS; c++) {
                x[c] = __builtin_amdgcn_alignbit(x[c], x[c], 25);
                x[c] = x[c] + y;
                x[c] = bop3<TT_XOR3>(x[c], z, y);
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; c++) acc ^= x[c];
    if (acc == seed) out[0] = t;  // keeps the chains live; practically never taken
}

// Grid-stride 16-byte loads over the buffer, XOR-folded so that nothing is
// dropped.
__global__ __launch_bounds__(256) void read_probe_kernel(const uint4 *__restrict__ p, uint64_t n16, uint32_t *out) {
    uint32_t acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const uint4 v = p[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x12345678u) out[0] = acc;
}

uint64_t alu_probe_ops(uint32_t blocks, uint32_t steps) {
    return (uint64_t)blocks * 256 * steps * 16 * PROBE_CHAINS * 3;
}

hipError_t launch_alu_probe(uint32_t blocks, uint32_t steps, uint32_t *out, hipStream_t s) {
    alu_probe_kernel<<<blocks, 256, 0, s>>>(0x2545f491u, steps, out);
    return hipGetLastError();
}

hipError_t launch_read_probe(const uint8_t *p, uint64_t len, uint32_t *out, hipStream_t s) {
    const uint64_t n16 = len / 16;
    if (n16 == 0) return hipSuccess;
    // 16 workgroups of 256 lanes per CU keep enough loads in flight.
    read_probe_kernel<<<256 * 16, 256, 0, s>>>((const uint4 *)p, n16, out);
    return hipGetLastError();
}

}  // namespace hg
