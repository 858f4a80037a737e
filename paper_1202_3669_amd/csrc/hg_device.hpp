// hg_device.hpp -- MD5 and SHA-1 compression functions for gfx950 (CDNA4).
//
// The two sequential Merkle-Damgard hashes that HashGPU uses as building
// blocks (paper Sec. 3.2.2; MD5 per RFC 1321, SHA-1 per FIPS 180-4).  State
// and message words stay in VGPRs; every boolean round function is one
// v_bitop3_b32 (a 3-input truth table), rotates lower to v_alignbit_b32 and
// the sums to v_add3_u32, so an MD5 step is five VALU ops and a SHA-1 round
// five plus three for its message schedule.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hg_rounds.hpp"

namespace hg {

template <uint32_t TT>
__device__ __forceinline__ uint32_t bop3(uint32_t x, uint32_t y, uint32_t z) {
    return __builtin_amdgcn_bitop3_b32(x, y, z, TT);
}
__device__ __forceinline__ uint32_t rotl(uint32_t x, uint32_t s) {
    return __builtin_rotateleft32(x, s);
}
__device__ __forceinline__ uint32_t bswap(uint32_t x) { return __builtin_bswap32(x); }

// Full compression of one 64-byte block (16 little-endian words).
__device__ __forceinline__ void md5_compress(uint32_t st[4], const uint32_t X[16]) {
    uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
    HG_MD5_ROUNDS_0_60(X, a, b, c, d)
    HG_MD5_ROUNDS_61_63(X, a, b, c, d)
    st[0] += a; st[1] += b; st[2] += c; st[3] += d;
}

// First digest word only.  Step 60 is the last step that writes register a,
// so the final A word is IV + a after step 60; steps 61..63 only feed B, C
// and D and are skipped.
__device__ __forceinline__ uint32_t md5_compress_word0(const uint32_t st[4], const uint32_t X[16]) {
    uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
    HG_MD5_ROUNDS_0_60(X, a, b, c, d)
    return st[0] + a;
}

// -------------------------------------------------------------- SHA-1 ----
// W holds the 16 big-endian message words and is overwritten by the schedule.
__device__ __forceinline__ void sha1_compress(uint32_t H[5], uint32_t W[16]) {
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4];
    HG_SHA1_5(TT_SEL, SHA1_K0, W, 0, HG_SHA1_WIN)
    HG_SHA1_5(TT_SEL, SHA1_K0, W, 5, HG_SHA1_WIN)
    HG_SHA1_5(TT_SEL, SHA1_K0, W, 10, HG_SHA1_WIN)
    HG_SHA1_R(TT_SEL, SHA1_K0, a, b, c, d, e, W[15])
    HG_SHA1_R(TT_SEL, SHA1_K0, e, a, b, c, d, HG_SHA1_W(W, 16))
    HG_SHA1_R(TT_SEL, SHA1_K0, d, e, a, b, c, HG_SHA1_W(W, 17))
    HG_SHA1_R(TT_SEL, SHA1_K0, c, d, e, a, b, HG_SHA1_W(W, 18))
    HG_SHA1_R(TT_SEL, SHA1_K0, b, c, d, e, a, HG_SHA1_W(W, 19))
    HG_SHA1_5(TT_XOR3, SHA1_K1, W, 20, HG_SHA1_W)
    HG_SHA1_5(TT_XOR3, SHA1_K1, W, 25, HG_SHA1_W)
    HG_SHA1_5(TT_XOR3, SHA1_K1, W, 30, HG_SHA1_W)
    HG_SHA1_5(TT_XOR3, SHA1_K1, W, 35, HG_SHA1_W)
    HG_SHA1_5(TT_MAJ, SHA1_K2, W, 40, HG_SHA1_W)
    HG_SHA1_5(TT_MAJ, SHA1_K2, W, 45, HG_SHA1_W)
    HG_SHA1_5(TT_MAJ, SHA1_K2, W, 50, HG_SHA1_W)
    HG_SHA1_5(TT_MAJ, SHA1_K2, W, 55, HG_SHA1_W)
    HG_SHA1_5(TT_XOR3, SHA1_K3, W, 60, HG_SHA1_W)
    HG_SHA1_5(TT_XOR3, SHA1_K3, W, 65, HG_SHA1_W)
    HG_SHA1_5(TT_XOR3, SHA1_K3, W, 70, HG_SHA1_W)
    HG_SHA1_5(TT_XOR3, SHA1_K3, W, 75, HG_SHA1_W)
    H[0] += a; H[1] += b; H[2] += c; H[3] += d; H[4] += e;
}

// ------------------------------------------------------ digest kinds ----
enum Kind : int { KIND_MD5 = 0, KIND_SHA1 = 1 };

template <int KIND> struct Hash;

template <> struct Hash<KIND_MD5> {
    static constexpr int NWORDS = 4;
    static constexpr int DIGEST = 16;
    static constexpr bool BIG_ENDIAN_WORDS = false;
    __device__ static __forceinline__ void init(uint32_t st[5]) {
        st[0] = MD5_IV0; st[1] = MD5_IV1; st[2] = MD5_IV2; st[3] = MD5_IV3; st[4] = 0;
    }
    // X: 16 message words as loaded little-endian from memory.
    __device__ static __forceinline__ void block(uint32_t st[5], uint32_t X[16]) {
        md5_compress(st, X);
    }
    // Little-endian value of digest bytes 0..3.
    __device__ static __forceinline__ uint32_t word0(const uint32_t st[5]) { return st[0]; }
    // Digest word j as it is stored (little-endian bytes).
    __device__ static __forceinline__ uint32_t out_word(const uint32_t st[5], int j) { return st[j]; }
    __device__ static __forceinline__ void length_words(uint32_t X[16], uint64_t bits) {
        X[14] = (uint32_t)bits; X[15] = (uint32_t)(bits >> 32);
    }
};

template <> struct Hash<KIND_SHA1> {
    static constexpr int NWORDS = 5;
    static constexpr int DIGEST = 20;
    static constexpr bool BIG_ENDIAN_WORDS = true;
    __device__ static __forceinline__ void init(uint32_t st[5]) {
        st[0] = MD5_IV0; st[1] = MD5_IV1; st[2] = MD5_IV2; st[3] = MD5_IV3; st[4] = SHA1_IV4;
    }
    // X: 16 words as loaded little-endian; they are byte-swapped here.
    __device__ static __forceinline__ void block(uint32_t st[5], uint32_t X[16]) {
#pragma unroll
        for (int j = 0; j < 16; j++) X[j] = bswap(X[j]);
        sha1_compress(st, X);
    }
    __device__ static __forceinline__ uint32_t word0(const uint32_t st[5]) { return bswap(st[0]); }
    __device__ static __forceinline__ uint32_t out_word(const uint32_t st[5], int j) { return bswap(st[j]); }
    // Length goes big-endian; X is still in load (little-endian) order here,
    // so the words are pre-swapped to come out right after block()'s bswap.
    __device__ static __forceinline__ void length_words(uint32_t X[16], uint64_t bits) {
        X[14] = bswap((uint32_t)(bits >> 32)); X[15] = bswap((uint32_t)bits);
    }
};

// ------------------------------------------------ message tail helpers ----
// Little-endian byte mask of the low n bytes of a word (n in 0..4).
__device__ __forceinline__ uint32_t low_bytes_mask(int n) {
    return n >= 4 ? 0xffffffffu : ((1u << (8 * n)) - 1u);
}

// Finish a message whose last `rem` (< 64) bytes are in X (little-endian
// load order, bytes at and beyond `rem` arbitrary): append 0x80, zero-fill,
// append the bit length, and compress one or two blocks.
template <int KIND>
__device__ __forceinline__ void finish_tail(uint32_t st[5], uint32_t X[16], int rem, uint64_t total_len) {
#pragma unroll
    for (int j = 0; j < 16; j++) {
        int valid = rem - 4 * j;
        valid = valid < 0 ? 0 : (valid > 4 ? 4 : valid);
        uint32_t w = X[j] & low_bytes_mask(valid);
        if (j == (rem >> 2)) w |= 0x80u << (8 * (rem & 3));
        X[j] = w;
    }
    uint64_t bits = total_len * 8u;
    if (rem < 56) {
        Hash<KIND>::length_words(X, bits);
        Hash<KIND>::block(st, X);
    } else {
        Hash<KIND>::block(st, X);
#pragma unroll
        for (int j = 0; j < 16; j++) X[j] = 0;
        Hash<KIND>::length_words(X, bits);
        Hash<KIND>::block(st, X);
    }
}

// Loads bytes p[0..n) (n < 64) into X in little-endian word order; bytes
// beyond n are zero.  Byte loads only, so nothing past p + n is touched.
__device__ __forceinline__ void load_partial(const uint8_t *p, int n, uint32_t X[16]) {
#pragma unroll
    for (int j = 0; j < 16; j++) {
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            int idx = 4 * j + b;
            if (idx < n) w |= (uint32_t)p[idx] << (8 * b);
        }
        X[j] = w;
    }
}

// 64 bytes from p into X (little-endian words); p may have any alignment.
__device__ __forceinline__ void load_block(const uint8_t *p, uint32_t X[16]) {
    __builtin_memcpy(X, p, 64);
}

// Tail of a message: the last n (< 64) bytes at p.  When a whole 64-byte
// block starting at p lies before buf_end it is loaded (one vector load; the
// caller masks what lies beyond n); otherwise the bytes are read one at a
// time so that nothing at or past buf_end is touched.
__device__ __forceinline__ void load_tail(const uint8_t *p, int n, const uint8_t *buf_end,
                                          uint32_t X[16]) {
    if (n == 0) {
        // Nothing to read (a message that ends on a block boundary).
#pragma unroll
        for (int j = 0; j < 16; j++) X[j] = 0;
    } else if (p + 64 <= buf_end) {
        load_block(p, X);
    } else {
        load_partial(p, n, X);
    }
}

// 128 bytes (two blocks) from p into X; p may have any alignment.
__device__ __forceinline__ void load_pair(const uint8_t *p, uint32_t X[32]) {
    __builtin_memcpy(X, p, 128);
}

// Hash the n bytes at p with one lane (p: any alignment; buf_end bounds the
// readable buffer); hash_rest continues a message of `total` bytes whose
// `rest` last bytes start at p (the state holds everything before).  Bytes
// are read in pairs of blocks, i.e. whole 128-byte
// lines for aligned input: with one lane per segment, the lanes of a wave
// read 64 different lines at a time, and a line read in two halves at
// different times is easily evicted from L2 in between and fetched twice.
// The loop double-buffers: pair q+1 is in flight while pair q is compressed.
template <int KIND>
__device__ __forceinline__ void hash_rest(const uint8_t *p, uint64_t rest, uint64_t total, const uint8_t *buf_end,
                                          uint32_t st[5]) {
    const uint64_t full = rest >> 6, pairs = full >> 1;
    uint32_t X[32], Y[32];
    uint64_t q = 0;
    if (pairs > 0) load_pair(p, X);
    while (q + 1 < pairs) {
        load_pair(p + ((q + 1) << 7), Y);
        // Keep the loads ahead of the rounds: left alone, the scheduler sinks
        // them next to their first use to save registers, and their latency
        // is then exposed.
        __builtin_amdgcn_sched_barrier(0);
        Hash<KIND>::block(st, X);
        Hash<KIND>::block(st, X + 16);
        // Unconditional prefetch (clamped to the last pair) keeps the loop
        // free of branches and register copies.
        const uint64_t nq = q + 2 < pairs ? q + 2 : pairs - 1;
        load_pair(p + (nq << 7), X);
        __builtin_amdgcn_sched_barrier(0);
        Hash<KIND>::block(st, Y);
        Hash<KIND>::block(st, Y + 16);
        q += 2;
    }
    if (q < pairs) {
        Hash<KIND>::block(st, X);
        Hash<KIND>::block(st, X + 16);
    }
    if (full & 1) {
        load_block(p + ((full - 1) << 6), X);
        Hash<KIND>::block(st, X);
    }
    const int rem = (int)(rest & 63);
    load_tail(p + (full << 6), rem, buf_end, X);
    finish_tail<KIND>(st, X, rem, total);
}

template <int KIND>
__device__ __forceinline__ void hash_range(const uint8_t *p, uint64_t n, const uint8_t *buf_end,
                                           uint32_t st[5]) {
    Hash<KIND>::init(st);
    hash_rest<KIND>(p, n, n, buf_end, st);
}

// MD5 and SHA-1 of the same n bytes in one pass (each block is read once
// and compressed by both; SHA-1 overwrites the block's words, so MD5 goes
// first).
__device__ __forceinline__ void dual_block(uint32_t sm[5], uint32_t ss[5], uint32_t X[16]) {
    Hash<KIND_MD5>::block(sm, X);
    Hash<KIND_SHA1>::block(ss, X);
}

__device__ __forceinline__ void hash_range_dual(const uint8_t *p, uint64_t n, const uint8_t *buf_end,
                                                uint32_t sm[5], uint32_t ss[5]) {
    Hash<KIND_MD5>::init(sm);
    Hash<KIND_SHA1>::init(ss);
    const uint64_t full = n >> 6, pairs = full >> 1;
    uint32_t X[32], Y[32];
    uint64_t q = 0;
    if (pairs > 0) load_pair(p, X);
    while (q + 1 < pairs) {
        load_pair(p + ((q + 1) << 7), Y);
        __builtin_amdgcn_sched_barrier(0);
        dual_block(sm, ss, X);
        dual_block(sm, ss, X + 16);
        const uint64_t nq = q + 2 < pairs ? q + 2 : pairs - 1;
        load_pair(p + (nq << 7), X);
        __builtin_amdgcn_sched_barrier(0);
        dual_block(sm, ss, Y);
        dual_block(sm, ss, Y + 16);
        q += 2;
    }
    if (q < pairs) {
        dual_block(sm, ss, X);
        dual_block(sm, ss, X + 16);
    }
    if (full & 1) {
        load_block(p + ((full - 1) << 6), X);
        dual_block(sm, ss, X);
    }
    const int rem = (int)(n & 63);
    load_tail(p + (full << 6), rem, buf_end, X);
    uint32_t T[16];
#pragma unroll
    for (int j = 0; j < 16; j++) T[j] = X[j];
    finish_tail<KIND_MD5>(sm, T, rem, n);
    finish_tail<KIND_SHA1>(ss, X, rem, n);
}

// Digests are uniformly distributed, so their first 8 bytes serve as a hash
// table key directly.
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

// Store a digest at `out` (any alignment).
template <int KIND>
__device__ __forceinline__ void store_digest(uint8_t *out, const uint32_t st[5]) {
    uint32_t w[5];
#pragma unroll
    for (int j = 0; j < Hash<KIND>::NWORDS; j++) w[j] = Hash<KIND>::out_word(st, j);
    __builtin_memcpy(out, w, Hash<KIND>::DIGEST);
}

}  // namespace hg
