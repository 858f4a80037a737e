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

namespace hg {

// Truth tables for v_bitop3_b32(x, y, z): bit i of the table is f(xi, yi, zi)
// where the three inputs enumerate as x = 0xF0, y = 0xCC, z = 0xAA.
constexpr uint32_t TX = 0xF0, TY = 0xCC, TZ = 0xAA;
constexpr uint32_t TT_SEL = ((TX & TY) | (~TX & TZ)) & 0xFF;          // x ? y : z  (MD5 F, SHA-1 Ch)
constexpr uint32_t TT_SELZ = ((TX & TZ) | (TY & ~TZ)) & 0xFF;         // z ? x : y  (MD5 G)
constexpr uint32_t TT_XOR3 = (TX ^ TY ^ TZ) & 0xFF;                   // MD5 H, SHA-1 Parity
constexpr uint32_t TT_MD5I = (TY ^ (TX | (~TZ & 0xFF))) & 0xFF;       // y ^ (x | ~z)  (MD5 I)
constexpr uint32_t TT_MAJ = ((TX & TY) | (TX & TZ) | (TY & TZ)) & 0xFF; // SHA-1 Maj

template <uint32_t TT>
__device__ __forceinline__ uint32_t bop3(uint32_t x, uint32_t y, uint32_t z) {
    return __builtin_amdgcn_bitop3_b32(x, y, z, TT);
}
__device__ __forceinline__ uint32_t rotl(uint32_t x, uint32_t s) {
    return __builtin_rotateleft32(x, s);
}
__device__ __forceinline__ uint32_t bswap(uint32_t x) { return __builtin_bswap32(x); }

constexpr uint32_t MD5_IV0 = 0x67452301u, MD5_IV1 = 0xefcdab89u, MD5_IV2 = 0x98badcfeu,
                   MD5_IV3 = 0x10325476u;
constexpr uint32_t SHA1_IV4 = 0xc3d2e1f0u;

// ---------------------------------------------------------------- MD5 ----
// One step: a = b + rotl(a + f(b, c, d) + X[k] + T[i], s).
#define HG_MD5_STEP(TT, a, b, c, d, x, t, s) \
    a = b + rotl(a + bop3<TT>(b, c, d) + ((x) + (t)), s)

// The 64 steps in RFC 1321 order (message word index, sine constant,
// rotation).  X is an indexable expression (array or macro argument).
#define HG_MD5_ROUNDS_0_60(X, a, b, c, d)                                   \
    HG_MD5_STEP(TT_SEL, a, b, c, d, X[0], 0xd76aa478u, 7);                  \
    HG_MD5_STEP(TT_SEL, d, a, b, c, X[1], 0xe8c7b756u, 12);                 \
    HG_MD5_STEP(TT_SEL, c, d, a, b, X[2], 0x242070dbu, 17);                 \
    HG_MD5_STEP(TT_SEL, b, c, d, a, X[3], 0xc1bdceeeu, 22);                 \
    HG_MD5_STEP(TT_SEL, a, b, c, d, X[4], 0xf57c0fafu, 7);                  \
    HG_MD5_STEP(TT_SEL, d, a, b, c, X[5], 0x4787c62au, 12);                 \
    HG_MD5_STEP(TT_SEL, c, d, a, b, X[6], 0xa8304613u, 17);                 \
    HG_MD5_STEP(TT_SEL, b, c, d, a, X[7], 0xfd469501u, 22);                 \
    HG_MD5_STEP(TT_SEL, a, b, c, d, X[8], 0x698098d8u, 7);                  \
    HG_MD5_STEP(TT_SEL, d, a, b, c, X[9], 0x8b44f7afu, 12);                 \
    HG_MD5_STEP(TT_SEL, c, d, a, b, X[10], 0xffff5bb1u, 17);                \
    HG_MD5_STEP(TT_SEL, b, c, d, a, X[11], 0x895cd7beu, 22);                \
    HG_MD5_STEP(TT_SEL, a, b, c, d, X[12], 0x6b901122u, 7);                 \
    HG_MD5_STEP(TT_SEL, d, a, b, c, X[13], 0xfd987193u, 12);                \
    HG_MD5_STEP(TT_SEL, c, d, a, b, X[14], 0xa679438eu, 17);                \
    HG_MD5_STEP(TT_SEL, b, c, d, a, X[15], 0x49b40821u, 22);                \
    HG_MD5_STEP(TT_SELZ, a, b, c, d, X[1], 0xf61e2562u, 5);                 \
    HG_MD5_STEP(TT_SELZ, d, a, b, c, X[6], 0xc040b340u, 9);                 \
    HG_MD5_STEP(TT_SELZ, c, d, a, b, X[11], 0x265e5a51u, 14);               \
    HG_MD5_STEP(TT_SELZ, b, c, d, a, X[0], 0xe9b6c7aau, 20);                \
    HG_MD5_STEP(TT_SELZ, a, b, c, d, X[5], 0xd62f105du, 5);                 \
    HG_MD5_STEP(TT_SELZ, d, a, b, c, X[10], 0x02441453u, 9);                \
    HG_MD5_STEP(TT_SELZ, c, d, a, b, X[15], 0xd8a1e681u, 14);               \
    HG_MD5_STEP(TT_SELZ, b, c, d, a, X[4], 0xe7d3fbc8u, 20);                \
    HG_MD5_STEP(TT_SELZ, a, b, c, d, X[9], 0x21e1cde6u, 5);                 \
    HG_MD5_STEP(TT_SELZ, d, a, b, c, X[14], 0xc33707d6u, 9);                \
    HG_MD5_STEP(TT_SELZ, c, d, a, b, X[3], 0xf4d50d87u, 14);                \
    HG_MD5_STEP(TT_SELZ, b, c, d, a, X[8], 0x455a14edu, 20);                \
    HG_MD5_STEP(TT_SELZ, a, b, c, d, X[13], 0xa9e3e905u, 5);                \
    HG_MD5_STEP(TT_SELZ, d, a, b, c, X[2], 0xfcefa3f8u, 9);                 \
    HG_MD5_STEP(TT_SELZ, c, d, a, b, X[7], 0x676f02d9u, 14);                \
    HG_MD5_STEP(TT_SELZ, b, c, d, a, X[12], 0x8d2a4c8au, 20);               \
    HG_MD5_STEP(TT_XOR3, a, b, c, d, X[5], 0xfffa3942u, 4);                 \
    HG_MD5_STEP(TT_XOR3, d, a, b, c, X[8], 0x8771f681u, 11);                \
    HG_MD5_STEP(TT_XOR3, c, d, a, b, X[11], 0x6d9d6122u, 16);               \
    HG_MD5_STEP(TT_XOR3, b, c, d, a, X[14], 0xfde5380cu, 23);               \
    HG_MD5_STEP(TT_XOR3, a, b, c, d, X[1], 0xa4beea44u, 4);                 \
    HG_MD5_STEP(TT_XOR3, d, a, b, c, X[4], 0x4bdecfa9u, 11);                \
    HG_MD5_STEP(TT_XOR3, c, d, a, b, X[7], 0xf6bb4b60u, 16);                \
    HG_MD5_STEP(TT_XOR3, b, c, d, a, X[10], 0xbebfbc70u, 23);               \
    HG_MD5_STEP(TT_XOR3, a, b, c, d, X[13], 0x289b7ec6u, 4);                \
    HG_MD5_STEP(TT_XOR3, d, a, b, c, X[0], 0xeaa127fau, 11);                \
    HG_MD5_STEP(TT_XOR3, c, d, a, b, X[3], 0xd4ef3085u, 16);                \
    HG_MD5_STEP(TT_XOR3, b, c, d, a, X[6], 0x04881d05u, 23);                \
    HG_MD5_STEP(TT_XOR3, a, b, c, d, X[9], 0xd9d4d039u, 4);                 \
    HG_MD5_STEP(TT_XOR3, d, a, b, c, X[12], 0xe6db99e5u, 11);               \
    HG_MD5_STEP(TT_XOR3, c, d, a, b, X[15], 0x1fa27cf8u, 16);               \
    HG_MD5_STEP(TT_XOR3, b, c, d, a, X[2], 0xc4ac5665u, 23);                \
    HG_MD5_STEP(TT_MD5I, a, b, c, d, X[0], 0xf4292244u, 6);                 \
    HG_MD5_STEP(TT_MD5I, d, a, b, c, X[7], 0x432aff97u, 10);                \
    HG_MD5_STEP(TT_MD5I, c, d, a, b, X[14], 0xab9423a7u, 15);               \
    HG_MD5_STEP(TT_MD5I, b, c, d, a, X[5], 0xfc93a039u, 21);                \
    HG_MD5_STEP(TT_MD5I, a, b, c, d, X[12], 0x655b59c3u, 6);                \
    HG_MD5_STEP(TT_MD5I, d, a, b, c, X[3], 0x8f0ccc92u, 10);                \
    HG_MD5_STEP(TT_MD5I, c, d, a, b, X[10], 0xffeff47du, 15);               \
    HG_MD5_STEP(TT_MD5I, b, c, d, a, X[1], 0x85845dd1u, 21);                \
    HG_MD5_STEP(TT_MD5I, a, b, c, d, X[8], 0x6fa87e4fu, 6);                 \
    HG_MD5_STEP(TT_MD5I, d, a, b, c, X[15], 0xfe2ce6e0u, 10);               \
    HG_MD5_STEP(TT_MD5I, c, d, a, b, X[6], 0xa3014314u, 15);                \
    HG_MD5_STEP(TT_MD5I, b, c, d, a, X[13], 0x4e0811a1u, 21);               \
    HG_MD5_STEP(TT_MD5I, a, b, c, d, X[4], 0xf7537e82u, 6);

#define HG_MD5_ROUNDS_61_63(X, a, b, c, d)                                  \
    HG_MD5_STEP(TT_MD5I, d, a, b, c, X[11], 0xbd3af235u, 10);               \
    HG_MD5_STEP(TT_MD5I, c, d, a, b, X[2], 0x2ad7d2bbu, 15);                \
    HG_MD5_STEP(TT_MD5I, b, c, d, a, X[9], 0xeb86d391u, 21);

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
constexpr uint32_t SHA1_K0 = 0x5a827999u, SHA1_K1 = 0x6ed9eba1u, SHA1_K2 = 0x8f1bbcdcu,
                   SHA1_K3 = 0xca62c1d6u;

// Round t with the register names rotated: e += rotl(a,5) + f(b,c,d) + K + W;
// b = rotl(b, 30).  The next round uses (e, a, b, c, d).
#define HG_SHA1_R(TT, K, a, b, c, d, e, w) \
    e += rotl(a, 5) + bop3<TT>(b, c, d) + ((w) + (K)); \
    b = rotl(b, 30);

// Message schedule in a 16-word ring: W[t] = rotl1(W[t-3]^W[t-8]^W[t-14]^W[t-16]).
#define HG_SHA1_W(W, t) \
    (W[(t) & 15] = rotl(bop3<TT_XOR3>(W[((t) - 3) & 15], W[((t) - 8) & 15], W[((t) - 14) & 15]) ^ W[(t) & 15], 1))

#define HG_SHA1_5(TT, K, W, t0, WEXPR)                \
    HG_SHA1_R(TT, K, a, b, c, d, e, WEXPR(W, t0 + 0)) \
    HG_SHA1_R(TT, K, e, a, b, c, d, WEXPR(W, t0 + 1)) \
    HG_SHA1_R(TT, K, d, e, a, b, c, WEXPR(W, t0 + 2)) \
    HG_SHA1_R(TT, K, c, d, e, a, b, WEXPR(W, t0 + 3)) \
    HG_SHA1_R(TT, K, b, c, d, e, a, WEXPR(W, t0 + 4))

#define HG_SHA1_WIN(W, t) W[(t) & 15]

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
