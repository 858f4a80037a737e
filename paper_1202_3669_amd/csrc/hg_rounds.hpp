// hg_rounds.hpp -- the MD5 and SHA-1 round sequences as macros, and their
// constants, shared by the device kernels (hg_device.hpp) and the host's
// sequential hashes (host_hash.cpp).  RFC 1321 / FIPS 180-4 order and
// constants.  Plain C++: the macros expand with whatever bop3<TT>(x, y, z)
// (three-input boolean function by truth table) and rotl(x, s) are in scope.
#pragma once

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

}  // namespace hg
