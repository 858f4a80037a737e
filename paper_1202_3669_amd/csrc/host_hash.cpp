// host_hash.cpp -- sequential MD5 / SHA-1 on the host and the host thread
// pool (see host_hash.hpp).
//
// The round sequences are the library's own macros from hg_rounds.hpp
// (RFC 1321 / FIPS 180-4 order and constants); here they expand with host
// versions of the three-input boolean functions and the rotate.  SHA-1 also
// has a path on the x86 SHA extensions: sha1rnds4 runs four rounds on the
// packed (A, B, C, D) state, sha1nexte derives the next four rounds' E from
// the A of four rounds earlier, and sha1msg1 / sha1msg2 extend the message
// schedule four words at a time.
#include "host_hash.hpp"

#include <cpuid.h>
#include <immintrin.h>

#include <atomic>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "hg_rounds.hpp"

namespace hg {
namespace host {

namespace {

// Host forms of the truth tables the device evaluates with v_bitop3_b32.
template <uint32_t TT>
inline uint32_t bop3(uint32_t x, uint32_t y, uint32_t z) {
    if constexpr (TT == TT_SEL) {
        return z ^ (x & (y ^ z));
    } else if constexpr (TT == TT_SELZ) {
        return y ^ (z & (x ^ y));
    } else if constexpr (TT == TT_XOR3) {
        return x ^ y ^ z;
    } else if constexpr (TT == TT_MD5I) {
        return y ^ (x | ~z);
    } else {
        static_assert(TT == TT_MAJ, "truth table without a host form");
        return (x & y) | (z & (x | y));
    }
}

inline uint32_t rotl(uint32_t x, uint32_t s) { return (x << s) | (x >> (32 - s)); }

inline uint32_t le32(const uint8_t *p) {
    uint32_t w;
    memcpy(&w, p, 4);
    return w;
}

void md5_blocks(uint32_t st[5], const uint8_t *p, uint64_t nblocks) {
    for (uint64_t k = 0; k < nblocks; k++, p += 64) {
        uint32_t X[16];
        for (int j = 0; j < 16; j++) X[j] = le32(p + 4 * j);
        uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
        HG_MD5_ROUNDS_0_60(X, a, b, c, d)
        HG_MD5_ROUNDS_61_63(X, a, b, c, d)
        st[0] += a; st[1] += b; st[2] += c; st[3] += d;
    }
}

void sha1_blocks_portable(uint32_t H[5], const uint8_t *p, uint64_t nblocks) {
    for (uint64_t k = 0; k < nblocks; k++, p += 64) {
        uint32_t W[16];
        for (int j = 0; j < 16; j++) W[j] = __builtin_bswap32(le32(p + 4 * j));
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
}

// SHA-1 on the SHA extensions.  The packed state holds A in its top 32-bit
// lane (then B, C, D); E travels in the top lane of its own register.  Each
// group g of four rounds uses message words W[4g..4g+3] (W[4g] in the top
// lane) with E added to the first: for g = 0 the initial E, afterwards
// sha1nexte of the state before the previous group (E after four rounds is
// the A four rounds earlier rotated by 30).  The boolean function changes
// every five groups.
#define HG_NI_GROUP(F, wk)                        \
    do {                                          \
        const __m128i wk_ = (wk);                 \
        prev = abcd;                              \
        abcd = _mm_sha1rnds4_epu32(abcd, wk_, F); \
    } while (0)
// Next four schedule words from the previous sixteen (m0 oldest).
#define HG_NI_SCHED(m0, m1, m2, m3) \
    _mm_sha1msg2_epu32(_mm_xor_si128(_mm_sha1msg1_epu32(m0, m1), m2), m3)

__attribute__((target("sha,sse4.1,ssse3"))) void sha1_blocks_ni(uint32_t H[5], const uint8_t *p,
                                                                uint64_t nblocks) {
    // Reverses the 16 bytes: each 32-bit word becomes big-endian and the
    // first word lands in the top lane.
    const __m128i rev = _mm_set_epi8(0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15);
    __m128i abcd = _mm_set_epi32((int)H[0], (int)H[1], (int)H[2], (int)H[3]);
    __m128i e0 = _mm_set_epi32((int)H[4], 0, 0, 0);
    for (uint64_t k = 0; k < nblocks; k++, p += 64) {
        const __m128i abcd_in = abcd, e_in = e0;
        __m128i m0 = _mm_shuffle_epi8(_mm_loadu_si128((const __m128i *)(p + 0)), rev);
        __m128i m1 = _mm_shuffle_epi8(_mm_loadu_si128((const __m128i *)(p + 16)), rev);
        __m128i m2 = _mm_shuffle_epi8(_mm_loadu_si128((const __m128i *)(p + 32)), rev);
        __m128i m3 = _mm_shuffle_epi8(_mm_loadu_si128((const __m128i *)(p + 48)), rev);
        __m128i prev;
        HG_NI_GROUP(0, _mm_add_epi32(e0, m0));        // rounds 0-3
        HG_NI_GROUP(0, _mm_sha1nexte_epu32(prev, m1)); // 4-7
        HG_NI_GROUP(0, _mm_sha1nexte_epu32(prev, m2)); // 8-11
        HG_NI_GROUP(0, _mm_sha1nexte_epu32(prev, m3)); // 12-15
        // Groups 4..19: each needs the four schedule words after the last
        // sixteen; the ring (m0..m3) advances one register per group.
#define HG_NI_NEXT(F)                                    \
    do {                                                 \
        __m128i m4 = HG_NI_SCHED(m0, m1, m2, m3);        \
        m0 = m1; m1 = m2; m2 = m3; m3 = m4;              \
        HG_NI_GROUP(F, _mm_sha1nexte_epu32(prev, m4));   \
    } while (0)
        HG_NI_NEXT(0);  // 16-19
        HG_NI_NEXT(1); HG_NI_NEXT(1); HG_NI_NEXT(1); HG_NI_NEXT(1); HG_NI_NEXT(1);  // 20-39
        HG_NI_NEXT(2); HG_NI_NEXT(2); HG_NI_NEXT(2); HG_NI_NEXT(2); HG_NI_NEXT(2);  // 40-59
        HG_NI_NEXT(3); HG_NI_NEXT(3); HG_NI_NEXT(3); HG_NI_NEXT(3); HG_NI_NEXT(3);  // 60-79
#undef HG_NI_NEXT
        // E after the last group, plus the block's input E (feed-forward).
        e0 = _mm_sha1nexte_epu32(prev, e_in);
        abcd = _mm_add_epi32(abcd, abcd_in);
    }
    H[0] = (uint32_t)_mm_extract_epi32(abcd, 3);
    H[1] = (uint32_t)_mm_extract_epi32(abcd, 2);
    H[2] = (uint32_t)_mm_extract_epi32(abcd, 1);
    H[3] = (uint32_t)_mm_extract_epi32(abcd, 0);
    H[4] = (uint32_t)_mm_extract_epi32(e0, 3);
}
#undef HG_NI_GROUP
#undef HG_NI_SCHED

bool cpu_has_sha() {
    unsigned a, b, c, d;
    // Leaf 1 ECX: bit 9 SSSE3, bit 19 SSE4.1 (used beside the SHA
    // instructions); leaf 7 sub-leaf 0 EBX bit 29: SHA extensions.
    if (!__get_cpuid(1, &a, &b, &c, &d) || !((c >> 9) & 1u) || !((c >> 19) & 1u)) return false;
    if (!__get_cpuid_count(7, 0, &a, &b, &c, &d)) return false;
    return (b >> 29) & 1u;
}

const bool g_has_sha = cpu_has_sha();
// HG_HOST_SHA1_PORTABLE set in the environment: the portable SHA-1 runs
// even where the SHA extensions exist (so that tests can check both paths).
std::atomic<bool> g_force_portable{getenv("HG_HOST_SHA1_PORTABLE") != nullptr};

void sha1_blocks(uint32_t H[5], const uint8_t *p, uint64_t nblocks) {
    if (g_has_sha && !g_force_portable.load(std::memory_order_relaxed))
        sha1_blocks_ni(H, p, nblocks);
    else
        sha1_blocks_portable(H, p, nblocks);
}

}  // namespace

bool sha1_accelerated() { return g_has_sha && !g_force_portable.load(); }

void digest(int kind, const uint8_t *p, uint64_t n, uint8_t *out) {
    if (kind != 0 && kind != 1) return;
    uint32_t st[5] = {MD5_IV0, MD5_IV1, MD5_IV2, MD5_IV3, SHA1_IV4};
    auto blocks = kind == 0 ? md5_blocks : sha1_blocks;
    const uint64_t full = n / 64;
    if (full) blocks(st, p, full);
    // Padding: 0x80, zeros to 56 mod 64, the bit length (64 bits; little-
    // endian for MD5, big-endian for SHA-1).
    uint8_t tail[128] = {0};
    const uint64_t rem = n - 64 * full;
    if (rem) memcpy(tail, p + 64 * full, rem);
    tail[rem] = 0x80;
    const int nb = rem < 56 ? 1 : 2;
    const uint64_t bits = n * 8;
    for (int j = 0; j < 8; j++) tail[64 * nb - 8 + j] = (uint8_t)(kind == 0 ? bits >> (8 * j) : bits >> (56 - 8 * j));
    blocks(st, tail, (uint64_t)nb);
    for (int j = 0; j < (kind == 0 ? 4 : 5); j++) {
        const uint32_t w = kind == 0 ? st[j] : __builtin_bswap32(st[j]);
        memcpy(out + 4 * j, &w, 4);
    }
}

// ------------------------------------------------------------- pool ----
namespace {

struct Job {
    const std::function<void(uint64_t)> *fn;
    uint64_t n;
    std::atomic<uint64_t> next{0}, done{0};
    int users = 0;  // pool threads working on it (guarded by the pool mutex)
};

class Pool {
  public:
    Pool() {
        // One thread per host core but the caller's, at most 15.
        const unsigned hw = std::thread::hardware_concurrency();
        const int n = (int)std::max(1u, std::min(15u, hw > 1 ? hw - 1 : 1u));
        for (int i = 0; i < n; i++) threads_.emplace_back([this] { work(); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : threads_) t.join();
    }
    int threads() const { return (int)threads_.size(); }

    void run(uint64_t n, const std::function<void(uint64_t)> &fn) {
        if (n == 0) return;
        Job job;
        job.fn = &fn;
        job.n = n;
        if (n > 1) {
            std::lock_guard<std::mutex> g(m_);
            queue_.push_back(&job);
        }
        if (n > 1) cv_.notify_all();
        drain(job);
        std::unique_lock<std::mutex> g(m_);
        for (auto it = queue_.begin(); it != queue_.end(); ++it)
            if (*it == &job) {
                queue_.erase(it);
                break;
            }
        // Every index has been claimed; wait for the pool threads still
        // finishing theirs (and holding a pointer to the job).
        done_cv_.wait(g, [&] { return job.done.load() == job.n && job.users == 0; });
    }

  private:
    static void drain(Job &j) {
        for (;;) {
            const uint64_t i = j.next.fetch_add(1);
            if (i >= j.n) return;
            (*j.fn)(i);
            j.done.fetch_add(1);
        }
    }
    void work() {
        std::unique_lock<std::mutex> g(m_);
        for (;;) {
            cv_.wait(g, [&] { return stop_ || !queue_.empty(); });
            if (stop_) return;
            Job *j = queue_.front();
            if (j->next.load() >= j->n) {  // exhausted: its caller removes it
                queue_.pop_front();
                continue;
            }
            j->users++;
            g.unlock();
            drain(*j);
            g.lock();
            j->users--;
            done_cv_.notify_all();
        }
    }

    std::mutex m_;
    std::condition_variable cv_, done_cv_;
    std::deque<Job *> queue_;
    std::vector<std::thread> threads_;
    bool stop_ = false;
};

Pool &pool() {
    static Pool p;
    return p;
}

}  // namespace

void parallel_for(uint64_t n, const std::function<void(uint64_t)> &fn) { pool().run(n, fn); }
int pool_threads() { return pool().threads(); }

}  // namespace host
}  // namespace hg
