// Host-side driver for the sanitizer builds of the library's host hashing
// (host_hash.cpp): prints the digest of every prefix length 0..1100 (and a
// few large ones) of a deterministic buffer, for comparison with an
// independent implementation, then hammers the host thread pool from
// several caller threads at once, each checking that every index of its
// calls ran exactly once.
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <thread>
#include <vector>

#include "host_hash.hpp"

int main() {
    std::vector<uint8_t> buf((1u << 20) + 64);
    uint32_t x = 12345u;
    for (auto &b : buf) {  // xorshift bytes
        x ^= x << 13; x ^= x >> 17; x ^= x << 5;
        b = (uint8_t)x;
    }
    std::vector<uint64_t> lens;
    for (uint64_t n = 0; n <= 1100; n++) lens.push_back(n);
    for (uint64_t n : {4095ull, 4096ull, 4097ull, 65536ull, (1ull << 20) + 13}) lens.push_back(n);
    for (int kind = 0; kind < 2; kind++)
        for (uint64_t n : lens) {
            uint8_t d[20];
            hg::host::digest(kind, buf.data(), n, d);
            printf("%d %llu ", kind, (unsigned long long)n);
            for (int j = 0; j < (kind ? 20 : 16); j++) printf("%02x", d[j]);
            printf("\n");
        }
    // The pool: 8 callers, 300 calls each, 0..63 indices per call.
    std::atomic<int> bad{0};
    std::vector<std::thread> callers;
    for (int t = 0; t < 8; t++)
        callers.emplace_back([&, t] {
            uint32_t y = 777u + t;
            for (int c = 0; c < 300; c++) {
                y ^= y << 13; y ^= y >> 17; y ^= y << 5;
                const uint64_t n = y % 64;
                std::vector<std::atomic<int>> hits(n);
                std::vector<uint8_t> out(n * 20);
                hg::host::parallel_for(n, [&](uint64_t i) {
                    hits[i].fetch_add(1);
                    hg::host::digest((int)(i & 1), buf.data() + i, 100 + i, out.data() + 20 * i);
                });
                for (uint64_t i = 0; i < n; i++)
                    if (hits[i].load() != 1) bad++;
            }
        });
    for (auto &th : callers) th.join();
    printf("pool %s threads=%d\n", bad.load() ? "BAD" : "ok", hg::host::pool_threads());
    return bad.load() ? 1 : 0;
}
