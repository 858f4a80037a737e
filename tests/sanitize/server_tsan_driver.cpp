// ThreadSanitizer driver for the serving loop's host logic, built against
// the stub device layer (stub/hip/hip_runtime.h, server_stub_device.cpp):
// four submitter threads (callbacks and hg_wait), a load replay
// (hg_server_play) on another thread, a statistics reader polling
// throughout, injected failures, host payloads competing for a small
// staging budget, requests larger than a group (served alone), and a stop
// with requests still queued.  Every request's status and outputs are
// checked against what the stub layer writes for it (and, for the second
// levels the worker computes on the host, against the host digest of the
// segment digests).
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "hashgpu.h"
#include "host_hash.hpp"

namespace {

constexpr uint64_t POOL = 8u << 20, BLOCK = 4096;
std::vector<uint8_t> g_pool(POOL);
std::atomic<int> g_bad{0}, g_callbacks{0};

struct Out {
    hg_request r{};
    std::vector<uint8_t> leaves, root = std::vector<uint8_t>(20), dig;
    std::vector<uint64_t> ends;
    uint64_t n_chunks = ~0ull;
    std::atomic<int> status{1};
    bool inject = false;
};

void make(Out &o, std::mt19937_64 &rng, bool allow_inject) {
    hg_request &r = o.r;
    const uint64_t len = rng() % 3 == 0 ? rng() % (1u << 21) : rng() % (64u << 10);  // some beyond a group
    r.len = len;
    r.payload = g_pool.data() + rng() % (POOL - len);
    r.flags = rng() % 2 ? HG_IN_DEVICE : 0;
    if (r.flags == 0 && len > (1u << 20)) r.flags = HG_IN_DEVICE;  // host payloads stay within the budget
    o.inject = allow_inject && rng() % 25 == 0;
    if (o.inject) r.flags |= HG_REQ_FAIL_INJECT;
    if (rng() % 3) {
        r.kind = HG_REQ_BLOCK;
        r.block_size = BLOCK;
        r.digest = rng() % 2 ? HG_SHA1 : HG_MD5;
        const int d = r.digest == HG_MD5 ? 16 : 20;
        o.leaves.assign((len + BLOCK - 1) / BLOCK * d + 1, 0);
        r.leaf_out = o.leaves.data();
        r.root_out = o.root.data();
    } else {
        r.kind = HG_REQ_CHUNK;
        r.chunk = hg_chunk_params{20, 1, 0xFFF, 0, 2048, 0, HG_MD5, HG_SHA1, 0};
        r.capacity = len / 2048 + 1;
        o.ends.assign(r.capacity + 1, 0);
        o.dig.assign((r.capacity + 1) * 20, 0);
        r.chunk_ends = o.ends.data();
        r.chunk_digests = o.dig.data();
        r.n_chunks = &o.n_chunks;
    }
}

void check(const Out &o) {
    const hg_request &r = o.r;
    const int st = o.status.load();
    if (o.inject) {
        if (st != HG_EDEVICE) g_bad++;
        return;
    }
    if (st != HG_OK) {
        g_bad++;
        return;
    }
    if (r.kind == HG_REQ_BLOCK) {
        const int d = r.digest == HG_MD5 ? 16 : 20;
        const uint64_t nl = (r.len + BLOCK - 1) / BLOCK;
        for (uint64_t i = 0; i < nl * d; i++)
            if (o.leaves[i] != (uint8_t)((r.len * 7 + BLOCK) & 0xff)) {
                g_bad++;
                return;
            }
        // Grouped requests get their second level from the host hash of the
        // segment digests; a request larger than a group runs alone through
        // the stub's hg_block_hash, which writes a pattern.
        uint8_t want[20];
        if (r.len > (1u << 20)) {
            memset(want, (uint8_t)((r.len * 13) & 0xff), sizeof want);
        } else {
            hg::host::digest(r.digest, o.leaves.data(), nl * d, want);
        }
        if (memcmp(o.root.data(), want, (size_t)d) != 0) {
            g_bad++;
            return;
        }
    } else {
        // grouped: no candidates, no chunks; alone: one chunk ending at len
        if (!(o.n_chunks == 0 || (o.n_chunks == 1 && r.len && o.ends[0] == r.len))) g_bad++;
    }
}

void on_done(uint64_t, int status, void *user) {
    static_cast<Out *>(user)->status.store(status);
    g_callbacks++;
}

}  // namespace

int main() {
    std::mt19937_64 seed_rng(7);
    for (auto &b : g_pool) b = (uint8_t)seed_rng();
    hg_server_cfg cfg{3, 8, 2u << 20, 1u << 20, 0, 0};
    hg_server *s = nullptr;
    if (hg_server_start(0, &cfg, &s) != HG_OK) return 2;
    // A host payload larger than the staging budget can never be admitted.
    {
        Out o;
        std::mt19937_64 rng(1);
        make(o, rng, false);
        o.r.flags = 0;
        o.r.len = 3u << 20;
        o.r.payload = g_pool.data();
        uint64_t id;
        if (hg_submit(s, &o.r, nullptr, nullptr, &id) != HG_EBUSY) g_bad++;
    }
    std::atomic<bool> done{false};
    std::thread stats([&] {
        while (!done.load()) {
            hg_server_stats st;
            if (hg_server_stats_read(s, &st) != HG_OK || st.completed > st.submitted) g_bad++;
            std::this_thread::yield();
        }
    });
    constexpr int PER = 150;
    std::vector<std::vector<Out>> outs(4);
    for (auto &v : outs) v = std::vector<Out>(PER);
    std::vector<std::thread> subs;
    int expect_cb = 0;
    std::mutex cb_mu;
    for (int t = 0; t < 4; t++)
        subs.emplace_back([&, t] {
            std::mt19937_64 rng(100 + t);
            std::vector<std::pair<uint64_t, int>> waited;
            int cbs = 0;
            for (int i = 0; i < PER; i++) {
                Out &o = outs[t][i];
                make(o, rng, true);
                uint64_t id = 0;
                const bool cb = i % 3 == 0;
                if (hg_submit(s, &o.r, cb ? on_done : nullptr, cb ? &o : nullptr, &id) != HG_OK) {
                    g_bad++;
                    continue;
                }
                if (cb) cbs++;
                else waited.push_back({id, i});
            }
            std::shuffle(waited.begin(), waited.end(), rng);
            for (auto &w : waited) {
                int st = -100;
                if (hg_wait(s, w.first, -1, &st) != HG_OK) g_bad++;
                outs[t][w.second].status.store(st);
            }
            std::lock_guard<std::mutex> g(cb_mu);
            expect_cb += cbs;
        });
    // A load replay beside the submitters.
    std::vector<Out> play(100);
    std::thread player([&] {
        std::mt19937_64 rng(200);
        std::vector<hg_request> reqs(play.size());
        std::vector<double> arr(play.size()), lat(play.size());
        std::vector<int32_t> sts(play.size());
        for (size_t i = 0; i < play.size(); i++) {
            make(play[i], rng, true);
            reqs[i] = play[i].r;
            arr[i] = 0.0005 * (double)i;
        }
        if (hg_server_play(s, reqs.data(), arr.data(), reqs.size(), lat.data(), sts.data()) != HG_OK) g_bad++;
        for (size_t i = 0; i < play.size(); i++) play[i].status.store(sts[i]);
    });
    for (auto &th : subs) th.join();
    player.join();
    // Callbacks have all run once every waited request is back? Not
    // necessarily: wait for the callback count.
    while (g_callbacks.load() < expect_cb) std::this_thread::yield();
    for (auto &v : outs)
        for (auto &o : v) check(o);
    for (auto &o : play) check(o);
    // Stop with requests still queued: they are served first, callbacks run.
    std::vector<Out> tail(60);
    std::mt19937_64 rng(300);
    const int cb_before = g_callbacks.load();
    for (auto &o : tail) {
        make(o, rng, false);
        uint64_t id;
        if (hg_submit(s, &o.r, on_done, &o, &id) != HG_OK) g_bad++;
    }
    done.store(true);
    stats.join();
    if (hg_server_stop(s) != HG_OK) g_bad++;
    if (g_callbacks.load() != cb_before + (int)tail.size()) g_bad++;
    for (auto &o : tail) check(o);
    printf("server tsan driver: %s (%d callbacks)\n", g_bad.load() ? "BAD" : "ok", g_callbacks.load());
    return g_bad.load() ? 1 : 0;
}
