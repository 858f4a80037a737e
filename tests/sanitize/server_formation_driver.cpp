// Group formation of the serving loop, built against the stub device layer:
// one worker is held inside a request served alone (a chunk request above
// 32 MiB) while seven more are queued behind it -- block and chunk requests
// in device memory, a block request in host memory and a second chunk
// request served alone.  Once released, the worker forms a group of the
// head's kind, passing over device requests of the other kind and the chunk
// request served alone (they stay queued) and taking the host payload of
// its own kind; then a chunk group; then the request served alone.  The
// callbacks' order shows the groups: H | B1 B3 B5 B7 | C2 C6 | C4, and the
// server counts four groups.
#include <atomic>
#include <cstdio>
#include <mutex>
#include <thread>
#include <vector>

#include "hashgpu.h"

namespace stubhook {
extern std::atomic<uint64_t> hold_len;
extern std::atomic<int> entered, released;
}  // namespace stubhook

namespace {

constexpr uint64_t MiB = 1u << 20, BIG = 40 * MiB, SMALL = 8192, BLOCK = 4096;
std::mutex g_mu;
std::vector<int> g_order;
std::atomic<int> g_bad{0};

struct Req {
    int tag = 0;
    hg_request r{};
    std::vector<uint8_t> leaves, root = std::vector<uint8_t>(20), dig;
    std::vector<uint64_t> ends;
    uint64_t n_chunks = 0;
};

void on_done(uint64_t, int status, void *user) {
    const Req *q = static_cast<const Req *>(user);
    if (status != HG_OK) g_bad++;
    std::lock_guard<std::mutex> g(g_mu);
    g_order.push_back(q->tag);
}

void make(Req &q, int tag, bool block, bool device, uint64_t len, const uint8_t *payload) {
    q.tag = tag;
    hg_request &r = q.r;
    r.kind = block ? HG_REQ_BLOCK : HG_REQ_CHUNK;
    r.flags = device ? HG_IN_DEVICE : 0;
    r.payload = payload;
    r.len = len;
    if (block) {
        r.block_size = BLOCK;
        r.digest = HG_SHA1;
        q.leaves.assign((len + BLOCK - 1) / BLOCK * 20, 0);
        r.leaf_out = q.leaves.data();
        r.root_out = q.root.data();
    } else {
        r.chunk = hg_chunk_params{20, 1, 0xFFF, 0, 2048, 0, HG_MD5, HG_SHA1, 0};
        r.capacity = len / 2048 + 1;
        q.ends.assign(r.capacity, 0);
        q.dig.assign(r.capacity * 20, 0);
        r.chunk_ends = q.ends.data();
        r.chunk_digests = q.dig.data();
        r.n_chunks = &q.n_chunks;
    }
}

}  // namespace

int main() {
    std::vector<uint8_t> big(BIG), small(SMALL, 7);
    hg_server_cfg cfg{1, 16, 16 * MiB, 64 * MiB, 0, 0};
    hg_server *s = nullptr;
    if (hg_server_start(0, &cfg, &s) != HG_OK) return 2;
    std::vector<Req> q(8);
    // H (tag 0): served alone and held; then B1 C2 B3 C4 B5 C6 B7 (tags 1-7).
    make(q[0], 0, false, true, BIG, big.data());
    make(q[1], 1, true, true, SMALL, small.data());
    make(q[2], 2, false, true, SMALL, small.data());
    make(q[3], 3, true, true, SMALL, small.data());
    make(q[4], 4, false, true, BIG, big.data());
    make(q[5], 5, true, false, SMALL, small.data());
    make(q[6], 6, false, true, SMALL, small.data());
    make(q[7], 7, true, true, SMALL, small.data());
    stubhook::hold_len.store(BIG);
    uint64_t id;
    if (hg_submit(s, &q[0].r, on_done, &q[0], &id) != HG_OK) g_bad++;
    while (!stubhook::entered.load()) std::this_thread::yield();
    stubhook::hold_len.store(0);  // C4 is not held
    for (int i = 1; i < 8; i++)
        if (hg_submit(s, &q[i].r, on_done, &q[i], &id) != HG_OK) g_bad++;
    stubhook::released.store(1);
    for (;;) {
        std::lock_guard<std::mutex> g(g_mu);
        if (g_order.size() == q.size()) break;
    }
    hg_server_stats st{};
    if (hg_server_stats_read(s, &st) != HG_OK) g_bad++;
    if (hg_server_stop(s) != HG_OK) g_bad++;
    const std::vector<int> want = {0, 1, 3, 5, 7, 2, 6, 4};
    printf("order:");
    for (int t : g_order) printf(" %d", t);
    printf("\ngroups: %llu\n", (unsigned long long)st.groups);
    if (g_order != want || st.groups != 4) g_bad++;
    printf("server formation driver: %s\n", g_bad.load() ? "BAD" : "ok");
    return g_bad.load() ? 1 : 0;
}
