// Stress of the serving loop through the C ABI (admission, group formation,
// completion, waiters, callbacks, statistics): four submitter threads,
// callbacks and waiters mixed, injected failures, a statistics reader
// running concurrently, then a stop with requests still queued.  Every
// served result must equal the single call on its own context.  Built and
// run by tests/test_gpu_server_stress.py; exit status 0 on success.
#include "hashgpu.h"

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t MiB = 1ull << 20;
constexpr int THREADS = 4, PER_THREAD = 60;

struct Job {
    hg_request r{};
    std::vector<uint8_t> leaves, root, digests;
    std::vector<uint64_t> ends;
    uint64_t n_chunks = 0;
    bool waitable = false, inject = false;
    int status = 1;
};

std::atomic<int> callbacks_done{0};

void on_done(uint64_t, int status, void *user) {
    static_cast<Job *>(user)->status = status;
    callbacks_done.fetch_add(1);
}

int fail(const char *what, int st) {
    std::fprintf(stderr, "FAIL: %s (status %d)\n", what, st);
    return 1;
}

}  // namespace

int main() {
    std::mt19937_64 rng(1234);
    std::vector<uint8_t> payload(48 * MiB);
    for (auto &b : payload) b = (uint8_t)rng();

    hg_server_cfg cfg{};
    cfg.slots = 3;
    cfg.max_requests = 16;
    cfg.device_budget = 64 * MiB;
    cfg.max_group_bytes = 16 * MiB;
    hg_server *srv = nullptr;
    int st = hg_server_start(0, &cfg, &srv);
    if (st != HG_OK) return fail("hg_server_start", st);

    std::vector<Job> jobs(THREADS * PER_THREAD);
    for (size_t i = 0; i < jobs.size(); i++) {
        Job &j = jobs[i];
        const uint64_t off = rng() % (payload.size() - 8 * MiB);
        const uint64_t len = (i % 7 == 0) ? rng() % (6 * MiB) : rng() % (512 * 1024);
        j.r.payload = payload.data() + off;
        j.r.len = len;
        j.waitable = i % 3 != 0;
        j.inject = i % 17 == 5;
        if (j.inject) j.r.flags |= HG_REQ_FAIL_INJECT;
        if (i % 2 == 0) {
            j.r.kind = HG_REQ_BLOCK;
            j.r.block_size = 64 * 1024;
            j.r.digest = (i % 4 == 0) ? HG_SHA1 : HG_MD5;
            const int d = hg_digest_size(j.r.digest);
            j.leaves.assign(((len + 65535) / 65536) * d + 1, 0);
            j.root.assign(d, 0);
            j.r.leaf_out = j.leaves.data();
            j.r.root_out = j.root.data();
        } else {
            j.r.kind = HG_REQ_CHUNK;
            j.r.chunk = hg_chunk_params{20, 1, 0xFFF, 0, 2048, 0, HG_MD5, HG_SHA1, 0};
            j.r.capacity = len / 2048 + 2;
            j.ends.assign(j.r.capacity, 0);
            j.digests.assign(j.r.capacity * 20, 0);
            j.r.chunk_ends = j.ends.data();
            j.r.chunk_digests = j.digests.data();
            j.r.n_chunks = &j.n_chunks;
        }
    }

    std::atomic<bool> reading{true};
    std::thread reader([&] {
        hg_server_stats s{};
        while (reading.load()) {
            if (hg_server_stats_read(srv, &s) != HG_OK) std::abort();
            std::this_thread::yield();
        }
    });
    std::vector<std::thread> submitters;
    std::atomic<int> errors{0};
    for (int t = 0; t < THREADS; t++) {
        submitters.emplace_back([&, t] {
            std::vector<uint64_t> ids;
            for (int k = 0; k < PER_THREAD; k++) {
                Job &j = jobs[t * PER_THREAD + k];
                uint64_t id = 0;
                const int s = j.waitable ? hg_submit(srv, &j.r, nullptr, nullptr, &id)
                                         : hg_submit(srv, &j.r, on_done, &j, &id);
                if (s != HG_OK) errors.fetch_add(1);
                ids.push_back(j.waitable ? id : 0);
            }
            for (int k = 0; k < PER_THREAD; k++) {
                Job &j = jobs[t * PER_THREAD + k];
                if (!j.waitable) continue;
                int status = 0;
                if (hg_wait(srv, ids[k], -1, &status) != HG_OK) errors.fetch_add(1);
                j.status = status;
            }
        });
    }
    for (auto &th : submitters) th.join();
    int expected_cb = 0;
    for (const Job &j : jobs) expected_cb += j.waitable ? 0 : 1;
    while (callbacks_done.load() < expected_cb) std::this_thread::yield();
    reading.store(false);
    reader.join();
    if (errors.load()) return fail("submit or wait", errors.load());

    // A few more requests left queued at stop: stop serves them.
    for (int k = 0; k < 8; k++) {
        uint64_t id;
        hg_request r = jobs[k].r;
        r.flags &= ~(uint32_t)HG_REQ_FAIL_INJECT;
        if ((st = hg_submit(srv, &r, nullptr, nullptr, &id)) != HG_OK) return fail("late submit", st);
    }
    if ((st = hg_server_stop(srv)) != HG_OK) return fail("hg_server_stop", st);

    // Results against the single calls.
    hg_ctx *ctx = nullptr;
    if ((st = hg_create(0, 0, 0, &ctx)) != HG_OK) return fail("hg_create", st);
    int checked = 0;
    for (size_t i = 0; i < jobs.size(); i++) {
        Job &j = jobs[i];
        if (j.inject) {
            if (j.status != HG_EDEVICE) return fail("injected failure status", j.status);
            continue;
        }
        if (j.status != HG_OK) return fail("request status", j.status);
        if (j.r.kind == HG_REQ_BLOCK) {
            std::vector<uint8_t> lv(j.leaves.size()), rt(j.root.size());
            st = hg_block_hash(ctx, j.r.payload, j.r.len, j.r.block_size, j.r.digest, lv.data(), rt.data(), 0,
                               nullptr);
            if (st != HG_OK) return fail("hg_block_hash", st);
            if (lv != j.leaves || rt != j.root) return fail("block result differs from the single call", (int)i);
        } else {
            std::vector<uint64_t> e(j.ends.size());
            std::vector<uint8_t> dg(j.digests.size());
            uint64_t n = 0;
            st = hg_chunk(ctx, j.r.payload, j.r.len, &j.r.chunk, e.data(), e.size(), &n, dg.data(), 0, nullptr);
            if (st != HG_OK) return fail("hg_chunk", st);
            if (n != j.n_chunks || std::memcmp(e.data(), j.ends.data(), n * 8) != 0 ||
                std::memcmp(dg.data(), j.digests.data(), n * 20) != 0)
                return fail("chunk result differs from the single call", (int)i);
        }
        checked++;
    }
    hg_destroy(ctx);
    std::printf("server stress ok: %d results checked, %d callbacks\n", checked, callbacks_done.load());
    return 0;
}
