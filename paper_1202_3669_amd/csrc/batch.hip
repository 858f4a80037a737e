// batch.hip -- many direct-hash jobs in few launches (batch-oriented
// computation, paper Sec. 3.1 and Sec. 3.2.4; a stream of hashing jobs,
// Sec. 4.1).
//
// A job is one block to direct-hash: its segments (leaves) and, optionally,
// the second-level hash of its segment digests (Sec. 3.2.2).
//
//   plan    one workgroup lists the jobs of each digest kind in the given
//           order and assigns every segment a task number (prefix sums);
//   leaves  a persistent grid of one-wavefront workgroups (so that the
//           first tasks, the longest chains, spread over all CUs); each
//           workgroup serves one digest kind; a lane's first task follows
//           from its workgroup index, later ones come from an atomic counter
//           (one atomic per wavefront per refill), hashes that segment 64
//           bytes per iteration, stores the digest and takes another, so
//           uneven segments never leave a wavefront idle behind its longest
//           lane.  Tasks are handed out in job order: callers list jobs
//           with the longest sequential chains first;
//   roots   one lane per job hashes the job's segment-digest buffer.  It is
//           a separate launch: the kernel boundary makes every segment
//           digest visible without per-segment cache write-backs across the
//           XCDs' L2 caches.
// Waves working on long chains raise their issue priority (s_setprio) so
// that throughput work running beside them does not stretch the chain.
#include "hashgpu.h"
#include "hg_device.hpp"
#include "hg_internal.hpp"

namespace hg {

// 64- and 128-byte loads (load_block, load_pair) through the global address
// space, for pointers read from memory (job records): the compiler cannot
// tell that such a generic pointer addresses global memory and would issue
// flat loads, which may complete out of order, so that every wait on one of
// them waits for all loads in flight.  Global loads complete in order and let a loop wait for the older
// of two line buffers only.  p: any alignment, global (device or mapped
// host) memory.
typedef uint32_t hg_u32x4u __attribute__((ext_vector_type(4), aligned(1)));
typedef const __attribute__((address_space(1))) hg_u32x4u *hg_gptr4;

__device__ __forceinline__ void load_words_g(const uint8_t *p, uint32_t *X, int n16) {
#pragma unroll
    for (int i = 0; i < n16; i++) {
        const hg_u32x4u v = ((hg_gptr4)p)[i];
        X[4 * i] = v.x;
        X[4 * i + 1] = v.y;
        X[4 * i + 2] = v.z;
        X[4 * i + 3] = v.w;
    }
}
__device__ __forceinline__ void load_block_g(const uint8_t *p, uint32_t X[16]) { load_words_g(p, X, 4); }
__device__ __forceinline__ void load_pair_g(const uint8_t *p, uint32_t X[32]) { load_words_g(p, X, 8); }

struct Plan {
    uint32_t n_cls[2];           // jobs per digest kind
    uint32_t pad0[2];
    unsigned long long tasks[2];  // segments per kind
    unsigned long long blocks[2]; // 64-byte blocks per kind (work estimate)
    unsigned long long next[2];   // task counters
    // followed by: uint32_t cls_job[2][n_jobs]; uint64_t cls_base[2][n_jobs + 1]
};

static_assert(sizeof(hg_block_job) == 48, "hg_block_job layout");

__device__ __forceinline__ uint32_t *plan_jobs(Plan *p, uint32_t n_jobs, int c) {
    return (uint32_t *)(p + 1) + (size_t)c * n_jobs;
}
__device__ __forceinline__ unsigned long long *plan_base(Plan *p, uint32_t n_jobs, int c) {
    uint8_t *q = (uint8_t *)((uint32_t *)(p + 1) + 2 * (size_t)n_jobs);
    q = (uint8_t *)(((uintptr_t)q + 7) & ~(uintptr_t)7);
    return (unsigned long long *)q + (size_t)c * (n_jobs + 1);
}

size_t batch_plan_bytes(uint32_t n_jobs) {
    return sizeof(Plan) + 2 * (size_t)n_jobs * 4 + 8 + 2 * ((size_t)n_jobs + 1) * 8 + 256;
}

// Jobs with block_size 0 have no segments (device tables are not checked
// on the host).
__device__ __forceinline__ uint64_t job_leaves(const hg_block_job &j) {
    return (j.len && j.block_size) ? (j.len + j.block_size - 1) / j.block_size : 0;
}

constexpr int PLAN_TPB = 1024;

// Single workgroup.  Thread t owns the contiguous job range [lo, hi).
__global__ __launch_bounds__(PLAN_TPB) void batch_plan_kernel(const hg_block_job *__restrict__ jobs,
                                                              uint32_t n_jobs, Plan *__restrict__ plan) {
    __shared__ unsigned long long s_cnt[2][PLAN_TPB], s_task[2][PLAN_TPB], s_blk[2][PLAN_TPB];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (n_jobs + PLAN_TPB - 1) / PLAN_TPB;
    const uint32_t lo = min(t * per, n_jobs), hi = min(lo + per, n_jobs);
    unsigned long long cnt[2] = {0, 0}, task[2] = {0, 0}, blk[2] = {0, 0};
    for (uint32_t i = lo; i < hi; i++) {
        const hg_block_job j = jobs[i];
        const int c = j.digest == HG_SHA1 ? 1 : 0;
        const uint64_t n = job_leaves(j);
        cnt[c] += 1;
        task[c] += n;
        blk[c] += (j.len >> 6) + n;
    }
    for (int c = 0; c < 2; c++) {
        s_cnt[c][t] = cnt[c];
        s_task[c][t] = task[c];
        s_blk[c][t] = blk[c];
    }
    __syncthreads();
    for (int off = 1; off < PLAN_TPB; off <<= 1) {
        unsigned long long v[6];
        for (int c = 0; c < 2; c++) {
            v[3 * c + 0] = t >= (uint32_t)off ? s_cnt[c][t - off] : 0;
            v[3 * c + 1] = t >= (uint32_t)off ? s_task[c][t - off] : 0;
            v[3 * c + 2] = t >= (uint32_t)off ? s_blk[c][t - off] : 0;
        }
        __syncthreads();
        for (int c = 0; c < 2; c++) {
            s_cnt[c][t] += v[3 * c + 0];
            s_task[c][t] += v[3 * c + 1];
            s_blk[c][t] += v[3 * c + 2];
        }
        __syncthreads();
    }
    unsigned long long pos[2], base[2];
    for (int c = 0; c < 2; c++) {
        pos[c] = s_cnt[c][t] - cnt[c];
        base[c] = s_task[c][t] - task[c];
    }
    for (uint32_t i = lo; i < hi; i++) {
        const hg_block_job j = jobs[i];
        const int c = j.digest == HG_SHA1 ? 1 : 0;
        plan_jobs(plan, n_jobs, c)[pos[c]] = i;
        plan_base(plan, n_jobs, c)[pos[c]] = base[c];
        pos[c] += 1;
        base[c] += job_leaves(j);
    }
    if (t == PLAN_TPB - 1) {
        for (int c = 0; c < 2; c++) {
            plan->n_cls[c] = (uint32_t)s_cnt[c][t];
            plan->tasks[c] = s_task[c][t];
            plan->blocks[c] = s_blk[c][t];
            plan->next[c] = 0;
            plan_base(plan, n_jobs, c)[s_cnt[c][t]] = s_task[c][t];
        }
    }
}

// Index of the class job that owns task `tk`: largest i with base[i] <= tk.
__device__ __forceinline__ uint32_t find_job(const unsigned long long *base, uint32_t n, uint64_t tk) {
    uint32_t lo = 0, hi = n;  // base[lo] <= tk < base[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= tk) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Segments at least this long mark a wave as running a long chain.
constexpr uint64_t LONG_CHAIN_BYTES = 32 * 1024;

// first_task: this lane's first task (static, by workgroup index, so that
// the first tasks -- the longest chains -- land on consecutive workgroups,
// which the dispatcher spreads over the CUs); dyn_base: the first task
// handed out by the refill counter.
template <int KIND>
__device__ void leaves_worker(const hg_block_job *__restrict__ jobs, uint32_t n_jobs, Plan *plan,
                              bool boost, uint64_t first_task, uint64_t dyn_base) {
    constexpr int c = KIND == KIND_SHA1 ? 1 : 0;
    constexpr int D = Hash<KIND>::DIGEST;
    const uint32_t ncls = plan->n_cls[c];
    const unsigned long long ntask = plan->tasks[c];
    const uint32_t *cjob = plan_jobs(plan, n_jobs, c);
    const unsigned long long *cbase = plan_base(plan, n_jobs, c);
    const int lane = threadIdx.x & 63;

    // Lane state: message [p, p+n), bytes done, where its digest goes.
    const uint8_t *p = nullptr, *end = nullptr;
    uint64_t n = 0, done = 0;
    uint8_t *out = nullptr;
    int phase = 2;  // 0 data, 1 length block pending, 2 idle, 3 finished
    uint32_t st[5] = {0, 0, 0, 0, 0};
    // The lane's next full blocks -- two (one 128-byte line when aligned) or
    // the last one -- loaded an iteration ahead so that their latency hides
    // behind the current compression.  Lanes read whole lines at once: a
    // line read in two halves at different times is easily evicted from L2
    // in between and fetched twice.
    uint32_t Y[32];
    // Cached job range of the last task for the fast lookup path.
    uint32_t ci = 0;
    unsigned long long cb0 = 1, cb1 = 0;
    int prio = 0;

    bool initial = true;
    while (true) {
        const uint64_t idle = __ballot(phase == 2);
        if (idle) {
            unsigned long long first = first_task;
            if (!initial) {
                const uint32_t want = __builtin_popcountll(idle);
                const int leader = __builtin_ctzll(idle);
                if (lane == leader) first = dyn_base + atomicAdd(&plan->next[c], (unsigned long long)want);
                first = __shfl(first, leader, 64);
            }
            if (phase == 2) {
                const unsigned long long tk =
                    initial ? first : first + __builtin_popcountll(idle & ((1ull << lane) - 1ull));
                if (tk < ntask) {
                    if (!(cb0 <= tk && tk < cb1)) {
                        ci = find_job(cbase, ncls, tk);
                        cb0 = cbase[ci];
                        cb1 = cbase[ci + 1];
                    }
                    const hg_block_job j = jobs[cjob[ci]];
                    const uint64_t k = tk - cb0;
                    const uint64_t s0 = k * j.block_size;
                    p = (const uint8_t *)j.in + s0;
                    end = (const uint8_t *)j.in + j.len;
                    n = j.len - s0 < j.block_size ? j.len - s0 : j.block_size;
                    out = (uint8_t *)j.leaf_out + k * D;
                    done = 0;
                    phase = 0;
                    Hash<KIND>::init(st);
                    if (n >= 128) load_pair_g(p, Y);
                    else if (n >= 64) load_block_g(p, Y);
                } else {
                    phase = 3;
                }
            }
            initial = false;
            const int want_prio = (boost && __ballot(phase == 0 && n >= LONG_CHAIN_BYTES)) ? 2 : 0;
            if (want_prio != prio) {
                if (want_prio) __builtin_amdgcn_s_setprio(2);
                else __builtin_amdgcn_s_setprio(0);
                prio = want_prio;
            }
        }
        if (__ballot(phase < 2) == 0) break;
        // Fast path: every active lane has at least m full blocks left (the
        // next two already in Y), so m / 2 pair iterations need no tail
        // handling.  Lanes without work do not limit m; a lane in its tail
        // makes m 0.  The loop alternates two line buffers (Y, Z) so that no
        // buffer is copied per pair, and every lane loads unconditionally:
        // a working lane's next pair, clamped to its last full pair (the
        // surplus load of the last iteration is not used), an idle lane the
        // start of the plan record (in bounds, not used).
        {
            const uint64_t fb = phase == 0 ? (n - done) >> 6 : (phase == 1 ? 0 : ~0ull);
            uint64_t m = fb;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const uint64_t o = __shfl_xor(m, off, 64);
                m = o < m ? o : m;
            }
            const uint64_t m2 = m == ~0ull ? 0 : m >> 1;
            if (m2 > 0) {
                const uint8_t *q = phase == 0 ? p + done + 128 : (const uint8_t *)plan;
                const uint8_t *last = phase == 0 ? p + done + ((fb >> 1) - 1) * 128 : q;
                const uint64_t step = phase == 0 ? 128 : 0;
                uint32_t Z[32];
                uint64_t k = 0;
                // Y's loads complete here, so that inside the loop each
                // buffer's first use waits only for its own loads.
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
                for (; k + 2 <= m2; k += 2) {
                    load_pair_g(q < last ? q : last, Z);
                    q += step;
                    __builtin_amdgcn_sched_barrier(0);
                    Hash<KIND>::block(st, Y);
                    Hash<KIND>::block(st, Y + 16);
                    load_pair_g(q < last ? q : last, Y);
                    q += step;
                    __builtin_amdgcn_sched_barrier(0);
                    Hash<KIND>::block(st, Z);
                    Hash<KIND>::block(st, Z + 16);
                }
                if (k < m2) {
                    load_pair_g(q < last ? q : last, Z);
                    __builtin_amdgcn_sched_barrier(0);
                    Hash<KIND>::block(st, Y);
                    Hash<KIND>::block(st, Y + 16);
#pragma unroll
                    for (int i = 0; i < 32; i++) Y[i] = Z[i];
                }
                if (phase == 0) {
                    done += 128 * m2;
                    // One full block left: Y holds a stale pair; the single-
                    // block path below expects that block in Y[0..15].
                    if (fb - 2 * m2 == 1) load_block_g(p + done, Y);
                }
            }
        }
        if (phase < 2) {
            uint32_t X[16];
            bool last = false;
            if (phase == 1) {
#pragma unroll
                for (int i = 0; i < 16; i++) X[i] = 0;
                Hash<KIND>::length_words(X, n * 8u);
                last = true;
            } else if (n - done >= 64) {
                // One block from Y; its second block moves down, and the
                // block after it is loaded behind it.
                const uint64_t avail = (n - done) >> 6;
#pragma unroll
                for (int i = 0; i < 16; i++) {
                    X[i] = Y[i];
                    Y[i] = Y[i + 16];
                }
                done += 64;
                if (avail >= 3) load_block_g(p + done + 64, Y + 16);
            } else {
                const int rem = (int)(n - done);
                load_tail(p + done, rem, end, X);
#pragma unroll
                for (int i = 0; i < 16; i++) {
                    int valid = rem - 4 * i;
                    valid = valid < 0 ? 0 : (valid > 4 ? 4 : valid);
                    uint32_t v = X[i] & low_bytes_mask(valid);
                    if (i == (rem >> 2)) v |= 0x80u << (8 * (rem & 3));
                    X[i] = v;
                }
                if (rem < 56) {
                    Hash<KIND>::length_words(X, n * 8u);
                    last = true;
                } else {
                    phase = 1;
                }
                done = n;
            }
            Hash<KIND>::block(st, X);
            if (last) {
                store_digest<KIND>(out, st);
                phase = 2;
            }
        }
    }
}

// Workgroups of one to four wavefronts; every wavefront works on its own
// (ballots and shuffles only, no workgroup barrier), numbered w across the
// grid.
__global__ __launch_bounds__(256) void leaves_batch_kernel(const hg_block_job *__restrict__ jobs,
                                                           uint32_t n_jobs, Plan *plan, int boost) {
    // Split the grid's wavefronts between the two digest kinds in proportion
    // to their VALU work (an MD5 block costs about half a SHA-1 block).
    const double w0 = (double)plan->blocks[0] * 328.0, w1 = (double)plan->blocks[1] * 618.0;
    const uint32_t wpg = blockDim.x >> 6;
    const uint32_t g = gridDim.x * wpg;
    const uint32_t w = blockIdx.x * wpg + (threadIdx.x >> 6);
    uint32_t g0;
    if (plan->tasks[1] == 0) g0 = g;
    else if (plan->tasks[0] == 0) g0 = 0;
    else {
        g0 = (uint32_t)(g * (w0 / (w0 + w1)) + 0.5);
        g0 = g0 < 1 ? 1 : (g0 > g - 1 ? g - 1 : g0);
    }
    const int lane = threadIdx.x & 63;
    if (w < g0)
        leaves_worker<KIND_MD5>(jobs, n_jobs, plan, boost != 0, (uint64_t)w * 64 + lane, (uint64_t)g0 * 64);
    else
        leaves_worker<KIND_SHA1>(jobs, n_jobs, plan, boost != 0, (uint64_t)(w - g0) * 64 + lane,
                                 (uint64_t)(g - g0) * 64);
}

template <int KIND>
__device__ void root_lane(const hg_block_job &j) {
    const uint64_t n = job_leaves(j) * (uint64_t)Hash<KIND>::DIGEST;
    uint32_t st[5];
    hash_range<KIND>((const uint8_t *)j.leaf_out, n, (const uint8_t *)j.leaf_out + n, st);
    store_digest<KIND>((uint8_t *)j.root_out, st);
}

// Workgroups [0, g0) take MD5 jobs, the rest SHA-1 jobs, 64 per workgroup.
__global__ __launch_bounds__(64) void roots_batch_kernel(const hg_block_job *__restrict__ jobs,
                                                         uint32_t n_jobs, const Plan *__restrict__ plan, int boost) {
    if (boost) __builtin_amdgcn_s_setprio(3);
    const uint32_t g0 = (plan->n_cls[0] + 63) / 64;
    const int c = blockIdx.x < g0 ? 0 : 1;
    const uint32_t i = (c == 0 ? blockIdx.x : blockIdx.x - g0) * 64 + threadIdx.x;
    if (i >= plan->n_cls[c]) return;
    const hg_block_job j = jobs[plan_jobs((Plan *)plan, n_jobs, c)[i]];
    if (!j.root_out) return;
    if (c == 0) root_lane<KIND_MD5>(j);
    else root_lane<KIND_SHA1>(j);
}

// Second levels computed elsewhere (on the host): root j of `roots` (20-byte
// records by job index) goes to jobs[j].root_out, one lane per job.
__global__ __launch_bounds__(256) void roots_scatter_kernel(const hg_block_job *__restrict__ jobs, uint32_t n_jobs,
                                                            const uint8_t *__restrict__ roots) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_jobs) return;
    const hg_block_job j = jobs[i];
    if (!j.root_out) return;
    const int d = j.digest == KIND_MD5 ? 16 : 20;
    uint8_t *out = (uint8_t *)j.root_out;
    for (int b = 0; b < d; b++) out[b] = roots[20ull * i + b];
}

hipError_t launch_roots_scatter(const hg_block_job *jobs, uint32_t n_jobs, const uint8_t *roots, hipStream_t s) {
    if (n_jobs == 0) return hipSuccess;
    roots_scatter_kernel<<<(n_jobs + 255) / 256, 256, 0, s>>>(jobs, n_jobs, roots);
    return hipGetLastError();
}

hipError_t launch_batch_plan(const hg_block_job *jobs, uint32_t n_jobs, void *plan, hipStream_t s) {
    batch_plan_kernel<<<1, PLAN_TPB, 0, s>>>(jobs, n_jobs, (Plan *)plan);
    return hipGetLastError();
}

hipError_t launch_leaves_batch(const hg_block_job *jobs, uint32_t n_jobs, void *plan, uint32_t waves,
                               uint32_t wg_waves, bool boost, hipStream_t s) {
    if (wg_waves != 1 && wg_waves != 2 && wg_waves != 4) return hipErrorInvalidValue;
    const uint32_t grid = (waves + wg_waves - 1) / wg_waves;
    leaves_batch_kernel<<<grid, 64 * wg_waves, 0, s>>>(jobs, n_jobs, (Plan *)plan, boost ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_roots_batch(const hg_block_job *jobs, uint32_t n_jobs, void *plan, bool boost, hipStream_t s) {
    // Enough workgroups for every job of either kind; surplus ones return.
    if (n_jobs == 0) return hipSuccess;
    const uint32_t grid = 2 * ((n_jobs + 63) / 64);
    roots_batch_kernel<<<grid, 64, 0, s>>>(jobs, n_jobs, (const Plan *)plan, boost ? 1 : 0);
    return hipGetLastError();
}

}  // namespace hg
