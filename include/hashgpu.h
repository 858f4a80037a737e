/*
 * hashgpu.h -- C ABI of the MI355X (gfx950) HashGPU hashing library.
 *
 * The library implements the two hashing primitives of "GPUs as Storage
 * System Accelerators" (Al-Kiswany, Gharaibeh, Ripeanu), Sec. 2.1 and
 * Sec. 3.2.2:
 *   - direct hashing of a large block with the parallel Merkle-Damgard
 *     construction (segment digests, then the hash of the digest buffer);
 *   - content-based chunking: sliding-window hashing at every stride-aligned
 *     offset, boundary detection, per-chunk digests, and the similarity of
 *     two versions' chunk digests (the block-map comparison of Sec. 3.2.1).
 * Every step runs in the library's HIP kernels on the GPU.
 *
 * Conventions for every entry point
 *   - Return value: HG_OK (0) or a negative HG_E* status; nothing throws
 *     across the ABI.  hg_last_error() gives the text of the last failure.
 *   - Pointers: `in`-type arguments are device pointers when `flags` has
 *     HG_IN_DEVICE, host pointers otherwise; output arguments (digests,
 *     offsets, counts) are device pointers when `flags` has HG_OUT_DEVICE,
 *     host pointers otherwise.  Host input is copied to device memory owned
 *     by the context; host output is copied back before the call returns.
 *   - Stream: `stream` is a hipStream_t (NULL = the default stream).  All
 *     GPU work of the call is ordered on it.
 *   - Synchrony: without HG_ASYNC the call returns when its results are in
 *     the caller's memory.  HG_ASYNC (valid with HG_IN_DEVICE and
 *     HG_OUT_DEVICE for hg_block_hash, hg_block_hash_dual, hg_window_scan,
 *     hg_similarity, hg_chunk and the chunking stages below; with a device
 *     job table for the batch calls; with HG_OUT_DEVICE for the streaming
 *     chunker's feeds) returns after enqueueing; results are valid once the
 *     stream has completed, and truncation can then only be seen by
 *     comparing the written count with the capacity (hg_chunk and the
 *     chunker still wait for the counts they need, see there).
 *   - Sizes: lengths and offsets are 64-bit; inputs may exceed 4 GiB.  Work
 *     that needs 2^31 or more candidates, chunks, two-level chunk segments
 *     or similarity digests in one call is refused with HG_EINVAL (split the
 *     input); segment counts and window counts have no such limit.
 *   - Ownership: the caller owns every buffer it passes and keeps it alive
 *     until the results are valid; the library retains no caller pointer
 *     after that.  A context owns its device scratch, pinned staging memory
 *     and helper streams.
 *   - Concurrency: one context serves one caller thread and one stream at a
 *     time (its scratch is reused from call to call); use one context per
 *     concurrent stream.
 *   - Digest bytes are in the standard byte order of each hash (MD5 words
 *     little-endian, SHA-1 words big-endian), i.e. exactly the bytes a
 *     sequential implementation prints.
 */
#ifndef HASHGPU_H
#define HASHGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hg_ctx hg_ctx;

/* Digest types (the paper's experiments use MD5; SHA-1 is the second
 * standard sequential hash offered). */
enum { HG_MD5 = 0, HG_SHA1 = 1 };

/* Status codes. */
enum {
    HG_OK = 0,
    HG_EINVAL = -1,  /* bad argument: NULL required pointer, zero size, unknown digest, flag misuse */
    HG_ENOMEM = -2,  /* device or pinned allocation failed */
    HG_EDEVICE = -3, /* no usable gfx950 device, or a HIP runtime error (see hg_last_error) */
    HG_ETRUNC = -4,  /* output capacity too small; counts hold the full size, outputs the first
                        `capacity` entries */
    HG_EBUSY = -5    /* resource temporarily unavailable */
};

/* Flags.  HG_LEN_ENDS applies to hg_similarity and hg_blockmap_write only; HG_BACKGROUND to the
 * batch calls only; HG_COUNT_HOST to hg_chunk and the chunker's feed and finish only;
 * HG_HOST_ROOTS to hg_roots_batch and hg_block_hash_batch only; HG_IN_READY to the chunker's
 * feed only. */
enum {
    HG_IN_DEVICE = 1u,
    HG_OUT_DEVICE = 2u,
    HG_ASYNC = 4u,
    HG_LEN_ENDS = 8u,
    HG_BACKGROUND = 16u,
    HG_COUNT_HOST = 32u,
    HG_HOST_ROOTS = 64u,
    HG_IN_READY = 128u
};

/* Limits of the sliding-window primitive. */
enum { HG_MAX_WINDOW = 4096 };

/* ------------------------------------------------------------- context -- */

/* Creates a context on HIP device `device` (that device becomes current for
 * the calling thread).  Returns HG_EDEVICE if the device does not exist or
 * is not a gfx950 GPU, HG_ENOMEM if a pool cannot be allocated.  *out
 * receives the context.  The paper's buffer reuse (Sec. 3.1: buffers are
 * allocated once and reused; Sec. 3.2.3: a queue of pre-allocated buffers):
 *   device_pool_bytes  0: the scratch of the calls on this context is
 *                      allocated when a call first needs it and reused (and
 *                      grown) by later calls.  > 0: one device region of that
 *                      size is allocated now and all call scratch is carved
 *                      from it (first fit, 64 KiB units); a call whose
 *                      scratch does not fit fails with HG_ENOMEM, and calls
 *                      allocate no device memory.  (Batches, chunkers and
 *                      block maps allocate their own memory when created.)
 *   pinned_pool_bytes  0: hg_host_alloc allocates pinned memory per call.
 *                      > 0: one pinned region of that size is allocated now
 *                      and hg_host_alloc carves from it (first fit, 256-byte
 *                      units), HG_ENOMEM when no free range is large enough.
 *                      (The context's own staging for pageable input is
 *                      separate.) */
int hg_create(int device, size_t device_pool_bytes, size_t pinned_pool_bytes, hg_ctx **out);

/* Pool use and allocation counts of a context, e.g. to check that a
 * steady-state loop allocates nothing. */
typedef struct {
    uint64_t device_pool_bytes, device_pool_used;  /* 0, 0 without a device pool */
    uint64_t pinned_pool_bytes, pinned_pool_used;  /* 0, 0 without a pinned pool */
    uint64_t device_allocs;  /* device allocations the context has made (the pool counts once) */
    uint64_t pinned_allocs;  /* pinned host allocations the context has made (pool, staging,
                                hg_host_alloc without a pool) */
    uint64_t host_blocks;    /* hg_host_alloc blocks not yet freed */
} hg_ctx_stats;
int hg_ctx_stats_read(const hg_ctx *ctx, hg_ctx_stats *out);

/* Synchronizes the context's work and frees everything it owns.  NULL is a
 * no-op. */
void hg_destroy(hg_ctx *ctx);

/* Static text of a status code. */
const char *hg_strerror(int status);

/* Copies the text of the context's last failure (NUL-terminated, truncated
 * to n bytes) into buf; returns the status of that failure (HG_OK if none). */
int hg_last_error(const hg_ctx *ctx, char *buf, size_t n);

/* Digest size in bytes: 16 for HG_MD5, 20 for HG_SHA1, HG_EINVAL otherwise. */
int hg_digest_size(int digest);

/* The standard digest of a host buffer, computed on the calling thread by
 * the library's own sequential MD5 / SHA-1 for the host: the routine with
 * which the host computes the last step of direct hashing (Sec. 3.2.2: the
 * CPU hashes the buffer of segment digests into the final value).  in: len
 * bytes of host memory (may be NULL when len is 0); out: digest_size bytes.
 * Needs no context and no GPU.  SHA-1 uses the processor's SHA extensions
 * when it has them (HG_HOST_SHA1_PORTABLE set in the environment when the
 * library loads selects the portable code).  HG_EINVAL for an unknown
 * digest or a NULL pointer. */
int hg_host_hash(int digest, const void *in, uint64_t len, void *out);

/* Pinned (page-locked) host memory from the context, for one-copy transfers
 * (Sec. 3.1: data handed to the GPU should already sit in non-pageable
 * memory, and such buffers should be allocated once and reused; Sec. 3.2.4:
 * buffers are allocated through the library).  With a pinned pool
 * (hg_create) the block is carved from it and HG_ENOMEM means the pool has
 * no free range that large; without one, each call allocates.  *out is NULL
 * on failure.  hg_host_free returns a block (NULL is a no-op); a pointer
 * that is not a live block of this context (foreign, or already freed)
 * gives HG_EINVAL.  hg_destroy frees every block. */
int hg_host_alloc(hg_ctx *ctx, size_t bytes, void **out);
int hg_host_free(hg_ctx *ctx, void *p);

/* ------------------------------------------------------ direct hashing -- */

/* Direct hash with the parallel Merkle-Damgard construction (Sec. 3.2.2,
 * "Direct Hashing").
 *   in, len     the block (len may be 0; in may then be NULL).
 *   block_size  segment size B >= 1.  Segment k covers
 *               [k*B, min((k+1)*B, len)); a short last segment is hashed as
 *               it is, with the standard padding.  n = ceil(len / B).
 *   digest      HG_MD5 or HG_SHA1 (used for both levels).
 *   leaf_out    n * digest_size bytes: segment digests in segment order; may
 *               be NULL when only the root is wanted.
 *   root_out    digest_size bytes: digest of the concatenated segment
 *               digests (for len = 0, the digest of the empty string); may be
 *               NULL.  At least one of leaf_out, root_out is required.
 * With a host `in` the block is streamed to the GPU in pieces through pinned
 * staging buffers, overlapping copies with hashing.
 * The second level is computed on the host, as the paper places it
 * (Sec. 3.2.2: the CPU hashes the buffer of segment digests), when the
 * digest buffer holds at least 16 KiB: the segment digests are copied back
 * and the call waits for them on the host even with HG_ASYNC (which then
 * only leaves the root's copy to a device root_out enqueued).  A smaller
 * second level runs in one GPU lane and needs no host wait. */
int hg_block_hash(hg_ctx *ctx, const void *in, uint64_t len, uint64_t block_size, int digest,
                  void *leaf_out, void *root_out, uint32_t flags, void *stream);

/* Both digests in one pass over the input: the MD5 and the SHA-1 direct
 * hash of the block (the same segments; each byte is read once).  Equal to
 * hg_block_hash with HG_MD5 and with HG_SHA1.  Outputs as there; each may
 * be NULL, not all four.  Second levels as for hg_block_hash (the two host
 * ones run at once). */
int hg_block_hash_dual(hg_ctx *ctx, const void *in, uint64_t len, uint64_t block_size, void *md5_leaf_out,
                       void *md5_root_out, void *sha1_leaf_out, void *sha1_root_out, uint32_t flags,
                       void *stream);

/* ------------------------------------------------- batched direct hash -- */

/* One direct-hash job of a batch.  All pointers are device pointers. */
typedef struct {
    const void *in;       /* the job's bytes (may be NULL when len = 0) */
    uint64_t len;         /* bytes */
    uint64_t block_size;  /* segment size B >= 1 */
    void *leaf_out;       /* ceil(len / B) * digest_size bytes, segment order */
    void *root_out;       /* digest_size bytes, or NULL for no second level */
    int32_t digest;       /* HG_MD5 or HG_SHA1 */
    int32_t reserved;     /* must be 0 */
} hg_block_job;

/* Segment digests of every job of a batch in one persistent launch
 * (batch-oriented computation, Sec. 3.1; Sec. 3.2.4).  Segments are handed
 * to lanes in job order, so jobs with the longest sequential work should be
 * listed first.  `jobs` (n_jobs records) is in device memory with
 * HG_IN_DEVICE (then it is used as is and not validated: a record with
 * block_size 0 is treated as empty) and in host memory otherwise (then every
 * record is validated and the table copied).  Outputs always go to the
 * device pointers inside the records; HG_OUT_DEVICE is implied.  HG_ASYNC
 * requires HG_IN_DEVICE.  The same results as one hg_block_hash call per
 * job.  Wavefronts working on segments of 32 KiB or more raise their issue
 * priority so that the launch is not stretched by its longest chains;
 * HG_BACKGROUND keeps every wavefront at normal priority, for batches that
 * run beside latency-critical work on another stream. */
int hg_leaves_batch(hg_ctx *ctx, const hg_block_job *jobs, uint32_t n_jobs, uint32_t flags,
                    void *stream);

/* Second level of every job whose root_out is not NULL: root_out receives
 * the digest of the job's leaf_out buffer (ceil(len/B) digests), as
 * hg_block_hash does.  Reads leaf_out, so it must be ordered after the
 * hg_leaves_batch call that wrote it.  One GPU lane per job (many small
 * second levels).  Arguments as for hg_leaves_batch.
 * With HG_HOST_ROOTS (host job table only) the second levels run on the
 * host's cores instead, where the paper computes them (Sec. 3.2.2; a few
 * long second levels): the call copies every job's segment digests back,
 * waits for them on the host, hashes them on the library's host threads
 * (longest first), and copies the roots to their root_out pointers on
 * `stream`; with HG_ASYNC it returns once those copies are enqueued. */
int hg_roots_batch(hg_ctx *ctx, const hg_block_job *jobs, uint32_t n_jobs, uint32_t flags,
                   void *stream);

/* hg_leaves_batch followed by hg_roots_batch on the same stream. */
int hg_block_hash_batch(hg_ctx *ctx, const hg_block_job *jobs, uint32_t n_jobs, uint32_t flags,
                        void *stream);

/* ---------------------------------------------- content-based chunking -- */

/* Sliding-window hashing (Sec. 2.1, "Content-based chunking"; Sec. 3.2.2).
 *   window      w, 1 <= w <= HG_MAX_WINDOW bytes.
 *   stride      s >= 1.  Windows start at i = k*s (k >= 0) and satisfy
 *               i + w <= len, so there are floor((len - w)/s) + 1 windows
 *               when len >= w and none otherwise (not an error).
 *   mask,target a window is a boundary candidate iff
 *               (u32le(D[0..3]) & mask) == target, where D is the standard
 *               digest (`digest`) of the w window bytes and u32le reads its
 *               first four bytes as a little-endian integer.
 *   starts      capacity entries of uint64: ascending start offsets of the
 *               candidates (may be NULL when capacity is 0).
 *   count       one uint64: the number of candidates (always the full number).
 * Returns HG_ETRUNC (after writing the first `capacity` starts) when more
 * candidates exist than fit. */
int hg_window_scan(hg_ctx *ctx, const void *in, uint64_t len, uint32_t window, uint32_t stride,
                   uint32_t mask, uint32_t target, int digest, uint64_t *starts,
                   uint64_t capacity, uint64_t *count, uint32_t flags, void *stream);

/* hg_window_scan without any allocation, for callers that cannot allocate
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The same scan and results as hg_window_scan with
 * HG_IN_DEVICE | HG_OUT_DEVICE | HG_ASYNC: in, starts and count are device
 * pointers, the call returns after enqueueing on `stream`, and *count holds
 * the full number of candidates once the stream has completed (truncation
 * shows as *count > capacity).  Its scratch (the per-tile bookkeeping, about
 * 80 bytes per 4096 windows for w = 20 at stride 1 or 4, up to twice that
 * for other windows) lives in a fixed array of HG_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU until the process ends (set up by
 * hg_create); the call allocates nothing and returns HG_EINVAL when the
 * scan would need more (for w = 20, stride 1: inputs up to about 1.6 GiB).
 * Every call on a GPU shares that GPU's array and leaves it holding its
 * bookkeeping: calls that overlap on one GPU (other streams, other threads,
 * other contexts) race and must be serialized by the caller. */
enum { HG_NOALLOC_SCRATCH_BYTES = 32 << 20 };
int hg_window_scan_noalloc(hg_ctx *ctx, const void *in, uint64_t len, uint32_t window, uint32_t stride,
                           uint32_t mask, uint32_t target, int digest, uint64_t *starts,
                           uint64_t capacity, uint64_t *count, void *stream);

typedef struct {
    uint32_t window, stride, mask, target; /* as for hg_window_scan */
    uint64_t min_chunk;   /* minimum chunk size in bytes (0 = none) */
    uint64_t max_chunk;   /* maximum chunk size in bytes (0 = none; else >= max(min_chunk, 1)) */
    int32_t window_digest; /* digest of the sliding windows */
    int32_t chunk_digest;  /* digest of each chunk */
    uint64_t chunk_segment; /* 0: a chunk's digest is the standard digest of its
                             * bytes.  S > 0: each chunk is direct-hashed by the
                             * parallel construction (Sec. 3.2.2, applied to every
                             * detected chunk as in Sec. 3.2.4): cut into segments
                             * of S bytes from its start (the last one shorter),
                             * digest = H(H(seg_0) || ... || H(seg_m-1)), m =
                             * ceil(len / S) -- what hg_block_hash gives as the
                             * root of the chunk's bytes at block size S. */
} hg_chunk_params;

/* Content-based chunking of one block: window scan, boundary decision and
 * chunk digests (Fig. 3 legend; Sec. 3.2.4).
 * Boundary decision: a candidate window starting at i proposes the cut
 * e = i + w; scanning candidates in ascending order, e becomes a cut iff
 * e < len and e - last >= max(min_chunk, 1), where last is the previous cut
 * (initially 0).  The final chunk ends at len.  len = 0 gives no chunks.
 * With max_chunk > 0 (Sec. 4.3 names a maximum chunk size; this is the
 * reading taken): whenever the next cut by that rule -- or len, when there
 * is none -- lies more than max_chunk past `last`, a cut is forced at
 * last + max_chunk and the rule applies again from there; so no chunk is
 * longer than max_chunk, and at most len / max_chunk cuts are forced.
 *   ends           capacity entries of uint64: ascending chunk end offsets
 *                  (the last one is len).  Chunk j is [ends[j-1], ends[j])
 *                  with ends[-1] = 0.
 *   n_chunks       one uint64: the number of chunks (always the full number).
 *   chunk_digests  capacity * digest_size(chunk_digest) bytes, or NULL.
 * Returns HG_ETRUNC when n_chunks > capacity (outputs hold the first
 * `capacity` chunks).
 * The call waits on the host for two counts it needs to size its launches:
 * the candidates after the window scan and the chunks after the boundary
 * decision.  With HG_ASYNC (and HG_IN_DEVICE, HG_OUT_DEVICE) it returns
 * right after enqueueing the chunk digests and the output copies, so that
 * the digests can overlap the caller's next work on another stream; the
 * outputs are valid once the stream has completed.  With HG_COUNT_HOST,
 * n_chunks is a host pointer (written before the call returns) even when
 * the other outputs are device pointers. */
int hg_chunk(hg_ctx *ctx, const void *in, uint64_t len, const hg_chunk_params *params,
             uint64_t *ends, uint64_t capacity, uint64_t *n_chunks, void *chunk_digests,
             uint32_t flags, void *stream);

/* Similarity of two versions' chunk digests (the block-map comparison of
 * Sec. 3.2.1): *matched = number of B's chunks, counted with multiplicity,
 * whose digest occurs among A's n_a digests; *matched_bytes = sum of the
 * lengths of those chunks (0 when len_b is NULL).  len_b holds n_b chunk
 * lengths, or with HG_LEN_ENDS the n_b ascending chunk end offsets that
 * hg_chunk returns (chunk j is then ends[j] - ends[j-1] long, ends[-1] = 0).
 * dig_a, dig_b, len_b are inputs (HG_IN_DEVICE); matched, matched_bytes are
 * outputs (HG_OUT_DEVICE).  matched_bytes may be NULL. */
int hg_similarity(hg_ctx *ctx, const void *dig_a, uint64_t n_a, const void *dig_b,
                  const uint64_t *len_b, uint64_t n_b, int digest, uint64_t *matched,
                  uint64_t *matched_bytes, uint32_t flags, void *stream);

/* --------------------------------------------- the chunking stages alone -- */
/* The stages of hg_chunk as separate calls (Sec. 3.2.2: window digests, then
 * the boundary decision, then a direct hash of each chunk; Fig. 3).  Counts
 * produced on the device feed the next stage on the device, so a pipeline
 * of hg_window_scan (HG_ASYNC), hg_chunk_select, hg_chunk_digests and
 * hg_similarity_n runs without waiting on the host, and its stages can be
 * placed on different streams with events between them. */

/* Boundary decision from candidate window starts, by the rule of hg_chunk
 * (minimum, and maximum when max_chunk > 0), for a block of len bytes.
 *   starts     ascending window start offsets, as hg_window_scan writes them;
 *              max_starts entries of room.
 *   n_starts   one uint64: the number of candidates.  When *n_starts exceeds
 *              max_starts (the scan found more than it could store), the
 *              list is incomplete: *n_chunks is set to UINT64_MAX, and a
 *              call that waits returns HG_ETRUNC.
 *   ends       capacity entries; capacity must be at least max_starts + 1
 *              (+ len / max_chunk + 1 with a maximum), else HG_EINVAL.
 *   n_chunks   one uint64: the number of chunks.
 * starts and n_starts are device pointers with HG_IN_DEVICE; ends and
 * n_chunks with HG_OUT_DEVICE.  With HG_ASYNC (both flags) nothing waits on
 * the host.  Starts that do not ascend give meaningless cuts, never writes
 * outside `ends`. */
int hg_chunk_select(hg_ctx *ctx, const uint64_t *starts, const uint64_t *n_starts, uint64_t max_starts,
                    uint64_t len, uint32_t window, uint64_t min_chunk, uint64_t max_chunk, uint64_t *ends,
                    uint64_t capacity, uint64_t *n_chunks, uint32_t flags, void *stream);

/* Chunk digests (Fig. 3 legend, Sec. 3.2.4) of in[0, len): chunk j is
 * [ends[j-1], ends[j]) with ends[-1] = 0, for min(*n_chunks, max_chunks)
 * chunks; `digests` has room for max_chunks digests.  chunk_segment as in
 * hg_chunk_params (0: standard digest; S > 0: two-level with S-byte
 * segments).  Ends past len are read as len and a decreasing end as an empty
 * chunk, so no input leads outside the buffers.  in, ends and n_chunks are
 * device pointers with HG_IN_DEVICE, digests with HG_OUT_DEVICE; HG_ASYNC
 * (both flags) returns after enqueueing. */
int hg_chunk_digests(hg_ctx *ctx, const void *in, uint64_t len, const uint64_t *ends, const uint64_t *n_chunks,
                     uint64_t max_chunks, int digest, uint64_t chunk_segment, void *digests, uint32_t flags,
                     void *stream);

/* hg_similarity with B's count read when the work runs: B has
 * min(*n_b, max_b) chunks; dig_b and len_b have room for max_b entries.
 * n_b is a device pointer with HG_IN_DEVICE (as hg_chunk_select writes it),
 * a host pointer otherwise.  Other arguments and flags as hg_similarity. */
int hg_similarity_n(hg_ctx *ctx, const void *dig_a, uint64_t n_a, const void *dig_b, const uint64_t *len_b,
                    const uint64_t *n_b, uint64_t max_b, int digest, uint64_t *matched, uint64_t *matched_bytes,
                    uint32_t flags, void *stream);

/* ------------------------------------------------------------ block map -- */

/* The block-map of a content-addressable store (Sec. 3.2.1: written data is
 * cut into chunks identified by their digests, and only chunks the store
 * does not hold yet are stored): the digests of every chunk stored so far,
 * kept on the device across writes. */
typedef struct hg_blockmap hg_blockmap;

/* capacity: the most digests the map will hold (1 .. 2^30). */
int hg_blockmap_create(hg_ctx *ctx, int digest, uint64_t capacity, hg_blockmap **out);
void hg_blockmap_destroy(hg_blockmap *m);
int hg_blockmap_size(const hg_blockmap *m, uint64_t *n);

/* Writes one version's n chunk digests, in order: chunk i is a duplicate iff
 * its digest is in the map already or equals the digest of a chunk j < i of
 * this write; every other chunk is new and its digest is added.  is_dup
 * (n bytes, 1 = duplicate) may be NULL; *dup_chunks and *dup_bytes (host
 * pointers, may be NULL) receive the number of duplicates and the sum of
 * their lengths (len_b: n lengths, or with HG_LEN_ENDS the chunk end offsets
 * hg_chunk returns; NULL: bytes not counted) -- the bytes a store need not
 * write.  digests and len_b are device pointers with HG_IN_DEVICE, is_dup
 * with HG_OUT_DEVICE.  Synchronous.  HG_EBUSY when the map could overflow
 * (size + n > capacity); nothing is changed then. */
int hg_blockmap_write(hg_blockmap *m, const void *digests, const uint64_t *len_b, uint64_t n, uint32_t flags,
                      uint8_t *is_dup, uint64_t *dup_chunks, uint64_t *dup_bytes, void *stream);

/* ---------------------------------------------------- streaming chunker -- */

/* Content-based chunking of a stream fed in pieces (Sec. 3.2.4: data is
 * buffered, each buffer is chunked on the GPU, and the bytes after its last
 * boundary carry over to the next buffer).  The concatenation of the chunks
 * that all feeds and the finish return is exactly what hg_chunk returns for
 * the whole stream with the same parameters.  The device holds only the
 * carry (the bytes from the last decided cut, and w - 1 before it, to the end
 * of the data fed) plus the piece being fed.  A chunker serves one caller at
 * a time on its context. */
typedef struct hg_chunker hg_chunker;

int hg_chunker_create(hg_ctx *ctx, const hg_chunk_params *params, hg_chunker **out);
void hg_chunker_destroy(hg_chunker *c);

/* *bound = the most chunks one feed of len bytes (or the finish, len = 0)
 * can return; the capacity passed must be at least this. */
int hg_chunker_bound(const hg_chunker *c, uint64_t len, uint64_t *bound);

/* Appends data[0, len) (HG_IN_DEVICE: device memory, else host memory) and
 * returns the chunks the bytes known so far determine: *n_chunks of them,
 * ends[] as absolute stream offsets ascending (a chunk starts where the
 * previous one -- of this or an earlier call -- ended, the first at 0), and
 * their digests (NULL: not wanted).  Outputs are device pointers with
 * HG_OUT_DEVICE (then n_chunks too, unless HG_COUNT_HOST), host pointers
 * otherwise.  Synchronous, unless HG_ASYNC (with HG_OUT_DEVICE; the input
 * may be host memory): then the call returns once the input has been read
 * and the cuts decided, and ends[], the digests and a device *n_chunks are
 * written in stream order on `stream`, valid after it synchronizes.  The
 * input may be reused when the call returns; the outputs may not be read
 * or reused before the stream synchronizes.  A feed's copy, window scan
 * and boundary decision run on a stream of the chunker's own and end with
 * one host wait; its ends, digests and count are written on `stream`, so
 * with HG_ASYNC the digests left running overlap the next feed's copy and
 * window scan.  Device input is read after the work already queued on
 * `stream` (which may produce it) -- that includes the previous feed's
 * digests -- unless the caller passes HG_IN_READY: the device input is
 * complete when the call is made (nothing pending on `stream` writes it).
 * HG_EINVAL when capacity < hg_chunker_bound, or HG_ASYNC without
 * HG_OUT_DEVICE. */
int hg_chunker_feed(hg_chunker *c, const void *data, uint64_t len, uint32_t flags, uint64_t *ends,
                    uint64_t capacity, uint64_t *n_chunks, void *chunk_digests, void *stream);

/* Ends the stream: returns the remaining chunks, the last one ending at the
 * stream's length.  Afterwards only hg_chunker_reset (start a new stream)
 * or hg_chunker_destroy are accepted. */
int hg_chunker_finish(hg_chunker *c, uint32_t flags, uint64_t *ends, uint64_t capacity, uint64_t *n_chunks,
                      void *chunk_digests, void *stream);
int hg_chunker_reset(hg_chunker *c);

/* -------------------------------------------------------- file batches -- */

/* A planned batch of many files held in one device arena: every file gets
 * the direct hash (segments + optional second level) and content-based
 * chunking with chunk digests, exactly as one hg_block_hash and one hg_chunk
 * call per file would give (batch-oriented computation, Sec. 3.1; the
 * buffered, batched chunking of Sec. 3.2.4).  The plan uploads the file
 * layout once and owns all scratch, so runs allocate nothing and a run can
 * be captured into a HIP graph and replayed. */
typedef struct hg_batch hg_batch;

typedef struct {
    uint64_t block_size;      /* direct-hash segment size; 0 = no direct hash */
    int32_t block_digest;     /* HG_MD5 or HG_SHA1 */
    int32_t roots;            /* nonzero: also the second level of every file */
    hg_chunk_params chunk;    /* chunk.window == 0: no chunking */
    uint64_t max_candidates;  /* boundary-candidate capacity over all files; 0 = twice the
                                 expectation for random data (mask bits) plus slack */
} hg_batch_params;

/* Outputs of a run, all device pointers (sizes from hg_batch_layout). */
typedef struct {
    void *leaf_digests;     /* n_leaves_total * d: file f's segments start at leaf_first[f] */
    void *roots;            /* n_files * d, file order (or NULL) */
    uint64_t *chunk_ends;   /* max_chunks: ends relative to the file start, files in order */
    void *chunk_digests;    /* max_chunks * d_chunk, same order (or NULL) */
    uint64_t *chunk_off;    /* n_files + 1: chunks of file f are [chunk_off[f], chunk_off[f+1]) */
    uint64_t *status;       /* 4 words: candidates, chunks, overflow (nonzero: the candidate
                               capacity was too small and the chunk outputs are incomplete;
                               re-plan with a larger max_candidates), 0 */
} hg_batch_out;

/* file_off, file_len: host arrays of n_files byte offsets/lengths inside the
 * arena that runs will pass.  Files may overlap and need no alignment. */
int hg_batch_create(hg_ctx *ctx, const uint64_t *file_off, const uint64_t *file_len, uint32_t n_files,
                    const hg_batch_params *params, hg_batch **out);
void hg_batch_destroy(hg_batch *b);

/* Sizes of the outputs; leaf_first (host, n_files + 1 entries) may be NULL. */
int hg_batch_layout(const hg_batch *b, uint64_t *leaf_first, uint64_t *n_leaves_total, uint64_t *max_chunks);

/* Enqueues the whole batch on `stream` (asynchronous: results are valid when
 * the stream has completed; no host synchronization inside).  The direct
 * hash and the chunking run as two concurrent branches. */
int hg_batch_run(hg_batch *b, const void *arena, const hg_batch_out *out, void *stream);

/* Captures one hg_batch_run with these arguments into a HIP graph owned by
 * the batch; hg_batch_replay launches it (one launch per batch). */
int hg_batch_capture(hg_batch *b, const void *arena, const hg_batch_out *out, void *stream);
int hg_batch_replay(hg_batch *b, void *stream);

/* Schedule autotuner: times the direct-hash part of the batch under each
 * candidate segment-to-lane schedule (file order: longest first or as
 * given; persistent grid: 1024-8192 wavefronts; lanes per workgroup: 64,
 * 128 or 256) with HIP events, keeps the fastest for later runs (and captures),
 * and writes a one-line report of what it measured.  Synchronous. */
int hg_batch_tune(hg_batch *b, const void *arena, const hg_batch_out *out, void *stream, char *report,
                  size_t report_len);

/* ------------------------------------------------------------- serving -- */

/* A serving loop for hash requests (the job lifecycle of the paper's
 * CrystalGPU layer, Sec. 3.2.3: jobs are handed to an outstanding queue, run
 * on the GPU with buffers allocated once and reused, and reported by
 * callback; Sec. 3.1: batching and overlap of transfers with work).
 *
 * Continuous batching: `slots` workers each own a stream pair and a
 * pre-allocated group (job table, segment and chunk scratch, pinned output
 * buffer).  A worker that becomes idle takes the waiting requests from the
 * head of the queue, in arrival order, while they fit its group and the
 * device staging budget, and runs them as one group: one persistent launch
 * for the segment digests of all its block requests (their second levels
 * then on the host's cores, as Sec. 3.2.2 places them, from the digests
 * copied back), and the sliding-window chunking of all its chunk requests
 * through one tile map.  Groups of different workers overlap on the device;
 * a request that arrives while groups run joins the next group that frees
 * up, without waiting for the others to drain.  A request that does not fit
 * an empty group -- and a chunk request of more than 32 MiB, whose boundary
 * decision the single call makes faster -- is served alone by a worker
 * through the single-call entry point.  A request in device memory whose
 * kind (block or chunk) differs from the group's, or a chunk request in
 * device memory served alone for its size or parameters, does not close the
 * group being formed: it stays at its place in the queue for the next idle
 * worker, and the requests behind it that fit join the group -- so groups
 * of device payloads hold one kind.  (Host payloads keep strict arrival
 * order: they are admitted by staging room at the head of the queue.)
 *
 * Admission by device memory: a payload in host memory is admitted only
 * when its bytes fit the staging region (device_budget bytes, allocated once
 * at start and carved first-fit); it is copied there on the worker's stream
 * and its bytes return to the region when the request completes.  A payload
 * in device memory (HG_IN_DEVICE) takes no staging bytes.
 *
 * Each request's results are those of the single call of its primitive
 * (hg_block_hash with its block size and digest, or hg_chunk with its
 * parameters), bit for bit.  Outputs are host memory. */
typedef struct hg_server hg_server;

enum { HG_REQ_BLOCK = 0, HG_REQ_CHUNK = 1 };

/* Request flag for tests of failure handling: the worker fails the request
 * with HG_EDEVICE at its staging step, before any of its work is enqueued;
 * the other requests of its group are served normally. */
enum { HG_REQ_FAIL_INJECT = 1u << 8 };

typedef struct {
    int32_t kind;           /* HG_REQ_BLOCK or HG_REQ_CHUNK */
    uint32_t flags;         /* HG_IN_DEVICE (payload in device memory), HG_REQ_FAIL_INJECT */
    const void *payload;    /* len bytes (may be NULL when len is 0) */
    uint64_t len;
    /* HG_REQ_BLOCK: the direct hash (hg_block_hash) */
    uint64_t block_size;    /* segment size B >= 1 */
    int32_t digest;         /* HG_MD5 or HG_SHA1 */
    int32_t reserved;
    void *leaf_out;         /* ceil(len / B) digests, or NULL */
    void *root_out;         /* one digest, or NULL (not both NULL) */
    /* HG_REQ_CHUNK: content-based chunking (hg_chunk) */
    hg_chunk_params chunk;
    uint64_t *chunk_ends;   /* capacity entries (may be NULL when capacity is 0) */
    uint64_t capacity;
    uint64_t *n_chunks;     /* one word: the full number of chunks */
    void *chunk_digests;    /* capacity digests, or NULL */
} hg_request;

typedef struct {
    uint32_t slots;           /* workers (groups in flight), 1..64 */
    uint32_t max_requests;    /* requests per group, >= 1 */
    uint64_t device_budget;   /* staging bytes for host payloads, >= 1 */
    uint64_t max_group_bytes; /* payload bytes per group, >= 1 MiB; a larger request runs alone */
    uint32_t flags;           /* HG_BACKGROUND: no raised issue priority for long segments */
    uint32_t reserved;
} hg_server_cfg;

typedef struct {
    uint64_t submitted, completed, failed; /* failed: status other than HG_OK and HG_ETRUNC */
    uint64_t bytes;                        /* payload bytes of completed requests */
    uint64_t groups;                       /* groups run */
    uint64_t queued;                       /* waiting now */
    uint32_t in_flight, max_in_flight;     /* requests admitted and not completed */
    double p50_ms, p99_ms, mean_ms, max_ms; /* latency submit -> completion over the last 2^20
                                             * completed requests (since the last reset) */
} hg_server_stats;

/* Starts the workers on `device`; allocates every group and the staging
 * region now (HG_ENOMEM if that fails).  Streams are created with default
 * priority. */
int hg_server_start(int device, const hg_server_cfg *cfg, hg_server **out);

/* Queues a copy of *req (the payload and output buffers are not copied: the
 * caller keeps them alive until completion).  Thread-safe.  *id receives the
 * request id.  With a callback, cb(id, status, user) runs on a worker thread
 * after the outputs are written, and the request is released after it; the
 * caller must not hg_wait on it.  Without a callback the caller must
 * hg_wait on the id.  HG_EINVAL for a malformed request, HG_EBUSY when the
 * server is stopping or a host payload exceeds device_budget (it could never
 * be admitted). */
int hg_submit(hg_server *s, const hg_request *req, void (*cb)(uint64_t id, int status, void *user), void *user,
              uint64_t *id);

/* Waits for request `id` (timeout_ms < 0: no limit) and releases it;
 * *status receives its status (HG_OK, HG_ETRUNC when the chunk capacity was
 * too small, or the failure).  Returns HG_EBUSY on timeout (the request
 * stays), HG_EINVAL for an unknown id. */
int hg_wait(hg_server *s, uint64_t id, int timeout_ms, int *status);

/* Load replay: submits req[i] at start + arrival_s[i] (arrival_s ascending,
 * seconds) from a native submitter thread, waits for all, and writes each
 * request's latency (completion minus its scheduled arrival, ms) and status.
 * The arrival schedule is kept even when the server falls behind. */
int hg_server_play(hg_server *s, const hg_request *req, const double *arrival_s, uint64_t n, double *latency_ms,
                   int32_t *status);

int hg_server_stats_read(hg_server *s, hg_server_stats *out);
int hg_server_stats_reset(hg_server *s);

/* Stops admitting, serves every queued request, joins the workers and frees
 * everything.  Requests not yet waited for are released. */
int hg_server_stop(hg_server *s);

/* ------------------------------------------------------ kernel timing -- */

/* Kernel classes for the timing counters. */
enum {
    HG_K_LEAVES = 0,         /* segment digests of hg_block_hash */
    HG_K_ROOT = 1,           /* second level of hg_block_hash */
    HG_K_WINDOW_TILES = 2,   /* window hashing + per-tile counts (hg_window_scan, hg_chunk) */
    HG_K_WINDOW_EMIT = 3,    /* tile prefix + ordered candidate output */
    HG_K_CHUNK_SELECT = 4,   /* boundary decision */
    HG_K_CHUNK_DIGESTS = 5,  /* chunk digests */
    HG_K_SIMILARITY = 6,     /* digest set build + probe */
    HG_K_LEAVES_BATCH = 7,   /* hg_leaves_batch */
    HG_K_ROOTS_BATCH = 8,    /* hg_roots_batch */
    HG_K_COUNT = 9
};

/* Measurement support.  While enabled, the context records a pair of HIP
 * events on the call's stream around every launch of each kernel class
 * above.  hg_timing_read waits for the recorded events and returns, for one
 * class, the number of launches and the summed GPU duration (ms) since the
 * last reset.  Disabled by default; recording adds two event records per
 * launch. */
int hg_timing_enable(hg_ctx *ctx, int enable);
int hg_timing_read(hg_ctx *ctx, int kernel_class, uint64_t *launches, double *total_ms);
int hg_timing_reset(hg_ctx *ctx);

/* Per-launch intervals, for launches that overlap (several streams): after
 * hg_timing_origin(ctx, event) -- `event` is a hipEvent_t with timing,
 * already recorded before the launches to be measured and kept alive by the
 * caller until the reads are done (NULL turns this off) -- every timed
 * launch also records its start and end in ms after that event.
 * hg_timing_intervals copies up to `capacity` of them for one kernel class
 * (launch order) and sets *count to the number recorded since the last
 * reset (HG_ETRUNC when that exceeds capacity).  Contexts given the same
 * origin share one time axis, so their intervals can be merged. */
int hg_timing_origin(hg_ctx *ctx, void *event);

/* Measured ceilings (synchronous, best of three timed runs after a warm-up).
 * hg_probe_alu: int32 VALU issue rate in Tops/s, from independent chains of
 * rotate, add and three-input logic ops (the hash rounds' mix) on every
 * SIMD.  hg_probe_read: HBM read rate in GB/s (1e9 B/s), 16-byte loads over
 * the device buffer buf of len bytes (len >= 16; use one larger than the
 * caches). */
int hg_probe_alu(hg_ctx *ctx, double *tops, void *stream);
int hg_probe_read(hg_ctx *ctx, const void *buf, uint64_t len, double *gbps, void *stream);
int hg_timing_intervals(hg_ctx *ctx, int kernel_class, double *start_ms, double *end_ms, uint64_t capacity,
                        uint64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* HASHGPU_H */
