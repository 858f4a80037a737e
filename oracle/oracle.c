/*
 * oracle.c -- plain, single-threaded CPU reference for the HashGPU hashing
 * path ("GPUs as Storage System Accelerators", Al-Kiswany, Gharaibeh,
 * Ripeanu).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or constant with the GPU library: the MD5 sine table
 * and the SHA-1 round constants are derived here from their defining formulas
 * at first use, and every routine is written for clarity, not speed.
 *
 * What it computes (each function names the passage it follows):
 *   - MD5 (RFC 1321) and SHA-1 (FIPS 180-4): the sequential Merkle-Damgard
 *     hashes used as building blocks (paper Sec. 3.2.2, "Direct Hashing";
 *     the paper's experiments use MD5).
 *   - Direct hashing with the parallel Merkle-Damgard construction: split a
 *     block into fixed-size segments, hash each segment, place the segment
 *     digests in one buffer, hash that buffer (Sec. 3.2.2).
 *   - Sliding-window hashing: hash every overlapping window and declare a
 *     boundary where the window hash matches a predefined value (Sec. 2.1
 *     "Content-based chunking"; Sec. 3.2.2).
 *   - Boundary selection with a minimum chunk size (Sec. 3.2.2 last stage on
 *     the host; Sec. 4.3 gives min/max chunk sizes of the system).
 *   - Chunk digests: direct hash of each detected chunk (Fig. 3 legend;
 *     Sec. 3.2.4 "Content-based Chunking Integration").
 *   - Similarity: fraction of the new version's chunks whose hash appears in
 *     the previous version's block-map (Sec. 3.2.1; similarity percentages
 *     of Sec. 4.3).
 *   - The block-map write of a content-addressable store: which chunks of a
 *     write are already held (and need not be stored) and the digests held
 *     afterwards (Sec. 3.2.1).
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   - a short last segment is hashed as-is with standard padding;
 *   - the second level uses the same hash as the segments, two levels only;
 *   - a window digest is the full padded standard hash of the w-byte window;
 *   - the boundary predicate reads the first four digest bytes as a
 *     little-endian 32-bit integer: (u32le(D[0..3]) & mask) == target;
 *   - windows start at multiples of the stride from the buffer start and
 *     never extend past its end;
 *   - a chunk ends right after a matching window (end = start + w); the
 *     greedy rule keeps a candidate end e iff e - last >= min_chunk,
 *     e > last and e < len; the final chunk ends at len.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MD5 0
#define ORACLE_SHA1 1

static uint32_t rotl32(uint32_t x, int s) {
    s &= 31;
    if (s == 0) return x;
    return (x << s) | (x >> (32 - s));
}

static uint32_t load_le32(const uint8_t *p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) |
           ((uint32_t)p[3] << 24);
}

static uint32_t load_be32(const uint8_t *p) {
    return ((uint32_t)p[0] << 24) | ((uint32_t)p[1] << 16) | ((uint32_t)p[2] << 8) |
           (uint32_t)p[3];
}

static void store_le32(uint8_t *p, uint32_t v) {
    p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8);
    p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}

static void store_be32(uint8_t *p, uint32_t v) {
    p[0] = (uint8_t)(v >> 24); p[1] = (uint8_t)(v >> 16);
    p[2] = (uint8_t)(v >> 8); p[3] = (uint8_t)v;
}

/* ------------------------------------------------------------------ MD5 -- */
/* RFC 1321: T[i] = floor(2^32 * |sin(i)|) for i = 1..64 (radians). */
static uint32_t md5_T[64];
static int md5_T_ready = 0;

static void md5_make_table(void) {
    if (md5_T_ready) return;
    for (int i = 0; i < 64; i++)
        md5_T[i] = (uint32_t)floor(4294967296.0 * fabs(sin((double)(i + 1))));
    md5_T_ready = 1;
}

/* Per-round rotation amounts, RFC 1321 section 3.4. */
static const int md5_rot[4][4] = {
    {7, 12, 17, 22}, {5, 9, 14, 20}, {4, 11, 16, 23}, {6, 10, 15, 21}};

/* One MD5 compression of a 64-byte block into the state (a, b, c, d). */
static void md5_compress(uint32_t st[4], const uint8_t block[64]) {
    uint32_t X[16];
    for (int j = 0; j < 16; j++) X[j] = load_le32(block + 4 * j);
    uint32_t a = st[0], b = st[1], c = st[2], d = st[3];
    for (int i = 0; i < 64; i++) {
        int round = i / 16;
        uint32_t f;
        int k;
        if (round == 0) {        /* F(X,Y,Z) = XY v not(X) Z */
            f = (b & c) | (~b & d);
            k = i;
        } else if (round == 1) { /* G(X,Y,Z) = XZ v Y not(Z) */
            f = (b & d) | (c & ~d);
            k = (1 + 5 * i) % 16;
        } else if (round == 2) { /* H(X,Y,Z) = X xor Y xor Z */
            f = b ^ c ^ d;
            k = (5 + 3 * i) % 16;
        } else {                 /* I(X,Y,Z) = Y xor (X v not(Z)) */
            f = c ^ (b | ~d);
            k = (7 * i) % 16;
        }
        uint32_t t = a + f + X[k] + md5_T[i];
        a = d;
        d = c;
        c = b;
        b = b + rotl32(t, md5_rot[round][i % 4]);
    }
    st[0] += a; st[1] += b; st[2] += c; st[3] += d;
}

/* ---------------------------------------------------------------- SHA-1 -- */
/* FIPS 180-4: the four round constants are floor(2^30 * sqrt(n)) for
 * n = 2, 3, 5, 10. */
static uint32_t sha1_K[4];
static int sha1_K_ready = 0;

static void sha1_make_constants(void) {
    if (sha1_K_ready) return;
    const double n[4] = {2.0, 3.0, 5.0, 10.0};
    for (int i = 0; i < 4; i++) sha1_K[i] = (uint32_t)floor(1073741824.0 * sqrt(n[i]));
    sha1_K_ready = 1;
}

static void sha1_compress(uint32_t H[5], const uint8_t block[64]) {
    uint32_t W[80];
    for (int t = 0; t < 16; t++) W[t] = load_be32(block + 4 * t);
    for (int t = 16; t < 80; t++) W[t] = rotl32(W[t - 3] ^ W[t - 8] ^ W[t - 14] ^ W[t - 16], 1);
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4];
    for (int t = 0; t < 80; t++) {
        uint32_t f;
        if (t < 20)
            f = (b & c) ^ (~b & d);            /* Ch */
        else if (t < 40 || t >= 60)
            f = b ^ c ^ d;                     /* Parity */
        else
            f = (b & c) ^ (b & d) ^ (c & d);   /* Maj */
        uint32_t T = rotl32(a, 5) + f + e + sha1_K[t / 20] + W[t];
        e = d;
        d = c;
        c = rotl32(b, 30);
        b = a;
        a = T;
    }
    H[0] += a; H[1] += b; H[2] += c; H[3] += d; H[4] += e;
}

/* Builds both constant tables; the loader calls it once before any use, so
 * later calls from several threads only read them. */
void oracle_init(void) {
    md5_make_table();
    sha1_make_constants();
}

/* ------------------------------------------------- generic whole message -- */
int oracle_digest_size(int kind) {
    if (kind == ORACLE_MD5) return 16;
    if (kind == ORACLE_SHA1) return 20;
    return -1;
}

/* Standard Merkle-Damgard message processing with the length padding of both
 * standards: append 0x80, zero-fill to 56 mod 64, append the 64-bit message
 * length in bits (little-endian for MD5, big-endian for SHA-1). */
int oracle_hash(int kind, const uint8_t *msg, uint64_t len, uint8_t *out) {
    uint32_t st[5];
    if (kind == ORACLE_MD5) {
        md5_make_table();
        st[0] = 0x67452301u; st[1] = 0xefcdab89u; st[2] = 0x98badcfeu; st[3] = 0x10325476u;
    } else if (kind == ORACLE_SHA1) {
        sha1_make_constants();
        st[0] = 0x67452301u; st[1] = 0xefcdab89u; st[2] = 0x98badcfeu; st[3] = 0x10325476u;
        st[4] = 0xc3d2e1f0u;
    } else {
        return -1;
    }
    uint64_t full = len / 64;
    for (uint64_t blk = 0; blk < full; blk++) {
        if (kind == ORACLE_MD5) md5_compress(st, msg + 64 * blk);
        else sha1_compress(st, msg + 64 * blk);
    }
    uint8_t tail[128];
    memset(tail, 0, sizeof tail);
    uint64_t rem = len - 64 * full;
    if (rem) memcpy(tail, msg + 64 * full, (size_t)rem);
    tail[rem] = 0x80;
    int nblk = rem < 56 ? 1 : 2;
    uint64_t bits = len * 8u;
    uint8_t *lenp = tail + 64 * nblk - 8;
    for (int j = 0; j < 8; j++) {
        if (kind == ORACLE_MD5) lenp[j] = (uint8_t)(bits >> (8 * j));
        else lenp[7 - j] = (uint8_t)(bits >> (8 * j));
    }
    for (int blk = 0; blk < nblk; blk++) {
        if (kind == ORACLE_MD5) md5_compress(st, tail + 64 * blk);
        else sha1_compress(st, tail + 64 * blk);
    }
    if (kind == ORACLE_MD5) {
        for (int j = 0; j < 4; j++) store_le32(out + 4 * j, st[j]);
    } else {
        for (int j = 0; j < 5; j++) store_be32(out + 4 * j, st[j]);
    }
    return 0;
}

/* ------------------------------------------------------- direct hashing -- */
/* Number of fixed-size segments of a len-byte block: ceil(len / B), 0 for an
 * empty block. */
uint64_t oracle_leaf_count(uint64_t len, uint64_t block) {
    if (block == 0 || len == 0) return 0;
    return (len + block - 1) / block;
}

/* Segment digests of the parallel Merkle-Damgard construction (Sec. 3.2.2):
 * segment k covers [k*B, min((k+1)*B, len)); digests are written in segment
 * order into one buffer of leaf_count * d bytes. Segments [k0, k1) only. */
int oracle_leaves_range(int kind, const uint8_t *in, uint64_t len, uint64_t block,
                        uint64_t k0, uint64_t k1, uint8_t *out) {
    int d = oracle_digest_size(kind);
    if (d < 0 || block == 0) return -1;
    uint64_t n = oracle_leaf_count(len, block);
    if (k1 > n) k1 = n;
    for (uint64_t k = k0; k < k1; k++) {
        uint64_t start = k * block;
        uint64_t end = start + block < len ? start + block : len;
        oracle_hash(kind, in + start, end - start, out + (k - k0) * (uint64_t)d);
    }
    return 0;
}

int oracle_leaves(int kind, const uint8_t *in, uint64_t len, uint64_t block, uint8_t *out) {
    return oracle_leaves_range(kind, in, len, block, 0, oracle_leaf_count(len, block), out);
}

/* Second level: the segment-digest buffer is itself hashed (Sec. 3.2.2). */
int oracle_root(int kind, const uint8_t *leaves, uint64_t n, uint8_t *out) {
    int d = oracle_digest_size(kind);
    if (d < 0) return -1;
    return oracle_hash(kind, leaves, n * (uint64_t)d, out);
}

/* ----------------------------------------------- sliding-window hashing -- */
uint64_t oracle_window_count(uint64_t len, uint64_t w, uint64_t s) {
    if (w == 0 || s == 0 || len < w) return 0;
    return (len - w) / s + 1;
}

/* Brute force over windows k in [k0, k1): window k starts at i = k*s and
 * covers [i, i+w).  Its digest D is the full standard hash of those w bytes;
 * the window is a boundary candidate iff (u32le(D[0..3]) & mask) == target
 * (Sec. 2.1: "declaring a block boundary when the hash value matches a
 * predefined value").  Writes up to cap candidate start offsets in ascending
 * order and returns how many candidates exist in the range. */
uint64_t oracle_window_scan_range(int kind, const uint8_t *in, uint64_t len, uint64_t w,
                                  uint64_t s, uint32_t mask, uint32_t target, uint64_t k0,
                                  uint64_t k1, uint64_t *starts, uint64_t cap) {
    uint64_t nwin = oracle_window_count(len, w, s);
    if (k1 > nwin) k1 = nwin;
    uint8_t D[20];
    uint64_t found = 0;
    for (uint64_t k = k0; k < k1; k++) {
        uint64_t i = k * s;
        oracle_hash(kind, in + i, w, D);
        if ((load_le32(D) & mask) == target) {
            if (found < cap) starts[found] = i;
            found++;
        }
    }
    return found;
}

uint64_t oracle_window_scan(int kind, const uint8_t *in, uint64_t len, uint64_t w, uint64_t s,
                            uint32_t mask, uint32_t target, uint64_t *starts, uint64_t cap) {
    return oracle_window_scan_range(kind, in, len, w, s, mask, target, 0,
                                    oracle_window_count(len, w, s), starts, cap);
}

/* Greedy boundary decision over ascending candidate starts: a candidate ends
 * a chunk at e = start + w; it is taken iff e > last, e - last >= min_chunk
 * and e < len; the final chunk ends at len.  An empty block has no chunks.
 * Returns the number of chunk ends; writes up to cap of them. */
uint64_t oracle_chunk_select(const uint64_t *starts, uint64_t n, uint64_t w, uint64_t len,
                             uint64_t min_chunk, uint64_t *ends, uint64_t cap) {
    uint64_t last = 0, m = 0;
    if (len == 0) return 0;
    for (uint64_t j = 0; j < n; j++) {
        uint64_t e = starts[j] + w;
        if (e > last && e - last >= min_chunk && e < len) {
            if (m < cap) ends[m] = e;
            m++;
            last = e;
        }
    }
    if (m < cap) ends[m] = len;
    m++;
    return m;
}

/* Boundary decision with a minimum and a maximum chunk size (Sec. 4.3 names
 * both as system parameters; the reading here: the maximum is kept by forced
 * cuts).  step = max(min_chunk, 1).  From the previous cut `last`, the next
 * natural cut is the first candidate end e = start + w with e >= last + step
 * and e < len (or, when there is none, the end of the block).  If that lies
 * more than max_chunk past `last`, a cut is forced at last + max_chunk and
 * the search starts again from there; otherwise the natural cut is taken.
 * The final chunk ends at len.  max_chunk = 0: no maximum (the same result as
 * oracle_chunk_select).  Returns the number of chunk ends (writes up to cap),
 * or UINT64_MAX when 0 < max_chunk < step. */
uint64_t oracle_chunk_select_max(const uint64_t *starts, uint64_t n, uint64_t w, uint64_t len,
                                 uint64_t min_chunk, uint64_t max_chunk, uint64_t *ends, uint64_t cap) {
    const uint64_t step = min_chunk > 0 ? min_chunk : 1;
    uint64_t last = 0, m = 0, j = 0;
    if (max_chunk != 0 && max_chunk < step) return UINT64_MAX;
    if (len == 0) return 0;
    for (;;) {
        while (j < n && starts[j] + w < last + step) j++;
        const int natural = j < n && starts[j] + w < len;
        const uint64_t next = natural ? starts[j] + w : len;
        if (max_chunk != 0 && next - last > max_chunk) {
            last += max_chunk;
            if (m < cap) ends[m] = last;
            m++;
            continue;
        }
        if (!natural) break;
        if (m < cap) ends[m] = next;
        m++;
        last = next;
        j++;
    }
    if (m < cap) ends[m] = len;
    m++;
    return m;
}

/* Direct hash of every chunk [ends[j-1], ends[j]) with ends[-1] = 0. */
int oracle_chunk_digests(int kind, const uint8_t *in, const uint64_t *ends, uint64_t n,
                         uint8_t *out) {
    int d = oracle_digest_size(kind);
    if (d < 0) return -1;
    uint64_t start = 0;
    for (uint64_t j = 0; j < n; j++) {
        oracle_hash(kind, in + start, ends[j] - start, out + j * (uint64_t)d);
        start = ends[j];
    }
    return 0;
}

/* ------------------------------------------------------------ similarity -- */
static int cmp_md5(const void *x, const void *y) { return memcmp(x, y, 16); }
static int cmp_sha1(const void *x, const void *y) { return memcmp(x, y, 20); }

/* Counts the chunks of version B (with multiplicity) whose digest appears
 * among version A's digests; if len_b is given, also sums their lengths. The
 * set lookup sorts a copy of A's digests and binary-searches each B digest. */
uint64_t oracle_similarity(int kind, const uint8_t *dig_a, uint64_t n_a, const uint8_t *dig_b,
                           const uint64_t *len_b, uint64_t n_b, uint64_t *matched_bytes) {
    int d = oracle_digest_size(kind);
    if (d < 0) return 0;
    uint8_t *sorted = NULL;
    if (n_a) {
        sorted = (uint8_t *)malloc((size_t)(n_a * (uint64_t)d));
        if (!sorted) return 0;
        memcpy(sorted, dig_a, (size_t)(n_a * (uint64_t)d));
        qsort(sorted, (size_t)n_a, (size_t)d, d == 16 ? cmp_md5 : cmp_sha1);
    }
    uint64_t matched = 0, bytes = 0;
    for (uint64_t j = 0; j < n_b; j++) {
        if (n_a && bsearch(dig_b + j * (uint64_t)d, sorted, (size_t)n_a, (size_t)d,
                           d == 16 ? cmp_md5 : cmp_sha1)) {
            matched++;
            if (len_b) bytes += len_b[j];
        }
    }
    free(sorted);
    if (matched_bytes) *matched_bytes = bytes;
    return matched;
}

/* ------------------------------------------------------------- block map -- */
/* The block-map of a content-addressable store (Sec. 3.2.1): data written to
 * the store is cut into chunks named by their digests, the block-map holds
 * the digests of every chunk stored so far, and a chunk whose digest is
 * already held is not stored again.  A write hands over n chunk digests in
 * order; chunk i is a duplicate iff its digest is held when its turn comes,
 * i.e. it was stored by an earlier write or it equals an earlier chunk j < i
 * of the same write (chunk j's digest is held from then on, whether j was
 * stored or was itself a duplicate).  Every other chunk is stored and its
 * digest added.  The held digests are kept as a sorted array; membership is
 * a binary search.  Capacity is a limit of the interface, not of the paper:
 * a write that could exceed it (size + n > capacity) is refused and changes
 * nothing. */
typedef struct {
    int kind, d;
    uint64_t capacity, n;
    uint8_t *dig; /* n sorted digests */
} oracle_blockmap;

typedef struct {
    uint8_t dig[20];
    uint64_t idx;
} bm_rec;

/* Records in digest order; equal digests in chunk order.  An MD5 digest
 * fills the first 16 bytes and the rest are zero, so comparing all 20
 * bytes orders both digest sizes. */
static int bm_cmp_rec(const void *x, const void *y) {
    const bm_rec *a = (const bm_rec *)x, *b = (const bm_rec *)y;
    int c = memcmp(a->dig, b->dig, sizeof a->dig);
    if (c) return c;
    return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

oracle_blockmap *oracle_blockmap_create(int kind, uint64_t capacity) {
    int d = oracle_digest_size(kind);
    if (d < 0) return NULL;
    oracle_blockmap *m = (oracle_blockmap *)calloc(1, sizeof *m);
    if (!m) return NULL;
    m->kind = kind;
    m->d = d;
    m->capacity = capacity;
    return m;
}

void oracle_blockmap_destroy(oracle_blockmap *m) {
    if (!m) return;
    free(m->dig);
    free(m);
}

uint64_t oracle_blockmap_size(const oracle_blockmap *m) { return m ? m->n : 0; }

/* One write: dig holds n digests (chunk order), len their lengths (or NULL).
 * is_dup (n bytes, may be NULL) receives 1 for a duplicate, 0 for a stored
 * chunk; *dup_chunks / *dup_bytes the number of duplicates and the sum of
 * their lengths.  Returns 0, -1 for bad arguments, -5 when refused for
 * capacity. */
int oracle_blockmap_write(oracle_blockmap *m, const uint8_t *dig, const uint64_t *len, uint64_t n,
                          uint8_t *is_dup, uint64_t *dup_chunks, uint64_t *dup_bytes) {
    if (!m || (n && !dig)) return -1;
    if (m->n + n > m->capacity) return -5;
    const int d = m->d;
    uint64_t count = 0, bytes = 0, added = 0;
    bm_rec *r = NULL;
    uint8_t *dup = NULL, *grown = NULL;
    if (n) {
        r = (bm_rec *)malloc((size_t)n * sizeof *r);
        dup = (uint8_t *)malloc((size_t)n);
        grown = (uint8_t *)realloc(m->dig, (size_t)((m->n + n) * (uint64_t)d));
        if (!r || !dup || !grown) {
            free(r);
            free(dup);
            if (grown) m->dig = grown;
            return -1;
        }
        m->dig = grown;
    }
    for (uint64_t i = 0; i < n; i++) {
        memset(r[i].dig, 0, sizeof r[i].dig);
        memcpy(r[i].dig, dig + i * (uint64_t)d, (size_t)d);
        r[i].idx = i;
    }
    if (n) qsort(r, (size_t)n, sizeof *r, bm_cmp_rec);
    for (uint64_t k = 0; k < n; k++) {
        const uint64_t i = r[k].idx;
        const int repeat = k > 0 && memcmp(r[k - 1].dig, r[k].dig, (size_t)d) == 0;
        const int held = m->n && bsearch(r[k].dig, m->dig, (size_t)m->n, (size_t)d,
                                         d == 16 ? cmp_md5 : cmp_sha1) != NULL;
        dup[i] = (uint8_t)(repeat || held);
    }
    for (uint64_t i = 0; i < n; i++) {
        if (dup[i]) {
            count++;
            if (len) bytes += len[i];
        } else {
            memcpy(m->dig + (m->n + added) * (uint64_t)d, dig + i * (uint64_t)d, (size_t)d);
            added++;
        }
    }
    m->n += added;
    if (m->n) qsort(m->dig, (size_t)m->n, (size_t)d, d == 16 ? cmp_md5 : cmp_sha1);
    if (is_dup && n) memcpy(is_dup, dup, (size_t)n);
    if (dup_chunks) *dup_chunks = count;
    if (dup_bytes) *dup_bytes = bytes;
    free(r);
    free(dup);
    return 0;
}
