/*
 * Exact frequent-k-mer oracle.  TEST INFRASTRUCTURE ONLY: the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load this library;
 * the GPU product path never calls it, and it shares no code with it.
 *
 * Plain, slow, obviously-correct C following Roy, Bhattacharya & Schliep,
 * "Turtle: identifying frequent k-mers with cache-efficient algorithms"
 * (arXiv 1305.1861):
 *
 *  - §2.1 "k-mer extraction and bit-encoding": k-mers are taken only from
 *    stretches of A/C/G/T (reads are cut at ambiguous calls), each base is
 *    two bits, and a k-mer and its reverse complement are the same object,
 *    represented by whichever encoding is numerically smaller.
 *  - §2.1 "Counting frequencies with sorting and compaction" (and Fig. 1):
 *    items are sorted by k-mer value so equal k-mers become neighbours, and
 *    one linear pass folds each run of equal k-mers into a single item whose
 *    count is the run length (run-length encoding).
 *  - Algorithm 1 (scTurtle outline), final step: report the k-mers that
 *    survive with their counts.
 *  - §3: 64-bit keys for short k, 128-bit keys for long k.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *  - base codes A=0, C=1, G=2, T=3, first base most significant, so numeric
 *    order of codes is lexicographic order of strings; complement = 3 - code;
 *  - upper and lower case ACGT are bases; every other byte breaks windows;
 *  - windows never span two reads; a read shorter than k has no window;
 *  - k in [1, 63]; k <= 31 gives a one-word key, 32..63 a two-word key;
 *  - output: every distinct canonical k-mer whose TRUE count is >= c, in
 *    ascending key order, with that count (the paper's "+1" correction of
 *    §2.1 is replaced by exact counting);
 *  - functions marked "Bloom model" follow the pattern-blocked Bloom filter of
 *    §2.1 ("Identification of frequent k-mers with Pattern-blocked Bloom
 *    Filter") with per-bit two-plane semantics: a bit of the second plane is
 *    set iff its position in the first plane was touched at least twice.
 *
 * All keys are held as unsigned __int128 regardless of k (the top bits are
 * zero for short k).  Sorting uses the C library qsort.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ECAP (-3)

/* Base code of one byte, or -1 if the byte is not a base (§2.1 extraction). */
static int base_code(uint8_t b)
{
    switch (b) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

/*
 * Canonical key of the k bases at s (§2.1 extraction): the forward encoding
 * and the encoding of the reverse complement, each with its first base most
 * significant; the smaller one is the key.  Returns 0 if some byte of the
 * window is not a base.
 */
static int window_key(const uint8_t *s, int k, u128 *key)
{
    u128 fwd = 0, rc = 0;
    for (int j = 0; j < k; j++) {
        int c = base_code(s[j]);
        if (c < 0)
            return 0;
        fwd = (fwd << 2) | (u128)c;
    }
    /* reverse complement: read the window backwards, complementing */
    for (int j = k - 1; j >= 0; j--)
        rc = (rc << 2) | (u128)(3 - base_code(s[j]));
    *key = fwd < rc ? fwd : rc;
    return 1;
}

static int cmp_u128(const void *a, const void *b)
{
    u128 x = *(const u128 *)a, y = *(const u128 *)b;
    return (x > y) - (x < y);
}

static int check_args(const uint64_t *offsets, uint64_t n_reads, int k)
{
    if (k < 1 || k > 63 || offsets == NULL)
        return OR_EINVAL;
    for (uint64_t r = 0; r < n_reads; r++)
        if (offsets[r + 1] < offsets[r])
            return OR_EINVAL;
    return OR_OK;
}

/*
 * Every valid window's canonical key, in read order then position order.
 * *keys_out is malloc'ed (may be NULL when there is no window).
 */
static int enumerate_keys(const uint8_t *bases, const uint64_t *offsets,
                          uint64_t n_reads, int k, u128 **keys_out,
                          uint64_t *n_out)
{
    uint64_t cap = 0;
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t len = offsets[r + 1] - offsets[r];
        if (len >= (uint64_t)k)
            cap += len - (uint64_t)k + 1;
    }
    u128 *keys = cap ? (u128 *)malloc(cap * sizeof(u128)) : NULL;
    if (cap && !keys)
        return OR_ENOMEM;
    uint64_t n = 0;
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t lo = offsets[r], hi = offsets[r + 1];
        if (hi - lo < (uint64_t)k)
            continue;
        for (uint64_t i = lo; i + (uint64_t)k <= hi; i++) {
            u128 key;
            if (window_key(bases + i, k, &key))
                keys[n++] = key;
        }
    }
    *keys_out = keys;
    *n_out = n;
    return OR_OK;
}

/*
 * Sort-and-compact (§2.1, Fig. 1): sort the items by key, then fold each run
 * of equal keys into one (key, run length) pair.  Operates in place: on
 * return keys[0..*n_runs) hold the distinct keys in ascending order and
 * counts[0..*n_runs) their run lengths.
 */
static void sort_and_compact(u128 *keys, uint64_t n, uint64_t *counts,
                             uint64_t *n_runs)
{
    if (n == 0) {
        *n_runs = 0;
        return;
    }
    qsort(keys, n, sizeof(u128), cmp_u128);
    uint64_t r = 0;
    counts[0] = 1;
    for (uint64_t i = 1; i < n; i++) {
        if (keys[i] == keys[r]) {
            counts[r] += 1;
        } else {
            r += 1;
            keys[r] = keys[i];
            counts[r] = 1;
        }
    }
    *n_runs = r + 1;
}

/* Number of valid k-mer windows (windows of k bases inside one read). */
int64_t oracle_count_windows(const uint8_t *bases, const uint64_t *offsets,
                             uint64_t n_reads, int k)
{
    if (check_args(offsets, n_reads, k) != OR_OK)
        return OR_EINVAL;
    int64_t n = 0;
    for (uint64_t r = 0; r < n_reads; r++) {
        uint64_t lo = offsets[r], hi = offsets[r + 1];
        for (uint64_t i = lo; i + (uint64_t)k <= hi; i++) {
            u128 key;
            n += window_key(bases + i, k, &key);
        }
    }
    return n;
}

/*
 * Sort-and-compact over explicit items (§2.1): keys given as (hi, lo) words.
 * Writes the distinct keys ascending and their multiplicities; returns the
 * number of distinct keys or a negative status.
 */
int64_t oracle_sort_compact(const uint64_t *in_hi, const uint64_t *in_lo,
                            uint64_t n, uint64_t *out_hi, uint64_t *out_lo,
                            uint64_t *out_count)
{
    u128 *keys = n ? (u128 *)malloc(n * sizeof(u128)) : NULL;
    uint64_t *counts = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (n && (!keys || !counts)) {
        free(keys);
        free(counts);
        return OR_ENOMEM;
    }
    for (uint64_t i = 0; i < n; i++)
        keys[i] = ((u128)in_hi[i] << 64) | in_lo[i];
    uint64_t runs = 0;
    sort_and_compact(keys, n, counts, &runs);
    for (uint64_t i = 0; i < runs; i++) {
        out_hi[i] = (uint64_t)(keys[i] >> 64);
        out_lo[i] = (uint64_t)keys[i];
        out_count[i] = counts[i];
    }
    free(keys);
    free(counts);
    return (int64_t)runs;
}

/*
 * The exact answer: every canonical k-mer with count >= c, ascending, with
 * its count.  Output arrays hold `capacity` entries; returns the number of
 * entries written, OR_ECAP if they do not fit, or another negative status.
 * *n_windows receives the number of valid windows and *n_distinct the number
 * of distinct canonical k-mers.
 */
int64_t oracle_kmer_count(const uint8_t *bases, const uint64_t *offsets,
                          uint64_t n_reads, int k, uint64_t c,
                          uint64_t *out_hi, uint64_t *out_lo,
                          uint64_t *out_count, uint64_t capacity,
                          uint64_t *n_windows, uint64_t *n_distinct)
{
    int st = check_args(offsets, n_reads, k);
    if (st != OR_OK || c == 0)
        return OR_EINVAL;
    u128 *keys = NULL;
    uint64_t n = 0;
    st = enumerate_keys(bases, offsets, n_reads, k, &keys, &n);
    if (st != OR_OK)
        return st;
    uint64_t *counts = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (n && !counts) {
        free(keys);
        return OR_ENOMEM;
    }
    uint64_t runs = 0;
    sort_and_compact(keys, n, counts, &runs);
    uint64_t m = 0;
    for (uint64_t i = 0; i < runs; i++) {
        if (counts[i] < c)
            continue;
        if (m >= capacity) {
            free(keys);
            free(counts);
            return OR_ECAP;
        }
        out_hi[m] = (uint64_t)(keys[i] >> 64);
        out_lo[m] = (uint64_t)keys[i];
        out_count[m] = counts[i];
        m++;
    }
    *n_windows = n;
    *n_distinct = runs;
    free(keys);
    free(counts);
    return (int64_t)m;
}

/*
 * The canonical keys of every window whose key lies in one range of the key
 * space, for libraries too large to hold all their keys at once: range r of
 * 2^range_bits is the set of keys whose top range_bits bits (of the 2k-bit
 * value) equal r.  The ranges are ordered like the keys, so the exact answer
 * of a library is the concatenation, in range order, of the sort-and-compact
 * of each range's keys.  Occurrences come in read order then position
 * order.  *hi and *lo receive malloc'ed arrays of *n entries (NULL when
 * there are none); release them with oracle_free.
 */
int oracle_keys_in_range(const uint8_t *bases, const uint64_t *offsets,
                         uint64_t n_reads, int k, int range_bits,
                         uint64_t range_index, uint64_t **hi, uint64_t **lo,
                         uint64_t *n)
{
    if (check_args(offsets, n_reads, k) != OR_OK || range_bits < 0 ||
        range_bits > 2 * k || range_bits > 16 ||
        range_index >= ((uint64_t)1 << range_bits) || !hi || !lo || !n)
        return OR_EINVAL;
    uint64_t cap = 0, m = 0;
    uint64_t *h = NULL, *l = NULL;
    for (uint64_t r = 0; r < n_reads; r++) {
        for (uint64_t i = offsets[r]; i + (uint64_t)k <= offsets[r + 1]; i++) {
            u128 key;
            if (!window_key(bases + i, k, &key))
                continue;
            if (range_bits && (uint64_t)(key >> (2 * k - range_bits)) != range_index)
                continue;
            if (m == cap) {
                uint64_t nc = cap ? 2 * cap : 4096;
                uint64_t *nh = (uint64_t *)realloc(h, nc * sizeof(uint64_t));
                if (nh)
                    h = nh;
                uint64_t *nl = nh ? (uint64_t *)realloc(l, nc * sizeof(uint64_t)) : NULL;
                if (!nh || !nl) {
                    free(h);
                    free(l);
                    return OR_ENOMEM;
                }
                l = nl;
                cap = nc;
            }
            h[m] = (uint64_t)(key >> 64);
            l[m] = (uint64_t)key;
            m++;
        }
    }
    *hi = h;
    *lo = l;
    *n = m;
    return OR_OK;
}

void oracle_free(void *p)
{
    free(p);
}

/*
 * Exact counts of chosen keys over all windows of a library, for checking
 * sampled outputs of very large runs.  `q_hi`/`q_lo` must be sorted
 * ascending by (hi, lo) and distinct; counts[i] receives the number of
 * windows whose canonical key equals query i.  The scan over reads may use
 * several threads (each keeps private counts), `n_threads` <= 0 meaning one.
 */
int oracle_count_queries(const uint8_t *bases, const uint64_t *offsets,
                         uint64_t n_reads, int k, const uint64_t *q_hi,
                         const uint64_t *q_lo, uint64_t n_q, uint64_t *counts,
                         int n_threads)
{
    if (check_args(offsets, n_reads, k) != OR_OK)
        return OR_EINVAL;
    u128 *q = n_q ? (u128 *)malloc(n_q * sizeof(u128)) : NULL;
    if (n_q && !q)
        return OR_ENOMEM;
    for (uint64_t i = 0; i < n_q; i++) {
        q[i] = ((u128)q_hi[i] << 64) | q_lo[i];
        counts[i] = 0;
    }
    if (n_threads < 1)
        n_threads = 1;
    uint64_t *priv = (uint64_t *)calloc((size_t)n_threads * (n_q ? n_q : 1),
                                        sizeof(uint64_t));
    if (!priv) {
        free(q);
        return OR_ENOMEM;
    }
#pragma omp parallel for num_threads(n_threads) schedule(dynamic, 4096)
    for (int64_t r = 0; r < (int64_t)n_reads; r++) {
#ifdef _OPENMP
        uint64_t *mine = priv + (size_t)omp_get_thread_num() * n_q;
#else
        uint64_t *mine = priv;
#endif
        uint64_t lo = offsets[r], hi = offsets[r + 1];
        for (uint64_t i = lo; i + (uint64_t)k <= hi; i++) {
            u128 key;
            if (!window_key(bases + i, k, &key))
                continue;
            /* binary search in the sorted queries */
            uint64_t a = 0, b = n_q;
            while (a < b) {
                uint64_t mid = a + (b - a) / 2;
                if (q[mid] < key)
                    a = mid + 1;
                else
                    b = mid;
            }
            if (a < n_q && q[a] == key)
                mine[a] += 1;
        }
    }
    for (int t = 0; t < n_threads; t++)
        for (uint64_t i = 0; i < n_q; i++)
            counts[i] += priv[(size_t)t * n_q + i];
    free(priv);
    free(q);
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Bloom model: pattern-blocked Bloom filter of §2.1 with two planes.
 *
 * The filter is n_blocks blocks; a block has a 256-bit first plane (S) and a
 * 256-bit second plane (T), each seen as four 64-bit words.  A key picks its
 * block from a 64-bit hash h of the key, block = floor(h * n_blocks / 2^64).
 * Its pattern is multiplexed from one precomputed table of n_patterns
 * entries (n_patterns a power of two, lg = log2(n_patterns)): word w of the
 * block receives table entry (h >> (w * lg)) mod n_patterns, an entry being
 * a set of `n_bits` distinct bit positions in [0, 64).  Every window touches
 * its pattern bits; a T bit holds iff the bit was touched at least twice.
 * A key is a candidate iff all its pattern bits hold in T.
 *
 * Hash: the 64-bit finaliser of MurmurHash3 (Appleby), fmix64; a two-word key
 * hashes as fmix64(lo XOR fmix64(hi)).
 * Pattern table: SplitMix64 (Steele, Lea & Flood 2014) seeded with `seed`;
 * entries are filled in order, each drawing outputs and taking the top six
 * bits as a bit position, skipping repeats, until it has `n_bits` distinct
 * positions.
 * ------------------------------------------------------------------------ */

#define BLOCK_WORDS 4

static uint64_t fmix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static uint64_t key_hash(u128 key, int two_words)
{
    if (!two_words)
        return fmix64((uint64_t)key);
    return fmix64((uint64_t)key ^ fmix64((uint64_t)(key >> 64)));
}

static int log2_exact(uint32_t v)
{
    if (v == 0 || (v & (v - 1)) != 0)
        return -1;
    int lg = 0;
    while ((1u << lg) < v)
        lg++;
    return lg;
}

static int bloom_params_ok(uint64_t n_blocks, uint32_t n_patterns,
                           uint32_t n_bits)
{
    int lg = log2_exact(n_patterns);
    return n_blocks > 0 && lg >= 0 && lg * BLOCK_WORDS <= 64 && n_bits >= 1 &&
           n_bits <= 64;
}

/*
 * Pattern table as bit positions: positions[e * n_bits + j] is the j-th
 * position (in [0, 64)) drawn for entry e, in draw order.
 */
int oracle_pattern_positions(uint64_t seed, uint32_t n_patterns,
                             uint32_t n_bits, uint8_t *positions)
{
    if (n_patterns == 0 || n_bits == 0 || n_bits > 64)
        return OR_EINVAL;
    uint64_t state = seed;
    for (uint32_t e = 0; e < n_patterns; e++) {
        uint32_t have = 0;
        while (have < n_bits) {
            uint8_t p = (uint8_t)(splitmix64_next(&state) >> 58);
            int seen = 0;
            for (uint32_t j = 0; j < have; j++)
                if (positions[(size_t)e * n_bits + j] == p)
                    seen = 1;
            if (!seen)
                positions[(size_t)e * n_bits + have++] = p;
        }
    }
    return OR_OK;
}

/* Block index and the table entry used by each block word (Bloom model). */
int oracle_block_of(uint64_t hi, uint64_t lo, int two_words, uint64_t n_blocks,
                    uint32_t n_patterns, uint64_t *block, uint32_t *entries)
{
    int lg = log2_exact(n_patterns);
    if (n_blocks == 0 || lg < 0 || lg * BLOCK_WORDS > 64)
        return OR_EINVAL;
    uint64_t h = key_hash(((u128)hi << 64) | lo, two_words);
    *block = (uint64_t)(((u128)h * n_blocks) >> 64);
    for (int w = 0; w < BLOCK_WORDS; w++)
        entries[w] = (uint32_t)((h >> (w * lg)) & (n_patterns - 1));
    return OR_OK;
}

/*
 * Bloom model over an explicit multiset of keys (each array entry is one
 * occurrence).  touch[] counts touches per filter bit of the first plane,
 * saturating at 2 (a count of 2 is a set second-plane bit).
 * Outputs: *n_cand_occ = occurrences whose key is a candidate, *n_cand =
 * distinct candidate keys, *n_cand_single = distinct candidates that occur
 * exactly once (false positives of the screen).  When cand_flags is not NULL
 * it receives 1/0 per occurrence.
 */
int oracle_bloom_model_keys(const uint64_t *hi, const uint64_t *lo, uint64_t n,
                            int two_words, uint64_t n_blocks,
                            uint32_t n_patterns, uint32_t n_bits,
                            uint64_t seed, uint64_t *n_cand_occ,
                            uint64_t *n_cand, uint64_t *n_cand_single,
                            uint8_t *cand_flags)
{
    if (!bloom_params_ok(n_blocks, n_patterns, n_bits))
        return OR_EINVAL;
    uint8_t *pos = (uint8_t *)malloc((size_t)n_patterns * n_bits);
    uint8_t *touch = (uint8_t *)calloc((size_t)n_blocks * 64 * BLOCK_WORDS, 1);
    u128 *cand = n ? (u128 *)malloc(n * sizeof(u128)) : NULL;
    uint64_t *cnt = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (!pos || !touch || (n && (!cand || !cnt))) {
        free(pos); free(touch); free(cand); free(cnt);
        return OR_ENOMEM;
    }
    oracle_pattern_positions(seed, n_patterns, n_bits, pos);
    /* screen: every occurrence touches its pattern bits */
    for (uint64_t i = 0; i < n; i++) {
        uint64_t blk;
        uint32_t ent[BLOCK_WORDS];
        oracle_block_of(hi[i], lo[i], two_words, n_blocks, n_patterns, &blk, ent);
        for (int w = 0; w < BLOCK_WORDS; w++)
            for (uint32_t j = 0; j < n_bits; j++) {
                size_t bit = (size_t)w * 64 + pos[(size_t)ent[w] * n_bits + j];
                uint8_t *t = &touch[blk * 64 * BLOCK_WORDS + bit];
                if (*t < 2)
                    *t += 1;
            }
    }
    /* collect: occurrences whose every pattern bit was touched twice */
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t blk;
        uint32_t ent[BLOCK_WORDS];
        oracle_block_of(hi[i], lo[i], two_words, n_blocks, n_patterns, &blk, ent);
        int all = 1;
        for (int w = 0; w < BLOCK_WORDS; w++)
            for (uint32_t j = 0; j < n_bits; j++) {
                size_t bit = (size_t)w * 64 + pos[(size_t)ent[w] * n_bits + j];
                if (touch[blk * 64 * BLOCK_WORDS + bit] < 2)
                    all = 0;
            }
        if (cand_flags)
            cand_flags[i] = (uint8_t)all;
        if (all)
            cand[m++] = ((u128)hi[i] << 64) | lo[i];
    }
    uint64_t runs = 0;
    sort_and_compact(cand, m, cnt, &runs);
    uint64_t single = 0;
    for (uint64_t r = 0; r < runs; r++)
        single += (cnt[r] == 1);
    *n_cand_occ = m;
    *n_cand = runs;
    *n_cand_single = single;
    free(pos); free(touch); free(cand); free(cnt);
    return OR_OK;
}

/*
 * Bloom model over a read library: the windows' canonical keys (in the same
 * enumeration as oracle_kmer_count) fed to oracle_bloom_model_keys.
 */
int oracle_bloom_model(const uint8_t *bases, const uint64_t *offsets,
                       uint64_t n_reads, int k, uint64_t n_blocks,
                       uint32_t n_patterns, uint32_t n_bits, uint64_t seed,
                       uint64_t *n_cand_occ, uint64_t *n_cand,
                       uint64_t *n_cand_single)
{
    int st = check_args(offsets, n_reads, k);
    if (st != OR_OK)
        return st;
    u128 *keys = NULL;
    uint64_t n = 0;
    st = enumerate_keys(bases, offsets, n_reads, k, &keys, &n);
    if (st != OR_OK)
        return st;
    uint64_t *hi = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    uint64_t *lo = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (n && (!hi || !lo)) {
        free(keys); free(hi); free(lo);
        return OR_ENOMEM;
    }
    for (uint64_t i = 0; i < n; i++) {
        hi[i] = (uint64_t)(keys[i] >> 64);
        lo[i] = (uint64_t)keys[i];
    }
    st = oracle_bloom_model_keys(hi, lo, n, k > 31, n_blocks, n_patterns,
                                 n_bits, seed, n_cand_occ, n_cand,
                                 n_cand_single, NULL);
    free(keys); free(hi); free(lo);
    return st;
}

/*
 * Bloom model with one filter per bucket: a key's bucket is the top D bits of
 * its 2k-bit value; bucket s with n_s occurrences has its own two-plane filter
 * of max(1, ceil(beta * n_s / 256)) blocks, used only by the keys of s.  The
 * result is the sum over buckets of oracle_bloom_model_keys.
 */
int oracle_bloom_model_buckets_keys(const uint64_t *hi, const uint64_t *lo,
                                    uint64_t n, int k, int D, uint32_t beta,
                                    uint32_t n_patterns, uint32_t n_bits,
                                    uint64_t seed, uint64_t *n_cand_occ,
                                    uint64_t *n_cand, uint64_t *n_cand_single)
{
    if (k < 1 || k > 63 || D < 0 || D > 2 * k || D > 24 || beta == 0)
        return OR_EINVAL;
    uint64_t n_buckets = (uint64_t)1 << D;
    uint64_t *count = (uint64_t *)calloc(n_buckets + 1, sizeof(uint64_t));
    uint32_t *bucket = n ? (uint32_t *)malloc(n * sizeof(uint32_t)) : NULL;
    uint64_t *order = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    uint64_t *ghi = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    uint64_t *glo = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (!count || (n && (!bucket || !order || !ghi || !glo))) {
        free(count); free(bucket); free(order); free(ghi); free(glo);
        return OR_ENOMEM;
    }
    for (uint64_t i = 0; i < n; i++) {
        u128 key = ((u128)hi[i] << 64) | lo[i];
        bucket[i] = D ? (uint32_t)(key >> (2 * k - D)) : 0;
        count[bucket[i] + 1] += 1;
    }
    /* counting sort of the occurrences by bucket */
    for (uint64_t b = 0; b < n_buckets; b++)
        count[b + 1] += count[b];
    for (uint64_t i = 0; i < n; i++)
        order[count[bucket[i]]++] = i;
    uint64_t start = 0;
    *n_cand_occ = *n_cand = *n_cand_single = 0;
    for (uint64_t b = 0; b < n_buckets; b++) {
        uint64_t end = count[b]; /* after the placement loop count[b] = end of b */
        uint64_t ns = end - start;
        if (ns) {
            for (uint64_t j = 0; j < ns; j++) {
                ghi[j] = hi[order[start + j]];
                glo[j] = lo[order[start + j]];
            }
            uint64_t blocks = ((uint64_t)beta * ns + 255) / 256;
            if (blocks == 0)
                blocks = 1;
            uint64_t a = 0, c = 0, d = 0;
            int st = oracle_bloom_model_keys(ghi, glo, ns, k > 31, blocks, n_patterns,
                                             n_bits, seed, &a, &c, &d, NULL);
            if (st != OR_OK) {
                free(count); free(bucket); free(order); free(ghi); free(glo);
                return st;
            }
            *n_cand_occ += a;
            *n_cand += c;
            *n_cand_single += d;
        }
        start = end;
    }
    free(count); free(bucket); free(order); free(ghi); free(glo);
    return OR_OK;
}

/* The per-bucket Bloom model over the windows of a read library. */
int oracle_bloom_model_buckets(const uint8_t *bases, const uint64_t *offsets,
                               uint64_t n_reads, int k, int D, uint32_t beta,
                               uint32_t n_patterns, uint32_t n_bits,
                               uint64_t seed, uint64_t *n_cand_occ,
                               uint64_t *n_cand, uint64_t *n_cand_single)
{
    int st = check_args(offsets, n_reads, k);
    if (st != OR_OK)
        return st;
    u128 *keys = NULL;
    uint64_t n = 0;
    st = enumerate_keys(bases, offsets, n_reads, k, &keys, &n);
    if (st != OR_OK)
        return st;
    uint64_t *hi = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    uint64_t *lo = n ? (uint64_t *)malloc(n * sizeof(uint64_t)) : NULL;
    if (n && (!hi || !lo)) {
        free(keys); free(hi); free(lo);
        return OR_ENOMEM;
    }
    for (uint64_t i = 0; i < n; i++) {
        hi[i] = (uint64_t)(keys[i] >> 64);
        lo[i] = (uint64_t)keys[i];
    }
    st = oracle_bloom_model_buckets_keys(hi, lo, n, k, D, beta, n_patterns, n_bits,
                                         seed, n_cand_occ, n_cand, n_cand_single);
    free(keys); free(hi); free(lo);
    return st;
}

/*
 * Approximate variants, run sequentially over the windows in read order.
 * The filter is n_words 64-bit words; a key's first pattern is the OR of
 * table entries e0 and e1 (e_w = (h >> (w * lg)) mod P, h the key hash) in
 * word floor(h * n_words / 2^64), its second pattern the OR of e2 and e3 in
 * the next word (word 0 after the last).
 *   mode 1, cTurtle (§2.2): if the first pattern is not all set, set it;
 *     otherwise, if the second pattern is not all set, set it and report the
 *     key.  Output: the reported keys in ascending order, count 0.
 *   mode 2, the single pass of Algorithm 1 as printed (§2.1): if the first
 *     pattern is all set, store the key, else set it.  Output: the stored
 *     keys sorted and compacted, count = run length + 1 (the "+1"), kept
 *     when >= c.
 * *n_reported receives the number of reported (mode 1) or stored (mode 2)
 * sightings.  Returns OR_ECAP when more than `capacity` records result.
 * Pinned: with a filter large enough to have no collisions both modes equal
 * the exact counting above; whatever the collisions, mode 2 counts are the
 * true count or one more and miss no k-mer seen twice, mode 1 reports every
 * key once.  Which keys a colliding filter misreports is parity unpinned:
 * the paper fixes none of the filter's constants.
 */
int oracle_approx(const uint8_t *bases, const uint64_t *offsets,
                  uint64_t n_reads, int k, int mode, uint32_t c,
                  uint64_t n_words, uint32_t n_patterns, uint32_t n_bits,
                  uint64_t seed, uint64_t *out_hi, uint64_t *out_lo,
                  uint64_t *out_count, uint64_t capacity, uint64_t *n_out,
                  uint64_t *n_reported)
{
    int st = check_args(offsets, n_reads, k);
    int lg = log2_exact(n_patterns);
    if (st != OR_OK || (mode != 1 && mode != 2) || n_words == 0 || lg < 0 ||
        lg * BLOCK_WORDS > 64 || n_bits == 0 || n_bits > 64 || c == 0)
        return OR_EINVAL;
    uint8_t *pos = (uint8_t *)malloc((size_t)n_patterns * n_bits);
    uint64_t *mask = (uint64_t *)calloc(n_patterns, sizeof(uint64_t));
    uint64_t *filter = (uint64_t *)calloc(n_words, sizeof(uint64_t));
    u128 *keys = NULL;
    uint64_t n = 0;
    if (!pos || !mask || !filter) {
        free(pos); free(mask); free(filter);
        return OR_ENOMEM;
    }
    oracle_pattern_positions(seed, n_patterns, n_bits, pos);
    for (uint32_t e = 0; e < n_patterns; e++)
        for (uint32_t j = 0; j < n_bits; j++)
            mask[e] |= 1ull << pos[(size_t)e * n_bits + j];
    free(pos);
    st = enumerate_keys(bases, offsets, n_reads, k, &keys, &n);
    if (st != OR_OK) {
        free(mask); free(filter);
        return st;
    }
    const int two = k > 31;
    uint64_t kept = 0;  /* keys[0..kept) are the reported or stored sightings */
    for (uint64_t i = 0; i < n; i++) {
        uint64_t h = key_hash(keys[i], two);
        uint64_t w1 = (uint64_t)(((u128)h * n_words) >> 64);
        uint64_t m1 = mask[h & (n_patterns - 1)] | mask[(h >> lg) & (n_patterns - 1)];
        int seen = (filter[w1] & m1) == m1;
        filter[w1] |= m1;
        if (!seen)
            continue;
        if (mode == 2) {
            keys[kept++] = keys[i];
            continue;
        }
        uint64_t w2 = w1 + 1 < n_words ? w1 + 1 : 0;
        uint64_t m2 = mask[(h >> (2 * lg)) & (n_patterns - 1)] |
                      mask[(h >> (3 * lg)) & (n_patterns - 1)];
        int done = (filter[w2] & m2) == m2;
        filter[w2] |= m2;
        if (!done)
            keys[kept++] = keys[i];
    }
    *n_reported = kept;
    free(mask);
    free(filter);
    uint64_t *runs = kept ? (uint64_t *)malloc(kept * sizeof(uint64_t)) : NULL;
    if (kept && !runs) {
        free(keys);
        return OR_ENOMEM;
    }
    uint64_t n_runs = 0;
    sort_and_compact(keys, kept, runs, &n_runs);
    uint64_t o = 0;
    for (uint64_t r = 0; r < n_runs; r++) {
        uint64_t cnt = mode == 1 ? 0 : runs[r] + 1;
        if (mode == 2 && cnt < c)
            continue;
        if (o >= capacity) {
            free(keys); free(runs);
            return OR_ECAP;
        }
        out_hi[o] = (uint64_t)(keys[r] >> 64);
        out_lo[o] = (uint64_t)keys[r];
        out_count[o] = cnt;
        o++;
    }
    *n_out = o;
    free(keys);
    free(runs);
    return OR_OK;
}
