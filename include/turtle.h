/*
 * turtle.h -- exact frequent-k-mer counting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libturtle.so.  Every entry point returns a tk_status; errors are
 * returned, never thrown or aborted, and outputs are left untouched on
 * error.  A thread-local message with details is available from
 * tk_last_error().  Calls are reentrant; calls that share a workspace or a
 * stream are ordered by that stream.
 *
 * The method is the exact-count path of Roy, Bhattacharya & Schliep, "Turtle:
 * identifying frequent k-mers with cache-efficient algorithms" (arXiv
 * 1305.1861), §2.1:
 *   1. k-mers are extracted from the reads, 2 bits per base, cut at every
 *      byte that is not A/C/G/T (upper or lower case), never across reads;
 *      a k-mer and its reverse complement are one object represented by the
 *      numerically smaller encoding ("k-mer extraction and bit-encoding");
 *   2. a pattern-blocked Bloom filter screens out k-mers seen only once
 *      ("Identification of frequent k-mers with Pattern-blocked Bloom
 *      Filter");
 *   3. the surviving occurrences are counted by sorting and run-length
 *      compaction instead of a hash table ("Counting frequencies with sorting
 *      and compaction", Fig. 1, Algorithm 1).
 *
 * Result contract (bit-exact): every canonical k-mer whose TRUE number of
 * occurrences is >= c, in ascending key order, with that number.  Keys:
 *   - base codes A=0, C=1, G=2, T=3, first base most significant, so the
 *     numeric order of keys is the lexicographic order of the k-mers;
 *   - k in [1, 31]: one 64-bit word per key (key_words = 1);
 *   - k in [32, 63]: two 64-bit words per key stored {hi, lo} (key_words =
 *     2), ordered by (hi, lo).
 * Counts are exact even for keys the Bloom screen let through by mistake:
 * every occurrence of a candidate key is collected, so a false positive shows
 * up with its true count 1 and is dropped (and counted in n_singletons).
 * This replaces the paper's "+1" correction of §2.1, which assumes a key's
 * first sighting was never a false positive.
 *
 * Bloom screen (used when c >= 2; c = 1 counts every window directly):
 *   - buckets (default, partitioned path): the windows are grouped by the top
 *     D bits of their key (2k-bit value) and every bucket has a filter of its
 *     own, sized from its own number of windows n_s:
 *     n_blocks = max(1, ceil(bloom_beta * n_s / 256)).  D follows the size
 *     rule: W = max(n_bases - n_reads * (k - 1), 1), L = ceil(log2 W),
 *     D = L - 11 for one-word keys and L - 10 for two-word keys, clamped to
 *     [0, min(20, 2k)] (or D = part_bits when set).  With TK_FLAG_GLOBAL_FILTER
 *     one filter covers the whole library (size rule below);
 *   - n_blocks blocks of 64 bytes: words 0..3 are the first plane S (256
 *     bits), words 4..7 the second plane T;
 *   - h = fmix64(key) for one-word keys, fmix64(lo ^ fmix64(hi)) for
 *     two-word keys (fmix64: the 64-bit finaliser of MurmurHash3);
 *   - block = floor(h * n_blocks / 2^64);
 *   - word w (0..3) of the block gets pattern table entry
 *     (h >> (w * table_bits)) mod 2^table_bits, a 64-bit mask with
 *     `bloom_bits` set bits; the table is precomputed with SplitMix64 seeded
 *     with `bloom_seed`, entries filled in order, each drawing outputs and
 *     taking the top six bits as a bit position, skipping repeats;
 *   - screen pass: for each window and each word, old = atomicOr(S[w], m);
 *     atomicOr(T[w], old & m).  A T bit therefore holds iff its position was
 *     touched at least twice, whatever the order of the windows, so the set
 *     of candidates is deterministic;
 *   - collect pass: a window is collected iff all its pattern bits hold in T.
 *     Every key seen at least twice is collected (no false negatives);
 *   - global filter size: W = max(n_bases - n_reads * (k - 1), 1) estimated
 *     windows, n_blocks = max(1, ceil(bloom_beta * W / 256)).
 */
#ifndef TURTLE_H
#define TURTLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define TK_API __attribute__((visibility("default")))
#else
#define TK_API
#endif

typedef enum {
    TK_OK = 0,
    TK_EINVAL = -1,    /* bad argument: k outside [1, 63], c = 0, null
                          pointer, decreasing offsets, workspace too small,
                          misaligned device pointer, bad option value */
    TK_ENOMEM = -2,    /* host or device allocation failed */
    TK_EDEVICE = -3,   /* a HIP call failed (message in tk_last_error) */
    TK_EOVERFLOW = -4  /* input too large: n_bases must be < 2^32 so that
                          positions and counts fit 32 bits */
} tk_status;
/* Every failure is reported as a status (with a message in tk_last_error);
 * no function lets a C++ exception out of the library. */

/* Stages whose device time is reported when TK_FLAG_TIMING is set.  The
 * partitioned path (default) runs PACK, PARTITION, BUCKET, FALLBACK and
 * GATHER; the global-filter path runs PACK, SCREEN, COLLECT, SORT, COMPACT. */
enum {
    TK_STAGE_PACK = 0,       /* 2-bit packing and window validity           */
    TK_STAGE_SCREEN = 1,     /* global filter: screen pass (atomicOr)       */
    TK_STAGE_COLLECT = 2,    /* global filter: collect pass (append)        */
    TK_STAGE_SORT = 3,       /* global filter: LSD radix sort               */
    TK_STAGE_COMPACT = 4,    /* global filter: run-length compaction        */
    TK_STAGE_PARTITION = 5,  /* partitioned: radix passes on the top bits   */
    TK_STAGE_BUCKET = 6,     /* partitioned: per-bucket screen, sort, RLE   */
    TK_STAGE_FALLBACK = 7,   /* partitioned: buckets too large for LDS      */
    TK_STAGE_GATHER = 8,     /* partitioned: records into final order       */
    TK_STAGE_COUNT = 9
};

#define TK_FLAG_TIMING 1u         /* record HIP events around each stage     */
#define TK_FLAG_CTURTLE 4u        /* approximate: cTurtle (§2.2), see below   */
#define TK_FLAG_SINGLE_PASS 8u    /* approximate: single pass with "+1" (§2.1)
                                     see below                               */
#define TK_FLAG_GLOBAL_FILTER 2u  /* one filter for the whole library in HBM
                                     (device-scope atomics) instead of one
                                     filter per bucket                       */

/*
 * Approximate variants (one library per call; tk_count / tk_count_device):
 *   TK_FLAG_CTURTLE: the counting Bloom filter of cTurtle (§2.2).  A k-mer's
 *     first pattern (two table entries ORed, in 64-bit word
 *     floor(h * W / 2^64) of a filter of W words) is set at its first
 *     sighting; a sighting that finds it set tries its second pattern (two
 *     more entries, in the next word): if not all set, it sets them and the
 *     k-mer is reported.  Result: the reported k-mers, ascending, counts 0;
 *     c must be 2.  False positives and negatives come from collisions.
 *   TK_FLAG_SINGLE_PASS: the single pass of Algorithm 1 as printed: a
 *     sighting that finds its first pattern set is stored; counts are the
 *     stored sightings plus one; records with count >= c are kept.
 * W = max(1, ceil(bloom_beta * windows_estimate / 64)) (bloom_beta up to
 * 1024 here), or 8 * bloom_blocks when set.  n_collected = stored or
 * reported sightings.  Not combinable with each other or with batches.
 */
typedef struct {
    uint32_t bloom_beta;        /* first-plane bits per window (4); the
                                   partitioned path accepts 1..32          */
    uint32_t bloom_table_bits;  /* log2 of pattern table entries, 1..10 (10) */
    uint32_t bloom_bits;        /* set bits per table entry, 1..16 (2)       */
    uint32_t flags;             /* TK_FLAG_* */
    uint64_t bloom_blocks;      /* global filter only: explicit size in
                                   blocks; 0 = size rule                    */
    uint64_t bloom_seed;        /* SplitMix64 seed of the table (1305)       */
    int32_t part_bits;          /* partitioned path: bucket bits D, 0..20;
                                   -1 (default) = size rule                 */
    uint32_t shard_count;       /* key-range shards, 0 or 1 = none; <= 1024  */
    uint32_t shard_index;       /* the shard this call counts, < shard_count */
    uint32_t bucket_tile;       /* partitioned path: tile shape of the
                                   bucket kernel, 0 (default: 7168 one-word
                                   or 3584 two-word windows per group) or 1
                                   (6144 or 3072); results never depend on
                                   it                                      */
} tk_options;

/*
 * Key-range shards (partitioned path, one library per call): the share of
 * the work one of G devices does when the library is split among G devices
 * that each hold all of its reads -- the counterpart of the paper's routing
 * of every k-mer to the one consumer that owns its filter (§2.1,
 * parallelization), with key ranges as owners.  Every window is extracted,
 * and the first partition pass counts the library's top-digit histogram
 * (the top D1 bits of the canonical key: D1 = D for D <= 10, else D - 10,
 * the second pass taking the other 10).  Digit d goes to shard
 * min(G - 1, floor(G * (below(d) + n(d) / 2) / M)), where n(d) is its
 * window count, below(d) that of the digits before it, and M the library's
 * window count.  The owners are contiguous and the shares even to within one
 * digit's mass.  A call with shard_index = g keeps only the keys of its
 * digits from then on: the rest of the partition, the per-bucket filters, the
 * sort and the compaction see only the shard.  Every
 * bucket lies in one shard and meets exactly the filter it meets unsharded.
 * So the results of g = 0..G-1, concatenated in order, are the unsharded
 * result record for record, and every statistic (n_windows: the shard's
 * windows) adds up to the unsharded one.  Not combinable with the global
 * filter, the approximate variants, batches or the phased call.
 */

typedef struct {
    uint64_t n;             /* records in keys/counts (count >= c)           */
    uint32_t k;
    uint32_t key_words;     /* 1 for k <= 31, 2 for k >= 32                  */
    uint64_t *keys;         /* n * key_words words, ascending                */
    uint32_t *counts;       /* n counts                                      */
    uint64_t n_windows;     /* valid k-mer windows in the input              */
    uint64_t n_collected;   /* occurrences passed to the sort                */
    uint64_t n_distinct;    /* distinct keys among the collected             */
    uint64_t n_singletons;  /* collected keys seen once (screen false
                               positives when c >= 2)                        */
    uint64_t n_below_c;     /* collected keys with 2 <= count < c            */
    uint64_t bloom_blocks;  /* global filter: blocks used (0 when c = 1 or
                               partitioned)                                  */
    uint32_t sort_passes;   /* global filter: radix passes run               */
    int32_t part_bits;      /* partitioned: bucket bits D used; -1 global    */
    uint64_t n_fallback;    /* partitioned: buckets too large for LDS        */
    double stage_ms[TK_STAGE_COUNT]; /* device time per stage when timed     */
} tk_result;

/* Fill *opts with the defaults listed in tk_options. */
TK_API tk_status tk_default_options(tk_options *opts);

/* Short text for a status code (static storage). */
TK_API const char *tk_strerror(tk_status st);

/* Detail of the last error raised on the calling thread ("" if none). */
TK_API const char *tk_last_error(void);

/*
 * Count the k-mers of a read library held in HOST memory.
 *   bases   : n_bases ASCII bytes, all reads concatenated (read-only);
 *   offsets : n_reads + 1 non-decreasing values, offsets[0] = 0 and
 *             offsets[n_reads] = n_bases; read r is bases[offsets[r] ..
 *             offsets[r+1]) (read-only);
 *   k       : 1..63;  c : threshold >= 1;  opts : NULL for defaults.
 * On success *out receives a library-allocated result whose keys/counts are
 * host arrays; release it with tk_result_free.  Device memory is allocated
 * and freed inside the call on the current HIP device; the reads and the
 * records cross PCIe through two pinned 64 MB host slices, also released
 * before the call returns.
 */
TK_API tk_status tk_count(const uint8_t *bases, const uint64_t *offsets,
                   uint64_t n_reads, int k, uint32_t c,
                   const tk_options *opts, tk_result **out);

/* Release a result returned by tk_count (NULL is ignored). */
TK_API void tk_result_free(tk_result *res);

/*
 * Device workspace needed by tk_count_device for a library of n_bases bases
 * and n_reads reads at this k, c and options.  The size is an upper bound
 * that does not depend on the read contents.
 */
TK_API tk_status tk_workspace_size(uint64_t n_bases, uint64_t n_reads, int k,
                            uint32_t c, const tk_options *opts,
                            size_t *bytes);

/*
 * Count the k-mers of a read library held in DEVICE memory.
 *   d_bases      : device pointer, n_bases bytes (16-byte alignment takes
 *                  the vector-load path; any alignment is accepted);
 *   d_offsets    : device pointer, n_reads + 1 uint64 as in tk_count (the
 *                  values are trusted: offsets[n_reads] must equal n_bases
 *                  and they must not decrease);
 *   d_workspace  : device buffer of ws_bytes >= tk_workspace_size(...),
 *                  256-byte aligned, owned by the caller;
 *   stream       : hipStream_t to launch on (NULL = the null stream).
 * On success *out is filled in: out->keys and out->counts are DEVICE
 * pointers into the workspace (valid until the workspace is reused), the
 * other fields are host values.  The call blocks until the result is
 * complete on the device.  The workspace may be reused by the next call
 * once this one has returned.
 */
TK_API tk_status tk_count_device(const uint8_t *d_bases, const uint64_t *d_offsets,
                          uint64_t n_bases, uint64_t n_reads, int k,
                          uint32_t c, const tk_options *opts,
                          void *d_workspace, size_t ws_bytes, void *stream,
                          tk_result *out);

/*
 * tk_count_device without any allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The workspace is a static device array of
 * TK_STATIC_WORKSPACE_BYTES (256 MiB) inside the library, one per device,
 * held until the process ends; its address is looked up once per device.
 * That bounds the library: about 7e6 bases for k <= 31 and 4e6 for k >= 32
 * (tk_workspace_size <= TK_STATIC_WORKSPACE_BYTES); a larger one is refused
 * with TK_EINVAL before anything runs.  Arguments as tk_count_device, plus:
 *   d_out_keys   : device buffer of out_capacity * key_words uint64 (caller's);
 *   d_out_counts : device buffer of out_capacity uint32 (caller's);
 * On success the records are copied there (out->keys / out->counts are
 * these pointers); more records than out_capacity (at most n_bases can
 * occur) give TK_EINVAL and leave the buffers unspecified.  TK_FLAG_TIMING
 * is refused (timing creates events).  The call allocates nothing: no
 * hipMalloc, hipFree, event or stream.  Every call on a device shares that
 * device's array and finds the previous call's contents, which the counting
 * path clears or overwrites as it goes; calls on one device are serialised
 * by a lock inside the library (the call returns only when its work on the
 * stream is finished).  Other processes have arrays of their own.
 */
#define TK_STATIC_WORKSPACE_BYTES (256ull << 20)
TK_API tk_status tk_count_device_static(const uint8_t *d_bases, const uint64_t *d_offsets,
                                        uint64_t n_bases, uint64_t n_reads, int k, uint32_t c,
                                        const tk_options *opts, uint64_t *d_out_keys,
                                        uint32_t *d_out_counts, uint64_t out_capacity,
                                        void *stream, tk_result *out);

/*
 * Batches: several read libraries counted in one call, each with its own
 * k, buckets, Bloom filters, threshold and result -- the libraries are
 * independent counting jobs (§2.1 applied to each library) that share the
 * kernels' launches.  Library j owns reads [lib_reads[j], lib_reads[j+1])
 * and bases [lib_bases[j], lib_bases[j+1]) of one bases/offsets pair as in
 * tk_count_device (offsets[lib_reads[j]] must equal lib_bases[j]);
 * lib_bases and lib_reads are HOST arrays of n_libs + 1 non-decreasing
 * values starting at 0, k a HOST array of n_libs k-mer lengths (1..63), c a
 * HOST array of n_libs thresholds (>= 1).  Each library takes its bucket
 * bits D from the size rule on its own bases, reads and k (or
 * options.part_bits).  The libraries with one-word keys (k <= 31) and those
 * with two-word keys (k >= 32) are counted in two passes, one after the
 * other on the stream, each in its own part of the workspace; a batch of one
 * key width is one pass.  Not available with TK_FLAG_GLOBAL_FILTER, the
 * approximate variants or key-range shards.
 * Errors: TK_EINVAL (bad boundaries, c = 0, k, options, a pass needing
 * 2^31 buckets or more), TK_EOVERFLOW (n_bases >= 2^32).
 */
TK_API tk_status tk_batch_workspace_size(uint64_t n_libs, const uint64_t *lib_bases,
                                         const uint64_t *lib_reads, const int *k,
                                         const uint32_t *c, const tk_options *opts,
                                         size_t *bytes);

/*
 * Count a batch held in DEVICE memory.  out is a HOST array of n_libs
 * results; out[j] describes library j exactly as tk_count_device describes
 * it counted alone (its own k and key_words; keys and counts are device
 * pointers into the workspace; stage_ms holds the timings of the whole
 * call).  The call blocks until every result is complete on the device.
 */
TK_API tk_status tk_count_batch_device(const uint8_t *d_bases, const uint64_t *d_offsets,
                                       uint64_t n_libs, const uint64_t *lib_bases,
                                       const uint64_t *lib_reads, const int *k, const uint32_t *c,
                                       const tk_options *opts, void *d_workspace,
                                       size_t ws_bytes, void *stream, tk_result *out);

/*
 * Phased sort-and-compact (§2.1, "Counting frequencies with sorting and
 * compaction", Fig. 1): a library in HOST memory (as tk_count) is streamed to
 * the device in chunks of consecutive reads of at most chunk_bases bases (a
 * longer read forms a chunk alone).  Pass 1 screens every window of every
 * chunk into one filter of the global-filter size rule; pass 2 collects each
 * chunk's candidates, sorts and compacts them into (key, count) records and
 * merges those into a resident sorted-and-compacted array (SAC) of at most
 * sac_capacity records (0: as many as bases), adding the counts of keys
 * present in both.  The answer keeps the SAC records with count >= c.
 * Device memory is bounded by the chunk size and the SAC capacity, not by
 * the library size; the result does not depend on chunk_bases and equals
 * tk_count's with TK_FLAG_GLOBAL_FILTER (same filter, same statistics).
 * Host memory: when c >= 2 every chunk is packed once, in pass 1, and its
 * packed words and validity bits (0.5 byte per base) wait in pinned host
 * memory for pass 2; host copies go through two pinned 64 MB slices.  Both
 * are released before the call returns.
 * *out is allocated as in tk_count (free with tk_result_free);
 * *device_bytes (may be NULL) receives the device memory used.
 * Errors: as tk_count; TK_ENOMEM also when the SAC outgrows sac_capacity.
 */
TK_API tk_status tk_count_phased(const uint8_t *bases, const uint64_t *offsets,
                                 uint64_t n_reads, int k, uint32_t c,
                                 uint64_t chunk_bases, uint64_t sac_capacity,
                                 const tk_options *opts, tk_result **out,
                                 size_t *device_bytes);

/*
 * The pattern table the screen uses for these options: 2^bloom_table_bits
 * 64-bit masks written to host array `masks` of `capacity` entries.
 */
TK_API tk_status tk_pattern_table(const tk_options *opts, uint64_t *masks,
                           uint64_t capacity);

/* Global-filter size in 64-byte blocks for a library at these options. */
TK_API tk_status tk_bloom_blocks(uint64_t n_bases, uint64_t n_reads, int k,
                          const tk_options *opts, uint64_t *n_blocks);

/* Bucket bits D the partitioned path uses for a library at these options. */
TK_API tk_status tk_part_bits(uint64_t n_bases, uint64_t n_reads, int k,
                              const tk_options *opts, int *part_bits);

/* ---------------------------------------------------------------------
 * Stage entry points (device memory, caller's stream), used to check each
 * kernel on its own.  All pointers are device pointers.
 * --------------------------------------------------------------------- */

/*
 * 2-bit packing (§2.1 extraction).  packed[w] holds bases 32w..32w+31, base
 * 32w+t in bits (63-2t, 62-2t) (first base most significant; a non-base
 * byte packs as 0).  valid[w] bit t is set iff the k bases ending at base
 * 32w+t lie in one read and are all A/C/G/T.  n_words = ceil(n_bases/32);
 * packed and valid hold n_words entries; *n_windows (device, uint64)
 * receives the number of valid windows.  d_scratch holds n_words uint32.
 */
TK_API tk_status tk_pack_device(const uint8_t *d_bases, const uint64_t *d_offsets,
                         uint64_t n_bases, uint64_t n_reads, int k,
                         uint64_t *d_packed, uint32_t *d_valid,
                         uint32_t *d_scratch, uint64_t *d_n_windows,
                         void *stream);

/*
 * Stable LSD radix sort of n keys of key_words 64-bit words ({hi, lo} when
 * 2), on the low `key_bits` bits (bits above must be zero).  d_keys holds
 * the input; d_alt is a buffer of the same size; d_scratch holds
 * tk_sort_scratch_size(n) bytes.  *d_sorted_out (host) receives whichever
 * of d_keys / d_alt holds the sorted keys.
 */
TK_API tk_status tk_sort_scratch_size(uint64_t n, int key_words, size_t *bytes);
TK_API tk_status tk_sort_keys_device(uint64_t *d_keys, uint64_t *d_alt, uint64_t n,
                              int key_words, int key_bits, void *d_scratch,
                              size_t scratch_bytes, void *stream,
                              uint64_t **d_sorted_out);

/*
 * Run-length compaction and threshold of n sorted keys (§2.1 sorting and
 * compaction): writes the distinct keys with count >= c to d_out_keys and
 * their counts to d_out_counts (both sized for n entries), and to *stats
 * (host) n_out, n_distinct, n_singletons, n_below_c in that order.
 * d_scratch holds tk_compact_scratch_size(n) bytes.
 */
TK_API tk_status tk_compact_scratch_size(uint64_t n, size_t *bytes);
TK_API tk_status tk_compact_device(const uint64_t *d_keys, uint64_t n, int key_words,
                            uint32_t c, uint64_t *d_out_keys,
                            uint32_t *d_out_counts, void *d_scratch,
                            size_t scratch_bytes, void *stream,
                            uint64_t stats[4]);

#ifdef __cplusplus
}
#endif

#endif /* TURTLE_H */
