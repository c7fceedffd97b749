// Host-side launchers shared between the translation units of libturtle.
// Every launcher enqueues work on `stream` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

namespace tk {

// Device counters of one counting call (zeroed before the call).
struct DevCounters {
    unsigned long long n_windows;
    unsigned long long n_collected;
    unsigned long long n_runs;
    unsigned long long n_out;
    unsigned long long n_single;
    unsigned long long n_below;
    unsigned long long pad[2];
};

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Clears n bytes (n a multiple of 4, p 4-byte aligned) with fill kernels.
hipError_t zero_bytes(void *p, size_t n, hipStream_t stream);


// ---- bloom.hip ------------------------------------------------------------
struct BloomArgs {
    const uint64_t *packed;
    const uint32_t *valid;
    uint64_t n_words;
    int k;
    const uint64_t *table;  // 2^table_bits masks in device memory
    uint32_t table_bits;
    uint64_t n_blocks;
    uint64_t *filter;       // n_blocks * 8 words
};
hipError_t launch_screen(const BloomArgs &a, int grid, hipStream_t stream);
// screen = false collects every valid window (c = 1).
hipError_t launch_collect(const BloomArgs &a, bool screen, void *keys, uint64_t capacity,
                          unsigned long long *n_collected, int grid, hipStream_t stream);

// ---- libraries of a batch --------------------------------------------------
// Device table, one entry per library.  The libraries' reads are consecutive
// in the bases/offsets arrays; a window belongs to the library holding its
// last base, and window positions are base positions.
struct LibDesc {
    uint64_t pos0, pos1;  // window positions [pos0, pos1)
    uint64_t h1;          // partition pass 1: first count entry of the library
    uint32_t cb1, nch1;   // pass 1: first chunk, number of chunks
    uint32_t seg0;        // pass 2: first segment (2^D1 segments per library)
    uint32_t bucket0;     // first bucket id (2^D buckets per library)
    uint32_t c;           // threshold
    int D, D1, D2;        // bucket bits D = D1 (pass 1) + D2 (pass 2)
    int k;                // k-mer length of the library
};

// ---- pack.hip -------------------------------------------------------------
// starts: n_words uint32, must be zero on entry.  n_windows may be null.
// libs (device, n_libs entries ordered by position): when given, the
// validity bits of each library's positions use that library's k (k is
// then unused) and positions outside the listed libraries stay clear.
hipError_t launch_pack(const uint8_t *bases, const uint64_t *offsets, uint64_t n_bases,
                       uint64_t n_reads, int k, uint64_t *packed, uint32_t *valid,
                       uint32_t *starts, unsigned long long *n_windows, hipStream_t stream,
                       const LibDesc *libs = nullptr, uint32_t n_libs = 0);

// ---- partition.hip --------------------------------------------------------
// Keys of every valid window, ordered by (library, top D bits) as far as the
// bucket kernel needs.  Pass 1 extracts the canonical keys from the packed
// reads and orders them by (library, top D1 bits): every "segment" is one
// contiguous range.  Pass 2, run when some library has D2 > 0, cuts every
// segment into tiles and orders each tile by the next D2 bits in place
// (D2 = 0: the tile is left as it is, in some order).  Pass-1 chunks are per
// library: chunk i of library j covers window positions
// [floor32(pos0) + i * chunk, ...) inside [pos0, pos1).
uint64_t partition_chunk(int key_words);  // window positions (pass 1) or keys (pass 2) per chunk
uint64_t partition_tile2(int key_words);  // keys per second-pass tile
struct PartPlan {
    const uint64_t *packed;
    const uint32_t *valid;
    const LibDesc *libs;  // device; every library has its own k
    uint32_t n_libs;
    uint32_t nch1;        // pass-1 chunks of all libraries
    uint64_t n_hist1;     // pass-1 count entries of all libraries
    uint32_t nseg;        // pass-2 segments of all libraries
    int D2max;            // largest pass-2 digit; 0: no second pass
    uint64_t cap;         // key capacity of tmp and out
    uint32_t shard_count; // key-range shards (one library): 1 = none
    uint32_t shard_index; // the shard whose keys are kept
    uint32_t n_buckets;   // buckets of all libraries
};
// Where the keys of a bucket are after the partition (device pointers into
// its scratch).  Without a second pass (tiled = 0), and for the libraries
// with D2 = 0, bucket b is the range [bucket_starts[b], bucket_starts[b + 1])
// of the output.  With one, a bucket of a library with D2 > 0 is digit d2
// (its low D2 bits) of segment s = seg0 + (its top D1 bits): the segment's
// keys [seg[s], seg[s + 1]) form its T = tt[s + 1] - tt[s] tiles of
// tile_keys keys each (tile i of the segment starts at seg[s] + i *
// tile_keys), and in tile i digit d occupies [px[x + d * T + i],
// px[x + (d + 1) * T + i]) relative to the tile's start, x = tt[s] * pw.
// bucket_starts then holds the exclusive prefix of the bucket sizes:
// disjoint index ranges of the right sizes, in (library, bucket) order, that
// coincide with the key positions of the contiguous buckets.
struct KeyLayout {
    int tiled;
    const uint32_t *seg, *tt;
    const uint16_t *px;
    uint32_t pw, tile_keys;
};
size_t partition_scratch_words(const PartPlan &p, int key_words);
// out receives the keys; lib_keys (device, n_libs + 1) the first key of
// every library and the number of keys; bucket_starts (device,
// n_buckets + 1) the first index of every bucket and the number of keys;
// *layout where the buckets are.
hipError_t partition_keys(const PartPlan &p, int key_words, void *tmp, void *out, uint32_t *scratch,
                          size_t scratch_words, uint32_t *lib_keys, uint32_t *bucket_starts, KeyLayout *layout,
                          hipStream_t stream);

// ---- bucket.hip -----------------------------------------------------------
struct BucketArgs {
    const void *keys;         // keys ordered by (library, bucket)
    const LibDesc *libs;      // device
    uint32_t n_libs;
    const uint32_t *lib_keys; // first key of every library, number of keys (device)
    uint32_t beta;
    const uint64_t *table;
    uint32_t table_bits;
    void *gap_keys;        // records of a group start at the group's first index
    uint32_t *gap_counts;
    uint32_t *rec_start;   // per bucket id: first index, number of records
    uint32_t *rec_nout;
    unsigned long long *lib_stats;  // per library: collected, runs, singletons, below c
    uint32_t *fb_list;     // oversized buckets: (bucket id, start, size)
    uint32_t *fb_count;
    uint32_t fb_cap;
    // the schedule: chunk c holds the bucket ids [c * chunk_buckets,
    // (c + 1) * chunk_buckets); launch_bucket cuts each chunk into groups of
    // whole buckets (first and last non-empty bucket of group g at
    // grp_first/grp_last[c * chunk_buckets + g], grp_count[c] groups) and
    // lists the buckets too large for a group in fb_list
    uint32_t n_buckets;
    const uint32_t *bucket_starts;  // n_buckets + 1 key positions (from the partition)
    uint32_t n_chunks, chunk_buckets;
    uint32_t *grp_first, *grp_last, *grp_count;
    uint32_t *chunk_next;           // chunk counter, zero before the launch
    int tile;                       // tile shape (keys per thread), 0 or 1
    KeyLayout layout;               // where the buckets' keys are (from the partition)
    uint4 *grp_piece;               // per group of a tiled library: first tile, tiles,
                                    // segment start, first | (last digit << 16); others: tiles = 0
};
int bucket_grid();
constexpr uint32_t BK_CHUNK_MAX = 32;  // bucket ids per chunk of the bucket kernel's schedule
constexpr uint32_t BK_TILES_MAX = 256;  // tiles a group of a tiled library may span
int bucket_capacity(int key_words, int tile);
hipError_t launch_bucket(const BucketArgs &a, int key_words, int grid, hipStream_t stream);
// Oversized buckets (more keys than a workgroup holds) of one library, in
// key order.
struct FbEntry {
    uint32_t d, start, ns;  // bucket within the library, first key, number of keys
    uint32_t wpre, fpre;    // keys and filter blocks of the entries before
    uint32_t nb;            // filter blocks of this bucket
};
// Copies the keys of the listed oversized buckets of one library (first
// segment seg0, D2 second-pass bits) to dst + each bucket's first index
// (ent[i].start), from src laid out as `layout` describes.
hipError_t launch_fb_gather(const void *src, void *dst, const FbEntry *ent, uint32_t n_ent, int key_words,
                            const KeyLayout &layout, uint32_t seg0, int D2, hipStream_t stream);
hipError_t launch_fb_screen(const void *keys, const FbEntry *ent, uint32_t n_ent, uint64_t n, int key_words,
                            const uint64_t *table, uint32_t table_bits, uint64_t *filter, hipStream_t stream);
hipError_t launch_fb_collect(const void *keys, const FbEntry *ent, uint32_t n_ent, uint64_t n, int key_words,
                             const uint64_t *table, uint32_t table_bits, const uint64_t *filter, bool screen,
                             void *out, unsigned long long *n_out, hipStream_t stream);
// Copies each bucket's records (sorted records of all entries, c->n_out of
// them) to its slot, sets rec_nout[bucket0 + d], and adds the counters to
// the library's statistics.
hipError_t launch_fb_distribute(const void *rec_keys, const uint32_t *rec_counts, const DevCounters *c,
                                const FbEntry *ent, uint32_t n_ent, int key_words, int k, int D, uint32_t bucket0,
                                void *gap_keys, uint32_t *gap_counts, uint32_t *rec_nout,
                                unsigned long long *lib_stats, hipStream_t stream);
hipError_t launch_gather(const uint32_t *rec_start, const uint32_t *rec_nout, const uint32_t *rec_off,
                         uint64_t n_buckets, const uint64_t *gap_keys, const uint32_t *gap_counts, int key_words,
                         uint64_t *out_keys, uint32_t *out_counts, hipStream_t stream);
// Per-library counters: windows from lib_keys, records and their first
// index from the scanned record counts (rec_off, total), the rest from
// lib_stats.  out_first[j]: first output record of library j.
hipError_t launch_lib_stats(const LibDesc *libs, uint32_t n_libs, const uint32_t *lib_keys, const uint32_t *rec_off,
                            const uint32_t *rec_total, const unsigned long long *lib_stats, DevCounters *ctr,
                            uint32_t *out_first, hipStream_t stream);

// ---- scan.hip -------------------------------------------------------------
// Exclusive prefix sum of n uint32 values (in may equal out).  *total (device)
// receives the sum.  scratch holds scan_scratch_words(n) uint32.
uint64_t scan_scratch_words(uint64_t n);
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *scratch,
                                 uint32_t *total, hipStream_t stream);

// ---- radix.hip ------------------------------------------------------------
size_t radix_scratch_bytes(uint64_t n, int key_words);
// Sorts n keys on bits [0, key_bits); returns in *sorted which buffer holds
// the result and in *passes the number of passes run.
hipError_t radix_sort(uint64_t *keys, uint64_t *alt, uint64_t n, int key_words, int key_bits,
                      void *scratch, size_t scratch_bytes, hipStream_t stream, uint64_t **sorted,
                      int *passes);

// ---- compact.hip ----------------------------------------------------------
size_t compact_scratch_bytes(uint64_t n);
// Run-length compaction of n sorted keys with threshold c.  Writes
// n_runs, n_out, n_single and n_below into *ctr (device).
hipError_t compact(const uint64_t *keys, uint64_t n, int key_words, uint32_t c, uint64_t *out_keys,
                   uint32_t *out_counts, void *scratch, size_t scratch_bytes, DevCounters *ctr,
                   hipStream_t stream);

// ---- phased.hip -----------------------------------------------------------
// Merge of two sorted (key, count) lists with unique keys into one list with
// unique keys, counts of equal keys added (*n_out, device).  tmp_k/tmp_c and
// flag hold na + nb entries, scan_tmp scan_scratch_words(na + nb); out holds
// na + nb records.
hipError_t merge_compact(const uint64_t *ak, const uint32_t *ac, uint64_t na, const uint64_t *bk, const uint32_t *bc,
                         uint64_t nb, int key_words, uint64_t *tmp_k, uint32_t *tmp_c, uint32_t *flag,
                         uint32_t *scan_tmp, uint64_t *out_k, uint32_t *out_c, uint32_t *n_out, hipStream_t stream);
// Records with count >= c, in order (*n_out, device); stats[0] += records of
// count 1, stats[1] += records of count in [2, c).  flag holds 2n entries.
hipError_t select_records(const uint64_t *keys, const uint32_t *cnt, uint64_t n, int key_words, uint32_t c,
                          uint32_t *flag, uint32_t *scan_tmp, uint64_t *out_k, uint32_t *out_c, uint32_t *n_out,
                          unsigned long long *stats, hipStream_t stream);

// ---- approx.hip -----------------------------------------------------------
// One pass of cTurtle (cturtle) or of the single-pass "+1" variant over the
// packed windows: reported keys appended to out (at most capacity; *n_out
// counts every report).
hipError_t launch_approx(const uint64_t *packed, const uint32_t *valid, uint64_t n_words, int k,
                         const uint64_t *table, uint32_t table_bits, uint64_t *filter, uint64_t n_filter_words,
                         bool cturtle, void *out, uint64_t capacity, unsigned long long *n_out, int grid,
                         hipStream_t stream);
// counts[0, c->n_out) += add, or = 0 when add is 0.
hipError_t launch_adjust_counts(uint32_t *counts, const DevCounters *c, uint32_t add, hipStream_t stream);

// Number of compute units of the current device (cached).
int device_cu_count();

}  // namespace tk
