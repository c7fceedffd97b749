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

// ---- pack.hip -------------------------------------------------------------
// starts: n_words uint32, must be zero on entry.  n_windows may be null.
hipError_t launch_pack(const uint8_t *bases, const uint64_t *offsets, uint64_t n_bases,
                       uint64_t n_reads, int k, uint64_t *packed, uint32_t *valid,
                       uint32_t *starts, unsigned long long *n_windows, hipStream_t stream);

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

// ---- partition.hip --------------------------------------------------------
// Keys of every valid window ordered by their top D = bits bits (D <= 20),
// in one pass (D <= 10) or two; the order inside a bucket is unspecified.
// Input: the packed reads (n_elems = n_words * 32 window positions).  tmp
// (pass-1 output when D > 10) and out hold n_elems keys each; out receives
// the result and *total (device) the number of keys; *total2 (device) the
// number moved by pass 2.
struct PartArgs {
    const uint64_t *packed;
    const uint32_t *valid;
    const void *keys_in;  // pass 2: the pass-1 output
    uint64_t n_elems;
    int k;
    int shift, bits;
    uint64_t n_chunks;    // pass 1: chunks
    const uint32_t *seg;  // pass 2: segment starts (nseg + 1)
    const uint32_t *cb;   // pass 2: first chunk of each segment (nseg + 1)
    uint32_t nseg;
};
size_t partition_scratch_words(uint64_t n_pos, int key_words);
hipError_t partition_keys(const PartArgs &a, void *tmp, void *out, uint32_t *scratch, size_t scratch_words,
                          uint32_t *total, uint32_t *total2, hipStream_t stream);

// ---- bucket.hip -----------------------------------------------------------
struct BucketArgs {
    const void *keys;         // keys ordered by bucket (top D bits)
    const uint32_t *n_dev;    // number of keys (device)
    int k, D;
    uint32_t c;
    int screen;
    uint32_t beta;
    const uint64_t *table;
    uint32_t table_bits;
    void *gap_keys;        // records of a bucket start at the bucket's first index
    uint32_t *gap_counts;
    uint32_t *rec_start;   // per bucket: first index, number of records
    uint32_t *rec_nout;
    unsigned long long *wg_stats;  // per workgroup: collected, runs, singletons, below c
    uint32_t *fb_list;     // oversized buckets: (bucket, start, size)
    uint32_t *fb_count;
    uint32_t fb_cap;
};
int bucket_grid();
int bucket_capacity(int key_words);
hipError_t launch_bucket(const BucketArgs &a, int key_words, int grid, hipStream_t stream);
// Oversized buckets (more keys than a workgroup holds), in key order.
struct FbEntry {
    uint32_t d, start, ns;  // bucket, first key, number of keys
    uint32_t wpre, fpre;    // keys and filter blocks of the entries before
    uint32_t nb;            // filter blocks of this bucket
};
hipError_t launch_fb_screen(const void *keys, const FbEntry *ent, uint32_t n_ent, uint64_t n, int key_words,
                            const uint64_t *table, uint32_t table_bits, uint64_t *filter, hipStream_t stream);
hipError_t launch_fb_collect(const void *keys, const FbEntry *ent, uint32_t n_ent, uint64_t n, int key_words,
                             const uint64_t *table, uint32_t table_bits, const uint64_t *filter, bool screen,
                             void *out, unsigned long long *n_out, hipStream_t stream);
// Copies each bucket's records (sorted records of all entries, c->n_out of
// them) to its slot, sets rec_nout, and adds the counters to fb_stats.
hipError_t launch_fb_distribute(const void *rec_keys, const uint32_t *rec_counts, const DevCounters *c,
                                const FbEntry *ent, uint32_t n_ent, int key_words, int k, int D, void *gap_keys,
                                uint32_t *gap_counts, uint32_t *rec_nout, unsigned long long *fb_stats,
                                hipStream_t stream);
hipError_t launch_gather(const uint32_t *rec_start, const uint32_t *rec_nout, const uint32_t *rec_off,
                         uint64_t n_buckets, const uint64_t *gap_keys, const uint32_t *gap_counts, int key_words,
                         uint64_t *out_keys, uint32_t *out_counts, hipStream_t stream);
hipError_t launch_stats(const unsigned long long *wg_stats, uint64_t n_wg, const unsigned long long *fb_stats,
                        const uint32_t *totals, DevCounters *ctr, hipStream_t stream);

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

// Number of compute units of the current device (cached).
int device_cu_count();

}  // namespace tk
