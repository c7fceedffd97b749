// K4: stable LSD radix sort of k-mer keys (one or two 64-bit words).
//
// Paper §2.1 (Counting frequencies with sorting and compaction): the
// collected occurrences are sorted by k-mer value so that equal k-mers become
// neighbours for the run-length pass; the paper argues (§2.1, running-time
// analysis) that the sequential access of sorting beats the random access of
// a hash table.
//
// Each pass over an 8-bit digit runs three kernels:
//   hist    : per tile, digit counts -> counts[digit * n_tiles + tile];
//   scan    : exclusive prefix sum of counts in (digit, tile) order gives
//             every tile the global start of each of its digits;
//   scatter : per tile, a stable local rank (wave match over the 8 digit bits
//             + per-wave digit counters in LDS), a local reorder through LDS,
//             then coalesced writes of each digit run to its global place.
// Tiles are wave-striped: wave w of the block owns a contiguous quarter of
// the tile, and item i of lane l is element i*64 + l of that quarter, so the
// (wave, item, lane) order is the input order and the sort is stable.
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int RADIX_THREADS = 256;
constexpr int RADIX_BITS = 8;
constexpr int RADIX_BINS = 1 << RADIX_BITS;
constexpr int RADIX_WAVES = RADIX_THREADS / WAVE;

template <typename K>
struct Tile;
template <>
struct Tile<uint64_t> {
    static constexpr int ITEMS = 16;
};
template <>
struct Tile<Key2> {
    static constexpr int ITEMS = 8;
};

template <typename K>
constexpr uint64_t tile_size() {
    return (uint64_t)RADIX_THREADS * Tile<K>::ITEMS;
}

template <typename K>
__global__ __launch_bounds__(RADIX_THREADS) void radix_hist(const K *__restrict__ in, uint64_t n, int shift,
                                                            uint32_t *__restrict__ counts, uint64_t n_tiles) {
    constexpr int ITEMS = Tile<K>::ITEMS;
    __shared__ uint32_t s_h[RADIX_BINS];
    const int tid = threadIdx.x;
    s_h[tid] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * tile_size<K>();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint64_t idx = base + (uint64_t)i * RADIX_THREADS + tid;
        if (idx < n)
            atomicAdd(&s_h[digit_of(in[idx], shift, RADIX_BINS - 1)], 1u);
    }
    __syncthreads();
    counts[(uint64_t)tid * n_tiles + blockIdx.x] = s_h[tid];
}

template <typename K>
__global__ __launch_bounds__(RADIX_THREADS) void radix_scatter(const K *__restrict__ in, K *__restrict__ out,
                                                               uint64_t n, int shift,
                                                               const uint32_t *__restrict__ starts,
                                                               uint64_t n_tiles) {
    constexpr int ITEMS = Tile<K>::ITEMS;
    constexpr int TILE = RADIX_THREADS * ITEMS;
    __shared__ uint32_t s_wcnt[RADIX_WAVES][RADIX_BINS];  // per-wave digit counters, then offsets
    __shared__ uint32_t s_dstart[RADIX_BINS];              // tile-local start of each digit
    __shared__ uint32_t s_gstart[RADIX_BINS];              // global start of each digit
    __shared__ K s_keys[TILE];
    const int tid = threadIdx.x;
    const int wave = tid / WAVE;
    const uint32_t lane = lane_id();
    const uint64_t tile = blockIdx.x;
    for (int i = tid; i < RADIX_WAVES * RADIX_BINS; i += RADIX_THREADS)
        (&s_wcnt[0][0])[i] = 0;
    s_gstart[tid] = starts[(uint64_t)tid * n_tiles + tile];
    __syncthreads();

    const uint64_t wbase = tile * TILE + (uint64_t)wave * (ITEMS * WAVE);
    K keys[ITEMS];
    uint32_t rank[ITEMS];
    uint32_t dig[ITEMS];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint64_t idx = wbase + (uint64_t)i * WAVE + lane;
        keys[i] = idx < n ? in[idx] : K{};
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint64_t idx = wbase + (uint64_t)i * WAVE + lane;
        const bool act = idx < n;
        const uint32_t d = digit_of(keys[i], shift, RADIX_BINS - 1);
        dig[i] = d;
        // lanes holding the same digit (match over the 8 digit bits)
        uint64_t peers = __ballot(act);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = __popcll(peers & lt);
        const uint32_t prior = s_wcnt[wave][d];
        // the lowest lane of each group advances the wave's counter; all
        // lanes of the wave have read it above (LDS ops of a wave are ordered)
        if (act && below == 0)
            s_wcnt[wave][d] = prior + (uint32_t)__popcll(peers);
        rank[i] = prior + below;
    }
    __syncthreads();
    {
        const int d = tid;  // RADIX_THREADS == RADIX_BINS
        uint32_t c[RADIX_WAVES];
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < RADIX_WAVES; w++) {
            c[w] = s_wcnt[w][d];
            tot += c[w];
        }
        uint32_t all;
        const uint32_t ex = block_exclusive_sum<RADIX_THREADS>(tot, &all);
        s_dstart[d] = ex;
        uint32_t run = ex;
#pragma unroll
        for (int w = 0; w < RADIX_WAVES; w++) {
            s_wcnt[w][d] = run;  // only thread d touches column d
            run += c[w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint64_t idx = wbase + (uint64_t)i * WAVE + lane;
        if (idx < n)
            s_keys[s_wcnt[wave][dig[i]] + rank[i]] = keys[i];
    }
    __syncthreads();
    const uint64_t left = n - tile * TILE;
    const uint32_t tile_n = left < (uint64_t)TILE ? (uint32_t)left : (uint32_t)TILE;
    for (uint32_t j = tid; j < tile_n; j += RADIX_THREADS) {
        const K key = s_keys[j];
        const uint32_t d = digit_of(key, shift, RADIX_BINS - 1);
        out[(uint64_t)s_gstart[d] + (j - s_dstart[d])] = key;
    }
}

template <typename K>
hipError_t sort_impl(K *keys, K *alt, uint64_t n, int key_bits, void *scratch, size_t scratch_bytes,
                     hipStream_t stream, K **sorted, int *passes) {
    *sorted = keys;
    *passes = 0;
    if (n <= 1)
        return hipSuccess;
    const uint64_t n_tiles = ceil_div(n, tile_size<K>());
    const uint64_t n_counts = n_tiles * RADIX_BINS;
    uint32_t *counts = static_cast<uint32_t *>(scratch);
    uint32_t *total = counts + n_counts;
    uint32_t *scan_tmp = total + 1;
    if ((n_counts + 1 + scan_scratch_words(n_counts)) * sizeof(uint32_t) > scratch_bytes)
        return hipErrorInvalidValue;
    K *src = keys, *dst = alt;
    for (int shift = 0; shift < key_bits; shift += RADIX_BITS) {
        radix_hist<K><<<dim3((unsigned)n_tiles), dim3(RADIX_THREADS), 0, stream>>>(src, n, shift, counts, n_tiles);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        e = launch_exclusive_scan(counts, counts, n_counts, scan_tmp, total, stream);
        if (e != hipSuccess)
            return e;
        radix_scatter<K><<<dim3((unsigned)n_tiles), dim3(RADIX_THREADS), 0, stream>>>(src, dst, n, shift, counts,
                                                                                     n_tiles);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        K *t = src;
        src = dst;
        dst = t;
        ++*passes;
    }
    *sorted = src;
    return hipSuccess;
}

}  // namespace

size_t radix_scratch_bytes(uint64_t n, int key_words) {
    const uint64_t tile = key_words == 2 ? tile_size<Key2>() : tile_size<uint64_t>();
    const uint64_t n_counts = ceil_div(n ? n : 1, tile) * RADIX_BINS;
    return (n_counts + 1 + scan_scratch_words(n_counts)) * sizeof(uint32_t);
}

hipError_t radix_sort(uint64_t *keys, uint64_t *alt, uint64_t n, int key_words, int key_bits, void *scratch,
                      size_t scratch_bytes, hipStream_t stream, uint64_t **sorted, int *passes) {
    if (key_words == 2) {
        Key2 *out = nullptr;
        hipError_t e = sort_impl<Key2>(reinterpret_cast<Key2 *>(keys), reinterpret_cast<Key2 *>(alt), n, key_bits,
                                       scratch, scratch_bytes, stream, &out, passes);
        *sorted = reinterpret_cast<uint64_t *>(out);
        return e;
    }
    uint64_t *out = nullptr;
    hipError_t e = sort_impl<uint64_t>(keys, alt, n, key_bits, scratch, scratch_bytes, stream, &out, passes);
    *sorted = out;
    return e;
}

}  // namespace tk
