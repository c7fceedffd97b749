// Partitioning of the window keys by their top D bits (D <= 20) with at most
// two stable radix passes of <= 10-bit digits.  The first pass reads the
// windows straight from the packed reads (fused canonical extraction, paper
// §2.1 k-mer extraction); a second pass, when D > 10, reorders the keys by the
// upper digit.  After both, every partition ("bucket": keys sharing their top
// D bits) is one contiguous range and the buckets are in key order, so the
// per-bucket sort-and-compact results concatenate into the sorted answer.
//
// Each block owns a chunk of PT_SUBTILES sub-tiles.  hist: per-chunk digit
// counts -> hist[bin * n_chunks + chunk].  After an exclusive scan, scatter
// keeps one cursor per bin in LDS; for each sub-tile it ranks the keys by
// digit (wave match over the digit bits + per-wave counters), reorders them
// through LDS and writes each bin's run at its cursor.
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int PT_THREADS = 256;
constexpr int PT_WAVES = PT_THREADS / WAVE;
constexpr int PT_MAX_BITS = 10;
constexpr int PT_MAX_BINS = 1 << PT_MAX_BITS;
constexpr int PT_BINS_PER_THREAD = PT_MAX_BINS / PT_THREADS;  // 4
constexpr int PT_SUBTILES = 64;

template <typename K>
struct PtItems;
template <>
struct PtItems<uint64_t> {
    static constexpr int value = 16;  // 4096 keys per sub-tile
};
template <>
struct PtItems<Key2> {
    static constexpr int value = 8;  // 2048 keys per sub-tile
};

template <typename K>
constexpr uint64_t pt_sub() {
    return (uint64_t)PT_THREADS * PtItems<K>::value;
}

// Element e of the pass: a window position (FROM_WIN) or a key index.
template <typename K, bool FROM_WIN>
__device__ __forceinline__ bool load_elem(const PartArgs &a, uint64_t e, K &key) {
    if (FROM_WIN) {
        if (e >= a.n_elems)
            return false;
        const uint64_t w = e >> 5;
        const uint32_t t = (uint32_t)e & 31u;
        if (!((a.valid[w] >> t) & 1u))
            return false;
        key = KeyOf<std::is_same<K, Key2>::value>::get(a.packed, w, t, a.k);
        return true;
    }
    if (e >= a.n_elems)
        return false;
    key = static_cast<const K *>(a.keys_in)[e];
    return true;
}

__device__ __forceinline__ PartArgs resolve_count(PartArgs a) {
    if (a.n_dev)
        a.n_elems = min(a.n_elems, (uint64_t)*a.n_dev);
    return a;
}

template <typename K, bool FROM_WIN>
__global__ __launch_bounds__(PT_THREADS) void pt_hist(PartArgs a0, uint32_t *__restrict__ hist) {
    const PartArgs a = resolve_count(a0);
    __shared__ uint32_t s_h[PT_MAX_BINS];
    const int tid = threadIdx.x;
    const uint32_t bins = 1u << a.bits, mask = bins - 1;
    for (uint32_t b = tid; b < bins; b += PT_THREADS)
        s_h[b] = 0;
    __syncthreads();
    const uint64_t chunk = blockIdx.x;
    const uint64_t base = chunk * pt_sub<K>() * PT_SUBTILES;
    for (int st = 0; st < PT_SUBTILES; st++) {
        const uint64_t sbase = base + (uint64_t)st * pt_sub<K>();
        if (sbase >= a.n_elems)
            break;
#pragma unroll 4
        for (int i = 0; i < PtItems<K>::value; i++) {
            K key;
            if (load_elem<K, FROM_WIN>(a, sbase + (uint64_t)i * PT_THREADS + tid, key))
                atomicAdd(&s_h[digit_of(key, a.shift, mask)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t b = tid; b < bins; b += PT_THREADS)
        hist[(uint64_t)b * a.n_chunks + chunk] = s_h[b];
}

template <typename K, bool FROM_WIN>
__global__ __launch_bounds__(PT_THREADS) void pt_scatter(PartArgs a0, const uint32_t *__restrict__ offs,
                                                         K *__restrict__ out) {
    const PartArgs a = resolve_count(a0);
    constexpr int ITEMS = PtItems<K>::value;
    constexpr int SUB = PT_THREADS * ITEMS;
    __shared__ uint16_t s_cnt[PT_WAVES][PT_MAX_BINS];  // per-wave digit counters, then offsets
    __shared__ uint32_t s_dstart[PT_MAX_BINS];          // sub-tile-local start of each digit
    __shared__ uint32_t s_cursor[PT_MAX_BINS];          // global write position of each digit
    __shared__ K s_stage[SUB];
    const int tid = threadIdx.x;
    const int wave = tid / WAVE;
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const uint32_t bins = 1u << a.bits, mask = bins - 1;
    const uint64_t chunk = blockIdx.x;
    for (uint32_t b = tid; b < bins; b += PT_THREADS)
        s_cursor[b] = offs[(uint64_t)b * a.n_chunks + chunk];

    const uint64_t base = chunk * (uint64_t)SUB * PT_SUBTILES;
    for (int st = 0; st < PT_SUBTILES; st++) {
        const uint64_t sbase = base + (uint64_t)st * SUB;
        if (sbase >= a.n_elems)
            break;  // uniform over the block
        for (int i = tid; i < PT_WAVES * PT_MAX_BINS; i += PT_THREADS)
            (&s_cnt[0][0])[i] = 0;
        __syncthreads();

        K keys[ITEMS];
        uint32_t rank[ITEMS];
        uint32_t dig[ITEMS];
        bool act[ITEMS];
        const uint64_t wbase = sbase + (uint64_t)wave * (ITEMS * WAVE);
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
            act[i] = load_elem<K, FROM_WIN>(a, wbase + (uint64_t)i * WAVE + lane, keys[i]);
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint32_t d = act[i] ? digit_of(keys[i], a.shift, mask) : 0u;
            dig[i] = d;
            uint64_t peers = __ballot(act[i]);
            for (int b = 0; b < a.bits; b++) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            const uint32_t below = __popcll(peers & lt);
            const uint32_t prior = s_cnt[wave][d];
            if (act[i] && below == 0)
                s_cnt[wave][d] = (uint16_t)(prior + (uint32_t)__popcll(peers));
            rank[i] = prior + below;
        }
        __syncthreads();
        // digit totals, sub-tile starts and per-wave offsets; thread t owns
        // bins 4t .. 4t+3
        uint32_t tot[PT_BINS_PER_THREAD];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < PT_BINS_PER_THREAD; j++) {
            const uint32_t b = tid * PT_BINS_PER_THREAD + j;
            uint32_t t = 0;
            if (b < bins)
                for (int w = 0; w < PT_WAVES; w++)
                    t += s_cnt[w][b];
            tot[j] = t;
            sum += t;
        }
        uint32_t n_sub;
        uint32_t run = block_exclusive_sum<PT_THREADS>(sum, &n_sub);
#pragma unroll
        for (int j = 0; j < PT_BINS_PER_THREAD; j++) {
            const uint32_t b = tid * PT_BINS_PER_THREAD + j;
            if (b < bins) {
                s_dstart[b] = run;
                uint32_t r = run;
                for (int w = 0; w < PT_WAVES; w++) {
                    const uint32_t c = s_cnt[w][b];
                    s_cnt[w][b] = (uint16_t)r;
                    r += c;
                }
            }
            run += tot[j];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
            if (act[i])
                s_stage[s_cnt[wave][dig[i]] + rank[i]] = keys[i];
        __syncthreads();
        for (uint32_t j = tid; j < n_sub; j += PT_THREADS) {
            const K key = s_stage[j];
            const uint32_t d = digit_of(key, a.shift, mask);
            out[(uint64_t)s_cursor[d] + (j - s_dstart[d])] = key;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PT_BINS_PER_THREAD; j++) {
            const uint32_t b = tid * PT_BINS_PER_THREAD + j;
            if (b < bins)
                s_cursor[b] += tot[j];
        }
        __syncthreads();
    }
}

template <typename K, bool FROM_WIN>
hipError_t run_pass(const PartArgs &a0, void *out, uint32_t *scratch, size_t scratch_words, uint32_t *total,
                    hipStream_t stream) {
    PartArgs a = a0;
    a.n_chunks = ceil_div(a.n_elems ? a.n_elems : 1, pt_sub<K>() * PT_SUBTILES);
    const uint64_t n_hist = a.n_chunks << a.bits;
    if (a.bits < 0 || a.bits > PT_MAX_BITS || n_hist + scan_scratch_words(n_hist) > scratch_words)
        return hipErrorInvalidValue;
    uint32_t *hist = scratch;
    uint32_t *tmp = scratch + n_hist;
    const dim3 grid((unsigned)a.n_chunks), block(PT_THREADS);
    pt_hist<K, FROM_WIN><<<grid, block, 0, stream>>>(a, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if ((e = launch_exclusive_scan(hist, hist, n_hist, tmp, total, stream)) != hipSuccess)
        return e;
    pt_scatter<K, FROM_WIN><<<grid, block, 0, stream>>>(a, hist, static_cast<K *>(out));
    return hipGetLastError();
}

}  // namespace

size_t partition_scratch_words(uint64_t n_elems, int key_words) {
    const uint64_t per_chunk = (key_words == 2 ? pt_sub<Key2>() : pt_sub<uint64_t>()) * PT_SUBTILES;
    const uint64_t n_hist = ceil_div(n_elems ? n_elems : 1, per_chunk) << PT_MAX_BITS;
    return n_hist + scan_scratch_words(n_hist);
}

hipError_t partition_pass(const PartArgs &a, bool from_windows, void *out, uint32_t *scratch, size_t scratch_words,
                          uint32_t *total, hipStream_t stream) {
    const bool two = a.k > 31;
    if (from_windows)
        return two ? run_pass<Key2, true>(a, out, scratch, scratch_words, total, stream)
                   : run_pass<uint64_t, true>(a, out, scratch, scratch_words, total, stream);
    return two ? run_pass<Key2, false>(a, out, scratch, scratch_words, total, stream)
               : run_pass<uint64_t, false>(a, out, scratch, scratch_words, total, stream);
}

}  // namespace tk
