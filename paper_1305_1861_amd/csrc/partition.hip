// Partitioning of the window keys by their top D bits (D <= 20) -- the GPU
// counterpart of routing every k-mer to the consumer that owns its filter
// (paper §2.1, parallelization): afterwards every bucket (keys sharing their
// top D bits) is one contiguous range and the buckets are in key order, so
// per-bucket sort-and-compact results concatenate into the sorted answer.
//
// Pass 1 extracts the canonical keys straight from the packed reads (§2.1,
// k-mer extraction) and orders them by their top D1 = min(D, 10) bits
// ("segments").  When D > 10, pass 2 orders every segment by the next
// D2 = D - 10 bits.  The order of keys inside a bucket is not kept -- the
// bucket kernel sorts each bucket -- so both passes rank keys with LDS atomic
// counters instead of a stable ranking.
//
// Work unit: a chunk of up to PT_CH tiles, one workgroup each.  hist counts
// the chunk's digits; the counts are laid out so that one exclusive scan
// gives every (chunk, digit) its write position.  scatter, per tile: rank
// every key within its digit (LDS atomics), stage the tile in LDS in digit
// order, write each digit's run contiguously at the chunk's cursor for that
// digit.  Pass-2 chunks never straddle a segment: chunk j of segment s covers
// keys [seg[s] + j * CHUNK, min(seg[s] + (j + 1) * CHUNK, seg[s + 1])).
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int PT_THREADS = 1024;
constexpr int PT_WAVES = PT_THREADS / WAVE;
constexpr int PT_MAX_BITS = 10;
constexpr int PT_MAX_BINS = 1 << PT_MAX_BITS;
constexpr int PT_BPT = PT_MAX_BINS / PT_THREADS;  // digit bins per thread
constexpr int PT_CH = 8;                          // tiles per chunk
constexpr int SEG_THREADS = 1024;                 // one thread per segment
static_assert(PT_BPT * PT_THREADS == PT_MAX_BINS, "bins spread evenly over the threads");

template <typename K>
struct PtItems;
template <>
struct PtItems<uint64_t> {
    static constexpr int value = 16;  // 16384 keys per tile (128 KB of LDS)
};
template <>
struct PtItems<Key2> {
    static constexpr int value = 8;  // 8192 keys per tile (128 KB of LDS)
};

template <typename K>
constexpr uint64_t pt_tile() {
    return (uint64_t)PT_THREADS * PtItems<K>::value;
}
template <typename K>
constexpr uint64_t pt_chunk() {
    return pt_tile<K>() * PT_CH;
}

// Segment s and chunk index j of pass-2 workgroup b; false for workgroups
// beyond the last chunk.  cb[s] is the first chunk of segment s, cb[nseg]
// the number of chunks.
__device__ __forceinline__ bool seg_chunk(const uint32_t *__restrict__ cb, uint32_t nseg, uint32_t b, uint32_t &s,
                                          uint32_t &j) {
    if (b >= cb[nseg])
        return false;
    uint32_t lo = 0, hi = nseg;  // largest s with cb[s] <= b
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (cb[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    s = lo;
    j = b - cb[lo];
    return true;
}

// Keys of one tile into registers.  Pass 1: the tile is PT_TILE window
// positions; thread t takes ITEMS consecutive windows of one packed word.
// Pass 2: keys [k0, k1) of the pass-1 output, item-major.  Bit i of the
// result: item i holds a key.
template <typename K, bool FROM_WIN>
__device__ __forceinline__ uint32_t load_tile(const PartArgs &a, uint64_t t0, uint64_t t1, K (&key)[PtItems<K>::value]) {
    constexpr int ITEMS = PtItems<K>::value;
    const int tid = threadIdx.x;
    uint32_t vm = 0;
    if (FROM_WIN) {
        constexpr int PER_WORD = 32 / ITEMS;  // threads per packed word
        const uint64_t w = t0 / 32 + (uint64_t)(tid / PER_WORD);
        const uint32_t first = (uint32_t)(tid % PER_WORD) * ITEMS;
        if (w * 32 + first < t1) {
            const uint64_t w0 = a.packed[w];
            const uint64_t w1 = w ? a.packed[w - 1] : 0;
            const uint64_t w2 = (std::is_same<K, Key2>::value && w > 1) ? a.packed[w - 2] : 0;
            const uint32_t ok = (a.valid[w] >> first) & (ITEMS == 32 ? ~0u : (1u << (ITEMS & 31)) - 1u);
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                key[i] = K{};
                if ((ok >> i) & 1u) {
                    key[i] = KeyOf<std::is_same<K, Key2>::value>::get(w0, w1, w2, first + i, a.k);
                    vm |= 1u << i;
                }
            }
        }
    } else {
        const K *__restrict__ in = static_cast<const K *>(a.keys_in);
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint64_t e = t0 + (uint64_t)i * PT_THREADS + tid;
            key[i] = K{};
            if (e < t1) {
                key[i] = in[e];
                vm |= 1u << i;
            }
        }
    }
    return vm;
}

// Element range of the chunk this workgroup owns: [c0, c1).
template <typename K, bool FROM_WIN>
__device__ __forceinline__ bool chunk_range(const PartArgs &a, uint64_t &c0, uint64_t &c1, uint64_t &hidx,
                                            uint32_t &hstride) {
    const uint32_t b = blockIdx.x;
    if (FROM_WIN) {
        c0 = (uint64_t)b * pt_chunk<K>();
        c1 = min(c0 + pt_chunk<K>(), a.n_elems);
        hidx = b;                        // entry of digit d: d * n_chunks + b
        hstride = (uint32_t)a.n_chunks;  // chunks of pass 1
        return c0 < c1;
    }
    uint32_t s, j;
    if (!seg_chunk(a.cb, a.nseg, b, s, j))
        return false;
    const uint64_t s0 = a.seg[s], s1 = a.seg[s + 1];
    c0 = s0 + (uint64_t)j * pt_chunk<K>();
    c1 = min(c0 + pt_chunk<K>(), s1);
    const uint32_t nch = a.cb[s + 1] - a.cb[s];
    hidx = (uint64_t)a.cb[s] * (1u << a.bits) + j;  // entry of digit d: cb[s] * bins + d * nch + j
    hstride = nch;
    return true;
}

template <typename K, bool FROM_WIN>
__global__ __launch_bounds__(PT_THREADS) void pt_hist(PartArgs a, uint32_t *__restrict__ hist) {
    constexpr int ITEMS = PtItems<K>::value;
    __shared__ uint32_t s_h[PT_MAX_BINS];
    const int tid = threadIdx.x;
    const uint32_t bins = 1u << a.bits, mask = bins - 1;
    uint64_t c0, c1, hidx;
    uint32_t hstride;
    if (!chunk_range<K, FROM_WIN>(a, c0, c1, hidx, hstride)) {
        if (!FROM_WIN) {
            // beyond the last pass-2 chunk: clear this block's share of the
            // unused tail of the count array
            const uint64_t z = (uint64_t)blockIdx.x * bins;
            for (uint32_t d = tid; d < bins; d += PT_THREADS)
                hist[z + d] = 0;
        }
        return;
    }
    for (int d = tid; d < PT_MAX_BINS; d += PT_THREADS)
        s_h[d] = 0;
    __syncthreads();
    for (uint64_t t0 = c0; t0 < c1; t0 += pt_tile<K>()) {
        K key[ITEMS];
        const uint32_t vm = load_tile<K, FROM_WIN>(a, t0, min(t0 + pt_tile<K>(), c1), key);
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
            if ((vm >> i) & 1u)
                atomicAdd(&s_h[digit_of(key[i], a.shift, mask)], 1u);
    }
    __syncthreads();
    for (uint32_t d = tid; d < bins; d += PT_THREADS)
        hist[hidx + (uint64_t)d * hstride] = s_h[d];
}

template <typename K, bool FROM_WIN>
__global__ __launch_bounds__(PT_THREADS) void pt_scatter(PartArgs a, const uint32_t *__restrict__ offs,
                                                         K *__restrict__ out) {
    constexpr int ITEMS = PtItems<K>::value;
    constexpr int TILE = PT_THREADS * ITEMS;
    __shared__ uint32_t s_cnt[PT_MAX_BINS];  // digit counts of the tile, then their starts
    __shared__ uint32_t s_cur[PT_MAX_BINS];  // write position of each digit
    __shared__ uint32_t s_wt[PT_WAVES];
    __shared__ K s_stage[TILE];
    const int tid = threadIdx.x;
    const int wave = tid / WAVE;
    const uint32_t lane = lane_id();
    const uint32_t bins = 1u << a.bits, mask = bins - 1;
    uint64_t c0, c1, hidx;
    uint32_t hstride;
    if (!chunk_range<K, FROM_WIN>(a, c0, c1, hidx, hstride))
        return;  // uniform over the block
    // thread t owns digits t * PT_BPT .. t * PT_BPT + PT_BPT - 1
    const uint32_t d0 = (uint32_t)tid * PT_BPT;
#pragma unroll
    for (int j = 0; j < PT_BPT; j++) {
        if (d0 + j < bins)
            s_cur[d0 + j] = offs[hidx + (uint64_t)(d0 + j) * hstride];
        s_cnt[d0 + j] = 0;
    }
    __syncthreads();
    for (uint64_t t0 = c0; t0 < c1; t0 += TILE) {
        K key[ITEMS];
        const uint32_t vm = load_tile<K, FROM_WIN>(a, t0, min(t0 + (uint64_t)TILE, c1), key);
        uint32_t rd[ITEMS];  // (rank << 10) | digit
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            rd[i] = 0;
            if ((vm >> i) & 1u) {
                const uint32_t d = digit_of(key[i], a.shift, mask);
                rd[i] = (atomicAdd(&s_cnt[d], 1u) << PT_MAX_BITS) | d;
            }
        }
        __syncthreads();
        // starts of the digits in the tile
        uint32_t c[PT_BPT];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < PT_BPT; j++) {
            c[j] = s_cnt[d0 + j];
            sum += c[j];
        }
        const uint32_t inc = wave_inclusive_sum(sum);
        if (lane == WAVE - 1)
            s_wt[wave] = inc;
        __syncthreads();
        uint32_t before = 0, n_tile = 0;
#pragma unroll
        for (int w = 0; w < PT_WAVES; w++) {
            const uint32_t t = s_wt[w];
            before += w < wave ? t : 0u;
            n_tile += t;
        }
        uint32_t run = before + inc - sum;
#pragma unroll
        for (int j = 0; j < PT_BPT; j++) {
            s_cnt[d0 + j] = run;
            run += c[j];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
            if ((vm >> i) & 1u)
                s_stage[s_cnt[rd[i] & (PT_MAX_BINS - 1)] + (rd[i] >> PT_MAX_BITS)] = key[i];
        __syncthreads();
        // each digit's run goes to its cursor; consecutive threads write
        // consecutive positions of a run
        for (uint32_t j = tid; j < n_tile; j += PT_THREADS) {
            const K x = s_stage[j];
            const uint32_t d = digit_of(x, a.shift, mask);
            out[(uint64_t)s_cur[d] + (j - s_cnt[d])] = x;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PT_BPT; j++) {
            if (d0 + j < bins)
                s_cur[d0 + j] += c[j];
            s_cnt[d0 + j] = 0;
        }
        __syncthreads();
    }
}

// Segment starts and the first pass-2 chunk of each segment, from the
// scanned pass-1 counts (entry d * n_chunks of the scan is the start of
// digit d).  One block.
template <typename K>
__global__ __launch_bounds__(SEG_THREADS) void pt_segments(const uint32_t *__restrict__ offs1, uint64_t n_chunks1,
                                                          uint32_t nseg, const uint32_t *__restrict__ total,
                                                          uint32_t *__restrict__ seg, uint32_t *__restrict__ cb) {
    const uint32_t s = threadIdx.x;
    const uint32_t n = *total;
    uint32_t start = n, end = n;
    if (s < nseg)
        start = offs1[(uint64_t)s * n_chunks1];
    if (s + 1 < nseg)
        end = offs1[(uint64_t)(s + 1) * n_chunks1];
    const uint32_t ch = s < nseg ? (uint32_t)(((uint64_t)(end - start) + pt_chunk<K>() - 1) / pt_chunk<K>()) : 0u;
    uint32_t n_ch;
    const uint32_t first = block_exclusive_sum<SEG_THREADS>(ch, &n_ch);
    if (s < nseg) {
        seg[s] = start;
        cb[s] = first;
    }
    if (s == 0) {
        seg[nseg] = n;
        cb[nseg] = n_ch;
    }
}

template <typename K>
hipError_t run_partition(const PartArgs &a0, void *tmp, void *out, uint32_t *scratch, size_t scratch_words,
                         uint32_t *total, uint32_t *total2, hipStream_t stream) {
    const int D = a0.bits;
    const int D1 = D < PT_MAX_BITS ? D : PT_MAX_BITS;
    const int D2 = D - D1;
    if (D < 0 || D2 > PT_MAX_BITS || 2 * a0.k < D)
        return hipErrorInvalidValue;
    const uint64_t n_pos = a0.n_elems;  // window positions
    uint32_t *seg = scratch;
    uint32_t *cb = scratch + (PT_MAX_BINS + 1);
    uint32_t *hist = scratch + 2 * (PT_MAX_BINS + 1);
    const size_t hist_words = scratch_words - 2 * (PT_MAX_BINS + 1);
    const dim3 block(PT_THREADS);

    // pass 1: windows -> (D2 ? tmp : out), by the top D1 bits
    PartArgs a = a0;
    a.shift = 2 * a0.k - D1;
    a.bits = D1;
    a.n_chunks = ceil_div(n_pos ? n_pos : 1, pt_chunk<K>());
    const uint64_t n_hist1 = a.n_chunks << D1;
    if (n_hist1 + scan_scratch_words(n_hist1) > hist_words)
        return hipErrorInvalidValue;
    void *out1 = D2 ? tmp : out;
    if (n_pos) {
        pt_hist<K, true><<<dim3((unsigned)a.n_chunks), block, 0, stream>>>(a, hist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    } else {
        a.n_chunks = 0;
    }
    hipError_t e = launch_exclusive_scan(hist, hist, a.n_chunks << D1, hist + n_hist1, total, stream);
    if (e != hipSuccess)
        return e;
    if (!n_pos)
        return hipSuccess;  // no key: nothing to move
    pt_scatter<K, true><<<dim3((unsigned)a.n_chunks), block, 0, stream>>>(a, hist, static_cast<K *>(out1));
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (!D2)
        return hipSuccess;

    // pass 2: tmp -> out, each segment by the next D2 bits
    const uint32_t nseg = 1u << D1;
    pt_segments<K><<<dim3(1), dim3(SEG_THREADS), 0, stream>>>(hist, a.n_chunks, nseg, total, seg, cb);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    PartArgs b = a0;
    b.keys_in = tmp;
    b.shift = 2 * a0.k - D;
    b.bits = D2;
    b.seg = seg;
    b.cb = cb;
    b.nseg = nseg;
    const uint64_t grid2 = ceil_div(n_pos, pt_chunk<K>()) + nseg;  // bound on the number of chunks
    const uint64_t n_hist2 = grid2 << D2;
    if (n_hist2 + scan_scratch_words(n_hist2) > hist_words)
        return hipErrorInvalidValue;
    pt_hist<K, false><<<dim3((unsigned)grid2), block, 0, stream>>>(b, hist);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = launch_exclusive_scan(hist, hist, n_hist2, hist + n_hist2, total2, stream)) != hipSuccess)
        return e;
    pt_scatter<K, false><<<dim3((unsigned)grid2), block, 0, stream>>>(b, hist, static_cast<K *>(out));
    return hipGetLastError();
}

}  // namespace

size_t partition_scratch_words(uint64_t n_pos, int key_words) {
    const uint64_t chunk = key_words == 2 ? pt_chunk<Key2>() : pt_chunk<uint64_t>();
    const uint64_t n1 = ceil_div(n_pos ? n_pos : 1, chunk) << PT_MAX_BITS;
    const uint64_t n2 = (ceil_div(n_pos, chunk) + PT_MAX_BINS) << PT_MAX_BITS;
    const uint64_t h = std::max(n1 + scan_scratch_words(n1), n2 + scan_scratch_words(n2));
    return 2 * (PT_MAX_BINS + 1) + h;
}

hipError_t partition_keys(const PartArgs &a, void *tmp, void *out, uint32_t *scratch, size_t scratch_words,
                          uint32_t *total, uint32_t *total2, hipStream_t stream) {
    return a.k > 31 ? run_partition<Key2>(a, tmp, out, scratch, scratch_words, total, total2, stream)
                    : run_partition<uint64_t>(a, tmp, out, scratch, scratch_words, total, total2, stream);
}

}  // namespace tk
