// K2 screen and K3 collect: fused canonical k-mer extraction and the
// two-plane pattern-blocked Bloom filter.
//
// Paper §2.1 (Identification of frequent k-mers with Pattern-blocked Bloom
// Filter; Algorithm 1): a key selects one block of the filter by a hash and
// sets a precomputed pattern of bits inside it, so each test/update touches a
// single cache line.  Paper §2.1 (k-mer extraction): the key of a window is
// the smaller of its forward and reverse-complement encodings.
//
// Filter block (64 bytes, 8 words): words 0..3 = first plane S, words 4..7 =
// second plane T.  The pattern is multiplexed from one table: word w of the
// block gets entry (h >> (w * table_bits)) mod 2^table_bits.
//
// screen : for every valid window, old = atomicOr(S[w], m_w) and, for the
//          bits that were already set, atomicOr(T[w], old & m_w), skipped for
//          words whose bits are all in T already.  A T bit is set iff its
//          position was touched at least twice, in any order.
// collect: a window is a candidate iff all its pattern bits are set in T.
//          Candidates are staged per block in LDS (ballot + popcount for
//          the lane offsets) and appended a buffer at a time with one
//          atomicAdd.  Every key seen at least twice is a candidate.
//
// Threads map one-to-one onto base positions: position p = 32w + t is the
// last base of the window handled by that lane.  A persistent grid strides
// over the positions so the pattern table is loaded into LDS once per block.
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int BLOOM_THREADS = 256;

__device__ __forceinline__ void load_table(const uint64_t *__restrict__ table, uint32_t n, uint64_t *s_table) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        s_table[i] = table[i];
    __syncthreads();
}

template <bool TWO>
__global__ __launch_bounds__(BLOOM_THREADS) void screen_kernel(BloomArgs a) {
    extern __shared__ uint64_t s_table[];
    const uint32_t n_tab = 1u << a.table_bits;
    load_table(a.table, n_tab, s_table);
    const uint64_t n_pos = a.n_words * 32;
    const uint64_t stride = (uint64_t)gridDim.x * BLOOM_THREADS;
    for (uint64_t p = (uint64_t)blockIdx.x * BLOOM_THREADS + threadIdx.x; p < n_pos; p += stride) {
        const uint64_t w = p >> 5;
        const uint32_t t = (uint32_t)p & 31u;
        if (!((a.valid[w] >> t) & 1u))
            continue;
        const auto key = KeyOf<TWO>::get(a.packed, w, t, a.k);
        const uint64_t h = key_hash(key);
        const uint64_t blk = __umul64hi(h, a.n_blocks);
        uint64_t *b = a.filter + blk * 8;
        uint64_t m[4];
#pragma unroll
        for (int i = 0; i < 4; i++)
            m[i] = s_table[(h >> (i * a.table_bits)) & (n_tab - 1)];
        // Bits are only ever set and a T bit implies its S bit, so a word
        // whose pattern bits are already all in T needs neither atomic: the
        // T half of the block (the same cache line) is read first.  A stale
        // read only costs atomics that change nothing.
        const ulonglong2 *tp = reinterpret_cast<const ulonglong2 *>(b + 4);
        const ulonglong2 t01 = tp[0], t23 = tp[1];
        const uint64_t tw[4] = {t01.x, t01.y, t23.x, t23.y};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            if ((tw[i] & m[i]) == m[i])
                continue;
            const uint64_t old = __hip_atomic_fetch_or(b + i, m[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t again = old & m[i];
            if (again)
                __hip_atomic_fetch_or(b + 4 + i, again, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

constexpr int COLLECT_BUF = 2048;  // candidates staged per block

template <bool TWO, bool SCREEN>
__global__ __launch_bounds__(BLOOM_THREADS) void collect_kernel(BloomArgs a, typename KeyOf<TWO>::type *__restrict__ out,
                                                                uint64_t capacity,
                                                                unsigned long long *__restrict__ n_out) {
    using K = typename KeyOf<TWO>::type;
    extern __shared__ uint64_t s_table[];
    __shared__ K s_buf[COLLECT_BUF];
    __shared__ uint32_t s_wc[BLOOM_THREADS / WAVE];
    __shared__ uint32_t s_n;
    __shared__ unsigned long long s_base;
    const uint32_t n_tab = 1u << a.table_bits;
    if (SCREEN)
        load_table(a.table, n_tab, s_table);
    const int tid = threadIdx.x;
    BlockAppender<K, BLOOM_THREADS, COLLECT_BUF> app{s_buf, s_wc, &s_n, &s_base, out, capacity, n_out};
    app.init();
    const uint64_t n_pos = a.n_words * 32;
    const uint64_t stride = (uint64_t)gridDim.x * BLOOM_THREADS;
    // every lane of a block runs the same number of iterations, so the wave
    // ballots and the barriers below always see every thread
    const uint64_t first = (uint64_t)blockIdx.x * BLOOM_THREADS;
    for (uint64_t base = first; base < n_pos; base += stride) {
        const uint64_t p = base + tid;
        bool cand = false;
        K key{};
        if (p < n_pos) {
            const uint64_t w = p >> 5;
            const uint32_t t = (uint32_t)p & 31u;
            if ((a.valid[w] >> t) & 1u) {
                key = KeyOf<TWO>::get(a.packed, w, t, a.k);
                if (SCREEN) {
                    const uint64_t h = key_hash(key);
                    const uint64_t blk = __umul64hi(h, a.n_blocks);
                    const ulonglong2 *tp = reinterpret_cast<const ulonglong2 *>(a.filter + blk * 8 + 4);
                    const ulonglong2 t01 = tp[0];
                    const ulonglong2 t23 = tp[1];
                    const uint64_t m0 = s_table[h & (n_tab - 1)];
                    const uint64_t m1 = s_table[(h >> a.table_bits) & (n_tab - 1)];
                    const uint64_t m2 = s_table[(h >> (2 * a.table_bits)) & (n_tab - 1)];
                    const uint64_t m3 = s_table[(h >> (3 * a.table_bits)) & (n_tab - 1)];
                    cand = ((t01.x & m0) == m0) & ((t01.y & m1) == m1) & ((t23.x & m2) == m2) &
                           ((t23.y & m3) == m3);
                } else {
                    cand = true;
                }
            }
        }
        app.push(cand, key);
    }
    app.finish();
}

}  // namespace

hipError_t launch_screen(const BloomArgs &a, int grid, hipStream_t stream) {
    if (a.n_words == 0)
        return hipSuccess;
    const size_t lds = sizeof(uint64_t) << a.table_bits;
    if (a.k <= 31)
        screen_kernel<false><<<dim3(grid), dim3(BLOOM_THREADS), lds, stream>>>(a);
    else
        screen_kernel<true><<<dim3(grid), dim3(BLOOM_THREADS), lds, stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_collect(const BloomArgs &a, bool screen, void *keys, uint64_t capacity,
                          unsigned long long *n_collected, int grid, hipStream_t stream) {
    if (a.n_words == 0)
        return hipSuccess;
    const size_t lds = screen ? sizeof(uint64_t) << a.table_bits : 0;
    if (a.k <= 31) {
        if (screen)
            collect_kernel<false, true><<<dim3(grid), dim3(BLOOM_THREADS), lds, stream>>>(
                a, static_cast<uint64_t *>(keys), capacity, n_collected);
        else
            collect_kernel<false, false><<<dim3(grid), dim3(BLOOM_THREADS), lds, stream>>>(
                a, static_cast<uint64_t *>(keys), capacity, n_collected);
    } else {
        if (screen)
            collect_kernel<true, true><<<dim3(grid), dim3(BLOOM_THREADS), lds, stream>>>(
                a, static_cast<Key2 *>(keys), capacity, n_collected);
        else
            collect_kernel<true, false><<<dim3(grid), dim3(BLOOM_THREADS), lds, stream>>>(
                a, static_cast<Key2 *>(keys), capacity, n_collected);
    }
    return hipGetLastError();
}

}  // namespace tk
