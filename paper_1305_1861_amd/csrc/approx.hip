// Approximate one-pass variants of the paper, kept for their error rates
// against the exact path:
//   cTurtle (§2.2): a pattern-blocked counting Bloom filter.  The first
//     sighting of a k-mer sets its first pattern in block h(x); a later
//     sighting that finds those bits set checks its second pattern in the
//     next block: if not all set, it sets them and reports the k-mer (once).
//     Reports k-mers seen more than once, without counts; false positives
//     (first stage) and false negatives (second stage) come from collisions.
//   single pass with "+1" (§2.1, Algorithm 1 as printed): a sighting that
//     finds its pattern set is stored; the count is the number of stored
//     sightings plus one, which over-counts by one when the first sighting
//     was a false positive.
// A block here is one 64-bit word and every stage is one atomicOr, so a
// k-mer whose words no other k-mer touches goes through the stages exactly
// as in a sequential run, whatever the order of the lanes.
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int AP_THREADS = 256;
constexpr int AP_BUF = 2048;  // reported keys staged per block

template <bool TWO, bool CTURTLE>
__global__ __launch_bounds__(AP_THREADS) void approx_kernel(const uint64_t *__restrict__ packed,
                                                            const uint32_t *__restrict__ valid, uint64_t n_words,
                                                            int k, const uint64_t *__restrict__ table,
                                                            uint32_t table_bits, uint64_t *__restrict__ filter,
                                                            uint64_t n_fw, typename KeyOf<TWO>::type *__restrict__ out,
                                                            uint64_t capacity, unsigned long long *__restrict__ n_out) {
    using K = typename KeyOf<TWO>::type;
    __shared__ uint64_t s_table[1024];
    __shared__ K s_buf[AP_BUF];
    __shared__ uint32_t s_wc[AP_THREADS / WAVE];
    __shared__ uint32_t s_n;
    __shared__ unsigned long long s_base;
    BlockAppender<K, AP_THREADS, AP_BUF> app{s_buf, s_wc, &s_n, &s_base, out, capacity, n_out};
    const uint32_t n_tab = 1u << table_bits, tm = n_tab - 1;
    for (uint32_t i = threadIdx.x; i < n_tab; i += AP_THREADS)
        s_table[i] = table[i];
    app.init();  // (its barrier also publishes the table)
    const uint64_t n_pos = n_words * 32;
    const uint64_t stride = (uint64_t)gridDim.x * AP_THREADS;
    // every lane of a block runs the same number of iterations (wave ballots)
    for (uint64_t base = (uint64_t)blockIdx.x * AP_THREADS; base < n_pos; base += stride) {
        const uint64_t p = base + threadIdx.x;
        bool emit = false;
        K key{};
        if (p < n_pos) {
            const uint64_t w = p >> 5;
            const uint32_t t = (uint32_t)p & 31u;
            if ((valid[w] >> t) & 1u) {
                key = KeyOf<TWO>::get(packed, w, t, k);
                const uint64_t h = key_hash(key);
                const uint64_t w1 = __umul64hi(h, n_fw);
                const uint64_t m1 = s_table[h & tm] | s_table[(h >> table_bits) & tm];
                // Bits are only ever set: a read that finds a pattern's bits
                // all set decides exactly as the atomic would have (which
                // would change nothing), so the atomic is issued only when
                // the read finds a bit missing (a stale read only costs it).
                bool seen = (filter[w1] & m1) == m1;
                if (!seen) {
                    const uint64_t old1 = __hip_atomic_fetch_or(filter + w1, m1, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                    seen = (old1 & m1) == m1;
                }
                if (seen) {
                    if (CTURTLE) {
                        const uint64_t w2 = w1 + 1 < n_fw ? w1 + 1 : 0;
                        const uint64_t m2 = s_table[(h >> (2 * table_bits)) & tm] |
                                            s_table[(h >> (3 * table_bits)) & tm];
                        if ((filter[w2] & m2) != m2) {
                            const uint64_t old2 = __hip_atomic_fetch_or(filter + w2, m2, __ATOMIC_RELAXED,
                                                                        __HIP_MEMORY_SCOPE_AGENT);
                            emit = (old2 & m2) != m2;
                        }
                    } else {
                        emit = true;
                    }
                }
            }
        }
        app.push(emit, key);
    }
    app.finish();
}

// counts[i] += add (or = 0 when add is 0)
__global__ __launch_bounds__(256) void adjust_counts(uint32_t *__restrict__ counts, const DevCounters *__restrict__ c,
                                                     uint32_t add) {
    const uint64_t n = c->n_out;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        counts[i] = add ? counts[i] + add : 0u;
}

}  // namespace

hipError_t launch_approx(const uint64_t *packed, const uint32_t *valid, uint64_t n_words, int k,
                         const uint64_t *table, uint32_t table_bits, uint64_t *filter, uint64_t n_filter_words,
                         bool cturtle, void *out, uint64_t capacity, unsigned long long *n_out, int grid,
                         hipStream_t stream) {
    if (n_words == 0)
        return hipSuccess;
    const dim3 g(grid), b(AP_THREADS);
    if (k > 31) {
        if (cturtle)
            approx_kernel<true, true><<<g, b, 0, stream>>>(packed, valid, n_words, k, table, table_bits, filter,
                                                           n_filter_words, static_cast<Key2 *>(out), capacity, n_out);
        else
            approx_kernel<true, false><<<g, b, 0, stream>>>(packed, valid, n_words, k, table, table_bits, filter,
                                                            n_filter_words, static_cast<Key2 *>(out), capacity, n_out);
    } else {
        if (cturtle)
            approx_kernel<false, true><<<g, b, 0, stream>>>(packed, valid, n_words, k, table, table_bits, filter,
                                                            n_filter_words, static_cast<uint64_t *>(out), capacity,
                                                            n_out);
        else
            approx_kernel<false, false><<<g, b, 0, stream>>>(packed, valid, n_words, k, table, table_bits, filter,
                                                             n_filter_words, static_cast<uint64_t *>(out), capacity,
                                                             n_out);
    }
    return hipGetLastError();
}

hipError_t launch_adjust_counts(uint32_t *counts, const DevCounters *c, uint32_t add, hipStream_t stream) {
    adjust_counts<<<dim3((unsigned)std::min<int>(device_cu_count() * 8, 65535)), dim3(256), 0, stream>>>(counts, c,
                                                                                                        add);
    return hipGetLastError();
}

}  // namespace tk
