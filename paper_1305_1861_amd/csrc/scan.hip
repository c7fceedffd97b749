// Exclusive prefix sum of uint32 arrays (reduce, scan of block sums,
// down-sweep).  Used for radix histograms and compaction offsets; all sums
// stay below 2^32 because every count is bounded by the number of bases.
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr uint64_t SCAN_TILE = (uint64_t)SCAN_THREADS * SCAN_ITEMS;  // 4096
constexpr int PART_THREADS = 1024;

// Each thread sums SCAN_ITEMS consecutive values of the block's tile.
__global__ __launch_bounds__(SCAN_THREADS) void scan_reduce(const uint32_t *__restrict__ in, uint64_t n,
                                                            uint32_t *__restrict__ partials) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++)
        if (base + i < n)
            s += in[base + i];
    uint32_t total;
    block_exclusive_sum<SCAN_THREADS>(s, &total);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = total;
}

// One block scans the block sums in chunks, carrying the running total.
__global__ __launch_bounds__(PART_THREADS) void scan_partials(uint32_t *__restrict__ partials, uint64_t n_parts,
                                                              uint32_t *__restrict__ total) {
    uint32_t carry = 0;
    for (uint64_t c0 = 0; c0 < n_parts; c0 += PART_THREADS) {
        const uint64_t i = c0 + threadIdx.x;
        const uint32_t v = i < n_parts ? partials[i] : 0;
        uint32_t chunk;
        const uint32_t ex = block_exclusive_sum<PART_THREADS>(v, &chunk);
        if (i < n_parts)
            partials[i] = carry + ex;
        carry += chunk;
    }
    if (threadIdx.x == 0)
        *total = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                          uint64_t n, const uint32_t *__restrict__ partials) {
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_sum<SCAN_THREADS>(s, &total) + partials[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        if (base + i < n)
            out[base + i] = run;
        run += v[i];
    }
}

}  // namespace

uint64_t scan_scratch_words(uint64_t n) { return ceil_div(n, SCAN_TILE) + 1; }

hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *scratch, uint32_t *total,
                                 hipStream_t stream) {
    const uint64_t parts = ceil_div(n, SCAN_TILE);
    if (parts) {
        scan_reduce<<<dim3((unsigned)parts), dim3(SCAN_THREADS), 0, stream>>>(in, n, scratch);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    scan_partials<<<dim3(1), dim3(PART_THREADS), 0, stream>>>(scratch, parts, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !parts)
        return e;
    scan_down<<<dim3((unsigned)parts), dim3(SCAN_THREADS), 0, stream>>>(in, out, n, scratch);
    return hipGetLastError();
}

}  // namespace tk
