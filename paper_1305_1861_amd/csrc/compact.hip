// K5: run-length compaction of sorted keys and the count threshold.
//
// Paper §2.1 (Counting frequencies with sorting and compaction, Fig. 1):
// after sorting, one linear pass folds each run of equal k-mers into one item
// whose count is the run length (the paper likens it to run-length encoding);
// Algorithm 1 then reports the k-mers with their counts.  Here the counts are
// the true run lengths (every occurrence of a candidate was collected), so a
// Bloom false positive has count 1 and is dropped by the threshold c.
//
// Kernels (tiles of 4096 elements, wave-striped as in the radix sort):
//   heads_count : head[i] = (i == 0 || key[i] != key[i-1]); heads per tile
//   scan        : tile offsets of the heads; the total is the number of runs
//   heads_write : run_start[r] = index of the r-th head; run_start[R] = n
//   runs_count  : count[r] = run_start[r+1] - run_start[r]; kept per tile,
//                 singletons and 2 <= count < c tallied
//   scan        : tile offsets of the kept runs; the total is n_out
//   runs_write  : (key, count) of every kept run, in order
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int CT_THREADS = 256;
constexpr int CT_ITEMS = 16;
constexpr uint64_t CT_TILE = (uint64_t)CT_THREADS * CT_ITEMS;
constexpr int CT_WAVES = CT_THREADS / WAVE;

__device__ __forceinline__ uint64_t striped_index(uint64_t tile, int wave, int item, uint32_t lane) {
    return tile * CT_TILE + (uint64_t)wave * (CT_ITEMS * WAVE) + (uint64_t)item * WAVE + lane;
}

template <typename K>
__device__ __forceinline__ bool is_head(const K *__restrict__ keys, uint64_t i, uint64_t n) {
    return i < n && (i == 0 || keys[i] != keys[i - 1]);
}

template <typename K>
__global__ __launch_bounds__(CT_THREADS) void heads_count(const K *__restrict__ keys, uint64_t n,
                                                          uint32_t *__restrict__ tile_cnt) {
    const int wave = threadIdx.x / WAVE;
    const uint32_t lane = lane_id();
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < CT_ITEMS; i++)
        c += is_head(keys, striped_index(blockIdx.x, wave, i, lane), n);
    uint32_t total;
    block_exclusive_sum<CT_THREADS>(c, &total);
    if (threadIdx.x == 0)
        tile_cnt[blockIdx.x] = total;
}

template <typename K>
__global__ __launch_bounds__(CT_THREADS) void heads_write(const K *__restrict__ keys, uint64_t n,
                                                          const uint32_t *__restrict__ tile_off,
                                                          const uint32_t *__restrict__ n_runs,
                                                          uint32_t *__restrict__ run_start) {
    __shared__ uint32_t s_w[CT_WAVES];
    const int wave = threadIdx.x / WAVE;
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    uint64_t balls[CT_ITEMS];
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < CT_ITEMS; i++) {
        balls[i] = __ballot(is_head(keys, striped_index(blockIdx.x, wave, i, lane), n));
        c += (uint32_t)__popcll(balls[i]);
    }
    if (lane == 0)
        s_w[wave] = c;
    __syncthreads();
    uint32_t run = tile_off[blockIdx.x];
    for (int w = 0; w < wave; w++)
        run += s_w[w];
#pragma unroll
    for (int i = 0; i < CT_ITEMS; i++) {
        if ((balls[i] >> lane) & 1u)
            run_start[run + __popcll(balls[i] & lt)] = (uint32_t)striped_index(blockIdx.x, wave, i, lane);
        run += (uint32_t)__popcll(balls[i]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        run_start[*n_runs] = (uint32_t)n;
}

__device__ __forceinline__ uint32_t run_count(const uint32_t *__restrict__ run_start, uint64_t r) {
    return run_start[r + 1] - run_start[r];
}

__global__ __launch_bounds__(CT_THREADS) void runs_count(const uint32_t *__restrict__ run_start,
                                                         const uint32_t *__restrict__ n_runs_p, uint32_t c,
                                                         uint32_t *__restrict__ tile_cnt,
                                                         unsigned long long *__restrict__ n_single,
                                                         unsigned long long *__restrict__ n_below) {
    const uint64_t n_runs = *n_runs_p;
    const int wave = threadIdx.x / WAVE;
    const uint32_t lane = lane_id();
    uint32_t kept = 0, single = 0, below = 0;
#pragma unroll
    for (int i = 0; i < CT_ITEMS; i++) {
        const uint64_t r = striped_index(blockIdx.x, wave, i, lane);
        if (r < n_runs) {
            const uint32_t cnt = run_count(run_start, r);
            kept += cnt >= c;
            single += cnt == 1;
            below += cnt >= 2 && cnt < c;
        }
    }
    uint32_t tk, ts, tb;
    block_exclusive_sum<CT_THREADS>(kept, &tk);
    block_exclusive_sum<CT_THREADS>(single, &ts);
    block_exclusive_sum<CT_THREADS>(below, &tb);
    if (threadIdx.x == 0) {
        tile_cnt[blockIdx.x] = tk;
        if (ts)
            atomicAdd(n_single, (unsigned long long)ts);
        if (tb)
            atomicAdd(n_below, (unsigned long long)tb);
    }
}

template <typename K>
__global__ __launch_bounds__(CT_THREADS) void runs_write(const K *__restrict__ keys,
                                                         const uint32_t *__restrict__ run_start,
                                                         const uint32_t *__restrict__ n_runs_p, uint32_t c,
                                                         const uint32_t *__restrict__ tile_off,
                                                         K *__restrict__ out_keys, uint32_t *__restrict__ out_counts) {
    __shared__ uint32_t s_w[CT_WAVES];
    const uint64_t n_runs = *n_runs_p;
    const int wave = threadIdx.x / WAVE;
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    uint64_t balls[CT_ITEMS];
    uint32_t cnts[CT_ITEMS];
    uint32_t tot = 0;
#pragma unroll
    for (int i = 0; i < CT_ITEMS; i++) {
        const uint64_t r = striped_index(blockIdx.x, wave, i, lane);
        cnts[i] = r < n_runs ? run_count(run_start, r) : 0;
        balls[i] = __ballot(r < n_runs && cnts[i] >= c);
        tot += (uint32_t)__popcll(balls[i]);
    }
    if (lane == 0)
        s_w[wave] = tot;
    __syncthreads();
    uint32_t at = tile_off[blockIdx.x];
    for (int w = 0; w < wave; w++)
        at += s_w[w];
#pragma unroll
    for (int i = 0; i < CT_ITEMS; i++) {
        if ((balls[i] >> lane) & 1u) {
            const uint64_t r = striped_index(blockIdx.x, wave, i, lane);
            const uint32_t o = at + (uint32_t)__popcll(balls[i] & lt);
            out_keys[o] = keys[run_start[r]];
            out_counts[o] = cnts[i];
        }
        at += (uint32_t)__popcll(balls[i]);
    }
}

// Layout of the compaction scratch for n keys.
struct CompactScratch {
    uint32_t *run_start;  // n + 1
    uint32_t *tile_cnt;   // tiles
    uint32_t *scan_tmp;   // scan_scratch_words(tiles)
    uint32_t *totals;     // [0] = n_runs, [1] = n_out
    size_t bytes;
};

CompactScratch compact_layout(void *base, uint64_t n) {
    CompactScratch s{};
    const uint64_t tiles = ceil_div(n ? n : 1, CT_TILE);
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *r = p ? p + off : nullptr;
        off = align_up(off + bytes, 256);
        return r;
    };
    s.run_start = reinterpret_cast<uint32_t *>(take((n + 1) * sizeof(uint32_t)));
    s.tile_cnt = reinterpret_cast<uint32_t *>(take(tiles * sizeof(uint32_t)));
    s.scan_tmp = reinterpret_cast<uint32_t *>(take(scan_scratch_words(tiles) * sizeof(uint32_t)));
    s.totals = reinterpret_cast<uint32_t *>(take(4 * sizeof(uint32_t)));
    s.bytes = off;
    return s;
}

__global__ void totals_to_counters(const uint32_t *__restrict__ totals, DevCounters *__restrict__ ctr) {
    ctr->n_runs = totals[0];
    ctr->n_out = totals[1];
}

template <typename K>
hipError_t compact_impl(const K *keys, uint64_t n, uint32_t c, K *out_keys, uint32_t *out_counts, void *scratch,
                        size_t scratch_bytes, DevCounters *ctr, hipStream_t stream) {
    if (n == 0)
        return hipSuccess;  // counters already zero
    CompactScratch s = compact_layout(scratch, n);
    if (s.bytes > scratch_bytes)
        return hipErrorInvalidValue;
    const uint64_t tiles = ceil_div(n, CT_TILE);
    const dim3 grid((unsigned)tiles), block(CT_THREADS);
    heads_count<K><<<grid, block, 0, stream>>>(keys, n, s.tile_cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if ((e = launch_exclusive_scan(s.tile_cnt, s.tile_cnt, tiles, s.scan_tmp, &s.totals[0], stream)) != hipSuccess)
        return e;
    heads_write<K><<<grid, block, 0, stream>>>(keys, n, s.tile_cnt, &s.totals[0], s.run_start);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    // there are at most n runs: size the run passes for n and let each block
    // read the true number of runs
    runs_count<<<grid, block, 0, stream>>>(s.run_start, &s.totals[0], c, s.tile_cnt, &ctr->n_single, &ctr->n_below);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = launch_exclusive_scan(s.tile_cnt, s.tile_cnt, tiles, s.scan_tmp, &s.totals[1], stream)) != hipSuccess)
        return e;
    runs_write<K><<<grid, block, 0, stream>>>(keys, s.run_start, &s.totals[0], c, s.tile_cnt, out_keys, out_counts);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    totals_to_counters<<<1, 1, 0, stream>>>(s.totals, ctr);
    return hipGetLastError();
}

}  // namespace

size_t compact_scratch_bytes(uint64_t n) { return compact_layout(nullptr, n).bytes; }

hipError_t compact(const uint64_t *keys, uint64_t n, int key_words, uint32_t c, uint64_t *out_keys,
                   uint32_t *out_counts, void *scratch, size_t scratch_bytes, DevCounters *ctr, hipStream_t stream) {
    if (key_words == 2)
        return compact_impl<Key2>(reinterpret_cast<const Key2 *>(keys), n, c, reinterpret_cast<Key2 *>(out_keys),
                                  out_counts, scratch, scratch_bytes, ctr, stream);
    return compact_impl<uint64_t>(keys, n, c, out_keys, out_counts, scratch, scratch_bytes, ctr, stream);
}

}  // namespace tk
