// Phased sort-and-compact (paper §2.1, "Counting frequencies with sorting
// and compaction", Fig. 1, and the running-time analysis): the counted
// (key, count) records of the library so far -- the sorted and compacted
// array, "SAC" -- stay resident; the records of every new chunk of reads,
// sorted and compacted on their own, are merged into it by one linear pass
// that adds up the counts of keys present in both.
//
// merge     : merge path of two sorted record lists with unique keys (the
//             SAC first on equal keys); every thread finds its own start on
//             its diagonal by binary search and merges MG_ITEMS outputs.
// heads     : flag of every merged record whose key differs from the one
//             before (a key occurs at most twice: once per list).
// reduce    : after an exclusive scan of the flags, every head writes its
//             key and its count plus the count of an equal successor.
// select    : flags of the records with count >= c (and the statistics of
//             the others); the same scan and a gather write the answer.
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int MG_THREADS = 256;
constexpr int MG_ITEMS = 8;

template <typename K>
__device__ __forceinline__ bool key_le(const K &a, const K &b) {
    return !(b < a);
}

template <typename K>
__global__ __launch_bounds__(MG_THREADS) void merge_kernel(const K *__restrict__ ak, const uint32_t *__restrict__ ac,
                                                           uint64_t na, const K *__restrict__ bk,
                                                           const uint32_t *__restrict__ bc, uint64_t nb,
                                                           K *__restrict__ ck, uint32_t *__restrict__ cc) {
    const uint64_t n = na + nb;
    const uint64_t d = ((uint64_t)blockIdx.x * MG_THREADS + threadIdx.x) * MG_ITEMS;
    if (d >= n)
        return;
    // split of diagonal d: i items from A, d - i from B, A first on ties
    uint64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (key_le(ak[mid], bk[d - mid - 1]))
            lo = mid + 1;
        else
            hi = mid;
    }
    uint64_t i = lo, j = d - lo;
    const uint64_t e = min(d + MG_ITEMS, n);
    for (uint64_t o = d; o < e; o++) {
        const bool take_a = j >= nb || (i < na && key_le(ak[i], bk[j]));
        if (take_a) {
            ck[o] = ak[i];
            cc[o] = ac[i];
            i++;
        } else {
            ck[o] = bk[j];
            cc[o] = bc[j];
            j++;
        }
    }
}

template <typename K>
__global__ __launch_bounds__(256) void heads_kernel(const K *__restrict__ keys, uint64_t n, uint32_t *__restrict__ flag) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        flag[p] = (p == 0 || keys[p] != keys[p - 1]) ? 1u : 0u;
}

// pos: exclusive scan of the head flags (flag[p] = pos[p + 1] - pos[p], with
// pos[n] the total).
template <typename K>
__global__ __launch_bounds__(256) void reduce_kernel(const K *__restrict__ keys, const uint32_t *__restrict__ cnt,
                                                     uint64_t n, const uint32_t *__restrict__ pos,
                                                     const uint32_t *__restrict__ total, K *__restrict__ out_k,
                                                     uint32_t *__restrict__ out_c) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const uint32_t next = p + 1 < n ? pos[p + 1] : *total;
        if (next == pos[p])
            continue;  // not a head
        uint32_t c = cnt[p];
        if (p + 1 < n && keys[p + 1] == keys[p])
            c += cnt[p + 1];
        out_k[pos[p]] = keys[p];
        out_c[pos[p]] = c;
    }
}

// flag = count >= c; stats[0] += records of count 1, stats[1] += records of
// count in [2, c)
__global__ __launch_bounds__(256) void select_flags(const uint32_t *__restrict__ cnt, uint64_t n, uint32_t c,
                                                    uint32_t *__restrict__ flag,
                                                    unsigned long long *__restrict__ stats) {
    __shared__ unsigned long long s[2];
    if (threadIdx.x < 2)
        s[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long one = 0, below = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const uint32_t v = cnt[p];
        flag[p] = v >= c ? 1u : 0u;
        one += v == 1;
        below += v >= 2 && v < c;
    }
    atomicAdd(&s[0], one);
    atomicAdd(&s[1], below);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&stats[0], s[0]);
        atomicAdd(&stats[1], s[1]);
    }
}

template <typename K>
__global__ __launch_bounds__(256) void gather_selected(const K *__restrict__ keys, const uint32_t *__restrict__ cnt,
                                                       uint64_t n, const uint32_t *__restrict__ flag,
                                                       const uint32_t *__restrict__ pos, K *__restrict__ out_k,
                                                       uint32_t *__restrict__ out_c) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        if (flag[p]) {
            out_k[pos[p]] = keys[p];
            out_c[pos[p]] = cnt[p];
        }
    }
}

unsigned grid_for(uint64_t n) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(n, 256), (uint64_t)device_cu_count() * 16));
}

template <typename K>
hipError_t merge_compact_impl(const K *ak, const uint32_t *ac, uint64_t na, const K *bk, const uint32_t *bc,
                              uint64_t nb, K *tk_, uint32_t *tc, uint32_t *flag, uint32_t *scan_tmp, K *out_k,
                              uint32_t *out_c, uint32_t *n_out, hipStream_t stream) {
    const uint64_t n = na + nb;
    if (n == 0)
        return launch_exclusive_scan(flag, flag, 0, scan_tmp, n_out, stream);  // writes 0
    const uint64_t per_block = (uint64_t)MG_THREADS * MG_ITEMS;
    merge_kernel<K><<<dim3((unsigned)ceil_div(n, per_block)), dim3(MG_THREADS), 0, stream>>>(ak, ac, na, bk, bc, nb,
                                                                                            tk_, tc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    heads_kernel<K><<<grid_for(n), 256, 0, stream>>>(tk_, n, flag);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = launch_exclusive_scan(flag, flag, n, scan_tmp, n_out, stream)) != hipSuccess)
        return e;
    reduce_kernel<K><<<grid_for(n), 256, 0, stream>>>(tk_, tc, n, flag, n_out, out_k, out_c);
    return hipGetLastError();
}

template <typename K>
hipError_t select_impl(const K *keys, const uint32_t *cnt, uint64_t n, uint32_t c, uint32_t *flag, uint32_t *scan_tmp,
                       K *out_k, uint32_t *out_c, uint32_t *n_out, unsigned long long *stats, hipStream_t stream) {
    if (n == 0)
        return launch_exclusive_scan(flag, flag, 0, scan_tmp, n_out, stream);
    select_flags<<<grid_for(n), 256, 0, stream>>>(cnt, n, c, flag, stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // keep the flags: the scan writes positions to the second half
    uint32_t *pos = flag + n;
    if ((e = launch_exclusive_scan(flag, pos, n, scan_tmp, n_out, stream)) != hipSuccess)
        return e;
    gather_selected<K><<<grid_for(n), 256, 0, stream>>>(keys, cnt, n, flag, pos, out_k, out_c);
    return hipGetLastError();
}

}  // namespace

hipError_t merge_compact(const uint64_t *ak, const uint32_t *ac, uint64_t na, const uint64_t *bk, const uint32_t *bc,
                         uint64_t nb, int key_words, uint64_t *tmp_k, uint32_t *tmp_c, uint32_t *flag,
                         uint32_t *scan_tmp, uint64_t *out_k, uint32_t *out_c, uint32_t *n_out, hipStream_t stream) {
    if (key_words == 2)
        return merge_compact_impl<Key2>(reinterpret_cast<const Key2 *>(ak), ac, na, reinterpret_cast<const Key2 *>(bk),
                                        bc, nb, reinterpret_cast<Key2 *>(tmp_k), tmp_c, flag, scan_tmp,
                                        reinterpret_cast<Key2 *>(out_k), out_c, n_out, stream);
    return merge_compact_impl<uint64_t>(ak, ac, na, bk, bc, nb, tmp_k, tmp_c, flag, scan_tmp, out_k, out_c, n_out,
                                        stream);
}

hipError_t select_records(const uint64_t *keys, const uint32_t *cnt, uint64_t n, int key_words, uint32_t c,
                          uint32_t *flag, uint32_t *scan_tmp, uint64_t *out_k, uint32_t *out_c, uint32_t *n_out,
                          unsigned long long *stats, hipStream_t stream) {
    if (key_words == 2)
        return select_impl<Key2>(reinterpret_cast<const Key2 *>(keys), cnt, n, c, flag, scan_tmp,
                                 reinterpret_cast<Key2 *>(out_k), out_c, n_out, stats, stream);
    return select_impl<uint64_t>(keys, cnt, n, c, flag, scan_tmp, out_k, out_c, n_out, stats, stream);
}

}  // namespace tk
