// Phased sort-and-compact (paper §2.1, "Counting frequencies with sorting
// and compaction", Fig. 1, and the running-time analysis): the counted
// (key, count) records of the library so far -- the sorted and compacted
// array, "SAC" -- stay resident; the records of every new chunk of reads,
// sorted and compacted on their own, are merged into it by one linear pass
// that adds up the counts of keys present in both.
//
// merge     : merge path of two sorted record lists with unique keys (the
//             SAC first on equal keys), a tile of MG_TILE outputs per
//             workgroup: the tiles' splits are found first (one binary
//             search per tile), then each workgroup stages its two input
//             ranges in LDS, every thread merges MG_ITEMS outputs there, and
//             the tile is written back coalesced.
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
constexpr int MG_TILE = MG_THREADS * MG_ITEMS;

template <typename K>
__device__ __forceinline__ bool key_le(const K &a, const K &b) {
    return !(b < a);
}

// Split of diagonal d of the merge of A (na) and B (nb): the number of A
// records among the first d outputs, A first on equal keys.
template <typename K, typename AtA, typename AtB>
__device__ __forceinline__ uint64_t merge_split(uint64_t na, uint64_t nb, uint64_t d, AtA at_a, AtB at_b) {
    uint64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (key_le<K>(at_a(mid), at_b(d - mid - 1)))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// splits[t]: split of diagonal min(t * MG_TILE, na + nb), t <= n_tiles
template <typename K>
__global__ __launch_bounds__(256) void merge_splits_kernel(const K *__restrict__ ak, uint64_t na,
                                                           const K *__restrict__ bk, uint64_t nb, uint64_t n_tiles,
                                                           uint64_t *__restrict__ splits) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t > n_tiles)
        return;
    const uint64_t d = min(t * (uint64_t)MG_TILE, na + nb);
    splits[t] = merge_split<K>(na, nb, d, [&](uint64_t i) { return ak[i]; }, [&](uint64_t j) { return bk[j]; });
}

template <typename K>
__global__ __launch_bounds__(MG_THREADS) void merge_kernel(const K *__restrict__ ak, const uint32_t *__restrict__ ac,
                                                           uint64_t na, const K *__restrict__ bk,
                                                           const uint32_t *__restrict__ bc, uint64_t nb,
                                                           const uint64_t *__restrict__ splits,
                                                           K *__restrict__ ck, uint32_t *__restrict__ cc) {
    __shared__ K s_k[MG_TILE];  // the tile's inputs: its A records, then its B records
    __shared__ uint32_t s_c[MG_TILE];
    __shared__ K s_ok[MG_TILE];  // the tile's outputs
    __shared__ uint32_t s_oc[MG_TILE];
    const int tid = threadIdx.x;
    const uint64_t d0 = (uint64_t)blockIdx.x * MG_TILE, d1 = min(d0 + MG_TILE, na + nb);
    const uint64_t i0 = splits[blockIdx.x], i1 = splits[blockIdx.x + 1];
    const uint32_t la = (uint32_t)(i1 - i0), lb = (uint32_t)((d1 - i1) - (d0 - i0));  // la + lb = d1 - d0
    const uint64_t j0 = d0 - i0;
    // the tile's A records, then its B records
    for (uint32_t u = tid; u < la; u += MG_THREADS) {
        s_k[u] = ak[i0 + u];
        s_c[u] = ac[i0 + u];
    }
    for (uint32_t u = tid; u < lb; u += MG_THREADS) {
        s_k[la + u] = bk[j0 + u];
        s_c[la + u] = bc[j0 + u];
    }
    __syncthreads();
    const uint32_t n = la + lb, t0 = (uint32_t)tid * MG_ITEMS;
    if (t0 < n) {
        uint32_t i = (uint32_t)merge_split<K>(la, lb, t0, [&](uint64_t x) { return s_k[x]; },
                                              [&](uint64_t y) { return s_k[la + y]; });
        uint32_t j = t0 - i;
        const uint32_t m = min((uint32_t)MG_ITEMS, n - t0);  // outputs of this thread
        for (uint32_t u = 0; u < m; u++) {
            const bool take_a = j >= lb || (i < la && key_le(s_k[i], s_k[la + j]));
            const uint32_t x = take_a ? i : la + j;
            s_ok[t0 + u] = s_k[x];
            s_oc[t0 + u] = s_c[x];
            i += take_a ? 1u : 0u;
            j += take_a ? 0u : 1u;
        }
    }
    __syncthreads();
    for (uint32_t u = tid; u < n; u += MG_THREADS) {
        ck[d0 + u] = s_ok[u];
        cc[d0 + u] = s_oc[u];
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
    // the tiles' splits live in the flag array until the heads overwrite it
    // (it holds 2 n >= 2 (n_tiles + 1) words)
    const uint64_t n_tiles = ceil_div(n, (uint64_t)MG_TILE);
    uint64_t *splits = reinterpret_cast<uint64_t *>(flag);
    merge_splits_kernel<K><<<dim3((unsigned)ceil_div(n_tiles + 1, 256)), dim3(256), 0, stream>>>(ak, na, bk, nb,
                                                                                                n_tiles, splits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    merge_kernel<K><<<dim3((unsigned)n_tiles), dim3(MG_THREADS), 0, stream>>>(ak, ac, na, bk, bc, nb, splits, tk_, tc);
    if ((e = hipGetLastError()) != hipSuccess)
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
