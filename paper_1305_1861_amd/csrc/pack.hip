// K1: 2-bit packing of reads and k-mer window validity.
//
// Paper §2.1 (k-mer extraction and bit-encoding): each base is stored in
// two bits and k-mers are only taken from stretches of A/C/G/T, the reads
// being cut at ambiguous calls; windows never span two reads.
//
// Layout produced (one entry per 32 bases, n_words = ceil(n_bases / 32)):
//   packed[w] : bases 32w..32w+31, base 32w+t in bits (63-2t, 62-2t), codes
//               A=0 C=1 G=2 T=3 (a non-base byte packs as 0);
//   valid[w]  : bit t set iff the window of k bases ENDING at base 32w+t lies
//               inside one read and holds only A/C/G/T (upper or lower case).
// With the first base most significant, the forward encoding of a window is
// a contiguous bit field of the big-endian concatenation of packed words.
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int PACK_THREADS = 256;  // one word (32 bases) per thread

// 4 bytes -> their four 2-bit codes, first byte highest (g, 8 bits), and
// their non-base flags (bad4, bit j: byte j).  Upper-casing by clearing bit
// 5 maps a/c/g/t onto A/C/G/T and no other byte onto them.
__device__ __forceinline__ void classify4(uint32_t x, uint32_t &g, uint32_t &bad4) {
    const uint32_t u = x & 0xDFDFDFDFu;
    // ((u >> 1) ^ (u >> 2)) & 3 per byte: A(0x41)->0, C(0x43)->1, G(0x47)->2, T(0x54)->3
    uint32_t codes = ((u >> 1) ^ (u >> 2)) & 0x03030303u;
    // a byte is a base iff it equals the letter of its code, picked per byte
    // from the bytes of 0x54474341 (A, C, G, T) by a byte permute; exact
    // per-byte zero test: 0x80 in every byte of v that is zero
    auto zero_bytes = [](uint32_t v) { return ~(((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v | 0x7F7F7F7Fu); };
    const uint32_t ok = zero_bytes(u ^ __builtin_amdgcn_perm(0u, 0x54474341u, codes));
    codes &= (ok >> 6) | (ok >> 7);  // a non-base byte packs as code 0
    // one multiply gathers the four codes (byte j to bits 7-2j, 6-2j),
    // another the four flags; their partial products never overlap
    g = (codes * 0x40100401u) >> 24;
    bad4 = ((((~ok) >> 7) & 0x01010101u) * 0x00204081u) >> 21 & 0xFu;
}

// Packed codes and non-base mask of word w.  Bytes past n_bases count as
// non-bases.  `aligned` says the byte array is 16-byte aligned.
__device__ __forceinline__ void load_word(const uint8_t *__restrict__ bases, uint64_t n_bases, uint64_t w,
                                          bool aligned, uint64_t &code, uint32_t &bad) {
    const uint64_t p0 = w * 32;
    uint32_t x[8];
    if (aligned && p0 + 32 <= n_bases) {
        const uint4 *src = reinterpret_cast<const uint4 *>(bases + p0);
        const uint4 a = src[0];
        const uint4 b = src[1];
        x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
        x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    } else {
#pragma unroll
        for (int i = 0; i < 8; i++) {
            uint32_t v = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint64_t p = p0 + 4 * i + j;
                const uint32_t byte = p < n_bases ? bases[p] : (uint32_t)'N';
                v |= byte << (8 * j);
            }
            x[i] = v;
        }
    }
    uint32_t hi = 0, lo = 0;
    bad = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        uint32_t g, b4;
        classify4(x[i], g, b4);  // bases 4i..4i+3 (byte j = base 4i+j)
        if (i < 4)
            hi |= g << (24 - 8 * i);
        else
            lo |= g << (56 - 8 * i);
        bad |= b4 << (4 * i);
    }
    code = ((uint64_t)hi << 32) | lo;
}

// Bit t of the result: bits t - L + 1 .. t of x are all set (bits below bit
// 0 count as clear); 0 <= L <= 32.  Windows of length 1, 2, 4, ... are
// formed by doubling and combined along the binary digits of L.
__device__ __forceinline__ uint32_t runs_of(uint32_t x, int L) {
    uint32_t res = ~0u, pw = x;
    int cov = 0;  // length combined so far, below the current digit
#pragma unroll
    for (int p = 1; p <= 32; p <<= 1) {
        if (L & p) {
            res &= pw << cov;
            cov += p;
        }
        if (p < 32)
            pw &= pw << p;
    }
    return res;
}

// Validity bits of one word: bit t is set iff the k-base window ending at
// base t of the word lies in one read and holds only bases.  bad, st: the
// word's non-base and read-start masks; run0 (<= 64): length of the base run
// of one read that ends just before the word.  A window reaching back
// before the word (t < k - 1) needs bases 0..t free of non-bases and read
// starts and run0 >= k - 1 - t; a window inside the word needs its k bases
// free of non-bases and its last k - 1 free of read starts (its first base
// may start a read).
__device__ __forceinline__ uint32_t window_bits(uint32_t bad, uint32_t st, int run0, int k) {
    const uint32_t g = ~bad, ns = ~st;
    const uint32_t pre = (g & ~(g + 1u)) & (ns & ~(ns + 1u));  // bits below the first break
    const uint32_t before = k - 1 >= 32 ? ~0u : (1u << (k - 1)) - 1u;  // t < k - 1
    const int need = max(0, k - 1 - run0);
    uint32_t v = pre & before & (need >= 32 ? 0u : ~0u << need);
    if (k <= 32)
        v |= runs_of(g, k) & runs_of(ns, k - 1) & (~0u << (k - 1));
    return v;
}

__global__ void mark_read_starts(const uint64_t *__restrict__ offsets, uint64_t n_reads, uint64_t n_bases,
                                 uint32_t *__restrict__ starts) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_reads)
        return;
    const uint64_t p = offsets[r];
    if (p < n_bases)
        atomicOr(&starts[p >> 5], 1u << (p & 31));
}

// Validity bits of word w when the libraries of a batch have different k:
// each library overlapping the word (libraries ordered by position, maybe
// with gaps) sets the bits of its own positions with its own k; positions of
// no listed library stay clear.
__device__ __forceinline__ uint32_t window_bits_libs(uint32_t bad, uint32_t st, int run0, uint64_t w,
                                                     const LibDesc *__restrict__ libs, uint32_t n_libs) {
    const uint64_t p0 = w * 32, p1 = p0 + 32;
    // first library ending after p0
    uint32_t lo = 0, hi = n_libs;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (libs[mid].pos1 <= p0)
            lo = mid + 1;
        else
            hi = mid;
    }
    uint32_t v = 0;
    for (uint32_t j = lo; j < n_libs && libs[j].pos0 < p1; j++) {
        const uint64_t a = max(libs[j].pos0, p0), b = min(libs[j].pos1, p1);
        if (a >= b)
            continue;
        const uint32_t na = (uint32_t)(a - p0), nb = (uint32_t)(b - p0);  // bits [na, nb)
        const uint32_t mask = (nb == 32 ? ~0u : (1u << nb) - 1u) & (~0u << na);
        v |= window_bits(bad, st, run0, libs[j].k) & mask;
    }
    return v;
}

__global__ __launch_bounds__(PACK_THREADS) void pack_kernel(const uint8_t *__restrict__ bases, uint64_t n_bases,
                                                            uint64_t n_words, bool aligned,
                                                            const uint32_t *__restrict__ starts, int k,
                                                            const LibDesc *__restrict__ libs, uint32_t n_libs,
                                                            uint64_t *__restrict__ packed,
                                                            uint32_t *__restrict__ valid,
                                                            unsigned long long *__restrict__ n_windows) {
    // non-base and read-start masks of this block's words, plus the two
    // words before them (a window of up to 63 bases reaches two words back)
    __shared__ uint32_t s_bad[PACK_THREADS + 2];
    __shared__ uint32_t s_st[PACK_THREADS + 2];
    const int tid = threadIdx.x;
    const uint64_t w0 = (uint64_t)blockIdx.x * PACK_THREADS;
    const uint64_t w = w0 + tid;
    uint64_t code = 0;
    uint32_t bad = 0xFFFFFFFFu, st = 0;
    if (w < n_words) {
        load_word(bases, n_bases, w, aligned, code, bad);
        st = starts[w];
    }
    s_bad[tid + 2] = bad;
    s_st[tid + 2] = st;
    if (tid < 2) {
        const int64_t hw = (int64_t)w0 - 2 + tid;
        uint32_t hb = 0xFFFFFFFFu, hs = 0;  // before base 0: nothing is a base
        if (hw >= 0) {
            uint64_t hc;
            load_word(bases, n_bases, (uint64_t)hw, aligned, hc, hb);
            hs = starts[hw];
        }
        s_bad[tid] = hb;
        s_st[tid] = hs;
    }
    __syncthreads();

    uint32_t vbits = 0;
    if (w < n_words) {
        packed[w] = code;
        // length of the base run that ends just before this word (capped at
        // 64): it begins after the last non-base, or at the last read start
        const uint64_t bad64 = (uint64_t)s_bad[tid] | ((uint64_t)s_bad[tid + 1] << 32);
        const uint64_t st64 = (uint64_t)s_st[tid] | ((uint64_t)s_st[tid + 1] << 32);
        const int qb = bad64 ? 63 - __clzll(bad64) : -1;
        const int qs = st64 ? 63 - __clzll(st64) : -1;
        const int run0 = 64 - max(qb + 1, qs);
        vbits = libs ? window_bits_libs(bad, st, run0, w, libs, n_libs) : window_bits(bad, st, run0, k);
        valid[w] = vbits;
    }
    // valid windows of the block -> one atomic per block
    if (!n_windows)
        return;
    uint64_t cnt = wave_sum64((uint64_t)__popc(vbits));
    __shared__ unsigned long long s_cnt[PACK_THREADS / WAVE];
    if (lane_id() == 0)
        s_cnt[tid / WAVE] = cnt;
    __syncthreads();
    if (tid == 0) {
        unsigned long long sum = 0;
        for (int i = 0; i < PACK_THREADS / WAVE; i++)
            sum += s_cnt[i];
        if (sum)
            atomicAdd(n_windows, sum);
    }
}

}  // namespace

hipError_t launch_pack(const uint8_t *bases, const uint64_t *offsets, uint64_t n_bases, uint64_t n_reads, int k,
                       uint64_t *packed, uint32_t *valid, uint32_t *starts, unsigned long long *n_windows,
                       hipStream_t stream, const LibDesc *libs, uint32_t n_libs) {
    const uint64_t n_words = ceil_div(n_bases, 32);
    if (n_words == 0)
        return hipSuccess;
    if (n_reads) {
        const uint64_t g = ceil_div(n_reads, 256);
        mark_read_starts<<<dim3((unsigned)g), dim3(256), 0, stream>>>(offsets, n_reads, n_bases, starts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    const bool aligned = ((uintptr_t)bases & 15u) == 0;
    const uint64_t g = ceil_div(n_words, PACK_THREADS);
    pack_kernel<<<dim3((unsigned)g), dim3(PACK_THREADS), 0, stream>>>(bases, n_bases, n_words, aligned, starts, k,
                                                                     libs, n_libs, packed, valid, n_windows);
    return hipGetLastError();
}

}  // namespace tk
