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

// Byte -> (code, is_base) for 4 bytes at once.  Upper-casing by clearing
// bit 5 maps a/c/g/t onto A/C/G/T and no other byte onto them.
__device__ __forceinline__ void classify4(uint32_t x, uint32_t &codes, uint32_t &bad4) {
    const uint32_t u = x & 0xDFDFDFDFu;
    // ((u >> 1) ^ (u >> 2)) & 3 per byte: A(0x41)->0, C(0x43)->1, G(0x47)->2, T(0x54)->3
    codes = ((u >> 1) ^ (u >> 2)) & 0x03030303u;
    // exact per-byte zero test: 0x80 in every byte of v that is zero
    auto zero_bytes = [](uint32_t v) { return ~(((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v | 0x7F7F7F7Fu); };
    const uint32_t ok = zero_bytes(u ^ 0x41414141u) | zero_bytes(u ^ 0x43434343u) |
                        zero_bytes(u ^ 0x47474747u) | zero_bytes(u ^ 0x54545454u);
    codes &= (ok >> 7) * 3u;  // a non-base byte packs as code 0
    const uint32_t nb = ~ok & 0x80808080u;
    bad4 = ((nb >> 7) & 1u) | ((nb >> 14) & 2u) | ((nb >> 21) & 4u) | ((nb >> 28) & 8u);
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
    code = 0;
    bad = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        uint32_t c4, b4;
        classify4(x[i], c4, b4);
        // bases 4i..4i+3 (byte j = base 4i+j) -> 8 bits, first base highest
        const uint32_t g = ((c4 & 3u) << 6) | (((c4 >> 8) & 3u) << 4) | (((c4 >> 16) & 3u) << 2) |
                           ((c4 >> 24) & 3u);
        code |= (uint64_t)g << (56 - 8 * i);
        bad |= b4 << (4 * i);
    }
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

__global__ __launch_bounds__(PACK_THREADS) void pack_kernel(const uint8_t *__restrict__ bases, uint64_t n_bases,
                                                            uint64_t n_words, bool aligned,
                                                            const uint32_t *__restrict__ starts, int k,
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
        int run = 64 - max(qb + 1, qs);
        for (int t = 0; t < 32; t++) {
            const bool b = (bad >> t) & 1u;
            const bool s = (st >> t) & 1u;
            run = b ? 0 : (s ? 1 : min(run + 1, 64));
            vbits |= (uint32_t)(run >= k) << t;
        }
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
                       hipStream_t stream) {
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
                                                                     packed, valid, n_windows);
    return hipGetLastError();
}

}  // namespace tk
