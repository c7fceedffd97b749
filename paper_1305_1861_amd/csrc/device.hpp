// Device-side helpers shared by the kernels of libturtle (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tk {

constexpr int WAVE = 64;

// Two-word key, stored {hi, lo} in memory and ordered by (hi, lo).
struct Key2 {
    uint64_t hi, lo;
};

__device__ __forceinline__ bool operator==(const Key2 &a, const Key2 &b) { return a.hi == b.hi && a.lo == b.lo; }
__device__ __forceinline__ bool operator!=(const Key2 &a, const Key2 &b) { return !(a == b); }
__device__ __forceinline__ bool operator<(const Key2 &a, const Key2 &b) {
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// 64-bit finaliser of MurmurHash3 (fmix64).
__device__ __forceinline__ uint64_t fmix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

__device__ __forceinline__ uint64_t key_hash(uint64_t key) { return fmix64(key); }
__device__ __forceinline__ uint64_t key_hash(const Key2 &key) { return fmix64(key.lo ^ fmix64(key.hi)); }

// Reverse the order of the 32 two-bit groups of a word (bit reversal, then
// swap the two bits inside each group back).
__device__ __forceinline__ uint64_t group_reverse(uint64_t x) {
    uint64_t y = __builtin_bitreverse64(x);
    return ((y >> 1) & 0x5555555555555555ull) | ((y & 0x5555555555555555ull) << 1);
}

// Radix digit of a key.
__device__ __forceinline__ uint32_t digit_of(uint64_t key, int shift, uint32_t mask) {
    return (uint32_t)(key >> shift) & mask;
}
__device__ __forceinline__ uint32_t digit_of(const Key2 &key, int shift, uint32_t mask) {
    if (shift >= 64)
        return (uint32_t)(key.hi >> (shift - 64)) & mask;
    if (shift == 0)
        return (uint32_t)key.lo & mask;
    // a digit may straddle the two words
    return (uint32_t)((key.lo >> shift) | (key.hi << (64 - shift))) & mask;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t l = lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

// Value of x held by lane `src` of the wave (every lane must be active).
__device__ __forceinline__ uint64_t read_lane64(uint64_t x, int src) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t read_lane(uint64_t x, int src) { return read_lane64(x, src); }
__device__ __forceinline__ Key2 read_lane(const Key2 &x, int src) {
    return Key2{read_lane64(x.hi, src), read_lane64(x.lo, src)};
}

// Inclusive prefix sum across the wave, with DPP moves only (no LDS round
// trips): shifts by 1, 2, 4 and 8 lanes within each row of 16 lanes (lanes
// shifted in from outside the row add 0), then lane 15 of rows 0 and 2 into
// rows 1 and 3, then lane 31 into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111 /* row_shr:1 */, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112 /* row_shr:2 */, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114 /* row_shr:4 */, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118 /* row_shr:8 */, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142 /* row_bcast:15 */, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143 /* row_bcast:31 */, 0xC, 0xF, false);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1)
        v += __shfl_xor(v, d, WAVE);
    return v;
}

// Exclusive prefix sum over the threads of a block of NT threads (NT a
// multiple of 64, at most 1024).  Every thread must call it.  *total gets
// the block-wide sum.  Uses a small static LDS array.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t *total) {
    constexpr int NW = NT / WAVE;
    __shared__ uint32_t s_wave[NW];
    __shared__ uint32_t s_total;
    const int tid = threadIdx.x;
    const int w = tid / WAVE;
    uint32_t inc = wave_inclusive_sum(v);
    if (lane_id() == WAVE - 1)
        s_wave[w] = inc;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int i = 0; i < NW; i++) {
            uint32_t t = s_wave[i];
            s_wave[i] = run;
            run += t;
        }
        s_total = run;
    }
    __syncthreads();
    uint32_t r = s_wave[w] + inc - v;
    *total = s_total;
    __syncthreads();  // s_wave / s_total may be reused by the next call
    return r;
}

// Appending items found by the threads of a block to one output array: the
// items are staged in LDS (wave ballots for the offsets) and a full buffer
// is appended with one atomicAdd on the output counter and copied out
// coalesced, instead of one atomic on that counter per wave.  Every thread
// of the block calls push() the same number of times, then finish().  The
// LDS arrays belong to the caller's kernel.
template <typename K, int THREADS, int BUF>
struct BlockAppender {
    K *s_buf;                      // BUF items
    uint32_t *s_wc;                // THREADS / WAVE counts
    uint32_t *s_n;                 // items staged
    unsigned long long *s_base;    // output position of the buffer
    K *out;
    uint64_t capacity;             // items beyond it are counted, not written
    unsigned long long *n_out;
    static_assert(BUF >= THREADS, "a buffer holds at least one round");

    __device__ void init() {
        if (threadIdx.x == 0)
            *s_n = 0;
        __syncthreads();
    }
    __device__ void flush() {
        const uint32_t n = *s_n;
        if (threadIdx.x == 0)
            *s_base = atomicAdd(n_out, (unsigned long long)n);
        __syncthreads();
        const uint64_t base = *s_base;
        for (uint32_t j = threadIdx.x; j < n; j += THREADS)
            if (base + j < capacity)
                out[base + j] = s_buf[j];
        __syncthreads();
        if (threadIdx.x == 0)
            *s_n = 0;
        __syncthreads();
    }
    __device__ void push(bool emit, const K &item) {
        const int wave = (int)threadIdx.x / WAVE;
        const uint64_t ball = __ballot(emit);
        if (__lane_id() == 0)
            s_wc[wave] = (uint32_t)__popcll(ball);
        __syncthreads();
        uint32_t off = *s_n, tot = 0;
        for (int v = 0; v < THREADS / WAVE; v++) {
            off += v < wave ? s_wc[v] : 0u;
            tot += s_wc[v];
        }
        if (emit)
            s_buf[off + (uint32_t)__popcll(ball & lanemask_lt())] = item;
        __syncthreads();
        if (threadIdx.x == 0)
            *s_n += tot;
        __syncthreads();
        if (*s_n + THREADS > BUF)
            flush();
    }
    __device__ void finish() {
        if (*s_n)
            flush();
    }
};

// ---------------------------------------------------------------------------
// Canonical key of a k-mer window (paper §2.1, k-mer extraction): the window
// ending at base p = 32w + t is a contiguous 2k-bit field of the big-endian
// concatenation of packed words (first base most significant); the reverse
// complement is the complemented field with its 2-bit groups reversed; the
// key is the smaller of the two.
// ---------------------------------------------------------------------------
// Forward/reverse-complement extraction of the window ending at base
// p = 32w + t from the packed words w0 = packed[w], w1 = packed[w - 1] and
// w2 = packed[w - 2] (zero before the first word).
// k <= 31: one-word key.
__device__ __forceinline__ uint64_t window_key1(uint64_t w0, uint64_t w1, uint32_t t, int k) {
    const uint32_t s = 62 - 2 * t;  // bit of the window's last base in w0
    const uint64_t cat = s ? (w0 >> s) | (w1 << (64 - s)) : w0;
    const uint64_t fwd = cat & ((1ull << (2 * k)) - 1);
    const uint64_t rc = ~group_reverse(fwd) >> (64 - 2 * k);
    return fwd < rc ? fwd : rc;
}

// 32 <= k <= 63: two-word key {hi, lo}.
__device__ __forceinline__ Key2 window_key2(uint64_t w0, uint64_t w1, uint64_t w2, uint32_t t, int k) {
    const uint32_t s = 62 - 2 * t;
    uint64_t lo, hi;
    if (s) {
        lo = (w0 >> s) | (w1 << (64 - s));
        hi = (w1 >> s) | (w2 << (64 - s));
    } else {
        lo = w0;
        hi = w1;
    }
    const int hb = 2 * k - 64;  // bits of the key in hi, 0..62
    hi &= (1ull << hb) - 1;
    // reverse complement of the 2k-bit value: reverse the 64 groups of the
    // 128-bit word, complement, shift right by 128 - 2k
    const uint64_t a_hi = ~group_reverse(lo);
    const uint64_t a_lo = ~group_reverse(hi);
    const int sh = 128 - 2 * k;  // 2..64
    uint64_t rlo, rhi;
    if (sh == 64) {
        rlo = a_hi;
        rhi = 0;
    } else {
        rlo = (a_lo >> sh) | (a_hi << (64 - sh));
        rhi = a_hi >> sh;
    }
    const bool fwd_smaller = hi < rhi || (hi == rhi && lo <= rlo);
    return fwd_smaller ? Key2{hi, lo} : Key2{rhi, rlo};
}

__device__ __forceinline__ uint64_t window_key1(const uint64_t *__restrict__ packed, uint64_t w, uint32_t t, int k) {
    return window_key1(packed[w], w ? packed[w - 1] : 0, t, k);
}
__device__ __forceinline__ Key2 window_key2(const uint64_t *__restrict__ packed, uint64_t w, uint32_t t, int k) {
    return window_key2(packed[w], w ? packed[w - 1] : 0, w > 1 ? packed[w - 2] : 0, t, k);
}

// Rolling extraction along the consecutive windows of one packed word: the
// window ending at base t + 1 is the one ending at t with the base of t + 1
// appended (forward: shift left, new code at the bottom; reverse complement:
// shift right, complemented code at the top).  init() takes the window
// ending at t as above; key() equals window_key1/2 for every window reached.
struct Roll1 {
    uint64_t fwd, rc, mask;
    int top;  // 2k - 2: bit of the first base of the reverse complement
    __device__ __forceinline__ void init(uint64_t w0, uint64_t w1, uint64_t, uint32_t t, int k) {
        const uint32_t s = 62 - 2 * t;
        const uint64_t cat = s ? (w0 >> s) | (w1 << (64 - s)) : w0;
        mask = (1ull << (2 * k)) - 1;
        fwd = cat & mask;
        rc = ~group_reverse(fwd) >> (64 - 2 * k);
        top = 2 * k - 2;
    }
    __device__ __forceinline__ void step(uint32_t b) {
        fwd = ((fwd << 2) | b) & mask;
        rc = (rc >> 2) | ((uint64_t)(3u - b) << top);
    }
    __device__ __forceinline__ uint64_t key() const { return fwd < rc ? fwd : rc; }
};

struct Roll2 {
    uint64_t hi, lo, rhi, rlo, hmask;
    int top;  // 2k - 2
    __device__ __forceinline__ void init(uint64_t w0, uint64_t w1, uint64_t w2, uint32_t t, int k) {
        const uint32_t s = 62 - 2 * t;
        if (s) {
            lo = (w0 >> s) | (w1 << (64 - s));
            hi = (w1 >> s) | (w2 << (64 - s));
        } else {
            lo = w0;
            hi = w1;
        }
        hmask = (1ull << (2 * k - 64)) - 1;
        hi &= hmask;
        const uint64_t a_hi = ~group_reverse(lo);
        const uint64_t a_lo = ~group_reverse(hi);
        const int sh = 128 - 2 * k;  // 2..64
        if (sh == 64) {
            rlo = a_hi;
            rhi = 0;
        } else {
            rlo = (a_lo >> sh) | (a_hi << (64 - sh));
            rhi = a_hi >> sh;
        }
        top = 2 * k - 2;
    }
    __device__ __forceinline__ void step(uint32_t b) {
        hi = ((hi << 2) | (lo >> 62)) & hmask;
        lo = (lo << 2) | b;
        const uint64_t c = 3u - b;
        rlo = (rlo >> 2) | (rhi << 62);
        rhi >>= 2;
        if (top >= 64)
            rhi |= c << (top - 64);
        else
            rlo |= c << top;  // k = 32
    }
    __device__ __forceinline__ Key2 key() const {
        const bool fwd_smaller = hi < rhi || (hi == rhi && lo <= rlo);
        return fwd_smaller ? Key2{hi, lo} : Key2{rhi, rlo};
    }
};

template <bool TWO>
struct KeyOf;
template <>
struct KeyOf<false> {
    using type = uint64_t;
    using Roll = Roll1;
    __device__ __forceinline__ static uint64_t get(const uint64_t *packed, uint64_t w, uint32_t t, int k) {
        return window_key1(packed, w, t, k);
    }
    __device__ __forceinline__ static uint64_t get(uint64_t w0, uint64_t w1, uint64_t, uint32_t t, int k) {
        return window_key1(w0, w1, t, k);
    }
};
template <>
struct KeyOf<true> {
    using type = Key2;
    using Roll = Roll2;
    __device__ __forceinline__ static Key2 get(const uint64_t *packed, uint64_t w, uint32_t t, int k) {
        return window_key2(packed, w, t, k);
    }
    __device__ __forceinline__ static Key2 get(uint64_t w0, uint64_t w1, uint64_t w2, uint32_t t, int k) {
        return window_key2(w0, w1, w2, t, k);
    }
};

}  // namespace tk
