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
    return shift >= 64 ? ((uint32_t)(key.hi >> (shift - 64)) & mask)
                       : (uint32_t)(key.lo >> shift) & mask;
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

// Inclusive prefix sum across the wave.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t t = __shfl_up(v, d, WAVE);
        if (l >= (uint32_t)d)
            v += t;
    }
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

}  // namespace tk
