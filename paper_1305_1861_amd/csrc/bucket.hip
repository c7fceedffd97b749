// Per-bucket screen, sort and compaction in LDS.
//
// The keys arrive partitioned by bucket (top D bits): a bucket is one range,
// or, after a second partition pass, one piece per tile of its segment (the
// kernel reads the tiles' prefix tables to find them).  Every bucket owns a
// pattern-blocked Bloom filter sized from its own number of windows, so the
// filter of one bucket fits in LDS and is touched by one workgroup only -- the
// GPU counterpart of the paper's per-consumer filters (§2.1, parallelization:
// a k-mer always meets the same filter because it is routed by a function of
// its value).  Within a group of whole buckets (§2.1 PBF, sorting and
// compaction, Algorithm 1):
//   screen : per window and pattern word, old = atomicOr(S[w], m_w) and
//            atomicOr(T[w], old & m_w) -- skipped when T[w] already holds
//            m_w, since bits are only ever set and T is a subset of S;
//   collect: a window survives iff all its pattern bits hold in T (decided
//            in the screen for the windows that found them all set);
//   sort   : one MSD pass on the top bits of (bucket - first bucket, key
//            bits below the bucket digit) into 4096 bins, then the bins that
//            hold different keys ranked by waves, two bins of at most 64
//            keys side by side or a larger bin alone (LSD passes only for
//            groups whose bins are too large for that);
//   compact: run-length compaction, threshold c, (key, count) records written
//            at the group's first window index (gathered into place after).
//
// Groups are planned before the launch (plan_groups: whole buckets of one
// library within the register and filter capacity); persistent workgroups
// take chunks of groups from a counter.  A bucket with more windows than fit
// in registers is listed for the fallback path (global-memory kernels with
// the same filter semantics).
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int BK_THREADS = 512;
constexpr int BK_WAVES = BK_THREADS / WAVE;
constexpr int BK_SORT_BITS = 9;
constexpr int BK_BINS = 1 << BK_SORT_BITS;  // == BK_THREADS: one bin per thread
constexpr int BK_TABLE_BITS = 10;         // log2 of the largest pattern table (the default)
constexpr int BK_TABLE = 1 << BK_TABLE_BITS;  // pattern table entries held in LDS (max)

// Keys per thread of a group (tile shape; options.bucket_tile picks one):
// tile 0 holds 7168 one-word or 3584 two-word windows per group in
// registers, tile 1 holds 6144 or 3072 (fewer registers, smaller groups).
template <typename K, int TILE>
struct BkItems;
template <int TILE>
struct BkItems<uint64_t, TILE> {
    static constexpr int value = TILE ? 12 : 14;
};
template <int TILE>
struct BkItems<Key2, TILE> {
    static constexpr int value = TILE ? 6 : 7;
};
constexpr int BK_RMAX = 1024;  // buckets per group
constexpr int BK_MSD_BITS = 12;  // first (MSD) sort pass: 4096 bins, 16-bit counters in the LSD counter array
constexpr int BK_MSD_BINS = 1 << BK_MSD_BITS;
constexpr int BK_PMAX = 2 * (BK_RMAX + 1);  // keys of mixed bins radix-sorted through a position map
constexpr int BK_LIST_MAX = BK_PMAX / 2;     // mixed bins listed for the rank sort
constexpr int BK_RANK_MAX = 256;             // largest bin the rank sort takes (4 keys per lane)
static_assert(BK_MSD_BINS == 8 * BK_THREADS, "bin starts: eight bins per thread");
static_assert(BK_MSD_BINS / 2 == BK_WAVES * BK_BINS / 2, "MSD counters reuse the LSD counter array");

template <typename K>
__device__ __forceinline__ uint32_t bucket_of(const K &key, int k, int D) {
    return digit_of(key, 2 * k - D, (1u << D) - 1u);
}

// Library of bucket id b: the largest j with libs[j].bucket0 <= b.
__device__ __forceinline__ uint32_t library_of_bucket(const BucketArgs &a, uint32_t b) {
    uint32_t lo = 0, hi = a.n_libs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (a.libs[mid].bucket0 <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <typename K>
__device__ __forceinline__ K sentinel();
template <>
__device__ __forceinline__ uint64_t sentinel<uint64_t>() { return ~0ull; }
template <>
__device__ __forceinline__ Key2 sentinel<Key2>() { return Key2{~0ull, ~0ull}; }

// A group's virtual sort key V = ((bucket - d0) << SB) | (key bits below
// the bucket digit) is key - (d0 << SB): the group's keys belong to one
// library and their buckets are at least d0.  vbase = d0 << SB.
template <typename K>
__device__ __forceinline__ K group_base(uint32_t d0, int SB);
template <>
__device__ __forceinline__ uint64_t group_base<uint64_t>(uint32_t d0, int SB) {
    return SB < 64 ? (uint64_t)d0 << SB : 0ull;  // SB <= 62 for one-word keys
}
template <>
__device__ __forceinline__ Key2 group_base<Key2>(uint32_t d0, int SB) {
    if (SB >= 64)
        return Key2{(uint64_t)d0 << (SB - 64), 0ull};
    if (SB == 0)
        return Key2{0ull, (uint64_t)d0};
    return Key2{(uint64_t)d0 >> (64 - SB), (uint64_t)d0 << SB};
}
__device__ __forceinline__ uint64_t key_sub(uint64_t a, uint64_t b) { return a - b; }
__device__ __forceinline__ Key2 key_sub(const Key2 &a, const Key2 &b) {
    return Key2{a.hi - b.hi - (a.lo < b.lo ? 1ull : 0ull), a.lo - b.lo};
}

// Bits [shift, shift + nbits) of V, nbits <= 12.
template <typename K>
__device__ __forceinline__ uint32_t vdigit(const K &key, int shift, int nbits, const K &vbase) {
    return digit_of(key_sub(key, vbase), shift, (1u << nbits) - 1u);
}

// Start and size of bin d of the MSD pass (starts packed two per word).
__device__ __forceinline__ uint32_t msd_bin_start(const uint32_t *s_c32, uint32_t d) {
    return (s_c32[d >> 1] >> ((d & 1u) * 16u)) & 0xFFFFu;
}
__device__ __forceinline__ uint32_t msd_bin_size(const uint32_t *s_c32, uint32_t d, uint32_t n) {
    const uint32_t end = d + 1 < (uint32_t)BK_MSD_BINS ? msd_bin_start(s_c32, d + 1) : n;
    return end - msd_bin_start(s_c32, d);
}

// In-place exclusive prefix of m <= 2 * WAVE counters v[0, m), run by the
// lanes of one wave; lane WAVE - 1 returns the total.
__device__ __forceinline__ uint32_t exclusive_parts(uint32_t *v, int m, int lane) {
    const uint32_t v0 = 2 * lane < m ? v[2 * lane] : 0u;
    const uint32_t v1 = 2 * lane + 1 < m ? v[2 * lane + 1] : 0u;
    const uint32_t inc = wave_inclusive_sum(v0 + v1);
    const uint32_t ex = inc - v0 - v1;
    if (2 * lane < m)
        v[2 * lane] = ex;
    if (2 * lane + 1 < m)
        v[2 * lane + 1] = ex + v0;
    return inc;
}

// The value of lane - 1 (lane 0 receives its own value): a wave-wide DPP
// shift by one lane.
__device__ __forceinline__ uint32_t shift_up_lane(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
}
__device__ __forceinline__ uint64_t shift_up_lane(uint64_t x) {
    return ((uint64_t)shift_up_lane((uint32_t)(x >> 32)) << 32) | shift_up_lane((uint32_t)x);
}
__device__ __forceinline__ Key2 shift_up_lane(const Key2 &x) { return Key2{shift_up_lane(x.hi), shift_up_lane(x.lo)}; }

// Number of lanes whose flag is set in a ballot.
__device__ __forceinline__ uint32_t wave_count(uint64_t ball) { return (uint32_t)__popcll(ball); }

// Orders NB bins of at most WAVE keys each side by side, run by one wave,
// one key per lane and bin: bin b's keys s_ex[st[b], st[b] + m[b]) (m[b] =
// 0: no bin).  A key's place in its bin is the number of smaller keys plus
// the number of equal keys before it.  Each step takes one pending distinct
// value of every bin; the bins' steps are independent, so one bin's waits
// overlap the others' work.  Past 8 + m / 16 values, a bin's remaining keys
// scan the bin instead.
template <typename K, int NB>
__device__ __forceinline__ void rank_bins(K *s_ex, const uint32_t (&st)[NB], const uint32_t (&m)[NB], uint32_t lane,
                                          uint64_t lt) {
    K x[NB];
    uint32_t rk[NB], cap[NB];
    bool pend[NB];  // the lane's key has no place yet
#pragma unroll
    for (int b = 0; b < NB; b++) {
        cap[b] = 8u + m[b] / 16u;
        rk[b] = 0;
        pend[b] = lane < m[b];
        x[b] = pend[b] ? s_ex[st[b] + lane] : sentinel<K>();
    }
    for (uint32_t it = 0;; it++) {
        uint64_t first[NB], any = 0;  // lanes with a pending key
#pragma unroll
        for (int b = 0; b < NB; b++) {
            first[b] = __ballot(it < cap[b] && pend[b]);
            any |= first[b];
        }
        if (!any)
            break;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const K v = read_lane(x[b], first[b] ? (int)__builtin_ctzll(first[b]) : 0);
            const uint32_t less = (uint32_t)__popcll(__ballot(x[b] < v));  // empty lanes hold the sentinel
            const bool eq = first[b] && pend[b] && x[b] == v;
            const uint64_t qb = __ballot(eq);
            rk[b] = eq ? less + (uint32_t)__popcll(qb & lt) : rk[b];
            pend[b] = pend[b] && !eq;
        }
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        if (__ballot(pend[b])) {
            for (uint32_t j = 0; j < m[b]; j++) {
                const K y = s_ex[st[b] + j];
                if (pend[b])
                    rk[b] += (y < x[b] || (y == x[b] && j < lane)) ? 1u : 0u;
            }
        }
        if (lane < m[b])
            s_ex[st[b] + rk[b]] = x[b];
    }
}

// TBITS: log2 of the pattern table entries when fixed at compile time (the
// default table: the pattern fields of the hash become constant shifts), or
// 0 to take it from the arguments.
template <typename K, int TBITS, int TILE>
// Two workgroups per CU (LDS < 80 KB each) hide more latency than the
// registers saved by running one.
__global__ __launch_bounds__(BK_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void bucket_kernel(BucketArgs a) {
    constexpr int ITEMS = BkItems<K, TILE>::value;
    constexpr int CAP = BK_THREADS * ITEMS;
    // filter blocks that fit in the exchange buffer
    constexpr uint32_t FMAX = (uint32_t)((CAP + 2) * sizeof(K) / 64);
    __shared__ uint64_t s_table[BK_TABLE];
    __shared__ __align__(16) uint16_t s_cnt[BK_WAVES][BK_BINS];
    // exchange buffer with a sentinel slot on each side; holds the filters
    // during screen/collect
    __shared__ __align__(16) K s_exs[CAP + 2];
    // first index of each bucket of the group, then the first filter block of
    // each bucket; during the sort, the position map of the mixed bins
    __shared__ __align__(16) uint16_t s_aux[2 * (BK_RMAX + 1)];
    uint16_t *const s_start = s_aux;
    uint16_t *const s_fo = s_aux + BK_RMAX + 1;
    __shared__ uint32_t s_mix[BK_MSD_BINS / 32];  // mixed-bin flags of the MSD pass
    __shared__ uint32_t s_part[ITEMS][BK_WAVES];
    __shared__ uint32_t s_w[2][BK_WAVES];
    __shared__ uint32_t s_u[4];
    __shared__ uint32_t s_chunk;
    // statistics accumulated over the workgroup's groups: per wave (false
    // positives, counts in [2, c), runs) and per workgroup (survivors); every
    // sum is below the number of windows, hence below 2^32
    __shared__ uint32_t s_acc[BK_WAVES][3];
    __shared__ uint32_t s_tot[1];
    // pieces of the next group of a tiled library (one per tile of its
    // segment): s_pc[p] piece p's size, then the group index of its first
    // key; s_lo[p] its first key's offset in its tile.  Row r (group indices
    // 64 r .. 64 r + 63, the keys of item r / BK_WAVES of wave r % BK_WAVES)
    // has one record, read by the wave at one address: x = key offset of the
    // piece holding index 64 r (key position of group index e: segment start
    // + offset + e), y = that of a piece starting inside the row, z = that
    // piece's first lane (WAVE if none), w = pieces starting inside the row
    // | (piece of index 64 r << 16).
    constexpr int ROWS = (CAP + WAVE - 1) / WAVE;
    static_assert(ROWS == ITEMS * BK_WAVES, "one row per item and wave");
    __shared__ uint16_t s_pc[BK_TILES_MAX], s_lo[BK_TILES_MAX];
    __shared__ uint4 s_row[ROWS];
    constexpr int PPL = BK_TILES_MAX / WAVE;  // rounds of pieces of wave 0
    static_assert(PPL * WAVE == BK_TILES_MAX, "whole rounds of pieces");

    K *const s_ex = s_exs + 1;
    uint64_t *s_filter = reinterpret_cast<uint64_t *>(s_exs);
    const int tid0 = threadIdx.x;
    const K *__restrict__ keys = static_cast<const K *>(a.keys);
    K *__restrict__ gap_keys = static_cast<K *>(a.gap_keys);
    const int tbits = TBITS ? TBITS : (int)a.table_bits;
    const uint32_t n_tab = 1u << tbits;
    const uint32_t tmask = n_tab - 1;
    for (uint32_t i = tid0; i < n_tab; i += BK_THREADS)
        s_table[i] = a.table[i];
    if (tid0 < 3 * BK_WAVES)
        (&s_acc[0][0])[tid0] = 0;
    if (tid0 == 0)
        s_tot[0] = 0;

    __syncthreads();
    // Chunks of the key array (whole groups; bounds precomputed) are taken
    // from a counter: a group's cost is not proportional to its keys (small
    // groups of large buckets pay the same per-group overhead), so equal key
    // ranges per workgroup would finish unevenly.
    uint32_t jl = 0;  // library of the groups being processed (0: nothing gathered yet)
    // statistics of library jl gathered so far go to its counters (thread 0;
    // the counters it reads were written before a barrier)
    auto flush_stats = [&](uint32_t j) {
        unsigned long long t[3] = {0, 0, 0};
        for (int w = 0; w < BK_WAVES; w++)
            for (int q = 0; q < 3; q++) {
                t[q] += s_acc[w][q];
                s_acc[w][q] = 0;
            }
        unsigned long long *o = a.lib_stats + 4 * (uint64_t)j;
        atomicAdd(o + 0, (unsigned long long)s_tot[0]);
        atomicAdd(o + 1, t[2]);
        atomicAdd(o + 2, t[0]);
        atomicAdd(o + 3, t[1]);
        s_tot[0] = 0;
    };
    // keys [p, p + n) of a group (item-major, sentinel past them); every
    // element is assigned so that no value is carried from one group to the
    // next
    K key[ITEMS];
    auto load_group = [&](uint64_t p, uint32_t n, int t) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint32_t e = (uint32_t)i * BK_THREADS + t;
            key[i] = sentinel<K>();
            if (e < n)
                key[i] = keys[p + e];
        }
    };
    // A group of a tiled library is one piece per tile of its segment
    // (descriptor gp: first tile, tiles, segment start, digits): (1) thread
    // t < tiles reads tile t's prefix entries of the group's first digit and
    // of the digit after its last, (2) writes the piece's size and offset,
    // (3) after a barrier wave 0 turns the sizes into the group indices of
    // the pieces and fills the row records, (4) after another barrier every
    // thread loads its keys: one LDS round trip for the rows of all its
    // items, the rare rows with two or more piece starts walked afterwards.
    const uint32_t tile_keys = a.layout.tile_keys, pw = a.layout.pw;
    auto piece_read = [&](const uint4 &gp, int t, uint32_t &lo, uint32_t &hi) __attribute__((always_inline)) {
        lo = hi = 0;
        if ((uint32_t)t < gp.y) {
            const uint16_t *col = a.layout.px + (uint64_t)gp.x * pw + (uint32_t)t;
            lo = col[(gp.w & 0xFFFFu) * gp.y];
            hi = col[((gp.w >> 16) + 1) * gp.y];
        }
    };
    auto piece_write = [&](const uint4 &gp, int t, uint32_t lo, uint32_t hi) __attribute__((always_inline)) {
        if ((uint32_t)t < gp.y) {
            s_pc[t] = (uint16_t)(hi - lo);
            s_lo[t] = (uint16_t)lo;
        }
    };
    auto piece_index = [&](const uint4 &gp, uint32_t ln) __attribute__((always_inline)) {  // wave 0
        const uint32_t np = gp.y;  // <= BK_TILES_MAX = PPL * WAVE
        for (uint32_t r = ln; r < (uint32_t)ROWS; r += WAVE) {
            s_row[r].z = WAVE;
            s_row[r].w = 0;
        }
        // piece p on lane p % WAVE, in rounds of WAVE pieces (one round for
        // most groups); run: the group index of the piece's first key
        uint32_t base = 0;
#pragma unroll
        for (int q = 0; q < PPL; q++) {
            if ((uint32_t)q * WAVE < np) {
                const uint32_t p = (uint32_t)q * WAVE + ln;
                const uint32_t v = p < np ? (uint32_t)s_pc[p] : 0u;
                const uint32_t o = p < np ? (uint32_t)s_lo[p] : 0u;
                const uint32_t inc = wave_inclusive_sum(v);
                const uint32_t run = base + inc - v;
                base += (uint32_t)__shfl(inc, WAVE - 1);
                if (p < np) {
                    s_pc[p] = (uint16_t)run;
                    if (v) {
                        const uint32_t dl = p * tile_keys + o - run;
                        if (run & (WAVE - 1)) {
                            const uint32_t r = run / WAVE;
                            atomicAdd(&s_row[r].w, 1u);
                            s_row[r].y = dl;
                            s_row[r].z = run & (WAVE - 1);
                        }
                        for (uint32_t r = (run + WAVE - 1) / WAVE; r * WAVE < run + v; r++) {
                            s_row[r].x = dl;
                            atomicOr(&s_row[r].w, p << 16);
                        }
                    }
                }
            }
        }
    };
    auto piece_load = [&](const uint4 &gp, uint32_t n, int t) __attribute__((always_inline)) {
        const uint32_t np = gp.y, ln = (uint32_t)t % WAVE;
        uint32_t dl[ITEMS];
        uint32_t many = 0;  // bit i: two or more pieces start inside item i's row
        const uint32_t wv = (uint32_t)t / WAVE;
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint32_t e = (uint32_t)i * BK_THREADS + (uint32_t)t;
            const uint4 rec = s_row[(uint32_t)i * BK_WAVES + wv];  // the row of e
            dl[i] = ln >= rec.z ? rec.y : rec.x;
            many |= (uint32_t)(e < n && (rec.w & 0xFFFFu) > 1) << i;
        }
        if (many) {
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if ((many >> i) & 1u) {
                    const uint32_t e = (uint32_t)i * BK_THREADS + (uint32_t)t;
                    uint32_t p = s_row[e / WAVE].w >> 16;
                    while (p + 1 < np && (uint32_t)s_pc[p + 1] <= e)
                        p++;
                    dl[i] = p * tile_keys + s_lo[p] - s_pc[p];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint32_t e = (uint32_t)i * BK_THREADS + (uint32_t)t;
            key[i] = sentinel<K>();
            if (e < n)
                key[i] = keys[(uint32_t)(gp.z + dl[i] + e)];
        }
    };
    for (;;) {
    if (tid0 == 0)
        s_chunk = atomicAdd(a.chunk_next, 1u);
    __syncthreads();
    const uint32_t chunk = s_chunk;
    __syncthreads();  // s_chunk is rewritten only after every thread has read it
    if (chunk >= a.n_chunks)
        break;
    const uint32_t n_grp = a.grp_count[chunk];
    const uint32_t gbase = chunk * a.chunk_buckets;
    if (n_grp == 0)
        continue;
    // the chunk's first group: buckets [b0, b1], keys [pos, pos + n_sb)
    uint32_t b0 = a.grp_first[gbase], b1 = a.grp_last[gbase];
    uint64_t pos = a.bucket_starts[b0];
    uint32_t n_sb = a.bucket_starts[b1 + 1] - (uint32_t)pos;
    {
        // (thread index laundered as in the group loop below, so that the
        // compiler does not hoist per-item addresses out of the chunk loop)
        int tidc = tid0;
        asm volatile("" : "+v"(tidc));
        const uint4 gp = a.grp_piece[gbase];
        if (gp.y) {
            uint32_t lo, hi;
            piece_read(gp, tidc, lo, hi);
            piece_write(gp, tidc, lo, hi);
            __syncthreads();
            if (tidc < WAVE)
                piece_index(gp, (uint32_t)tidc);
            __syncthreads();
            piece_load(gp, n_sb, tidc);
        } else {
            load_group(pos, n_sb, tidc);
        }
    }

    for (uint32_t g = 0; g < n_grp; g++) {
        // Thread indices are passed through an empty asm each iteration so
        // the compiler recomputes what depends on them inside the loop
        // instead of keeping dozens of hoisted lane masks alive across it.
        int tid = tid0;
        asm volatile("" : "+v"(tid));
        const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
        const uint32_t lane = (uint32_t)tid % WAVE;
        const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
        // the chunk's next group: buckets, and its pieces for a tiled library
        uint32_t nb0 = 0, nb1 = 0;
        uint4 ngp = make_uint4(0, 0, 0, 0);
        if (g + 1 < n_grp) {
            nb0 = a.grp_first[gbase + g + 1];
            nb1 = a.grp_last[gbase + g + 1];
            ngp = a.grp_piece[gbase + g + 1];
        }

        // ---- the group's library ----
        {
            const uint32_t jn = library_of_bucket(a, b0);
            if (jn != jl) {
                if (tid == 0)
                    flush_stats(jl);
                jl = jn;
            }
        }
        const int D = a.libs[jl].D;            // bucket bits of the library
        const int kk = a.libs[jl].k;           // its k
        const uint32_t c = a.libs[jl].c;       // its threshold
        const bool screen = c >= 2;
        const uint32_t bucket0 = a.libs[jl].bucket0;
        const int SB = 2 * kk - D;  // key bits below the bucket digit

        // ---- a group of whole buckets b0..b1 of one library (planned
        // before the launch; keys loaded by the previous iteration) ----
        const int n_items = (int)((n_sb + BK_THREADS - 1) / BK_THREADS);
        const uint32_t d0 = b0 - bucket0;
        const uint32_t R = b1 - b0 + 1;  // bucket ids spanned, <= BK_RMAX
        const K vbase = group_base<K>(d0, SB);
        // start of every bucket in the group, then its first filter block
        for (uint32_t r = tid; r <= R; r += BK_THREADS)
            s_start[r] = (uint16_t)(a.bucket_starts[b0 + r] - (uint32_t)pos);
        __syncthreads();
        if (wave == 0) {
            uint32_t carry = 0;
            for (uint32_t r0 = 0; r0 < R; r0 += WAVE) {
                const uint32_t r = r0 + lane;
                uint32_t nb = 0;
                if (r < R) {
                    const uint32_t ns = (uint32_t)s_start[r + 1] - s_start[r];
                    nb = (screen && ns) ? max(1u, (a.beta * ns + 255) / 256) : 0u;
                }
                const uint32_t inc = wave_inclusive_sum(nb);
                if (r < R)
                    s_fo[r] = (uint16_t)(carry + inc - nb);
                carry += (uint32_t)__shfl(inc, WAVE - 1);
            }
            if (lane == 0)
                s_fo[R] = (uint16_t)carry;
        }
        __syncthreads();
        const uint32_t blocks_cut = s_fo[R];
        uint32_t rb[ITEMS];  // bucket of each key, relative to b0; after the screen its filter block
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            rb[i] = 0;
            if (i < n_items && (uint32_t)i * BK_THREADS + tid < n_sb)
                rb[i] = bucket_of(key[i], kk, D) - d0;
        }
        // span of bucket ids in the group -> bits of the bucket part of the sort key
        const uint32_t span = R - 1;
        const int RB = span ? 32 - __clz(span) : 0;

        // ---- screen and collect, each bucket against its own filter ----
        // In LDS the group's filters are stored as 8 word planes (word q of
        // block x at q * blocks_cut + x) so that the lanes of a wave touching
        // the same word of different blocks fall in different banks.
        uint32_t sv = 0;  // bit i: item i survives
        if (screen) {
            for (uint32_t i = tid; i < blocks_cut * 8; i += BK_THREADS)
                s_filter[i] = 0;
            __syncthreads();
            // Bits are only ever set, and a second-plane bit implies its
            // first-plane bit, so a word whose pattern bits are all in the
            // second plane already needs no update: one read replaces both
            // atomics (on deep libraries, for most sightings).  A sighting
            // that finds all its bits set in either plane sets them all in
            // the second plane, so its key is a candidate whatever comes
            // later: it is marked now and skips the collect test.
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (i < n_items && (uint32_t)i * BK_THREADS + tid < n_sb) {
                    const uint32_t f0 = s_fo[rb[i]], nb = (uint32_t)s_fo[rb[i] + 1] - f0;
                    const uint64_t h = key_hash(key[i]);
                    rb[i] = f0 + (uint32_t)__umul64hi(h, nb);  // from here on: the key's filter block
                    uint64_t *b = s_filter + rb[i];
                    // the four pattern words and second-plane words are
                    // read together, then the first-plane atomics of the
                    // words that need them are issued together, so that a
                    // key waits for LDS three times rather than nine
                    uint64_t m[4], o[4];
                    uint32_t need = 0;  // bit w: word w lacks some of its bits in the second plane
#pragma unroll
                    for (int w = 0; w < 4; w++) {
                        m[w] = s_table[(h >> (w * tbits)) & tmask];
                        const uint64_t t = b[(4 + w) * blocks_cut];
                        need |= (uint32_t)((t & m[w]) != m[w]) << w;
                    }
#pragma unroll
                    for (int w = 0; w < 4; w++) {
                        o[w] = m[w];
                        if ((need >> w) & 1u)
                            o[w] = atomicOr((unsigned long long *)(b + w * blocks_cut), (unsigned long long)m[w]);
                    }
                    bool seen = true;
#pragma unroll
                    for (int w = 0; w < 4; w++) {
                        const uint64_t hit = o[w] & m[w];
                        if (((need >> w) & 1u) && hit)
                            atomicOr((unsigned long long *)(b + (4 + w) * blocks_cut), (unsigned long long)hit);
                        seen &= hit == m[w];
                    }
                    sv |= (uint32_t)seen << i;
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (i < n_items && (uint32_t)i * BK_THREADS + tid < n_sb && !((sv >> i) & 1u)) {
                    const uint64_t h = key_hash(key[i]);
                    const uint64_t *b = s_filter + rb[i] + 4 * blocks_cut;  // the block the screen chose
                    bool all = true;
#pragma unroll
                    for (int w = 0; w < 4; w++) {
                        const uint64_t m = s_table[(h >> (w * tbits)) & tmask];
                        all &= (b[w * blocks_cut] & m) == m;
                    }
                    sv |= (uint32_t)all << i;
                }
            }
            __syncthreads();  // the filter area becomes the exchange buffer
        } else {
#pragma unroll
            for (int i = 0; i < ITEMS; i++)
                if (i < n_items && (uint32_t)i * BK_THREADS + tid < n_sb)
                    sv |= 1u << i;
        }

        // ---- sort the survivors by the virtual key V = ((bucket - d0) << SB) |
        // (key bits below the bucket digit), TB bits; within the group V is
        // a bijection of the key, so sorting by V sorts the keys ----
        // (1) one MSD pass on the top MB <= 12 bits of V into 4096 bins
        //     (unordered within a bin: LDS atomics on packed 16-bit counters);
        // (2) a bin whose keys are not all equal is "mixed";
        // (3) the keys of mixed bins (a quarter of the survivors on deep
        //     libraries with repeats: copies and error k-mers share
        //     prefixes) are ranked within their bins by waves; groups with a
        //     bin of more than BK_RANK_MAX keys, or too many mixed bins, take
        //     an LSD radix sort (9-bit digits, stable wave-match ranking)
        //     over just the mixed bins' positions, or over the whole group
        //     when there are too many of them to map.
        const int TB = SB + RB;
        const int MB = min(BK_MSD_BITS, TB);
        const int mshift = TB - MB;
        uint32_t *const s_c32 = reinterpret_cast<uint32_t *>(&s_cnt[0][0]);
        for (int i = tid; i < BK_WAVES * BK_BINS / 4; i += BK_THREADS)
            reinterpret_cast<uint64_t *>(&s_cnt[0][0])[i] = 0;
        if (tid < BK_MSD_BINS / 32)
            s_mix[tid] = 0;
        __syncthreads();
        uint32_t rd[ITEMS];  // MSD pass: (rank << 12) | bin; LSD passes: (rank << 9) | digit
        // four items at a time: their counter updates are issued before any
        // of their results is used
#pragma unroll
        for (int i0 = 0; i0 < ITEMS; i0 += 4) {
            uint32_t old[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int i = i0 + j;
                if (i < ITEMS) {
                    rd[i] = 0;
                    old[j] = 0;
                    if (i < n_items && ((sv >> i) & 1u)) {
                        rd[i] = vdigit(key[i], mshift, MB, vbase);
                        old[j] = atomicAdd(&s_c32[rd[i] >> 1], 1u << ((rd[i] & 1u) * 16u));
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int i = i0 + j;
                if (i < ITEMS)
                    rd[i] |= ((old[j] >> ((rd[i] & 1u) * 16u)) & 0xFFFFu) << BK_MSD_BITS;
            }
        }
        __syncthreads();
        uint32_t n_surv;
        {
            // bin starts; thread t owns bins 8t .. 8t+7 (words 4t .. 4t+3)
            uint4 w = reinterpret_cast<const uint4 *>(s_c32)[tid];
            const uint32_t c0 = w.x & 0xFFFFu, c1 = w.x >> 16, c2 = w.y & 0xFFFFu, c3 = w.y >> 16;
            const uint32_t c4 = w.z & 0xFFFFu, c5 = w.z >> 16, c6 = w.w & 0xFFFFu, c7 = w.w >> 16;
            const uint32_t s0 = block_exclusive_sum<BK_THREADS>(c0 + c1 + c2 + c3 + c4 + c5 + c6 + c7, &n_surv);
            const uint32_t s1 = s0 + c0, s2 = s1 + c1, s3 = s2 + c2, s4 = s3 + c3, s5 = s4 + c4, s6 = s5 + c5,
                           s7 = s6 + c6;
            w = make_uint4(s0 | (s1 << 16), s2 | (s3 << 16), s4 | (s5 << 16), s6 | (s7 << 16));
            reinterpret_cast<uint4 *>(s_c32)[tid] = w;
        }
        __syncthreads();
        // four items at a time: their bin starts are read before any key is
        // written (rd is 0 for items that hold no survivor: bin 0, in bounds)
#pragma unroll
        for (int i0 = 0; i0 < ITEMS; i0 += 4) {
            if (i0 < n_items) {
                uint32_t w[4];
#pragma unroll
                for (int j = 0; j < 4; j++)
                    if (i0 + j < ITEMS)
                        w[j] = s_c32[(rd[i0 + j] & (BK_MSD_BINS - 1)) >> 1];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int i = i0 + j;
                    if (i < ITEMS && ((sv >> i) & 1u)) {
                        const uint32_t st = (w[j] >> ((rd[i] & 1u) * 16u)) & 0xFFFFu;
                        s_ex[st + (rd[i] >> BK_MSD_BITS)] = key[i];
                    }
                }
            }
        }
        __syncthreads();
        // the keys are in s_ex: the next group's prefix entries are requested
        // now, written to LDS after the mixed-bin detection, indexed by wave 0
        // after the mixed-bin count, its keys loaded after the ordering
        uint32_t plo = 0, phi = 0;
        if (ngp.y)
            piece_read(ngp, tid, plo, phi);
        // mixed bins: a key differing from its left neighbour in the same bin
        const int n_ch = (int)((n_surv + BK_THREADS - 1) / BK_THREADS);
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint32_t e = (uint32_t)i * BK_THREADS + tid;
            if (i < n_ch && e > 0 && e < n_surv) {
                const K x = s_ex[e], y = s_ex[e - 1];
                if (x != y) {
                    const uint32_t dx = vdigit(x, mshift, MB, vbase);
                    if (dx == vdigit(y, mshift, MB, vbase))
                        atomicOr(&s_mix[dx >> 5], 1u << (dx & 31u));
                }
            }
        }
        __syncthreads();
        if (ngp.y)
            piece_write(ngp, tid, plo, phi);
        // mixed bins of this thread (bins 8t .. 8t+7): number, keys, oversized
        // ones, packed into one sum (each field stays below 2^13, 2^13, 2^6)
        const uint32_t mixw = (s_mix[tid >> 2] >> ((tid & 3u) * 8u)) & 0xFFu;
        uint32_t mine = 0;
        if (mixw) {
            for (int j = 0; j < 8; j++) {
                if ((mixw >> j) & 1u) {
                    const uint32_t m = msd_bin_size(s_c32, tid * 8 + j, n_surv);
                    mine += m | (1u << 13) | ((m > BK_RANK_MAX ? 1u : 0u) << 26);
                }
            }
        }
        uint32_t mix_tot;
        const uint32_t mix_ex = block_exclusive_sum<BK_THREADS>(mine, &mix_tot);
        if (ngp.y && wave == 0)
            piece_index(ngp, lane);  // read by piece_load after a barrier
        uint32_t n_sort = mix_tot & 0x1FFFu;
        const uint32_t n_mb = (mix_tot >> 13) & 0x1FFFu, n_big = mix_tot >> 26;
        if (n_sort > 0 && n_big == 0 && n_mb <= BK_LIST_MAX) {
            // one wave per mixed bin, keys in registers (up to 4 per lane).
            // A key's place in its bin is the number of smaller keys in the
            // bin plus the number of equal keys before it.  Distinct values
            // are taken one at a time (a value of a pending lane, its number
            // of smaller keys by ballots); a bin with many distinct values
            // finishes with a scan of the bin per key instead.
            uint32_t *const s_list = reinterpret_cast<uint32_t *>(s_aux);  // (start, size) of each mixed bin
            if (mixw) {
                uint32_t idx = (mix_ex >> 13) & 0x1FFFu;
                for (int j = 0; j < 8; j++) {
                    if ((mixw >> j) & 1u) {
                        const uint32_t d = tid * 8 + j;
                        s_list[idx++] = msd_bin_start(s_c32, d) | (msd_bin_size(s_c32, d, n_surv) << 16);
                    }
                }
            }
            if (tid == 0)
                s_u[2] = 0;
            __syncthreads();
            // A wave takes two list entries at a time.  Those of at most a
            // wave's keys are ranked side by side, one key per lane each:
            // their ranking steps are independent and issued together, so
            // that one bin's waits overlap the other's work (more bins in
            // flight measured slower).  A larger bin goes through the
            // general ranking below.
            constexpr int NB = 2;
            for (;;) {
                uint32_t idx = 0;
                if (lane == 0)
                    idx = atomicAdd(&s_u[2], (uint32_t)NB);
                idx = __builtin_amdgcn_readfirstlane(idx);
                if (idx >= n_mb)
                    break;
                uint32_t es[NB], sm = 0;  // entries (0: none); bit b: entry b is small
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    es[b] = idx + b < n_mb ? __builtin_amdgcn_readfirstlane(s_list[idx + b]) : 0u;
                    sm |= (uint32_t)(es[b] != 0 && (es[b] >> 16) <= WAVE) << b;
                }
                if (sm) {
                    uint32_t sts[NB], ms[NB];
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        sts[b] = es[b] & 0xFFFFu;
                        ms[b] = ((sm >> b) & 1u) ? es[b] >> 16 : 0u;
                    }
                    rank_bins<K, NB>(s_ex, sts, ms, lane, lt);
                }
                for (int b = 0; b < NB; b++) {
                    const uint32_t ent = es[b];
                    if (ent == 0 || ((sm >> b) & 1u))
                        continue;
                    const uint32_t st = ent & 0xFFFFu, m = ent >> 16;
                    constexpr int Q = BK_RANK_MAX / WAVE;
                    const int nq = (int)((m + WAVE - 1) / WAVE);
                    K x[Q];
                    uint32_t rk[Q];
                    uint32_t pend = 0;  // bit q: key q of this lane has no place yet
#pragma unroll
                    for (int q = 0; q < Q; q++) {
                        rk[q] = 0;
                        x[q] = sentinel<K>();
                        if ((uint32_t)(q * WAVE) + lane < m) {
                            x[q] = s_ex[st + q * WAVE + lane];
                            pend |= 1u << q;
                        }
                    }
                    const uint32_t cap = 8u + m / 16u;  // distinct values taken before switching
                    for (uint32_t it = 0;; it++) {
                        int q0 = -1;
                        uint64_t b0 = 0;
#pragma unroll
                        for (int q = 0; q < Q; q++) {
                            if (q < nq) {
                                const uint64_t b = __ballot((pend >> q) & 1u);
                                if (q0 < 0 && b) {
                                    q0 = q;
                                    b0 = b;
                                }
                            }
                        }
                        if (q0 < 0 || it == cap)
                            break;
                        const int l0 = (int)__builtin_ctzll(b0);
                        K v = sentinel<K>();
#pragma unroll
                        for (int q = 0; q < Q; q++)
                            if (q == q0)
                                v = read_lane(x[q], l0);
                        uint32_t less = 0;
#pragma unroll
                        for (int q = 0; q < Q; q++)
                            if (q < nq)
                                less += (uint32_t)__popcll(__ballot(x[q] < v));  // invalid slots hold the sentinel
#pragma unroll
                        for (int q = 0; q < Q; q++) {
                            if (q < nq) {
                                const bool eq = ((pend >> q) & 1u) && x[q] == v;
                                const uint64_t b = __ballot(eq);
                                if (eq) {
                                    rk[q] = less + (uint32_t)__popcll(b & lt);
                                    pend &= ~(1u << q);
                                }
                                less += (uint32_t)__popcll(b);
                            }
                        }
                    }
                    if (__ballot(pend != 0)) {
                        // remaining keys: scan the whole bin (four keys per step)
                        for (uint32_t j0 = 0; j0 < m; j0 += 4) {
                            K y[4];
#pragma unroll
                            for (int u = 0; u < 4; u++)
                                y[u] = j0 + u < m ? s_ex[st + j0 + u] : sentinel<K>();
#pragma unroll
                            for (int u = 0; u < 4; u++) {
                                const uint32_t j = j0 + u;
#pragma unroll
                                for (int q = 0; q < Q; q++)
                                    if (q < nq && ((pend >> q) & 1u))
                                        rk[q] += (y[u] < x[q] || (y[u] == x[q] && j < (uint32_t)(q * WAVE) + lane)) ? 1u : 0u;
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < Q; q++)
                        if ((uint32_t)(q * WAVE) + lane < m)
                            s_ex[st + rk[q]] = x[q];
                }
            }
            __syncthreads();
            n_sort = 0;
        }
        if (n_sort > 0) {
            // radix fallback over the keys of the mixed bins
            for (int i = tid; i < BK_WAVES * BK_BINS / 4; i += BK_THREADS)
                reinterpret_cast<uint64_t *>(&s_cnt[0][0])[i] = 0;
            uint32_t fm = 0;  // bit i: position i * BK_THREADS + tid lies in a mixed bin
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (i < n_ch) {
                    const uint32_t e = (uint32_t)i * BK_THREADS + tid;
                    bool f = false;
                    if (e < n_surv) {
                        const uint32_t d = vdigit(s_ex[e], mshift, MB, vbase);
                        f = (s_mix[d >> 5] >> (d & 31u)) & 1u;
                    }
                    fm |= (uint32_t)f << i;
                    const uint64_t fb = __ballot(f);
                    if (lane == 0)
                        s_part[i][wave] = (uint32_t)__popcll(fb);
                }
            }
            __syncthreads();
            if (tid < WAVE)
                exclusive_parts(&s_part[0][0], n_ch * BK_WAVES, tid);
            __syncthreads();
            const bool mapped = n_sort <= BK_PMAX;
            uint16_t *const s_map = s_aux;  // sorted position j lives at s_ex[s_map[j]]
            if (mapped) {
#pragma unroll
                for (int i = 0; i < ITEMS; i++) {
                    if (i < n_ch) {
                        const bool f = (fm >> i) & 1u;
                        const uint64_t fb = __ballot(f);
                        if (f)
                            s_map[s_part[i][wave] + (uint32_t)__popcll(fb & lt)] =
                                (uint16_t)((uint32_t)i * BK_THREADS + tid);
                    }
                }
            } else {
                n_sort = n_surv;
            }
            __syncthreads();
            // keys to sort, wave-striped: element (wave, item, lane)
            int act_items = (int)((n_sort + BK_THREADS - 1) / BK_THREADS);
            sv = 0;
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (i < act_items) {
                    const uint32_t e = (uint32_t)(wave * act_items + i) * WAVE + lane;
                    if (e < n_sort) {
                        key[i] = s_ex[mapped ? (uint32_t)s_map[e] : e];
                        sv |= 1u << i;
                    }
                }
            }
            __syncthreads();
            const int passes = (TB + BK_SORT_BITS - 1) / BK_SORT_BITS;
            for (int p = 0; p < passes; p++) {
                const int shift = p * BK_SORT_BITS;
#pragma unroll
                for (int i = 0; i < ITEMS; i++)
                    rd[i] = 0;
                constexpr int IL = 3;  // items ranked together (independent ballot chains)
#pragma unroll
                for (int i0 = 0; i0 < ITEMS; i0 += IL) {
                    if (i0 < act_items) {
                        uint32_t dg[IL];
                        uint64_t peers[IL];
                        bool act[IL];
#pragma unroll
                        for (int j = 0; j < IL; j++) {
                            const int i = i0 + j;
                            act[j] = i < ITEMS && ((sv >> i) & 1u);
                            dg[j] = act[j] ? vdigit(key[i], shift, BK_SORT_BITS, vbase) : 0u;
                            peers[j] = __ballot(act[j]);
                        }
#pragma unroll
                        for (int b = 0; b < BK_SORT_BITS; b++) {
#pragma unroll
                            for (int j = 0; j < IL; j++) {
                                const bool bit = (dg[j] >> b) & 1u;
                                const uint64_t m = __ballot(bit);
                                peers[j] &= bit ? m : ~m;
                            }
                        }
#pragma unroll
                        for (int j = 0; j < IL; j++) {
                            const int i = i0 + j;
                            if (i < ITEMS) {
                                const uint32_t below = __popcll(peers[j] & lt);
                                const uint32_t prior = s_cnt[wave][dg[j]];
                                if (act[j] && below == 0)
                                    s_cnt[wave][dg[j]] = (uint16_t)(prior + (uint32_t)__popcll(peers[j]));
                                rd[i] = ((prior + below) << BK_SORT_BITS) | dg[j];
                            }
                        }
                    }
                }
                __syncthreads();
                // bin `tid`: total over waves; exclusive prefix over bins by a
                // wave scan plus the totals of the waves before
                uint32_t c[BK_WAVES];
                uint32_t tot = 0;
#pragma unroll
                for (int w = 0; w < BK_WAVES; w++) {
                    c[w] = s_cnt[w][tid];
                    tot += c[w];
                }
                const uint32_t inc = wave_inclusive_sum(tot);
                if (lane == WAVE - 1)
                    s_w[0][wave] = inc;
                __syncthreads();
                uint32_t r = inc - tot;
#pragma unroll
                for (int w = 0; w < BK_WAVES; w++)
                    r += w < wave ? s_w[0][w] : 0u;
#pragma unroll
                for (int w = 0; w < BK_WAVES; w++) {
                    s_cnt[w][tid] = (uint16_t)r;
                    r += c[w];
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < ITEMS; i++) {
                    if (i < act_items && ((sv >> i) & 1u)) {
                        const uint32_t dst = s_cnt[wave][rd[i] & (BK_BINS - 1)] + (rd[i] >> BK_SORT_BITS);
                        s_ex[mapped ? (uint32_t)s_map[dst] : dst] = key[i];
                    }
                }
                __syncthreads();
                // counters are free again: clear them for the next pass while
                // reloading the keys wave-striped
#pragma unroll
                for (int w = 0; w < BK_WAVES; w++)
                    s_cnt[w][tid] = 0;
                if (p + 1 < passes) {
                    sv = 0;
#pragma unroll
                    for (int i = 0; i < ITEMS; i++) {
                        if (i < act_items) {
                            const uint32_t e = (uint32_t)(wave * act_items + i) * WAVE + lane;
                            if (e < n_sort) {
                                key[i] = s_ex[mapped ? (uint32_t)s_map[e] : e];
                                sv |= 1u << i;
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }

        // the next group's keys are requested now (the sorted keys are in
        // s_ex), so that their latency overlaps the run-length pass, the
        // record writes and the bookkeeping below
        uint32_t n_next = 0;
        uint64_t p_next = 0;
        if (g + 1 < n_grp) {
            p_next = a.bucket_starts[nb0];
            n_next = a.bucket_starts[nb1 + 1] - (uint32_t)p_next;
        }
        if (ngp.y) {
            __syncthreads();  // the piece table of the next group is complete
            piece_load(ngp, n_next, tid);
        } else {
            load_group(p_next, n_next, tid);
        }
        // ---- run-length compaction of s_ex[0, n_surv) ----
        // positions in (wave, item, lane) order with n_it items per wave.  A
        // run's count is its tail position minus its head position plus one;
        // the head of a tail is the last head at or before it, found from the
        // head ballots of this wave (and, for the first run of a wave, the
        // last head of the waves before).
        // (n_it equals n_ch; passed through an empty asm so that the compiler
        // does not keep the detection loop's per-item masks alive until here)
        int n_it = (int)((n_surv + BK_THREADS - 1) / BK_THREADS);
        asm volatile("" : "+s"(n_it));
        if (tid == 0) {
            s_ex[-1] = sentinel<K>();
            s_ex[n_surv] = sentinel<K>();
        }
        __syncthreads();
        uint32_t rh = 0, rt = 0;  // bit i: item i is a run head / a run tail
        uint32_t last = 0;        // 1 + position of this wave's last head (0: none)
        uint32_t nh = 0;          // heads (runs) in this wave, wave-uniform
        // items in pairs, each pair's reads issued together; positions past
        // n_surv read in-bounds slots (below CAP + 1) and count as nothing
#pragma unroll
        for (int i0 = 0; i0 < ITEMS; i0 += 2) {
            if (i0 < n_it) {
                K x[2], y[2], z[2];
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const uint32_t e = (uint32_t)(wave * n_it + i0 + j) * WAVE + lane;
                    if (i0 + j < ITEMS) {
                        x[j] = s_ex[e];
                        y[j] = s_ex[(int)e - 1];
                        z[j] = s_ex[e + 1];
                    }
                }
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const int i = i0 + j;
                    if (i < ITEMS) {
                        const uint32_t base = (uint32_t)(wave * n_it + i) * WAVE;
                        const bool in = i < n_it && base + lane < n_surv;
                        const bool h = in && y[j] != x[j], t = in && z[j] != x[j];
                        rh |= (uint32_t)h << i;
                        rt |= (uint32_t)t << i;
                        const uint64_t hb = __ballot(h);
                        nh += wave_count(hb);
                        if (hb)
                            last = base + 64u - (uint32_t)__clzll(hb);
                    }
                }
            }
        }
        if (lane == 0)
            s_w[1][wave] = last;
        __syncthreads();
        uint32_t carry = 0;  // position of the last head before the current item
#pragma unroll
        for (int w = 0; w < BK_WAVES; w++) {
            const uint32_t l = s_w[1][w];
            if (w < wave && l)
                carry = l - 1;
        }
        uint32_t cnt[ITEMS];
        uint32_t below = 0;  // runs of 2 .. c - 1 keys ending in this wave, wave-uniform
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            cnt[i] = 0;
            if (i < n_it) {
                const uint32_t base = (uint32_t)(wave * n_it + i) * WAVE;
                const uint64_t hb = __ballot((rh >> i) & 1u);
                const uint64_t upto = hb & (lt | (1ull << lane));  // heads at lanes <= this one
                const uint32_t hp = upto ? base + 63u - (uint32_t)__clzll(upto) : carry;
                if ((rt >> i) & 1u)
                    cnt[i] = base + lane - hp + 1;
                if (hb)
                    carry = base + 63u - (uint32_t)__clzll(hb);
                if (c > 2)
                    below += wave_count(__ballot(cnt[i] >= 2 && cnt[i] < c));
            }
        }
        // the runs ending in this wave (one per tail), those of one key (a
        // head and a tail at once) and the kept ones
        const uint32_t tw = wave_inclusive_sum((uint32_t)__popc(rt) | ((uint32_t)__popc(rh & rt) << 16));
        const uint32_t tt = (uint32_t)__builtin_amdgcn_readlane((int)tw, WAVE - 1);
        const uint32_t single = tt >> 16;
        const uint32_t nk = (tt & 0xFFFFu) - below - (c >= 2 ? single : 0u);
        if (lane == 0)
            s_w[0][wave] = nk;
        __syncthreads();
        uint32_t kbase = 0, n_kept = 0;
        for (int w = 0; w < BK_WAVES; w++) {
            kbase += w < wave ? s_w[0][w] : 0;
            n_kept += s_w[0][w];
        }
        uint32_t *gcnt = a.gap_counts + pos;
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            if (i < n_it) {
                const bool keep = cnt[i] >= c;
                const uint64_t kb = __ballot(keep);
                if (keep) {
                    const uint32_t o = kbase + (uint32_t)__popcll(kb & lt);
                    gap_keys[pos + o] = s_ex[(uint32_t)(wave * n_it + i) * WAVE + lane];
                    gcnt[o] = cnt[i];
                }
                kbase += wave_count(kb);
            }
        }
        if (lane == 0) {
            s_acc[wave][0] += single;
            s_acc[wave][1] += below;
            s_acc[wave][2] += nh;
        }
        if (tid == 0) {
            // the group's records are filed under its first bucket
            a.rec_start[bucket0 + d0] = (uint32_t)pos;
            a.rec_nout[bucket0 + d0] = n_kept;
            s_tot[0] += n_surv;
        }
        pos = p_next;
        n_sb = n_next;
        b0 = nb0;
        b1 = nb1;
        __syncthreads();  // shared buffers are reused by the next group
    }
    }
    // statistics of the last library of this workgroup
    __syncthreads();
    if (tid0 == 0)
        flush_stats(jl);
}

// ---- fallback: oversized buckets, all at once, with global-memory kernels --
// Entry i of the table (buckets in key order): bucket d, first key start,
// ns keys, wpre = windows of the entries before, fpre = filter blocks of the
// entries before, nb = filter blocks.  Every bucket keeps its own filter of
// nb blocks (the same rule as in LDS); the survivors of all of them are
// sorted together -- buckets partition the key space in order -- compacted,
// and each bucket's records are copied to its own slot.

// Entry holding window g: the largest i with e[i].wpre <= g.
__device__ __forceinline__ uint32_t fb_entry_of(const FbEntry *__restrict__ e, uint32_t n, uint64_t g) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (e[mid].wpre <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Keys of oversized bucket ent[blockIdx.x] to dst + its first index: one
// range, or in a tiled layout one piece per tile of its segment.
template <typename K>
__global__ __launch_bounds__(256) void fb_gather(const K *__restrict__ src, K *__restrict__ dst,
                                                 const FbEntry *__restrict__ ent, KeyLayout lay, uint32_t seg0,
                                                 int D2) {
    const FbEntry e = ent[blockIdx.x];
    K *const out = dst + e.start;
    if (!lay.tiled || D2 == 0) {
        for (uint32_t i = threadIdx.x; i < e.ns; i += 256)
            out[i] = src[(uint64_t)e.start + i];
        return;
    }
    const uint32_t sg = seg0 + (e.d >> D2), d2 = e.d & ((1u << D2) - 1u);
    const uint32_t t0 = lay.tt[sg], nt = lay.tt[sg + 1] - t0;
    const uint16_t *const col = lay.px + (uint64_t)t0 * lay.pw;
    uint64_t at = lay.seg[sg];
    uint32_t o = 0;
    for (uint32_t i = 0; i < nt; i++, at += lay.tile_keys) {
        const uint32_t lo = col[(uint64_t)d2 * nt + i], hi = col[(uint64_t)(d2 + 1) * nt + i];
        for (uint32_t i = threadIdx.x; i < hi - lo; i += 256)
            out[o + i] = src[at + lo + i];
        o += hi - lo;
    }
}

template <typename K>
__global__ __launch_bounds__(256) void fb_screen(const K *__restrict__ keys, const FbEntry *__restrict__ ent,
                                                 uint32_t n_ent, uint64_t n, const uint64_t *__restrict__ table,
                                                 uint32_t table_bits, uint64_t *__restrict__ filter) {
    const uint32_t tmask = (1u << table_bits) - 1u;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += stride) {
        const FbEntry e = ent[fb_entry_of(ent, n_ent, g)];
        const uint64_t h = key_hash(keys[e.start + (g - e.wpre)]);
        uint64_t *b = filter + ((uint64_t)e.fpre + __umul64hi(h, (uint64_t)e.nb)) * 8;
        for (int w = 0; w < 4; w++) {
            const uint64_t m = table[(h >> (w * table_bits)) & tmask];
            if ((b[4 + w] & m) == m)
                continue;  // already in the second plane: the atomics would change nothing
            const uint64_t old = __hip_atomic_fetch_or(b + w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (old & m)
                __hip_atomic_fetch_or(b + 4 + w, old & m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <typename K>
__global__ __launch_bounds__(256) void fb_collect(const K *__restrict__ keys, const FbEntry *__restrict__ ent,
                                                  uint32_t n_ent, uint64_t n, const uint64_t *__restrict__ table,
                                                  uint32_t table_bits, const uint64_t *__restrict__ filter, int screen,
                                                  K *__restrict__ out, unsigned long long *__restrict__ n_out) {
    constexpr int FB_BUF = 1024;
    __shared__ K s_buf[FB_BUF];
    __shared__ uint32_t s_wc[256 / WAVE];
    __shared__ uint32_t s_n;
    __shared__ unsigned long long s_base;
    BlockAppender<K, 256, FB_BUF> app{s_buf, s_wc, &s_n, &s_base, out, n, n_out};
    app.init();
    const uint32_t tmask = (1u << table_bits) - 1u;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // every thread of a block runs the same number of iterations
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const uint64_t g = base + threadIdx.x;
        bool keep = false;
        K key{};
        if (g < n) {
            const FbEntry e = ent[fb_entry_of(ent, n_ent, g)];
            key = keys[e.start + (g - e.wpre)];
            keep = true;
            if (screen) {
                const uint64_t h = key_hash(key);
                const uint64_t *b = filter + ((uint64_t)e.fpre + __umul64hi(h, (uint64_t)e.nb)) * 8 + 4;
                for (int w = 0; w < 4; w++) {
                    const uint64_t m = table[(h >> (w * table_bits)) & tmask];
                    keep &= (b[w] & m) == m;
                }
            }
        }
        app.push(keep, key);
    }
    app.finish();
}

// One block per entry: the records of bucket d (a contiguous range of the
// sorted records) go to the bucket's slot in gap_keys / gap_counts.
template <typename K>
__global__ __launch_bounds__(256) void fb_distribute(const K *__restrict__ rec_keys, const uint32_t *__restrict__ rec_counts,
                                                     const DevCounters *__restrict__ c, const FbEntry *__restrict__ ent,
                                                     int k, int D, uint32_t bucket0, K *__restrict__ gap_keys,
                                                     uint32_t *__restrict__ gap_counts, uint32_t *__restrict__ rec_nout) {
    __shared__ uint64_t s_r[2];
    const FbEntry e = ent[blockIdx.x];
    const uint64_t n = c->n_out;
    if (threadIdx.x < 2) {
        // first record with bucket >= d (+ threadIdx.x)
        const uint32_t want = e.d + threadIdx.x;
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (bucket_of(rec_keys[mid], k, D) < want)
                lo = mid + 1;
            else
                hi = mid;
        }
        s_r[threadIdx.x] = lo;
    }
    __syncthreads();
    const uint64_t r0 = s_r[0], m = s_r[1] - r0;
    for (uint64_t i = threadIdx.x; i < m; i += blockDim.x) {
        gap_keys[e.start + i] = rec_keys[r0 + i];
        gap_counts[e.start + i] = rec_counts[r0 + i];
    }
    if (threadIdx.x == 0)
        rec_nout[bucket0 + e.d] = (uint32_t)m;
}

// Folds the fallback's compaction counters into the library's statistics.
__global__ void fb_fold(const DevCounters *__restrict__ c, unsigned long long *__restrict__ stats) {
    stats[0] += c->n_collected;
    stats[1] += c->n_runs;
    stats[2] += c->n_single;
    stats[3] += c->n_below;
}

// ---- gather: records of every bucket, in bucket order, into place ---------

// One wave copies n records from src to dst, four per lane in flight: every
// load of a round is issued before its stores.
template <typename R>
__device__ __forceinline__ void gather_records(const R *__restrict__ gk, const uint32_t *__restrict__ gc, uint64_t src,
                                               uint64_t dst, uint32_t n, R *__restrict__ ok,
                                               uint32_t *__restrict__ oc) {
    constexpr int U = 4;
    const uint32_t lane = lane_id();
    for (uint32_t i0 = 0; i0 < n; i0 += U * WAVE) {
        R kv[U];
        uint32_t cv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t i = i0 + (uint32_t)u * WAVE + lane;
            if (i < n) {
                kv[u] = gk[src + i];
                cv[u] = gc[src + i];
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t i = i0 + (uint32_t)u * WAVE + lane;
            if (i < n) {
                ok[dst + i] = kv[u];
                oc[dst + i] = cv[u];
            }
        }
    }
}

__global__ __launch_bounds__(256) void gather_kernel(const uint32_t *__restrict__ rec_start,
                                                     const uint32_t *__restrict__ rec_nout,
                                                     const uint32_t *__restrict__ rec_off, uint64_t n_buckets,
                                                     const uint64_t *__restrict__ gap_keys,
                                                     const uint32_t *__restrict__ gap_counts, int key_words,
                                                     uint64_t *__restrict__ out_keys, uint32_t *__restrict__ out_counts) {
    const uint64_t b = (uint64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (b >= n_buckets)
        return;
    const uint32_t n = rec_nout[b];
    if (!n)
        return;
    const uint64_t src = rec_start[b], dst = rec_off[b];
    if (key_words == 1)
        gather_records(gap_keys, gap_counts, src, dst, n, out_keys, out_counts);
    else
        gather_records(reinterpret_cast<const ulonglong2 *>(gap_keys), gap_counts, src, dst, n,
                       reinterpret_cast<ulonglong2 *>(out_keys), out_counts);
}

// Per-library counters; one thread per library.
__global__ __launch_bounds__(256) void lib_stats_kernel(const LibDesc *__restrict__ libs, uint32_t n_libs,
                                                        const uint32_t *__restrict__ lib_keys,
                                                        const uint32_t *__restrict__ rec_off,
                                                        const uint32_t *__restrict__ rec_total,
                                                        const unsigned long long *__restrict__ stats,
                                                        DevCounters *__restrict__ ctr, uint32_t *__restrict__ out_first) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_libs)
        return;
    const uint32_t first = rec_off[libs[j].bucket0];
    const uint32_t next = j + 1 < n_libs ? rec_off[libs[j + 1].bucket0] : *rec_total;
    DevCounters c{};
    c.n_windows = lib_keys[j + 1] - lib_keys[j];
    c.n_out = next - first;
    c.n_collected = stats[4 * (uint64_t)j + 0];
    c.n_runs = stats[4 * (uint64_t)j + 1];
    c.n_single = stats[4 * (uint64_t)j + 2];
    c.n_below = stats[4 * (uint64_t)j + 3];
    ctr[j] = c;
    out_first[j] = first;
}

// The schedule's groups (one thread per chunk of chunk_buckets bucket ids):
// greedy, in key order, a group takes whole non-empty buckets of one library
// while its keys fit the registers (CAP), its filters the exchange buffer
// (FMAX blocks) and its bucket ids span at most BK_RMAX.  A bucket too large
// on its own goes to the fallback list instead (its records are filed under
// it by the fallback kernels).  Groups never cross a chunk boundary.  In a
// tiled layout, a group of a library with a second pass stays in one
// segment and records where its pieces are (grp_piece); the buckets of a
// segment with more than BK_TILES_MAX tiles all go to the fallback list.
template <typename K, int TILE>
__global__ __launch_bounds__(256) void plan_groups(BucketArgs a) {
    constexpr uint32_t CAP = BK_THREADS * BkItems<K, TILE>::value;
    constexpr uint32_t FMAX = (uint32_t)((CAP + 2) * sizeof(K) / 64);
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chunks)
        return;
    const uint32_t b_lo = c * a.chunk_buckets;
    const uint32_t b_hi = min(b_lo + a.chunk_buckets, a.n_buckets);
    const uint32_t *bs = a.bucket_starts;
    uint32_t j = library_of_bucket(a, b_lo);
    uint32_t ng = 0;
    for (uint32_t b = b_lo; b < b_hi;) {
        while (j + 1 < a.n_libs && a.libs[j + 1].bucket0 <= b)
            j++;
        const LibDesc &L = a.libs[j];
        const uint32_t lib_end = j + 1 < a.n_libs ? a.libs[j + 1].bucket0 : a.n_buckets;
        const bool screen = L.c >= 2;
        const uint32_t s0 = bs[b], ns = bs[b + 1] - s0;
        if (ns == 0) {
            b++;
            continue;
        }
        // tiled: the bucket's segment, its tiles and the segment's last bucket
        const bool tiled = a.layout.tiled && L.D2 > 0;
        uint32_t seg_end = lib_end, t0 = 0, nt = 0, sgs = 0;
        if (tiled) {
            const uint32_t sg = L.seg0 + ((b - L.bucket0) >> L.D2);
            seg_end = L.bucket0 + ((sg - L.seg0 + 1) << L.D2);
            t0 = a.layout.tt[sg];
            nt = a.layout.tt[sg + 1] - t0;
            sgs = a.layout.seg[sg];
        }
        const uint32_t nb = screen ? max(1u, (a.beta * ns + 255) / 256) : 0u;
        if (ns > CAP || nb > FMAX || nt > BK_TILES_MAX) {
            const uint32_t slot = atomicAdd(a.fb_count, 1u);
            if (slot < a.fb_cap) {
                a.fb_list[3 * slot + 0] = b;
                a.fb_list[3 * slot + 1] = s0;
                a.fb_list[3 * slot + 2] = ns;
            }
            a.rec_start[b] = s0;
            b++;
            continue;
        }
        uint32_t n_keys = ns, n_blocks = nb, last = b;
        const uint32_t e_max = min(min(min(b_hi, lib_end), seg_end), b + (uint32_t)BK_RMAX);
        for (uint32_t e = b + 1; e < e_max; e++) {
            const uint32_t ne = bs[e + 1] - bs[e];
            if (ne == 0)
                continue;
            const uint32_t nbe = screen ? max(1u, (a.beta * ne + 255) / 256) : 0u;
            if (n_keys + ne > CAP || n_blocks + nbe > FMAX)
                break;
            n_keys += ne;
            n_blocks += nbe;
            last = e;
        }
        a.grp_first[b_lo + ng] = b;
        a.grp_last[b_lo + ng] = last;
        const uint32_t m = (1u << L.D2) - 1u;
        a.grp_piece[b_lo + ng] = make_uint4(t0, nt, sgs, ((b - L.bucket0) & m) | (((last - L.bucket0) & m) << 16));
        ng++;
        b = last + 1;
    }
    a.grp_count[c] = ng;
}

}  // namespace

int bucket_grid() { return device_cu_count() * 2; }

int bucket_capacity(int key_words, int tile) {
    if (key_words == 2)
        return BK_THREADS * (tile ? BkItems<Key2, 1>::value : BkItems<Key2, 0>::value);
    return BK_THREADS * (tile ? BkItems<uint64_t, 1>::value : BkItems<uint64_t, 0>::value);
}

template <typename K, int TILE>
hipError_t launch_bucket_tile(const BucketArgs &a, int grid, hipStream_t stream) {
    // the groups of every chunk (grp_* and *a.chunk_next, zero on entry,
    // belong to the caller's workspace)
    const unsigned cg = (unsigned)((a.n_chunks + 255) / 256);
    plan_groups<K, TILE><<<dim3(cg), dim3(256), 0, stream>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (a.table_bits == BK_TABLE_BITS)
        bucket_kernel<K, BK_TABLE_BITS, TILE><<<dim3(grid), dim3(BK_THREADS), 0, stream>>>(a);
    else
        bucket_kernel<K, 0, TILE><<<dim3(grid), dim3(BK_THREADS), 0, stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_bucket(const BucketArgs &a, int key_words, int grid, hipStream_t stream) {
    if (key_words == 2)
        return a.tile ? launch_bucket_tile<Key2, 1>(a, grid, stream) : launch_bucket_tile<Key2, 0>(a, grid, stream);
    return a.tile ? launch_bucket_tile<uint64_t, 1>(a, grid, stream) : launch_bucket_tile<uint64_t, 0>(a, grid, stream);
}

hipError_t launch_fb_gather(const void *src, void *dst, const FbEntry *ent, uint32_t n_ent, int key_words,
                            const KeyLayout &layout, uint32_t seg0, int D2, hipStream_t stream) {
    if (!n_ent)
        return hipSuccess;
    if (key_words == 2)
        fb_gather<Key2><<<n_ent, 256, 0, stream>>>(static_cast<const Key2 *>(src), static_cast<Key2 *>(dst), ent,
                                                   layout, seg0, D2);
    else
        fb_gather<uint64_t><<<n_ent, 256, 0, stream>>>(static_cast<const uint64_t *>(src),
                                                       static_cast<uint64_t *>(dst), ent, layout, seg0, D2);
    return hipGetLastError();
}

hipError_t launch_fb_screen(const void *keys, const FbEntry *ent, uint32_t n_ent, uint64_t n, int key_words,
                            const uint64_t *table, uint32_t table_bits, uint64_t *filter, hipStream_t stream) {
    const unsigned g = (unsigned)std::min<uint64_t>(ceil_div(n ? n : 1, 256), (uint64_t)device_cu_count() * 8);
    if (key_words == 2)
        fb_screen<Key2><<<g, 256, 0, stream>>>(static_cast<const Key2 *>(keys), ent, n_ent, n, table, table_bits,
                                               filter);
    else
        fb_screen<uint64_t><<<g, 256, 0, stream>>>(static_cast<const uint64_t *>(keys), ent, n_ent, n, table,
                                                   table_bits, filter);
    return hipGetLastError();
}

hipError_t launch_fb_collect(const void *keys, const FbEntry *ent, uint32_t n_ent, uint64_t n, int key_words,
                             const uint64_t *table, uint32_t table_bits, const uint64_t *filter, bool screen,
                             void *out, unsigned long long *n_out, hipStream_t stream) {
    const unsigned g = (unsigned)std::min<uint64_t>(ceil_div(n ? n : 1, 256), (uint64_t)device_cu_count() * 8);
    if (key_words == 2)
        fb_collect<Key2><<<g, 256, 0, stream>>>(static_cast<const Key2 *>(keys), ent, n_ent, n, table, table_bits,
                                                filter, screen, static_cast<Key2 *>(out), n_out);
    else
        fb_collect<uint64_t><<<g, 256, 0, stream>>>(static_cast<const uint64_t *>(keys), ent, n_ent, n, table,
                                                    table_bits, filter, screen, static_cast<uint64_t *>(out), n_out);
    return hipGetLastError();
}

hipError_t launch_fb_distribute(const void *rec_keys, const uint32_t *rec_counts, const DevCounters *c,
                                const FbEntry *ent, uint32_t n_ent, int key_words, int k, int D, uint32_t bucket0,
                                void *gap_keys, uint32_t *gap_counts, uint32_t *rec_nout,
                                unsigned long long *lib_stats, hipStream_t stream) {
    if (n_ent) {
        if (key_words == 2)
            fb_distribute<Key2><<<n_ent, 256, 0, stream>>>(static_cast<const Key2 *>(rec_keys), rec_counts, c, ent, k,
                                                           D, bucket0, static_cast<Key2 *>(gap_keys), gap_counts,
                                                           rec_nout);
        else
            fb_distribute<uint64_t><<<n_ent, 256, 0, stream>>>(static_cast<const uint64_t *>(rec_keys), rec_counts, c,
                                                               ent, k, D, bucket0, static_cast<uint64_t *>(gap_keys),
                                                               gap_counts, rec_nout);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    fb_fold<<<1, 1, 0, stream>>>(c, lib_stats);
    return hipGetLastError();
}

hipError_t launch_gather(const uint32_t *rec_start, const uint32_t *rec_nout, const uint32_t *rec_off,
                         uint64_t n_buckets, const uint64_t *gap_keys, const uint32_t *gap_counts, int key_words,
                         uint64_t *out_keys, uint32_t *out_counts, hipStream_t stream) {
    const uint64_t per_block = 256 / WAVE;
    const uint64_t g = ceil_div(n_buckets, per_block);
    if (!g)
        return hipSuccess;
    gather_kernel<<<dim3((unsigned)g), dim3(256), 0, stream>>>(rec_start, rec_nout, rec_off, n_buckets, gap_keys,
                                                               gap_counts, key_words, out_keys, out_counts);
    return hipGetLastError();
}

hipError_t launch_lib_stats(const LibDesc *libs, uint32_t n_libs, const uint32_t *lib_keys, const uint32_t *rec_off,
                            const uint32_t *rec_total, const unsigned long long *lib_stats, DevCounters *ctr,
                            uint32_t *out_first, hipStream_t stream) {
    if (!n_libs)
        return hipSuccess;
    lib_stats_kernel<<<dim3((unsigned)ceil_div(n_libs, 256)), dim3(256), 0, stream>>>(
        libs, n_libs, lib_keys, rec_off, rec_total, lib_stats, ctr, out_first);
    return hipGetLastError();
}

}  // namespace tk
