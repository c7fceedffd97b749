// Partitioning of the window keys by (library, top D bits), D <= 20 -- the
// GPU counterpart of routing every k-mer to the consumer that owns its filter
// (paper §2.1, parallelization): afterwards the keys of every bucket (keys of
// one library sharing their top D bits) can be found without a search, and
// libraries and buckets follow each other in key order, so per-bucket
// sort-and-compact results concatenate into each library's sorted answer.
//
// Pass 1 extracts the canonical keys straight from the packed reads (§2.1,
// k-mer extraction) and orders them by (library, top D1 bits), D1 = D - 10
// for D > 10 and D otherwise: the "segments", each one contiguous range.  Pass 2 (run when some library
// has D2 = D - D1 > 0) cuts every segment into tiles of PtItems * PT_THREADS
// keys and orders each tile by the next D2 bits in place, recording for
// every tile the first position of every digit (a prefix table of 16-bit
// entries).  A bucket is then digit d of its segment: one piece per tile of
// the segment, found from the prefix tables, and its size is the sum of its
// pieces.  Ordering tiles rather than whole segments spares a histogram pass
// over all keys and turns the second pass's writes into one sequential
// stream.  The order of keys inside a bucket is not kept -- the bucket
// kernel sorts each bucket -- so both passes rank keys with LDS atomic
// counters instead of a stable ranking.
//
// Pass-1 work unit: a chunk of up to PT_CH tiles, one workgroup each; chunks
// never straddle a library.  hist counts the chunk's digits; the counts are
// laid out (library, digit, chunk) so that one exclusive scan gives every
// (chunk, digit) its write position.  scatter, per tile: rank every window
// within its digit (LDS atomics), stage the tile's window positions in LDS in
// digit order, rebuild each key from the tile's packed words as its digit's
// run is written contiguously at its cursor.  Pass 2 takes chunks of up to
// PT_CH / PT2_ROUNDS tiles of one segment and writes every tile back in digit
// order.
#include "device.hpp"
#include "internal.hpp"

namespace tk {
namespace {

constexpr int PT_THREADS = 1024;
constexpr int PT_WAVES = PT_THREADS / WAVE;
constexpr int PT_MAX_BITS = 10;
constexpr int PT_MAX_BINS = 1 << PT_MAX_BITS;
constexpr int PT_BPT = PT_MAX_BINS / PT_THREADS;  // digit bins per thread
constexpr int PT_CH = 8;                          // tiles per chunk
constexpr int SEG_THREADS = 256;
static_assert(PT_BPT * PT_THREADS == PT_MAX_BINS, "bins spread evenly over the threads");

template <typename K>
struct PtItems;
template <>
struct PtItems<uint64_t> {
    static constexpr int value = 16;  // 16384 keys per tile (128 KB of LDS)
};
template <>
struct PtItems<Key2> {
    static constexpr int value = 8;  // 8192 keys per tile (128 KB of LDS)
};

template <typename K>
constexpr uint64_t pt_tile() {
    return (uint64_t)PT_THREADS * PtItems<K>::value;
}
template <typename K>
constexpr uint64_t pt_chunk() {
    return pt_tile<K>() * PT_CH;
}
// Pass-2 tiles hold PT2_ROUNDS pass-1 tiles' worth of keys, staged through
// the same LDS buffer in that many rounds: fewer, larger pieces per bucket.
constexpr int PT2_ROUNDS = 2;
template <typename K>
constexpr uint64_t pt2_tile() {
    return pt_tile<K>() * PT2_ROUNDS;
}
static_assert(PT_CH % PT2_ROUNDS == 0, "a pass-2 chunk holds whole tiles");


// Largest i in [0, n) with at(i) <= v, for a non-decreasing at(); 0 if none.
template <typename F>
__device__ __forceinline__ uint32_t last_le(uint32_t n, uint64_t v, F at) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (at(mid) <= v)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

struct PassArgs {
    const uint64_t *packed;
    const uint32_t *valid;
    const void *keys_in;     // pass 2: the pass-1 output
    const LibDesc *libs;
    uint32_t n_libs;
    const uint32_t *seg;     // pass 2: start of every segment (nseg + 1)
    const uint32_t *cb;      // pass 2: first chunk of every segment (nseg + 1)
    const uint32_t *tt;      // pass 2: first tile of every segment (nseg + 1)
    uint32_t nseg;
    const uint32_t *own;     // pass 1 of a key-range shard: its digits
                             // [own[0], own[1]); nullptr: every digit
    uint64_t cap;            // keys the output can hold
};

// The chunk of this workgroup: elements [c0, c1) (window positions of pass
// 1, below which `lo` masks positions of the previous library; keys of pass
// 2), its count entries hidx + d * hstride, and its digit (shift, bits).
struct Chunk {
    uint64_t c0, c1, lo, hidx;
    uint32_t hstride;
    int shift, bits;
    int k;         // the library's k-mer length
    uint32_t tile;  // pass 2: global index of the chunk's first tile
};

template <typename K, bool FROM_WIN>
__device__ __forceinline__ bool chunk_of(const PassArgs &a, Chunk &ch) {
    const uint32_t b = blockIdx.x;
    if (FROM_WIN) {
        const uint32_t j = last_le(a.n_libs, b, [&](uint32_t i) { return (uint64_t)a.libs[i].cb1; });
        const LibDesc L = a.libs[j];
        if (b < L.cb1 || b >= L.cb1 + L.nch1)
            return false;
        const uint32_t i = b - L.cb1;
        ch.c0 = (L.pos0 & ~31ull) + (uint64_t)i * pt_chunk<K>();
        ch.c1 = min(ch.c0 + pt_chunk<K>(), L.pos1);
        ch.lo = L.pos0;
        ch.hidx = L.h1 + i;
        ch.hstride = L.nch1;
        ch.shift = 2 * L.k - L.D1;
        ch.bits = L.D1;
        ch.k = L.k;
        ch.tile = 0;
        return true;
    }
    if (b >= a.cb[a.nseg])
        return false;
    const uint32_t s = last_le(a.nseg, b, [&](uint32_t i) { return (uint64_t)a.cb[i]; });
    const uint32_t j = last_le(a.n_libs, s, [&](uint32_t i) { return (uint64_t)a.libs[i].seg0; });
    const uint32_t i = b - a.cb[s];
    ch.c0 = a.seg[s] + (uint64_t)i * pt_chunk<K>();
    ch.c1 = min(ch.c0 + pt_chunk<K>(), (uint64_t)a.seg[s + 1]);
    ch.lo = ch.c0;
    ch.hidx = 0;
    ch.hstride = 0;
    ch.shift = 2 * a.libs[j].k - a.libs[j].D;
    ch.bits = a.libs[j].D2;
    ch.k = a.libs[j].k;
    ch.tile = a.tt[s] + i * (PT_CH / PT2_ROUNDS);
    return true;
}

// Pass-1 tiles: pt_tile window positions starting at a word boundary;
// thread t takes ITEMS consecutive windows of one packed word, and positions
// outside [lo, t1) are skipped.  fetch_win issues the loads of one thread's
// packed words and validity bits, so that the next tile's loads can be in
// flight while the current tile is processed.
struct RawWin {
    uint64_t w0, w1, w2;  // packed words w, w - 1, w - 2 (0 before the first)
    uint32_t vword;       // valid[w]
    uint32_t okmask;      // this thread's items inside [lo, t1)
};

template <typename K>
__device__ __forceinline__ RawWin fetch_win(const PassArgs &a, uint64_t t0, uint64_t t1, uint64_t lo) {
    constexpr int ITEMS = PtItems<K>::value;
    constexpr int PER_WORD = 32 / ITEMS;  // threads per packed word
    const int tid = threadIdx.x;
    const uint64_t w = t0 / 32 + (uint64_t)(tid / PER_WORD);
    const uint32_t first = (uint32_t)(tid % PER_WORD) * ITEMS;
    const uint64_t p0 = w * 32 + first;  // position of item 0
    RawWin r{0, 0, 0, 0, 0};
    if (p0 < t1 && p0 + ITEMS > lo) {
        r.w0 = a.packed[w];
        r.w1 = w ? a.packed[w - 1] : 0;
        r.w2 = (std::is_same<K, Key2>::value && w > 1) ? a.packed[w - 2] : 0;
        r.vword = a.valid[w];
        uint32_t ok = ITEMS == 32 ? ~0u : (1u << (ITEMS & 31)) - 1u;
        if (p0 < lo)
            ok &= ~0u << (uint32_t)(lo - p0);  // lo - p0 < ITEMS
        if (p0 + ITEMS > t1)
            ok &= (1u << (uint32_t)(t1 - p0)) - 1u;  // t1 - p0 < ITEMS
        r.okmask = ok;
    }
    return r;
}

// Two-bit codes of the 32 bases ending at base 32w + u (that base in bits
// 1..0), -64 <= u <= 31, from the packed words w, w - 1 and w - 2 held in
// r; bases before word w - 2 read as 0.
__device__ __forceinline__ uint64_t codes_ending_at(const RawWin &r, int u) {
    uint64_t a = r.w0, b = r.w1;
    if (u < 0) {
        a = r.w1;
        b = r.w2;
        u += 32;
    }
    if (u < 0) {
        a = r.w2;
        b = 0;
        u += 32;
    }
    const uint32_t s = 62 - 2 * u;
    return s ? (a >> s) | (b << (64 - s)) : a;
}

// Pass 1: digit counts of every chunk.
template <typename K>
__global__ __launch_bounds__(PT_THREADS) void pt_hist(PassArgs a, uint32_t *__restrict__ hist) {
    constexpr int ITEMS = PtItems<K>::value;
    __shared__ uint32_t s_h[PT_MAX_BINS];
    const int tid = threadIdx.x;
    Chunk ch;
    if (!chunk_of<K, true>(a, ch))
        return;  // uniform over the block
    const uint32_t bins = 1u << ch.bits, mask = bins - 1;
    for (int d = tid; d < PT_MAX_BINS; d += PT_THREADS)
        s_h[d] = 0;
    __syncthreads();
    // the next tile's words are requested before this tile's keys are
    // rolled out and counted
    RawWin cur = ch.c0 < ch.c1 ? fetch_win<K>(a, ch.c0, min(ch.c0 + pt_tile<K>(), ch.c1), ch.lo)
                               : RawWin{0, 0, 0, 0, 0};
    for (uint64_t t0 = ch.c0; t0 < ch.c1; t0 += pt_tile<K>()) {
        const uint64_t tn = t0 + pt_tile<K>();
        RawWin nxt{0, 0, 0, 0, 0};
        if (tn < ch.c1)
            nxt = fetch_win<K>(a, tn, min(tn + pt_tile<K>(), ch.c1), ch.lo);
        if (cur.okmask && ch.k >= 5) {
            // The top bits of the canonical key, the smaller of the
            // forward code and its reverse complement, are the smaller
            // of the two codes' top bits.  So a window's digit (at most
            // 10 bits) needs only its first five bases, forward, and its
            // last five, reverse-complemented: two fields of words
            // assembled once per thread, instead of the whole key.
            constexpr int PER_WORD = 32 / ITEMS;
            const int first = (tid % PER_WORD) * ITEMS;
            const uint32_t ok = (cur.vword >> first) & cur.okmask;
            const uint64_t last5 = ~group_reverse(codes_ending_at(cur, first + ITEMS - 1));
            const uint64_t first5 = codes_ending_at(cur, first + ITEMS + 4 - ch.k);
            const int drop = 10 - ch.bits;
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if ((ok >> i) & 1u) {
                    const uint32_t f = (uint32_t)(first5 >> (2 * (ITEMS - 1 - i))) & 0x3FFu;
                    const uint32_t r = (uint32_t)(last5 >> (56 - 2 * ITEMS + 2 * i)) & 0x3FFu;
                    atomicAdd(&s_h[min(f, r) >> drop], 1u);
                }
            }
        } else if (cur.okmask) {
            // k < 5: each key is counted as it is rolled out
            constexpr int PER_WORD = 32 / ITEMS;
            const uint32_t first = (uint32_t)(tid % PER_WORD) * ITEMS;
            const uint32_t ok = (cur.vword >> first) & cur.okmask;
            typename KeyOf<std::is_same<K, Key2>::value>::Roll rl;
            rl.init(cur.w0, cur.w1, cur.w2, first, ch.k);
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (i)
                    rl.step((uint32_t)(cur.w0 >> (62 - 2 * (first + i))) & 3u);
                if ((ok >> i) & 1u)
                    atomicAdd(&s_h[digit_of(rl.key(), ch.shift, mask)], 1u);
            }
        }
        cur = nxt;
    }
    __syncthreads();
    for (uint32_t d = tid; d < bins; d += PT_THREADS)
        hist[ch.hidx + (uint64_t)d * ch.hstride] = s_h[d];
}

// Pass 1: keys of every chunk to their (library, digit, chunk) places.
// Per tile: every window's digit from its first and last five bases (as in
// pt_hist; k < 5: from the whole key), ranked within its digit by LDS
// atomics; the tile's window positions (2 bytes each, not the 8- or 16-byte
// keys) staged in digit order; then each staged window's key rebuilt from
// the tile's packed words, kept in LDS, and written to its digit's run.
// Staging positions instead of keys keeps the workgroup small enough for
// two to share a CU, so one's loads and barriers overlap the other's work.
template <typename K>
__global__ __launch_bounds__(PT_THREADS) __attribute__((amdgpu_waves_per_eu(8))) void pt_scatter(PassArgs a, const uint32_t *__restrict__ offs,
                                                            K *__restrict__ out) {
    constexpr int ITEMS = PtItems<K>::value;
    constexpr int TILE = PT_THREADS * ITEMS;  // window positions per tile
    constexpr int PER_WORD = 32 / ITEMS;      // threads per packed word
    constexpr int WORDS = TILE / 32;
    constexpr int BACK = std::is_same<K, Key2>::value ? 2 : 1;  // words before the tile a key may reach into
    constexpr uint32_t SPARE = PT_MAX_BINS;   // rank record of a window that is not kept
    static_assert(TILE <= 65536, "positions are 16 bits");
    __shared__ uint32_t s_cnt[PT_MAX_BINS];       // digit counts of the tile
    __shared__ uint32_t s_start[PT_MAX_BINS];     // first slot of every digit
    __shared__ uint32_t s_base[PT_MAX_BINS];      // output position minus slot, per digit
    __shared__ uint32_t s_wt[PT_WAVES];
    __shared__ uint64_t s_words[2][BACK + WORDS];  // the tile's packed words (two tiles in turn)
    __shared__ uint16_t s_idx[TILE];               // window positions in digit order
    const int tid = threadIdx.x;
    const int wave = tid / WAVE;
    const uint32_t lane = lane_id();
    Chunk ch;
    if (!chunk_of<K, true>(a, ch))
        return;  // uniform over the block
    const uint32_t bins = 1u << ch.bits, mask = bins - 1;
    static_assert(PT_BPT == 1, "one digit per thread");
    // a shard keeps the keys of its digits only (one library)
    uint32_t own_lo = 0, own_hi = bins;
    if (a.own) {
        own_lo = a.own[0];
        own_hi = a.own[1];
    }
    // thread t owns digit t: its write position stays in a register
    uint32_t cur = (uint32_t)tid < bins ? offs[ch.hidx + (uint64_t)tid * ch.hstride] : 0u;
    s_cnt[tid] = 0;
    __syncthreads();
    uint32_t par = 0;
    for (uint64_t t0 = ch.c0; t0 < ch.c1; t0 += pt_tile<K>(), par ^= 1u) {
        // (the thread index passes through an empty asm each tile, so that
        // the compiler recomputes the per-lane shifts rather than keeping
        // them across the loop, where they would not fit the registers)
        int tix = tid;
        asm volatile("" : "+v"(tix));
        const int first = (tix % PER_WORD) * ITEMS;  // this thread's first window in its word
        const RawWin r = fetch_win<K>(a, t0, min(t0 + pt_tile<K>(), ch.c1), ch.lo);
        uint64_t *const words = s_words[par];
        // every thread that loaded its word stores it (a window's bases lie in
        // words that hold some window of [lo, t1)); thread 0 also the words
        // before the tile
        if (r.okmask) {
            words[BACK + tix / PER_WORD] = r.w0;
            if (tix == 0) {
                words[BACK - 1] = r.w1;
                if (BACK == 2)
                    words[0] = r.w2;
            }
        }
        // digits, ranked; a window that is not kept (not valid, or outside
        // a shard's digits) takes no counter: one shared spare counter
        // would serialise the atomics of every such window of a wave
        const uint32_t ok = r.okmask ? (r.vword >> first) & r.okmask : 0u;
        uint32_t rd[ITEMS];  // (rank << 11) | digit (SPARE: not kept)
        auto rank = [&](int i, uint32_t dg) __attribute__((always_inline)) {
            const bool keep = ((ok >> i) & 1u) && dg >= own_lo && dg < own_hi;
            rd[i] = SPARE;
            if (keep)
                rd[i] = (atomicAdd(&s_cnt[dg], 1u) << (PT_MAX_BITS + 1)) | dg;
        };
        if (ch.k >= 5) {
            // the canonical key's top 10 bits are the smaller of the forward
            // code's first five bases and the reverse complement's
            const uint64_t last5 = ~group_reverse(codes_ending_at(r, first + ITEMS - 1));
            const uint64_t first5 = codes_ending_at(r, first + ITEMS + 4 - ch.k);
            const int drop = 10 - ch.bits;
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                const uint32_t f = (uint32_t)(first5 >> (2 * (ITEMS - 1 - i))) & 0x3FFu;
                const uint32_t b = (uint32_t)(last5 >> (56 - 2 * ITEMS + 2 * i)) & 0x3FFu;
                rank(i, min(f, b) >> drop);
            }
        } else {
            typename KeyOf<std::is_same<K, Key2>::value>::Roll rl;
            rl.init(r.w0, r.w1, r.w2, (uint32_t)first, ch.k);
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (i)
                    rl.step((uint32_t)(r.w0 >> (62 - 2 * (first + i))) & 3u);
                rank(i, digit_of(rl.key(), ch.shift, mask));
            }
        }
        __syncthreads();
        // starts of the digits in the tile
        const uint32_t c = s_cnt[tid];
        const uint32_t inc = wave_inclusive_sum(c);
        if (lane == WAVE - 1)
            s_wt[wave] = inc;
        s_cnt[tid] = 0;  // read by its owner only until the next tile's atomics
        __syncthreads();
        uint32_t before = 0, n_tile = 0;
#pragma unroll
        for (int w = 0; w < PT_WAVES; w++) {
            const uint32_t t = s_wt[w];
            before += w < wave ? t : 0u;
            n_tile += t;
        }
        const uint32_t start = before + inc - c;
        s_start[tid] = start;
        s_base[tid] = cur - start;
        cur += c;
        __syncthreads();
        const uint32_t pos0 = (uint32_t)(tix / PER_WORD) * 32 + (uint32_t)first;
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint32_t d = rd[i] & (2 * PT_MAX_BINS - 1);
            if (d != SPARE)
                s_idx[s_start[d] + (rd[i] >> (PT_MAX_BITS + 1))] = (uint16_t)(pos0 + i);
        }
        __syncthreads();
        // each digit's run goes to its cursor; consecutive threads write
        // consecutive positions of a run
        for (uint32_t j = tid; j < n_tile; j += PT_THREADS) {
            const uint32_t p = s_idx[j];
            const uint32_t w = BACK + p / 32, u = p % 32;
            K x;
            if constexpr (std::is_same<K, Key2>::value)
                x = window_key2(words[w], words[w - 1], words[w - 2], u, ch.k);
            else
                x = window_key1(words[w], words[w - 1], u, ch.k);
            const uint64_t o = (uint32_t)(s_base[digit_of(x, ch.shift, mask)] + j);
            if (o < a.cap)  // holds whenever the counts match the keys
                out[o] = x;
        }
    }
}

// Pass 2: every tile of a segment (up to PT_CH / PT2_ROUNDS per workgroup)
// ordered by its library's next D2 bits in place; pt[t * pw + d] receives
// the first position of digit d in tile t, entries past the last digit the
// tile's size.  A tile holds at most 2^15 keys, so the entries fit 16 bits.
// The keys stay in registers while the tile's digit order is staged in LDS
// and written out, PtItems keys per thread and round.
template <typename K>
__global__ __launch_bounds__(PT_THREADS) void pt_tiles(PassArgs a, uint16_t *__restrict__ pt, uint32_t pw,
                                                       K *__restrict__ out) {
    constexpr int STAGE = PT_THREADS * PtItems<K>::value;  // keys staged per round
    constexpr int ITEMS = PtItems<K>::value * PT2_ROUNDS;
    constexpr int TILE = PT_THREADS * ITEMS;
    static_assert(TILE <= 65535, "prefix entries are 16 bits");
    static_assert(TILE < (1 << (32 - PT_MAX_BITS)), "(rank, digit) fits a word");
    __shared__ uint32_t s_cnt[PT_MAX_BINS];  // digit counts of the tile, then their starts
    __shared__ uint32_t s_wt[PT_WAVES];
    __shared__ K s_stage[STAGE];
    const int tid = threadIdx.x;
    const int wave = tid / WAVE;
    const uint32_t lane = lane_id();
    Chunk ch;
    if (!chunk_of<K, false>(a, ch))
        return;  // uniform over the block
    const uint32_t bins = 1u << ch.bits, mask = bins - 1;
    const uint32_t d0 = (uint32_t)tid * PT_BPT;
    const K *__restrict__ in = static_cast<const K *>(a.keys_in);
#pragma unroll
    for (int j = 0; j < PT_BPT; j++)
        s_cnt[d0 + j] = 0;
    __syncthreads();
    uint32_t tile = ch.tile;
    for (uint64_t t0 = ch.c0; t0 < ch.c1; t0 += TILE, tile++) {
        const uint32_t n_tile = (uint32_t)min((uint64_t)TILE, ch.c1 - t0);
        // all of the tile's loads first, then the ranking (the LDS atomics
        // would otherwise hold each load back)
        K key[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const uint32_t e = (uint32_t)i * PT_THREADS + tid;
            key[i] = K{};
            if (e < n_tile)
                key[i] = in[t0 + e];
        }
        uint32_t rd[ITEMS];  // (rank << 10) | digit, then the slot; ~0 for no key
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            rd[i] = ~0u;
            if ((uint32_t)i * PT_THREADS + tid < n_tile) {
                const uint32_t d = digit_of(key[i], ch.shift, mask);
                rd[i] = (atomicAdd(&s_cnt[d], 1u) << PT_MAX_BITS) | d;
            }
        }
        __syncthreads();
        // starts of the digits in the tile, also its prefix table
        uint32_t c[PT_BPT];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < PT_BPT; j++) {
            c[j] = s_cnt[d0 + j];
            sum += c[j];
        }
        const uint32_t inc = wave_inclusive_sum(sum);
        if (lane == WAVE - 1)
            s_wt[wave] = inc;
        __syncthreads();
        uint32_t before = 0;
#pragma unroll
        for (int w = 0; w < PT_WAVES; w++)
            before += w < wave ? s_wt[w] : 0u;
        uint32_t run = before + inc - sum;
        uint16_t *const row = pt + (uint64_t)tile * pw;
#pragma unroll
        for (int j = 0; j < PT_BPT; j++) {
            s_cnt[d0 + j] = run;
            if (d0 + j < pw)
                row[d0 + j] = (uint16_t)(d0 + j < bins ? run : n_tile);
            run += c[j];
        }
        for (uint32_t d = PT_MAX_BINS + tid; d < pw; d += PT_THREADS)
            row[d] = (uint16_t)n_tile;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
            if (rd[i] != ~0u)
                rd[i] = s_cnt[rd[i] & (PT_MAX_BINS - 1)] + (rd[i] >> PT_MAX_BITS);
        // the tile back to its own positions in digit order, one stage of
        // slots per round
#pragma unroll
        for (int r = 0; r < PT2_ROUNDS; r++) {
            const uint32_t lo = (uint32_t)r * STAGE;
            if (lo >= n_tile)
                break;  // uniform
#pragma unroll
            for (int i = 0; i < ITEMS; i++)
                if (rd[i] - lo < (uint32_t)STAGE)  // false for ~0 (no key): lo + STAGE <= 2^16
                    s_stage[rd[i] - lo] = key[i];
            __syncthreads();
            const uint32_t n = min((uint32_t)STAGE, n_tile - lo);
            for (uint32_t j = tid; j < n; j += PT_THREADS)
                out[t0 + lo + j] = s_stage[j];
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < PT_BPT; j++)
            s_cnt[d0 + j] = 0;
        __syncthreads();
    }
}

// Key-range shards of one library (pass 1, before the scan).  Window count
// of every digit d: the sum of its n_ch chunk counts hist[d * n_ch + i].
__global__ __launch_bounds__(256) void shard_totals(const uint32_t *__restrict__ hist, uint32_t n_ch,
                                                    uint32_t *__restrict__ tot) {
    __shared__ uint32_t s_w[256 / WAVE];
    const uint32_t d = blockIdx.x;
    uint32_t sum = 0;
    for (uint32_t i = threadIdx.x; i < n_ch; i += 256)
        sum += hist[(uint64_t)d * n_ch + i];
    sum = wave_inclusive_sum(sum);
    if (lane_id() == WAVE - 1)
        s_w[threadIdx.x / WAVE] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < 256 / WAVE; w++)
            t += s_w[w];
        tot[d] = t;
    }
}

// Owner of digit d (one workgroup, n_dig <= SH_THREADS digits):
// min(G - 1, floor(G * (below(d) + tot(d) / 2) / M)), non-decreasing in d, so
// shard g owns the digits [own[0], own[1]) = [#{owner < g}, #{owner <= g}).
constexpr int SH_THREADS = 1024;
__global__ __launch_bounds__(SH_THREADS) void shard_select(const uint32_t *__restrict__ tot, uint32_t n_dig,
                                                            uint32_t G, uint32_t g, uint32_t *__restrict__ own) {
    __shared__ uint32_t s_w[SH_THREADS / WAVE];
    const uint32_t d = threadIdx.x;
    const uint32_t t = d < n_dig ? tot[d] : 0u;
    const uint32_t inc = wave_inclusive_sum(t);
    if (lane_id() == WAVE - 1)
        s_w[d / WAVE] = inc;
    __syncthreads();
    uint64_t before = inc - t, M = 0;
    for (int w = 0; w < SH_THREADS / WAVE; w++) {
        before += (uint32_t)w < d / WAVE ? s_w[w] : 0u;
        M += s_w[w];
    }
    uint32_t owner = 0;
    if (M)
        owner = (uint32_t)min<uint64_t>(G - 1, (uint64_t)G * (2 * before + t) / (2 * M));
    const int below = __syncthreads_count(d < n_dig && owner < g);
    const int upto = __syncthreads_count(d < n_dig && owner <= g);
    if (d == 0) {
        own[0] = (uint32_t)below;
        own[1] = (uint32_t)upto;
    }
}

// Counts of the digits a shard does not own become 0, so that the scan
// places only its keys.
__global__ __launch_bounds__(256) void shard_clear(uint32_t *__restrict__ hist, uint32_t n_ch,
                                                   const uint32_t *__restrict__ own) {
    const uint32_t d = blockIdx.x;
    if (d >= own[0] && d < own[1])
        return;
    for (uint32_t i = threadIdx.x; i < n_ch; i += 256)
        hist[(uint64_t)d * n_ch + i] = 0;
}

// Start of segment s (library j, top digit d) from the scanned pass-1
// counts (n_hist1 entries, total1 keys).  Count entry h1 + d * nch1 of a
// library is the first chunk of digit d; an empty library has no entries and
// reads the start of what follows it.
__device__ __forceinline__ uint32_t segment_start(const PassArgs &a, const uint32_t *__restrict__ scan1,
                                                  uint64_t n_hist1, uint32_t total1, uint32_t s) {
    if (s >= a.nseg)
        return total1;
    const uint32_t j = last_le(a.n_libs, s, [&](uint32_t i) { return (uint64_t)a.libs[i].seg0; });
    const LibDesc &L = a.libs[j];
    const uint64_t e = L.h1 + (uint64_t)(s - L.seg0) * L.nch1;
    return e < n_hist1 ? scan1[e] : total1;
}

// Per segment: its start, its number of pass-2 chunks and of pass-2 tiles;
// the first key of every library.
template <typename K>
__global__ __launch_bounds__(SEG_THREADS) void pt_segments(PassArgs a, const uint32_t *__restrict__ scan1,
                                                           uint64_t n_hist1, const uint32_t *__restrict__ total1p,
                                                           uint32_t *__restrict__ seg, uint32_t *__restrict__ chs,
                                                           uint32_t *__restrict__ tiles, uint32_t *__restrict__ lib_keys) {
    const uint32_t total1 = *total1p;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= a.nseg; t += stride) {
        const uint32_t s = (uint32_t)t;
        const uint32_t start = segment_start(a, scan1, n_hist1, total1, s);
        seg[s] = start;
        if (s < a.nseg) {
            const uint32_t end = segment_start(a, scan1, n_hist1, total1, s + 1);
            chs[s] = (uint32_t)(((uint64_t)(end - start) + pt_chunk<K>() - 1) / pt_chunk<K>());
            tiles[s] = (uint32_t)(((uint64_t)(end - start) + pt2_tile<K>() - 1) / pt2_tile<K>());
        }
    }
    // first key of every library: the start of its first segment
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= a.n_libs; t += stride) {
        const uint32_t j = (uint32_t)t;
        lib_keys[j] = j < a.n_libs ? segment_start(a, scan1, n_hist1, total1, a.libs[j].seg0) : total1;
    }
}

// First key of every bucket (global id b = bucket0 of its library + its top
// D bits; entry n_buckets: the number of keys) when there is no second pass:
// every bucket is a segment.
__global__ __launch_bounds__(256) void pt_bucket_starts(PassArgs a, const uint32_t *__restrict__ total1p,
                                                        uint32_t n_buckets, uint32_t *__restrict__ starts) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= n_buckets; t += stride) {
        const uint32_t b = (uint32_t)t;
        if (b == n_buckets) {
            starts[b] = *total1p;
            continue;
        }
        const uint32_t j = last_le(a.n_libs, b, [&](uint32_t i) { return (uint64_t)a.libs[i].bucket0; });
        const LibDesc &L = a.libs[j];
        starts[b] = a.seg[L.seg0 + (b - L.bucket0)];
    }
}

// The prefix tables of every segment transposed (px: the segment's tiles
// side by side per digit, digit d of tile tt[s] + i at tt[s] * pw + d * T + i
// for the segment's T tiles, so that one digit's entries over all tiles are
// contiguous), and the size of every bucket (into sizes[b], b = bucket0 of
// its library + its top D bits): digit d2 of its segment summed over the
// segment's tiles.  One workgroup per segment and block of 64 digits (the
// block's sums need the entries of the digit after it too), 64 tiles at a
// time through LDS.
constexpr int TR_THREADS = 256;
constexpr int TR_B = 64;
__global__ __launch_bounds__(TR_THREADS) void pt_transpose(PassArgs a, const uint16_t *__restrict__ pt, uint32_t pw,
                                                           uint16_t *__restrict__ px, uint32_t *__restrict__ sizes) {
    __shared__ uint16_t s_b[TR_B][TR_B + 2];  // 64 tiles x 65 digits
    __shared__ uint32_t s_rs[TR_B + 1];
    const uint32_t s = blockIdx.x, dd = blockIdx.y * TR_B;
    if (s >= a.nseg)
        return;
    const int tid = threadIdx.x;
    const uint32_t j = last_le(a.n_libs, s, [&](uint32_t i) { return (uint64_t)a.libs[i].seg0; });
    const LibDesc &L = a.libs[j];
    const uint32_t bins = 1u << L.D2, nd = bins + 1;  // prefix entries of a tile: digits 0 .. bins
    if (dd >= bins)
        return;  // uniform
    const uint32_t t0 = a.tt[s], T = a.tt[s + 1] - t0;
    uint16_t *const out = px + (uint64_t)t0 * pw;
    uint32_t acc = 0;  // sum over the segment's tiles of digit dd + tid's entry (tid <= TR_B)
    for (uint32_t tb = 0; tb < T; tb += TR_B) {
        for (int x = tid; x < TR_B * (TR_B + 1); x += TR_THREADS) {
            const uint32_t ti = (uint32_t)x / (TR_B + 1), di = (uint32_t)x % (TR_B + 1);
            s_b[ti][di] = (tb + ti < T && dd + di < nd) ? pt[(uint64_t)(t0 + tb + ti) * pw + dd + di] : 0;
        }
        __syncthreads();
        // rows dd .. dd + 63, and the last block also row `bins` (the
        // tiles' sizes)
        for (int x = tid; x < TR_B * (TR_B + 1); x += TR_THREADS) {
            const uint32_t di = (uint32_t)x / TR_B, ti = (uint32_t)x % TR_B;
            if (tb + ti < T && dd + di < nd && (di < TR_B || dd + di == bins))
                out[(uint64_t)(dd + di) * T + tb + ti] = s_b[ti][di];
        }
        if (tid <= TR_B)
            for (int ti = 0; ti < TR_B; ti++)
                acc += s_b[ti][tid];
        __syncthreads();
    }
    if (tid <= TR_B)
        s_rs[tid] = acc;
    __syncthreads();
    const uint32_t b0 = L.bucket0 + ((s - L.seg0) << L.D2);
    if (tid < TR_B && dd + tid < bins)
        sizes[b0 + dd + tid] = s_rs[tid + 1] - s_rs[tid];
}

// Scratch words of the partition, in order: pass-1 counts and their scan
// scratch, segment starts, pass-2 chunks and tiles per segment, their scan
// scratch, totals, shard digits; with a second pass also the bucket-size
// scan scratch and the tiles' prefix tables, as written and transposed.
struct ScratchMap {
    uint64_t hist, seg, cb, tt, sscan, total1, own, bscan, pt, px, words;
    uint64_t n_tiles;  // bound on pass-2 tiles
    uint32_t pw;       // prefix entries per tile
};

ScratchMap scratch_map(const PartPlan &p, uint64_t tile) {
    ScratchMap m{};
    const uint64_t n1 = p.n_hist1;
    const uint64_t ns = (uint64_t)p.nseg + 1;
    m.hist = 0;
    m.seg = n1 + scan_scratch_words(n1);
    m.cb = m.seg + ns;
    m.tt = m.cb + ns;
    m.sscan = m.tt + ns;
    m.total1 = m.sscan + scan_scratch_words(p.nseg);
    m.own = m.total1 + 4;
    uint64_t w = m.own + (p.shard_count > 1 ? p.nseg + 2 : 0);
    if (p.D2max) {
        m.bscan = w;
        w += scan_scratch_words(p.n_buckets);
        m.pw = (1u << p.D2max) + 1;
        m.n_tiles = ceil_div(p.cap, tile) + p.nseg;  // pass-2 tiles
        m.pt = align_up(w, 4);
        w = m.pt + ceil_div(m.n_tiles * m.pw, 2);
        m.px = align_up(w, 4);
        w = m.px + ceil_div(m.n_tiles * m.pw, 2);
    }
    m.words = w;
    return m;
}

template <typename K>
hipError_t run_partition(const PartPlan &p, void *tmp, void *out, uint32_t *scratch, size_t scratch_words,
                         uint32_t *lib_keys, uint32_t *bucket_starts, KeyLayout *layout, hipStream_t stream) {
    if (p.D2max < 0 || p.D2max > PT_MAX_BITS)
        return hipErrorInvalidValue;
    const ScratchMap m = scratch_map(p, pt2_tile<K>());
    const bool shard = p.shard_count > 1;
    if (m.words > scratch_words || (shard && (p.n_libs != 1 || p.nseg > SH_THREADS)))
        return hipErrorInvalidValue;
    const uint64_t n1 = p.n_hist1;
    uint32_t *hist = scratch + m.hist;
    uint32_t *seg = scratch + m.seg;
    uint32_t *cb = scratch + m.cb;
    uint32_t *tt = scratch + m.tt;
    uint32_t *sscan = scratch + m.sscan;
    uint32_t *total1 = scratch + m.total1;
    uint32_t *own = scratch + m.own;  // shards: owned digits, then the digit totals
    uint32_t *dig_tot = own + 2;
    const dim3 block(PT_THREADS);

    PassArgs a{};
    a.packed = p.packed;
    a.valid = p.valid;
    a.libs = p.libs;
    a.n_libs = p.n_libs;
    a.seg = seg;
    a.cb = cb;
    a.tt = tt;
    a.nseg = p.nseg;
    a.cap = p.cap;
    *layout = KeyLayout{};

    // pass 1: windows -> (second pass ? tmp : out), by (library, top D1 bits)
    void *out1 = p.D2max ? tmp : out;
    hipError_t e;
    if (p.nch1) {
        pt_hist<K><<<dim3(p.nch1), block, 0, stream>>>(a, hist);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (shard) {  // one library: nseg digits of nch1 counts each
            shard_totals<<<dim3(p.nseg), dim3(256), 0, stream>>>(hist, p.nch1, dig_tot);
            shard_select<<<dim3(1), dim3(SH_THREADS), 0, stream>>>(dig_tot, p.nseg, p.shard_count, p.shard_index,
                                                                   own);
            shard_clear<<<dim3(p.nseg), dim3(256), 0, stream>>>(hist, p.nch1, own);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
            a.own = own;
        }
    }
    if ((e = launch_exclusive_scan(hist, hist, n1, hist + n1, total1, stream)) != hipSuccess)
        return e;
    if (p.nch1) {
        pt_scatter<K><<<dim3(p.nch1), block, 0, stream>>>(a, hist, static_cast<K *>(out1));
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const unsigned sgrid = (unsigned)std::min<uint64_t>(ceil_div((uint64_t)p.nseg + 1, SEG_THREADS), 4096);
    pt_segments<K><<<dim3(sgrid), dim3(SEG_THREADS), 0, stream>>>(a, hist, n1, total1, seg, cb, tt, lib_keys);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (!p.D2max) {
        const unsigned bgrid = (unsigned)std::min<uint64_t>(ceil_div((uint64_t)p.n_buckets + 1, 256), 8192);
        pt_bucket_starts<<<dim3(bgrid), dim3(256), 0, stream>>>(a, total1, p.n_buckets, bucket_starts);
        return hipGetLastError();
    }

    // pass 2: tmp -> out, every tile of every segment by its library's next
    // D2 bits, in place
    if ((e = launch_exclusive_scan(cb, cb, p.nseg, sscan, cb + p.nseg, stream)) != hipSuccess ||
        (e = launch_exclusive_scan(tt, tt, p.nseg, sscan, tt + p.nseg, stream)) != hipSuccess)
        return e;
    a.keys_in = tmp;
    uint16_t *pt = reinterpret_cast<uint16_t *>(scratch + m.pt);
    const uint64_t grid2 = ceil_div(p.cap, pt_chunk<K>()) + p.nseg;  // bound on pass-2 chunks
    pt_tiles<K><<<dim3((unsigned)grid2), block, 0, stream>>>(a, pt, m.pw, static_cast<K *>(out));
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    // transposed prefix tables and bucket sizes, then the sizes' exclusive
    // scan: the first index of every bucket in (library, bucket) order and,
    // in entry n_buckets, the number of keys
    uint16_t *px = reinterpret_cast<uint16_t *>(scratch + m.px);
    if (p.nseg) {
        const unsigned dblocks = (unsigned)ceil_div(1ull << p.D2max, TR_B);
        pt_transpose<<<dim3(p.nseg, dblocks), dim3(TR_THREADS), 0, stream>>>(a, pt, m.pw, px, bucket_starts);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    if ((e = launch_exclusive_scan(bucket_starts, bucket_starts, p.n_buckets, scratch + m.bscan,
                                   bucket_starts + p.n_buckets, stream)) != hipSuccess)
        return e;
    layout->tiled = 1;
    layout->seg = seg;
    layout->tt = tt;
    layout->px = px;
    layout->pw = m.pw;
    layout->tile_keys = (uint32_t)pt2_tile<K>();
    return hipSuccess;
}

}  // namespace

uint64_t partition_chunk(int key_words) { return key_words == 2 ? pt_chunk<Key2>() : pt_chunk<uint64_t>(); }
uint64_t partition_tile2(int key_words) { return key_words == 2 ? pt2_tile<Key2>() : pt2_tile<uint64_t>(); }

size_t partition_scratch_words(const PartPlan &p, int key_words) {
    return key_words == 2 ? scratch_map(p, pt2_tile<Key2>()).words : scratch_map(p, pt2_tile<uint64_t>()).words;
}

hipError_t partition_keys(const PartPlan &p, int key_words, void *tmp, void *out, uint32_t *scratch,
                          size_t scratch_words, uint32_t *lib_keys, uint32_t *bucket_starts, KeyLayout *layout,
                          hipStream_t stream) {
    return key_words == 2
               ? run_partition<Key2>(p, tmp, out, scratch, scratch_words, lib_keys, bucket_starts, layout, stream)
               : run_partition<uint64_t>(p, tmp, out, scratch, scratch_words, lib_keys, bucket_starts, layout,
                                         stream);
}

}  // namespace tk
