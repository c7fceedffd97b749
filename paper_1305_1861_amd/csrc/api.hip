// C ABI of libturtle: argument checks, workspace planning and the launch
// order of the counting path on one HIP stream.
//
//   pack (K1) -> screen (K2) -> collect (K3) -> [read n_collected]
//             -> radix sort (K4) -> compact (K5) -> [read counters]
//
// The only host synchronisations are the two small counter reads.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "turtle.h"

namespace tk {
namespace {

thread_local char g_err[512];

tk_status fail(tk_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

#define TK_HIP(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(TK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));            \
    } while (0)

constexpr uint32_t DEF_BETA = 4, DEF_TABLE_BITS = 10, DEF_BITS = 2;
constexpr uint64_t DEF_SEED = 1305;
constexpr int BLOCKS_PER_CU = 16;

struct Opts {
    uint32_t beta, table_bits, bits, flags;
    uint64_t blocks, seed;
    int part_bits;
    uint32_t shard_count, shard_index;
    int tile;
};

tk_status resolve(const tk_options *o, Opts *r) {
    r->beta = DEF_BETA;
    r->table_bits = DEF_TABLE_BITS;
    r->bits = DEF_BITS;
    r->flags = 0;
    r->blocks = 0;
    r->seed = DEF_SEED;
    r->part_bits = -1;
    r->shard_count = 1;
    r->shard_index = 0;
    r->tile = 0;
    if (o) {
        if (o->bloom_beta)
            r->beta = o->bloom_beta;
        if (o->bloom_table_bits)
            r->table_bits = o->bloom_table_bits;
        if (o->bloom_bits)
            r->bits = o->bloom_bits;
        r->flags = o->flags;
        r->blocks = o->bloom_blocks;
        r->seed = o->bloom_seed ? o->bloom_seed : DEF_SEED;
        r->part_bits = o->part_bits;
        r->shard_count = o->shard_count ? o->shard_count : 1;
        r->shard_index = o->shard_index;
        if (o->bucket_tile > 1)
            return fail(TK_EINVAL, "bucket_tile %u out of range [0, 1]", o->bucket_tile);
        r->tile = (int)o->bucket_tile;
    }
    const bool global = r->flags & (TK_FLAG_GLOBAL_FILTER | TK_FLAG_CTURTLE | TK_FLAG_SINGLE_PASS);
    if ((r->flags & TK_FLAG_CTURTLE) && (r->flags & (TK_FLAG_SINGLE_PASS | TK_FLAG_GLOBAL_FILTER)))
        return fail(TK_EINVAL, "TK_FLAG_CTURTLE combines with no other path flag");
    if ((r->flags & TK_FLAG_SINGLE_PASS) && (r->flags & TK_FLAG_GLOBAL_FILTER))
        return fail(TK_EINVAL, "TK_FLAG_SINGLE_PASS combines with no other path flag");
    if (r->beta > (global ? 1024u : 32u))
        return fail(TK_EINVAL, "bloom_beta %u out of range [1, %u]", r->beta, global ? 1024u : 32u);
    if (r->table_bits < 1 || r->table_bits > 10)
        return fail(TK_EINVAL, "bloom_table_bits %u out of range [1, 10]", r->table_bits);
    if (r->part_bits < -1 || r->part_bits > 20)
        return fail(TK_EINVAL, "part_bits %d out of range [-1, 20]", r->part_bits);
    if (r->bits < 1 || r->bits > 16)
        return fail(TK_EINVAL, "bloom_bits %u out of range [1, 16]", r->bits);
    if (r->shard_count > 1024 || r->shard_index >= r->shard_count)
        return fail(TK_EINVAL, "shard %u of %u: need shard_index < shard_count <= 1024", r->shard_index,
                    r->shard_count);
    if (r->shard_count > 1 && global)
        return fail(TK_EINVAL, "key-range shards need the partitioned path");
    return TK_OK;
}

uint64_t splitmix64_next(uint64_t &state) {
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Pattern table: SplitMix64(seed); each entry takes the top six bits of
// successive outputs as bit positions, skipping repeats, until it has `bits`
// distinct positions.  Cached for the life of the process (its storage is the
// source of asynchronous uploads).
const std::vector<uint64_t> &pattern_table(uint64_t seed, uint32_t table_bits, uint32_t bits) {
    static std::mutex mu;
    static std::map<std::tuple<uint64_t, uint32_t, uint32_t>, std::vector<uint64_t>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(seed, table_bits, bits);
    auto it = cache.find(key);
    if (it != cache.end())
        return it->second;
    std::vector<uint64_t> t(size_t(1) << table_bits, 0);
    uint64_t state = seed;
    for (auto &m : t) {
        uint32_t have = 0;
        while (have < bits) {
            const uint64_t bit = 1ull << (splitmix64_next(state) >> 58);
            if (!(m & bit)) {
                m |= bit;
                ++have;
            }
        }
    }
    return cache.emplace(key, std::move(t)).first->second;
}

uint64_t bloom_blocks_for(uint64_t n_bases, uint64_t n_reads, int k, const Opts &o) {
    if (o.blocks)
        return o.blocks;
    const uint64_t cut = n_reads * (uint64_t)(k - 1);
    const uint64_t w = n_bases > cut ? n_bases - cut : 0;
    const uint64_t est = w ? w : 1;
    const uint64_t b = ceil_div((uint64_t)o.beta * est, 256);
    return b ? b : 1;
}

// Bucket bits of the partitioned path (size rule documented in turtle.h).
int part_bits_for(uint64_t n_bases, uint64_t n_reads, int k, const Opts &o) {
    const int cap = std::min(20, 2 * k);
    if (o.part_bits >= 0)
        return std::min(o.part_bits, cap);
    const uint64_t cut = n_reads * (uint64_t)(k - 1);
    const uint64_t w = n_bases > cut ? n_bases - cut : 1;
    int lg = 0;
    while ((1ull << lg) < w)
        ++lg;
    const int d = lg - (k <= 31 ? 11 : 10);
    return std::max(0, std::min(d, cap));
}

constexpr uint64_t MAX_BUCKET_GRID = 4096;

struct Plan {
    int approx;            // 0 exact; 1 cTurtle; 2 single pass with "+1"
    uint64_t approx_words; // filter words of the approximate variants
    int k, key_words;      // k: the largest k of the libraries
    bool mixed_k;          // the libraries do not all have the same k
    uint32_t c;            // global path
    bool screen, global;   // screen: some library has c >= 2
    Opts opts;
    uint64_t n_bases, n_reads, n_words, cap, n_blocks;
    size_t key_bytes;
    // per-bucket path: the libraries of the batch
    uint32_t n_libs;
    std::vector<LibDesc> libs;
    uint64_t n_buckets, fb_cap, fb_nb_max;
    PartPlan part;
    size_t part_words;
    // workspace offsets
    size_t off_ctr, off_table, off_packed, off_valid, off_starts, off_filter;
    size_t off_keys_a, off_keys_b, off_counts, off_sort, off_compact;
    size_t off_gapc, off_f, off_part, off_rec_start, off_rec_nout, off_rec_off, off_rec_scan;
    size_t off_fb_list, off_fb_ent, off_fbc, off_misc, off_bstart, off_grp_first, off_grp_last, off_grp_count;
    size_t off_grp_piece, total;
    size_t off_libs, off_lib_keys, off_lib_stats, off_lib_ctr, off_lib_first;
    size_t sort_bytes, compact_bytes;
};

// small device values of the partitioned path
struct Misc {
    uint32_t fb_count;
    uint32_t totals[3];  // [1] records out
    DevCounters fb_ctr;
    uint32_t chunk_next;  // bucket kernel: next chunk to take
    uint32_t pad[3];
};

// One library of a plan: window positions [pos0, pos1) of the bases array,
// its number of reads, k and threshold.
struct LibSpec {
    uint64_t pos0, pos1, n_reads;
    int k;
    uint32_t c;
};

// Plan of one counting pass over the libraries `ls` (ordered by position,
// all with keys of the same width) of one bases/offsets pair of n_bases
// bases and n_reads reads.
tk_status make_plan(const LibSpec *ls, uint64_t n_libs, uint64_t n_bases, uint64_t n_reads, const tk_options *o,
                    Plan *p) {
    if (n_libs == 0 || !ls)
        return fail(TK_EINVAL, "a batch needs at least one library");
    if (n_libs >= (1ull << 24))
        return fail(TK_EINVAL, "%llu libraries are too many", (unsigned long long)n_libs);
    if (n_bases >= (1ull << 32))
        return fail(TK_EOVERFLOW, "n_bases = %llu must be below 2^32", (unsigned long long)n_bases);
    if (n_reads >= (1ull << 40))
        return fail(TK_EOVERFLOW, "n_reads = %llu too large", (unsigned long long)n_reads);
    int kmax = 0;
    uint64_t cap = 0;
    for (uint64_t j = 0; j < n_libs; j++) {
        if (ls[j].k < 1 || ls[j].k > 63)
            return fail(TK_EINVAL, "k = %d outside [1, 63]", ls[j].k);
        if (ls[j].c == 0)
            return fail(TK_EINVAL, "threshold c must be >= 1");
        if ((ls[j].k <= 31) != (ls[0].k <= 31))
            return fail(TK_EINVAL, "one counting pass takes keys of one width");
        if (ls[j].pos1 < ls[j].pos0 || ls[j].pos1 > n_bases || (j && ls[j].pos0 < ls[j - 1].pos1))
            return fail(TK_EINVAL, "library %llu lies outside the bases or before the previous one",
                        (unsigned long long)j);
        kmax = std::max(kmax, ls[j].k);
        cap += ls[j].pos1 - ls[j].pos0;  // windows <= bases
    }
    tk_status st = resolve(o, &p->opts);
    if (st != TK_OK)
        return st;
    const int k = kmax;
    p->k = k;
    p->mixed_k = false;
    for (uint64_t j = 0; j < n_libs; j++)
        p->mixed_k = p->mixed_k || ls[j].k != k;
    p->c = ls[0].c;
    p->key_words = k <= 31 ? 1 : 2;
    p->key_bytes = 8 * (size_t)p->key_words;
    p->screen = false;
    for (uint64_t j = 0; j < n_libs; j++)
        p->screen = p->screen || ls[j].c >= 2;
    p->approx = (p->opts.flags & TK_FLAG_CTURTLE) ? 1 : (p->opts.flags & TK_FLAG_SINGLE_PASS) ? 2 : 0;
    p->global = (p->opts.flags & TK_FLAG_GLOBAL_FILTER) || p->approx;
    if (p->global && n_libs != 1)
        return fail(TK_EINVAL, "the global-filter path and the approximate variants count one library per call");
    if (p->opts.shard_count > 1 && n_libs != 1)
        return fail(TK_EINVAL, "key-range shards split one library per call");
    if (p->approx == 1 && p->c != 2)
        return fail(TK_EINVAL, "cTurtle reports k-mers seen more than once: c must be 2");
    if (p->approx)
        p->screen = true;
    p->n_bases = n_bases;
    p->n_reads = n_reads;
    p->n_words = ceil_div(n_bases, 32);
    p->cap = cap;
    p->n_blocks = (p->screen && p->global) ? bloom_blocks_for(n_bases, n_reads, k, p->opts) : 0;
    p->approx_words = 0;
    if (p->approx) {
        const uint64_t cut = n_reads * (uint64_t)(k - 1);
        const uint64_t est = n_bases > cut ? n_bases - cut : 1;
        p->approx_words = p->opts.blocks ? 8 * p->opts.blocks : std::max<uint64_t>(1, ceil_div(p->opts.beta * est, 64));
        p->n_blocks = ceil_div(p->approx_words, 8);
    }
    if (p->n_blocks > (1ull << 40))
        return fail(TK_EINVAL, "filter of %llu blocks is too large", (unsigned long long)p->n_blocks);
    p->n_libs = (uint32_t)n_libs;
    p->libs.clear();
    if (!p->global) {
        const uint64_t chunk = partition_chunk(p->key_words);
        uint64_t n_ch = 0, n_hist = 0, n_seg = 0, n_bk = 0;
        int d2max = 0;
        p->libs.resize(n_libs);
        for (uint64_t j = 0; j < n_libs; j++) {
            LibDesc &L = p->libs[j];
            L.pos0 = ls[j].pos0;
            L.pos1 = ls[j].pos1;
            L.c = ls[j].c;
            L.k = ls[j].k;
            L.D = part_bits_for(L.pos1 - L.pos0, ls[j].n_reads, L.k, p->opts);
            // the second pass orders its tiles in place, so its digit count
            // does not shape its writes: it takes 10 bits, and the first
            // pass (whose digit runs are shorter the more digits it has)
            // only the rest
            L.D1 = L.D > 10 ? L.D - 10 : L.D;
            L.D2 = L.D - L.D1;
            L.nch1 = L.pos1 > L.pos0 ? (uint32_t)ceil_div(L.pos1 - (L.pos0 & ~31ull), chunk) : 0u;
            L.cb1 = (uint32_t)n_ch;
            L.h1 = n_hist;
            L.seg0 = (uint32_t)n_seg;
            L.bucket0 = (uint32_t)n_bk;
            n_ch += L.nch1;
            n_hist += (uint64_t)L.nch1 << L.D1;
            n_seg += 1ull << L.D1;
            n_bk += 1ull << L.D;
            d2max = std::max(d2max, L.D2);
        }
        if (n_bk >= (1ull << 31) || n_seg >= (1ull << 28) || n_ch >= (1ull << 31))
            return fail(TK_EINVAL, "the batch needs %llu buckets: too many (lower part_bits or split the batch)",
                        (unsigned long long)n_bk);
        p->n_buckets = n_bk;
        p->part = PartPlan{};
        p->part.n_libs = (uint32_t)n_libs;
        p->part.nch1 = (uint32_t)n_ch;
        p->part.n_hist1 = n_hist;
        p->part.nseg = (uint32_t)n_seg;
        p->part.D2max = d2max;
        p->part.cap = p->cap;
        p->part.shard_count = p->opts.shard_count;
        p->part.shard_index = p->opts.shard_index;
        // fallback list: buckets larger than a group, and every bucket of a
        // segment with more second-pass tiles than a group may span (more
        // than BK_TILES_MAX tiles of keys each)
        p->fb_cap = p->cap / ((uint64_t)bucket_capacity(p->key_words, p->opts.tile) + 1) + 1;
        if (d2max)
            p->fb_cap += (p->cap / (BK_TILES_MAX * partition_tile2(p->key_words)) + 1) << d2max;
        p->fb_nb_max = p->screen ? ceil_div((uint64_t)p->opts.beta * std::max<uint64_t>(p->cap, 1), 256) + p->fb_cap : 0;
        p->part.n_buckets = (uint32_t)n_bk;
        p->part_words = partition_scratch_words(p->part, p->key_words);
    }
    p->sort_bytes = radix_scratch_bytes(p->cap, p->key_words);
    p->compact_bytes = compact_scratch_bytes(p->cap);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t r = off;
        off = align_up(off + bytes, 256);
        return r;
    };
    p->off_ctr = take(sizeof(DevCounters));
    p->off_table = take(sizeof(uint64_t) << p->opts.table_bits);
    p->off_packed = take(p->n_words * sizeof(uint64_t));
    p->off_valid = take(p->n_words * sizeof(uint32_t));
    p->off_starts = take(p->n_words * sizeof(uint32_t));
    p->off_keys_a = take(p->cap * p->key_bytes);
    p->off_keys_b = take(p->cap * p->key_bytes);
    p->off_sort = take(p->sort_bytes);
    p->off_compact = take(p->compact_bytes);
    if (p->global) {
        p->off_filter = take(p->n_blocks * 64);
        p->off_counts = take(p->cap * sizeof(uint32_t));
    } else {
        p->off_filter = take(p->fb_nb_max * 64);
        p->off_gapc = take(p->cap * sizeof(uint32_t));
        p->off_f = take(p->cap * p->key_bytes);
        p->off_part = take(p->part_words * sizeof(uint32_t));
        p->off_rec_start = take(p->n_buckets * sizeof(uint32_t));
        p->off_rec_nout = take(p->n_buckets * sizeof(uint32_t));
        p->off_rec_off = take(p->n_buckets * sizeof(uint32_t));
        p->off_rec_scan = take(scan_scratch_words(p->n_buckets) * sizeof(uint32_t));
        p->off_fb_list = take(p->fb_cap * 3 * sizeof(uint32_t));
        p->off_fb_ent = take(p->fb_cap * sizeof(FbEntry));
        p->off_fbc = take(p->cap * sizeof(uint32_t));
        p->off_misc = take(sizeof(Misc));
        p->off_bstart = take((p->n_buckets + 1) * sizeof(uint32_t));
        // the group plan for any chunk size up to BK_CHUNK_MAX bucket ids
        // (chosen per call from the device): at most n_buckets groups and
        // chunks
        p->off_grp_first = take((p->n_buckets + BK_CHUNK_MAX) * sizeof(uint32_t));
        p->off_grp_last = take((p->n_buckets + BK_CHUNK_MAX) * sizeof(uint32_t));
        p->off_grp_count = take((p->n_buckets + 1) * sizeof(uint32_t));
        p->off_grp_piece = take((p->n_buckets + BK_CHUNK_MAX) * sizeof(uint4));
        p->off_libs = take(n_libs * sizeof(LibDesc));
        p->off_lib_keys = take((n_libs + 1) * sizeof(uint32_t));
        p->off_lib_stats = take(n_libs * 4 * sizeof(unsigned long long));
        p->off_lib_ctr = take(n_libs * sizeof(DevCounters));
        p->off_lib_first = take(n_libs * sizeof(uint32_t));
    }
    p->total = off;
    return TK_OK;
}

tk_status make_plan(uint64_t n_bases, uint64_t n_reads, int k, uint32_t c, const tk_options *o, Plan *p) {
    const LibSpec one{0, n_bases, n_reads, k, c};
    return make_plan(&one, 1, n_bases, n_reads, o, p);
}

// A batch of libraries (library j: reads [lib_reads[j], lib_reads[j + 1]),
// bases [lib_bases[j], lib_bases[j + 1])) in at most two counting passes,
// one per key width, each in its own part of the workspace: member[q] lists
// the libraries of pass q, ws_off[q] the start of its part.
struct BatchPlan {
    std::vector<Plan> plans;
    std::vector<std::vector<uint32_t>> member;
    std::vector<size_t> ws_off;
    size_t total = 0;
};

tk_status make_batch_plan(uint64_t n_libs, const uint64_t *lib_bases, const uint64_t *lib_reads, const int *k,
                          const uint32_t *c, const tk_options *o, BatchPlan *bp) {
    if (n_libs == 0 || !lib_bases || !lib_reads || !k || !c)
        return fail(TK_EINVAL, "a batch needs at least one library and its boundaries, k and thresholds");
    if (n_libs >= (1ull << 24))
        return fail(TK_EINVAL, "%llu libraries are too many", (unsigned long long)n_libs);
    if (lib_bases[0] != 0 || lib_reads[0] != 0)
        return fail(TK_EINVAL, "library boundaries must start at 0");
    for (uint64_t j = 0; j < n_libs; j++) {
        if (lib_bases[j + 1] < lib_bases[j] || lib_reads[j + 1] < lib_reads[j])
            return fail(TK_EINVAL, "library boundaries decrease at library %llu", (unsigned long long)j);
        if (c[j] == 0)
            return fail(TK_EINVAL, "threshold c of library %llu must be >= 1", (unsigned long long)j);
        if (k[j] < 1 || k[j] > 63)
            return fail(TK_EINVAL, "k = %d of library %llu outside [1, 63]", k[j], (unsigned long long)j);
    }
    const uint64_t n_bases = lib_bases[n_libs], n_reads = lib_reads[n_libs];
    bp->plans.clear();
    bp->member.clear();
    bp->ws_off.clear();
    bp->total = 0;
    for (int width = 1; width <= 2; width++) {
        std::vector<LibSpec> ls;
        std::vector<uint32_t> mem;
        for (uint64_t j = 0; j < n_libs; j++) {
            if ((k[j] <= 31 ? 1 : 2) != width)
                continue;
            ls.push_back(LibSpec{lib_bases[j], lib_bases[j + 1], lib_reads[j + 1] - lib_reads[j], k[j], c[j]});
            mem.push_back((uint32_t)j);
        }
        if (ls.empty())
            continue;
        Plan p;
        tk_status st = make_plan(ls.data(), ls.size(), n_bases, n_reads, o, &p);
        if (st != TK_OK)
            return st;
        if (p.global)
            return fail(TK_EINVAL, "batches run the partitioned path only");
        bp->ws_off.push_back(bp->total);
        bp->total = align_up(bp->total + p.total, 256);
        bp->plans.push_back(std::move(p));
        bp->member.push_back(std::move(mem));
    }
    return TK_OK;
}

__global__ void zero_vec(uint4 *__restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void zero_u32(uint32_t *__restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0;
}

}  // namespace

// Clears n bytes (n a multiple of 4, p 4-byte aligned) with kernels rather
// than memset nodes, so the sequence stays safe under stream capture.
hipError_t zero_bytes(void *p, size_t n, hipStream_t s) {
    if (n < 4)
        return hipSuccess;
    uint64_t words = n / 4;
    uint32_t *q = static_cast<uint32_t *>(p);
    if (((uintptr_t)q & 15u) == 0 && words >= 4) {
        const uint64_t vec = words / 4;
        const uint64_t g = std::min<uint64_t>(ceil_div(vec, 256), 65536);
        zero_vec<<<dim3((unsigned)g), dim3(256), 0, s>>>(reinterpret_cast<uint4 *>(q), vec);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        q += vec * 4;
        words -= vec * 4;
    }
    if (!words)
        return hipSuccess;
    const uint64_t g = std::min<uint64_t>(ceil_div(words, 256), 65536);
    zero_u32<<<dim3((unsigned)g), dim3(256), 0, s>>>(q, words);
    return hipGetLastError();
}

namespace {

int g_cu_cache[64];

// memcpy split over up to 8 host threads (slices of at least 4 MB)
void parallel_memcpy(void *dst, const void *src, size_t bytes) {
    constexpr size_t MIN_PART = size_t(4) << 20;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t parts = std::min<size_t>({8, (size_t)hw, std::max<size_t>(1, bytes / MIN_PART)});
    if (parts <= 1) {
        memcpy(dst, src, bytes);
        return;
    }
    std::vector<std::thread> pool;
    const size_t step = (bytes + parts - 1) / parts;
    auto part = [=](size_t a, size_t b) {
        memcpy(static_cast<char *>(dst) + a, static_cast<const char *>(src) + a, b - a);
    };
    for (size_t i = 1; i < parts; i++) {
        const size_t a = i * step, b = std::min(bytes, a + step);
        if (a >= b)
            continue;
        try {  // no exception may cross the C boundary: a part without a thread is copied here
            pool.emplace_back(part, a, b);
        } catch (...) {
            part(a, b);
        }
    }
    part(0, std::min(bytes, step));
    for (auto &t : pool)
        t.join();
}

}  // namespace

class Stager {
  public:
    static constexpr size_t SLICE = size_t(64) << 20;
    Stager() = default;
    Stager(const Stager &) = delete;
    Stager &operator=(const Stager &) = delete;
    ~Stager() { (void)release(); }
    hipError_t copy(void *dst, const void *src, size_t bytes, bool to_device, hipStream_t stream);
    hipError_t release();

  private:
    hipError_t reserve(size_t slice);
    void *pin_[2] = {nullptr, nullptr};
    hipEvent_t ev_[2] = {nullptr, nullptr};
    size_t cap_ = 0;
};

// Copies between pageable host memory and device memory through two pinned
// staging slices: the DMA of one slice overlaps the multi-threaded host copy
// of the other (the runtime's own pageable copies ran at about 4 GB/s here).
// A slice is reused only after its last DMA has finished, whatever stream
// that DMA was on.  Host to device: returns once the last slice's DMA is
// enqueued on `stream` (later work on that stream sees the data); device to
// host: returns once the data is in dst.
hipError_t Stager::reserve(size_t slice) {
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; i++)
        if (!ev_[i])
            e = hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming);
    if (e != hipSuccess || cap_ >= slice)
        return e;
    for (int i = 0; i < 2; i++) {
        if ((e = hipEventSynchronize(ev_[i])) != hipSuccess)
            return e;
        if (pin_[i])
            (void)hipHostFree(pin_[i]);
        pin_[i] = nullptr;
    }
    cap_ = 0;
    for (int i = 0; i < 2; i++)
        if ((e = hipHostMalloc(&pin_[i], slice)) != hipSuccess)
            return e;
    cap_ = slice;
    return hipSuccess;
}

hipError_t Stager::copy(void *dst, const void *src, size_t bytes, bool to_device, hipStream_t stream) {
    if (!bytes)
        return hipSuccess;
    hipError_t e = reserve(std::min(bytes, SLICE));
    if (e != hipSuccess)
        return e;
    const size_t n_slices = (bytes + SLICE - 1) / SLICE;
    auto drain = [&](size_t i) -> hipError_t {  // device to host: slice i from its slot to dst
        const size_t off = i * SLICE, len = std::min(SLICE, bytes - off);
        hipError_t w = hipEventSynchronize(ev_[i % 2]);
        if (w == hipSuccess)
            parallel_memcpy(static_cast<char *>(dst) + off, pin_[i % 2], len);
        return w;
    };
    for (size_t i = 0; i < n_slices; i++) {
        const size_t off = i * SLICE, len = std::min(SLICE, bytes - off);
        const int b = (int)(i % 2);
        if ((e = hipEventSynchronize(ev_[b])) != hipSuccess)  // the slot's last DMA
            return e;
        if (to_device) {
            parallel_memcpy(pin_[b], static_cast<const char *>(src) + off, len);
            if ((e = hipMemcpyAsync(static_cast<char *>(dst) + off, pin_[b], len, hipMemcpyHostToDevice, stream)) !=
                    hipSuccess ||
                (e = hipEventRecord(ev_[b], stream)) != hipSuccess)
                return e;
        } else {
            if ((e = hipMemcpyAsync(pin_[b], static_cast<const char *>(src) + off, len, hipMemcpyDeviceToHost,
                                    stream)) != hipSuccess ||
                (e = hipEventRecord(ev_[b], stream)) != hipSuccess)
                return e;
            if (i > 0 && (e = drain(i - 1)) != hipSuccess)  // slice i - 1 while slice i travels
                return e;
        }
    }
    return to_device ? hipSuccess : drain(n_slices - 1);
}

hipError_t Stager::release() {
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2; i++) {
        if (ev_[i]) {
            const hipError_t w = hipEventSynchronize(ev_[i]);  // the slot's last DMA
            if (e == hipSuccess)
                e = w;
            (void)hipEventDestroy(ev_[i]);
            ev_[i] = nullptr;
        }
        if (pin_[i])
            (void)hipHostFree(pin_[i]);
        pin_[i] = nullptr;
    }
    cap_ = 0;
    return e;
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        dev = 0;
    int *slot = dev < 64 ? &g_cu_cache[dev] : nullptr;
    if (slot && *slot)
        return *slot;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
        cu = 256;
    if (slot)
        *slot = cu;
    return cu;
}

namespace {

struct Timer {
    bool on = false;
    hipEvent_t ev[2 * TK_STAGE_COUNT] = {};
    bool used[TK_STAGE_COUNT] = {};
    ~Timer() {
        for (auto &e : ev)
            if (e)
                (void)hipEventDestroy(e);
    }
    tk_status init(bool enable) {
        on = enable;
        if (!on)
            return TK_OK;
        for (auto &e : ev)
            TK_HIP(hipEventCreate(&e));
        return TK_OK;
    }
    tk_status mark(int i, hipStream_t s) {
        if (on) {
            TK_HIP(hipEventRecord(ev[2 * i], s));
            used[i] = true;
        }
        return TK_OK;
    }
    tk_status end(int i, hipStream_t s) {
        if (on)
            TK_HIP(hipEventRecord(ev[2 * i + 1], s));
        return TK_OK;
    }
    void read(double *ms) {
        for (int i = 0; i < TK_STAGE_COUNT; i++) {
            float t = 0.f;
            ms[i] = (on && used[i] && hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) ? (double)t
                                                                                                       : 0.0;
        }
    }
};

int persistent_grid(uint64_t n_pos) {
    const uint64_t want = ceil_div(n_pos ? n_pos : 1, 256);
    const uint64_t cap = (uint64_t)device_cu_count() * BLOCKS_PER_CU;
    return (int)std::min(want, cap);
}

tk_status run_global(const uint8_t *d_bases, const uint64_t *d_offsets, const Plan &p, char *ws, hipStream_t s,
                     tk_result *out) {
    DevCounters *ctr = reinterpret_cast<DevCounters *>(ws + p.off_ctr);
    uint64_t *table = reinterpret_cast<uint64_t *>(ws + p.off_table);
    uint64_t *packed = reinterpret_cast<uint64_t *>(ws + p.off_packed);
    uint32_t *valid = reinterpret_cast<uint32_t *>(ws + p.off_valid);
    uint32_t *starts = reinterpret_cast<uint32_t *>(ws + p.off_starts);
    uint64_t *filter = reinterpret_cast<uint64_t *>(ws + p.off_filter);
    uint64_t *keys_a = reinterpret_cast<uint64_t *>(ws + p.off_keys_a);
    uint64_t *keys_b = reinterpret_cast<uint64_t *>(ws + p.off_keys_b);
    uint32_t *counts = reinterpret_cast<uint32_t *>(ws + p.off_counts);

    Timer tm;
    tk_status st = tm.init(p.opts.flags & TK_FLAG_TIMING);
    if (st != TK_OK)
        return st;

    TK_HIP(zero_bytes(ctr, sizeof(DevCounters), s));
    TK_HIP(zero_bytes(starts, p.n_words * sizeof(uint32_t), s));
    if (p.screen) {
        TK_HIP(zero_bytes(filter, p.n_blocks * 64, s));
        const auto &tab = pattern_table(p.opts.seed, p.opts.table_bits, p.opts.bits);
        TK_HIP(hipMemcpyAsync(table, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    }

    if ((st = tm.mark(TK_STAGE_PACK, s)) != TK_OK)
        return st;
    TK_HIP(launch_pack(d_bases, d_offsets, p.n_bases, p.n_reads, p.k, packed, valid, starts, &ctr->n_windows, s));
    if ((st = tm.end(TK_STAGE_PACK, s)) != TK_OK || (st = tm.mark(TK_STAGE_SCREEN, s)) != TK_OK)
        return st;
    BloomArgs a{packed, valid, p.n_words, p.k, table, p.opts.table_bits, p.n_blocks, filter};
    const int grid = persistent_grid(p.n_words * 32);
    if (p.screen && !p.approx)
        TK_HIP(launch_screen(a, grid, s));
    if ((st = tm.end(TK_STAGE_SCREEN, s)) != TK_OK || (st = tm.mark(TK_STAGE_COLLECT, s)) != TK_OK)
        return st;
    if (p.approx)
        TK_HIP(launch_approx(packed, valid, p.n_words, p.k, table, p.opts.table_bits, filter, p.approx_words,
                             p.approx == 1, keys_a, p.cap, &ctr->n_collected, grid, s));
    else
        TK_HIP(launch_collect(a, p.screen, keys_a, p.cap, &ctr->n_collected, grid, s));
    if ((st = tm.end(TK_STAGE_COLLECT, s)) != TK_OK)
        return st;

    DevCounters h{};
    TK_HIP(hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));
    const uint64_t n = h.n_collected;
    if (n > p.cap)
        return fail(TK_EDEVICE, "collected %llu keys into a buffer of %llu", (unsigned long long)n,
                    (unsigned long long)p.cap);

    if ((st = tm.mark(TK_STAGE_SORT, s)) != TK_OK)
        return st;
    uint64_t *sorted = nullptr;
    int passes = 0;
    TK_HIP(radix_sort(keys_a, keys_b, n, p.key_words, 2 * p.k, ws + p.off_sort, p.sort_bytes, s, &sorted, &passes));
    uint64_t *out_keys = sorted == keys_a ? keys_b : keys_a;
    if ((st = tm.end(TK_STAGE_SORT, s)) != TK_OK || (st = tm.mark(TK_STAGE_COMPACT, s)) != TK_OK)
        return st;
    // cTurtle reports every key once (kept, counts cleared); the single pass
    // counts stored sightings, one short of the count
    const uint32_t c_eff = p.approx == 1 ? 1u : p.approx == 2 ? std::max(1u, p.c - 1) : p.c;
    TK_HIP(compact(sorted, n, p.key_words, c_eff, out_keys, counts, ws + p.off_compact, p.compact_bytes, ctr, s));
    if (p.approx)
        TK_HIP(launch_adjust_counts(counts, ctr, p.approx == 1 ? 0u : 1u, s));
    if ((st = tm.end(TK_STAGE_COMPACT, s)) != TK_OK)
        return st;
    TK_HIP(hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));

    memset(out, 0, sizeof *out);
    out->n = h.n_out;
    out->k = (uint32_t)p.k;
    out->key_words = (uint32_t)p.key_words;
    out->keys = out_keys;
    out->counts = counts;
    out->n_windows = h.n_windows;
    out->n_collected = h.n_collected;
    out->n_distinct = h.n_runs;
    out->n_singletons = h.n_single;
    out->n_below_c = h.n_below;
    out->bloom_blocks = p.n_blocks;
    out->sort_passes = (uint32_t)passes;
    out->part_bits = -1;
    tm.read(out->stage_ms);
    return TK_OK;
}

// The per-bucket path over the plan's libraries; out[j] receives library j.
tk_status run_partitioned(const uint8_t *d_bases, const uint64_t *d_offsets, const Plan &p, char *ws,
                          hipStream_t s, tk_result *out) {
    uint64_t *table = reinterpret_cast<uint64_t *>(ws + p.off_table);
    uint64_t *packed = reinterpret_cast<uint64_t *>(ws + p.off_packed);
    uint32_t *valid = reinterpret_cast<uint32_t *>(ws + p.off_valid);
    uint32_t *starts = reinterpret_cast<uint32_t *>(ws + p.off_starts);
    uint64_t *filter = reinterpret_cast<uint64_t *>(ws + p.off_filter);
    uint64_t *keys_a = reinterpret_cast<uint64_t *>(ws + p.off_keys_a);
    uint64_t *keys_b = reinterpret_cast<uint64_t *>(ws + p.off_keys_b);
    uint32_t *gap_counts = reinterpret_cast<uint32_t *>(ws + p.off_gapc);
    uint64_t *fbuf = reinterpret_cast<uint64_t *>(ws + p.off_f);
    uint32_t *part = reinterpret_cast<uint32_t *>(ws + p.off_part);
    uint32_t *rec_start = reinterpret_cast<uint32_t *>(ws + p.off_rec_start);
    uint32_t *rec_nout = reinterpret_cast<uint32_t *>(ws + p.off_rec_nout);
    uint32_t *rec_off = reinterpret_cast<uint32_t *>(ws + p.off_rec_off);
    uint32_t *rec_scan = reinterpret_cast<uint32_t *>(ws + p.off_rec_scan);
    uint32_t *fb_list = reinterpret_cast<uint32_t *>(ws + p.off_fb_list);
    Misc *misc = reinterpret_cast<Misc *>(ws + p.off_misc);
    LibDesc *d_libs = reinterpret_cast<LibDesc *>(ws + p.off_libs);
    uint32_t *lib_keys = reinterpret_cast<uint32_t *>(ws + p.off_lib_keys);
    unsigned long long *lib_stats = reinterpret_cast<unsigned long long *>(ws + p.off_lib_stats);
    DevCounters *lib_ctr = reinterpret_cast<DevCounters *>(ws + p.off_lib_ctr);
    uint32_t *lib_first = reinterpret_cast<uint32_t *>(ws + p.off_lib_first);
    const int kw = p.key_words;
    const uint32_t L = p.n_libs;

    Timer tm;
    tk_status st = tm.init(p.opts.flags & TK_FLAG_TIMING);
    if (st != TK_OK)
        return st;

    TK_HIP(zero_bytes(misc, sizeof(Misc), s));
    TK_HIP(zero_bytes(starts, p.n_words * sizeof(uint32_t), s));
    TK_HIP(zero_bytes(rec_nout, p.n_buckets * sizeof(uint32_t), s));
    TK_HIP(zero_bytes(lib_stats, (size_t)L * 4 * sizeof(unsigned long long), s));
    TK_HIP(hipMemcpyAsync(d_libs, p.libs.data(), (size_t)L * sizeof(LibDesc), hipMemcpyHostToDevice, s));
    if (p.screen) {
        const auto &tab = pattern_table(p.opts.seed, p.opts.table_bits, p.opts.bits);
        TK_HIP(hipMemcpyAsync(table, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    }

    if ((st = tm.mark(TK_STAGE_PACK, s)) != TK_OK)
        return st;
    TK_HIP(launch_pack(d_bases, d_offsets, p.n_bases, p.n_reads, p.k, packed, valid, starts, nullptr, s,
                       p.mixed_k ? d_libs : nullptr, L));
    if ((st = tm.end(TK_STAGE_PACK, s)) != TK_OK || (st = tm.mark(TK_STAGE_PARTITION, s)) != TK_OK)
        return st;

    // keys ordered by (library, bucket): windows -> A (through B for D > 10)
    PartPlan pp = p.part;
    pp.packed = packed;
    pp.valid = valid;
    pp.libs = d_libs;
    uint32_t *bstart = reinterpret_cast<uint32_t *>(ws + p.off_bstart);
    KeyLayout lay{};
    TK_HIP(partition_keys(pp, kw, keys_b, keys_a, part, p.part_words, lib_keys, bstart, &lay, s));
    uint64_t *sorted = keys_a, *other = keys_b;
    if ((st = tm.end(TK_STAGE_PARTITION, s)) != TK_OK || (st = tm.mark(TK_STAGE_BUCKET, s)) != TK_OK)
        return st;

    const int grid = (int)std::min<uint64_t>((uint64_t)bucket_grid(), MAX_BUCKET_GRID);
    BucketArgs ba{};
    ba.keys = sorted;
    ba.libs = d_libs;
    ba.n_libs = L;
    ba.lib_keys = lib_keys;
    ba.beta = p.opts.beta;
    ba.table = table;
    ba.table_bits = p.opts.table_bits;
    ba.gap_keys = other;
    ba.gap_counts = gap_counts;
    ba.rec_start = rec_start;
    ba.rec_nout = rec_nout;
    ba.lib_stats = lib_stats;
    ba.fb_list = fb_list;
    ba.fb_count = &misc->fb_count;
    ba.fb_cap = (uint32_t)p.fb_cap;
    ba.n_buckets = (uint32_t)p.n_buckets;
    ba.bucket_starts = bstart;
    // chunks of BK_CHUNK_MAX bucket ids (about 64K keys under the size
    // rule), fewer when that leaves under two chunks per workgroup
    ba.chunk_buckets = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(BK_CHUNK_MAX, p.n_buckets / (2 * (uint64_t)grid)));
    ba.n_chunks = (uint32_t)std::max<uint64_t>(1, ceil_div(p.n_buckets, ba.chunk_buckets));
    ba.grp_first = reinterpret_cast<uint32_t *>(ws + p.off_grp_first);
    ba.grp_last = reinterpret_cast<uint32_t *>(ws + p.off_grp_last);
    ba.grp_count = reinterpret_cast<uint32_t *>(ws + p.off_grp_count);
    ba.chunk_next = &misc->chunk_next;
    ba.tile = p.opts.tile;
    ba.layout = lay;
    ba.grp_piece = reinterpret_cast<uint4 *>(ws + p.off_grp_piece);
    TK_HIP(launch_bucket(ba, kw, grid, s));
    if ((st = tm.end(TK_STAGE_BUCKET, s)) != TK_OK)
        return st;

    Misc hm{};
    TK_HIP(hipMemcpyAsync(&hm, misc, sizeof hm, hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));
    if (hm.fb_count > p.fb_cap)
        return fail(TK_EDEVICE, "%u oversized buckets exceed the list of %llu", hm.fb_count,
                    (unsigned long long)p.fb_cap);

    // buckets too large for LDS: global-memory kernels, same filter rule, all
    // oversized buckets of a library at once
    if ((st = tm.mark(TK_STAGE_FALLBACK, s)) != TK_OK)
        return st;
    std::vector<uint32_t> fb_per_lib(L, 0);
    if (hm.fb_count) {
        const uint32_t nf = hm.fb_count;
        std::vector<uint32_t> list(3 * (size_t)nf);
        TK_HIP(hipMemcpyAsync(list.data(), fb_list, list.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        // (library, entry) in key order
        std::vector<std::pair<uint32_t, FbEntry>> all(nf);
        for (uint32_t i = 0; i < nf; i++) {
            const uint32_t id = list[3 * i];
            uint32_t lo = 0, hi = L;  // library: largest j with bucket0 <= id
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) / 2;
                if (p.libs[mid].bucket0 <= id)
                    lo = mid;
                else
                    hi = mid;
            }
            all[i] = {lo, FbEntry{id - p.libs[lo].bucket0, list[3 * i + 1], list[3 * i + 2], 0, 0, 0}};
        }
        std::sort(all.begin(), all.end(), [](const std::pair<uint32_t, FbEntry> &x, const std::pair<uint32_t, FbEntry> &y) {
            return x.first != y.first ? x.first < y.first : x.second.d < y.second.d;
        });
        // every library's entries with their windows (wpre: inside the
        // library) and filter blocks (fpre: over the whole batch)
        std::vector<FbEntry> ent(nf);
        struct Group {
            uint32_t lib, e0, ne;
            uint64_t w0, n_win;  // survivors go to fbuf + w0 (at most n_win of them)
        };
        std::vector<Group> groups;
        uint64_t n_blk = 0, w_all = 0;
        for (uint32_t i = 0; i < nf;) {
            const uint32_t j = all[i].first;
            const bool screen = p.libs[j].c >= 2;
            Group gr{j, i, 0, w_all, 0};
            for (; i < nf && all[i].first == j; i++) {
                FbEntry e = all[i].second;
                e.wpre = (uint32_t)gr.n_win;
                e.fpre = (uint32_t)n_blk;
                e.nb = screen ? (uint32_t)std::max<uint64_t>(1, ceil_div((uint64_t)p.opts.beta * e.ns, 256)) : 0u;
                gr.n_win += e.ns;
                n_blk += e.nb;
                ent[i] = e;
                gr.ne++;
            }
            w_all += gr.n_win;
            fb_per_lib[j] = gr.ne;
            groups.push_back(gr);
        }
        if (n_blk > p.fb_nb_max)
            return fail(TK_EDEVICE, "fallback filters of %llu blocks exceed the reserved %llu",
                        (unsigned long long)n_blk, (unsigned long long)p.fb_nb_max);
        FbEntry *d_ent = reinterpret_cast<FbEntry *>(ws + p.off_fb_ent);
        uint32_t *fb_counts = reinterpret_cast<uint32_t *>(ws + p.off_fbc);
        TK_HIP(hipMemcpyAsync(d_ent, ent.data(), nf * sizeof(FbEntry), hipMemcpyHostToDevice, s));
        TK_HIP(zero_bytes(lib_ctr, (size_t)L * sizeof(DevCounters), s));  // per-library fallback counters
        if (p.screen)
            TK_HIP(zero_bytes(filter, n_blk * 64, s));
        // every oversized bucket's keys to its own index range of `other`
        // (free there: the bucket kernel files records only in the ranges of
        // its groups), where they are screened and collected; `sorted`
        // becomes free
        for (const Group &gr : groups)
            TK_HIP(launch_fb_gather(sorted, other, d_ent + gr.e0, gr.ne, kw, lay, p.libs[gr.lib].seg0,
                                    p.libs[gr.lib].D2, s));
        for (const Group &gr : groups) {
            const bool screen = p.libs[gr.lib].c >= 2;
            if (screen)
                TK_HIP(launch_fb_screen(other, d_ent + gr.e0, gr.ne, gr.n_win, kw, table, p.opts.table_bits, filter,
                                        s));
            TK_HIP(launch_fb_collect(other, d_ent + gr.e0, gr.ne, gr.n_win, kw, table, p.opts.table_bits, filter,
                                     screen, fbuf + gr.w0 * kw, &lib_ctr[gr.lib].n_collected, s));
        }
        std::vector<DevCounters> fc(L);
        TK_HIP(hipMemcpyAsync(fc.data(), lib_ctr, (size_t)L * sizeof(DevCounters), hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));  // ent, fc
        // sort the survivors of each library (buckets partition its key
        // space in order), compact them and file every bucket's records
        for (const Group &gr : groups) {
            const LibDesc &lib = p.libs[gr.lib];
            const uint64_t n_surv = fc[gr.lib].n_collected;
            uint64_t *src = fbuf + gr.w0 * kw, *alt = sorted + gr.w0 * kw;
            uint64_t *srt = nullptr;
            int passes = 0;
            TK_HIP(radix_sort(src, alt, n_surv, kw, 2 * lib.k, ws + p.off_sort, p.sort_bytes, s, &srt, &passes));
            uint64_t *dst = srt == src ? alt : src;
            TK_HIP(compact(srt, n_surv, kw, lib.c, dst, fb_counts + gr.w0, ws + p.off_compact, p.compact_bytes,
                           &lib_ctr[gr.lib], s));
            TK_HIP(launch_fb_distribute(dst, fb_counts + gr.w0, &lib_ctr[gr.lib], d_ent + gr.e0, gr.ne, kw, lib.k,
                                        lib.D, lib.bucket0, other, gap_counts, rec_nout,
                                        lib_stats + 4 * (size_t)gr.lib, s));
        }
    }
    if ((st = tm.end(TK_STAGE_FALLBACK, s)) != TK_OK || (st = tm.mark(TK_STAGE_GATHER, s)) != TK_OK)
        return st;

    // records of every bucket in (library, bucket) order: final keys in
    // `sorted`, final counts in F
    uint32_t *out_counts = reinterpret_cast<uint32_t *>(fbuf);
    TK_HIP(launch_exclusive_scan(rec_nout, rec_off, p.n_buckets, rec_scan, &misc->totals[1], s));
    TK_HIP(launch_gather(rec_start, rec_nout, rec_off, p.n_buckets, other, gap_counts, kw, sorted, out_counts, s));
    TK_HIP(launch_lib_stats(d_libs, L, lib_keys, rec_off, &misc->totals[1], lib_stats, lib_ctr, lib_first, s));
    if ((st = tm.end(TK_STAGE_GATHER, s)) != TK_OK)
        return st;
    std::vector<DevCounters> h(L);
    std::vector<uint32_t> first(L);
    TK_HIP(hipMemcpyAsync(h.data(), lib_ctr, (size_t)L * sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    TK_HIP(hipMemcpyAsync(first.data(), lib_first, (size_t)L * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));

    double ms[9] = {0};
    tm.read(ms);
    for (uint32_t j = 0; j < L; j++) {
        tk_result &o = out[j];
        memset(&o, 0, sizeof o);
        o.n = h[j].n_out;
        o.k = (uint32_t)p.libs[j].k;
        o.key_words = (uint32_t)kw;
        o.keys = sorted + (size_t)first[j] * kw;
        o.counts = out_counts + first[j];
        o.n_windows = h[j].n_windows;
        o.n_collected = h[j].n_collected;
        o.n_distinct = h[j].n_runs;
        o.n_singletons = h[j].n_single;
        o.n_below_c = h[j].n_below;
        o.bloom_blocks = 0;
        o.sort_passes = 0;
        o.part_bits = p.libs[j].D;
        o.n_fallback = fb_per_lib[j];
        memcpy(o.stage_ms, ms, sizeof ms);
    }
    return TK_OK;
}

tk_status run_count(const uint8_t *d_bases, const uint64_t *d_offsets, const Plan &p, char *ws, hipStream_t s,
                    tk_result *out) {
    return p.global ? run_global(d_bases, d_offsets, p, ws, s, out)
                    : run_partitioned(d_bases, d_offsets, p, ws, s, out);
}

}  // namespace
}  // namespace tk

using namespace tk;

namespace {

// Workspace of tk_count_device_static: a file-scope device array, one copy
// per device, held until the process ends.  Host code never passes its name
// to a kernel (on the host the name is only a stand-in); it uses the device
// address from hipGetSymbolAddress, looked up once per device with that
// device current.
constexpr size_t STATIC_WORKSPACE_BYTES = TK_STATIC_WORKSPACE_BYTES;
__device__ __align__(256) unsigned char scratch[STATIC_WORKSPACE_BYTES];

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu[STATIC_MAX_DEVICES];  // one call at a time per device
void *g_static_ptr[STATIC_MAX_DEVICES];       // address of `scratch` on each device


// Runs a cleanup when the scope ends, also when a C++ exception (a failed
// host allocation inside the counting path) unwinds it; the cleanup must be
// safe to run more than once.
template <typename F>
struct OnExit {
    F f;
    ~OnExit() { f(); }
};
template <typename F>
OnExit<F> on_exit(F f) {
    return OnExit<F>{f};
}

// Entry points return a status: a C++ exception (a host allocation that
// fails, a thread that cannot start) never leaves the library.
template <typename F>
tk_status guarded(F &&body) {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(TK_ENOMEM, "host memory allocation failed");
    } catch (...) {
        return fail(TK_EDEVICE, "unexpected host-side error");
    }
}

}  // namespace

extern "C" {

tk_status tk_default_options(tk_options *opts) {
    if (!opts)
        return fail(TK_EINVAL, "opts is NULL");
    memset(opts, 0, sizeof *opts);
    opts->bloom_beta = DEF_BETA;
    opts->bloom_table_bits = DEF_TABLE_BITS;
    opts->bloom_bits = DEF_BITS;
    opts->bloom_seed = DEF_SEED;
    opts->part_bits = -1;
    return TK_OK;
}

const char *tk_strerror(tk_status st) {
    switch (st) {
    case TK_OK: return "ok";
    case TK_EINVAL: return "invalid argument";
    case TK_ENOMEM: return "out of memory";
    case TK_EDEVICE: return "device error";
    case TK_EOVERFLOW: return "input too large";
    }
    return "unknown status";
}

const char *tk_last_error(void) { return g_err; }

tk_status tk_workspace_size(uint64_t n_bases, uint64_t n_reads, int k, uint32_t c, const tk_options *opts,
                            size_t *bytes) {
    return guarded([&]() -> tk_status {
        if (!bytes)
            return fail(TK_EINVAL, "bytes is NULL");
        Plan p;
        tk_status st = make_plan(n_bases, n_reads, k, c, opts, &p);
        if (st != TK_OK)
            return st;
        *bytes = p.total;
        return TK_OK;
    });
}

tk_status tk_bloom_blocks(uint64_t n_bases, uint64_t n_reads, int k, const tk_options *opts, uint64_t *n_blocks) {
    return guarded([&]() -> tk_status {
        if (!n_blocks)
            return fail(TK_EINVAL, "n_blocks is NULL");
        if (k < 1 || k > 63)
            return fail(TK_EINVAL, "k = %d outside [1, 63]", k);
        Opts o;
        tk_status st = resolve(opts, &o);
        if (st != TK_OK)
            return st;
        *n_blocks = bloom_blocks_for(n_bases, n_reads, k, o);
        return TK_OK;
    });
}

tk_status tk_part_bits(uint64_t n_bases, uint64_t n_reads, int k, const tk_options *opts, int *part_bits) {
    return guarded([&]() -> tk_status {
        if (!part_bits)
            return fail(TK_EINVAL, "part_bits is NULL");
        if (k < 1 || k > 63)
            return fail(TK_EINVAL, "k = %d outside [1, 63]", k);
        Opts o;
        tk_status st = resolve(opts, &o);
        if (st != TK_OK)
            return st;
        *part_bits = part_bits_for(n_bases, n_reads, k, o);
        return TK_OK;
    });
}

tk_status tk_pattern_table(const tk_options *opts, uint64_t *masks, uint64_t capacity) {
    return guarded([&]() -> tk_status {
        Opts o;
        tk_status st = resolve(opts, &o);
        if (st != TK_OK)
            return st;
        const auto &t = pattern_table(o.seed, o.table_bits, o.bits);
        if (!masks || capacity < t.size())
            return fail(TK_EINVAL, "pattern table needs %zu entries", t.size());
        memcpy(masks, t.data(), t.size() * sizeof(uint64_t));
        return TK_OK;
    });
}

tk_status tk_count_device(const uint8_t *d_bases, const uint64_t *d_offsets, uint64_t n_bases, uint64_t n_reads,
                          int k, uint32_t c, const tk_options *opts, void *d_workspace, size_t ws_bytes,
                          void *stream, tk_result *out) {
    return guarded([&]() -> tk_status {
        if (!out)
            return fail(TK_EINVAL, "out is NULL");
        if (!d_offsets)
            return fail(TK_EINVAL, "offsets is NULL");
        if (n_bases && !d_bases)
            return fail(TK_EINVAL, "bases is NULL");
        if (!d_workspace)
            return fail(TK_EINVAL, "workspace is NULL");
        if ((uintptr_t)d_workspace & 255u)
            return fail(TK_EINVAL, "workspace must be 256-byte aligned");
        Plan p;
        tk_status st = make_plan(n_bases, n_reads, k, c, opts, &p);
        if (st != TK_OK)
            return st;
        if (ws_bytes < p.total)
            return fail(TK_EINVAL, "workspace of %zu bytes is below the %zu needed", ws_bytes, p.total);
        return run_count(d_bases, d_offsets, p, static_cast<char *>(d_workspace), static_cast<hipStream_t>(stream),
                         out);
    });
}

tk_status tk_count_device_static(const uint8_t *d_bases, const uint64_t *d_offsets, uint64_t n_bases,
                                 uint64_t n_reads, int k, uint32_t c, const tk_options *opts, uint64_t *d_out_keys,
                                 uint32_t *d_out_counts, uint64_t out_capacity, void *stream, tk_result *out) {
    return guarded([&]() -> tk_status {
        if (!out)
            return fail(TK_EINVAL, "out is NULL");
        if (!d_offsets)
            return fail(TK_EINVAL, "offsets is NULL");
        if (n_bases && !d_bases)
            return fail(TK_EINVAL, "bases is NULL");
        if (out_capacity && (!d_out_keys || !d_out_counts))
            return fail(TK_EINVAL, "output buffers are NULL");
        if (opts && (opts->flags & TK_FLAG_TIMING))
            return fail(TK_EINVAL, "TK_FLAG_TIMING creates events: not available without allocation");
        Plan p;
        tk_status st = make_plan(n_bases, n_reads, k, c, opts, &p);
        if (st != TK_OK)
            return st;
        if (p.total > STATIC_WORKSPACE_BYTES)
            return fail(TK_EINVAL,
                        "the library needs a workspace of %zu bytes; the static workspace holds %zu "
                        "(use tk_count_device with a workspace of its own)",
                        p.total, STATIC_WORKSPACE_BYTES);
        int dev = -1;
        TK_HIP(hipGetDevice(&dev));
        if (dev < 0 || dev >= STATIC_MAX_DEVICES)
            return fail(TK_EDEVICE, "device %d is beyond the %d the static workspace serves", dev,
                        STATIC_MAX_DEVICES);
        std::lock_guard<std::mutex> lock(g_static_mu[dev]);
        hipStream_t s = static_cast<hipStream_t>(stream);
        // whatever happens below, the stream's work on the array is finished
        // before the next call on this device may start
        auto drain = on_exit([&]() { (void)hipStreamSynchronize(s); });
        if (!g_static_ptr[dev]) {
            void *ptr = nullptr;
            TK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr || ((uintptr_t)ptr & 255u))
                return fail(TK_EDEVICE, "static workspace has no usable device address");
            g_static_ptr[dev] = ptr;
        }
        tk_result dev_res{};
        st = run_count(d_bases, d_offsets, p, static_cast<char *>(g_static_ptr[dev]), s, &dev_res);
        if (st != TK_OK)
            return st;
        if (dev_res.n > out_capacity)
            return fail(TK_EINVAL, "%llu records do not fit the output capacity of %llu",
                        (unsigned long long)dev_res.n, (unsigned long long)out_capacity);
        if (dev_res.n) {
            TK_HIP(hipMemcpyAsync(d_out_keys, dev_res.keys, dev_res.n * dev_res.key_words * sizeof(uint64_t),
                                  hipMemcpyDeviceToDevice, s));
            TK_HIP(hipMemcpyAsync(d_out_counts, dev_res.counts, dev_res.n * sizeof(uint32_t),
                                  hipMemcpyDeviceToDevice, s));
        }
        TK_HIP(hipStreamSynchronize(s));
        dev_res.keys = d_out_keys;
        dev_res.counts = d_out_counts;
        *out = dev_res;
        return TK_OK;
    });
}

tk_status tk_batch_workspace_size(uint64_t n_libs, const uint64_t *lib_bases, const uint64_t *lib_reads,
                                  const int *k, const uint32_t *c, const tk_options *opts, size_t *bytes) {
    return guarded([&]() -> tk_status {
        if (!bytes)
            return fail(TK_EINVAL, "bytes is NULL");
        BatchPlan bp;
        tk_status st = make_batch_plan(n_libs, lib_bases, lib_reads, k, c, opts, &bp);
        if (st != TK_OK)
            return st;
        *bytes = bp.total;
        return TK_OK;
    });
}

tk_status tk_count_batch_device(const uint8_t *d_bases, const uint64_t *d_offsets, uint64_t n_libs,
                                const uint64_t *lib_bases, const uint64_t *lib_reads, const int *k, const uint32_t *c,
                                const tk_options *opts, void *d_workspace, size_t ws_bytes, void *stream,
                                tk_result *out) {
    return guarded([&]() -> tk_status {
        if (!out)
            return fail(TK_EINVAL, "out is NULL");
        if (!d_offsets)
            return fail(TK_EINVAL, "offsets is NULL");
        if (!d_workspace)
            return fail(TK_EINVAL, "workspace is NULL");
        if ((uintptr_t)d_workspace & 255u)
            return fail(TK_EINVAL, "workspace must be 256-byte aligned");
        BatchPlan bp;
        tk_status st = make_batch_plan(n_libs, lib_bases, lib_reads, k, c, opts, &bp);
        if (st != TK_OK)
            return st;
        if (lib_bases[n_libs] && !d_bases)
            return fail(TK_EINVAL, "bases is NULL");
        if (ws_bytes < bp.total)
            return fail(TK_EINVAL, "workspace of %zu bytes is below the %zu needed", ws_bytes, bp.total);
        // one counting pass per key width, one after the other on the stream,
        // each in its own part of the workspace
        double ms[TK_STAGE_COUNT] = {0};
        std::vector<tk_result> part;
        for (size_t q = 0; q < bp.plans.size(); q++) {
            part.assign(bp.member[q].size(), tk_result{});
            st = run_partitioned(d_bases, d_offsets, bp.plans[q], static_cast<char *>(d_workspace) + bp.ws_off[q],
                                 static_cast<hipStream_t>(stream), part.data());
            if (st != TK_OK)
                return st;
            for (size_t i = 0; i < part.size(); i++)
                out[bp.member[q][i]] = part[i];
            for (int t = 0; t < TK_STAGE_COUNT; t++)
                ms[t] += part.empty() ? 0.0 : part[0].stage_ms[t];
        }
        for (uint64_t j = 0; j < n_libs; j++)
            memcpy(out[j].stage_ms, ms, sizeof ms);
        return TK_OK;
    });
}

tk_status tk_count(const uint8_t *bases, const uint64_t *offsets, uint64_t n_reads, int k, uint32_t c,
                   const tk_options *opts, tk_result **out) {
    return guarded([&]() -> tk_status {
        if (!out)
            return fail(TK_EINVAL, "out is NULL");
        if (!offsets)
            return fail(TK_EINVAL, "offsets is NULL");
        if (offsets[0] != 0)
            return fail(TK_EINVAL, "offsets[0] must be 0");
        for (uint64_t r = 0; r < n_reads; r++)
            if (offsets[r + 1] < offsets[r])
                return fail(TK_EINVAL, "offsets decrease at read %llu", (unsigned long long)r);
        const uint64_t n_bases = offsets[n_reads];
        if (n_bases && !bases)
            return fail(TK_EINVAL, "bases is NULL");
        Plan p;
        tk_status st = make_plan(n_bases, n_reads, k, c, opts, &p);
        if (st != TK_OK)
            return st;
    
        uint8_t *d_bases = nullptr;
        uint64_t *d_offsets = nullptr;
        void *d_ws = nullptr;
        tk_result *res = nullptr;
        hipStream_t s = nullptr;
        Stager stage;  // pinned slices of the host copies
        auto cleanup = [&]() {  // idempotent: also runs when the scope ends
            (void)stage.release();
            if (s) (void)hipStreamSynchronize(s);
            if (d_bases) (void)hipFree(d_bases);
            if (d_offsets) (void)hipFree(d_offsets);
            if (d_ws) (void)hipFree(d_ws);
            if (s) (void)hipStreamDestroy(s);
            d_bases = nullptr;
            d_offsets = nullptr;
            d_ws = nullptr;
            s = nullptr;
        };
        auto guard = on_exit(cleanup);
        auto dev_fail = [&](const char *what, hipError_t e) {
            cleanup();
            if (res) {
                free(res->keys);
                free(res->counts);
                free(res);
            }
            if (e == hipErrorOutOfMemory)
                return fail(TK_ENOMEM, "%s: %s", what, hipGetErrorString(e));
            return fail(TK_EDEVICE, "%s: %s", what, hipGetErrorString(e));
        };
        hipError_t e;
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
            return dev_fail("hipStreamCreate", e);
        if ((e = hipMalloc(&d_bases, n_bases ? n_bases : 1)) != hipSuccess)
            return dev_fail("hipMalloc(bases)", e);
        if ((e = hipMalloc(&d_offsets, (n_reads + 1) * sizeof(uint64_t))) != hipSuccess)
            return dev_fail("hipMalloc(offsets)", e);
        if ((e = hipMalloc(&d_ws, p.total ? p.total : 256)) != hipSuccess)
            return dev_fail("hipMalloc(workspace)", e);
        if ((e = stage.copy(d_bases, bases, n_bases, true, s)) != hipSuccess)
            return dev_fail("copy of the reads", e);
        if ((e = hipMemcpyAsync(d_offsets, offsets, (n_reads + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return dev_fail("hipMemcpy(offsets)", e);
    
        tk_result dev{};
        st = run_count(d_bases, d_offsets, p, static_cast<char *>(d_ws), s, &dev);
        if (st != TK_OK) {
            cleanup();
            return st;
        }
        res = static_cast<tk_result *>(calloc(1, sizeof(tk_result)));
        if (!res) {
            cleanup();
            return fail(TK_ENOMEM, "result allocation failed");
        }
        *res = dev;
        res->keys = static_cast<uint64_t *>(malloc((dev.n ? dev.n : 1) * dev.key_words * sizeof(uint64_t)));
        res->counts = static_cast<uint32_t *>(malloc((dev.n ? dev.n : 1) * sizeof(uint32_t)));
        if (!res->keys || !res->counts) {
            cleanup();
            free(res->keys);
            free(res->counts);
            free(res);
            return fail(TK_ENOMEM, "result allocation failed");
        }
        if ((e = stage.copy(res->keys, dev.keys, dev.n * dev.key_words * sizeof(uint64_t), false, s)) != hipSuccess)
            return dev_fail("copy of the keys", e);
        if ((e = stage.copy(res->counts, dev.counts, dev.n * sizeof(uint32_t), false, s)) != hipSuccess)
            return dev_fail("copy of the counts", e);
        if ((e = hipStreamSynchronize(s)) != hipSuccess)
            return dev_fail("hipStreamSynchronize", e);
        cleanup();
        *out = res;
        return TK_OK;
    });
}

tk_status tk_count_phased(const uint8_t *bases, const uint64_t *offsets, uint64_t n_reads, int k, uint32_t c,
                          uint64_t chunk_bases, uint64_t sac_capacity, const tk_options *opts, tk_result **out,
                          size_t *device_bytes) {
    return guarded([&]() -> tk_status {
        if (!out)
            return fail(TK_EINVAL, "out is NULL");
        if (!offsets)
            return fail(TK_EINVAL, "offsets is NULL");
        if (offsets[0] != 0)
            return fail(TK_EINVAL, "offsets[0] must be 0");
        for (uint64_t r = 0; r < n_reads; r++)
            if (offsets[r + 1] < offsets[r])
                return fail(TK_EINVAL, "offsets decrease at read %llu", (unsigned long long)r);
        if (k < 1 || k > 63)
            return fail(TK_EINVAL, "k = %d outside [1, 63]", k);
        if (c == 0)
            return fail(TK_EINVAL, "threshold c must be >= 1");
        if (chunk_bases == 0)
            return fail(TK_EINVAL, "chunk_bases must be >= 1");
        const uint64_t n_bases = offsets[n_reads];
        if (n_bases && !bases)
            return fail(TK_EINVAL, "bases is NULL");
        if (n_bases >= (1ull << 32))
            return fail(TK_EOVERFLOW, "n_bases = %llu must be below 2^32", (unsigned long long)n_bases);
        Opts o;
        tk_status st = resolve(opts, &o);
        if (st != TK_OK)
            return st;
        if (o.shard_count > 1)
            return fail(TK_EINVAL, "key-range shards need the partitioned path");
        const int kw = k <= 31 ? 1 : 2;
        const size_t kb = 8 * (size_t)kw;
        const bool screen = c >= 2;
        // chunks: consecutive reads of at most chunk_bases bases (a longer read
        // alone)
        std::vector<uint64_t> cuts{0};
        uint64_t cb_max = 0, cr_max = 0;
        for (uint64_t r0 = 0; r0 < n_reads;) {
            uint64_t r1 = r0 + 1;
            while (r1 < n_reads && offsets[r1 + 1] - offsets[r0] <= chunk_bases)
                r1++;
            cb_max = std::max(cb_max, offsets[r1] - offsets[r0]);
            cr_max = std::max(cr_max, r1 - r0);
            cuts.push_back(r1);
            r0 = r1;
        }
        const uint64_t n_chunks = cuts.size() - 1;
        const uint64_t CB = std::max<uint64_t>(cb_max, 1), CW = ceil_div(CB, 32);
        const uint64_t sac_cap = sac_capacity ? sac_capacity : std::max<uint64_t>(n_bases, 1);
        const uint64_t n_blocks = screen ? bloom_blocks_for(n_bases, n_reads, k, o) : 0;
        const uint64_t merged = sac_cap + CB;  // records of one merge
        // device memory
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t r = off;
            off = align_up(off + bytes, 256);
            return r;
        };
        const size_t o_ctr = take(2 * sizeof(DevCounters)), o_misc = take(64), o_table = take(sizeof(uint64_t) << o.table_bits);
        const size_t o_filter = take(n_blocks * 64), o_bases = take(CB), o_offs = take((cr_max + 1) * sizeof(uint64_t));
        const size_t o_packed = take(CW * 8), o_valid = take(CW * 4), o_starts = take(CW * 4);
        // second packed/valid buffer: the next chunk's words arrive while this
        // chunk is collected (second pass)
        const size_t o_packed2 = screen ? take(CW * 8) : 0, o_valid2 = screen ? take(CW * 4) : 0;
        const size_t o_ka = take(CB * kb), o_kb = take(CB * kb), o_rk = take(CB * kb), o_rc = take(CB * 4);
        const size_t sort_bytes = radix_scratch_bytes(CB, kw), cmp_bytes = compact_scratch_bytes(CB);
        const size_t o_sort = take(sort_bytes), o_cmp = take(cmp_bytes);
        const size_t o_sk[2] = {take(merged * kb), take(merged * kb)}, o_sc[2] = {take(merged * 4), take(merged * 4)};
        const size_t o_tk = take(merged * kb), o_tc = take(merged * 4), o_flag = take(2 * merged * 4);
        const size_t o_scan = take(scan_scratch_words(2 * merged) * 4);
        const size_t total = off;
        if (device_bytes)
            *device_bytes = total;
    
        // packed words and validity bits of every chunk, kept in pinned host
        // memory between the passes (0.5 B per base instead of the 1 B per base
        // of the reads, and no pageable staging in the second pass)
        std::vector<uint64_t> wfirst(n_chunks + 1, 0);  // first word of every chunk in the pinned arrays
        for (uint64_t q = 0; q < n_chunks; q++)
            wfirst[q + 1] = wfirst[q] + ceil_div(offsets[cuts[q + 1]] - offsets[cuts[q]], 32);
    
        char *ws = nullptr;
        hipStream_t s = nullptr, cs = nullptr;  // kernels; copies of the next chunk
        hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
        uint64_t *h_packed = nullptr;
        uint32_t *h_valid = nullptr;
        uint64_t *h_roff = nullptr;  // relative read offsets of two chunks (pinned)
        Stager up;                   // pinned slices of the reads' and the answer's copies
        tk_result *res = nullptr;
        auto cleanup = [&]() {  // idempotent: also runs when the scope ends
            (void)up.release();
            if (s) (void)hipStreamSynchronize(s);
            if (cs) (void)hipStreamSynchronize(cs);
            if (ws) (void)hipFree(ws);
            for (hipEvent_t &e : ev) {
                if (e) (void)hipEventDestroy(e);
                e = nullptr;
            }
            if (h_packed) (void)hipHostFree(h_packed);
            if (h_valid) (void)hipHostFree(h_valid);
            if (h_roff) (void)hipHostFree(h_roff);
            if (cs) (void)hipStreamDestroy(cs);
            if (s) (void)hipStreamDestroy(s);
            ws = nullptr;
            h_packed = nullptr;
            h_valid = nullptr;
            h_roff = nullptr;
            cs = nullptr;
            s = nullptr;
        };
        auto guard = on_exit(cleanup);
        auto dev_fail = [&](const char *what, hipError_t e) {
            cleanup();
            if (res) {
                free(res->keys);
                free(res->counts);
                free(res);
            }
            if (e == hipErrorOutOfMemory)
                return fail(TK_ENOMEM, "%s: %s", what, hipGetErrorString(e));
            return fail(TK_EDEVICE, "%s: %s", what, hipGetErrorString(e));
        };
    #define TK_PH(call, what)                   \
        do {                                    \
            hipError_t e_ = (call);             \
            if (e_ != hipSuccess)               \
                return dev_fail(what, e_);      \
        } while (0)
        TK_PH(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
        TK_PH(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
        for (hipEvent_t &e : ev)
            TK_PH(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        TK_PH(hipHostMalloc(reinterpret_cast<void **>(&h_roff), 2 * (cr_max + 1) * sizeof(uint64_t)), "hipHostMalloc");
        if (screen && wfirst[n_chunks]) {
            TK_PH(hipHostMalloc(reinterpret_cast<void **>(&h_packed), wfirst[n_chunks] * sizeof(uint64_t)),
                  "hipHostMalloc(packed)");
            TK_PH(hipHostMalloc(reinterpret_cast<void **>(&h_valid), wfirst[n_chunks] * sizeof(uint32_t)),
                  "hipHostMalloc(valid)");
        }
        TK_PH(hipMalloc(&ws, total), "hipMalloc(workspace)");
        DevCounters *ctr = reinterpret_cast<DevCounters *>(ws + o_ctr);  // [0] windows, collected; [1] chunk compaction
        uint32_t *misc = reinterpret_cast<uint32_t *>(ws + o_misc);        // [0] SAC size, [1] selected
        unsigned long long *stats = reinterpret_cast<unsigned long long *>(ws + o_misc + 16);
        uint64_t *table = reinterpret_cast<uint64_t *>(ws + o_table);
        uint64_t *filter = reinterpret_cast<uint64_t *>(ws + o_filter);
        uint8_t *d_bases = reinterpret_cast<uint8_t *>(ws + o_bases);
        uint64_t *d_offs = reinterpret_cast<uint64_t *>(ws + o_offs);
        uint64_t *packed = reinterpret_cast<uint64_t *>(ws + o_packed);
        uint32_t *valid = reinterpret_cast<uint32_t *>(ws + o_valid), *starts = reinterpret_cast<uint32_t *>(ws + o_starts);
        uint64_t *packed2[2] = {packed, reinterpret_cast<uint64_t *>(ws + o_packed2)};
        uint32_t *valid2[2] = {valid, reinterpret_cast<uint32_t *>(ws + o_valid2)};
        uint64_t *keys_a = reinterpret_cast<uint64_t *>(ws + o_ka), *keys_b = reinterpret_cast<uint64_t *>(ws + o_kb);
        uint64_t *run_k = reinterpret_cast<uint64_t *>(ws + o_rk);
        uint32_t *run_c = reinterpret_cast<uint32_t *>(ws + o_rc);
        uint64_t *sac_k[2] = {reinterpret_cast<uint64_t *>(ws + o_sk[0]), reinterpret_cast<uint64_t *>(ws + o_sk[1])};
        uint32_t *sac_c[2] = {reinterpret_cast<uint32_t *>(ws + o_sc[0]), reinterpret_cast<uint32_t *>(ws + o_sc[1])};
        uint64_t *tmp_k = reinterpret_cast<uint64_t *>(ws + o_tk);
        uint32_t *tmp_c = reinterpret_cast<uint32_t *>(ws + o_tc), *flag = reinterpret_cast<uint32_t *>(ws + o_flag);
        uint32_t *scan_tmp = reinterpret_cast<uint32_t *>(ws + o_scan);
        TK_PH(zero_bytes(ws, o_table, s), "zero");  // counters and misc
        if (screen) {
            const auto &tab = pattern_table(o.seed, o.table_bits, o.bits);
            TK_PH(hipMemcpyAsync(table, tab.data(), tab.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s), "table");
            TK_PH(zero_bytes(filter, n_blocks * 64, s), "zero filter");
        }
        BloomArgs ba{};
        ba.packed = packed;
        ba.valid = valid;
        ba.k = k;
        ba.table = table;
        ba.table_bits = o.table_bits;
        ba.n_blocks = n_blocks;
        ba.filter = filter;
        // Chunk q's reads and relative read offsets go to the device on the copy
        // stream (offsets staged in pinned slot q % 2) while the kernel stream
        // still screens the chunk before; pack then runs on the kernel stream.
        // ev[0]: chunk copied; ev[1]: chunk packed (its reads are consumed, so
        // the next chunk may overwrite them; the host waits for it, whatever the
        // runtime does with pageable sources); ev[2 + q % 2]: the offsets of
        // slot q % 2 are on the device.
        auto send_chunk = [&](uint64_t q) -> hipError_t {
            const uint64_t r0 = cuts[q], r1 = cuts[q + 1], b0 = offsets[r0], nb = offsets[r1] - b0;
            uint64_t *ro = h_roff + (q % 2) * (cr_max + 1);
            hipError_t e = hipEventSynchronize(ev[2 + q % 2]);  // slot free (chunk q - 2 sent)
            if (e != hipSuccess)
                return e;
            for (uint64_t r = r0; r <= r1; r++)
                ro[r - r0] = offsets[r] - b0;
            if ((e = hipEventSynchronize(ev[1])) != hipSuccess)
                return e;
            if ((e = up.copy(d_bases, bases + b0, nb, true, cs)) != hipSuccess)
                return e;
            if ((e = hipMemcpyAsync(d_offs, ro, (r1 - r0 + 1) * 8, hipMemcpyHostToDevice, cs)) != hipSuccess)
                return e;
            if ((e = hipEventRecord(ev[2 + q % 2], cs)) != hipSuccess)
                return e;
            return hipEventRecord(ev[0], cs);
        };
        auto pack_chunk = [&](uint64_t q, bool count) -> hipError_t {
            const uint64_t nb = offsets[cuts[q + 1]] - offsets[cuts[q]];
            hipError_t e = hipStreamWaitEvent(s, ev[0], 0);
            if (e != hipSuccess || (e = zero_bytes(starts, CW * 4, s)) != hipSuccess)
                return e;
            ba.packed = packed;
            ba.valid = valid;
            ba.n_words = ceil_div(nb, 32);
            e = launch_pack(d_bases, d_offs, nb, cuts[q + 1] - cuts[q], k, packed, valid, starts,
                            count ? &ctr[0].n_windows : nullptr, s);
            if (e == hipSuccess)
                e = hipEventRecord(ev[1], s);
            return e;
        };
        // pass 1: every window of every chunk into the filter; the next chunk's
        // reads travel while this one is screened; the packed words are kept
        if (screen) {
            if (n_chunks)
                TK_PH(send_chunk(0), "pass 1");
            for (uint64_t q = 0; q < n_chunks; q++) {
                TK_PH(pack_chunk(q, true), "pass 1");
                const uint64_t nw = wfirst[q + 1] - wfirst[q];
                TK_PH(launch_screen(ba, persistent_grid(ba.n_words * 32), s), "screen");
                if (nw) {
                    TK_PH(hipMemcpyAsync(h_packed + wfirst[q], packed, nw * 8, hipMemcpyDeviceToHost, s), "keep");
                    TK_PH(hipMemcpyAsync(h_valid + wfirst[q], valid, nw * 4, hipMemcpyDeviceToHost, s), "keep");
                }
                if (q + 1 < n_chunks)
                    TK_PH(send_chunk(q + 1), "pass 1");
            }
            // the pinned words are complete before the second pass reads them
            TK_PH(hipEventRecord(ev[1], s), "record");
            TK_PH(hipStreamWaitEvent(cs, ev[1], 0), "wait");
        }
        // second pass input of chunk q: packed words and validity bits from
        // pinned memory into buffer q % 2 (screen), or the reads, packed again
        auto second_pass_input = [&](uint64_t q) -> hipError_t {
            const uint64_t nw = wfirst[q + 1] - wfirst[q];
            hipError_t e;
            if (nw && (e = hipMemcpyAsync(packed2[q % 2], h_packed + wfirst[q], nw * 8, hipMemcpyHostToDevice, cs)) !=
                          hipSuccess)
                return e;
            if (nw && (e = hipMemcpyAsync(valid2[q % 2], h_valid + wfirst[q], nw * 4, hipMemcpyHostToDevice, cs)) !=
                          hipSuccess)
                return e;
            return hipEventRecord(ev[q % 2], cs);
        };
        // pass 2: per chunk, collect, sort, compact, merge into the SAC
        uint64_t n_sac = 0, n_coll = 0;
        int cur = 0;
        if (screen && n_chunks)
            TK_PH(second_pass_input(0), "pass 2");
        for (uint64_t q = 0; q < n_chunks; q++) {
            if (screen) {
                // buffer (q + 1) % 2 was last read by chunk q - 1, whose collect
                // finished before its survivor count was read back
                if (q + 1 < n_chunks)
                    TK_PH(second_pass_input(q + 1), "pass 2");
                TK_PH(hipStreamWaitEvent(s, ev[q % 2], 0), "wait");
                ba.packed = packed2[q % 2];
                ba.valid = valid2[q % 2];
                ba.n_words = wfirst[q + 1] - wfirst[q];
            } else {
                TK_PH(send_chunk(q), "pass 2");
                TK_PH(pack_chunk(q, true), "pass 2");
            }
            TK_PH(zero_bytes(&ctr[1], sizeof(DevCounters), s), "zero");
            TK_PH(launch_collect(ba, screen, keys_a, CB, &ctr[1].n_collected, persistent_grid(ba.n_words * 32), s),
                  "collect");
            unsigned long long n_surv = 0;
            TK_PH(hipMemcpyAsync(&n_surv, &ctr[1].n_collected, 8, hipMemcpyDeviceToHost, s), "read");
            TK_PH(hipStreamSynchronize(s), "sync");
            n_coll += n_surv;
            uint64_t *srt = nullptr;
            int passes = 0;
            TK_PH(radix_sort(keys_a, keys_b, n_surv, kw, 2 * k, ws + o_sort, sort_bytes, s, &srt, &passes), "sort");
            TK_PH(compact(srt, n_surv, kw, 1, run_k, run_c, ws + o_cmp, cmp_bytes, &ctr[1], s), "compact");
            unsigned long long n_runs = 0;
            TK_PH(hipMemcpyAsync(&n_runs, &ctr[1].n_out, 8, hipMemcpyDeviceToHost, s), "read");
            TK_PH(hipStreamSynchronize(s), "sync");
            TK_PH(merge_compact(sac_k[cur], sac_c[cur], n_sac, run_k, run_c, n_runs, kw, tmp_k, tmp_c, flag, scan_tmp,
                                sac_k[1 - cur], sac_c[1 - cur], &misc[0], s),
                  "merge");
            uint32_t ns = 0;
            TK_PH(hipMemcpyAsync(&ns, &misc[0], 4, hipMemcpyDeviceToHost, s), "read");
            TK_PH(hipStreamSynchronize(s), "sync");
            n_sac = ns;
            cur = 1 - cur;
            if (n_sac > sac_cap) {
                cleanup();
                return fail(TK_ENOMEM, "%llu counted k-mers exceed the sorted-and-compacted array of %llu",
                            (unsigned long long)n_sac, (unsigned long long)sac_cap);
            }
        }
        // the answer: records with count >= c
        TK_PH(select_records(sac_k[cur], sac_c[cur], n_sac, kw, c, flag, scan_tmp, tmp_k, tmp_c, &misc[1], stats, s),
              "select");
        uint32_t n_out = 0;
        unsigned long long st2[2] = {0, 0}, n_win = 0;
        TK_PH(hipMemcpyAsync(&n_out, &misc[1], 4, hipMemcpyDeviceToHost, s), "read");
        TK_PH(hipMemcpyAsync(st2, stats, 16, hipMemcpyDeviceToHost, s), "read");
        TK_PH(hipMemcpyAsync(&n_win, &ctr[0].n_windows, 8, hipMemcpyDeviceToHost, s), "read");
        TK_PH(hipStreamSynchronize(s), "sync");
        res = static_cast<tk_result *>(calloc(1, sizeof(tk_result)));
        if (!res) {
            cleanup();
            return fail(TK_ENOMEM, "result allocation failed");
        }
        res->n = n_out;
        res->k = (uint32_t)k;
        res->key_words = (uint32_t)kw;
        res->n_windows = n_win;
        res->n_collected = n_coll;
        res->n_distinct = n_sac;
        res->n_singletons = st2[0];
        res->n_below_c = st2[1];
        res->bloom_blocks = n_blocks;
        res->part_bits = -1;
        res->keys = static_cast<uint64_t *>(malloc((n_out ? n_out : 1) * kb));
        res->counts = static_cast<uint32_t *>(malloc((n_out ? n_out : 1) * sizeof(uint32_t)));
        if (!res->keys || !res->counts)
            return dev_fail("result allocation", hipErrorOutOfMemory);
        TK_PH(up.copy(res->keys, tmp_k, n_out * kb, false, s), "copy keys");
        TK_PH(up.copy(res->counts, tmp_c, n_out * 4, false, s), "copy counts");
        TK_PH(hipStreamSynchronize(s), "sync");
    #undef TK_PH
        cleanup();
        *out = res;
        return TK_OK;
    });
}

void tk_result_free(tk_result *res) {
    if (!res)
        return;
    free(res->keys);
    free(res->counts);
    free(res);
}

tk_status tk_pack_device(const uint8_t *d_bases, const uint64_t *d_offsets, uint64_t n_bases, uint64_t n_reads,
                         int k, uint64_t *d_packed, uint32_t *d_valid, uint32_t *d_scratch,
                         uint64_t *d_n_windows, void *stream) {
    return guarded([&]() -> tk_status {
        if (k < 1 || k > 63)
            return fail(TK_EINVAL, "k = %d outside [1, 63]", k);
        if (n_bases >= (1ull << 32))
            return fail(TK_EOVERFLOW, "n_bases must be below 2^32");
        if (!d_offsets || !d_n_windows || (n_bases && (!d_bases || !d_packed || !d_valid || !d_scratch)))
            return fail(TK_EINVAL, "NULL device pointer");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const uint64_t n_words = ceil_div(n_bases, 32);
        TK_HIP(zero_bytes(d_n_windows, 8, s));
        if ((uintptr_t)d_n_windows & 7u || (uintptr_t)d_scratch & 3u)
            return fail(TK_EINVAL, "misaligned device pointer");
        TK_HIP(zero_bytes(d_scratch, n_words * 4, s));
        TK_HIP(launch_pack(d_bases, d_offsets, n_bases, n_reads, k, d_packed, d_valid, d_scratch,
                           reinterpret_cast<unsigned long long *>(d_n_windows), s));
        return TK_OK;
    });
}

tk_status tk_sort_scratch_size(uint64_t n, int key_words, size_t *bytes) {
    return guarded([&]() -> tk_status {
        if (!bytes || (key_words != 1 && key_words != 2))
            return fail(TK_EINVAL, "bad arguments");
        *bytes = radix_scratch_bytes(n, key_words);
        return TK_OK;
    });
}

tk_status tk_sort_keys_device(uint64_t *d_keys, uint64_t *d_alt, uint64_t n, int key_words, int key_bits,
                              void *d_scratch, size_t scratch_bytes, void *stream, uint64_t **d_sorted_out) {
    return guarded([&]() -> tk_status {
        if (key_words != 1 && key_words != 2)
            return fail(TK_EINVAL, "key_words must be 1 or 2");
        if (key_bits < 0 || key_bits > 64 * key_words)
            return fail(TK_EINVAL, "key_bits out of range");
        if (!d_sorted_out || (n && (!d_keys || !d_alt || !d_scratch)))
            return fail(TK_EINVAL, "NULL pointer");
        if (n >= (1ull << 32))
            return fail(TK_EOVERFLOW, "at most 2^32 - 1 keys");
        if (scratch_bytes < radix_scratch_bytes(n, key_words))
            return fail(TK_EINVAL, "scratch too small");
        int passes = 0;
        TK_HIP(radix_sort(d_keys, d_alt, n, key_words, key_bits, d_scratch, scratch_bytes,
                          static_cast<hipStream_t>(stream), d_sorted_out, &passes));
        return TK_OK;
    });
}

tk_status tk_compact_scratch_size(uint64_t n, size_t *bytes) {
    return guarded([&]() -> tk_status {
        if (!bytes)
            return fail(TK_EINVAL, "bytes is NULL");
        *bytes = align_up(sizeof(DevCounters), 256) + compact_scratch_bytes(n);
        return TK_OK;
    });
}

tk_status tk_compact_device(const uint64_t *d_keys, uint64_t n, int key_words, uint32_t c, uint64_t *d_out_keys,
                            uint32_t *d_out_counts, void *d_scratch, size_t scratch_bytes, void *stream,
                            uint64_t stats[4]) {
    return guarded([&]() -> tk_status {
        if (key_words != 1 && key_words != 2)
            return fail(TK_EINVAL, "key_words must be 1 or 2");
        if (c == 0)
            return fail(TK_EINVAL, "threshold c must be >= 1");
        if (!stats || !d_scratch || (n && (!d_keys || !d_out_keys || !d_out_counts)))
            return fail(TK_EINVAL, "NULL pointer");
        if ((uintptr_t)d_scratch & 255u)
            return fail(TK_EINVAL, "scratch must be 256-byte aligned");
        if (n >= (1ull << 32))
            return fail(TK_EOVERFLOW, "at most 2^32 - 1 keys");
        const size_t head = align_up(sizeof(DevCounters), 256);
        if (scratch_bytes < head + compact_scratch_bytes(n))
            return fail(TK_EINVAL, "scratch too small");
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevCounters *ctr = static_cast<DevCounters *>(d_scratch);
        TK_HIP(zero_bytes(ctr, sizeof(DevCounters), s));
        TK_HIP(compact(d_keys, n, key_words, c, d_out_keys, d_out_counts, static_cast<char *>(d_scratch) + head,
                       scratch_bytes - head, ctr, s));
        DevCounters h{};
        TK_HIP(hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        stats[0] = h.n_out;
        stats[1] = h.n_runs;
        stats[2] = h.n_single;
        stats[3] = h.n_below;
        return TK_OK;
    });
}

}  // extern "C"
