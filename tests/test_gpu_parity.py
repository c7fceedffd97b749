"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every comparison is bit-exact (integer work): keys, counts, order, the number
of valid windows, and the screen's statistics (collected occurrences,
distinct candidates, false positives) against the oracle's Bloom model.
"""
import sys

import numpy as np
import pytest

import readsim
from oracle import brute

pytestmark = pytest.mark.gpu

KS = [1, 2, 3, 4, 5, 15, 21, 31, 32, 33, 55, 63]


def case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1305_1861_amd as tk
    tk.load_library()
    return tk


def to_device(bases, offsets, shift=0):
    """Device copies; `shift` > 0 places the bases at a misaligned address."""
    import torch
    b = torch.zeros(bases.size + shift + 1, dtype=torch.uint8)
    b[shift:shift + bases.size] = torch.from_numpy(bases)
    db = b.cuda()[shift:shift + bases.size]
    do = torch.from_numpy(offsets.astype(np.uint64).view(np.int64)).cuda()
    return db, do


def gpu_count(tk, bases, offsets, k, c, opts=None, shift=0):
    import torch
    db, do = to_device(bases, offsets, shift)
    r = tk.tk_count_device(db, do, k, c, opts)
    torch.cuda.synchronize()
    keys = r.keys.cpu().numpy().view(np.uint64).reshape(r.n, r.key_words)
    counts = r.counts.cpu().numpy().view(np.uint32)
    return keys, counts, r


def assert_same(keys, counts, res, k):
    if k <= 31:
        assert keys.shape[1] == 1
        assert not res.hi.any()
        got = keys[:, 0]
        assert got.size == res.lo.size, (got.size, res.lo.size)
        assert (got == res.lo).all()
    else:
        assert keys.shape[1] == 2
        assert keys.shape[0] == res.lo.size, (keys.shape[0], res.lo.size)
        assert (keys[:, 0] == res.hi).all() and (keys[:, 1] == res.lo).all()
    assert (counts.astype(np.uint64) == res.count).all()


def expected_bloom(oracle_lib, bases, offsets, k, opts=None):
    """The oracle's Bloom statistics for the filter layout these options select."""
    opts = dict(opts or {})
    n_reads = offsets.size - 1
    beta = opts.get("bloom_beta", 4)
    tb = 1 << opts.get("bloom_table_bits", 10)
    bits = opts.get("bloom_bits", 2)
    seed = opts.get("bloom_seed", 1305)
    if opts.get("flags", 0) & 2:  # one global filter
        nb = opts.get("bloom_blocks") or oracle_lib.default_blocks(bases.size, n_reads, k, beta)
        return oracle_lib.bloom_model(bases, offsets, k, nb, tb, bits, seed), nb, -1
    D = oracle_lib.partition_bits(bases.size, n_reads, k, opts.get("part_bits", -1))
    return oracle_lib.bloom_model_buckets(bases, offsets, k, D, beta, tb, bits, seed), 0, D


def check_against_oracle(tk, oracle_lib, bases, offsets, k, c, shift=0, opts=None):
    keys, counts, r = gpu_count(tk, bases, offsets, k, c, opts=opts, shift=shift)
    ora = oracle_lib.kmer_count(bases, offsets, k, c)
    assert_same(keys, counts, ora, k)
    assert r.n_windows == ora.n_windows
    if c == 1:
        assert r.n_collected == ora.n_windows
        assert r.n_distinct == ora.n_distinct
        assert r.bloom_blocks == 0
    else:
        m, nb, D = expected_bloom(oracle_lib, bases, offsets, k, opts)
        assert r.bloom_blocks == nb and r.part_bits == D
        assert (r.n_collected, r.n_distinct, r.n_singletons) == (m.n_cand_occ, m.n_cand, m.n_cand_single)
        all2 = oracle_lib.kmer_count(bases, offsets, k, 2)
        assert r.n_below_c == int(((all2.count >= 2) & (all2.count < c)).sum())
    return r


GLOBAL = dict(flags=2)


def library(seed, n_reads, max_len, k, dup=0.3):
    bases, offsets = readsim.random_reads(seed, n_reads, 0, max_len, n_rate=0.01,
                                          lower_rate=0.02, junk_rate=0.002)
    reads = readsim.to_strings(bases, offsets)
    reads = reads + reads[: int(len(reads) * dup)] + \
        [brute.revcomp(brute.ascii_upper(x)) for x in reads[: int(len(reads) * dup / 2)]]
    return readsim.from_strings(reads)


# --------------------------------------------------------------------------
# stages
# --------------------------------------------------------------------------

def host_pack(bases, offsets, k):
    """Packed words and window-validity bits from the documented layout."""
    n = bases.size
    n_words = (n + 31) // 32
    up = bases & 0xDF
    code = np.zeros(n, np.uint64)
    code[up == ord("C")] = 1
    code[up == ord("G")] = 2
    code[up == ord("T")] = 3
    isbase = np.isin(up, np.frombuffer(b"ACGT", np.uint8))
    packed = np.zeros(n_words, np.uint64)
    pos = np.arange(n)
    np.bitwise_or.at(packed, pos // 32, code << (np.uint64(62) - np.uint64(2) * (pos % 32).astype(np.uint64)))
    valid = np.zeros(n_words, np.uint64)
    for r in range(offsets.size - 1):
        a, b = int(offsets[r]), int(offsets[r + 1])
        run = 0
        for p in range(a, b):
            run = run + 1 if isbase[p] else 0
            if run >= k:
                valid[p // 32] |= np.uint64(1) << np.uint64(p % 32)
    return packed, valid.astype(np.uint32)


@pytest.mark.parametrize("k", [1, 5, 31, 32, 63])
def test_pack_stage(tk, oracle_lib, k):
    bases, offsets = library(7 + k, 400, 3 * k + 20, k)
    case(f"pack k={k} n_bases={bases.size}")
    db, do = to_device(bases, offsets)
    packed, valid, nw = tk.tk_pack_device(db, do, k)
    hp, hv = host_pack(bases, offsets, k)
    gp = packed.cpu().numpy().view(np.uint64)
    gv = valid.cpu().numpy().view(np.uint32)
    assert (gp == hp).all()
    assert (gv == hv).all()
    assert int(nw.cpu().item()) == oracle_lib.count_windows(bases, offsets, k)


def word_edge_library(k, seed):
    """Reads whose starts, ends and N bases fall at every offset around the
    32-base words: lengths about k and about multiples of 32, one N at each
    position of a 96-base read, and single bases between them, shuffled;
    every read twice."""
    rng = np.random.default_rng(seed)
    rand = lambda n: "".join("ACGT"[x] for x in rng.integers(0, 4, n))
    reads = []
    for L in sorted({k - 1, k, k + 1, 31, 32, 33, 63, 64, 65, 95, 96, 97}):
        reads += [rand(L) for _ in range(3)] if L > 0 else [""]
    base = rand(96)
    reads += [base[:p] + "N" + base[p + 1:] for p in range(96)]
    reads += [rand(1) for _ in range(40)]
    rng.shuffle(reads)
    return readsim.from_strings(reads + reads)


@pytest.mark.parametrize("k", [2, 4, 5, 6, 31, 32, 33, 62, 63])
def test_pack_and_count_at_word_edges(tk, oracle_lib, k):
    for seed in range(3):
        bases, offsets = word_edge_library(k, 40 * k + seed)
        case(f"word edges k={k} seed={seed} n_bases={bases.size}")
        db, do = to_device(bases, offsets)
        packed, valid, nw = tk.tk_pack_device(db, do, k)
        hp, hv = host_pack(bases, offsets, k)
        assert (packed.cpu().numpy().view(np.uint64) == hp).all()
        assert (valid.cpu().numpy().view(np.uint32) == hv).all()
        check_against_oracle(tk, oracle_lib, bases, offsets, k, 2)


@pytest.mark.parametrize("n", [0, 1, 2, 100, 4095, 4096, 4097, 100_003])
@pytest.mark.parametrize("bits", [62, 20, 7])
def test_sort_stage_one_word(tk, n, bits):
    import torch
    case(f"sort u64 n={n} bits={bits}")
    rng = np.random.default_rng(n + bits)
    keys = rng.integers(0, 1 << bits, size=n, dtype=np.uint64)
    out = tk.tk_sort_keys_device(torch.from_numpy(keys.view(np.int64)).cuda(), 1, bits)
    got = out.cpu().numpy().view(np.uint64)
    assert (got == np.sort(keys)).all()


@pytest.mark.parametrize("n", [1, 2047, 2048, 2049, 50_001])
def test_sort_stage_two_words(tk, n):
    import torch
    case(f"sort u128 n={n}")
    rng = np.random.default_rng(n)
    hi = rng.integers(0, 1 << 20, size=n, dtype=np.uint64)  # repeats in hi
    lo = rng.integers(0, 1 << 63, size=n, dtype=np.uint64)
    lo[::3] = lo[0]
    flat = np.stack([hi, lo], axis=1).ravel()
    out = tk.tk_sort_keys_device(torch.from_numpy(flat.view(np.int64)).cuda(), 2, 84)
    got = out.cpu().numpy().view(np.uint64).reshape(n, 2)
    order = np.lexsort((lo, hi))
    assert (got[:, 0] == hi[order]).all() and (got[:, 1] == lo[order]).all()


@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097, 70_001])
@pytest.mark.parametrize("c", [1, 2, 3, 7])
def test_compact_stage(tk, n, c):
    import torch
    case(f"compact n={n} c={c}")
    rng = np.random.default_rng(n * 10 + c)
    keys = np.sort(rng.geometric(0.02, size=n).astype(np.uint64) * np.uint64(977))
    ok, oc, st = tk.tk_compact_device(torch.from_numpy(keys.view(np.int64)).cuda(), 1, c)
    u, cnt = np.unique(keys, return_counts=True)
    keep = cnt >= c
    assert (ok.cpu().numpy().view(np.uint64)[:, 0] == u[keep]).all()
    assert (oc.cpu().numpy() == cnt[keep]).all()
    assert st["n_out"] == int(keep.sum())
    assert st["n_distinct"] == u.size
    assert st["n_singletons"] == int((cnt == 1).sum())
    assert st["n_below_c"] == int(((cnt >= 2) & (cnt < c)).sum())


def test_compact_stage_two_words(tk):
    import torch
    case("compact u128")
    rng = np.random.default_rng(3)
    n = 9000
    hi = np.sort(rng.integers(0, 50, size=n, dtype=np.uint64))
    lo = rng.integers(0, 3, size=n, dtype=np.uint64)
    order = np.lexsort((lo, hi))
    hi, lo = hi[order], lo[order]
    flat = np.stack([hi, lo], axis=1).ravel()
    ok, oc, st = tk.tk_compact_device(torch.from_numpy(flat.view(np.int64)).cuda(), 2, 2)
    import collections
    cnt = collections.Counter(zip(hi.tolist(), lo.tolist()))
    want = sorted((h, l, v) for (h, l), v in cnt.items() if v >= 2)
    got = ok.cpu().numpy().view(np.uint64)
    assert [(int(a), int(b), int(v)) for (a, b), v in zip(got, oc.cpu().numpy())] == want


# --------------------------------------------------------------------------
# end to end
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", KS)
@pytest.mark.parametrize("c", [1, 2, 3])
def test_count_matches_oracle(tk, oracle_lib, k, c):
    bases, offsets = library(100 + 3 * k + c, 600, 2 * k + 120, k)
    case(f"count k={k} c={c} n_bases={bases.size}")
    check_against_oracle(tk, oracle_lib, bases, offsets, k, c)


@pytest.mark.parametrize("shift", [1, 3, 7, 13])
def test_misaligned_bases(tk, oracle_lib, shift):
    bases, offsets = library(55 + shift, 300, 150, 31)
    case(f"misaligned shift={shift}")
    check_against_oracle(tk, oracle_lib, bases, offsets, 31, 2, shift=shift)


def test_empty_inputs(tk, oracle_lib):
    case("empty library")
    for reads in ([], [""], ["", "", ""], ["ACG", "TT"], ["NNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNNN"]):
        bases, offsets = readsim.from_strings(reads)
        for k, c in ((31, 2), (5, 1), (63, 3)):
            keys, counts, r = gpu_count(tk, bases, offsets, k, c)
            assert keys.shape[0] == 0 and counts.size == 0
            assert r.n_windows == oracle_lib.count_windows(bases, offsets, k) if bases.size else r.n_windows == 0


@pytest.mark.parametrize("k", [1, 31, 32, 63])
def test_single_huge_run(tk, oracle_lib, k):
    """One all-A read: a single key whose count is the read length - k + 1."""
    L = 200_000
    bases, offsets = readsim.from_strings(["A" * L])
    case(f"all-A L={L} k={k}")
    keys, counts, r = gpu_count(tk, bases, offsets, k, 2)
    assert keys.shape[0] == 1 and int(keys[0].max()) == 0
    assert counts.tolist() == [L - k + 1]
    assert r.n_windows == L - k + 1


def test_exact_length_reads(tk, oracle_lib):
    k = 31
    rng = np.random.default_rng(1)
    reads = ["".join("ACGT"[x] for x in rng.integers(0, 4, k)) for _ in range(50)]
    reads = reads * 3
    bases, offsets = readsim.from_strings(reads)
    case("reads of exactly k bases")
    check_against_oracle(tk, oracle_lib, bases, offsets, k, 2)


@pytest.mark.parametrize("k", [5, 7])
def test_de_bruijn(tk, oracle_lib, k):
    s = readsim.de_bruijn("ACGT", k)
    bases, offsets = readsim.from_strings([s])
    case(f"de Bruijn k={k}")
    keys, counts, r = gpu_count(tk, bases, offsets, k, 2)
    assert keys.shape[0] == 4 ** k // 2 and (counts == 2).all()
    check_against_oracle(tk, oracle_lib, bases, offsets, k, 2)


def test_host_entry_point(tk, oracle_lib):
    bases, offsets = library(999, 500, 200, 31)
    case("tk_count host entry point")
    for k, c in ((31, 2), (45, 2), (12, 1)):
        r = tk.tk_count(bases, offsets, k, c)
        ora = oracle_lib.kmer_count(bases, offsets, k, c)
        assert_same(r.keys, r.counts, ora, k)
        assert r.n_windows == ora.n_windows


@pytest.mark.parametrize("k,c", [(31, 1), (63, 1), (31, 2)])
def test_host_entry_point_beyond_one_staging_slice(tk, k, c):
    """Reads (90 MB) and records (up to 0.3 GB at c = 1) larger than one
    64 MB staging slice of the host copies: the host entry point returns
    exactly the device entry point's records."""
    lib = readsim.large_library(scale=0.06)
    case(f"host entry point, staged copies, k={k} c={c} n_bases={lib.n_bases}")
    h = tk.tk_count(lib.bases, lib.offsets, k, c)
    keys, counts, r = gpu_count(tk, lib.bases, lib.offsets, k, c)
    assert h.keys.shape == keys.shape and np.array_equal(h.keys, keys)
    assert np.array_equal(h.counts, counts)
    assert (h.n_windows, h.n_collected, h.n_distinct) == (r.n_windows, r.n_collected, r.n_distinct)
    if c == 1:
        assert keys.nbytes > 64 << 20


@pytest.mark.parametrize("opts", [None, GLOBAL])
def test_repeat_runs_identical(tk, opts):
    """The screen's outcome does not depend on the order atomics land in."""
    lib = readsim.small_library(scale=0.2)
    case(f"repeatability {opts}")
    first = None
    for _ in range(3):
        keys, counts, r = gpu_count(tk, lib.bases, lib.offsets, 31, 2, opts=opts)
        cur = (keys.tobytes(), counts.tobytes(), r.n_collected, r.n_distinct, r.n_singletons)
        if first is None:
            first = cur
        assert cur == first


@pytest.mark.parametrize("opts", [dict(bloom_beta=1), dict(bloom_bits=1, bloom_table_bits=4),
                                  dict(bloom_bits=5, bloom_seed=77), dict(bloom_beta=32),
                                  dict(part_bits=0), dict(part_bits=3), dict(part_bits=16),
                                  dict(GLOBAL, bloom_beta=1), dict(GLOBAL, bloom_blocks=3),
                                  dict(GLOBAL, bloom_bits=5, bloom_seed=77)])
def test_bloom_options(tk, oracle_lib, opts):
    """Other filter layouts, sizes and tables: same exact answer, model-exact statistics."""
    bases, offsets = library(4242, 800, 160, 31, dup=0.5)
    case(f"bloom options {opts}")
    check_against_oracle(tk, oracle_lib, bases, offsets, 31, 2, opts=opts)


@pytest.mark.parametrize("k", [5, 31, 32, 63])
@pytest.mark.parametrize("c", [1, 2, 3])
def test_global_filter_path(tk, oracle_lib, k, c):
    bases, offsets = library(300 + 3 * k + c, 500, 2 * k + 100, k)
    case(f"global filter k={k} c={c}")
    check_against_oracle(tk, oracle_lib, bases, offsets, k, c, opts=GLOBAL)


@pytest.mark.parametrize("k,part_bits", [(31, 0), (31, 2), (63, 0), (63, 3), (21, 1)])
@pytest.mark.parametrize("c", [1, 2])
def test_oversized_buckets_fallback(tk, oracle_lib, k, part_bits, c):
    """Buckets larger than the LDS capacity go through the global-memory
    fallback with the same per-bucket filter rule."""
    bases, offsets = library(900 + k + part_bits, 3000, 2 * k + 120, k, dup=0.4)
    case(f"fallback k={k} part_bits={part_bits} c={c} n_bases={bases.size}")
    r = check_against_oracle(tk, oracle_lib, bases, offsets, k, c, opts=dict(part_bits=part_bits))
    assert r.n_fallback >= 1


@pytest.mark.parametrize("which,part_bits", [("small", 6), ("small", 8), ("long_k", 10)])
def test_many_oversized_buckets(tk, oracle_lib, which, part_bits):
    """Dozens to hundreds of oversized buckets, alone or mixed with buckets
    that fit a workgroup, all through one fallback batch."""
    lib = readsim.small_library(scale=0.2) if which == "small" else readsim.long_k_library(scale=0.01)
    case(f"many oversized buckets {lib.name} part_bits={part_bits} n_bases={lib.n_bases}")
    r = check_against_oracle(tk, oracle_lib, lib.bases, lib.offsets, lib.k, lib.c, opts=dict(part_bits=part_bits))
    assert r.n_fallback >= 8


@pytest.mark.parametrize("which,scale,part_bits", [("large", 0.03, 11), ("long_k", 0.05, 12)])
def test_oversized_buckets_in_tiles(tk, oracle_lib, which, scale, part_bits):
    """With a second pass, a bucket is one piece per tile of its segment:
    buckets too large for a workgroup are gathered piece by piece for the
    fallback kernels, the others are loaded piece by piece by the bucket
    kernel."""
    lib = readsim.large_library(scale=scale) if which == "large" else readsim.long_k_library(scale=scale)
    case(f"oversized buckets in tiles {lib.name} part_bits={part_bits} n_bases={lib.n_bases}")
    r = check_against_oracle(tk, oracle_lib, lib.bases, lib.offsets, lib.k, lib.c, opts=dict(part_bits=part_bits))
    assert r.part_bits > 10 and r.n_fallback >= 8


@pytest.mark.parametrize("over", [False, True])
@pytest.mark.parametrize("k", [31, 63])
def test_segment_with_more_tiles_than_a_group_spans(tk, oracle_lib, k, over):
    """One k-mer repeated millions of times fills one segment with many
    second-pass tiles.  Up to 256 tiles, the segment's small buckets are
    loaded from up to 256 pieces (four per lane of the wave that indexes
    them) and only the giant bucket goes through the fallback; past 256,
    the small buckets go through the fallback as well (gathered from the
    tiles).  Every count stays exact."""
    rng = np.random.default_rng(404 + k)
    # about 137 (142) or 275 (283) tiles of 32768 (16384) keys
    n_same = (50_000 if k <= 31 else 40_000) * (2 if over else 1)
    reads = ["A" * 120] * n_same
    # random reads: k-mers in the same segment (a leading run of A) and elsewhere
    reads += ["A" * 6 + "".join("ACGT"[x] for x in rng.integers(0, 4, 114)) for _ in range(4000)]
    reads += ["".join("ACGT"[x] for x in rng.integers(0, 4, 120)) for _ in range(4000)]
    bases, offsets = readsim.from_strings(reads)
    case(f"hot segment k={k} over={over} n_bases={bases.size}")
    r = check_against_oracle(tk, oracle_lib, bases, offsets, k, 2, opts=dict(part_bits=13))
    assert r.part_bits == 13
    assert r.n_fallback >= 2 if over else r.n_fallback == 1, r.n_fallback


def _bin_reads(rng, k, prefix, n_distinct, copies):
    """Reads of exactly k bases (one window each): n_distinct k-mers that
    start with ``prefix`` and end in A (so the forward strand is the
    canonical one and the key keeps the prefix), each repeated ``copies``
    times."""
    out = []
    for _ in range(n_distinct):
        mid = "".join("ACGT"[x] for x in rng.integers(0, 4, k - len(prefix) - 1))
        out += [prefix + mid + "A"] * copies
    return out


@pytest.mark.parametrize("k", [31, 63])
def test_mixed_bins_past_the_rank_cap(tk, oracle_lib, k):
    """Mixed bins of every ordering path.  With one bucket (part_bits 0) the
    sort's first pass bins keys by their first six bases, so each prefix
    below is one bin.  The bins are taken two at a time in key order:
    (small, large) then (small, small).  The small bins, ranked side by
    side, and the large one, ranked alone, all hold more distinct values
    than the value-at-a-time ranking takes before it scans the bin (8 +
    keys / 16), except the last.  A separate library has one bin of more
    than 256 keys, which sends its group through the radix passes."""
    rng = np.random.default_rng(1303 + k)
    reads = (_bin_reads(rng, k, "AAAAAC", 20, 2)     # 40 keys, 20 values: small, past the cap
             + _bin_reads(rng, k, "AAAAAG", 40, 3)   # 120 keys, 40 values: large, past the cap
             + _bin_reads(rng, k, "AAAACA", 12, 3)   # 36 keys, 12 values: small, past the cap
             + _bin_reads(rng, k, "AAAACC", 5, 8))   # 40 keys, 5 values: small, within the cap
    rng.shuffle(reads)
    bases, offsets = readsim.from_strings(reads)
    case(f"mixed bins k={k} windows={len(reads)}")
    check_against_oracle(tk, oracle_lib, bases, offsets, k, 2, opts=dict(part_bits=0))
    reads = _bin_reads(rng, k, "AAAAGA", 150, 2) + _bin_reads(rng, k, "AAAAGC", 10, 4)
    rng.shuffle(reads)
    bases, offsets = readsim.from_strings(reads)
    case(f"mixed bin over 256 keys k={k} windows={len(reads)}")
    check_against_oracle(tk, oracle_lib, bases, offsets, k, 2, opts=dict(part_bits=0))


def test_bucket_capacity_edges(tk, oracle_lib):
    """One bucket (part_bits 0) of exactly the register capacity, one less
    and one more: 512 threads x 14 one-word keys = 7168, x 7 two-word keys =
    3584 windows.  A second read repeats the first third of the first, so
    the bucket holds frequent and single k-mers."""
    rng = np.random.default_rng(77)
    for k, caps in ((31, (7167, 7168, 7169, 3584)), (63, (3583, 3584, 3585, 7168))):
        for total in caps:
            m = total // 3  # windows of the second read
            L1 = total - m + k - 1
            read = "".join("ACGT"[x] for x in rng.integers(0, 4, L1))
            bases, offsets = readsim.from_strings([read, read[: m + k - 1]])
            case(f"capacity edge windows={total} k={k}")
            r = check_against_oracle(tk, oracle_lib, bases, offsets, k, 2, opts=dict(part_bits=0))
            assert r.n_windows == total
            cap = 7168 if k <= 31 else 3584
            assert r.n_fallback == (1 if total > cap else 0), (total, r.n_fallback)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def test_small_library_full(tk, oracle_lib):
    lib = readsim.small_library()
    case(f"{lib.name} full n_bases={lib.n_bases}")
    r = check_against_oracle(tk, oracle_lib, lib.bases, lib.offsets, lib.k, lib.c)
    assert r.n_windows == lib.n_reads * (100 - 31 + 1)
    case(f"{lib.name} full, global filter")
    check_against_oracle(tk, oracle_lib, lib.bases, lib.offsets, lib.k, lib.c, opts=GLOBAL)


def test_large_library_reduced(tk, oracle_lib):
    lib = readsim.large_library(scale=0.02)
    case(f"{lib.name} scale=0.02 n_bases={lib.n_bases}")
    check_against_oracle(tk, oracle_lib, lib.bases, lib.offsets, lib.k, lib.c)


def test_long_k_library_reduced(tk, oracle_lib):
    lib = readsim.long_k_library(scale=0.03)
    case(f"{lib.name} scale=0.03 n_bases={lib.n_bases}")
    check_against_oracle(tk, oracle_lib, lib.bases, lib.offsets, lib.k, lib.c)


def sampled_full_size_check(tk, oracle_lib, lib, n_sample=1500):
    """Full-size run in the benchmark's launch configuration, checked on
    sampled keys (exact counts recounted by the oracle) and by properties."""
    keys, counts, r = gpu_count(tk, lib.bases, lib.offsets, lib.k, lib.c)
    kw = keys.shape[1]
    # strictly ascending, every count >= c, counts add up
    if kw == 1:
        assert (keys[1:, 0] > keys[:-1, 0]).all()
    else:
        h, l = keys[:, 0], keys[:, 1]
        asc = (h[1:] > h[:-1]) | ((h[1:] == h[:-1]) & (l[1:] > l[:-1]))
        assert asc.all()
    assert (counts >= lib.c).all()
    if lib.c == 2:
        # every collected occurrence is either in the output or a false positive
        assert int(counts.astype(np.uint64).sum()) == r.n_collected - r.n_singletons
    rng = np.random.default_rng(12345)
    # sampled output keys
    pick = rng.choice(keys.shape[0], size=min(n_sample, keys.shape[0]), replace=False)
    # sampled input windows (their canonical keys, from the strings)
    raw = lib.bases
    L = int(lib.offsets[1] - lib.offsets[0])
    win = []
    while len(win) < n_sample:
        rd = int(rng.integers(0, lib.n_reads))
        p = int(rng.integers(0, L - lib.k + 1))
        s = raw[rd * L + p: rd * L + p + lib.k].tobytes().decode()
        if set(s) <= set("ACGT"):
            win.append(brute.encode(brute.canonical(s)))
    qs = set(win)
    for i in pick:
        qs.add((int(keys[i, 0]) << 64 | int(keys[i, 1])) if kw == 2 else int(keys[i, 0]))
    q = sorted(qs)
    q_hi = np.array([x >> 64 for x in q], np.uint64)
    q_lo = np.array([x & ((1 << 64) - 1) for x in q], np.uint64)
    truth = oracle_lib.count_queries(lib.bases, lib.offsets, lib.k, q_hi, q_lo, n_threads=16)
    truth = dict(zip(q, truth.tolist()))
    if kw == 1:
        gk = keys[:, 0]
        find = lambda x: np.searchsorted(gk, np.uint64(x))  # noqa: E731
    else:
        def find(x):
            hi, lo = np.uint64(x >> 64), np.uint64(x & ((1 << 64) - 1))
            a = np.searchsorted(keys[:, 0], hi, side="left")
            b = np.searchsorted(keys[:, 0], hi, side="right")
            return a + np.searchsorted(keys[a:b, 1], lo)
    for x in q:
        i = int(find(x))
        have = i < keys.shape[0] and ((int(keys[i, 0]) << 64 | int(keys[i, 1])) if kw == 2 else int(keys[i, 0])) == x
        if truth[x] >= lib.c:
            assert have, hex(x)
            assert int(counts[i]) == truth[x]
        else:
            assert not have, hex(x)
    return r


@pytest.mark.slow
def test_large_library_full_sampled(tk, oracle_lib):
    lib = readsim.large_library()
    case(f"{lib.name} full n_bases={lib.n_bases}")
    r = sampled_full_size_check(tk, oracle_lib, lib)
    assert r.n_windows == lib.n_reads * (100 - 31 + 1)  # no N bases in this workload


@pytest.mark.slow
def test_long_k_library_full_sampled(tk, oracle_lib):
    lib = readsim.long_k_library()
    case(f"{lib.name} full n_bases={lib.n_bases}")
    sampled_full_size_check(tk, oracle_lib, lib)
