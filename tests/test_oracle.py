"""Pins of the CPU oracle against things other than itself (no GPU).

Each test checks the oracle against brute force, a closed form, an invariant
or a library routine, so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import os
import re

import numpy as np
import pytest

import readsim
from oracle import brute

KS = [1, 2, 3, 5, 15, 21, 31, 32, 33, 55, 63]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def as_pairs(res, k):
    """Oracle result as sorted [(kmer string, count)] for comparison with brute force."""
    out = []
    for hi, lo, n in zip(res.hi.tolist(), res.lo.tolist(), res.count.tolist()):
        out.append((brute.decode((hi << 64) | lo, k), n))
    return out


@pytest.mark.parametrize("k", KS)
@pytest.mark.parametrize("c", [1, 2, 3, 5])
def test_oracle_matches_brute_force(oracle_lib, k, c):
    seed = 1000 + 17 * k + c
    bases, offsets = readsim.random_reads(seed, 60, min_len=0, max_len=2 * k + 40,
                                          n_rate=0.03, lower_rate=0.1, junk_rate=0.01)
    # add a few repeated reads so that counts >= c occur
    reads = readsim.to_strings(bases, offsets)
    reads = reads + reads[:20] + [brute.revcomp(brute.ascii_upper(r)) for r in reads[:10]]
    b, o = readsim.from_strings(reads)
    res = oracle_lib.kmer_count(b, o, k, c)
    want = brute.count(reads, k, c)
    assert as_pairs(res, k) == want
    assert res.n_windows == brute.n_windows(reads, k)
    assert oracle_lib.count_windows(b, o, k) == res.n_windows
    if k <= 31:
        assert not res.hi.any()


def test_base_codes_and_order(oracle_lib):
    # A<C<G<T and first base most significant: AC.. < CA..
    b, o = readsim.from_strings(["AAC", "ACA", "AAG"])
    res = oracle_lib.kmer_count(b, o, 3, 1)
    # canonical: AAC (rc GTT) -> AAC=1; ACA (rc TGT) -> ACA=4; AAG (rc CTT) -> AAG=2
    assert res.lo.tolist() == [1, 2, 4]
    assert res.count.tolist() == [1, 1, 1]


def test_palindrome_counts_once(oracle_lib):
    # "AT" is its own reverse complement: one key per window, never doubled
    b, o = readsim.from_strings(["ATATAT"])
    res = oracle_lib.kmer_count(b, o, 2, 1)
    # windows: AT TA AT TA AT ; TA's rc is TA (palindrome too)
    assert as_pairs(res, 2) == [("AT", 3), ("TA", 2)]


def test_all_a_read(oracle_lib):
    for L, k in [(100, 31), (1000, 63), (5000, 1), (31, 31), (30, 31)]:
        b, o = readsim.from_strings(["A" * L])
        res = oracle_lib.kmer_count(b, o, k, 1)
        if L < k:
            assert res.lo.size == 0 and res.n_windows == 0
        else:
            assert res.hi.tolist() == [0] and res.lo.tolist() == [0]
            assert res.count.tolist() == [L - k + 1]


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7])
def test_de_bruijn_closed_form(oracle_lib, k):
    s = readsim.de_bruijn("ACGT", k)
    assert len(s) == 4 ** k + k - 1
    b, o = readsim.from_strings([s])
    res = oracle_lib.kmer_count(b, o, k, 1)
    counts = res.count
    n_pal = 4 ** (k // 2) if k % 2 == 0 else 0
    # every k-mer occurs once; a class {x, rc(x)} has 2 members unless x is a palindrome
    assert res.n_windows == 4 ** k
    assert int((counts == 1).sum()) == n_pal
    assert int((counts == 2).sum()) == (4 ** k - n_pal) // 2
    assert counts.size == n_pal + (4 ** k - n_pal) // 2
    # at c = 2 only the non-palindromic classes remain
    res2 = oracle_lib.kmer_count(b, o, k, 2)
    assert res2.count.size == (4 ** k - n_pal) // 2


def _tiny_library(seed, n=80, max_len=90):
    bases, offsets = readsim.random_reads(seed, n, min_len=0, max_len=max_len,
                                          n_rate=0.02, lower_rate=0.05, junk_rate=0.005)
    reads = readsim.to_strings(bases, offsets)
    return reads + reads[: n // 3]


def _count(oracle_lib, reads, k, c):
    b, o = readsim.from_strings(reads)
    return oracle_lib.kmer_count(b, o, k, c)


def _as_dict(res):
    return {(h, l): n for h, l, n in zip(res.hi.tolist(), res.lo.tolist(), res.count.tolist())}


@pytest.mark.parametrize("k", [5, 21, 31, 33, 63])
def test_reverse_complement_invariance(oracle_lib, k):
    reads = _tiny_library(50 + k, max_len=3 * k)
    rc_reads = [brute.revcomp(brute.ascii_upper(r)) for r in reads]
    a = _count(oracle_lib, reads, k, 1)
    b = _count(oracle_lib, rc_reads, k, 1)
    assert _as_dict(a) == _as_dict(b)
    assert a.n_windows == b.n_windows


@pytest.mark.parametrize("k", [7, 31, 40])
def test_adding_rc_reads_doubles_counts(oracle_lib, k):
    reads = _tiny_library(70 + k, max_len=3 * k)
    a = _as_dict(_count(oracle_lib, reads, k, 1))
    b = _as_dict(_count(oracle_lib, reads + [brute.revcomp(brute.ascii_upper(r)) for r in reads], k, 1))
    assert b == {key: 2 * v for key, v in a.items()}


@pytest.mark.parametrize("k", [3, 31, 63])
def test_read_permutation_invariance(oracle_lib, k):
    reads = _tiny_library(90 + k, max_len=3 * k)
    rng = np.random.default_rng(k)
    perm = [reads[i] for i in rng.permutation(len(reads))]
    assert _as_dict(_count(oracle_lib, reads, k, 2)) == _as_dict(_count(oracle_lib, perm, k, 2))


@pytest.mark.parametrize("k", [4, 31, 50])
def test_n_split_identity(oracle_lib, k):
    """A read with a non-base byte at p counts like r[:p] and r[p+1:] as two reads."""
    reads = _tiny_library(110 + k, max_len=3 * k)
    split = []
    for r in reads:
        split.extend(re.split(r"[^ACGTacgt]", r))
    a = _count(oracle_lib, reads, k, 1)
    b = _count(oracle_lib, split, k, 1)
    assert _as_dict(a) == _as_dict(b)
    assert a.n_windows == b.n_windows


@pytest.mark.parametrize("k", [1, 6, 31, 32, 63])
def test_counts_sum_to_windows(oracle_lib, k):
    reads = _tiny_library(130 + k, max_len=3 * k)
    res = _count(oracle_lib, reads, k, 1)
    runs = [len(m) for r in reads for m in re.findall(r"[ACGTacgt]+", r)]
    expect = sum(max(0, L - k + 1) for L in runs)
    assert res.n_windows == expect
    assert int(res.count.sum()) == expect


@pytest.mark.parametrize("k", [9, 31, 45])
def test_additivity_over_libraries(oracle_lib, k):
    r1 = _tiny_library(150 + k, max_len=3 * k)
    r2 = _tiny_library(170 + k, max_len=3 * k)
    a, b = _as_dict(_count(oracle_lib, r1, k, 1)), _as_dict(_count(oracle_lib, r2, k, 1))
    ab = _as_dict(_count(oracle_lib, r1 + r2, k, 1))
    merged = dict(a)
    for key, v in b.items():
        merged[key] = merged.get(key, 0) + v
    assert ab == merged


@pytest.mark.parametrize("k", [5, 31, 63])
def test_threshold_monotone(oracle_lib, k):
    reads = _tiny_library(190 + k, max_len=3 * k)
    prev = _as_dict(_count(oracle_lib, reads, k, 1))
    for c in range(2, 6):
        cur = _as_dict(_count(oracle_lib, reads, k, c))
        assert set(cur) <= set(prev)
        assert all(prev[key] == v and v >= c for key, v in cur.items())
        assert {key for key, v in prev.items() if v >= c} == set(cur)
        prev = cur


@pytest.mark.parametrize("k", [11, 31, 33, 63])
def test_sort_compact_is_np_unique(oracle_lib, k):
    """At c = 1 sort-and-compact equals numpy.unique on brute-force encodings."""
    reads = _tiny_library(210 + k, n=150, max_len=3 * k)
    keys = [brute.encode(brute.canonical(w)) for r in reads for w in brute.windows(r, k)]
    res = _count(oracle_lib, reads, k, 1)
    got = [(h << 64) | l for h, l in zip(res.hi.tolist(), res.lo.tolist())]
    if k <= 31:
        u, cnt = np.unique(np.array(keys, dtype=np.uint64), return_counts=True)
        assert got == u.tolist()
    else:
        u, cnt = np.unique(np.array(keys, dtype=object), return_counts=True)
        assert got == list(u)
    assert res.count.tolist() == cnt.tolist()


def test_paper_toy_example():
    """§2.1 sorting-and-compaction toy example (golden fixture)."""
    import oracle
    inp, expect = None, []
    with open(os.path.join(GOLDEN, "sac_toy_example.txt")) as f:
        for line in f:
            if line.startswith("input"):
                inp = [int(x) for x in line.split()[1:]]
            elif line.startswith("expect"):
                _, key, n = line.split()
                expect.append((int(key), int(n)))
    hi = np.zeros(len(inp), np.uint64)
    lo = np.array(inp, np.uint64)
    h, l, c = oracle.sort_compact(hi, lo)
    assert list(zip(l.tolist(), c.tolist())) == expect
    assert not h.any()


def test_sort_compact_two_word_order():
    """Two-word keys order by (hi, lo): the high word decides first."""
    import oracle
    hi = np.array([1, 0, 1, 0, 2], np.uint64)
    lo = np.array([0, 2**64 - 1, 0, 5, 0], np.uint64)
    h, l, c = oracle.sort_compact(hi, lo)
    assert list(zip(h.tolist(), l.tolist(), c.tolist())) == [
        (0, 5, 1), (0, 2**64 - 1, 1), (1, 0, 2), (2, 0, 1)]


def test_empty_and_degenerate_inputs(oracle_lib):
    # no reads at all
    b = np.zeros(0, np.uint8)
    o = np.zeros(1, np.uint64)
    res = oracle_lib.kmer_count(b, o, 31, 2)
    assert res.lo.size == 0 and res.n_windows == 0
    # only empty / short / all-N reads
    res = _count(oracle_lib, ["", "ACG", "NNNNNNNNNN", ""], 5, 1)
    assert res.lo.size == 0 and res.n_windows == 0
    # k out of range and c = 0 are errors
    with pytest.raises(ValueError):
        _count(oracle_lib, ["ACGT"], 0, 1)
    with pytest.raises(ValueError):
        _count(oracle_lib, ["ACGT"], 64, 1)
    with pytest.raises(ValueError):
        _count(oracle_lib, ["ACGT"], 2, 0)
    # decreasing offsets are an error
    with pytest.raises(ValueError):
        oracle_lib.kmer_count(np.frombuffer(b"ACGTACGT", np.uint8).copy(),
                              np.array([0, 6, 3, 8], np.uint64), 2, 1)


def test_key_width_boundary(oracle_lib):
    # k = 31 uses 62 bits of one word; k = 32 and up use (hi, lo)
    s = "T" * 40
    for k in (31, 32, 33, 40):
        res = _count(oracle_lib, [s], k, 1)
        # canonical of T^k is A^k = 0
        assert res.hi.tolist() == [0] and res.lo.tolist() == [0]
    s = "C" * 63
    res = _count(oracle_lib, [s], 63, 1)
    # canonical of C^63 is C^63 (rc = G^63 is larger): all codes 1 over 126 bits
    v = int("1" * 63, 4)
    assert res.hi.tolist() == [v >> 64] and res.lo.tolist() == [v & (2**64 - 1)]


def test_count_queries_matches_full_count(oracle_lib):
    reads = _tiny_library(333, n=200, max_len=70)
    for k in (9, 31, 40):
        res = _count(oracle_lib, reads, k, 1)
        b, o = readsim.from_strings(reads)
        # query every other key plus a few absent keys
        qh = list(res.hi[::2]) + [2**63 - 1]
        ql = list(res.lo[::2]) + [12345]
        order = sorted(range(len(qh)), key=lambda i: (int(qh[i]), int(ql[i])))
        qh = np.array([qh[i] for i in order], np.uint64)
        ql = np.array([ql[i] for i in order], np.uint64)
        got = oracle_lib.count_queries(b, o, k, qh, ql, n_threads=3)
        want = _as_dict(res)
        for h, l, n in zip(qh.tolist(), ql.tolist(), got.tolist()):
            assert n == want.get((h, l), 0)
