"""Pins of the oracle's key-range enumeration (no GPU).

``oracle.keys_in_range`` lets the full-size workloads be counted exactly one
key range at a time.  It is pinned against brute force on Python strings
(the top bits of a key are the leading bases of its canonical string) and
against the whole-library oracle: the ranges partition the windows, and the
per-range sort-and-compact results concatenate, in range order, into the
exact answer.
"""
from collections import Counter

import numpy as np
import pytest

import readsim
from oracle import brute


def _reads(seed, k):
    bases, offsets = readsim.random_reads(seed, 40, min_len=0, max_len=2 * k + 30,
                                          n_rate=0.03, lower_rate=0.1, junk_rate=0.01)
    reads = readsim.to_strings(bases, offsets)
    reads = reads + reads[:15] + [brute.revcomp(brute.ascii_upper(r)) for r in reads[:8]]
    return reads


@pytest.mark.parametrize("k", [1, 2, 3, 5, 21, 31, 32, 33, 63])
def test_range_keys_match_brute_force(oracle_lib, k):
    reads = _reads(7000 + k, k)
    b, o = readsim.from_strings(reads)
    canon = [brute.encode(brute.canonical(w)) for r in reads for w in brute.windows(r, k)]
    for rb in sorted({0, 1, 2, 3, 4, 5} & set(range(0, min(2 * k, 16) + 1))):
        for ri in range(1 << rb):
            hi, lo = oracle_lib.keys_in_range(b, o, k, rb, ri)
            got = Counter((int(h) << 64) | int(l) for h, l in zip(hi.tolist(), lo.tolist()))
            want = Counter(v for v in canon if (v >> (2 * k - rb)) == ri)
            assert got == want, (k, rb, ri)


@pytest.mark.parametrize("k,rb", [(21, 3), (31, 4), (33, 4), (63, 6)])
def test_ranges_concatenate_to_the_exact_answer(oracle_lib, k, rb):
    bases, offsets = readsim.random_reads(8100 + k, 300, min_len=0, max_len=160)
    # duplicated reads so that counts above 1 occur
    bases = np.concatenate([bases, bases])
    offsets = np.concatenate([offsets, offsets[1:] + offsets[-1]])
    full = oracle_lib.kmer_count(bases, offsets, k, 1)
    parts_hi, parts_lo, parts_n = [], [], []
    n_win = 0
    for ri in range(1 << rb):
        hi, lo = oracle_lib.keys_in_range(bases, offsets, k, rb, ri)
        n_win += hi.size
        key = (hi.astype(object) << 64) | lo.astype(object) if hi.size else np.zeros(0, object)
        assert all((int(x) >> (2 * k - rb)) == ri for x in key)
        uh, ul, uc = oracle_lib.sort_compact(hi, lo)
        parts_hi.append(uh)
        parts_lo.append(ul)
        parts_n.append(uc)
    assert n_win == full.n_windows == oracle_lib.count_windows(bases, offsets, k)
    assert np.array_equal(np.concatenate(parts_hi), full.hi)
    assert np.array_equal(np.concatenate(parts_lo), full.lo)
    assert np.array_equal(np.concatenate(parts_n), full.count)


def test_range_argument_checks(oracle_lib):
    b, o = readsim.from_strings(["ACGTACGT"])
    for k, rb, ri in [(3, 7, 0), (3, 2, 4), (31, 17, 0), (64, 0, 0)]:
        with pytest.raises(ValueError):
            oracle_lib.keys_in_range(b, o, k, rb, ri)
