"""Pins of the oracle's pattern-blocked Bloom model (paper §2.1, §2.2) -- no GPU.

The screen never changes the exact answer; it only decides which keys are
collected.  These tests pin the model against: the no-false-negative property,
an explicit per-bit touch count, the false-positive rate predicted by theory,
the paper's 9.6-bits-per-item figure for an ordinary Bloom filter, and the
invertibility of the hash (a dropped or altered step breaks the inverse).
"""
import math
from collections import Counter

import numpy as np
import pytest

import readsim
from oracle import brute

M64 = (1 << 64) - 1


def test_standard_bloom_figure(oracle_lib):
    # §2.2: about 9.6 bits per item give a 1 % false-positive rate (7 hashes)
    assert abs(oracle_lib.standard_bloom_fpr(9.6, 7) - 0.01) < 0.0005


@pytest.mark.parametrize("n_bits", [1, 2, 4, 7])
def test_pattern_table_shape(oracle_lib, n_bits):
    pos = oracle_lib.pattern_positions(512, n_bits, seed=99)
    assert pos.shape == (512, n_bits)
    for row in pos:
        assert len(set(row.tolist())) == n_bits  # distinct positions
        assert row.max() < 64
    masks = oracle_lib.pattern_masks(512, n_bits, seed=99)
    pop = np.array([bin(int(m)).count("1") for m in masks])
    assert (pop == n_bits).all()
    # deterministic and seed-dependent
    assert (oracle_lib.pattern_positions(512, n_bits, seed=99) == pos).all()
    assert not (oracle_lib.pattern_positions(512, n_bits, seed=100) == pos).all()
    # positions roughly uniform over the 256 bits
    hist = np.bincount(pos.ravel(), minlength=64)
    assert hist.size == 64
    assert hist.max() < 2 * pos.size / 64 + 10 and hist.min() > pos.size / 64 / 2 - 10


def _inv_xorshift33(x):
    return x ^ (x >> 33)


def _inv_fmix64(h):
    c1, c2 = 0xff51afd7ed558ccd, 0xc4ceb9fe1a85ec53
    i1, i2 = pow(c1, -1, 1 << 64), pow(c2, -1, 1 << 64)
    x = _inv_xorshift33(h)
    x = (x * i2) & M64
    x = _inv_xorshift33(x)
    x = (x * i1) & M64
    return _inv_xorshift33(x)


def _full_hash(oracle_lib, hi, lo, two):
    # with n_blocks = 2^63 the block is h >> 1; with a 2^16-entry table word w
    # gets bits [16w, 16w + 16) of h
    blk, ent = oracle_lib.block_of(hi, lo, two, 1 << 63, 1 << 16)
    h = sum(e << (16 * w) for w, e in enumerate(ent))
    assert blk == h >> 1
    return h


def test_hash_is_invertible_finaliser(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(200):
        lo = int(rng.integers(0, 1 << 62))
        h = _full_hash(oracle_lib, 0, lo, False)
        assert _inv_fmix64(h) == lo
        hi = int(rng.integers(0, 1 << 62))
        h2 = _full_hash(oracle_lib, hi, lo, True)
        # two-word hash: fmix64(lo ^ fmix64(hi)); undo the outer step, then the xor
        inner = _inv_fmix64(h2)
        assert _inv_fmix64(inner ^ lo) == hi


def test_block_mapping_multiply_shift(oracle_lib):
    for n_blocks in (1, 3, 1000, 12345677):
        for key in (0, 1, 77, 2**61 + 5):
            blk, ent = oracle_lib.block_of(0, key, False, n_blocks, 1024)
            h = _full_hash(oracle_lib, 0, key, False)
            assert blk == (h * n_blocks) >> 64
            assert ent == [(h >> (10 * w)) % 1024 for w in range(4)]
            assert 0 <= blk < n_blocks


def _window_keys(reads, k):
    keys = [brute.encode(brute.canonical(w)) for r in reads for w in brute.windows(r, k)]
    hi = np.array([x >> 64 for x in keys], np.uint64)
    lo = np.array([x & M64 for x in keys], np.uint64)
    return keys, hi, lo


@pytest.mark.parametrize("k", [9, 31, 45])
def test_no_false_negatives_and_touch_semantics(oracle_lib, k):
    """Candidates = keys whose every pattern bit is touched twice (explicit count)."""
    bases, offsets = readsim.random_reads(400 + k, 300, 0, 3 * k, 0.02, 0.05, 0.0)
    reads = readsim.to_strings(bases, offsets)
    reads = reads + reads[:100]
    keys, hi, lo = _window_keys(reads, k)
    two = k > 31
    n_blocks = 37  # small filter so that false positives occur
    st = oracle_lib.bloom_model_keys(hi, lo, two, n_blocks, want_flags=True)
    pos = oracle_lib.pattern_positions()
    touches = Counter()
    loc = []
    for x in keys:
        blk, ent = oracle_lib.block_of(x >> 64, x & M64, two, n_blocks)
        bits = [(blk, 64 * w + int(p)) for w, e in enumerate(ent) for p in pos[e]]
        loc.append(bits)
        for b in bits:
            touches[b] += 1
    flags = [all(touches[b] >= 2 for b in bits) for bits in loc]
    assert st.flags.astype(bool).tolist() == flags
    mult = Counter(keys)
    # every key seen at least twice is collected (no false negatives)
    for x, f in zip(keys, flags):
        if mult[x] >= 2:
            assert f
    cand = {x for x, f in zip(keys, flags) if f}
    assert st.n_cand == len(cand)
    assert st.n_cand_occ == sum(flags)
    assert st.n_cand_single == sum(1 for x in cand if mult[x] == 1)
    # the library-level entry point agrees with the key-level one
    b, o = readsim.from_strings(reads)
    st2 = oracle_lib.bloom_model(b, o, k, n_blocks)
    assert (st2.n_cand_occ, st2.n_cand, st2.n_cand_single) == (st.n_cand_occ, st.n_cand, st.n_cand_single)


def test_touch_order_independence(oracle_lib):
    """The candidate set does not depend on the order the windows are seen in."""
    rng = np.random.default_rng(11)
    lo = rng.integers(0, 1 << 40, size=3000).astype(np.uint64)
    lo = np.concatenate([lo, lo[:800]])
    hi = np.zeros_like(lo)
    a = oracle_lib.bloom_model_keys(hi, lo, False, 20, want_flags=True)
    perm = rng.permutation(lo.size)
    b = oracle_lib.bloom_model_keys(hi[perm], lo[perm], False, 20, want_flags=True)
    assert (a.n_cand_occ, a.n_cand, a.n_cand_single) == (b.n_cand_occ, b.n_cand, b.n_cand_single)
    assert (a.flags[perm] == b.flags).all()


@pytest.mark.parametrize("bits_per_key,n_patterns,n_bits",
                         [(6.0, 1024, 2), (12.0, 1024, 2), (9.0, 64, 2), (16.0, 256, 3)])
def test_false_positive_rate_matches_theory(oracle_lib, bits_per_key, n_patterns, n_bits):
    """Singletons only: measured false positives vs the blocked-filter theory (4 sigma)."""
    n = 60_000
    rng = np.random.default_rng(int(bits_per_key * 10) + n_patterns)
    lo = np.unique(rng.integers(0, 1 << 62, size=n + 100, dtype=np.int64).astype(np.uint64))[:n]
    hi = np.zeros_like(lo)
    n_blocks = max(1, int(round(n * bits_per_key / 256)))
    st = oracle_lib.bloom_model_keys(hi, lo, False, n_blocks, n_patterns=n_patterns,
                                     n_bits=n_bits)
    masks = oracle_lib.pattern_masks(n_patterns, n_bits)
    p = oracle_lib.blocked_singleton_fp_prob(masks, n_blocks, n - 1)
    expect = n * p
    sigma = math.sqrt(n * p * (1 - p))
    assert st.n_cand == st.n_cand_single  # all keys are singletons
    assert abs(st.n_cand_single - expect) <= 4 * sigma + 1, (st.n_cand_single, expect, sigma)


def test_theory_approaches_standard_bloom(oracle_lib):
    """With many bits per key the blocked rate is near the ordinary Bloom rate."""
    masks = oracle_lib.pattern_masks(1024)
    n = 100_000
    for b in (10.0, 16.0):
        n_blocks = int(n * b / 256)
        blocked = oracle_lib.blocked_singleton_fp_prob(masks, n_blocks, n - 1)
        std = oracle_lib.standard_bloom_fpr(b, 8)
        # blocking costs some accuracy but stays within a small factor
        assert std < blocked < 6 * std, (b, std, blocked)


def test_default_block_rule(oracle_lib):
    assert oracle_lib.default_blocks(0, 0, 31) == 1
    assert oracle_lib.default_blocks(100, 1, 31) == math.ceil(4 * 70 / 256)
    assert oracle_lib.default_blocks(10_000_000, 100_000, 31) == math.ceil(4 * 7_000_000 / 256)
    assert oracle_lib.default_blocks(10, 5, 31) == 1


def test_bucket_model_single_bucket_equals_global(oracle_lib):
    """With D = 0 there is one bucket whose filter is sized from all windows."""
    rng = np.random.default_rng(21)
    lo = rng.integers(0, 1 << 62, size=5000, dtype=np.int64).astype(np.uint64)
    lo = np.concatenate([lo, lo[:2000], lo[:300]])
    hi = np.zeros_like(lo)
    for beta in (1, 4, 9):
        a = oracle_lib.bloom_model_buckets_keys(hi, lo, 31, 0, beta)
        nb = max(1, -(-beta * lo.size // 256))
        b = oracle_lib.bloom_model_keys(hi, lo, False, nb)
        assert (a.n_cand_occ, a.n_cand, a.n_cand_single) == (b.n_cand_occ, b.n_cand, b.n_cand_single)


@pytest.mark.parametrize("k,D", [(31, 6), (63, 9), (33, 4), (5, 10), (2, 4)])
def test_bucket_model_is_sum_over_buckets(oracle_lib, k, D):
    """Grouping by the top D bits (done here in Python) and summing the
    one-filter model per group reproduces the per-bucket model."""
    bases, offsets = readsim.random_reads(700 + k + D, 400, 0, 3 * k + 10, 0.01, 0.0, 0.0)
    reads = readsim.to_strings(bases, offsets)
    reads = reads + reads[:150]
    keys, hi, lo = _window_keys(reads, k)
    beta = 3
    want = [0, 0, 0]
    groups = {}
    for x in keys:
        groups.setdefault(x >> (2 * k - D), []).append(x)
    for g in groups.values():
        gh = np.array([x >> 64 for x in g], np.uint64)
        gl = np.array([x & M64 for x in g], np.uint64)
        nb = max(1, -(-beta * len(g) // 256))
        st = oracle_lib.bloom_model_keys(gh, gl, k > 31, nb)
        want[0] += st.n_cand_occ
        want[1] += st.n_cand
        want[2] += st.n_cand_single
    got = oracle_lib.bloom_model_buckets_keys(hi, lo, k, D, beta)
    assert [got.n_cand_occ, got.n_cand, got.n_cand_single] == want
    b, o = readsim.from_strings(reads)
    lib_level = oracle_lib.bloom_model_buckets(b, o, k, D, beta)
    assert (lib_level.n_cand_occ, lib_level.n_cand, lib_level.n_cand_single) == tuple(want)
    # every key seen at least twice is a candidate
    mult = Counter(keys)
    assert got.n_cand_occ >= sum(v for v in mult.values() if v >= 2)
