"""The sequential models of the approximate variants (cTurtle of §2.2, the
single pass of Algorithm 1 with "+1") against the exact oracle: the
properties that hold whatever the filter collisions, and error rates that
fall as the filter grows."""
import numpy as np
import pytest

import oracle
import readsim


@pytest.fixture(scope="module")
def lib():
    return readsim.small_library(scale=0.05, seed=9)


def rates(exact_keys, got_keys):
    fn = np.setdiff1d(exact_keys, got_keys).size / max(exact_keys.size, 1)
    fp = np.setdiff1d(got_keys, exact_keys).size / max(exact_keys.size, 1)
    return fn, fp


@pytest.mark.parametrize("beta", [4, 16, 256])
def test_single_pass_counts_are_exact_or_one_over(lib, beta):
    all1 = oracle.kmer_count(lib.bases, lib.offsets, 31, 1)
    W = oracle.approx_words(lib.n_bases, lib.n_reads, 31, beta)
    got, stored = oracle.approx_count(lib.bases, lib.offsets, 31, "single_pass", 2, W)
    idx = np.searchsorted(all1.lo, got.lo)
    assert (all1.lo[idx] == got.lo).all()
    diff = got.count.astype(np.int64) - all1.count[idx].astype(np.int64)
    assert ((diff == 0) | (diff == 1)).all()
    # every k-mer seen twice is stored at its second sighting: no false negative
    frequent = all1.lo[all1.count >= 2]
    assert np.isin(frequent, got.lo).all()
    # stored sightings: all but the first of every reported key, plus the
    # false-positive first sightings
    assert stored == int(got.count.sum()) - got.lo.size


@pytest.mark.parametrize("beta", [4, 16, 256])
def test_cturtle_reports_each_key_once(lib, beta):
    all1 = oracle.kmer_count(lib.bases, lib.offsets, 31, 1)
    W = oracle.approx_words(lib.n_bases, lib.n_reads, 31, beta)
    got, reported = oracle.approx_count(lib.bases, lib.offsets, 31, "cturtle", 2, W)
    assert reported == got.lo.size  # one report per key
    assert (got.count == 0).all()
    assert np.isin(got.lo, all1.lo).all()  # only k-mers of the library


def test_errors_fall_as_the_filter_grows(lib):
    exact = oracle.kmer_count(lib.bases, lib.offsets, 31, 2)
    prev = None
    for beta in (4, 16, 64, 1024):
        W = oracle.approx_words(lib.n_bases, lib.n_reads, 31, beta)
        ct, _ = oracle.approx_count(lib.bases, lib.offsets, 31, "cturtle", 2, W)
        sp, _ = oracle.approx_count(lib.bases, lib.offsets, 31, "single_pass", 2, W)
        fn_c, fp_c = rates(exact.lo, ct.lo)
        fn_s, fp_s = rates(exact.lo, sp.lo)
        assert fn_s == 0
        tot = fn_c + fp_c + fp_s
        if prev is not None:
            assert tot <= prev
        prev = tot
    assert prev < 1e-3


def test_large_filter_is_nearly_exact(lib):
    exact = oracle.kmer_count(lib.bases, lib.offsets, 31, 2)
    W = 1 << 26  # 64 Mi words for 3.5e5 windows
    ct, _ = oracle.approx_count(lib.bases, lib.offsets, 31, "cturtle", 2, W)
    sp, _ = oracle.approx_count(lib.bases, lib.offsets, 31, "single_pass", 2, W)
    assert np.array_equal(ct.lo, exact.lo)
    assert np.array_equal(sp.lo, exact.lo) and np.array_equal(sp.count, exact.count)
