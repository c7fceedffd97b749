"""Phased sort-and-compact: the library streamed in chunks, each chunk's
records merged into a resident sorted-and-compacted array.  The answer must
not depend on the chunk size and equals the oracle's, with the global
filter's exact statistics."""
import sys

import numpy as np
import pytest

import readsim

pytestmark = pytest.mark.gpu


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


def check(oracle_lib, bases, offsets, k, c, r):
    ora = oracle_lib.kmer_count(bases, offsets, k, c)
    assert r.keys.shape[0] == ora.lo.size
    if k <= 31:
        assert (r.keys[:, 0] == ora.lo).all()
    else:
        assert (r.keys[:, 0] == ora.hi).all() and (r.keys[:, 1] == ora.lo).all()
    assert (r.counts.astype(np.uint64) == ora.count).all()
    assert r.n_windows == ora.n_windows
    if c >= 2:
        nb = oracle_lib.default_blocks(bases.size, offsets.size - 1, k, 4)
        m = oracle_lib.bloom_model(bases, offsets, k, nb, 1024, 2, 1305)
        assert (r.n_collected, r.n_distinct, r.n_singletons) == (m.n_cand_occ, m.n_cand, m.n_cand_single)
        assert r.bloom_blocks == nb


@pytest.mark.parametrize("k", [21, 31, 63])
@pytest.mark.parametrize("chunk", [137, 5_000, 60_000, 10 ** 9])
def test_phased_independent_of_chunk_size(tk, oracle_lib, k, chunk):
    lib = readsim.small_library(scale=0.05, seed=3 + k)
    case(f"phased k={k} chunk={chunk} n_bases={lib.n_bases}")
    r = tk.tk_count_phased(lib.bases, lib.offsets, k, 2, chunk)
    check(oracle_lib, lib.bases, lib.offsets, k, 2, r)


@pytest.mark.parametrize("c", [1, 3])
def test_phased_thresholds_and_noise(tk, oracle_lib, c):
    bases, offsets = readsim.random_reads(61, 3000, 0, 160, n_rate=0.01, lower_rate=0.02, junk_rate=0.002)
    dup = readsim.to_strings(bases, offsets)
    bases, offsets = readsim.from_strings(dup + dup[::3])
    case(f"phased noisy reads c={c}")
    r = tk.tk_count_phased(bases, offsets, 31, c, 2_000)
    check(oracle_lib, bases, offsets, 31, c, r)


def test_phased_matches_global_filter_path(tk, oracle_lib):
    lib = readsim.small_library(scale=0.2)
    case("phased vs global-filter host path")
    r = tk.tk_count_phased(lib.bases, lib.offsets, lib.k, lib.c, 100_000)
    g = tk.tk_count(lib.bases, lib.offsets, lib.k, lib.c, dict(flags=2))
    assert np.array_equal(r.keys, g.keys) and np.array_equal(r.counts, g.counts)
    assert (r.n_windows, r.n_collected, r.n_distinct, r.n_singletons) == \
        (g.n_windows, g.n_collected, g.n_distinct, g.n_singletons)


def test_phased_capacity_bounds_memory_and_is_enforced(tk, oracle_lib):
    lib = readsim.small_library(scale=0.2)
    case("phased memory bound")
    full = tk.tk_count_phased(lib.bases, lib.offsets, lib.k, lib.c, 200_000, sac_capacity=0)
    tight = tk.tk_count_phased(lib.bases, lib.offsets, lib.k, lib.c, 200_000, sac_capacity=full.n_distinct)
    assert np.array_equal(full.keys, tight.keys) and np.array_equal(full.counts, tight.counts)
    assert tight.device_bytes < full.device_bytes
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_count_phased(lib.bases, lib.offsets, lib.k, lib.c, 200_000, sac_capacity=full.n_distinct // 2)
    assert e.value.status == tk.TK_ENOMEM


def test_phased_empty_and_tiny(tk, oracle_lib):
    for reads in ([], [""], ["ACGT"], ["A" * 50, "N" * 10, "ACGTACGTAC" * 8]):
        bases, offsets = readsim.from_strings(reads)
        r = tk.tk_count_phased(bases, offsets, 5, 2, 16)
        check(oracle_lib, bases, offsets, 5, 2, r)
