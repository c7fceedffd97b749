"""The autotuner: it times every candidate (bucket bits around the size
rule, filter bits per window), and the options it returns count the library
exactly like the defaults (the counts never depend on those options)."""
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


def host(r):
    return (r.keys.cpu().numpy().view(np.uint64).reshape(r.n, r.key_words).copy(),
            r.counts.cpu().numpy().view(np.uint32).copy())


@pytest.mark.parametrize("k", [31, 63])
def test_autotune_picks_a_timed_candidate_with_the_same_counts(tk, oracle_lib, k):
    import torch
    from paper_1305_1861_amd.tune import autotune
    lib = readsim.small_library(scale=0.1, seed=11)
    case(f"autotune k={k} n_bases={lib.n_bases}")
    b = torch.from_numpy(lib.bases).cuda()
    o = torch.from_numpy(lib.offsets.view(np.int64)).cuda()
    t = autotune(b, o, k, 2, betas=(2, 4), repeats=2)
    D = tk.tk_part_bits(lib.n_bases, lib.n_reads, k)
    assert {(d, be) for d, be, _, _ in t.timings} == {(d, be) for d in (D - 1, D, D + 1) for be in (2, 4)}
    assert all(ms > 0 for _, _, ms, _ in t.timings)
    assert t.ms == min(ms for _, _, ms, _ in t.timings)
    keys, counts = host(tk.tk_count_device(b, o, k, 2, t.options()))
    ref_k, ref_c = host(tk.tk_count_device(b, o, k, 2))
    assert np.array_equal(keys, ref_k) and np.array_equal(counts, ref_c)
    ora = oracle_lib.kmer_count(lib.bases, lib.offsets, k, 2)
    assert np.array_equal(keys[:, -1], ora.lo) and np.array_equal(counts.astype(np.uint64), ora.count)


def test_autotune_workspace_bound(tk):
    import torch
    from paper_1305_1861_amd.tune import autotune
    lib = readsim.small_library(scale=0.02, seed=12)
    b = torch.from_numpy(lib.bases).cuda()
    o = torch.from_numpy(lib.offsets.view(np.int64)).cuda()
    case("autotune with a workspace bound that nothing fits")
    with pytest.raises(ValueError):
        autotune(b, o, 31, 2, max_workspace_bytes=1)
