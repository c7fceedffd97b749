"""The autotuner: it times every candidate (bucket bits around the size
rule, filter bits per window, pattern bits, bucket-kernel tile shape), the
options it returns count the library exactly like the defaults (the counts
never depend on those options), and a cached choice is reused untimed by the
tuner, by batches and by the server."""
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
    t = autotune(b, o, k, 2, betas=(2, 4), bloom_bits=(2, 3), tiles=(0, 1), repeats=2, cache="")
    D = tk.tk_part_bits(lib.n_bases, lib.n_reads, k)
    assert {x[:4] for x in t.timings} == {(d, be, bi, ti) for d in (D - 1, D, D + 1) for be in (2, 4)
                                          for bi in (2, 3) for ti in (0, 1)}
    assert all(x[4] > 0 for x in t.timings)
    assert t.ms == min(x[4] for x in t.timings)
    ref_k, ref_c = host(tk.tk_count_device(b, o, k, 2))
    ora = oracle_lib.kmer_count(lib.bases, lib.offsets, k, 2)
    assert np.array_equal(ref_k[:, -1], ora.lo) and np.array_equal(ref_c.astype(np.uint64), ora.count)
    # every candidate, not only the fastest, counts exactly
    for D_, be, bi, ti, _, _ in t.timings:
        opt = tk.tk_default_options()
        opt.part_bits, opt.bloom_beta, opt.bloom_bits, opt.bucket_tile = D_, be, bi, ti
        keys, counts = host(tk.tk_count_device(b, o, k, 2, opt))
        assert np.array_equal(keys, ref_k) and np.array_equal(counts, ref_c), (D_, be, bi, ti)


def test_tile_shapes_and_fallback(tk, oracle_lib):
    """Tile 1 holds fewer keys per group, so more buckets go to the fallback
    at a small D; the counts stay exact."""
    import torch
    lib = readsim.small_library(scale=0.2, seed=13)
    b = torch.from_numpy(lib.bases).cuda()
    o = torch.from_numpy(lib.offsets.view(np.int64)).cuda()
    ora = oracle_lib.kmer_count(lib.bases, lib.offsets, 31, 2)
    fb = []
    for tile in (0, 1):
        opt = tk.tk_default_options()
        opt.bucket_tile, opt.part_bits = tile, 9
        r = tk.tk_count_device(b, o, 31, 2, opt)
        keys, counts = host(r)
        assert np.array_equal(keys[:, 0], ora.lo) and np.array_equal(counts.astype(np.uint64), ora.count)
        fb.append(r.n_fallback)
    assert fb[1] >= fb[0]


def test_cached_choice_is_reused(tk, oracle_lib, tmp_path, monkeypatch):
    import torch
    from paper_1305_1861_amd import tune
    from paper_1305_1861_amd.serve import Job, Server
    path = str(tmp_path / "tune.json")
    lib = readsim.small_library(scale=0.05, seed=14)
    b = torch.from_numpy(lib.bases).cuda()
    o = torch.from_numpy(lib.offsets.view(np.int64)).cuda()
    case("autotune with a cache file")
    t1 = tune.autotune(b, o, 31, 2, betas=(2, 8), bloom_bits=(2,), tiles=(0, 1), repeats=1, cache=path)
    assert not t1.cached and len(t1.timings) == 3 * 2 * 2
    t2 = tune.autotune(b, o, 31, 2, cache=path)
    assert t2.cached and t2.timings == []
    assert (t2.part_bits, t2.bloom_beta, t2.bloom_bits, t2.bucket_tile) == \
        (t1.part_bits, t1.bloom_beta, t1.bloom_bits, t1.bucket_tile)
    # a batch and the server take the cached batch-wide options
    monkeypatch.setenv(tune.CACHE_ENV, path)
    want = tk.tk_count_device(b, o, 31, 2, t2.options(with_part_bits=False))
    wk, wc = host(want)
    (r,) = tk.tk_count_batch_device(b, o, [0, lib.n_bases], [0, lib.n_reads], 31, 2)
    gk, gc = host(r)
    assert np.array_equal(gk, wk) and np.array_equal(gc, wc)
    assert (r.n_collected, r.n_singletons) == (want.n_collected, want.n_singletons)
    srv = Server(hbm_bytes=1 << 29, workers=1)
    try:
        res = srv.submit(Job(lib.bases, lib.offsets, 31, 2)).result(timeout=120)
    finally:
        srv.close()
    assert np.array_equal(res.keys, wk) and np.array_equal(res.counts, wc)
    assert (res.n_collected, res.n_singletons) == (want.n_collected, want.n_singletons)
    ora = oracle_lib.kmer_count(lib.bases, lib.offsets, 31, 2)
    assert np.array_equal(res.keys[:, 0], ora.lo) and np.array_equal(res.counts.astype(np.uint64), ora.count)


def test_autotune_workspace_bound(tk):
    import torch
    from paper_1305_1861_amd.tune import autotune
    lib = readsim.small_library(scale=0.02, seed=12)
    b = torch.from_numpy(lib.bases).cuda()
    o = torch.from_numpy(lib.offsets.view(np.int64)).cuda()
    case("autotune with a workspace bound that nothing fits")
    with pytest.raises(ValueError):
        autotune(b, o, 31, 2, max_workspace_bytes=1, cache="")
