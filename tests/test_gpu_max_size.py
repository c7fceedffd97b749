"""GPU parity at the largest input the boundary accepts (n_bases < 2^32).

The library is one tile of 10^4 noisy 100-base reads repeated T = 4294
times: 4.294e9 bases, just below 2^32, so window positions, key indices,
bucket starts and scan totals all run near the top of their 32-bit range.
Reads never cross a tile, so every canonical k-mer's count is exactly T
times its count in one tile, which the oracle computes on the tile alone;
with c = 2 every k-mer of the tile is in the answer.  Most buckets hold
more windows than a workgroup (each k-mer occurs T times), so the run also
drives the global-memory fallback at full size.  Device memory: 4.3 GB of
reads and a 162 GB workspace.

A second case takes two-word keys (k = 63) past 2^31 windows, so that
their 64-bit word offsets pass 2^32: one read of 3e9 bases, a random tile
of 10^6 bases repeated R = 3000 times.  Window p is the tile's cyclic
k-mer at p mod 10^6, so a key's count is R times its multiplicity among
the tile's cyclic windows less its multiplicity among the k - 1 windows
that wrap (those occur R - 1 times); the oracle counts both on short
strings.  Device memory: 3 GB of reads and a 186 GB workspace."""
import gc
import sys

import numpy as np
import pytest

import readsim

pytestmark = pytest.mark.gpu

T = 4294
READS, L, K, C = 10_000, 100, 31, 2


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


def test_largest_accepted_library(tk, oracle_lib):
    import torch
    tile_b, tile_o = readsim.random_reads(4242, READS, L, L, n_rate=0.01, lower_rate=0.02, junk_rate=0.002)
    assert tile_b.size == READS * L
    n_bases = T * tile_b.size
    assert n_bases < 1 << 32
    ora = oracle_lib.kmer_count(tile_b, tile_o, K, 1)
    case(f"max size: {T} tiles, n_bases={n_bases}, tile distinct={ora.lo.size}")
    gc.collect()
    torch.cuda.empty_cache()
    db = torch.from_numpy(np.tile(tile_b, T)).cuda()
    do = torch.arange(0, n_bases + 1, L, dtype=torch.int64).cuda()
    assert do.numel() == T * READS + 1
    ws = torch.empty(tk.tk_workspace_size(n_bases, T * READS, K, C), dtype=torch.uint8, device="cuda")
    case(f"max size: workspace {ws.numel() / 1e9:.1f} GB, counting")
    r = tk.tk_count_device(db, do, K, C, workspace=ws)
    torch.cuda.synchronize()
    keys = r.keys.cpu().numpy().view(np.uint64).reshape(-1, 1)[:, 0].copy()
    counts = r.counts.cpu().numpy().view(np.uint32).copy()
    n_windows = r.n_windows
    case(f"max size: {keys.size} records, {r.n_fallback} oversized buckets")
    del r, ws, db, do
    gc.collect()
    torch.cuda.empty_cache()
    assert n_windows == T * ora.n_windows
    assert keys.size == ora.lo.size
    assert np.array_equal(keys, ora.lo)
    assert np.array_equal(counts.astype(np.uint64), ora.count * np.uint64(T))


def test_longest_read_two_word_keys(tk, oracle_lib):
    import torch
    P, R, k = 1_000_000, 3000, 63
    rng = np.random.default_rng(6363)
    tile = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, P)]
    cyc = np.concatenate([tile, tile[:k - 1]])  # every cyclic window once
    wrap = cyc[P - k + 1:]                     # the k - 1 windows that wrap
    one = lambda x: np.array([0, x.size], np.uint64)  # noqa: E731
    m = oracle_lib.kmer_count(cyc, one(cyc), k, 1)
    w = oracle_lib.kmer_count(wrap, one(wrap), k, 1)
    mk = (m.hi.astype(object) << 64) | m.lo.astype(object)
    wk = (w.hi.astype(object) << 64) | w.lo.astype(object)
    pos = np.searchsorted(mk, wk)
    assert (mk[pos] == wk).all()
    want = m.count * np.uint64(R)
    np.subtract.at(want, pos, w.count)
    n_bases = P * R
    case(f"longest read: k={k}, n_bases={n_bases}, tile distinct={m.lo.size}")
    gc.collect()
    torch.cuda.empty_cache()
    db = torch.from_numpy(np.tile(tile, R)).cuda()
    do = torch.tensor([0, n_bases], dtype=torch.int64).cuda()
    ws = torch.empty(tk.tk_workspace_size(n_bases, 1, k, C), dtype=torch.uint8, device="cuda")
    case(f"longest read: workspace {ws.numel() / 1e9:.1f} GB, counting")
    r = tk.tk_count_device(db, do, k, C, workspace=ws)
    torch.cuda.synchronize()
    keys = r.keys.cpu().numpy().view(np.uint64).reshape(-1, 2).copy()
    counts = r.counts.cpu().numpy().view(np.uint32).copy()
    n_windows = r.n_windows
    case(f"longest read: {keys.shape[0]} records, {r.n_fallback} oversized buckets")
    del r, ws, db, do
    gc.collect()
    torch.cuda.empty_cache()
    assert n_windows == n_bases - k + 1 > 1 << 31
    assert keys.shape[0] == m.lo.size
    assert np.array_equal(keys[:, 0], m.hi) and np.array_equal(keys[:, 1], m.lo)
    assert np.array_equal(counts.astype(np.uint64), want)
