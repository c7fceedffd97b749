"""GPU parity at the largest input the boundary accepts (n_bases < 2^32).

The library is one tile of 10^4 noisy 100-base reads repeated T = 4294
times: 4.294e9 bases, just below 2^32, so window positions, key indices,
bucket starts and scan totals all run near the top of their 32-bit range.
Reads never cross a tile, so every canonical k-mer's count is exactly T
times its count in one tile, which the oracle computes on the tile alone;
with c = 2 every k-mer of the tile is in the answer.  Most buckets hold
more windows than a workgroup (each k-mer occurs T times), so the run also
drives the global-memory fallback at full size.  Device memory: 4.3 GB of
reads and a 162 GB workspace."""
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
