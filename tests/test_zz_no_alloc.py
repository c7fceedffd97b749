"""The allocation-free entry point (static device workspace) against
tk_count_device, through the C ABI, on the GPU."""
import numpy as np
import pytest

import readsim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1305_1861_amd as tk
    tk.load_library()
    return tk


def _dev(lib):
    import torch
    b = torch.from_numpy(lib.bases).cuda()
    o = torch.from_numpy(lib.offsets.view(np.int64)).cuda()
    return b, o


def _same(a, b):
    import torch
    assert a.n == b.n and a.key_words == b.key_words
    assert torch.equal(a.keys.cpu(), b.keys.cpu())
    assert torch.equal(a.counts.cpu(), b.counts.cpu())
    for f in ("n_windows", "n_collected", "n_distinct", "n_singletons", "n_below_c", "part_bits", "n_fallback"):
        assert getattr(a, f) == getattr(b, f), f


def test_static_workspace_matches_device_call_twice(tk):
    """Two calls in a row, the second on a smaller library: the array keeps
    the first call's contents and the second must not see them."""
    import torch
    big = readsim.small_library(scale=0.5, seed=21)       # 5e6 bases, ~190 MB of workspace
    small = readsim.small_library(scale=0.08, seed=22)
    assert tk.tk_workspace_size(big.n_bases, big.n_reads, 31, 2) <= tk.STATIC_WORKSPACE_BYTES
    out_k = torch.empty(big.n_bases, dtype=torch.int64, device="cuda")
    out_c = torch.empty(big.n_bases, dtype=torch.int32, device="cuda")
    for lib in (big, small):
        b, o = _dev(lib)
        print(f"static workspace: {lib.name} {lib.n_bases} bases", flush=True)
        want = tk.tk_count_device(b, o, lib.k, lib.c)
        got = tk.tk_count_device_static(b, o, lib.k, lib.c, out_k, out_c)
        torch.cuda.synchronize()
        _same(got, want)
        assert got.keys.data_ptr() == out_k.data_ptr()


@pytest.mark.parametrize("k,c", [(63, 2), (21, 1), (33, 3)])
def test_static_workspace_other_k(tk, k, c):
    import torch
    bases, offsets = readsim.random_reads(3100 + k, 20000, min_len=0, max_len=150)
    bases = np.concatenate([bases, bases])
    offsets = np.concatenate([offsets, offsets[1:] + offsets[-1]])
    lib = readsim.Library("random", k, c, bases, offsets)
    b, o = _dev(lib)
    out_k = torch.empty(2 * lib.n_bases, dtype=torch.int64, device="cuda")
    out_c = torch.empty(lib.n_bases, dtype=torch.int32, device="cuda")
    want = tk.tk_count_device(b, o, k, c)
    got = tk.tk_count_device_static(b, o, k, c, out_k, out_c)
    torch.cuda.synchronize()
    _same(got, want)


def test_static_workspace_refuses_what_does_not_fit(tk):
    import torch
    lib = readsim.small_library(scale=1.0, seed=23)  # 1e7 bases: ~360 MB of workspace
    b, o = _dev(lib)
    out_k = torch.empty(16, dtype=torch.int64, device="cuda")
    out_c = torch.empty(16, dtype=torch.int32, device="cuda")
    with pytest.raises(tk.TurtleError, match="static workspace"):
        tk.tk_count_device_static(b, o, lib.k, lib.c, out_k, out_c)
    # a library that fits but whose records exceed the output buffers
    small = readsim.small_library(scale=0.05, seed=24)
    b, o = _dev(small)
    with pytest.raises(tk.TurtleError, match="output capacity"):
        tk.tk_count_device_static(b, o, small.k, small.c, out_k, out_c)
    # the next call still gives the right answer
    out_k = torch.empty(small.n_bases, dtype=torch.int64, device="cuda")
    out_c = torch.empty(small.n_bases, dtype=torch.int32, device="cuda")
    want = tk.tk_count_device(b, o, small.k, small.c)
    got = tk.tk_count_device_static(b, o, small.k, small.c, out_k, out_c)
    torch.cuda.synchronize()
    _same(got, want)
