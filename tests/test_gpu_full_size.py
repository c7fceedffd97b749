"""Full-size parity: the benchmarked libraries counted on the GPU, record by
record against the oracle's exact answer, and the full batched workload
(256 libraries, about 2.8e10 bases, in waves) against single calls and the
oracle.

The oracle's answers are stored as per-key-range digests in
``tests/golden/full_<workload>.json`` (written by
``tests/golden/make_full_digests.py``, which calls only ``oracle/`` and
``readsim/``).  Here the same libraries are generated, counted with
``tk_count_device`` in the bench's configuration (default options, timing
on), and the GPU's records -- split by the same top key bits -- must give the
same counts, sums and SHA-256 digests in every range, and the Bloom
statistics must equal the per-bucket model's.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import readsim

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def tk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1305_1861_amd as tk
    tk.load_library()
    return tk


def _golden(name):
    path = os.path.join(GOLDEN, f"full_{name}.json")
    if not os.path.exists(path):
        pytest.fail(f"{path} is missing: run tests/golden/make_full_digests.py")
    with open(path) as f:
        return json.load(f)


def range_digests(keys: np.ndarray, counts: np.ndarray, k: int, range_bits: int):
    """Per key range (top range_bits bits of the 2k-bit key): records, sum of
    counts and SHA-256 of keys and counts in the output layout."""
    if range_bits == 0:
        top = np.zeros(keys.shape[0], np.uint64)
    elif keys.shape[1] == 1:
        top = keys[:, 0] >> np.uint64(2 * k - range_bits)
    else:
        top = keys[:, 0] >> np.uint64(2 * k - 64 - range_bits)
    assert (np.diff(top.astype(np.int64)) >= 0).all(), "records not in key order"
    edges = np.searchsorted(top, np.arange((1 << range_bits) + 1, dtype=np.uint64))
    out = []
    for r in range(1 << range_bits):
        a, b = int(edges[r]), int(edges[r + 1])
        out.append(dict(n_out=b - a, sum_counts=int(counts[a:b].astype(np.uint64).sum()),
                        sha256_keys=hashlib.sha256(np.ascontiguousarray(keys[a:b], dtype="<u8").tobytes()).hexdigest(),
                        sha256_counts=hashlib.sha256(np.ascontiguousarray(counts[a:b], dtype="<u4").tobytes()).hexdigest()))
    return out


@pytest.mark.parametrize("name", ["large", "long_k"])
def test_full_size_equals_oracle_record_by_record(tk, name):
    import torch
    gold = _golden(name)
    print(f"full size {name}: generating", flush=True)
    lib = readsim.WORKLOADS[name](scale=1.0)
    assert (lib.name, lib.n_bases, lib.n_reads, lib.k, lib.c) == (
        gold["workload"], gold["n_bases"], gold["n_reads"], gold["k"], gold["c"])
    bases = torch.from_numpy(lib.bases).cuda()
    offsets = torch.from_numpy(lib.offsets.view(np.int64)).cuda()
    del lib
    opts = tk.tk_default_options()
    opts.flags = tk.TK_FLAG_TIMING
    print(f"full size {name}: counting", flush=True)
    r = tk.tk_count_device(bases, offsets, gold["k"], gold["c"], opts)
    keys = r.keys.cpu().numpy().view(np.uint64)
    counts = r.counts.cpu().numpy().view(np.uint32)
    assert r.part_bits == gold["part_bits"]
    assert r.n_windows == gold["n_windows"]
    assert r.n == gold["n_out"]
    assert int(counts.astype(np.uint64).sum()) == gold["sum_counts"]
    assert (counts >= gold["c"]).all()
    # Bloom screen statistics: the per-bucket model, exactly
    assert r.n_collected == gold["bloom_n_collected"]
    assert r.n_distinct == gold["bloom_n_distinct"]
    assert r.n_singletons == gold["bloom_n_singletons"]
    got = range_digests(keys, counts, gold["k"], gold["range_bits"])
    for g, want in zip(got, gold["ranges"]):
        for f in ("n_out", "sum_counts", "sha256_keys", "sha256_counts"):
            assert g[f] == want[f], (name, want["index"], f)


def test_batched_workload_full_size(tk):
    """All 256 libraries of the batched workload in waves of at most 2e9
    bases: every library's batch result equals its single call (records and
    statistics), and the smallest, median and largest of every wave equal
    the oracle's digests."""
    import torch
    gold = _golden("batched")
    print("batched full size: generating", flush=True)
    bases, offsets, lib_bases, lib_reads = readsim.batched_workload(gold["n_libs"], 1.0, gold["base_seed"],
                                                                    workers=16)
    waves = readsim.batched_waves(gold["n_libs"], 1.0, gold["base_seed"], gold["wave_bases"])
    db_all = torch.from_numpy(bases).cuda()
    del bases
    need = 0
    plan = []
    for w in waves:
        b0, b1 = int(lib_bases[w[0]]), int(lib_bases[w[-1] + 1])
        r0, r1 = int(lib_reads[w[0]]), int(lib_reads[w[-1] + 1])
        lb = [int(lib_bases[j]) - b0 for j in w] + [b1 - b0]
        lr = [int(lib_reads[j]) - r0 for j in w] + [r1 - r0]
        plan.append((w, b0, b1, r0, r1, lb, lr))
        need = max(need, tk.tk_batch_workspace_size(lb, lr, 31, 2))
        for q in range(len(w)):
            need = max(need, tk.tk_workspace_size(lb[q + 1] - lb[q], lr[q + 1] - lr[q], 31, 2))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")  # the batches' and the single calls'
    print(f"batched full size: {len(plan)} waves, workspace {need / 1e9:.1f} GB", flush=True)
    checked = 0
    for w, b0, b1, r0, r1, lb, lr in plan:
        db = db_all[b0:b1]
        do = torch.from_numpy((offsets[r0:r1 + 1] - np.uint64(b0)).view(np.int64)).cuda()
        res = tk.tk_count_batch_device(db, do, lb, lr, 31, 2, workspace=ws)
        kept = [(r.keys.clone(), r.counts.clone(), r) for r in res]
        for q, (j, (keys, counts, r)) in enumerate(zip(w, kept)):
            s1 = tk.tk_count_device(db[lb[q]:lb[q + 1]], do[lr[q]:lr[q + 1] + 1] - lb[q], 31, 2, workspace=ws)
            assert torch.equal(keys, s1.keys) and torch.equal(counts, s1.counts), j
            assert (r.n_windows, r.n_collected, r.n_distinct, r.n_singletons, r.part_bits) == \
                (s1.n_windows, s1.n_collected, s1.n_distinct, s1.n_singletons, s1.part_bits), j
            g = gold["libraries"].get(str(j))
            if g is None:
                continue
            assert (r.n_windows, r.n, r.part_bits) == (g["n_windows"], g["n_out"], g["part_bits"]), j
            assert (r.n_collected, r.n_distinct, r.n_singletons) == \
                (g["bloom_n_collected"], g["bloom_n_distinct"], g["bloom_n_singletons"]), j
            got = range_digests(keys.cpu().numpy().view(np.uint64), counts.cpu().numpy().view(np.uint32),
                                g["k"], g["range_bits"])
            for a, want in zip(got, g["ranges"]):
                for f in ("n_out", "sum_counts", "sha256_keys", "sha256_counts"):
                    assert a[f] == want[f], (j, want["index"], f)
            checked += 1
        del kept, res
    assert checked == len(gold["libraries"])
