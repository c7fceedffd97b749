"""GPU parity of key-range shards: the results of shards 0..G-1 of one
library, concatenated in order, equal the oracle (and the unsharded call)
record for record; every shard holds exactly the keys of the pass-1 digits
the ownership rule gives it; the statistics of the shards add up to the
unsharded ones (every bucket meets the same filter)."""
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


def run(tk, bases, offsets, k, c, opts):
    import torch
    db = torch.from_numpy(bases).cuda() if bases.size else torch.zeros(1, dtype=torch.uint8).cuda()[:0]
    do = torch.from_numpy(offsets.view(np.int64)).cuda()
    r = tk.tk_count_device(db, do, k, c, opts)
    torch.cuda.synchronize()
    keys = r.keys.cpu().numpy().view(np.uint64).reshape(r.n, r.key_words).copy()
    counts = r.counts.cpu().numpy().view(np.uint32).copy()
    return keys, counts, r


def first_pass_bits(D):
    """Bits of the first partition pass: all D up to 10, else D - 10 (the
    second pass takes 10)."""
    return D - 10 if D > 10 else D


def expected_owners(oracle_lib, bases, offsets, k, D, G):
    """Pass-1 digit (top first_pass_bits(D) bits of the canonical key) of
    every window, from the oracle's counts at c = 1, and the owner of each
    digit: min(G - 1, floor(G * (below + n / 2) / M))."""
    D1 = first_pass_bits(D)
    allk = oracle_lib.kmer_count(bases, offsets, k, 1)
    if k <= 31:
        dig = (allk.lo >> np.uint64(2 * k - D1)) if D1 else np.zeros(allk.lo.size, np.uint64)
    else:  # 2k - D1 >= 64 - 10 > 64 only for k > 37; split over the two words
        sh = 2 * k - D1
        if sh >= 64:
            dig = allk.hi >> np.uint64(sh - 64)
        else:
            dig = (allk.hi << np.uint64(64 - sh)) | (allk.lo >> np.uint64(sh))
        dig = dig & np.uint64((1 << D1) - 1)
    n = np.bincount(dig.astype(np.int64), weights=allk.count.astype(np.float64), minlength=1 << D1).astype(np.int64)
    M = int(n.sum())
    below = np.concatenate([[0], np.cumsum(n)[:-1]])
    owner = np.minimum(G - 1, (G * (2 * below + n)) // (2 * M)) if M else np.zeros(1 << D1, np.int64)
    return dig, owner, n


def check_shards(tk, oracle_lib, bases, offsets, k, c, G, part_bits=-1):
    base = {"part_bits": part_bits}
    full_k, full_c, full = run(tk, bases, offsets, k, c, base)
    parts = [run(tk, bases, offsets, k, c, dict(base, shard_count=G, shard_index=g)) for g in range(G)]
    keys = np.concatenate([p[0] for p in parts]) if parts else full_k
    counts = np.concatenate([p[1] for p in parts])
    ora = oracle_lib.kmer_count(bases, offsets, k, c)
    if k <= 31:
        assert np.array_equal(keys[:, 0], ora.lo)
    else:
        assert np.array_equal(keys[:, 0], ora.hi) and np.array_equal(keys[:, 1], ora.lo)
    assert np.array_equal(counts.astype(np.uint64), ora.count)
    assert np.array_equal(keys, full_k) and np.array_equal(counts, full_c)
    for f in ("n_windows", "n_collected", "n_distinct", "n_singletons", "n_below_c", "n_fallback"):
        assert sum(getattr(p[2], f) for p in parts) == getattr(full, f), f
    for p in parts:
        assert p[2].part_bits == full.part_bits
    # every shard holds exactly its digits' keys and windows
    D = full.part_bits
    _, owner, n = expected_owners(oracle_lib, bases, offsets, k, D, G)
    D1 = first_pass_bits(D)
    for g, (pk, _, pr) in enumerate(parts):
        assert pr.n_windows == int(n[owner == g].sum()), (g, pr.n_windows)
        if pk.shape[0] and D1:
            sh = 2 * k - D1
            if k <= 31:
                d = pk[:, 0] >> np.uint64(sh)
            elif sh >= 64:
                d = pk[:, 0] >> np.uint64(sh - 64)
            else:
                d = ((pk[:, 0] << np.uint64(64 - sh)) | (pk[:, 1] >> np.uint64(sh))) & np.uint64((1 << D1) - 1)
            assert (owner[d.astype(np.int64)] == g).all()
    return parts


@pytest.mark.parametrize("k", [21, 31, 63])
@pytest.mark.parametrize("G", [2, 3, 8])
def test_shards_concatenate_to_the_full_result(tk, oracle_lib, k, G):
    lib = readsim.small_library(scale=0.05, seed=70 + k)
    case(f"shards G={G} k={k} n_bases={lib.n_bases}")
    parts = check_shards(tk, oracle_lib, lib.bases, lib.offsets, k, 2, G)
    # shares are even to within one digit's windows
    M = sum(p[2].n_windows for p in parts)
    for p in parts:
        assert abs(p[2].n_windows - M / G) <= 0.05 * M, [q[2].n_windows for q in parts]


@pytest.mark.parametrize("c", [1, 3])
def test_shards_thresholds(tk, oracle_lib, c):
    lib = readsim.small_library(scale=0.03, seed=5)
    case(f"shards c={c}")
    check_shards(tk, oracle_lib, lib.bases, lib.offsets, 31, c, 4)


@pytest.mark.parametrize("part_bits", [0, 2, 12])
def test_shards_coarse_digits_and_oversized_buckets(tk, oracle_lib, part_bits):
    """D = 0 (one digit: one shard takes all), D = 2 (four digits, more
    shards than digits, every bucket oversized: the fallback runs per shard),
    D = 12 (two partition passes)."""
    lib = readsim.small_library(scale=0.03, seed=6)
    case(f"shards part_bits={part_bits}")
    check_shards(tk, oracle_lib, lib.bases, lib.offsets, 31, 2, 6, part_bits=part_bits)


def test_shards_noisy_and_empty(tk, oracle_lib):
    b, o = readsim.random_reads(77, 400, 0, 150, n_rate=0.01, lower_rate=0.02, junk_rate=0.002)
    case("shards noisy reads k=33")
    check_shards(tk, oracle_lib, b, o, 33, 2, 5)
    case("shards empty library")
    e_b, e_o = np.zeros(0, np.uint8), np.zeros(1, np.uint64)
    check_shards(tk, oracle_lib, e_b, e_o, 31, 2, 3)
    case("shards one short read")
    s_b, s_o = readsim.from_strings(["ACGTACGTAC"])
    check_shards(tk, oracle_lib, s_b, s_o, 31, 2, 3)
