"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol declared in include/turtle.h, and its host logic (options, filter size
rule, pattern table, argument checks) agrees with the oracle's independent
implementation of the same documented rules."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1305_1861_amd as tk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "turtle.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tk.LIB_PATH):
        from paper_1305_1861_amd import build
        build.build()
    return tk.load_library()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"TK_API\s+[\w\s\*]*?\b(tk_\w+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for want in ("tk_count", "tk_count_device", "tk_workspace_size", "tk_result_free", "tk_strerror"):
        assert want in names
    assert sorted(tk.exported_symbols()) == names


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(tk.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name


def test_default_options(lib):
    o = tk.tk_default_options()
    assert (o.bloom_beta, o.bloom_table_bits, o.bloom_bits, o.bloom_seed, o.bloom_blocks) == (4, 10, 2, 1305, 0)
    assert o.part_bits == -1 and o.flags == 0


def test_strerror(lib):
    assert tk.tk_strerror(0) == "ok"
    assert "invalid" in tk.tk_strerror(-1)
    assert tk.tk_strerror(-4)


def test_pattern_table_matches_oracle(oracle_lib, lib):
    for bits, table_bits, seed in [(2, 10, 1305), (1, 4, 7), (3, 9, 99), (16, 6, 5)]:
        got = tk.tk_pattern_table(dict(bloom_bits=bits, bloom_table_bits=table_bits, bloom_seed=seed))
        want = oracle_lib.pattern_masks(1 << table_bits, bits, seed)
        assert (got == want).all()


@pytest.mark.parametrize("n_bases,n_reads,k", [(0, 0, 31), (10_000_000, 100_000, 31), (99, 1, 63),
                                               (5, 5, 21), (1_500_000_000, 15_000_000, 31)])
def test_bloom_size_rule_matches_oracle(oracle_lib, lib, n_bases, n_reads, k):
    for beta in (1, 4, 7):
        assert tk.tk_bloom_blocks(n_bases, n_reads, k, dict(bloom_beta=beta)) == \
            oracle_lib.default_blocks(n_bases, n_reads, k, beta)
    assert tk.tk_bloom_blocks(n_bases, n_reads, k, dict(bloom_blocks=12345)) == 12345


@pytest.mark.parametrize("n_bases,n_reads,k", [(0, 0, 31), (10_000_000, 100_000, 31), (99, 1, 63),
                                               (5, 5, 2), (1_500_000_000, 15_000_000, 31),
                                               (800_000_000, 5_333_333, 63), (4095, 1, 1), (1 << 31, 1, 40)])
def test_partition_rule_matches_oracle(oracle_lib, lib, n_bases, n_reads, k):
    assert tk.tk_part_bits(n_bases, n_reads, k) == oracle_lib.partition_bits(n_bases, n_reads, k)
    for explicit in (0, 3, 20):
        assert tk.tk_part_bits(n_bases, n_reads, k, dict(part_bits=explicit)) == \
            oracle_lib.partition_bits(n_bases, n_reads, k, explicit)


def test_partition_rule_values(lib):
    # the workloads: about 2^11 (one-word keys) or 2^10 (two-word keys) windows per bucket
    assert tk.tk_part_bits(1_500_000_000, 15_000_000, 31) == 19
    assert tk.tk_part_bits(10_000_000, 100_000, 31) == 12
    assert tk.tk_part_bits(800_000_000, 5_333_333, 63) == 19
    assert tk.tk_part_bits(100, 1, 1) == 0


def test_workspace_size_grows(lib):
    a = tk.tk_workspace_size(1000, 10, 31, 2)
    b = tk.tk_workspace_size(100_000, 1000, 31, 2)
    c = tk.tk_workspace_size(100_000, 1000, 63, 2)
    assert 0 < a < b < c
    # c = 1 needs no filter
    assert tk.tk_workspace_size(100_000, 1000, 31, 1) < b
    assert tk.tk_workspace_size(0, 0, 5, 2) > 0


@pytest.mark.parametrize("k,c", [(0, 2), (64, 2), (-3, 2), (31, 0)])
def test_bad_arguments_rejected(lib, k, c):
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_workspace_size(100, 1, k, c)
    assert e.value.status == tk.TK_EINVAL
    # the host entry point checks before touching any device
    b = np.frombuffer(b"ACGTACGT", np.uint8).copy()
    o = np.array([0, 8], np.uint64)
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_count(b, o, k, c)
    assert e.value.status == tk.TK_EINVAL


def test_bad_offsets_rejected(lib):
    b = np.frombuffer(b"ACGTACGT", np.uint8).copy()
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_count(b, np.array([0, 6, 3, 8], np.uint64), 3, 2)
    assert e.value.status == tk.TK_EINVAL and "decrease" in str(e.value)
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_count(b, np.array([1, 8], np.uint64), 3, 2)
    assert e.value.status == tk.TK_EINVAL


def test_overflow_rejected(lib):
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_workspace_size(1 << 32, 10, 31, 2)
    assert e.value.status == tk.TK_EOVERFLOW


def test_bad_options_rejected(lib):
    for bad in (dict(bloom_table_bits=11), dict(bloom_bits=17), dict(bloom_beta=5000),
                dict(bloom_beta=33), dict(part_bits=21), dict(part_bits=-2)):
        with pytest.raises(tk.TurtleError) as e:
            tk.tk_workspace_size(1000, 10, 31, 2, bad)
        assert e.value.status == tk.TK_EINVAL


def test_last_error_message(lib):
    with pytest.raises(tk.TurtleError):
        tk.tk_workspace_size(100, 1, 99, 2)
    assert "k = 99" in tk.tk_last_error()


def test_batch_workspace_of_one_library_equals_single(lib):
    for n_bases, n_reads, k, c in [(100_000, 1000, 31, 2), (10_000_000, 100_000, 63, 2), (0, 0, 5, 1)]:
        assert tk.tk_batch_workspace_size([0, n_bases], [0, n_reads], k, [c]) == \
            tk.tk_workspace_size(n_bases, n_reads, k, c)


@pytest.mark.parametrize("n_libs", [2, 7, 100])
def test_batch_workspace_bounded_by_its_libraries(lib, n_libs):
    """A batch needs at least its largest library's workspace and at most
    the sum of its libraries' workspaces."""
    rng = np.random.default_rng(n_libs)
    nb = rng.integers(0, 400_000, n_libs)
    nr = nb // 100
    lb = np.concatenate([[0], np.cumsum(nb)])
    lr = np.concatenate([[0], np.cumsum(nr)])
    singles = [tk.tk_workspace_size(int(b), int(r), 31, 2) for b, r in zip(nb, nr)]
    batch = tk.tk_batch_workspace_size(lb, lr, 31, 2)
    assert max(singles) <= batch <= sum(singles)


@pytest.mark.parametrize("lb,lr,c,opts,what", [
    ([0, 10, 5], [0, 1, 2], [2, 2], None, "decrease"),
    ([0, 10, 20], [0, 2, 1], [2, 2], None, "decrease"),
    ([1, 10], [0, 1], [2], None, "start at 0"),
    ([0, 10, 20], [0, 1, 2], [2, 0], None, "threshold"),
    ([0, 10, 20], [0, 1, 2], [2, 2], dict(flags=2), "one library"),
    ([0, 10, 20], [0, 1, 2], [2, 2], dict(part_bits=20), "buckets"),
])
def test_batch_bad_arguments_rejected(lib, lb, lr, c, opts, what):
    if what == "buckets":
        # 2^20 buckets per library: too many over 2048 libraries
        lb = list(range(0, 20 * 2049, 20))
        lr = list(range(0, 2049))
        c = [2] * 2048
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_batch_workspace_size(lb, lr, 31, c, opts)
    assert e.value.status == tk.TK_EINVAL and what in str(e.value)


@pytest.mark.parametrize("opts,what", [
    (dict(shard_count=4, shard_index=4), "shard"),
    (dict(shard_count=2000, shard_index=0), "shard"),
    (dict(shard_count=0, shard_index=1), "shard"),
    (dict(shard_count=2, shard_index=0, flags=2), "partitioned"),
    (dict(shard_count=2, shard_index=1, flags=4), "partitioned"),
])
def test_bad_shards_rejected(lib, opts, what):
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_workspace_size(100_000, 1000, 31, 2, opts)
    assert e.value.status == tk.TK_EINVAL and what in str(e.value)


def test_shards_split_one_library_per_call(lib):
    with pytest.raises(tk.TurtleError) as e:
        tk.tk_batch_workspace_size([0, 500, 1000], [0, 5, 10], 31, [2, 2], dict(shard_count=2, shard_index=0))
    assert e.value.status == tk.TK_EINVAL and "shard" in str(e.value)
    # one shard of one library: the same buffers plus the digit table
    one = tk.tk_workspace_size(10_000_000, 100_000, 31, 2)
    sh = tk.tk_workspace_size(10_000_000, 100_000, 31, 2, dict(shard_count=8, shard_index=3))
    assert one <= sh <= one + 8192


# ---- binding-side checks of device arguments (rejected before the library
# is called, so CPU tensors reach every check but the device one) ----

def _t():
    import torch
    return torch


@pytest.mark.parametrize("case", ["bases_dtype", "offsets_int32", "offsets_float", "noncontig", "empty_offsets"])
def test_binding_rejects_bad_device_reads(lib, case):
    torch = _t()
    bases = torch.zeros(64, dtype=torch.uint8)
    offsets = torch.tensor([0, 32, 64], dtype=torch.int64)
    if case == "bases_dtype":
        bases = bases.to(torch.int16)
    elif case == "offsets_int32":
        offsets = offsets.to(torch.int32)
    elif case == "offsets_float":
        offsets = offsets.to(torch.float64)
    elif case == "noncontig":
        bases = torch.zeros(128, dtype=torch.uint8)[::2]
    elif case == "empty_offsets":
        offsets = torch.zeros(0, dtype=torch.int64)
    with pytest.raises(ValueError):
        tk.tk_count_device(bases, offsets, 31, 2)
    with pytest.raises(ValueError):
        tk.tk_count_batch_device(bases, offsets, [0, 64], [0, 2], 31, 2)


def test_binding_rejects_host_tensors(lib):
    torch = _t()
    with pytest.raises(ValueError, match="CUDA"):
        tk.tk_count_device(torch.zeros(64, dtype=torch.uint8), torch.tensor([0, 64]), 31, 2)


@pytest.mark.parametrize("lb,lr", [([0, 65], [0, 2]), ([0, 64], [0, 3]), ([0, 32, 70], [0, 1, 2])])
def test_binding_rejects_short_batch_tensors(lib, lb, lr):
    torch = _t()
    bases = torch.zeros(64, dtype=torch.uint8)
    offsets = torch.tensor([0, 32, 64], dtype=torch.int64)
    with pytest.raises(ValueError, match="at least"):
        tk.tk_count_batch_device(bases, offsets, lb, lr, 31, 2)


def test_batch_workspace_mixed_k(lib):
    """Libraries of both key widths: two counting passes, each in its own
    part of the workspace."""
    lb, lr = [0, 5000, 9000, 20000], [0, 50, 90, 200]
    one = tk.tk_batch_workspace_size(lb, lr, [21, 31, 31], 2)
    two = tk.tk_batch_workspace_size(lb, lr, [55, 63, 33], 2)
    mixed = tk.tk_batch_workspace_size(lb, lr, [21, 63, 31], 2)
    assert mixed > 0 and mixed < one + two
    assert mixed >= tk.tk_batch_workspace_size(lb, lr, [21, 31, 31], 2) * 0.5


@pytest.mark.parametrize("k", [[31, 0, 31], [31, 64, 21], [-1, 21, 21]])
def test_batch_bad_k_rejected(lib, k):
    with pytest.raises(tk.TurtleError):
        tk.tk_batch_workspace_size([0, 100, 200, 300], [0, 1, 2, 3], k, 2)
