"""Host-side checks of the autotuner's cache (no GPU): choices are stored per
(k, size class) and read back as options."""
import pytest

from paper_1305_1861_amd import tune


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    assert tune.cached_result(31, 10 ** 9, path) is None
    r = tune.TuneResult(part_bits=18, bloom_beta=8, ms=1.5, bloom_bits=3, bucket_tile=1)
    tune._store(path, 31, 10 ** 9, r)
    tune._store(path, 63, 10 ** 9, tune.TuneResult(20, 2, 2.0, 2, 0))
    got = tune.cached_result(31, 10 ** 9 + 5, path)  # same size class
    assert got.cached and (got.part_bits, got.bloom_beta, got.bloom_bits, got.bucket_tile) == (18, 8, 3, 1)
    assert tune.cached_result(31, 10 ** 8, path) is None  # another size class
    assert tune.cached_result(21, 10 ** 9, path) is None  # another k
    o = tune.cached_options(31, 10 ** 9, path)
    assert (o.part_bits, o.bloom_beta, o.bloom_bits, o.bucket_tile) == (18, 8, 3, 1)
    ob = tune.cached_options(31, 10 ** 9, path, with_part_bits=False)
    assert ob.part_bits == -1 and ob.bloom_beta == 8


def test_cache_from_environment(tmp_path, monkeypatch):
    path = str(tmp_path / "env.json")
    tune._store(path, 21, 5000, tune.TuneResult(7, 4, 0.1, 2, 0))
    monkeypatch.setenv(tune.CACHE_ENV, path)
    assert tune.cached_result(21, 5000) is not None
    assert tune.cached_result(21, 5000, cache="") is None  # an empty path turns the cache off
