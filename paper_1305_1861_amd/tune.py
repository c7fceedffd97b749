"""Autotuning of the counting options on one device, with a persistent cache.

The result of a counting call does not depend on the options tuned here --
every count is exact; only the number of screen false positives (and so the
work of the sort) and the speed change -- so they can be chosen for speed
alone:

* ``part_bits``  -- bucket bits D around the size rule (the buckets'
  filters and sorts live in one workgroup's LDS; smaller D means larger
  buckets, some too large for a group and sent to the fallback kernels);
* ``bloom_beta`` -- first-plane filter bits per window (filter size);
* ``bloom_bits`` -- bits each pattern table entry sets in a 64-bit block
  word (K/4 of the pattern bits a key sets in its 64-byte block);
* ``bucket_tile`` -- the bucket kernel's tile shape: 14 one-word (7
  two-word) keys per thread per group, or 12 (6).

The filter block (64 bytes: a 256-bit first plane and a 256-bit second
plane) and the sort digit widths (12-bit MSD pass, 9-bit LSD passes inside
the bucket kernel, 8-bit LSD passes of the global-memory sorts) are fixed by
the kernels' LDS layouts and are not tuned.

``autotune`` times ``tk_count_device`` on the caller's device-resident
library for every candidate and returns the fastest options with every
timing.  With a cache file (argument, or the environment variable
``TK_TUNE_CACHE``), the choice is stored per (k, size class = bit length of
the number of bases) and a later call for the same class returns it without
timing; ``cached_options`` reads it back for ``tk_count_batch_device`` and
the server.
"""
from __future__ import annotations

import json
import os
import threading
from dataclasses import dataclass, field

from . import STAGES, _torch, tk_count_device, tk_default_options, tk_part_bits, tk_workspace_size

CACHE_ENV = "TK_TUNE_CACHE"
_lock = threading.Lock()


@dataclass
class TuneResult:
    part_bits: int
    bloom_beta: int
    ms: float
    bloom_bits: int = 2
    bucket_tile: int = 0
    timings: list = field(default_factory=list)  # (part_bits, bloom_beta, bloom_bits, bucket_tile, ms, n_fallback)
    cached: bool = False

    def options(self, flags: int = 0, with_part_bits: bool = True):
        o = tk_default_options()
        if with_part_bits:
            o.part_bits = self.part_bits
        o.bloom_beta = self.bloom_beta
        o.bloom_bits = self.bloom_bits
        o.bucket_tile = self.bucket_tile
        o.flags = flags
        return o


def size_class(n_bases: int) -> int:
    return int(n_bases).bit_length()


def cache_key(k: int, n_bases: int) -> str:
    return f"k{int(k)}/b{size_class(n_bases)}"


def _cache_path(cache):
    if cache is None:
        return os.environ.get(CACHE_ENV) or None
    return cache or None


def _read(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def cached_result(k: int, n_bases: int, cache=None) -> TuneResult | None:
    """The stored choice for (k, size class of n_bases), or None."""
    path = _cache_path(cache)
    if not path:
        return None
    with _lock:
        e = _read(path).get(cache_key(k, n_bases))
    if not e:
        return None
    return TuneResult(e["part_bits"], e["bloom_beta"], e["ms"], e["bloom_bits"], e["bucket_tile"], cached=True)


def cached_options(k: int, n_bases: int, cache=None, with_part_bits: bool = True, flags: int = 0):
    """Options of the stored choice, or None when there is none.  For a
    batch (``with_part_bits=False``) every library keeps the size rule's D
    and only the batch-wide options are taken."""
    r = cached_result(k, n_bases, cache)
    return r.options(flags, with_part_bits) if r else None


def _store(path, k, n_bases, r: TuneResult):
    with _lock:
        doc = _read(path)
        doc[cache_key(k, n_bases)] = dict(part_bits=r.part_bits, bloom_beta=r.bloom_beta, bloom_bits=r.bloom_bits,
                                          bucket_tile=r.bucket_tile, ms=r.ms)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def autotune(bases, offsets, k: int, c: int, part_bits=None, betas=(2, 4, 8), bloom_bits=(2, 3), tiles=(0, 1),
             repeats: int = 3, max_workspace_bytes: int | None = None, stream=None, cache=None,
             refresh: bool = False) -> TuneResult:
    """Fastest (part_bits, bloom_beta, bloom_bits, bucket_tile) for this library.

    ``bases``/``offsets``: device tensors as for ``tk_count_device``.
    ``part_bits``: candidate D values (default: the size rule's D - 1, D,
    D + 1, within 0..20).  Device time per candidate: the summed stage
    times (HIP events) of the fastest of ``repeats`` calls after one warm-up.
    ``cache``: cache file (default: ``$TK_TUNE_CACHE``; None there: no
    cache); a stored choice for this (k, size class) is returned untimed
    unless ``refresh``.
    """
    torch = _torch()
    n_bases = int(bases.numel())
    n_reads = int(offsets.numel()) - 1
    path = _cache_path(cache)
    if path and not refresh:
        hit = cached_result(k, n_bases, path)
        if hit is not None:
            return hit
    if part_bits is None:
        d = tk_part_bits(n_bases, n_reads, k)
        part_bits = sorted({x for x in (d - 1, d, d + 1) if 0 <= x <= 20})
    timings = []
    best = None
    ws = None
    for D in part_bits:
        for beta in betas:
            for bits in bloom_bits:
                for tile in tiles:
                    o = tk_default_options()
                    o.part_bits, o.bloom_beta, o.bloom_bits, o.bucket_tile = D, beta, bits, tile
                    o.flags = 1  # stage timing
                    need = tk_workspace_size(n_bases, n_reads, k, c, o)
                    if max_workspace_bytes is not None and need > max_workspace_bytes:
                        continue
                    if ws is None or ws.numel() < need:
                        ws = None
                        ws = torch.empty(need, dtype=torch.uint8, device=bases.device)
                    tk_count_device(bases, offsets, k, c, o, workspace=ws, stream=stream)
                    ms = float("inf")
                    for _ in range(repeats):
                        r = tk_count_device(bases, offsets, k, c, o, workspace=ws, stream=stream)
                        ms = min(ms, sum(r.stage_ms[s] for s in STAGES))
                    timings.append((D, beta, bits, tile, ms, int(r.n_fallback)))
                    if best is None or ms < best[4]:
                        best = (D, beta, bits, tile, ms)
    if best is None:
        raise ValueError("no candidate fits the workspace bound")
    res = TuneResult(best[0], best[1], best[4], best[2], best[3], timings)
    if path:
        _store(path, k, n_bases, res)
    return res
