"""Write the exact answers of the full-size workloads as digests.

    python tests/golden/make_full_digests.py [--workers 4] [--only large,long_k,batched]

Calls only the CPU oracle (``oracle/``) and the input generators
(``readsim/``).  For each full-size library -- the plain large library
(50 Mbp with repeats, 30x, 100 bp, k = 31, c = 2) and the long-k library
(20 Mbp, 40x, 150 bp, 0.5 % substitutions, 0.1 % N, k = 63, c = 2) -- the
key space is cut into 2^RANGE_BITS ranges by the keys' top bits, so that no
step holds more than one range's keys.  Per range it records the windows,
the distinct keys, the records with count >= c, the sum of their counts and
SHA-256 digests of the records in the library's output layout (keys as
little-endian uint64 words, {hi, lo} per record for two-word keys; counts as
little-endian uint32), plus the per-bucket Bloom model's statistics for the
bucket bits D the counting library's size rule gives (every range holds
whole buckets since D >= RANGE_BITS).  The result goes to
``tests/golden/full_<workload>.json``.

The batched workload (256 libraries, genomes log-uniform in 0.1-20 Mbp,
coverage U[5, 60], counted in waves of at most 2e9 bases) is digested for a
spread of its libraries: the smallest, the median and the largest of every
wave, each on its own (libraries above 2e8 bases in 8 key ranges).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import readsim  # noqa: E402

RANGE_BITS = 4
WORKLOADS = ("large", "long_k", "batched")
# the batched workload: 256 libraries in waves of at most 2e9 bases; per
# wave the smallest, the median and the largest library are digested
BATCH_LIBS = 256
BATCH_WAVE_BASES = 2_000_000_000
BATCH_SPLIT_BASES = 200_000_000  # libraries above this are digested in 8 key ranges
_LIBS: dict = {}


def batched_selection():
    """Indices of the digested batched libraries: per wave, the smallest,
    the median and the largest."""
    sel = set()
    for wave in readsim.batched_waves(BATCH_LIBS, 1.0, 4000, BATCH_WAVE_BASES):
        by_size = sorted(wave, key=lambda j: (readsim.batched_library_size(j)[0], j))
        sel.update((by_size[0], by_size[len(by_size) // 2], by_size[-1]))
    return sorted(sel)


def _range_task(args):
    name, rbits, ri = args
    lib = _LIBS[name]
    k, c = lib.k, lib.c
    D = oracle.partition_bits(lib.n_bases, lib.n_reads, k)
    assert D >= rbits
    t0 = time.time()
    hi, lo = oracle.keys_in_range(lib.bases, lib.offsets, k, rbits, ri)
    n_win = int(hi.size)
    bloom = oracle.bloom_model_buckets_keys(hi, lo, k, D, oracle.BLOOM_BETA)
    uh, ul, uc = oracle.sort_compact(hi, lo)
    del hi, lo
    keep = uc >= c
    kh, kl, kc = uh[keep], ul[keep], uc[keep]
    if k <= 31:
        key_bytes = np.ascontiguousarray(kl, dtype="<u8").tobytes()
    else:
        key_bytes = np.ascontiguousarray(np.stack([kh, kl], axis=1), dtype="<u8").tobytes()
    out = dict(index=ri, n_windows=n_win, n_distinct=int(uh.size), n_out=int(kc.size),
               sum_counts=int(kc.sum()), n_singletons=int((uc == 1).sum()),
               sha256_keys=hashlib.sha256(key_bytes).hexdigest(),
               sha256_counts=hashlib.sha256(np.ascontiguousarray(kc, dtype="<u4").tobytes()).hexdigest(),
               bloom_n_collected=bloom.n_cand_occ, bloom_n_distinct=bloom.n_cand,
               bloom_n_singletons=bloom.n_cand_single)
    print(f"{name} range {ri}/{1 << rbits}: {n_win} windows, {out['n_out']} records ({time.time() - t0:.0f} s)",
          flush=True)
    return name, out


def _summary(lib, name, rbits, rs, scale):
    rs = sorted(rs, key=lambda r: r["index"])
    return dict(
        workload=lib.name, generator=name, scale=scale, k=lib.k, c=lib.c, n_bases=lib.n_bases,
        n_reads=lib.n_reads, range_bits=rbits,
        part_bits=oracle.partition_bits(lib.n_bases, lib.n_reads, lib.k), bloom_beta=oracle.BLOOM_BETA,
        n_windows=sum(r["n_windows"] for r in rs), n_distinct=sum(r["n_distinct"] for r in rs),
        n_out=sum(r["n_out"] for r in rs), sum_counts=sum(r["sum_counts"] for r in rs),
        bloom_n_collected=sum(r["bloom_n_collected"] for r in rs),
        bloom_n_distinct=sum(r["bloom_n_distinct"] for r in rs),
        bloom_n_singletons=sum(r["bloom_n_singletons"] for r in rs),
        ranges=rs)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--only", default=",".join(WORKLOADS))
    ap.add_argument("--scale", type=float, default=1.0, help="library scale (1.0 for the stored digests)")
    ap.add_argument("--out-dir", default=HERE)
    args = ap.parse_args()
    names = [n for n in args.only.split(",") if n]
    oracle.build(force=False)
    tasks = []
    batched = []
    for n in names:
        t0 = time.time()
        if n == "batched":
            batched = batched_selection()
            for j in batched:
                _LIBS[f"batched/{j}"] = readsim.batched_library(j, args.scale)
            print(f"generated {len(batched)} batched libraries ({time.time() - t0:.0f} s)", flush=True)
            continue
        _LIBS[n] = readsim.WORKLOADS[n](scale=args.scale)
        print(f"generated {n}: {_LIBS[n].n_bases} bases ({time.time() - t0:.0f} s)", flush=True)
    # largest ranges first: canonical keys are denser at the low end
    for ri in range(1 << RANGE_BITS):
        tasks += [(n, RANGE_BITS, ri) for n in names if n != "batched"]
    for j in sorted(batched, key=lambda j: -_LIBS[f"batched/{j}"].n_bases):
        rb = 3 if _LIBS[f"batched/{j}"].n_bases > BATCH_SPLIT_BASES else 0
        tasks += [(f"batched/{j}", rb, ri) for ri in range(1 << rb)]
    with mp.get_context("fork").Pool(args.workers) as pool:
        results = pool.map(_range_task, tasks, chunksize=1)
    bits = {t[0]: t[1] for t in tasks}
    for n in names:
        if n == "batched":
            doc = dict(workload="batched-256-libraries", scale=args.scale, n_libs=BATCH_LIBS,
                       wave_bases=BATCH_WAVE_BASES, base_seed=4000,
                       libraries={str(j): _summary(_LIBS[f"batched/{j}"], f"batched/{j}", bits[f"batched/{j}"],
                                                   [r for m, r in results if m == f"batched/{j}"], args.scale)
                                  for j in batched})
        else:
            doc = _summary(_LIBS[n], n, RANGE_BITS, [r for m, r in results if m == n], args.scale)
        path = os.path.join(args.out_dir, f"full_{n}.json")
        with open(path, "w") as f:
            json.dump(doc, f, indent=1)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
