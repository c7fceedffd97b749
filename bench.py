#!/usr/bin/env python3
"""Throughput of exact frequent-k-mer counting on one MI355X.

One step = one whole counting call (pack, Bloom screen, collect, radix sort,
run-length compaction) over one synthetic read library already resident in
HBM, through the C ABI entry point tk_count_device with a preallocated
workspace.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload large|small|long_k]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frequent k-mers/sec counted (exact) + % HBM peak; p50/p99 job latency served"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1305_1861_amd", "csrc")
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE; used
# only while the kernel sources still hash to the recorded digest
def traffic_file(workload: str) -> str:
    """Counter record of a workload: profiles/traffic_<workload>-library.json."""
    return os.path.join(ROOT, "profiles", f"traffic_{workload.replace('_', '-')}-library.json")
STAGE_SOURCES = {
    "bucket": ["bucket.hip", "device.hpp", "internal.hpp"],
    "partition": ["partition.hip", "scan.hip", "device.hpp", "internal.hpp"],
    "pack": ["pack.hip", "device.hpp", "internal.hpp"],
    "gather": ["bucket.hip", "device.hpp", "internal.hpp"],
}
# kernels of each stage of the partitioned path (name prefixes in rocprofv3
# records; the shared scan kernels are left out)
STAGE_KERNELS = {
    "pack": ["mark_read_starts", "pack_kernel"],
    "partition": ["pt_hist", "pt_scatter", "pt_segments", "pt_bucket_starts", "pt_tiles", "pt_transpose"],
    "bucket": ["plan_groups", "bucket_kernel"],
    "gather": ["gather_kernel"],
}
# stages made of one main kernel: the roofline's "dominant kernel" is the
# slowest of these (the partition is a sequence of radix passes)
SINGLE_KERNEL_STAGES = ("bucket", "gather", "screen", "collect", "pack")

WORKLOAD_INFO = {
    "phased": dict(library="the large library, streamed from host memory in chunks into a resident SAC"),
    "served": dict(jobs="Poisson arrivals, mean 50/s; batched-style libraries, k in {21, 31, 55}"),
    "batched": dict(libraries="log-uniform genomes 1e5..2e7 bp, coverage U[5, 60]"),
    "small": dict(genome_bp=1_000_000, coverage=10, read_len=100, sub_rate=0.01, n_rate=0.0, repeats=None),
    "large": dict(genome_bp=50_000_000, coverage=30, read_len=100, sub_rate=0.01, n_rate=0.0,
                  repeats="20% as 5 kbp copies, 2-10 per family, 2% divergence"),
    "long_k": dict(genome_bp=20_000_000, coverage=40, read_len=150, sub_rate=0.005, n_rate=0.001, repeats=None),
}


def algorithmic_bytes(n_bases: int, n_windows: int, n_collected: int, n_out: int, key_bytes: int,
                      passes: int, screen: bool, part_bits: int) -> dict:
    """Bytes each stage must move (the least traffic its structures need).

    Global-filter path (one 64-byte filter block per window per Bloom pass):
      pack    : 1 B/base read + 0.375 B/base written (2-bit codes + validity bit)
      screen  : 0.375 B/base read + 64 B read + 64 B written per window
      collect : 0.375 B/base read + 64 B read per window + key bytes per survivor
      sort    : 2 x key bytes per survivor per radix pass
      compact : key bytes per survivor + (key bytes + 4) per output record
    Partitioned path (filters, sort and compaction of a bucket live in LDS):
      pack      : as above
      partition : 0.375 B/base read + key bytes per window written, plus one
                  read and one write of every key for the second pass (D > 10;
                  its prefix tables, 2 B per digit and tile of 16384 keys,
                  are left out)
      bucket    : key bytes per window read + (key bytes + 4) per record written
      gather    : (key bytes + 4) per record read and written
    """
    pack = 1.375 * n_bases
    if part_bits < 0:
        scr = (0.375 * n_bases + 128.0 * n_windows) if screen else 0.0
        col = 0.375 * n_bases + (64.0 * n_windows if screen else 0.0) + key_bytes * n_collected
        srt = 2.0 * key_bytes * passes * n_collected
        cmp_ = key_bytes * n_collected + (key_bytes + 4) * n_out
        return dict(pack=pack, screen=scr, collect=col, sort=srt, compact=cmp_)
    part = 0.375 * n_bases + key_bytes * n_windows + (2.0 * key_bytes * n_windows if part_bits > 10 else 0.0)
    bucket = key_bytes * n_windows + (key_bytes + 4) * n_out
    gather = 2.0 * (key_bytes + 4) * n_out
    return dict(pack=pack, partition=part, bucket=bucket, gather=gather)


def sources_digest(stage: str) -> str:
    """sha256 over the HIP sources that define a stage's kernels."""
    import hashlib
    h = hashlib.sha256()
    for name in STAGE_SOURCES.get(stage, []):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(path: str, stage: str, workload: str):
    """HBM bytes per launch of `stage` from the counter record, or None when
    the record is missing, covers another workload or not this stage, or
    predates the stage's current kernel sources."""
    if not path or not os.path.exists(path):
        return None, "no counter record"
    with open(path) as f:
        tr = json.load(f)
    if tr.get("workload") != workload:
        return None, f"counter record covers {tr.get('workload')}"
    st = tr.get("stages", {}).get(stage)
    if st is None:
        return None, f"counter record has no {stage} stage"
    if st.get("sources_sha256") != sources_digest(stage):
        return None, "kernel sources changed since the counters were taken"
    return st.get("bytes"), tr.get("source", path)


WORKLOAD_NAMES = {"small": "uniform-1Mbp-10x-L100-k31", "large": "repeats-50Mbp-30x-L100-k31",
                  "long_k": "uniform-20Mbp-40x-L150-k63-N"}


def record_traffic(fetch_csv: str, write_csv: str, copy_bytes: int, workload: str, source: str, out: str) -> dict:
    """Per-stage HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE, in KiB per dispatch) of one bench step (--steps 1
    --warmup 0) that ends with plain device copies of copy_bytes each
    (--calibrate-copy-mib): each counter is scaled by what it reads for one
    of those copies."""
    import csv
    import re
    from collections import defaultdict

    def per_kernel(path):
        d = defaultdict(list)
        with open(path) as f:
            for r in csv.DictReader(f):
                name = re.sub(r"^void\s+", "", r["Kernel_Name"]).replace("tk::(anonymous namespace)::", "")
                d[name].append(float(r["Counter_Value"]))
        return d
    fe, wr = per_kernel(fetch_csv), per_kernel(write_csv)
    copies = [n for n in fe if "copyBuffer" in n]
    if not copies:
        raise SystemExit("no calibration copy in the counter records (run the step with --calibrate-copy-mib)")
    cf = max(max(fe[n]) for n in copies)
    cw = max(max(wr[n]) for n in copies)
    fs, ws_ = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    rec = {"workload": workload, "source": source, "copy_bytes": copy_bytes, "copy_fetch_size_kib": cf,
           "copy_write_size_kib": cw, "fetch_scale": fs, "write_scale": ws_, "stages": {}}
    for stage, prefixes in STAGE_KERNELS.items():
        names = sorted(n for n in fe if any(n.startswith(q) for q in prefixes))
        if not names:
            continue
        f_kib = sum(fe[n][0] for n in names)
        w_kib = sum(wr[n][0] for n in names if n in wr)
        rd, wt = f_kib * 1024.0 * fs, w_kib * 1024.0 * ws_
        rec["stages"][stage] = {"kernels": [n.split("(")[0] for n in names], "fetch_size_kib": round(f_kib, 3),
                                "write_size_kib": round(w_kib, 3), "read_bytes": int(rd), "written_bytes": int(wt),
                                "bytes": int(rd + wt), "sources_sha256": sources_digest(stage)}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


def cpu_baseline(lib, target_s: float = 12.0) -> dict:
    """The oracle, as it stands, on a bounded prefix of the same library."""
    import numpy as np
    import oracle
    n_reads = lib.n_reads
    read_len = int(lib.offsets[1] - lib.offsets[0]) if n_reads else 1
    # calibrate on a small prefix, then size the timed sample to ~target_s
    probe = min(n_reads, 20_000)
    t0 = time.perf_counter()
    oracle.kmer_count(lib.bases[:probe * read_len], lib.offsets[:probe + 1], lib.k, lib.c)
    dt = max(time.perf_counter() - t0, 1e-3)
    sample = int(min(n_reads, max(probe, probe * target_s / dt)))
    b = lib.bases[:int(lib.offsets[sample])]
    o = np.ascontiguousarray(lib.offsets[:sample + 1])
    t0 = time.perf_counter()
    res = oracle.kmer_count(b, o, lib.k, lib.c)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": res.n_windows / dt, "unit": "k-mer windows/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample} of {n_reads} reads ({res.n_windows} windows, {dt:.1f} s), "
                      f"single-threaded on 1 of {os.cpu_count()} host cores ({cpu})"}


def batched_digest_check(res_by_lib, gold, np):
    """Per-range digests of selected batched libraries' records against the
    oracle's (tests/golden/full_batched.json); returns (checked, mismatched)."""
    import hashlib
    checked, bad = 0, []
    for js, g in gold["libraries"].items():
        j = int(js)
        if j not in res_by_lib:
            continue
        keys, counts = res_by_lib[j]
        k, rb = g["k"], g["range_bits"]
        top = keys[:, 0] >> np.uint64(2 * k - rb) if rb else np.zeros(keys.shape[0], np.uint64)
        edges = np.searchsorted(top, np.arange((1 << rb) + 1, dtype=np.uint64))
        ok = True
        for r, want in enumerate(g["ranges"]):
            a, b = int(edges[r]), int(edges[r + 1])
            ok &= (b - a) == want["n_out"]
            ok &= hashlib.sha256(np.ascontiguousarray(keys[a:b], dtype="<u8").tobytes()).hexdigest() == \
                want["sha256_keys"]
            ok &= hashlib.sha256(np.ascontiguousarray(counts[a:b], dtype="<u4").tobytes()).hexdigest() == \
                want["sha256_counts"]
        checked += 1
        if not ok:
            bad.append(j)
    return checked, bad


def gen_progress(done: int, total: int):
    if done % 64 == 0 or done == total:
        print(f"[bench] drawn {done}/{total} libraries", file=sys.stderr, flush=True)


def bench_batched(args, tk, readsim, torch, np, dev) -> int:
    """The batched workload: 256 libraries of uneven size counted in waves
    (one tk_count_batch_device call per wave, every library with its own
    buckets, filters and result) against one tk_count_device call per
    library, on the same resident reads.  After timing, every library's
    batch result is compared with its single call and a spread of them
    (smallest, median and largest of every wave) with the oracle's digests."""
    t0 = time.perf_counter()
    n_libs, scale = args.batch_libs, args.batch_scale
    bases, offsets, lib_bases, lib_reads = readsim.batched_workload(n_libs, scale, workers=args.gen_workers,
                                                                    progress=gen_progress)
    waves = readsim.batched_waves(n_libs, scale, wave_bases=int(args.wave_bases))
    print(f"[bench] generated {n_libs} libraries, {bases.size} bases, {len(waves)} waves in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    k, c = 31, 2
    opts = tk.tk_default_options()
    opts.flags = tk.TK_FLAG_TIMING
    db_all = torch.from_numpy(bases).to(dev)
    wave_data = []
    for w in waves:
        b0, b1 = int(lib_bases[w[0]]), int(lib_bases[w[-1] + 1])
        r0, r1 = int(lib_reads[w[0]]), int(lib_reads[w[-1] + 1])
        lb = [int(lib_bases[j]) - b0 for j in w] + [b1 - b0]
        lr = [int(lib_reads[j]) - r0 for j in w] + [r1 - r0]
        do = torch.from_numpy((offsets[r0:r1 + 1] - np.uint64(b0)).view(np.int64)).to(dev)
        db = db_all[b0:b1]
        single = [(db[lb[q]:lb[q + 1]], do[lr[q]:lr[q + 1] + 1] - lb[q]) for q in range(len(w))]
        wave_data.append(dict(db=db, do=do, lb=lb, lr=lr, libs=w, single=single))
    del bases, offsets
    ws_bytes = max(tk.tk_batch_workspace_size(wd["lb"], wd["lr"], k, c, opts) for wd in wave_data)
    ws_bytes = max(ws_bytes, max(tk.tk_workspace_size(int(lib_bases[j + 1] - lib_bases[j]),
                                                      int(lib_reads[j + 1] - lib_reads[j]), k, c, opts)
                                 for j in range(n_libs)))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    print(f"[bench] resident: {db_all.numel() / 1e9:.1f} GB of reads, workspace {ws_bytes / 1e9:.1f} GB",
          file=sys.stderr, flush=True)

    def batched():
        n_win = n_out = 0
        for wd in wave_data:
            for r in tk.tk_count_batch_device(wd["db"], wd["do"], wd["lb"], wd["lr"], k, c, opts, workspace=ws,
                                              stream=stream):
                n_win += r.n_windows
                n_out += r.n
        return n_win, n_out

    def sequential():
        n_win = n_out = 0
        for wd in wave_data:
            for b, o in wd["single"]:
                r = tk.tk_count_device(b, o, k, c, opts, workspace=ws, stream=stream)
                n_win += r.n_windows
                n_out += r.n
        return n_win, n_out

    results = {}
    for name, fn in (("batched", batched), ("sequential", sequential)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            n_win, n_out = fn()
        torch.cuda.synchronize()
        results[name] = ((time.perf_counter() - t) / args.steps, n_win, n_out)
        print(f"[bench] {name}: {1e3 * results[name][0]:.2f} ms per pass", file=sys.stderr, flush=True)
    tb, n_win, n_out = results["batched"]
    ts = results["sequential"][0]
    # parity: every library's batch result against its single call, and the
    # digested spread against the oracle
    gold_path = os.path.join(ROOT, "tests", "golden", "full_batched.json")
    gold = None
    if scale == 1.0 and n_libs == 256 and os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)
    want = set(int(j) for j in gold["libraries"]) if gold else set()
    same, got = 0, {}
    for wd in wave_data:
        res = tk.tk_count_batch_device(wd["db"], wd["do"], wd["lb"], wd["lr"], k, c, opts, workspace=ws,
                                       stream=stream)
        kept = [(r.keys.clone(), r.counts.clone(), r) for r in res]
        for j, (b, o), (kk, cc, r) in zip(wd["libs"], wd["single"], kept):
            s1 = tk.tk_count_device(b, o, k, c, opts, workspace=ws, stream=stream)
            same += int(torch.equal(kk, s1.keys) and torch.equal(cc, s1.counts) and
                        (r.n_windows, r.n_collected, r.n_distinct, r.n_singletons) ==
                        (s1.n_windows, s1.n_collected, s1.n_distinct, s1.n_singletons))
            if j in want:
                got[j] = (kk.cpu().numpy().view(np.uint64), cc.cpu().numpy().view(np.uint32))
        del kept
    checked, bad = batched_digest_check(got, gold, np) if gold else (0, [])
    plain = getattr(args, "plain_windows_per_s", None)
    out = {
        "metric": METRIC, "value": n_win / tb, "unit": "k-mer windows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * tb, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"batched-{n_libs}-libraries" + ("" if scale == 1.0 else f"-scale-{scale:g}"),
                   "genome_bp": "log-uniform 1e5..2e7" + ("" if scale == 1.0 else f" times {scale:g}"),
                   "coverage": "U[5, 60]", "read_len": 100, "sub_rate": 0.01, "k": k, "c": c,
                   "n_bases": int(lib_bases[-1]), "waves": len(waves), "wave_bases": int(args.wave_bases)},
        "result": {"n_windows": n_win, "n_frequent": n_out,
                   "libraries_equal_to_single_call": f"{same}/{n_libs}",
                   "libraries_equal_to_oracle_digests": f"{checked - len(bad)}/{checked}" if gold else None,
                   "digest_mismatches": bad},
        "frequent_kmers_per_s": n_out / tb,
        "sequential": {"ms_per_step": 1e3 * ts, "value": n_win / ts, "calls": n_libs},
        "speedup_vs_sequential": ts / tb,
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0 if same == n_libs and not bad else 1


def bench_served(args, tk, readsim, torch, np, dev) -> int:
    """Jobs arriving as a Poisson process (mean args.rate per second), each a
    library drawn as in the batched workload (job j: seed 5000000 + j mod
    the pool) with k drawn from {21, 31, 55}, served by continuous batching
    with admission by HBM footprint; latency per job from arrival to result
    on the host, throughput against the plain path on the same device."""
    from paper_1305_1861_amd.serve import Job, Server
    pool_n = min(args.pool, args.jobs)
    t0 = time.perf_counter()
    bases, offsets, lib_bases, lib_reads = readsim.batched_workload(pool_n, args.batch_scale, base_seed=5_000_000,
                                                                    workers=args.gen_workers, progress=gen_progress)
    pool = []
    for q in range(pool_n):
        b0, b1, r0, r1 = int(lib_bases[q]), int(lib_bases[q + 1]), int(lib_reads[q]), int(lib_reads[q + 1])
        pool.append((bases[b0:b1], offsets[r0:r1 + 1] - np.uint64(b0)))
    print(f"[bench] generated {pool_n} job libraries ({bases.size} bases) in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    rng = np.random.Generator(np.random.PCG64(5))
    gaps = rng.exponential(1.0 / args.rate, args.jobs)
    ks = rng.choice([21, 31, 55], args.jobs)
    arrivals = np.cumsum(gaps)
    free, _ = torch.cuda.mem_get_info(dev)
    hbm = int(args.serve_hbm_frac * free)
    srv = Server(hbm_bytes=hbm, max_batch_libs=64, workers=2, device="cuda:0")
    try:
        # warm-up: one job of each k
        for k in (21, 31, 55):
            srv.submit(Job(pool[0][0], pool[0][1], int(k), 2)).result()
        futs = []
        start = time.perf_counter()
        for j in range(args.jobs):
            wait = start + arrivals[j] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            b, o = pool[j % pool_n]
            futs.append(srv.submit(Job(b, o, int(ks[j]), 2, t_submit=time.perf_counter())))
            if (j + 1) % 200 == 0:
                print(f"[bench] {j + 1} jobs submitted", file=sys.stderr, flush=True)
        res = [f.result() for f in futs]
        end = max(r.t_done for r in res)
    finally:
        srv.close()
    lat = np.array([r.latency_s for r in res]) * 1e3
    n_win = sum(r.n_windows for r in res)
    span = end - start
    batches = len({(r.t_start, r.t_done) for r in res})
    # the plain path on the same device: the largest pool library alone
    q = int(np.argmax(lib_bases[1:] - lib_bases[:-1]))
    b, o = pool[q]
    db = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    do = torch.from_numpy(o.view(np.int64)).to(dev)
    ws = torch.empty(tk.tk_workspace_size(int(b.size), int(o.size - 1), 31, 2), dtype=torch.uint8, device=dev)
    tk.tk_count_device(db, do, 31, 2, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        r = tk.tk_count_device(db, do, 31, 2, workspace=ws)
    torch.cuda.synchronize()
    plain = r.n_windows / ((time.perf_counter() - t) / 3)
    distinct = "" if pool_n >= args.jobs else f"-pool-{pool_n}"
    out = {
        "metric": METRIC, "value": n_win / span, "unit": "k-mer windows/s", "n_gpus": 1, "steps": args.jobs,
        "warmup": 3, "ms_per_step": 1e3 * span / args.jobs, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64/u128", "data": "synthetic",
        "config": {"workload": f"served-{args.jobs}-jobs-{args.rate:g}-per-s{distinct}"
                               + ("" if args.batch_scale == 1.0 else f"-scale-{args.batch_scale:g}"),
                   "jobs": args.jobs, "rate_per_s": args.rate, "k": "U{21, 31, 55}", "c": 2,
                   "distinct_libraries": pool_n, "job_library": "batched recipe, seed 5000000 + (j mod pool)",
                   "workers": 2, "hbm_bytes": hbm, "admission": "HBM footprint per batch"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "result": {"n_windows": n_win, "n_frequent": sum(int(r.counts.size) for r in res), "batches": batches,
                   "mean_jobs_per_batch": args.jobs / batches,
                   "offered_windows_per_s": n_win / arrivals[-1]},
        "plain_path_windows_per_s": plain,
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_phased(args, tk, readsim, torch, np, dev) -> int:
    """The large library in host memory, counted in chunks merged into a
    resident SAC (two passes over the host data), against its device
    footprint and the plain path's."""
    lib = readsim.WORKLOADS["large"]()
    chunk, cap = int(args.chunk_bases), int(args.sac_capacity)
    for _ in range(args.warmup):
        tk.tk_count_phased(lib.bases, lib.offsets, lib.k, lib.c, chunk, cap)
    t = time.perf_counter()
    for _ in range(args.steps):
        r = tk.tk_count_phased(lib.bases, lib.offsets, lib.k, lib.c, chunk, cap)
    dt = (time.perf_counter() - t) / args.steps
    plain = tk.tk_workspace_size(lib.n_bases, lib.n_reads, lib.k, lib.c)
    out = {
        "metric": METRIC, "value": r.n_windows / dt, "unit": "k-mer windows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"phased-{lib.name}", "chunk_bases": chunk, "sac_capacity": cap,
                   "input": "host memory (pageable), host-to-device copies timed"},
        "result": {"n_windows": r.n_windows, "n_frequent": r.n, "n_collected": r.n_collected,
                   "n_distinct_collected": r.n_distinct},
        "device_bytes": r.device_bytes, "plain_path_workspace_bytes": plain,
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_approx(args, tk, readsim, torch, np, dev) -> int:
    """An approximate variant (cTurtle or the single pass with "+1") on a
    resident workload: throughput, and false positives / negatives / count
    errors against the exact per-bucket path on the same input."""
    lib = readsim.WORKLOADS[args.workload]()
    bases = torch.from_numpy(lib.bases).to(dev)
    offsets = torch.from_numpy(lib.offsets.view(np.int64)).to(dev)
    flag = 4 if args.approx == "cturtle" else 8
    opts = tk.tk_default_options()
    opts.flags = tk.TK_FLAG_TIMING | flag
    opts.bloom_beta = args.approx_beta
    ws = torch.empty(tk.tk_workspace_size(lib.n_bases, lib.n_reads, lib.k, lib.c, opts), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        tk.tk_count_device(bases, offsets, lib.k, lib.c, opts, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        r = tk.tk_count_device(bases, offsets, lib.k, lib.c, opts, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    got_k = r.keys[:, -1].clone()
    got_c = r.counts.clone()
    ex = tk.tk_count_device(bases, offsets, lib.k, lib.c)
    ex_k, ex_c = ex.keys[:, -1], ex.counts
    if lib.k > 31:  # two-word keys: compare (hi, lo) pairs through their rank in the union
        raise SystemExit("approximate bench compares one-word keys")
    fn = int((~torch.isin(ex_k, got_k)).sum())
    fp = int((~torch.isin(got_k, ex_k)).sum())
    over = None
    if args.approx == "single_pass":
        idx = torch.searchsorted(ex_k, got_k).clamp(max=ex_k.numel() - 1)
        hit = ex_k[idx] == got_k
        over = int((got_c[hit] != ex_c[idx[hit]]).sum())
    n_ex = int(ex_k.numel())
    out = {
        "metric": METRIC, "value": r.n_windows / dt, "unit": "k-mer windows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{args.approx}-{lib.name}", "bits_per_window": args.approx_beta,
                   "filter_words": int(r.bloom_blocks) * 8},
        "result": {"n_windows": r.n_windows, "n_reported": int(got_k.numel()), "n_frequent_exact": n_ex,
                   "false_negative_rate": fn / n_ex, "false_positive_rate": fp / n_ex,
                   "count_one_over_rate": (over / n_ex) if over is not None else None},
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_shards(args, tk, readsim, torch, np, dev) -> int:
    """Key-range shards of one library on one device: each shard's call is
    the work one of G devices would do on its share (all windows extracted,
    only the shard's keys partitioned, screened, sorted and compacted).
    Reports every shard's device time; the step of G devices would take the
    slowest shard plus the broadcast of the packed reads, which one device
    cannot show."""
    G = args.shards
    lib = readsim.WORKLOADS[args.workload]()
    bases = torch.from_numpy(lib.bases).to(dev)
    offsets = torch.from_numpy(lib.offsets.view(np.int64)).to(dev)
    stream = torch.cuda.current_stream()
    full_o = tk.tk_default_options()
    full_o.flags = tk.TK_FLAG_TIMING
    opts = []
    for g in range(G):
        o = tk.tk_default_options()
        o.flags = tk.TK_FLAG_TIMING
        o.shard_count, o.shard_index = G, g
        opts.append(o)
    need = max(tk.tk_workspace_size(lib.n_bases, lib.n_reads, lib.k, lib.c, o) for o in opts + [full_o])
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    full = tk.tk_count_device(bases, offsets, lib.k, lib.c, full_o, workspace=ws, stream=stream)
    full_keys, full_counts = full.keys.clone(), full.counts.clone()
    full_ms = sum(full.stage_ms.values())
    # parity of the concatenation with the unsharded result
    got_k, got_c, wins = [], [], []
    for o in opts:
        r = tk.tk_count_device(bases, offsets, lib.k, lib.c, o, workspace=ws, stream=stream)
        got_k.append(r.keys.clone())
        got_c.append(r.counts.clone())
        wins.append(r.n_windows)
    same = bool(torch.equal(torch.cat(got_k), full_keys) and torch.equal(torch.cat(got_c), full_counts))
    del got_k, got_c
    for _ in range(args.warmup):
        for o in opts:
            tk.tk_count_device(bases, offsets, lib.k, lib.c, o, workspace=ws, stream=stream)
    ms = np.zeros((args.steps, G))
    stages = {s: np.zeros(G) for s in tk.STAGES}
    for i in range(args.steps):
        for g, o in enumerate(opts):
            r = tk.tk_count_device(bases, offsets, lib.k, lib.c, o, workspace=ws, stream=stream)
            ms[i, g] = sum(r.stage_ms.values())
            for s in tk.STAGES:
                stages[s][g] += r.stage_ms[s] / args.steps
    torch.cuda.synchronize()
    per = ms.mean(axis=0)
    total = float(per.sum())
    out = {
        "metric": METRIC, "value": full.n_windows / (total * 1e-3), "unit": "k-mer windows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": total,
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "u64" if lib.k <= 31 else "u128",
        "data": "synthetic",
        "config": {"workload": f"{lib.name}-shard-of-{G}", "shards": G, "k": lib.k, "c": lib.c},
        "note": "one device runs the G shards one after the other; value: the library's windows over "
                "their summed device time.  slowest_shard_ms is what each of G devices would spend on its "
                "share, before the broadcast of the packed reads",
        "result": {"concatenation_equals_unsharded": same, "unsharded_ms": full_ms,
                   "slowest_shard_ms": round(float(per.max()), 3),
                   "shard_ms": [round(float(x), 3) for x in per],
                   "shard_windows": wins,
                   "shard_stage_ms_mean": {s: round(float(v.mean()), 3) for s, v in stages.items() if v.any()}},
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    return 0 if same else 1


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOAD_INFO))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--global-filter", action="store_true",
                    help="one Bloom filter in HBM for the whole library (device-scope atomics)")
    ap.add_argument("--part-bits", type=int, default=-1,
                    help="bucket bits D of the per-bucket plan (-1: the library's size rule)")
    ap.add_argument("--traffic", default=None,
                    help="JSON record of measured HBM bytes per launch of the dominant kernel")
    ap.add_argument("--batch-libs", type=int, default=256, help="batched workload: number of libraries")
    ap.add_argument("--batch-scale", type=float, default=1.0,
                    help="batched workload: factor on every library's genome size (1: the stated config)")
    ap.add_argument("--wave-bases", type=float, default=2.0e9,
                    help="batched workload: bases per batch call (waves sized to HBM)")
    ap.add_argument("--gen-workers", type=int, default=16,
                    help="batched workload: processes drawing the libraries")
    ap.add_argument("--jobs", type=int, default=1000, help="served workload: number of jobs")
    ap.add_argument("--rate", type=float, default=50.0, help="served workload: mean arrivals per second")
    ap.add_argument("--pool", type=int, default=1000,
                    help="served workload: distinct job libraries (jobs cycle over them when fewer than --jobs)")
    ap.add_argument("--serve-hbm-frac", type=float, default=0.6,
                    help="served workload: fraction of free device memory the server holds")
    ap.add_argument("--chunk-bases", type=float, default=1.0e8, help="phased workload: bases per chunk")
    ap.add_argument("--sac-capacity", type=float, default=6.0e7,
                    help="phased workload: records of the resident sorted-and-compacted array")
    ap.add_argument("--approx", choices=["cturtle", "single_pass"], default=None,
                    help="time an approximate variant on the workload and report its errors against the exact path")
    ap.add_argument("--approx-beta", type=int, default=16, help="approximate variants: filter bits per window")
    ap.add_argument("--shards", type=int, default=1,
                    help="time every key-range shard of the workload in turn (the share of one of this many "
                         "devices) and check that their results concatenate to the unsharded one")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="write the per-stage HBM byte record (--traffic) from two rocprofv3 --pmc counter "
                         "files of one step of --workload run with --calibrate-copy-mib, then exit")
    ap.add_argument("--autotune", action="store_true",
                    help="time bucket bits, filter bits per window, pattern bits and the bucket kernel's tile "
                         "shape; print the fastest (stored in $TK_TUNE_CACHE when set)")
    ap.add_argument("--no-end-to-end", action="store_true",
                    help="skip the end-to-end run from host buffers (reported beside the timed value)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times with a plain "
                         "device copy kernel (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.traffic is None:
        args.traffic = traffic_file(args.workload)

    if args.record_traffic:
        rec = record_traffic(args.record_traffic[0], args.record_traffic[1], args.calibrate_copy_mib << 20,
                             WORKLOAD_NAMES[args.workload], f"profiles/kernels_{args.workload.replace('_', '-')}-library_per-bucket.md",
                             args.traffic)
        print(json.dumps({s: v["bytes"] for s, v in rec["stages"].items()}))
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "the library counts on one device (tk_options.shard_count/shard_index give one device's share "
              "of a key-range split).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1305_1861_amd as tk
    import readsim

    tk.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batched":
        return bench_batched(args, tk, readsim, torch, np, dev)
    if args.workload == "served":
        return bench_served(args, tk, readsim, torch, np, dev)
    if args.workload == "phased":
        return bench_phased(args, tk, readsim, torch, np, dev)
    if args.approx:
        return bench_approx(args, tk, readsim, torch, np, dev)
    if args.shards > 1:
        return bench_shards(args, tk, readsim, torch, np, dev)
    if args.autotune:
        from paper_1305_1861_amd.tune import autotune
        lib = readsim.WORKLOADS[args.workload]()
        bases = torch.from_numpy(lib.bases).to(dev)
        offsets = torch.from_numpy(lib.offsets.view(np.int64)).to(dev)
        t = autotune(bases, offsets, lib.k, lib.c, repeats=max(1, args.steps))
        print(json.dumps({"workload": lib.name, "cached": t.cached,
                          "best": {"part_bits": t.part_bits, "bloom_beta": t.bloom_beta, "bloom_bits": t.bloom_bits,
                                   "bucket_tile": t.bucket_tile, "ms": t.ms},
                          "timings": [{"part_bits": d, "bloom_beta": be, "bloom_bits": bi, "bucket_tile": ti,
                                       "ms": ms, "n_fallback": nf} for d, be, bi, ti, ms, nf in t.timings],
                          "host": platform.node()}), flush=True)
        return 0

    t0 = time.perf_counter()
    lib = readsim.WORKLOADS[args.workload]()
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated {lib.name}: {lib.n_bases} bases, {lib.n_reads} reads in {gen_s:.1f} s",
          file=sys.stderr, flush=True)
    bases = torch.from_numpy(lib.bases).to(dev)
    offsets = torch.from_numpy(lib.offsets.view(np.int64)).to(dev)
    opts = tk.tk_default_options()
    opts.flags = tk.TK_FLAG_TIMING | (tk.TK_FLAG_GLOBAL_FILTER if args.global_filter else 0)
    opts.part_bits = args.part_bits
    need = tk.tk_workspace_size(lib.n_bases, lib.n_reads, lib.k, lib.c, opts)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        tk.tk_count_device(bases, offsets, lib.k, lib.c, opts, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    stage_sum = {s: 0.0 for s in tk.STAGES}
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        r = tk.tk_count_device(bases, offsets, lib.k, lib.c, opts, workspace=ws, stream=stream)
        lat.append(time.perf_counter() - ts)
        for s in tk.STAGES:
            stage_sum[s] += r.stage_ms[s]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    stage_ms = {s: stage_sum[s] / args.steps for s in tk.STAGES}

    key_bytes = 8 * r.key_words
    model = algorithmic_bytes(lib.n_bases, r.n_windows, r.n_collected, r.n, key_bytes, r.sort_passes,
                              lib.c >= 2, r.part_bits)
    single = [s for s in model if s in SINGLE_KERNEL_STAGES] or list(model)
    dominant = max(single, key=lambda s: stage_ms.get(s, 0.0))
    achieved = model[dominant] / (stage_ms[dominant] * 1e-3) / 1e9
    traffic, traffic_src = measured_traffic(args.traffic, dominant, lib.name)
    stages = {}
    for st, b in model.items():
        ms = stage_ms.get(st, 0.0)
        ach = b / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        tr_b, _ = measured_traffic(args.traffic, st, lib.name)
        stages[st] = {"ms": ms, "algorithmic_bytes": int(b), "achieved": ach, "frac": ach / HBM_PEAK_GBS,
                      "traffic": tr_b}
    path_bytes = sum(model.values())
    step_s = ms_per_step * 1e-3
    out = {
        "metric": METRIC,
        "value": r.n_windows / step_s,
        "unit": "k-mer windows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64" if r.key_words == 1 else "u128",
        "data": "synthetic",
        "config": {
            "workload": lib.name,
            **WORKLOAD_INFO[args.workload],
            "n_reads": lib.n_reads, "n_bases": lib.n_bases, "k": lib.k, "c": lib.c,
            "filter": "global" if args.global_filter else "per-bucket",
            "bloom_blocks": r.bloom_blocks, "part_bits": r.part_bits,
        },
        "result": {
            "n_windows": r.n_windows, "n_frequent": r.n, "n_collected": r.n_collected,
            "n_distinct_collected": r.n_distinct, "n_false_pos": r.n_singletons,
            "false_pos_rate_of_distinct": (r.n_singletons / r.n_distinct) if r.n_distinct else 0.0,
            "sort_passes": r.sort_passes, "n_fallback_buckets": r.n_fallback,
        },
        "frequent_kmers_per_s": r.n / step_s,
        "hbm_frac_path": path_bytes / step_s / (HBM_PEAK_GBS * 1e9),
        "model_bytes": {k: int(v) for k, v in model.items()},
        "stage_ms": {k: v for k, v in stage_ms.items() if k in model},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99))},
        "roofline": {
            "bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": traffic_src,
            "algorithmic_bytes": int(model[dominant]), "launch_ms": stage_ms[dominant],
        },
        "stages": stages,
    }
    if not args.no_end_to_end:
        # host buffers in, host result out (tk_count: device allocation, both
        # PCIe copies and the same kernels); reported beside, never as value
        del ws, r
        torch.cuda.empty_cache()
        tk.tk_count(lib.bases, lib.offsets, lib.k, lib.c)
        t = time.perf_counter()
        e2e = tk.tk_count(lib.bases, lib.offsets, lib.k, lib.c)
        e2e_s = time.perf_counter() - t
        out["end_to_end"] = {"ms": 1e3 * e2e_s, "windows_per_s": e2e.n_windows / e2e_s,
                             "what": "tk_count on pageable host buffers: workspace allocation, copy of the "
                                     "reads to the device, the timed path, copy of the records back"}
    if args.calibrate_copy_mib:
        src = torch.ones(args.calibrate_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = int(src.numel())
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(lib)
    out["host"] = platform.node()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
