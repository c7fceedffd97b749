"""Continuous batching: every job's result from the server (mixed with other
jobs of several k and thresholds, in batches formed by arrival) is
bit-identical to a single-library call on the job alone, and one of them to
the oracle."""
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


def jobs_mix():
    from paper_1305_1861_amd.serve import Job
    jobs = []
    for j in range(14):
        k = (21, 31, 55)[j % 3]
        c = 3 if j % 4 == 3 else 2
        if j % 5 == 0:
            lib = readsim.small_library(scale=0.02, seed=700 + j)
            b, o = lib.bases, lib.offsets
        else:
            b, o = readsim.random_reads(800 + j, 150 + 40 * j, 0, 200, n_rate=0.01)
            dup = readsim.to_strings(b, o)
            b, o = readsim.from_strings(dup + dup[: len(dup) // 2])
        jobs.append(Job(b, o, k, c))
    return jobs


def alone(tk, job):
    import torch
    db = torch.from_numpy(job.bases).cuda() if job.bases.size else torch.zeros(1, dtype=torch.uint8).cuda()[:0]
    do = torch.from_numpy(job.offsets.astype(np.uint64).view(np.int64)).cuda()
    r = tk.tk_count_device(db, do, job.k, job.c)
    torch.cuda.synchronize()
    return (r.keys.cpu().numpy().view(np.uint64).reshape(r.n, r.key_words), r.counts.cpu().numpy().view(np.uint32),
            r)


def test_served_results_identical_to_single_calls(tk, oracle_lib):
    from paper_1305_1861_amd.serve import Server
    jobs = jobs_mix()
    case(f"served mix of {len(jobs)} jobs")
    srv = Server(max_batch_bases=1 << 22, max_batch_reads=1 << 16, max_batch_libs=6, workers=2)
    try:
        futs = [srv.submit(j) for j in jobs]
        results = [f.result(timeout=120) for f in futs]
    finally:
        srv.close()
    for q, (job, res) in enumerate(zip(jobs, results)):
        keys, counts, r = alone(tk, job)
        assert np.array_equal(res.keys, keys), q
        assert np.array_equal(res.counts, counts), q
        assert (res.n_windows, res.n_collected, res.n_distinct, res.n_singletons) == \
            (r.n_windows, r.n_collected, r.n_distinct, r.n_singletons), q
        assert res.t_submit <= res.t_start <= res.t_done
    job, res = jobs[1], results[1]
    ora = oracle_lib.kmer_count(job.bases, job.offsets, job.k, job.c)
    assert np.array_equal(res.keys[:, 0], ora.lo) and np.array_equal(res.counts.astype(np.uint64), ora.count)


def test_server_refuses_oversized_job(tk):
    from paper_1305_1861_amd.serve import Job, Server
    srv = Server(max_batch_bases=1 << 12, max_batch_reads=64, max_batch_libs=2, workers=1)
    try:
        b, o = readsim.random_reads(1, 100, 50, 60)
        with pytest.raises(ValueError):
            srv.submit(Job(b, o, 31))
    finally:
        srv.close()
