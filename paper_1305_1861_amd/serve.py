"""Continuous batching of counting jobs on one GPU.

A job is one read library (host ``bases``/``offsets`` arrays) with its k and
threshold c.  Every job's device footprint is computed from the library's own
sizing rules -- the workspace ``tk_batch_workspace_size`` gives for it plus
its input bytes -- and a job is admitted only while the footprint of its
batch fits the device memory a worker holds.  The server reserves that
memory once, at start: ``hbm_bytes`` (by default 60 % of the device memory
free at start) split evenly over the workers, each share one resident device
arena that holds a batch's workspace (filters, key and sort buffers), its
reads and its offsets, reused from batch to batch, so admitting a job never
allocates device memory.

Jobs wait in arrival order; when a worker is free, the dispatcher hands it
the oldest waiting job plus every later waiting job that still fits the
worker's arena (at most ``max_batch_libs`` jobs), whatever their k: one
``tk_count_batch_device`` call counts the batch, every library with its own
k, buckets, filters, threshold and result.  Each worker owns a HIP stream, so
one batch's copies overlap the other's kernels.  Jobs reach the device
through a pinned host buffer per worker (one host copy per job into its
slice, then one transfer per batch, offsets rebased on the host), and
results come back through pinned buffers into ordinary host arrays: copies
from pageable memory ran at about 4 GB/s.

Options: the ``opts`` given to the server, else, per batch, the
autotuner's cached choice for the batch's largest job when ``$TK_TUNE_CACHE``
names a cache file (``tune.py``), else the defaults.  Results are host
arrays, identical to what a single ``tk_count_device`` call on the job alone
(with the same options) returns.
"""
from __future__ import annotations

import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass

import numpy as np

from . import _torch, load_library, tk_batch_workspace_size, tk_count_batch_device

_ALIGN = 256


def _align(x: int) -> int:
    return (x + _ALIGN - 1) // _ALIGN * _ALIGN


@dataclass
class Job:
    bases: np.ndarray    # uint8
    offsets: np.ndarray  # uint64, n_reads + 1
    k: int
    c: int = 2
    t_submit: float = 0.0


@dataclass
class JobResult:
    keys: np.ndarray     # uint64 [n, key_words]
    counts: np.ndarray   # uint32 [n]
    n_windows: int
    n_collected: int
    n_distinct: int
    n_singletons: int
    t_submit: float
    t_start: float
    t_done: float
    batch_jobs: int = 1  # jobs counted in the same call

    @property
    def latency_s(self) -> float:
        return self.t_done - self.t_submit


class Server:
    """Counting server: ``submit(job)`` returns a Future of a JobResult.

    ``hbm_bytes``: device memory the server holds (default: 60 % of what is
    free at start), split evenly over ``workers``; a job whose footprint
    exceeds one worker's share is refused at submission.
    ``max_batch_libs``: jobs per batch.  ``linger_s``: how long the
    dispatcher waits for more arrivals before handing out a batch.
    """

    def __init__(self, hbm_bytes: int | None = None, workers: int = 2, max_batch_libs: int = 64, opts=None,
                 device: str = "cuda:0", linger_s: float = 0.0):
        torch = _torch()
        load_library()
        self.torch = torch
        self.device = torch.device(device)
        if hbm_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_bytes = int(0.6 * free)
        self.share = (int(hbm_bytes) // workers) // _ALIGN * _ALIGN
        if self.share < (1 << 20):
            raise ValueError("the server needs at least 1 MiB of device memory per worker")
        self.max_libs = int(max_batch_libs)
        # None: per batch, the autotuner's cached choice ($TK_TUNE_CACHE)
        # for its largest job, else the defaults (tk_count_batch_device)
        self.opts = opts
        self.linger_s = linger_s
        self._pending: list[tuple[Job, Future, int]] = []  # job, future, its own footprint
        self._cv = threading.Condition()
        self._idle: queue.Queue = queue.Queue()
        self._stop = False
        self._workers = []
        for i in range(workers):
            w = dict(
                stream=torch.cuda.Stream(device=self.device),
                arena=torch.empty(self.share, dtype=torch.uint8, device=self.device),
                h_bases=None, h_offsets=None, h_keys=None, h_counts=None,
                inbox=queue.Queue(),
            )
            t = threading.Thread(target=self._work, args=(w,), daemon=True, name=f"tk-worker-{i}")
            w["thread"] = t
            self._workers.append(w)
            t.start()
            self._idle.put(w)
        self._dispatcher = threading.Thread(target=self._dispatch, daemon=True, name="tk-dispatch")
        self._dispatcher.start()

    # -- footprints ------------------------------------------------------------
    def footprint(self, jobs) -> int:
        """Device bytes of one batch of these jobs: the library's workspace
        for them, then their reads and offsets, in one arena."""
        lb, lr = [0], [0]
        for j in jobs:
            lb.append(lb[-1] + int(j.bases.size))
            lr.append(lr[-1] + int(j.offsets.size - 1))
        ws = tk_batch_workspace_size(lb, lr, [int(j.k) for j in jobs], [int(j.c) for j in jobs], self.opts)
        return _align(ws) + _align(lb[-1]) + 8 * (lr[-1] + 1)

    # -- client side ---------------------------------------------------------
    @staticmethod
    def check_job(job: Job):
        """Refuse a malformed job before it can share a batch: its offsets
        are rebased into the batch's arrays, so an offset past its own bases
        would cut windows of the next job, and a bad k or c would fail the
        whole batch."""
        b, o = job.bases, job.offsets
        if not isinstance(b, np.ndarray) or b.dtype != np.uint8 or b.ndim != 1:
            raise ValueError("job.bases must be a 1-D uint8 array")
        if not isinstance(o, np.ndarray) or o.dtype not in (np.uint64, np.int64) or o.ndim != 1 or o.size < 1:
            raise ValueError("job.offsets must be a 1-D array of n_reads + 1 uint64 values")
        if int(o[0]) != 0 or int(o[-1]) != b.size:
            raise ValueError("job.offsets must start at 0 and end at bases.size")
        if o.size > 1 and (np.diff(o.astype(np.int64)) < 0).any():
            raise ValueError("job.offsets must not decrease")
        if not (isinstance(job.k, (int, np.integer)) and 1 <= int(job.k) <= 63):
            raise ValueError("job.k must be in [1, 63]")
        if not (isinstance(job.c, (int, np.integer)) and int(job.c) >= 1):
            raise ValueError("job.c must be >= 1")

    def submit(self, job: Job) -> Future:
        self.check_job(job)
        fp = self.footprint([job])
        if fp > self.share:
            raise ValueError(f"job needs {fp} bytes of device memory; a worker holds {self.share}")
        fut: Future = Future()
        job.t_submit = job.t_submit or time.perf_counter()
        with self._cv:
            self._pending.append((job, fut, fp))
            self._cv.notify()
        return fut

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        self._dispatcher.join()
        for w in self._workers:
            w["inbox"].put(None)
            w["thread"].join()

    # -- scheduling ------------------------------------------------------------
    _SCAN = 256  # waiting jobs looked at per batch

    def _take_batch(self):
        """The oldest waiting job plus later ones while the batch's footprint
        fits a worker's arena; jobs of every k share a batch."""
        take, rest = [self._pending[0]], []
        for i, item in enumerate(self._pending[1:], 1):
            if len(take) >= self.max_libs or i >= self._SCAN or \
                    sum(t[2] for t in take) + item[2] > 2 * self.share:
                rest.append(item)
                continue
            if self.footprint([t[0] for t in take] + [item[0]]) <= self.share:
                take.append(item)
            else:
                rest.append(item)
        self._pending = rest
        return [(j, f) for j, f, _ in take]

    def _dispatch(self):
        while True:
            w = self._idle.get()  # a free worker first, then the jobs
            with self._cv:
                while not self._pending and not self._stop:
                    self._cv.wait()
                if not self._pending and self._stop:
                    self._idle.put(w)
                    return
                if self.linger_s:
                    self._cv.wait(self.linger_s)
                batch = self._take_batch()
            w["inbox"].put(batch)

    def _work(self, w):
        while True:
            batch = w["inbox"].get()
            if batch is None:
                return
            t_start = time.perf_counter()
            try:
                self._run(w, batch, t_start)
            except Exception as e:  # every job of the batch learns the failure
                for _, fut in batch:
                    if not fut.done():
                        fut.set_exception(e)
            self._idle.put(w)

    def _pinned(self, w, name, n, dtype):
        """Worker w's pinned host buffer `name` of at least n elements
        (grown by half again when too small)."""
        buf = w[name]
        if buf is None or buf.numel() < n:
            w[name] = None
            buf = self.torch.empty(max(n + n // 2, 1 << 16), dtype=dtype, pin_memory=True)
            w[name] = buf
        return buf

    def _run(self, w, batch, t_start):
        torch = self.torch
        jobs = [j for j, _ in batch]
        lb, lr = [0], [0]
        for j in jobs:
            lb.append(lb[-1] + int(j.bases.size))
            lr.append(lr[-1] + int(j.offsets.size - 1))
        ks, cs = [int(j.k) for j in jobs], [int(j.c) for j in jobs]
        ws_bytes = _align(tk_batch_workspace_size(lb, lr, ks, cs, self.opts))
        b_off = ws_bytes
        o_off = b_off + _align(lb[-1])
        assert o_off + 8 * (lr[-1] + 1) <= self.share, "admission let in a batch larger than the arena"
        arena = w["arena"]
        stream = w["stream"]
        # every job into its slice of the pinned input buffers, its offsets
        # rebased to its first base (the previous batch's transfer from these
        # buffers ended with that batch's stream synchronisation); torch runs
        # the host copies on its thread pool without holding the interpreter
        # lock, so both workers' copies and the dispatcher proceed together
        hb = self._pinned(w, "h_bases", max(lb[-1], 1), torch.uint8)
        ho = self._pinned(w, "h_offsets", lr[-1] + 1, torch.int64)
        ho[:1].zero_()
        for q, j in enumerate(jobs):
            if j.bases.size:
                hb[lb[q]:lb[q + 1]].copy_(torch.from_numpy(j.bases))
            if lr[q + 1] > lr[q]:
                off = torch.from_numpy(j.offsets[1:].astype(np.uint64, copy=False).view(np.int64))
                torch.add(off, lb[q], out=ho[lr[q] + 1:lr[q + 1] + 1])
        with torch.cuda.stream(stream):
            db = arena[b_off:b_off + lb[-1]]
            do = arena[o_off:o_off + 8 * (lr[-1] + 1)].view(torch.int64)
            db.copy_(hb[:lb[-1]], non_blocking=True)
            do.copy_(ho[:lr[-1] + 1], non_blocking=True)
            res = tk_count_batch_device(db, do, lb, lr, ks, cs, self.opts, workspace=arena[:ws_bytes],
                                        stream=stream)
            hk = self._pinned(w, "h_keys", sum(int(r.keys.numel()) for r in res), torch.int64)
            hc = self._pinned(w, "h_counts", sum(int(r.counts.numel()) for r in res), torch.int32)
            back, ok, oc = [], 0, 0
            for r in res:
                nk, nc = int(r.keys.numel()), int(r.counts.numel())
                pk, pc = hk[ok:ok + nk].view(r.keys.shape), hc[oc:oc + nc]
                pk.copy_(r.keys, non_blocking=True)
                pc.copy_(r.counts, non_blocking=True)
                back.append((pk, pc, r))
                ok += nk
                oc += nc
            stream.synchronize()
            # own copies: the pinned buffer serves the worker's next batch
            host = [(pk.clone().numpy().view(np.uint64).reshape(r.n, r.key_words), pc.clone().numpy().view(np.uint32),
                     r) for pk, pc, r in back]
        t_done = time.perf_counter()
        for (keys, counts, r), (job, fut) in zip(host, batch):
            fut.set_result(JobResult(keys, counts, r.n_windows, r.n_collected, r.n_distinct, r.n_singletons,
                                     job.t_submit, t_start, t_done, len(jobs)))
