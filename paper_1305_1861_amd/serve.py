"""Continuous batching of counting jobs on one GPU.

A job is one read library (host ``bases``/``offsets`` arrays) with its k and
threshold c.  Jobs wait in arrival order; a dispatcher takes the oldest job
and every other waiting job of the same k, up to a budget of bases, and hands
them to a free worker as one batch (``tk_count_batch_device``: every library
keeps its own buckets, filters, threshold and result).  Each worker owns a
HIP stream and keeps its device buffers -- input bases and offsets and the
counting workspace -- for the whole life of the server, sized once for the
budget, so admitting a job never allocates device memory.  Two workers let
one batch's host-to-device copy and result copy overlap the other's kernels.
Jobs reach the device through pinned host buffers of the same size (one
host copy per job into its slice, then one transfer per batch, offsets
rebased on the host), and results come back through a pinned buffer per
worker (grown to the largest batch's records) into ordinary host arrays:
copies from pageable memory ran at about 4 GB/s.

Results are host arrays, identical to what a single ``tk_count_device``
call on the job alone returns.
"""
from __future__ import annotations

import queue
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass

import numpy as np

from . import _torch, load_library, tk_batch_workspace_size, tk_count_batch_device, tk_default_options


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

    @property
    def latency_s(self) -> float:
        return self.t_done - self.t_submit


class Server:
    """Counting server: ``submit(job)`` returns a Future of a JobResult.

    ``max_batch_bases`` bounds the bases of one batch (and of one job: a
    larger job is refused); ``max_batch_reads`` bounds its reads;
    ``max_batch_libs`` its number of jobs.  Device memory per worker: the
    input buffers plus the workspace of the largest batch these bounds
    allow.  Pinned host memory per worker: input buffers of the same size,
    and a result buffer grown to the largest batch's records seen so far.
    """

    def __init__(self, max_batch_bases: int = 1 << 28, max_batch_reads: int = 1 << 22, max_batch_libs: int = 64,
                 workers: int = 2, opts=None, device: str = "cuda:0", linger_s: float = 0.0):
        torch = _torch()
        load_library()
        self.torch = torch
        self.device = torch.device(device)
        self.max_bases = int(max_batch_bases)
        self.max_reads = int(max_batch_reads)
        self.max_libs = int(max_batch_libs)
        self.opts = opts if opts is not None else tk_default_options()
        self.linger_s = linger_s
        # workspace bound: the largest of one library of all the bases and of
        # max_libs equal libraries sharing them, for the widest key
        ws = 0
        for k in (31, 63):
            one = tk_batch_workspace_size([0, self.max_bases], [0, self.max_reads], k, [2], self.opts)
            nb = np.linspace(0, self.max_bases, self.max_libs + 1).astype(np.uint64)
            nr = np.linspace(0, self.max_reads, self.max_libs + 1).astype(np.uint64)
            many = tk_batch_workspace_size(nb, nr, k, [2] * self.max_libs, self.opts)
            ws = max(ws, one, many)
        # a quarter more for other splits of the budget (bucket and chunk
        # tables grow with rounding per library); a batch that still needs
        # more fails with the library's workspace error
        ws = int(ws * 1.25) // 256 * 256 + 256
        self.ws_bytes = ws
        self._pending: list[tuple[Job, Future]] = []
        self._cv = threading.Condition()
        self._idle: queue.Queue = queue.Queue()
        self._stop = False
        self._workers = []
        for i in range(workers):
            w = dict(
                stream=torch.cuda.Stream(device=self.device),
                ws=torch.empty(ws, dtype=torch.uint8, device=self.device),
                bases=torch.empty(max(self.max_bases, 1), dtype=torch.uint8, device=self.device),
                offsets=torch.empty(self.max_reads + 1 + self.max_libs, dtype=torch.int64, device=self.device),
                h_bases=torch.empty(max(self.max_bases, 1), dtype=torch.uint8, pin_memory=True),
                h_offsets=torch.empty(self.max_reads + 1 + self.max_libs, dtype=torch.int64, pin_memory=True),
                h_keys=None,
                h_counts=None,
                inbox=queue.Queue(),
            )
            t = threading.Thread(target=self._work, args=(w,), daemon=True, name=f"tk-worker-{i}")
            w["thread"] = t
            self._workers.append(w)
            t.start()
            self._idle.put(w)
        self._dispatcher = threading.Thread(target=self._dispatch, daemon=True, name="tk-dispatch")
        self._dispatcher.start()

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
        if job.bases.size > self.max_bases or job.offsets.size - 1 > self.max_reads:
            raise ValueError("job larger than the server's batch budget")
        fut: Future = Future()
        job.t_submit = job.t_submit or time.perf_counter()
        with self._cv:
            self._pending.append((job, fut))
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
    def _take_batch(self):
        """Oldest waiting job plus later ones of the same k within budget."""
        job0, _ = self._pending[0]
        take, rest, bases, reads = [], [], 0, 0
        for item in self._pending:
            j = item[0]
            fits = (j.k == job0.k and len(take) < self.max_libs and bases + j.bases.size <= self.max_bases
                    and reads + j.offsets.size - 1 <= self.max_reads)
            if fits:
                take.append(item)
                bases += j.bases.size
                reads += j.offsets.size - 1
            else:
                rest.append(item)
        self._pending = rest
        return take

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
        torch = self.torch
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
        stream = w["stream"]
        # every job into its slice of the pinned input buffers, its offsets
        # rebased to its first base (the previous batch's transfer from these
        # buffers ended with that batch's stream synchronisation)
        # (host copies through torch, which runs them on its thread pool
        # without holding the interpreter lock, so both workers' copies and
        # the dispatcher proceed together)
        hb, ho = w["h_bases"], w["h_offsets"]
        ho[:1].zero_()
        for q, j in enumerate(jobs):
            if j.bases.size:
                hb[lb[q]:lb[q + 1]].copy_(torch.from_numpy(j.bases))
            if lr[q + 1] > lr[q]:
                off = torch.from_numpy(j.offsets[1:].astype(np.uint64, copy=False).view(np.int64))
                torch.add(off, lb[q], out=ho[lr[q] + 1:lr[q + 1] + 1])
        with torch.cuda.stream(stream):
            db = w["bases"][:lb[-1]]
            do = w["offsets"][:lr[-1] + 1]
            db.copy_(w["h_bases"][:lb[-1]], non_blocking=True)
            do.copy_(w["h_offsets"][:lr[-1] + 1], non_blocking=True)
            res = tk_count_batch_device(db, do, lb, lr, jobs[0].k, [j.c for j in jobs], self.opts,
                                        workspace=w["ws"], stream=stream)
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
                                     job.t_submit, t_start, t_done))
