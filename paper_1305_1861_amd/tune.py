"""Autotuning of the counting options for one library on one device.

The result of a counting call does not depend on the bucket bits D or on
the filter bits per window (every count is exact; only the number of
screen false positives changes), so those two can be chosen for speed
alone.  ``autotune`` times ``tk_count_device`` on the caller's device-resident
library for each candidate pair, around the size rule's D, and returns the
fastest options with every timing.

Candidates whose workspace does not fit ``max_workspace_bytes`` are
skipped.  Candidates that make buckets overflow a workgroup fall back to the
slower global-memory kernels; they are timed like the others.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import STAGES, _torch, tk_count_device, tk_default_options, tk_part_bits, tk_workspace_size


@dataclass
class TuneResult:
    part_bits: int
    bloom_beta: int
    ms: float
    timings: list = field(default_factory=list)  # (part_bits, bloom_beta, ms, n_fallback)

    def options(self, flags: int = 0):
        o = tk_default_options()
        o.part_bits = self.part_bits
        o.bloom_beta = self.bloom_beta
        o.flags = flags
        return o


def autotune(bases, offsets, k: int, c: int, part_bits=None, betas=(2, 4, 8), repeats: int = 3,
             max_workspace_bytes: int | None = None, stream=None) -> TuneResult:
    """Fastest (part_bits, bloom_beta) for this library.

    ``bases``/``offsets``: device tensors as for ``tk_count_device``.
    ``part_bits``: candidate D values (default: the size rule's D - 1, D,
    D + 1, within 0..20).  Device time per candidate: the summed stage
    times (HIP events) of the fastest of ``repeats`` calls after one warm-up.
    """
    torch = _torch()
    n_bases = int(bases.numel())
    n_reads = int(offsets.numel()) - 1
    if part_bits is None:
        d = tk_part_bits(n_bases, n_reads, k)
        part_bits = sorted({x for x in (d - 1, d, d + 1) if 0 <= x <= 20})
    timings = []
    best = None
    ws = None
    for D in part_bits:
        for beta in betas:
            o = tk_default_options()
            o.part_bits = D
            o.bloom_beta = beta
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
            timings.append((D, beta, ms, int(r.n_fallback)))
            if best is None or ms < best[2]:
                best = (D, beta, ms)
    if best is None:
        raise ValueError("no candidate fits the workspace bound")
    return TuneResult(best[0], best[1], best[2], timings)
