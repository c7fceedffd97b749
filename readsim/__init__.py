"""Seeded synthetic read libraries.

This module only draws inputs: genomes, reads sampled from both strands,
substitution errors and ambiguous ``N`` calls.  It holds none of the counting
method's arithmetic (no 2-bit encoding, no canonical form, no hashing), so both
the CPU oracle and the GPU path can take their inputs from it without sharing
any code with each other.

A read library is returned as two numpy arrays:

* ``bases``   -- ``uint8[n_bases]``, the ASCII bytes of all reads concatenated;
* ``offsets`` -- ``uint64[n_reads + 1]``, read ``r`` is
  ``bases[offsets[r]:offsets[r + 1]]``.

The workloads stand in for the read libraries the paper benchmarks (its
Table 2), which are not available here; their recipe is stated in each
function.  Every draw comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ASCII_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8).copy()
N_BYTE = ord("N")


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_genome(rng: np.random.Generator, g: int) -> np.ndarray:
    """``g`` bases drawn i.i.d. uniform over A, C, G, T, as symbol ids 0..3."""
    return rng.integers(0, 4, size=g, dtype=np.uint8)


def mutate(rng: np.random.Generator, sym: np.ndarray, rate: float) -> np.ndarray:
    """Substitute each symbol with probability ``rate`` by one of the other three."""
    out = sym.copy()
    if rate <= 0.0 or out.size == 0:
        return out
    hit = rng.random(out.shape, dtype=np.float32) < np.float32(rate)
    n = int(hit.sum())
    if n:
        out[hit] = (out[hit] + rng.integers(1, 4, size=n, dtype=np.uint8)) & np.uint8(3)
    return out


def repeat_genome(rng: np.random.Generator, g_unique: int, n_copies: int,
                  seg_len: int, copies_lo: int, copies_hi: int,
                  divergence: float) -> np.ndarray:
    """Uniform sequence of ``g_unique`` bases with ``n_copies`` repeat copies inserted.

    Repeat families are drawn until ``n_copies`` copies exist: each family has
    a uniform source segment of ``seg_len`` bases and U{copies_lo..copies_hi}
    copies (the last family is truncated to the total), each copy being the
    source with i.i.d. ``divergence`` substitutions.  The copies are inserted
    at uniform random points of the unique sequence, in random order.
    """
    unique = uniform_genome(rng, g_unique)
    copies = []
    while len(copies) < n_copies:
        src = uniform_genome(rng, seg_len)
        m = int(rng.integers(copies_lo, copies_hi + 1))
        for _ in range(min(m, n_copies - len(copies))):
            copies.append(mutate(rng, src, divergence))
    order = rng.permutation(n_copies)
    points = np.sort(rng.integers(0, g_unique + 1, size=n_copies))
    pieces = []
    prev = 0
    for p, ci in zip(points, order):
        pieces.append(unique[prev:p])
        pieces.append(copies[ci])
        prev = int(p)
    pieces.append(unique[prev:])
    return np.concatenate(pieces)


def sample_reads(rng: np.random.Generator, genome: np.ndarray, n_reads: int,
                 read_len: int, sub_rate: float, n_rate: float = 0.0,
                 chunk_reads: int = 1 << 18) -> tuple[np.ndarray, np.ndarray]:
    """Fixed-length reads with uniform starts in ``[0, G - L]``.

    Each read is taken from the reverse-complement strand with probability
    1/2 (symbols reversed and complemented as 3 - s).  Then every base is
    substituted with probability ``sub_rate`` (to one of the 3 others,
    uniformly) and afterwards replaced by ``N`` with probability ``n_rate``.
    """
    g = int(genome.size)
    if g < read_len:
        raise ValueError("genome shorter than the read length")
    starts = rng.integers(0, g - read_len + 1, size=n_reads)
    minus = rng.random(n_reads) < 0.5
    bases = np.empty(n_reads * read_len, dtype=np.uint8)
    col = np.arange(read_len)
    for c0 in range(0, n_reads, chunk_reads):
        c1 = min(n_reads, c0 + chunk_reads)
        sym = genome[starts[c0:c1, None] + col[None, :]]
        m = minus[c0:c1]
        sym[m] = np.uint8(3) - sym[m, ::-1]
        sym = mutate(rng, sym, sub_rate)
        asc = ASCII_ACGT[sym]
        if n_rate > 0.0:
            asc[rng.random(asc.shape, dtype=np.float32) < np.float32(n_rate)] = N_BYTE
        bases[c0 * read_len:c1 * read_len] = asc.ravel()
    offsets = np.arange(n_reads + 1, dtype=np.uint64) * np.uint64(read_len)
    return bases, offsets


@dataclass(frozen=True)
class Library:
    """One synthetic read library plus the counting parameters it is run at."""
    name: str
    k: int
    c: int
    bases: np.ndarray = field(repr=False)
    offsets: np.ndarray = field(repr=False)

    @property
    def n_reads(self) -> int:
        return int(self.offsets.size - 1)

    @property
    def n_bases(self) -> int:
        return int(self.bases.size)


def small_library(scale: float = 1.0, seed: int = 1) -> Library:
    """1 Mbp uniform genome, 100 bp reads at 10x, 1 % substitutions, k=31, c=2.

    About 1e5 reads and 7e6 k-mer windows at ``scale=1``.
    """
    rng = rng_for(seed)
    g = max(200, int(round(1_000_000 * scale)))
    genome = uniform_genome(rng, g)
    n = int(round(10 * g / 100))
    b, o = sample_reads(rng, genome, n, 100, 0.01)
    return Library("uniform-1Mbp-10x-L100-k31", 31, 2, b, o)


def large_library(scale: float = 1.0, seed: int = 2) -> Library:
    """50 Mbp genome with repeats, 100 bp reads at 30x, 1 % substitutions, k=31, c=2.

    80 % of the genome is unique uniform sequence; 20 % is 5 kbp repeat
    copies (families of 2-10 copies, 2 % divergence from the family source).
    About 1.5e7 reads and 1.05e9 windows at ``scale=1``.
    """
    rng = rng_for(seed)
    g = max(20_000, int(round(50_000_000 * scale)))
    n_copies = max(1, int(round(0.2 * g / 5000)))
    genome = repeat_genome(rng, g - n_copies * 5000, n_copies, 5000, 2, 10, 0.02)
    n = int(round(30 * genome.size / 100))
    b, o = sample_reads(rng, genome, n, 100, 0.01)
    return Library("repeats-50Mbp-30x-L100-k31", 31, 2, b, o)


def long_k_library(scale: float = 1.0, seed: int = 3) -> Library:
    """20 Mbp uniform genome, 150 bp reads at 40x, 0.5 % subs + 0.1 % N, k=63, c=2.

    About 5.3e6 reads and 4.4e8 windows at ``scale=1``.
    """
    rng = rng_for(seed)
    g = max(300, int(round(20_000_000 * scale)))
    genome = uniform_genome(rng, g)
    n = int(round(40 * g / 150))
    b, o = sample_reads(rng, genome, n, 150, 0.005, 0.001)
    return Library("uniform-20Mbp-40x-L150-k63-N", 63, 2, b, o)


WORKLOADS = {
    "small": small_library,
    "large": large_library,
    "long_k": long_k_library,
}


def _batched_draws(j: int, scale: float, base_seed: int):
    """Generator, genome size and coverage of batched library j (the first
    draws of its generator)."""
    rng = rng_for(base_seed + j)
    g = int(round(math.exp(rng.uniform(math.log(1e5), math.log(2e7))) * scale))
    g = max(g, 200)
    cov = rng.uniform(5.0, 60.0)
    return rng, g, cov


def batched_library_size(j: int, scale: float = 1.0, base_seed: int = 4000) -> tuple[int, int]:
    """(n_bases, n_reads) of batched library j without generating it."""
    _, g, cov = _batched_draws(j, scale, base_seed)
    n = max(1, int(round(cov * g / 100)))
    return 100 * n, n


def batched_library(j: int, scale: float = 1.0, base_seed: int = 4000) -> Library:
    """Library j of the batched workload: genome log-uniform in 0.1-20 Mbp,
    coverage U[5, 60], 100 bp reads, 1 % substitutions, k=31, c=2, drawn
    from seed ``base_seed + j``.  ``scale`` multiplies the genome size."""
    rng, g, cov = _batched_draws(j, scale, base_seed)
    genome = uniform_genome(rng, g)
    n = max(1, int(round(cov * g / 100)))
    b, o = sample_reads(rng, genome, n, 100, 0.01)
    return Library(f"lib{j}-{g}bp-{cov:.1f}x", 31, 2, b, o)


def batched_libraries(n_libs: int = 256, scale: float = 1.0, base_seed: int = 4000):
    """Libraries of uneven size: genome log-uniform in 0.1-20 Mbp, coverage U[5, 60].

    100 bp reads, 1 % substitutions, k=31, c=2; library ``j`` uses seed
    ``base_seed + j``.  ``scale`` multiplies every genome size.
    """
    return [batched_library(j, scale, base_seed) for j in range(n_libs)]


def batched_waves(n_libs: int = 256, scale: float = 1.0, base_seed: int = 4000,
                  wave_bases: int = 2_000_000_000) -> list[list[int]]:
    """Consecutive batched libraries grouped into waves of at most
    ``wave_bases`` bases each (a larger library forms a wave alone)."""
    waves, cur, acc = [], [], 0
    for j in range(n_libs):
        nb, _ = batched_library_size(j, scale, base_seed)
        if cur and acc + nb > wave_bases:
            waves.append(cur)
            cur, acc = [], 0
        cur.append(j)
        acc += nb
    if cur:
        waves.append(cur)
    return waves


# ---------------------------------------------------------------------------
# Small adversarial inputs for tests
# ---------------------------------------------------------------------------

def random_reads(seed: int, n_reads: int, min_len: int = 0, max_len: int = 120,
                 n_rate: float = 0.02, lower_rate: float = 0.05,
                 junk_rate: float = 0.005) -> tuple[np.ndarray, np.ndarray]:
    """Reads of random length in ``[min_len, max_len]`` over ``ACGT`` with noise.

    Bases are uniform ACGT, then each byte independently becomes ``N``
    (``n_rate``), lower case (``lower_rate``) or an arbitrary non-ACGT byte
    (``junk_rate``).  Empty reads occur when ``min_len`` is 0.
    """
    rng = rng_for(seed)
    lens = rng.integers(min_len, max_len + 1, size=n_reads)
    offsets = np.zeros(n_reads + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(lens)
    total = int(offsets[-1])
    bases = ASCII_ACGT[rng.integers(0, 4, size=total, dtype=np.uint8)]
    u = rng.random(total)
    lower = u < lower_rate
    bases[lower] = bases[lower] | np.uint8(0x20)
    bases[(u >= lower_rate) & (u < lower_rate + n_rate)] = N_BYTE
    junk = (u >= lower_rate + n_rate) & (u < lower_rate + n_rate + junk_rate)
    if junk.any():
        pool = np.array([b for b in range(256) if chr(b) not in "ACGTacgt"], dtype=np.uint8)
        bases[junk] = pool[rng.integers(0, pool.size, size=int(junk.sum()))]
    return bases, offsets


def de_bruijn(alphabet: str, n: int) -> str:
    """Linear de Bruijn sequence B(|alphabet|, n): every length-n word over the
    alphabet occurs exactly once (Fredricksen-Kessler-Maiorana construction,
    plus the n - 1 wrap-around symbols)."""
    kk = len(alphabet)
    a = [0] * kk * n
    seq = []

    def db(t, p):
        if t > n:
            if n % p == 0:
                seq.extend(a[1:p + 1])
        else:
            a[t] = a[t - p]
            db(t + 1, p)
            for j in range(a[t - p] + 1, kk):
                a[t] = j
                db(t + 1, t)

    db(1, 1)
    cyc = "".join(alphabet[i] for i in seq)
    return cyc + cyc[:n - 1]


def from_strings(reads) -> tuple[np.ndarray, np.ndarray]:
    """Pack a list of ``str``/``bytes`` reads into the (bases, offsets) layout."""
    raw = [r.encode("latin-1") if isinstance(r, str) else bytes(r) for r in reads]
    offsets = np.zeros(len(raw) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum([len(r) for r in raw]) if raw else []
    bases = np.frombuffer(b"".join(raw), dtype=np.uint8).copy()
    return bases, offsets


def to_strings(bases: np.ndarray, offsets: np.ndarray) -> list[str]:
    raw = bases.tobytes()
    return [raw[int(offsets[i]):int(offsets[i + 1])].decode("latin-1")
            for i in range(offsets.size - 1)]


_SHARED = None  # (bases map, offsets map) of the workload being drawn


def _fill_batched(args):
    """Draw batched library j into its slice of the shared bases and offsets."""
    j, scale, base_seed, b0, r0, nb, nr = args
    lib = batched_library(j, scale, base_seed)
    bases = np.frombuffer(_SHARED[0], dtype=np.uint8, count=nb)
    offs = np.frombuffer(_SHARED[1], dtype=np.uint64, count=nr + 1)
    bases[b0:b0 + lib.n_bases] = lib.bases
    offs[r0 + 1:r0 + lib.n_reads + 1] = lib.offsets[1:] + np.uint64(b0)
    return j


def batched_workload(n_libs: int = 256, scale: float = 1.0, base_seed: int = 4000, workers: int = 8,
                     progress=None):
    """All batched libraries laid end to end in one bases/offsets pair:
    returns (bases, offsets, lib_bases, lib_reads), library j owning bases
    [lib_bases[j], lib_bases[j+1]) and reads [lib_reads[j], lib_reads[j+1]).
    The libraries are the ones ``batched_library`` draws (identical bytes);
    ``workers`` forked processes draw them in parallel into shared memory;
    ``progress(done, total)`` is called as libraries are finished."""
    import mmap
    import multiprocessing as mp
    global _SHARED
    sizes = [batched_library_size(j, scale, base_seed) for j in range(n_libs)]
    lib_bases = np.zeros(n_libs + 1, np.uint64)
    lib_reads = np.zeros(n_libs + 1, np.uint64)
    lib_bases[1:] = np.cumsum([s[0] for s in sizes])
    lib_reads[1:] = np.cumsum([s[1] for s in sizes])
    nb, nr = int(lib_bases[-1]), int(lib_reads[-1])
    _SHARED = (mmap.mmap(-1, max(nb, 1)), mmap.mmap(-1, 8 * (nr + 1)))
    tasks = [(j, scale, base_seed, int(lib_bases[j]), int(lib_reads[j]), nb, nr)
             for j in sorted(range(n_libs), key=lambda j: -sizes[j][0])]
    try:
        if workers > 1:
            with mp.get_context("fork").Pool(workers) as pool:
                for done, _ in enumerate(pool.imap_unordered(_fill_batched, tasks), 1):
                    if progress:
                        progress(done, n_libs)
        else:
            for done, t in enumerate(tasks, 1):
                _fill_batched(t)
                if progress:
                    progress(done, n_libs)
        bases = np.frombuffer(_SHARED[0], dtype=np.uint8, count=nb)
        offsets = np.frombuffer(_SHARED[1], dtype=np.uint64, count=nr + 1)
    finally:
        _SHARED = None
    return bases, offsets, lib_bases, lib_reads
