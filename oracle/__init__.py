"""CPU oracle for exact frequent-k-mer counting.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the GPU
path (``paper_1305_1861_amd``) and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc into
``liboracle.so``); this module only marshals numpy arrays.  ``brute`` holds an
independent pure-Python string implementation used to pin the C oracle on
tiny inputs.

Paper: Roy, Bhattacharya & Schliep, "Turtle: identifying frequent k-mers with
cache-efficient algorithms", arXiv 1305.1861 -- §2.1 (extraction and
bit-encoding; pattern-blocked Bloom filter; sorting and compaction) and
Algorithm 1.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-fopenmp", "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_count_windows.restype = ctypes.c_int64
        lib.oracle_count_windows.argtypes = [_u8p, _u64p, ctypes.c_uint64, ctypes.c_int]
        lib.oracle_sort_compact.restype = ctypes.c_int64
        lib.oracle_sort_compact.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p, _u64p, _u64p]
        lib.oracle_kmer_count.restype = ctypes.c_int64
        lib.oracle_kmer_count.argtypes = [_u8p, _u64p, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_uint64, _u64p, _u64p, _u64p,
                                          ctypes.c_uint64, _u64p, _u64p]
        lib.oracle_count_queries.restype = ctypes.c_int
        lib.oracle_count_queries.argtypes = [_u8p, _u64p, ctypes.c_uint64, ctypes.c_int,
                                             _u64p, _u64p, ctypes.c_uint64, _u64p, ctypes.c_int]
        lib.oracle_pattern_positions.restype = ctypes.c_int
        lib.oracle_pattern_positions.argtypes = [ctypes.c_uint64, ctypes.c_uint32,
                                                 ctypes.c_uint32, _u8p]
        lib.oracle_block_of.restype = ctypes.c_int
        lib.oracle_block_of.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_uint64, ctypes.c_uint32, _u64p, _u32p]
        lib.oracle_bloom_model_keys.restype = ctypes.c_int
        lib.oracle_bloom_model_keys.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_int,
                                                ctypes.c_uint64, ctypes.c_uint32,
                                                ctypes.c_uint32, ctypes.c_uint64,
                                                _u64p, _u64p, _u64p, _u8p]
        lib.oracle_bloom_model_buckets_keys.restype = ctypes.c_int
        lib.oracle_bloom_model_buckets_keys.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_int,
                                                        ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                                                        ctypes.c_uint32, ctypes.c_uint64,
                                                        _u64p, _u64p, _u64p]
        lib.oracle_bloom_model_buckets.restype = ctypes.c_int
        lib.oracle_bloom_model_buckets.argtypes = [_u8p, _u64p, ctypes.c_uint64, ctypes.c_int,
                                                   ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                                                   ctypes.c_uint32, ctypes.c_uint64,
                                                   _u64p, _u64p, _u64p]
        lib.oracle_approx.restype = ctypes.c_int
        lib.oracle_approx.argtypes = [_u8p, _u64p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint64, _u64p, _u64p, _u64p, ctypes.c_uint64, _u64p, _u64p]
        lib.oracle_keys_in_range.restype = ctypes.c_int
        lib.oracle_keys_in_range.argtypes = [_u8p, _u64p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_uint64, ctypes.POINTER(_u64p), ctypes.POINTER(_u64p),
                                             _u64p]
        lib.oracle_free.restype = None
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_bloom_model.restype = ctypes.c_int
        lib.oracle_bloom_model.argtypes = [_u8p, _u64p, ctypes.c_uint64, ctypes.c_int,
                                           ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint64, _u64p, _u64p, _u64p]
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _reads(bases, offsets):
    b = np.ascontiguousarray(bases, dtype=np.uint8)
    o = np.ascontiguousarray(offsets, dtype=np.uint64)
    if b.size == 0:
        b = np.zeros(1, dtype=np.uint8)
    return b, o, int(o.size - 1)


@dataclass
class Counted:
    """Exact result: ascending keys with their counts (count >= c)."""
    hi: np.ndarray        # uint64, zero when k <= 31
    lo: np.ndarray        # uint64
    count: np.ndarray     # uint64
    n_windows: int
    n_distinct: int


def count_windows(bases, offsets, k: int) -> int:
    """Number of valid k-mer windows of a library."""
    b, o, n = _reads(bases, offsets)
    r = _load().oracle_count_windows(_p(b, _u8p), _p(o, _u64p), n, k)
    if r < 0:
        raise ValueError(f"oracle_count_windows: status {r}")
    return int(r)


def kmer_count(bases, offsets, k: int, c: int) -> Counted:
    """Every canonical k-mer with count >= c, ascending, with its exact count."""
    b, o, n = _reads(bases, offsets)
    cap = max(1, int(b.size))
    hi = np.empty(cap, np.uint64)
    lo = np.empty(cap, np.uint64)
    cnt = np.empty(cap, np.uint64)
    nw = ctypes.c_uint64(0)
    nd = ctypes.c_uint64(0)
    r = _load().oracle_kmer_count(_p(b, _u8p), _p(o, _u64p), n, k, c,
                                  _p(hi, _u64p), _p(lo, _u64p), _p(cnt, _u64p), cap,
                                  ctypes.byref(nw), ctypes.byref(nd))
    if r < 0:
        raise ValueError(f"oracle_kmer_count: status {r}")
    return Counted(hi[:r].copy(), lo[:r].copy(), cnt[:r].copy(), int(nw.value), int(nd.value))


def keys_in_range(bases, offsets, k: int, range_bits: int, range_index: int):
    """Canonical keys (hi, lo occurrence arrays, read order) of the windows
    whose key has top ``range_bits`` bits (of its 2k-bit value) equal to
    ``range_index``.  Range by range, a library too large for host memory
    can be counted exactly: the answer is the concatenation over ranges, in
    order, of ``sort_compact`` of each range's keys."""
    b, o, n = _reads(bases, offsets)
    ph, pl = _u64p(), _u64p()
    m = ctypes.c_uint64(0)
    lib = _load()
    r = lib.oracle_keys_in_range(_p(b, _u8p), _p(o, _u64p), n, k, range_bits, range_index,
                                 ctypes.byref(ph), ctypes.byref(pl), ctypes.byref(m))
    if r != 0:
        raise ValueError(f"oracle_keys_in_range: status {r}")
    q = int(m.value)
    try:
        if q == 0:
            return np.zeros(0, np.uint64), np.zeros(0, np.uint64)
        hi = np.ctypeslib.as_array(ph, shape=(q,)).copy()
        lo = np.ctypeslib.as_array(pl, shape=(q,)).copy()
        return hi, lo
    finally:
        lib.oracle_free(ph)
        lib.oracle_free(pl)


def approx_words(n_bases: int, n_reads: int, k: int, beta: int) -> int:
    """Filter words of the approximate variants: max(1, ceil(beta * W / 64))
    with W = max(n_bases - n_reads * (k - 1), 1) estimated windows."""
    w = max(n_bases - n_reads * (k - 1), 1)
    return max(1, -(-beta * w // 64))


def approx_count(bases, offsets, k: int, mode: str, c: int, n_words: int,
                 n_patterns: int = 1024, n_bits: int = 2, seed: int = 1305):
    """The approximate variants run sequentially in read order: mode
    "cturtle" (reported keys, count 0) or "single_pass" (stored sightings
    compacted, count = run + 1, kept when >= c).  Returns (Counted, number
    of reported or stored sightings)."""
    b, o, n = _reads(bases, offsets)
    cap = max(1, int(b.size))
    hi, lo, cnt = np.empty(cap, np.uint64), np.empty(cap, np.uint64), np.empty(cap, np.uint64)
    n_out, n_rep = ctypes.c_uint64(0), ctypes.c_uint64(0)
    m = {"cturtle": 1, "single_pass": 2}[mode]
    r = _load().oracle_approx(_p(b, _u8p), _p(o, _u64p), n, k, m, c, n_words, n_patterns, n_bits, seed,
                              _p(hi, _u64p), _p(lo, _u64p), _p(cnt, _u64p), cap,
                              ctypes.byref(n_out), ctypes.byref(n_rep))
    if r != 0:
        raise ValueError(f"oracle_approx: status {r}")
    q = int(n_out.value)
    return Counted(hi[:q].copy(), lo[:q].copy(), cnt[:q].copy(), 0, q), int(n_rep.value)


def sort_compact(hi, lo):
    """Sort-and-compact of explicit items: (distinct hi, distinct lo, counts)."""
    hi = np.ascontiguousarray(hi, dtype=np.uint64)
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    n = int(hi.size)
    m = max(1, n)
    oh, ol, oc = np.empty(m, np.uint64), np.empty(m, np.uint64), np.empty(m, np.uint64)
    ih = hi if n else np.zeros(1, np.uint64)
    il = lo if n else np.zeros(1, np.uint64)
    r = _load().oracle_sort_compact(_p(ih, _u64p), _p(il, _u64p), n,
                                    _p(oh, _u64p), _p(ol, _u64p), _p(oc, _u64p))
    if r < 0:
        raise ValueError(f"oracle_sort_compact: status {r}")
    return oh[:r].copy(), ol[:r].copy(), oc[:r].copy()


def count_queries(bases, offsets, k: int, q_hi, q_lo, n_threads: int = 1) -> np.ndarray:
    """Exact counts of the given (sorted, distinct) keys over every window."""
    b, o, n = _reads(bases, offsets)
    q_hi = np.ascontiguousarray(q_hi, dtype=np.uint64)
    q_lo = np.ascontiguousarray(q_lo, dtype=np.uint64)
    nq = int(q_hi.size)
    out = np.zeros(max(1, nq), np.uint64)
    qh = q_hi if nq else np.zeros(1, np.uint64)
    ql = q_lo if nq else np.zeros(1, np.uint64)
    r = _load().oracle_count_queries(_p(b, _u8p), _p(o, _u64p), n, k, _p(qh, _u64p),
                                     _p(ql, _u64p), nq, _p(out, _u64p), n_threads)
    if r != 0:
        raise ValueError(f"oracle_count_queries: status {r}")
    return out[:nq]


# --------------------------------------------------------------------------
# Bloom model (pattern-blocked Bloom filter, §2.1, with two-plane semantics)
# --------------------------------------------------------------------------

#: Default Bloom parameters of the counting interface (bits per table entry,
#: i.e. per 64-bit block word; number of table entries; SplitMix64 seed;
#: first-plane bits per estimated window).  A key sets 4 * BLOOM_BITS bits.
BLOCK_WORDS = 4
BLOOM_BITS = 2
BLOOM_PATTERNS = 1024
BLOOM_SEED = 1305
BLOOM_BETA = 4


def default_blocks(n_bases: int, n_reads: int, k: int, beta: int = BLOOM_BETA) -> int:
    """Filter size rule of the counting interface.

    W = max(n_bases - n_reads * (k - 1), 1) estimates the windows; the first
    plane gets ``beta`` bits per estimated window, 256 bits per block:
    ``n_blocks = max(1, ceil(beta * W / 256))``.
    """
    w = max(n_bases - n_reads * (k - 1), 1)
    return max(1, -(-beta * w // 256))


def pattern_positions(n_patterns: int = BLOOM_PATTERNS, n_bits: int = BLOOM_BITS,
                      seed: int = BLOOM_SEED) -> np.ndarray:
    """``uint8[n_patterns, n_bits]`` bit positions in [0, 64) of the table entries."""
    out = np.zeros(n_patterns * n_bits, np.uint8)
    r = _load().oracle_pattern_positions(seed, n_patterns, n_bits, _p(out, _u8p))
    if r != 0:
        raise ValueError(f"oracle_pattern_positions: status {r}")
    return out.reshape(n_patterns, n_bits)


def pattern_masks(n_patterns: int = BLOOM_PATTERNS, n_bits: int = BLOOM_BITS,
                  seed: int = BLOOM_SEED) -> np.ndarray:
    """Pattern table as one ``uint64`` word mask per entry."""
    pos = pattern_positions(n_patterns, n_bits, seed).astype(np.uint64)
    masks = np.zeros(n_patterns, np.uint64)
    for j in range(n_bits):
        masks |= np.uint64(1) << pos[:, j]
    return masks


def block_of(hi: int, lo: int, two_words: bool, n_blocks: int,
             n_patterns: int = BLOOM_PATTERNS) -> tuple[int, list[int]]:
    """(block index, table entry of each of the 4 block words) of one key."""
    blk = ctypes.c_uint64(0)
    ent = (ctypes.c_uint32 * BLOCK_WORDS)()
    r = _load().oracle_block_of(hi, lo, int(two_words), n_blocks, n_patterns,
                                ctypes.byref(blk), ent)
    if r != 0:
        raise ValueError("oracle_block_of")
    return int(blk.value), [int(x) for x in ent]


@dataclass
class BloomStats:
    n_cand_occ: int      # occurrences collected by the screen
    n_cand: int          # distinct candidate keys
    n_cand_single: int   # candidates seen once (false positives of the screen)
    flags: np.ndarray | None = None


def bloom_model_keys(hi, lo, two_words: bool, n_blocks: int,
                     n_patterns: int = BLOOM_PATTERNS, n_bits: int = BLOOM_BITS,
                     seed: int = BLOOM_SEED, want_flags: bool = False) -> BloomStats:
    hi = np.ascontiguousarray(hi, dtype=np.uint64)
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    n = int(hi.size)
    flags = np.zeros(max(1, n), np.uint8) if want_flags else None
    a, b, c = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    ih = hi if n else np.zeros(1, np.uint64)
    il = lo if n else np.zeros(1, np.uint64)
    r = _load().oracle_bloom_model_keys(_p(ih, _u64p), _p(il, _u64p), n, int(two_words),
                                        n_blocks, n_patterns, n_bits, seed,
                                        ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                        _p(flags, _u8p) if want_flags else None)
    if r != 0:
        raise ValueError(f"oracle_bloom_model_keys: status {r}")
    return BloomStats(int(a.value), int(b.value), int(c.value),
                      flags[:n] if want_flags else None)


def bloom_model(bases, offsets, k: int, n_blocks: int, n_patterns: int = BLOOM_PATTERNS,
                n_bits: int = BLOOM_BITS, seed: int = BLOOM_SEED) -> BloomStats:
    b, o, n = _reads(bases, offsets)
    a, bb, c = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    r = _load().oracle_bloom_model(_p(b, _u8p), _p(o, _u64p), n, k, n_blocks, n_patterns,
                                   n_bits, seed, ctypes.byref(a), ctypes.byref(bb),
                                   ctypes.byref(c))
    if r != 0:
        raise ValueError(f"oracle_bloom_model: status {r}")
    return BloomStats(int(a.value), int(bb.value), int(c.value))


def partition_bits(n_bases: int, n_reads: int, k: int, part_bits: int = -1) -> int:
    """Bucket bits D of the per-bucket filters (rule of the counting interface).

    W = max(n_bases - n_reads * (k - 1), 1), L = ceil(log2 W); D = L - 11 for
    one-word keys (k <= 31) and L - 10 for two-word keys, clamped to
    [0, min(20, 2k)]; an explicit ``part_bits`` >= 0 is clamped the same way.
    """
    cap = min(20, 2 * k)
    if part_bits >= 0:
        return min(part_bits, cap)
    w = max(n_bases - n_reads * (k - 1), 1)
    lg = (w - 1).bit_length()
    return max(0, min(lg - (11 if k <= 31 else 10), cap))


def bloom_model_buckets_keys(hi, lo, k: int, D: int, beta: int = BLOOM_BETA,
                             n_patterns: int = BLOOM_PATTERNS, n_bits: int = BLOOM_BITS,
                             seed: int = BLOOM_SEED) -> BloomStats:
    hi = np.ascontiguousarray(hi, dtype=np.uint64)
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    n = int(hi.size)
    ih = hi if n else np.zeros(1, np.uint64)
    il = lo if n else np.zeros(1, np.uint64)
    a, b, c = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    r = _load().oracle_bloom_model_buckets_keys(_p(ih, _u64p), _p(il, _u64p), n, k, D, beta,
                                                n_patterns, n_bits, seed, ctypes.byref(a),
                                                ctypes.byref(b), ctypes.byref(c))
    if r != 0:
        raise ValueError(f"oracle_bloom_model_buckets_keys: status {r}")
    return BloomStats(int(a.value), int(b.value), int(c.value))


def bloom_model_buckets(bases, offsets, k: int, D: int, beta: int = BLOOM_BETA,
                        n_patterns: int = BLOOM_PATTERNS, n_bits: int = BLOOM_BITS,
                        seed: int = BLOOM_SEED) -> BloomStats:
    """Per-bucket Bloom model over the windows of a library."""
    b, o, n = _reads(bases, offsets)
    a, bb, c = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
    r = _load().oracle_bloom_model_buckets(_p(b, _u8p), _p(o, _u64p), n, k, D, beta, n_patterns,
                                           n_bits, seed, ctypes.byref(a), ctypes.byref(bb),
                                           ctypes.byref(c))
    if r != 0:
        raise ValueError(f"oracle_bloom_model_buckets: status {r}")
    return BloomStats(int(a.value), int(bb.value), int(c.value))


# --------------------------------------------------------------------------
# Theory used to pin the Bloom model
# --------------------------------------------------------------------------

def standard_bloom_fpr(bits_per_item: float, n_hashes: int) -> float:
    """False-positive rate of an ordinary Bloom filter, (1 - e^{-K/b})^K."""
    return (1.0 - math.exp(-n_hashes / bits_per_item)) ** n_hashes


def blocked_singleton_fp_prob(masks: np.ndarray, n_blocks: int, n_others: int,
                              words: int = BLOCK_WORDS) -> float:
    """Probability that a key seen once passes the two-plane screen.

    A key seen once is a candidate iff every bit of its pattern is also
    touched by another key.  Other keys fall in its block independently with
    probability 1/n_blocks, and each of their ``words`` block words carries a
    table entry drawn uniformly and independently.  For j other keys in the
    block, inclusion-exclusion over subsets J of the key's own bits gives
        P(all covered) = sum_J (-1)^|J| f(J)^j,
    with f(J) = probability that one other key misses all of J.  Because the
    words are independent, f(J) is a product over words and the sum factors
    into a product over words; averaging over the key's own (independent)
    entries gives  E[P | j] = (E_o g(o, j))^words  with
        g(o, j) = sum_{J subset of o} (-1)^|J| f1(J)^j,
    f1(J) = fraction of table entries disjoint from J.  The result averages
    over j ~ Binomial(n_others, 1/n_blocks).
    """
    tab = [int(m) for m in masks.tolist()]
    n_pat = len(tab)
    p = 1.0 / n_blocks
    jmax = int(min(n_others, n_others * p + 12 * math.sqrt(n_others * p + 1) + 30))
    j = np.arange(jmax + 1)
    logw = (np.array([math.lgamma(n_others + 1) - math.lgamma(x + 1)
                      - math.lgamma(n_others - x + 1) for x in j])
            + j * math.log(p) + (n_others - j) * (math.log1p(-p) if p < 1 else 0.0))
    if p >= 1.0:
        logw = np.where(j == n_others, 0.0, -np.inf)
    w = np.exp(logw)
    f_cache: dict[int, float] = {}

    def f1(sub: int) -> float:
        if sub not in f_cache:
            f_cache[sub] = sum(1 for t in tab if t & sub == 0) / n_pat
        return f_cache[sub]

    eg = np.zeros(jmax + 1)
    for own in tab:
        bits = [1 << b for b in range(64) if (own >> b) & 1]
        g = np.zeros(jmax + 1)
        for sel in range(1 << len(bits)):
            sub = 0
            for i, bb in enumerate(bits):
                if (sel >> i) & 1:
                    sub |= bb
            sign = -1.0 if bin(sel).count("1") % 2 else 1.0
            g += sign * f1(sub) ** j
        eg += g
    eg /= n_pat
    return float(np.dot(w, eg ** words))
