"""Brute-force k-mer counting on Python strings.  TEST INFRASTRUCTURE ONLY.

Independent of the C oracle: no 2-bit encoding and no integer sort.  Windows
are substrings, the reverse complement is built with ``str.translate`` and
reversal, the canonical form is the lexicographically smaller string, and a
``collections.Counter`` counts.  Only for tiny inputs.

It pins the C oracle's readings of the paper's extraction rules (§2.1,
k-mer extraction and bit-encoding): case folding, cuts at non-ACGT bytes,
no window across reads, canonical = smaller of the pair, and ascending order
(for codes A<C<G<T with the first base most significant, numeric order of the
encoding is the lexicographic order of the strings).
"""
from __future__ import annotations

from collections import Counter

_COMP = str.maketrans("ACGT", "TGCA")
_UPPER = str.maketrans("abcdefghijklmnopqrstuvwxyz", "ABCDEFGHIJKLMNOPQRSTUVWXYZ")
_ACGT = set("ACGT")


def ascii_upper(s: str) -> str:
    """Upper-case ASCII letters only (str.upper would also change other bytes)."""
    return s.translate(_UPPER)


def revcomp(s: str) -> str:
    return s.translate(_COMP)[::-1]


def canonical(s: str) -> str:
    r = revcomp(s)
    return s if s <= r else r


def windows(read: str, k: int):
    """Every length-k substring of the upper-cased read made of A/C/G/T only."""
    up = ascii_upper(read)
    for i in range(len(up) - k + 1):
        w = up[i:i + k]
        if set(w) <= _ACGT:
            yield w


def count(reads, k: int, c: int):
    """Sorted list of (canonical k-mer string, count) with count >= c."""
    cnt = Counter()
    for r in reads:
        for w in windows(r, k):
            cnt[canonical(w)] += 1
    return sorted((s, n) for s, n in cnt.items() if n >= c)


def n_windows(reads, k: int) -> int:
    return sum(1 for r in reads for _ in windows(r, k))


def encode(s: str) -> int:
    """Integer of a k-mer string: A=0, C=1, G=2, T=3, first base most significant."""
    return int(s.translate(str.maketrans("ACGT", "0123")), 4) if s else 0


def decode(v: int, k: int) -> str:
    out = []
    for _ in range(k):
        out.append("ACGT"[v & 3])
        v >>= 2
    return "".join(reversed(out))
