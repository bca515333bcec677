"""Brute-force BWT of a string set by sorting rotations (tiny inputs only).

TEST INFRASTRUCTURE ONLY (see oracle/oracle.py).  This is a second, independent
reading of the definition in Section 2 of Pantaleoni, arXiv:1410.0562, written
in pure Python so that it shares nothing with the C oracle either:

* every terminator is its own symbol: $_j is the integer j, and a base is the
  integer m + 1 + (its index in ACGT), so $_0 < ... < $_{m-1} < A < C < G < T
  is plain integer order;
* T = S_0 $_0 ... S_{m-1} $_{m-1}; since the terminators are all distinct, all
  n rotations of T are distinct, and sorting rotations sorts suffixes;
* Eq. 1: B[i] is the last symbol of the i-th smallest rotation, i.e.
  T[(SA[i] - 1) mod n].
"""
from __future__ import annotations

from typing import Sequence

_BASES = "ACGT"


def tokens(reads: Sequence[str]) -> list:
    m = len(reads)
    T = []
    for j, s in enumerate(reads):
        for ch in s:
            T.append(m + 1 + _BASES.index(ch))
        T.append(j)
    return T


def bwt(reads: Sequence[str]) -> str:
    m = len(reads)
    T = tokens(reads)
    n = len(T)
    rots = sorted(range(n), key=lambda i: T[i:] + T[:i])
    out = []
    for i in rots:
        x = T[(i - 1) % n]
        out.append("$" if x < m else _BASES[x - m - 1])
    return "".join(out)


def suffix_array(reads: Sequence[str]) -> list:
    T = tokens(reads)
    n = len(T)
    return sorted(range(n), key=lambda i: T[i:] + T[:i])


def old_smaller(old: Sequence[str], new: Sequence[str]) -> list:
    """For every suffix of the new strings (in text order of the new strings'
    concatenation P_0 $ P_1 $ ...), the number of suffixes of the old strings'
    text that are smaller, with the new strings numbered after the old ones."""
    allr = list(old) + list(new)
    T = tokens(allr)
    n_old = sum(len(s) + 1 for s in old)
    res = []
    for p in range(n_old, len(T)):
        sp = T[p:]
        res.append(sum(1 for q in range(n_old) if T[q:] < sp))
    return res


def occurrences(reads: Sequence[str], pattern: str) -> int:
    """Occurrences of pattern inside the strings (overlaps counted); the
    empty pattern occurs once per suffix, terminators included."""
    if pattern == "":
        return sum(len(s) + 1 for s in reads)
    L = len(pattern)
    return sum(1 for s in reads for i in range(len(s) - L + 1) if s[i:i + L] == pattern)


def rows_below(reads: Sequence[str], pattern: str) -> int:
    """Suffixes smaller than the pattern: the suffix (up to and including its
    terminator, the smallest symbols) compared with the pattern's symbols,
    a suffix that has the pattern as a prefix not counted."""
    m = len(reads)
    T = tokens(reads)
    P = [m + 1 + _BASES.index(ch) for ch in pattern]
    below = 0
    for p in range(len(T)):
        end = p
        while T[end] >= m + 1:
            end += 1
        head = T[p:end + 1][:len(P)]
        # a suffix shorter than P ends in its terminator, which differs from
        # (and is smaller than) the pattern's base at that offset
        if head != P and head < P:
            below += 1
    return below


def reverse_complement(s: str) -> str:
    return s[::-1].translate(str.maketrans("ACGT", "TGCA"))
