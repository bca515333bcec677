"""CPU oracle for the BWT of a string set and for each step of set-bwte.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library and never imports it.

Everything here follows Pantaleoni, arXiv:1410.0562:

* the BWT of a string set is the BWT (Eq. 1) of T = S_0 $_0 ... S_{m-1} $_{m-1}
  with $_0 < ... < $_{m-1} < A < C < G < T (Section 2);
* rank(c, k, B) counts c in B[0..k) (Eq. 2);
* set-bwte (Algorithm 1) adds blocks of whole strings to a partial BWT B_ext:
  suffix-sort the block, take the preceding symbol of every sorted suffix
  (B_int), rank every block suffix among the old suffixes (ComputeRanks,
  Section 4), reorder the ranks into suffix order (g_sa), and insert B_int[i]
  into B_ext before old row g_sa[i] (Insert, Section 5).

Beyond the construction, two things the paper names around it:

* the FM-index use of the BWT (the BWT with rank, Eq. 2): for a pattern, the
  rows of the sorted suffixes that start with it, by a scan over every suffix
  (pattern_rows);
* reversal, which Section 2 notes is possible, and the set with every string's
  reverse complement beside it (reverse_strings, with_reverse_complements),
  as plain transformations of the input strings.

The ranks are taken from their definition -- the number of old suffixes smaller
than each new suffix -- out of one suffix array of the old and new text
together, not by LF steps; Lemma 1's recurrence is only a cross-check in the
tests.

Readings taken where the paper is silent or inconsistent (each listed with its
reason in the design notes of the repository):

* g is indexed by off_j + k where off is the exclusive prefix sum of |P_j|+1;
* every terminator is printed as '$';
* strings appended later get larger terminators (arrival order);
* blocks are whole strings, cut greedily before the string that would make the
  block exceed M suffixes (terminators included); a longer string is a block
  by itself.

Symbol codes inside the oracle: 0 = terminator, 1..4 = A, C, G, T.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bwt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ASCII = np.frombuffer(b"$ACGT", dtype=np.uint8)
_CODE_OF_ASCII = np.full(256, 255, dtype=np.uint8)
for _i, _ch in enumerate(b"$ACGT"):
    _CODE_OF_ASCII[_ch] = _i


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (plain -O2, no GPU code)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u64 = ctypes.c_uint64
    lib.oracle_sa.argtypes = [u8p, u64, u64p]
    lib.oracle_sa.restype = None
    lib.oracle_sa_threads.argtypes = [u8p, u64, u64p, ctypes.c_int]
    lib.oracle_sa_threads.restype = ctypes.c_int
    lib.oracle_bwt.argtypes = [u8p, u64, u64p, u8p]
    lib.oracle_bwt.restype = None
    lib.oracle_count_smaller.argtypes = [u8p, u64, u64]
    lib.oracle_count_smaller.restype = u64
    lib.oracle_lf_invert.argtypes = [u8p, u64, u64p, u64, u64p, u8p, u64p]
    lib.oracle_lf_invert.restype = ctypes.c_int
    lib.oracle_count_old_smaller.argtypes = [u8p, u64, u64]
    lib.oracle_count_old_smaller.restype = u64
    lib.oracle_pattern_rows.argtypes = [u8p, u64, u8p, u64, u64p, u64p]
    lib.oracle_pattern_rows.restype = None
    _lib = lib
    return lib


def _p8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


# --------------------------------------------------------------------------
# Input handling (the oracle's own; nothing here is shared with the library)
# --------------------------------------------------------------------------

def unpack_2bit(packed: np.ndarray, nsym: int) -> np.ndarray:
    """Codes 0..3 (A,C,G,T) of symbols 0..nsym-1 of a 2-bit, LSB-first packing:
    symbol s sits in byte s // 4 at bits 2*(s % 4) .. 2*(s % 4)+1."""
    packed = np.asarray(packed, dtype=np.uint8)
    out = np.empty(len(packed) * 4, dtype=np.uint8)
    for q in range(4):
        out[q::4] = (packed >> (2 * q)) & 3
    return out[:nsym]


def reads_from_packed(packed: np.ndarray, offsets: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(codes 1..4 of all read symbols concatenated, offsets) from the packed
    input format; read j is codes[offsets[j]-offsets[0] : offsets[j+1]-offsets[0]]."""
    offsets = np.asarray(offsets, dtype=np.uint64)
    nsym = int(offsets[-1]) if len(offsets) else 0
    codes = unpack_2bit(packed, nsym).astype(np.uint8) + 1
    base = int(offsets[0]) if len(offsets) else 0
    return codes[base:nsym], (offsets - np.uint64(base)).astype(np.uint64)


def strings_to_codes(reads: Sequence[str]) -> tuple[np.ndarray, np.ndarray]:
    """ASCII reads over ACGT -> (codes 1..4 concatenated, offsets[m+1])."""
    joined = "".join(reads).encode("ascii")
    codes = _CODE_OF_ASCII[np.frombuffer(joined, dtype=np.uint8)] if joined else np.zeros(0, np.uint8)
    if codes.size and (codes.min() < 1 or codes.max() > 4):
        raise ValueError("reads must use only A, C, G, T")
    offsets = np.zeros(len(reads) + 1, dtype=np.uint64)
    if reads:
        offsets[1:] = np.cumsum([len(r) for r in reads], dtype=np.uint64)
    return codes.astype(np.uint8), offsets


def concat_text(codes: np.ndarray, offsets: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """T = S_0 $ S_1 $ ... S_{m-1} $ (codes, terminator 0) and soff, the start
    of every string in T (exclusive prefix sum of |S_j|+1), soff[m] = len(T)."""
    offsets = np.asarray(offsets, dtype=np.uint64)
    m = len(offsets) - 1
    lens = (offsets[1:] - offsets[:-1]).astype(np.int64)
    n = int(lens.sum()) + m
    T = np.zeros(n, dtype=np.uint8)
    soff = np.zeros(m + 1, dtype=np.uint64)
    if m:
        soff[1:] = np.cumsum(lens + 1).astype(np.uint64)
        # every non-terminator position of T, in order, takes the next code
        is_sym = np.ones(n, dtype=bool)
        is_sym[(soff[1:] - 1).astype(np.int64)] = False
        T[is_sym] = codes[:int(offsets[-1]) - int(offsets[0])]
    return T, soff


# --------------------------------------------------------------------------
# The definition: suffix array and BWT of the whole set
# --------------------------------------------------------------------------

def suffix_array(T: np.ndarray, threads: int = 1) -> np.ndarray:
    """SA of T (terminators 0, T[-1] == 0) by comparison sort; with threads >
    1, sorted runs merged pairwise (the same order)."""
    T = np.ascontiguousarray(T, dtype=np.uint8)
    n = len(T)
    sa = np.empty(n, dtype=np.uint64)
    if n:
        if threads > 1:
            if _load().oracle_sa_threads(_p8(T), n, _p64(sa), int(threads)) != 0:
                raise MemoryError("oracle_sa_threads")
        else:
            _load().oracle_sa(_p8(T), n, _p64(sa))
    return sa


def bwt_from_text(T: np.ndarray, sa: np.ndarray | None = None, threads: int = 1) -> bytes:
    """Eq. 1 over T, every terminator printed '$'."""
    T = np.ascontiguousarray(T, dtype=np.uint8)
    n = len(T)
    if n == 0:
        return b""
    if sa is None:
        sa = suffix_array(T, threads)
    sa = np.ascontiguousarray(sa, dtype=np.uint64)
    B = np.empty(n, dtype=np.uint8)
    _load().oracle_bwt(_p8(T), n, _p64(sa), _p8(B))
    return B.tobytes()


def bwt_of_codes(codes: np.ndarray, offsets: np.ndarray, threads: int = 1) -> bytes:
    T, _ = concat_text(codes, offsets)
    return bwt_from_text(T, threads=threads)


def bwt(reads: Sequence[str]) -> bytes:
    """BWT of a string set given as ASCII strings over ACGT (Section 2)."""
    codes, offsets = strings_to_codes(reads)
    return bwt_of_codes(codes, offsets)


def rank(B: bytes, c: str, k: int) -> int:
    """Eq. 2: number of occurrences of c in B[0..k)."""
    return B[:k].count(c.encode("ascii"))


def count_smaller(T: np.ndarray, p: int) -> int:
    """Number of suffixes of T smaller than T^p (one SA row, by brute force)."""
    T = np.ascontiguousarray(T, dtype=np.uint8)
    return int(_load().oracle_count_smaller(_p8(T), len(T), int(p)))


def lf_invert(B: bytes, rows: Iterable[int], max_len: int) -> list:
    """For each row r, walk B backwards by LF from r until a '$'; returns the
    spelled strings reversed back into reading order (None for a walk that
    fails: runs past max_len symbols or meets a byte outside $ACGT)."""
    rows = np.ascontiguousarray(list(rows), dtype=np.uint64)
    nr = len(rows)
    Bn = np.frombuffer(B, dtype=np.uint8).copy()
    out_off = np.arange(nr + 1, dtype=np.uint64) * np.uint64(max_len)
    out = np.zeros(max(1, nr * max_len), dtype=np.uint8)
    lens = np.zeros(max(1, nr), dtype=np.uint64)
    if nr:
        rc = _load().oracle_lf_invert(_p8(Bn), len(Bn), _p64(rows), nr, _p64(out_off),
                                      _p8(out), _p64(lens))
        if rc != 0:
            raise MemoryError("oracle_lf_invert")
    res = []
    for t in range(nr):
        L = int(lens[t])
        if L == 2**64 - 1:
            res.append(None)
        else:
            s = out[t * max_len:t * max_len + L].tobytes()[::-1]
            res.append(s.decode("ascii"))
    return res


# --------------------------------------------------------------------------
# set-bwte step by step (Algorithm 1)
# --------------------------------------------------------------------------

def split_blocks(offsets: np.ndarray, M: int) -> list:
    """Greedy partition into blocks of whole strings of at most M suffixes
    (|S_j|+1 per string); a string with more than M suffixes is a block by
    itself.  Returns a list of (j_begin, j_end)."""
    offsets = np.asarray(offsets, dtype=np.uint64)
    m = len(offsets) - 1
    blocks = []
    j = 0
    while j < m:
        k = j
        total = 0
        while k < m:
            s = int(offsets[k + 1] - offsets[k]) + 1
            if k > j and total + s > M:
                break
            total += s
            k += 1
        blocks.append((j, k))
        j = k
    return blocks


def construct_sa(block_codes: np.ndarray, block_offsets: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """ConstructSA (Section 3): the suffix array of the block text
    P_0 $_0 ... P_{mb-1} $_{mb-1} with block-local terminators in string order.
    Returns (SA_int, block text)."""
    T, _ = concat_text(block_codes, block_offsets)
    return suffix_array(T), T


def b_int(T_block: np.ndarray, sa_int: np.ndarray) -> bytes:
    """B_int: the symbol preceding each sorted block suffix; '$' when the suffix
    starts a string (the preceding symbol is some terminator)."""
    T = np.asarray(T_block, dtype=np.uint8)
    sa = np.asarray(sa_int, dtype=np.int64)
    prev = np.where(sa == 0, 0, T[np.maximum(sa - 1, 0)])
    return ASCII[prev].tobytes()


def compute_ranks(T_old: np.ndarray, T_block: np.ndarray, threads: int = 1) -> np.ndarray:
    """What ComputeRanks returns (Section 4, the quantity Lemma 1 computes):
    g[p] for every block position p = the number of suffixes of the old strings
    that are smaller than the block suffix at p.

    Taken from its definition: the old text T_old (every string already in the
    index, terminators 0) and the block text are laid end to end, so the block's
    terminators come after the old ones (strings added later get larger
    terminators), and one suffix array of the whole is sorted.  A suffix that
    starts in the old text ends at its own terminator, so it compares with a
    block suffix exactly as in the set's text.  g of a block suffix is then the
    number of old suffixes that precede it in that order."""
    T_old = np.ascontiguousarray(T_old, dtype=np.uint8)
    T_block = np.ascontiguousarray(T_block, dtype=np.uint8)
    n_old = len(T_old)
    G = np.concatenate([T_old, T_block])
    sa = suffix_array(G, threads).astype(np.int64)
    is_old = sa < n_old
    old_before = np.cumsum(is_old, dtype=np.int64) - is_old
    g = np.zeros(len(T_block), dtype=np.uint64)
    new_rows = ~is_old
    g[sa[new_rows] - n_old] = old_before[new_rows].astype(np.uint64)
    return g


def count_old_smaller(G: np.ndarray, n_old: int, p: int) -> int:
    """Brute-force value of g: old suffixes (the first n_old positions of the
    global text G) smaller than the suffix of G starting at p."""
    G = np.ascontiguousarray(G, dtype=np.uint8)
    return int(_load().oracle_count_old_smaller(_p8(G), int(n_old), int(p)))


def reorder(g: np.ndarray, sa_int: np.ndarray) -> np.ndarray:
    """g_sa[i] = g[SA_int[i]] (Algorithm 1)."""
    return np.asarray(g, dtype=np.uint64)[np.asarray(sa_int, dtype=np.int64)]


def insert(B_ext: bytes, B_int: bytes, g_sa: np.ndarray) -> bytes:
    """Insert (Section 5): B_int[i] goes in front of old row g_sa[i]; new
    symbols with the same g_sa keep their B_int order (numpy.insert does
    exactly this for a non-decreasing index list)."""
    old = np.frombuffer(B_ext, dtype=np.uint8)
    new = np.frombuffer(B_int, dtype=np.uint8)
    idx = np.asarray(g_sa, dtype=np.int64)
    return np.insert(old, idx, new).tobytes()


def set_bwte(codes: np.ndarray, offsets: np.ndarray, M: int,
             prior: tuple | None = None, trace: list | None = None) -> bytes:
    """Algorithm 1 over the strings (codes 1..4, offsets).  prior = (B_ext,
    T_old): the index built so far and the text of the strings in it (for the
    definition of g); None for an empty index.  When `trace` is a list, each
    block appends a dict of its intermediates."""
    offsets = np.asarray(offsets, dtype=np.uint64)
    base = int(offsets[0]) if len(offsets) else 0
    if prior is None:
        B_ext, T_old = b"", np.zeros(0, dtype=np.uint8)
    else:
        B_ext, T_old = prior
    for (j0, j1) in split_blocks(offsets, M):
        bo = offsets[j0:j1 + 1] - offsets[j0]
        bc = codes[int(offsets[j0]) - base:int(offsets[j1]) - base]
        sa_int, T_blk = construct_sa(bc, bo)
        bint = b_int(T_blk, sa_int)
        g = compute_ranks(T_old, T_blk)
        g_sa = reorder(g, sa_int)
        if trace is not None:
            trace.append(dict(block=(j0, j1), sa_int=sa_int, b_int=bint, g=g,
                              g_sa=g_sa, B_ext_before=B_ext))
        B_ext = insert(B_ext, bint, g_sa)
        T_old = np.concatenate([T_old, T_blk])
    return B_ext


def bwt_rank_all(B: bytes, c: str) -> np.ndarray:
    """rank(c, k, B) for every k in [0, n] (naive prefix counting)."""
    Bn = np.frombuffer(B, dtype=np.uint8)
    hits = (Bn == ord(c)).astype(np.uint64)
    out = np.zeros(len(Bn) + 1, dtype=np.uint64)
    out[1:] = np.cumsum(hits)
    return out


# --------------------------------------------------------------------------
# FM-index queries (the BWT and its rank function form an FM-index; Eq. 2)
# --------------------------------------------------------------------------

def pattern_rows(T: np.ndarray, pattern: np.ndarray) -> tuple[int, int]:
    """(lo, hi): the rows of the sorted suffixes of T that start with the
    pattern (codes 1..4).  lo = suffixes smaller than the pattern, hi - lo =
    occurrences of the pattern in the strings.  The empty pattern gives all
    rows [0, n)."""
    T = np.ascontiguousarray(T, dtype=np.uint8)
    P = np.ascontiguousarray(pattern, dtype=np.uint8)
    if len(P) == 0:
        return 0, len(T)
    lo = np.zeros(1, dtype=np.uint64)
    cnt = np.zeros(1, dtype=np.uint64)
    Pb = P if len(P) else np.zeros(1, np.uint8)
    _load().oracle_pattern_rows(_p8(T), len(T), _p8(Pb), len(P), _p64(lo), _p64(cnt))
    return int(lo[0]), int(lo[0] + cnt[0])


# --------------------------------------------------------------------------
# Strand variants of the input (Section 2 notes that reversal is possible)
# --------------------------------------------------------------------------

def _strings(codes: np.ndarray, offsets: np.ndarray) -> list:
    offsets = np.asarray(offsets, dtype=np.int64)
    base = int(offsets[0]) if len(offsets) else 0
    return [codes[int(offsets[j]) - base:int(offsets[j + 1]) - base]
            for j in range(len(offsets) - 1)]


def _from_strings(strs: list) -> tuple[np.ndarray, np.ndarray]:
    offsets = np.zeros(len(strs) + 1, dtype=np.uint64)
    if strs:
        offsets[1:] = np.cumsum([len(x) for x in strs], dtype=np.uint64)
    codes = np.concatenate(strs).astype(np.uint8) if strs else np.zeros(0, np.uint8)
    return codes, offsets


def reverse_strings(codes: np.ndarray, offsets: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Every string written backwards, in the same order (codes 1..4)."""
    return _from_strings([x[::-1] for x in _strings(codes, offsets)])


def with_reverse_complements(codes: np.ndarray,
                             offsets: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Every string followed by its reverse complement (A<->T, C<->G, read
    backwards): strings 2j and 2j + 1 come from string j (codes 1..4)."""
    out = []
    for x in _strings(codes, offsets):
        out.append(x)
        out.append((5 - x[::-1]).astype(np.uint8))
    return _from_strings(out)
