"""Pins of the CPU oracle against what the paper and the mathematics fix.

The oracle (oracle/) is checked here against things other than itself: an
independent pure-Python rotation sort, hand-checkable small cases, a closed
form, invariants that any BWT of a string set satisfies, and brute-force
counts.  None of these tests touch the GPU library.
"""
import itertools
import os
import random

import numpy as np
import pytest

from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_pins():
    rows = []
    with open(os.path.join(GOLDEN, "set_bwt_pins.tsv")) as f:
        for line in f:
            if line.startswith("#") or not line.strip("\n"):
                continue
            reads_s, B, sa = line.rstrip("\n").split("\t")
            reads = reads_s.split(",")
            rows.append((reads, B, [int(x) for x in sa.split()]))
    return rows


def test_textbook_single_string(oracle_mod):
    # Single string: the string-set BWT reduces to the classic BWT of S$.
    assert oracle_mod.bwt(["GATTACA"]) == b"ACTGA$TA"
    assert brute.bwt(["GATTACA"]) == "ACTGA$TA"


@pytest.mark.parametrize("row", _read_pins(), ids=lambda r: ",".join(r[0]) or "empty")
def test_golden_pins(oracle_mod, row):
    reads, B, sa = row
    assert oracle_mod.bwt(reads).decode() == B
    assert brute.bwt(reads) == B
    T, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(reads))
    assert [int(x) for x in oracle_mod.suffix_array(T)] == sa


def _all_sets(alphabet, max_m, max_total):
    for m in range(1, max_m + 1):
        for lens in itertools.product(range(max_total + 1), repeat=m):
            if sum(lens) > max_total:
                continue
            for syms in itertools.product(alphabet, repeat=sum(lens)):
                s = "".join(syms)
                out, p = [], 0
                for L in lens:
                    out.append(s[p:p + L])
                    p += L
                yield out


def test_exhaustive_small_sets_acgt(oracle_mod):
    n = 0
    for reads in _all_sets("ACGT", 3, 3):
        assert oracle_mod.bwt(reads).decode() == brute.bwt(reads), reads
        n += 1
    assert n > 1000


def test_exhaustive_small_sets_binary(oracle_mod):
    # Two letters reach longer strings (more repeats, longer common prefixes).
    for reads in _all_sets("AC", 3, 6):
        assert oracle_mod.bwt(reads).decode() == brute.bwt(reads), reads


def test_random_sets_vs_rotation_sort(oracle_mod):
    rng = random.Random(1410)
    for _ in range(400):
        m = rng.randint(1, 6)
        alpha = rng.choice(["A", "AC", "ACGT", "GT"])
        reads = ["".join(rng.choice(alpha) for _ in range(rng.randint(0, 9))) for _ in range(m)]
        assert oracle_mod.bwt(reads).decode() == brute.bwt(reads), reads


def _single_bwt(s):
    # classic BWT of s$ by sorting rotations of a single string (one terminator)
    t = s + "\0"
    rots = sorted(range(len(t)), key=lambda i: t[i:] + t[:i])
    return "".join("$" if t[i - 1] == "\0" else t[i - 1] for i in rots)


def test_closed_form_identical_strings(oracle_mod):
    # m copies of S: every row of BWT(S$) splits into m adjacent rows, one per
    # copy, all with the same preceding symbol.
    rng = random.Random(7)
    for _ in range(60):
        s = "".join(rng.choice("ACGT") for _ in range(rng.randint(0, 12)))
        m = rng.randint(1, 5)
        expect = "".join(ch * m for ch in _single_bwt(s))
        assert oracle_mod.bwt([s] * m).decode() == expect


def _check_invariants(O, reads, B):
    n = sum(len(r) + 1 for r in reads)
    assert len(B) == n
    # B is a permutation of T with every terminator printed '$'
    for ch in "ACGT":
        assert B.count(ch.encode()) == sum(r.count(ch) for r in reads)
    assert B.count(b"$") == len(reads)
    # rank totals and monotonicity (Eq. 2)
    ranks = {c: O.bwt_rank_all(B, c) for c in "$ACGT"}
    tot = sum(ranks[c] for c in "$ACGT")
    assert np.array_equal(tot, np.arange(n + 1, dtype=np.uint64))
    # LF inversion from row j spells S_j backwards
    maxlen = max([len(r) for r in reads] + [1])
    got = O.lf_invert(B, range(len(reads)), maxlen + 1)
    assert got == list(reads)


def test_invariants_random(oracle_mod):
    rng = random.Random(11)
    for _ in range(60):
        m = rng.randint(1, 40)
        reads = ["".join(rng.choice("ACGT") for _ in range(rng.randint(0, 30))) for _ in range(m)]
        _check_invariants(oracle_mod, reads, oracle_mod.bwt(reads))


def test_invariants_repetitive(oracle_mod):
    # reads cut from one short reference: long shared prefixes and duplicates
    rng = random.Random(12)
    ref = "".join(rng.choice("ACGT") for _ in range(60))
    reads = []
    for _ in range(80):
        a = rng.randint(0, 50)
        reads.append(ref[a:a + rng.randint(0, 10)])
    _check_invariants(oracle_mod, reads, oracle_mod.bwt(reads))


def test_rank_pins(oracle_mod):
    B = oracle_mod.bwt(["TTAG", "GAT", "ATT", "TAG"])
    assert B == b"GTTGTTG$AA$ATT$A$"
    expect = {"$": [0, 0, 1, 4], "A": [0, 0, 2, 4], "C": [0, 0, 0, 0],
              "G": [0, 2, 3, 3], "T": [0, 3, 4, 6]}
    for c, vals in expect.items():
        for k, v in zip([0, 5, 10, 17], vals):
            assert oracle_mod.rank(B, c, k) == v


def test_count_smaller_is_sa_row(oracle_mod):
    rng = random.Random(3)
    reads = ["".join(rng.choice("ACGT") for _ in range(rng.randint(0, 15))) for _ in range(30)]
    T, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(reads))
    sa = oracle_mod.suffix_array(T)
    inv = np.empty_like(sa)
    inv[sa.astype(np.int64)] = np.arange(len(sa), dtype=np.uint64)
    for p in rng.sample(range(len(T)), 40):
        assert oracle_mod.count_smaller(T, p) == int(inv[p])


def _incremental():
    vals = {}
    with open(os.path.join(GOLDEN, "incremental_step.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            k, v = line.rstrip("\n").split("\t")
            vals[k] = v
    return vals


def test_incremental_step_pin(oracle_mod):
    v = _incremental()
    codes, offs = oracle_mod.strings_to_codes(["TTAG", "GAT", "ATT", "TAG"])
    trace = []
    B = oracle_mod.set_bwte(codes, offs, 9, trace=trace)
    t = trace[1]
    assert t["B_ext_before"].decode() == v["B_ext"]
    assert " ".join(map(str, t["sa_int"])) == v["sa_int"]
    assert t["b_int"].decode() == v["b_int"]
    assert " ".join(map(str, t["g"])) == v["g"]
    assert " ".join(map(str, t["g_sa"])) == v["g_sa"]
    assert B.decode() == v["merged"] == brute.bwt(["TTAG", "GAT", "ATT", "TAG"])


def test_compute_ranks_vs_brute_force(oracle_mod):
    # g from its definition (one joint suffix array) against direct counting,
    # two independent ways: the C brute-force row count and the pure-Python
    # rotation sort.
    rng = random.Random(5)
    for _ in range(120):
        old = ["".join(rng.choice("ACG") for _ in range(rng.randint(0, 7))) for _ in range(rng.randint(1, 5))]
        new = ["".join(rng.choice("ACG") for _ in range(rng.randint(0, 7))) for _ in range(rng.randint(1, 4))]
        T_old, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(old))
        bc, bo = oracle_mod.strings_to_codes(new)
        T_blk, soff = oracle_mod.concat_text(bc, bo)
        g = [int(x) for x in oracle_mod.compute_ranks(T_old, T_blk)]
        assert g == brute.old_smaller(old, new), (old, new)
        G, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(old + new))
        n_old = sum(len(s) + 1 for s in old)
        assert g == [oracle_mod.count_old_smaller(G, n_old, n_old + p) for p in range(len(T_blk))]


def _lemma1_ranks(O, B_ext, T_blk, soff, start):
    # Lemma 1 used as a recurrence: if X has rank r among the old suffixes,
    # then cX has rank C[c] + rank(c, r, B_ext).  Every string's terminator
    # suffix is given the rank `start`, and the recurrence is applied from the
    # string's end towards its beginning.
    cnt = {c: B_ext.count(c.encode()) for c in "$ACGT"}
    C, acc = {}, 0
    for c in "$ACGT":
        C[c] = acc
        acc += cnt[c]
    g = [0] * len(T_blk)
    for j in range(len(soff) - 1):
        a, e = int(soff[j]), int(soff[j + 1]) - 1     # e: the terminator
        r = start
        g[e] = r
        for p in range(e - 1, a - 1, -1):
            c = "$ACGT"[int(T_blk[p])]
            r = C[c] + O.rank(B_ext, c, r)
            g[p] = r
    return g


def test_lemma1_matches_definition(oracle_mod):
    # Cross-check: Lemma 1's recurrence from the terminator rank m_ext gives
    # the definition of g on random sets (this is what the GPU walks compute).
    rng = random.Random(55)
    for _ in range(80):
        old = _rand_reads(rng, rng.randint(1, 8), 0, 9, "ACGT")
        new = _rand_reads(rng, rng.randint(1, 6), 0, 9, "ACGT")
        T_old, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(old))
        B_ext = oracle_mod.bwt(old)
        T_blk, soff = oracle_mod.concat_text(*oracle_mod.strings_to_codes(new))
        want = [int(x) for x in oracle_mod.compute_ranks(T_old, T_blk)]
        assert _lemma1_ranks(oracle_mod, B_ext, T_blk, soff, len(old)) == want


def _rand_reads(rng, m, lo, hi, alpha):
    return ["".join(rng.choice(alpha) for _ in range(rng.randint(lo, hi))) for _ in range(m)]


def test_printed_lf_start_is_wrong_reading(oracle_mod):
    # Algorithm 2 as printed starts each walk at i = n_ext; with the terminator
    # order of Section 2 the new terminator beats only the m_ext old ones, so
    # the start must be m_ext.  The planted variant fails the brute force.
    old, new = ["AC"], ["A"]
    B_ext = oracle_mod.bwt(old)
    assert B_ext == b"C$A"
    bc, bo = oracle_mod.strings_to_codes(new)
    T_blk, soff = oracle_mod.concat_text(bc, bo)
    truth = brute.old_smaller(old, new)
    assert truth == [1, 1]
    assert _lemma1_ranks(oracle_mod, B_ext, T_blk, soff, 1) == truth   # m_ext
    assert _lemma1_ranks(oracle_mod, B_ext, T_blk, soff, 3) != truth   # n_ext
    T_old, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(old))
    assert [int(x) for x in oracle_mod.compute_ranks(T_old, T_blk)] == truth


def test_set_bwte_blocking_invariance(oracle_mod):
    # Algorithm 1 gives the BWT of the whole set for any block size.
    rng = random.Random(9)
    for _ in range(150):
        m = rng.randint(1, 14)
        reads = ["".join(rng.choice("ACGT") for _ in range(rng.randint(0, 8))) for _ in range(m)]
        codes, offs = oracle_mod.strings_to_codes(reads)
        want = oracle_mod.bwt(reads)
        for M in (1, 3, rng.randint(2, 40), 10_000):
            assert oracle_mod.set_bwte(codes, offs, M) == want


def test_append_split_invariance(oracle_mod):
    # Appending in several calls equals one call on the concatenation.
    rng = random.Random(10)
    for _ in range(60):
        m = rng.randint(2, 12)
        reads = ["".join(rng.choice("ACGT") for _ in range(rng.randint(0, 8))) for _ in range(m)]
        cut = rng.randint(1, m - 1)
        prior = None
        for part in (reads[:cut], reads[cut:]):
            c, o = oracle_mod.strings_to_codes(part)
            B = oracle_mod.set_bwte(c, o, rng.randint(1, 30), prior=prior)
            T_part, _ = oracle_mod.concat_text(c, o)
            prior = (B, T_part if prior is None else np.concatenate([prior[1], T_part]))
        assert B == oracle_mod.bwt(reads)


def test_split_blocks_rule(oracle_mod):
    offs = np.array([0, 3, 6, 6, 20, 21], dtype=np.uint64)   # lens 3,3,0,14,1
    # suffixes per string: 4,4,1,15,2
    assert oracle_mod.split_blocks(offs, 8) == [(0, 2), (2, 3), (3, 4), (4, 5)]
    assert oracle_mod.split_blocks(offs, 9) == [(0, 3), (3, 4), (4, 5)]
    assert oracle_mod.split_blocks(offs, 100) == [(0, 5)]


def test_unpack_literal_bytes(oracle_mod):
    # The input layout written out by hand: code = index in "ACGT", symbol s
    # in byte s >> 2 at bits 2(s & 3), lowest bits first.  "ACGT" is
    # 00 01 10 11 read from bit 0 up, i.e. 0b11100100 = 0xE4; "TTGA" is
    # 11 11 10 00 from bit 0 up = 0b00101111 = 0x2F.
    assert list(oracle_mod.unpack_2bit(np.array([0xE4], np.uint8), 4)) == [0, 1, 2, 3]
    assert list(oracle_mod.unpack_2bit(np.array([0x2F], np.uint8), 4)) == [3, 3, 2, 0]
    assert list(oracle_mod.unpack_2bit(np.array([0xE4, 0x03], np.uint8), 5)) == [0, 1, 2, 3, 3]
    codes, offs = oracle_mod.reads_from_packed(np.array([0xE4, 0x2F], np.uint8),
                                                np.array([0, 4, 8], np.uint64))
    assert list(codes) == [1, 2, 3, 4, 4, 4, 3, 1]
    # the BWT of "ACGT" from the literal byte, rotations written out by hand:
    # $ACGT T | ACGT$ $ | CGT$A A | GT$AC C | T$ACG G  -> T$ACG
    c1, o1 = oracle_mod.reads_from_packed(np.array([0xE4], np.uint8), np.array([0, 4], np.uint64))
    assert oracle_mod.bwt_of_codes(c1, o1) == b"T$ACG"


def test_pack_literal_bytes():
    from paper_1410_0562_amd import synth
    assert list(synth.pack_codes(np.array([0, 1, 2, 3], np.uint8))) == [0xE4]
    assert list(synth.pack_codes(np.array([3, 3, 2, 0, 3], np.uint8))) == [0x2F, 0x03]
    p, o = synth.strings_to_input(["ACGT", "TTGA"])
    assert list(p) == [0xE4, 0x2F] and list(o) == [0, 4, 8]


def test_threaded_sort_is_the_same_order(oracle_mod):
    # Sorted runs merged pairwise give the single-threaded comparison sort,
    # for run counts that do and do not divide the input evenly.
    rng = random.Random(21)
    for trial in range(12):
        reads = _rand_reads(rng, rng.randint(1, 300), 0, rng.choice([5, 30, 120]),
                            rng.choice(["ACGT", "AC", "A"]))
        T, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(reads))
        want = oracle_mod.suffix_array(T)
        for th in (2, 3, 5, 8):
            assert np.array_equal(oracle_mod.suffix_array(T, threads=th), want), (trial, th)
    T, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(["GATTACA"]))
    assert [int(x) for x in oracle_mod.suffix_array(T, threads=3)] == [7, 6, 4, 1, 5, 0, 3, 2]


def test_unpack_roundtrip(oracle_mod):
    from paper_1410_0562_amd import synth
    reads = ["ACGTTGCA", "", "G", "TTTTA"]
    packed, offs = synth.strings_to_input(reads)
    codes, o2 = oracle_mod.reads_from_packed(packed, offs)
    c2, o3 = oracle_mod.strings_to_codes(reads)
    assert np.array_equal(codes, c2) and np.array_equal(o2, o3)


# ---- FM-index rows of a pattern (count queries) ---------------------------

def _rows(oracle_mod, reads, pattern):
    T, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(reads))
    P = oracle_mod.strings_to_codes([pattern])[0] if pattern else np.zeros(0, np.uint8)
    return oracle_mod.pattern_rows(T, P)


def test_pattern_rows_vs_brute_force(oracle_mod):
    rng = random.Random(562)
    for _ in range(300):
        m = rng.randint(1, 5)
        alpha = rng.choice(["AC", "ACGT", "GT"])
        reads = ["".join(rng.choice(alpha) for _ in range(rng.randint(0, 9))) for _ in range(m)]
        for _ in range(4):
            P = "".join(rng.choice("ACGT") for _ in range(rng.randint(0, 4)))
            lo, hi = _rows(oracle_mod, reads, P)
            assert hi - lo == brute.occurrences(reads, P), (reads, P)
            assert lo == brute.rows_below(reads, P), (reads, P)


def test_pattern_rows_are_the_sa_rows_with_that_prefix(oracle_mod):
    reads = ["ACGTTACG", "CGTA", "", "TTAC", "ACG"]
    T, _ = oracle_mod.concat_text(*oracle_mod.strings_to_codes(reads))
    sa = oracle_mod.suffix_array(T).astype(np.int64)
    for P in ["A", "AC", "ACG", "CG", "T", "TA", "GTT", "CCC"]:
        lo, hi = _rows(oracle_mod, reads, P)
        Pc = [" ACGT".index(ch) for ch in P]
        pref = [list(T[p:p + len(P)]) == Pc for p in sa]
        assert [i for i, x in enumerate(pref) if x] == list(range(lo, hi)), P


def test_pattern_rows_closed_form(oracle_mod):
    # m copies of ACGT: rows are $ (m), ACGT$ (m), CGT$ (m), GT$ (m), T$ (m)
    m = 7
    reads = ["ACGT"] * m
    assert _rows(oracle_mod, reads, "") == (0, 5 * m)
    assert _rows(oracle_mod, reads, "A") == (m, 2 * m)
    assert _rows(oracle_mod, reads, "CG") == (2 * m, 3 * m)
    assert _rows(oracle_mod, reads, "GT") == (3 * m, 4 * m)
    assert _rows(oracle_mod, reads, "TA") == (5 * m, 5 * m)
    assert _rows(oracle_mod, reads, "AA") == (m, m)


# ---- strand variants ------------------------------------------------------

def test_reverse_and_reverse_complement_by_hand(oracle_mod):
    codes, offs = oracle_mod.strings_to_codes(["ACG", "", "TTA"])
    rc, ro = oracle_mod.reverse_strings(codes, offs)
    assert list(ro) == [0, 3, 3, 6] and "".join(" ACGT"[c] for c in rc) == "GCAATT"
    wc, wo = oracle_mod.with_reverse_complements(codes, offs)
    assert list(wo) == [0, 3, 6, 6, 6, 9, 12]
    assert "".join(" ACGT"[c] for c in wc) == "ACGCGTTTATAA"
    assert brute.reverse_complement("ACGTT") == "AACGT"
    # AC with its reverse complement GT: T = A C $0 G T $1, sorted suffixes
    # $0 $1 AC$0 C$0 GT$1 T$1, preceded by C T $ A $ G
    wc, wo = oracle_mod.with_reverse_complements(*oracle_mod.strings_to_codes(["AC"]))
    assert oracle_mod.bwt_of_codes(wc, wo) == b"CT$A$G" == brute.bwt(["AC", "GT"]).encode()


def test_reverse_complement_set_is_strand_symmetric(oracle_mod):
    # with every string's reverse complement in the set, every pattern occurs
    # as often as its reverse complement
    rng = random.Random(1014)
    reads = ["".join(rng.choice("ACGT") for _ in range(rng.randint(0, 12))) for _ in range(6)]
    codes, offs = oracle_mod.strings_to_codes(reads)
    wc, wo = oracle_mod.with_reverse_complements(codes, offs)
    T, _ = oracle_mod.concat_text(wc, wo)
    for _ in range(60):
        P = "".join(rng.choice("ACGT") for _ in range(rng.randint(1, 4)))
        a = oracle_mod.pattern_rows(T, oracle_mod.strings_to_codes([P])[0])
        b = oracle_mod.pattern_rows(T, oracle_mod.strings_to_codes([brute.reverse_complement(P)])[0])
        assert a[1] - a[0] == b[1] - b[0], P
    rs = [brute.reverse_complement(r) for r in reads]
    both = [x for pair in zip(reads, rs) for x in pair]
    assert oracle_mod.bwt_of_codes(wc, wo).decode() == brute.bwt(both)
