"""Writes the expected values in tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
It imports only oracle/ (the pure-Python rotation sort and the C oracle, which
must agree before anything is written).
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import brute, oracle  # noqa: E402

# Small string sets chosen so that each exercises one part of the order of
# Section 2 (Eq. 1 and the terminator order $_0 < ... < $_{m-1} < A).
PIN_SETS = [
    ["GATTACA"],                    # one string: the textbook BWT of GATTACA$
    ["ACGT", "ACGT", "ACGT"],       # identical strings: terminator tie-break
    ["GATTACA", "GATTACA"],
    ["GA", "GA"],
    ["T", "A"],                     # terminator rows follow string order
    ["A", "T"],
    ["ACG", "CG", "G", ""],         # an empty string contributes one '$'
    [""],
    ["", ""],
    ["TTAG", "GAT", "ATT", "TAG"],
    ["AAAA", "AAA", "AA", "A"],     # nested prefixes: '$' below every base
    ["CCCC", "C", "CC", "CCC"],
    ["TGCA", "ACGT", "TTTT", "GGGG", "CATG"],
]


def main():
    rows = []
    for reads in PIN_SETS:
        b1 = brute.bwt(reads)
        b2 = oracle.bwt(reads).decode()
        if b1 != b2:
            raise SystemExit("oracles disagree on %r: %s vs %s" % (reads, b1, b2))
        sa = brute.suffix_array(reads)
        rows.append("%s\t%s\t%s" % (",".join(reads) if reads != [""] else "",
                                    b1, " ".join(map(str, sa))))
    with open(os.path.join(HERE, "set_bwt_pins.tsv"), "w") as f:
        f.write("# BWT of small string sets (Section 2: Eq. 1 over T = S_0 $_0 ... S_{m-1} $_{m-1},\n")
        f.write("# $_0 < ... < $_{m-1} < A < C < G < T).  Columns: reads (comma-separated,\n")
        f.write("# an empty field is an empty string), B with every terminator printed '$',\n")
        f.write("# suffix array of T.  Written by tests/golden/make_golden.py from oracle/.\n")
        f.write("# Hand check of two rows, sorted rotations with their last symbol:\n")
        f.write("#   GATTACA: $GATTACA A | A$GATTAC C | ACA$GATT T | ATTACA$G G | CA$GATTA A |\n")
        f.write("#            GATTACA$ $ | TACA$GAT T | TTACA$GA A            -> ACTGA$TA\n")
        f.write("#   T,A:     $0 A $1 T -> T | $1 T $0 A -> A | A $1 T $0 -> $ | T $0 A $1 -> $\n")
        f.write("#                                                           -> TA$$\n")
        for r in rows:
            f.write(r + "\n")

    # one full incremental step of Algorithm 1: B_ext from the first two
    # strings, then the block of the last two
    import numpy as np
    codes, offs = oracle.strings_to_codes(["TTAG", "GAT", "ATT", "TAG"])
    trace = []
    B = oracle.set_bwte(codes, offs, 9, trace=trace)
    assert B.decode() == brute.bwt(["TTAG", "GAT", "ATT", "TAG"])
    t = trace[1]
    assert t["block"] == (2, 4)
    olds = brute.old_smaller(["TTAG", "GAT"], ["ATT", "TAG"])
    assert olds == [int(x) for x in t["g"]], (olds, t["g"])
    with open(os.path.join(HERE, "incremental_step.txt"), "w") as f:
        f.write("# Algorithm 1, one block: B_ext = BWT{TTAG, GAT}; block = {ATT, TAG}.\n")
        f.write("# g (text order of ATT$TAG$) is the number of old suffixes smaller than\n")
        f.write("# each new suffix (Lemma 1), checked against a brute-force count.\n")
        f.write("# Written by tests/golden/make_golden.py from oracle/.\n")
        f.write("B_ext\t%s\n" % t["B_ext_before"].decode())
        f.write("sa_int\t%s\n" % " ".join(map(str, t["sa_int"])))
        f.write("b_int\t%s\n" % t["b_int"].decode())
        f.write("g\t%s\n" % " ".join(map(str, t["g"])))
        f.write("g_sa\t%s\n" % " ".join(map(str, t["g_sa"])))
        f.write("merged\t%s\n" % B.decode())


if __name__ == "__main__":
    main()
