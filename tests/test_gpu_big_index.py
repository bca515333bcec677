"""An index above 2^32 symbols: the 64-bit superblock counts of the rank
dictionary (rank, ComputeRanks and Insert all add them once a position
reaches 2^32).

The index is m copies of the string ACGT, whose BWT has a closed form: the
BWT of ACGT$ is T$ACG, and each of its symbols repeated m times is the BWT of
the m copies (equal suffixes of different copies are ordered by their
terminators, and the copies' rows of one kind are consecutive).  With
m = 2^32 / 5 + 200,000 it holds 2^32 + 999,999 symbols and is loaded with
bwt_set_import.  A block of random reads is then appended, which ranks and
inserts on both sides of 2^32.  The expected result follows from the oracle
on ONE copy plus the same reads: no new suffix sorts between two old copies
of one kind (that would need a terminator between two old terminators), so
the expected BWT is the oracle's BWT of (ACGT + reads) with each row of the
old copy repeated m times.
"""
import numpy as np
import pytest

from paper_1410_0562_amd import synth

M_COPIES = (1 << 32) // 5 + 200_000
N_OLD = 5 * M_COPIES


def _log(msg):
    print("[big-index] " + msg, flush=True)


def test_closed_form_of_copies(oracle_mod):
    """The closed form the test relies on, checked by the oracle (small m)."""
    for m in (1, 2, 5):
        assert oracle_mod.bwt(["ACGT"] * m) == b"T" * m + b"$" * m + b"A" * m + b"C" * m + b"G" * m


def _closed_rank(c, k):
    seg = "T$ACG".index(c)
    return int(min(max(k - seg * M_COPIES, 0), M_COPIES))


@pytest.mark.gpu
def test_index_above_2_32_symbols(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0562_amd import bwtset
    m = M_COPIES
    _log("building the closed-form BWT of %d copies of ACGT (%d symbols)" % (m, N_OLD))
    B_old = torch.empty(N_OLD, dtype=torch.uint8, device="cuda")
    for k, ch in enumerate(b"T$ACG"):
        B_old[k * m:(k + 1) * m].fill_(ch)
    idx = bwtset.BwtSet()
    try:
        _log("import")
        idx.import_bwt(B_old)
        del B_old
        torch.cuda.empty_cache()
        assert idx.size() == (N_OLD, m)
        ks = [0, 1, m - 1, m, 4 * m, (1 << 32) - 7, (1 << 32) - 1, 1 << 32, (1 << 32) + 1,
              (1 << 32) + 127, (1 << 32) + 128, (1 << 32) + 65_537, N_OLD - 1, N_OLD]
        _log("rank on both sides of 2^32")
        for c in "$ACGT":
            for k in ks:
                assert idx.rank(c, k) == _closed_rank(c, k), (c, k)

        # a block of reads on top: ComputeRanks and Insert above 2^32
        packed, offs = synth.random_reads(4242, 2000, 0, 120)
        codes, o = oracle_mod.reads_from_packed(packed, offs)
        one = np.array([1, 2, 3, 4], dtype=np.uint8)      # ACGT as oracle codes
        allc = np.concatenate([one, codes])
        allo = np.concatenate([np.array([0], np.uint64), o + np.uint64(4)])
        T, _ = oracle_mod.concat_text(allc, allo)
        sa = oracle_mod.suffix_array(T)
        B1 = np.frombuffer(oracle_mod.bwt_from_text(T, sa), dtype=np.uint8)
        reps = np.where(sa.astype(np.int64) < 5, m, 1).astype(np.int64)
        n_new = int(o[-1]) + 2000
        _log("append %d suffixes" % n_new)
        idx.append(packed, offs)
        n, mm = idx.size()
        assert (n, mm) == (N_OLD + n_new, m + 2000)
        # The expected BWT and its ranks are formed on the host: row r of the
        # one-copy BWT stands for reps[r] consecutive rows.
        want = np.repeat(B1, reps)
        assert len(want) == n
        got = torch.empty(n, dtype=torch.uint8, device="cuda")
        _log("export and compare")
        idx.export(got)
        got_h = got.cpu().numpy()
        del got
        torch.cuda.empty_cache()
        CH = 1 << 28
        for a in range(0, n, CH):
            g, w = got_h[a:a + CH], want[a:a + CH]
            if not np.array_equal(g, w):
                bad = (a + np.flatnonzero(g != w)[:5]).tolist()
                raise AssertionError("rows differ from the expected BWT, first at %s" % bad)
        del got_h, want
        # the new rows land at both ends (suffixes before and after the
        # copies' rows), so counts at 2^32 and above include new symbols
        ends = np.cumsum(reps)
        for c in "$ACGT":
            cw = np.cumsum(np.where(B1 == ord(c), reps, 0))
            for k in (1 << 32, (1 << 32) + 12_345, n - 1, n):
                r = int(np.searchsorted(ends, k, side="right"))   # rows wholly before k
                w = int(cw[r - 1]) if r else 0
                if r < len(B1) and B1[r] == ord(c):
                    w += k - (int(ends[r - 1]) if r else 0)
                assert idx.rank(c, k) == w, (c, k)
    finally:
        idx.close()
        torch.cuda.empty_cache()
