"""Parity at the benchmark's full size, in the launch configuration bench.py
times (4,000,000 x 100 bp short reads, block M = 2^26 suffixes, device
inputs).  The oracle cannot sort 404 M suffixes in a test, so it checks what
it can compute one by one, plus properties that hold at any size:

* sampled rows: for a text position p the oracle counts, by brute force, the
  suffixes smaller than T^p; that row of B must hold the symbol before p;
* LF inversion from sampled rows j spells read j (every read is recovered);
* B is a permutation of T (symbol counts) with one '$' per read;
* rank(c, k) at sampled k against direct counting.
"""
import numpy as np
import pytest

from paper_1410_0562_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def built(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0562_amd import bwtset
    print("[scale] generating 4,000,000 x 100 bp", flush=True)
    packed, offs = synth.short_reads()
    dev_reads = torch.from_numpy(packed).cuda()
    dev_offs = torch.from_numpy(offs.view(np.int64)).cuda()
    idx = bwtset.BwtSet(block_size=1 << 26)
    print("[scale] building on the GPU", flush=True)
    idx.append(dev_reads, dev_offs)
    B = idx.export()
    ranks = {}
    rng = np.random.default_rng(7)
    ks = rng.integers(0, len(B) + 1, 6)
    for c in "$ACGT":
        ranks[c] = [(int(k), idx.rank(c, int(k))) for k in ks]
    size = idx.size()
    idx.close()
    del dev_reads, dev_offs
    torch.cuda.empty_cache()
    print("[scale] built %d symbols" % len(B), flush=True)
    return packed, offs, B, ranks, size


def test_counts_and_size(built, oracle_mod):
    packed, offs, B, ranks, size = built
    m = len(offs) - 1
    n = int(offs[-1]) + m
    assert size == (n, m) and len(B) == n
    codes = oracle_mod.unpack_2bit(packed, int(offs[-1]))
    want = np.bincount(codes, minlength=4)
    got = np.bincount(np.frombuffer(B, np.uint8), minlength=256)
    for i, ch in enumerate(b"ACGT"):
        assert got[ch] == want[i]
    assert got[ord("$")] == m


def test_sampled_rank_queries(built):
    packed, offs, B, ranks, size = built
    Bn = np.frombuffer(B, np.uint8)
    for c, pairs in ranks.items():
        for k, r in pairs:
            assert r == int(np.count_nonzero(Bn[:k] == ord(c)))


def test_lf_inversion_sampled_reads(built, oracle_mod):
    packed, offs, B, ranks, size = built
    rng = np.random.default_rng(8)
    m = len(offs) - 1
    rows = np.concatenate([[0, 1, m - 1], rng.integers(0, m, 2000)]).astype(np.int64)
    got = oracle_mod.lf_invert(B, rows, 101)
    codes = oracle_mod.unpack_2bit(packed, int(offs[-1]))
    for j, s in zip(rows, got):
        a, b = int(offs[j]), int(offs[j + 1])
        assert s == "".join("ACGT"[x] for x in codes[a:b]), j


def test_sampled_rows_by_brute_force(built, oracle_mod):
    packed, offs, B, ranks, size = built
    codes, o = oracle_mod.reads_from_packed(packed, offs)
    T, soff = oracle_mod.concat_text(codes, o)
    rng = np.random.default_rng(9)
    # a read start, a terminator, and interior positions
    ps = [0, int(soff[1]) - 1, int(soff[2_000_000]), int(rng.integers(0, len(T)))]
    for p in ps:
        r = oracle_mod.count_smaller(T, p)
        prev = T[p - 1] if p > 0 else 0
        assert B[r] == b"$ACGT"[prev], p
