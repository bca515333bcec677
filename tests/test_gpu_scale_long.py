"""Parity at the long-read workload's full size: 250,000 reads, lognormal
lengths (mean 5 kbp, 1-50 kbp), ~1.25 Gbp from a 100 Mbp reference with 10%
noise, block M = 2^27 suffixes.  Checked as in test_gpu_scale.py: sampled rows
against the oracle's brute-force row count, LF inversion of sampled reads,
symbol counts, and sampled rank queries."""
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
    print("[long] generating 250,000 long reads", flush=True)
    packed, offs = synth.long_reads(threads=16)
    dev_reads = torch.from_numpy(packed).cuda()
    dev_offs = torch.from_numpy(offs.view(np.int64)).cuda()
    idx = bwtset.BwtSet(block_size=1 << 27)
    idx.enable_timing(True)
    print("[long] building on the GPU (%d bases)" % int(offs[-1]), flush=True)
    idx.append(dev_reads, dev_offs)
    st = idx.stats()
    print("[long] stats %s" % {k: st[k] for k in ("blocks", "tied_suffixes", "fallback_blocks",
                                                  "ranks_kernel_ms", "sort_pass_ms",
                                                  "refine_ms")}, flush=True)
    B = idx.export()
    rng = np.random.default_rng(17)
    ks = rng.integers(0, len(B) + 1, 4)
    ranks = {c: [(int(k), idx.rank(c, int(k))) for k in ks] for c in "$ACGT"}
    size = idx.size()
    idx.close()
    del dev_reads, dev_offs
    torch.cuda.empty_cache()
    print("[long] built %d symbols" % len(B), flush=True)
    return packed, offs, B, ranks, size


def test_long_counts_and_size(built, oracle_mod):
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


def test_long_sampled_rank_queries(built):
    packed, offs, B, ranks, size = built
    Bn = np.frombuffer(B, np.uint8)
    for c, pairs in ranks.items():
        for k, r in pairs:
            assert r == int(np.count_nonzero(Bn[:k] == ord(c)))


def test_long_lf_inversion_sampled_reads(built, oracle_mod):
    packed, offs, B, ranks, size = built
    rng = np.random.default_rng(18)
    m = len(offs) - 1
    rows = np.concatenate([[0, m - 1], rng.integers(0, m, 150)]).astype(np.int64)
    maxlen = int(np.max(np.diff(offs.astype(np.int64)))) + 1
    got = oracle_mod.lf_invert(B, rows, maxlen)
    codes = oracle_mod.unpack_2bit(packed, int(offs[-1]))
    for j, s in zip(rows, got):
        a, b = int(offs[j]), int(offs[j + 1])
        assert s == "".join("ACGT"[x] for x in codes[a:b]), j


def test_long_sampled_rows_by_brute_force(built, oracle_mod):
    packed, offs, B, ranks, size = built
    codes, o = oracle_mod.reads_from_packed(packed, offs)
    T, soff = oracle_mod.concat_text(codes, o)
    rng = np.random.default_rng(19)
    ps = [int(soff[123_456]), int(rng.integers(0, len(T)))]
    for p in ps:
        r = oracle_mod.count_smaller(T, p)
        prev = T[p - 1] if p > 0 else 0
        assert B[r] == b"$ACGT"[prev], p
