"""Strand variants of an append (bwt_set_append_strands): every read indexed
backwards, or followed by its reverse complement, against the oracle's BWT
of the transformed strings (oracle.reverse_strings and
oracle.with_reverse_complements, pinned by hand in test_oracle.py)."""
import numpy as np
import pytest

from paper_1410_0562_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _want(oracle_mod, parts, mode):
    """Oracle BWT of the transformed strings of several appends, in order."""
    from paper_1410_0562_amd import bwtset
    strs = []
    for packed, offs in parts:
        codes, o = oracle_mod.reads_from_packed(packed, offs)
        if mode == bwtset.BWT_STRAND_REVERSE:
            codes, o = oracle_mod.reverse_strings(codes, o)
        elif mode == bwtset.BWT_STRAND_BOTH:
            codes, o = oracle_mod.with_reverse_complements(codes, o)
        o = np.asarray(o, np.int64)
        strs += [codes[o[j] - o[0]:o[j + 1] - o[0]] for j in range(len(o) - 1)]
    offs = np.zeros(len(strs) + 1, np.uint64)
    offs[1:] = np.cumsum([len(x) for x in strs])
    codes = np.concatenate(strs) if strs else np.zeros(0, np.uint8)
    return oracle_mod.bwt_of_codes(codes, offs)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("where", ["host", "device", "device-offsets-host-reads"])
def test_strands_equal_the_oracle(torch_dev, oracle_mod, mode, where):
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    a = synth.random_reads(91, 1500, 0, 130)          # ragged, empty reads included
    b = synth.random_reads(92, 700, 90, 400)
    # b with its reads starting inside the packed buffer (offsets[0] > 0)
    pb, ob = b
    ob = ob.copy()
    ob[0] += np.uint64(3)
    b = (pb, ob)
    with bwtset.BwtSet(block_size=80_000) as idx:
        for packed, offs in (a, b):
            if where == "host":
                idx.append_strands(packed, offs, mode)
            elif where == "device":
                idx.append_strands(torch.from_numpy(packed).cuda(),
                                   torch.from_numpy(offs.view(np.int64)).cuda(), mode)
            else:
                idx.append_strands(packed, torch.from_numpy(offs.view(np.int64)).cuda(), mode)
        got = idx.export()
        assert idx.size()[1] == (1 if mode == 1 else 2) * (len(a[1]) + len(b[1]) - 2)
    assert got == _want(oracle_mod, [a, b], mode)


def test_both_strands_make_counts_symmetric(torch_dev, oracle_mod):
    """With every read's reverse complement indexed, a pattern and its
    reverse complement occur equally often (FM-index count on the GPU)."""
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    packed, offs = synth.short_reads(m=3000, length=100, ref_len=20_000, seed=93)
    rng = np.random.default_rng(93)
    pats = [rng.integers(0, 4, int(rng.integers(1, 12)), dtype=np.uint8) for _ in range(400)]
    rcs = [(3 - p[::-1]).astype(np.uint8) for p in pats]
    allp = pats + rcs
    codes = np.concatenate(allp)
    po = np.zeros(len(allp) + 1, np.uint64)
    po[1:] = np.cumsum([len(p) for p in allp])
    dp = torch.from_numpy(synth.pack_codes(codes)).cuda()
    do = torch.from_numpy(po.view(np.int64)).cuda()
    lo = torch.empty(len(allp), dtype=torch.int64, device="cuda")
    hi = torch.empty(len(allp), dtype=torch.int64, device="cuda")
    with bwtset.BwtSet(block_size=150_000) as idx:
        idx.append_strands(packed, offs, bwtset.BWT_STRAND_BOTH)
        idx.count_many(dp, do, lo, hi)
        torch.cuda.synchronize()
    occ = (hi - lo).cpu().numpy()
    k = len(pats)
    assert np.array_equal(occ[:k], occ[k:])
    assert (occ[:k] > 0).sum() > 100


def test_strands_reject_bad_input(torch_dev):
    from paper_1410_0562_amd import bwtset
    packed, offs = synth.random_reads(94, 50, 0, 40)
    with bwtset.BwtSet() as idx:
        idx.append(packed, offs)
        before = idx.export()
        with pytest.raises(bwtset.BwtSetError) as e:
            idx.append_strands(packed, offs, 7)
        assert e.value.code == bwtset.BWT_EINVAL
        bad = offs.copy()
        bad[10], bad[11] = bad[11] + np.uint64(5), bad[10]
        import torch
        for o in (bad, torch.from_numpy(bad.view(np.int64)).cuda()):
            with pytest.raises(bwtset.BwtSetError) as e:
                idx.append_strands(packed, o, bwtset.BWT_STRAND_BOTH)
            assert e.value.code == bwtset.BWT_EINVAL
        assert idx.export() == before
