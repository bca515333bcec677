"""bwt_set_block_sort_noalloc (ConstructSA and B_int of one block on the
library's fixed per-GPU workspace) against bwt_set_block_sort, the entry
point it is a variant of, and against the oracle.

Two calls in a row share the workspace, the second on a smaller block, so a
count or table the first call left behind would show in the second.  Both are
compared element by element: the suffix array and B_int are integers, so the
bar is bit-exact.
"""
import numpy as np
import pytest

from paper_1410_0562_amd import synth

pytestmark = pytest.mark.gpu

MAX_SUFFIXES = 1 << 18


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _log(msg):
    print("[no-alloc] " + msg, flush=True)


def _dev(torch, packed, offs):
    return (torch.from_numpy(packed).cuda(),
            torch.from_numpy(np.asarray(offs, np.uint64).view(np.int64)).cuda())


def _run(torch, fn, packed, offs):
    n = int(offs[-1]) - int(offs[0]) + len(offs) - 1
    reads, o = _dev(torch, packed, offs)
    sa = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    bint = torch.zeros(n, dtype=torch.uint8, device="cuda")
    fn(reads, o, sa, bint)
    torch.cuda.synchronize()
    return sa.cpu().numpy(), bint.cpu().numpy()


def _repeats(seed):
    """Reads that leave tied groups above the LDS refinement limit (prefix
    doubling) beside ordinary ones."""
    rng = np.random.default_rng(seed)
    ref = rng.integers(0, 4, 2000, dtype=np.uint8)
    reads = [ref[a:a + 900] for a in rng.integers(0, 100, 60)] + [ref[:23]] * 700
    codes = np.concatenate(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    return synth.pack_codes(codes), offs


def test_noalloc_equals_block_sort_on_two_calls(torch_dev, oracle_mod):
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    cases = [
        ("ragged 2400 reads of 0..200 bp", synth.random_reads(71, 2400, 0, 200)),
        ("smaller: 300 reads of 0..90 bp", synth.random_reads(72, 300, 0, 90)),
        ("repeats (doubling fallback)", _repeats(73)),
        ("smaller again: 50 reads at 10x coverage",
         synth.short_reads(m=50, length=100, ref_len=500, seed=74)),
    ]
    with bwtset.BwtSet() as idx, bwtset.BwtSet() as ref_idx:
        mem0 = idx.memory()
        for name, (packed, offs) in cases:
            n = int(offs[-1]) - int(offs[0]) + len(offs) - 1
            assert n <= MAX_SUFFIXES
            _log("%s: %d suffixes" % (name, n))
            sa1, b1 = _run(torch, idx.block_sort_noalloc, packed, offs)
            sa0, b0 = _run(torch, ref_idx.block_sort, packed, offs)
            assert np.array_equal(sa1, sa0), name
            assert np.array_equal(b1, b0), name
            codes, o = oracle_mod.reads_from_packed(packed, offs)
            sa_want, T = oracle_mod.construct_sa(codes, o)
            assert np.array_equal(sa1.astype(np.uint64), sa_want), name
            assert b1.tobytes() == oracle_mod.b_int(T, sa_want), name
        # the handle's own device memory did not grow
        assert idx.memory() == mem0


def test_noalloc_at_the_size_limit_and_offset_reads(torch_dev, oracle_mod):
    """A block of exactly 2^18 suffixes whose reads start inside the packed
    buffer (offsets[0] > 0), then a small one."""
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    packed, offs = synth.random_reads(75, 2600, 100, 100)     # 262,600 suffixes
    j1 = 2600
    # drop reads from the front until the block holds exactly 2^18 suffixes
    j0 = 0
    while int(offs[j1]) - int(offs[j0]) + (j1 - j0) > MAX_SUFFIXES:
        j0 += 1
    sub = offs[j0:j1 + 1]
    extra = MAX_SUFFIXES - (int(sub[-1]) - int(sub[0]) + len(sub) - 1)
    # grow the first read by `extra` symbols (taken from the read before it)
    sub = sub.copy()
    sub[0] -= np.uint64(extra)
    assert int(sub[-1]) - int(sub[0]) + len(sub) - 1 == MAX_SUFFIXES
    with bwtset.BwtSet() as idx, bwtset.BwtSet() as ref_idx:
        for name, (p, o) in [("2^18 suffixes, reads from offset %d" % int(sub[0]), (packed, sub)),
                             ("then 40 reads", synth.random_reads(76, 40, 0, 60))]:
            _log(name)
            sa1, b1 = _run(torch, idx.block_sort_noalloc, p, o)
            sa0, b0 = _run(torch, ref_idx.block_sort, p, o)
            assert np.array_equal(sa1, sa0), name
            assert np.array_equal(b1, b0), name


def test_noalloc_rejects_too_large_and_host_buffers(torch_dev):
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    packed, offs = synth.random_reads(77, 2700, 100, 100)     # 272,700 suffixes
    n = int(offs[-1]) + len(offs) - 1
    assert n > MAX_SUFFIXES
    reads, o = _dev(torch, packed, offs)
    sa = torch.empty(n, dtype=torch.int32, device="cuda")
    bint = torch.empty(n, dtype=torch.uint8, device="cuda")
    with bwtset.BwtSet() as idx:
        _log("over the limit")
        with pytest.raises(bwtset.BwtSetError) as e:
            idx.block_sort_noalloc(reads, o, sa, bint)
        assert e.value.code == bwtset.BWT_EINVAL
        _log("host inputs")
        small_p, small_o = synth.random_reads(78, 10, 0, 20)
        with pytest.raises(bwtset.BwtSetError) as e:
            idx.block_sort_noalloc(small_p, small_o, sa, bint)
        assert e.value.code == bwtset.BWT_EINVAL
        # the handle still works after the refusals
        _log("a valid call after the refusals")
        sa1, b1 = _run(torch, idx.block_sort_noalloc, small_p, small_o)
        sa0, b0 = _run(torch, idx.block_sort, small_p, small_o)
        assert np.array_equal(sa1, sa0) and np.array_equal(b1, b0)
