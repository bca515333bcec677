"""Batched form: many independent sets appended by one call.  Every set's
index must equal the oracle BWT of its reads (after whatever it held), and be
the same bytes as one plain append per set, whatever the mix of set sizes,
blocks per set, host or device inputs, and sets left out (m = 0)."""
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


def _set(seed, m, lo=36, hi=250, ref_len=20_000):
    """m reads sampled from a small random reference (so suffixes tie deep
    into the reads), uniform lengths in [lo, hi]."""
    rng = np.random.default_rng(seed)
    ref = rng.integers(0, 4, ref_len, dtype=np.uint8)
    lens = rng.integers(lo, hi + 1, m)
    offs = np.zeros(m + 1, np.uint64)
    offs[1:] = np.cumsum(lens)
    parts = []
    for L in lens:
        a = int(rng.integers(0, ref_len - L + 1))
        c = ref[a:a + L].copy()
        if rng.random() < 0.5:
            c = (3 - c)[::-1]
        hit = rng.random(L) < 0.01
        c[hit] = (c[hit] + 1) & 3
        parts.append(c)
    codes = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return synth.pack_codes(codes), offs


def _oracle(oracle_mod, parts):
    codes, offs = [], [np.zeros(1, np.uint64)]
    base = 0
    for p, o in parts:
        c, oo = oracle_mod.reads_from_packed(p, o)
        codes.append(c)
        offs.append(oo[1:] + np.uint64(base))
        base += int(oo[-1])
    allc = np.concatenate(codes) if codes else np.zeros(0, np.uint8)
    return oracle_mod.bwt_of_codes(allc, np.concatenate(offs))


def _dev(torch, p, o):
    return (torch.from_numpy(p).cuda(), torch.from_numpy(o.astype(np.int64)).cuda())


def test_batch_equals_oracle_and_plain(torch_dev, oracle_mod):
    from paper_1410_0562_amd import bwtset
    sizes = [1, 3, 40, 200, 700, 1500, 5, 0, 2600, 90]
    data = [_set(100 + k, m) for k, m in enumerate(sizes)]
    hs = [bwtset.BwtSet(block_size=1 << 16) for _ in sizes]
    try:
        reads = [torch_dev.from_numpy(p).cuda() if k % 2 == 0 else p
                 for k, (p, _) in enumerate(data)]
        offs = [torch_dev.from_numpy(o.astype(np.int64)).cuda() if k % 3 != 1 else o
                for k, (_, o) in enumerate(data)]
        bwtset.append_many(hs, reads, offs)
        for k, (p, o) in enumerate(data):
            want = _oracle(oracle_mod, [(p, o)]) if sizes[k] else b""
            got = hs[k].export()
            assert got == want, (k, sizes[k])
            with bwtset.BwtSet(block_size=1 << 16) as one:
                one.append(p, o)
                assert one.export() == got
            assert hs[k].size() == (len(want), sizes[k])
    finally:
        for h in hs:
            h.close()


def test_batch_on_top_of_existing_indices_multi_block(torch_dev, oracle_mod):
    """Sets that already hold reads, sets cut into several blocks (small M),
    a read longer than M, empty reads, and two batches in a row."""
    from paper_1410_0562_amd import bwtset
    first = [_set(200 + k, m) for k, m in enumerate([300, 0, 50, 1200, 10])]
    second = [_set(300 + k, m) for k, m in enumerate([2000, 400, 0, 900, 3])]
    # a set with empty reads and one read longer than the block size
    p, o = synth.strings_to_input(["", "ACGT" * 1100, "", "GATTACA", "T" * 40])
    second[4] = (p, o)
    hs = [bwtset.BwtSet(block_size=1 << 12) for _ in first]
    try:
        for k, (p, o) in enumerate(first):
            if len(o) > 1:
                hs[k].append(p, o)
        bwtset.append_many(hs, [p for p, _ in second], [o for _, o in second])
        for k in range(len(hs)):
            parts = [x for x in (first[k], second[k]) if len(x[1]) > 1]
            assert hs[k].export() == _oracle(oracle_mod, parts), k
        third = [_set(400 + k, 150) for k in range(len(hs))]
        bwtset.append_many(hs, [_dev(torch_dev, *x)[0] for x in third],
                           [_dev(torch_dev, *x)[1] for x in third])
        for k in range(len(hs)):
            parts = [x for x in (first[k], second[k], third[k]) if len(x[1]) > 1]
            want = _oracle(oracle_mod, parts)
            assert hs[k].export() == want, k
            for c in "$ACGT":
                kk = len(want) // 3
                assert hs[k].rank(c, kk) == oracle_mod.rank(want, c, kk)
    finally:
        for h in hs:
            h.close()


def test_batch_errors_leave_every_index_unchanged(torch_dev):
    from paper_1410_0562_amd import bwtset
    data = [_set(500 + k, 100) for k in range(3)]
    hs = [bwtset.BwtSet() for _ in range(3)]
    try:
        for h, (p, o) in zip(hs, data):
            h.append(p, o)
        before = [h.export() for h in hs]
        bad = data[1][1].copy()
        bad[5], bad[6] = bad[6], bad[5]          # decreasing offsets
        with pytest.raises(bwtset.BwtSetError):
            bwtset.append_many(hs, [p for p, _ in data], [data[0][1], bad, data[2][1]])
        badd = torch_dev.from_numpy(bad.astype(np.int64)).cuda()
        with pytest.raises(bwtset.BwtSetError):
            bwtset.append_many(hs, [p for p, _ in data], [data[0][1], badd, data[2][1]])
        with pytest.raises(bwtset.BwtSetError):  # the same handle twice
            bwtset.append_many([hs[0], hs[0]], [data[0][0]] * 2, [data[0][1]] * 2)
        assert [h.export() for h in hs] == before
        bwtset.append_many([], [], [])
    finally:
        for h in hs:
            h.close()


def test_batch_workload_generator_small(torch_dev, oracle_mod):
    """The device generator of the batched workload at a small size, through
    the batch, against the oracle per set."""
    from paper_1410_0562_amd import bwtset
    sets = synth.batch_sets_gpu(count=6, ref_len=30_000, min_reads=10, max_reads=3000)
    hs = [bwtset.BwtSet(block_size=1 << 17) for _ in sets]
    try:
        bwtset.append_many(hs, [p for p, _, _ in sets], [o for _, o, _ in sets])
        for h, (p, o, b) in zip(hs, sets):
            hp, ho = p.cpu().numpy(), o.cpu().numpy().astype(np.uint64)
            assert int(ho[-1]) == b
            lens = np.diff(ho.astype(np.int64))
            assert lens.min() >= 36 and lens.max() <= 250
            assert h.export() == _oracle(oracle_mod, [(hp, ho)])
    finally:
        for h in hs:
            h.close()


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_batch_lanes_do_not_change_the_result(torch_dev, oracle_mod, lanes):
    """Blocks of one level run side by side on `lanes` streams; several
    levels (small M, a few large sets) and many blocks per level."""
    from paper_1410_0562_amd import bwtset
    sizes = [900, 30, 2500, 7, 1200, 400, 0, 1800]
    data = [_set(600 + k, m) for k, m in enumerate(sizes)]
    hs = [bwtset.BwtSet(block_size=1 << 15) for _ in sizes]
    try:
        hs[0].set_param(bwtset.BWT_PARAM_BATCH_LANES, lanes)
        hs[0].enable_timing(True)
        bwtset.append_many(hs, [p for p, _ in data], [o for _, o in data])
        st = hs[0].stats()
        assert st["blocks"] > 4 and st["insert_new_symbols"] == sum(
            int(o[-1]) + len(o) - 1 for _, o in data)
        for k, (p, o) in enumerate(data):
            want = _oracle(oracle_mod, [(p, o)]) if sizes[k] else b""
            assert hs[k].export() == want, k
        with pytest.raises(bwtset.BwtSetError):
            hs[0].set_param(bwtset.BWT_PARAM_BATCH_LANES, 5)
    finally:
        for h in hs:
            h.close()
