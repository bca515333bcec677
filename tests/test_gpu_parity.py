"""GPU parity: every step of the HIP path against the CPU oracle, through the
C ABI.  Integer work, so the bar is bit-exact equality everywhere."""
import random

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


@pytest.fixture(scope="module")
def B(torch_dev):
    from paper_1410_0562_amd import bwtset
    return bwtset


def _pins():
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "set_bwt_pins.tsv")) as f:
        for line in f:
            if line.startswith("#") or not line.strip("\n"):
                continue
            reads_s, Bs, _ = line.rstrip("\n").split("\t")
            rows.append((reads_s.split(","), Bs))
    return rows


def _dev(torch, arr, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(arr).view(np.int64) if arr.dtype == np.uint64
                         else np.ascontiguousarray(arr))
    return t.cuda()


def _oracle_inputs(O, packed, offsets):
    codes, offs = O.reads_from_packed(packed, offsets)
    return codes, offs


@pytest.mark.parametrize("row", _pins(), ids=lambda r: ",".join(r[0]) or "empty")
def test_pins_host_inputs(B, oracle_mod, row):
    reads, want = row
    packed, offs = synth.strings_to_input(reads)
    with B.BwtSet() as idx:
        idx.append(packed, offs)
        assert idx.export().decode() == want
        assert idx.size() == (len(want), len(reads))


def test_pins_device_inputs(B, torch_dev, oracle_mod):
    for reads, want in _pins():
        packed, offs = synth.strings_to_input(reads)
        with B.BwtSet() as idx:
            idx.append(_dev(torch_dev, np.concatenate([packed, np.zeros(8, np.uint8)])),
                       _dev(torch_dev, offs))
            assert idx.export().decode() == want, reads


def _random_set(rng, m, lo, hi, alpha="ACGT"):
    return ["".join(rng.choice(alpha) for _ in range(rng.randint(lo, hi))) for _ in range(m)]


def test_random_small_sets(B, oracle_mod):
    rng = random.Random(20)
    for trial in range(40):
        reads = _random_set(rng, rng.randint(1, 60), 0, rng.choice([3, 12, 40]),
                            rng.choice(["ACGT", "AC", "A", "GT"]))
        packed, offs = synth.strings_to_input(reads)
        with B.BwtSet(block_size=rng.randint(1, 200)) as idx:
            idx.append(packed, offs)
            got = idx.export()
        assert got == oracle_mod.bwt(reads), (trial, reads)


def test_uniform_reads_workload(B, oracle_mod):
    # 10,000 reads x 100 bp, block size 262,144 suffixes (4 blocks, ragged last)
    packed, offs = synth.uniform_reads()
    codes, o = _oracle_inputs(oracle_mod, packed, offs)
    want = oracle_mod.bwt_of_codes(codes, o)
    with B.BwtSet(block_size=262_144) as idx:
        idx.enable_timing(True)
        idx.append(packed, offs)
        got = idx.export()
        st = idx.stats()
    assert st["blocks"] == 4
    assert got == want


def test_block_sort_vs_oracle(B, torch_dev, oracle_mod):
    torch = torch_dev
    cases = [
        synth.random_reads(31, 2595, 100, 100),            # one block of the 10k x 100 workload
        synth.random_reads(32, 3000, 0, 300),              # ragged, empty reads included
        synth.random_reads(33, 500, 0, 40, alphabet=2),    # long common prefixes
        synth.short_reads(m=20_000, length=100, ref_len=200_000, seed=34),  # 10x coverage
    ]
    for packed, offs in cases:
        codes, o = _oracle_inputs(oracle_mod, packed, offs)
        sa_want, T = oracle_mod.construct_sa(codes, o)
        bint_want = oracle_mod.b_int(T, sa_want)
        n = len(T)
        sa = torch.empty(n, dtype=torch.int32, device="cuda")
        bint = torch.empty(n, dtype=torch.uint8, device="cuda")
        with B.BwtSet() as idx:
            idx.block_sort(packed, offs, sa, bint)
        assert np.array_equal(sa.cpu().numpy().astype(np.uint64), sa_want)
        assert bint.cpu().numpy().tobytes() == bint_want


def test_block_sort_repeats(B, torch_dev, oracle_mod):
    # identical reads and reads that are shifts of one long string: long LCPs,
    # many prefix-doubling rounds, groups spanning several scan tiles
    torch = torch_dev
    rng = np.random.default_rng(35)
    ref = rng.integers(0, 4, 3000, dtype=np.uint8)
    reads = []
    for k in range(400):
        a = int(rng.integers(0, 200))
        reads.append(ref[a:a + 2500])
    for k in range(5000):
        reads.append(ref[:37])
    codes = np.concatenate(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    packed = synth.pack_codes(codes)
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    sa_want, T = oracle_mod.construct_sa(c1, o1)
    n = len(T)
    sa = torch.empty(n, dtype=torch.int32, device="cuda")
    bint = torch.empty(n, dtype=torch.uint8, device="cuda")
    with B.BwtSet() as idx:
        idx.block_sort(packed, offs, sa, bint)
    assert np.array_equal(sa.cpu().numpy().astype(np.uint64), sa_want)
    assert bint.cpu().numpy().tobytes() == oracle_mod.b_int(T, sa_want)


def _split(packed, offs, j):
    return synth.take_reads(packed, offs, 0, j), synth.take_reads(packed, offs, j, len(offs) - 1)


def test_compute_ranks_vs_oracle(B, torch_dev, oracle_mod):
    torch = torch_dev
    packed, offs = synth.short_reads(m=12_000, length=100, ref_len=300_000, seed=36)
    (pa, oa), (pb, ob) = _split(packed, offs, 9_000)
    ca, oa2 = _oracle_inputs(oracle_mod, pa, oa)
    B_ext = oracle_mod.bwt_of_codes(ca, oa2)
    T_old, _ = oracle_mod.concat_text(ca, oa2)
    cb, ob2 = _oracle_inputs(oracle_mod, pb, ob)
    T, soff = oracle_mod.concat_text(cb, ob2)
    want = oracle_mod.compute_ranks(T_old, T)
    g = torch.empty(len(T), dtype=torch.int64, device="cuda")
    with B.BwtSet() as idx:
        idx.append(pa, oa)
        assert idx.export() == B_ext
        idx.compute_ranks(pb, ob, g)
    assert np.array_equal(g.cpu().numpy().astype(np.uint64), want)


@pytest.mark.parametrize("shift", [3, 16])
def test_compute_ranks_into_an_offset_buffer(B, torch_dev, oracle_mod, shift):
    """The walks write g in whole 128-byte chunks only where the output is
    128-byte aligned, word by word elsewhere: g written into a view that
    starts `shift` words into a buffer (24 bytes: unaligned; 128: aligned) is
    the oracle's, short and segmented reads alike, and the words around the
    view are left as they were."""
    torch = torch_dev
    old = synth.random_reads(71, 600, 50, 3000)
    new = synth.random_reads(72, 400, 0, 2500)
    ca, oa2 = _oracle_inputs(oracle_mod, *old)
    T_old, _ = oracle_mod.concat_text(ca, oa2)
    cb, ob2 = _oracle_inputs(oracle_mod, *new)
    T, _ = oracle_mod.concat_text(cb, ob2)
    want = oracle_mod.compute_ranks(T_old, T)
    guard = -7
    buf = torch.full((len(T) + shift + 40,), guard, dtype=torch.int64, device="cuda")
    g = buf[shift:shift + len(T)]
    with B.BwtSet() as idx:
        idx.set_param(B.BWT_PARAM_RANK_SEGMENT, 512)
        idx.append(*old)
        idx.compute_ranks(*new, g)
    h = buf.cpu().numpy()
    assert np.array_equal(h[shift:shift + len(T)].astype(np.uint64), want)
    assert (h[:shift] == guard).all() and (h[shift + len(T):] == guard).all()


def test_insert_vs_oracle(B, torch_dev, oracle_mod):
    torch = torch_dev
    packed, offs = synth.random_reads(37, 5000, 20, 180)
    (pa, oa), (pb, ob) = _split(packed, offs, 3000)
    ca, oa2 = _oracle_inputs(oracle_mod, pa, oa)
    B_ext = oracle_mod.bwt_of_codes(ca, oa2)
    cb, ob2 = _oracle_inputs(oracle_mod, pb, ob)
    sa_int, T = oracle_mod.construct_sa(cb, ob2)
    bint = oracle_mod.b_int(T, sa_int)
    T_old, _ = oracle_mod.concat_text(ca, oa2)
    g = oracle_mod.compute_ranks(T_old, T)
    gsa = oracle_mod.reorder(g, sa_int)
    want = oracle_mod.insert(B_ext, bint, gsa)
    codes_all, o_all = _oracle_inputs(oracle_mod, packed, offs)
    assert want == oracle_mod.bwt_of_codes(codes_all, o_all)
    with B.BwtSet() as idx:
        idx.append(pa, oa)
        idx.insert(_dev(torch, np.frombuffer(bint, np.uint8).copy()), _dev(torch, gsa))
        assert idx.export() == want
        assert idx.size() == (len(want), 5000)


def test_rank_queries(B, torch_dev, oracle_mod):
    torch = torch_dev
    packed, offs = synth.random_reads(38, 3000, 0, 150)
    codes, o = _oracle_inputs(oracle_mod, packed, offs)
    Bw = oracle_mod.bwt_of_codes(codes, o)
    n = len(Bw)
    rng = np.random.default_rng(39)
    ks = np.concatenate([[0, 1, 127, 128, 129, n - 1, n], rng.integers(0, n + 1, 500)]).astype(np.int64)
    with B.BwtSet() as idx:
        idx.append(packed, offs)
        tables = {c: oracle_mod.bwt_rank_all(Bw, c) for c in "$ACGT"}
        for c in "$ACGT":
            for k in ks[:40]:
                assert idx.rank(c, int(k)) == int(tables[c][k])
        cs = np.array([ord(c) for c in "$ACGT"] * len(ks), np.uint8)
        kk = np.repeat(ks, 5)
        out = torch.empty(len(kk), dtype=torch.int64, device="cuda")
        idx.rank_many(_dev(torch, cs), _dev(torch, kk), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = np.array([tables[chr(c)][k] for c, k in zip(cs, kk)], dtype=np.int64)
        assert np.array_equal(got, want)


def test_blocking_and_append_split_invariance(B, oracle_mod):
    packed, offs = synth.random_reads(40, 4000, 0, 120)
    codes, o = _oracle_inputs(oracle_mod, packed, offs)
    want = oracle_mod.bwt_of_codes(codes, o)
    for M in (1, 97, 4096, 1 << 20):
        with B.BwtSet(block_size=M) as idx:
            idx.append(packed, offs)
            assert idx.export() == want, M
    with B.BwtSet(block_size=5000) as idx:
        for j0, j1 in ((0, 1), (1, 1000), (1000, 1001), (1001, 4000)):
            p, oo = synth.take_reads(packed, offs, j0, j1)
            idx.append(p, oo)
        assert idx.export() == want


def test_long_reads(B, oracle_mod):
    # reads of 5k-60k symbols cut from one reference: long LF walks and long
    # shared prefixes (many doubling rounds)
    rng = np.random.default_rng(41)
    ref = rng.integers(0, 4, 120_000, dtype=np.uint8)
    reads = []
    for _ in range(12):
        a = int(rng.integers(0, 50_000))
        L = int(rng.integers(5_000, 60_000))
        r = ref[a:a + L].copy()
        hit = rng.random(len(r)) < 0.001
        r[hit] = (r[hit] + 1) & 3
        reads.append(r)
    codes = np.concatenate(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    packed = synth.pack_codes(codes)
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    want = oracle_mod.bwt_of_codes(c1, o1)
    with B.BwtSet(block_size=100_000) as idx:
        idx.append(packed, offs)
        assert idx.export() == want


def test_misaligned_device_reads(B, torch_dev, oracle_mod):
    # reads starting at an odd symbol offset inside an unaligned device buffer
    torch = torch_dev
    packed, offs = synth.random_reads(42, 700, 1, 90)
    shift = 5  # symbols
    codes = oracle_mod.unpack_2bit(packed, int(offs[-1]))
    shifted = synth.pack_codes(np.concatenate([np.zeros(shift, np.uint8), codes]))
    offs2 = offs + np.uint64(shift)
    buf = torch.zeros(len(shifted) + 16, dtype=torch.uint8, device="cuda")
    buf[3:3 + len(shifted)] = torch.from_numpy(shifted).cuda()
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    with B.BwtSet(block_size=9999) as idx:
        idx.append(buf[3:], _dev(torch, offs2))
        assert idx.export() == oracle_mod.bwt_of_codes(c1, o1)


def test_errors_leave_index_unchanged(B, torch_dev, oracle_mod):
    torch = torch_dev
    with pytest.raises(B.BwtSetError) as e:
        B.BwtSet("ACGU")
    assert e.value.code == B.BWT_EALPHABET
    packed, offs = synth.random_reads(43, 200, 0, 50)
    with B.BwtSet() as idx:
        idx.append(packed, offs)
        before = idx.export()
        bad = offs.copy()
        bad[5], bad[6] = bad[6] + 3, bad[5]
        with pytest.raises(B.BwtSetError) as e:
            idx.append(packed, bad)
        assert e.value.code == B.BWT_EINVAL
        with pytest.raises(B.BwtSetError):
            idx.append(_dev(torch, packed), _dev(torch, bad))
        n, m = idx.size()
        with pytest.raises(B.BwtSetError):
            idx.rank("A", n + 1)
        with pytest.raises(B.BwtSetError):
            idx.rank("N", 0)
        gsa = np.array([3, 2], np.uint64)
        with pytest.raises(B.BwtSetError):
            idx.insert(_dev(torch, np.frombuffer(b"A$", np.uint8).copy()), _dev(torch, gsa))
        with pytest.raises(B.BwtSetError):
            idx.insert(_dev(torch, np.frombuffer(b"AX", np.uint8).copy()),
                       _dev(torch, np.array([0, 1], np.uint64)))
        assert idx.export() == before
        assert idx.size() == (n, m)
        idx.reset()
        assert idx.size() == (0, 0) and idx.export() == b""
        idx.append(packed, offs)
        assert idx.export() == before


def test_deterministic(B, oracle_mod):
    packed, offs = synth.short_reads(m=30_000, length=100, ref_len=500_000, seed=44)
    outs = []
    for _ in range(2):
        with B.BwtSet(block_size=1 << 20) as idx:
            idx.append(packed, offs)
            outs.append(idx.export())
    assert outs[0] == outs[1]
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    assert outs[0] == oracle_mod.bwt_of_codes(c1, o1)


@pytest.mark.parametrize("copies", [255, 256, 257, 600])
def test_group_size_around_refine_limit(B, torch_dev, oracle_mod, copies):
    # `copies` identical reads give tied groups of exactly that size: up to
    # 256 they are finished in LDS, above that by prefix doubling
    torch = torch_dev
    rng = np.random.default_rng(100 + copies)
    base = rng.integers(0, 4, 80, dtype=np.uint8)
    other = [rng.integers(0, 4, int(rng.integers(0, 120)), dtype=np.uint8) for _ in range(300)]
    reads = [base] * copies + other
    codes = np.concatenate(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    packed = synth.pack_codes(codes)
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    sa_want, T = oracle_mod.construct_sa(c1, o1)
    n = len(T)
    sa = torch.empty(n, dtype=torch.int32, device="cuda")
    bint = torch.empty(n, dtype=torch.uint8, device="cuda")
    with B.BwtSet() as idx:
        idx.block_sort(packed, offs, sa, bint)
        assert np.array_equal(sa.cpu().numpy().astype(np.uint64), sa_want)
        # and through the whole path, split so that later blocks rank against
        # an index that already holds copies of the same read
        idx.set_block_size(9000)
        idx.append(packed, offs)
        assert idx.export() == oracle_mod.bwt_of_codes(c1, o1)


def test_identical_long_reads(B, oracle_mod):
    # three copies of a 6,000-symbol read: the tied group needs ~200 chunk passes
    rng = np.random.default_rng(45)
    r = rng.integers(0, 4, 6000, dtype=np.uint8)
    reads = [r, r[:5000], r, rng.integers(0, 4, 3000, dtype=np.uint8), r]
    codes = np.concatenate(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(x) for x in reads])
    packed = synth.pack_codes(codes)
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    want = oracle_mod.bwt_of_codes(c1, o1)
    for M in (1 << 20, 7000):
        with B.BwtSet(block_size=M) as idx:
            idx.append(packed, offs)
            assert idx.export() == want, M


@pytest.mark.parametrize("key_bits", [16, 24, 40, 48, 56, 64])
@pytest.mark.parametrize("block", [400_000, 1_100_000])
def test_key_width_does_not_change_the_result(B, oracle_mod, key_bits, block):
    # the first sort key holds g and as many symbols as fit; narrower keys
    # leave more ties to the LDS refinement (or, for huge groups, doubling);
    # blocks of 2^20 suffixes and more take the bucket finish
    packed, offs = synth.short_reads(m=30_000, length=100, ref_len=600_000, seed=46)
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    want = oracle_mod.bwt_of_codes(c1, o1)
    with B.BwtSet(block_size=block) as idx:
        idx.set_key_bits(key_bits)
        idx.enable_timing(True)
        idx.append(packed, offs)
        assert idx.export() == want
        st = idx.stats()
    assert st["blocks"] >= 3
    assert (st["bucket_ms"] > 0) == (block >= (1 << 20))


def test_key_width_with_large_groups(B, oracle_mod):
    # many identical reads force the doubling fallback, which widens the key
    rng = np.random.default_rng(47)
    base = rng.integers(0, 4, 60, dtype=np.uint8)
    reads = [base] * 700 + [rng.integers(0, 4, 90, dtype=np.uint8) for _ in range(3000)]
    codes = np.concatenate(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    packed = synth.pack_codes(codes)
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    want = oracle_mod.bwt_of_codes(c1, o1)
    for kb in (16, 40):
        with B.BwtSet(block_size=60_000) as idx:
            idx.set_key_bits(kb)
            idx.enable_timing(True)
            idx.append(packed, offs)
            assert idx.export() == want, kb
            assert idx.stats()["fallback_blocks"] >= 1


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4, 5, 6, 7, 8])
def test_radix_tile_shapes(B, torch_dev, oracle_mod, cfg):
    torch = torch_dev
    packed, offs = synth.random_reads(48, 4000, 0, 160)
    c1, o1 = _oracle_inputs(oracle_mod, packed, offs)
    sa_want, T = oracle_mod.construct_sa(c1, o1)
    n = len(T)
    sa = torch.empty(n, dtype=torch.int32, device="cuda")
    bint = torch.empty(n, dtype=torch.uint8, device="cuda")
    with B.BwtSet() as idx:
        idx.set_param(B.BWT_PARAM_RADIX_TILE, cfg)
        idx.block_sort(packed, offs, sa, bint)
        assert np.array_equal(sa.cpu().numpy().astype(np.uint64), sa_want)
        idx.set_block_size(50_000)
        idx.append(packed, offs)
        assert idx.export() == oracle_mod.bwt_of_codes(c1, o1)


@pytest.mark.parametrize("seg,ov", [(0, 0), (256, 0), (256, 16), (256, 128), (1024, 64)])
def test_segmented_compute_ranks(B, torch_dev, oracle_mod, seg, ov):
    # long reads walked in segments that start with a backward search: exact
    # whether the interval closes within the overlap or the read falls back
    torch = torch_dev
    rng = np.random.default_rng(49)
    ref = rng.integers(0, 4, 40_000, dtype=np.uint8)
    reads = []
    for _ in range(60):
        a = int(rng.integers(0, 30_000))
        r = ref[a:a + int(rng.integers(300, 9000))].copy()
        hit = rng.random(len(r)) < 0.05
        r[hit] = (r[hit] + 1) & 3
        reads.append(r)
    reads += [rng.integers(0, 4, int(rng.integers(0, 400)), dtype=np.uint8) for _ in range(200)]
    codes = np.concatenate(reads)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(x) for x in reads])
    packed = synth.pack_codes(codes)
    (pa, oa), (pb, ob) = _split(packed, offs, 130)
    ca, oa2 = _oracle_inputs(oracle_mod, pa, oa)
    B_ext = oracle_mod.bwt_of_codes(ca, oa2)
    T_old, _ = oracle_mod.concat_text(ca, oa2)
    cb, ob2 = _oracle_inputs(oracle_mod, pb, ob)
    T, soff = oracle_mod.concat_text(cb, ob2)
    want = oracle_mod.compute_ranks(T_old, T)
    g = torch.empty(len(T), dtype=torch.int64, device="cuda")
    with B.BwtSet() as idx:
        idx.set_param(B.BWT_PARAM_RANK_SEGMENT, seg)
        idx.set_param(B.BWT_PARAM_RANK_OVERLAP, ov)
        idx.append(pa, oa)
        idx.compute_ranks(pb, ob, g)
        assert np.array_equal(g.cpu().numpy().astype(np.uint64), want)
        idx.append(pb, ob)
        assert idx.export() == oracle_mod.bwt_of_codes(*_oracle_inputs(oracle_mod, packed, offs))


@pytest.mark.parametrize("seg,ov,exact_copies", [(256, 16, False), (512, 8, True),
                                                  (300, 0, True)])
def test_segment_retry_and_fallback(B, torch_dev, oracle_mod, seg, ov, exact_copies):
    """Segments whose FM-index interval is still open at their end start
    again with a 4x longer overlap (at least 256), then a 16x one (at least
    1024); a read with a repeat longer than that (an exact copy of an old
    string) is walked whole.  Noisy
    copies of one region (5% substitutions) make the first attempts of short
    overlaps fail; the ranks are exact either way, and the statistics show
    that both paths ran."""
    torch = torch_dev
    rng = np.random.default_rng(57)
    ref = rng.integers(0, 4, 20_000, dtype=np.uint8)

    def noisy(n):
        out = []
        for _ in range(n):
            a = int(rng.integers(0, 15_000))
            r = ref[a:a + int(rng.integers(600, 5000))].copy()
            hit = rng.random(len(r)) < 0.05
            r[hit] = (r[hit] + 1) & 3
            out.append(r)
        return out

    old = noisy(40)
    new = noisy(30)
    if exact_copies:
        new += [old[k][100:100 + 2500].copy() for k in range(3) if len(old[k]) > 2700]
        new += [rng.integers(0, 4, int(rng.integers(0, 50)), dtype=np.uint8) for _ in range(20)]

    def pack(rs):
        codes = np.concatenate(rs)
        offs = np.zeros(len(rs) + 1, np.uint64)
        offs[1:] = np.cumsum([len(x) for x in rs])
        return synth.pack_codes(codes), offs

    pa, oa = pack(old)
    pb, ob = pack(new)
    ca, oa2 = _oracle_inputs(oracle_mod, pa, oa)
    T_old, _ = oracle_mod.concat_text(ca, oa2)
    cb, ob2 = _oracle_inputs(oracle_mod, pb, ob)
    T, _ = oracle_mod.concat_text(cb, ob2)
    want = oracle_mod.compute_ranks(T_old, T)
    g = torch.empty(len(T), dtype=torch.int64, device="cuda")
    with B.BwtSet() as idx:
        idx.set_param(B.BWT_PARAM_RANK_SEGMENT, seg)
        idx.set_param(B.BWT_PARAM_RANK_OVERLAP, ov)
        idx.append(pa, oa)
        idx.enable_timing(True)
        idx.stats(reset=True)
        idx.compute_ranks(pb, ob, g)
        st = idx.stats(reset=True)
        assert np.array_equal(g.cpu().numpy().astype(np.uint64), want)
        assert st["ranks_retries"] > 0
        if exact_copies:
            assert st["ranks_fallback_reads"] >= 1
        # every base of the new reads was ranked by the segment kernel (all
        # reads fit the queue)
        assert st["ranks_seg_symbols"] == int(ob[-1])
        idx.append(pb, ob)
        allc = pack(old + new)
        assert idx.export() == oracle_mod.bwt_of_codes(*_oracle_inputs(oracle_mod, *allc))


@pytest.mark.parametrize("buckets", [0, 1])
def test_sort_modes_agree(B, torch_dev, oracle_mod, buckets):
    """The first sort either runs radix passes over the whole key, or only
    over its top digits and finishes each bucket in LDS (piles of identical
    short suffixes, larger than a bucket can hold, take the gathered radix
    path).  Both give the oracle's suffix array and BWT, on one block and
    through appends that rank against a growing index."""
    torch = torch_dev
    cases = [
        synth.short_reads(m=30_000, length=100, ref_len=300_000, seed=51),   # 10x, $-pile of 30k
        synth.random_reads(52, 12_000, 0, 200),                              # ragged, empty reads
        synth.random_reads(53, 60_000, 0, 50, alphabet=2),                   # few distinct keys
        synth.random_reads(54, 40, 0, 6),                                    # tiny block
    ]
    for k, (packed, offs) in enumerate(cases):
        codes, o = _oracle_inputs(oracle_mod, packed, offs)
        sa_want, T = oracle_mod.construct_sa(codes, o)
        n = len(T)
        sa = torch.empty(n, dtype=torch.int32, device="cuda")
        bint = torch.empty(n, dtype=torch.uint8, device="cuda")
        with B.BwtSet() as idx:
            idx.set_param(B.BWT_PARAM_SORT_BUCKETS, buckets)
            idx.enable_timing(True)
            idx.block_sort(packed, offs, sa, bint)
            assert np.array_equal(sa.cpu().numpy().astype(np.uint64), sa_want), k
            assert (idx.stats()["bucket_ms"] > 0) == bool(buckets and n >= (1 << 20)), k
        with B.BwtSet(block_size=max(64, n // 5)) as idx:
            idx.set_param(B.BWT_PARAM_SORT_BUCKETS, buckets)
            idx.append(packed, offs)
            assert idx.export() == oracle_mod.bwt_of_codes(codes, o), k
