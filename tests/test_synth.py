"""The seeded input generators (host side).  The batched and served workloads
are drawn on the GPU with torch and again on the host with numpy for the
full-size expected values, so both must give the same bits; this is checked
here with torch on the CPU, which runs the same integer operations."""
import numpy as np
import pytest

from paper_1410_0562_amd import synth


def test_fmix32_published_vectors():
    # MurmurHash3_x86_32 of the empty input is fmix32(seed): the published
    # test vectors for seeds 0, 1 and 0xFFFFFFFF.
    assert synth.fmix32(0) == 0
    assert synth.fmix32(1) == 0x514E28B7
    assert synth.fmix32(0xFFFFFFFF) == 0x81F16F39


def test_mul32_is_wrapping_product():
    rng = np.random.default_rng(3)
    xs = rng.integers(0, 1 << 32, 2000, dtype=np.int64)
    for c in (0x85EBCA6B, 0xC2B2AE35, 3, 0xFFFFFFFF):
        got = synth._mul32(xs, c)
        want = np.array([(int(x) * c) & 0xFFFFFFFF for x in xs], dtype=np.int64)
        assert np.array_equal(got, want)


def test_counter_draws_same_in_numpy_and_torch():
    torch = pytest.importorskip("torch")
    i = np.arange(0, 1 << 32, 9_999_991, dtype=np.int64)
    k = synth.stream_key(14100566, 7, 4)
    a = synth.counter_u32(k, i)
    b = synth.counter_u32(k, torch.from_numpy(i)).numpy()
    assert np.array_equal(a, b)
    assert a.min() >= 0 and a.max() < (1 << 32)


def test_batch_set_same_on_both_backends():
    torch = pytest.importorskip("torch")
    c1, o1 = synth.batch_set_codes(3, 4000, ref_len=80_000, chunk=555)
    c2, o2 = synth.batch_set_codes(3, 4000, ref_len=80_000, device="cpu")
    assert np.array_equal(c1, c2.numpy()) and np.array_equal(o1, o2.numpy())
    assert np.array_equal(synth.pack_codes(c1), synth._pack_torch(c2).numpy())
    lens = np.diff(o1)
    assert lens.min() >= 36 and lens.max() <= 250 and abs(lens.mean() - 143) < 3


def test_batch_set_statistics():
    # strand 1/2, 1% substitutions: every read is its reference window
    # (reverse-complemented on the minus strand) up to the substituted bases
    ref_len, m = 60_000, 3000
    codes, offs = synth.batch_set_codes(5, m, ref_len=ref_len)
    key = synth.stream_key(synth.SEED_BASE + 4, 5, 0)
    ref = (synth.counter_u32(key, np.arange(ref_len, dtype=np.int64)) >> 30).astype(np.uint8)
    r = np.arange(m, dtype=np.int64)
    lens = np.diff(offs)
    starts = synth.uniform_below(synth.stream_key(synth.SEED_BASE + 4, 5, 2), r, ref_len - lens + 1)
    minus = (synth.counter_u32(synth.stream_key(synth.SEED_BASE + 4, 5, 3), r) >> 31) == 1
    assert 0.45 < minus.mean() < 0.55
    diff = tot = 0
    for j in range(m):
        src = ref[starts[j]:starts[j] + lens[j]]
        if minus[j]:
            src = (3 - src)[::-1]
        diff += int(np.count_nonzero(codes[offs[j]:offs[j + 1]] != src))
        tot += int(lens[j])
    assert 0.008 < diff / tot < 0.012


def test_served_requests_same_on_both_backends():
    torch = pytest.importorskip("torch")
    tids, ms = synth.served_plan(tenants=3, count=6, min_reads=100, max_reads=3000)
    assert tids.min() >= 0 and tids.max() < 3
    ref = synth.served_reference(1, ref_len=70_000)
    reft = synth.served_reference(1, ref_len=70_000, device="cpu")
    assert np.array_equal(ref, reft.numpy())
    for k in range(6):
        a, oa = synth.served_request_codes(k, ref, int(ms[k]), chunk=333)
        b, ob = synth.served_request_codes(k, reft, int(ms[k]), device="cpu")
        assert np.array_equal(a, b.numpy()) and np.array_equal(oa, ob.numpy())
        assert len(a) == 150 * int(ms[k])


def test_full_size_plan_matches_the_workload_recipe():
    ms = synth.batch_sizes()
    assert len(ms) == 64 and ms.min() >= 1000 and ms.max() <= 2_000_000
    tids, rm = synth.served_plan()
    assert len(tids) == 512 and set(tids.tolist()) == set(range(16))
    assert rm.min() >= 10_000 and rm.max() <= 1_000_000
