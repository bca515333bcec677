"""Serving form: several tenants, requests arriving while others run.  Each
tenant's index must equal the oracle BWT of its requests in arrival order,
and be the same bytes whether the tenant ran alone or in the mix, and
whether or not it was spilled to host memory and restored in between."""
import random
import time

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


def _requests(seed, tenants, count):
    rng = random.Random(seed)
    refs = [np.random.default_rng(seed * 100 + t).integers(0, 4, 200_000, dtype=np.uint8)
            for t in range(tenants)]
    reqs = []
    for k in range(count):
        t = rng.randrange(tenants)
        m = int(np.exp(rng.uniform(np.log(200), np.log(6000))))
        r = np.random.default_rng(seed * 7919 + k)
        starts = r.integers(0, len(refs[t]) - 150, m)
        codes = refs[t][starts[:, None] + np.arange(150)[None, :]].copy()
        hit = r.random(codes.shape) < 0.01
        codes[hit] = (codes[hit] + 1) & 3
        offs = np.arange(m + 1, dtype=np.uint64) * np.uint64(150)
        reqs.append((t, synth.pack_codes(codes.reshape(-1)), offs))
    return reqs


def _oracle_of(oracle_mod, reqs, t):
    parts = [(p, o) for (tt, p, o) in reqs if tt == t]
    if not parts:
        return b""
    codes = [oracle_mod.reads_from_packed(p, o) for p, o in parts]
    allc = np.concatenate([c for c, _ in codes])
    lens = np.concatenate([np.diff(o.astype(np.int64)) for _, o in codes])
    offs = np.zeros(len(lens) + 1, np.uint64)
    offs[1:] = np.cumsum(lens)
    return oracle_mod.bwt_of_codes(allc, offs)


def _run(reqs, tenants, budget, workers, gap_s=0.0, block=1 << 20, per_append=None):
    from paper_1410_0562_amd.serve import BwtService
    svc = BwtService(tenants, budget_bytes=budget, workers=workers, block_size=block,
                     per_append_bytes=per_append)
    try:
        for (t, p, o) in reqs:
            svc.submit(t, p, o)
            if gap_s:
                time.sleep(gap_s)
        svc.drain(timeout=120)
        out = [svc.export(t) for t in range(tenants)]
        summ = svc.latency_summary()
    finally:
        svc.close()
    return out, summ


def test_mix_equals_alone_and_oracle(torch_dev, oracle_mod):
    tenants = 4
    reqs = _requests(5, tenants, 24)
    mixed, summ = _run(reqs, tenants, budget=64 << 30, workers=3, gap_s=0.002)
    assert summ["errors"] == 0 and summ["requests"] == len(reqs)
    for t in range(tenants):
        alone, _ = _run([r for r in reqs if r[0] == t], tenants, budget=64 << 30, workers=1)
        assert mixed[t] == alone[t], t
        assert mixed[t] == _oracle_of(oracle_mod, reqs, t), t


def test_spill_and_restore_under_a_small_budget(torch_dev, oracle_mod):
    tenants = 5
    reqs = _requests(6, tenants, 30)
    # a budget that holds about one tenant's working set forces spills
    out, summ = _run(reqs, tenants, budget=24 << 20, workers=2, block=1 << 18,
                     per_append=16 << 20)
    assert summ["errors"] == 0
    assert summ["spills"] > 0 and summ["restores"] > 0
    for t in range(tenants):
        assert out[t] == _oracle_of(oracle_mod, reqs, t), t


def test_import_roundtrip(torch_dev, oracle_mod):
    from paper_1410_0562_amd import bwtset
    packed, offs = synth.random_reads(50, 3000, 0, 200)
    c1, o1 = oracle_mod.reads_from_packed(packed, offs)
    want = oracle_mod.bwt_of_codes(c1, o1)
    with bwtset.BwtSet() as a:
        a.import_bwt(want)
        assert a.export() == want and a.size() == (len(want), 3000)
        for c in "$ACGT":
            assert a.rank(c, len(want) // 2) == oracle_mod.rank(want, c, len(want) // 2)
        # device input, then an append on top of the imported index
        dev = torch_dev.from_numpy(np.frombuffer(want, np.uint8).copy()).cuda()
        a.import_bwt(dev)
        more_p, more_o = synth.random_reads(51, 500, 0, 120)
        a.append(more_p, more_o)
        cm, om = oracle_mod.reads_from_packed(more_p, more_o)
        allc = np.concatenate([c1, cm])
        allo = np.concatenate([o1, om[1:] + o1[-1]])
        assert a.export() == oracle_mod.bwt_of_codes(allc, allo)
        with pytest.raises(bwtset.BwtSetError):
            a.import_bwt(b"ACGTN$")
        before = a.export()
        assert a.size()[0] == len(before)
        a.trim()
        assert a.export() == before
        assert a.memory() > 0


def test_served_generator_through_service(torch_dev, oracle_mod):
    """The device-side request generator used by the served benchmark, at a
    small size: every tenant's index equals the oracle BWT of its requests."""
    tenants = 3
    tids, reqs = synth.served_requests_gpu(tenants=tenants, count=9, ref_len=50_000,
                                           min_reads=100, max_reads=2000, length=150)
    host = [(int(t), p.cpu().numpy(), o.cpu().numpy().astype(np.uint64))
            for t, (p, o, _) in zip(tids, reqs)]
    for (_, p, o), (_, _, b) in zip(host, reqs):
        assert int(o[-1]) == b and len(p) == (b + 3) // 4
    from paper_1410_0562_amd.serve import BwtService
    svc = BwtService(tenants, budget_bytes=64 << 30, workers=2, block_size=1 << 18)
    try:
        for t, (p, o, _) in zip(tids, reqs):
            svc.submit(int(t), p, o)
        svc.drain(timeout=120)
        out = [svc.export(t) for t in range(tenants)]
        assert svc.latency_summary()["errors"] == 0
    finally:
        svc.close()
    for t in range(tenants):
        assert out[t] == _oracle_of(oracle_mod, host, t), t


def test_failed_restore_keeps_the_spill_and_stops_the_tenant(torch_dev, oracle_mod, monkeypatch):
    """An import that fails while a spilled tenant is restored (as it may under
    the memory pressure that caused the spill) must leave the tenant spilled
    with its index intact, fail its later requests rather than apply them
    without the failed one, and serve it again after resume()."""
    from paper_1410_0562_amd import bwtset
    from paper_1410_0562_amd.serve import BwtService, TenantFailed
    tenants = 3
    reqs = _requests(9, tenants, 12)
    real_import = bwtset.BwtSet.import_bwt
    calls = {"n": 0}

    def flaky_import(self, B, stream=None):
        calls["n"] += 1
        if calls["n"] == 1:
            raise bwtset.BwtSetError(bwtset.BWT_ENOMEM, "bwt_set_import")
        return real_import(self, B, stream)

    monkeypatch.setattr(bwtset.BwtSet, "import_bwt", flaky_import)
    # a budget below one batch's workspace: every batch runs alone, and every
    # idle tenant is spilled before it, so each tenant's next request restores
    svc = BwtService(tenants, budget_bytes=1 << 20, workers=1, block_size=1 << 18,
                     per_append_bytes=1 << 20)
    try:
        handles = [svc.submit(t, p, o) for (t, p, o) in reqs]
        svc.drain(timeout=120)
        failed = [k for k, r in enumerate(handles) if r.error is not None]
        assert failed, "the injected import failure did not happen"
        first = failed[0]
        bad_t = reqs[first][0]
        assert isinstance(handles[first].error, bwtset.BwtSetError)
        assert svc.failure(bad_t) is not None
        # every later request of that tenant failed, none of another tenant
        for k, r in enumerate(handles):
            if reqs[k][0] == bad_t and k > first:
                assert isinstance(r.error, TenantFailed), k
            elif reqs[k][0] != bad_t:
                assert r.error is None, k
        # the tenant still holds exactly its requests before the failure
        done = [r for k, r in enumerate(reqs) if r[0] != bad_t or k < first]
        assert svc.export(bad_t) == _oracle_of(oracle_mod, done, bad_t)
        # after resume, the failed and later requests go through in order
        svc.resume(bad_t)
        for k in range(first, len(reqs)):
            if reqs[k][0] == bad_t:
                svc.submit(*reqs[k])
        svc.drain(timeout=120)
        assert svc.failure(bad_t) is None
        out = [svc.export(t) for t in range(tenants)]
    finally:
        svc.close()
    for t in range(tenants):
        assert out[t] == _oracle_of(oracle_mod, reqs, t), t


def test_queued_requests_share_one_batch(torch_dev, oracle_mod):
    """Requests of different tenants queued together run as one batched
    append (bwt_set_append_many), and each tenant's index is still the oracle
    BWT of its own requests."""
    from paper_1410_0562_amd.serve import BwtService
    tenants = 6
    reqs = _requests(11, tenants, 36)
    svc = BwtService(tenants, budget_bytes=64 << 30, workers=1, block_size=1 << 20, max_batch=6)
    try:
        # one worker: whatever queues while it runs a batch forms the next one
        for (t, p, o) in reqs:
            svc.submit(t, p, o)
        svc.drain(timeout=120)
        summ = svc.latency_summary()
        out = [svc.export(t) for t in range(tenants)]
    finally:
        svc.close()
    assert summ["errors"] == 0 and summ["requests"] == len(reqs)
    assert summ["mean_batch"] > 1.5, summ
    for t in range(tenants):
        assert out[t] == _oracle_of(oracle_mod, reqs, t), t


def test_batches_run_on_the_workers_own_handles(torch_dev, oracle_mod):
    """Every batch is led by a handle of its worker that holds no strings, so
    the block workspace lives on the workers' handles and a tenant's handle
    holds only its index buffers (trimming a tenant frees nothing a later
    batch has to allocate again)."""
    from paper_1410_0562_amd.serve import BwtService
    tenants = 4
    reqs = _requests(11, tenants, 16)
    svc = BwtService(tenants, budget_bytes=64 << 30, workers=2, block_size=1 << 20)
    try:
        for (t, p, o) in reqs:
            svc.submit(t, p, o)
        svc.drain(timeout=120)
        lead = max(h.memory() for h in svc._leaders)
        held = [t.index.memory() for t in svc.tenants if t.index is not None]
        assert held and lead > 0
        # the workspace of a block of up to 2^20 suffixes is far larger than
        # the few-million-symbol indices of these tenants
        assert max(held) * 4 < lead, (held, lead)
        out = [svc.export(t) for t in range(tenants)]
        assert svc.latency_summary()["errors"] == 0
    finally:
        svc.close()
    for t in range(tenants):
        assert out[t] == _oracle_of(oracle_mod, reqs, t), t

