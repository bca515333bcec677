"""Parity at full size: the whole exported BWT of every benchmark workload,
built in the launch configuration bench.py times (device inputs, the same
block sizes), against the SHA-256 of the oracle's BWT of the same draws.

The digests are written by tests/golden/make_full_size.py, which runs only
the oracle (a comparison sort of all suffixes in Section 2's order, then
Eq. 1) on the seeded generators; a workload whose digest has not been
computed is skipped with that reason.  The BWT is unique (all suffixes are
distinct), so equal digests mean the GPU result is the oracle's, byte for
byte.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1410_0562_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "full_size_sha256.json")


def _golden(key):
    try:
        with open(GOLDEN) as f:
            d = json.load(f)
    except OSError:
        pytest.skip("no full-size digests (run tests/golden/make_full_size.py)")
    if key not in d:
        pytest.skip("no full-size digest for %s yet (tests/golden/make_full_size.py --only)" % key)
    return d[key]


def _log(msg):
    print("[full-size] " + msg, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _sha_of_index(torch, idx):
    n = idx.size()[0]
    out = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
    idx.export(out)
    host = out[:n].cpu().numpy()
    del out
    return hashlib.sha256(host.tobytes()).hexdigest(), n


@pytest.mark.parametrize("key,block,where", [("uniform_10k", 1 << 18, "device"),
                                             ("short_reads_4M", 1 << 26, "device"),
                                             ("long_reads_250k", 1 << 27, "device"),
                                             ("short_reads_4M", 1 << 26, "host, pipelined"),
                                             ("long_reads_250k", 1 << 27, "host, pipelined")])
def test_plain_workload_bwt_digest(torch_dev, key, block, where):
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    want = _golden(key)
    _log("%s: generating" % key)
    if key == "uniform_10k":
        packed, offs = synth.uniform_reads()
    elif key == "short_reads_4M":
        packed, offs = synth.short_reads()
    else:
        packed, offs = synth.long_reads(threads=16)
    assert int(offs[-1]) == want["bases"] and len(offs) - 1 == want["strings"]
    if where == "device":
        dev_reads = torch.from_numpy(packed).cuda()
        dev_offs = torch.from_numpy(offs.view(np.int64)).cuda()
    else:
        dev_reads, dev_offs = packed, offs       # streamed block by block
    _log("%s: building %d bases, block %d, input %s" % (key, want["bases"], block, where))
    with bwtset.BwtSet(block_size=block) as idx:
        idx.append(dev_reads, dev_offs)
        sha, n = _sha_of_index(torch, idx)
    del dev_reads, dev_offs
    torch.cuda.empty_cache()
    assert n == want["symbols"]
    assert sha == want["sha256"], key


def test_batched_workload_digests(torch_dev):
    """All 64 sets of the batched workload in one bwt_set_append_many call
    (bench.py --batched's launch configuration), every set's BWT against the
    oracle's digest of that set."""
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    want = _golden("batched_64_sets")
    _log("batched: generating 64 sets on the GPU")
    sets = synth.batch_sets_gpu()
    assert len(sets) == len(want)
    hs = [bwtset.BwtSet(block_size=1 << 26) for _ in sets]
    try:
        _log("batched: building")
        bwtset.append_many(hs, [p for p, _, _ in sets], [o for _, o, _ in sets])
        for s, (h, w) in enumerate(zip(hs, want)):
            assert h.size() == (w["symbols"], w["strings"]), s
            sha, _ = _sha_of_index(torch, h)
            assert sha == w["sha256"], s
    finally:
        for h in hs:
            h.close()
        del sets
        torch.cuda.empty_cache()


def test_served_workload_digests(torch_dev):
    """All 512 requests of the served workload through the service (requests
    of different tenants batched and overlapping), every tenant's BWT against
    the oracle's digest of its requests in arrival order."""
    torch = torch_dev
    from paper_1410_0562_amd.serve import BwtService
    want = _golden("served_16_tenants")
    if len(want) < 16:
        pytest.skip("served digests for %d of 16 tenants so far (tests/golden/make_full_size.py)"
                    % len(want))
    _log("served: generating 512 requests on the GPU")
    tids, reqs = synth.served_requests_gpu()
    svc = BwtService(16, budget_bytes=100 << 30, workers=4, block_size=1 << 26)
    try:
        _log("served: submitting")
        for t, (p, o, _) in zip(tids, reqs):
            svc.submit(int(t), p, o)
        svc.drain(timeout=900)
        assert svc.latency_summary()["errors"] == 0
        for t in range(16):
            B = svc.export(t)
            assert len(B) == want[t]["symbols"], t
            assert hashlib.sha256(B).hexdigest() == want[t]["sha256"], t
    finally:
        svc.close()
        del reqs
        torch.cuda.empty_cache()
