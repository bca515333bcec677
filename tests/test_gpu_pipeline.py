"""Pipelined blocks (BWT_PARAM_PIPELINE): reads in host memory streamed to
the device block by block on a copy stream while earlier blocks run.  The
index must not depend on it: pipelined, unpipelined and device-input appends
give the oracle's BWT."""
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


def _log(msg):
    print("[pipeline] " + msg, flush=True)


CASES = {
    "short reads, many blocks": (lambda: synth.short_reads(m=30_000, length=100,
                                                             ref_len=300_000, seed=131), 90_000),
    "ragged with empty reads": (lambda: synth.random_reads(132, 5000, 0, 300), 60_000),
    "long reads, segments": (lambda: synth.random_reads(133, 400, 800, 6000), 250_000),
    "one block": (lambda: synth.random_reads(134, 300, 10, 90), 1 << 20),
}


@pytest.mark.parametrize("name", list(CASES))
def test_pipelined_equals_unpipelined_and_oracle(torch_dev, oracle_mod, name):
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    make, M = CASES[name]
    packed, offs = make()
    want = oracle_mod.bwt_of_codes(*oracle_mod.reads_from_packed(packed, offs))
    got = {}
    for mode in ("pipelined", "unpipelined", "device", "device offsets"):
        _log("%s: %s" % (name, mode))
        with bwtset.BwtSet(block_size=M) as h:
            h.set_param(bwtset.BWT_PARAM_PIPELINE, 0 if mode == "unpipelined" else 1)
            h.enable_timing(True)
            if mode == "device":
                h.append(torch.from_numpy(packed).cuda(),
                         torch.from_numpy(offs.view(np.int64)).cuda())
            elif mode == "device offsets":
                h.append(packed, torch.from_numpy(offs.view(np.int64)).cuda())
            else:
                h.append(packed, offs)
            got[mode] = h.export()
            assert h.size() == (len(want), len(offs) - 1)
    for mode, b in got.items():
        assert b == want, mode


def test_pipelined_appends_on_a_growing_index(torch_dev, oracle_mod):
    """Several pipelined appends, one starting inside its packed buffer, on
    top of an index built from device input."""
    torch = torch_dev
    from paper_1410_0562_amd import bwtset
    parts = [synth.random_reads(140 + k, 2500, 0, 220) for k in range(3)]
    p1, o1 = parts[1]
    o1 = o1.copy()
    o1[0] += np.uint64(5)                          # first read starts at symbol 5
    parts[1] = (p1, o1)
    allc = [oracle_mod.reads_from_packed(p, o) for p, o in parts]
    codes = np.concatenate([c for c, _ in allc])
    offs = np.zeros(sum(len(o) - 1 for _, o in allc) + 1, np.uint64)
    offs[1:] = np.cumsum(np.concatenate([np.diff(o.astype(np.int64)) for _, o in allc]))
    want = oracle_mod.bwt_of_codes(codes, offs)
    with bwtset.BwtSet(block_size=40_000) as h:
        h.append(torch.from_numpy(parts[0][0]).cuda(),
                 torch.from_numpy(parts[0][1].view(np.int64)).cuda())
        h.append(*parts[1])
        h.append(*parts[2])
        assert h.export() == want
