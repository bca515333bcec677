"""Seeded synthetic read sets in the library's input format.

This module only draws random DNA and packs it; it holds none of the BWT
arithmetic, and it is the one piece shared by the tests, the benchmark and the
CPU oracle's callers.

Input format (the one ``bwt_set_append`` takes):

* ``packed``: uint8, 2 bits per symbol, code = index in "ACGT", symbol s at
  byte s >> 2, bits 2*(s & 3) and up (LSB first);
* ``offsets``: uint64[m + 1], non-decreasing; read j is symbols
  [offsets[j], offsets[j+1]).

Workloads (seed = 14100562 + workload number):

1. ``uniform_reads``: 10,000 reads x 100 bp, i.i.d. uniform bases.
2. ``short_reads``: 4,000,000 x 100 bp sampled from a uniform random 50 Mbp
   reference at uniform start positions, either strand with probability 1/2
   (reverse complement), 1% i.i.d. substitutions to one of the other three
   bases.  Stands in for a large Illumina short-read set.
3. ``long_reads``: 250,000 reads, lengths lognormal (mean 5 kbp, sigma of the
   log 0.5, clipped to [1,000, 50,000]) from a uniform 100 Mbp reference, either
   strand, 10% noise per base split 6% substitution / 2% insertion / 2%
   deletion.  Stands in for a long-read (Sanger-like) set.
4. ``batch_sets_gpu``: 64 independent sets, each from its own uniform 10 Mbp
   reference, floor(exp(U(ln 1e3, ln 2e6))) reads per set of uniform length
   in [36, 250], either strand, 1% substitutions (drawn on the GPU).
5. ``served_requests_gpu``: 16 tenants with their own uniform 100 Mbp
   references; 512 append requests of floor(exp(U(ln 1e4, ln 1e6))) reads x
   150 bp, forward strand, 1% substitutions (drawn on the GPU).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 14100562
_RC = np.array([3, 2, 1, 0], dtype=np.uint8)


def pack_codes(codes: np.ndarray) -> np.ndarray:
    """Pack codes 0..3 four per byte, LSB first; pads with zero bits."""
    codes = np.asarray(codes, dtype=np.uint8)
    n = len(codes)
    pad = (-n) % 4
    if pad:
        codes = np.concatenate([codes, np.zeros(pad, dtype=np.uint8)])
    c = codes.reshape(-1, 4)
    return (c[:, 0] | (c[:, 1] << 2) | (c[:, 2] << 4) | (c[:, 3] << 6)).astype(np.uint8)


def strings_to_input(reads) -> tuple[np.ndarray, np.ndarray]:
    """ASCII reads over ACGT -> (packed, offsets)."""
    lut = np.full(256, 255, dtype=np.uint8)
    for i, ch in enumerate(b"ACGT"):
        lut[ch] = i
    joined = "".join(reads).encode("ascii")
    codes = lut[np.frombuffer(joined, dtype=np.uint8)] if joined else np.zeros(0, np.uint8)
    if codes.size and codes.max() > 3:
        raise ValueError("reads must use only A, C, G, T")
    offsets = np.zeros(len(reads) + 1, dtype=np.uint64)
    if len(reads):
        offsets[1:] = np.cumsum([len(r) for r in reads], dtype=np.uint64)
    return pack_codes(codes), offsets


def random_reads(seed: int, m: int, min_len: int, max_len: int, alphabet: int = 4):
    """m reads with lengths uniform in [min_len, max_len], i.i.d. bases drawn
    from the first `alphabet` letters of ACGT.  Returns (packed, offsets)."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(min_len, max_len + 1, size=m, dtype=np.int64)
    offsets = np.zeros(m + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(lens).astype(np.uint64)
    codes = rng.integers(0, alphabet, size=int(offsets[-1]), dtype=np.uint8)
    return pack_codes(codes), offsets


def uniform_reads(m: int = 10_000, length: int = 100, seed: int = SEED_BASE + 1):
    """Workload 1: m reads x length bp, i.i.d. uniform over ACGT."""
    return random_reads(seed, m, length, length)


def _substitute(rng, codes: np.ndarray, rate: float) -> None:
    hit = rng.random(codes.shape) < rate
    k = int(hit.sum())
    if k:
        codes[hit] = (codes[hit] + rng.integers(1, 4, size=k, dtype=np.uint8)) & 3


def short_reads(m: int = 4_000_000, length: int = 100, ref_len: int = 50_000_000,
                sub_rate: float = 0.01, seed: int = SEED_BASE + 2,
                chunk: int = 1 << 18):
    """Workload 2: fixed-length reads sampled from a random reference, both
    strands, i.i.d. substitutions.  Returns (packed, offsets)."""
    rng = np.random.default_rng(seed)
    ref = rng.integers(0, 4, size=ref_len, dtype=np.uint8)
    total = m * length
    codes_all = np.empty(total, dtype=np.uint8)
    ar = np.arange(length, dtype=np.int64)
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        k = r1 - r0
        starts = rng.integers(0, ref_len - length + 1, size=k, dtype=np.int64)
        minus = rng.random(k) < 0.5
        blk = ref[starts[:, None] + ar[None, :]]
        if minus.any():
            blk[minus] = _RC[blk[minus][:, ::-1]]
        _substitute(rng, blk, sub_rate)
        codes_all[r0 * length:r1 * length] = blk.reshape(-1)
    offsets = np.arange(m + 1, dtype=np.uint64) * np.uint64(length)
    return pack_codes(codes_all), offsets


def _long_chunk(child_seed, ref, L, sub, ins, dele):
    rng = np.random.default_rng(child_seed)
    ref_len = len(ref)
    k = len(L)
    starts = rng.integers(0, ref_len - L + 1, dtype=np.int64)
    minus = rng.random(k) < 0.5
    seg = np.zeros(k + 1, dtype=np.int64)
    seg[1:] = np.cumsum(L)
    total = int(seg[-1])
    # source index of every base; a minus-strand read walks its window
    # backwards and is complemented
    step = np.where(minus, -1, 1)
    first = np.where(minus, starts + L - 1, starts)
    idx = np.repeat(first - step * seg[:-1], L) + np.repeat(step, L) * np.arange(total, dtype=np.int64)
    base = ref[idx]
    mrep = np.repeat(minus, L)
    base[mrep] = _RC[base[mrep]]
    # per-base event drawn at a resolution of 1/10,000
    u = rng.integers(0, 10_000, size=total, dtype=np.uint16)
    t_del, t_ins = int(round(dele * 1e4)), int(round((dele + ins) * 1e4))
    t_sub = int(round((dele + ins + sub) * 1e4))
    copies = np.ones(total, dtype=np.int8)
    copies[u < t_del] = 0
    copies[(u >= t_del) & (u < t_ins)] = 2
    subm = (u >= t_ins) & (u < t_sub)
    ks = int(subm.sum())
    if ks:
        base[subm] = (base[subm] + rng.integers(1, 4, size=ks, dtype=np.uint8)) & 3
    rep = np.repeat(base, copies)
    ins_pos = np.flatnonzero(copies == 2)
    if len(ins_pos):
        # the second copy of an inserted base becomes a random base
        out_idx = np.cumsum(copies, dtype=np.int64) - 1
        rep[out_idx[ins_pos]] = rng.integers(0, 4, size=len(ins_pos), dtype=np.uint8)
    return rep, np.add.reduceat(copies.astype(np.int64), seg[:-1])


def long_reads(m: int = 250_000, mean_len: float = 5000.0, sigma: float = 0.5,
               min_len: int = 1000, max_len: int = 50_000,
               ref_len: int = 100_000_000, sub: float = 0.06, ins: float = 0.02,
               dele: float = 0.02, seed: int = SEED_BASE + 3, chunk: int = 4096,
               threads: int = 8):
    """Workload 3: lognormal-length noisy reads from a random reference.
    Each source base is deleted (prob. dele), followed by an inserted random
    base (ins), substituted (sub) or kept.  Chunks of reads draw from child
    seeds, so the output does not depend on `threads`.  Returns (packed, offsets)."""
    from concurrent.futures import ThreadPoolExecutor
    ss = np.random.SeedSequence(seed)
    s_ref, s_len, s_chunks = ss.spawn(3)
    ref = np.random.default_rng(s_ref).integers(0, 4, size=ref_len, dtype=np.uint8)
    mu = np.log(mean_len) - sigma * sigma / 2.0
    lens = np.clip(np.rint(np.random.default_rng(s_len).lognormal(mu, sigma, size=m)),
                   min_len, max_len).astype(np.int64)
    bounds = list(range(0, m, chunk))
    seeds = s_chunks.spawn(len(bounds))
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        res = list(ex.map(lambda a: _long_chunk(seeds[a[0]], ref, lens[a[1]:min(m, a[1] + chunk)],
                                                sub, ins, dele), enumerate(bounds)))
    out_lens = np.concatenate([r[1] for r in res]) if res else np.zeros(0, np.int64)
    offsets = np.zeros(m + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(out_lens).astype(np.uint64)
    codes = np.concatenate([r[0] for r in res]) if res else np.zeros(0, np.uint8)
    return pack_codes(codes), offsets


def take_reads(packed: np.ndarray, offsets: np.ndarray, j0: int, j1: int):
    """Reads j0..j1-1 of an input as a new (packed, offsets) pair whose first
    read starts at symbol 0."""
    offsets = np.asarray(offsets, dtype=np.uint64)
    s0, s1 = int(offsets[j0]), int(offsets[j1])
    n = s1 - s0
    # unpack the symbol range and repack from symbol 0
    b0, b1 = s0 // 4, (s1 + 3) // 4
    sub = np.asarray(packed[b0:b1], dtype=np.uint8)
    codes = np.empty(len(sub) * 4, dtype=np.uint8)
    for q in range(4):
        codes[q::4] = (sub >> (2 * q)) & 3
    codes = codes[s0 - 4 * b0:s0 - 4 * b0 + n]
    return pack_codes(codes), (offsets[j0:j1 + 1] - np.uint64(s0)).astype(np.uint64)


# ---------------------------------------------------------------------------
# Counter-based draws for the batched and served workloads.
#
# These two workloads are drawn on the GPU (billions of bases), and their
# full-size expected BWTs are computed offline on the CPU, so every random
# value must come out the same from numpy on the host and from torch on the
# device.  Each value is a pure function of (stream key, index): MurmurHash3's
# 32-bit finalizer (Appleby, "fmix32") applied twice to the index mixed with
# the key.  Every step is a 64-bit integer operation whose result stays below
# 2^63 (the 32x32-bit products are split into 16-bit halves), so numpy and
# torch, on either device, compute exactly the same bits.
# ---------------------------------------------------------------------------
_M32 = 0xFFFFFFFF
_SUB_THRESHOLD = 42_949_673          # round(0.01 * 2^32): a 1% substitution draw


def _mul32(x, c: int):
    """(x * c) mod 2^32 for x in [0, 2^32) held in int64, c a 32-bit constant."""
    return (x * (c & 0xFFFF) + (((x * (c >> 16)) & 0xFFFF) << 16)) & _M32


def fmix32(h):
    """MurmurHash3's 32-bit finalizer on values in [0, 2^32) (int64 arrays or
    tensors, or Python ints)."""
    h = h ^ (h >> 16)
    h = _mul32(h, 0x85EBCA6B)
    h = h ^ (h >> 13)
    h = _mul32(h, 0xC2B2AE35)
    return h ^ (h >> 16)


def stream_key(*parts: int) -> int:
    """A 32-bit stream key from small non-negative integers (seed, set, purpose)."""
    k = 0x9E3779B9
    for p in parts:
        k = fmix32((k ^ (int(p) & _M32)) & _M32)
        k = fmix32((k + 0x7F4A7C15) & _M32)
    return k


def counter_u32(key: int, i):
    """Uniform 32-bit value number i (0 <= i < 2^32) of stream `key`."""
    k1 = fmix32(key & _M32)
    k2 = fmix32((key ^ 0x85EBCA77) & _M32)
    return fmix32(fmix32(i ^ k1) ^ k2)


def uniform_below(key: int, i, bound):
    """floor(u * bound / 2^32) for u = counter_u32(key, i): an integer in
    [0, bound) for bound < 2^31 (scalar or array)."""
    return (counter_u32(key, i) * bound) >> 32


class _NumpyOps:
    device = "cpu"

    def arange(self, a, b=None):
        return np.arange(a, b, dtype=np.int64) if b is not None else np.arange(a, dtype=np.int64)

    def cumsum0(self, x):
        out = np.zeros(len(x) + 1, dtype=np.int64)
        out[1:] = np.cumsum(x)
        return out

    def repeat(self, x, counts):
        return np.repeat(x, counts)

    def where(self, c, a, b):
        return np.where(c, a, b)

    def u8(self, x):
        return x.astype(np.uint8)

    def cat(self, xs):
        return np.concatenate(xs)

    def scalar(self, x):
        return int(x)


class _TorchOps:
    def __init__(self, device):
        import torch
        self.t = torch
        self.device = device

    def arange(self, a, b=None):
        t = self.t
        if b is None:
            return t.arange(a, dtype=t.int64, device=self.device)
        return t.arange(a, b, dtype=t.int64, device=self.device)

    def cumsum0(self, x):
        t = self.t
        out = t.zeros(x.numel() + 1, dtype=t.int64, device=self.device)
        t.cumsum(x, 0, out=out[1:])
        return out

    def repeat(self, x, counts):
        return self.t.repeat_interleave(x, counts)

    def where(self, c, a, b):
        return self.t.where(c, a, b)

    def u8(self, x):
        return x.to(self.t.uint8)

    def cat(self, xs):
        return self.t.cat(xs)

    def scalar(self, x):
        return int(x.item())


def _ops(device):
    return _NumpyOps() if device is None or device == "numpy" else _TorchOps(device)


def _reference(ops, key: int, ref_len: int):
    """A uniform random reference: base i = top two bits of draw i."""
    out = []
    step = 1 << 26
    for a in range(0, ref_len, step):
        out.append(ops.u8(counter_u32(key, ops.arange(a, min(ref_len, a + step))) >> 30))
    return ops.cat(out)


def _substitute_counter(ops, codes, pos, key_hit: int, key_delta: int):
    """1% i.i.d. substitutions to one of the other three bases; the draws of
    base number `pos` (an int64 array the shape of codes)."""
    hit = counter_u32(key_hit, pos) < _SUB_THRESHOLD
    delta = 1 + uniform_below(key_delta, pos, 3)
    return ops.where(hit, (codes + delta) & 3, codes)


def batch_set_codes(s: int, m: int, ref_len: int = 10_000_000, min_len: int = 36,
                    max_len: int = 250, seed: int = SEED_BASE + 4, device=None,
                    chunk: int = 1 << 18):
    """Set s of the batched workload with m reads: its own uniform reference of
    ref_len bases; read r has length uniform in [min_len, max_len], a start
    uniform over the positions it fits, the minus strand (reverse complement)
    with probability 1/2, and 1% substitutions.  device None: numpy arrays;
    otherwise torch tensors on that device.  Returns (codes 0..3 as uint8,
    offsets int64[m + 1]); the values do not depend on the device or chunk."""
    ops = _ops(device)
    ref = _reference(ops, stream_key(seed, s, 0), ref_len)
    r = ops.arange(m)
    span = max_len - min_len + 1
    lens = min_len + uniform_below(stream_key(seed, s, 1), r, span)
    starts = uniform_below(stream_key(seed, s, 2), r, ref_len - lens + 1)
    minus = (counter_u32(stream_key(seed, s, 3), r) >> 31) == 1
    offs = ops.cumsum0(lens)
    total = ops.scalar(offs[-1])
    if total >= 1 << 32:
        raise ValueError("set too large for 32-bit draw indices")
    parts = []
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        L = lens[r0:r1]
        rid = ops.repeat(ops.arange(r0, r1), L)
        pos = ops.arange(ops.scalar(offs[r0]), ops.scalar(offs[r1]))
        within = pos - offs[rid]
        fwd = starts[rid] + within
        rev = starts[rid] + lens[rid] - 1 - within
        mr = minus[rid]
        c = ref[ops.where(mr, rev, fwd)]
        c = ops.where(mr, 3 - c, c)
        c = _substitute_counter(ops, c, pos, stream_key(seed, s, 4), stream_key(seed, s, 5))
        parts.append(ops.u8(c))
    codes = ops.cat(parts) if parts else ops.u8(ops.arange(0))
    return codes, offs


def batch_sizes(count: int = 64, min_reads: int = 1_000, max_reads: int = 2_000_000,
                seed: int = SEED_BASE + 4):
    """Reads per set of the batched workload: floor(exp(U(ln min, ln max)))."""
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(np.log(min_reads), np.log(max_reads), count))).astype(np.int64)


def served_plan(tenants: int = 16, count: int = 512, min_reads: int = 10_000,
                max_reads: int = 1_000_000, seed: int = SEED_BASE + 5):
    """Tenant and read count of every request of the served workload."""
    rng = np.random.default_rng(seed)
    tids = rng.integers(0, tenants, count)
    ms = np.floor(np.exp(rng.uniform(np.log(min_reads), np.log(max_reads), count))).astype(np.int64)
    return tids, ms


def served_reference(t: int, ref_len: int = 100_000_000, seed: int = SEED_BASE + 5, device=None):
    return _reference(_ops(device), stream_key(seed, 1_000_000 + t, 0), ref_len)


def served_request_codes(k: int, ref, m: int, length: int = 150, seed: int = SEED_BASE + 5,
                         device=None, chunk: int = 1 << 18):
    """Request k of the served workload against its tenant's reference `ref`:
    m reads x length bp at uniform forward-strand starts, 1% substitutions.
    Returns (codes uint8, offsets int64[m + 1]) as numpy (device None) or torch."""
    ops = _ops(device)
    ref_len = int(ref.shape[0])
    r = ops.arange(m)
    starts = uniform_below(stream_key(seed, k, 2), r, ref_len - length + 1)
    offs = ops.arange(m + 1) * length
    if m * length >= 1 << 32:
        raise ValueError("request too large for 32-bit draw indices")
    parts = []
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        pos = ops.arange(r0 * length, r1 * length)
        rid = pos // length
        c = ref[starts[rid] + (pos - rid * length)]
        c = _substitute_counter(ops, c, pos, stream_key(seed, k, 4), stream_key(seed, k, 5))
        parts.append(ops.u8(c))
    codes = ops.cat(parts) if parts else ops.u8(ops.arange(0))
    return codes, offs


def _pack_torch(codes):
    import torch
    shifts = torch.tensor([0, 2, 4, 6], device=codes.device, dtype=torch.uint8)
    pad = (-codes.numel()) % 4
    if pad:
        codes = torch.cat([codes, torch.zeros(pad, dtype=torch.uint8, device=codes.device)])
    return (codes.view(-1, 4) << shifts).sum(dim=1, dtype=torch.uint8)


def served_requests_gpu(tenants: int = 16, count: int = 512, ref_len: int = 100_000_000,
                        min_reads: int = 10_000, max_reads: int = 1_000_000, length: int = 150,
                        seed: int = SEED_BASE + 5):
    """Workload 5 drawn on the GPU: per-tenant uniform random references,
    `count` requests to uniformly drawn tenants with log-uniform read counts,
    reads sampled at uniform positions (forward strand) with i.i.d.
    substitutions (the counter-based draws above, so the host can draw the
    same requests).  Returns (tenant ids, list of (packed device tensor,
    offsets device int64 tensor, bases))."""
    tids, ms = served_plan(tenants, count, min_reads, max_reads, seed)
    refs = [served_reference(t, ref_len, seed, device="cuda") for t in range(tenants)]
    out = []
    for k, (t, m) in enumerate(zip(tids, ms)):
        codes, offs = served_request_codes(k, refs[int(t)], int(m), length, seed, device="cuda")
        out.append((_pack_torch(codes), offs, int(m) * length))
    del refs
    return tids, out


def batch_sets_gpu(count: int = 64, ref_len: int = 10_000_000, min_reads: int = 1_000,
                   max_reads: int = 2_000_000, min_len: int = 36, max_len: int = 250,
                   sub_rate: float = 0.01, seed: int = SEED_BASE + 4):
    """Workload 4 drawn on the GPU: `count` independent sets, each with its own
    uniform random reference of ref_len bases and floor(exp(U(ln min_reads,
    ln max_reads))) reads (batch_set_codes, the same values the host draws).
    Returns a list of (packed device tensor, offsets device int64 tensor, bases)."""
    if sub_rate != 0.01:
        raise ValueError("the counter-based draws use a 1% substitution rate")
    ms = batch_sizes(count, min_reads, max_reads, seed)
    out = []
    for s, m in enumerate(ms):
        codes, offs = batch_set_codes(s, int(m), ref_len, min_len, max_len, seed, device="cuda")
        out.append((_pack_torch(codes), offs, int(offs[-1].item())))
        del codes
    return out
