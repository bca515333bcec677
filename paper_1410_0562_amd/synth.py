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


def served_requests_gpu(tenants: int = 16, count: int = 512, ref_len: int = 100_000_000,
                        min_reads: int = 10_000, max_reads: int = 1_000_000, length: int = 150,
                        sub_rate: float = 0.01, seed: int = SEED_BASE + 5):
    """Workload 5 drawn on the GPU with torch: per-tenant uniform random
    references, `count` requests to uniformly drawn tenants with
    log-uniform read counts, reads sampled at uniform positions (forward
    strand) with i.i.d. substitutions.  Returns (tenant ids, list of
    (packed device tensor, offsets device int64 tensor, bases))."""
    import torch
    rng = np.random.default_rng(seed)
    tids = rng.integers(0, tenants, count)
    ms = np.floor(np.exp(rng.uniform(np.log(min_reads), np.log(max_reads), count))).astype(np.int64)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    refs = [torch.randint(0, 4, (ref_len,), dtype=torch.uint8, device="cuda", generator=gen)
            for _ in range(tenants)]
    ar = torch.arange(length, device="cuda", dtype=torch.int64)
    shifts = torch.tensor([0, 2, 4, 6], device="cuda", dtype=torch.uint8)
    out = []
    for t, m in zip(tids, ms):
        starts = torch.randint(0, ref_len - length + 1, (int(m),), device="cuda", generator=gen)
        codes = refs[int(t)][starts[:, None] + ar[None, :]].reshape(-1)
        hit = torch.rand(codes.shape, device="cuda", generator=gen) < sub_rate
        delta = torch.randint(1, 4, codes.shape, dtype=torch.uint8, device="cuda", generator=gen)
        codes = torch.where(hit, (codes + delta) & 3, codes)
        pad = (-codes.numel()) % 4
        if pad:
            codes = torch.cat([codes, torch.zeros(pad, dtype=torch.uint8, device="cuda")])
        packed = (codes.view(-1, 4) << shifts).sum(dim=1, dtype=torch.uint8)
        offs = torch.arange(int(m) + 1, device="cuda", dtype=torch.int64) * length
        out.append((packed, offs, int(m) * length))
    del refs
    return tids, out


def batch_sets_gpu(count: int = 64, ref_len: int = 10_000_000, min_reads: int = 1_000,
                   max_reads: int = 2_000_000, min_len: int = 36, max_len: int = 250,
                   sub_rate: float = 0.01, seed: int = SEED_BASE + 4):
    """Workload 4 drawn on the GPU with torch: `count` independent sets, each
    with its own uniform random reference of ref_len bases and
    floor(exp(U(ln min_reads, ln max_reads))) reads of uniform integer
    length in [min_len, max_len], sampled at uniform positions on a random
    strand (reverse complement for the minus strand) with i.i.d.
    substitutions to one of the other three bases.  Returns a list of
    (packed device tensor, offsets device int64 tensor, bases)."""
    import torch
    rng = np.random.default_rng(seed)
    ms = np.floor(np.exp(rng.uniform(np.log(min_reads), np.log(max_reads), count))).astype(np.int64)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    shifts = torch.tensor([0, 2, 4, 6], device="cuda", dtype=torch.uint8)
    out = []
    for m in ms:
        m = int(m)
        ref = torch.randint(0, 4, (ref_len,), dtype=torch.uint8, device="cuda", generator=gen)
        lens = torch.randint(min_len, max_len + 1, (m,), device="cuda", generator=gen)
        offs = torch.zeros(m + 1, dtype=torch.int64, device="cuda")
        torch.cumsum(lens, 0, out=offs[1:])
        total = int(offs[-1].item())
        starts = (torch.rand(m, device="cuda", generator=gen, dtype=torch.float64) *
                  (ref_len - lens + 1).to(torch.float64)).to(torch.int64)
        minus = torch.rand(m, device="cuda", generator=gen) < 0.5
        rid = torch.repeat_interleave(torch.arange(m, device="cuda"), lens)
        within = torch.arange(total, device="cuda", dtype=torch.int64) - offs[:-1][rid]
        fwd = starts[rid] + within
        rev = starts[rid] + lens[rid] - 1 - within
        mr = minus[rid]
        codes = ref[torch.where(mr, rev, fwd)]
        codes = torch.where(mr, 3 - codes, codes)
        del rid, within, fwd, rev, mr
        hit = torch.rand(total, device="cuda", generator=gen) < sub_rate
        delta = torch.randint(1, 4, (total,), dtype=torch.uint8, device="cuda", generator=gen)
        codes = torch.where(hit, (codes + delta) & 3, codes)
        del hit, delta
        pad = (-total) % 4
        if pad:
            codes = torch.cat([codes, torch.zeros(pad, dtype=torch.uint8, device="cuda")])
        packed = (codes.view(-1, 4) << shifts).sum(dim=1, dtype=torch.uint8)
        out.append((packed, offs, total))
        del ref, codes
    return out
