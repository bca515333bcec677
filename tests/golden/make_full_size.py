"""Writes tests/golden/full_size_sha256.json: the SHA-256 of the oracle's BWT
of every benchmark workload at its full size.

Run from the repository root (hours of CPU for the served workload):

    python tests/golden/make_full_size.py [--threads N] [--only uniform,short,long,batched,served]

The inputs come from the seeded generators in paper_1410_0562_amd/synth.py
(the same draws the GPU tests and bench.py make), packed into the library's
2-bit input format, and unpacked again by the oracle's own reader.  The BWT is
the definition (Section 2, Eq. 1): one comparison sort of all suffixes of
T = S_0 $_0 ... S_{m-1} $_{m-1}, run as sorted runs merged pairwise on N
threads.  Nothing here loads the GPU library.

Entries are merged into the existing file, so workloads can be computed in
separate runs.  Each entry records the oracle's wall time, its thread count,
and the host it ran on.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle  # noqa: E402
from paper_1410_0562_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "full_size_sha256.json")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_sha(packed, offs, threads):
    """SHA-256 of the oracle BWT of (packed, offsets), with its size and time."""
    codes, o = oracle.reads_from_packed(packed, offs)
    T, _ = oracle.concat_text(codes, o)
    del codes
    t0 = time.perf_counter()
    B = oracle.bwt_from_text(T, threads=threads)
    dt = time.perf_counter() - t0
    return {"sha256": hashlib.sha256(B).hexdigest(), "symbols": len(B),
            "strings": len(o) - 1, "bases": int(o[-1]), "oracle_s": round(dt, 1)}


def concat_parts(parts):
    """(packed, offsets) of several (codes, offsets) parts laid end to end."""
    codes = np.concatenate([c for c, _ in parts]) if parts else np.zeros(0, np.uint8)
    lens = np.concatenate([np.diff(np.asarray(o, np.int64)) for _, o in parts]) \
        if parts else np.zeros(0, np.int64)
    offs = np.zeros(len(lens) + 1, np.uint64)
    offs[1:] = np.cumsum(lens)
    return synth.pack_codes(codes), offs


def load():
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def save(d):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)


def log(msg):
    print("[golden] " + msg, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default="uniform,short,long,batched,served")
    args = ap.parse_args()
    todo = set(args.only.split(","))
    th = args.threads
    d = load()
    d["host"] = {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "threads": th,
                 "numpy": np.__version__}

    if "uniform" in todo:
        log("uniform reads: 10,000 x 100 bp")
        d["uniform_10k"] = oracle_sha(*synth.uniform_reads(), th)
        save(d)
    if "short" in todo:
        log("short reads: 4,000,000 x 100 bp")
        d["short_reads_4M"] = oracle_sha(*synth.short_reads(), th)
        save(d)
        log("  %s" % d["short_reads_4M"])
    if "long" in todo:
        log("long reads: 250,000, lognormal lengths")
        d["long_reads_250k"] = oracle_sha(*synth.long_reads(threads=th), th)
        save(d)
        log("  %s" % d["long_reads_250k"])
    if "batched" in todo:
        ms = synth.batch_sizes()
        sets = []
        for s, m in enumerate(ms):
            codes, offs = synth.batch_set_codes(s, int(m))
            e = oracle_sha(synth.pack_codes(codes), offs.astype(np.uint64), th)
            del codes
            sets.append(e)
            log("  set %d: %d reads, %.1f s" % (s, int(m), e["oracle_s"]))
        d["batched_64_sets"] = sets
        save(d)
    if "served" in todo:
        tids, ms = synth.served_plan()
        tenants = []
        for t in range(16):
            ref = synth.served_reference(t)
            parts = []
            for k in np.flatnonzero(tids == t):
                parts.append(synth.served_request_codes(int(k), ref, int(ms[k])))
            e = oracle_sha(*concat_parts(parts), th)
            e["requests"] = int(len(parts))
            del parts, ref
            tenants.append(e)
            log("  tenant %d: %d requests, %d bases, %.1f s" % (t, e["requests"], e["bases"],
                                                                 e["oracle_s"]))
            d["served_16_tenants"] = tenants
            save(d)
    save(d)


if __name__ == "__main__":
    main()
