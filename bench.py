"""Benchmark: incremental BWT construction (set-bwte, Algorithm 1) on one GPU.

One step = build the index of a whole workload from empty, every stage of the
hot path -- suffix sort, ComputeRanks, g_sa, Insert with the occurrence-counter
rebuild -- over all of its blocks.  Inputs are resident in HBM before the
timed region.  Prints one JSON line.

The headline is the largest plain workload that fits one GPU: 250,000 long
reads, lognormal lengths (mean 5 kbp, clipped to 1-50 kbp) from a random 100
Mbp reference with 10% noise, about 1.25 Gbp in blocks of M = 2^27 suffixes.
The short-read workload (4,000,000 x 100 bp from a random 50 Mbp reference,
both strands, 1% substitutions, M = 2^26) is measured after it and reported
under "also".

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload long|short|uniform]
    python bench.py --batched | --served
"""
import argparse
import hashlib
import json
import subprocess
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "input bases indexed/sec (incremental BWT) + HBM GB/s fraction; p99 append latency"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
# Algorithmic bytes: what the method must move, over-fetch excluded.
RANKS_BYTES_PER_STEP = 64 + 4 + 0.25   # one 64-byte rank record, a 4-byte rank, one 2-bit base
RADIX_BYTES_PER_KEY = 24               # read and write a 64-bit key and a 32-bit value
TILE_SORT_BYTES_PER_KEY = 25           # the same, plus one tie-flag byte written
# Insert per launch: n_ext/4 read + n_out/4 written (2-bit symbols) + n_out/8
# (occurrence counters at one bit per symbol) + 5 per new symbol (4-byte g_sa,
# one B_int byte) + 8 per new terminator (its position)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
GOLDEN_FILE = os.path.join(ROOT, "tests", "golden", "full_size_sha256.json")
CPU_THREADS_MAX = 16                    # the host share of one GPU on the box
COPY_BYTES = 1 << 30                    # the calibration copy (--calibrate-copy)

WORKLOADS = {
    # name: (key in the traffic and golden files, default block, description)
    "long": ("long_reads_250k", 1 << 27,
             "long reads: %d reads, lognormal lengths (mean 5 kbp, 1-50 kbp) from a random "
             "100 Mbp reference, both strands, 10%% noise; block M=%d suffixes"),
    "short": ("short_reads_4M", 1 << 26,
              "short reads: %d x 100 bp from a random 50 Mbp reference, both strands, 1%% "
              "substitutions; block M=%d suffixes"),
    "uniform": ("uniform_10k", 1 << 18,
                "uniform reads: %d x 100 bp i.i.d.; block M=%d suffixes"),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


_COMMON = ["paper_1410_0562_amd/csrc/dev_util.hpp", "paper_1410_0562_amd/csrc/bwt_internal.hpp"]
KERNEL_SOURCES = {
    "compute_ranks_kernel": ["paper_1410_0562_amd/csrc/k_ranks.hip"] + _COMMON,
    "rank_segments_kernel": ["paper_1410_0562_amd/csrc/k_ranks.hip"] + _COMMON,
    "radix_pass_kernel": ["paper_1410_0562_amd/csrc/k_radix.hip"] + _COMMON,
    "insert_kernel": ["paper_1410_0562_amd/csrc/k_insert.hip"] + _COMMON,
    "bucket_tile_sort_kernel": ["paper_1410_0562_amd/csrc/k_bucket.hip"] + _COMMON,
}


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary, or None when there is none or the kernel source
    changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("source_digest") != source_digest(KERNEL_SOURCES[kernel]):
        return None
    return e.get("bytes_per_launch")


def _kernel_base(full):
    """Short kernel name (no return type, namespace, template or arguments)
    and the name with its template arguments."""
    s = full.replace("(anonymous namespace)::", "").split("(")[0].strip()
    if s.startswith("void "):
        s = s[5:]
    s = s.replace("bwt::", "")
    return s.split("<")[0].split("::")[-1].strip(), s


def _csv_rows(folder, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(folder, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit("no *%s under %s" % (suffix, folder))
    return rows


def _counter_per_kernel(folder, counter):
    """{kernel base name: (dispatches, summed counter value)} from one
    rocprofv3 --pmc run."""
    acc = {}
    for r in _csv_rows(folder, "counter_collection.csv"):
        if r.get("Counter_Name", counter) != counter:
            continue
        base, _ = _kernel_base(r["Kernel_Name"])
        n, v = acc.get(base, (0, 0.0))
        acc[base] = (n + 1, v + float(r["Counter_Value"]))
    return acc


def summarize_profile(root, workload, command_note):
    """Turns the rocprofv3 output of one workload into the committed
    summaries: <key>_kernel_stats.md (kernel trace), <key>_hbm_traffic.md and
    the workload's entry of profiles/traffic.json (FETCH_SIZE and WRITE_SIZE
    per dispatch, scaled by what the same counters read for a plain 1 GiB
    device copy).  root holds the runs' folders: stats/, fetch/, write/,
    copy_fetch/, copy_write/."""
    key = WORKLOADS[workload][0]
    prof = os.path.join(ROOT, "profiles")
    rows = _csv_rows(os.path.join(root, "stats"), "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel time per kernel, %s" % key, "",
             "Commands (`$R` = the repository root where they ran):", "", "```", command_note.strip(),
             "```", "", "| kernel | calls | total ms | avg us | min us | max us | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        _, name = _kernel_base(r["Name"])
        lines.append("| %s | %d | %.2f | %.1f | %.1f | %.1f | %.1f |" % (
            name, int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    with open(os.path.join(prof, key + "_kernel_stats.md"), "w") as f:
        f.write("\n".join(lines) + "\n")

    fetch = _counter_per_kernel(os.path.join(root, "fetch"), "FETCH_SIZE")
    write = _counter_per_kernel(os.path.join(root, "write"), "WRITE_SIZE")
    cf = _counter_per_kernel(os.path.join(root, "copy_fetch"), "FETCH_SIZE")
    cw = _counter_per_kernel(os.path.join(root, "copy_write"), "WRITE_SIZE")
    copy = [k for k in cf if "copyBuffer" in k]
    if not copy or copy[0] not in cw:
        raise SystemExit("no copy kernel in the calibration runs")
    n, v = cf[copy[0]]
    f_scale = COPY_BYTES / (v / n * 1024)          # bytes per counter KiB, reads
    n, v = cw[copy[0]]
    w_scale = COPY_BYTES / (v / n * 1024)          # bytes per counter KiB, writes
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        t = {}
    t = {k: v for k, v in t.items() if isinstance(v, dict) and k in
         {w[0] for w in WORKLOADS.values()}}
    entry = {"_note": "HBM bytes per launch, one index build of the workload: FETCH_SIZE x %.3f "
                      "+ WRITE_SIZE x %.3f (KiB x 1024), the factors being what a plain 1 GiB "
                      "device copy reads on the same counters" % (f_scale, w_scale)}
    table = ["# HBM traffic per kernel launch, %s" % key, "",
             "Commands (`$R` = the repository root where they ran; each counter in a run of its own):",
             "", "```", command_note.strip(), "```", "",
             "Scale: a plain 1 GiB device copy reads FETCH_SIZE x 1024 x %.3f and WRITE_SIZE x "
             "1024 x %.3f bytes per launch." % (f_scale, w_scale), "",
             "| kernel | launches | fetch MB/launch | write MB/launch | total MB/launch |",
             "|---|---:|---:|---:|---:|"]
    order = sorted(fetch, key=lambda k: -(fetch[k][1] * f_scale +
                                          write.get(k, (1, 0.0))[1] * w_scale))
    for k in order:
        nf, vf = fetch[k]
        nw, vw = write.get(k, (nf, 0.0))
        fb = vf / nf * 1024 * f_scale
        wb = vw / max(nw, 1) * 1024 * w_scale
        table.append("| %s | %d | %.1f | %.1f | %.1f |" % (k, nf, fb / 1e6, wb / 1e6,
                                                          (fb + wb) / 1e6))
        if k in KERNEL_SOURCES:
            entry[k] = {"launches": nf, "fetch_bytes_per_launch": int(fb),
                        "write_bytes_per_launch": int(wb), "bytes_per_launch": int(fb + wb),
                        "source_digest": source_digest(KERNEL_SOURCES[k])}
    t[key] = entry
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
        f.write("\n")
    with open(os.path.join(prof, key + "_hbm_traffic.md"), "w") as f:
        f.write("\n".join(table) + "\n")


def summarize_overlap(folder, command_note, out_name):
    """From a rocprofv3 kernel trace: how much of the time kernels of
    different HIP streams ran at the same moment on the device (the served
    form's batches on their own streams).  Writes profiles/<out_name>.md."""
    rows = _csv_rows(folder, "kernel_trace.csv")
    ev = []
    for r in rows:
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if b > a:
            sid = (r.get("Queue_Id"), r.get("Stream_Id"))
            ev.append((a, 1, sid))
            ev.append((b, -1, sid))
    ev.sort(key=lambda e: (e[0], e[1]))
    active = {}
    t_prev = ev[0][0]
    busy = multi = 0
    hist = {}
    for t, d, sid in ev:
        nact = sum(1 for v in active.values() if v > 0)
        dt = t - t_prev
        if nact >= 1:
            busy += dt
        if nact >= 2:
            multi += dt
        hist[nact] = hist.get(nact, 0) + dt
        active[sid] = active.get(sid, 0) + d
        t_prev = t
    span = ev[-1][0] - ev[0][0]
    streams = {sid for _, _, sid in ev}
    lines = ["# Kernels of different streams running at once: %s" % out_name, "",
             "Commands (`$R` = the repository root where they ran):", "", "```",
             command_note.strip(), "```", "",
             "Kernel dispatches: %d on %d streams.  Span from the first kernel start to the last "
             "kernel end: %.1f ms; time with at least one kernel running: %.1f ms; time with "
             "kernels of two or more streams running at once: %.1f ms (%.1f%% of the busy time)."
             % (len(rows), len(streams), span / 1e6, busy / 1e6, multi / 1e6,
                100.0 * multi / max(busy, 1)), "",
             "| streams with a kernel running | ms | share of busy time |", "|---:|---:|---:|"]
    for k in sorted(hist):
        if k >= 1:
            lines.append("| %d | %.1f | %.1f%% |" % (k, hist[k] / 1e6, 100.0 * hist[k] / max(busy, 1)))
    with open(os.path.join(ROOT, "profiles", out_name + ".md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(packed, offs, sample_bases, golden_key):
    """The oracle (a comparison sort of all suffixes, Section 2's order, then
    Eq. 1) on the host cores, on the first reads of the workload holding about
    sample_bases bases."""
    import numpy as np
    from oracle import oracle
    from paper_1410_0562_amd import synth
    offs = np.asarray(offs, dtype=np.uint64)
    nreads = int(np.searchsorted(offs, np.uint64(int(offs[0]) + sample_bases), side="right")) - 1
    nreads = max(1, min(len(offs) - 1, nreads))
    p, o = synth.take_reads(packed, offs, 0, nreads)
    codes, oo = oracle.reads_from_packed(p, o)
    T, _ = oracle.concat_text(codes, oo)
    del codes
    bases = int(oo[-1])
    threads = max(1, min(CPU_THREADS_MAX, os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.bwt_from_text(T, threads=threads)
    dt = time.perf_counter() - t0
    out = {"value": bases / dt, "unit": "bases/s", "cores": threads, "kind": "oracle",
           "sample": "first %d reads (%d bases) of the same workload; comparison sort of all "
                     "suffixes as %d sorted runs merged pairwise (%.1f s)"
                     % (nreads, bases, threads, dt),
           "nproc": os.cpu_count(), "cpu_model": cpu_model()}
    try:
        with open(GOLDEN_FILE) as f:
            g = json.load(f)
        e = g.get(golden_key)
        if e:
            host = g.get("host", {})
            out["full_size"] = {"oracle_s": e["oracle_s"], "bases": e["bases"],
                                "bases_per_s": e["bases"] / e["oracle_s"],
                                "threads": host.get("threads"), "cpu_model": host.get("cpu_model"),
                                "note": "the whole workload, timed when its parity digest was "
                                        "written (tests/golden/make_full_size.py)"}
    except (OSError, ValueError, KeyError):
        pass
    return out


def run_batched(args, torch, bwtset, synth):
    """Batched form: `sets` independent read sets appended to fresh indices,
    one bwt_set_append_many call per step, timed beside the plain loop of one
    bwt_set_append per set on the same GPU.  Both build the same indices (the
    exports are compared on the device).  Prints one JSON line."""
    block = args.block or (1 << 26)
    log("generating %d sets on the GPU" % args.sets)
    lo_r, hi_r = (1000, 2_000_000)
    if args.set_reads:
        lo_r, hi_r = (int(x) for x in args.set_reads.split(","))
    sets = synth.batch_sets_gpu(count=args.sets, min_reads=lo_r, max_reads=hi_r)
    torch.cuda.synchronize()
    bases = sum(b for _, _, b in sets)
    reads = sum(int(o.numel()) - 1 for _, o, _ in sets)
    reads_l = [p for p, _, _ in sets]
    offs_l = [o for _, o, _ in sets]
    hb = [bwtset.BwtSet(block_size=block) for _ in sets]
    hl = [bwtset.BwtSet(block_size=block) for _ in sets]
    if args.lanes is not None:
        hb[0].set_param(bwtset.BWT_PARAM_BATCH_LANES, args.lanes)
    if args.graph:
        hb[0].set_param(bwtset.BWT_PARAM_GRAPH, 1)
    for h in hb + hl:
        if args.key_bits is not None:
            h.set_key_bits(args.key_bits)
        if args.radix_tile is not None:
            h.set_param(bwtset.BWT_PARAM_RADIX_TILE, args.radix_tile)

    def timed(run, hs):
        total = 0.0
        for k in range(args.warmup + args.steps):
            for h in hs:
                h.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            if k >= args.warmup:
                total += time.perf_counter() - t0
        return total

    def batched():
        bwtset.append_many(hb, reads_l, offs_l)

    def loop():
        for h, p, o in zip(hl, reads_l, offs_l):
            h.append(p, o)

    t_batch = timed(batched, hb)
    log("batched: %.3f s for %d steps" % (t_batch, args.steps))
    t_loop = timed(loop, hl)
    log("per-set loop: %.3f s for %d steps" % (t_loop, args.steps))
    same = 0
    for a, b in zip(hb, hl):
        n = a.size()[0]
        assert n == b.size()[0]
        ea = torch.empty(n, dtype=torch.uint8, device="cuda")
        eb = torch.empty(n, dtype=torch.uint8, device="cuda")
        a.export(ea)
        b.export(eb)
        same += bool(torch.equal(ea, eb))
        del ea, eb
    assert same == len(sets), "batched and per-set indices differ"
    for h in hb + hl:
        h.close()
    v_batch = bases * args.steps / t_batch
    v_loop = bases * args.steps / t_loop
    out = {
        "metric": METRIC,
        "value": v_batch,
        "unit": "bases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "batched: %d independent sets, each from its own random 10 Mbp "
                               "reference, %d-%d reads per set (log-uniform), 36-250 bp, both "
                               "strands, 1%% substitutions; block M=%d suffixes" % (
                                   len(sets), lo_r, hi_r, block),
                   "sets": len(sets), "reads": reads, "bases": bases, "block_suffixes": block,
                   "lanes": args.lanes, "graph": bool(args.graph)},
        "batched": {"per_set_loop_bases_per_s": v_loop,
                    "per_set_loop_ms_per_step": t_loop / args.steps * 1e3,
                    "speedup_vs_per_set_loop": v_batch / v_loop,
                    "identical_indices": same},
    }
    print(json.dumps(out), flush=True)


def run_served(args, torch, bwtset, synth):
    """Served form: tenants' append requests arrive as a Poisson process at
    `load` times the measured single-stream capacity; a continuous-batching
    service (paper_1410_0562_amd.serve) runs them.  Prints one JSON line."""
    import numpy as np
    from paper_1410_0562_amd.serve import BwtService
    tenants = 16
    log("generating %d requests on the GPU" % args.requests)
    tids, reqs = synth.served_requests_gpu(tenants=tenants, count=args.requests)
    torch.cuda.synchronize()
    mean_bases = float(np.mean([b for _, _, b in reqs]))
    # single-stream capacity: one fresh index, requests appended back to back
    log("measuring single-stream capacity")
    cal = bwtset.BwtSet(block_size=1 << 26)
    cal_reqs = sorted(reqs, key=lambda r: r[2])[len(reqs) // 2: len(reqs) // 2 + 4]
    cal.append(cal_reqs[0][0], cal_reqs[0][1])  # warm the workspace
    cal.reset()
    t0 = time.perf_counter()
    nb = 0
    for p, o, b in cal_reqs:
        cal.append(p, o)
        nb += b
    torch.cuda.synchronize()
    capacity = nb / (time.perf_counter() - t0)
    cal.close()
    rate = args.load * capacity / mean_bases       # requests per second
    rng = np.random.default_rng(14100562 + 55)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
    svc = BwtService(tenants, budget_bytes=int(args.budget_gb * (1 << 30)), workers=args.workers,
                     block_size=1 << 26)
    log("serving %d requests at %.1f req/s" % (len(reqs), rate))
    t_start = time.perf_counter()
    for k, ((p, o, b), t) in enumerate(zip(reqs, tids)):
        delay = t_start + arrivals[k] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        svc.submit(int(t), p, o)
        if k % 64 == 63:
            log("submitted %d" % (k + 1))
    svc.drain(timeout=600)
    summ = svc.latency_summary()
    svc.close()
    out = {
        "metric": METRIC,
        "value": summ["bases_per_s"],
        "unit": "bases/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": (max(r.finish for r in svc.completed) - t_start) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "served: %d tenants with random 100 Mbp references, %d append "
                               "requests of 10k-1M reads (log-uniform) x 150 bp, 1%% "
                               "substitutions, Poisson arrivals at %.0f%% of single-stream "
                               "capacity; %g GB budget, %d workers" % (
                                   tenants, len(reqs), args.load * 100, args.budget_gb,
                                   args.workers)},
        "served": {"p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"], "mean_ms": summ["mean_ms"],
                   "requests": summ["requests"], "errors": summ["errors"],
                   "spills": summ["spills"], "restores": summ["restores"], "trims": summ["trims"],
                   "single_stream_bases_per_s": capacity, "arrival_rate_per_s": rate},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["short", "long", "uniform"], default="long",
                    help="long: 250k lognormal reads, mean 5 kbp, M = 2^27 (default, the "
                         "headline); short: 4M x 100 bp, M = 2^26; uniform: 10k x 100 bp, "
                         "M = 2^18")
    ap.add_argument("--no-also", action="store_true",
                    help="with the long workload: skip the short-read measurement after it")
    ap.add_argument("--reads", type=int, default=None)
    ap.add_argument("--block", type=int, default=None)
    ap.add_argument("--key-bits", type=int, default=None,
                    help="width of the first suffix-sort key (library default if omitted)")
    ap.add_argument("--radix-tile", type=int, default=None,
                    help="radix pass tile shape (library default if omitted)")
    ap.add_argument("--graph", action="store_true",
                    help="capture each append in a HIP graph and replay it (BWT_PARAM_GRAPH)")
    ap.add_argument("--host-input", action="store_true",
                    help="pass the reads from host memory (the host-to-device copy is timed)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="with --host-input: copy all reads before the first block")
    ap.add_argument("--host-index", action="store_true",
                    help="keep the index in pinned host memory (BWT_PARAM_HOST_INDEX)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner on the workload first (untimed)")
    ap.add_argument("--cpu-sample-bases", type=int, default=None,
                    help="bases of the oracle's sample (default: a sixth of the workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-random", action="store_true",
                    help="run bench_random_reads (dependent random reads per second, the "
                         "ceiling of the LF walks) and print its table")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (for scaling HBM counters)")
    ap.add_argument("--summarize-profile", metavar="DIR", default=None,
                    help="no GPU work: write profiles/ summaries for --workload from the "
                         "rocprofv3 runs under DIR (stats/, fetch/, write/, copy_fetch/, "
                         "copy_write/)")
    ap.add_argument("--summarize-overlap", metavar="DIR", default=None,
                    help="no GPU work: write profiles/served_16_tenants_overlap.md from the "
                         "rocprofv3 kernel trace under DIR")
    ap.add_argument("--profile-commands", metavar="FILE", default=None,
                    help="with --summarize-profile: text file holding the commands that made "
                         "the runs")
    ap.add_argument("--served", action="store_true",
                    help="served form: 16 tenants, Poisson append requests (p50/p99 latency)")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--budget-gb", type=float, default=100.0)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--load", type=float, default=0.7,
                    help="offered load as a fraction of the single-stream capacity")
    ap.add_argument("--batched", action="store_true",
                    help="batched form: 64 independent sets in one call, against one append "
                         "per set")
    ap.add_argument("--sets", type=int, default=64)
    ap.add_argument("--lanes", type=int, default=None,
                    help="batched form: blocks run side by side (library default if omitted)")
    ap.add_argument("--set-reads", type=str, default=None,
                    help="batched form: MIN,MAX reads per set (default 1000,2000000)")
    args = ap.parse_args()
    if args.summarize_overlap:
        note = open(args.profile_commands).read() if args.profile_commands else ""
        summarize_overlap(args.summarize_overlap, note, "served_16_tenants_overlap")
        return
    if args.summarize_profile:
        note = open(args.profile_commands).read() if args.profile_commands else ""
        summarize_profile(args.summarize_profile, args.workload, note)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the per-block path runs on a single MI355X "
              "(how it would shard across GPUs is described in the design notes, not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1410_0562_amd import bwtset, synth

    if not os.path.exists(bwtset.LIB_PATH):
        from paper_1410_0562_amd import build
        build.build()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_random:
        from paper_1410_0562_amd import build as hipbuild
        if not os.path.exists(hipbuild.RANDOM_READS_BIN):
            print("bench_random_reads is not built; run __graft_entry__.build()", file=sys.stderr)
            sys.exit(2)
        sys.exit(subprocess.run([hipbuild.RANDOM_READS_BIN]).returncode)

    if args.calibrate_copy:
        # a plain copy of known size: the HBM byte counters read on it give the
        # factor between counter units and bytes moved (1 GiB read + 1 GiB written)
        src = torch.ones(COPY_BYTES, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 3}))
        return

    if args.served:
        return run_served(args, torch, bwtset, synth)
    if args.batched:
        return run_batched(args, torch, bwtset, synth)

    res = run_plain(args, torch, bwtset, synth, args.workload, args.steps, args.warmup,
                    cpu=not args.no_cpu_baseline)
    if not args.no_also and args.workload == "long":
        log("also: the short-read workload")
        extra = run_plain(args, torch, bwtset, synth, "short", args.steps, args.warmup, cpu=False)
        res["also"] = {"short_reads_4M": {k: extra[k] for k in (
            "value", "unit", "ms_per_step", "config", "roofline", "kernels", "stages_ms_per_step")}}
    print(json.dumps(res), flush=True)


def run_plain(args, torch, bwtset, synth, workload, steps, warmup, cpu=True):
    """Whole builds of one plain workload; returns the JSON object."""
    import numpy as np
    key, default_block, wdesc = WORKLOADS[workload]
    own = workload == args.workload          # --block / --reads apply to the headline only
    block = (args.block if own else None) or default_block
    nreads = args.reads if own else None
    log("generating the %s workload" % workload)
    if workload == "short":
        packed, offs = synth.short_reads(m=nreads or 4_000_000)
    elif workload == "long":
        packed, offs = synth.long_reads(m=nreads or 250_000, threads=CPU_THREADS_MAX)
    else:
        packed, offs = synth.uniform_reads(m=nreads or 10_000)
    bases = int(offs[-1]) - int(offs[0])
    m = len(offs) - 1
    if args.host_input and own:
        dev_reads, dev_offs = packed, offs          # host buffers: staged by the library
    else:
        dev_reads = torch.from_numpy(packed).cuda()
        dev_offs = torch.from_numpy(offs.view(np.int64)).cuda()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    idx = bwtset.BwtSet(block_size=block)
    if args.graph and own:
        idx.set_param(bwtset.BWT_PARAM_GRAPH, 1)
    if args.host_index and own:
        idx.set_param(bwtset.BWT_PARAM_HOST_INDEX, 1)
    if args.no_pipeline and own:
        idx.set_param(bwtset.BWT_PARAM_PIPELINE, 0)
    if args.key_bits is not None:
        idx.set_key_bits(args.key_bits)
    if args.radix_tile is not None:
        idx.set_param(bwtset.BWT_PARAM_RADIX_TILE, args.radix_tile)
    tune = None
    if args.autotune and own:
        tune = idx.autotune(dev_reads, dev_offs)
        log("autotune: %s" % tune)
    for w in range(warmup):
        idx.reset()
        idx.append(dev_reads, dev_offs, stream)
        log("warmup %d done" % w)
    # the timed steps run without per-kernel events; the same steps are then
    # run again with them for the kernel and stage breakdown
    idx.stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        idx.reset()
        idx.append(dev_reads, dev_offs, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    graph_replays = idx.stats(reset=True)["graph_replays"]
    n, mm = idx.size()
    assert n == bases + m and mm == m
    dt = t1 - t0
    log("timed %d steps in %.3f s" % (steps, dt))
    if args.graph and own:
        # captured appends record no per-kernel events: the breakdown comes
        # from the same steps run eagerly
        idx.set_param(bwtset.BWT_PARAM_GRAPH, 0)
    idx.enable_timing(True)
    for k in range(steps):
        idx.reset()
        idx.append(dev_reads, dev_offs, stream)
    torch.cuda.synchronize()
    st = idx.stats()
    idx.enable_timing(False)

    # LF steps: every base of every block with an index to rank against; the
    # library counts those of the reads its segment kernel walked
    seg_steps = st["ranks_seg_symbols"]
    main_steps = st["ranks_steps"] - seg_steps
    kernels = {}
    if st["ranks_launches"]:
        kernels["compute_ranks_kernel"] = (st["ranks_kernel_ms"], st["ranks_launches"],
                                           main_steps * RANKS_BYTES_PER_STEP)
    if st["ranks_seg_launches"] and seg_steps:
        kernels["rank_segments_kernel"] = (st["ranks_seg_ms"], st["ranks_seg_launches"],
                                           seg_steps * RANKS_BYTES_PER_STEP)
    if st["sort_pass_launches"]:
        kernels["radix_pass_kernel"] = (st["sort_pass_ms"], st["sort_pass_launches"],
                                        st["sort_pass_keys"] * RADIX_BYTES_PER_KEY)
    if st["tile_sort_launches"]:
        kernels["bucket_tile_sort_kernel"] = (st["tile_sort_ms"], st["tile_sort_launches"],
                                              st["tile_sort_keys"] * TILE_SORT_BYTES_PER_KEY)
    if st["insert_launches"]:
        n_old, n_new = st["insert_old_symbols"], st["insert_new_symbols"]
        kernels["insert_kernel"] = (
            st["insert_kernel_ms"], st["insert_launches"],
            n_old / 4 + (n_old + n_new) / 4 + (n_old + n_new) / 8 + 5 * n_new +
            8 * st["insert_terminators"])
    kinfo = {}
    for name, (ms, launches, nbytes) in kernels.items():
        gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        kinfo[name] = {"ms_per_step": ms / steps, "launches_per_step": launches / steps,
                       "avg_launch_ms": ms / launches, "bytes_per_launch": nbytes / launches,
                       "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
        if name in ("compute_ranks_kernel", "rank_segments_kernel") and ms > 0:
            # each LF step is one dependent read of a random 64-byte record:
            # compare with `bench.py --calibrate-random`
            kinfo[name]["lf_steps_G_per_s"] = nbytes / RANKS_BYTES_PER_STEP / (ms * 1e-3) / 1e9
    if kinfo:
        dom = max(kinfo, key=lambda k: kinfo[k]["ms_per_step"])
        d = kinfo[dom]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(d["achieved_GBs"], 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(d["frac"], 4),
                    "traffic": measured_traffic(key, dom)}
    else:
        roofline = None
    out = {
        "metric": METRIC,
        "value": bases * steps / dt,
        "unit": "bases/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": dt / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": wdesc % (m, block),
                   "reads": m, "bases": bases, "block_suffixes": block,
                   "blocks": st["blocks"] // steps, "key_bits": args.key_bits,
                   "radix_tile": args.radix_tile, "graph": bool(args.graph and own),
                   "graph_replays": graph_replays, "autotune": tune,
                   "host_index": bool(args.host_index and own),
                   "host_input": bool(args.host_input and own),
                   "pipeline": not (args.no_pipeline and own)},
        "roofline": roofline,
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in kinfo.items()},
        "stages_ms_per_step": {s: round(st["ms"][s] / steps, 3) for s in bwtset.STAGES},
        "sort_detail_ms_per_step": {
            "keys": round(st["keys_ms"] / steps, 3),
            "radix_passes": round(st["sort_pass_ms"] / steps, 3),
            "tie_detection": round(st["heads_ms"] / steps, 3),
            "bucket_finish": round(st["bucket_ms"] / steps, 3),
            "refine": round(st["refine_ms"] / steps, 3)},
        "ranks_detail_ms_per_step": {
            "read_walks": round(st["ranks_kernel_ms"] / steps, 3),
            "segment_walks": round(st["ranks_seg_ms"] / steps, 3),
            "fallback_and_counts": round(st["ranks_fb_ms"] / steps, 3),
            "segment_retries": st["ranks_retries"] / steps,
            "whole_read_fallbacks": st["ranks_fallback_reads"] / steps},
        "tied_fraction": st["tied_suffixes"] / float(steps * (bases + m)),
        "fallback_blocks_per_step": st["fallback_blocks"] / steps,
        "doubling_rounds_per_step": st["doubling_rounds"] / steps,
    }
    idx.close()
    del dev_reads, dev_offs
    torch.cuda.empty_cache()
    if cpu:
        sample = args.cpu_sample_bases or max(1, bases // 6)
        log("timing the CPU oracle on a sample of %d bases" % sample)
        out["cpu_baseline"] = cpu_baseline(packed, offs, sample, key)
    else:
        out["cpu_baseline"] = None
    return out


if __name__ == "__main__":
    main()
