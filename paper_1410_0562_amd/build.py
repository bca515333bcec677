"""Builds libbwtset.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1410_0562_amd.build

Every .hip / .cpp file under csrc/ is compiled to an object with
``--offload-arch=gfx950`` and linked into ``paper_1410_0562_amd/libbwtset.so``.
Packed FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libbwtset.so")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC, "-I", INCLUDE,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def build(verbose: bool = False, jobs: int = 8) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sources()
    objs = []
    procs = []
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        lang = ["-x", "hip"]
        cmd = [hipcc] + COMMON + lang + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    while procs:
        _wait(procs.pop(0))
    fd, tmp = tempfile.mkstemp(prefix="libbwtset.", suffix=".so.tmp", dir=HERE)
    os.close(fd)
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode != 0:
        os.unlink(tmp)
        raise RuntimeError("link failed:\n" + out.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    build_random_reads(hipcc, verbose)
    return LIB


# The random-read rate benchmark beside bench.py (the ceiling of the LF walks).
RANDOM_READS_SRC = os.path.join(os.path.dirname(HERE), "bench_random_reads.hip")
RANDOM_READS_BIN = os.path.join(os.path.dirname(HERE), "bench_random_reads")


def build_random_reads(hipcc: str, verbose: bool = False) -> str:
    cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=" + ARCH,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           RANDOM_READS_SRC, "-o", RANDOM_READS_BIN + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (RANDOM_READS_SRC,
                                                      out.stdout.decode(errors="replace")))
    os.replace(RANDOM_READS_BIN + ".tmp", RANDOM_READS_BIN)
    return RANDOM_READS_BIN


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    # hipcc's host pass does not know the device-only feature flag; that is harmless
    lines = [ln for ln in text.splitlines()
             if "packed-fp32-ops" not in ln and ln.strip() != "1 warning generated."
             and ln.strip() != "1 warning generated"]
    if p.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (src, text))
    if any(ln.strip() for ln in lines):
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
