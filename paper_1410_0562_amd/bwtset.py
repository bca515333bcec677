"""Python binding of libbwtset (C ABI in include/bwtset.h).

Argument marshalling only: every step of the BWT construction runs in the HIP
kernels of the library.  Host inputs are numpy arrays; device inputs and
outputs are torch tensors on a ROCm device (torch is used for device memory
and streams only).  The library must have been built
(``python -m paper_1410_0562_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbwtset.so")

BWT_OK = 0
BWT_EINVAL = -1
BWT_ENOMEM = -2
BWT_EHIP = -3
BWT_EALPHABET = -4
BWT_ESTATE = -5

STAGES = ("plan", "sort", "ranks", "gather", "insert")
U64_MAX = (1 << 64) - 1


class Stats(ctypes.Structure):
    _fields_ = [
        ("ms", ctypes.c_double * 5),
        ("launches", ctypes.c_uint64 * 5),
        ("ranks_kernel_ms", ctypes.c_double),
        ("ranks_launches", ctypes.c_uint64),
        ("ranks_steps", ctypes.c_uint64),
        ("insert_kernel_ms", ctypes.c_double),
        ("insert_launches", ctypes.c_uint64),
        ("insert_records_out", ctypes.c_uint64),
        ("insert_records_in", ctypes.c_uint64),
        ("insert_new_symbols", ctypes.c_uint64),
        ("sort_pass_ms", ctypes.c_double),
        ("sort_pass_launches", ctypes.c_uint64),
        ("sort_pass_keys", ctypes.c_uint64),
        ("blocks", ctypes.c_uint64),
        ("doubling_rounds", ctypes.c_uint64),
        ("keys_ms", ctypes.c_double),
        ("heads_ms", ctypes.c_double),
        ("refine_ms", ctypes.c_double),
        ("tied_suffixes", ctypes.c_uint64),
        ("fallback_blocks", ctypes.c_uint64),
        ("bucket_ms", ctypes.c_double),
        ("ranks_seg_ms", ctypes.c_double),
        ("ranks_seg_launches", ctypes.c_uint64),
        ("ranks_fb_ms", ctypes.c_double),
        ("tile_sort_ms", ctypes.c_double),
        ("tile_sort_launches", ctypes.c_uint64),
        ("tile_sort_keys", ctypes.c_uint64),
        ("insert_old_symbols", ctypes.c_uint64),
        ("insert_terminators", ctypes.c_uint64),
        ("ranks_retries", ctypes.c_uint64),
        ("ranks_fallback_reads", ctypes.c_uint64),
        ("ranks_seg_symbols", ctypes.c_uint64),
        ("graph_captures", ctypes.c_uint64),
        ("graph_replays", ctypes.c_uint64),
        ("graph_redos", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name in ("ms", "launches"):
                d[name] = {s: v[i] for i, s in enumerate(STAGES)}
            else:
                d[name] = v
        return d


EXPORTED = [
    "bwt_set_create", "bwt_set_destroy", "bwt_set_append", "bwt_set_rank",
    "bwt_set_rank_many", "bwt_set_export", "bwt_set_size", "bwt_set_reset",
    "bwt_set_set_block_size", "bwt_set_last_error", "bwt_set_strerror",
    "bwt_set_block_sort", "bwt_set_compute_ranks", "bwt_set_insert",
    "bwt_set_enable_timing", "bwt_set_get_stats", "bwt_set_set_param",
    "bwt_set_import", "bwt_set_memory", "bwt_set_trim", "bwt_set_append_many",
    "bwt_set_block_sort_noalloc", "bwt_set_count_many", "bwt_set_append_strands",
    "bwt_set_autotune",
]
BWT_STRAND_FORWARD = 0
BWT_STRAND_REVERSE = 1
BWT_STRAND_BOTH = 2
BWT_PARAM_KEY_BITS = 1
BWT_PARAM_RADIX_TILE = 2
BWT_PARAM_RANK_SEGMENT = 3
BWT_PARAM_RANK_OVERLAP = 4
BWT_PARAM_BATCH_LANES = 5
BWT_PARAM_SORT_BUCKETS = 6
BWT_PARAM_GRAPH = 7
BWT_PARAM_HOST_INDEX = 8
BWT_PARAM_PIPELINE = 9

_lib = None


def load(path: str = LIB_PATH):
    """Load libbwtset.so and declare its signatures (no GPU call is made)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libbwtset.so is not built (%s); run python -m paper_1410_0562_amd.build"
                          % path)
    L = ctypes.CDLL(path)
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    L.bwt_set_create.argtypes = [ctypes.c_char_p]
    L.bwt_set_create.restype = vp
    L.bwt_set_destroy.argtypes = [vp]
    L.bwt_set_destroy.restype = None
    L.bwt_set_append.argtypes = [vp, vp, vp, u64, vp]
    L.bwt_set_append.restype = i32
    L.bwt_set_rank.argtypes = [vp, ctypes.c_char, u64]
    L.bwt_set_rank.restype = u64
    L.bwt_set_rank_many.argtypes = [vp, vp, vp, vp, u64, vp]
    L.bwt_set_rank_many.restype = i32
    L.bwt_set_export.argtypes = [vp, vp]
    L.bwt_set_export.restype = ctypes.c_int64
    L.bwt_set_size.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    L.bwt_set_size.restype = i32
    L.bwt_set_reset.argtypes = [vp]
    L.bwt_set_reset.restype = i32
    L.bwt_set_set_block_size.argtypes = [vp, u64]
    L.bwt_set_set_block_size.restype = i32
    L.bwt_set_last_error.argtypes = [vp]
    L.bwt_set_last_error.restype = i32
    L.bwt_set_strerror.argtypes = [i32]
    L.bwt_set_strerror.restype = ctypes.c_char_p
    L.bwt_set_block_sort.argtypes = [vp, vp, vp, u64, vp, vp, vp]
    L.bwt_set_block_sort.restype = i32
    L.bwt_set_block_sort_noalloc.argtypes = [vp, vp, vp, u64, vp, vp, vp]
    L.bwt_set_block_sort_noalloc.restype = i32
    L.bwt_set_count_many.argtypes = [vp, vp, vp, u64, vp, vp, vp]
    L.bwt_set_count_many.restype = i32
    L.bwt_set_append_strands.argtypes = [vp, vp, vp, u64, i32, vp]
    L.bwt_set_append_strands.restype = i32
    L.bwt_set_autotune.argtypes = [vp, vp, vp, u64, i32, ctypes.POINTER(Tune)]
    L.bwt_set_autotune.restype = i32
    L.bwt_set_compute_ranks.argtypes = [vp, vp, vp, u64, vp, vp]
    L.bwt_set_compute_ranks.restype = i32
    L.bwt_set_insert.argtypes = [vp, vp, vp, u64, vp]
    L.bwt_set_insert.restype = i32
    L.bwt_set_enable_timing.argtypes = [vp, i32]
    L.bwt_set_enable_timing.restype = i32
    L.bwt_set_get_stats.argtypes = [vp, ctypes.POINTER(Stats), i32]
    L.bwt_set_get_stats.restype = i32
    L.bwt_set_set_param.argtypes = [vp, i32, ctypes.c_int64]
    L.bwt_set_set_param.restype = i32
    L.bwt_set_import.argtypes = [vp, vp, u64, vp]
    L.bwt_set_import.restype = i32
    L.bwt_set_memory.argtypes = [vp, ctypes.POINTER(u64)]
    L.bwt_set_memory.restype = i32
    L.bwt_set_trim.argtypes = [vp]
    L.bwt_set_trim.restype = i32
    L.bwt_set_append_many.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(u64), u64, vp]
    L.bwt_set_append_many.restype = i32
    if path == LIB_PATH:
        _lib = L
    return L


class Tune(ctypes.Structure):
    _fields_ = [("radix_tile", ctypes.c_int), ("key_bits", ctypes.c_int),
                ("rank_segment", ctypes.c_uint32), ("rank_overlap", ctypes.c_uint32),
                ("from_cache", ctypes.c_int), ("ms", ctypes.c_double), ("trials", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class BwtSetError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = load().bwt_set_strerror(code).decode()
        super().__init__("%s%s (%d)" % (what + ": " if what else "", msg, code))


def _ptr(x) -> int:
    """Address of a numpy array (host) or a torch tensor (device or host)."""
    if x is None:
        return 0
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError("expected a numpy array or a torch tensor, got %r" % type(x))


def _stream(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _len(x) -> int:
    return int(x.numel()) if hasattr(x, "numel") else int(x.size)


def _as_offsets(offsets):
    if isinstance(offsets, np.ndarray):
        return np.ascontiguousarray(offsets, dtype=np.uint64)
    import torch
    if offsets.dtype not in (torch.int64, torch.uint64):
        raise TypeError("device offsets must be int64 or uint64")
    return offsets.contiguous()


def _as_reads(reads):
    if isinstance(reads, np.ndarray):
        return np.ascontiguousarray(reads, dtype=np.uint8)
    return reads.contiguous()


class BwtSet:
    """One incremental BWT index on the current GPU."""

    def __init__(self, alphabet: str = "ACGT", block_size: Optional[int] = None):
        L = load()
        h = L.bwt_set_create(alphabet.encode("ascii"))
        if not h:
            raise BwtSetError(L.bwt_set_last_error(None), "bwt_set_create")
        self._h = h
        if block_size is not None:
            self.set_block_size(block_size)

    # -- lifecycle
    def close(self) -> None:
        if getattr(self, "_h", None):
            load().bwt_set_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc: int, what: str) -> int:
        if rc < 0:
            raise BwtSetError(int(rc), what)
        return rc

    # -- the ABI
    def set_block_size(self, M: int) -> None:
        self._check(load().bwt_set_set_block_size(self._h, int(M)), "bwt_set_set_block_size")

    def set_key_bits(self, bits: int) -> None:
        self.set_param(BWT_PARAM_KEY_BITS, bits)

    def set_param(self, param: int, value: int) -> None:
        self._check(load().bwt_set_set_param(self._h, int(param), int(value)), "bwt_set_set_param")

    def append(self, reads, offsets, stream=None) -> None:
        """Append m = len(offsets) - 1 reads (2-bit packed, see synth.py)."""
        reads = _as_reads(reads)
        offsets = _as_offsets(offsets)
        m = _len(offsets) - 1
        if m <= 0:
            return
        self._check(load().bwt_set_append(self._h, _ptr(reads), _ptr(offsets), m, _stream(stream)),
                    "bwt_set_append")

    def append_strands(self, reads, offsets, mode: int, stream=None) -> None:
        """Append the reads reversed (BWT_STRAND_REVERSE) or each followed by
        its reverse complement (BWT_STRAND_BOTH)."""
        reads = _as_reads(reads)
        offsets = _as_offsets(offsets)
        m = _len(offsets) - 1
        if m <= 0:
            return
        self._check(load().bwt_set_append_strands(self._h, _ptr(reads), _ptr(offsets), m,
                                                  int(mode), _stream(stream)),
                    "bwt_set_append_strands")

    def autotune(self, reads, offsets, force: bool = False) -> dict:
        """Pick the fastest tuning knobs for this input's shape class (see
        bwt_set_autotune) and apply them; returns the choice."""
        reads = _as_reads(reads)
        offsets = _as_offsets(offsets)
        t = Tune()
        self._check(load().bwt_set_autotune(self._h, _ptr(reads), _ptr(offsets),
                                            _len(offsets) - 1, 1 if force else 0,
                                            ctypes.byref(t)), "bwt_set_autotune")
        return t.as_dict()

    def rank(self, c: str, k: int) -> int:
        r = load().bwt_set_rank(self._h, c.encode("ascii"), int(k))
        if r == U64_MAX:
            raise BwtSetError(load().bwt_set_last_error(self._h), "bwt_set_rank")
        return int(r)

    def rank_many(self, cs, ks, out, stream=None) -> None:
        """Device tensors: cs uint8 (ASCII), ks int64, out int64 (same length)."""
        self._check(load().bwt_set_rank_many(self._h, _ptr(cs), _ptr(ks), _ptr(out), _len(ks),
                                             _stream(stream)), "bwt_set_rank_many")

    def count_many(self, pats, offsets, lo_out, hi_out, stream=None) -> None:
        """FM-index count: device tensors pats (2-bit packed uint8), offsets
        (int64, count + 1), lo_out / hi_out (int64, count)."""
        offsets = _as_offsets(offsets)
        self._check(load().bwt_set_count_many(self._h, _ptr(pats), _ptr(offsets),
                                              _len(offsets) - 1, _ptr(lo_out), _ptr(hi_out),
                                              _stream(stream)), "bwt_set_count_many")

    def size(self) -> tuple:
        n, m = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(load().bwt_set_size(self._h, ctypes.byref(n), ctypes.byref(m)), "bwt_set_size")
        return int(n.value), int(m.value)

    def export(self, out=None):
        """B as bytes, or written into `out` (a uint8 device tensor or numpy array)."""
        L = load()
        n = self._check(L.bwt_set_export(self._h, None), "bwt_set_export")
        if out is None:
            buf = np.empty(n, dtype=np.uint8)
            if n:
                self._check(L.bwt_set_export(self._h, _ptr(buf)), "bwt_set_export")
            return buf.tobytes()
        if _len(out) < n:
            raise ValueError("output too small: %d < %d" % (_len(out), n))
        self._check(L.bwt_set_export(self._h, _ptr(out)), "bwt_set_export")
        return out

    def reset(self) -> None:
        self._check(load().bwt_set_reset(self._h), "bwt_set_reset")

    def import_bwt(self, B, stream=None) -> None:
        """Load the index whose BWT is B (bytes, numpy uint8 array or device tensor)."""
        if isinstance(B, (bytes, bytearray)):
            B = np.frombuffer(bytes(B), dtype=np.uint8)
        self._check(load().bwt_set_import(self._h, _ptr(B) if _len(B) else None, _len(B),
                                          _stream(stream)), "bwt_set_import")

    def memory(self) -> int:
        b = ctypes.c_uint64()
        self._check(load().bwt_set_memory(self._h, ctypes.byref(b)), "bwt_set_memory")
        return int(b.value)

    def trim(self) -> None:
        self._check(load().bwt_set_trim(self._h), "bwt_set_trim")

    # -- single steps
    def block_sort(self, reads, offsets, sa_out, bint_out, stream=None) -> None:
        reads = _as_reads(reads)
        offsets = _as_offsets(offsets)
        self._check(load().bwt_set_block_sort(self._h, _ptr(reads), _ptr(offsets), _len(offsets) - 1,
                                              _ptr(sa_out), _ptr(bint_out), _stream(stream)),
                    "bwt_set_block_sort")

    def block_sort_noalloc(self, reads, offsets, sa_out, bint_out, stream=None) -> None:
        """block_sort on the library's fixed per-GPU workspace (no device
        allocation; device buffers only, at most 2^18 suffixes)."""
        self._check(load().bwt_set_block_sort_noalloc(self._h, _ptr(reads), _ptr(offsets),
                                                      _len(offsets) - 1, _ptr(sa_out),
                                                      _ptr(bint_out), _stream(stream)),
                    "bwt_set_block_sort_noalloc")

    def compute_ranks(self, reads, offsets, g_out, stream=None) -> None:
        reads = _as_reads(reads)
        offsets = _as_offsets(offsets)
        self._check(load().bwt_set_compute_ranks(self._h, _ptr(reads), _ptr(offsets),
                                                 _len(offsets) - 1, _ptr(g_out), _stream(stream)),
                    "bwt_set_compute_ranks")

    def insert(self, bint, gsa, stream=None) -> None:
        self._check(load().bwt_set_insert(self._h, _ptr(bint), _ptr(gsa), _len(bint),
                                          _stream(stream)), "bwt_set_insert")

    # -- timing
    def enable_timing(self, on: bool = True) -> None:
        self._check(load().bwt_set_enable_timing(self._h, 1 if on else 0), "bwt_set_enable_timing")

    def stats(self, reset: bool = False) -> dict:
        st = Stats()
        self._check(load().bwt_set_get_stats(self._h, ctypes.byref(st), 1 if reset else 0),
                    "bwt_set_get_stats")
        return st.as_dict()


def append_many(sets, reads_list, offsets_list, stream=None) -> None:
    """Batched form: sets[i].append(reads_list[i], offsets_list[i]) for every
    i, run as one schedule on sets[0]'s workspace and parameters (see
    bwt_set_append_many).  Same result on every set as one append each."""
    n = len(sets)
    if n != len(reads_list) or n != len(offsets_list):
        raise ValueError("sets, reads and offsets must have the same length")
    if n == 0:
        return
    reads_list = [_as_reads(r) for r in reads_list]
    offsets_list = [_as_offsets(o) for o in offsets_list]
    vp = ctypes.c_void_p
    hs = (vp * n)(*[s._h for s in sets])
    rp = (vp * n)(*[_ptr(r) for r in reads_list])
    op = (vp * n)(*[_ptr(o) for o in offsets_list])
    ms = (ctypes.c_uint64 * n)(*[max(_len(o) - 1, 0) for o in offsets_list])
    rc = load().bwt_set_append_many(hs, rp, op, ms, n, _stream(stream))
    if rc != 0:
        raise BwtSetError(rc, "bwt_set_append_many")
