"""The C-ABI library loads and exports every entry point declared in
include/bwtset.h.  No GPU work is started here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bwtset.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bwt_set_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1410_0562_amd import bwtset
    if not os.path.exists(bwtset.LIB_PATH):
        from paper_1410_0562_amd import build
        build.build()
    return bwtset.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("bwt_set_create", "bwt_set_append", "bwt_set_rank", "bwt_set_export"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1410_0562_amd import bwtset
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(bwtset.EXPORTED) == declared_functions()


def test_strerror_is_host_only(lib):
    assert lib.bwt_set_strerror(0) == b"ok"
    assert b"alphabet" in lib.bwt_set_strerror(-4)
    assert lib.bwt_set_strerror(-99) == b"unknown error"


def test_built_for_gfx950():
    from paper_1410_0562_amd import bwtset
    data = open(bwtset.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_product_does_not_import_oracle():
    # the GPU path must never route through the CPU oracle
    pkg = os.path.join(ROOT, "paper_1410_0562_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"(#|//).*", "", src).lower() or f == "synth.py", f
