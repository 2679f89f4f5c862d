"""The C-ABI library loads and exports every symbol include/krt.h declares (no
compute calls: these run without a GPU), and the product path is independent of
the oracle."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "krt.h")
LIB = os.path.join(ROOT, "paper_2608_09340_amd", "libkrt.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(krt_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["krt_create", "krt_destroy", "krt_last_error", "krt_grid_upload", "krt_tables_build",
              "krt_mc_run", "krt_levels_update"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkrt.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2608_09340_amd import krt
    assert sorted(krt.EXPORTS) == sorted(n for n in declared_functions())


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2608_09340_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "krt_oracle" not in txt and "orc_" not in txt, f


def test_oracle_shares_no_source_with_the_library():
    src = open(os.path.join(ROOT, "oracle", "krt_oracle.c")).read()
    assert "#include \"krt" not in src and "krt_internal" not in src


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2608_09340_amd import krt
    with pytest.raises(RuntimeError):
        krt.load.__wrapped__(str(tmp_path / "nope.so")) if hasattr(krt.load, "__wrapped__") else \
            _load_fresh(krt, str(tmp_path / "nope.so"))


def _load_fresh(krt, path):
    saved = krt._lib
    krt._lib = None
    try:
        return krt.load(path)
    finally:
        krt._lib = saved
