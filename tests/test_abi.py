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


def test_binding_structs_match_header_layout(tmp_path):
    """Every structure the binding mirrors has the header's size and the
    header's offset for each of its fields (a C program built against
    include/krt.h prints them; the binding's ctypes layout must agree)."""
    import shutil
    import subprocess
    from paper_2608_09340_amd import krt
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [krt.krt_grid_desc, krt.krt_line_desc, krt.krt_run_opts, krt.krt_tallies, krt.krt_levels_desc,
               krt.krt_image_desc, krt.krt_escape_cond]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "krt.h"', "int main(void) {"]
    for S in structs:
        name = S.__name__
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for fname, _ in S._fields_:
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    r = subprocess.run([cc, "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    got = {}
    for row in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        sname, field, value = row.split()
        got[(sname, field)] = int(value)
    for S in structs:
        name = S.__name__
        assert got[(name, "sizeof")] == ctypes.sizeof(S), name
        for fname, _ in S._fields_:
            assert got[(name, fname)] == getattr(S, fname).offset, (name, fname)
