"""The C ABI: every symbol include/dualip.h declares is exported by the built
library, and the binding's structs match the header's layout (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dualip.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dl_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("dl_problem_create", "dl_problem_destroy", "dl_dual_grad", "dl_project", "dl_solve",
                 "dl_solver_create", "dl_solver_step", "dl_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2606_07777_amd as dl
    if not os.path.exists(dl.LIB_PATH):
        pytest.skip("libdualip.so not built")
    lib = ctypes.CDLL(dl.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(dl.SIGNATURES)


def test_struct_layouts_match_header():
    import paper_2606_07777_amd as dl
    src = f"""
#include <stddef.h>
#include <stdio.h>
#include "dualip.h"
int main(void) {{
  printf("%zu %zu %zu %zu %zu\\n", sizeof(dl_problem_desc), sizeof(dl_problem_info), sizeof(dl_solve_opts),
         sizeof(dl_solve_stats), sizeof(dl_timing));
  printf("%zu %zu %zu\\n", offsetof(dl_problem_desc, radius), offsetof(dl_problem_desc, stream),
         offsetof(dl_solve_opts, step_scale));
  return 0;
}}
"""
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(td, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe], text=True).split()
    sizes = [int(v) for v in out]
    assert sizes[:5] == [ctypes.sizeof(dl.dl_problem_desc), ctypes.sizeof(dl.dl_problem_info),
                         ctypes.sizeof(dl.dl_solve_opts), ctypes.sizeof(dl.dl_solve_stats),
                         ctypes.sizeof(dl.dl_timing)]
    assert sizes[5:] == [dl.dl_problem_desc.radius.offset, dl.dl_problem_desc.stream.offset,
                         dl.dl_solve_opts.step_scale.offset]


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_2606_07777_amd as dl
    saved = dl._lib
    dl._lib = None
    try:
        with pytest.raises(RuntimeError):
            dl.load(str(tmp_path / "missing.so"))
    finally:
        dl._lib = saved
