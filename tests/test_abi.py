"""The C-ABI library loads and exports every function include/lcs.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lcs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lcs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for f in ["lcs_solve_global", "lcs_build_local_domain", "lcs_solve_local",
              "lcs_solve_local_then_global"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2001_01158_amd import lcs
    if not os.path.exists(lcs.LIB_PATH):
        pytest.fail("liblcs.so is not built (python -m paper_2001_01158_amd.build)")
    L = lcs.load_library()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)
    assert sorted(lcs.EXPORTED) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2001_01158_amd import lcs
    with pytest.raises(ImportError):
        lcs.load_library(str(tmp_path / "missing.so"))


def test_default_options_without_gpu():
    from paper_2001_01158_amd import lcs
    L = lcs.load_library()
    o = lcs._Options()
    L.lcs_default_options(ctypes.byref(o))
    assert o.eps == 1e-10 and o.precond == lcs.PC_JACOBI and o.n_smooth == 1


def test_ctypes_structs_match_the_header_layout(tmp_path):
    """sizeof and every field offset of the structs the binding mirrors, as
    gcc lays them out from include/lcs.h."""
    import shutil
    import subprocess
    from paper_2001_01158_amd import lcs
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"lcs_matrix": lcs._Matrix, "lcs_options": lcs._Options, "lcs_stats": lcs._Stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lcs.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
