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


def _fake_matrix(lcs, kind, nx, ny, nz, with32=False):
    """A matrix description with placeholder device addresses: the workspace
    size is host arithmetic and never dereferences them."""
    m = lcs._Matrix(kind, nx, ny, nz, ctypes.c_void_p(0x10000), None)
    if with32:
        m.coef32 = ctypes.c_void_p(0x20000)
    if kind == lcs.CSR:
        m.row_ptr, m.col, m.val = ctypes.c_void_p(0x30000), ctypes.c_void_p(0x40000), ctypes.c_void_p(0x50000)
        m.nnz = 5 * nx
    return m


def test_workspace_bytes_without_gpu():
    """lcs_workspace_bytes is host arithmetic: the fixed head plus every
    buffer of the path at K = N, each rounded up to 256 bytes.  Its per-row
    cost matches the buffers the path uses (FP64 PCG: nine FP64 vectors,
    domain and restricted ELL of width W; mixed: FP32 vectors and the FP32
    copy of B), and invalid input gives 0."""
    from paper_2001_01158_amd import lcs
    L = lcs.load_library()
    o = lcs._Options()
    L.lcs_default_options(ctypes.byref(o))

    def nbytes(m, opts):
        return L.lcs_workspace_bytes(ctypes.byref(m), ctypes.byref(opts) if opts is not None else None)

    head = nbytes(_fake_matrix(lcs, lcs.STENCIL5_2D, 1, 1, 1), o)
    n = 1 << 20
    b5 = nbytes(_fake_matrix(lcs, lcs.STENCIL5_2D, 1024, 1024, 1), o)
    # per row: score 8, stamp 1, inv 4, idx 4, B (W = 5) 5 x 12, diag 8, colour 1,
    # rhs 8, rowlen 4, local correction 8, nine FP64 PCG vectors 72
    per_row = 8 + 1 + 4 + 4 + 5 * 12 + 8 + 1 + 8 + 4 + 8 + 72
    assert abs((b5 - head) - per_row * n) < 64 * 1024, (b5 - head) / n
    om = lcs._Options()
    L.lcs_default_options(ctypes.byref(om))
    om.precision = lcs.PREC_MIXED
    b9m = nbytes(_fake_matrix(lcs, lcs.STENCIL9_2D, 1024, 1024, 1, with32=True), om)
    # ... plus the second buffer of the nine-point paired-colour sweeps
    per_row = 8 + 1 + 4 + 4 + 9 * 12 + 8 + 1 + 8 + 4 + 8 + 9 * 4 + 4 + 8 + 11 * 4 + 8
    assert abs((b9m - head) - per_row * n) < 64 * 1024, (b9m - head) / n
    # without a caller FP32 copy the library casts the five arrays itself
    b9c = nbytes(_fake_matrix(lcs, lcs.STENCIL9_2D, 1024, 1024, 1), om)
    assert abs((b9c - b9m) - 5 * 4 * n) < 4096
    # general sparse input counts B and its own ELL copy at the largest width,
    # 64 (indices, values, diagonal, colour)
    bc = nbytes(_fake_matrix(lcs, lcs.CSR, n, 1, 1), o)
    per_row = 8 + 1 + 4 + 4 + 64 * 12 + 8 + 1 + 8 + 4 + 8 + 72 + 64 * 4 + 65 * 8 + 1
    assert abs((bc - head) - per_row * n) < 64 * 1024, (bc - head) / n
    assert nbytes(_fake_matrix(lcs, lcs.STENCIL5_2D, 1024, 1024, 1), None) == b5
    # batched: four FP64 vectors, stamps and indices per cell and system, plus results
    G = 64
    bb = L.lcs_workspace_bytes_batched(ctypes.byref(_fake_matrix(lcs, lcs.STENCIL9_2D, 88, 80, 1)), G,
                                       ctypes.byref(o))
    assert abs((bb - head) - G * 7040 * (32 + 1 + 4)) < 64 * 1024
    bad = _fake_matrix(lcs, lcs.STENCIL5_2D, 0, 4, 1)
    assert nbytes(bad, o) == 0
    assert L.lcs_workspace_bytes_batched(ctypes.byref(_fake_matrix(lcs, lcs.STENCIL5_2D, 8, 8, 1)), 0,
                                         ctypes.byref(o)) == 0
