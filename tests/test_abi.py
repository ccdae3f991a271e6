"""CPU-side checks of the C ABI library: it loads, exports every symbol that
include/gplhr.h declares, and validates host-visible arguments (no GPU work)."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_symbols():
    text = (ROOT / "include" / "gplhr.h").read_text()
    return sorted(set(re.findall(r"\b(gplhr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["gplhr_create", "gplhr_iterate", "gplhr_get_schur", "gplhr_eig_backward",
              "gplhr_destroy", "gplhr_last_error", "gplhr_spmm", "gplhr_csr_plane",
              "gplhr_gram", "gplhr_block_update", "gplhr_jacobi"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_1506_06829_amd import gplhr
    L = gplhr.lib()
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(gplhr.EXPORTS) <= set(declared_symbols())


def test_default_options():
    from paper_1506_06829_amd import gplhr
    L = gplhr.lib()
    o = gplhr._Options()
    L.gplhr_default_options(ctypes.byref(o))
    assert o.precision == 0 and o.tol == 1e-10 and o.max_iter == 500 and o.arnoldi_m == 1
    assert o.p_mode == 0 and o.switch_tol == 1e-8 and o.stall_window == 3


def test_argument_errors_without_device_work():
    from paper_1506_06829_amd import gplhr
    L = gplhr.lib()
    h = ctypes.c_void_p()
    # NULL A -> ERR_ARG, message available through gplhr_last_error(NULL)
    st = L.gplhr_create(None, None, 0.0, 0.0, 1, 1, None, None, ctypes.byref(h))
    assert st == -1 and h.value is None
    assert b"A must be" in L.gplhr_last_error(None)
    assert L.gplhr_create(None, None, 0.0, 0.0, 1, 1, None, None, None) == -1
    # bad block widths for the single-kernel entry points
    assert L.gplhr_spmm(0, 10, 0, None, None, None, None, 4, None, 4, 0, 0, None) == -1
    assert L.gplhr_spmm(0, 10, 0, None, None, None, None, 2, None, 4, 4, 0, None) == -1
    # the plane must divide n and be a multiple of 8
    assert L.gplhr_spmm(0, 48, 0, None, None, None, None, 4, None, 4, 4, 12, None) == -1
    assert L.gplhr_spmm(0, 40, 0, None, None, None, None, 4, None, 4, 4, 16, None) == -1
    assert L.gplhr_spmm(0, 40, 0, None, None, None, None, 4, None, 4, 4, -8, None) == -1
    # negative nnz
    assert L.gplhr_spmm(0, 10, -1, None, None, None, None, 4, None, 4, 4, 0, None) == -1
    # Jacobi: sweeps, omega, widths, nnz, plane
    for args in [(0, 10, 30, 0.7, 0, 4, 4, 4, 0), (0, 10, 30, 0.7, 65, 4, 4, 4, 0),
                 (0, 10, 30, 0.0, 3, 4, 4, 4, 0), (0, 10, 30, float("nan"), 3, 4, 4, 4, 0),
                 (0, 10, 30, 0.7, 3, 2, 4, 4, 0), (0, 10, 30, 0.7, 3, 4, 4, 65, 0),
                 (0, 10, -1, 0.7, 3, 4, 4, 4, 0), (2, 10, 30, 0.7, 3, 4, 4, 4, 0),
                 (0, 48, 30, 0.7, 3, 4, 4, 4, 12)]:
        dt, n, nnz, om, sw, ldr, ldy, b, plane = args
        assert L.gplhr_jacobi(dt, n, nnz, None, None, None, ctypes.c_double(om), sw, None, ldr,
                              None, ldy, b, plane, None) == -1
    assert b"gplhr_jacobi" in L.gplhr_last_error(None)
    assert L.gplhr_csr_plane(10, None, None, None, None) == -1
    assert L.gplhr_gram(0, 10, None, 4, 4, None, 4, 65, None, None) == -1
    # the allocation-free Gram rejects the same arguments before any device call
    assert L.gplhr_gram_noalloc(0, 10, None, 4, 4, None, 4, 65, None, None) == -1
    assert L.gplhr_gram_noalloc(0, 0, None, 4, 4, None, 4, 4, None, None) == -1
    assert L.gplhr_gram_noalloc(2, 10, None, 4, 4, None, 4, 4, None, None) == -1
    assert b"gplhr_gram_noalloc" in L.gplhr_last_error(None)
    for wx, wy in [(0, 4), (129, 4), (4, 0), (4, 49)]:
        assert L.gplhr_block_update(0, 10, None, 200, wx, None, 200, None, 200, wy,
                                    ctypes.c_double(0.0), ctypes.c_double(0.0), None) == -1
    # projection + Cholesky-QR: widths, passes, leading dimension, dtype, NULL block
    for dt, n, ld, wy, w, passes in [(0, 10, 64, 0, 0, 2), (0, 10, 64, 0, 49, 2),
                                     (0, 10, 64, 49, 8, 2), (0, 10, 64, 24, 48, 2),
                                     (0, 10, 64, 16, 16, 0), (0, 10, 64, 16, 16, 4),
                                     (0, 10, 31, 16, 16, 2), (2, 10, 64, 16, 16, 2),
                                     (0, 0, 64, 16, 16, 2)]:
        assert L.gplhr_proj_orth(dt, n, ctypes.c_void_p(16), ld, wy, w, passes, None) == -1
    assert L.gplhr_proj_orth(0, 10, None, 64, 16, 16, 2, None) == -1
    assert b"gplhr_proj_orth" in L.gplhr_last_error(None)
    assert L.gplhr_iterate(None, 1, None, None) == -1


def test_ctypes_structs_match_header(tmp_path):
    # a C probe compiled against the header prints sizeof and every field
    # offset; the ctypes mirrors of the binding must agree field by field
    import subprocess
    from paper_1506_06829_amd import gplhr
    structs = {"gplhr_csr": gplhr._Csr, "gplhr_precond": gplhr._Precond,
               "gplhr_options": gplhr._Options, "gplhr_stats": gplhr._Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gplhr.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", str(ROOT / "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
