"""The C ABI library loads on the host, exports every symbol include/psfd.h
declares, matches the binding's struct layout, and rejects bad arguments
before touching any device memory.  No compute call is made (no GPU here)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psfd.h")


@pytest.fixture(scope="module")
def L():
    from paper_2607_25330_amd import psfd
    return psfd.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(psfd_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for need in ["psfd_plan", "psfd_apply", "psfd_precond", "psfd_solve", "psfd_adjoint",
                 "psfd_rhs", "psfd_destroy", "psfd_last_error"]:
        assert need in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_struct_layout_matches_c(tmp_path):
    from paper_2607_25330_amd.psfd import Desc, Info
    prog = tmp_path / "layout.c"
    fields = [f for f, _ in Desc._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "psfd.h"', 'int main(void){',
             'printf("%zu %zu\\n", sizeof(psfd_desc), sizeof(psfd_info));']
    for f in fields:
        cf = "lambda" if f == "lambda_" else f
        lines.append(f'printf("%zu\\n", offsetof(psfd_desc, {cf}));')
    lines.append("return 0;}")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(Desc)
    assert int(out[1]) == ctypes.sizeof(Info)
    for f, off in zip(fields, out[2:]):
        assert getattr(Desc, f).offset == int(off), f


def test_invalid_arguments_return_err_arg(L):
    from paper_2607_25330_amd import psfd
    from psfd_synth import config_c1
    h = ctypes.c_void_p()
    assert L.psfd_plan(None, None, None, ctypes.byref(h)) == psfd.PSFD_ERR_ARG
    assert b"NULL" in L.psfd_last_error()
    d, keep = psfd.make_desc(config_c1())
    for field, bad in [("nx", 20), ("ny", 0), ("nz_gap_bot", 0), ("pol", 2), ("prec", 7),
                       ("dz", -1.0), ("nz_abs", 9)]:
        d2, keep2 = psfd.make_desc(config_c1())
        setattr(d2, field, bad)
        st = L.psfd_plan(ctypes.byref(d2), ctypes.c_void_p(1), None, ctypes.byref(h))
        assert st == psfd.PSFD_ERR_ARG, field
    assert L.psfd_apply(None, None, None) == psfd.PSFD_ERR_ARG
    assert L.psfd_solve(None, None, None, None, ctypes.c_double(1e-6), 10, 0, None) == psfd.PSFD_ERR_ARG
    assert L.psfd_layout_eps(ctypes.byref(d), None, None, ctypes.c_double(1.0), None, None) == psfd.PSFD_ERR_ARG
    assert L.psfd_layered_eps(ctypes.byref(d), 0, None, None, None, None) == psfd.PSFD_ERR_ARG
    neg = (ctypes.c_double * 2)(2.0, 0.0)
    thick = (ctypes.c_double * 1)(-1.0)
    assert L.psfd_layered_eps(ctypes.byref(d), 1, neg, thick, ctypes.c_void_p(1), None) == psfd.PSFD_ERR_ARG
    assert L.psfd_specular(None, None, None) == psfd.PSFD_ERR_ARG
    one = ctypes.c_void_p(1)
    assert L.psfd_contour_segments(None, 64, 64, 1, 4096, 1.0, 1.0, 10, 0.15, 0.05, 8, one, one,
                                   None) == psfd.PSFD_ERR_ARG
    assert L.psfd_contour_segments(one, 2048, 64, 1, 2048 * 64, 1.0, 1.0, 10, 0.15, 0.05, 8, one,
                                   one, None) == psfd.PSFD_ERR_ARG
    assert L.psfd_contour_segments(one, 64, 64, 1, 100, 1.0, 1.0, 10, 0.15, 0.05, 8, one, one,
                                   None) == psfd.PSFD_ERR_ARG
    st5 = (ctypes.c_double * 5)()
    assert L.psfd_contour_deviation(one, one, one, one, 64, 64, 1, 1.0, 1.0, 10, 8, 0.0, 1.0, one,
                                    st5, None) == psfd.PSFD_ERR_ARG
    assert L.psfd_field_size(None) == 0
    L.psfd_destroy(None)
