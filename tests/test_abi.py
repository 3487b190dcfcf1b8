"""The C-ABI library loads and exports every entry point of include/imrt.h
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

from paper_0908_4421_amd import imrt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "imrt.h")


def declared_functions():
    text = open(HEADER).read()
    return re.findall(r"IMRT_API\s+(?:const\s+)?\w+\s*\*?\s*(imrt_\w+)\s*\(", text)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("imrt_build_dose_matrix", "imrt_set_structures", "imrt_set_penalties",
                     "imrt_evaluate_objective", "imrt_gradient", "imrt_project", "imrt_solve"):
        assert required in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(imrt.LIB_PATH):
        pytest.skip("libimrt.so not built")
    lib = imrt.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_the_header_with_the_same_names():
    names = set(declared_functions())
    assert names == set(imrt.SIGNATURES)
    for name in names:
        assert callable(getattr(imrt, name)), name


STRUCTS = ("imrt_penalty", "imrt_geometry", "imrt_solve_params", "imrt_trace_entry", "imrt_solve_result",
           "imrt_request", "imrt_serve_times")


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Size and every field offset of each ctypes structure equal what the C
    compiler gives for the declaration in include/imrt.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "imrt.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(imrt, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            cfield = "lambda" if field == "lambda_" else field
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {cfield}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, stdout=subprocess.PIPE, text=True).stdout.split("\n")
    for line in filter(None, out):
        name, field, value = line.split()
        cls = getattr(imrt, name)
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(value), line


def test_host_side_argument_errors_without_device_work():
    """Validation that happens before any HIP call returns IMRT_EINVAL."""
    if not os.path.exists(imrt.LIB_PATH):
        pytest.skip("libimrt.so not built")
    lib = imrt.load()
    assert lib.imrt_ctx_create(0, None, None) == imrt.IMRT_EINVAL
    assert lib.imrt_dose_info(None, None, None, None) == imrt.IMRT_EINVAL
    assert "NULL" in imrt.last_error()
    assert lib.imrt_plan_create(None, None, None) == imrt.IMRT_EINVAL
    assert lib.imrt_solve(None, None, None, None) == imrt.IMRT_EINVAL
    assert lib.imrt_evaluate_objective(None, None, None, None) == imrt.IMRT_EINVAL
    # destroying NULL handles is a no-op
    assert lib.imrt_ctx_destroy(None) == imrt.IMRT_OK
    assert lib.imrt_dose_destroy(None) == imrt.IMRT_OK
    assert lib.imrt_plan_destroy(None) == imrt.IMRT_OK
