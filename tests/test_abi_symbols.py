"""CPU checks of the boundary: libcib.so loads and exports every function that
include/cib.h declares; the Python binding lists the same set; the host-side
argument checks reject bad calls without touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2110_10765_amd import cib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cib.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(cib_[a-z_A-Z0-9]+)\s*\(", txt))
    # typedef'd function-pointer members are not functions
    return sorted(n for n in names)


def test_library_exports_every_declared_function():
    lib = cib.load()
    declared = header_functions()
    assert declared, "no functions parsed from cib.h"
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", cib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (cib_\w+)", out))
    assert set(declared) <= exported
    assert set(declared) == set(cib.EXPORTS)


def test_null_arguments_are_rejected():
    lib = cib.load()
    h = ctypes.c_void_p()
    assert lib.cib_build_basis(None, None, ctypes.byref(h), None) == cib.CIB_E_INVALID
    assert b"NULL" in lib.cib_last_error()
    assert lib.cib_apply_H(None, None, None, 1, None, 1, 1) == cib.CIB_E_INVALID
    assert lib.cib_matrix_info(None, None, None, None) == cib.CIB_E_INVALID
    # free functions accept NULL
    lib.cib_basis_free(None)
    lib.cib_matrix_free(None)
    lib.cib_destroy(None)


def test_status_codes_match_header():
    txt = open(HEADER).read()
    for name, val in re.findall(r"#define (CIB_E?_?[A-Z_]+) \(?(-?\d+)\)?", txt):
        assert getattr(cib, name) == int(val), name


def test_missing_library_fails_loudly():
    """No CPU fallback: without the built library every entry point raises."""
    code = ("import paper_2110_10765_amd.cib as c\n"
            "try:\n"
            "    c.load('/nonexistent/libcib.so')\n"
            "except RuntimeError as e:\n"
            "    print('raised', 'not found' in str(e))\n")
    out = subprocess.run(["python", "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert "raised True" in out.stdout, out.stdout + out.stderr
