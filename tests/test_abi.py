"""The C-ABI library loads on the host and exports every function that
include/fgfft.h declares (no device calls)."""
import os
import re

from paper_2411_16583_amd import fgfft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fgfft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_lists_the_binding_functions():
    assert declared_functions() == sorted(fgfft.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = fgfft.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_argument_errors_without_device():
    lib = fgfft.load_library()
    assert lib.fg_status_string(fgfft.FG_E_SIZE) == b"unsupported size"
    import ctypes
    out = ctypes.c_void_p()
    g = (ctypes.c_int * 3)(16, 16, 10)  # N2/2 = 5 is not a supported length
    h = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert lib.fg_plan_create(g, h, 0, None, ctypes.byref(out)) == fgfft.FG_E_SIZE
    g = (ctypes.c_int * 3)(16, 16, 16)
    h = (ctypes.c_double * 3)(1.0, -1.0, 1.0)
    assert lib.fg_plan_create(g, h, 0, None, ctypes.byref(out)) == fgfft.FG_E_ARG
    assert lib.fg_plan_workspace_bytes(None) == 0
