"""C-ABI checks that need no GPU: the library loads, exports every entry point that
include/fot.h declares, and rejects invalid plans before touching the device."""
import ctypes
import os

import pytest

from paper_2512_19072_amd import fot as F


def test_library_exists_and_loads():
    assert os.path.exists(F.LIB_PATH), "build libfot.so first (python -m paper_2512_19072_amd.build)"
    F.load()


def test_exports_every_header_symbol():
    lib = F.load()
    names = F.header_functions()
    assert set(names) >= {"fot_plan", "fot_solve", "fot_potentials", "fot_backward", "fot_destroy",
                          "fot_last_error", "fot_version"}
    for name in names:
        assert hasattr(lib, name), f"{name} declared in fot.h but not exported"


def test_version_string():
    assert "gfx950" in F.fot_version()


@pytest.mark.parametrize("desc, msg", [
    ((0, 1, 1, 10, 0, 0), "n must be"),
    ((9000, 1, 1, 10, 0, 0), "n must be"),
    ((64, 0, 1, 10, 0, 0), "batch"),
    ((64, 1, 7, 10, 0, 0), "precision"),
    ((64, 1, 1, 0, 0, 0), "max_iters"),
    ((64, 1, 1, 10, -1, 0), "checkpoint_every"),
    ((64, 1, 1, 10, 0, 128), "flag bits"),
])
def test_plan_rejects_invalid_desc(desc, msg):
    lib = F.load()
    d = F.fot_plan_desc(*desc)
    h = ctypes.c_void_p()
    st = lib.fot_plan(ctypes.byref(d), None, ctypes.byref(h))
    assert st == F.FOT_E_INVALID
    assert msg in F.fot_last_error()
    assert h.value is None


def test_null_arguments_are_rejected():
    lib = F.load()
    assert lib.fot_plan(None, None, None) == F.FOT_E_INVALID
    assert lib.fot_solve(None, None, None, None, 1, 1, 0, None, None) == F.FOT_E_INVALID
    assert lib.fot_potentials(None, None, None, None, None) == F.FOT_E_INVALID
    assert lib.fot_backward(None, None, None, None) == F.FOT_E_INVALID
    assert lib.fot_output_beam(None, None, None, None, None, None) == F.FOT_E_INVALID
    assert lib.fot_polish_gs(None, None, None, None, 1) == F.FOT_E_INVALID
    assert lib.fot_destroy(None) == F.FOT_E_INVALID


def test_header_structs_match_binding():
    """Field order of the ctypes structs follows the header."""
    text = open(F.HEADER).read()
    for field, _ in F.fot_plan_desc._fields_:
        assert field in text
    for field, _ in F.fot_report._fields_:
        assert field in text


def test_header_enum_values_match_binding():
    """Every FOT_* constant that fot.h defines with an explicit value has the same value in the
    Python binding (statuses, precisions, flags)."""
    import re
    text = open(F.HEADER).read()
    pairs = re.findall(r"\b(FOT_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)
    assert len(pairs) >= 15
    for name, val in pairs:
        assert getattr(F, name) == int(val), name
    assert F.PRECISIONS["bf16x3"] == F.FOT_BF16X3


@pytest.mark.parametrize("desc, msg", [
    ((64, 1, 1, 10, 0, 8), "FOT_F64"),             # cFOT with FP32 operands
    ((64, 1, 0, 10, 5, 8), "reverse mode"),        # cFOT with a tape
    ((3000, 1, 0, 10, 0, 8), "n <= 2048"),         # FFT length beyond 4096
])
def test_cfot_plan_limits(desc, msg):
    lib = F.load()
    d = F.fot_plan_desc(*desc)
    h = ctypes.c_void_p()
    st = lib.fot_plan(ctypes.byref(d), None, ctypes.byref(h))
    assert st == F.FOT_E_UNSUPPORTED
    assert msg in F.fot_last_error()
    assert h.value is None
