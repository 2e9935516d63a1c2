"""CPU checks of the C-ABI library: it loads and exports every entry point
include/sparstencil.h declares (no compute calls without a GPU), and the
binding's structures match the header's."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparstencil.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sparstencil_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def native():
    from paper_2506_22969_amd import native as n
    if not os.path.exists(n.LIB_PATH):
        pytest.fail("libsparstencil.so is not built (run __graft_entry__.build())")
    return n


def test_every_declared_symbol_is_exported(native):
    lib = ctypes.CDLL(native.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    assert set(native.EXPORTS) <= set(names)


def test_status_strings(native):
    assert native.status_string(0) == "ok"
    assert native.status_string(-1) == "invalid argument"
    assert native.status_string(-2) == "unsupported"
    assert native.status_string(12345) == "unknown status"


def test_struct_sizes_match_header(native):
    # ss_plan_opts: 7 x 4-byte fields; ss_plan_info: 18 int32, 2 doubles, 3 int64
    assert ctypes.sizeof(native.PlanOpts) == 28
    assert ctypes.sizeof(native.PlanInfo) == 18 * 4 + 2 * 8 + 3 * 8


def test_null_arguments_rejected_without_device(native):
    # argument validation happens before any HIP call
    lib = native.lib()
    h = ctypes.c_void_p()
    assert lib.sparstencil_plan(ctypes.byref(h), 0, 1, None, 2, None, 3, None) == native.SS_E_INVALID
    assert lib.sparstencil_run(None, None, None, 1, None) == native.SS_E_INVALID
    assert lib.sparstencil_plan_destroy(None) == native.SS_OK
    assert lib.sparstencil_launch_count(None, 5) == 0
