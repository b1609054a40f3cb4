"""The C-ABI library loads on the CPU and exports every function that
include/fthms.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "fthms.h")
LIB = os.path.join(ROOT, "paper_2507_05725_amd", "libfthms.so")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fthms_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2507_05725_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_path():
    names = declared()
    for must in ("fthms_create", "fthms_arc_create", "fthms_solve_dev",
                 "fthms_eval_field_dev", "fthms_freq_to_time_dev",
                 "fthms_problem_run_dev", "fthms_rhs_dev"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header(lib):
    from paper_2507_05725_amd import EXPORTED
    assert sorted(EXPORTED) == declared()


def test_host_only_calls(lib):
    """Calls that need no device: node table and argument checks."""
    import numpy as np
    lib.fthms_cheb_nodes.argtypes = [ctypes.c_int, ctypes.c_void_p]
    t = np.empty(9)
    assert lib.fthms_cheb_nodes(9, t.ctypes.data_as(ctypes.c_void_p)) == 0
    ref = np.cos((2 * np.arange(1, 10) - 1) * np.pi / 18)
    assert np.max(np.abs(t - ref)) < 2e-16
    assert lib.fthms_cheb_nodes(1, t.ctypes.data_as(ctypes.c_void_p)) == -1
    lib.fthms_abi_version.restype = ctypes.c_int
    assert lib.fthms_abi_version() == 2
