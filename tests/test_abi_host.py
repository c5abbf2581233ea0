"""Host-side checks of the C-ABI library: it loads, exports every symbol that
include/csel.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2307_11648_amd import csel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(csel_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(csel.LIB_PATH):
        pytest.skip("libcsel.so not built")
    lib = csel.load()
    names = _declared_symbols()
    assert "csel_select_and_factor" in names
    for name in sorted(names):
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def test_version_and_limits():
    if not os.path.exists(csel.LIB_PATH):
        pytest.skip("libcsel.so not built")
    lib = csel.load()
    assert lib.csel_version() == 1
    assert lib.csel_max_pool() >= 512
    assert lib.csel_max_select() >= 32


def test_argument_validation_without_gpu():
    """Validation runs on the host before any HIP call, so it works here."""
    if not os.path.exists(csel.LIB_PATH):
        pytest.skip("libcsel.so not built")
    lib = csel.load()
    kp = csel.KernelParams(4, 0.1, 1.0, 0.0)
    rc = lib.csel_select_and_factor(None, 10, 2, ctypes.byref(kp), 1, None, None, None, 8, 4, 0, None, None, None,
                                    None, None, None)
    assert rc == -4
    assert b"two_nu" in lib.csel_last_error()
    kp = csel.KernelParams(3, -1.0, 1.0, 0.0)
    rc = lib.csel_select_and_factor(None, 10, 2, ctypes.byref(kp), 1, None, None, None, 8, 4, 0, None, None, None,
                                    None, None, None)
    assert rc == -1
    kp = csel.KernelParams(3, 0.1, 1.0, 0.0)
    rc = lib.csel_select_and_factor(None, 10, 2, ctypes.byref(kp), 1, None, None, None, 8, 4, 0, None, None, None,
                                    None, None, None)
    assert rc == -1 and b"NULL" in lib.csel_last_error()
    rc = lib.csel_select_and_factor(None, 10, 5, ctypes.byref(kp), 1, None, None, None, 8, 4, 0, None, None, None,
                                    None, None, None)
    assert rc == -1 and b"dim" in lib.csel_last_error()
    rc = lib.csel_select_and_factor(None, 10, 2, ctypes.byref(kp), 1, None, None, None, 8, 99, 0, None, None, None,
                                    None, None, None)
    assert rc == -4
    rc = lib.csel_select_and_factor(None, 10, 2, ctypes.byref(kp), 0, None, None, None, 8, 4, 0, None, None, None,
                                    None, None, None)
    assert rc == 0
    assert lib.csel_sum(None, -1, None, None) == -1
