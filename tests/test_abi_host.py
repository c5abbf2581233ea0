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


def test_screen_groups_validation_without_gpu():
    """csel_screen_groups rejects bad sizes and missing arrays on the host."""
    if not os.path.exists(csel.LIB_PATH):
        pytest.skip("libcsel.so not built")
    lib = csel.load()
    kp = csel.KernelParams(5, 0.03, 1.0, 0.0)
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below fails validation first

    def call(dim=2, n_groups=1, n_members=4, stride=2048, params=fake, keep=512, thr=0.5, kept=fake, features=None,
             group_ptr=fake):
        return lib.csel_screen_groups(fake, 100, dim, ctypes.byref(kp), n_groups, group_ptr, fake, n_members, fake,
                                      fake, stride, params, fake if params is not None else None, keep, thr, kept,
                                      fake, fake, None, features, None)

    assert call(dim=4) == -1 and b"dim" in lib.csel_last_error()
    assert call(stride=2049) == -4 and b"pool_stride" in lib.csel_last_error()
    assert call(stride=0) == -4
    assert call(keep=0) == -1 and b"keep" in lib.csel_last_error()
    assert call(keep=600, stride=512) == -1
    assert call(thr=-1.0) == -1 and b"fallback_threshold" in lib.csel_last_error()
    assert call(n_groups=-1) == -1
    assert call(n_members=-1) == -1
    assert call(params=None, features=None) == -1 and b"features" in lib.csel_last_error()
    assert call(kept=None) == -1 and b"NULL" in lib.csel_last_error()
    assert call(group_ptr=None) == -1 and b"NULL" in lib.csel_last_error()
    # no groups: nothing to do
    assert call(n_groups=0) == 0
    kp_bad = csel.KernelParams(2, 0.03, 1.0, 0.0)
    assert lib.csel_screen_groups(fake, 100, 2, ctypes.byref(kp_bad), 1, fake, fake, 4, fake, fake, 64, fake, fake,
                                  8, 0.5, fake, fake, fake, None, None, None) == -4


def test_transpose_factor_validation_without_gpu():
    if not os.path.exists(csel.LIB_PATH):
        pytest.skip("libcsel.so not built")
    lib = csel.load()
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below fails validation first
    assert lib.csel_transpose_factor_workspace_size(-1, 0) == -1
    assert lib.csel_transpose_factor_workspace_size(10, -1) == -1
    assert lib.csel_transpose_factor_workspace_size(2 ** 31, 0) == -1
    assert lib.csel_transpose_factor_workspace_size(10, 2 ** 31) == -1
    assert lib.csel_transpose_factor_workspace_size(10, 0) == 0
    assert lib.csel_transpose_factor(10, None, fake, fake, 5, fake, fake, fake, fake, 1 << 30, None) == -1
    assert b"NULL" in lib.csel_last_error()
    assert lib.csel_transpose_factor(10, fake, None, fake, 5, fake, fake, fake, fake, 1 << 30, None) == -1
    assert lib.csel_transpose_factor(10, fake, fake, fake, 5, fake, fake, fake, None, 0, None) == -1
    assert b"workspace" in lib.csel_last_error()


def test_screen_rejects_order_longer_than_the_fallback_list():
    """Each processed order position may append one fallback entry, and the
    list holds n_targets entries: an order longer than that is refused on the
    host, before anything is enqueued."""
    if not os.path.exists(csel.LIB_PATH):
        pytest.skip("libcsel.so not built")
    lib = csel.load()
    kp = csel.KernelParams(3, 0.05, 1.0, 0.0)
    fake = ctypes.c_void_p(16)  # never dereferenced: the call fails validation first

    def call(n_order):
        return lib.csel_screen(fake, 100, 3, ctypes.byref(kp), 5, fake, fake, fake, 64, fake, fake, 8, 0.5, fake,
                               fake, fake, None, fake, fake, fake, n_order, None)

    assert call(6) == -1 and b"n_order" in lib.csel_last_error()
    assert call(-1) == -1 and b"n_order" in lib.csel_last_error()


def test_select_global_and_sched_validation_without_gpu():
    if not os.path.exists(csel.LIB_PATH):
        pytest.skip("libcsel.so not built")
    lib = csel.load()
    fake = ctypes.c_void_p(16)  # never dereferenced: every call below fails validation first
    kp = csel.KernelParams(3, 0.05, 1.0, 0.0)
    assert lib.csel_select_global_workspace_size(10, 0) == -4
    assert lib.csel_select_global_workspace_size(10, 33) == -4
    assert lib.csel_select_global_workspace_size(-1, 8) == -1
    assert lib.csel_select_global_workspace_size(10, 8) > 0

    def glob(budget=5, k_max=8, ws=fake, ws_bytes=1 << 40):
        return lib.csel_select_global(fake, 100, 3, ctypes.byref(kp), 10, fake, fake, fake, 64, k_max, budget, 0,
                                      ws, ws_bytes, fake, fake, fake, None, None, fake, None)

    assert glob(budget=-1) == -1 and b"budget" in lib.csel_last_error()
    assert glob(k_max=40) == -4
    assert glob(ws=None) == -1 and b"workspace" in lib.csel_last_error()
    assert glob(ws_bytes=8) == -1
    # the scheduled selection: only 1 or the multi-wave count of the pool width
    assert lib.csel_select_waves_per_column(128) == 2 and lib.csel_select_waves_per_column(512) == 4
    assert lib.csel_select_waves_per_column(600) == -1
    rc = lib.csel_select_and_factor_sched(fake, 100, 3, ctypes.byref(kp), 10, fake, fake, fake, 128, 8, 0, None,
                                          None, 0, 3, fake, fake, None, fake, None)
    assert rc == -4 and b"waves_per_column" in lib.csel_last_error()
    rc = lib.csel_select_and_factor_sched(fake, 100, 3, ctypes.byref(kp), 10, fake, fake, fake, 128, 8, 0, fake,
                                          None, 5, 2, fake, fake, None, fake, None)
    assert rc == -1 and b"col_list" in lib.csel_last_error()
