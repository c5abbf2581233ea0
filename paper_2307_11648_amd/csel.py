"""Python binding of libcsel (ctypes).  Argument marshalling only: every step
of the hot path runs in the library's HIP kernels; torch supplies device
memory and the current stream.  There is no CPU fallback: a missing library
or a non-GPU tensor is an error.

Entry points mirror include/csel.h:
    select_and_factor  -- greedy single-target selection + eq. L_col columns
    aggregated_select  -- multi-target selection, aggregated columns, GP posterior variances
    apply_factor       -- y = L^T x or y = L x with the sparse factor
    sum                -- deterministic FP64 sum (KL data term)
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsel.so")
_lib = None

_c = ctypes
_vp = ctypes.c_void_p

CSEL_FP64 = 0
CSEL_MIXED = 1
_PREC = {"fp64": CSEL_FP64, "mixed": CSEL_MIXED}


class CselError(RuntimeError):
    """A non-OK return of the C ABI, with csel_last_error()'s message."""

    def __init__(self, code, msg):
        super().__init__(f"csel error {code}: {msg}")
        self.code = code


class KernelParams(ctypes.Structure):
    _fields_ = [("two_nu", ctypes.c_int32), ("length_scale", ctypes.c_double), ("variance", ctypes.c_double),
                ("nugget", ctypes.c_double)]


def kernel_struct(kernel) -> KernelParams:
    return KernelParams(int(kernel.two_nu), float(kernel.length_scale), float(kernel.variance), float(kernel.nugget))


def load():
    """Load libcsel.so (built in-tree by paper_2307_11648_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2307_11648_amd.build.build_hip()")
    lib = ctypes.CDLL(LIB_PATH)
    lib.csel_last_error.restype = ctypes.c_char_p
    lib.csel_version.restype = ctypes.c_int32
    lib.csel_max_pool.restype = ctypes.c_int32
    lib.csel_max_select.restype = ctypes.c_int32
    lib.csel_select_and_factor.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _c.c_int64,
                                           _vp, _vp, _vp, _c.c_int32, _c.c_int32, _c.c_int32, _vp, _vp, _vp, _vp,
                                           _vp, _vp]
    lib.csel_select_and_factor.restype = ctypes.c_int
    lib.csel_apply_factor.argtypes = [_c.c_int64, _vp, _vp, _vp, _c.c_int32, _vp, _vp, _vp]
    lib.csel_apply_factor.restype = ctypes.c_int
    lib.csel_transpose_factor_workspace_size.argtypes = [_c.c_int64, _c.c_int64]
    lib.csel_transpose_factor_workspace_size.restype = ctypes.c_int64
    lib.csel_transpose_factor.argtypes = [_c.c_int64, _vp, _vp, _vp, _c.c_int64, _vp, _vp, _vp, _vp, _c.c_int64, _vp]
    lib.csel_transpose_factor.restype = ctypes.c_int
    lib.csel_aggregated_workspace_size.argtypes = [_c.c_int64, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_int32]
    lib.csel_aggregated_workspace_size.restype = ctypes.c_int64
    lib.csel_aggregated_max_block.restype = ctypes.c_int32
    lib.csel_aggregated_select.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _c.c_int64,
                                           _vp, _vp, _c.c_int32, _vp, _vp, _c.c_int32, _c.c_int32, _c.c_int32,
                                           _vp, _c.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.csel_aggregated_select.restype = ctypes.c_int
    lib.csel_aggregated_select_sched.argtypes = lib.csel_aggregated_select.argtypes[:-1] + [_c.c_int32, _vp]
    lib.csel_aggregated_select_sched.restype = ctypes.c_int
    lib.csel_partial_select.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _c.c_int64,
                                        _vp, _vp, _c.c_int32, _vp, _vp, _c.c_int32, _c.c_int32, _vp, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _vp, _vp]
    lib.csel_partial_select.restype = ctypes.c_int
    lib.csel_later_knn_workspace_size.argtypes = [_c.c_int64, _c.c_int32]
    lib.csel_later_knn_workspace_size.restype = ctypes.c_int64
    lib.csel_later_knn.argtypes = [_vp, _c.c_int64, _c.c_int32, _c.c_int32, _vp, _c.c_int64, _vp, _vp, _vp]
    lib.csel_later_knn.restype = ctypes.c_int
    lib.csel_reverse_maximin_workspace_size.argtypes = [_c.c_int64, _c.c_int32]
    lib.csel_reverse_maximin_workspace_size.restype = ctypes.c_int64
    lib.csel_reverse_maximin.argtypes = [_vp, _c.c_int64, _c.c_int32, _vp, _c.c_int64, _vp, _vp,
                                         ctypes.POINTER(_c.c_int32), _vp]
    lib.csel_reverse_maximin.restype = ctypes.c_int
    lib.csel_select_and_factor_list.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams),
                                                _c.c_int64, _vp, _vp, _vp, _c.c_int32, _c.c_int32, _c.c_int32,
                                                _vp, _vp, _c.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.csel_select_and_factor_list.restype = ctypes.c_int
    lib.csel_mlp_num_params.restype = ctypes.c_int32
    lib.csel_screen_features.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _c.c_int64,
                                         _vp, _vp, _vp, _c.c_int32, _vp, _vp]
    lib.csel_screen_features.restype = ctypes.c_int
    lib.csel_screen.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _c.c_int64, _vp, _vp,
                                _vp, _c.c_int32, _vp, _vp, _c.c_int32, _c.c_float, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, _c.c_int64, _vp]
    lib.csel_screen.restype = ctypes.c_int
    lib.csel_screen_groups.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _c.c_int64,
                                       _vp, _vp, _c.c_int64, _vp, _vp, _c.c_int32, _vp, _vp, _c.c_int32,
                                       _c.c_float, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.csel_screen_groups.restype = ctypes.c_int
    lib.csel_spatial_order_workspace_size.argtypes = [_c.c_int64]
    lib.csel_spatial_order_workspace_size.restype = ctypes.c_int64
    lib.csel_spatial_order.argtypes = [_vp, _c.c_int64, _c.c_int32, _c.c_int64, _vp, _vp, _c.c_int64, _vp, _vp]
    lib.csel_spatial_order.restype = ctypes.c_int
    lib.csel_mlp_forward.argtypes = [_vp, _vp, _vp, _c.c_int64, _vp, _vp]
    lib.csel_mlp_forward.restype = ctypes.c_int
    lib.csel_mlp_grad_workspace_size.argtypes = [_c.c_int64]
    lib.csel_mlp_grad_workspace_size.restype = ctypes.c_int64
    lib.csel_mlp_grad.argtypes = [_vp, _vp, _vp, _vp, _c.c_int64, _c.c_float, _vp, _c.c_int64, _vp, _vp]
    lib.csel_mlp_grad.restype = ctypes.c_int
    lib.csel_select_waves_per_column.argtypes = [_c.c_int32]
    lib.csel_select_waves_per_column.restype = ctypes.c_int32
    lib.csel_select_and_factor_sched.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams),
                                                 _c.c_int64, _vp, _vp, _vp, _c.c_int32, _c.c_int32, _c.c_int32,
                                                 _vp, _vp, _c.c_int64, _c.c_int32, _vp, _vp, _vp, _vp, _vp]
    lib.csel_select_and_factor_sched.restype = ctypes.c_int
    lib.csel_select_global_workspace_size.argtypes = [_c.c_int64, _c.c_int32]
    lib.csel_select_global_workspace_size.restype = ctypes.c_int64
    lib.csel_select_global.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _c.c_int64, _vp,
                                       _vp, _vp, _c.c_int32, _c.c_int32, _c.c_int64, _c.c_int32, _vp, _c.c_int64,
                                       _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.csel_select_global.restype = ctypes.c_int
    lib.csel_kernel_matvec_workspace_size.argtypes = [_c.c_int64]
    lib.csel_kernel_matvec_workspace_size.restype = ctypes.c_int64
    lib.csel_kernel_matvec.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _vp, _vp, _vp,
                                       _c.c_int64, _vp]
    lib.csel_kernel_matvec.restype = ctypes.c_int
    lib.csel_pcg_workspace_size.argtypes = [_c.c_int64]
    lib.csel_pcg_workspace_size.restype = ctypes.c_int64
    lib.csel_pcg.argtypes = [_vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _vp, _vp, _vp, _vp, _vp, _vp,
                             _vp, _vp, _c.c_double, _c.c_int32, _vp, _c.c_int64, ctypes.POINTER(_c.c_int32),
                             ctypes.POINTER(_c.c_double), _vp]
    lib.csel_pcg.restype = ctypes.c_int
    lib.csel_plan_create.argtypes = [ctypes.POINTER(_vp), _c.c_int64, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_int32,
                                     _c.c_uint32]
    lib.csel_plan_create.restype = ctypes.c_int
    lib.csel_plan_destroy.argtypes = [_vp]
    lib.csel_plan_destroy.restype = None
    lib.csel_plan_set_order.argtypes = [_vp, _vp, _c.c_int64, _c.c_int32, _vp, _vp]
    lib.csel_plan_set_order.restype = ctypes.c_int
    lib.csel_screened_select.argtypes = [_vp, _vp, _c.c_int64, _c.c_int32, ctypes.POINTER(KernelParams), _vp, _vp,
                                         _vp, _vp, _vp, _c.c_float, _vp, _vp, _vp, _vp, _vp]
    lib.csel_screened_select.restype = ctypes.c_int
    lib.csel_plan_info.argtypes = [_vp, ctypes.POINTER(_c.c_int32), ctypes.POINTER(_c.c_int32),
                                   ctypes.POINTER(_c.c_float)]
    lib.csel_plan_info.restype = ctypes.c_int
    lib.csel_plan_screen_outputs.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.csel_plan_screen_outputs.restype = ctypes.c_int
    lib.csel_mlp_grad_noalloc.argtypes = [_vp, _vp, _vp, _vp, _c.c_int64, _c.c_float, _vp, _vp]
    lib.csel_mlp_grad_noalloc.restype = ctypes.c_int
    lib.csel_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, _vp, _c.c_int32, _c.c_float, _c.c_float, _c.c_float,
                                  _c.c_float, _c.c_int32, _vp]
    lib.csel_mlp_adam.restype = ctypes.c_int
    lib.csel_mlp_to_bf16.argtypes = [_vp, _vp, _c.c_int32, _vp]
    lib.csel_mlp_to_bf16.restype = ctypes.c_int
    lib.csel_sum.argtypes = [_vp, _c.c_int64, _vp, _vp]
    lib.csel_sum.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise CselError(rc, load().csel_last_error().decode())


def _dev(t: torch.Tensor, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def select_and_factor(points, kernel, targets, pool, pool_len, k: int, precision: str = "fp64",
                      want_gap: bool = False, out: dict | None = None, stream=None) -> dict:
    """Greedy selection + factor columns for every target (csel_select_and_factor).

    points [n, dim] float64, targets [T] int32, pool [T, stride] int32,
    pool_len [T] int32 -- all on the GPU.  Returns a dict of GPU tensors:
    sel [T, k] int32, factor [T, k+1] float64, log_condvar [T] float64,
    status [T] uint8 and, if want_gap, gap [T, k] float32.  Pass `out` (same
    keys) to reuse buffers."""
    lib = load()
    _dev(points, torch.float64, "points")
    _dev(targets, torch.int32, "targets")
    _dev(pool, torch.int32, "pool")
    _dev(pool_len, torch.int32, "pool_len")
    if points.dim() != 2:
        raise ValueError("points must be [n, dim]")
    T = targets.shape[0]
    stride = pool.shape[1] if pool.dim() == 2 else 0
    dev = points.device
    if out is None:
        out = {
            "sel": torch.empty((T, k), dtype=torch.int32, device=dev),
            "factor": torch.empty((T, k + 1), dtype=torch.float64, device=dev),
            "log_condvar": torch.empty(T, dtype=torch.float64, device=dev),
            "status": torch.empty(T, dtype=torch.uint8, device=dev),
        }
        if want_gap:
            out["gap"] = torch.empty((T, k), dtype=torch.float32, device=dev)
    kp = kernel_struct(kernel)
    rc = lib.csel_select_and_factor(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), T,
                                    targets.data_ptr(), pool.data_ptr(), pool_len.data_ptr(), stride, int(k),
                                    _PREC[precision], _ptr(out["sel"]), _ptr(out["factor"]),
                                    _ptr(out.get("log_condvar")), _ptr(out.get("gap")), _ptr(out["status"]),
                                    _stream(stream))
    _check(rc)
    return out


def select_and_factor_list(points, kernel, targets, pool, pool_len, k: int, precision: str, col_list, col_count,
                           max_cols: int, out: dict, stream=None) -> dict:
    """csel_select_and_factor on the listed columns only, writing into `out`
    (the dict returned by select_and_factor for the same targets)."""
    lib = load()
    _dev(col_list, torch.int32, "col_list")
    _dev(col_count, torch.int32, "col_count")
    if col_list.numel() < max_cols or col_count.numel() < 1:
        raise ValueError("col_list must hold max_cols entries and col_count one")
    T = targets.shape[0]
    stride = pool.shape[1] if pool.dim() == 2 else 0
    kp = kernel_struct(kernel)
    rc = lib.csel_select_and_factor_list(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), T,
                                         targets.data_ptr(), pool.data_ptr(), pool_len.data_ptr(), stride, int(k),
                                         _PREC[precision], col_list.data_ptr(), col_count.data_ptr(), int(max_cols),
                                         _ptr(out["sel"]), _ptr(out["factor"]), _ptr(out.get("log_condvar")),
                                         _ptr(out.get("gap")), _ptr(out["status"]), _stream(stream))
    _check(rc)
    return out


def select_waves_per_column(pool_stride: int) -> int:
    """The multi-wave schedule's wavefronts per column for this pool width."""
    return int(load().csel_select_waves_per_column(int(pool_stride)))


def select_and_factor_sched(points, kernel, targets, pool, pool_len, k: int, precision: str = "fp64",
                            waves: int = 1, col_list=None, col_count=None, max_cols: int = 0,
                            out: dict | None = None, stream=None) -> dict:
    """csel_select_and_factor_sched: the selection under an explicit schedule
    (waves per column, optional column list); the same outputs as
    select_and_factor without the gap."""
    lib = load()
    _dev(points, torch.float64, "points")
    _dev(targets, torch.int32, "targets")
    _dev(pool, torch.int32, "pool")
    _dev(pool_len, torch.int32, "pool_len")
    if col_list is not None:
        _dev(col_list, torch.int32, "col_list")
        _dev(col_count, torch.int32, "col_count")
        if col_list.numel() < max_cols or col_count.numel() < 1:
            raise ValueError("col_list must hold max_cols entries and col_count one")
    T = targets.shape[0]
    stride = pool.shape[1] if pool.dim() == 2 else 0
    dev = points.device
    if out is None:
        out = {"sel": torch.empty((T, k), dtype=torch.int32, device=dev),
               "factor": torch.empty((T, k + 1), dtype=torch.float64, device=dev),
               "log_condvar": torch.empty(T, dtype=torch.float64, device=dev),
               "status": torch.empty(T, dtype=torch.uint8, device=dev)}
    kp = kernel_struct(kernel)
    _check(lib.csel_select_and_factor_sched(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), T,
                                            targets.data_ptr(), pool.data_ptr(), pool_len.data_ptr(), stride, int(k),
                                            _PREC[precision], _ptr(col_list), _ptr(col_count), int(max_cols),
                                            int(waves), _ptr(out["sel"]), _ptr(out["factor"]),
                                            _ptr(out.get("log_condvar")), _ptr(out["status"]), _stream(stream)))
    return out


def select_global(points, kernel, targets, pool, pool_len, k_max: int, budget: int, precision: str = "fp64",
                  want_gain: bool = False, out: dict | None = None, workspace=None, stream=None) -> dict:
    """csel_select_global: greedy selection with the nonzeros allocated over
    the columns by global greedy selection.  Returns GPU tensors k_alloc [T],
    sel [T, k_max], factor [T, k_max+1], log_condvar [T], status [T] and,
    with want_gain, gain [T, k_max]; plus the workspace."""
    lib = load()
    _dev(points, torch.float64, "points")
    _dev(targets, torch.int32, "targets")
    _dev(pool, torch.int32, "pool")
    _dev(pool_len, torch.int32, "pool_len")
    T = targets.shape[0]
    stride = pool.shape[1] if pool.dim() == 2 else 0
    dev = points.device
    if out is None:
        out = {"k_alloc": torch.empty(T, dtype=torch.int32, device=dev),
               "sel": torch.empty((T, k_max), dtype=torch.int32, device=dev),
               "factor": torch.empty((T, k_max + 1), dtype=torch.float64, device=dev),
               "log_condvar": torch.empty(T, dtype=torch.float64, device=dev),
               "status": torch.empty(T, dtype=torch.uint8, device=dev)}
        if want_gain:
            out["gain"] = torch.empty((T, k_max), dtype=torch.float64, device=dev)
    need = int(lib.csel_select_global_workspace_size(T, int(k_max)))
    if need < 0:
        _check(-1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    kp = kernel_struct(kernel)
    _check(lib.csel_select_global(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), T,
                                  targets.data_ptr(), pool.data_ptr(), pool_len.data_ptr(), stride, int(k_max),
                                  int(budget), _PREC[precision], workspace.data_ptr(), workspace.numel(),
                                  _ptr(out["k_alloc"]), _ptr(out["sel"]), _ptr(out["factor"]),
                                  _ptr(out.get("log_condvar")), _ptr(out.get("gain")), _ptr(out["status"]),
                                  _stream(stream)))
    out["workspace"] = workspace
    return out


def kernel_matvec(points, kernel, x, out=None, workspace=None, stream=None):
    """csel_kernel_matvec: y = Theta x, matrix-free in FP64.  Returns (y,
    workspace)."""
    lib = load()
    _dev(points, torch.float64, "points")
    _dev(x, torch.float64, "x")
    n = points.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=points.device)
    need = int(lib.csel_kernel_matvec_workspace_size(n))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=points.device)
    kp = kernel_struct(kernel)
    _check(lib.csel_kernel_matvec(points.data_ptr(), n, points.shape[1], ctypes.byref(kp), x.data_ptr(),
                                  out.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream(stream)))
    return out, workspace


def pcg(points, kernel, y, factor=None, factor_t=None, x0=None, rel_tol: float = 1e-12, max_iter: int = 1000,
        workspace=None, stream=None):
    """csel_pcg: solve Theta x = y by the conjugate gradient preconditioned by
    L L^T.  factor = (col_ptr, rows, vals) of L in CSC form, factor_t the same
    for L^T (transpose_factor); factor None runs the plain conjugate
    gradient.  Returns (x, iterations, relative residual)."""
    lib = load()
    _dev(points, torch.float64, "points")
    _dev(y, torch.float64, "y")
    n = points.shape[0]
    x = torch.zeros(n, dtype=torch.float64, device=points.device) if x0 is None else x0.clone()
    need = int(lib.csel_pcg_workspace_size(n))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=points.device)
    lc = lr = lv = tc = tr = tv = None
    if factor is not None:
        lc, lr, lv = (_ptr(a) for a in factor)
        tc, tr, tv = (_ptr(a) for a in factor_t)
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    kp = kernel_struct(kernel)
    _check(lib.csel_pcg(points.data_ptr(), n, points.shape[1], ctypes.byref(kp), lc, lr, lv, tc, tr, tv, y.data_ptr(),
                        x.data_ptr(), float(rel_tol), int(max_iter), workspace.data_ptr(), workspace.numel(),
                        ctypes.byref(it), ctypes.byref(res), _stream(stream)))
    return x, int(it.value), float(res.value)


# --------------------------------------------------------------------------
# the screened-selection plan (one call per learned-screened step)
# --------------------------------------------------------------------------
class Plan:
    """csel_plan: the buffers, tuned column schedule and (graph=True) captured
    HIP graph of the learned-screened step over n_targets columns with pools
    of pool_stride candidates kept to `keep` before the selection of k."""

    def __init__(self, n_targets: int, pool_stride: int, keep: int, k: int, precision: str = "mixed",
                 graph: bool = False):
        lib = load()
        self._lib = lib
        self._h = ctypes.c_void_p()
        self.n_targets, self.pool_stride, self.keep, self.k = int(n_targets), int(pool_stride), int(keep), int(k)
        self.precision = precision
        _check(lib.csel_plan_create(ctypes.byref(self._h), self.n_targets, self.pool_stride, self.keep, self.k,
                                    _PREC[precision], 1 if graph else 0))

    def close(self):
        if self._h:
            self._lib.csel_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass

    def set_order(self, points, targets, stream=None):
        """The Morton processing order of the columns (csel_plan_set_order)."""
        _dev(points, torch.float64, "points")
        _dev(targets, torch.int32, "targets")
        _check(self._lib.csel_plan_set_order(self._h, points.data_ptr(), points.shape[0], points.shape[1],
                                             targets.data_ptr(), _stream(stream)))

    def step(self, points, kernel, targets, pool, pool_len, params, params_bf16, fallback_threshold: float,
             out: dict | None = None, stream=None) -> dict:
        """One screened step (csel_screened_select); returns sel, factor,
        log_condvar and status as GPU tensors (reusing `out`)."""
        _dev(points, torch.float64, "points")
        _dev(targets, torch.int32, "targets")
        _dev(pool, torch.int32, "pool")
        _dev(pool_len, torch.int32, "pool_len")
        T, k = self.n_targets, self.k
        if targets.shape[0] != T or pool.shape != (T, self.pool_stride):
            raise ValueError("targets / pool do not match the plan's shape")
        dev = points.device
        if out is None:
            out = {"sel": torch.empty((T, k), dtype=torch.int32, device=dev),
                   "factor": torch.empty((T, k + 1), dtype=torch.float64, device=dev),
                   "log_condvar": torch.empty(T, dtype=torch.float64, device=dev),
                   "status": torch.empty(T, dtype=torch.uint8, device=dev)}
        kp = kernel_struct(kernel)
        _check(self._lib.csel_screened_select(self._h, points.data_ptr(), points.shape[0], points.shape[1],
                                              ctypes.byref(kp), targets.data_ptr(), pool.data_ptr(),
                                              pool_len.data_ptr(), params.data_ptr(), params_bf16.data_ptr(),
                                              float(fallback_threshold), _ptr(out["sel"]), _ptr(out["factor"]),
                                              _ptr(out.get("log_condvar")), _ptr(out["status"]), _stream(stream)))
        return out

    def screen_outputs(self, out: dict | None = None, stream=None) -> dict:
        """Copies of the last step's kept lists, fallback flags, fallback list
        and count (csel_plan_screen_outputs)."""
        T, dev = self.n_targets, torch.cuda.current_device()
        if out is None:
            out = {"kept": torch.empty((T, self.keep), dtype=torch.int32, device=dev),
                   "kept_len": torch.empty(T, dtype=torch.int32, device=dev),
                   "fallback": torch.empty(T, dtype=torch.uint8, device=dev),
                   "fallback_list": torch.empty(T, dtype=torch.int32, device=dev),
                   "fallback_count": torch.empty(1, dtype=torch.int32, device=dev)}
        _check(self._lib.csel_plan_screen_outputs(self._h, _ptr(out.get("kept")), _ptr(out.get("kept_len")),
                                                  _ptr(out.get("fallback")), _ptr(out.get("fallback_list")),
                                                  _ptr(out.get("fallback_count")), _stream(stream)))
        return out

    def info(self) -> dict:
        """The tuned schedules (None before the first step): the kept-pool
        selection's ("natural", "spatial", "natural/mw" or "spatial/mw") and
        the fallback launch's waves per column, with the tuning times in ms."""
        sc = ctypes.c_int32(-1)
        fw = ctypes.c_int32(1)
        ms = (ctypes.c_float * 6)()
        _check(self._lib.csel_plan_info(self._h, ctypes.byref(sc), ctypes.byref(fw), ms))
        names = ("natural", "spatial", "natural/mw", "spatial/mw")
        name = names[sc.value] if 0 <= sc.value < 4 else None
        return {"schedule": name, "fallback_waves": int(fw.value) if name else None,
                "ms": {n: float(ms[i]) for i, n in enumerate(names)},
                "fallback_ms": {"1": float(ms[4]), "mw": float(ms[5])}}


# --------------------------------------------------------------------------
# learned screen
# --------------------------------------------------------------------------
def mlp_num_params() -> int:
    return int(load().csel_mlp_num_params())


def mlp_to_bf16(params, out=None, stream=None):
    """BF16 copy (as int16 bit patterns) of FP32 parameters."""
    lib = load()
    _dev(params, torch.float32, "params")
    if out is None:
        out = torch.empty(params.numel(), dtype=torch.int16, device=params.device)
    _check(lib.csel_mlp_to_bf16(params.data_ptr(), out.data_ptr(), params.numel(), _stream(stream)))
    return out


def screen_features(points, kernel, targets, pool, pool_len, stream=None):
    """Features [T, stride, 16] float32 of every pool slot (zeros past pool_len)."""
    lib = load()
    T = targets.shape[0]
    stride = pool.shape[1]
    feats = torch.zeros((T, stride, 16), dtype=torch.float32, device=points.device)
    kp = kernel_struct(kernel)
    _check(lib.csel_screen_features(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), T,
                                    targets.data_ptr(), pool.data_ptr(), pool_len.data_ptr(), stride,
                                    feats.data_ptr(), _stream(stream)))
    return feats


def spatial_order(points, targets, out=None, workspace=None, stream=None):
    """csel_spatial_order: int32 [T] processing order of the columns by the
    Morton code of their targets.  Returns (order, workspace)."""
    lib = load()
    T = targets.shape[0]
    dev = points.device
    if out is None:
        out = torch.empty(max(T, 1), dtype=torch.int32, device=dev)
    need = int(lib.csel_spatial_order_workspace_size(T))
    if need < 0:
        raise CselError(lib.csel_last_error().decode())
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib.csel_spatial_order(points.data_ptr(), points.shape[0], points.shape[1], T, targets.data_ptr(),
                                  workspace.data_ptr(), workspace.numel(), out.data_ptr(), _stream(stream)))
    return out[:T], workspace


def screen(points, kernel, targets, pool, pool_len, params, params_bf16, keep: int, fallback_threshold=0.5,
           want_logits=False, out=None, order=None, stream=None) -> dict:
    """csel_screen: kept [T, keep] ids in distance order, kept_len [T],
    fallback [T] u8, fallback_list [T] int32 with fallback_count [1].
    `order` (int32 device tensor, optional) lists the columns to process, in
    processing order (all of them, e.g. csel.spatial_order, or a subset)."""
    lib = load()
    _dev(params, torch.float32, "params")
    if order is not None:
        _dev(order, torch.int32, "order")
    T = targets.shape[0]
    stride = pool.shape[1]
    dev = points.device
    if out is None:
        out = {"kept": torch.empty((T, keep), dtype=torch.int32, device=dev),
               "kept_len": torch.empty(T, dtype=torch.int32, device=dev),
               "fallback": torch.empty(T, dtype=torch.uint8, device=dev),
               "fallback_list": torch.empty(max(T, 1), dtype=torch.int32, device=dev),
               "fallback_count": torch.empty(1, dtype=torch.int32, device=dev)}
        if want_logits:
            out["logits"] = torch.zeros((T, stride), dtype=torch.float32, device=dev)
    kp = kernel_struct(kernel)
    _check(lib.csel_screen(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), T,
                           targets.data_ptr(), pool.data_ptr(), pool_len.data_ptr(), stride, params.data_ptr(),
                           params_bf16.data_ptr(), int(keep), float(fallback_threshold), out["kept"].data_ptr(),
                           out["kept_len"].data_ptr(), out["fallback"].data_ptr(), _ptr(out.get("logits")),
                           out["fallback_list"].data_ptr(), out["fallback_count"].data_ptr(), _ptr(order),
                           0 if order is None else order.numel(), _stream(stream)))
    return out


def screen_groups(points, kernel, group_ptr, members, pool, pool_len, params, params_bf16, keep: int,
                  fallback_threshold=0.5, want_logits=False, want_features=False, out=None, stream=None) -> dict:
    """csel_screen_groups: kept [G, keep] ids in slot order, kept_len [G],
    fallback [G] u8; optionally logits [G, stride] and features [G, stride,
    16].  With params None only the features are computed."""
    lib = load()
    for t, nm in ((group_ptr, "group_ptr"), (members, "members"), (pool, "pool"), (pool_len, "pool_len")):
        _dev(t, torch.int32, nm)
    _dev(points, torch.float64, "points")
    if params is not None:
        _dev(params, torch.float32, "params")
    G = group_ptr.numel() - 1
    stride = pool.shape[1]
    dev = points.device
    if out is None:
        out = {}
        if params is not None:
            out.update(kept=torch.empty((G, keep), dtype=torch.int32, device=dev),
                       kept_len=torch.empty(G, dtype=torch.int32, device=dev),
                       fallback=torch.empty(G, dtype=torch.uint8, device=dev))
        if want_logits:
            out["logits"] = torch.zeros((G, stride), dtype=torch.float32, device=dev)
        if want_features or params is None:
            out["features"] = torch.zeros((G, stride, 16), dtype=torch.float32, device=dev)
    kp = kernel_struct(kernel)
    _check(lib.csel_screen_groups(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), G,
                                  group_ptr.data_ptr(), members.data_ptr(), members.numel(), pool.data_ptr(),
                                  pool_len.data_ptr(), stride, _ptr(params), _ptr(params_bf16), int(keep),
                                  float(fallback_threshold), _ptr(out.get("kept")), _ptr(out.get("kept_len")),
                                  _ptr(out.get("fallback")), _ptr(out.get("logits")), _ptr(out.get("features")),
                                  _stream(stream)))
    return out


def mlp_forward(params, params_bf16, x, out=None, stream=None):
    lib = load()
    _dev(x, torch.float32, "x")
    n = x.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=x.device)
    _check(lib.csel_mlp_forward(params.data_ptr(), params_bf16.data_ptr(), x.data_ptr(), n, out.data_ptr(),
                                _stream(stream)))
    return out


def mlp_grad(params, params_bf16, x, labels, pos_weight: float, grad=None, workspace=None, stream=None):
    """Gradient [P+1] (last = summed weighted loss) of the mean weighted BCE."""
    lib = load()
    _dev(x, torch.float32, "x")
    _dev(labels, torch.uint8, "labels")
    n = x.shape[0]
    need = lib.csel_mlp_grad_workspace_size(n)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 4), dtype=torch.uint8, device=x.device)
    if grad is None:
        grad = torch.empty(mlp_num_params() + 1, dtype=torch.float32, device=x.device)
    _check(lib.csel_mlp_grad(params.data_ptr(), params_bf16.data_ptr(), x.data_ptr(), labels.data_ptr(), n,
                             float(pos_weight), workspace.data_ptr(), workspace.numel(), grad.data_ptr(),
                             _stream(stream)))
    return grad, workspace


MLP_GRAD_NOALLOC_MAX_ROWS = 65536  # CSEL_MLP_GRAD_NOALLOC_MAX_ROWS


def mlp_grad_noalloc(params, params_bf16, x, labels, pos_weight: float, grad, stream=None):
    """csel_mlp_grad_noalloc: mlp_grad without a workspace and without any
    device allocation (the caller passes `grad`, [P+1] float32); at most
    MLP_GRAD_NOALLOC_MAX_ROWS rows."""
    lib = load()
    _dev(x, torch.float32, "x")
    _dev(labels, torch.uint8, "labels")
    _dev(grad, torch.float32, "grad")
    _check(lib.csel_mlp_grad_noalloc(params.data_ptr(), params_bf16.data_ptr(), x.data_ptr(), labels.data_ptr(),
                                     x.shape[0], float(pos_weight), grad.data_ptr(), _stream(stream)))
    return grad


def mlp_adam(params, params_bf16, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    lib = load()
    _check(lib.csel_mlp_adam(params.data_ptr(), params_bf16.data_ptr(), grad.data_ptr(), m.data_ptr(),
                             v.data_ptr(), params.numel(), float(lr), float(beta1), float(beta2), float(eps),
                             int(step), _stream(stream)))


def aggregated_val_ptr(group_ptr, pool_len, k: int):
    """Offsets of the aggregated member columns (layout glue): member a of a
    group with m members and min(k, pool_len) selections owns m - a + that
    many values, rows ascending."""
    gp = group_ptr.to(torch.int64)
    m = gp[1:] - gp[:-1]
    ns = torch.clamp(pool_len.to(torch.int64), max=k)
    g_of = torch.repeat_interleave(torch.arange(len(m), device=gp.device), m)
    a = torch.arange(int(gp[-1].item()), device=gp.device) - gp[:-1][g_of]
    sizes = m[g_of] - a + ns[g_of]
    vp = torch.zeros(len(sizes) + 1, dtype=torch.int64, device=gp.device)
    vp[1:] = torch.cumsum(sizes, 0)
    return vp


AGG_SCHEDULES = {"auto": 0, "one_group": 1, "register": 2, "split256": 3, "split512": 4, "split1024": 5}


def aggregated_select(points, kernel, group_ptr, members, max_members: int, pool, pool_len, k: int,
                      precision: str = "mixed", want_factor: bool = False, want_post_var: bool = False,
                      want_gap: bool = False, out: dict | None = None, workspace=None, stream=None,
                      schedule: str = "auto") -> dict:
    """Multi-target (aggregated) greedy selection (csel_aggregated_select,
    or csel_aggregated_select_sched for a schedule other than "auto": one of
    AGG_SCHEDULES).

    group_ptr [G+1] int32 CSR offsets into members [sum m] int32; pool [G,
    stride] int32, pool_len [G] int32.  Returns GPU tensors: sel [G, k],
    logdet [G], status [G]; with want_post_var post_var [sum m]; with
    want_factor val_ptr, rows, vals, member_log_condvar; with want_gap gap."""
    lib = load()
    _dev(points, torch.float64, "points")
    for t, nm in ((group_ptr, "group_ptr"), (members, "members"), (pool, "pool"), (pool_len, "pool_len")):
        _dev(t, torch.int32, nm)
    G = group_ptr.numel() - 1
    stride = pool.shape[1] if pool.dim() == 2 else 0
    dev = points.device
    nm_total = members.numel()
    if out is None:
        out = {"sel": torch.empty((G, k), dtype=torch.int32, device=dev),
               "logdet": torch.empty(G, dtype=torch.float64, device=dev),
               "status": torch.empty(G, dtype=torch.uint8, device=dev)}
        if want_gap:
            out["gap"] = torch.empty((G, k), dtype=torch.float32, device=dev)
        if want_post_var:
            out["post_var"] = torch.empty(nm_total, dtype=torch.float64, device=dev)
        if want_factor:
            vp = aggregated_val_ptr(group_ptr, pool_len, k)
            nnz = int(vp[-1].item())
            out.update(val_ptr=vp, rows=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
                       vals=torch.empty(max(nnz, 1), dtype=torch.float64, device=dev),
                       member_log_condvar=torch.empty(nm_total, dtype=torch.float64, device=dev))
    prec = _PREC[precision]
    need = lib.csel_aggregated_workspace_size(G, stride, int(max_members), int(k), prec)
    if need < 0:
        _check(-1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    out["workspace"] = workspace
    kp = kernel_struct(kernel)
    if schedule not in AGG_SCHEDULES:
        raise ValueError(f"schedule must be one of {sorted(AGG_SCHEDULES)}")
    rc = lib.csel_aggregated_select_sched(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), G,
                                          group_ptr.data_ptr(), members.data_ptr(), int(max_members),
                                          pool.data_ptr(), pool_len.data_ptr(), stride, int(k), prec,
                                          workspace.data_ptr(), workspace.numel(), _ptr(out["sel"]),
                                          _ptr(out.get("gap")), _ptr(out.get("logdet")), _ptr(out.get("post_var")),
                                          _ptr(out.get("val_ptr")), _ptr(out.get("rows")), _ptr(out.get("vals")),
                                          _ptr(out.get("member_log_condvar")), _ptr(out["status"]),
                                          AGG_SCHEDULES[schedule], _stream(stream))
    _check(rc)
    return out


def partial_select(points, kernel, group_ptr, members, max_members: int, pool, pool_len, k: int,
                   want_factor: bool = False, want_gap: bool = False, out: dict | None = None, stream=None) -> dict:
    """Partial (non-adjacent) aggregated selection, FP64 (csel_partial_select):
    candidates may lie between a group's members and condition only the
    members they follow.  Returns GPU tensors sel [G, k], logdet [G] (the
    group term), status [G]; with want_gap gap; with want_factor val_ptr,
    rows, vals, member_log_condvar (the aggregated member columns)."""
    lib = load()
    _dev(points, torch.float64, "points")
    for t, nm in ((group_ptr, "group_ptr"), (members, "members"), (pool, "pool"), (pool_len, "pool_len")):
        _dev(t, torch.int32, nm)
    G = group_ptr.numel() - 1
    stride = pool.shape[1] if pool.dim() == 2 else 0
    dev = points.device
    if out is None:
        out = {"sel": torch.empty((G, k), dtype=torch.int32, device=dev),
               "logdet": torch.empty(G, dtype=torch.float64, device=dev),
               "status": torch.empty(G, dtype=torch.uint8, device=dev)}
        if want_gap:
            out["gap"] = torch.empty((G, k), dtype=torch.float32, device=dev)
        if want_factor:
            vp = aggregated_val_ptr(group_ptr, pool_len, k)
            nnz = int(vp[-1].item())
            out.update(val_ptr=vp, rows=torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
                       vals=torch.empty(max(nnz, 1), dtype=torch.float64, device=dev),
                       member_log_condvar=torch.empty(members.numel(), dtype=torch.float64, device=dev))
    kp = kernel_struct(kernel)
    rc = lib.csel_partial_select(points.data_ptr(), points.shape[0], points.shape[1], ctypes.byref(kp), G,
                                 group_ptr.data_ptr(), members.data_ptr(), int(max_members), pool.data_ptr(),
                                 pool_len.data_ptr(), stride, int(k), _ptr(out["sel"]), _ptr(out.get("gap")),
                                 _ptr(out.get("logdet")), _ptr(out.get("val_ptr")), _ptr(out.get("rows")),
                                 _ptr(out.get("vals")), _ptr(out.get("member_log_condvar")), _ptr(out["status"]),
                                 _stream(stream))
    _check(rc)
    return out


def later_knn_pools(points, C: int, out=None, workspace=None, stream=None, check: bool = True):
    """Later-ordered kNN pools on the GPU (csel_later_knn): (pool [n, C]
    int32, pool_len [n] int32) for points [n, dim] FP64 in ordering-position
    order.  With check, raises if a row could not be built (more than 2048
    later points tied at one distance)."""
    lib = load()
    _dev(points, torch.float64, "points")
    n, dim = points.shape
    dev = points.device
    if out is None:
        out = (torch.empty((n, C), dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
    need = lib.csel_later_knn_workspace_size(n, dim)
    if need < 0:
        _check(-1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib.csel_later_knn(points.data_ptr(), n, dim, int(C), workspace.data_ptr(), workspace.numel(),
                              out[0].data_ptr(), out[1].data_ptr(), _stream(stream)))
    if check and n > 0 and int(out[1].min().item()) < 0:
        raise CselError(-4, "later_knn: more than 2048 later points tie at one distance")
    return out


def reverse_maximin(points, out=None, workspace=None, stream=None):
    """Reverse-maximin ordering on the GPU (csel_reverse_maximin): (order [n]
    int32, ell [n] FP64, rounds) for points [n, dim] FP64 in id order;
    order[pos] is the id at position pos.  Returns after the stream drained."""
    lib = load()
    _dev(points, torch.float64, "points")
    n, dim = points.shape
    dev = points.device
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.float64, device=dev))
    need = lib.csel_reverse_maximin_workspace_size(n, dim)
    if need < 0:
        _check(-1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    rounds = _c.c_int32(0)
    _check(lib.csel_reverse_maximin(points.data_ptr(), n, dim, workspace.data_ptr(), workspace.numel(),
                                    out[0].data_ptr(), out[1].data_ptr(), ctypes.byref(rounds), _stream(stream)))
    return out[0], out[1], int(rounds.value)


def apply_factor(col_ptr, row_idx, val, x, transpose: bool, out=None, stream=None):
    """y = L^T x (transpose) or y = L x for L in CSC form (csel_apply_factor)."""
    lib = load()
    _dev(col_ptr, torch.int64, "col_ptr")
    _dev(row_idx, torch.int32, "row_idx")
    _dev(val, torch.float64, "val")
    _dev(x, torch.float64, "x")
    n = col_ptr.numel() - 1
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=x.device)
    _check(lib.csel_apply_factor(n, col_ptr.data_ptr(), row_idx.data_ptr(), val.data_ptr(), int(bool(transpose)),
                                 x.data_ptr(), out.data_ptr(), _stream(stream)))
    return out


def transpose_factor(col_ptr, row_idx, val, out=None, workspace=None, stream=None):
    """(t_col_ptr, t_row_idx, t_val): L^T in CSC form (csel_transpose_factor),
    so that apply_factor(..., transpose=True) on it computes L x."""
    lib = load()
    _dev(col_ptr, torch.int64, "col_ptr")
    _dev(row_idx, torch.int32, "row_idx")
    _dev(val, torch.float64, "val")
    n = col_ptr.numel() - 1
    n_slots = row_idx.numel()
    dev = col_ptr.device
    if out is None:
        out = (torch.empty(n + 1, dtype=torch.int64, device=dev),
               torch.empty(max(n_slots, 1), dtype=torch.int32, device=dev),
               torch.empty(max(n_slots, 1), dtype=torch.float64, device=dev))
    need = lib.csel_transpose_factor_workspace_size(n, n_slots)
    if need < 0:
        _check(-1)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib.csel_transpose_factor(n, col_ptr.data_ptr(), row_idx.data_ptr(), val.data_ptr(), n_slots,
                                     out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), workspace.data_ptr(),
                                     workspace.numel(), _stream(stream)))
    return out


def single_target_csc(targets, sel, factor):
    """CSC view of select_and_factor outputs for targets 0..n-1 in order:
    column i holds [i, sel[i]...] with factor[i] (layout glue, no arithmetic)."""
    T, k = sel.shape
    rows = torch.cat([targets.view(T, 1), sel], dim=1).contiguous().view(-1)
    col_ptr = torch.arange(T + 1, dtype=torch.int64, device=sel.device) * (k + 1)
    return col_ptr, rows, factor.contiguous().view(-1)


def sum(x, out=None, stream=None):
    """Deterministic FP64 sum of a GPU float64 vector (csel_sum) -> 1-element tensor."""
    lib = load()
    _dev(x, torch.float64, "x")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(lib.csel_sum(x.data_ptr(), x.numel(), out.data_ptr(), _stream(stream)))
    return out
