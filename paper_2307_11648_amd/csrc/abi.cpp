// abi.cpp -- extern "C" entry points of libcsel: host-side validation, schedule
// choice and kernel launches.  No exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "csel.h"
#include "launch.hpp"

#define CSEL_API extern "C" __attribute__((visibility("default")))

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(CSEL_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int check_kernel(const csel_kernel* k) {
    if (!k) return fail(CSEL_EINVAL, "kernel is NULL");
    if (k->two_nu != 1 && k->two_nu != 3 && k->two_nu != 5)
        return fail(CSEL_EUNSUPPORTED, "two_nu must be 1, 3 or 5 (got %d)", k->two_nu);
    if (!(k->length_scale > 0.0) || !std::isfinite(k->length_scale))
        return fail(CSEL_EINVAL, "length_scale must be positive and finite");
    if (!(k->variance > 0.0) || !std::isfinite(k->variance))
        return fail(CSEL_EINVAL, "variance must be positive and finite");
    if (!(k->nugget >= 0.0) || !std::isfinite(k->nugget)) return fail(CSEL_EINVAL, "nugget must be >= 0 and finite");
    return CSEL_OK;
}

double c_nu(const csel_kernel* k) { return std::sqrt((double)k->two_nu) / k->length_scale; }

constexpr int kMaxPool = 512;
constexpr int kMaxSelect = 32;

}  // namespace

CSEL_API const char* csel_last_error(void) { return g_err; }

// the error slot, for the entry points defined in other sources (plan.cpp);
// code 0 clears it
extern "C" int csel_internal_fail(int code, const char* msg) {
    if (code == CSEL_OK) {
        g_err[0] = 0;
        return CSEL_OK;
    }
    return fail(code, "%s", msg);
}

CSEL_API int32_t csel_version(void) { return 1; }

CSEL_API int32_t csel_max_pool(void) { return kMaxPool; }

CSEL_API int32_t csel_max_select(void) { return kMaxSelect; }

CSEL_API int csel_select_and_factor(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                    int64_t n_targets, const int32_t* targets, const int32_t* pool_idx,
                                    const int32_t* pool_len, int32_t pool_stride, int32_t k, int32_t precision,
                                    int32_t* sel_idx, double* factor_val, double* log_condvar, float* top2_gap,
                                    uint8_t* status, hipStream_t stream) {
    g_err[0] = 0;
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n_targets < 0) return fail(CSEL_EINVAL, "n_targets must be >= 0");
    if (pool_stride < 0 || pool_stride > kMaxPool)
        return fail(CSEL_EUNSUPPORTED, "pool_stride must be in [0, %d] (got %d)", kMaxPool, pool_stride);
    if (k < 0 || k > kMaxSelect) return fail(CSEL_EUNSUPPORTED, "k must be in [0, %d] (got %d)", kMaxSelect, k);
    if (precision != CSEL_FP64 && precision != CSEL_MIXED)
        return fail(CSEL_EINVAL, "precision must be CSEL_FP64 or CSEL_MIXED");
    if (n_targets == 0) return CSEL_OK;
    if (!pts || !targets || !pool_len || !status || !factor_val || (k > 0 && !sel_idx) ||
        (pool_stride > 0 && !pool_idx))
        return fail(CSEL_EINVAL, "a required array is NULL");

    csel::SelectArgs a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.two_nu = kernel->two_nu;
    a.c_nu = c_nu(kernel);
    a.s2 = kernel->variance;
    a.nugget = kernel->nugget;
    a.n_targets = n_targets;
    a.targets = targets;
    a.pool = pool_idx;
    a.pool_len = pool_len;
    a.stride = pool_stride;
    a.k = k;
    a.sel = sel_idx;
    a.fac = factor_val;
    a.logcv = log_condvar;
    a.gap = top2_gap;
    a.status = status;
    a.col_list = nullptr;
    a.col_count = nullptr;
    a.n_waves = n_targets;
    const int rpl = pool_stride <= 64 ? 1 : pool_stride <= 128 ? 2 : pool_stride <= 256 ? 4 : 8;
    const int kmax = k <= 16 ? 16 : 32;
    hipError_t e = csel::launch_select_factor(a, precision, rpl, kmax, stream);
    if (e != hipSuccess) return hip_fail(e, "select_and_factor launch");
    return CSEL_OK;
}

CSEL_API int32_t csel_select_waves_per_column(int32_t pool_stride) {
    if (pool_stride < 0 || pool_stride > kMaxPool) return -1;
    return csel::select_mw_waves(pool_stride);
}

CSEL_API int csel_select_and_factor_sched(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                          int64_t n_targets, const int32_t* targets, const int32_t* pool_idx,
                                          const int32_t* pool_len, int32_t pool_stride, int32_t k, int32_t precision,
                                          const int32_t* col_list, const int32_t* col_count, int64_t max_cols,
                                          int32_t waves_per_column, int32_t* sel_idx, double* factor_val,
                                          double* log_condvar, uint8_t* status, hipStream_t stream) {
    g_err[0] = 0;
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n_targets < 0 || max_cols < 0) return fail(CSEL_EINVAL, "n_targets and max_cols must be >= 0");
    if (pool_stride < 0 || pool_stride > kMaxPool)
        return fail(CSEL_EUNSUPPORTED, "pool_stride must be in [0, %d] (got %d)", kMaxPool, pool_stride);
    if (k < 0 || k > kMaxSelect) return fail(CSEL_EUNSUPPORTED, "k must be in [0, %d] (got %d)", kMaxSelect, k);
    if (precision != CSEL_FP64 && precision != CSEL_MIXED)
        return fail(CSEL_EINVAL, "precision must be CSEL_FP64 or CSEL_MIXED");
    const int mw = csel::select_mw_waves(pool_stride);
    if (waves_per_column != 1 && waves_per_column != mw)
        return fail(CSEL_EUNSUPPORTED, "waves_per_column must be 1 or %d for pool_stride %d (got %d)", mw,
                    pool_stride, waves_per_column);
    if ((col_list == nullptr) != (col_count == nullptr)) return fail(CSEL_EINVAL, "col_list and col_count go together");
    const int64_t cols = col_list ? max_cols : n_targets;
    if (n_targets == 0 || cols == 0) return CSEL_OK;
    if (!pts || !targets || !pool_len || !status || !factor_val || (k > 0 && !sel_idx) ||
        (pool_stride > 0 && !pool_idx))
        return fail(CSEL_EINVAL, "a required array is NULL");
    csel::SelectArgs a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.two_nu = kernel->two_nu;
    a.c_nu = c_nu(kernel);
    a.s2 = kernel->variance;
    a.nugget = kernel->nugget;
    a.n_targets = n_targets;
    a.targets = targets;
    a.pool = pool_idx;
    a.pool_len = pool_len;
    a.stride = pool_stride;
    a.k = k;
    a.sel = sel_idx;
    a.fac = factor_val;
    a.logcv = log_condvar;
    a.gap = nullptr;
    a.status = status;
    a.col_list = col_list;
    a.col_count = col_count;
    a.n_waves = cols;
    const int rpl = pool_stride <= 64 ? 1 : pool_stride <= 128 ? 2 : pool_stride <= 256 ? 4 : 8;
    const int kmax = k <= 16 ? 16 : 32;
    hipError_t e = waves_per_column == 1 ? csel::launch_select_factor(a, precision, rpl, kmax, stream)
                                         : csel::launch_select_factor_mw(a, precision, kmax, stream);
    if (e != hipSuccess) return hip_fail(e, "select_and_factor_sched launch");
    return CSEL_OK;
}

CSEL_API int64_t csel_select_global_workspace_size(int64_t n_targets, int32_t k_max) {
    g_err[0] = 0;
    if (n_targets < 0 || n_targets > INT32_MAX)
        return fail(CSEL_EINVAL, "n_targets must be in [0, 2^31) (got %lld)", (long long)n_targets);
    if (k_max < 1 || k_max > kMaxSelect) return fail(CSEL_EUNSUPPORTED, "k_max must be in [1, %d]", kMaxSelect);
    return csel::global_workspace(n_targets, k_max);
}

CSEL_API int csel_select_global(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                int64_t n_targets, const int32_t* targets, const int32_t* pool_idx,
                                const int32_t* pool_len, int32_t pool_stride, int32_t k_max, int64_t budget,
                                int32_t precision, void* workspace, int64_t workspace_bytes, int32_t* k_alloc,
                                int32_t* sel_idx, double* factor_val, double* log_condvar, double* gain,
                                uint8_t* status, hipStream_t stream) {
    g_err[0] = 0;
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n_targets < 0 || n_targets > INT32_MAX)
        return fail(CSEL_EINVAL, "n_targets must be in [0, 2^31) (got %lld)", (long long)n_targets);
    if (pool_stride < 0 || pool_stride > kMaxPool)
        return fail(CSEL_EUNSUPPORTED, "pool_stride must be in [0, %d] (got %d)", kMaxPool, pool_stride);
    if (k_max < 1 || k_max > kMaxSelect) return fail(CSEL_EUNSUPPORTED, "k_max must be in [1, %d]", kMaxSelect);
    if (budget < 0) return fail(CSEL_EINVAL, "budget must be >= 0");
    if (precision != CSEL_FP64 && precision != CSEL_MIXED)
        return fail(CSEL_EINVAL, "precision must be CSEL_FP64 or CSEL_MIXED");
    if (n_targets == 0) return CSEL_OK;
    if (!pts || !targets || !pool_len || !status || !factor_val || !sel_idx || !k_alloc ||
        (pool_stride > 0 && !pool_idx))
        return fail(CSEL_EINVAL, "a required array is NULL");
    const int64_t need = csel::global_workspace(n_targets, k_max);
    if (!workspace || workspace_bytes < need)
        return fail(CSEL_EINVAL, "workspace must hold csel_select_global_workspace_size() = %lld bytes",
                    (long long)need);
    csel::SelectArgs a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.two_nu = kernel->two_nu;
    a.c_nu = c_nu(kernel);
    a.s2 = kernel->variance;
    a.nugget = kernel->nugget;
    a.n_targets = n_targets;
    a.targets = targets;
    a.pool = pool_idx;
    a.pool_len = pool_len;
    a.stride = pool_stride;
    a.k = k_max;
    a.sel = sel_idx;
    a.logcv = log_condvar;
    a.gain = gain;
    a.status = status;
    a.n_waves = n_targets;
    const int rpl = pool_stride <= 64 ? 1 : pool_stride <= 128 ? 2 : pool_stride <= 256 ? 4 : 8;
    hipError_t e = csel::launch_global(a, precision, rpl, budget, workspace, k_alloc, factor_val, stream);
    if (e != hipSuccess) return hip_fail(e, "select_global launch");
    return CSEL_OK;
}

CSEL_API int64_t csel_kernel_matvec_workspace_size(int64_t n) {
    g_err[0] = 0;
    if (n < 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [0, 2^31) (got %lld)", (long long)n);
    return csel::kmatvec_workspace(n);
}

CSEL_API int csel_kernel_matvec(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel, const double* x,
                                double* y, void* workspace, int64_t workspace_bytes, hipStream_t stream) {
    g_err[0] = 0;
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n < 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [0, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n == 0) return CSEL_OK;
    if (!pts || !x || !y) return fail(CSEL_EINVAL, "a required array is NULL");
    if (x == y) return fail(CSEL_EINVAL, "x and y must not alias");
    const int64_t need = csel::kmatvec_workspace(n);
    if (!workspace || workspace_bytes < need)
        return fail(CSEL_EINVAL, "workspace must hold csel_kernel_matvec_workspace_size() = %lld bytes",
                    (long long)need);
    hipError_t e = csel::launch_kmatvec(pts, n, dim, kernel->two_nu, c_nu(kernel), kernel->variance, kernel->nugget,
                                        x, y, workspace, stream);
    if (e != hipSuccess) return hip_fail(e, "kernel_matvec launch");
    return CSEL_OK;
}

CSEL_API int64_t csel_pcg_workspace_size(int64_t n) {
    g_err[0] = 0;
    if (n < 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [0, 2^31) (got %lld)", (long long)n);
    return csel::pcg_workspace(n);
}

CSEL_API int csel_pcg(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel, const int64_t* l_col_ptr,
                      const int32_t* l_row_idx, const double* l_val, const int64_t* lt_col_ptr,
                      const int32_t* lt_row_idx, const double* lt_val, const double* y, double* x, double rel_tol,
                      int32_t max_iter, void* workspace, int64_t workspace_bytes, int32_t* iterations,
                      double* rel_residual, hipStream_t stream) {
    g_err[0] = 0;
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n < 1 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (!(rel_tol > 0.0)) return fail(CSEL_EINVAL, "rel_tol must be > 0");
    if (max_iter < 0) return fail(CSEL_EINVAL, "max_iter must be >= 0");
    if (!pts || !y || !x || !iterations || !rel_residual) return fail(CSEL_EINVAL, "a required array is NULL");
    const bool precond = l_col_ptr != nullptr;
    if (precond && (!l_row_idx || !l_val || !lt_col_ptr || !lt_row_idx || !lt_val))
        return fail(CSEL_EINVAL, "the preconditioner needs L and L^T in CSC form");
    if (x == y) return fail(CSEL_EINVAL, "x and y must not alias");
    const int64_t need = csel::pcg_workspace(n);
    if (!workspace || workspace_bytes < need)
        return fail(CSEL_EINVAL, "workspace must hold csel_pcg_workspace_size() = %lld bytes", (long long)need);
    int it = 0;
    double res = 0.0;
    hipError_t e = csel::run_pcg(pts, n, dim, kernel->two_nu, c_nu(kernel), kernel->variance, kernel->nugget,
                                 l_col_ptr, l_row_idx, l_val, lt_col_ptr, lt_row_idx, lt_val, y, x, rel_tol, max_iter,
                                 workspace, &it, &res, stream);
    if (e != hipSuccess) return hip_fail(e, "pcg");
    *iterations = it;
    *rel_residual = res;
    return CSEL_OK;
}

CSEL_API int csel_sum(const double* x, int64_t n, double* out, hipStream_t stream) {
    g_err[0] = 0;
    if (n < 0) return fail(CSEL_EINVAL, "n must be >= 0");
    if (!out || (n > 0 && !x)) return fail(CSEL_EINVAL, "a required array is NULL");
    hipError_t e = csel::launch_sum(x, n, out, stream);
    if (e != hipSuccess) return hip_fail(e, "sum launch");
    return CSEL_OK;
}

CSEL_API int csel_apply_factor(int64_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* val,
                               int32_t transpose, const double* x, double* y, hipStream_t stream) {
    g_err[0] = 0;
    if (n < 0) return fail(CSEL_EINVAL, "n must be >= 0");
    if (transpose != 0 && transpose != 1) return fail(CSEL_EINVAL, "transpose must be 0 or 1");
    if (n == 0) return CSEL_OK;
    if (!col_ptr || !x || !y) return fail(CSEL_EINVAL, "a required array is NULL");
    if (x == y) return fail(CSEL_EINVAL, "x and y must not alias");
    hipError_t e = csel::launch_apply(n, col_ptr, row_idx, val, transpose, x, y, stream);
    if (e != hipSuccess) return hip_fail(e, "apply_factor launch");
    return CSEL_OK;
}

CSEL_API int64_t csel_transpose_factor_workspace_size(int64_t n, int64_t n_slots) {
    g_err[0] = 0;
    if (n < 0 || n >= INT32_MAX) return fail(CSEL_EINVAL, "n must be in [0, 2^31 - 1) (got %lld)", (long long)n);
    if (n_slots < 0 || n_slots > INT32_MAX)
        return fail(CSEL_EINVAL, "n_slots must be in [0, 2^31) (got %lld)", (long long)n_slots);
    const int64_t w = csel::transpose_factor_workspace(n, n_slots);
    if (w < 0) return fail(CSEL_EHIP, "radix sort could not size its temporary storage");
    return w;
}

CSEL_API int csel_transpose_factor(int64_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* val,
                                   int64_t n_slots, int64_t* t_col_ptr, int32_t* t_row_idx, double* t_val,
                                   void* workspace, int64_t workspace_bytes, hipStream_t stream) {
    g_err[0] = 0;
    const int64_t need = csel_transpose_factor_workspace_size(n, n_slots);
    if (need < 0) return (int)need;
    if (!col_ptr || !t_col_ptr) return fail(CSEL_EINVAL, "a required array is NULL");
    if (n_slots > 0 && (!row_idx || !val || !t_row_idx || !t_val)) return fail(CSEL_EINVAL, "a required array is NULL");
    if (n_slots > 0 && (!workspace || workspace_bytes < need))
        return fail(CSEL_EINVAL, "workspace too small: %lld bytes needed", (long long)need);
    hipError_t e = csel::launch_transpose_factor(n, col_ptr, row_idx, val, n_slots, t_col_ptr, t_row_idx, t_val,
                                                 workspace, stream);
    if (e != hipSuccess) return hip_fail(e, "transpose_factor launch");
    return CSEL_OK;
}

namespace {
constexpr int kAggMaxPool = 4096;
constexpr int kAggMaxMembers = 256;
constexpr int kAggMaxSelect = 256;

int check_agg(int64_t n_groups, int32_t pool_stride, int32_t max_members, int32_t k, int32_t precision) {
    if (n_groups < 0) return fail(CSEL_EINVAL, "n_groups must be >= 0");
    if (pool_stride < 0 || pool_stride > kAggMaxPool)
        return fail(CSEL_EUNSUPPORTED, "pool_stride must be in [0, %d] (got %d)", kAggMaxPool, pool_stride);
    if (max_members < 1 || max_members > kAggMaxMembers)
        return fail(CSEL_EUNSUPPORTED, "max_members must be in [1, %d] (got %d)", kAggMaxMembers, max_members);
    if (k < 0 || k > kAggMaxSelect) return fail(CSEL_EUNSUPPORTED, "k must be in [0, %d] (got %d)", kAggMaxSelect, k);
    if (pool_stride + max_members > 4096)
        return fail(CSEL_EUNSUPPORTED, "pool_stride + max_members must be <= 4096");
    if (precision != CSEL_FP64 && precision != CSEL_MIXED)
        return fail(CSEL_EINVAL, "precision must be CSEL_FP64 or CSEL_MIXED");
    return CSEL_OK;
}
}  // namespace

CSEL_API int64_t csel_aggregated_workspace_size(int64_t n_groups, int32_t pool_stride, int32_t max_members, int32_t k,
                                                int32_t precision) {
    g_err[0] = 0;
    if (check_agg(n_groups, pool_stride, max_members, k, precision)) return -1;
    return csel::plan_aggregated(n_groups, pool_stride, max_members, k, precision).ws_bytes;
}

CSEL_API int32_t csel_aggregated_max_block(void) { return csel::agg_factor_max_m(); }

CSEL_API int csel_aggregated_select_sched(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                          int64_t n_groups, const int32_t* group_ptr, const int32_t* members,
                                          int32_t max_members, const int32_t* pool_idx, const int32_t* pool_len,
                                          int32_t pool_stride, int32_t k, int32_t precision, void* workspace,
                                          int64_t workspace_bytes, int32_t* sel_idx, float* top2_gap,
                                          double* group_logdet, double* post_var, const int64_t* val_ptr,
                                          int32_t* factor_rows, double* factor_val, double* member_log_condvar,
                                          uint8_t* status, int32_t schedule, hipStream_t stream) {
    g_err[0] = 0;
    if (schedule < CSEL_AGG_AUTO || schedule > CSEL_AGG_SPLIT_1024)
        return fail(CSEL_EINVAL, "schedule must be one of the CSEL_AGG_ values (got %d)", schedule);
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    rc = check_agg(n_groups, pool_stride, max_members, k, precision);
    if (rc) return rc;
    if (n_groups == 0) return CSEL_OK;
    const bool want_factor = factor_val != nullptr;
    if (!pts || !group_ptr || !members || !pool_len || !status || (k > 0 && !sel_idx) ||
        (pool_stride > 0 && !pool_idx))
        return fail(CSEL_EINVAL, "a required array is NULL");
    if (want_factor && (!val_ptr || !factor_rows))
        return fail(CSEL_EINVAL, "factor output needs val_ptr, factor_rows and factor_val");
    if (post_var && precision != CSEL_FP64)
        return fail(CSEL_EUNSUPPORTED,
                    "post_var needs CSEL_FP64: the FP32 factor of the picks does not resolve posterior variances "
                    "far below the prior variance");
    const csel::AggPlan pl = csel::plan_aggregated(n_groups, pool_stride, max_members, k, precision);
    if (!workspace || workspace_bytes < pl.ws_bytes)
        return fail(CSEL_EINVAL, "workspace must hold csel_aggregated_workspace_size() = %lld bytes",
                    (long long)pl.ws_bytes);
    csel::AggArgs a;
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.two_nu = kernel->two_nu;
    a.c_nu = c_nu(kernel);
    a.s2 = kernel->variance;
    a.nugget = kernel->nugget;
    a.n_groups = n_groups;
    a.group_ptr = group_ptr;
    a.members = members;
    a.max_members = max_members;
    a.pool = pool_idx;
    a.pool_len = pool_len;
    a.stride = pool_stride;
    a.k = k;
    a.later_only = want_factor ? 1 : 0;
    a.ws = workspace;
    a.slab_bytes = pl.slab_bytes;
    a.rmax = pl.rmax;
    a.sel = sel_idx;
    a.gap = top2_gap;
    a.logdet = group_logdet;
    a.post_var = post_var;
    a.status = status;
    a.val_ptr = val_ptr;
    a.fac_rows = factor_rows;
    a.fac_val = factor_val;
    a.member_logcv = member_log_condvar;
    hipError_t e = csel::launch_aggregated(a, pl, precision, want_factor, schedule, stream);
    if (e == hipErrorNotSupported)
        return fail(CSEL_EUNSUPPORTED, "schedule %d does not apply to this request (register: mixed, no post_var, "
                    "pools <= 512, groups <= 32, k <= 64; split: no factor output, <= 1024 groups, k <= 256, "
                    "groups <= 128)", schedule);
    if (e == hipErrorCooperativeLaunchTooLarge)
        return fail(CSEL_EUNSUPPORTED, "the split schedule's workgroups do not all fit on the device at once");
    if (e != hipSuccess) return hip_fail(e, "aggregated_select launch");
    return CSEL_OK;
}

CSEL_API int csel_aggregated_select(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                    int64_t n_groups, const int32_t* group_ptr, const int32_t* members,
                                    int32_t max_members, const int32_t* pool_idx, const int32_t* pool_len,
                                    int32_t pool_stride, int32_t k, int32_t precision, void* workspace,
                                    int64_t workspace_bytes, int32_t* sel_idx, float* top2_gap,
                                    double* group_logdet, double* post_var, const int64_t* val_ptr,
                                    int32_t* factor_rows, double* factor_val, double* member_log_condvar,
                                    uint8_t* status, hipStream_t stream) {
    return csel_aggregated_select_sched(pts, n, dim, kernel, n_groups, group_ptr, members, max_members, pool_idx,
                                        pool_len, pool_stride, k, precision, workspace, workspace_bytes, sel_idx,
                                        top2_gap, group_logdet, post_var, val_ptr, factor_rows, factor_val,
                                        member_log_condvar, status, CSEL_AGG_AUTO, stream);
}

CSEL_API int64_t csel_later_knn_workspace_size(int64_t n, int32_t dim) {
    g_err[0] = 0;
    if (n < 0 || n > INT32_MAX) {
        fail(CSEL_EINVAL, "n must be in [0, 2^31)");
        return -1;
    }
    if (dim < 1 || dim > 3) {
        fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
        return -1;
    }
    const int64_t b = csel::later_knn_workspace(n, dim);
    if (b < 0) fail(CSEL_EUNSUPPORTED, "later_knn: cannot size the workspace");
    return b;
}

CSEL_API int csel_later_knn(const double* pts, int64_t n, int32_t dim, int32_t C, void* workspace,
                            int64_t workspace_bytes, int32_t* pool_idx, int32_t* pool_len, hipStream_t stream) {
    g_err[0] = 0;
    if (n < 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [0, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (C < 0 || C > csel::later_knn_max_pool())
        return fail(CSEL_EUNSUPPORTED, "C must be in [0, %d] (got %d)", csel::later_knn_max_pool(), C);
    if (n == 0) return CSEL_OK;
    if (!pts || !pool_len || (C > 0 && !pool_idx)) return fail(CSEL_EINVAL, "a required array is NULL");
    const int64_t need = csel::later_knn_workspace(n, dim);
    if (need < 0) return fail(CSEL_EUNSUPPORTED, "later_knn: cannot size the workspace");
    if (!workspace || workspace_bytes < need)
        return fail(CSEL_EINVAL, "workspace must hold csel_later_knn_workspace_size() = %lld bytes",
                    (long long)need);
    hipError_t e = csel::launch_later_knn(pts, n, dim, C, workspace, pool_idx, pool_len, stream);
    if (e != hipSuccess) return hip_fail(e, "later_knn launch");
    return CSEL_OK;
}

CSEL_API int64_t csel_reverse_maximin_workspace_size(int64_t n, int32_t dim) {
    g_err[0] = 0;
    if (n < 0 || n > INT32_MAX) {
        fail(CSEL_EINVAL, "n must be in [0, 2^31)");
        return -1;
    }
    if (dim < 1 || dim > 3) {
        fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
        return -1;
    }
    const int64_t b = csel::reverse_maximin_workspace(n, dim);
    if (b < 0) fail(CSEL_EUNSUPPORTED, "reverse_maximin: cannot size the workspace");
    return b;
}

CSEL_API int csel_reverse_maximin(const double* pts, int64_t n, int32_t dim, void* workspace, int64_t workspace_bytes,
                                  int32_t* order, double* ell, int32_t* rounds, hipStream_t stream) {
    g_err[0] = 0;
    if (n < 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [0, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (rounds) *rounds = 0;
    if (n == 0) return CSEL_OK;
    if (!pts || !order || !ell) return fail(CSEL_EINVAL, "a required array is NULL");
    const int64_t need = csel::reverse_maximin_workspace(n, dim);
    if (need < 0) return fail(CSEL_EUNSUPPORTED, "reverse_maximin: cannot size the workspace");
    if (!workspace || workspace_bytes < need)
        return fail(CSEL_EINVAL, "workspace must hold csel_reverse_maximin_workspace_size() = %lld bytes",
                    (long long)need);
    hipError_t e = csel::launch_reverse_maximin(pts, n, dim, workspace, order, ell, stream, rounds);
    if (e == hipErrorUnknown) return fail(CSEL_EHIP, "reverse_maximin: the rounds stopped making progress");
    if (e != hipSuccess) return hip_fail(e, "reverse_maximin");
    return CSEL_OK;
}

CSEL_API int csel_partial_select(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                 int64_t n_groups, const int32_t* group_ptr, const int32_t* members,
                                 int32_t max_members, const int32_t* pool_idx, const int32_t* pool_len,
                                 int32_t pool_stride, int32_t k, int32_t* sel_idx, float* top2_gap,
                                 double* group_logdet, const int64_t* val_ptr, int32_t* factor_rows,
                                 double* factor_val, double* member_log_condvar, uint8_t* status,
                                 hipStream_t stream) {
    g_err[0] = 0;
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n_groups < 0 || n_groups > INT32_MAX) return fail(CSEL_EINVAL, "n_groups must be in [0, 2^31)");
    if (pool_stride < 0 || pool_stride > csel::partial_max_pool())
        return fail(CSEL_EUNSUPPORTED, "pool_stride must be in [0, %d] (got %d)", csel::partial_max_pool(),
                    pool_stride);
    if (max_members < 1 || max_members > csel::partial_max_members())
        return fail(CSEL_EUNSUPPORTED, "max_members must be in [1, %d] (got %d)", csel::partial_max_members(),
                    max_members);
    if (k < 0 || k > csel::partial_max_k())
        return fail(CSEL_EUNSUPPORTED, "k must be in [0, %d] (got %d)", csel::partial_max_k(), k);
    if (n_groups == 0) return CSEL_OK;
    const bool want_factor = factor_val != nullptr;
    if (!pts || !group_ptr || !members || !pool_len || !status || (k > 0 && !sel_idx) ||
        (pool_stride > 0 && !pool_idx))
        return fail(CSEL_EINVAL, "a required array is NULL");
    if (want_factor && (!val_ptr || !factor_rows))
        return fail(CSEL_EINVAL, "factor output needs val_ptr, factor_rows and factor_val");
    csel::AggArgs a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.two_nu = kernel->two_nu;
    a.c_nu = c_nu(kernel);
    a.s2 = kernel->variance;
    a.nugget = kernel->nugget;
    a.n_groups = n_groups;
    a.group_ptr = group_ptr;
    a.members = members;
    a.max_members = max_members;
    a.pool = pool_idx;
    a.pool_len = pool_len;
    a.stride = pool_stride;
    a.k = k;
    a.sel = sel_idx;
    a.gap = top2_gap;
    a.logdet = group_logdet;
    a.status = status;
    a.val_ptr = val_ptr;
    a.fac_rows = factor_rows;
    a.fac_val = factor_val;
    a.member_logcv = member_log_condvar;
    hipError_t e = csel::launch_partial(a, want_factor, stream);
    if (e != hipSuccess) return hip_fail(e, "partial_select launch");
    return CSEL_OK;
}

CSEL_API int csel_select_and_factor_list(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                         int64_t n_targets, const int32_t* targets, const int32_t* pool_idx,
                                         const int32_t* pool_len, int32_t pool_stride, int32_t k, int32_t precision,
                                         const int32_t* col_list, const int32_t* col_count, int64_t max_cols,
                                         int32_t* sel_idx, double* factor_val, double* log_condvar,
                                         float* top2_gap, uint8_t* status, hipStream_t stream) {
    g_err[0] = 0;
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n_targets < 0 || max_cols < 0) return fail(CSEL_EINVAL, "n_targets and max_cols must be >= 0");
    if (pool_stride < 0 || pool_stride > kMaxPool)
        return fail(CSEL_EUNSUPPORTED, "pool_stride must be in [0, %d] (got %d)", kMaxPool, pool_stride);
    if (k < 0 || k > kMaxSelect) return fail(CSEL_EUNSUPPORTED, "k must be in [0, %d] (got %d)", kMaxSelect, k);
    if (precision != CSEL_FP64 && precision != CSEL_MIXED)
        return fail(CSEL_EINVAL, "precision must be CSEL_FP64 or CSEL_MIXED");
    if (n_targets == 0 || max_cols == 0) return CSEL_OK;
    if (!col_list || !col_count) return fail(CSEL_EINVAL, "col_list and col_count are required");
    if (!pts || !targets || !pool_len || !status || !factor_val || (k > 0 && !sel_idx) ||
        (pool_stride > 0 && !pool_idx))
        return fail(CSEL_EINVAL, "a required array is NULL");
    csel::SelectArgs a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.two_nu = kernel->two_nu;
    a.c_nu = c_nu(kernel);
    a.s2 = kernel->variance;
    a.nugget = kernel->nugget;
    a.n_targets = n_targets;
    a.targets = targets;
    a.pool = pool_idx;
    a.pool_len = pool_len;
    a.stride = pool_stride;
    a.k = k;
    a.sel = sel_idx;
    a.fac = factor_val;
    a.logcv = log_condvar;
    a.gap = top2_gap;
    a.status = status;
    a.col_list = col_list;
    a.col_count = col_count;
    const int rpl = pool_stride <= 64 ? 1 : pool_stride <= 128 ? 2 : pool_stride <= 256 ? 4 : 8;
    const int kmax = k <= 16 ? 16 : 32;
    // the grid covers max_cols list entries; waves beyond *col_count exit at once
    a.n_waves = max_cols;
    hipError_t e = csel::launch_select_factor(a, precision, rpl, kmax, stream);
    if (e != hipSuccess) return hip_fail(e, "select_and_factor_list launch");
    return CSEL_OK;
}

namespace {
constexpr int kScreenMaxPool = 512;
}

static int screen_common(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel, int64_t n_targets,
                         const int32_t* targets, const int32_t* pool_idx, const int32_t* pool_len,
                         int32_t pool_stride, csel::ScreenArgs& a) {
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n_targets < 0 || n_targets > INT32_MAX)
        return fail(CSEL_EINVAL, "n_targets must be in [0, 2^31) (got %lld)", (long long)n_targets);
    if (pool_stride < 1 || pool_stride > kScreenMaxPool)
        return fail(CSEL_EUNSUPPORTED, "pool_stride must be in [1, %d] (got %d)", kScreenMaxPool, pool_stride);
    if (n_targets > 0 && (!pts || !targets || !pool_idx || !pool_len))
        return fail(CSEL_EINVAL, "a required array is NULL");
    a = csel::ScreenArgs{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.two_nu = kernel->two_nu;
    a.c_nu = c_nu(kernel);
    a.s2 = kernel->variance;
    a.nugget = kernel->nugget;
    a.ell = kernel->length_scale;
    a.n_targets = n_targets;
    a.targets = targets;
    a.pool = pool_idx;
    a.pool_len = pool_len;
    a.stride = pool_stride;
    return CSEL_OK;
}

static int screen_rpl(int32_t stride) { return stride <= 64 ? 1 : stride <= 128 ? 2 : stride <= 256 ? 4 : 8; }

CSEL_API int32_t csel_mlp_num_params(void) { return csel::mlp_nparams(); }

CSEL_API int csel_screen_features(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                  int64_t n_targets, const int32_t* targets, const int32_t* pool_idx,
                                  const int32_t* pool_len, int32_t pool_stride, float* features,
                                  hipStream_t stream) {
    g_err[0] = 0;
    csel::ScreenArgs a;
    int rc = screen_common(pts, n, dim, kernel, n_targets, targets, pool_idx, pool_len, pool_stride, a);
    if (rc) return rc;
    if (n_targets == 0) return CSEL_OK;
    if (!features) return fail(CSEL_EINVAL, "features is NULL");
    a.mode = 1;
    a.feats = features;
    a.keep = 1;
    a.kept = nullptr;
    a.kept_len = nullptr;
    a.fallback = nullptr;
    hipError_t e = csel::launch_screen(a, screen_rpl(pool_stride), stream);
    if (e != hipSuccess) return hip_fail(e, "screen_features launch");
    return CSEL_OK;
}

CSEL_API int csel_screen(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel, int64_t n_targets,
                         const int32_t* targets, const int32_t* pool_idx, const int32_t* pool_len,
                         int32_t pool_stride, const float* params, const uint16_t* params_bf16, int32_t keep,
                         float fallback_threshold, int32_t* kept_idx, int32_t* kept_len, uint8_t* fallback,
                         float* logits, int32_t* fallback_list, int32_t* fallback_count, const int32_t* order,
                         int64_t n_order, hipStream_t stream) {
    g_err[0] = 0;
    csel::ScreenArgs a;
    int rc = screen_common(pts, n, dim, kernel, n_targets, targets, pool_idx, pool_len, pool_stride, a);
    if (rc) return rc;
    if (keep < 1 || keep > pool_stride) return fail(CSEL_EINVAL, "keep must be in [1, pool_stride]");
    if (!(fallback_threshold >= 0.0f)) return fail(CSEL_EINVAL, "fallback_threshold must be >= 0");
    if ((fallback_list == nullptr) != (fallback_count == nullptr))
        return fail(CSEL_EINVAL, "fallback_list and fallback_count go together");
    if (n_targets == 0) {
        if (fallback_count) {
            hipError_t e = csel::launch_fill_i32(fallback_count, 1, 0, stream);
            if (e != hipSuccess) return hip_fail(e, "fill launch");
        }
        return CSEL_OK;
    }
    if (!params || !params_bf16 || !kept_idx || !kept_len || !fallback)
        return fail(CSEL_EINVAL, "a required array is NULL");
    a.params = params;
    a.params_bf16 = params_bf16;
    a.keep = keep;
    a.fb_thr = fallback_threshold;
    a.mode = 0;
    a.logits = logits;
    a.kept = kept_idx;
    a.kept_len = kept_len;
    a.fallback = fallback;
    a.fb_list = fallback_list;
    a.fb_count = fallback_count;
    // each processed position appends at most one entry to the fallback list,
    // which holds n_targets entries
    if (order && (n_order < 0 || n_order > n_targets))
        return fail(CSEL_EINVAL, "n_order must be in [0, n_targets] (got %lld)", (long long)n_order);
    a.order = order;
    a.n_order = order ? n_order : n_targets;
    if (fallback_count) {
        hipError_t e = csel::launch_fill_i32(fallback_count, 1, 0, stream);
        if (e != hipSuccess) return hip_fail(e, "fill launch");
    }
    hipError_t e = csel::launch_screen(a, screen_rpl(pool_stride), stream);
    if (e != hipSuccess) return hip_fail(e, "screen launch");
    return CSEL_OK;
}

CSEL_API int csel_screen_groups(const double* pts, int64_t n, int32_t dim, const csel_kernel* kernel,
                                int64_t n_groups, const int32_t* group_ptr, const int32_t* members,
                                int64_t n_members, const int32_t* pool_idx, const int32_t* pool_len,
                                int32_t pool_stride, const float* params, const uint16_t* params_bf16,
                                int32_t keep, float fallback_threshold, int32_t* kept_idx, int32_t* kept_len,
                                uint8_t* fallback, float* logits, float* features, hipStream_t stream) {
    g_err[0] = 0;
    int rc = check_kernel(kernel);
    if (rc) return rc;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n_groups < 0 || n_groups > INT32_MAX)
        return fail(CSEL_EINVAL, "n_groups must be in [0, 2^31) (got %lld)", (long long)n_groups);
    if (n_members < 0) return fail(CSEL_EINVAL, "n_members must be >= 0");
    if (pool_stride < 1 || pool_stride > csel::kGroupScreenMaxPool)
        return fail(CSEL_EUNSUPPORTED, "pool_stride must be in [1, %d] (got %d)", csel::kGroupScreenMaxPool,
                    pool_stride);
    const bool features_only = params == nullptr;
    if (features_only && !features) return fail(CSEL_EINVAL, "params and features are both NULL");
    if (!features_only) {
        if (keep < 1 || keep > pool_stride) return fail(CSEL_EINVAL, "keep must be in [1, pool_stride]");
        if (!(fallback_threshold >= 0.0f)) return fail(CSEL_EINVAL, "fallback_threshold must be >= 0");
    }
    if (n_groups == 0) return CSEL_OK;
    if (!pts || !group_ptr || !members || !pool_idx || !pool_len) return fail(CSEL_EINVAL, "a required array is NULL");
    if (!features_only && (!params_bf16 || !kept_idx || !kept_len || !fallback))
        return fail(CSEL_EINVAL, "a required array is NULL");
    csel::GroupScreenArgs a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.two_nu = kernel->two_nu;
    a.c_nu = c_nu(kernel);
    a.ell = kernel->length_scale;
    a.n_groups = n_groups;
    a.group_ptr = group_ptr;
    a.members = members;
    a.n_members = n_members;
    a.pool = pool_idx;
    a.pool_len = pool_len;
    a.stride = pool_stride;
    a.params = params;
    a.params_bf16 = params_bf16;
    a.keep = keep;
    a.fb_thr = fallback_threshold;
    a.mode = features_only ? 1 : 0;
    a.feats = features;
    a.logits = logits;
    a.kept = kept_idx;
    a.kept_len = kept_len;
    a.fallback = fallback;
    hipError_t e = csel::launch_screen_groups(a, stream);
    if (e != hipSuccess) return hip_fail(e, "screen_groups launch");
    return CSEL_OK;
}

CSEL_API int64_t csel_spatial_order_workspace_size(int64_t n_targets) {
    g_err[0] = 0;
    if (n_targets < 0 || n_targets > INT32_MAX)
        return fail(CSEL_EINVAL, "n_targets must be in [0, 2^31) (got %lld)", (long long)n_targets);
    const int64_t w = csel::spatial_order_workspace(n_targets);
    if (w < 0) return fail(CSEL_EHIP, "radix sort could not size its temporary storage");
    return w;
}

CSEL_API int csel_spatial_order(const double* pts, int64_t n, int32_t dim, int64_t n_targets,
                                const int32_t* targets, void* workspace, int64_t workspace_bytes, int32_t* order,
                                hipStream_t stream) {
    g_err[0] = 0;
    if (n <= 0 || n > INT32_MAX) return fail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return fail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (n_targets < 0 || n_targets > INT32_MAX)
        return fail(CSEL_EINVAL, "n_targets must be in [0, 2^31) (got %lld)", (long long)n_targets);
    if (n_targets == 0) return CSEL_OK;
    if (!pts || !targets || !order) return fail(CSEL_EINVAL, "a required array is NULL");
    const int64_t need = csel::spatial_order_workspace(n_targets);
    if (need < 0) return fail(CSEL_EHIP, "radix sort could not size its temporary storage");
    if (!workspace || workspace_bytes < need)
        return fail(CSEL_EINVAL, "workspace too small: %lld bytes needed", (long long)need);
    hipError_t e = csel::launch_spatial_order(pts, n, dim, n_targets, targets, workspace, order, stream);
    if (e != hipSuccess) return hip_fail(e, "spatial order launch");
    return CSEL_OK;
}

CSEL_API int64_t csel_mlp_grad_workspace_size(int64_t n_rows) {
    g_err[0] = 0;
    if (n_rows < 0) return fail(CSEL_EINVAL, "n_rows must be >= 0");
    return csel::mlp_grad_nparts(n_rows) * (int64_t)(csel::mlp_nparams() + 1) * (int64_t)sizeof(float);
}

CSEL_API int csel_mlp_forward(const float* params, const uint16_t* params_bf16, const float* x, int64_t n_rows,
                              float* logits, hipStream_t stream) {
    g_err[0] = 0;
    if (n_rows < 0) return fail(CSEL_EINVAL, "n_rows must be >= 0");
    if (n_rows == 0) return CSEL_OK;
    if (!params || !params_bf16 || !x || !logits) return fail(CSEL_EINVAL, "a required array is NULL");
    csel::MlpTrainArgs a{};
    a.params = params;
    a.params_bf16 = params_bf16;
    a.x = x;
    a.n_rows = n_rows;
    hipError_t e = csel::launch_mlp_forward(a, logits, stream);
    if (e != hipSuccess) return hip_fail(e, "mlp_forward launch");
    return CSEL_OK;
}

CSEL_API int csel_mlp_grad(const float* params, const uint16_t* params_bf16, const float* x, const uint8_t* labels,
                           int64_t n_rows, float pos_weight, void* workspace, int64_t workspace_bytes, float* grad,
                           hipStream_t stream) {
    g_err[0] = 0;
    if (n_rows < 0) return fail(CSEL_EINVAL, "n_rows must be >= 0");
    if (!(pos_weight > 0.0f)) return fail(CSEL_EINVAL, "pos_weight must be > 0");
    if (!params || !params_bf16 || !grad || (n_rows > 0 && (!x || !labels)))
        return fail(CSEL_EINVAL, "a required array is NULL");
    const int64_t need = csel::mlp_grad_nparts(n_rows) * (int64_t)(csel::mlp_nparams() + 1) * (int64_t)sizeof(float);
    if (need > 0 && (!workspace || workspace_bytes < need))
        return fail(CSEL_EINVAL, "workspace must hold csel_mlp_grad_workspace_size() = %lld bytes", (long long)need);
    csel::MlpTrainArgs a{};
    a.params = params;
    a.params_bf16 = params_bf16;
    a.x = x;
    a.y = labels;
    a.n_rows = n_rows;
    a.pos_weight = pos_weight;
    a.inv_n = n_rows > 0 ? 1.0f / (float)n_rows : 0.0f;
    a.partials = reinterpret_cast<float*>(workspace);
    hipError_t e = csel::launch_mlp_grad(a, grad, stream);
    if (e != hipSuccess) return hip_fail(e, "mlp_grad launch");
    return CSEL_OK;
}

CSEL_API int csel_mlp_grad_noalloc(const float* params, const uint16_t* params_bf16, const float* x,
                                   const uint8_t* labels, int64_t n_rows, float pos_weight, float* grad,
                                   hipStream_t stream) {
    g_err[0] = 0;
    static_assert(CSEL_MLP_GRAD_NOALLOC_MAX_ROWS == csel::kMlpGradNoAllocMaxRows, "header and library agree");
    if (n_rows < 0) return fail(CSEL_EINVAL, "n_rows must be >= 0");
    if (n_rows > CSEL_MLP_GRAD_NOALLOC_MAX_ROWS)
        return fail(CSEL_EUNSUPPORTED, "n_rows must be <= %d for csel_mlp_grad_noalloc (got %lld); use csel_mlp_grad",
                    CSEL_MLP_GRAD_NOALLOC_MAX_ROWS, (long long)n_rows);
    if (!(pos_weight > 0.0f)) return fail(CSEL_EINVAL, "pos_weight must be > 0");
    if (!params || !params_bf16 || !grad || (n_rows > 0 && (!x || !labels)))
        return fail(CSEL_EINVAL, "a required array is NULL");
    csel::MlpTrainArgs a{};
    a.params = params;
    a.params_bf16 = params_bf16;
    a.x = x;
    a.y = labels;
    a.n_rows = n_rows;
    a.pos_weight = pos_weight;
    a.inv_n = n_rows > 0 ? 1.0f / (float)n_rows : 0.0f;
    hipError_t e = csel::launch_mlp_grad_noalloc(a, grad, stream);
    if (e != hipSuccess) return hip_fail(e, "mlp_grad_noalloc");
    return CSEL_OK;
}

CSEL_API int csel_mlp_adam(float* params, uint16_t* params_bf16, const float* grad, float* m, float* v,
                           int32_t n_params, float lr, float beta1, float beta2, float eps, int32_t step,
                           hipStream_t stream) {
    g_err[0] = 0;
    if (n_params != csel::mlp_nparams()) return fail(CSEL_EINVAL, "n_params must be csel_mlp_num_params()");
    if (step < 1) return fail(CSEL_EINVAL, "step counts from 1");
    if (!params || !params_bf16 || !grad || !m || !v) return fail(CSEL_EINVAL, "a required array is NULL");
    hipError_t e = csel::launch_adam(params, params_bf16, grad, m, v, n_params, lr, beta1, beta2, eps, step, stream);
    if (e != hipSuccess) return hip_fail(e, "adam launch");
    return CSEL_OK;
}

CSEL_API int csel_mlp_to_bf16(const float* params, uint16_t* params_bf16, int32_t n_params, hipStream_t stream) {
    g_err[0] = 0;
    if (n_params < 0) return fail(CSEL_EINVAL, "n_params must be >= 0");
    if (n_params == 0) return CSEL_OK;
    if (!params || !params_bf16) return fail(CSEL_EINVAL, "a required array is NULL");
    hipError_t e = csel::launch_to_bf16(params, params_bf16, n_params, stream);
    if (e != hipSuccess) return hip_fail(e, "to_bf16 launch");
    return CSEL_OK;
}
