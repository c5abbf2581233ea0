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

    csel::SelectArgs a;
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
    const int rpl = pool_stride <= 64 ? 1 : pool_stride <= 128 ? 2 : pool_stride <= 256 ? 4 : 8;
    const int kmax = k <= 16 ? 16 : 32;
    hipError_t e = csel::launch_select_factor(a, precision, rpl, kmax, stream);
    if (e != hipSuccess) return hip_fail(e, "select_and_factor launch");
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
