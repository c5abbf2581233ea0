// plan.cpp -- the screened-selection plan: one C call for the whole learned-
// screened step (screen, greedy selection on the kept pools, greedy selection
// on the full pools of the fallback columns), with the buffers between the
// stages, the tuned column schedule and an optional captured HIP graph owned
// by the plan.  No exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "csel.h"
#include "launch.hpp"

#define CSEL_API extern "C" __attribute__((visibility("default")))

// the error slot of the calling thread (abi.cpp)
extern "C" int csel_internal_fail(int code, const char* msg);

namespace {

int pfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return csel_internal_fail(code, buf);
}

int phip(hipError_t e, const char* what) { return pfail(CSEL_EHIP, "%s: %s", what, hipGetErrorString(e)); }

constexpr int kPlanMaxPool = 512;
constexpr int kPlanMaxSelect = 32;
// below this many columns the natural order is used untimed
constexpr int64_t kTuneMinColumns = 4096;

// the arguments a captured graph was recorded with
struct StepKey {
    const double* pts;
    int64_t n;
    int32_t dim;
    csel_kernel kernel;
    const int32_t* targets;
    const int32_t* pool_idx;
    const int32_t* pool_len;
    const float* params;
    const uint16_t* params_bf16;
    float threshold;
    int32_t* sel;
    double* fac;
    double* logcv;
    uint8_t* status;
};

bool same_key(const StepKey& a, const StepKey& b) {
    return a.pts == b.pts && a.n == b.n && a.dim == b.dim && a.kernel.two_nu == b.kernel.two_nu &&
           a.kernel.length_scale == b.kernel.length_scale && a.kernel.variance == b.kernel.variance &&
           a.kernel.nugget == b.kernel.nugget && a.targets == b.targets && a.pool_idx == b.pool_idx &&
           a.pool_len == b.pool_len && a.params == b.params && a.params_bf16 == b.params_bf16 &&
           a.threshold == b.threshold && a.sel == b.sel && a.fac == b.fac && a.logcv == b.logcv &&
           a.status == b.status;
}

}  // namespace

struct csel_plan {
    int device = 0;
    int64_t n_targets = 0;
    int32_t stride = 0, keep = 0, k = 0, precision = 0;
    uint32_t flags = 0;
    // device buffers between the stages
    int32_t* kept = nullptr;      // [T][keep]
    int32_t* kept_len = nullptr;  // [T]
    uint8_t* fallback = nullptr;  // [T]
    int32_t* fb_list = nullptr;   // [T]
    int32_t* fb_count = nullptr;  // [1]
    int32_t* order = nullptr;     // [T] processing order (valid when has_order)
    int32_t* n_all = nullptr;     // [1] = T, the count of the order as a list
    void* order_ws = nullptr;
    int64_t order_ws_bytes = 0;
    bool has_order = false;
    // the kept-pool selection's schedule, -1 untuned: bit 0 the Morton column
    // order (else natural), bit 1 the multi-wave schedule (else one wave per
    // column); and the fallback launch's waves per column
    int schedule = -1;
    int fb_waves = 1;
    float tune_ms[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    // the captured step
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool has_graph = false;
    StepKey key{};
};

namespace {

void free_plan(csel_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    void* bufs[] = {p->kept, p->kept_len, p->fallback, p->fb_list, p->fb_count, p->order, p->n_all, p->order_ws};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

csel::SelectArgs select_args(const csel_plan* p, const StepKey& a) {
    csel::SelectArgs s{};
    s.pts = a.pts;
    s.n = a.n;
    s.dim = a.dim;
    s.two_nu = a.kernel.two_nu;
    s.c_nu = std::sqrt((double)a.kernel.two_nu) / a.kernel.length_scale;
    s.s2 = a.kernel.variance;
    s.nugget = a.kernel.nugget;
    s.n_targets = p->n_targets;
    s.targets = a.targets;
    s.k = p->k;
    s.sel = a.sel;
    s.fac = a.fac;
    s.logcv = a.logcv;
    s.gap = nullptr;
    s.status = a.status;
    return s;
}

int rpl_of(int32_t stride) { return stride <= 64 ? 1 : stride <= 128 ? 2 : stride <= 256 ? 4 : 8; }
int kmax_of(int32_t k) { return k <= 16 ? 16 : 32; }

// the greedy selection on the kept pools under a schedule (see csel_plan)
hipError_t enqueue_kept(const csel_plan* p, const StepKey& a, int schedule, hipStream_t s) {
    csel::SelectArgs sa = select_args(p, a);
    sa.pool = p->kept;
    sa.pool_len = p->kept_len;
    sa.stride = p->keep;
    if (schedule & 1) {
        sa.col_list = p->order;
        sa.col_count = p->n_all;
    }
    sa.n_waves = p->n_targets;
    if (schedule & 2) return csel::launch_select_factor_mw(sa, p->precision, kmax_of(p->k), s);
    return csel::launch_select_factor(sa, p->precision, rpl_of(p->keep), kmax_of(p->k), s);
}

hipError_t enqueue_screen(const csel_plan* p, const StepKey& a, hipStream_t s) {
    hipError_t e = csel::launch_fill_i32(p->fb_count, 1, 0, s);
    if (e != hipSuccess) return e;
    csel::ScreenArgs sa{};
    sa.pts = a.pts;
    sa.n = a.n;
    sa.dim = a.dim;
    sa.two_nu = a.kernel.two_nu;
    sa.c_nu = std::sqrt((double)a.kernel.two_nu) / a.kernel.length_scale;
    sa.s2 = a.kernel.variance;
    sa.nugget = a.kernel.nugget;
    sa.ell = a.kernel.length_scale;
    sa.n_targets = p->n_targets;
    sa.targets = a.targets;
    sa.pool = a.pool_idx;
    sa.pool_len = a.pool_len;
    sa.stride = p->stride;
    sa.params = a.params;
    sa.params_bf16 = a.params_bf16;
    sa.keep = p->keep;
    sa.fb_thr = a.threshold;
    sa.mode = 0;
    sa.kept = p->kept;
    sa.kept_len = p->kept_len;
    sa.fallback = p->fallback;
    sa.fb_list = p->fb_list;
    sa.fb_count = p->fb_count;
    sa.order = p->has_order ? p->order : nullptr;
    sa.n_order = p->n_targets;
    return csel::launch_screen(sa, rpl_of(p->stride), s);
}

// full-pool selection of the listed fallback columns: the launch covers
// every column's list position (the list's capacity), and the waves past the
// device-side count exit at once, so the launch needs no host read of the
// count (a grid-stride loop over the list would keep the selection's
// invariants live across the column body and double its registers)
hipError_t enqueue_fallback(const csel_plan* p, const StepKey& a, hipStream_t s) {
    csel::SelectArgs sa = select_args(p, a);
    sa.pool = a.pool_idx;
    sa.pool_len = a.pool_len;
    sa.stride = p->stride;
    sa.col_list = p->fb_list;
    sa.col_count = p->fb_count;
    sa.n_waves = p->n_targets;
    if (p->fb_waves > 1) return csel::launch_select_factor_mw(sa, p->precision, kmax_of(p->k), s);
    return csel::launch_select_factor(sa, p->precision, rpl_of(p->stride), kmax_of(p->k), s);
}

hipError_t enqueue_step(const csel_plan* p, const StepKey& a, hipStream_t s) {
    hipError_t e = enqueue_screen(p, a, s);
    if (e == hipSuccess) e = enqueue_kept(p, a, p->schedule < 0 ? 0 : p->schedule, s);
    if (e == hipSuccess) e = enqueue_fallback(p, a, s);
    return e;
}

// one warm-up and one timed run of `run` on the caller's stream (HIP events)
template <typename F>
hipError_t time_once(F run, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms) {
    hipError_t e = run();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = run();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    return e;
}

// time the kept-pool selection under each schedule (natural or Morton order
// when the plan has one; one wave or several per column) and the fallback
// launch under one wave or several per column, on the caller's stream after
// its screen, and keep the fastest of each (ties to the lower number)
hipError_t tune(csel_plan* p, const StepKey& a, hipStream_t s) {
    if (p->n_targets < kTuneMinColumns) {
        p->schedule = 0;
        p->fb_waves = 1;
        return hipSuccess;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best = 0;
    for (int sc = 0; sc < 4 && e == hipSuccess; ++sc) {
        if ((sc & 1) && !p->has_order) continue;
        e = time_once([&] { return enqueue_kept(p, a, sc, s); }, s, e0, e1, &p->tune_ms[sc]);
        if (e == hipSuccess && p->tune_ms[sc] < p->tune_ms[best]) best = sc;
    }
    const int mw = csel::select_mw_waves(p->stride);
    for (int v = 0; v < 2 && e == hipSuccess; ++v) {
        p->fb_waves = v ? mw : 1;
        e = time_once([&] { return enqueue_fallback(p, a, s); }, s, e0, e1, &p->tune_ms[4 + v]);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e == hipSuccess) {
        p->schedule = best;
        p->fb_waves = p->tune_ms[5] < p->tune_ms[4] ? mw : 1;
    }
    return e;
}

hipError_t capture(csel_plan* p, const StepKey& a) {
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    p->has_graph = false;
    hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t enq = enqueue_step(p, a, p->cap_stream);
    e = hipStreamEndCapture(p->cap_stream, &p->graph);
    if (enq != hipSuccess) return enq;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiateWithFlags(&p->exec, p->graph, 0);
    if (e != hipSuccess) return e;
    p->key = a;
    p->has_graph = true;
    return hipSuccess;
}

}  // namespace

CSEL_API int csel_plan_create(csel_plan** plan, int64_t n_targets, int32_t pool_stride, int32_t keep, int32_t k,
                              int32_t precision, uint32_t flags) {
    csel_internal_fail(CSEL_OK, "");
    if (!plan) return pfail(CSEL_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (n_targets < 1 || n_targets > INT32_MAX)
        return pfail(CSEL_EINVAL, "n_targets must be in [1, 2^31) (got %lld)", (long long)n_targets);
    if (pool_stride < 1 || pool_stride > kPlanMaxPool)
        return pfail(CSEL_EUNSUPPORTED, "pool_stride must be in [1, %d] (got %d)", kPlanMaxPool, pool_stride);
    if (keep < 1 || keep > pool_stride) return pfail(CSEL_EINVAL, "keep must be in [1, pool_stride]");
    if (k < 0 || k > kPlanMaxSelect) return pfail(CSEL_EUNSUPPORTED, "k must be in [0, %d] (got %d)", kPlanMaxSelect, k);
    if (precision != CSEL_FP64 && precision != CSEL_MIXED)
        return pfail(CSEL_EINVAL, "precision must be CSEL_FP64 or CSEL_MIXED");
    if (flags & ~(uint32_t)CSEL_PLAN_GRAPH) return pfail(CSEL_EINVAL, "unknown plan flags 0x%x", flags);
    csel_plan* p = new (std::nothrow) csel_plan();
    if (!p) return pfail(CSEL_ENOMEM, "plan allocation failed");
    p->n_targets = n_targets;
    p->stride = pool_stride;
    p->keep = keep;
    p->k = k;
    p->precision = precision;
    p->flags = flags;
    hipError_t e = hipGetDevice(&p->device);
    const int64_t T = n_targets;
    p->order_ws_bytes = csel::spatial_order_workspace(T);
    if (e == hipSuccess && p->order_ws_bytes < 0) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipMalloc(&p->kept, sizeof(int32_t) * T * keep);
    if (e == hipSuccess) e = hipMalloc(&p->kept_len, sizeof(int32_t) * T);
    if (e == hipSuccess) e = hipMalloc(&p->fallback, T);
    if (e == hipSuccess) e = hipMalloc(&p->fb_list, sizeof(int32_t) * T);
    if (e == hipSuccess) e = hipMalloc(&p->fb_count, sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&p->order, sizeof(int32_t) * T);
    if (e == hipSuccess) e = hipMalloc(&p->n_all, sizeof(int32_t));
    if (e == hipSuccess && p->order_ws_bytes > 0) e = hipMalloc(&p->order_ws, p->order_ws_bytes);
    if (e == hipSuccess) {
        const int32_t t32 = (int32_t)T;
        e = hipMemcpy(p->n_all, &t32, sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && (flags & CSEL_PLAN_GRAPH)) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        const int rc = e == hipErrorOutOfMemory ? pfail(CSEL_ENOMEM, "plan buffers: %s", hipGetErrorString(e))
                                                : phip(e, "plan creation");
        free_plan(p);
        return rc;
    }
    *plan = p;
    return CSEL_OK;
}

CSEL_API void csel_plan_destroy(csel_plan* plan) {
    if (plan) (void)hipDeviceSynchronize();
    free_plan(plan);
}

CSEL_API int csel_plan_set_order(csel_plan* plan, const double* pts, int64_t n, int32_t dim, const int32_t* targets,
                                 hipStream_t stream) {
    csel_internal_fail(CSEL_OK, "");
    if (!plan) return pfail(CSEL_EINVAL, "plan is NULL");
    if (n <= 0 || n > INT32_MAX) return pfail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return pfail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (!pts || !targets) return pfail(CSEL_EINVAL, "a required array is NULL");
    hipError_t e = csel::launch_spatial_order(pts, n, dim, plan->n_targets, targets, plan->order_ws, plan->order, stream);
    if (e != hipSuccess) return phip(e, "plan order");
    plan->has_order = true;
    plan->schedule = -1;  // tune again: the schedules' speeds depend on the order
    plan->has_graph = false;
    return CSEL_OK;
}

CSEL_API int csel_plan_info(const csel_plan* plan, int32_t* kept_schedule, int32_t* fallback_waves, float* tune_ms) {
    csel_internal_fail(CSEL_OK, "");
    if (!plan) return pfail(CSEL_EINVAL, "plan is NULL");
    if (kept_schedule) *kept_schedule = plan->schedule;
    if (fallback_waves) *fallback_waves = plan->fb_waves;
    if (tune_ms)
        for (int i = 0; i < 6; ++i) tune_ms[i] = plan->tune_ms[i];
    return CSEL_OK;
}

CSEL_API int csel_plan_screen_outputs(const csel_plan* plan, int32_t* kept_idx, int32_t* kept_len, uint8_t* fallback,
                                      int32_t* fallback_list, int32_t* fallback_count, hipStream_t stream) {
    csel_internal_fail(CSEL_OK, "");
    if (!plan) return pfail(CSEL_EINVAL, "plan is NULL");
    const int64_t T = plan->n_targets;
    struct {
        void* dst;
        const void* src;
        size_t bytes;
    } cp[] = {{kept_idx, plan->kept, sizeof(int32_t) * (size_t)(T * plan->keep)},
              {kept_len, plan->kept_len, sizeof(int32_t) * (size_t)T},
              {fallback, plan->fallback, (size_t)T},
              {fallback_list, plan->fb_list, sizeof(int32_t) * (size_t)T},
              {fallback_count, plan->fb_count, sizeof(int32_t)}};
    for (const auto& c : cp) {
        if (!c.dst) continue;
        const hipError_t e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return phip(e, "plan screen outputs");
    }
    return CSEL_OK;
}

CSEL_API int csel_screened_select(csel_plan* plan, const double* pts, int64_t n, int32_t dim,
                                  const csel_kernel* kernel, const int32_t* targets, const int32_t* pool_idx,
                                  const int32_t* pool_len, const float* params, const uint16_t* params_bf16,
                                  float fallback_threshold, int32_t* sel_idx, double* factor_val,
                                  double* log_condvar, uint8_t* status, hipStream_t stream) {
    csel_internal_fail(CSEL_OK, "");
    if (!plan) return pfail(CSEL_EINVAL, "plan is NULL");
    if (!kernel) return pfail(CSEL_EINVAL, "kernel is NULL");
    if (kernel->two_nu != 1 && kernel->two_nu != 3 && kernel->two_nu != 5)
        return pfail(CSEL_EUNSUPPORTED, "two_nu must be 1, 3 or 5 (got %d)", kernel->two_nu);
    if (!(kernel->length_scale > 0.0) || !std::isfinite(kernel->length_scale))
        return pfail(CSEL_EINVAL, "length_scale must be positive and finite");
    if (!(kernel->variance > 0.0) || !std::isfinite(kernel->variance))
        return pfail(CSEL_EINVAL, "variance must be positive and finite");
    if (!(kernel->nugget >= 0.0) || !std::isfinite(kernel->nugget))
        return pfail(CSEL_EINVAL, "nugget must be >= 0 and finite");
    if (n <= 0 || n > INT32_MAX) return pfail(CSEL_EINVAL, "n must be in [1, 2^31) (got %lld)", (long long)n);
    if (dim < 1 || dim > 3) return pfail(CSEL_EINVAL, "dim must be 1, 2 or 3 (got %d)", dim);
    if (!(fallback_threshold >= 0.0f)) return pfail(CSEL_EINVAL, "fallback_threshold must be >= 0");
    if (!pts || !targets || !pool_idx || !pool_len || !params || !params_bf16 || !factor_val || !status ||
        (plan->k > 0 && !sel_idx))
        return pfail(CSEL_EINVAL, "a required array is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return phip(e, "hipGetDevice");
    if (dev != plan->device) return pfail(CSEL_EINVAL, "the plan was created on device %d, not %d", plan->device, dev);
    StepKey a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.kernel = *kernel;
    a.targets = targets;
    a.pool_idx = pool_idx;
    a.pool_len = pool_len;
    a.params = params;
    a.params_bf16 = params_bf16;
    a.threshold = fallback_threshold;
    a.sel = sel_idx;
    a.fac = factor_val;
    a.logcv = log_condvar;
    a.status = status;
    if (plan->schedule < 0) {
        // first step of the plan (or of a new order): run it eagerly, tuning
        // the kept-pool schedule between the screen and the fallback
        e = enqueue_screen(plan, a, stream);
        if (e == hipSuccess) e = tune(plan, a, stream);
        if (e == hipSuccess) e = enqueue_kept(plan, a, plan->schedule, stream);
        if (e == hipSuccess) e = enqueue_fallback(plan, a, stream);
        if (e != hipSuccess) return phip(e, "screened_select");
        return CSEL_OK;
    }
    if (plan->flags & CSEL_PLAN_GRAPH) {
        if (!plan->has_graph || !same_key(plan->key, a)) {
            e = capture(plan, a);
            if (e != hipSuccess) return phip(e, "screened_select graph capture");
        }
        e = hipGraphLaunch(plan->exec, stream);
        if (e != hipSuccess) return phip(e, "screened_select graph launch");
        return CSEL_OK;
    }
    e = enqueue_step(plan, a, stream);
    if (e != hipSuccess) return phip(e, "screened_select");
    return CSEL_OK;
}
