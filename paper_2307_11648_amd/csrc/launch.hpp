// launch.hpp -- internal launcher interface between the C ABI (abi.cpp) and
// the kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csel {

struct SelectArgs {
    const double* pts;
    int64_t n;
    int32_t dim;
    int32_t two_nu;
    double c_nu;  // sqrt(2 nu) / length_scale
    double s2;    // kernel variance
    double nugget;
    int64_t n_targets;
    const int32_t* targets;
    const int32_t* pool;
    const int32_t* pool_len;
    int32_t stride;
    int32_t k;
    int32_t* sel;
    double* fac;
    double* logcv;
    float* gap;
    // (top-two variant only, may be null) per step, the fraction of the
    // target's conditional variance the pick removes (its squared conditional
    // correlation, eq. global_obj)
    double* gain;
    uint8_t* status;
    // optional indirection: run only columns col_list[0 .. *col_count)
    const int32_t* col_list;
    const int32_t* col_count;
    int64_t n_waves;  // waves launched: n_targets, or the list capacity
};

struct ScreenArgs {
    const double* pts;
    int64_t n;
    int32_t dim;
    int32_t two_nu;
    double c_nu;
    double s2;
    double nugget;
    double ell;
    int64_t n_targets;
    const int32_t* targets;
    const int32_t* pool;
    const int32_t* pool_len;
    int32_t stride;
    const float* params;
    const uint16_t* params_bf16;
    int32_t keep;
    float fb_thr;
    int32_t mode;  // 0 screen, 1 features only
    float* feats;
    float* logits;
    int32_t* kept;
    int32_t* kept_len;
    uint8_t* fallback;
    int32_t* fb_list;
    int32_t* fb_count;
    const int32_t* order;  // processing order of the columns (nullptr: 0, 1, ...)
    int64_t n_order;       // positions of `order` to process (n_targets without an order)
};

// learned screen of multi-target groups: one workgroup per group
struct GroupScreenArgs {
    const double* pts;
    int64_t n;
    int32_t dim;
    int32_t two_nu;
    double c_nu;
    double ell;
    int64_t n_groups;
    const int32_t* group_ptr;  // [n_groups + 1] offsets into members
    const int32_t* members;
    int64_t n_members;         // length of members
    const int32_t* pool;       // [n_groups][stride], sorted by distance to the nearest member
    const int32_t* pool_len;
    int32_t stride;
    const float* params;
    const uint16_t* params_bf16;
    int32_t keep;
    float fb_thr;
    int32_t mode;  // 0 screen, 1 features only
    float* feats;
    float* logits;
    int32_t* kept;
    int32_t* kept_len;
    uint8_t* fallback;
};

constexpr int kGroupScreenMaxPool = 2048;
constexpr int kGroupScreenMaxMembers = 64;

struct MlpTrainArgs {
    const float* params;
    const uint16_t* params_bf16;
    const float* x;
    const uint8_t* y;
    int64_t n_rows;
    float pos_weight;
    float inv_n;
    float* partials;
};

hipError_t launch_screen(const ScreenArgs& a, int rpl, hipStream_t s);
hipError_t launch_screen_groups(const GroupScreenArgs& a, hipStream_t s);
int mlp_nparams();
int64_t mlp_grad_nparts(int64_t n_rows);
hipError_t launch_mlp_grad(const MlpTrainArgs& a, float* grad, hipStream_t s);
// rows handled by the allocation-free gradient (its partials live in a
// file-scope device array of about 5.4 MB per GPU)
constexpr int64_t kMlpGradNoAllocMaxRows = 65536;
hipError_t launch_mlp_grad_noalloc(MlpTrainArgs a, float* grad, hipStream_t s);
hipError_t launch_mlp_forward(const MlpTrainArgs& a, float* z, hipStream_t s);
hipError_t launch_adam(float* p, uint16_t* pb, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
hipError_t launch_to_bf16(const float* p, uint16_t* pb, int n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s);

// spatial (Morton) processing order of the target columns
int64_t spatial_order_workspace(int64_t n_targets);
hipError_t launch_spatial_order(const double* pts, int64_t n, int dim, int64_t n_targets, const int32_t* targets,
                                void* workspace, int32_t* order, hipStream_t s);

struct AggArgs {
    const double* pts;
    int64_t n;
    int32_t dim;
    int32_t two_nu;
    double c_nu;
    double s2;
    double nugget;
    int64_t n_groups;
    const int32_t* group_ptr;
    const int32_t* members;
    int32_t max_members;
    const int32_t* pool;
    const int32_t* pool_len;
    int32_t stride;
    int32_t k;
    int32_t later_only;  // pool ids must exceed every member id (factor output)
    void* ws;
    int64_t slab_bytes;  // bytes of one workgroup's slab
    int32_t rmax;
    int32_t* sel;
    float* gap;
    double* logdet;
    double* post_var;
    uint8_t* status;
    const int64_t* val_ptr;
    int32_t* fac_rows;
    double* fac_val;
    double* member_logcv;
    // the slab kernel with one row per thread keeps the first cache_b columns
    // of factor B and cache_a of factor A in LDS instead of the slab (set at
    // its launch)
    int32_t cache_a = 0, cache_b = 0;
};

struct AggPlan {
    int rmax, rpt, threads, slots;
    int64_t slab_bytes, ws_bytes;
    size_t smem;
};

AggPlan plan_aggregated(int64_t n_groups, int32_t stride, int32_t max_members, int32_t k, int precision);
// schedules of the multi-target selection (kAggAuto: the library's rule)
enum AggSchedule { kAggAuto = 0, kAggOneGroup = 1, kAggRegister = 2, kAggSplit256 = 3, kAggSplit512 = 4, kAggSplit1024 = 5 };
hipError_t launch_aggregated(const AggArgs& a, const AggPlan& pl, int precision, bool want_factor, int schedule,
                             hipStream_t s);
int agg_factor_max_m();
// reverse-maximin ordering (Sec. 2.2, eq. maximin, p = 1); blocks until done
int64_t reverse_maximin_workspace(int64_t n, int dim);
hipError_t launch_reverse_maximin(const double* pts, int64_t n, int dim, void* workspace, int32_t* order, double* ell,
                                  hipStream_t s, int32_t* rounds_out);

// multi-target selection with each group's rows over several workgroups
// (cooperative launch; factor A in FP64 or, mixed, FP32);
// hipErrorCooperativeLaunchTooLarge when the grid cannot be resident at once
int64_t agg_coop_workspace(int64_t n_groups, int32_t stride, int32_t max_members, int32_t k);
// (block_threads 256, 512 or 1024; 0 picks by the group count)
hipError_t launch_aggregated_coop(const AggArgs& a, int precision, int block_threads, void* workspace, hipStream_t s);
bool agg_coop_applies(int64_t n_groups, int32_t stride, int32_t max_members, int32_t k, int precision);
// the workspace also holds the split-row schedule
bool agg_split_possible(int64_t n_groups, int32_t max_members, int32_t k);
bool agg_reg_applies(int32_t stride, int32_t max_members, int32_t k, int precision, bool want_post_var);

// the aggregated member columns (eq. L_col on s_q = {j in sort(T u S) : j >= q})
hipError_t launch_agg_factor(const AggArgs& a, hipStream_t s);

// later-ordered kNN pools (Sec. 4) on the GPU
int64_t later_knn_workspace(int64_t n, int dim);
int later_knn_max_pool();
hipError_t launch_later_knn(const double* pts, int64_t n, int dim, int C, void* workspace, int32_t* pool,
                            int32_t* pool_len, hipStream_t s);

// partial (non-adjacent) aggregated selection, FP64, then (want_factor) the
// member columns
hipError_t launch_partial(const AggArgs& a, bool want_factor, hipStream_t s);
int partial_max_members();
int partial_max_k();
int partial_max_pool();

// rpl: pool rows per lane (1, 2, 4, 8); kmax: 16 or 32.
hipError_t launch_select_factor(const SelectArgs& a, int precision, int rpl, int kmax, hipStream_t s);
// the multi-wave schedule (no gap output): select_mw_waves(stride) waves per
// column, 2 for pools <= 128, 4 up to 512
int select_mw_waves(int32_t stride);
hipError_t launch_select_factor_mw(const SelectArgs& a, int precision, int kmax, hipStream_t s);
// the kernel matrix-vector product and the preconditioned conjugate gradient (pcg.hip)
int64_t kmatvec_workspace(int64_t n);
hipError_t launch_kmatvec(const double* pts, int64_t n, int dim, int two_nu, double c_nu, double s2, double nugget,
                          const double* v, double* y, void* ws, hipStream_t s);
int64_t pcg_workspace(int64_t n);
hipError_t run_pcg(const double* pts, int64_t n, int dim, int two_nu, double c_nu, double s2, double nugget,
                   const int64_t* l_cp, const int32_t* l_ri, const double* l_v, const int64_t* lt_cp,
                   const int32_t* lt_ri, const double* lt_v, const double* y, double* x, double rel_tol,
                   int max_iter, void* ws, int* iterations, double* rel_res, hipStream_t s);
// global greedy allocation of nonzeros (global.hip)
int64_t global_workspace(int64_t n_targets, int k_max);
hipError_t launch_global(const SelectArgs& sel_args, int precision, int rpl, int64_t budget, void* workspace,
                         int32_t* k_alloc, double* factor_val, hipStream_t s);
int64_t transpose_factor_workspace(int64_t n, int64_t n_slots);
hipError_t launch_transpose_factor(int64_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* val,
                                   int64_t n_slots, int64_t* t_col_ptr, int32_t* t_row_idx, double* t_val,
                                   void* workspace, hipStream_t s);
hipError_t launch_apply(int64_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* val, int transpose,
                        const double* x, double* y, hipStream_t s);
hipError_t launch_sum(const double* x, int64_t n, double* out, hipStream_t s);

}  // namespace csel
