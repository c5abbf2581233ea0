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
    uint8_t* status;
};

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
    int64_t slab_elems;
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
};

struct AggPlan {
    int rmax, rpt, threads, slots;
    int64_t slab_elems, ws_bytes;
    size_t smem;
};

AggPlan plan_aggregated(int64_t n_groups, int32_t stride, int32_t max_members, int32_t k, int precision);
hipError_t launch_aggregated(const AggArgs& a, const AggPlan& pl, int precision, bool want_factor, hipStream_t s);
int agg_factor_max_m();

// rpl: pool rows per lane (1, 2, 4, 8); kmax: 16 or 32.
hipError_t launch_select_factor(const SelectArgs& a, int precision, int rpl, int kmax, hipStream_t s);
hipError_t launch_apply(int64_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* val, int transpose,
                        const double* x, double* y, hipStream_t s);
hipError_t launch_sum(const double* x, int64_t n, double* out, hipStream_t s);

}  // namespace csel
