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

// rpl: pool rows per lane (1, 2, 4, 8); kmax: 16 or 32.
hipError_t launch_select_factor(const SelectArgs& a, int precision, int rpl, int kmax, hipStream_t s);
hipError_t launch_sum(const double* x, int64_t n, double* out, hipStream_t s);

}  // namespace csel
