// select.hip -- dispatch of the single-target kernel families and the
// deterministic FP64 sum.  The kernels themselves live in select_kernel.hpp
// and are instantiated by select_inst.hip (one object per family).
#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

#define CSEL_DECL(T, NU)                                                              \
    hipError_t launch_select_##T##_##NU##_0(const SelectArgs&, int, int, hipStream_t); \
    hipError_t launch_select_##T##_##NU##_1(const SelectArgs&, int, int, hipStream_t);
CSEL_DECL(float, 1)
CSEL_DECL(float, 3)
CSEL_DECL(float, 5)
CSEL_DECL(double, 1)
CSEL_DECL(double, 3)
CSEL_DECL(double, 5)
#undef CSEL_DECL

hipError_t launch_select_factor(const SelectArgs& a, int precision, int rpl, int kmax, hipStream_t s) {
    if (a.n_targets == 0 || a.n_waves == 0) return hipSuccess;
    const bool gap = a.gap != nullptr;
#define CSEL_CASE(T, NU) \
    return gap ? launch_select_##T##_##NU##_1(a, rpl, kmax, s) : launch_select_##T##_##NU##_0(a, rpl, kmax, s);
    if (precision == 0) {
        switch (a.two_nu) {
            case 1: CSEL_CASE(double, 1)
            case 3: CSEL_CASE(double, 3)
            case 5: CSEL_CASE(double, 5)
        }
    } else {
        switch (a.two_nu) {
            case 1: CSEL_CASE(float, 1)
            case 3: CSEL_CASE(float, 3)
            case 5: CSEL_CASE(float, 5)
        }
    }
#undef CSEL_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// deterministic FP64 sum: one block of 1024 threads, fixed order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void sum_kernel(const double* __restrict__ x, int64_t n, double* out) {
    __shared__ double part[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += x[i];
    // wave reduction in a fixed order
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane_id() == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += part[w];
        *out = t;
    }
}

hipError_t launch_sum(const double* x, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1024), 0, s, x, n, out);
    return hipGetLastError();
}

}  // namespace csel
