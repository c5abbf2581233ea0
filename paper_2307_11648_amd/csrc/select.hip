// select.hip -- dispatch of the single-target kernel families and the
// deterministic FP64 sum.  The kernels themselves live in select_kernel.hpp
// and are instantiated by select_inst.hip (one object per family and pool width).
#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

#define CSEL_DECL1(T, NU, G, R) hipError_t launch_select_##T##_##NU##_##G##_##R(const SelectArgs&, int, hipStream_t);
#define CSEL_DECL(T, NU)        \
    CSEL_DECL1(T, NU, 0, 1)     \
    CSEL_DECL1(T, NU, 0, 2)     \
    CSEL_DECL1(T, NU, 0, 4)     \
    CSEL_DECL1(T, NU, 0, 8)     \
    CSEL_DECL1(T, NU, 1, 1)     \
    CSEL_DECL1(T, NU, 1, 2)     \
    CSEL_DECL1(T, NU, 1, 4)     \
    CSEL_DECL1(T, NU, 1, 8)
CSEL_DECL(float, 1)
CSEL_DECL(float, 3)
CSEL_DECL(float, 5)
CSEL_DECL(double, 1)
CSEL_DECL(double, 3)
CSEL_DECL(double, 5)
#undef CSEL_DECL
#undef CSEL_DECL1

// the family's launcher for pool width rpl (1, 2, 4 or 8 entries per lane)
#define CSEL_RPL(T, NU, G)                                               \
    switch (rpl) {                                                       \
        case 1: return launch_select_##T##_##NU##_##G##_1(a, kmax, s); \
        case 2: return launch_select_##T##_##NU##_##G##_2(a, kmax, s); \
        case 4: return launch_select_##T##_##NU##_##G##_4(a, kmax, s); \
        case 8: return launch_select_##T##_##NU##_##G##_8(a, kmax, s); \
    }                                                                    \
    return hipErrorInvalidValue;

template <int PREC, int NU>
static hipError_t launch_family(const SelectArgs& a, bool gap, int rpl, int kmax, hipStream_t s);

#define CSEL_FAMILY(PREC, T, NU)                                                                              \
    template <>                                                                                              \
    hipError_t launch_family<PREC, NU>(const SelectArgs& a, bool gap, int rpl, int kmax, hipStream_t s) { \
        if (gap) {                                                                                           \
            CSEL_RPL(T, NU, 1)                                                                               \
        }                                                                                                    \
        CSEL_RPL(T, NU, 0)                                                                                   \
    }
CSEL_FAMILY(0, double, 1)
CSEL_FAMILY(0, double, 3)
CSEL_FAMILY(0, double, 5)
CSEL_FAMILY(1, float, 1)
CSEL_FAMILY(1, float, 3)
CSEL_FAMILY(1, float, 5)
#undef CSEL_FAMILY
#undef CSEL_RPL

hipError_t launch_select_factor(const SelectArgs& a, int precision, int rpl, int kmax, hipStream_t s) {
    if (a.n_targets == 0 || a.n_waves == 0) return hipSuccess;
    // the top-two variant also records each step's gain
    const bool gap = a.gap != nullptr || a.gain != nullptr;
    if (precision == 0) {
        switch (a.two_nu) {
            case 1: return launch_family<0, 1>(a, gap, rpl, kmax, s);
            case 3: return launch_family<0, 3>(a, gap, rpl, kmax, s);
            case 5: return launch_family<0, 5>(a, gap, rpl, kmax, s);
        }
    } else {
        switch (a.two_nu) {
            case 1: return launch_family<1, 1>(a, gap, rpl, kmax, s);
            case 3: return launch_family<1, 3>(a, gap, rpl, kmax, s);
            case 5: return launch_family<1, 5>(a, gap, rpl, kmax, s);
        }
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// the multi-wave schedule: (waves per column, rows per lane) for each pool width
// ---------------------------------------------------------------------------
#define CSEL_MW_DECL1(T, NU, W, R) hipError_t launch_select_mw_##T##_##NU##_##W##_##R(const SelectArgs&, int, hipStream_t);
#define CSEL_MW_DECL(T, NU)     \
    CSEL_MW_DECL1(T, NU, 2, 1)  \
    CSEL_MW_DECL1(T, NU, 4, 1)  \
    CSEL_MW_DECL1(T, NU, 4, 2)
CSEL_MW_DECL(float, 1)
CSEL_MW_DECL(float, 3)
CSEL_MW_DECL(float, 5)
CSEL_MW_DECL(double, 1)
CSEL_MW_DECL(double, 3)
CSEL_MW_DECL(double, 5)
#undef CSEL_MW_DECL
#undef CSEL_MW_DECL1

int select_mw_waves(int32_t stride) { return stride <= 128 ? 2 : 4; }

#define CSEL_MW_PICK(T, NU)                                                            \
    if (stride <= 128) return launch_select_mw_##T##_##NU##_2_1(a, kmax, s);           \
    if (stride <= 256) return launch_select_mw_##T##_##NU##_4_1(a, kmax, s);           \
    return launch_select_mw_##T##_##NU##_4_2(a, kmax, s);

hipError_t launch_select_factor_mw(const SelectArgs& a, int precision, int kmax, hipStream_t s) {
    if (a.n_targets == 0 || a.n_waves == 0) return hipSuccess;
    if (a.gap != nullptr || a.stride > 512) return hipErrorInvalidValue;
    const int32_t stride = a.stride;
    if (precision == 0) {
        switch (a.two_nu) {
            case 1: { CSEL_MW_PICK(double, 1) }
            case 3: { CSEL_MW_PICK(double, 3) }
            case 5: { CSEL_MW_PICK(double, 5) }
        }
    } else {
        switch (a.two_nu) {
            case 1: { CSEL_MW_PICK(float, 1) }
            case 3: { CSEL_MW_PICK(float, 3) }
            case 5: { CSEL_MW_PICK(float, 5) }
        }
    }
    return hipErrorInvalidValue;
}
#undef CSEL_MW_PICK

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
