// apply.hip -- products with the sparse factor L (CSC, FP64), the way the
// factor is used once built (e.g. as a preconditioner L L^T, Sec. 6.3).
//
//   transpose = 1:  y = L^T x  -- gather-dot per column; 16 lanes per column
//                   read the column's entries contiguously (coalesced) and
//                   reduce with DPP inside their 16-lane row.  Deterministic.
//   transpose = 0:  y = L x    -- scatter per column with FP64 atomic adds
//                   into y (cleared first by a fill kernel).  The summation
//                   order depends on scheduling, so results can differ in the
//                   last bits between runs.
//
// HBM-bound: per entry 12 B (int32 row, FP64 value) plus the x gather, which
// mostly hits L2 for factors whose rows are spatial neighbours.
#include <algorithm>
#include <type_traits>

#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

constexpr int kApplyLanesPerCol = 16;

__device__ __forceinline__ double row16_sum(double v) {
    // all-reduce inside each row of 16 lanes (quad butterflies, row rotations)
    auto step = [](double x, auto ctrl_tag) {
        constexpr int CTRL = decltype(ctrl_tag)::value;
        int64_t b = __double_as_longlong(x);
        int32_t lo = __builtin_amdgcn_update_dpp(0, (int32_t)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
        int32_t hi = __builtin_amdgcn_update_dpp(0, (int32_t)(b >> 32), CTRL, 0xF, 0xF, false);
        return x + __longlong_as_double(((int64_t)(uint32_t)lo) | ((int64_t)hi << 32));
    };
    v = step(v, std::integral_constant<int, kDppQuadXor1>{});
    v = step(v, std::integral_constant<int, kDppQuadXor2>{});
    v = step(v, std::integral_constant<int, kDppRowRor4>{});
    v = step(v, std::integral_constant<int, kDppRowRor8>{});
    return v;
}

__global__ __launch_bounds__(256) void apply_lt_kernel(int64_t n, const int64_t* __restrict__ col_ptr,
                                                       const int32_t* __restrict__ row_idx,
                                                       const double* __restrict__ val, const double* __restrict__ x,
                                                       double* __restrict__ y) {
    const int64_t col = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kApplyLanesPerCol;
    const int sub = threadIdx.x & (kApplyLanesPerCol - 1);
    double s = 0.0;
    const bool active = col < n;
    if (active) {
        const int64_t b = col_ptr[col], e = col_ptr[col + 1];
        // three entries per lane in flight: the index and value loads of a
        // chunk of 48 entries first, then their x gathers, so a column of up to
        // 48 entries waits for two dependent memory round trips instead of six;
        // the sum runs over the lane's entries in the same order as one at a time
        for (int64_t p0 = b + sub; p0 < e; p0 += 3 * kApplyLanesPerCol) {
            int32_t r[3];
            double v[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int64_t p = p0 + u * kApplyLanesPerCol;
                r[u] = p < e ? row_idx[p] : -1;
                v[u] = p < e ? val[p] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 3; ++u)
                if (r[u] >= 0 && (int64_t)r[u] < n) s += v[u] * x[r[u]];
        }
    }
    s = row16_sum(s);
    if (active && sub == 0) y[col] = s;
}

__global__ __launch_bounds__(256) void fill_kernel(double* __restrict__ y, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = v;
}

__global__ __launch_bounds__(256) void apply_l_kernel(int64_t n, const int64_t* __restrict__ col_ptr,
                                                      const int32_t* __restrict__ row_idx,
                                                      const double* __restrict__ val, const double* __restrict__ x,
                                                      double* __restrict__ y) {
    const int64_t col = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kApplyLanesPerCol;
    const int sub = threadIdx.x & (kApplyLanesPerCol - 1);
    if (col >= n) return;
    const double xc = x[col];
    const int64_t b = col_ptr[col], e = col_ptr[col + 1];
    for (int64_t p = b + sub; p < e; p += kApplyLanesPerCol) {
        const int32_t r = row_idx[p];
        if (r >= 0 && (int64_t)r < n) atomicAdd(&y[r], val[p] * xc);
    }
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* __restrict__ x, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

hipError_t launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned b = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(b), dim3(256), 0, s, x, n, v);
    return hipGetLastError();
}

hipError_t launch_apply(int64_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* val, int transpose,
                        const double* x, double* y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int64_t threads = n * kApplyLanesPerCol;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    if (transpose) {
        hipLaunchKernelGGL(apply_lt_kernel, dim3(blocks), dim3(256), 0, s, n, col_ptr, row_idx, val, x, y);
    } else {
        const unsigned fb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(fill_kernel, dim3(fb), dim3(256), 0, s, y, n, 0.0);
        hipLaunchKernelGGL(apply_l_kernel, dim3(blocks), dim3(256), 0, s, n, col_ptr, row_idx, val, x, y);
    }
    return hipGetLastError();
}

}  // namespace csel
