// order.hip -- spatial processing order of the target columns.
//
// Not part of the paper's method: a schedule.  Columns are independent, so
// any order gives the same results; processing columns whose targets are
// close in space at the same time lets their candidate pools (which then
// overlap) share cache lines.  The order is the Morton (Z-order) code of
// the target's coordinates quantised over the targets' bounding box
// (30 bits: 10 per coordinate in 3-D, 15 in 2-D, 30 in 1-D), sorted with a
// stable radix sort so equal codes keep increasing column order.
#include <rocprim/device/device_radix_sort.hpp>

#include "launch.hpp"

namespace csel {

// order-preserving image of a double in uint64 (for atomic min / max)
__device__ __forceinline__ uint64_t ordered_bits(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered(uint64_t o) {
    const uint64_t b = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
    return __longlong_as_double((long long)b);
}

__device__ __forceinline__ double target_coord(const double* pts, int64_t n, int dim, const int32_t* targets,
                                               int64_t t, int c) {
    const int32_t i = targets[t];
    return (c < dim && i >= 0 && (int64_t)i < n) ? pts[(int64_t)i * dim + c] : 0.0;
}

// bb[0..3) = min, bb[3..6) = max (ordered bits), initialised by bbox_init_kernel
__global__ __launch_bounds__(64) void bbox_init_kernel(uint64_t* bb) {
    const int i = threadIdx.x;
    if (i < 3) bb[i] = ~0ull;
    else if (i < 6) bb[i] = 0ull;
}

__global__ __launch_bounds__(256) void bbox_kernel(const double* __restrict__ pts, int64_t n, int dim,
                                                   const int32_t* __restrict__ targets, int64_t T,
                                                   uint64_t* __restrict__ bb) {
    __shared__ uint64_t smin[3][256], smax[3][256];
    uint64_t lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0ull, 0ull, 0ull};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T; t += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint64_t o = ordered_bits(target_coord(pts, n, dim, targets, t, c));
            lo[c] = o < lo[c] ? o : lo[c];
            hi[c] = o > hi[c] ? o : hi[c];
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        smin[c][threadIdx.x] = lo[c];
        smax[c][threadIdx.x] = hi[c];
    }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint64_t a = smin[c][threadIdx.x + s], b = smax[c][threadIdx.x + s];
                if (a < smin[c][threadIdx.x]) smin[c][threadIdx.x] = a;
                if (b > smax[c][threadIdx.x]) smax[c][threadIdx.x] = b;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        atomicMin((unsigned long long*)&bb[threadIdx.x], (unsigned long long)smin[threadIdx.x][0]);
        atomicMax((unsigned long long*)&bb[3 + threadIdx.x], (unsigned long long)smax[threadIdx.x][0]);
    }
}

// spread the low `bits` bits of v so that consecutive bits land `step` apart
__device__ __forceinline__ uint32_t spread_bits(uint32_t v, int bits, int step) {
    uint32_t r = 0u;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1u) << (b * step);
    return r;
}

__global__ __launch_bounds__(256) void morton_kernel(const double* __restrict__ pts, int64_t n, int dim,
                                                     const int32_t* __restrict__ targets, int64_t T,
                                                     const uint64_t* __restrict__ bb, uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ vals) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int bits = dim >= 3 ? 10 : (dim == 2 ? 15 : 30);
    const double cells = (double)((1u << bits) - 1u);
    uint32_t code = 0u;
    for (int c = 0; c < dim && c < 3; ++c) {
        const double lo = from_ordered(bb[c]), hi = from_ordered(bb[3 + c]);
        const double ext = hi - lo;
        double u = ext > 0.0 ? (target_coord(pts, n, dim, targets, t, c) - lo) / ext : 0.0;
        u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
        // separately rounded product and sum (no contraction), so the cell
        // index is reproducible in any IEEE FP64 arithmetic
        const uint32_t q = (uint32_t)__dadd_rn(__dmul_rn(u, cells), 0.5);
        code |= spread_bits(q, bits, dim >= 3 ? 3 : dim) << c;
    }
    keys[t] = code;
    vals[t] = (int32_t)t;
}

// workspace: [bbox 6 x u64][keys in T][keys out T][vals in T][radix-sort temporary]
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t sort_temp_bytes(int64_t T) {
    size_t bytes = 0;
    const hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                                   (const int32_t*)nullptr, (int32_t*)nullptr, (unsigned int)T,
                                                   0u, 30u);
    return e == hipSuccess ? bytes : SIZE_MAX;
}

// bytes of workspace, or -1 when the radix sort cannot size its temporary
int64_t spatial_order_workspace(int64_t T) {
    if (T <= 0) return 0;
    const size_t temp = sort_temp_bytes(T);
    if (temp == SIZE_MAX) return -1;
    return (int64_t)(align256(6 * sizeof(uint64_t)) + 3 * align256((size_t)T * 4) + align256(temp));
}

hipError_t launch_spatial_order(const double* pts, int64_t n, int dim, int64_t T, const int32_t* targets,
                                void* workspace, int32_t* order, hipStream_t s) {
    if (T <= 0) return hipSuccess;
    char* w = static_cast<char*>(workspace);
    uint64_t* bb = reinterpret_cast<uint64_t*>(w);
    w += align256(6 * sizeof(uint64_t));
    uint32_t* keys_in = reinterpret_cast<uint32_t*>(w);
    w += align256((size_t)T * 4);
    uint32_t* keys_out = reinterpret_cast<uint32_t*>(w);
    w += align256((size_t)T * 4);
    int32_t* vals_in = reinterpret_cast<int32_t*>(w);
    w += align256((size_t)T * 4);
    size_t temp = sort_temp_bytes(T);
    hipLaunchKernelGGL(bbox_init_kernel, dim3(1), dim3(64), 0, s, bb);
    const unsigned nb = (unsigned)std::min<int64_t>((T + 255) / 256, 1024);
    hipLaunchKernelGGL(bbox_kernel, dim3(nb), dim3(256), 0, s, pts, n, dim, targets, T, bb);
    hipLaunchKernelGGL(morton_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, pts, n, dim, targets, T,
                       (const uint64_t*)bb, keys_in, vals_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return rocprim::radix_sort_pairs(w, temp, keys_in, keys_out, vals_in, order, (unsigned int)T, 0u, 30u, s);
}

}  // namespace csel
