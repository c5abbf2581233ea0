// pcg.hip -- the kernel matrix-vector product and the conjugate gradient
// preconditioned by the sparse inverse-Cholesky factor (Sec. 6.3: L L^T
// approximates Theta^{-1}, so M^{-1} = L L^T).
//
// y = Theta x is matrix-free, FP64: Theta(x_i, x_j) is evaluated as it is
// used.  Workgroups tile the rows (256 per workgroup, one per thread) and
// split the columns into chunks; each stages its chunk's points and x values
// in LDS 256 at a time and every thread sums its row over them; the chunks'
// partial sums are then added in a fixed order, so the product is
// deterministic.  Dot products reduce per workgroup and then in one
// workgroup, also in a fixed order.  The iteration itself is the textbook
// preconditioned conjugate gradient; its scalars stay on the device and the
// host reads the residual norm once per iteration to stop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

constexpr int kMvThreads = 256;
constexpr int kMvTile = 256;

// partial[c][i] = sum over the columns j of chunk c of Theta(x_i, x_j) v_j
template <int TWO_NU>
__global__ __launch_bounds__(kMvThreads) void kmatvec_partial_kernel(const double* __restrict__ pts, int64_t n,
                                                                     int dim, double c_nu, double s2, double nugget,
                                                                     const double* __restrict__ v, int64_t chunk,
                                                                     double* __restrict__ partial) {
    __shared__ double sx[kMvTile][4];  // x, y, z, v_j
    const int64_t i = (int64_t)blockIdx.x * kMvThreads + threadIdx.x;
    const int64_t c = blockIdx.y;
    const int64_t j0 = c * chunk, j1 = min(j0 + chunk, n);
    double xi[3] = {0.0, 0.0, 0.0};
    if (i < n)
        for (int d = 0; d < dim; ++d) xi[d] = pts[i * dim + d];
    double acc = 0.0;
    for (int64_t jt = j0; jt < j1; jt += kMvTile) {
        const int64_t j = jt + threadIdx.x;
        __syncthreads();
        if (j < j1) {
            sx[threadIdx.x][0] = pts[j * dim];
            sx[threadIdx.x][1] = dim > 1 ? pts[j * dim + 1] : 0.0;
            sx[threadIdx.x][2] = dim > 2 ? pts[j * dim + 2] : 0.0;
            sx[threadIdx.x][3] = v[j];
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)kMvTile, j1 - jt);
        for (int q = 0; q < cnt; ++q) {
            const double e0 = xi[0] - sx[q][0], e1 = xi[1] - sx[q][1], e2 = xi[2] - sx[q][2];
            const double r = dist64(e0 * e0 + e1 * e1 + e2 * e2);
            acc = fma(matern_f64<TWO_NU>(r, c_nu, s2), sx[q][3], acc);
        }
    }
    if (i < n) {
        // the nugget sits on the diagonal, by index
        if (i >= j0 && i < j1) acc = fma(nugget, v[i], acc);
        partial[c * n + i] = acc;
    }
}

__global__ __launch_bounds__(256) void sum_chunks_kernel(const double* __restrict__ partial, int chunks, int64_t n,
                                                         double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * n + i];
    y[i] = s;
}

// chunks of columns: enough workgroups to fill the chip several times over
static int mv_chunks(int64_t n) {
    const int64_t row_blocks = (n + kMvThreads - 1) / kMvThreads;
    const int64_t want = (4096 + row_blocks - 1) / row_blocks;
    const int64_t max_chunks = std::max<int64_t>(1, (n + kMvTile - 1) / kMvTile);
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, std::min<int64_t>(max_chunks, 64)));
}

int64_t kmatvec_workspace(int64_t n) { return (int64_t)mv_chunks(n) * n * (int64_t)sizeof(double); }

hipError_t launch_kmatvec(const double* pts, int64_t n, int dim, int two_nu, double c_nu, double s2, double nugget,
                          const double* v, double* y, void* ws, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int chunks = mv_chunks(n);
    const int64_t chunk = ((n + chunks - 1) / chunks + kMvTile - 1) / kMvTile * kMvTile;
    const dim3 grid((unsigned)((n + kMvThreads - 1) / kMvThreads), (unsigned)chunks);
    double* partial = reinterpret_cast<double*>(ws);
    switch (two_nu) {
        case 1:
            hipLaunchKernelGGL(kmatvec_partial_kernel<1>, grid, dim3(kMvThreads), 0, s, pts, n, dim, c_nu, s2, nugget,
                               v, chunk, partial);
            break;
        case 3:
            hipLaunchKernelGGL(kmatvec_partial_kernel<3>, grid, dim3(kMvThreads), 0, s, pts, n, dim, c_nu, s2, nugget,
                               v, chunk, partial);
            break;
        case 5:
            hipLaunchKernelGGL(kmatvec_partial_kernel<5>, grid, dim3(kMvThreads), 0, s, pts, n, dim, c_nu, s2, nugget,
                               v, chunk, partial);
            break;
        default:
            return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, partial, chunks, n, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the iteration's vector kernels; scalars live in a small device array
// ---------------------------------------------------------------------------
constexpr int kDotBlocks = 256;
enum { S_RZ = 0, S_RZ_NEW, S_PQ, S_RR, S_YY, S_ALPHA, S_BETA, S_COUNT };

// per-workgroup partial sums of a . b (fixed grid, so a fixed order)
__global__ __launch_bounds__(256) void dot_partial_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                                          int64_t n, double* __restrict__ part) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) s = fma(a[i], b[i], s);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// scal[slot] = the sum of the partials; then the step's scalar update:
// op 1: alpha = rz / pq;  op 2: beta = rz_new / rz, then rz = rz_new
__global__ __launch_bounds__(kDotBlocks) void dot_final_kernel(const double* __restrict__ part, double* scal,
                                                               int slot, int op) {
    __shared__ double sh[kDotBlocks / 64];
    double s = part[threadIdx.x];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kDotBlocks / 64; ++w) t += sh[w];
        scal[slot] = t;
        if (op == 1) scal[S_ALPHA] = scal[S_RZ] / t;
        if (op == 2) {
            scal[S_BETA] = t / scal[S_RZ];
            scal[S_RZ] = t;
        }
    }
}

// x += alpha p, r -= alpha q
__global__ __launch_bounds__(256) void cg_update_xr_kernel(double* __restrict__ x, double* __restrict__ r,
                                                           const double* __restrict__ p, const double* __restrict__ q,
                                                           const double* __restrict__ scal, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double a = scal[S_ALPHA];
    x[i] = fma(a, p[i], x[i]);
    r[i] = fma(-a, q[i], r[i]);
}

// p = z + beta p (beta = 0: p = z)
__global__ __launch_bounds__(256) void cg_update_p_kernel(double* __restrict__ p, const double* __restrict__ z,
                                                          const double* __restrict__ scal, int use_beta, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    p[i] = use_beta ? fma(scal[S_BETA], p[i], z[i]) : z[i];
}

// r = y - r (r holds Theta x on entry)
__global__ __launch_bounds__(256) void residual_kernel(const double* __restrict__ y, double* __restrict__ r, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) r[i] = y[i] - r[i];
}

__global__ void copy_kernel(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// workspace: r, z, p, q, w (n each), matvec partials, dot partials, scalars
int64_t pcg_workspace(int64_t n) {
    return 5 * n * (int64_t)sizeof(double) + kmatvec_workspace(n) + (kDotBlocks + 16) * (int64_t)sizeof(double);
}

hipError_t run_pcg(const double* pts, int64_t n, int dim, int two_nu, double c_nu, double s2, double nugget,
                   const int64_t* l_cp, const int32_t* l_ri, const double* l_v, const int64_t* lt_cp,
                   const int32_t* lt_ri, const double* lt_v, const double* y, double* x, double rel_tol,
                   int max_iter, void* ws, int* iterations, double* rel_res, hipStream_t s) {
    double* r = reinterpret_cast<double*>(ws);
    double* z = r + n;
    double* p = z + n;
    double* q = p + n;
    double* w = q + n;
    double* mv = w + n;
    double* part = mv + kmatvec_workspace(n) / (int64_t)sizeof(double);
    double* scal = part + kDotBlocks;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    const bool precond = l_cp != nullptr;
    hipError_t e;
#define CSEL_TRY(x)              \
    do {                         \
        e = (x);                 \
        if (e != hipSuccess) return e; \
    } while (0)
    auto dot = [&](const double* a, const double* bb, int slot, int op) -> hipError_t {
        hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotBlocks), dim3(256), 0, s, a, bb, n, part);
        hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kDotBlocks), 0, s, part, scal, slot, op);
        return hipGetLastError();
    };
    // z = M^{-1} r = L (L^T r): w = L^T r as a gather on L, then L w as the
    // same gather on L^T
    auto precondition = [&]() -> hipError_t {
        if (!precond) {
            hipLaunchKernelGGL(copy_kernel, g, b, 0, s, r, z, n);
            return hipGetLastError();
        }
        hipError_t e2 = launch_apply(n, l_cp, l_ri, l_v, 1, r, w, s);
        if (e2 != hipSuccess) return e2;
        return launch_apply(n, lt_cp, lt_ri, lt_v, 1, w, z, s);
    };
    auto host_scalar = [&](int slot, double* out) -> hipError_t {
        hipError_t e2 = hipMemcpyAsync(out, scal + slot, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e2 != hipSuccess) return e2;
        return hipStreamSynchronize(s);
    };
    // r = y - Theta x, z = M^{-1} r, p = z, rz = r . z
    CSEL_TRY(launch_kmatvec(pts, n, dim, two_nu, c_nu, s2, nugget, x, r, mv, s));
    hipLaunchKernelGGL(residual_kernel, g, b, 0, s, y, r, n);
    CSEL_TRY(hipGetLastError());
    CSEL_TRY(dot(y, y, S_YY, 0));
    CSEL_TRY(precondition());
    hipLaunchKernelGGL(cg_update_p_kernel, g, b, 0, s, p, z, scal, 0, n);
    CSEL_TRY(hipGetLastError());
    CSEL_TRY(dot(r, z, S_RZ, 0));
    CSEL_TRY(dot(r, r, S_RR, 0));
    double yy = 0.0, rr = 0.0;
    CSEL_TRY(host_scalar(S_YY, &yy));
    CSEL_TRY(host_scalar(S_RR, &rr));
    const double ynorm = std::sqrt(yy);
    int it = 0;
    double res = ynorm > 0.0 ? std::sqrt(rr) / ynorm : 0.0;
    while (it < max_iter && res > rel_tol) {
        CSEL_TRY(launch_kmatvec(pts, n, dim, two_nu, c_nu, s2, nugget, p, q, mv, s));
        CSEL_TRY(dot(p, q, S_PQ, 1));  // alpha = rz / (p . q)
        hipLaunchKernelGGL(cg_update_xr_kernel, g, b, 0, s, x, r, p, q, scal, n);
        CSEL_TRY(hipGetLastError());
        CSEL_TRY(dot(r, r, S_RR, 0));
        CSEL_TRY(precondition());
        CSEL_TRY(dot(r, z, S_RZ_NEW, 2));  // beta = rz_new / rz
        hipLaunchKernelGGL(cg_update_p_kernel, g, b, 0, s, p, z, scal, 1, n);
        CSEL_TRY(hipGetLastError());
        CSEL_TRY(host_scalar(S_RR, &rr));
        ++it;
        res = std::sqrt(rr) / ynorm;
    }
#undef CSEL_TRY
    *iterations = it;
    *rel_res = res;
    return hipSuccess;
}

}  // namespace csel
