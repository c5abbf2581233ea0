// global.hip -- global greedy allocation of a budget of nonzeros over the
// columns (Sec. 5.4, eq. global_obj).
//
// The paper keeps a priority queue over all columns, keyed by the fraction of
// the target's conditional variance that the column's next greedy pick
// removes (its squared conditional correlation: eq. global_obj, a monotone
// image of the pick's exact decrease of the KL divergence, eq. obj_chol),
// and pops the largest until the budget is spent.  A column's own greedy
// sequence does not depend on the other columns, so the queue's outcome has
// a closed form: with m_{i,t} = min_{s <= t} gain_{i,s} (the prefix minima of
// column i's gains, non-increasing in t), the queue pops the steps in
// decreasing order of m (equal m: smaller column, then earlier step), so
// the budget takes, per column, a prefix of its steps: those with m above a
// threshold tau, plus the steps with m == tau of the first columns in column
// order.  Here:
//   1. the selection runs every column to its cap (select_factor_kernel,
//      selection only) and records each step's gain;
//   2. prefix_min_kernel: m and the number of picks per column;
//   3. allocate_kernel (one workgroup): tau by bisection over the bit
//      patterns of the non-negative doubles m (count of steps with m >= x by
//      binary search in each column's non-increasing m), then each column's
//      count with a workgroup scan of the tied steps in column order;
//   4. factor_prefix_kernel: the eq. L_col column on each allocated prefix
//      (by prefix consistency, the greedy pattern of that many picks).
#include "select_kernel.hpp"

namespace csel {

// m = prefix minima of the gains (clamped at 0; the first NaN or a missing
// pick ends the column), npick = the number of picks
__global__ __launch_bounds__(256) void prefix_min_kernel(const double* __restrict__ gain,
                                                         const int32_t* __restrict__ sel, int64_t T, int K,
                                                         double* __restrict__ m, int32_t* __restrict__ npick) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T) return;
    double run = __builtin_inf();
    int n = 0;
    for (int t = 0; t < K; ++t) {
        const double g = gain[i * K + t];
        if (!(sel[i * K + t] >= 0) || !(g == g)) break;
        run = fmin(run, fmax(g, 0.0));
        m[i * K + t] = run;
        n = t + 1;
    }
    npick[i] = n;
}

// number of steps of column i whose m (as ordered bits) is >= key
__device__ __forceinline__ int count_ge(const double* m, int64_t i, int K, int n, uint64_t key) {
    int lo = 0, hi = n;  // the first step below key lies in [lo, hi]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const uint64_t b = (uint64_t)__double_as_longlong(m[i * K + mid]);
        if (b >= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

constexpr int kAllocThreads = 1024;

template <typename V>
__device__ __forceinline__ V block_sum(V v, V* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    V tot = 0;
    for (int w = 0; w < kAllocThreads / 64; ++w) tot += sh[w];
    return tot;
}

__global__ __launch_bounds__(kAllocThreads) void allocate_kernel(const double* __restrict__ m,
                                                                 const int32_t* __restrict__ npick, int64_t T, int K,
                                                                 int64_t budget, int32_t* __restrict__ k_alloc) {
    __shared__ long long sh_sum[kAllocThreads / 64];
    __shared__ int sh_scan[kAllocThreads];
    const int tid = threadIdx.x;
    // total steps; with no more than the budget, every step is taken
    long long part = 0;
    for (int64_t i = tid; i < T; i += kAllocThreads) part += npick[i];
    const long long total = block_sum<long long>(part, sh_sum);
    if (total <= budget) {
        for (int64_t i = tid; i < T; i += kAllocThreads) k_alloc[i] = npick[i];
        return;
    }
    // tau: the largest bit pattern with at least `budget` steps at or above it
    uint64_t lo = 0ull, hi = 0x7FF0000000000000ull;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        long long c = 0;
        for (int64_t i = tid; i < T; i += kAllocThreads) c += count_ge(m, i, K, npick[i], mid);
        c = block_sum<long long>(c, sh_sum);
        if (c >= budget) lo = mid;
        else hi = mid - 1;
    }
    const uint64_t tau = lo;
    long long gt = 0;
    for (int64_t i = tid; i < T; i += kAllocThreads) gt += count_ge(m, i, K, npick[i], tau + 1);
    gt = block_sum<long long>(gt, sh_sum);
    const long long need = budget - gt;  // steps with m == tau still to take, in column order
    long long carry = 0;
    for (int64_t base = 0; base < T; base += kAllocThreads) {
        const int64_t i = base + tid;
        int above = 0, ties = 0;
        if (i < T) {
            above = count_ge(m, i, K, npick[i], tau + 1);
            ties = count_ge(m, i, K, npick[i], tau) - above;
        }
        // inclusive scan of the tied steps over the chunk's columns
        __syncthreads();
        sh_scan[tid] = ties;
        __syncthreads();
        for (int off = 1; off < kAllocThreads; off <<= 1) {
            const int v = tid >= off ? sh_scan[tid - off] : 0;
            __syncthreads();
            sh_scan[tid] += v;
            __syncthreads();
        }
        const long long before = carry + sh_scan[tid] - ties;
        if (i < T) {
            const long long take = need - before;
            k_alloc[i] = above + (int)(take <= 0 ? 0 : (take >= ties ? ties : take));
        }
        carry += sh_scan[kAllocThreads - 1];
    }
}

// the factor column on each allocated prefix of the greedy selection, one
// wavefront per column
template <int TWO_NU, int KMAX>
__global__ __launch_bounds__(256) void factor_prefix_kernel(SelectArgs p, const int32_t* __restrict__ k_alloc) {
    __shared__ __align__(16) double sh_r[kSelWavesPerBlock][KMAX + 1][KMAX + 2];
    __shared__ double sh_pt[kSelWavesPerBlock][KMAX + 1][4];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * kSelWavesPerBlock + wib;
    if (col >= p.n_targets) return;
    if (p.status[col] >= 2) {
        // bad input (status 3): the selection wrote -1 picks; no column
        for (int r = lane; r <= p.k; r += kWave) p.fac[col * (p.k + 1) + r] = __builtin_nan("");
        if (lane == 0 && p.logcv) p.logcv[col] = __builtin_nan("");
        return;
    }
    const int kk = __builtin_amdgcn_readfirstlane(k_alloc[col]);
    const int32_t tgt = __builtin_amdgcn_readfirstlane(p.targets[col]);
    const int32_t my_sel = lane < kk ? p.sel[col * p.k + lane] : -1;
    // the allocation never exceeds the picks, so no column stopped short of it
    factor_column<TWO_NU, KMAX>(p, col, lane, kk, my_sel, __builtin_nanf(""), tgt, 0, sh_r[wib], sh_pt[wib]);
}

template <int TWO_NU, int KMAX>
static hipError_t launch_factor_prefix(const SelectArgs& a, const int32_t* k_alloc, hipStream_t s) {
    const int64_t blocks = (a.n_targets + kSelWavesPerBlock - 1) / kSelWavesPerBlock;
    hipLaunchKernelGGL((factor_prefix_kernel<TWO_NU, KMAX>), dim3((unsigned)blocks), dim3(256), 0, s, a, k_alloc);
    return hipGetLastError();
}

// workspace: m [T][K] FP64, gains [T][K] FP64 (used when the caller keeps
// none), npick [T] int32
static int64_t ws_block(int64_t T, int K) { return ((T * K * (int64_t)sizeof(double) + 255) / 256) * 256; }

int64_t global_workspace(int64_t n_targets, int k_max) {
    return 2 * ws_block(n_targets, k_max) + n_targets * (int64_t)sizeof(int32_t);
}

hipError_t launch_global(const SelectArgs& sel_args, int precision, int rpl, int64_t budget, void* workspace,
                         int32_t* k_alloc, double* factor_val, hipStream_t s) {
    const int64_t T = sel_args.n_targets;
    const int K = sel_args.k;
    if (T == 0) return hipSuccess;
    const int kmax = K <= 16 ? 16 : 32;
    char* ws = reinterpret_cast<char*>(workspace);
    double* m = reinterpret_cast<double*>(ws);
    double* gain_ws = reinterpret_cast<double*>(ws + ws_block(T, K));
    int32_t* npick = reinterpret_cast<int32_t*>(ws + 2 * ws_block(T, K));
    // 1. every column to its cap: picks and gains, no factor
    SelectArgs a = sel_args;
    a.fac = nullptr;
    a.logcv = nullptr;
    if (!a.gain) a.gain = gain_ws;
    hipError_t e = launch_select_factor(a, precision, rpl, kmax, s);
    if (e != hipSuccess) return e;
    // 2. prefix minima
    hipLaunchKernelGGL(prefix_min_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, a.gain, a.sel, T, K, m,
                       npick);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 3. the allocation
    hipLaunchKernelGGL(allocate_kernel, dim3(1), dim3(kAllocThreads), 0, s, m, npick, T, K, budget, k_alloc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 4. the factor columns on the allocated prefixes
    SelectArgs f = sel_args;
    f.fac = factor_val;
    f.gap = nullptr;
    switch (f.two_nu) {
        case 1: return kmax == 16 ? launch_factor_prefix<1, 16>(f, k_alloc, s) : launch_factor_prefix<1, 32>(f, k_alloc, s);
        case 3: return kmax == 16 ? launch_factor_prefix<3, 16>(f, k_alloc, s) : launch_factor_prefix<3, 32>(f, k_alloc, s);
        case 5: return kmax == 16 ? launch_factor_prefix<5, 16>(f, k_alloc, s) : launch_factor_prefix<5, 32>(f, k_alloc, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace csel
