// agg_coop.hip -- multi-target selection (Sec. 5.2, eq. greedy_mult; App.
// C.2) with each group's rows split over several workgroups, for runs with
// few groups (GP prediction batches: 64 groups of 64 targets with pools of
// 2,048) that one workgroup per group leaves on a quarter of the CUs.
//
// The computation is the slab kernel's (aggregate.hip), rounded the same way
// (the same expressions, fused multiply-adds and summation orders), so the two
// schedules give bit-identical results: factor B
// conditions on the targets and then on every pick, factor A on the picks
// only, both column-major in a per-group slab in global memory; every pick
// maximizes 1 - var2 / var1.  W workgroups share a group, each owning a
// contiguous block of its rows.  The grid is launched cooperatively, so every
// workgroup is resident, and the W workgroups of a group meet at a barrier of
// their own (an arrival counter per group in global memory) once per target
// column and once per pick:
//   * target column c: the pivot row's owner publishes its var2 and
//     coordinates; after the barrier every workgroup of the group reads them
//     (and the pivot's B row from the slab) and writes column c for its rows;
//   * pick t: each workgroup publishes its best two keys with its best
//     candidate's var1, var2, coordinates and id; after the barrier every
//     workgroup merges the W records of its group, reads the winner's A and
//     B rows from the slab and writes columns t (A) and m + t (B) for its
//     rows.
// Published records are double-buffered by the parity of the step, so a
// workgroup that runs ahead writes the next step's record while a slower one
// still reads the current step's.  Every workgroup of a group takes the same
// steps (the group's size, pool length, validity and early stop are known to
// all of them), so the groups need not wait for each other.
#include <algorithm>

#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

constexpr int kAggMaxSelectCoop = 256;
constexpr int kAggMaxMembersCoop = 128;

struct CoopPub {
    uint64_t k1, k2;          // the workgroup's best two keys
    double v1, v2, x0, x1, x2;  // its best candidate's variances and coordinates
    int32_t id, pad;
};

struct CoopArgs {
    AggArgs a;
    int32_t W;          // workgroups per group
    int32_t rows_wg;    // rows per workgroup (= the block size)
    CoopPub* pub;       // [2][n_groups][W]
    double* piv;        // [2][n_groups][5]: pivot var2, coordinates, id
    uint32_t* sync;     // [n_groups][kSyncStride]: [0] arrivals, [1] invalid row seen, [2] wait abandoned
    int32_t cache_b;    // factor B's first columns of the workgroup's own rows also kept in LDS
};

// one counter per 128-byte line
constexpr int kSyncStride = 32;
// polls (each a device-scope load, about a microsecond, after a short sleep)
// before a barrier wait is abandoned: far beyond any real wait (one step of
// one workgroup), it bounds the kernel should a workgroup never arrive
constexpr uint32_t kSpinLimit = 1u << 20;

__global__ void agg_coop_clear_kernel(uint32_t* sync, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) sync[i] = 0u;
}

// the W workgroups of a group meet: the n-th barrier of a launch completes
// when the group's arrival counter reaches n * W.  Every wave first waits for
// its own global stores to complete; one thread then releases at device scope
// (the L2 write-back that makes the workgroup's writes visible on the other
// XCDs), arrives, waits, and acquires at device scope (which invalidates the
// CU's caches for every wave of the workgroup).  Fencing from one thread
// rather than all keeps the device-wide cache maintenance to one release and
// one acquire per workgroup and barrier.  A wait that runs out of polls marks
// the group (its status then reports it) and the workgroup stops waiting at
// the group's later barriers, so the launch always ends.
__device__ __forceinline__ void group_barrier(uint32_t* gs, uint32_t target, bool& lost) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's stores are done
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(gs, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t polls = 0;
        while (!lost && __hip_atomic_load(gs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++polls == kSpinLimit) {
                __hip_atomic_store(gs + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                lost = true;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

__device__ __forceinline__ float matern_f32_rt(int two_nu, float r, float c, float s2) {
    if (two_nu == 1) return matern_f32<1>(r, c, s2);
    if (two_nu == 3) return matern_f32<3>(r, c, s2);
    return matern_f32<5>(r, c, s2);
}

// TA: the picks-only factor A and its covariance evaluations (double, or
// float in mixed precision); factor B and both variances stay FP64
template <typename TA, int NT>
__global__ __launch_bounds__(NT) void agg_select_coop_kernel(CoopArgs ca) {
    const AggArgs& p = ca.a;
    __shared__ TA rowA[kAggMaxSelectCoop];
    __shared__ double rowB[kAggMaxSelectCoop + kAggMaxMembersCoop];
    __shared__ Top2 wtop[NT / kWave];
    // the first nb columns of factor B for this workgroup's rows (entry tid of
    // column c at cB[c * NT + tid]): the rows' own reads come from here, the
    // slab keeps every column for the winner's and pivot's rows
    extern __shared__ __align__(16) double cB[];
    const int nb = ca.cache_b;

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    const int W = ca.W;
    const int64_t g = blockIdx.x / W;
    const int wg = blockIdx.x % W;
    const int rmax = p.rmax;
    const double prior = p.s2 + p.nugget;
    const double thr = 1e-12 * prior;
    const int dim = p.dim;
    double* slabB = reinterpret_cast<double*>(reinterpret_cast<char*>(p.ws) + g * p.slab_bytes);
    TA* slabA = reinterpret_cast<TA*>(slabB + (int64_t)(p.max_members + p.k) * rmax);

    const int32_t b0 = p.group_ptr[g];
    const int32_t m = p.group_ptr[g + 1] - b0;
    const int32_t C = p.pool_len[g];
    bool bad = m < 1 || m > p.max_members || C < 0 || C > p.stride;
    const int R = bad ? 0 : C + m;
    // my row
    const int r = wg * ca.rows_wg + tid;
    int32_t rid = -1;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0, v1 = prior, v2 = prior;
    bool live = false, my_bad = false;
    if (r < R) {
        const int32_t id = r < C ? p.pool[g * p.stride + r] : p.members[b0 + (r - C)];
        if (id < 0 || (int64_t)id >= p.n) {
            my_bad = true;
        } else {
            rid = id;
            x0 = p.pts[(int64_t)id * dim];
            if (dim > 1) x1 = p.pts[(int64_t)id * dim + 1];
            if (dim > 2) x2 = p.pts[(int64_t)id * dim + 2];
            live = r < C;
        }
    }
    uint32_t* gs = ca.sync + g * kSyncStride;
    uint32_t nbar = 0;
    bool lost = false;
    if (__syncthreads_or(my_bad) && tid == 0)
        __hip_atomic_store(gs + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    group_barrier(gs, ++nbar * W, lost);
    bad = bad || __hip_atomic_load(gs + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    const double cnu = p.c_nu, s2 = p.s2;

    // ---- factor B over the targets ----------------------------------------
    double ldT = 0.0;
    for (int c = 0; c < (bad ? 0 : m); ++c) {
        const int prow = C + c;
        double* pv = ca.piv + ((int64_t)(c & 1) * p.n_groups + g) * 5;
        if (r == prow) {
            pv[0] = v2;
            pv[1] = x0;
            pv[2] = x1;
            pv[3] = x2;
            pv[4] = (double)rid;
        }
        group_barrier(gs, ++nbar * W, lost);
        for (int q = tid; q < c; q += NT) rowB[q] = slabB[(int64_t)q * rmax + prow];
        __syncthreads();
        const double piv = pv[0], y0 = pv[1], y1 = pv[2], y2 = pv[3];
        const int32_t idw = (int32_t)pv[4];
        ldT += log(piv);
        const double inv_sd = 1.0 / sqrt(piv);
        if (r < R) {
            const double e0 = x0 - y0, e1 = x1 - y1, e2 = x2 - y2;
            double acc = matern_f64_rt(p.two_nu, sqrt(sqnorm3(e0, e1, e2)), cnu, s2);
            if (rid == idw) acc += p.nugget;
            acc = dot_down_cached<double>(acc, cB + threadIdx.x, NT, nb, slabB + r, rmax, rowB, c);
            const double u = acc * inv_sd;
            slabB[(int64_t)c * rmax + r] = u;
            if (c < nb) cB[c * NT + threadIdx.x] = u;
            v2 = fma(-u, u, v2);
        }
        __syncthreads();  // rowB is rewritten at the next column
    }

    // ---- the picks ------------------------------------------------------------
    const int kk = bad ? 0 : min(p.k, C);
    int32_t* sel_out = p.sel + g * p.k;
    double ld = 0.0;
    int nsel = 0, st = 0;
    for (int t = 0; t < kk; ++t) {
        CoopPub* pb = ca.pub + ((int64_t)(t & 1) * p.n_groups + g) * W;
        {
            uint64_t key = 0ull;
            if (live && v1 > thr && v2 > thr) key = make_key(fmax(0.0, 1.0 - v2 / v1), r);
            Top2 loc = {key, 0ull};
            const Top2 wv = wave_top2(loc);
            if (lane == 0) wtop[wave] = wv;
            __syncthreads();
            Top2 b = wtop[0];
            for (int q = 1; q < NT / kWave; ++q) b = merge(b, wtop[q]);
            // the workgroup's best candidate publishes its record
            if (b.k1 != 0ull && key == b.k1) {
                CoopPub rec;
                rec.k1 = b.k1;
                rec.k2 = b.k2;
                rec.v1 = v1;
                rec.v2 = v2;
                rec.x0 = x0;
                rec.x1 = x1;
                rec.x2 = x2;
                rec.id = rid;
                rec.pad = 0;
                pb[wg] = rec;
            } else if (b.k1 == 0ull && tid == 0) {
                CoopPub rec{};
                pb[wg] = rec;
            }
        }
        group_barrier(gs, ++nbar * W, lost);
        // the group's best over its W records
        Top2 best = {0ull, 0ull};
        int wbest = -1;
        for (int v = 0; v < W; ++v) {
            const uint64_t k1 = pb[v].k1, k2 = pb[v].k2;
            if (k1 > best.k1) wbest = v;
            best = merge(best, Top2{k1, k2});
        }
        if (best.k1 == 0ull) {
            st = 1;
            break;
        }
        const CoopPub wr = pb[wbest];
        const int slot = key_slot(best.k1);  // the winner's row within the group
        if (r == slot) live = false;
        for (int q = tid; q < t; q += NT) rowA[q] = slabA[(int64_t)q * rmax + slot];
        for (int q = tid; q < m + t; q += NT) rowB[q] = slabB[(int64_t)q * rmax + slot];
        __syncthreads();
        const double w1 = wr.v1, w2 = wr.v2;
        ld += log(w2) - log(w1);
        if (wg == 0 && tid == 0) {
            sel_out[t] = wr.id;
            if (p.gap) {
                const double sa = key_score(best.k1), sb = key_score(best.k2);
                p.gap[g * p.k + t] = (best.k2 == 0ull) ? 1.0f : (sa == 0.0 ? 0.0f : (float)((sa - sb) / sa));
            }
        }
        const double inv1 = 1.0 / sqrt(w1), inv2 = 1.0 / sqrt(w2);
        if (r < R) {
            const double e0 = x0 - wr.x0, e1 = x1 - wr.x1, e2 = x2 - wr.x2;
            double th = matern_f64_rt(p.two_nu, sqrt(sqnorm3(e0, e1, e2)), cnu, s2);
            if (rid == wr.id) th += p.nugget;
            TA a;
            if constexpr (sizeof(TA) == 8) {
                a = th;
            } else {
                const float f0 = (float)e0, f1 = (float)e1, f2 = (float)e2;
                a = matern_f32_rt(p.two_nu, sqrt(sqnorm3(f0, f1, f2)), (float)cnu, (float)s2);
                if (rid == wr.id) a += (float)p.nugget;
            }
            a = dot_down<TA>(a, slabA + r, rmax, rowA, t);
            const double bb = dot_down_cached<double>(th, cB + threadIdx.x, NT, nb, slabB + r, rmax, rowB, m + t);
            const TA u1 = a * (TA)inv1;
            const double u2 = bb * inv2;
            slabA[(int64_t)t * rmax + r] = u1;
            slabB[(int64_t)(m + t) * rmax + r] = u2;
            if (m + t < nb) cB[(m + t) * NT + threadIdx.x] = u2;
            const double d1 = (double)u1;
            v1 = fma(-d1, d1, v1);
            v2 = fma(-u2, u2, v2);
        }
        __syncthreads();  // rowA / rowB and wtop are rewritten at the next pick
        nsel = t + 1;
    }

    // ---- outputs -----------------------------------------------------------------
    if (bad) {
        if (wg == 0) {
            for (int t = tid; t < p.k; t += NT) {
                sel_out[t] = -1;
                if (p.gap) p.gap[g * p.k + t] = __builtin_nanf("");
            }
            if (tid == 0) {
                if (p.logdet) p.logdet[g] = __builtin_nan("");
                p.status[g] = 3;
            }
        }
        return;
    }
    if (wg == 0) {
        for (int t = nsel + tid; t < p.k; t += NT) {
            sel_out[t] = -1;
            if (p.gap) p.gap[g * p.k + t] = __builtin_nanf("");
        }
        if (tid == 0) {
            // a barrier wait abandoned (never seen in a complete launch)
            // leaves the group's results unusable: status 6
            const bool lost = __hip_atomic_load(gs + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
            if (p.logdet) p.logdet[g] = lost ? __builtin_nan("") : ldT + ld;
            p.status[g] = lost ? (uint8_t)6 : (uint8_t)st;
        }
    }
    if (p.post_var && r >= C && r < R) p.post_var[b0 + (r - C)] = v1;
}

// workgroups of each group for a block size
static int coop_split(int64_t rmax, int nt) { return (int)((rmax + nt - 1) / nt); }

// bytes of the cooperative run's workspace (slabs + exchange records, sized
// for the smallest block size)
int64_t agg_coop_workspace(int64_t n_groups, int32_t stride, int32_t max_members, int32_t k) {
    const int64_t rmax = (int64_t)stride + max_members;
    int64_t slab = ((int64_t)max_members + k + k) * rmax * 8;
    slab = (slab + 255) / 256 * 256;
    const int64_t pub = 2 * n_groups * coop_split(rmax, 256) * (int64_t)sizeof(CoopPub);
    const int64_t piv = 2 * n_groups * 5 * (int64_t)sizeof(double);
    return n_groups * slab + ((pub + 255) / 256) * 256 + ((piv + 255) / 256) * 256 +
           n_groups * kSyncStride * 4;
}

// LDS of one CU, and the most one workgroup's column cache takes
constexpr size_t kCoopCuLds = 160 * 1024;
constexpr size_t kCoopCacheLds = 152 * 1024;

template <typename TA, int NT>
static hipError_t launch_coop(CoopArgs& ca, int cus, hipStream_t s) {
    ca.W = coop_split(ca.a.rmax, NT);
    ca.rows_wg = NT;
    const int64_t nblocks = ca.a.n_groups * ca.W;
    const void* kern = (const void*)agg_select_coop_kernel<TA, NT>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0);
    if (e != hipSuccess) return e;
    if (nblocks > (int64_t)per_cu * cus || nblocks > INT32_MAX) return hipErrorCooperativeLaunchTooLarge;
    // B's first columns in the LDS the resident workgroups leave free (as
    // many workgroups per CU as without them)
    hipFuncAttributes fa;
    e = hipFuncGetAttributes(&fa, kern);
    if (e != hipSuccess) return e;
    const size_t lds = std::min<size_t>(kCoopCacheLds, kCoopCuLds / (size_t)std::max(1, per_cu));
    const size_t avail = lds > fa.sharedSizeBytes + 1024 ? lds - fa.sharedSizeBytes - 1024 : 0;
    ca.cache_b = (int)std::min<size_t>(avail / ((size_t)NT * sizeof(double)), (size_t)ca.a.max_members + ca.a.k);
    size_t smem = (size_t)ca.cache_b * NT * sizeof(double);
    if (smem > 0) {
        e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        int per_cu2 = 0;
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, kern, NT, smem);
        if (e != hipSuccess || per_cu2 < per_cu) {  // keep the residency: no caches
            (void)hipGetLastError();
            ca.cache_b = 0;
            smem = 0;
        }
    }
    // counters start at zero (a fill kernel: no memset node if the caller captures the stream)
    const int64_t ns = ca.a.n_groups * kSyncStride;
    hipLaunchKernelGGL(agg_coop_clear_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, ca.sync, ns);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* args[] = {&ca};
    return hipLaunchCooperativeKernel(kern, dim3((unsigned)nblocks), dim3(NT), args, (unsigned)smem, s);
}

// the cooperative launch, when every workgroup fits on the device at once;
// hipErrorCooperativeLaunchTooLarge otherwise (the caller then uses the
// one-workgroup-per-group kernel).  Each barrier costs every workgroup one
// device-scope release and acquire, so the block is as large (the split as
// coarse) as still leaves at least half the CUs a workgroup: 64 groups of
// 2,112 rows run 3 workgroups of 1,024 threads each (6.5 ms for k = 128 on
// MI355X, against 7.9 ms with 9 of 256), 8 such groups 9 of 256 (2.3 ms,
// against 4.3 ms with 1,024).
hipError_t launch_aggregated_coop(const AggArgs& a0, int precision, int block_threads, void* workspace, hipStream_t s) {
    if (a0.n_groups == 0) return hipSuccess;
    // (the later-only check of factor-producing runs stays with the slab kernel)
    if (a0.k > kAggMaxSelectCoop || a0.max_members > kAggMaxMembersCoop || a0.later_only)
        return hipErrorNotSupported;
    CoopArgs ca;
    ca.a = a0;
    const int64_t rmax = (int64_t)a0.stride + a0.max_members;
    ca.a.rmax = (int32_t)rmax;
    int64_t slab = ((int64_t)a0.max_members + a0.k + a0.k) * rmax * 8;
    slab = (slab + 255) / 256 * 256;
    ca.a.slab_bytes = slab;
    char* w = static_cast<char*>(workspace);
    ca.a.ws = w;
    w += a0.n_groups * slab;
    ca.pub = reinterpret_cast<CoopPub*>(w);
    const int64_t pub = 2 * a0.n_groups * coop_split(rmax, 256) * (int64_t)sizeof(CoopPub);
    w += ((pub + 255) / 256) * 256;
    ca.piv = reinterpret_cast<double*>(w);
    w += ((2 * a0.n_groups * 5 * (int64_t)sizeof(double) + 255) / 256) * 256;
    ca.sync = reinterpret_cast<uint32_t*>(w);
    int dev = 0, cus = 0, coop = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (!coop) return hipErrorCooperativeLaunchTooLarge;
    const int nt = block_threads == 256 || block_threads == 512 || block_threads == 1024 ? block_threads
                   : a0.n_groups * coop_split(rmax, 1024) >= cus / 2                    ? 1024
                   : a0.n_groups * coop_split(rmax, 512) >= cus / 2                     ? 512
                                                                                         : 256;
    if (precision == 0)
        return nt == 1024 ? launch_coop<double, 1024>(ca, cus, s)
               : nt == 512 ? launch_coop<double, 512>(ca, cus, s)
                           : launch_coop<double, 256>(ca, cus, s);
    return nt == 1024 ? launch_coop<float, 1024>(ca, cus, s)
           : nt == 512 ? launch_coop<float, 512>(ca, cus, s)
                       : launch_coop<float, 256>(ca, cus, s);
}

}  // namespace csel
