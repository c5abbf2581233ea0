// aggregate.hip -- multi-target (aggregated / supernodal) greedy selection and
// the aggregated factor columns.
//
// Selection (Sec. 5.2, eq. greedy_mult; App. C.2): for a group of targets T
// and a candidate pool P, two partial Cholesky factors are kept over the rows
// R = P u T:
//   factor B conditions on the targets first (m columns, left-looking), then
//            on every selected point: var2_j = Theta_jj | T, I
//   factor A conditions on the selected points only: var1_j = Theta_jj | I
// and each pick maximizes 1 - var2_j / var1_j, the monotone form of the
// log-determinant decrease log var2 - log var1 of eq. greedy_mult.
//
// Schedule: one workgroup per group (grid-stride over groups).  Rows are
// spread over the threads (row r = i*NT + tid, RPT rows per thread, static),
// each thread keeping its rows' coordinates and FP64 var1/var2 in registers.
// The factors live column-major in a per-workgroup slab of the workspace
// (A[q*rmax + r], B[q*rmax + r]), so the per-pick GEMVs read coalesced
// columns; for the group sizes of interest the slab stays in L2/MALL.
// A pick is: per-thread top-two -> wave top-two (DPP) -> LDS -> workgroup
// top-two; the winner's factor rows are staged in LDS; every thread then
// evaluates Theta(row, winner), runs the two GEMVs and the FP64 downdates.
//
// Aggregated columns (Sec. 5.1; App. A.4, eq. L_precision): with
// s_g = sort(T u selected), U = P chol(P Theta_sg P) P is upper triangular and
// L = U^{-T}; member q's column is L[:, p_q], nonzero on the suffix of s_g
// that starts at q.  A second kernel builds the reversed Theta_sg in packed
// LDS (FP64), factors it right-looking (one barrier per column) and solves
// one column per wavefront with readlane broadcasts.
#include <algorithm>

#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

template <typename T>
__device__ __forceinline__ T matern_any(int two_nu, T r, T c, T s2) {
    if constexpr (sizeof(T) == 4) {
        if (two_nu == 1) return matern_f32<1>(r, c, s2);
        if (two_nu == 3) return matern_f32<3>(r, c, s2);
        return matern_f32<5>(r, c, s2);
    } else {
        return matern_f64_rt(two_nu, r, c, s2);
    }
}

constexpr int kAggMaxWaves = 16;

// byte offset of the slab kernel's LDS column caches: past the wave top-two
// records, the winner scalars and the winner's B and A rows
inline __host__ __device__ size_t agg_cache_offset(int max_members, int k, size_t elem_a) {
    const size_t b = sizeof(Top2) * kAggMaxWaves + 8 * sizeof(double) + ((size_t)k + max_members) * sizeof(double) +
                     (size_t)k * elem_a;
    return (b + 15) / 16 * 16;
}

// TA: factor A (the selected points only) and its covariance evaluations;
// TB: factor B (the targets, then the selected points).  FP64: both double.
// Mixed: A in FP32, B in FP64 -- var2 = Theta_jj | T, I falls far below
// the prior when many targets cluster (GP batches), below what an FP32
// evaluation resolves, while var1 stays large.
template <typename TA, typename TB, int RPT>
__global__ __launch_bounds__(1024) void agg_select_kernel(AggArgs p) {
    // slab entries in flight per row in the left-looking updates: eight with one
    // row per thread; with 2-4 rows per thread the registers are already short
    constexpr int kUD = RPT == 1 ? 8 : 1;
    extern __shared__ __align__(16) unsigned char agg_smem[];
    // LDS layout: wave top-two [16], winner scalars, winner B row [mmax+k], A row [k]
    Top2* wtop = reinterpret_cast<Top2*>(agg_smem);
    double* wsc = reinterpret_cast<double*>(agg_smem + sizeof(Top2) * kAggMaxWaves);  // var1, var2, x0..x2
    int32_t* wid = reinterpret_cast<int32_t*>(wsc + 6);
    TB* rowB = reinterpret_cast<TB*>(agg_smem + sizeof(Top2) * kAggMaxWaves + 8 * sizeof(double));
    TA* rowA = reinterpret_cast<TA*>(rowB + p.max_members + p.k);
    // LDS column caches (one row per thread): B's first nb columns, then A's
    // first na, each column NT entries (row r at entry r)
    const int nb = RPT == 1 ? p.cache_b : 0;
    const int na = RPT == 1 ? p.cache_a : 0;
    TB* cB = reinterpret_cast<TB*>(agg_smem + agg_cache_offset(p.max_members, p.k, sizeof(TA)));
    TA* cA = reinterpret_cast<TA*>(cB + (size_t)nb * blockDim.x);

    const int tid = threadIdx.x;
    const int NT = blockDim.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    const int nwaves = NT >> 6;
    const int rmax = p.rmax;
    // slab: B [(mmax + k) * rmax] of TB, then A [k * rmax] of TA
    TB* slabB = reinterpret_cast<TB*>(reinterpret_cast<char*>(p.ws) + (int64_t)blockIdx.x * p.slab_bytes);
    TA* slabA = reinterpret_cast<TA*>(slabB + (int64_t)(p.max_members + p.k) * rmax);
    const TA cnuA = (TA)p.c_nu, s2A = (TA)p.s2;
    const TB cnuB = (TB)p.c_nu, s2B = (TB)p.s2;
    const double prior = p.s2 + p.nugget;
    const double thr = 1e-12 * prior;
    const int dim = p.dim;

    for (int64_t g = blockIdx.x; g < p.n_groups; g += gridDim.x) {
        const int32_t b0 = p.group_ptr[g];
        const int32_t m = p.group_ptr[g + 1] - b0;
        const int32_t C = p.pool_len[g];
        int32_t* sel_out = p.sel + g * p.k;
        // ---- validate (uniform) ------------------------------------------
        bool bad = m < 1 || m > p.max_members || C < 0 || C > p.stride;
        const int R = bad ? 0 : C + m;
        // stage my rows
        int32_t rid[RPT];
        double x0[RPT], x1[RPT], x2[RPT], v1[RPT], v2[RPT];
        uint32_t live = 0;  // candidate rows not yet taken
        bool my_bad = false;
        int32_t my_max_member = -1;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = i * NT + tid;
            rid[i] = -1;
            x0[i] = x1[i] = x2[i] = 0.0;
            v1[i] = v2[i] = prior;
            if (r < R) {
                const int32_t id = r < C ? p.pool[g * p.stride + r] : p.members[b0 + (r - C)];
                if (id < 0 || (int64_t)id >= p.n) {
                    my_bad = true;
                } else {
                    rid[i] = id;
                    x0[i] = p.pts[(int64_t)id * dim];
                    if (dim > 1) x1[i] = p.pts[(int64_t)id * dim + 1];
                    if (dim > 2) x2[i] = p.pts[(int64_t)id * dim + 2];
                    if (r < C) live |= 1u << i;
                }
            }
        }
        // later-only check needs the largest member id: members are few, every
        // thread scans them (uniform result)
        // (the factor columns also need the members strictly ascending: a
        // member's column length is counted from its rank)
        if (!bad && p.later_only) {
            for (int q = 0; q < m; ++q) {
                const int32_t v = p.members[b0 + q];
                if (q > 0 && v <= my_max_member) bad = true;
                my_max_member = max(my_max_member, v);
            }
        }
        bool my_early = false;
        if (p.later_only) {
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                if (((live >> i) & 1u) && rid[i] <= my_max_member) my_early = true;
        }
        bad = __syncthreads_or(bad || my_bad);
        const bool early = __syncthreads_or(my_early);
        if (bad || early) {
            for (int t = tid; t < p.k; t += NT) {
                sel_out[t] = -1;
                if (p.gap) p.gap[g * p.k + t] = __builtin_nanf("");
            }
            if (tid == 0) {
                if (p.logdet) p.logdet[g] = __builtin_nan("");
                p.status[g] = bad ? 3 : 4;
            }
            if (p.post_var && !bad)
                for (int q = tid; q < m; q += NT) p.post_var[b0 + q] = __builtin_nan("");
            __syncthreads();
            continue;
        }

        // ---- factor B over the targets (left-looking, Sec. 5.2) -------------
        double ldT = 0.0;
        for (int c = 0; c < m; ++c) {
            const int prow = C + c;
            // the previous column's writes (slab, LDS reads) complete first
            __syncthreads();
            // owner publishes the pivot's var2 and coordinates
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                if (i * NT + tid == prow) {
                    wsc[1] = v2[i];
                    wsc[2] = x0[i];
                    wsc[3] = x1[i];
                    wsc[4] = x2[i];
                    wid[0] = rid[i];
                }
            for (int q = tid; q < c; q += NT) rowB[q] = q < nb ? cB[q * NT + prow] : slabB[(int64_t)q * rmax + prow];
            __syncthreads();
            const double piv = wsc[1];
            const double y0 = wsc[2], y1 = wsc[3], y2 = wsc[4];
            const int32_t idw = wid[0];
            ldT += log(piv);
            const double inv_sd = 1.0 / sqrt(piv);
            const TB inv_sd_t = (TB)inv_sd;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = i * NT + tid;
                if (r < R) {
                    const TB e0 = (TB)(x0[i] - y0), e1 = (TB)(x1[i] - y1), e2 = (TB)(x2[i] - y2);
                    TB acc = matern_any<TB>(p.two_nu, sqrt(sqnorm3(e0, e1, e2)), cnuB, s2B);
                    if (rid[i] == idw) acc += (TB)p.nugget;
                    acc = dot_down_cached<TB, kUD>(acc, cB + r, NT, nb, slabB + r, rmax, rowB, c);
                    const TB u = acc * inv_sd_t;
                    if (c < nb) cB[c * NT + r] = u;
                    else slabB[(int64_t)c * rmax + r] = u;
                    const double ud = (double)u;
                    v2[i] -= ud * ud;
                }
            }
        }

        // ---- greedy multi-target selection ---------------------------------
        const int kk = min(p.k, C);
        double ld = 0.0;
        int nsel = 0;
        int st = 0;
        for (int t = 0; t < kk; ++t) {
            Top2 loc = {0ull, 0ull};
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                // conditioning on the targets never raises a variance (var2 <= var1),
                // so the score is >= 0; rounding can push it below, and a negative
                // double would compare as a huge key
                if (((live >> i) & 1u) && v1[i] > thr && v2[i] > thr)
                    insert(loc, make_key(fmax(0.0, 1.0 - v2[i] / v1[i]), i * NT + tid));
            }
            const Top2 wv = wave_top2(loc);
            if (lane == 0) wtop[wave] = wv;
            __syncthreads();  // also orders the previous pick's column writes before the staging below
            Top2 w = wtop[0];
            for (int q = 1; q < nwaves; ++q) w = merge(w, wtop[q]);
            if (w.k1 == 0ull) {
                st = 1;
                break;
            }
            const int slot = key_slot(w.k1);
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                if (i * NT + tid == slot) {
                    wsc[0] = v1[i];
                    wsc[1] = v2[i];
                    wsc[2] = x0[i];
                    wsc[3] = x1[i];
                    wsc[4] = x2[i];
                    wid[0] = rid[i];
                    live &= ~(1u << i);
                }
            for (int q = tid; q < t; q += NT) rowA[q] = q < na ? cA[q * NT + slot] : slabA[(int64_t)q * rmax + slot];
            for (int q = tid; q < m + t; q += NT)
                rowB[q] = q < nb ? cB[q * NT + slot] : slabB[(int64_t)q * rmax + slot];
            __syncthreads();
            const double w1 = wsc[0], w2 = wsc[1];
            const double y0 = wsc[2], y1 = wsc[3], y2 = wsc[4];
            const int32_t idw = wid[0];
            ld += log(w2) - log(w1);
            if (tid == 0) {
                sel_out[t] = idw;
                if (p.gap) {
                    const double sa = key_score(w.k1), sb = key_score(w.k2);
                    p.gap[g * p.k + t] = (w.k2 == 0ull) ? 1.0f : (sa == 0.0 ? 0.0f : (float)((sa - sb) / sa));
                }
            }
            const TA inv1 = (TA)(1.0 / sqrt(w1));
            const TB inv2 = (TB)(1.0 / sqrt(w2));
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = i * NT + tid;
                if (r < R) {
                    const TB e0 = (TB)(x0[i] - y0), e1 = (TB)(x1[i] - y1), e2 = (TB)(x2[i] - y2);
                    TB thb = matern_any<TB>(p.two_nu, sqrt(sqnorm3(e0, e1, e2)), cnuB, s2B);
                    if (rid[i] == idw) thb += (TB)p.nugget;
                    TA tha;
                    if constexpr (sizeof(TA) == sizeof(TB)) {
                        tha = thb;
                    } else {
                        const TA f0 = (TA)(x0[i] - y0), f1 = (TA)(x1[i] - y1), f2 = (TA)(x2[i] - y2);
                        tha = matern_any<TA>(p.two_nu, sqrt(sqnorm3(f0, f1, f2)), cnuA, s2A);
                        if (rid[i] == idw) tha += (TA)p.nugget;
                    }
                    TA a = tha;
                    TB bb = thb;
                    a = dot_down_cached<TA, kUD>(a, cA + r, NT, na, slabA + r, rmax, rowA, t);
                    bb = dot_down_cached<TB, kUD>(bb, cB + r, NT, nb, slabB + r, rmax, rowB, m + t);
                    const TA u1 = a * inv1;
                    const TB u2 = bb * inv2;
                    if (t < na) cA[t * NT + r] = u1;
                    else slabA[(int64_t)t * rmax + r] = u1;
                    if (m + t < nb) cB[(m + t) * NT + r] = u2;
                    else slabB[(int64_t)(m + t) * rmax + r] = u2;
                    const double d1 = (double)u1, d2 = (double)u2;
                    v1[i] -= d1 * d1;
                    v2[i] -= d2 * d2;
                }
            }
            nsel = t + 1;
        }
        // ---- outputs ----------------------------------------------------------
        for (int t = nsel + tid; t < p.k; t += NT) {
            sel_out[t] = -1;
            if (p.gap) p.gap[g * p.k + t] = __builtin_nanf("");
        }
        if (tid == 0) {
            if (p.logdet) p.logdet[g] = ldT + ld;
            p.status[g] = (uint8_t)st;
        }
        if (p.post_var) {
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = i * NT + tid;
                if (r >= C && r < R) p.post_var[b0 + (r - C)] = v1[i];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// register-resident multi-target selection (mixed precision, C <= 512,
// m <= 32, k <= KA): one workgroup of 512 threads per group, thread r owning
// pool row r with its rows of both partial factors in VGPRs
// ---------------------------------------------------------------------------
// The targets are conditioned first through chol(Theta_TT), computed in FP64
// by one wave (left-looking, lane r owning row r) and kept in LDS: each
// candidate row then solves for its B entries over the targets (forward
// substitution, FP32).  Factor A's row and B's target columns stay in
// VGPRs; B's pick columns live in LDS, column-major [t][row] (128 KB at
// k = 64), where each thread reads its own entries and the winner's as a
// broadcast.  A pick: FP64 score 1 - var2/var1 -> wave top-two -> LDS ->
// every thread merges the eight wave results; the winner stores its
// register rows, offset and variances in LDS; every thread evaluates
// Theta(row, winner) in FP32, runs both GEMVs and downdates var1, var2 in
// FP64.  Offsets are taken from the group's first
// member so FP32 differences stay accurate.  Posterior variances (target
// rows) are not tracked here: that mode uses the slab kernel.
constexpr int kAggRegThreads = 512;
constexpr int kAggRegMaxM = 32;

// a running product held as mantissa * 2^exponent, so a sum of logarithms
// costs one log at the end
struct LogProd {
    double mant = 1.0;
    int expo = 0;
    __device__ void mul(double x) {
        int e;
        mant = frexp(mant * x, &e);
        expo += e;
    }
    __device__ double log_value() const { return log(mant) + (double)expo * 0.69314718055994530942; }
};

template <int KA, bool GAP>
__global__ __launch_bounds__(kAggRegThreads, 1) void agg_select_reg_kernel(AggArgs p) {
    constexpr int MM = kAggRegMaxM;
    constexpr int NW = kAggRegThreads / 64;
    constexpr int NR = kAggRegThreads;  // rows (pool slots) per group
    extern __shared__ __align__(16) float sh_bp[];  // B pick columns [KA][NR]
    __shared__ double sh_th[MM][MM + 1];  // Theta_TT, then its Cholesky factor (rows)
    __shared__ float sh_lt[MM][MM];       // the factor in FP32 for the forward substitution
    __shared__ float sh_ltinv[MM];        // 1 / diagonal
    __shared__ float sh_tx[MM][4];        // target offsets from the reference point
    __shared__ int32_t sh_tid[MM];        // target ids
    __shared__ __align__(16) float sh_row[KA + MM + 4];  // winner: A row, B target part, offset
    __shared__ double sh_wv[4];           // winner var1, var2, id
    __shared__ Top2 sh_top[NW];
    __shared__ double sh_ldt;

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    const float cnu = (float)p.c_nu, s2f = (float)p.s2, nugf = (float)p.nugget;
    const double prior = p.s2 + p.nugget;
    const double thr = 1e-12 * prior;
    const int dim = p.dim;

    for (int64_t g = blockIdx.x; g < p.n_groups; g += gridDim.x) {
        const int32_t b0 = p.group_ptr[g];
        const int32_t m = p.group_ptr[g + 1] - b0;
        const int32_t C = p.pool_len[g];
        int32_t* sel_out = p.sel + g * p.k;
        bool bad = m < 1 || m > p.max_members || m > MM || C < 0 || C > p.stride || C > kAggRegThreads;
        // reference point: the first member
        double ref[3] = {0.0, 0.0, 0.0};
        int32_t max_member = -1;
        if (!bad) {
            const int32_t r0 = p.members[b0];
            if (r0 < 0 || (int64_t)r0 >= p.n) {
                bad = true;
            } else {
                for (int c = 0; c < dim; ++c) ref[c] = p.pts[(int64_t)r0 * dim + c];
                // factor columns need the members strictly ascending
                for (int q = 0; q < m; ++q) {
                    const int32_t v = p.members[b0 + q];
                    if (p.later_only && q > 0 && v <= max_member) bad = true;
                    max_member = max(max_member, v);
                }
            }
        }
        bool my_bad = false, my_early = false;
        // my pool row
        int32_t rid = -1;
        float dx0 = 0.f, dx1 = 0.f, dx2 = 0.f;
        if (!bad && tid < C) {
            const int32_t id = p.pool[g * p.stride + tid];
            if (id < 0 || (int64_t)id >= p.n) {
                my_bad = true;
            } else {
                rid = id;
                dx0 = (float)(p.pts[(int64_t)id * dim] - ref[0]);
                if (dim > 1) dx1 = (float)(p.pts[(int64_t)id * dim + 1] - ref[1]);
                if (dim > 2) dx2 = (float)(p.pts[(int64_t)id * dim + 2] - ref[2]);
                if (p.later_only && id <= max_member) my_early = true;
            }
        }
        // targets -> LDS
        if (!bad && tid < m) {
            const int32_t id = p.members[b0 + tid];
            if (id < 0 || (int64_t)id >= p.n) {
                my_bad = true;
            } else {
                sh_tid[tid] = id;
                sh_tx[tid][0] = (float)(p.pts[(int64_t)id * dim] - ref[0]);
                sh_tx[tid][1] = dim > 1 ? (float)(p.pts[(int64_t)id * dim + 1] - ref[1]) : 0.f;
                sh_tx[tid][2] = dim > 2 ? (float)(p.pts[(int64_t)id * dim + 2] - ref[2]) : 0.f;
            }
        }
        bad = __syncthreads_or(bad || my_bad);
        const bool early = __syncthreads_or(my_early);
        if (bad || early) {
            for (int t = tid; t < p.k; t += kAggRegThreads) {
                sel_out[t] = -1;
                if (p.gap) p.gap[g * p.k + t] = __builtin_nanf("");
            }
            if (tid == 0) {
                if (p.logdet) p.logdet[g] = __builtin_nan("");
                p.status[g] = bad ? 3 : 4;
            }
            __syncthreads();
            continue;
        }
        // ---- Theta_TT (FP64, one entry per thread) and its Cholesky factor --
        for (int e = tid; e < MM * (MM + 1) / 2; e += kAggRegThreads) {
            int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            while ((r + 1) * (r + 2) / 2 <= e) ++r;
            while (r * (r + 1) / 2 > e) --r;
            const int c = e - r * (r + 1) / 2;
            if (r < m) {
                const int32_t ir = p.members[b0 + r], ic = p.members[b0 + c];
                double d2 = 0.0;
                for (int q = 0; q < dim; ++q) {
                    const double df = p.pts[(int64_t)ir * dim + q] - p.pts[(int64_t)ic * dim + q];
                    d2 += df * df;
                }
                sh_th[r][c] = matern_f64_rt(p.two_nu, sqrt(d2), p.c_nu, p.s2) + (ir == ic ? p.nugget : 0.0);
            }
        }
        __syncthreads();
        bool pd = true;
        if (wave == 0) {
            // left-looking, lane r finishing row r of the factor in LDS
            LogProd ldt;
            for (int j = 0; j < m; ++j) {
                double sj = 0.0;
                if (lane >= j && lane < m) {
                    sj = sh_th[lane][j];
                    for (int c = 0; c < j; ++c) sj -= sh_th[lane][c] * sh_th[j][c];
                }
                const double piv = bcast(sj, j);
                if (!(piv > 0.0)) {
                    pd = false;
                    break;
                }
                const double inv = rsq64(piv);
                ldt.mul(piv);
                if (lane >= j && lane < m) sh_th[lane][j] = lane == j ? piv * inv : sj * inv;
                if (lane == j) sh_ltinv[j] = (float)inv;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            for (int e = lane; e < MM * MM; e += 64) {
                const int r = e / MM, c = e - (e / MM) * MM;
                sh_lt[r][c] = (c < r && r < m) ? (float)sh_th[r][c] : 0.0f;
            }
            if (lane == 0) sh_ldt = pd ? ldt.log_value() : __builtin_nan("");
        }
        pd = __syncthreads_and(wave != 0 || pd);
        if (!pd) {  // Theta_TT not positive definite in FP64: no selection
            for (int t = tid; t < p.k; t += kAggRegThreads) {
                sel_out[t] = -1;
                if (p.gap) p.gap[g * p.k + t] = __builtin_nanf("");
            }
            if (tid == 0) {
                if (p.logdet) p.logdet[g] = __builtin_nan("");
                p.status[g] = 2;
            }
            __syncthreads();
            continue;
        }
        // ---- condition my row on the targets: B[0, m) --------------------------
        float A[KA], B[MM];
#pragma unroll
        for (int q = 0; q < KA; ++q) A[q] = 0.0f;
#pragma unroll
        for (int q = 0; q < MM; ++q) B[q] = 0.0f;
        double v1 = rid >= 0 ? prior : -1.0;  // -1: never a candidate
        double v2 = prior;
#pragma unroll
        for (int c = 0; c < MM; ++c) {
            asm volatile("" ::: "memory");  // one row of the factor's LDS copy at a time
            if (c < m) {
                const float e0 = dx0 - sh_tx[c][0], e1 = dx1 - sh_tx[c][1], e2 = dx2 - sh_tx[c][2];
                float acc = matern_any<float>(p.two_nu, __builtin_amdgcn_sqrtf(e0 * e0 + e1 * e1 + e2 * e2), cnu, s2f);
                if (rid == sh_tid[c]) acc += nugf;
#pragma unroll
                for (int q = 0; q < c; ++q) acc -= B[q] * sh_lt[c][q];
                B[c] = acc * sh_ltinv[c];
                v2 -= (double)B[c] * (double)B[c];
            }
        }
        // ---- greedy multi-target selection ---------------------------------------
        const int kk = min(p.k, C);
        LogProd ld;  // prod of var2 / var1 of the winners (thread 0)
        int nsel = 0;
        int st = 0;
        bool stopped = false;
#pragma unroll
        for (int t = 0; t < KA; ++t) {
            if (t < kk && !stopped) {
                const bool valid = v1 > thr && v2 > thr;
                const uint64_t key = valid ? make_key(fmax(0.0, (v1 - v2) * rcp64(v1)), tid) : 0ull;
                Top2 w;
                if constexpr (GAP) {
                    w = wave_top2(Top2{key, 0ull});
                } else {
                    w.k1 = wave_max64(key);
                    w.k2 = 0ull;
                }
                if (lane == 0) sh_top[wave] = w;
                __syncthreads();  // also: every thread is done reading the previous winner
                w = sh_top[0];
#pragma unroll
                for (int q = 1; q < NW; ++q) {
                    if constexpr (GAP) {
                        w = merge(w, sh_top[q]);
                    } else {
                        w.k1 = max(w.k1, sh_top[q].k1);
                    }
                }
                if (w.k1 == 0ull) {
                    st = 1;
                    stopped = true;
                } else {
                    const int slot = key_slot(w.k1);
                    if (tid == slot) {
#pragma unroll
                        for (int q = 0; q < t; ++q) sh_row[q] = A[q];
#pragma unroll
                        for (int q = 0; q < MM; ++q) sh_row[KA + q] = B[q];
                        sh_row[KA + MM] = dx0;
                        sh_row[KA + MM + 1] = dx1;
                        sh_row[KA + MM + 2] = dx2;
                        sh_wv[0] = v1;
                        sh_wv[1] = v2;
                        sh_wv[2] = (double)rid;
                        v1 = -1.0;  // taken
                    }
                    __syncthreads();
                    const double w1 = sh_wv[0], w2 = sh_wv[1];
                    const int32_t idw = (int32_t)sh_wv[2];
                    if (tid == 0) {
                        sel_out[t] = idw;
                        ld.mul(w2 * rcp64(w1));
                        if constexpr (GAP) {
                            const double sa = key_score(w.k1), sb = key_score(w.k2);
                            if (p.gap)
                                p.gap[g * p.k + t] =
                                    (w.k2 == 0ull) ? 1.0f : (sa == 0.0 ? 0.0f : (float)((sa - sb) / sa));
                        }
                    }
                    const float inv1 = (float)rsq64(w1), inv2 = (float)rsq64(w2);
                    const float e0 = dx0 - sh_row[KA + MM], e1 = dx1 - sh_row[KA + MM + 1],
                                e2 = dx2 - sh_row[KA + MM + 2];
                    float th = matern_any<float>(p.two_nu, __builtin_amdgcn_sqrtf(e0 * e0 + e1 * e1 + e2 * e2), cnu, s2f);
                    if (rid == idw) th += nugf;
                    // GEMVs against the broadcast rows, 32 LDS values at a time
                    // (the empty asm keeps the compiler from hoisting every
                    // broadcast load of the pick into registers at once)
                    float a = th, b = th;
#pragma unroll
                    for (int q0 = 0; q0 < t; q0 += 32) {
                        asm volatile("" ::: "memory");
#pragma unroll
                        for (int q = q0; q < q0 + 32 && q < t; ++q) a -= A[q] * sh_row[q];
                    }
                    asm volatile("" ::: "memory");
#pragma unroll
                    for (int q4 = 0; q4 < MM / 4; ++q4) {
                        if (4 * q4 < m) {  // entries past m are zero on both sides
#pragma unroll
                            for (int q = 4 * q4; q < 4 * q4 + 4; ++q) b -= B[q] * sh_row[KA + q];
                        }
                    }
                    // B's pick columns: my entry and the winner's (a broadcast)
#pragma unroll
                    for (int q0 = 0; q0 < t; q0 += 32) {
                        asm volatile("" ::: "memory");
#pragma unroll
                        for (int q = q0; q < q0 + 32 && q < t; ++q) b -= sh_bp[q * NR + tid] * sh_bp[q * NR + slot];
                    }
                    const float u1 = a * inv1, u2 = b * inv2;
                    A[t] = u1;
                    sh_bp[t * NR + tid] = u2;
                    v1 -= (double)u1 * (double)u1;
                    v2 -= (double)u2 * (double)u2;
                    nsel = t + 1;
                }
            }
        }
        // ---- outputs ----------------------------------------------------------
        for (int t = nsel + tid; t < p.k; t += kAggRegThreads) {
            sel_out[t] = -1;
            if (p.gap) p.gap[g * p.k + t] = __builtin_nanf("");
        }
        if (tid == 0) {
            if (p.logdet) p.logdet[g] = sh_ldt + ld.log_value();
            p.status[g] = (uint8_t)st;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// aggregated factor columns (FP64)
// ---------------------------------------------------------------------------
constexpr int kAggFacMaxM = 96;  // |s_g| = m + selected
constexpr int kAggFacThreads = 128;

__host__ __device__ constexpr int tri(int i) { return i * (i + 1) / 2; }

// One 128-thread workgroup per group.  The reversed Theta_sg is built in
// packed LDS rows (its lower triangle spread evenly over the threads), then
// factored left-looking by columns: thread r keeps row r in VGPRs, reads
// row j of the factor from LDS as a broadcast, and stores its column-j entry
// back for the rows after it (two barriers per column).  One wave per member
// then back-substitutes its column against the stored rows.
__global__ __launch_bounds__(kAggFacThreads) void agg_factor_kernel(AggArgs p) {
    constexpr int MF = kAggFacMaxM;
    __shared__ double A[tri(MF)];       // reversed Theta_sg, then its Cholesky factor (packed rows)
    __shared__ double pc[MF][3];        // coordinates of s_g in reversed order
    __shared__ double dinv[MF];         // 1 / R[j][j]
    __shared__ int32_t sg[MF];
    __shared__ int32_t bad_piv;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    const int64_t g = blockIdx.x;
    if (g >= p.n_groups) return;
    if (p.status[g] >= 2) return;  // nothing to build (values were left untouched)
    const int32_t b0 = p.group_ptr[g];
    const int32_t m = p.group_ptr[g + 1] - b0;
    const int32_t* sel = p.sel + g * p.k;
    int nsel = 0;
    while (nsel < p.k && sel[nsel] >= 0) ++nsel;
    const int M = m + nsel;
    if (M > MF) {
        if (tid == 0) p.status[g] = 5;
        return;
    }
    const int dim = p.dim;
    // s_g sorted ascending: rank sort (ids are distinct); coordinates in reversed order
    for (int a = tid; a < M; a += kAggFacThreads) {
        const int32_t v = a < m ? p.members[b0 + a] : sel[a - m];
        int rank = 0;
        for (int c = 0; c < M; ++c) {
            const int32_t w = c < m ? p.members[b0 + c] : sel[c - m];
            rank += (w < v);
        }
        sg[rank] = v;
        for (int d = 0; d < 3; ++d) pc[M - 1 - rank][d] = d < dim ? p.pts[(int64_t)v * dim + d] : 0.0;
    }
    if (tid == 0) bad_piv = 0;
    __syncthreads();
    // reversed order: index i' = M-1-i; packed lower entries (i', c') with c' <= i'
    const double cnu = p.c_nu;
    for (int e = tid; e < tri(M); e += kAggFacThreads) {
        int i = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        while (tri(i + 1) <= e) ++i;
        while (tri(i) > e) --i;
        const int c = e - tri(i);
        const double d0 = pc[i][0] - pc[c][0], d1 = pc[i][1] - pc[c][1], d2 = pc[i][2] - pc[c][2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const double r = r2 > 0.0 ? r2 * rsq64(r2) : 0.0;
        A[e] = matern_f64_rt(p.two_nu, r, cnu, p.s2) + (i == c ? p.nugget : 0.0);
    }
    __syncthreads();
    // left-looking Cholesky, row r in thread r's registers
    {
        double a[MF];
#pragma unroll
        for (int c = 0; c < MF; ++c) a[c] = (c <= tid && tid < M) ? A[tri(tid) + c] : 0.0;
        __syncthreads();
        bool stop = false;  // uniform: past M or a non-positive pivot
#pragma unroll
        for (int j = 0; j < MF; ++j) {
            if (j >= M || stop) continue;
            // the row dot product in four independent partial sums (short
            // dependent FP64 chains), combined in a fixed order; the compiler
            // barrier every 16 entries keeps the row's LDS loads from all
            // being hoisted into registers at once
            double s4[4] = {a[j], 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < j; ++c) {
                if (c % 16 == 0 && c > 0) asm volatile("" ::: "memory");
                s4[c & 3] -= a[c] * A[tri(j) + c];
            }
            const double sj = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            if (tid == j) {
                if (sj > 0.0) {
                    const double inv = rsq64(sj);
                    a[j] = sj * inv;
                    A[tri(j) + j] = a[j];
                    dinv[j] = inv;
                } else {
                    bad_piv = 1;
                }
            }
            __syncthreads();
            if (bad_piv) {
                stop = true;
                continue;
            }
            if (tid > j && tid < M) {
                a[j] = sj * dinv[j];
                A[tri(tid) + j] = a[j];
            }
            __syncthreads();
        }
    }
    // member columns: member at sorted position pos -> reversed index jr = M-1-pos;
    // z = R^{-T} e_jr (entries z_i, i <= jr): column-oriented back-substitution.
    const int nw = kAggFacThreads / kWave;
    for (int a = wave; a < m; a += nw) {
        const int32_t q = p.members[b0 + a];
        int pos = 0;
        while (pos < M && sg[pos] != q) ++pos;
        const int jr = M - 1 - pos;
        double* vals = p.fac_val + p.val_ptr[b0 + a];
        int32_t* rows = p.fac_rows + p.val_ptr[b0 + a];
        const int len = M - pos;
        const int64_t budget = p.val_ptr[b0 + a + 1] - p.val_ptr[b0 + a];
        if (pos >= M || len > budget) {
            // members not strictly ascending (rejected by the selection kernels
            // before this runs): write nothing outside the member's slots
            if (lane == 0) p.status[g] = 3;
            continue;
        }
        if (bad_piv) {
            for (int l = lane; l < len; l += kWave) {
                vals[l] = __builtin_nan("");
                rows[l] = sg[pos + l];
            }
            if (lane == 0 && p.member_logcv) p.member_logcv[b0 + a] = __builtin_nan("");
            continue;
        }
        // lanes own reversed indices i = lane and lane + 64 (M <= 128)
        double acc0 = 0.0, acc1 = 0.0, z0 = 0.0, z1 = 0.0;
        for (int l = jr; l >= 0; --l) {
            const double il = dinv[l];  // 1 / R[l][l]
            double zl;
            if (l == jr) {
                zl = il;
            } else {
                const double al = (l < kWave) ? bcast(acc0, l) : bcast(acc1, l - kWave);
                zl = -al * il;
            }
            if (lane == l) z0 = zl;
            if (lane + kWave == l) z1 = zl;
            // rows i < l take R[l][i] * z_l
            if (lane < l) acc0 += A[tri(l) + lane] * zl;
            if (lane + kWave < l) acc1 += A[tri(l) + lane + kWave] * zl;
        }
        // reversed index i -> original position M-1-i -> output slot (M-1-i) - pos
        if (lane <= jr) {
            const int o = (M - 1 - lane) - pos;
            vals[o] = z0;
            rows[o] = sg[M - 1 - lane];
        }
        if (lane + kWave <= jr) {
            const int o = (M - 1 - lane - kWave) - pos;
            vals[o] = z1;
            rows[o] = sg[M - 1 - lane - kWave];
        }
        if (lane == 0 && p.member_logcv) p.member_logcv[b0 + a] = -2.0 * log(dinv[jr]);
        // pad the member's slot range if fewer points were selected than budgeted
        for (int64_t l = len + lane; l < budget; l += kWave) {
            vals[l] = 0.0;
            rows[l] = -1;
        }
    }
    if (tid == 0 && bad_piv) p.status[g] = 2;
}

// LDS of one CU, and the most one workgroup's column caches take
constexpr size_t kCuLds = 160 * 1024;
constexpr size_t kAggCacheLds = 152 * 1024;

template <typename TA, typename TB, int RPT>
static hipError_t launch_sel(const AggArgs& a0, int nt, unsigned grid, size_t smem, hipStream_t s) {
    AggArgs a = a0;
    auto kern = agg_select_kernel<TA, TB, RPT>;
    if (RPT == 1) {
        // Column caches in the LDS that the workgroups resident on a CU leave
        // free (as many as its registers allow without the caches): the first
        // columns of B (the target columns and the first picks, re-read by
        // every later step) take three quarters, A's first columns the rest.
        int res = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&res, (const void*)kern, nt, smem);
        if (e != hipSuccess) return e;
        const size_t per_cu = (size_t)std::max(1, res);
        const size_t lds = std::min(kAggCacheLds, kCuLds / per_cu - 1024);
        const size_t off = agg_cache_offset(a.max_members, a.k, sizeof(TA));
        const size_t avail = lds > off ? lds - off : 0;
        const size_t colB = (size_t)nt * sizeof(TB), colA = (size_t)nt * sizeof(TA);
        const int nb = (int)std::min<size_t>(avail * 3 / 4 / colB, (size_t)a.max_members + a.k);
        const int na = (int)std::min<size_t>((avail - nb * colB) / colA, (size_t)a.k);
        a.cache_b = nb;
        a.cache_a = na;
        smem = std::max(smem, off + nb * colB + na * colA);
    }
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(nt), smem, s, a);
    return hipGetLastError();
}

AggPlan plan_aggregated(int64_t n_groups, int32_t stride, int32_t max_members, int32_t k, int precision) {
    AggPlan pl;
    pl.rmax = stride + max_members;
    pl.rpt = (pl.rmax + 1023) / 1024;
    pl.rpt = pl.rpt <= 1 ? 1 : pl.rpt <= 2 ? 2 : 4;
    pl.threads = std::min(1024, std::max(64, ((pl.rmax + pl.rpt - 1) / pl.rpt + 63) / 64 * 64));
    // the slab kernel: factor B in FP64, factor A in FP64 or (mixed) FP32
    const int64_t elemA = precision == 0 ? 8 : 4;
    pl.slab_bytes = ((int64_t)max_members + k) * pl.rmax * 8 + (int64_t)k * pl.rmax * elemA;
    pl.slab_bytes = (pl.slab_bytes + 255) / 256 * 256;
    // enough slots to fill the chip several times over, capped by the group count
    pl.slots = (int)std::min<int64_t>(n_groups, 1024);
    if (pl.slots < 1) pl.slots = 1;
    pl.ws_bytes = pl.slab_bytes * pl.slots;
    if (agg_split_possible(n_groups, max_members, k))
        pl.ws_bytes = std::max<int64_t>(pl.ws_bytes, agg_coop_workspace(n_groups, stride, max_members, k));
    pl.smem = sizeof(Top2) * kAggMaxWaves + 8 * sizeof(double) + ((size_t)k + max_members) * 8 + (size_t)k * elemA;
    return pl;
}

template <int KA, bool GAP>
static hipError_t launch_reg(const AggArgs& a, hipStream_t s) {
    // one 512-thread workgroup per CU (its LDS holds B's pick columns)
    const size_t smem = (size_t)KA * kAggRegThreads * sizeof(float);
    auto kern = agg_select_reg_kernel<KA, GAP>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    const unsigned grid = (unsigned)std::min<int64_t>(a.n_groups, 4096);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kAggRegThreads), smem, s, a);
    return hipGetLastError();
}

// few groups with pools past one workgroup's rows: each group's rows split
// over several cooperatively launched workgroups (mixed runs the register
// kernel covers stay there)
bool agg_coop_applies(int64_t n_groups, int32_t stride, int32_t max_members, int32_t k, int precision) {
    return n_groups > 0 && n_groups <= 128 && k <= 256 && max_members <= 128 &&
           (int64_t)stride + max_members > 256;
}

// the register-resident kernel applies to mixed precision without posterior
// variances, pools <= 512, groups <= 32 and k <= 64
bool agg_split_possible(int64_t n_groups, int32_t max_members, int32_t k) {
    return n_groups > 0 && n_groups <= 1024 && k <= 256 && max_members <= 128;
}

bool agg_reg_applies(int32_t stride, int32_t max_members, int32_t k, int precision, bool want_post_var) {
    return precision != 0 && !want_post_var && stride <= kAggRegThreads && max_members <= kAggRegMaxM && k <= 64;
}

hipError_t launch_aggregated(const AggArgs& a, const AggPlan& pl, int precision, bool want_factor, int schedule,
                             hipStream_t s) {
    if (a.n_groups == 0) return hipSuccess;
    hipError_t e;
    const unsigned grid = (unsigned)pl.slots;
    const bool reg_ok = agg_reg_applies(a.stride, a.max_members, a.k, precision, a.post_var != nullptr);
    if (schedule == kAggRegister && !reg_ok) return hipErrorNotSupported;
    if (schedule >= kAggSplit256) {
        // explicit split rows: selection only, within the workspace's reach
        if (want_factor || !agg_split_possible(a.n_groups, a.max_members, a.k)) return hipErrorNotSupported;
        const int nt = schedule == kAggSplit256 ? 256 : schedule == kAggSplit512 ? 512 : 1024;
        return launch_aggregated_coop(a, precision, nt, a.ws, s);
    }
    if (reg_ok && (schedule == kAggAuto || schedule == kAggRegister)) {
        const bool gap = a.gap != nullptr;
        e = a.k <= 16 ? (gap ? launch_reg<16, true>(a, s) : launch_reg<16, false>(a, s))
            : a.k <= 32 ? (gap ? launch_reg<32, true>(a, s) : launch_reg<32, false>(a, s))
                        : (gap ? launch_reg<64, true>(a, s) : launch_reg<64, false>(a, s));
        if (e != hipSuccess) return e;
        if (want_factor) {
            hipLaunchKernelGGL(agg_factor_kernel, dim3((unsigned)a.n_groups), dim3(kAggFacThreads), 0, s, a);
            e = hipGetLastError();
        }
        return e;
    }
    if (schedule == kAggAuto && agg_coop_applies(a.n_groups, a.stride, a.max_members, a.k, precision)) {
        e = launch_aggregated_coop(a, precision, 0, a.ws, s);
        if (e == hipSuccess) {
            if (want_factor) {
                hipLaunchKernelGGL(agg_factor_kernel, dim3((unsigned)a.n_groups), dim3(kAggFacThreads), 0, s, a);
                e = hipGetLastError();
            }
            return e;
        }
        if (e != hipErrorCooperativeLaunchTooLarge && e != hipErrorNotSupported) return e;
        (void)hipGetLastError();  // the one-workgroup-per-group kernel instead
    }
    if (precision == 0) {
        e = pl.rpt == 1 ? launch_sel<double, double, 1>(a, pl.threads, grid, pl.smem, s)
            : pl.rpt == 2 ? launch_sel<double, double, 2>(a, pl.threads, grid, pl.smem, s)
                          : launch_sel<double, double, 4>(a, pl.threads, grid, pl.smem, s);
    } else {
        e = pl.rpt == 1 ? launch_sel<float, double, 1>(a, pl.threads, grid, pl.smem, s)
            : pl.rpt == 2 ? launch_sel<float, double, 2>(a, pl.threads, grid, pl.smem, s)
                          : launch_sel<float, double, 4>(a, pl.threads, grid, pl.smem, s);
    }
    if (e != hipSuccess) return e;
    if (want_factor) {
        hipLaunchKernelGGL(agg_factor_kernel, dim3((unsigned)a.n_groups), dim3(kAggFacThreads), 0, s, a);
        e = hipGetLastError();
    }
    return e;
}

int agg_factor_max_m() { return kAggFacMaxM; }

hipError_t launch_agg_factor(const AggArgs& a, hipStream_t s) {
    if (a.n_groups == 0) return hipSuccess;
    hipLaunchKernelGGL(agg_factor_kernel, dim3((unsigned)a.n_groups), dim3(kAggFacThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace csel
