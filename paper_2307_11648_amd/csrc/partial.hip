// partial.hip -- partial (non-adjacent) aggregated selection (Sec. 5.1 eq.
// chol_partial and eq. partial_kl; App. C.3 eq. chol_partial_update, eq.
// partial_diag, eq. obj_partial, eq. partial_induct).
//
// A group's candidates may lie between its targets; a candidate conditions
// only the targets it follows (larger id = later point).  The group's KL
// term is the log determinant of the partially conditioned target
// covariance, sum_q log L_qq^2 of the Cholesky factor L of Theta over the
// selected and target points sorted by decreasing id (the "columns"), with
// one row per target and candidate.
//
// Schedule: one 512-thread workgroup per group, FP64.
//   * candidate rows: thread j owns pool slot j and its row of L in VGPRs,
//     in column order (L[c], c < ncol <= 64), every index static;
//   * column points (targets and picks): their rows of L (the square part)
//     live in LDS at physical slots in insertion order (targets first), with
//     `ord` mapping column order to physical slots, so an insertion moves
//     nothing in LDS;
//   * one pick: every candidate's score by the induction over the columns
//     (with v its variance given the columns before c: at a target column
//     it conditions, the target's variance falls by 1 - L[c]^2 / v; then
//     v -= L[c]^2), a workgroup top-two, the winner's row broadcast; then
//     the new column u = (Theta(:, k) - L[:, :p] L[k, :p]^T) / sqrt(v_k) by
//     left-looking over the p columns before the pick (eq. chol_partial_update),
//     and the rank-one downdate of the columns after it by u: wave 0 runs
//     it on the square part (one column at a time, the pivot's running w by
//     readlane) and records each column's (cs, sn); every candidate row then
//     applies the same rotations to its own row and shifts its columns to
//     make room for u.
//   Three workgroup barriers per pick.
// The member columns (eq. L_col on s_q = {j in sort(T u S) : j >= q}) are
// built afterwards by the aggregated factor kernel, which handles picks
// between members.
#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

constexpr int kPartThreads = 512;           // pool slots (one row per thread)
constexpr int kPartCols = 64;               // members + picks
constexpr int kPartMaxMembers = 32;
constexpr int kPartMaxK = 32;

template <int TWO_NU>
__device__ __forceinline__ double part_cov(const double* a, const double* b, double c_nu, double s2) {
    const double r = dist64(sqnorm3(a[0] - b[0], a[1] - b[1], a[2] - b[2]));
    return matern_f64<TWO_NU>(r, c_nu, s2);
}

template <int TWO_NU>
__global__ __launch_bounds__(kPartThreads) void partial_select_kernel(AggArgs p) {
    __shared__ double Lsq[kPartCols][kPartCols];  // [physical row][physical column]
    __shared__ double cpt[kPartCols][3];          // column points' coordinates (physical)
    __shared__ int32_t cid[kPartCols];            // and ids
    __shared__ int32_t ord[kPartCols];            // column order -> physical slot
    __shared__ double bk[kPartCols];              // the winner's row (column order), first p entries
    __shared__ double bx[3];
    __shared__ double bv;                         // the winner's variance given the columns before it
    __shared__ int32_t bid, bp;
    __shared__ double rot_cs[kPartCols], rot_sn[kPartCols], rot_ics[kPartCols];
    __shared__ uint64_t wk1[kPartThreads / kWave], wk2[kPartThreads / kWave];
    __shared__ uint64_t tmask_sh;                 // bit c: column c is a target
    __shared__ int32_t bad_sh, notpd_sh;
    __shared__ int32_t sel_sh[kPartMaxK];
    __shared__ float gap_sh[kPartMaxK];

    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    const int64_t g = blockIdx.x;
    if (g >= p.n_groups) return;
    const int32_t b0 = p.group_ptr[g];
    const int32_t m = p.group_ptr[g + 1] - b0;
    const int32_t C = p.pool_len[g];
    const int dim = p.dim;
    const double c_nu = p.c_nu, s2 = p.s2, nug = p.nugget;
    const double prior = s2 + nug;
    const double thr = 1e-12 * prior;
    const int kk = min(p.k, max(C, 0));

    // ---- validation (the same decision in every thread) -------------------
    bool bad = m < 1 || m > p.max_members || m > kPartMaxMembers || C < 0 || C > p.stride || C > kPartThreads ||
               m + kk > kPartCols;
    if (tid == 0) {
        bad_sh = 0;
        notpd_sh = 0;
    }
    __syncthreads();
    if (!bad) {
        if (tid < m) {
            const int32_t q = p.members[b0 + tid];
            if (q < 0 || (int64_t)q >= p.n || (tid > 0 && !(p.members[b0 + tid - 1] < q))) bad_sh = 1;
            cid[tid] = q;
            for (int d = 0; d < 3; ++d) cpt[tid][d] = (d < dim && q >= 0 && (int64_t)q < p.n) ? p.pts[(int64_t)q * dim + d] : 0.0;
        }
    }
    __syncthreads();
    bad = bad || bad_sh != 0;
    // my candidate row
    int32_t my_id = -1;
    double xr[3] = {0.0, 0.0, 0.0};
    if (!bad && tid < C) {
        my_id = p.pool[g * p.stride + tid];
        bool ok = my_id >= 0 && (int64_t)my_id < p.n;
        for (int a = 0; a < m && ok; ++a) ok = cid[a] != my_id;
        for (int s = 0; s < tid && ok; ++s) ok = p.pool[g * p.stride + s] != my_id;
        if (!ok) {
            bad_sh = 1;
        } else {
            for (int d = 0; d < dim; ++d) xr[d] = p.pts[(int64_t)my_id * dim + d];
        }
    }
    __syncthreads();
    bad = bad || bad_sh != 0;
    if (bad) {
        for (int t = tid; t < p.k; t += kPartThreads) {
            p.sel[g * p.k + t] = -1;
            if (p.gap) p.gap[g * p.k + t] = __builtin_nanf("");
        }
        if (tid == 0) {
            if (p.logdet) p.logdet[g] = __builtin_nan("");
            p.status[g] = 3;
        }
        return;
    }

    // ---- the targets' columns: square part by wave 0, then every row ------
    // members ascend, so column c (decreasing id) is member m - 1 - c
    if (tid < m) ord[tid] = m - 1 - tid;
    if (tid == 0) tmask_sh = m >= 64 ? ~0ull : ((1ull << m) - 1ull);
    __syncthreads();
    if (wave == 0) {
        // lane i: column-order row i (physical m - 1 - i); left-looking by columns
        const int pi = m - 1 - lane;
        for (int c = 0; c < m; ++c) {
            const int pc = m - 1 - c;
            double v = 0.0;
            if (lane >= c && lane < m) {
                v = part_cov<TWO_NU>(cpt[pi], cpt[pc], c_nu, s2) + (lane == c ? nug : 0.0);
                for (int c2 = 0; c2 < c; ++c2) v = fma(-Lsq[pi][m - 1 - c2], Lsq[pc][m - 1 - c2], v);
                if (lane == c) {
                    if (!(v > 0.0)) notpd_sh = 1;
                    Lsq[pc][pc] = v > 0.0 ? v * rsq64(v) : 1.0;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (lane > c && lane < m) Lsq[pi][pc] = v / Lsq[pc][pc];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    double L[kPartCols];
#pragma unroll
    for (int c = 0; c < kPartCols; ++c) L[c] = 0.0;
    int q = 0;  // number of columns with a larger id than mine (my insertion point)
    bool cand = tid < C;
    if (cand) {
#pragma unroll
        for (int c = 0; c < kPartMaxMembers; ++c) {
            if (c < m) {
                const int pc = m - 1 - c;
                double v = part_cov<TWO_NU>(xr, cpt[pc], c_nu, s2);
#pragma unroll
                for (int c2 = 0; c2 < c; ++c2) v = fma(-L[c2], Lsq[pc][m - 1 - c2], v);
                L[c] = v / Lsq[pc][pc];
                q += cid[pc] > my_id ? 1 : 0;
            }
        }
    }

    // ---- the picks ----------------------------------------------------------
    int ncol = m;
    int nsel = 0;
    int st = 0;
    for (int t = 0; t < kk; ++t) {
        if (notpd_sh) break;
        const uint64_t tmask = tmask_sh;
        // score (eq. obj_partial with eq. partial_induct)
        uint64_t key = 0ull;
        if (cand) {
            double v = prior, prod = 1.0;
#pragma unroll
            for (int c = 0; c < kPartCols; ++c) {
                if (c < ncol) {
                    const double l = L[c];
                    if (((tmask >> c) & 1ull) && c >= q) {
                        double f = 1.0 - l * l * rcp64(v);
                        f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
                        prod *= f;
                    }
                    v = fma(-l, l, v);
                }
            }
            double sc = 1.0 - prod;
            sc = sc < 0.0 ? 0.0 : (sc > 1.0 ? 1.0 : sc);
            if (v > thr) key = make_key(sc, tid);
        }
        // workgroup top-two
        Top2 loc = {key, 0ull};
        Top2 wt = wave_top2(loc);
        if (lane == 0) {
            wk1[wave] = wt.k1;
            wk2[wave] = wt.k2;
        }
        __syncthreads();
        Top2 best = {0ull, 0ull};
#pragma unroll
        for (int w = 0; w < kPartThreads / kWave; ++w) best = merge(best, Top2{wk1[w], wk2[w]});
        if (best.k1 == 0ull) {
            st = 1;
            break;
        }
        const int ws = key_slot(best.k1);
        if (tid == ws) {
            double v = prior;
#pragma unroll
            for (int c = 0; c < kPartCols; ++c) {
                if (c < q) {
                    bk[c] = L[c];
                    v = fma(-L[c], L[c], v);
                }
            }
            bx[0] = xr[0];
            bx[1] = xr[1];
            bx[2] = xr[2];
            bv = v;
            bid = my_id;
            bp = q;
            sel_sh[t] = my_id;
            const double sa = key_score(best.k1), sb = key_score(best.k2);
            gap_sh[t] = best.k2 == 0ull ? 1.0f : (sa == 0.0 ? 0.0f : (float)((sa - sb) / sa));
            cand = false;
        }
        __syncthreads();
        const int pk = bp;
        const int32_t idk = bid;
        const double vk = bv;
        const double inv = rsq64(vk);
        const double xk[3] = {bx[0], bx[1], bx[2]};
        const int ph = ncol;  // the pick's physical slot
        // the new column on my candidate row
        double u = 0.0;
        if (cand) {
            double acc = part_cov<TWO_NU>(xr, xk, c_nu, s2);
#pragma unroll
            for (int c = 0; c < kPartCols; ++c)
                if (c < pk) acc = fma(-L[c], bk[c], acc);
            u = acc * inv;
        }
        if (wave == 0) {
            // square part: lane i is column-order row i of the old order
            const bool mine = lane < ncol;
            const int pi = mine ? ord[lane] : 0;
            // lane l also keeps ord[l] (column c's slot comes by readlane)
            const int my_ord = mine ? pi : 0;
            double w = 0.0;
            if (mine && lane >= pk) {
                double acc = part_cov<TWO_NU>(cpt[pi], xk, c_nu, s2);
#pragma unroll 4
                for (int c = 0; c < pk; ++c) acc = fma(-Lsq[pi][ord[c]], bk[c], acc);
                w = acc * inv;
            }
            if (mine) Lsq[pi][ph] = w;
            // the pick's own row: its entries before it, its pivot
            for (int c = lane; c < pk; c += kWave) Lsq[ph][ord[c]] = bk[c];
            if (lane == 0) {
                Lsq[ph][ph] = vk * inv;
                cid[ph] = idk;
                cpt[ph][0] = xk[0];
                cpt[ph][1] = xk[1];
                cpt[ph][2] = xk[2];
            }
            // rank-one downdate of the columns after the pick by u: column
            // c's pivot is row c (lane c), whose diagonal and its inverse
            // are read before the loop; each lane's entry of the next column
            // is loaded one column ahead, off the chain through w
            const double dg = (mine && lane >= pk) ? Lsq[pi][pi] : 1.0;
            const double idg = rcp64_acc(dg);
            double cur = 0.0;
            if (pk < ncol && mine && lane > pk) cur = Lsq[pi][__builtin_amdgcn_readlane(my_ord, pk)];
            for (int c = pk; c < ncol; ++c) {
                const int pc = __builtin_amdgcn_readlane(my_ord, c);
                double nxt = 0.0;
                if (c + 1 < ncol && mine && lane > c + 1) nxt = Lsq[pi][__builtin_amdgcn_readlane(my_ord, c + 1)];
                const double lcc = bcast(dg, c), il = bcast(idg, c);
                const double wc = bcast(w, c);
                const double r2 = (lcc - wc) * (lcc + wc);
                if (!(r2 > 0.0)) {
                    if (lane == 0) notpd_sh = 1;
                    break;
                }
                const double rr = rsq64(r2);
                const double r = r2 * rr;
                const double cs = r * il, sn = wc * il;
                const double ics = lcc * rr;
                if (lane == 0) {
                    rot_sn[c] = sn;
                    rot_cs[c] = cs;
                    rot_ics[c] = ics;
                }
                if (mine && lane > c) {
                    const double lic = (cur - sn * w) * ics;
                    w = cs * w - sn * lic;
                    Lsq[pi][pc] = lic;
                }
                if (lane == c) {
                    Lsq[pc][pc] = r;
                    w = 0.0;
                }
                cur = nxt;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // the new column order: the pick after every larger id
            if (lane == 0) {
                for (int c = ncol; c > pk; --c) ord[c] = ord[c - 1];
                ord[pk] = ph;
                const uint64_t lo = pk == 0 ? 0ull : (tmask & ((1ull << pk) - 1ull));
                const uint64_t hi = pk + 1 >= 64 ? 0ull : ((tmask >> pk) << (pk + 1));
                tmask_sh = lo | hi;
            }
        }
        __syncthreads();
        if (notpd_sh) break;
        // my row: the same rotations on the columns after the pick, then u
        // enters at column pk
        if (cand) {
            double w = u;
#pragma unroll
            for (int c = 0; c < kPartCols; ++c) {
                if (c >= pk && c < ncol) {
                    const double cs = rot_cs[c], sn = rot_sn[c];
                    const double lc = (L[c] - sn * w) * rot_ics[c];
                    w = cs * w - sn * lc;
                    L[c] = lc;
                }
            }
            // columns pk .. ncol - 1 move up by one and u enters at pk: pk and
            // ncol are uniform, and the empty asm keeps each move behind a
            // scalar branch (only the moved columns cost vector instructions)
#pragma unroll
            for (int c = kPartCols - 1; c >= 1; --c) {
                if (c > pk && c <= ncol) {
                    asm volatile("");
                    L[c] = L[c - 1];
                }
            }
#pragma unroll
            for (int c = 0; c < kPartCols; ++c) {
                if (c == pk) {
                    asm volatile("");
                    L[c] = u;
                }
            }
            q += idk > my_id ? 1 : 0;
        }
        ++ncol;
        nsel = t + 1;
    }
    if (notpd_sh) st = 2;

    // ---- outputs --------------------------------------------------------------
    __syncthreads();
    for (int t = tid; t < p.k; t += kPartThreads) {
        p.sel[g * p.k + t] = t < nsel ? sel_sh[t] : -1;
        if (p.gap) p.gap[g * p.k + t] = t < nsel ? gap_sh[t] : __builtin_nanf("");
    }
    if (wave == 0) {
        // the group term: sum over the targets of log L_qq^2 (physical slots 0 .. m-1)
        double s = 0.0;
        if (lane < m) s = 2.0 * log(Lsq[lane][lane]);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) {
            if (p.logdet) p.logdet[g] = st == 2 ? __builtin_nan("") : s;
            p.status[g] = (uint8_t)st;
        }
    }
}

hipError_t launch_partial(const AggArgs& a, bool want_factor, hipStream_t s) {
    if (a.n_groups == 0) return hipSuccess;
    switch (a.two_nu) {
        case 1: hipLaunchKernelGGL(partial_select_kernel<1>, dim3((unsigned)a.n_groups), dim3(kPartThreads), 0, s, a); break;
        case 3: hipLaunchKernelGGL(partial_select_kernel<3>, dim3((unsigned)a.n_groups), dim3(kPartThreads), 0, s, a); break;
        case 5: hipLaunchKernelGGL(partial_select_kernel<5>, dim3((unsigned)a.n_groups), dim3(kPartThreads), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !want_factor) return e;
    return launch_agg_factor(a, s);
}

int partial_max_members() { return kPartMaxMembers; }
int partial_max_k() { return kPartMaxK; }
int partial_max_pool() { return kPartThreads; }

}  // namespace csel
