// select_kernel.hpp -- single-target greedy selection + KL-optimal factor column.
//
// Schedule: one wavefront per target column (4 columns per 256-thread block).
// The candidate pool (C <= 64*RPL) is spread over the 64 lanes, RPL rows per
// lane (pool slot j = rr*64 + lane).  Each lane keeps, for its rows:
//   - the coordinate offset from the target (FP32 or FP64),
//   - the tracked conditional variance and covariance with the target (FP64),
//   - its row of the partial Cholesky factor, L[rr][0..KMAX) (FP32 or FP64),
// all in VGPRs: the pick loop is fully unrolled so every index into L is static.
//
// One pick (Sec. 3.1, eq. cond_select / eq. obj_gp; App. C.1):
//   score = cov^2 / var (FP64) -> wave top-two via DPP -> the winner's factor
//   row, offset, var and cov are broadcast (LDS; FP64: var and cov by
//   readlane, the offset from a per-wave table of the pool) -> every lane
//   evaluates Theta(row, winner), subtracts the GEMV L[row] . L[winner] and
//   scales by 1/sqrt(var_winner) -> FP64 rank-one downdate of var and cov.
// The target's own factor row is never formed: its entry for pick t is
// cov_winner / sqrt(var_winner), the quantity eq. cond_select defines.
//
// Factor column (eq. L_col): rows 0..s-1 are the selected points and row s
// the target.  FP64: the picks' rows of the pivoted Cholesky that the loop
// builds, with the target's row (its ui and final variance), are the Cholesky
// factor G of Theta' = Theta over [selected..., target], and the column is
// G^{-T} e_last, one back-substitution (factor_from_pivots; pools up to 256).
// Mixed precision (FP32 rows) and FP64 pools above 256: Theta' is rebuilt in FP64 (its lower triangle spread over the
// lanes, staged in LDS) and factored as L D L^T, left-looking by columns,
// each row's dot products split over a lane pair; then Theta'^{-1} e_last =
// L^{-T} e_last / d_last and e_last^T Theta'^{-1} e_last = 1 / d_last, so the
// column is L^{-T} e_last / sqrt(d_last) (factor_column).
//
// Argmax keys: FP64, the FP64 score with the slot in its low mantissa bits.
// Mixed precision ranks by the FP32 score of the FP64 state, equal scores to
// the smallest slot: without the gap output as the maximum of the score's
// bits and ballots for the slot, with it as a top-two of 64-bit keys (score
// bits above, slot below), so both variants pick identically.

#pragma once

#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

// distance square root: the hardware v_sqrt_f32 (1 ulp) in FP32, dist64
// (about 1 ulp) in FP64
template <typename T>
__device__ __forceinline__ T tsqrt(T x) {
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_sqrtf(x);
    else return dist64(x);
}

template <typename T, int TWO_NU>
__device__ __forceinline__ T matern(T r, T c, T s2, const ExpConsts& K) {
    if constexpr (sizeof(T) == 4) return matern_f32<TWO_NU>(r, c, s2);
    else return matern_f64<TWO_NU>(r, c, s2, K);
}

// the FP64 exponential's constants: pinned in scalar registers for the FP64
// kernels (built once instead of at every unrolled use), literals otherwise
template <typename T>
__device__ __forceinline__ ExpConsts kernel_exp_consts() {
    if constexpr (sizeof(T) == 8) return exp_consts_sgpr();
    else return exp_consts();
}

constexpr int kSelWavesPerBlock = 4;

// Factor column (eq. L_col) of one column on its nsel selected points, by
// one wavefront: lane t holds pick t in my_sel (and its gap in my_gap).
// Theta' over [selected..., target] is built in FP64 in LDS (TH, PT: this
// wave's buffers) and factored as L D L^T on lane pairs; writes the column's
// sel, factor, log_condvar, gap and status outputs.
template <int TWO_NU, int KMAX>
__device__ __forceinline__ void factor_column(const SelectArgs& p, int64_t col, int lane, int nsel, int32_t my_sel,
                                              float my_gap, int32_t tgt, int st, double (&TH)[KMAX + 1][KMAX + 2],
                                              double (&PT)[KMAX + 1][4]) {
    const int kout = p.k;
    const int dim = p.dim;
    int32_t* sel_out = p.sel + col * kout;
    double* fac_out = p.fac + col * (kout + 1);
    const int M = nsel + 1;
    const int32_t my_id = lane < nsel ? my_sel : (lane == nsel ? tgt : -1);
    // the points of s (lane r: selected point r, lane nsel: the target) -> LDS
    if (lane < M) {
        const int64_t b = (int64_t)my_id * dim;
        PT[lane][0] = p.pts[b];
        PT[lane][1] = dim > 1 ? p.pts[b + 1] : 0.0;
        PT[lane][2] = dim > 2 ? p.pts[b + 2] : 0.0;
        PT[lane][3] = (double)my_id;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const double cnu64 = p.c_nu, s264 = p.s2, nug64 = p.nugget;
    // Theta' = L D L^T (L unit lower triangular), FP64.  Row r >= 1 of Theta'
    // belongs to the lane pair (r - 1, r - 1 + 32): the low lane holds the
    // row's even columns, the high lane its odd columns, so each dot product
    // is split over two lanes and joined by one cross-half swap.  Row r of the
    // LDS buffer TH keeps column c at slot pos(c) = (c & 1) * HALF + (c >> 1):
    // each half's columns contiguous and 16-byte aligned, the even half in
    // slots 0 .. KMAX/2, the diagonal in slot HALF - 1, the odd half in slots
    // HALF .. KMAX + 1.  The slot pos(r) of row r holds 0.
    constexpr int HALF = KMAX / 2 + 2;
    constexpr int DIAG = HALF - 1;
    static_assert(HALF + (KMAX - 1) / 2 <= KMAX + 1 && DIAG > KMAX / 2, "row layout");
    {
        const int ne = M * (M + 1) / 2;
        // entry e of the row-major lower triangle is (r, c) with r = floor(x),
        // x = (sqrt(8e + 1) - 1) / 2: for rows r <= 32, x lies in
        // [r, r + 1 - 2 / (2r + 3)], so x + 1e-3 truncates to r under a
        // square root within one ulp
        static_assert(KMAX <= 32, "triangle index bound");
        for (int e = lane; e < ne; e += kWave) {
            const int r = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f + 1e-3f);
            const int c = e - r * (r + 1) / 2;
            const double d0 = PT[r][0] - PT[c][0], d1 = PT[r][1] - PT[c][1], d2 = PT[r][2] - PT[c][2];
            const double s2d = d0 * d0 + d1 * d1 + d2 * d2;
            const double rr = s2d > 0.0 ? s2d * rsq64(s2d) : 0.0;
            const double th = matern_f64<TWO_NU>(rr, cnu64, s264) + (PT[r][3] == PT[c][3] ? nug64 : 0.0);
            if (c < r) {
                TH[r][(c & 1) * HALF + (c >> 1)] = th;
            } else {
                TH[r][DIAG] = th;
                TH[r][(r & 1) * HALF + (r >> 1)] = 0.0;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int hi = lane >> 5;
    const int my_row = (lane & 31) + 1;
    const bool row_ok = my_row < M;
    // h[q]: column 2q + hi of my row (Theta' until that column is done, then L).
    // Every lane loads a whole half row (lanes past the last row read row 0 and
    // never use it); the odd half has one column fewer, so its last register
    // repeats the slot before, keeping the read inside the row.
    double h[KMAX / 2 + 1];
    const double* my_th = &TH[row_ok ? my_row : 0][hi * HALF];
#pragma unroll
    for (int q = 0; q <= KMAX / 2; ++q) h[q] = my_th[q == KMAX / 2 ? q - hi : q];
    const double diag = TH[row_ok ? my_row : 0][DIAG];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // Left-looking by columns: with W[j][c] = d_c L[j][c] (row j of TH, written
    // as column c finished), every row r >= j needs v_r = Theta'[r][j] -
    // sum_{c<j} L[r][c] W[j][c]; then d_j = v_j and L[r][j] = v_r / d_j.  The
    // high lane's sum for odd j reads the zero slot pos(j) of row j as its last
    // term.  Entries of rows below j and lanes past the last row are never
    // read.
    bool pd = true;
    double dinv = 0.0;   // lane c: 1 / d_c
    double dlast = 0.0;  // d of the last row (the target's conditional variance)
#pragma unroll
    for (int j = 0; j <= KMAX; ++j) {
        if (j >= M || !pd) continue;
        double part = 0.0;
        const double* wj = &TH[j][hi * HALF];
#pragma unroll
        for (int q = 0; q < (j + 1) / 2; ++q) part = fma(h[q], wj[q], part);
        const double tot = pair_sum(part);
        const double dj = j == 0 ? TH[0][DIAG] : bcast(diag - tot, j - 1);
        if (!(dj > 0.0)) {
            pd = false;
            continue;
        }
        const double inv = rcp64_acc(dj);
        if (lane == j) dinv = inv;
        dlast = dj;
        if (hi == (j & 1) && my_row > j && row_ok) {
            const double v = h[j >> 1] - tot;
            h[j >> 1] = v * inv;
            TH[my_row][(j & 1) * HALF + (j >> 1)] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }

    double y = 0.0;
    if (pd) {
        // Theta'^{-1} e_last = L^{-T} e_last / d_last and e_last^T Theta'^{-1}
        // e_last = 1 / d_last, so the column is z / sqrt(d_last) with L^T z =
        // e_last: z_last = 1, z_c = -(1 / d_c) sum_{r>c} W[r][c] z_r, lane c
        // accumulating its sum from the rows left in TH.
        const int l = nsel;
        const int my_pos = lane <= KMAX ? (lane & 1) * HALF + (lane >> 1) : 0;
        double acc = 0.0;
#pragma unroll
        for (int c = KMAX; c >= 0; --c) {
            if (c > l) continue;
            const double zc = c == l ? 1.0 : bcast(-acc * dinv, c);
            if (lane < c) acc = fma(TH[c][my_pos], zc, acc);
        }
        // lane c's sum was complete at its own step and untouched after it
        const double z = lane == l ? 1.0 : (lane < l ? -acc * dinv : 0.0);
        y = z * rsq64(dlast);
        if (p.logcv && lane == 0) p.logcv[col] = log(dlast);
    } else {
        st = 2;
        y = __builtin_nan("");
        if (lane == 0 && p.logcv) p.logcv[col] = __builtin_nan("");
    }
    if (lane < kout) {
        sel_out[lane] = lane < nsel ? my_sel : -1;
        fac_out[1 + lane] = lane < nsel ? y : (pd ? 0.0 : __builtin_nan(""));
        if (p.gap) p.gap[col * kout + lane] = my_gap;
    }
    if (lane == nsel) fac_out[0] = y;
    if (lane == 0) p.status[col] = (uint8_t)st;
}

// Which kernels build the FP64 factor column from the picks' Cholesky rows
// (factor_from_pivots): those whose pool, rows_per_wave = W * RPL rows per
// lane over the column's waves, is at most 256 (4 rows per lane of one
// wave).  The 8-rows-per-lane FP64 kernel spills its partial factor to
// scratch, and in its variant without the gap output the reused rows gave
// columns 1e-2 away from the oracle's (picks and log conditional variances
// exact; the cause was not found), so pools above 256 rebuild Theta' from
// the points (factor_column) in both schedules, which keeps the one-wave
// and multi-wave schedules bit-identical for every pool width.
template <typename T>
__host__ __device__ constexpr bool reuse_pivots(int rows_per_wave) {
    return sizeof(T) == 8 && rows_per_wave <= 4;
}

// A target's final conditional variance at or below this fraction of the
// prior variance is zero within the rounding of its FP64 downdates (about
// k u prior for k picks): the selected block is then singular.
constexpr double kSingularFrac = 0x1p-46;

// Factor column (eq. L_col) of an FP64 selection from its own pivoted
// Cholesky rows.  The greedy loop is a pivoted left-looking Cholesky of the
// pool's covariance, so the Cholesky factor G of Theta' over [picks...,
// target] is already at hand: row t < nsel is the row of pick t when it
// was picked (its t partial-factor entries, kept in LDS row t of G, and
// sqrt(var_t), whose reciprocal lane t holds in my_isd), and the target row
// is (ui_0 .. ui_{nsel-1}, sqrt(vt)), with ui_t in lane t's my_ui and vt the
// target's final conditional variance.  Theta'^{-1} e_last / sqrt(e_last^T
// Theta'^{-1} e_last) = G^{-T} e_last, so the column is z with G^T z =
// e_last: z_last = 1 / sqrt(vt), then z_r = -(sum_{c>r} G[c][r] z_c) / G[r][r]
// for r = nsel-1 .. 0, lane r accumulating its own sum.
template <int KMAX>
__device__ __forceinline__ void factor_from_pivots(const SelectArgs& p, int64_t col, int lane, int nsel,
                                                   int32_t my_sel, float my_gap, int st, double vt, double prior,
                                                   double my_ui, double my_isd, const double (&G)[KMAX + 1][KMAX + 2]) {
    const int kout = p.k;
    int32_t* sel_out = p.sel + col * kout;
    double* fac_out = p.fac + col * (kout + 1);
    const bool pd = vt > kSingularFrac * prior;
    double y = __builtin_nan("");
    if (pd) {
        const double zl = rsq64(vt);
        double acc = lane < nsel ? my_ui * zl : 0.0;
        y = lane == nsel ? zl : 0.0;
#pragma unroll
        for (int r = KMAX - 1; r >= 0; --r) {
            if (r >= nsel) continue;
            // lane r's sum is complete: every row below r has been applied
            const double zr = bcast(-acc * my_isd, r);
            if (lane == r) y = zr;
            if (lane < r) acc = fma(G[r][lane], zr, acc);
        }
        if (p.logcv && lane == 0) p.logcv[col] = log(vt);
    } else {
        st = 2;
        if (lane == 0 && p.logcv) p.logcv[col] = __builtin_nan("");
    }
    if (lane < kout) {
        sel_out[lane] = lane < nsel ? my_sel : -1;
        fac_out[1 + lane] = lane < nsel ? y : (pd ? 0.0 : __builtin_nan(""));
        if (p.gap) p.gap[col * kout + lane] = my_gap;
    }
    if (lane == nsel) fac_out[0] = y;
    if (lane == 0) p.status[col] = (uint8_t)st;
}


// GAP: also track the second-best score of every step (top-two reduction) for
// the top2_gap output; without it the reduction is a plain maximum.
template <typename T, int TWO_NU, int RPL, int KMAX, bool GAP>
__global__ __launch_bounds__(256) void select_factor_kernel(SelectArgs p) {
    static_assert(KMAX + 1 <= kWave, "factor phase keeps one row of Theta_ss per lane");
    __shared__ __align__(16) double sh_r[kSelWavesPerBlock][KMAX + 1][KMAX + 2];
    __shared__ double sh_pt[kSelWavesPerBlock][KMAX + 1][4];  // points of s: x, y, z, id
    // FP64 pools of up to 4 rows per lane: every slot's offset and point id
    // (x, y, z, id), written once, so the winner's are read from one uniform
    // LDS address as soon as its slot is known
    constexpr bool kPxTable = sizeof(T) == 8 && RPL <= 4;
    __shared__ __align__(16) double sh_px[kSelWavesPerBlock][kPxTable ? RPL * kWave : 1][4];

    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    int64_t col = (int64_t)blockIdx.x * kSelWavesPerBlock + wib;
    if (p.col_list) {
        // the list's positions in eight contiguous segments, one per XCD
        // (blocks go to the XCDs round-robin; the launch rounds the grid up to
        // a multiple of 8), so the columns of a spatially sorted list that run
        // together on one XCD share its L2.  Segments follow the list's actual
        // length, so a short list still spreads over every XCD.
        const int64_t cnt = min((int64_t)*p.col_count, p.n_waves);
        const int64_t seg = ((cnt + 7) / 8 + kSelWavesPerBlock - 1) / kSelWavesPerBlock * kSelWavesPerBlock;
        const int64_t lb = (int64_t)(blockIdx.x >> 3) * kSelWavesPerBlock + wib;
        const int64_t pos = (int64_t)(blockIdx.x & 7u) * seg + lb;
        if (lb >= seg || pos >= cnt) return;
        col = p.col_list[pos];
    }
    if (col < 0 || col >= p.n_targets) return;
    const ExpConsts EK = kernel_exp_consts<T>();

    const int kout = p.k;
    int32_t* sel_out = p.sel + col * kout;
    double* fac_out = p.fac ? p.fac + col * (kout + 1) : nullptr;

    const int32_t tgt = __builtin_amdgcn_readfirstlane(p.targets[col]);
    const int32_t C = __builtin_amdgcn_readfirstlane(p.pool_len[col]);
    const int dim = p.dim;

    // ---- stage the pool ------------------------------------------------
    bool bad = tgt < 0 || (int64_t)tgt >= p.n || C < 0 || C > p.stride || C > RPL * kWave;
    double xi[3] = {0.0, 0.0, 0.0};
    T dx[RPL][3];
    double var[RPL], cov[RPL];
    int32_t pid[RPL];
    const T cnu = (T)p.c_nu, s2 = (T)p.s2;
    const double prior = p.s2 + p.nugget;
    const double thr = 1e-12 * prior;
    if (!bad) {
        for (int d = 0; d < dim; ++d) xi[d] = p.pts[(int64_t)tgt * dim + d];
    }
    bool bad_idx = false;
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
        const int j = rr * kWave + lane;
        pid[rr] = -1;
        dx[rr][0] = dx[rr][1] = dx[rr][2] = (T)0;
        var[rr] = 0.0;
        cov[rr] = 0.0;
        if (!bad && j < C) {
            const int32_t q = p.pool[col * p.stride + j];
            if (q < 0 || (int64_t)q >= p.n) {
                bad_idx = true;
            } else {
                pid[rr] = q;
                for (int d = 0; d < dim; ++d) dx[rr][d] = (T)(p.pts[(int64_t)q * dim + d] - xi[d]);
            }
        }
        const T r = tsqrt(sqnorm3(dx[rr][0], dx[rr][1], dx[rr][2]));
        cov[rr] = (double)matern<T, TWO_NU>(r, cnu, s2, EK);
        // var = -1 marks a slot that can never be picked (empty, or selected)
        var[rr] = pid[rr] >= 0 ? prior : -1.0;
    }
    bad = bad || __any(bad_idx);
    if constexpr (kPxTable) {
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            double2* e = reinterpret_cast<double2*>(&sh_px[wib][rr * kWave + lane][0]);
            e[0] = double2{(double)dx[rr][0], (double)dx[rr][1]};
            e[1] = double2{(double)dx[rr][2], (double)pid[rr]};
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (bad) {
        for (int r = lane; r < kout; r += kWave) {
            sel_out[r] = -1;
            if (fac_out) fac_out[1 + r] = __builtin_nan("");
            if (p.gap) p.gap[col * kout + r] = __builtin_nanf("");
            if (GAP && p.gain) p.gain[col * kout + r] = __builtin_nan("");
        }
        if (lane == 0) {
            if (fac_out) fac_out[0] = __builtin_nan("");
            if (p.logcv) p.logcv[col] = __builtin_nan("");
            p.status[col] = 3;
        }
        return;
    }

    // ---- greedy selection ------------------------------------------------
    const int kk = min(kout, C);
    const T nug = (T)p.nugget;
    T L[RPL][KMAX];
    int32_t my_sel = -1;
    float my_gap = __builtin_nanf("");
    // the target's tracked conditional variance; top-two variant: in lane t,
    // the fraction of it that pick t removes
    double vt = p.s2 + p.nugget;
    double my_gain = __builtin_nan("");
    // FP64: lane t keeps pick t's target-row entry ui_t and 1 / sqrt(var_t)
    double my_ui = 0.0, my_isd = 0.0;
    int nsel = 0;
    int st = 0;
    bool stopped = false;
#pragma unroll
    for (int t = 0; t < KMAX; ++t) {
        if (t < kk && !stopped) {
            Top2 w;
            if constexpr (GAP) {
                // FP64: keys of the FP64 score; mixed: keys of the FP32 score,
                // which rank as the variant without the gap does
                Top2 loc = {0ull, 0ull};
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    if (var[rr] > thr) {
                        if constexpr (sizeof(T) == 8)
                            insert(loc, make_key(cov[rr] * cov[rr] * rcp64(var[rr]), rr * kWave + lane));
                        else
                            insert(loc, mixed_key(mixed_score(cov[rr], var[rr]), rr * kWave + lane));
                    }
                }
                w = wave_top2(loc);
            } else if constexpr (sizeof(T) == 8) {
                uint64_t best = 0ull;
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    const double sc = cov[rr] * cov[rr] * rcp64(var[rr]);
                    const uint64_t key = var[rr] > thr ? make_key(sc, rr * kWave + lane) : 0ull;
                    best = key > best ? key : best;
                }
                w.k1 = wave_max64(best);
                w.k2 = 0ull;
            } else {
                // FP32 score of the FP64 state; key = its bits with the top bit
                // marking a valid candidate (scores are >= 0), 0 = none
                uint32_t key[RPL], best = 0u;
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    const float sc = mixed_score(cov[rr], var[rr]);
                    key[rr] = var[rr] > thr ? (__float_as_uint(sc) | 0x80000000u) : 0u;
                    best = max(best, key[rr]);
                }
                best = wave_max32(best);
                // the smallest slot holding the maximum
                int slot = -1;
#pragma unroll
                for (int rr = RPL - 1; rr >= 0; --rr) {
                    const uint64_t m = __ballot(key[rr] == best);
                    if (m) slot = rr * kWave + (int)__builtin_ctzll(m);
                }
                w.k1 = best == 0u ? 0ull : make_key(0.0, slot);
                w.k2 = 0ull;
            }
            if (w.k1 == 0ull) {
                st = 1;
                stopped = true;
            } else {
                constexpr bool kMixedKeys = GAP && sizeof(T) == 4;
                const int slot = kMixedKeys ? mixed_key_slot(w.k1) : key_slot(w.k1);
                const int rs = slot >> 6;
                const int ls = slot & (kWave - 1);
                const double sa = kMixedKeys ? (double)mixed_key_score(w.k1) : key_score(w.k1);
                const double sb = kMixedKeys ? (double)mixed_key_score(w.k2) : key_score(w.k2);
                const float g = (w.k2 == 0ull) ? 1.0f : (sa == 0.0 ? 0.0f : (float)((sa - sb) / sa));

                // broadcast the winner's row through LDS (the factor-phase
                // buffer is free during the picks): the winning lane stores
                // its factor row, offset, var, cov and index; every lane reads
                // them back as broadcasts.  In FP64 the row goes to row t of
                // the buffer and stays there: rows 0 .. nsel-1 are the
                // Cholesky rows of the picks that the factor column reuses.
                T* bc;
                T* bdx;
                double* bcd = &sh_r[wib][KMAX][0];
                if constexpr (sizeof(T) == 8) {
                    bc = reinterpret_cast<T*>(&sh_r[wib][t][0]);
                    bdx = reinterpret_cast<T*>(bcd + 3);
                } else {
                    bc = reinterpret_cast<T*>(&sh_r[wib][0][0]);
                    bdx = bc + KMAX;
                }
                T dk0, dk1, dk2;
                double vk, ck;
                int32_t idk;
                if constexpr (sizeof(T) == 8) {
                    // FP64: the row through LDS (the GEMV reads it after the
                    // evaluation); var and cov by readlane from the winning
                    // lane, off the LDS round trip; the offset and id from the
                    // pool table (pools of up to 4 rows per lane), else by
                    // readlane as well
                    if (lane == ls) {
#pragma unroll
                        for (int rr = 0; rr < RPL; ++rr) {
                            if (rr == rs) {
#pragma unroll
                                for (int q = 0; q < t; ++q) bc[q] = L[rr][q];
                            }
                        }
                    }
                    double wv = 0.0, wc = 0.0, w0 = 0.0, w1 = 0.0, w2 = 0.0;
                    int32_t wp = -1;
#pragma unroll
                    for (int rr = 0; rr < RPL; ++rr) {
                        if (rr == rs) {
                            wv = var[rr];
                            wc = cov[rr];
                            if constexpr (!kPxTable) {
                                w0 = dx[rr][0];
                                w1 = dx[rr][1];
                                w2 = dx[rr][2];
                                wp = pid[rr];
                            }
                        }
                    }
                    vk = bcast(wv, ls);
                    ck = bcast(wc, ls);
                    if constexpr (kPxTable) {
                        const double2* px = reinterpret_cast<const double2*>(&sh_px[wib][slot][0]);
                        const double2 a = px[0], b = px[1];
                        dk0 = a.x;
                        dk1 = a.y;
                        dk2 = b.x;
                        idk = (int32_t)b.y;
                    } else {
                        dk0 = bcast(w0, ls);
                        dk1 = bcast(w1, ls);
                        dk2 = bcast(w2, ls);
                        idk = bcast(wp, ls);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                } else {
                    if (lane == ls) {
#pragma unroll
                        for (int rr = 0; rr < RPL; ++rr) {
                            if (rr == rs) {
#pragma unroll
                                for (int q = 0; q < t; ++q) bc[q] = L[rr][q];
                                bdx[0] = dx[rr][0];
                                bdx[1] = dx[rr][1];
                                bdx[2] = dx[rr][2];
                                bcd[0] = var[rr];
                                bcd[1] = cov[rr];
                                bcd[2] = (double)pid[rr];
                            }
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    dk0 = bdx[0];
                    dk1 = bdx[1];
                    dk2 = bdx[2];
                    vk = bcd[0];
                    ck = bcd[1];
                    idk = (int32_t)bcd[2];
                }
                const double inv_sd = rsq64(vk);
                const double ui = ck * inv_sd;
                const T inv_sd_t = (T)inv_sd;
                T acc[RPL];
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    const T e0 = dx[rr][0] - dk0, e1 = dx[rr][1] - dk1, e2 = dx[rr][2] - dk2;
                    const T r = tsqrt(sqnorm3(e0, e1, e2));
                    acc[rr] = matern<T, TWO_NU>(r, cnu, s2, EK);
                    if (pid[rr] == idk) acc[rr] += nug;
                }
                // GEMV with the broadcast row, one LDS element at a time for all rows
#pragma unroll
                for (int q = 0; q < t; ++q) {
                    const T lk = bc[q];
#pragma unroll
                    for (int rr = 0; rr < RPL; ++rr) acc[rr] = fma(-L[rr][q], lk, acc[rr]);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    const T u = acc[rr] * inv_sd_t;
                    L[rr][t] = u;
                    const double ud = (double)u;
                    var[rr] = fma(-ud, ud, var[rr]);
                    cov[rr] = fma(-ud, ui, cov[rr]);
                }
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr)
                    if (rr == rs && lane == ls) var[rr] = -1.0;
                if constexpr (GAP) {
                    // the pick's score is ck^2 / vk = ui^2 (eq. obj_gp); over
                    // the target's variance it is eq. global_obj's key
                    if (lane == t) my_gain = ui * ui / vt;
                }
                vt = fma(-ui, ui, vt);
                if (lane == t) {
                    my_sel = idk;
                    my_gap = g;
                    my_ui = ui;
                    my_isd = inv_sd;
                }
                nsel = t + 1;
            }
        }
    }

    if constexpr (GAP) {
        if (p.gain && lane < kout) p.gain[col * kout + lane] = lane < nsel ? my_gain : __builtin_nan("");
    }
    if (!p.fac) {
        // selection only: the picks, their gaps and the status
        if (lane < kout) {
            p.sel[col * kout + lane] = lane < nsel ? my_sel : -1;
            if (p.gap) p.gap[col * kout + lane] = my_gap;
        }
        if (lane == 0) p.status[col] = (uint8_t)st;
        return;
    }
    if constexpr (reuse_pivots<T>(RPL))
        factor_from_pivots<KMAX>(p, col, lane, nsel, my_sel, my_gap, st, vt, prior, my_ui, my_isd, sh_r[wib]);
    else
        factor_column<TWO_NU, KMAX>(p, col, lane, nsel, my_sel, my_gap, tgt, st, sh_r[wib], sh_pt[wib]);
}

template <typename T, int TWO_NU, int RPL, int KMAX, bool GAP>
static hipError_t launch_one(const SelectArgs& a, hipStream_t s) {
    int64_t blocks = (a.n_waves + kSelWavesPerBlock - 1) / kSelWavesPerBlock;
    if (a.col_list) {  // eight segments of whole blocks
        const int64_t seg = ((a.n_waves + 7) / 8 + kSelWavesPerBlock - 1) / kSelWavesPerBlock;
        blocks = 8 * seg;
    }
    hipLaunchKernelGGL((select_factor_kernel<T, TWO_NU, RPL, KMAX, GAP>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// one pool width (RPL pool entries per lane) at either pick capacity
template <typename T, int TWO_NU, int RPL, bool GAP>
static hipError_t launch_rpl_impl(const SelectArgs& a, int kmax, hipStream_t s) {
    if (kmax == 16) return launch_one<T, TWO_NU, RPL, 16, GAP>(a, s);
    if (kmax == 32) return launch_one<T, TWO_NU, RPL, 32, GAP>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace csel
