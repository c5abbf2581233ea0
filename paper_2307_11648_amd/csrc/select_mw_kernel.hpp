// select_mw_kernel.hpp -- the single-target selection with a column's pool
// split over W wavefronts of one workgroup (the multi-wave tile schedule).
//
// The one-wave schedule (select_kernel.hpp) keeps a column's whole pool in
// one wavefront's registers: RPL rows per lane and, per row, the partial
// Cholesky factor row L[rr][0..KMAX).  For FP64 on pools of 128 that is 226
// VGPRs (two waves per SIMD), and on pools of 512 more than a wave can hold
// (scratch spills, one wave per SIMD).  Here W wavefronts share a column:
// wave w owns pool slots (w*RPL + rr)*64 + lane, so each wave holds RPL rows
// per lane and the registers per wave fall W-fold.  One pick (Sec. 3.1, eq.
// cond_select / eq. obj_gp; App. C.1):
//   every wave: its best key (DPP) -> LDS; workgroup barrier;
//   every wave: the column's best of the W keys; the owner's winning lane
//     writes the winner's factor row, offset, var, cov and id to LDS;
//     workgroup barrier;
//   every wave: Theta(row, winner), the GEMV with the winner's row and the
//     FP64 rank-one downdate of its own rows.
// The keys are those of the one-wave kernel (the FP64 score with the slot in
// its low mantissa bits; in mixed precision the FP32 score, equal scores to
// the smallest slot), and each row's arithmetic is the same, so both
// schedules select and compute identically.  The workgroup holds 4/W
// columns; its barriers are executed at every pick step by every wave (a
// column that has stopped, or a slot without a column, passes them idle), so
// columns of different lengths share a workgroup safely.  After the picks,
// wave 0 of each column builds the factor column exactly as the one-wave
// kernel does (FP64 pools up to 256: from the picks' Cholesky rows,
// factor_from_pivots; otherwise factor_column).  No top-two gap output.

#pragma once

#include "select_kernel.hpp"

namespace csel {

template <typename T, int TWO_NU, int RPL, int KMAX, int W>
__global__ __launch_bounds__(256) void select_factor_mw_kernel(SelectArgs p) {
    static_assert(KMAX + 1 <= kWave, "factor phase keeps one row of Theta_ss per lane");
    static_assert(kSelWavesPerBlock % W == 0, "whole columns per workgroup");
    constexpr int CPB = kSelWavesPerBlock / W;  // columns per workgroup
    constexpr int POOL = W * RPL * kWave;       // largest pool
    static_assert(POOL <= kSlotMax, "slots fit the key");
    __shared__ __align__(16) double sh_r[CPB][KMAX + 1][KMAX + 2];
    __shared__ double sh_pt[CPB][KMAX + 1][4];
    __shared__ uint64_t sh_key[CPB][W];
    __shared__ int sh_bad[CPB][W];

    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int cib = wib / W;  // this wave's column within the workgroup
    const int w = wib % W;    // its share of the column's pool

    // the column of each of the workgroup's CPB slots (the same in every wave)
    auto column_of = [&](int c) -> int64_t {
        if (!p.col_list) {
            const int64_t v = (int64_t)blockIdx.x * CPB + c;
            return v < p.n_targets ? v : -1;
        }
        // the list's positions in eight contiguous segments, one per XCD (as
        // in the one-wave kernel, in units of whole workgroups)
        const int64_t cnt = min((int64_t)*p.col_count, p.n_waves);
        const int64_t seg = ((cnt + 7) / 8 + CPB - 1) / CPB * CPB;
        const int64_t lb = (int64_t)(blockIdx.x >> 3) * CPB + c;
        const int64_t pos = (int64_t)(blockIdx.x & 7u) * seg + lb;
        if (lb >= seg || pos >= cnt) return -1;
        const int64_t v = p.col_list[pos];
        return v >= 0 && v < p.n_targets ? v : -1;
    };
    bool any_col = false;
#pragma unroll
    for (int c = 0; c < CPB; ++c) any_col = any_col || column_of(c) >= 0;
    // a workgroup without any column leaves at once (the condition is the same
    // in all its waves, so no barrier is left waiting); one with at least one
    // column keeps every wave for the barriers
    if (!any_col) return;
    const ExpConsts EK = kernel_exp_consts<T>();
    const int64_t col = column_of(cib);
    const bool has_col = col >= 0;

    const int kout = p.k;
    const int32_t tgt = has_col ? __builtin_amdgcn_readfirstlane(p.targets[col]) : -1;
    const int32_t C = has_col ? __builtin_amdgcn_readfirstlane(p.pool_len[col]) : 0;
    const int dim = p.dim;

    // ---- stage my rows --------------------------------------------------
    bool bad = has_col && (tgt < 0 || (int64_t)tgt >= p.n || C < 0 || C > p.stride || C > POOL);
    double xi[3] = {0.0, 0.0, 0.0};
    T dx[RPL][3];
    double var[RPL], cov[RPL];
    int32_t pid[RPL];
    const T cnu = (T)p.c_nu, s2 = (T)p.s2;
    const double prior = p.s2 + p.nugget;
    const double thr = 1e-12 * prior;
    if (has_col && !bad) {
        for (int d = 0; d < dim; ++d) xi[d] = p.pts[(int64_t)tgt * dim + d];
    }
    bool bad_idx = false;
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
        const int j = (w * RPL + rr) * kWave + lane;
        pid[rr] = -1;
        dx[rr][0] = dx[rr][1] = dx[rr][2] = (T)0;
        if (has_col && !bad && j < C) {
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
    const bool my_bad = __any(bad_idx);
    if (lane == 0) sh_bad[cib][w] = my_bad ? 1 : 0;
    __syncthreads();
#pragma unroll
    for (int v = 0; v < W; ++v) bad = bad || (sh_bad[cib][v] != 0);

    // ---- greedy selection (every wave passes every pick's barriers) -------
    const int kk = (has_col && !bad) ? min(kout, C) : 0;
    const T nug = (T)p.nugget;
    T L[RPL][KMAX];
    int32_t my_sel = -1;
    int nsel = 0;
    int st = 0;
    bool stopped = false;
    // FP64: the target's tracked conditional variance, and in lane t pick t's
    // target-row entry ui_t and 1 / sqrt(var_t) (the factor column reuses the
    // picks' Cholesky rows, as in the one-wave kernel)
    double vt = prior, my_ui = 0.0, my_isd = 0.0;
    // the winner's factor row (FP64: row t of the buffer, kept), its offset,
    // var, cov and id
    double* bcd = &sh_r[cib][KMAX][0];
    T* bdx = sizeof(T) == 8 ? reinterpret_cast<T*>(bcd + 3) : reinterpret_cast<T*>(&sh_r[cib][0][0]) + KMAX;
#pragma unroll
    for (int t = 0; t < KMAX; ++t) {
        const bool active = t < kk && !stopped;  // the same in the column's W waves
        T* bc = reinterpret_cast<T*>(&sh_r[cib][sizeof(T) == 8 ? t : 0][0]);
        // this wave's best key: larger score first, then the smaller slot
        uint64_t lk = 0ull;
        if (active) {
            if constexpr (sizeof(T) == 8) {
                uint64_t best = 0ull;
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    const double sc = cov[rr] * cov[rr] * rcp64(var[rr]);
                    const uint64_t key = var[rr] > thr ? make_key(sc, (w * RPL + rr) * kWave + lane) : 0ull;
                    best = key > best ? key : best;
                }
                lk = wave_max64(best);
            } else {
                uint32_t key[RPL], best = 0u;
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    const float sc = mixed_score(cov[rr], var[rr]);
                    key[rr] = var[rr] > thr ? (__float_as_uint(sc) | 0x80000000u) : 0u;
                    best = max(best, key[rr]);
                }
                best = wave_max32(best);
                int slot = 0;
#pragma unroll
                for (int rr = RPL - 1; rr >= 0; --rr) {
                    const uint64_t m = __ballot(key[rr] == best);
                    if (m) slot = (w * RPL + rr) * kWave + (int)__builtin_ctzll(m);
                }
                // score bits above, the complement of the slot below
                lk = best == 0u ? 0ull : (((uint64_t)best << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)slot));
            }
        }
        if (lane == 0) sh_key[cib][w] = lk;
        __syncthreads();
        uint64_t gk = 0ull;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            const uint64_t o = sh_key[cib][v];
            gk = o > gk ? o : gk;
        }
        int slot = 0;
        if (active) {
            if (gk == 0ull) {
                st = 1;
                stopped = true;
            } else {
                if constexpr (sizeof(T) == 8) slot = key_slot(gk);
                else slot = (int)(0xFFFFFFFFu - (uint32_t)gk);
                const int wo = slot / (RPL * kWave);
                const int rs = (slot / kWave) % RPL;
                const int ls = slot & (kWave - 1);
                // the owner's winning lane broadcasts the winner's row
                if (w == wo && lane == ls) {
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
            }
        }
        __syncthreads();
        if (active && gk != 0ull) {
            const T dk0 = bdx[0], dk1 = bdx[1], dk2 = bdx[2];
            const double vk = bcd[0], ck = bcd[1];
            const int32_t idk = (int32_t)bcd[2];
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
                const T lk2 = bc[q];
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) acc[rr] = fma(-L[rr][q], lk2, acc[rr]);
            }
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
                const T u = acc[rr] * inv_sd_t;
                L[rr][t] = u;
                const double ud = (double)u;
                var[rr] = fma(-ud, ud, var[rr]);
                cov[rr] = fma(-ud, ui, cov[rr]);
            }
            const int wo = slot / (RPL * kWave);
            const int rs = (slot / kWave) % RPL;
            const int ls = slot & (kWave - 1);
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr)
                if (w == wo && rr == rs && lane == ls) var[rr] = -1.0;
            vt = fma(-ui, ui, vt);
            if (lane == t) {
                my_sel = idk;
                my_ui = ui;
                my_isd = inv_sd;
            }
            nsel = t + 1;
        }
    }
    // every wave is past its reads of the last pick's broadcast before wave
    // 0 reuses the buffer for the factor column
    __syncthreads();
    if (!has_col || w != 0) return;
    if (bad) {
        int32_t* sel_out = p.sel + col * kout;
        double* fac_out = p.fac ? p.fac + col * (kout + 1) : nullptr;
        for (int r = lane; r < kout; r += kWave) {
            sel_out[r] = -1;
            if (fac_out) fac_out[1 + r] = __builtin_nan("");
        }
        if (lane == 0) {
            if (fac_out) fac_out[0] = __builtin_nan("");
            if (p.logcv) p.logcv[col] = __builtin_nan("");
            p.status[col] = 3;
        }
        return;
    }
    if (!p.fac) {
        // selection only: the picks and the status
        if (lane < kout) p.sel[col * kout + lane] = lane < nsel ? my_sel : -1;
        if (lane == 0) p.status[col] = (uint8_t)st;
        return;
    }
    if constexpr (reuse_pivots<T>(W * RPL))
        factor_from_pivots<KMAX>(p, col, lane, nsel, my_sel, __builtin_nanf(""), st, vt, prior, my_ui, my_isd,
                                 sh_r[cib]);
    else
        factor_column<TWO_NU, KMAX>(p, col, lane, nsel, my_sel, __builtin_nanf(""), tgt, st, sh_r[cib], sh_pt[cib]);
}

template <typename T, int TWO_NU, int RPL, int KMAX, int W>
static hipError_t launch_mw_one(const SelectArgs& a, hipStream_t s) {
    constexpr int CPB = kSelWavesPerBlock / W;
    int64_t blocks = (a.n_waves + CPB - 1) / CPB;
    if (a.col_list) {  // eight segments of whole workgroups
        const int64_t seg = ((a.n_waves + 7) / 8 + CPB - 1) / CPB;
        blocks = 8 * seg;
    }
    hipLaunchKernelGGL((select_factor_mw_kernel<T, TWO_NU, RPL, KMAX, W>), dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T, int TWO_NU, int RPL, int W>
static hipError_t launch_mw_impl(const SelectArgs& a, int kmax, hipStream_t s) {
    if (kmax == 16) return launch_mw_one<T, TWO_NU, RPL, 16, W>(a, s);
    if (kmax == 32) return launch_mw_one<T, TWO_NU, RPL, 32, W>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace csel
