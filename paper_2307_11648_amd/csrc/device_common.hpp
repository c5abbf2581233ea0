// device_common.hpp -- wave-level building blocks shared by the CDNA4 kernels.
//
// Everything here is written for wave64 (gfx950): lane masks, DPP controls and
// readlane broadcasts assume 64 lanes per wavefront.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csel {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// ---------------------------------------------------------------------------
// uniform broadcasts (the source lane index must be wave-uniform)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ int32_t bcast(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
// broadcast from a lane that differs between lanes (ds_bpermute)
__device__ __forceinline__ int32_t bcast_dyn(int32_t v, int src_lane) { return __shfl(v, src_lane, 64); }
__device__ __forceinline__ double bcast(double v, int lane) {
    int64_t b = __double_as_longlong(v);
    int32_t lo = __builtin_amdgcn_readlane((int32_t)(b & 0xffffffff), lane);
    int32_t hi = __builtin_amdgcn_readlane((int32_t)(b >> 32), lane);
    return __longlong_as_double(((int64_t)(uint32_t)lo) | ((int64_t)hi << 32));
}
__device__ __forceinline__ uint64_t bcast(uint64_t v, int lane) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)v, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// DPP moves within rows of 16 lanes (all source lanes valid for these controls)
// ---------------------------------------------------------------------------
constexpr int kDppQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kDppRowRor4 = 0x124;  // row_ror:4
constexpr int kDppRowRor8 = 0x128;  // row_ror:8
// gfx9-family broadcasts across rows (rows not in the row mask keep `old`)
constexpr int kDppRowBcast15 = 0x142;  // row r + 1 reads lane 15 of row r
constexpr int kDppRowBcast31 = 0x143;  // rows 2 and 3 read lane 31

template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)(uint32_t)v, CTRL, 0xF, 0xF, false);
    uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// Top-two of distinct 64-bit keys; 0 means "no candidate".
struct Top2 {
    uint64_t k1, k2;
};

__device__ __forceinline__ Top2 merge(Top2 a, Top2 b) {
    Top2 r;
    r.k1 = a.k1 > b.k1 ? a.k1 : b.k1;
    uint64_t lo = a.k1 > b.k1 ? b.k1 : a.k1;
    uint64_t s = a.k2 > b.k2 ? a.k2 : b.k2;
    r.k2 = lo > s ? lo : s;
    return r;
}

__device__ __forceinline__ void insert(Top2 &a, uint64_t key) {
    if (key > a.k1) {
        a.k2 = a.k1;
        a.k1 = key;
    } else if (key > a.k2) {
        a.k2 = key;
    }
}

// Wave-wide top-two over disjoint per-lane sets; the result is uniform.
// Inside each row of 16 lanes: two quad butterflies and two row rotations
// (every step merges disjoint sets); across the four rows: readlane.
__device__ __forceinline__ Top2 wave_top2(Top2 v) {
    Top2 o;
    o.k1 = dpp64<kDppQuadXor1>(v.k1); o.k2 = dpp64<kDppQuadXor1>(v.k2); v = merge(v, o);
    o.k1 = dpp64<kDppQuadXor2>(v.k1); o.k2 = dpp64<kDppQuadXor2>(v.k2); v = merge(v, o);
    o.k1 = dpp64<kDppRowRor4>(v.k1); o.k2 = dpp64<kDppRowRor4>(v.k2); v = merge(v, o);
    o.k1 = dpp64<kDppRowRor8>(v.k1); o.k2 = dpp64<kDppRowRor8>(v.k2); v = merge(v, o);
    Top2 r0 = {bcast(v.k1, 0), bcast(v.k2, 0)};
    Top2 r1 = {bcast(v.k1, 16), bcast(v.k2, 16)};
    Top2 r2 = {bcast(v.k1, 32), bcast(v.k2, 32)};
    Top2 r3 = {bcast(v.k1, 48), bcast(v.k2, 48)};
    return merge(merge(r0, r1), merge(r2, r3));
}

// Wave-wide max of a 32-bit key (uniform result): DPP inside each row of 16
// lanes, then DPP broadcasts across rows -- rows 1 and 3 take the last lane of
// the row before, rows 2 and 3 take lane 31 -- so lane 63 holds the maximum.
// Rows outside a broadcast's row mask see 0, the identity of the maximum.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t wave_max32(uint32_t v) {
    v = max(v, dpp32<kDppQuadXor1>(v));
    v = max(v, dpp32<kDppQuadXor2>(v));
    v = max(v, dpp32<kDppRowRor4>(v));
    v = max(v, dpp32<kDppRowRor8>(v));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast15, 0xA, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast31, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Wave-wide sum of a float (uniform result): the DPP steps of wave_max32
// leave each row's sum of 16 lanes in every lane of the row; the four row
// sums are then added in a fixed order.  No lane-address registers (as a
// shuffle through ds_bpermute needs) and no LDS traffic.
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_sum_f32(float v) {
    v += dppf<kDppQuadXor1>(v);
    v += dppf<kDppQuadXor2>(v);
    v += dppf<kDppRowRor4>(v);
    v += dppf<kDppRowRor8>(v);
    return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}

// Wave-wide max of a 64-bit key (uniform result): the steps of wave_max32 on
// both 32-bit halves (rows outside a broadcast's row mask read 0, the
// identity of the maximum), then lane 63's value.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp64_rows(uint64_t v) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)(uint32_t)v, CTRL, ROWS, 0xF, false);
    uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)(uint32_t)(v >> 32), CTRL, ROWS, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_max64(uint64_t v) {
    uint64_t o;
    o = dpp64<kDppQuadXor1>(v); v = v > o ? v : o;
    o = dpp64<kDppQuadXor2>(v); v = v > o ? v : o;
    o = dpp64<kDppRowRor4>(v); v = v > o ? v : o;
    o = dpp64<kDppRowRor8>(v); v = v > o ? v : o;
    o = dpp64_rows<kDppRowBcast15, 0xA>(v); v = v > o ? v : o;
    o = dpp64_rows<kDppRowBcast31, 0xC>(v); v = v > o ? v : o;
    return bcast(v, 63);
}

// ---------------------------------------------------------------------------
// Selection keys: a non-negative FP64 score with its low kSlotBits mantissa
// bits replaced by (kSlotMax - slot).  Larger key = larger score, then
// smaller slot.  Any eligible candidate has key >= 1; 0 = none.  The score
// must be >= 0 (+0.0): the bits of a negative double compare as huge keys.
// ---------------------------------------------------------------------------
constexpr int kSlotBits = 13;
constexpr uint64_t kSlotMask = (1ull << kSlotBits) - 1;
constexpr int kSlotMax = (1 << kSlotBits) - 1;  // slots 0 .. kSlotMax-1

__device__ __forceinline__ uint64_t make_key(double score, int slot) {
    uint64_t b = (uint64_t)__double_as_longlong(score);
    return (b & ~kSlotMask) | (uint64_t)(kSlotMax - slot);
}
__device__ __forceinline__ int key_slot(uint64_t key) { return kSlotMax - (int)(key & kSlotMask); }
__device__ __forceinline__ double key_score(uint64_t key) {
    return __longlong_as_double((long long)(key & ~kSlotMask));
}

// Mixed-precision selection keys: the FP32 score cov^2 / var of the FP64
// state, its bits above (the top bit set: a valid candidate; scores are
// >= 0) and the complement of the slot below, so a larger key is a larger
// FP32 score, then a smaller slot; 0 = none.  The plain-maximum and the
// top-two reductions rank candidates identically with these keys.
__device__ __forceinline__ float mixed_score(double cov, double var) {
    const float cf = (float)cov;
    return cf * cf * __builtin_amdgcn_rcpf((float)var);
}
__device__ __forceinline__ uint64_t mixed_key(float score, int slot) {
    return ((uint64_t)(__float_as_uint(score) | 0x80000000u) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)slot);
}
__device__ __forceinline__ int mixed_key_slot(uint64_t key) { return (int)(0xFFFFFFFFu - (uint32_t)key); }
__device__ __forceinline__ float mixed_key_score(uint64_t key) {
    return __uint_as_float((uint32_t)(key >> 32) & 0x7FFFFFFFu);
}

// 1/v in FP64: hardware reciprocal refined by one Newton step (about 1 ulp)
__device__ __forceinline__ double rcp64(double v) {
    const double r = __builtin_amdgcn_rcp(v);
    return r * fma(-v, r, 2.0);
}

// 1/v in FP64 (v > 0 normal): hardware reciprocal refined by two Newton
// steps r <- r + r (1 - v r) (about 1 ulp)
__device__ __forceinline__ double rcp64_acc(double v) {
    double r = __builtin_amdgcn_rcp(v);
#pragma unroll
    for (int it = 0; it < 2; ++it) r = fma(r, fma(-v, r, 1.0), r);
    return r;
}

// x of lane i plus x of lane i ^ 32, the same bits in both lanes of the pair
// (gfx950's cross-half swap, once per 32-bit word; the two operands are added
// in either order, which rounds identically)
__device__ __forceinline__ double pair_sum(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    const double a0 = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
    const double a1 = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
    return a0 + a1;
}

// 1/sqrt(v) in FP64 (v > 0 normal): hardware reciprocal square root refined
// by two Newton steps r <- r + r/2 (1 - v r^2) (about 1 ulp)
__device__ __forceinline__ double rsq64(double v) {
    double r = __builtin_amdgcn_rsq(v);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-(v * r), r, 1.0);
        r = fma(0.5 * r, e, r);
    }
    return r;
}

// ---------------------------------------------------------------------------
// Matern kernels (half-integer smoothness).  `c` = sqrt(2 nu) / length_scale.
// ---------------------------------------------------------------------------
// (the polynomial factor with explicit fused multiply-adds, as in matern_f64)
template <int TWO_NU>
__device__ __forceinline__ float matern_f32(float r, float c, float s2) {
    const float a = c * r;
    const float e = __expf(-a);
    if constexpr (TWO_NU == 1) return s2 * e;
    if constexpr (TWO_NU == 3) return s2 * fmaf(c, r, 1.0f) * e;
    return s2 * fmaf(a, fmaf(a, 1.0f / 3.0f, 1.0f), 1.0f) * e;
}

// e^{-a} for finite a >= 0 in FP64, about 2 ulp: Cody-Waite reduction
// -a = k ln2 + r with k = rint(-a / ln2) and ln2 split into a 32-bit head
// (k * head exact for |k| < 2^21) and its tail, |r| <= ln2/2; then the
// degree-12 Taylor polynomial of e^r (truncation below 2.3e-16 relative) in
// Horner form, scaled by 2^k.  For a past ~745 the scaling underflows to 0.
// The argument is never infinite or NaN here, so the special-value checks of
// a general exp are left out.
//
// Its 64-bit constants (and the Matern 5/2 polynomial's 1/3) travel in an
// ExpConsts.  A kernel that evaluates the covariance in a fully unrolled pick
// loop builds them once with exp_consts_sgpr(), which pins each in a pair of
// scalar registers for the whole kernel; written as literals, each use would
// re-create its constant with two scalar moves (a thousand per column in the
// FP64 kept-pool selection).  The arithmetic is the same either way.
struct ExpConsts {
    double inv_ln2, ln2_hi, ln2_lo, third;
    double q[11];  // 1/12!, 1/11!, ..., 1/2! (the last two Horner steps add 1)
};

__device__ __forceinline__ ExpConsts exp_consts() {
    ExpConsts K;
    K.inv_ln2 = 1.4426950408889634;
    K.ln2_hi = 0x1.62e42ff000000p-1;
    K.ln2_lo = -0x1.718432a1b0e26p-35;
    K.third = 1.0 / 3.0;
    K.q[0] = 2.08767569878681e-09;
    K.q[1] = 2.505210838544172e-08;
    K.q[2] = 2.755731922398589e-07;
    K.q[3] = 2.7557319223985893e-06;
    K.q[4] = 2.48015873015873e-05;
    K.q[5] = 0.0001984126984126984;
    K.q[6] = 0.001388888888888889;
    K.q[7] = 0.008333333333333333;
    K.q[8] = 0.041666666666666664;
    K.q[9] = 0.16666666666666666;
    K.q[10] = 0.5;
    return K;
}

// the value in scalar registers, opaque to the compiler (so kept, not re-made)
__device__ __forceinline__ double pin_sgpr(double v) {
    asm volatile("" : "+s"(v));
    return v;
}

__device__ __forceinline__ ExpConsts exp_consts_sgpr() {
    ExpConsts K = exp_consts();
    K.inv_ln2 = pin_sgpr(K.inv_ln2);
    K.ln2_hi = pin_sgpr(K.ln2_hi);
    K.ln2_lo = pin_sgpr(K.ln2_lo);
    K.third = pin_sgpr(K.third);
#pragma unroll
    for (int i = 0; i < 10; ++i) K.q[i] = pin_sgpr(K.q[i]);  // q[10] = 0.5 is an inline constant
    return K;
}

__device__ __forceinline__ double exp_neg64(double a, const ExpConsts& K) {
    const double x = -a;
    const double k = __builtin_rint(x * K.inv_ln2);
    double r = fma(-k, K.ln2_hi, x);
    r = fma(-k, K.ln2_lo, r);
    double q = K.q[0];
#pragma unroll
    for (int i = 1; i < 11; ++i) q = fma(q, r, K.q[i]);
    q = fma(q, r, 1.0);
    q = fma(q, r, 1.0);
    return __builtin_amdgcn_ldexp(q, (int)k);
}

__device__ __forceinline__ double exp_neg64(double a) { return exp_neg64(a, exp_consts()); }

// sqrt(s) for s >= 0 in FP64, about 1 ulp: the hardware reciprocal square
// root, one Goldschmidt step (g -> sqrt(s), h -> 1/(2 sqrt(s))) and one
// Newton correction of g; 0 for s = 0.
__device__ __forceinline__ double dist64(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
    const double e = fma(-h, g, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    const double d = fma(-g, g, s);
    g = fma(d, h, g);
    return s > 0.0 ? g : 0.0;
}

// The polynomial factor is written with explicit fused multiply-adds, so
// every kernel that inlines this rounds it the same way (with contraction
// left to the compiler, a product with two uses may or may not be fused).
template <int TWO_NU>
__device__ __forceinline__ double matern_f64(double r, double c, double s2, const ExpConsts& K) {
    const double a = c * r;
    const double e = exp_neg64(a, K);
    if constexpr (TWO_NU == 1) return s2 * e;
    if constexpr (TWO_NU == 3) return s2 * fma(c, r, 1.0) * e;
    return s2 * fma(a, fma(a, K.third, 1.0), 1.0) * e;
}

template <int TWO_NU>
__device__ __forceinline__ double matern_f64(double r, double c, double s2) {
    return matern_f64<TWO_NU>(r, c, s2, exp_consts());
}

// |e|^2 of a 3-vector with explicit fused multiply-adds (the same rounding
// in every kernel that inlines it)
template <typename T>
__device__ __forceinline__ T sqnorm3(T e0, T e1, T e2) {
    return fma(e2, e2, fma(e1, e1, e0 * e0));
}

// acc - sum_{q < n} col[q * ld] * row[q], the fused multiply-adds in q order;
// the strided column entries are loaded U at a time, so that U global loads
// are in flight before the first is used (the multi-target
// kernels' left-looking updates of a row from a column-major slab)
template <typename T, int U = 16>
__device__ __forceinline__ T dot_down(T acc, const T* __restrict__ col, int64_t ld, const T* row, int n) {
    int q = 0;
    for (; q + U <= n; q += U) {
        T v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = col[(int64_t)(q + j) * ld];
#pragma unroll
        for (int j = 0; j < U; ++j) acc = fma(-v[j], row[q + j], acc);
    }
    for (; q < n; ++q) acc = fma(-col[(int64_t)q * ld], row[q], acc);
    return acc;
}

// dot_down over entries 0 .. n-1 of a column whose first nc entries sit in
// LDS (entry q at cache[q * cld]) and the rest in global memory: the same
// multiply-adds in the same order, so the same result as dot_down.
template <typename T, int U = 16>
__device__ __forceinline__ T dot_down_cached(T acc, const T* cache, int cld, int nc, const T* __restrict__ col,
                                             int64_t ld, const T* row, int n) {
    const int n1 = n < nc ? n : nc;
    int q = 0;
    for (; q + U <= n1; q += U) {
        T v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = cache[(q + j) * cld];
#pragma unroll
        for (int j = 0; j < U; ++j) acc = fma(-v[j], row[q + j], acc);
    }
    for (; q < n1; ++q) acc = fma(-cache[q * cld], row[q], acc);
    for (; q + U <= n; q += U) {
        T v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = col[(int64_t)(q + j) * ld];
#pragma unroll
        for (int j = 0; j < U; ++j) acc = fma(-v[j], row[q + j], acc);
    }
    for (; q < n; ++q) acc = fma(-col[(int64_t)q * ld], row[q], acc);
    return acc;
}

__device__ __forceinline__ double matern_f64_rt(int two_nu, double r, double c, double s2) {
    if (two_nu == 1) return matern_f64<1>(r, c, s2);
    if (two_nu == 3) return matern_f64<3>(r, c, s2);
    return matern_f64<5>(r, c, s2);
}

}  // namespace csel
