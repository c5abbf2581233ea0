// screen.hip -- learned candidate screen: per-candidate features, a BF16 MLP
// on MFMA (FP32 accumulation), top-`keep` selection and the fallback flag;
// plus the MLP's training kernels (forward + backward, Adam).
//
// Not part of the paper: the screen prunes a column's pool (sorted by
// distance) to the candidates an MLP scores highest, and the exact greedy
// selection (Sec. 3.1) then runs on the kept candidates.  Columns whose
// dropped candidates carry too much predicted probability fall back to the
// full pool.
//
// MLP 16 -> 64 -> 64 -> 1 (ReLU).  Computed transposed so the MFMA output of
// one layer is directly the B operand of the next: H^T = W^T X^T with
// v_mfma_f32_16x16x16_bf16 tiles (A: weights, 16 hidden x 16 k; B: 16 k x 16
// candidates; D: 16 hidden x 16 candidates).  Lane l of a 16x16x16 MFMA holds
// A[l%16][4(l/16)+i], B[4(l/16)+i][l%16] and D[4(l/16)+i][l%16], i = 0..3.
// The second hidden layer's activations are rounded to BF16 as well; the
// screen evaluates the last layer (64 -> 1) as an MFMA with w3 in the first
// row of A, the training kernels as a VALU dot product of the same rounded
// values.
//
// Parameters: one FP32 vector W1[16][64], b1[64], W2[64][64], b2[64],
// w3[64], b3 and its BF16 copy (same indexing); weights enter the MFMAs in
// BF16, biases stay FP32.
#include <algorithm>
#include <mutex>

#include "device_common.hpp"
#include "launch.hpp"


namespace csel {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kF = 16, kH = 64;
constexpr int kOffW1 = 0, kOffB1 = kF * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH, kNParams = kOffB3 + 1;

// round to the nearest bfloat16, ties to even (inputs are finite)
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float corr(int two_nu, float a) {
    const float e = __expf(-a);
    if (two_nu == 1) return e;
    if (two_nu == 3) return (1.0f + a) * e;
    return (1.0f + a + a * a * (1.0f / 3.0f)) * e;
}

// MLP weights in MFMA operand layout, held in registers by every wave
struct MlpRegs {
    short4_t a1[4];       // W1^T tile h: lane (hid 16h + l%16, feat 4g+i)
    short4_t a2[4][4];    // W2^T tile (h2, h): lane (out 16h2 + l%16, in 16h + 4g + i)
    float b1[4][4];       // b1[16h + 4g + i]
    float b2[4][4];
    float w3[4][4];       // bf16-rounded w3[16h + 4g + i]
    float b3;
};

__device__ __forceinline__ void load_mlp(MlpRegs& R, const float* __restrict__ p, const uint16_t* __restrict__ pb,
                                         int lane) {
    const int c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            R.a1[h][i] = (short)pb[kOffW1 + (4 * g + i) * kH + 16 * h + c];
            R.b1[h][i] = p[kOffB1 + 16 * h + 4 * g + i];
            R.b2[h][i] = p[kOffB2 + 16 * h + 4 * g + i];
            R.w3[h][i] = bf16_to_f32(pb[kOffW3 + 16 * h + 4 * g + i]);
        }
#pragma unroll
        for (int h2 = 0; h2 < 4; ++h2)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                R.a2[h2][h][i] = (short)pb[kOffW2 + (16 * h + 4 * g + i) * kH + 16 * h2 + c];
    }
    R.b3 = p[kOffB3];
}

typedef float float2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// two floats -> two bf16 (round to nearest even, v_cvt_pk_bf16_f32), as the
// low and high halves of a 32-bit word
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    const bf16x2_t v = __builtin_convertvector(float2_t{a, b}, bf16x2_t);
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ short4_t pack_bf16x4(float a, float b, float c, float d) {
    const uint2 v = {pack_bf16x2(a, b), pack_bf16x2(c, d)};
    return __builtin_bit_cast(short4_t, v);
}

// ReLU of packed bf16 values: rounding to bf16 keeps the sign, and a bf16
// with its sign bit set reads as a negative int16, so max(., 0) per 16-bit
// half (v_pk_max_i16) equals rounding max(x, 0).
__device__ __forceinline__ short4_t relu_bf16x4(short4_t v) {
    return __builtin_elementwise_max(v, short4_t{0, 0, 0, 0});
}

// Forward for one tile of 16 candidates; xb = B operand (feat 4g+i of candidate l%16).
// The biases seed the MFMA accumulators.  Returns the logit of candidate l%16
// (identical in the four lanes that share it); optionally exposes H1 (bf16
// operand form) and H2 (fp32) for the backward pass.
__device__ __forceinline__ float mlp_tile(const MlpRegs& R, short4_t xb, short4_t* h1q_out, float4_t* h2_out) {
    short4_t h1q[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        float4_t acc = {R.b1[h][0], R.b1[h][1], R.b1[h][2], R.b1[h][3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a1[h], xb, acc, 0, 0, 0);
        h1q[h] = relu_bf16x4(pack_bf16x4(acc[0], acc[1], acc[2], acc[3]));
    }
    float part = 0.0f;
#pragma unroll
    for (int h2 = 0; h2 < 4; ++h2) {
        float4_t acc = {R.b2[h2][0], R.b2[h2][1], R.b2[h2][2], R.b2[h2][3]};
#pragma unroll
        for (int h = 0; h < 4; ++h) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.a2[h2][h], h1q[h], acc, 0, 0, 0);
        const short4_t h2q = relu_bf16x4(pack_bf16x4(acc[0], acc[1], acc[2], acc[3]));
        float4_t hv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            hv[i] = bf16_to_f32((uint16_t)h2q[i]);
            part += hv[i] * R.w3[h2][i];
        }
        if (h2_out) h2_out[h2] = hv;
    }
    if (h1q_out)
#pragma unroll
        for (int h = 0; h < 4; ++h) h1q_out[h] = h1q[h];
    // the four lane groups (l/16) hold disjoint hidden units of the same candidate
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    return part + R.b3;
}

// Weight operands of the MFMAs staged in LDS (shared by the waves of a block)
// in per-lane operand order: A fragment f of lane l at [f][l].
// Layer 2 uses v_mfma_f32_16x16x32_bf16 (lane l: A[l%16][8(l/16)+j], B[8(l/16)+j][l%16],
// j = 0..7).  Its K = 32 block q covers hidden units 32q + 4g + (0..3) and
// 32q + 16 + 4g + (0..3) for lane group g, the order in which the layer-1
// output fragments of tiles 2q and 2q+1 sit in a lane, so B is their plain
// concatenation; W2 is staged in the same order.
// The last layer uses the same K = 32 blocks with A = w3 in row 0 (lanes
// l % 16 == 0), zeros elsewhere.
struct MlpLds {
    uint2 a1[4][64];
    uint4 a2[4][2][64];  // [h2][q][lane]
    uint4 a3[2][64];     // [q][lane]
    float4 b1[4][4];     // [h][lane group]: b1[16h + 4g + i]
    float4 b2[4][4];
    float b3;
};

__device__ __forceinline__ void stage_mlp(MlpLds& L, const float* __restrict__ pf, const uint16_t* __restrict__ pb) {
    for (int e = threadIdx.x; e < 16; e += blockDim.x) {
        const int h = e >> 2, g = e & 3;
        L.b1[h][g] = float4{pf[kOffB1 + 16 * h + 4 * g], pf[kOffB1 + 16 * h + 4 * g + 1],
                            pf[kOffB1 + 16 * h + 4 * g + 2], pf[kOffB1 + 16 * h + 4 * g + 3]};
        L.b2[h][g] = float4{pf[kOffB2 + 16 * h + 4 * g], pf[kOffB2 + 16 * h + 4 * g + 1],
                            pf[kOffB2 + 16 * h + 4 * g + 2], pf[kOffB2 + 16 * h + 4 * g + 3]};
    }
    if (threadIdx.x == 0) L.b3 = pf[kOffB3];
    for (int e = threadIdx.x; e < 14 * 64; e += blockDim.x) {
        const int f = e >> 6, l = e & 63, c = l & 15, g = l >> 4;
        if (f >= 12) {
            const int q = f - 12;
            uint32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int u0 = 32 * q + (2 * j < 4 ? 4 * g + 2 * j : 16 + 4 * g + (2 * j - 4));
                w[j] = c == 0 ? (uint32_t)pb[kOffW3 + u0] | ((uint32_t)pb[kOffW3 + u0 + 1] << 16) : 0u;
            }
            L.a3[q][l] = uint4{w[0], w[1], w[2], w[3]};
        } else if (f < 4) {
            short4_t v;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = (short)pb[kOffW1 + (4 * g + i) * kH + 16 * f + c];
            L.a1[f][l] = __builtin_bit_cast(uint2, v);
        } else {
            const int h2 = (f - 4) >> 1, q = (f - 4) & 1;
            short v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int unit = 32 * q + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
                v[j] = (short)pb[kOffW2 + unit * kH + 16 * h2 + c];
            }
            L.a2[h2][q][l] = uint4{(uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16),
                                   (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16),
                                   (uint32_t)(uint16_t)v[4] | ((uint32_t)(uint16_t)v[5] << 16),
                                   (uint32_t)(uint16_t)v[6] | ((uint32_t)(uint16_t)v[7] << 16)};
        }
    }
}

// The forward of mlp_tile for NT independent tiles at once, with the MFMA
// weight operands and the biases read from LDS: each weight operand is
// read from LDS once and applied to every tile, and the tiles' MFMA chains
// interleave.
template <int NT>
__device__ __forceinline__ void mlp_tiles_lds(const MlpLds& L, const short4_t (&xb)[NT], float (&z)[NT], int lane) {
    const int g = lane >> 4;
    short4_t h1q[NT][4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const short4_t a = __builtin_bit_cast(short4_t, L.a1[h][lane]);
        const float4 bb = L.b1[h][g];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float4_t acc = {bb.x, bb.y, bb.z, bb.w};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, xb[t], acc, 0, 0, 0);
            h1q[t][h] = relu_bf16x4(pack_bf16x4(acc[0], acc[1], acc[2], acc[3]));
        }
    }
    short4_t h2q[NT][4];
#pragma unroll
    for (int h2 = 0; h2 < 4; ++h2) {
        float4_t acc[NT];
        const float4 bb = L.b2[h2][g];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = float4_t{bb.x, bb.y, bb.z, bb.w};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const bf16x8_t a = __builtin_bit_cast(bf16x8_t, L.a2[h2][q][lane]);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const uint2 lo = __builtin_bit_cast(uint2, h1q[t][2 * q]);
                const uint2 hi = __builtin_bit_cast(uint2, h1q[t][2 * q + 1]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a, __builtin_bit_cast(bf16x8_t, uint4{lo.x, lo.y, hi.x, hi.y}), acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) h2q[t][h2] = relu_bf16x4(pack_bf16x4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]));
    }
    float4_t acc[NT];
    const float b3 = L.b3;
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = float4_t{b3, b3, b3, b3};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const bf16x8_t a = __builtin_bit_cast(bf16x8_t, L.a3[q][lane]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const uint2 lo = __builtin_bit_cast(uint2, h2q[t][2 * q]), hi = __builtin_bit_cast(uint2, h2q[t][2 * q + 1]);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8_t, uint4{lo.x, lo.y, hi.x, hi.y}),
                                                             acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) z[t] = acc[t][0];
}


// ---------------------------------------------------------------------------
// features of one candidate (FP32); see the feature list in the header
// ---------------------------------------------------------------------------
// Features of one candidate except the nearest-eight terms f6, f7 (which the
// caller accumulates with the neighbour loop outermost).  FP32; divisions use
// hardware reciprocals (the features feed BF16 MFMA operands).
struct ColumnConsts {
    float inv_ell, cnu, tiny, adiag, inv_adiag, r0, inv_r0g, log_r0g, rho_i0, inv_c, inv_log1p_c;
};

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Order-preserving 32-bit image of a finite float (a larger value gives a
// larger key); -0 maps to the key of +0, so equal values give equal keys.
// Every finite value maps to a key >= 2^23, so 0 is free to mark "none".
__device__ __forceinline__ uint32_t mono_key(float z) {
    uint32_t b = __float_as_uint(z);
    if (b == 0x80000000u) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ void candidate_features(const ScreenArgs& p, const ColumnConsts& k, int s, const float d[3],
                                                   float r, const float d0[3], float f[kF]) {
    const float rs = fmaxf(r, k.tiny);
    f[0] = __logf(rs) - k.log_r0g;
    f[1] = (float)s * k.inv_c;
    const float rho_i = corr(p.two_nu, k.cnu * r);
    f[2] = rho_i;
    f[3] = r * k.inv_ell;
    f[4] = k.r0 * k.inv_ell;
    const float dot0 = d[0] * d0[0] + d[1] * d0[1] + d[2] * d0[2];
    f[5] = r > 0.0f ? dot0 * frcp(rs) * k.inv_r0g : 1.0f;
    const float e0 = d[0] - d0[0], e1 = d[1] - d0[1], e2 = d[2] - d0[2];
    const float dj0 = __builtin_amdgcn_sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
    const float rho_j0c = corr(p.two_nu, k.cnu * dj0);
    f[8] = rho_j0c;
    const float cov1 = rho_i - k.rho_i0 * rho_j0c * k.inv_adiag;
    const float var1 = k.adiag - rho_j0c * rho_j0c * k.inv_adiag;
    f[9] = s == 0 ? 1.0f : (var1 > 1e-12f * k.adiag ? cov1 * cov1 * frcp(var1) * k.inv_adiag : 0.0f);
    f[10] = s == 0 ? 1.0f : 0.0f;
    f[11] = __logf(1.0f + (float)s) * k.inv_log1p_c;
#pragma unroll
    for (int q = 12; q < kF; ++q) f[q] = 0.0f;
}

// four waves per block share the staged MLP operands; with at most 128
// VGPRs (one spilled value) four waves per SIMD fit, which this latency-bound
// kernel turns into throughput
constexpr int kScrWaves = 4;
constexpr int kScrWavesPerSimd = 4;

// One wave per column; persistent waves walk through the processing order
// (each wave stages the MLP weights once).  The pool (<= 64*RPL*NCH candidates) is processed in NCH
// chunks of 64*RPL (RPL per lane) for features and the MLP, so only one
// chunk's candidate state is live; the logits of the whole pool then go
// through the top-keep selection.
template <int RPL, int NCH>
__global__ __launch_bounds__(kScrWaves * 64, kScrWavesPerSimd) void screen_kernel(ScreenArgs p) {
    constexpr int CH = 64 * RPL;
    constexpr int MAXC = CH * NCH;
    constexpr int KPL = RPL * NCH;  // keys per lane
    constexpr int kNT = 2;  // MLP tiles per LDS weight read
    static_assert((CH / 16) % kNT == 0, "tile groups must divide a chunk");
    __shared__ __align__(16) uint16_t sh_x[kScrWaves][CH][kF];
    __shared__ float sh_z[kScrWaves][MAXC];
    __shared__ float4 sh_nb[kScrWaves][8];  // nearest eight: offset from the target, distance
    __shared__ MlpLds sh_w;
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int cl = lane & 15, g = lane >> 4;
    if (p.mode == 0) stage_mlp(sh_w, p.params, p.params_bf16);
    __syncthreads();
    const int dim = p.dim;
    ColumnConsts kc0;
    kc0.inv_ell = (float)(1.0 / p.ell);
    kc0.cnu = (float)p.c_nu;
    kc0.tiny = 1e-9f * (float)p.ell;
    kc0.adiag = 1.0f + (float)(p.nugget / p.s2);
    kc0.inv_adiag = 1.0f / kc0.adiag;
    const int lim = min(p.stride, MAXC);  // pool entries a column may use
    // Positions in the processing order are split into eight contiguous
    // segments, one per XCD (workgroups go to the XCDs round-robin, so block
    // b runs on XCD b % 8): the waves of one XCD walk through their segment
    // side by side and share that XCD's L2.  The grid is a multiple of 8.
    const int64_t T = p.n_targets;
    const int64_t NP = p.order ? p.n_order : T;  // positions to process
    const int64_t seg = (NP + 7) / 8;
    const int64_t seg0 = (int64_t)(blockIdx.x & 7u) * seg;
    const int64_t seg1 = min(seg0 + seg, NP);
    const int64_t pstep = (int64_t)(gridDim.x >> 3) * kScrWaves;
    int64_t pos = seg0 + (int64_t)(blockIdx.x >> 3) * kScrWaves + wib;
    // the column at a position (-1 past the segment), loaded by lane 0
    auto col_load = [&](int64_t ps) -> int32_t {
        int32_t c = -1;
        if (ps < seg1 && lane == 0) c = p.order ? p.order[ps] : (int32_t)ps;
        return c;
    };
    // The next column's target, pool length, pool indices (slot kk*64 + lane)
    // and target coordinates (lane c < dim) are loaded while this column is
    // processed, and the column after it is looked up; the pool indices stay
    // in registers for the whole column.
    int32_t nx_pid[KPL];
    int32_t nx_tgt = -1, nx_len = 0;
    double nx_xc = 0.0;
    auto fetch_ids = [&](int64_t c) {
        nx_tgt = -1;
        nx_len = 0;
#pragma unroll
        for (int kk = 0; kk < KPL; ++kk) nx_pid[kk] = -1;
        if (c >= 0 && c < T) {
            if (lane == 0) {  // vector loads, so they complete in order with the gathers
                nx_tgt = p.targets[c];
                nx_len = p.pool_len[c];
            }
#pragma unroll
            for (int kk = 0; kk < KPL; ++kk)
                if (kk * 64 + lane < lim) nx_pid[kk] = p.pool[c * p.stride + kk * 64 + lane];
        }
    };
    auto fetch_xi = [&]() {
        const int32_t t = __builtin_amdgcn_readfirstlane(nx_tgt);
        nx_xc = 0.0;
        if (t >= 0 && (int64_t)t < p.n && lane < dim) nx_xc = p.pts[(int64_t)t * dim + lane];
    };
    int32_t c_cur = __builtin_amdgcn_readfirstlane(col_load(pos));
    fetch_ids(c_cur);
    fetch_xi();
    int32_t c_nx = col_load(pos + pstep);
    for (; pos < seg1; pos += pstep) {
        const int64_t col = c_cur;
        const int32_t tgt = __builtin_amdgcn_readfirstlane(nx_tgt);
        int32_t C = __builtin_amdgcn_readfirstlane(nx_len);
        int32_t pid[KPL];
#pragma unroll
        for (int kk = 0; kk < KPL; ++kk) pid[kk] = nx_pid[kk];
        const double xi[3] = {bcast(nx_xc, 0), bcast(nx_xc, 1), bcast(nx_xc, 2)};  // zero past dim
        c_cur = __builtin_amdgcn_readfirstlane(c_nx);
        fetch_ids(c_cur);
        c_nx = col_load(pos + 2 * pstep);
        if (col < 0 || col >= T) {  // an order entry out of range
            fetch_xi();
            continue;
        }
        const bool bad = tgt < 0 || (int64_t)tgt >= p.n || C < 0 || C > lim;
        bool my_bad = false;
#pragma unroll
        for (int kk = 0; kk < KPL; ++kk)
            if (kk * 64 + lane < C) my_bad |= pid[kk] < 0 || (int64_t)pid[kk] >= p.n;
        if (__any(my_bad) || bad) {
            // bad input: nothing kept; the column is listed with the fallback
            // columns, so the full-pool selection validates it and reports it
            if (lane == 0 && p.mode == 0) {
                p.kept_len[col] = 0;
                p.fallback[col] = 3;
                if (p.fb_list) {
                    const int fpos = atomicAdd(p.fb_count, 1);
                    p.fb_list[fpos] = (int32_t)col;
                }
            }
            fetch_xi();
            continue;
        }
        if (C == 0) fetch_xi();
        ColumnConsts kc = kc0;
        float d0[3] = {0.0f, 0.0f, 0.0f};
        const int nnear = min(8, C);
        for (int ch = 0; ch < NCH; ++ch) {
            if (ch * CH >= C) break;
            // this chunk's candidates: offsets from the target (one gather per coordinate)
            double xq[RPL][3];
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
                const int kk = ch * RPL + rr;
                const bool ok = kk * 64 + lane < C;
                const int64_t base = (int64_t)(ok ? pid[kk] : tgt) * dim;
                // branch-free (a clamped coordinate, zeroed past dim) so the
                // loads stay in flight together
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double v = p.pts[base + min(c, dim - 1)];
                    xq[rr][c] = c < dim ? v : 0.0;
                }
            }
            if (ch == 0) fetch_xi();  // the next target index was loaded before these gathers
            float d[RPL][3], r[RPL];
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
#pragma unroll
                for (int c = 0; c < 3; ++c) d[rr][c] = (float)(xq[rr][c] - xi[c]);
                r[rr] = __builtin_amdgcn_sqrtf(d[rr][0] * d[rr][0] + d[rr][1] * d[rr][1] + d[rr][2] * d[rr][2]);
            }
            if (ch == 0) {
                // the nearest eight (slots 0..7: lanes 0..7 of the first row) -> LDS
                if (lane < 8)
                    sh_nb[wib][lane] = lane < C ? float4{d[0][0], d[0][1], d[0][2], r[0]} : float4{0.f, 0.f, 0.f, 0.f};
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                const float4 nb0 = sh_nb[wib][0];
                d0[0] = nb0.x;
                d0[1] = nb0.y;
                d0[2] = nb0.z;
                kc.r0 = nb0.w;
                const float r0g = fmaxf(kc.r0, kc.tiny);
                kc.inv_r0g = frcp(r0g);
                kc.log_r0g = __logf(r0g);
                kc.rho_i0 = corr(p.two_nu, kc.cnu * kc.r0);
                kc.inv_c = frcp((float)max(C, 1));
                kc.inv_log1p_c = frcp(__logf(1.0f + (float)max(C, 1)));
            }
            // nearest-eight terms, neighbour outermost: squared distance to the
            // nearest other of slots 0..7 (f6) and the count of closer ones inside
            // the cos > 0.7 cone (f7, tested as d.d_l > 0.7 r_s max(r_l, tiny))
            float best2[RPL];
            int cnt[RPL];
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
                best2[rr] = INFINITY;
                cnt[rr] = 0;
            }
            for (int l = 0; l < nnear; ++l) {
                const float4 nl = sh_nb[wib][l];
                const float cone = 0.7f * fmaxf(nl.w, kc.tiny);
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    const float e0 = d[rr][0] - nl.x, e1 = d[rr][1] - nl.y, e2 = d[rr][2] - nl.z;
                    const float e2s = e0 * e0 + e1 * e1 + e2 * e2;
                    const float dl = d[rr][0] * nl.x + d[rr][1] * nl.y + d[rr][2] * nl.z;
                    // slot ch * CH + rr * 64 + lane is neighbour l (< 8) itself
                    // only in row 0 of chunk 0
                    const bool other = rr > 0 || ch > 0 || lane != l;
                    best2[rr] = other ? fminf(best2[rr], e2s) : best2[rr];
                    const float rsv = fmaxf(r[rr], kc.tiny);
                    cnt[rr] += (other && nl.w < r[rr] && dl > rsv * cone) ? 1 : 0;
                }
            }
            // features -> LDS (bf16), optionally -> global (fp32)
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
                const int sl = rr * 64 + lane;
                const int s = ch * CH + sl;
                float f[kF];
                candidate_features(p, kc, s, d[rr], r[rr], d0, f);
                const float rsv = fmaxf(r[rr], kc.tiny);
                f[6] = best2[rr] < INFINITY ? __builtin_amdgcn_sqrtf(best2[rr]) * frcp(rsv) : 0.0f;
                f[7] = (float)cnt[rr] * 0.125f;
                // rows of slots >= C hold finite values (of the target's own
                // offset); the MLP keeps candidates apart (one B column each)
                // and their logits are never read
                uint4* row = reinterpret_cast<uint4*>(&sh_x[wib][sl][0]);
                row[0] = uint4{pack_bf16x2(f[0], f[1]), pack_bf16x2(f[2], f[3]), pack_bf16x2(f[4], f[5]),
                               pack_bf16x2(f[6], f[7])};
                row[1] = uint4{pack_bf16x2(f[8], f[9]), pack_bf16x2(f[10], f[11]), pack_bf16x2(f[12], f[13]),
                               pack_bf16x2(f[14], f[15])};
                if (p.feats && s < C)
#pragma unroll
                    for (int q = 0; q < kF; ++q) p.feats[(col * p.stride + s) * kF + q] = f[q];
            }
            if (p.mode == 1) continue;  // features only
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // MLP over this chunk's tiles of 16 candidates, kNT tiles at a time
            // (CH / 16 is a multiple of kNT, so the rows a group reads past
            // ntiles are this chunk's; their logits are unused)
            const int ntiles = (min(C - ch * CH, CH) + 15) >> 4;
            for (int tile = 0; tile < ntiles; tile += kNT) {
                asm volatile("" ::: "memory");  // keep the weight operands in LDS (not hoisted to VGPRs)
                short4_t xb[kNT];
                float z[kNT];
#pragma unroll
                for (int t = 0; t < kNT; ++t)
                    xb[t] = __builtin_bit_cast(short4_t,
                                               *reinterpret_cast<const uint2*>(&sh_x[wib][(tile + t) * 16 + cl][4 * g]));
                mlp_tiles_lds<kNT>(sh_w, xb, z, lane);
#pragma unroll
                for (int t = 0; t < kNT; ++t)
                    if (g == 0) sh_z[wib][ch * CH + (tile + t) * 16 + cl] = z[t];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        if (p.mode == 1) continue;
        // 32-bit keys: the order-preserving image of the logit (equal logits,
        // equal keys); 0 marks an empty slot.  Slot s = kk*64 + lane.
        uint32_t key[KPL];
        float zz[KPL];
#pragma unroll
        for (int kk = 0; kk < KPL; ++kk) {
            const int s = kk * 64 + lane;
            zz[kk] = s < C ? sh_z[wib][s] : 0.0f;
            key[kk] = s < C ? mono_key(zz[kk]) : 0u;
            if (p.logits && s < C) p.logits[col * p.stride + s] = zz[kk];
        }
        const int keep = p.keep;
        // kept = key > thr, plus the first `need` slots with key == thr
        uint32_t thr = 0u;
        int need = 0;
        if (C > keep) {
            // bisection for the largest key value thr with at least `keep`
            // keys at or above it; it stops early at a midpoint with exactly
            // `keep` keys at or above it (that set is then the top `keep`)
            uint32_t lo = 0u, hi = 0xFFFFFFFFu;
            int cnt_lo = C;
            while (lo < hi) {
                const uint32_t mid = lo + (hi - lo) / 2u + 1u;
                int cntk = 0;
#pragma unroll
                for (int kk = 0; kk < KPL; ++kk) cntk += __popcll(__ballot(key[kk] >= mid));
                if (cntk >= keep) {
                    lo = mid;
                    cnt_lo = cntk;
                    if (cntk == keep) break;
                } else {
                    hi = mid - 1u;
                }
            }
            thr = lo;
            // keys equal to thr: as many as the top `keep` still needs
            int cnt_eq = 0;
#pragma unroll
            for (int kk = 0; kk < KPL; ++kk) cnt_eq += __popcll(__ballot(key[kk] != 0u && key[kk] == thr));
            need = keep - (cnt_lo - cnt_eq);
        } else {
            need = 0;  // every valid key (>= 1) exceeds thr = 0
        }
        // kept candidates in slot order; ties at thr go to the smaller slot
        int base = 0, tbase = 0;
        float drop = 0.0f;
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
        for (int kk = 0; kk < KPL; ++kk) {
            const bool eq = key[kk] != 0u && key[kk] == thr;
            const uint64_t me = __ballot(eq);
            const bool k = key[kk] > thr || (eq && tbase + __popcll(me & below) < need);
            tbase += __popcll(me);
            const uint64_t m = __ballot(k);
            if (k) p.kept[col * keep + base + __popcll(m & below)] = pid[kk];
            base += __popcll(m);
            if (key[kk] != 0u && !k) drop += frcp(1.0f + __expf(-zz[kk]));
        }
        drop = wave_sum_f32(drop);
        const bool fb = C > keep && drop > p.fb_thr;
        for (int q = base + lane; q < keep; q += 64) p.kept[col * keep + q] = -1;
        if (lane == 0) {
            p.kept_len[col] = base;
            p.fallback[col] = fb ? 1 : 0;
            if (fb && p.fb_list) {
                const int pos = atomicAdd(p.fb_count, 1);
                p.fb_list[pos] = (int32_t)col;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// training: forward + weighted BCE + backward for rows of features
// ---------------------------------------------------------------------------
// One wave per block of rows; tiles of 16 rows.  Weight gradients are
// reduced over rows with MFMAs whose operands are re-laid out through LDS,
// accumulated in registers over the wave's rows and written as one partial
// per wave; a second kernel sums the partials in a fixed order.
constexpr int kTrainTilesPerWave = 16;  // 256 rows per wave

__global__ __launch_bounds__(64) void mlp_grad_kernel(MlpTrainArgs p) {
    __shared__ __align__(16) uint16_t sh_h1[16][kH];   // H1q of the tile, [row][hid]
    __shared__ __align__(16) uint16_t sh_d2[16][kH];   // dH2 (bf16), [row][hid]
    __shared__ __align__(16) uint16_t sh_d1[16][kH];   // dH1 (bf16), [row][hid]
    __shared__ __align__(16) uint16_t sh_x[16][kF];    // X (bf16), [row][feat]
    const int lane = lane_id();
    const int cl = lane & 15, g = lane >> 4;
    MlpRegs R;
    load_mlp(R, p.params, p.params_bf16, lane);
    // W2 as the A operand of dH1^T = W2 dH2^T: lane (in 16h + l%16, out 16h2 + 4g + i)
    short4_t aw2[4][4];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int h2 = 0; h2 < 4; ++h2)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                aw2[h][h2][i] = (short)p.params_bf16[kOffW2 + (16 * h + cl) * kH + 16 * h2 + 4 * g + i];
    float4_t gW2[4][4], gW1[4];  // dW2^T tiles (out 16h2.., in 16h..), dW1^T tiles (hid 16h.., feat)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
    }
    float gw3[4][4] = {}, gb1[4][4] = {}, gb2[4][4] = {};
    float gb3 = 0.0f, loss = 0.0f;
    const int64_t row0 = (int64_t)blockIdx.x * kTrainTilesPerWave * 16;
    for (int tile = 0; tile < kTrainTilesPerWave; ++tile) {
        const int64_t row = row0 + tile * 16 + cl;
        const bool valid = row < p.n_rows;
        // inputs
        short4_t xb;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float v = valid ? p.x[row * kF + 4 * g + i] : 0.0f;
            xb[i] = (short)bf16_bits(v);
            sh_x[cl][4 * g + i] = (uint16_t)xb[i];
        }
        short4_t h1q[4];
        float4_t act2[4];
        const float z = mlp_tile(R, xb, h1q, act2);
        const float y = valid ? (float)p.y[row] : 0.0f;
        const float wgt = valid ? (y > 0.5f ? p.pos_weight : 1.0f) : 0.0f;
        const float sig = 1.0f / (1.0f + __expf(-z));
        const float dz = wgt * (sig - y) * p.inv_n;
        if (g == 0 && valid) loss += wgt * (fmaxf(z, 0.0f) - z * y + log1pf(__expf(-fabsf(z))));
        if (g == 0) gb3 += dz;
        // layer 3 and dH2 (D layout: hid 16h2 + 4g + i, row l%16)
        float4_t d2[4];
#pragma unroll
        for (int h2 = 0; h2 < 4; ++h2)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                gw3[h2][i] += dz * act2[h2][i];
                d2[h2][i] = act2[h2][i] > 0.0f ? dz * R.w3[h2][i] : 0.0f;
                gb2[h2][i] += d2[h2][i];
            }
        // dH1^T = W2 dH2^T (B operand = dH2^T in D layout, rounded to bf16)
        short4_t d2q[4];
#pragma unroll
        for (int h2 = 0; h2 < 4; ++h2)
#pragma unroll
            for (int i = 0; i < 4; ++i) d2q[h2][i] = (short)bf16_bits(d2[h2][i]);
        short4_t d1q[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int h2 = 0; h2 < 4; ++h2) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aw2[h][h2], d2q[h2], acc, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // relu' of layer 1: the pre-rounding activation is > 0 exactly when its bf16 is
                const float dv = bf16_to_f32((uint16_t)h1q[h][i]) > 0.0f ? acc[i] : 0.0f;
                gb1[h][i] += dv;
                d1q[h][i] = (short)bf16_bits(dv);
            }
        }
        // re-lay H1q, dH2, dH1 as [row][hid] through LDS
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                sh_h1[cl][16 * h + 4 * g + i] = (uint16_t)h1q[h][i];
                sh_d2[cl][16 * h + 4 * g + i] = (uint16_t)d2q[h][i];
                sh_d1[cl][16 * h + 4 * g + i] = (uint16_t)d1q[h][i];
            }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // dW2^T (out x in) += dH2^T (out x rows) * H1 (rows x in): A lane (out 16h2 + l%16, row 4g+i),
        // B lane (in 16h + l%16, row 4g+i)
#pragma unroll
        for (int h2 = 0; h2 < 4; ++h2) {
            short4_t a;
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = (short)sh_d2[4 * g + i][16 * h2 + cl];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                short4_t b;
#pragma unroll
                for (int i = 0; i < 4; ++i) b[i] = (short)sh_h1[4 * g + i][16 * h + cl];
                gW2[h2][h] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, gW2[h2][h], 0, 0, 0);
            }
        }
        // dW1^T (hid x feat) += dH1^T (hid x rows) * X (rows x feat)
        {
            short4_t b;
#pragma unroll
            for (int i = 0; i < 4; ++i) b[i] = (short)sh_x[4 * g + i][cl];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                short4_t a;
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = (short)sh_d1[4 * g + i][16 * h + cl];
                gW1[h] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, gW1[h], 0, 0, 0);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // reduce the per-lane bias / w3 partials over the 16 rows of a lane group
    auto row_sum = [](float v) {
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        return v;
    };
    float* out = p.partials + (int64_t)blockIdx.x * (kNParams + 1);
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float a = row_sum(gw3[h][i]), b1 = row_sum(gb1[h][i]), b2 = row_sum(gb2[h][i]);
            if (cl == 0) {
                out[kOffW3 + 16 * h + 4 * g + i] = a;
                out[kOffB1 + 16 * h + 4 * g + i] = b1;
                out[kOffB2 + 16 * h + 4 * g + i] = b2;
            }
        }
    // D layout of the gradient tiles: lane (row 4g+i of the tile, col l%16)
#pragma unroll
    for (int h2 = 0; h2 < 4; ++h2)
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i)  // dW2[in][out] with out = 16h2 + 4g + i, in = 16h + l%16
                out[kOffW2 + (16 * h + cl) * kH + 16 * h2 + 4 * g + i] = gW2[h2][h][i];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i)  // dW1[feat][hid] with hid = 16h + 4g + i, feat = l%16
            out[kOffW1 + cl * kH + 16 * h + 4 * g + i] = gW1[h][i];
    float lsum = row_sum(loss);
    lsum += __shfl_xor(lsum, 16, 64);
    lsum += __shfl_xor(lsum, 32, 64);
    float g3 = row_sum(gb3);
    if (lane == 0) {
        out[kOffB3] = g3;
        out[kNParams] = lsum;
    }
}

// grad[j] = sum over waves of partial[w][j] in a fixed order; slot kNParams = loss sum
__global__ __launch_bounds__(256) void reduce_partials_kernel(const float* __restrict__ partials, int nparts,
                                                              float* __restrict__ grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > kNParams) return;
    float s = 0.0f;
    for (int w = 0; w < nparts; ++w) s += partials[(int64_t)w * (kNParams + 1) + j];
    grad[j] = s;
}

// Adam (Kingma & Ba) on the FP32 master parameters; refreshes the BF16 copy.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, uint16_t* __restrict__ pb,
                                                   const float* __restrict__ g, float* __restrict__ m,
                                                   float* __restrict__ v, int n, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    const float pj = p[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    p[j] = pj;
    pb[j] = bf16_bits(pj);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ p, uint16_t* __restrict__ pb, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) pb[j] = bf16_bits(p[j]);
}

// forward only: logits of feature rows (for tests and evaluation)
__global__ __launch_bounds__(64) void mlp_forward_kernel(MlpTrainArgs p, float* __restrict__ z_out) {
    const int lane = lane_id();
    const int cl = lane & 15, g = lane >> 4;
    MlpRegs R;
    load_mlp(R, p.params, p.params_bf16, lane);
    const int64_t row0 = (int64_t)blockIdx.x * kTrainTilesPerWave * 16;
    for (int tile = 0; tile < kTrainTilesPerWave; ++tile) {
        const int64_t row = row0 + tile * 16 + cl;
        const bool valid = row < p.n_rows;
        short4_t xb;
#pragma unroll
        for (int i = 0; i < 4; ++i) xb[i] = (short)bf16_bits(valid ? p.x[row * kF + 4 * g + i] : 0.0f);
        const float z = mlp_tile(R, xb, nullptr, nullptr);
        if (g == 0 && valid) z_out[row] = z;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// Persistent grid: as many blocks as fit on the device at once (a multiple of
// 8, one share per XCD), fewer for small inputs; each wave loops over its
// segment of the processing order.
template <int RPL, int NCH>
static hipError_t launch_screen_t(const ScreenArgs& a, hipStream_t s) {
    static int resident[64] = {};  // blocks per device, by device id
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (resident[dev] == 0) {
        int per_cu = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, screen_kernel<RPL, NCH>, kScrWaves * 64, 0);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        resident[dev] = std::max(8, (std::max(per_cu, 1) * cus) / 8 * 8);
    }
    const int64_t np = a.order ? a.n_order : a.n_targets;
    const int64_t need = ((np + kScrWaves - 1) / kScrWaves + 7) / 8 * 8;
    const unsigned grid = (unsigned)std::min<int64_t>(need, resident[dev]);
    hipLaunchKernelGGL((screen_kernel<RPL, NCH>), dim3(grid), dim3(kScrWaves * 64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_screen(const ScreenArgs& a, int rpl, hipStream_t s) {
    if (a.n_targets == 0 || (a.order && a.n_order == 0)) return hipSuccess;
    switch (rpl) {
        case 1: return launch_screen_t<1, 1>(a, s);
        case 2: return launch_screen_t<2, 1>(a, s);
        // two rows per lane keeps the live state small enough for the 128-VGPR
        // budget of four waves per SIMD, and LDS at 37 KB per 4-wave block
        case 4: return launch_screen_t<2, 2>(a, s);
        case 8: return launch_screen_t<2, 4>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// screen of multi-target groups (GP prediction batches, supernodes)
// ---------------------------------------------------------------------------
// One 256-thread workgroup per group: pools of up to 2048 candidates (sorted
// by the distance to the nearest member) against up to 64 members.  Features
// (distances to the members, FP32) of a chunk of 512 candidates -> LDS (BF16)
// -> the same MLP as the column screen, each wave on its quarter of the
// chunk's tiles -> logits in LDS; then a workgroup-wide bisection for the
// keep-th largest logit (ties to the smaller slot) and the kept list in slot order.
constexpr int kGrpThreads = 256;
constexpr int kGrpWaves = kGrpThreads / 64;
constexpr int kGrpChunk = 512;
constexpr int kGrpSlots = kGroupScreenMaxPool / kGrpThreads;  // slots per thread: tid + 256 i

__device__ __forceinline__ uint32_t wave_min32(uint32_t v) {
    v = min(v, dpp32<kDppQuadXor1>(v));
    v = min(v, dpp32<kDppQuadXor2>(v));
    v = min(v, dpp32<kDppRowRor4>(v));
    v = min(v, dpp32<kDppRowRor8>(v));
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0), b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32), d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return min(min(a, b), min(c, d));
}

// distance of a candidate to a member (FP64 difference, FP32 norm); the one
// expression both passes use
__device__ __forceinline__ float member_dist(const double xj[3], const double* mq) {
    const float e0 = (float)(xj[0] - mq[0]), e1 = (float)(xj[1] - mq[1]), e2 = (float)(xj[2] - mq[2]);
    return __builtin_amdgcn_sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
}

__device__ __forceinline__ void group_candidate_features(const GroupScreenArgs& p, const double (*mem)[3], int m,
                                                         const uint32_t* dmin_bits, const double xj[3], int s, int C,
                                                         float log_r10, float f[kF]) {
    const float cnu = (float)p.c_nu, inv_ell = (float)(1.0 / p.ell), tiny = 1e-9f * (float)p.ell;
    float r1 = INFINITY, r2 = INFINITY, sr = 0.0f, sr2 = 0.0f, sd = 0.0f, rmin = INFINITY, sx = 0.0f;
    for (int q = 0; q < m; ++q) {
        const float r = member_dist(xj, mem[q]);
        const float ratio = fmaxf(r, tiny) * frcp(fmaxf(__uint_as_float(dmin_bits[q]), tiny));
        rmin = fminf(rmin, ratio);
        sx += __expf(1.0f - ratio);
        if (r < r1) {
            r2 = r1;
            r1 = r;
        } else if (r < r2) {
            r2 = r;
        }
        const float rho = corr(p.two_nu, cnu * r);
        sr += rho;
        sr2 += rho * rho;
        sd += r;
    }
    if (m == 1) r2 = r1;
    const float inv_m = frcp((float)m);
    f[0] = __logf(fmaxf(r1, tiny)) - log_r10;
    f[1] = (float)s * frcp((float)C);
    f[2] = corr(p.two_nu, cnu * r1);
    f[3] = r1 * inv_ell;
    f[4] = corr(p.two_nu, cnu * r2);
    f[5] = sr * inv_m;
    f[6] = sr2 * inv_m;
    f[7] = sd * inv_m * inv_ell;
    f[8] = (float)m * (1.0f / 64.0f);
    f[9] = s == 0 ? 1.0f : 0.0f;
    f[10] = __logf(1.0f + (float)s) * frcp(__logf(1.0f + (float)C));
    f[11] = __logf(rmin);
    f[12] = sx * inv_m;
#pragma unroll
    for (int q = 13; q < kF; ++q) f[q] = 0.0f;
}

__global__ __launch_bounds__(kGrpThreads) void screen_group_kernel(GroupScreenArgs p) {
    __shared__ MlpLds sh_w;
    __shared__ double sh_m[kGroupScreenMaxMembers][3];
    __shared__ __align__(16) uint16_t sh_x[kGrpChunk][kF];
    __shared__ float sh_z[kGroupScreenMaxPool];
    __shared__ int sh_cnt[kGrpSlots * kGrpWaves];
    __shared__ float sh_drop[kGrpWaves];
    __shared__ uint32_t sh_dmin[kGroupScreenMaxMembers];  // bits of each member's nearest-candidate distance
    const int tid = threadIdx.x, lane = lane_id(), wib = tid >> 6;
    const int cl = lane & 15, g4 = lane >> 4;
    const int64_t g = blockIdx.x;
    const int dim = p.dim;
    if (p.mode == 0) stage_mlp(sh_w, p.params, p.params_bf16);
    // group, pool length and member coordinates; a bad group (member range or
    // id, pool length or pool id out of range) is reported, not read past
    const int64_t b = p.group_ptr[g], e = p.group_ptr[g + 1];
    const int64_t m64 = e - b;
    const int C = p.pool_len[g];
    bool bad = b < 0 || e > p.n_members || m64 < 1 || m64 > kGroupScreenMaxMembers || C < 0 || C > p.stride ||
               C > kGroupScreenMaxPool;
    const int m = bad ? 0 : (int)m64;
    if (tid < kGroupScreenMaxMembers) sh_dmin[tid] = 0x7F800000u;  // +inf
    if (tid < m) {
        const int32_t id = p.members[b + tid];
        if (id < 0 || (int64_t)id >= p.n) {
            bad = true;
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) sh_m[tid][c] = c < dim ? p.pts[(int64_t)id * dim + c] : 0.0;
        }
    }
    for (int i = 0; i < kGrpSlots && !bad; ++i) {
        const int s = tid + kGrpThreads * i;
        if (s < C) {
            const int32_t q = p.pool[g * p.stride + s];
            if (q < 0 || (int64_t)q >= p.n) bad = true;
        }
    }
    if (__syncthreads_or(bad ? 1 : 0)) {
        if (tid == 0 && p.mode == 0) {
            p.kept_len[g] = 0;
            p.fallback[g] = 3;
        }
        return;
    }
    auto load_x = [&](int s, double xj[3]) {
        const int64_t q = p.pool[g * p.stride + s];
#pragma unroll
        for (int c = 0; c < 3; ++c) xj[c] = c < dim ? p.pts[q * dim + c] : 0.0;
    };
    // log of the nearest member distance of slot 0 (every thread computes it)
    float log_r10 = 0.0f;
    if (C > 0) {
        double x0[3];
        load_x(0, x0);
        float r1 = INFINITY;
        for (int q = 0; q < m; ++q) r1 = fminf(r1, member_dist(x0, sh_m[q]));
        log_r10 = __logf(fmaxf(r1, 1e-9f * (float)p.ell));
    }
    // each member's nearest-candidate distance: per member the minimum over a
    // thread's slots, over the wave (non-negative floats order as their bits),
    // then over the waves by LDS atomics
    {
        double xs[kGrpSlots][3];
#pragma unroll
        for (int i = 0; i < kGrpSlots; ++i) {
            const int s = tid + kGrpThreads * i;
            if (s < C) load_x(s, xs[i]);
        }
        for (int q = 0; q < m; ++q) {
            uint32_t best = 0x7F800000u;
#pragma unroll
            for (int i = 0; i < kGrpSlots; ++i)
                if (tid + kGrpThreads * i < C) best = min(best, __float_as_uint(member_dist(xs[i], sh_m[q])));
            best = wave_min32(best);
            if (lane == 0) atomicMin(&sh_dmin[q], best);
        }
    }
    __syncthreads();
    for (int c0 = 0; c0 < C; c0 += kGrpChunk) {
        for (int sl = tid; sl < kGrpChunk; sl += kGrpThreads) {
            const int s = c0 + sl;
            float f[kF];
            if (s < C) {
                double xj[3];
                load_x(s, xj);
                group_candidate_features(p, sh_m, m, sh_dmin, xj, s, C, log_r10, f);
                if (p.feats)
#pragma unroll
                    for (int q = 0; q < kF; ++q) p.feats[(g * p.stride + s) * kF + q] = f[q];
            } else {
                // rows past the pool: finite, and their logits are never read
#pragma unroll
                for (int q = 0; q < kF; ++q) f[q] = 0.0f;
            }
            uint4* row = reinterpret_cast<uint4*>(&sh_x[sl][0]);
            row[0] = uint4{pack_bf16x2(f[0], f[1]), pack_bf16x2(f[2], f[3]), pack_bf16x2(f[4], f[5]),
                           pack_bf16x2(f[6], f[7])};
            row[1] = uint4{pack_bf16x2(f[8], f[9]), pack_bf16x2(f[10], f[11]), pack_bf16x2(f[12], f[13]),
                           pack_bf16x2(f[14], f[15])};
        }
        __syncthreads();
        if (p.mode == 0) {
            // this chunk's 32 tiles of 16 candidates, 8 per wave, 2 at a time
            constexpr int kTilesPerWave = kGrpChunk / 16 / kGrpWaves;
            const int ntiles = (min(C - c0, kGrpChunk) + 15) >> 4;
            for (int t0 = wib * kTilesPerWave; t0 < (wib + 1) * kTilesPerWave && t0 < ntiles; t0 += 2) {
                short4_t xb[2];
                float z[2];
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    xb[t] = __builtin_bit_cast(short4_t, *reinterpret_cast<const uint2*>(&sh_x[(t0 + t) * 16 + cl][4 * g4]));
                mlp_tiles_lds<2>(sh_w, xb, z, lane);
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    if (g4 == 0) sh_z[c0 + (t0 + t) * 16 + cl] = z[t];
            }
        }
        __syncthreads();
    }
    if (p.mode == 1) return;
    // keys: the order-preserving image of the logit (equal logits, equal
    // keys); 0 marks an empty slot.  Slot s = tid + 256 i.
    uint32_t key[kGrpSlots];
    float zz[kGrpSlots];
#pragma unroll
    for (int i = 0; i < kGrpSlots; ++i) {
        const int s = tid + kGrpThreads * i;
        zz[i] = s < C ? sh_z[s] : 0.0f;
        key[i] = s < C ? mono_key(zz[i]) : 0u;
        if (p.logits && s < C) p.logits[g * p.stride + s] = zz[i];
    }
    const int keep = p.keep;
    // kept = key > thr, plus the first `need` slots (in slot order) with key == thr
    uint32_t thr = 0u;
    int cnt_ge = 0;  // keys >= thr
    if (C > keep) {
        // the largest thr with at least `keep` keys at or above it; stops early
        // at a midpoint with exactly `keep` keys at or above it
        uint32_t lo = 0u, hi = 0xFFFFFFFFu;
        cnt_ge = C;
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2u + 1u;
            int cw = 0;
#pragma unroll
            for (int i = 0; i < kGrpSlots; ++i) cw += __popcll(__ballot(key[i] >= mid));
            if (lane == 0) sh_cnt[wib] = cw;
            __syncthreads();
            int cnt = 0;
#pragma unroll
            for (int w = 0; w < kGrpWaves; ++w) cnt += sh_cnt[w];
            __syncthreads();
            if (cnt >= keep) {
                lo = mid;
                cnt_ge = cnt;
                if (cnt == keep) break;
            } else {
                hi = mid - 1u;
            }
        }
        thr = lo;
    }
    // ties at thr: per slot chunk (i, wave) -- slots 256 i + 64 w .. +63 --
    // the number of keys equal to thr, so a slot's rank among the ties in
    // slot order is the count of every chunk before it plus the lanes below
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t me[kGrpSlots];
#pragma unroll
    for (int i = 0; i < kGrpSlots; ++i) {
        me[i] = __ballot(key[i] != 0u && key[i] == thr);
        if (lane == 0) sh_cnt[i * kGrpWaves + wib] = __popcll(me[i]);
    }
    __syncthreads();
    int cnt_eq = 0;
    for (int c = 0; c < kGrpSlots * kGrpWaves; ++c) cnt_eq += sh_cnt[c];
    const int need = C > keep ? keep - (cnt_ge - cnt_eq) : 0;
    bool kp[kGrpSlots];
    float drop = 0.0f;
#pragma unroll
    for (int i = 0; i < kGrpSlots; ++i) {
        int rank = __popcll(me[i] & below);
        for (int c = 0; c < i * kGrpWaves + wib; ++c) rank += sh_cnt[c];
        kp[i] = key[i] > thr || (key[i] != 0u && key[i] == thr && rank < need);
        if (key[i] != 0u && !kp[i]) drop += frcp(1.0f + __expf(-zz[i]));
    }
    drop = wave_sum_f32(drop);
    __syncthreads();
    if (lane == 0) sh_drop[wib] = drop;
    // kept candidates in slot order: a chunk's offset counts the kept slots of
    // every chunk before it in (i, w) order
    uint64_t mk[kGrpSlots];
#pragma unroll
    for (int i = 0; i < kGrpSlots; ++i) {
        mk[i] = __ballot(kp[i]);
        if (lane == 0) sh_cnt[i * kGrpWaves + wib] = __popcll(mk[i]);
    }
    __syncthreads();
    float tot = 0.0f;
#pragma unroll
    for (int w = 0; w < kGrpWaves; ++w) tot += sh_drop[w];
    const bool fb = C > keep && tot > p.fb_thr;
    int total = 0;
    for (int c = 0; c < kGrpSlots * kGrpWaves; ++c) total += sh_cnt[c];
#pragma unroll
    for (int i = 0; i < kGrpSlots; ++i) {
        const int s = tid + kGrpThreads * i;
        if (kp[i]) {
            int off = 0;
            for (int c = 0; c < i * kGrpWaves + wib; ++c) off += sh_cnt[c];
            p.kept[g * keep + off + __popcll(mk[i] & below)] = p.pool[g * p.stride + s];
        }
    }
    for (int q = total + tid; q < keep; q += kGrpThreads) p.kept[g * keep + q] = -1;
    if (tid == 0) {
        p.kept_len[g] = total;
        p.fallback[g] = fb ? 1 : 0;
    }
}

hipError_t launch_screen_groups(const GroupScreenArgs& a, hipStream_t s) {
    if (a.n_groups == 0) return hipSuccess;
    hipLaunchKernelGGL(screen_group_kernel, dim3((unsigned)a.n_groups), dim3(kGrpThreads), 0, s, a);
    return hipGetLastError();
}

int mlp_nparams() { return kNParams; }
int64_t mlp_grad_nparts(int64_t n_rows) { return (n_rows + kTrainTilesPerWave * 16 - 1) / (kTrainTilesPerWave * 16); }

hipError_t launch_mlp_grad(const MlpTrainArgs& a, float* grad, hipStream_t s) {
    const int64_t parts = mlp_grad_nparts(a.n_rows);
    if (parts > 0) hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)parts), dim3(64), 0, s, a);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((kNParams + 1 + 255) / 256), dim3(256), 0, s, a.partials,
                       (int)parts, grad);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// allocation-free gradient: the per-wave partials in a file-scope device array
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocParts =
    (kMlpGradNoAllocMaxRows + kTrainTilesPerWave * 16 - 1) / (kTrainTilesPerWave * 16);
static __device__ __align__(256) float scratch[kNoAllocParts * (kNParams + 1)];

// The device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array).  In host code the
// array's name is only a stand-in: kernels get this address instead.
static hipError_t scratch_on_current_device(float** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static float* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<float*>(ptr);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_mlp_grad_noalloc(MlpTrainArgs a, float* grad, hipStream_t s) {
    if (a.n_rows > kMlpGradNoAllocMaxRows) return hipErrorInvalidValue;
    float* ws = nullptr;
    const hipError_t e = scratch_on_current_device(&ws);
    if (e != hipSuccess) return e;
    // every partial slot of the launched waves is written before it is summed,
    // so the array needs no clearing between calls
    a.partials = ws;
    return launch_mlp_grad(a, grad, s);
}

hipError_t launch_mlp_forward(const MlpTrainArgs& a, float* z, hipStream_t s) {
    const int64_t parts = mlp_grad_nparts(a.n_rows);
    if (parts > 0) hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)parts), dim3(64), 0, s, a, z);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, uint16_t* pb, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, pb, g, m, v, n, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* p, uint16_t* pb, int n, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, pb, n);
    return hipGetLastError();
}

}  // namespace csel
