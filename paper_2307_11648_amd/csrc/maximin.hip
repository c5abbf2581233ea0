// maximin.hip -- reverse-maximin ordering on the GPU (Sec. 2.2, eq. maximin,
// p = 1): the last position holds point 0; every earlier position holds the
// remaining point farthest from the points already placed after it (ties to
// the smaller id), and ell[pos] is that distance.
//
// The sequential rule places one point at a time.  With D_j the squared
// distance of a remaining point j to the placed points and the key (D_j, -j),
// take the remaining points sorted by decreasing key, q_1, q_2, ...: while
// none of q_1..q_{i-1} lies closer to q_i than sqrt(D_{q_i}), placing them
// leaves D_{q_i} unchanged and can only lower every other key, so q_i is the
// sequential rule's next pick.  A round places that prefix of the sorted
// order, then lowers D of every remaining point within sqrt(D_p) of a placed
// point p.  (About 3,000 rounds for 1e6 points.)
//
// Candidates.  A buffer holds every remaining point whose key is at least a
// threshold key theta (at most kMmCap points).  Keys only decrease, so the
// buffer's points still at or above theta, sorted, are exactly the top of the
// order; each round takes its prefix from them, and once none is left the
// buffer is refilled: theta comes from a radix descent over the 96-bit keys
// (D's bits, then the complement of the id), 11 bits per pass, each pass a
// histogram of the remaining points that share the digits fixed so far.
//
// Grid.  Levels l = 0..L with 2^l cells per dimension over the bounding box
// (a counting sort by cell: ids and coordinates per level).  The update for a
// placed point p scans the cells covering its ball of radius sqrt(D_p) on the
// finest level whose cells are at least that wide.
//
// Squared distances are summed coordinate by coordinate in order, without
// fused multiply-adds, as the definition reads; D is lowered with an atomic
// minimum on its bits (non-negative doubles order as their bit patterns), so
// the result does not depend on the order of the updates.  The host drives
// the rounds in batches and reads the number of points left after each batch.
#include <rocprim/device/device_scan.hpp>

#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

typedef unsigned __int128 u128;

constexpr int kMmCap = 2048;            // candidate buffer (points)
constexpr int kMmMin = 1024;            // a refill stops its descent once this many keys sit above theta
constexpr int kMmRoundThreads = 1024;   // the round kernel's one workgroup
constexpr int kMmBins = 2048;           // 11-bit radix digits
constexpr int kMmLastDigit = 8;         // digits 0..8 cover the 95 significant key bits
constexpr int kMmMaxLevels = 25;
constexpr int kMmStepsPerBatch = 32;    // rounds launched between two reads of the progress counter
constexpr int kMmGridBlocks = 512;      // grid-stride kernels over all points
constexpr int kMmLoadBatch = 8;         // points per thread whose loads a refill pass issues together
constexpr int kMmHash = 4096;           // buckets of the round's conflict grid
constexpr int kMmPassesPerStep = 2;     // histogram passes launched per round (a refill usually needs two)

struct MmLevel {
    int32_t G;         // cells per dimension (2^l)
    int64_t cells;     // G^dim
    int64_t cell_off;  // offset of the level's cell_start (cells + 1 entries)
    int64_t pt_off;    // offset of the level's points (n per level)
};

// device-resident control block
struct MmState {
    u128 prefix;        // key digits fixed by the descent so far (the key shifted right)
    u128 theta;         // the buffer holds every remaining point with key >= theta
    int32_t remaining;  // points not yet placed
    int32_t pos_next;   // the next position to fill (from n - 2 down)
    int32_t nb;         // points in the buffer
    int32_t phase;      // 0: buffer usable; 1: histogram pass pending; 2: gather pending
    int32_t lvl;        // digit of the pending histogram pass
    int32_t above;      // keys above the descent's current bin
    int32_t naccept;    // points placed by the last round
    int32_t done_hist;  // last-workgroup-done counters
    int32_t done_gather;
    int32_t overflow;   // set if a gather ever exceeded the buffer (not expected)
    int32_t rounds;     // rounds that placed points
    int32_t sorted;     // the buffer is in key order with its keys in bufD (a round wrote it)
};

struct MmArgs {
    const double* pts;
    int64_t n;
    int32_t dim;
    int32_t nlev;
    MmLevel lev[kMmMaxLevels];
    const double* prm;        // [level][3][2]: 1/h and h per dimension; then lo[3]; then hmin[level]
    const int32_t* cell_start;
    const int32_t* cell_ids;  // point ids grouped by cell, per level
    const double* cell_xyz;   // their coordinates
    uint64_t* D;              // [n] bits of the squared distance to the placed points
    int32_t* pos_of;          // [n] position of a placed point, -1 while remaining
    int32_t* buf;             // [kMmCap] candidate ids
    uint64_t* bufD;           // [kMmCap] their D bits when a round last wrote the buffer
    int32_t* acc;             // [kMmCap] points placed by the last round
    uint64_t* accD;           // [kMmCap] their D bits
    uint32_t* hist;           // [kMmBins]
    MmState* st;
    int32_t* order;
    double* ell;
};

// (x - q)^2 summed in coordinate order, products and sums rounded separately
__device__ __forceinline__ double mm_d2(const double* a, const double* q, int dim) {
#pragma clang fp contract(off)
    double e = a[0] - q[0];
    double s = e * e;
    if (dim > 1) {
        e = a[1] - q[1];
        s = s + e * e;
    }
    if (dim > 2) {
        e = a[2] - q[2];
        s = s + e * e;
    }
    return s;
}

__device__ __forceinline__ u128 mm_key(uint64_t dbits, int32_t id) {
    return ((u128)dbits << 32) | (u128)(uint32_t)~(uint32_t)id;
}
// digits: lvl 0..7 take bits [94 - 11 lvl, 84 - 11 lvl]; lvl 8 the last 7 bits, scaled by 16
__device__ __forceinline__ int mm_digit(u128 key, int lvl) {
    return lvl < kMmLastDigit ? (int)((key >> (84 - 11 * lvl)) & (u128)2047) : (int)((key & (u128)127) << 4);
}
// the key's digits above digit lvl
__device__ __forceinline__ u128 mm_prefix(u128 key, int lvl) { return key >> (95 - 11 * lvl); }
// the smallest key whose digits above lvl are `prefix` and whose digit lvl is >= b (b may be kMmBins)
__device__ __forceinline__ u128 mm_theta(u128 prefix, int lvl, int b) {
    if (lvl < kMmLastDigit) return ((prefix << 11) + (u128)b) << (84 - 11 * lvl);
    return (prefix << 7) + (u128)((b + 15) >> 4);
}

// ---------------------------------------------------------------------------
// sqrt rounded to nearest.  The device square root is within an ulp but not
// always the nearest double; the rounding is fixed with exact integer
// comparisons of squares (128-bit products of the 53-bit significands).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mm_split(double v, uint64_t& M, int& e) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const int ex = (int)((b >> 52) & 0x7FF);
    const uint64_t f = b & ((1ull << 52) - 1);
    if (ex == 0) {
        M = f;
        e = -1074;
    } else {
        M = f | (1ull << 52);
        e = ex - 1075;
    }
}
__device__ __forceinline__ int mm_bitlen(u128 x) {
    const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
    return hi ? 128 - __builtin_clzll(hi) : (lo ? 64 - __builtin_clzll(lo) : 0);
}
// sign of A 2^ea - B 2^eb for nonzero A, B below 2^120
__device__ __forceinline__ int mm_cmp2(u128 A, int ea, u128 B, int eb) {
    const int la = mm_bitlen(A), lb = mm_bitlen(B);
    if (ea + la != eb + lb) return ea + la > eb + lb ? 1 : -1;
    if (la < lb)
        A <<= (lb - la);
    else
        B <<= (la - lb);
    return A > B ? 1 : (A < B ? -1 : 0);
}
// sign of a^2 - D, and of (a + u/2)^2 - D with u the spacing above a (a, D > 0)
__device__ __forceinline__ int mm_sq_cmp(double a, double D) {
    uint64_t Ma, MD;
    int ea, eD;
    mm_split(a, Ma, ea);
    mm_split(D, MD, eD);
    return mm_cmp2((u128)Ma * Ma, 2 * ea, (u128)MD, eD);
}
__device__ __forceinline__ int mm_mid_cmp(double a, double D) {
    uint64_t Ma, MD;
    int ea, eD;
    mm_split(a, Ma, ea);
    mm_split(D, MD, eD);
    const u128 m = (u128)(2 * Ma + 1);
    return mm_cmp2(m * m, 2 * ea - 2, (u128)MD, eD);
}
__device__ double mm_sqrt_rn(double D) {
    const double y = sqrt(D);
    if (!(D > 0.0) || !(D <= 1.7976931348623157e308)) return y;
    // b: the largest double whose square is at most D
    uint64_t b = (uint64_t)__double_as_longlong(y);
    for (int it = 0; it < 4 && mm_sq_cmp(__longlong_as_double((long long)b), D) > 0; ++it) --b;
    for (int it = 0; it < 4 && mm_sq_cmp(__longlong_as_double((long long)(b + 1)), D) <= 0; ++it) ++b;
    // up when the midpoint above b lies below sqrt(D) (an exact tie cannot occur)
    if (mm_mid_cmp(__longlong_as_double((long long)b), D) < 0) ++b;
    return __longlong_as_double((long long)b);
}

// ordered image of a double (any sign) in uint64, for the bounding box
__device__ __forceinline__ uint64_t mm_ord(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double mm_unord(uint64_t u) {
    return __longlong_as_double((long long)((u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u));
}

__device__ __forceinline__ int mm_cell1(double x, double lo, double invh, int G) {
    const double t = (x - lo) * invh;
    int c = t > 0.0 ? (int)t : 0;  // floor for t >= 0
    return c < G ? c : G - 1;
}

// ---------------------------------------------------------------------------
// grid build
// ---------------------------------------------------------------------------
__global__ void mm_bbox_init_kernel(uint64_t* bb) {
    if (threadIdx.x < 3) {
        bb[threadIdx.x] = ~0ull;
        bb[3 + threadIdx.x] = 0ull;
    }
}

__global__ __launch_bounds__(256) void mm_bbox_kernel(const double* __restrict__ pts, int64_t n, int dim,
                                                      uint64_t* bb) {
    uint64_t mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < dim; ++k) {
            const uint64_t o = mm_ord(pts[i * dim + k]);
            mn[k] = o < mn[k] ? o : mn[k];
            mx[k] = o > mx[k] ? o : mx[k];
        }
    }
    for (int k = 0; k < dim; ++k) {
        atomicMin((unsigned long long*)&bb[k], (unsigned long long)mn[k]);
        atomicMax((unsigned long long*)&bb[3 + k], (unsigned long long)mx[k]);
    }
}

// per level and dimension 1/h and h (a zero extent puts every point in cell
// 0 of that dimension), the box's lower corner, and per level the smallest h
// over the dimensions with an extent
__global__ void mm_params_kernel(const uint64_t* bb, MmArgs a, double* prm) {
    if (threadIdx.x != 0) return;
    double lo[3] = {0.0, 0.0, 0.0}, ext[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < a.dim; ++k) {
        lo[k] = mm_unord(bb[k]);
        ext[k] = mm_unord(bb[3 + k]) - lo[k];
    }
    for (int l = 0; l < a.nlev; ++l) {
        double hmin = INFINITY;
        for (int k = 0; k < 3; ++k) {
            const double G = (double)a.lev[l].G;
            const bool flat = !(ext[k] > 0.0) || k >= a.dim;
            prm[(l * 3 + k) * 2 + 0] = flat ? 0.0 : G / ext[k];
            prm[(l * 3 + k) * 2 + 1] = flat ? 1.0 : ext[k] / G;
            if (!flat) hmin = fmin(hmin, ext[k] / G);
        }
        prm[a.nlev * 6 + 3 + l] = hmin;
    }
    for (int k = 0; k < 3; ++k) prm[a.nlev * 6 + k] = lo[k];
}

__device__ __forceinline__ int64_t mm_cell(const double* x, const double* prm, int l, int dim, int G, int nlev) {
    const double* lo = prm + nlev * 6;
    int64_t c = 0;
    for (int k = dim - 1; k >= 0; --k) c = c * G + mm_cell1(x[k], lo[k], prm[(l * 3 + k) * 2], G);
    return c;
}

__global__ __launch_bounds__(256) void mm_fill_kernel(int32_t* v, int64_t m, int32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = value;
}

// Coarse levels (at most kMmLdsCells cells) count and place their points
// through per-workgroup tallies in LDS, each workgroup taking a contiguous
// chunk of the points: a million atomic increments of a handful of counters
// would otherwise serialize.
constexpr int kMmLdsCells = 4096;

__global__ __launch_bounds__(256) void mm_count_kernel(MmArgs a, int l, int32_t* counts) {
    __shared__ int32_t h[kMmLdsCells];
    const MmLevel L = a.lev[l];
    const bool lds = L.cells <= kMmLdsCells;
    const int tid = threadIdx.x;
    if (lds) {
        for (int c = tid; c < L.cells; c += 256) h[c] = 0;
        __syncthreads();
    }
    const int64_t chunk = (a.n + gridDim.x - 1) / gridDim.x;
    const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = min(a.n, j0 + chunk);
    for (int64_t j = j0 + tid; j < j1; j += 256) {
        const int64_t c = mm_cell(a.pts + j * a.dim, a.prm, l, a.dim, L.G, a.nlev);
        if (lds)
            atomicAdd(&h[c], 1);
        else
            atomicAdd(&counts[c], 1);
    }
    if (lds) {
        __syncthreads();
        for (int c = tid; c < L.cells; c += 256)
            if (h[c]) atomicAdd(&counts[c], h[c]);
    }
}

__global__ __launch_bounds__(256) void mm_scatter_kernel(MmArgs a, int l, int32_t* fill, int32_t* cell_ids,
                                                         double* cell_xyz) {
    __shared__ int32_t h[kMmLdsCells];
    const MmLevel L = a.lev[l];
    const bool lds = L.cells <= kMmLdsCells;
    const int tid = threadIdx.x;
    const int64_t chunk = (a.n + gridDim.x - 1) / gridDim.x;
    const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = min(a.n, j0 + chunk);
    if (lds) {
        // this chunk's count per cell, then one reservation per cell
        for (int c = tid; c < L.cells; c += 256) h[c] = 0;
        __syncthreads();
        for (int64_t j = j0 + tid; j < j1; j += 256)
            atomicAdd(&h[mm_cell(a.pts + j * a.dim, a.prm, l, a.dim, L.G, a.nlev)], 1);
        __syncthreads();
        for (int c = tid; c < L.cells; c += 256)
            if (h[c]) h[c] = atomicAdd(&fill[c], h[c]);
        __syncthreads();
    }
    for (int64_t j = j0 + tid; j < j1; j += 256) {
        const double* x = a.pts + j * a.dim;
        const int64_t c = mm_cell(x, a.prm, l, a.dim, L.G, a.nlev);
        const int32_t slot = lds ? atomicAdd(&h[c], 1) : atomicAdd(&fill[c], 1);
        const int64_t at = L.pt_off + a.cell_start[L.cell_off + c] + slot;
        cell_ids[at] = (int32_t)j;
        for (int k = 0; k < a.dim; ++k) cell_xyz[at * a.dim + k] = x[k];
    }
}

// D_j = |x_j - x_0|^2; point 0 placed last
__global__ __launch_bounds__(256) void mm_init_kernel(MmArgs a) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < a.n) {
        const double d = mm_d2(a.pts + j * a.dim, a.pts, a.dim);
        a.D[j] = (uint64_t)__double_as_longlong(d);
        a.pos_of[j] = j == 0 ? (int32_t)(a.n - 1) : -1;
    }
    if (j == 0) {
        a.order[a.n - 1] = 0;
        a.ell[a.n - 1] = INFINITY;
        MmState s{};
        s.prefix = 0;
        s.theta = 0;
        s.remaining = (int32_t)(a.n - 1);
        s.pos_next = (int32_t)(a.n - 2);
        s.phase = a.n > 1 ? 1 : 0;
        *a.st = s;
    }
    if (j < kMmBins) a.hist[j] = 0u;
}

// ---------------------------------------------------------------------------
// refill: one histogram pass of the radix descent; the last workgroup to
// finish reads the histogram and either fixes theta or descends one digit
// ---------------------------------------------------------------------------
// h[dig] += 1 for the active lanes of a wave (called by every lane): lanes
// sharing a digit add once through their first lane (up to four distinct
// digits), the rest one by one -- the first digits of the keys are mostly
// equal, and thousands of increments of one LDS word would serialize
__device__ __forceinline__ void mm_hist_add(uint32_t* h, int dig, bool act) {
    const int lane = lane_id();
    uint64_t pending = __ballot(act);
    for (int it = 0; it < 4 && pending; ++it) {
        const int leader = (int)__builtin_ctzll(pending);
        const int dl = __shfl(dig, leader, kWave);
        const uint64_t m = __ballot(act && dig == dl) & pending;
        if (lane == leader) atomicAdd(&h[dl], (uint32_t)__popcll(m));
        if ((m >> lane) & 1ull) act = false;
        pending &= ~m;
    }
    if (act) atomicAdd(&h[dig], 1u);
}

__global__ __launch_bounds__(256) void mm_hist_kernel(MmArgs a) {
    __shared__ uint32_t h[kMmBins];
    __shared__ uint32_t tsum[256];
    __shared__ int sh_last;
    MmState* st = a.st;
    if (st->phase != 1) return;
    const int lvl = st->lvl;
    const u128 prefix = st->prefix;
    const int tid = threadIdx.x;
    for (int b = tid; b < kMmBins; b += 256) h[b] = 0u;
    __syncthreads();
    // kMmLoadBatch points per thread per pass, their loads issued together
    // (a workgroup-uniform loop: every thread takes the same passes)
    for (int64_t b0 = (int64_t)blockIdx.x * 256 * kMmLoadBatch; b0 < a.n; b0 += (int64_t)gridDim.x * 256 * kMmLoadBatch) {
        const int64_t j0 = b0 + tid;
        int32_t pv[kMmLoadBatch];
        uint64_t dv[kMmLoadBatch];
#pragma unroll
        for (int u = 0; u < kMmLoadBatch; ++u) {
            const int64_t j = j0 + (int64_t)u * 256;
            pv[u] = j < a.n ? a.pos_of[j] : 0;
            dv[u] = j < a.n ? a.D[j] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kMmLoadBatch; ++u) {
            const int64_t j = j0 + (int64_t)u * 256;
            const u128 key = mm_key(dv[u], (int32_t)j);
            const bool act = j < a.n && pv[u] < 0 && mm_prefix(key, lvl) == prefix;
            mm_hist_add(h, act ? mm_digit(key, lvl) : 0, act);
        }
    }
    __syncthreads();
    for (int b = tid; b < kMmBins; b += 256)
        if (h[b]) atomicAdd(&a.hist[b], h[b]);
    // every wave's atomics complete, then one device-scope release per
    // workgroup before it counts itself done (a fence from every thread would
    // write back the L2 thousands of times per pass)
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        sh_last = atomicAdd(&st->done_hist, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!sh_last) return;
    __threadfence();
    // the last workgroup: bins [8 tid, 8 tid + 8) per thread, suffix sums from the top
    uint32_t c[8];
    uint32_t mine = 0;
    for (int q = 0; q < 8; ++q) {
        c[q] = __hip_atomic_load(&a.hist[8 * tid + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        mine += c[q];
    }
    tsum[tid] = mine;
    __syncthreads();
    // exclusive suffix sum over threads (threads above tid)
    uint32_t above_me = 0;
    for (int t = tid + 1; t < 256; ++t) above_me += tsum[t];
    const int64_t A = st->above;
    // the overflow bin: the largest b with A + sum_{b' >= b} h[b'] > kMmCap
    int64_t cum = A + above_me;  // keys above my chunk
    int ob = -1;
    int64_t cum_above_ob = 0;
    for (int q = 7; q >= 0; --q) {
        if (cum + c[q] > kMmCap) {
            ob = 8 * tid + q;
            cum_above_ob = cum;
            break;
        }
        cum += c[q];
    }
    // only the chunk holding the transition finds an overflow bin whose keys
    // above it fit (a lower chunk sees a cumulative count already past the cap)
    const bool first = ob >= 0 && cum_above_ob <= kMmCap;
    __syncthreads();
    if (first) {
        if (cum_above_ob >= kMmMin || lvl == kMmLastDigit) {
            st->theta = mm_theta(prefix, lvl, ob + 1);
            st->phase = 2;
        } else {
            st->prefix = (prefix << 11) | (u128)ob;
            st->above = (int32_t)cum_above_ob;
            st->lvl = lvl + 1;
        }
    }
    if (tid == 0 && A + above_me + mine <= kMmCap) {
        // thread 0's chunk is the lowest: every key with this prefix fits
        st->theta = mm_theta(prefix, lvl, 0);
        st->phase = 2;
    }
    for (int q = 0; q < 8; ++q) a.hist[8 * tid + q] = 0u;
    if (tid == 0) st->done_hist = 0;
}

// refill: every remaining point with key >= theta into the buffer
__global__ __launch_bounds__(256) void mm_gather_kernel(MmArgs a) {
    __shared__ int sh_last, sh_n, sh_base;
    MmState* st = a.st;
    if (st->phase != 2) return;
    const u128 theta = st->theta;
    const int tid = threadIdx.x;
    // (a workgroup-uniform loop: every thread takes the same passes)
    for (int64_t b0 = (int64_t)blockIdx.x * 256 * kMmLoadBatch; b0 < a.n; b0 += (int64_t)gridDim.x * 256 * kMmLoadBatch) {
        const int64_t j0 = b0 + tid;
        int32_t pv[kMmLoadBatch];
        uint64_t dv[kMmLoadBatch];
#pragma unroll
        for (int u = 0; u < kMmLoadBatch; ++u) {
            const int64_t j = j0 + (int64_t)u * 256;
            pv[u] = j < a.n ? a.pos_of[j] : 0;
            dv[u] = j < a.n ? a.D[j] : 0ull;
        }
        // the workgroup's selected points take one range of the buffer
        int loc[kMmLoadBatch];
        if (tid == 0) sh_n = 0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kMmLoadBatch; ++u) {
            const int64_t j = j0 + (int64_t)u * 256;
            loc[u] = (j < a.n && pv[u] < 0 && mm_key(dv[u], (int32_t)j) >= theta) ? atomicAdd(&sh_n, 1) : -1;
        }
        __syncthreads();
        if (tid == 0) sh_base = sh_n > 0 ? atomicAdd(&st->nb, sh_n) : 0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kMmLoadBatch; ++u) {
            if (loc[u] < 0) continue;
            const int slot = sh_base + loc[u];
            if (slot < kMmCap)
                a.buf[slot] = (int32_t)(j0 + (int64_t)u * 256);
            else
                st->overflow = 1;
        }
        __syncthreads();  // sh_n is reset for the next pass
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's buffer stores are done
    __syncthreads();
    if (tid == 0) {
        __threadfence();  // one release per workgroup
        sh_last = atomicAdd(&st->done_gather, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!sh_last || tid != 0) return;
    __threadfence();
    st->done_gather = 0;
    st->sorted = 0;
    st->phase = 0;
    st->lvl = 0;
    st->prefix = 0;
    st->above = 0;
    if (st->nb > kMmCap) st->nb = kMmCap;
}

// ---------------------------------------------------------------------------
// one round: sort the buffer's valid points by key, place the prefix that no
// earlier point of it conflicts with, keep the rest
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool mm_before(uint64_t da, uint32_t ia, uint64_t db, uint32_t ib) {
    return da > db || (da == db && ia < ib);
}

// bitonic sort of sk/si[0 .. P) (P a power of two <= 2048) by descending key,
// by the whole workgroup: element i = tid + 1024 k (k = 0, 1) in registers;
// partners within a wave by shuffles, across waves through LDS
__device__ void mm_sort_desc(uint64_t* sk, uint32_t* si, int P, int tid) {
    uint64_t kd[2];
    uint32_t ki[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = tid + k * kMmRoundThreads;
        kd[k] = i < P ? sk[i] : 0ull;
        ki[k] = i < P ? si[i] : 0xFFFFFFFFu;
    }
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= kMmRoundThreads) {
                // i and i + 1024 in one thread (size 2048: the lower index holds the larger key)
                if (mm_before(kd[1], ki[1], kd[0], ki[0])) {
                    const uint64_t tk = kd[0];
                    kd[0] = kd[1];
                    kd[1] = tk;
                    const uint32_t ti = ki[0];
                    ki[0] = ki[1];
                    ki[1] = ti;
                }
                continue;
            }
            uint64_t od[2];
            uint32_t oi[2];
            if (stride >= kWave) {
                __syncthreads();  // the previous exchange's reads are done
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int i = tid + k * kMmRoundThreads;
                    if (i < P) {
                        sk[i] = kd[k];
                        si[i] = ki[k];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int i = tid + k * kMmRoundThreads;
                    od[k] = i < P ? sk[i ^ stride] : 0ull;
                    oi[k] = i < P ? si[i ^ stride] : 0xFFFFFFFFu;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const uint32_t lo = __shfl_xor((uint32_t)kd[k], stride, kWave);
                    const uint32_t hi = __shfl_xor((uint32_t)(kd[k] >> 32), stride, kWave);
                    od[k] = ((uint64_t)hi << 32) | lo;
                    oi[k] = __shfl_xor(ki[k], stride, kWave);
                }
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int i = tid + k * kMmRoundThreads;
                if (i >= P) continue;
                const bool lower = (i & stride) == 0, desc = (i & size) == 0;
                const bool keep = (lower == desc) ? !mm_before(od[k], oi[k], kd[k], ki[k])
                                                  : !mm_before(kd[k], ki[k], od[k], oi[k]);
                if (!keep) {
                    kd[k] = od[k];
                    ki[k] = oi[k];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = tid + k * kMmRoundThreads;
        if (i < P) {
            sk[i] = kd[k];
            si[i] = ki[k];
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kMmRoundThreads) void mm_round_kernel(MmArgs a) {
    extern __shared__ __align__(16) unsigned char mm_smem[];
    uint64_t* sk = reinterpret_cast<uint64_t*>(mm_smem);               // [kMmCap] D bits
    uint32_t* si = reinterpret_cast<uint32_t*>(sk + kMmCap);           // [kMmCap] ids (-1 pads)
    double* sx = reinterpret_cast<double*>(si + kMmCap);               // [kMmCap][3]
    int32_t* hcnt = reinterpret_cast<int32_t*>(sx + 3 * kMmCap);         // [kMmHash + 1] bucket starts
    int32_t* hfill = hcnt + (kMmHash + 1);                               // [kMmHash] fill counters
    int32_t* hidx = hfill + kMmHash;                                     // [kMmCap] candidates by bucket
    int32_t* hsum = hidx + kMmCap;                                       // [1024] per-thread totals
    __shared__ int sh_cnt, sh_first, sh_nu, sh_nc;
    __shared__ int sh_tot[2 * (kMmRoundThreads / kWave)][2];
    MmState* st = a.st;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid / kWave;
    constexpr int kWaves = kMmRoundThreads / kWave;
    const int phase = st->phase, nb = st->nb, remaining = st->remaining;
    const bool sorted = st->sorted != 0;
    const u128 theta = st->theta;
    const int dim = a.dim;
    __syncthreads();
    if (tid == 0) st->naccept = 0;
    if (phase != 0 || nb == 0 || remaining == 0) return;
    int nv;
    if (!sorted) {
        // a freshly gathered buffer: its valid points, then a full sort
        if (tid == 0) sh_cnt = 0;
        __syncthreads();
        for (int t = tid; t < nb; t += kMmRoundThreads) {
            const int32_t id = a.buf[t];
            if (a.pos_of[id] >= 0) continue;
            const uint64_t d = a.D[id];
            if (mm_key(d, id) >= theta) {
                const int s = atomicAdd(&sh_cnt, 1);
                sk[s] = d;
                si[s] = (uint32_t)id;
            }
        }
        __syncthreads();
        nv = sh_cnt;
        int P = 1;
        while (P < nv) P <<= 1;
        for (int t = nv + tid; t < P; t += kMmRoundThreads) {
            sk[t] = 0ull;
            si[t] = 0xFFFFFFFFu;
        }
        __syncthreads();
        mm_sort_desc(sk, si, P, tid);
    } else {
        // the buffer as the last round left it, in key order: the entries
        // whose D is unchanged keep that order (a stable compaction); the
        // few whose D the update lowered are sorted apart and merged in by
        // binary-search ranks.  (sx is free until the coordinates load.)
        uint64_t* uk = reinterpret_cast<uint64_t*>(sx);
        uint32_t* ui = reinterpret_cast<uint32_t*>(uk + kMmCap);
        uint64_t* ck = reinterpret_cast<uint64_t*>(ui + kMmCap);
        uint32_t* ci = reinterpret_cast<uint32_t*>(ck + kMmCap);
        bool fu[2], fc[2];
        uint64_t dk[2];
        uint32_t ik[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int t = tid + k * kMmRoundThreads;
            fu[k] = fc[k] = false;
            dk[k] = 0ull;
            ik[k] = 0u;
            if (t < nb) {
                const int32_t id = a.buf[t];
                if (a.pos_of[id] < 0) {
                    const uint64_t d = a.D[id];
                    if (mm_key(d, id) >= theta) {
                        dk[k] = d;
                        ik[k] = (uint32_t)id;
                        fu[k] = d == a.bufD[t];
                        fc[k] = !fu[k];
                    }
                }
            }
        }
        // positions in buffer order (t = tid, then tid + 1024): per wave and
        // half a prefix of ballots, then the 32 (half, wave) totals in order
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
        uint64_t bu[2], bcm[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            bu[k] = __ballot(fu[k]);
            bcm[k] = __ballot(fc[k]);
            if (lane == 0) {
                sh_tot[k * kWaves + wave][0] = __popcll(bu[k]);
                sh_tot[k * kWaves + wave][1] = __popcll(bcm[k]);
            }
        }
        __syncthreads();
        if (tid == 0) {
            int au = 0, ac = 0;
            for (int q = 0; q < 2 * kWaves; ++q) {
                const int tu = sh_tot[q][0], tc = sh_tot[q][1];
                sh_tot[q][0] = au;
                sh_tot[q][1] = ac;
                au += tu;
                ac += tc;
            }
            sh_nu = au;
            sh_nc = ac;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (fu[k]) {
                const int at = sh_tot[k * kWaves + wave][0] + __popcll(bu[k] & below);
                uk[at] = dk[k];
                ui[at] = ik[k];
            }
            if (fc[k]) {
                const int at = sh_tot[k * kWaves + wave][1] + __popcll(bcm[k] & below);
                ck[at] = dk[k];
                ci[at] = ik[k];
            }
        }
        const int nu = sh_nu, nc = sh_nc;
        nv = nu + nc;
        if (nc > 0) {
            int Pc = 1;
            while (Pc < nc) Pc <<= 1;
            for (int t = nc + tid; t < Pc; t += kMmRoundThreads) {
                ck[t] = 0ull;
                ci[t] = 0xFFFFFFFFu;
            }
            __syncthreads();
            mm_sort_desc(ck, ci, Pc, tid);
        } else {
            __syncthreads();
        }
        // ranks: own index plus the entries of the other list that come first
        for (int q = tid; q < nu; q += kMmRoundThreads) {
            int lo2 = 0, hi2 = nc;  // first c not before u_q
            while (lo2 < hi2) {
                const int mid = (lo2 + hi2) >> 1;
                if (mm_before(ck[mid], ci[mid], uk[q], ui[q]))
                    lo2 = mid + 1;
                else
                    hi2 = mid;
            }
            sk[q + lo2] = uk[q];
            si[q + lo2] = ui[q];
        }
        for (int q = tid; q < nc; q += kMmRoundThreads) {
            int lo2 = 0, hi2 = nu;  // first u not before c_q
            while (lo2 < hi2) {
                const int mid = (lo2 + hi2) >> 1;
                if (mm_before(uk[mid], ui[mid], ck[q], ci[q]))
                    lo2 = mid + 1;
                else
                    hi2 = mid;
            }
            sk[q + lo2] = ck[q];
            si[q + lo2] = ci[q];
        }
        __syncthreads();
    }
    for (int t = tid; t < nv; t += kMmRoundThreads)
        for (int k = 0; k < 3; ++k) sx[t * 3 + k] = k < dim ? a.pts[(int64_t)si[t] * dim + k] : 0.0;
    if (tid == 0) sh_first = nv;
    // the first point that an earlier one lies closer to than sqrt(D).  Two
    // such points lie within sqrt(D_0) (the largest D) of each other, so the
    // candidates are hashed by cells twice that wide: the ball around a
    // candidate reaches only the neighbour cell on the near side of each
    // dimension, 2^dim cells in all.  Each candidate checks the earlier
    // candidates of those cells; a conflict found bounds the first one, and
    // larger indices stop early.  The widths carry a 1e-5 margin, so a cell
    // coordinate t may err by up to 5e-6; past 2^30 cell widths across the box
    // its rounding could exceed that, and every candidate shares one bucket
    // instead.
    const double D0 = __longlong_as_double((long long)sk[0]);
    if (nv > 1 && D0 > 0.0) {
        const double inv_w = 1.0 / (2.0 * sqrt(D0) * (1.0 + 1e-5));  // room for the rounding of t below
        const double* lo = a.prm + a.nlev * 6;
        double ext = 0.0;
        for (int k = 0; k < dim; ++k) ext = fmax(ext, a.prm[k * 2 + 1]);  // level 0: h = the extent
        const bool one_bucket = ext * inv_w > 1073741824.0;
        for (int b = tid; b <= kMmHash; b += kMmRoundThreads) hcnt[b] = 0;
        for (int b = tid; b < kMmHash; b += kMmRoundThreads) hfill[b] = 0;
        __syncthreads();
        // cell coordinate of x along k, and the side (-1 or +1) of its nearer neighbour cell
        auto cell_of = [&](const double* x, int k, int* side) -> int64_t {
            if (k >= dim || one_bucket) {
                if (side) *side = 0;
                return 0;
            }
            const double t = (x[k] - lo[k]) * inv_w;
            const double c = floor(t);
            if (side) *side = t - c < 0.5 ? -1 : 1;
            return (int64_t)c;
        };
        auto bucket = [&](int64_t c0, int64_t c1, int64_t c2) -> int {
            const uint32_t h = (uint32_t)c0 * 73856093u ^ (uint32_t)c1 * 19349663u ^ (uint32_t)c2 * 83492791u;
            return (int)(h & (kMmHash - 1));
        };
        for (int t = tid; t < nv; t += kMmRoundThreads)
            atomicAdd(&hcnt[bucket(cell_of(sx + t * 3, 0, nullptr), cell_of(sx + t * 3, 1, nullptr),
                                   cell_of(sx + t * 3, 2, nullptr))], 1);
        __syncthreads();
        // exclusive scan of the kMmHash counts (kMmHash / 1024 per thread)
        constexpr int PER = kMmHash / kMmRoundThreads;
        int loc[PER], run = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            loc[q] = run;
            run += hcnt[tid * PER + q];
        }
        hsum[tid] = run;
        __syncthreads();
        if (tid < kWave) {
            // the 1024 thread totals, scanned by one wave (16 per lane)
            int v[16], acc = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                v[q] = acc;
                acc += hsum[tid * 16 + q];
            }
            int incl = acc;
            for (int off = 1; off < kWave; off <<= 1) {
                const int o = __shfl_up(incl, off, kWave);
                if (lane >= off) incl += o;
            }
            const int excl = incl - acc;
#pragma unroll
            for (int q = 0; q < 16; ++q) hsum[tid * 16 + q] = excl + v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) hcnt[tid * PER + q] = hsum[tid] + loc[q];
        if (tid == 0) hcnt[kMmHash] = nv;
        __syncthreads();
        for (int t = tid; t < nv; t += kMmRoundThreads) {
            const int b = bucket(cell_of(sx + t * 3, 0, nullptr), cell_of(sx + t * 3, 1, nullptr),
                                 cell_of(sx + t * 3, 2, nullptr));
            hidx[atomicAdd(&hfill[b], 1) + hcnt[b]] = t;
        }
        __syncthreads();
        for (int i = 1 + tid; i < nv; i += kMmRoundThreads) {
            if (__hip_atomic_load(&sh_first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <= i) break;
            const double Di = __longlong_as_double((long long)sk[i]);
            const double* q = sx + i * 3;
            int s0, s1, s2;
            const int64_t c0 = cell_of(q, 0, &s0), c1 = cell_of(q, 1, &s1), c2 = cell_of(q, 2, &s2);
            bool conf = false;
            const int ncell = one_bucket ? 1 : 1 << dim;
            for (int cm = 0; cm < ncell && !conf; ++cm) {
                const int b = bucket(c0 + ((cm & 1) ? s0 : 0), c1 + ((cm & 2) ? s1 : 0), c2 + ((cm & 4) ? s2 : 0));
                for (int e = hcnt[b]; e < hcnt[b + 1] && !conf; ++e) {
                    const int h = hidx[e];
                    if (h < i) conf = mm_d2(sx + h * 3, q, dim) < Di;
                    if ((e & 31) == 31 &&
                        __hip_atomic_load(&sh_first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <= i)
                        break;
                }
            }
            if (conf) atomicMin(&sh_first, i);
        }
    }
    __syncthreads();
    const int r = sh_first;
    const int pos0 = st->pos_next;
    for (int i = tid; i < r; i += kMmRoundThreads) {
        const int32_t id = (int32_t)si[i];
        const int pos = pos0 - i;
        const double Di = __longlong_as_double((long long)sk[i]);
        a.order[pos] = id;
        a.ell[pos] = mm_sqrt_rn(Di);
        a.pos_of[id] = pos;
        a.acc[i] = id;
        a.accD[i] = sk[i];
    }
    for (int i = r + tid; i < nv; i += kMmRoundThreads) {
        a.buf[i - r] = (int32_t)si[i];
        a.bufD[i - r] = sk[i];
    }
    __syncthreads();
    if (tid == 0) {
        st->naccept = r;
        st->pos_next = pos0 - r;
        st->remaining = remaining - r;
        st->nb = nv - r;
        st->sorted = 1;
        if (r > 0) st->rounds += 1;
        if (nv - r == 0 && remaining - r > 0) {
            st->phase = 1;
            st->lvl = 0;
            st->prefix = 0;
            st->above = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// update: D_j = min(D_j, |x_j - x_p|^2) for the remaining points near each
// placed point p; each placed point's cells are split over several workgroups
// when the round placed few points
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mm_update_kernel(MmArgs a) {
    const int r = a.st->naccept;
    if (r == 0) return;
    const int dim = a.dim;
    const int nparts = max(1, (int)gridDim.x / r);
    const double* lo = a.prm + a.nlev * 6;
    const double* hmin = lo + 3;
    for (int64_t w = blockIdx.x; w < (int64_t)r * nparts; w += gridDim.x) {
        const int ai = (int)(w % r);
        const int part = (int)(w / r);
        const uint64_t Dp = a.accD[ai];
        if (Dp == 0ull) continue;  // no remaining point can get closer than 0
        const int32_t p = a.acc[ai];
        double q[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < dim; ++k) q[k] = a.pts[(int64_t)p * dim + k];
        // every point with d2 < D_j <= D_p lies within rho (with room for rounding)
        const double rho = sqrt(__longlong_as_double((long long)Dp)) * (1.0 + 1e-6);
        int l = a.nlev - 1;
        while (l > 0 && hmin[l] < rho) --l;
        const MmLevel L = a.lev[l];
        int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) {
            const double invh = a.prm[(l * 3 + k) * 2];
            clo[k] = mm_cell1(q[k] - rho, lo[k], invh, L.G);
            chi[k] = mm_cell1(q[k] + rho, lo[k], invh, L.G);
        }
        const int ny = dim > 1 ? chi[1] - clo[1] + 1 : 1;
        const int nz = dim > 2 ? chi[2] - clo[2] + 1 : 1;
        const int rows = ny * nz;
        const int32_t* cs = a.cell_start + L.cell_off;
        // the rows' point ranges (each row of cells is contiguous)
        int64_t total = 0;
        for (int rr = 0; rr < rows; ++rr) {
            const int64_t y = dim > 1 ? clo[1] + rr % ny : 0;
            const int64_t z = dim > 2 ? clo[2] + rr / ny : 0;
            const int64_t base = (z * L.G + y) * L.G;
            total += cs[base + chi[0] + 1] - cs[base + clo[0]];
        }
        const int64_t e0 = total * part / nparts, e1 = total * (part + 1) / nparts;
        int64_t acc_len = 0;
        for (int rr = 0; rr < rows; ++rr) {
            const int64_t y = dim > 1 ? clo[1] + rr % ny : 0;
            const int64_t z = dim > 2 ? clo[2] + rr / ny : 0;
            const int64_t base = (z * L.G + y) * L.G;
            const int64_t b = cs[base + clo[0]], e = cs[base + chi[0] + 1];
            const int64_t len = e - b;
            // this row's share of [e0, e1)
            const int64_t s0 = max(e0, acc_len), s1 = min(e1, acc_len + len);
            for (int64_t f = s0 + threadIdx.x; f < s1; f += blockDim.x) {
                const int64_t k = L.pt_off + b + (f - acc_len);
                const int32_t j = a.cell_ids[k];
                if (a.pos_of[j] >= 0) continue;
                const double dd = mm_d2(a.cell_xyz + k * dim, q, dim);
                const uint64_t db = (uint64_t)__double_as_longlong(dd);
                if (db < a.D[j]) atomicMin((unsigned long long*)&a.D[j], (unsigned long long)db);
            }
            acc_len += len;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t mm_align(size_t b) { return (b + 255) & ~(size_t)255; }

static int mm_levels(int64_t n, int dim, MmLevel* lev) {
    // cells per level: (2^l)^dim up to about 2n (and 2^24)
    int nl = 0;
    int64_t cell_off = 0, pt_off = 0;
    for (int l = 0; l < kMmMaxLevels; ++l) {
        int64_t cells = 1;
        for (int k = 0; k < dim; ++k) cells <<= l;
        if (l > 0 && (cells > 2 * n || cells > (1 << 24))) break;
        MmLevel& L = lev[nl];
        L.G = 1 << l;
        L.cells = cells;
        L.cell_off = cell_off;
        L.pt_off = pt_off;
        cell_off += cells + 1;
        pt_off += n;
        ++nl;
    }
    return nl;
}

struct MmLayout {
    int nlev;
    MmLevel lev[kMmMaxLevels];
    int64_t total_cells, max_cells;
    size_t off_bb, off_prm, off_cs, off_fill, off_ids, off_xyz, off_D, off_pos, off_buf, off_bufD, off_acc, off_accD,
        off_hist, off_st, off_scan;
    size_t scan_bytes, bytes;
};

static bool mm_layout(int64_t n, int dim, MmLayout& y) {
    y.nlev = mm_levels(n, dim, y.lev);
    y.total_cells = y.max_cells = 0;
    for (int l = 0; l < y.nlev; ++l) {
        y.total_cells += y.lev[l].cells + 1;
        y.max_cells = std::max<int64_t>(y.max_cells, y.lev[l].cells + 1);
    }
    size_t scan = 0;
    if (rocprim::exclusive_scan(nullptr, scan, (const int32_t*)nullptr, (int32_t*)nullptr, 0, (size_t)y.max_cells,
                                rocprim::plus<int32_t>()) != hipSuccess)
        return false;
    y.scan_bytes = scan;
    size_t o = 0;
    y.off_bb = o; o += mm_align(6 * sizeof(uint64_t));
    y.off_prm = o; o += mm_align((size_t)(y.nlev * 7 + 3) * sizeof(double));
    y.off_cs = o; o += mm_align((size_t)y.total_cells * 4);
    y.off_fill = o; o += mm_align((size_t)y.max_cells * 4);
    y.off_ids = o; o += mm_align((size_t)y.nlev * n * 4);
    y.off_xyz = o; o += mm_align((size_t)y.nlev * n * dim * 8);
    y.off_D = o; o += mm_align((size_t)n * 8);
    y.off_pos = o; o += mm_align((size_t)n * 4);
    y.off_buf = o; o += mm_align((size_t)kMmCap * 4);
    y.off_bufD = o; o += mm_align((size_t)kMmCap * 8);
    y.off_acc = o; o += mm_align((size_t)kMmCap * 4);
    y.off_accD = o; o += mm_align((size_t)kMmCap * 8);
    y.off_hist = o; o += mm_align((size_t)kMmBins * 4);
    y.off_st = o; o += mm_align(sizeof(MmState));
    y.off_scan = o; o += mm_align(y.scan_bytes);
    y.bytes = o;
    return true;
}

int64_t reverse_maximin_workspace(int64_t n, int dim) {
    if (n <= 0) return 0;
    MmLayout y;
    if (!mm_layout(n, dim, y)) return -1;
    return (int64_t)y.bytes;
}

hipError_t launch_reverse_maximin(const double* pts, int64_t n, int dim, void* workspace, int32_t* order, double* ell,
                                  hipStream_t s, int32_t* rounds_out) {
    if (n <= 0) return hipSuccess;
    MmLayout y;
    if (!mm_layout(n, dim, y)) return hipErrorInvalidValue;
    char* w = static_cast<char*>(workspace);
    uint64_t* bb = reinterpret_cast<uint64_t*>(w + y.off_bb);
    double* prm = reinterpret_cast<double*>(w + y.off_prm);
    int32_t* cs = reinterpret_cast<int32_t*>(w + y.off_cs);
    int32_t* fill = reinterpret_cast<int32_t*>(w + y.off_fill);
    MmArgs a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.nlev = y.nlev;
    for (int l = 0; l < y.nlev; ++l) a.lev[l] = y.lev[l];
    a.prm = prm;
    a.cell_start = cs;
    a.cell_ids = reinterpret_cast<int32_t*>(w + y.off_ids);
    a.cell_xyz = reinterpret_cast<double*>(w + y.off_xyz);
    a.D = reinterpret_cast<uint64_t*>(w + y.off_D);
    a.pos_of = reinterpret_cast<int32_t*>(w + y.off_pos);
    a.buf = reinterpret_cast<int32_t*>(w + y.off_buf);
    a.bufD = reinterpret_cast<uint64_t*>(w + y.off_bufD);
    a.acc = reinterpret_cast<int32_t*>(w + y.off_acc);
    a.accD = reinterpret_cast<uint64_t*>(w + y.off_accD);
    a.hist = reinterpret_cast<uint32_t*>(w + y.off_hist);
    a.st = reinterpret_cast<MmState*>(w + y.off_st);
    a.order = order;
    a.ell = ell;
    hipLaunchKernelGGL(mm_bbox_init_kernel, dim3(1), dim3(64), 0, s, bb);
    const unsigned nbk = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(mm_bbox_kernel, dim3(nbk), dim3(256), 0, s, pts, n, dim, bb);
    hipLaunchKernelGGL(mm_params_kernel, dim3(1), dim3(64), 0, s, (const uint64_t*)bb, a, prm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned gb = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    for (int l = 0; l < y.nlev; ++l) {
        const MmLevel& L = y.lev[l];
        const unsigned gc = (unsigned)std::min<int64_t>((L.cells + 1 + 255) / 256, 4096);
        hipLaunchKernelGGL(mm_fill_kernel, dim3(gc), dim3(256), 0, s, fill, L.cells + 1, 0);
        hipLaunchKernelGGL(mm_count_kernel, dim3(gb), dim3(256), 0, s, a, l, fill);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        size_t sb = y.scan_bytes;
        e = rocprim::exclusive_scan(w + y.off_scan, sb, fill, cs + L.cell_off, 0, (size_t)(L.cells + 1),
                                    rocprim::plus<int32_t>(), s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(mm_fill_kernel, dim3(gc), dim3(256), 0, s, fill, L.cells + 1, 0);
        hipLaunchKernelGGL(mm_scatter_kernel, dim3(gb), dim3(256), 0, s, a, l, fill, const_cast<int32_t*>(a.cell_ids),
                           const_cast<double*>(a.cell_xyz));
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mm_init_kernel, dim3((unsigned)std::max<int64_t>((n + 255) / 256, kMmBins / 256)), dim3(256),
                       0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t smem = (size_t)kMmCap * (8 + 4 + 24) + (size_t)(2 * kMmHash + 1 + kMmCap + kMmRoundThreads) * 4;
    e = hipFuncSetAttribute((const void*)mm_round_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    const unsigned gh = (unsigned)std::min<int64_t>((n + 255) / 256, kMmGridBlocks);
    // each step places at least one point, or advances a refill by two
    // digits or runs its gather; a refill takes at most five steps, so every
    // batch of steps places points
    MmState hs{};
    int32_t left = (int32_t)(n - 1);
    for (;;) {
        for (int k = 0; k < kMmStepsPerBatch; ++k) {
            for (int pass = 0; pass < kMmPassesPerStep; ++pass)
                hipLaunchKernelGGL(mm_hist_kernel, dim3(gh), dim3(256), 0, s, a);
            hipLaunchKernelGGL(mm_gather_kernel, dim3(gh), dim3(256), 0, s, a);
            hipLaunchKernelGGL(mm_round_kernel, dim3(1), dim3(kMmRoundThreads), smem, s, a);
            hipLaunchKernelGGL(mm_update_kernel, dim3(1024), dim3(256), 0, s, a);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(&hs, a.st, sizeof(MmState), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (hs.overflow) return hipErrorUnknown;
        if (hs.remaining == 0) break;
        if (hs.remaining >= left) return hipErrorUnknown;  // no progress: not expected
        left = hs.remaining;
    }
    if (rounds_out) *rounds_out = hs.rounds;
    return hipSuccess;
}

}  // namespace csel
