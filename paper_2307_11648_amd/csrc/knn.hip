// knn.hip -- later-ordered nearest-neighbour candidate pools on the GPU
// (Sec. 4): for every ordering position i, the C nearest points among the
// positions after i, ascending by (squared distance, position); the squared
// distance is summed coordinate by coordinate in order, without fused
// multiply-adds, so ties and order are those of the plain definition.
//
// Levels: level l holds the positions [s_l, n) with n - s_l = ceil(n / 2^l),
// each in a uniform grid of about two points per cell (a counting sort by
// cell: counts, an exclusive scan, a scatter of positions and coordinates).
// A query at position i searches the finest level that still holds every
// position after i, so at least half of the points it meets are later ones.
// One wavefront per query, queries in the Morton order of their points:
//   * a radius rho from the level's density of later points, grown (volume
//     x 2) while fewer than min(C, n-1-i) later points lie within rho, or cut
//     by bisection while more than the LDS buffer holds;
//   * each pass walks the grid rows of the cells covering the ball (each
//     row's points are one contiguous range), lanes over the points, and
//     appends the later points within rho to the wave's LDS buffer (ballot
//     compaction); every point within rho is met, so once the count reaches
//     min(C, n-1-i) the pool is among them;
//   * a bitonic sort of the buffer by (squared distance, position).
#include <rocprim/device/device_scan.hpp>

#include "device_common.hpp"
#include "launch.hpp"

namespace csel {

constexpr int kKnnBuf = 2048;          // candidates per query in LDS
constexpr int kKnnWaves = 2;           // queries per workgroup
constexpr int kKnnMaxLevels = 32;
constexpr int64_t kKnnLastLevel = 4096;  // levels halve down to this many points

struct KnnLevel {
    int64_t s;         // first position held
    int64_t N;         // positions held (n - s)
    int32_t G;         // cells per dimension
    int64_t cells;     // G^dim
    int64_t cell_off;  // offset of the level's cell_start (cells + 1 entries)
    int64_t pt_off;    // offset of the level's points
};

struct KnnArgs {
    const double* pts;
    int64_t n;
    int32_t dim;
    int32_t C;
    int32_t nlev;
    KnnLevel lev[kKnnMaxLevels];
    const double* prm;        // [level][dim][2]: 1/h and h; then lo[3]
    const int32_t* cell_start;
    const int32_t* cell_pts;  // positions, grouped by cell
    const double* cell_xyz;   // their coordinates [.][dim]
    const int32_t* order;     // queries in Morton order
    int32_t* pool;
    int32_t* pool_len;
};

// (x - q)^2 summed in coordinate order, products and sums rounded separately
__device__ __forceinline__ double sq_dist_plain(const double* a, const double* q, int dim) {
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

// order-preserving image of a double in uint64 (for atomic min / max)
__device__ __forceinline__ uint64_t knn_ord(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double knn_unord(uint64_t u) {
    return __longlong_as_double((long long)((u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u));
}

__global__ void knn_bbox_init_kernel(uint64_t* bb) {
    if (threadIdx.x < 3) {
        bb[threadIdx.x] = ~0ull;
        bb[3 + threadIdx.x] = 0ull;
    }
}

__global__ __launch_bounds__(256) void knn_bbox_kernel(const double* __restrict__ pts, int64_t n, int dim,
                                                       uint64_t* bb) {
    uint64_t mn[3] = {~0ull, ~0ull, ~0ull}, mx[3] = {0ull, 0ull, 0ull};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < dim; ++k) {
            const uint64_t o = knn_ord(pts[i * dim + k]);
            mn[k] = o < mn[k] ? o : mn[k];
            mx[k] = o > mx[k] ? o : mx[k];
        }
    }
    for (int k = 0; k < dim; ++k) {
        atomicMin((unsigned long long*)&bb[k], (unsigned long long)mn[k]);
        atomicMax((unsigned long long*)&bb[3 + k], (unsigned long long)mx[k]);
    }
}

// per level and dimension: 1/h and h (h = extent / G; a zero extent puts
// every point in cell 0); then the box's lower corner
__global__ void knn_params_kernel(const uint64_t* bb, KnnArgs a, double* prm) {
    if (threadIdx.x != 0) return;
    double lo[3] = {0.0, 0.0, 0.0}, ext[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < a.dim; ++k) {
        lo[k] = knn_unord(bb[k]);
        ext[k] = knn_unord(bb[3 + k]) - lo[k];
    }
    for (int l = 0; l < a.nlev; ++l) {
        for (int k = 0; k < 3; ++k) {
            const double G = (double)a.lev[l].G;
            const bool flat = !(ext[k] > 0.0) || k >= a.dim;
            prm[(l * 3 + k) * 2 + 0] = flat ? 0.0 : G / ext[k];
            prm[(l * 3 + k) * 2 + 1] = flat ? 1.0 : ext[k] / G;
        }
    }
    for (int k = 0; k < 3; ++k) prm[a.nlev * 6 + k] = lo[k];
}

__device__ __forceinline__ int knn_cell1(double x, double lo, double invh, int G) {
    const double t = (x - lo) * invh;
    int c = t > 0.0 ? (int)t : 0;  // floor for t >= 0
    return c < G ? c : G - 1;
}

__device__ __forceinline__ int64_t knn_cell(const double* x, const double* prm, int l, int dim, int G, int nlev) {
    const double* lo = prm + nlev * 6;
    int64_t c = 0;
    for (int k = dim - 1; k >= 0; --k) c = c * G + knn_cell1(x[k], lo[k], prm[(l * 3 + k) * 2], G);
    return c;
}

__global__ __launch_bounds__(256) void knn_count_kernel(KnnArgs a, int l, int32_t* counts) {
    const KnnLevel L = a.lev[l];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= L.N) return;
    const int64_t p = L.s + j;
    const int64_t c = knn_cell(a.pts + p * a.dim, a.prm, l, a.dim, L.G, a.nlev);
    atomicAdd(&counts[c], 1);
}

__global__ __launch_bounds__(256) void knn_scatter_kernel(KnnArgs a, int l, int32_t* fill, int32_t* cell_pts,
                                                          double* cell_xyz) {
    const KnnLevel L = a.lev[l];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= L.N) return;
    const int64_t p = L.s + j;
    const double* x = a.pts + p * a.dim;
    const int64_t c = knn_cell(x, a.prm, l, a.dim, L.G, a.nlev);
    const int64_t at = L.pt_off + a.cell_start[L.cell_off + c] + atomicAdd(&fill[c], 1);
    cell_pts[at] = (int32_t)p;
    for (int k = 0; k < a.dim; ++k) cell_xyz[at * a.dim + k] = x[k];
}

__global__ __launch_bounds__(256) void knn_fill_kernel(int32_t* v, int64_t m, int32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = value;
}

__global__ __launch_bounds__(256) void knn_iota_kernel(int32_t* v, int64_t m) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (int32_t)i;
}

// one pass over the cells covering the ball of radius rho around q: the
// number of later points (position > i) with squared distance < rho^2; the
// first kKnnBuf of them go to (bd, bp)
__device__ int64_t knn_pass(const KnnArgs& a, int l, const double* q, int64_t i, double rho, double* bd,
                            int32_t* bp, int lane) {
    const KnnLevel L = a.lev[l];
    const int dim = a.dim;
    const double* lo = a.prm + a.nlev * 6;
    const double r2 = rho * rho;
    const double rc = rho * (1.0 + 1e-9);  // the cell range covers the ball with room for rounding
    int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) {
        const double invh = a.prm[(l * 3 + k) * 2];
        clo[k] = knn_cell1(q[k] - rc, lo[k], invh, L.G);
        chi[k] = knn_cell1(q[k] + rc, lo[k], invh, L.G);
    }
    const int ny = dim > 1 ? chi[1] - clo[1] + 1 : 1;
    const int nz = dim > 2 ? chi[2] - clo[2] + 1 : 1;
    const int64_t rows = (int64_t)ny * nz;
    const int32_t* cs = a.cell_start + L.cell_off;
    int64_t count = 0;
    for (int64_t r0 = 0; r0 < rows; r0 += kWave) {
        // lane t fetches the point range of row r0 + t
        int32_t rb = 0, re = 0;
        if (r0 + lane < rows) {
            const int64_t r = r0 + lane;
            const int64_t y = dim > 1 ? clo[1] + r % ny : 0;
            const int64_t z = dim > 2 ? clo[2] + r / ny : 0;
            const int64_t base = (z * L.G + y) * L.G;
            rb = cs[base + clo[0]];
            re = cs[base + chi[0] + 1];
        }
        const int nr = (int)min<int64_t>(kWave, rows - r0);
        for (int t = 0; t < nr; ++t) {
            const int32_t b = __builtin_amdgcn_readlane(rb, t), e = __builtin_amdgcn_readlane(re, t);
            for (int32_t j0 = b; j0 < e; j0 += kWave) {
                const int32_t j = j0 + lane;
                bool hit = false;
                double d2 = 0.0;
                int32_t p = -1;
                if (j < e) {
                    p = a.cell_pts[L.pt_off + j];
                    if ((int64_t)p > i) {
                        d2 = sq_dist_plain(a.cell_xyz + (L.pt_off + j) * dim, q, dim);
                        hit = d2 < r2;
                    }
                }
                const uint64_t m = __ballot(hit);
                if (hit) {
                    const int64_t at = count + __builtin_popcountll(m & ((1ull << lane) - 1ull));
                    if (at < kKnnBuf) {
                        bd[at] = d2;
                        bp[at] = p;
                    }
                }
                count += __builtin_popcountll(m);
            }
        }
    }
    return count;
}

__global__ __launch_bounds__(kKnnWaves * kWave) void knn_query_kernel(KnnArgs a) {
    __shared__ double sd[kKnnWaves][kKnnBuf];
    __shared__ int32_t sp[kKnnWaves][kKnnBuf];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    const int64_t qi = (int64_t)blockIdx.x * kKnnWaves + w;
    if (qi >= a.n) return;
    const int64_t i = a.order[qi];
    const int C = a.C;
    int32_t* prow = a.pool + i * C;
    const int64_t avail = a.n - 1 - i;
    const int want = (int)min<int64_t>(C, avail);
    if (want <= 0) {
        for (int t = lane; t < C; t += kWave) prow[t] = -1;
        if (lane == 0) a.pool_len[i] = 0;
        return;
    }
    int l = 0;
    while (l + 1 < a.nlev && a.lev[l + 1].s <= i + 1) ++l;
    const KnnLevel L = a.lev[l];
    const int dim = a.dim;
    double q[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) q[k] = a.pts[i * dim + k];
    // first radius: a ball that holds about 2 * want later points at the
    // level's mean density of later points
    double vcell = 1.0;
    double diam2 = 0.0;
    for (int k = 0; k < dim; ++k) {
        const double h = a.prm[(l * 3 + k) * 2 + 1];
        vcell *= h;
        diam2 += (h * L.G) * (h * L.G);
    }
    const double vd = dim == 1 ? 2.0 : (dim == 2 ? 3.141592653589793 : 4.188790204786391);
    const double dens = (double)avail / ((double)L.cells * vcell);
    double rho = pow(2.0 * want / (dens * vd), 1.0 / dim);
    const double rmax = 2.0 * sqrt(diam2) + 1.0;  // beyond the box: every point
    if (!(rho > 0.0) || !(rho < rmax)) rho = rmax;
    double rlo = 0.0, rhi = -1.0;  // below want at rlo, above the buffer at rhi
    double* bd = sd[w];
    int32_t* bp = sp[w];
    int64_t count = 0;
    bool ok = false;
    for (int it = 0; it < 200; ++it) {
        count = knn_pass(a, l, q, i, rho, bd, bp, lane);
        if (count < want) {
            rlo = rho;
            rho = rhi > 0.0 ? 0.5 * (rho + rhi) : (rho >= rmax ? rmax : fmin(rho * (dim == 1 ? 2.0 : dim == 2 ? 1.4142135623730951 : 1.2599210498948732), rmax));
            if (rlo >= rmax) break;  // cannot happen: every later point lies within rmax
            continue;
        }
        if (count > kKnnBuf) {
            rhi = rho;
            const double nr = 0.5 * (rlo + rho);
            if (!(nr < rho) || !(nr > rlo)) break;  // ties: no radius separates them
            rho = nr;
            continue;
        }
        ok = true;
        break;
    }
    if (!ok) {
        for (int t = lane; t < C; t += kWave) prow[t] = -1;
        if (lane == 0) a.pool_len[i] = -1;
        return;
    }
    // bitonic sort of the count candidates by (distance, position)
    int n2 = 64;
    while (n2 < count) n2 <<= 1;
    for (int t = (int)count + lane; t < n2; t += kWave) {
        bd[t] = __builtin_inf();
        bp[t] = INT32_MAX;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < n2; t += kWave) {
                const int u = t ^ j;
                if (u > t) {
                    const double dt = bd[t], du = bd[u];
                    const int32_t pt = bp[t], pu = bp[u];
                    const bool gt = dt > du || (dt == du && pt > pu);
                    const bool up = (t & k) == 0;
                    if (gt == up) {
                        bd[t] = du;
                        bd[u] = dt;
                        bp[t] = pu;
                        bp[u] = pt;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    for (int t = lane; t < C; t += kWave) prow[t] = t < want ? bp[t] : -1;
    if (lane == 0) a.pool_len[i] = want;
}

// ---------------------------------------------------------------------------
// host side: levels, workspace, launches
// ---------------------------------------------------------------------------
static size_t knn_align(size_t b) { return (b + 255) & ~(size_t)255; }

static int knn_levels(int64_t n, int dim, KnnLevel* lev) {
    int nl = 0;
    int64_t N = n, cell_off = 0, pt_off = 0;
    for (;;) {
        KnnLevel& L = lev[nl];
        L.s = n - N;
        L.N = N;
        int G = (int)floor(pow((double)N / 2.0, 1.0 / dim));
        if (G < 1) G = 1;
        if (dim == 1 && G > (1 << 24)) G = 1 << 24;
        L.G = G;
        L.cells = 1;
        for (int k = 0; k < dim; ++k) L.cells *= G;
        L.cell_off = cell_off;
        L.pt_off = pt_off;
        cell_off += L.cells + 1;
        pt_off += N;
        ++nl;
        if (N <= kKnnLastLevel || nl == kKnnMaxLevels) break;
        N = (N + 1) / 2;
    }
    return nl;
}

struct KnnLayout {
    int nlev;
    KnnLevel lev[kKnnMaxLevels];
    int64_t total_cells, total_pts, max_cells;
    size_t off_bb, off_prm, off_cs, off_fill, off_pts, off_xyz, off_iota, off_order, off_ord_ws, off_scan;
    size_t scan_bytes, ord_bytes, bytes;
};

static bool knn_layout(int64_t n, int dim, KnnLayout& y) {
    y.nlev = knn_levels(n, dim, y.lev);
    y.total_cells = y.total_pts = y.max_cells = 0;
    for (int l = 0; l < y.nlev; ++l) {
        y.total_cells += y.lev[l].cells + 1;
        y.total_pts += y.lev[l].N;
        y.max_cells = std::max<int64_t>(y.max_cells, y.lev[l].cells + 1);
    }
    size_t scan = 0;
    if (rocprim::exclusive_scan(nullptr, scan, (const int32_t*)nullptr, (int32_t*)nullptr, 0,
                                (size_t)y.max_cells, rocprim::plus<int32_t>()) != hipSuccess)
        return false;
    const int64_t ow = spatial_order_workspace(n);
    if (ow < 0) return false;
    y.scan_bytes = scan;
    y.ord_bytes = (size_t)ow;
    size_t o = 0;
    y.off_bb = o; o += knn_align(6 * sizeof(uint64_t));
    y.off_prm = o; o += knn_align((size_t)(y.nlev * 6 + 3) * sizeof(double));
    y.off_cs = o; o += knn_align((size_t)y.total_cells * 4);
    y.off_fill = o; o += knn_align((size_t)y.max_cells * 4);
    y.off_pts = o; o += knn_align((size_t)y.total_pts * 4);
    y.off_xyz = o; o += knn_align((size_t)y.total_pts * dim * 8);
    y.off_iota = o; o += knn_align((size_t)n * 4);
    y.off_order = o; o += knn_align((size_t)n * 4);
    y.off_ord_ws = o; o += knn_align(y.ord_bytes);
    y.off_scan = o; o += knn_align(y.scan_bytes);
    y.bytes = o;
    return true;
}

int64_t later_knn_workspace(int64_t n, int dim) {
    if (n <= 0) return 0;
    KnnLayout y;
    if (!knn_layout(n, dim, y)) return -1;
    return (int64_t)y.bytes;
}

int later_knn_max_pool() { return kKnnBuf; }

hipError_t launch_later_knn(const double* pts, int64_t n, int dim, int C, void* workspace, int32_t* pool,
                            int32_t* pool_len, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    KnnLayout y;
    if (!knn_layout(n, dim, y)) return hipErrorInvalidValue;
    char* w = static_cast<char*>(workspace);
    uint64_t* bb = reinterpret_cast<uint64_t*>(w + y.off_bb);
    double* prm = reinterpret_cast<double*>(w + y.off_prm);
    int32_t* cs = reinterpret_cast<int32_t*>(w + y.off_cs);
    int32_t* fill = reinterpret_cast<int32_t*>(w + y.off_fill);
    int32_t* cpts = reinterpret_cast<int32_t*>(w + y.off_pts);
    double* cxyz = reinterpret_cast<double*>(w + y.off_xyz);
    int32_t* iota = reinterpret_cast<int32_t*>(w + y.off_iota);
    int32_t* order = reinterpret_cast<int32_t*>(w + y.off_order);
    KnnArgs a{};
    a.pts = pts;
    a.n = n;
    a.dim = dim;
    a.C = C;
    a.nlev = y.nlev;
    for (int l = 0; l < y.nlev; ++l) a.lev[l] = y.lev[l];
    a.prm = prm;
    a.cell_start = cs;
    a.cell_pts = cpts;
    a.cell_xyz = cxyz;
    a.order = order;
    a.pool = pool;
    a.pool_len = pool_len;
    hipLaunchKernelGGL(knn_bbox_init_kernel, dim3(1), dim3(64), 0, s, bb);
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(knn_bbox_kernel, dim3(nb), dim3(256), 0, s, pts, n, dim, bb);
    hipLaunchKernelGGL(knn_params_kernel, dim3(1), dim3(64), 0, s, (const uint64_t*)bb, a, prm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = 0; l < y.nlev; ++l) {
        const KnnLevel& L = y.lev[l];
        const unsigned gc = (unsigned)std::min<int64_t>((L.cells + 1 + 255) / 256, 4096);
        const unsigned gp = (unsigned)((L.N + 255) / 256);
        // counts in cell_start[1 ..], then the exclusive scan in place
        hipLaunchKernelGGL(knn_fill_kernel, dim3(gc), dim3(256), 0, s, fill, L.cells + 1, 0);
        hipLaunchKernelGGL(knn_count_kernel, dim3(gp), dim3(256), 0, s, a, l, fill);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        size_t sb = y.scan_bytes;
        e = rocprim::exclusive_scan(w + y.off_scan, sb, fill, cs + L.cell_off, 0, (size_t)(L.cells + 1),
                                    rocprim::plus<int32_t>(), s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(knn_fill_kernel, dim3(gc), dim3(256), 0, s, fill, L.cells + 1, 0);
        hipLaunchKernelGGL(knn_scatter_kernel, dim3(gp), dim3(256), 0, s, a, l, fill, cpts, cxyz);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // queries in the Morton order of their points
    hipLaunchKernelGGL(knn_iota_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s,
                       iota, n);
    e = launch_spatial_order(pts, n, dim, n, iota, w + y.off_ord_ws, order, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(knn_query_kernel, dim3((unsigned)((n + kKnnWaves - 1) / kKnnWaves)), dim3(kKnnWaves * kWave),
                       0, s, a);
    return hipGetLastError();
}

}  // namespace csel
