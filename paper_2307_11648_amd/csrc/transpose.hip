// transpose.hip -- the CSC form of L^T from the CSC form of L (equivalently,
// L in CSR form), so that y = L x runs as the same deterministic per-column
// gather as y = L^T x instead of a scatter with atomics.
//
// The stored slots are sorted by row with a stable radix sort of (row, slot)
// pairs: inside a row the slots keep their CSC order, i.e. ascending column,
// so the result is canonical and the products built on it are deterministic.
// Slots with a row outside [0, n) (the padding of csel_select_and_factor's
// [T][k+1] layout), or not covered by any column, sort last and are dropped:
// t_col_ptr[n] counts the kept entries and the slots past it get row -1 and
// value 0.
#include <rocprim/device/device_radix_sort.hpp>

#include "launch.hpp"

namespace csel {

__global__ __launch_bounds__(256) void fill_neg_kernel(int32_t* __restrict__ a, int64_t m) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = -1;
}

// the column of every slot (slots outside [0, n_slots) are not written)
__global__ __launch_bounds__(256) void slot_column_kernel(int64_t n, const int64_t* __restrict__ col_ptr,
                                                          int64_t n_slots, int32_t* __restrict__ colof) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = max(col_ptr[c], (int64_t)0), e = min(col_ptr[c + 1], n_slots);
        for (int64_t p = b; p < e; ++p) colof[p] = (int32_t)c;
    }
}

// sort keys (the row, or n for a dropped slot) and the slot indices
__global__ __launch_bounds__(256) void slot_keys_kernel(int64_t n, const int32_t* __restrict__ row_idx,
                                                        const int32_t* __restrict__ colof, int64_t n_slots,
                                                        uint32_t* __restrict__ keys, int32_t* __restrict__ slots) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_slots;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = row_idx[p];
        const bool ok = colof[p] >= 0 && r >= 0 && (int64_t)r < n;
        keys[p] = ok ? (uint32_t)r : (uint32_t)n;
        slots[p] = (int32_t)p;
    }
}

// entries of L^T in sorted order, and its column offsets: t_col_ptr[r] is the
// number of sorted keys below r (written once per r, by the position where
// the keys step past it)
__global__ __launch_bounds__(256) void transposed_kernel(int64_t n, int64_t n_slots,
                                                         const uint32_t* __restrict__ keys,
                                                         const int32_t* __restrict__ perm,
                                                         const int32_t* __restrict__ colof,
                                                         const double* __restrict__ val,
                                                         int64_t* __restrict__ t_col_ptr,
                                                         int32_t* __restrict__ t_row_idx, double* __restrict__ t_val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n_slots;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kp = i == 0 ? -1 : (int64_t)keys[i - 1];
        const int64_t kc = i == n_slots ? n : (int64_t)keys[i];
        for (int64_t r = kp + 1; r <= kc && r <= n; ++r) t_col_ptr[r] = i;
        if (i < n_slots) {
            const int32_t p = perm[i];
            const bool ok = kc < n;
            t_row_idx[i] = ok ? colof[p] : -1;
            t_val[i] = ok ? val[p] : 0.0;
        }
    }
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static int key_bits(int64_t n) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) <= n) ++b;
    return b;
}

static size_t sort_temp(int64_t n_slots, int bits) {
    size_t bytes = 0;
    const hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                                   (const int32_t*)nullptr, (int32_t*)nullptr,
                                                   (unsigned int)n_slots, 0u, (unsigned int)bits);
    return e == hipSuccess ? bytes : SIZE_MAX;
}

// workspace: [keys in][keys out][slots in][slots out (the permutation)][slot columns][radix-sort temporary]
int64_t transpose_factor_workspace(int64_t n, int64_t n_slots) {
    if (n_slots <= 0) return 0;
    const size_t temp = sort_temp(n_slots, key_bits(n));
    if (temp == SIZE_MAX) return -1;
    return (int64_t)(5 * align256((size_t)n_slots * 4) + align256(temp));
}

hipError_t launch_transpose_factor(int64_t n, const int64_t* col_ptr, const int32_t* row_idx, const double* val,
                                   int64_t n_slots, int64_t* t_col_ptr, int32_t* t_row_idx, double* t_val,
                                   void* workspace, hipStream_t s) {
    const unsigned gb = (unsigned)std::min<int64_t>((std::max(n, n_slots) + 256) / 256, 8192);
    if (n_slots == 0) {
        // no stored entries: every column of L^T is empty
        hipLaunchKernelGGL(transposed_kernel, dim3(gb), dim3(256), 0, s, n, (int64_t)0, (const uint32_t*)nullptr,
                           (const int32_t*)nullptr, (const int32_t*)nullptr, (const double*)nullptr, t_col_ptr,
                           t_row_idx, t_val);
        return hipGetLastError();
    }
    char* w = static_cast<char*>(workspace);
    const size_t seg = align256((size_t)n_slots * 4);
    uint32_t* keys_in = reinterpret_cast<uint32_t*>(w);
    uint32_t* keys_out = reinterpret_cast<uint32_t*>(w + seg);
    int32_t* slots_in = reinterpret_cast<int32_t*>(w + 2 * seg);
    int32_t* perm = reinterpret_cast<int32_t*>(w + 3 * seg);
    int32_t* colof = reinterpret_cast<int32_t*>(w + 4 * seg);
    void* temp = w + 5 * seg;
    const int bits = key_bits(n);
    size_t temp_bytes = sort_temp(n_slots, bits);
    hipLaunchKernelGGL(fill_neg_kernel, dim3(gb), dim3(256), 0, s, colof, n_slots);
    hipLaunchKernelGGL(slot_column_kernel, dim3(gb), dim3(256), 0, s, n, col_ptr, n_slots, colof);
    hipLaunchKernelGGL(slot_keys_kernel, dim3(gb), dim3(256), 0, s, n, row_idx, (const int32_t*)colof, n_slots,
                       keys_in, slots_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, slots_in, perm, (unsigned int)n_slots, 0u,
                                  (unsigned int)bits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(transposed_kernel, dim3(gb), dim3(256), 0, s, n, n_slots, (const uint32_t*)keys_out,
                       (const int32_t*)perm, (const int32_t*)colof, val, t_col_ptr, t_row_idx, t_val);
    return hipGetLastError();
}

}  // namespace csel
