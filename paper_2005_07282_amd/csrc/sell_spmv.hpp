// Row loop of the sliced-ELL SpMV shared by the solver kernels: lane j of a
// wavefront computes row 64s+j of A x as a sequential fma chain over the
// row's stored entries in their original order (Section 4.3).
#pragma once

#include "kernels.hpp"

namespace rpcg {

// Entries of one row loaded per batch: loads of a batch are issued together
// so the wavefront waits for memory once per batch, not once per entry
// (9 divides the 27 entries of an interior 27-point row).
constexpr int SPMV_BATCH = 9;

__device__ __forceinline__ long long uniform_ll(long long v)
{
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xFFFFFFFFll));
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// The matrix is streamed once per iteration and is far larger than the
// caches: its loads are marked non-temporal so that they do not evict the
// gathered vector from L2.
template <bool COL16, typename T>
__device__ __forceinline__ int sell_col(const SellMat<T> &A, long long kk, int rbase)
{
    if constexpr (COL16) return rbase + (int)__builtin_nontemporal_load(&A.col16[kk]);
    else return __builtin_nontemporal_load(&A.col[kk]);
}

template <typename T>
__device__ __forceinline__ T sell_val(const T *pv, long long k)
{
    return __builtin_nontemporal_load(&pv[k]);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Row length of row i (0 for lanes past the last row).
template <typename T>
__device__ __forceinline__ int sell_len(const SellMat<T> &A, long long i)
{
    if (i >= A.n) return 0;
    return A.len8 ? (int)A.len8[i] : A.row_ptr[i + 1] - A.row_ptr[i];
}

// sum = fold over k < len of fma(a_ik, x[col_ik], sum) from +0 in T, for the
// row of this lane in slice s (base = off[s], width = slice width, both
// uniform). Every position up to the width holds a valid column (padding
// entries and the lanes past the last row point at a row of the matrix), so
// loads and gathers need no branch; only the fma is limited to the row's
// entries. With DIAG, *aii receives the value stored in column i (the last
// such entry) and *found whether there is one.
template <typename T, bool COL16, bool DIAG>
__device__ __forceinline__ T sell_row(const SellMat<T> &A, long long base, int width, long long i, int len,
                                      const T *__restrict__ x, T *aii, bool *found)
{
    const int lane = (int)(i & 63);
    const int rbase = i < A.n ? (int)i : A.n - 1;
    const long long kb = base + lane;
    const T *__restrict__ pv = A.val + kb;
    T sum = T(0);
    int k0 = 0;
    for (; k0 + SPMV_BATCH <= width; k0 += SPMV_BATCH) {
        int c[SPMV_BATCH];
        T a[SPMV_BATCH], g[SPMV_BATCH];
#pragma unroll
        for (int u = 0; u < SPMV_BATCH; ++u) c[u] = sell_col<COL16>(A, kb + 64 * (k0 + u), rbase);
#pragma unroll
        for (int u = 0; u < SPMV_BATCH; ++u) a[u] = sell_val(pv, 64 * (k0 + u));
#pragma unroll
        for (int u = 0; u < SPMV_BATCH; ++u) g[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < SPMV_BATCH; ++u) {
            const bool in = k0 + u < len;
            const T t = fma_t(a[u], g[u], sum);
            sum = in ? t : sum;
            if constexpr (DIAG) {
                if (in && c[u] == (int)i) { *aii = a[u]; *found = true; }
            }
        }
    }
    for (; k0 < width; ++k0) {
        const int c = sell_col<COL16>(A, kb + 64 * k0, rbase);
        const T a = sell_val(pv, 64 * k0);
        const bool in = k0 < len;
        const T t = fma_t(a, x[c], sum);
        sum = in ? t : sum;
        if constexpr (DIAG) {
            if (in && c == (int)i) { *aii = a; *found = true; }
        }
    }
    return sum;
}

} // namespace rpcg
