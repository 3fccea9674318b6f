// Row loop of the sliced-ELL SpMV shared by the solver kernels: lane j of a
// wavefront computes row 64s+j of A x as a sequential fma chain over the
// row's stored entries in their original order (Section 4.3). Layout and
// column encoding are described with SellMat.
#pragma once

#include "kernels.hpp"

namespace rpcg {

// Entries of one row loaded per batch: the loads of a batch are issued
// together so the wavefront waits for memory once per batch, not once per
// entry (14 with the two-entry interleave: an interior 27-point row is one
// batch of 14 and a last batch of 12 plus its single-entry last column; 9
// divides the 27 entries without it).
template <typename T>
__host__ __device__ constexpr int spmv_batch()
{
    return sell_vec<T>() == 2 ? 14 : 9;
}

__device__ __forceinline__ long long uniform_ll(long long v)
{
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xFFFFFFFFll));
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

typedef double d2_t __attribute__((ext_vector_type(2)));
typedef int i2_t __attribute__((ext_vector_type(2)));

// The matrix is streamed once per iteration and is far larger than the
// caches: its loads are marked non-temporal so that they do not evict the
// gathered vector from L2.
//
// One group = the V consecutive entries k = V*g .. V*g+V-1 of this lane's row
// at element index p (= off[s] + 64*V*g + V*lane). With 16-bit column codes
// the columns are decoded in rank order from `cur` (the previous column of
// the row) and `first` (min(i, n-1) + cfirst[s], the origin of rank 0).
template <typename T, bool COL16>
__device__ __forceinline__ void sell_group(const SellMat<T> &A, long long p, int k0, int first, int &cur,
                                           int (&c)[sell_vec<T>()], T (&a)[sell_vec<T>()])
{
    constexpr int V = sell_vec<T>();
    unsigned code[V];
    if constexpr (V == 2) {
        const d2_t v = __builtin_nontemporal_load((const d2_t *)(A.val + p));
        a[0] = v.x;
        a[1] = v.y;
        if constexpr (COL16) {
            const unsigned r = __builtin_nontemporal_load((const unsigned *)(A.col16 + p));
            code[0] = r & 0xFFFFu;
            code[1] = r >> 16;
        } else {
            const i2_t q = __builtin_nontemporal_load((const i2_t *)(A.col + p));
            c[0] = q.x;
            c[1] = q.y;
        }
    } else {
        a[0] = __builtin_nontemporal_load(A.val + p);
        if constexpr (COL16) code[0] = __builtin_nontemporal_load(A.col16 + p);
        else c[0] = __builtin_nontemporal_load(A.col + p);
    }
    if constexpr (COL16) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            cur = (k0 + v == 0) ? first + (int)(short)code[v] : cur + (int)code[v];
            c[v] = cur;
        }
    }
}

// Row length of row i (0 for lanes past the last row).
template <typename T>
__device__ __forceinline__ int sell_len(const SellMat<T> &A, long long i)
{
    if (i >= A.n) return 0;
    return A.len8 ? (int)A.len8[i] : A.row_ptr[i + 1] - A.row_ptr[i];
}

// R consecutive groups of this lane's row, from group g0, as one batch: all
// loads, then all gathers, then the fma chain in storage order (only the
// row's own entries enter it).
template <typename T, bool COL16, bool DIAG, int R, bool LAST = false>
__device__ __forceinline__ void sell_batch(const SellMat<T> &A, long long p0, int g0, int first, int &cur, int len,
                                           long long i, const T *__restrict__ x, T &sum, T *aii, bool *found,
                                           long long pl = 0, int kl = 0)
{
    constexpr int V = sell_vec<T>();
    int c[R + 1][V];
    T a[R + 1][V];
#pragma unroll
    for (int u = 0; u < R; ++u) sell_group<T, COL16>(A, p0 + 64ll * V * (g0 + u), V * (g0 + u), first, cur, c[u], a[u]);
    // LAST: the single-entry last column (entry kl = width-1 at pl)
    int cl = 0;
    T al = T(0);
    if constexpr (LAST) {
        al = __builtin_nontemporal_load(A.val + pl);
        if constexpr (COL16) {
            const unsigned code = __builtin_nontemporal_load(A.col16 + pl);
            cur = kl == 0 ? first + (int)(short)code : cur + (int)code;
            cl = cur;
        } else {
            cl = __builtin_nontemporal_load(A.col + pl);
        }
    }
    T g[R + 1][V];
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) g[u][v] = x[c[u][v]];
    T gl = T(0);
    if constexpr (LAST) gl = x[cl];
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool in = V * (g0 + u) + v < len;
            const T t = fma_t(a[u][v], g[u][v], sum);
            sum = in ? t : sum;
            if constexpr (DIAG) {
                if (in && c[u][v] == (int)i) { *aii = a[u][v]; *found = true; }
            }
        }
    if constexpr (LAST) {
        const bool in = kl < len;
        const T t = fma_t(al, gl, sum);
        sum = in ? t : sum;
        if constexpr (DIAG) {
            if (in && cl == (int)i) { *aii = al; *found = true; }
        }
    }
}

// The last rest < R groups as one batch of exactly that many (rest is
// wavefront-uniform, so the choice is a scalar branch and each batch is
// straight-line code).
template <typename T, bool COL16, bool DIAG, int R, bool LAST>
__device__ __forceinline__ void sell_rest(int rest, const SellMat<T> &A, long long p0, int g0, int first, int &cur,
                                          int len, long long i, const T *__restrict__ x, T &sum, T *aii, bool *found,
                                          long long pl, int kl)
{
    if constexpr (R > 0 || (LAST && R == 0)) {
        if (rest == R) sell_batch<T, COL16, DIAG, R, LAST>(A, p0, g0, first, cur, len, i, x, sum, aii, found, pl, kl);
        else if constexpr (R > 0)
            sell_rest<T, COL16, DIAG, R - 1, LAST>(rest, A, p0, g0, first, cur, len, i, x, sum, aii, found, pl, kl);
    }
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
    constexpr int V = sell_vec<T>();
    constexpr int BG = spmv_batch<T>() / V; // groups per batch
    const int lane = (int)(i & 63);
    const long long p0 = base + (long long)V * lane;
    int first = 0, cur = 0;
    if constexpr (COL16)
        first = (i < A.n ? (int)i : A.n - 1) + A.cfirst[__builtin_amdgcn_readfirstlane((int)(i >> 6))];
    const int groups = width / V;
    T sum = T(0);
    int g0 = 0;
    for (; g0 + BG <= groups; g0 += BG) sell_batch<T, COL16, DIAG, BG>(A, p0, g0, first, cur, len, i, x, sum, aii, found);
    // the remaining groups (fewer than a batch) as one more batch, so a
    // short row (a 7-point row is three groups and its last column) waits
    // for memory once
    if (V > 1 && (width % V) != 0) // odd width: the single-entry last column joins this batch
        sell_rest<T, COL16, DIAG, BG - 1, true>(groups - g0, A, p0, g0, first, cur, len, i, x, sum, aii, found,
                                                 base + 64ll * (width - 1) + lane, width - 1);
    else
        sell_rest<T, COL16, DIAG, BG - 1, false>(groups - g0, A, p0, g0, first, cur, len, i, x, sum, aii, found, 0, 0);
    return sum;
}

} // namespace rpcg
