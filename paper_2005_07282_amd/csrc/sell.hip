// Conversion of the caller's CSR matrix into the sliced-ELL layout used by
// the solver's SpMV (rows and their entry order unchanged; layout described
// with SellMat).
//
// Both passes give one wavefront to each slice of 64 rows: lane j owns row
// 64s+j, and the lanes stride together through the slice's contiguous CSR
// range, so every global read is coalesced. The row of entry e is found by a
// binary search over the slice's row starts, which sit one per lane.
#include "kernels.hpp"

namespace rpcg {

__device__ __forceinline__ int lane_of() { return threadIdx.x & 63; }

// Row (0..63 within the slice) of CSR entry e: the last of the first
// `nrows` lanes whose row start is <= e (row starts are non-decreasing and
// lane 0's start is <= e). Binary lifting with a fixed six steps, so every
// lane takes part in every shuffle.
__device__ __forceinline__ int slice_row_of(int start, long long e, int nrows)
{
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int cand = lo + step;
        const int sc = __shfl(start, min(cand, nrows - 1), 64);
        if (cand < nrows && sc <= e) lo = cand;
    }
    return lo;
}

// First row (0..63 within the slice) of maximal length: the slice's base row,
// whose first-column offset becomes the slice's cfirst.
__device__ __forceinline__ int slice_base_row(bool row, int len, int w)
{
    const unsigned long long m = __ballot(row && len == w);
    return m ? __builtin_ctzll(m) : 0;
}

// Rank-0 column code of a row (see SellMat): first column - min(i, n-1) -
// fb, or for a row without entries the shift that lands on a valid column.
__device__ __forceinline__ long long first_code(int n, long long rbase, long long fb, bool has_entry, int c0)
{
    if (has_entry) return (long long)c0 - rbase - fb;
    const long long t = rbase + fb;
    const long long tc = t < 0 ? 0 : (t >= n ? n - 1 : t);
    return tc - t;
}

// The slice's fb: first-column offset of its base row (0 if the slice has no
// entries). Every lane returns it; rows must be consistent.
__device__ __forceinline__ long long slice_fb(const int *__restrict__ col, long long s, bool row, int a, int len, int w)
{
    const int b = slice_base_row(row, len, w);
    const int ab = __shfl(a, b, 64);
    return w > 0 ? (long long)col[ab] - (s * 64 + b) : 0;
}

// Pass 1 (one wavefront per slice): structural check of the CSR (row_ptr[0] =
// 0, row_ptr[n] = nnz, non-decreasing, columns in [0, n)), slice widths
// (rounded up to a multiple of vec), the longest row, and whether the 16-bit
// column codes can represent the slice: *max_delta receives the largest
// |rank-0 code|, or 2^40 if a step between consecutive columns of a row is
// negative or above 65535.
__global__ void k_csr_scan(int n, int nnz, int nslices, const int *__restrict__ rp, const int *__restrict__ col,
                           int vec, long long *off_plus1, int *bad, int *max_len, long long *max_delta)
{
    const int lane = lane_of();
    const long long s = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (s >= nslices) return; // whole wavefronts leave together
    const long long i = s * 64 + lane;
    const bool row = i < n;
    const int nrows = (int)min(64ll, (long long)n - s * 64);
    int a = 0, b = 0;
    if (row) { a = rp[i]; b = rp[i + 1]; }
    bool ok = !row || (a >= 0 && a <= b && b <= nnz);
    if (row && i == 0 && a != 0) ok = false;
    if (row && i == n - 1 && b != nnz) ok = false;
    const int len = row ? b - a : 0;
    int w = len;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) w = max(w, __shfl_xor(w, off, 64));
    const bool all_ok = __ballot(!ok) == 0;
    if (lane == 0) {
        off_plus1[s] = 64ll * ((w + vec - 1) / vec * vec);
        atomicMax(max_len, w);
    }
    if (!all_ok) {
        if (lane == 0) atomicOr(bad, 1);
        return;
    }
    const long long fb = slice_fb(col, s, row, a, len, w);
    const long long rbase = row ? i : n - 1;
    long long d0 = first_code(n, rbase, fb, len > 0, len > 0 ? col[a] : 0);
    unsigned long long dmax = (unsigned long long)(d0 < 0 ? -d0 : d0);
    // rows are consistent: the slice's entries are [start of row 0, end of the last row)
    const int e0 = __shfl(a, 0, 64), e1 = __shfl(b, nrows - 1, 64);
    bool cok = true;
    // uniform trip count: every lane takes part in the shuffles of the search
    for (long long t = e0; t < e1; t += 64) {
        const long long e = t + lane;
        const bool in = e < e1;
        const int r = slice_row_of(a, in ? e : t, nrows);
        const int ar = __shfl(a, r, 64);
        if (in) {
            const int c = col[e];
            if (c < 0 || c >= n) cok = false;
            if (e > ar) {
                const long long step = (long long)c - (long long)col[e - 1];
                if (step < 0 || step > 65535) dmax = 1ull << 40;
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        dmax = max(dmax, (unsigned long long)__shfl_xor((long long)dmax, off, 64));
    if (__ballot(!cok) != 0 && lane == 0) atomicOr(bad, 1);
    if (lane == 0) atomicMax((unsigned long long *)max_delta, dmax);
}

// In-place inclusive prefix sum of off[1..nslices] with off[0] = 0, one workgroup of 1024.
__global__ void __launch_bounds__(1024) k_sell_scan(long long *off, int nslices)
{
    __shared__ long long part[1024];
    int t = threadIdx.x;
    long long chunk = (nslices + 1023) / 1024;
    long long b = 1 + t * chunk, e = min((long long)nslices + 1, b + chunk);
    long long s = 0;
    for (long long i = b; i < e; ++i) s += off[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        long long v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    long long run = t ? part[t - 1] : 0;
    for (long long i = b; i < e; ++i) { run += off[i]; off[i] = run; }
    if (t == 0) off[0] = 0;
}

// Pass 2 (one wavefront per slice): padding first, then every CSR entry e of
// the slice goes to the position of rank k = e - row start in row j of the
// slice (see SellMat). Padding entries hold the value 0 and a valid column
// (code 0 repeats the previous column; with 32-bit columns the row itself,
// or row n-1 for lanes past the last row). Columns are stored as 32-bit
// indices (scol) or as 16-bit codes (scol16 with cfirst). Values (type TIN)
// are written as binary64 to sval64 and rounded to nearest binary32 into
// sval32, for whichever of the two is non-null.
template <typename TIN>
__global__ void k_sell_fill(int n, int nslices, const int *__restrict__ rp, const int *__restrict__ col,
                            const TIN *__restrict__ val, int vec, const long long *__restrict__ off,
                            double *__restrict__ sval64, float *__restrict__ sval32, int *__restrict__ scol,
                            unsigned short *__restrict__ scol16, int *__restrict__ cfirst,
                            unsigned char *__restrict__ len8)
{
    const int lane = lane_of();
    const long long s = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (s >= nslices) return;
    const long long i = s * 64 + lane;
    const bool row = i < n;
    const int nrows = (int)min(64ll, (long long)n - s * 64);
    const long long base = off[s];
    const int width = (int)((off[s + 1] - base) >> 6);
    const int a = row ? rp[i] : 0;
    const int len = row ? rp[i + 1] - a : 0;
    const int rbase = row ? (int)i : n - 1;
    int w = len;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, 64));
    const long long fb = slice_fb(col, s, row, a, len, w);
    if (scol16 && lane == 0) cfirst[s] = (int)fb;
    auto pos = [&](int k, int j) { return base + 64ll * vec * (k / vec) + (long long)vec * j + (k % vec); };
    if (len8 && row) len8[i] = (unsigned char)len;
    for (int k = len; k < width; ++k) {
        const long long p = pos(k, lane);
        if (sval64) sval64[p] = 0.0;
        if (sval32) sval32[p] = 0.0f;
        if (scol16) scol16[p] = (k == 0) ? (unsigned short)(short)first_code(n, rbase, fb, false, 0) : 0;
        else scol[p] = rbase;
    }
    const int e0 = __shfl(a, 0, 64), e1 = __shfl(a + len, nrows - 1, 64);
    for (long long t = e0; t < e1; t += 64) { // uniform trip count (shuffles below)
        const long long e = t + lane;
        const bool in = e < e1;
        const int r = slice_row_of(a, in ? e : t, nrows);
        const int ar = __shfl(a, r, 64);
        if (in) {
            const int k = (int)(e - ar);
            const long long p = pos(k, r);
            const int c = col[e];
            const double v = (double)val[e]; // exact for either input type
            if (sval64) sval64[p] = v;
            if (sval32) sval32[p] = (float)v;
            if (scol16) {
                const long long code = k == 0 ? first_code(n, s * 64 + r, fb, true, c) : (long long)c - col[e - 1];
                scol16[p] = (unsigned short)code;
            } else {
                scol[p] = c;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Launch functions

hipError_t launch_csr_scan(int n, int nnz, const int *row_ptr, const int *col, int vec, long long *off_plus1,
                           int *bad, int *max_len, long long *max_delta, hipStream_t s)
{
    const int nslices = (n + 63) / 64;
    if (nslices == 0) return hipSuccess;
    if (vec < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_csr_scan, dim3((nslices + 3) / 4), dim3(256), 0, s, n, nnz, nslices, row_ptr, col, vec,
                       off_plus1, bad, max_len, max_delta);
    return hipGetLastError();
}

hipError_t launch_sell_scan(long long *off, int nslices, hipStream_t s)
{
    hipLaunchKernelGGL(k_sell_scan, dim3(1), dim3(1024), 0, s, off, nslices);
    return hipGetLastError();
}

hipError_t launch_sell_fill(int n, const int *row_ptr, const int *col, const double *val64_in,
                            const float *val32_in, int vec, const long long *off, double *sval64, float *sval32,
                            int *scol, unsigned short *scol16, int *cfirst, unsigned char *len8, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if ((val64_in == nullptr) == (val32_in == nullptr) || vec < 1 || (scol16 && !cfirst)) return hipErrorInvalidValue;
    const int nslices = (n + 63) / 64;
    const dim3 grid((nslices + 3) / 4), block(256);
    if (val64_in)
        hipLaunchKernelGGL(k_sell_fill<double>, grid, block, 0, s, n, nslices, row_ptr, col, val64_in, vec, off,
                           sval64, sval32, scol, scol16, cfirst, len8);
    else
        hipLaunchKernelGGL(k_sell_fill<float>, grid, block, 0, s, n, nslices, row_ptr, col, val32_in, vec, off,
                           sval64, sval32, scol, scol16, cfirst, len8);
    return hipGetLastError();
}

} // namespace rpcg
