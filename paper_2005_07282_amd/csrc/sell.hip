// Conversion of the caller's CSR matrix into the sliced-ELL layout used by
// the solver's SpMV (rows and their entry order unchanged; layout described
// with SellMat).
//
// Both passes work on slices of 64 rows with lane j owning row 64s+j. The
// scan strides the lanes together through the slice's contiguous CSR range
// (the row of entry e is found by a binary search over the slice's row
// starts, which sit one per lane); the fill gathers rank chunks row segment
// by row segment and writes them through LDS.
#include "kernels.hpp"
#include "sell_spmv.hpp"

#include <algorithm>

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

// Raise *p to v (an atomic max), skipping the atomic when a coherent read
// already shows a value >= v: the maxima settle early, so most wavefronts
// leave without touching the contended word.
__device__ __forceinline__ void max_to(int *p, int v)
{
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) atomicMax(p, v);
}
__device__ __forceinline__ void max_to(unsigned long long *p, unsigned long long v)
{
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) atomicMax(p, v);
}

// Pass 1, one slice at a time per wavefront (grid-stride): structural check
// of the CSR (row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing, columns in
// [0, n)), slice widths (the slice's longest row), the longest row,
// and whether the 16-bit column codes can represent the slice: *max_delta
// receives the largest |rank-0 code|, or 2^40 if a step between consecutive
// columns of a row is negative or above 65535. Each wavefront keeps its
// maxima in registers and publishes them once.
__global__ void k_csr_scan(int n, int nnz, int nslices, const int *__restrict__ rp, const int *__restrict__ col,
                           int vec, long long *off_plus1, int *bad, int *max_len, long long *max_delta)
{
    const int lane = lane_of();
    const long long wave0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    int wmax = 0;
    unsigned long long dmax = 0;
    bool failed = false;
    for (long long s = wave0; s < nslices; s += nwaves) { // wavefront-uniform
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
        if (lane == 0) off_plus1[s] = 64ll * w; // an odd width ends in a single-entry column
        wmax = max(wmax, w);
        if (__ballot(!ok) != 0) { // rows inconsistent: the entries are not read
            failed = true;
            continue;
        }
        const long long fb = slice_fb(col, s, row, a, len, w);
        const long long rbase = row ? i : n - 1;
        const long long d0 = first_code(n, rbase, fb, len > 0, len > 0 ? col[a] : 0);
        dmax = max(dmax, (unsigned long long)(d0 < 0 ? -d0 : d0));
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
        if (__ballot(!cok) != 0) failed = true;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        dmax = max(dmax, (unsigned long long)__shfl_xor((long long)dmax, off, 64));
    if (lane == 0) {
        if (failed) atomicOr(bad, 1);
        max_to(max_len, wmax);
        max_to((unsigned long long *)max_delta, dmax);
    }
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

// Pass 2, one workgroup of one wavefront per slice. Padding entries hold the
// value 0 and a valid column (code 0 repeats the previous column; with
// 32-bit columns the row itself, or row n-1 for lanes past the last row).
// Columns are stored as 32-bit indices (scol) or as 16-bit codes (scol16 with
// cfirst). Values (type TIN) are written as binary64 to sval64 and rounded
// to nearest binary32 into sval32, for whichever of the two is non-null.
//
// The slice's block is filled in chunks of FILL_RANKS ranks, which occupy a
// contiguous run of the layout (FILL_RANKS is a multiple of vec). A chunk is
// gathered with consecutive lanes on consecutive entries of a row (row
// segments of FILL_RANKS entries), transposed through LDS, and written out
// as one contiguous run, so both the CSR reads and the layout writes are
// coalesced (scattered narrow stores would leave partly written lines to be
// merged in HBM).
constexpr int FILL_RANKS = 16;
constexpr int FILL_PITCH = 65; // LDS row pitch: ranks apart land in different banks

template <typename TIN>
__global__ void __launch_bounds__(64) k_sell_fill(int n, int nslices, const int *__restrict__ rp,
                                                  const int *__restrict__ col, const TIN *__restrict__ val, int vec,
                                                  const long long *__restrict__ off, double *__restrict__ sval64,
                                                  float *__restrict__ sval32, int *__restrict__ scol,
                                                  unsigned short *__restrict__ scol16, int *__restrict__ cfirst,
                                                  unsigned char *__restrict__ len8)
{
    __shared__ double tv[FILL_RANKS * FILL_PITCH];
    __shared__ int tc[FILL_RANKS * FILL_PITCH];
    const int lane = threadIdx.x;
    const long long s = blockIdx.x;
    const long long i = s * 64 + lane;
    const bool row = i < n;
    const long long base = off[s];
    const int width = (int)((off[s + 1] - base) >> 6);
    const int a = row ? rp[i] : 0;
    const int len = row ? rp[i + 1] - a : 0;
    int w = len;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, 64));
    const long long fb = slice_fb(col, s, row, a, len, w);
    if (scol16 && lane == 0) cfirst[s] = (int)fb;
    if (len8 && row) len8[i] = (unsigned char)len;
    constexpr int ROWS_PER_STEP = 64 / FILL_RANKS;
    const int kk = lane % FILL_RANKS;   // rank within the chunk gathered by this lane
    const int rsub = lane / FILL_RANKS; // row within each group of ROWS_PER_STEP rows
    for (int k0 = 0; k0 < width; k0 += FILL_RANKS) {
        const int k = k0 + kk;
#pragma unroll 4
        for (int g = 0; g < 64 / ROWS_PER_STEP; ++g) {
            const int r = g * ROWS_PER_STEP + rsub;
            const int ar = __shfl(a, r, 64), lr = __shfl(len, r, 64);
            const long long rbase = (s * 64 + r < n) ? s * 64 + r : n - 1;
            double v = 0.0;
            int c;
            if (k < lr) {
                const long long e = (long long)ar + k;
                const int ce = col[e];
                v = (double)val[e]; // exact for either input type
                if (scol16) c = k == 0 ? (int)first_code(n, rbase, fb, true, ce) : ce - col[e - 1];
                else c = ce;
            } else {
                if (scol16) c = k == 0 ? (int)first_code(n, rbase, fb, false, 0) : 0;
                else c = (int)rbase;
            }
            tv[kk * FILL_PITCH + r] = v;
            tc[kk * FILL_PITCH + r] = c;
        }
        __syncthreads();
        // the chunk's run in layout order: t = 64 vec (q / vec) + vec j + q % vec for rank k0 + q of row j
        const int nk = min(FILL_RANKS, width - k0);
        const long long run = base + 64ll * k0;
        // chunk rank of the single-entry last column of an odd width (even,
        // as k0 is), past the chunk when there is none here
        const int tq = (vec > 1 && (width % vec) != 0) ? width - 1 - k0 : FILL_RANKS;
        for (int t = lane; t < 64 * nk; t += 64) {
            const bool last = t >= 64 * tq;
            const int q = last ? tq : vec * (t / (64 * vec)) + t % vec;
            const int j = last ? t - 64 * tq : (t % (64 * vec)) / vec;
            const double v = tv[q * FILL_PITCH + j];
            const int c = tc[q * FILL_PITCH + j];
            if (sval64) sval64[run + t] = v;
            if (sval32) sval32[run + t] = (float)v;
            if (scol16) scol16[run + t] = (unsigned short)c;
            else scol[run + t] = c;
        }
        __syncthreads();
    }
}

// y = A x on a prepared sliced-ELL copy (Section 4.3): lane j of a wavefront
// computes row 64 s + j as the sequential fma chain of sell_row (the same
// chain, from +0 in storage order, as the CSR kernel); wavefronts stride over
// the slices.
template <bool COL16>
__global__ void __launch_bounds__(256) k_sell_spmv(SellMat<double> A, const double *__restrict__ x,
                                                   double *__restrict__ y)
{
    const int lane = lane_of();
    const int W = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (long long s = (long long)blockIdx.x * W + wave; s < A.nslices; s += (long long)gridDim.x * W) {
        const long long base = uniform_ll(A.off[s]);
        const int width = __builtin_amdgcn_readfirstlane((int)((A.off[s + 1] - base) >> 6));
        const long long i = s * 64 + lane;
        const int len = sell_len(A, i);
        const double sum = sell_row<double, COL16, false>(A, base, width, i, len, x, nullptr, nullptr);
        if (i < A.n) y[i] = sum;
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
    const int grid = (int)std::min<long long>((nslices + 3) / 4, 4096);
    hipLaunchKernelGGL(k_csr_scan, dim3(grid), dim3(256), 0, s, n, nnz, nslices, row_ptr, col, vec, off_plus1, bad,
                       max_len, max_delta);
    return hipGetLastError();
}

hipError_t launch_sell_spmv(const SellMat<double> &A, const double *x, double *y, int grid, hipStream_t s)
{
    if (A.nslices == 0) return hipSuccess;
    if (grid < 1) return hipErrorInvalidValue;
    if (A.col16) hipLaunchKernelGGL(k_sell_spmv<true>, dim3(grid), dim3(256), 0, s, A, x, y);
    else hipLaunchKernelGGL(k_sell_spmv<false>, dim3(grid), dim3(256), 0, s, A, x, y);
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
    if ((val64_in == nullptr) == (val32_in == nullptr) || vec < 1 || FILL_RANKS % vec != 0 || (scol16 && !cfirst))
        return hipErrorInvalidValue;
    const int nslices = (n + 63) / 64;
    const dim3 grid(nslices), block(64);
    if (val64_in)
        hipLaunchKernelGGL(k_sell_fill<double>, grid, block, 0, s, n, nslices, row_ptr, col, val64_in, vec, off,
                           sval64, sval32, scol, scol16, cfirst, len8);
    else
        hipLaunchKernelGGL(k_sell_fill<float>, grid, block, 0, s, n, nslices, row_ptr, col, val32_in, vec, off,
                           sval64, sval32, scol, scol16, cfirst, len8);
    return hipGetLastError();
}

} // namespace rpcg
