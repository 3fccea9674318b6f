// Conversion of the caller's CSR matrix into the sliced-ELL layout used by
// the solver's SpMV (rows and their entry order unchanged).
#include "kernels.hpp"

namespace rpcg {

// ---------------------------------------------------------------------------
// SELL-64 construction

// Structural check of a CSR matrix: row_ptr[0] = 0, row_ptr[n] = nnz,
// non-decreasing, and every column index in [0, n). Sets *bad on failure.
// Every read stays inside row_ptr[0..n] and col[0..nnz).
__global__ void k_csr_check(int n, int nnz, const int *__restrict__ rp, const int *__restrict__ col, int *bad)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        int a = rp[i], b = rp[i + 1];
        bool ok = a >= 0 && a <= b && b <= nnz;
        if (i == 0 && a != 0) ok = false;
        if (i == n - 1 && b != nnz) ok = false;
        if (ok)
            for (int k = a; k < b; ++k)
                if (col[k] < 0 || col[k] >= n) { ok = false; break; }
        if (!ok) atomicOr(bad, 1);
    }
}

// Width of each slice (longest row), the longest row overall and the largest
// |column - row| (decides whether 16-bit column offsets suffice).
__global__ void k_sell_widths(int n, const int *__restrict__ rp, const int *__restrict__ col, long long *off_plus1,
                              int nslices, int *max_len, int *max_delta)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslices) return;
    int w = 0, dm = 0;
    int i0 = s * 64, i1 = min(n, i0 + 64);
    for (int i = i0; i < i1; ++i) {
        w = max(w, rp[i + 1] - rp[i]);
        for (int k = rp[i]; k < rp[i + 1]; ++k) dm = max(dm, abs(col[k] - i));
    }
    off_plus1[s] = 64ll * w;
    atomicMax(max_len, w);
    atomicMax(max_delta, dm);
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

// One thread per (slice, lane) position, including the lanes past the last
// row of the last slice: every stored position gets a valid column, so the
// SpMV can load and gather a whole slice width without bounds branches.
__global__ void k_sell_fill(int n, int nslices, const int *__restrict__ rp, const int *__restrict__ col,
                            const double *__restrict__ val, const long long *__restrict__ off,
                            double *__restrict__ sval, int *__restrict__ scol, short *__restrict__ scol16,
                            unsigned char *__restrict__ len8)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 64ll * nslices) return;
    long long s = i >> 6, j = i & 63;
    long long base = off[s] + j;
    int width = (int)((off[s + 1] - off[s]) >> 6);
    bool row = i < n;
    int r0 = row ? rp[i] : 0, len = row ? rp[i + 1] - r0 : 0;
    int pad_col = row ? (int)i : 0;
    int rbase = row ? (int)i : n - 1; // 16-bit offsets are relative to min(row, n-1)
    if (len8 && row) len8[i] = (unsigned char)len;
    for (int k = 0; k < width; ++k) {
        bool in = k < len;
        sval[base + 64ll * k] = in ? val[r0 + k] : 0.0;
        if (scol16) scol16[base + 64ll * k] = in ? (short)(col[r0 + k] - rbase) : (short)0;
        else scol[base + 64ll * k] = in ? col[r0 + k] : pad_col;
    }
}

// ---------------------------------------------------------------------------
// Launch functions

hipError_t launch_csr_check(int n, int nnz, const int *row_ptr, const int *col, int *bad, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    long long grid = ((long long)n + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_csr_check, dim3((unsigned)grid), dim3(256), 0, s, n, nnz, row_ptr, col, bad);
    return hipGetLastError();
}

hipError_t launch_sell_widths(int n, const int *row_ptr, const int *col, long long *off_plus1, int nslices,
                              int *max_len, int *max_delta, hipStream_t s)
{
    if (nslices == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sell_widths, dim3((nslices + 255) / 256), dim3(256), 0, s, n, row_ptr, col,
                       off_plus1, nslices, max_len, max_delta);
    return hipGetLastError();
}

hipError_t launch_sell_scan(long long *off, int nslices, hipStream_t s)
{
    hipLaunchKernelGGL(k_sell_scan, dim3(1), dim3(1024), 0, s, off, nslices);
    return hipGetLastError();
}

hipError_t launch_sell_fill(int n, const int *row_ptr, const int *col, const double *val,
                            const long long *off, double *sval, int *scol, short *scol16, unsigned char *len8,
                            hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int nslices = (n + 63) / 64;
    hipLaunchKernelGGL(k_sell_fill, dim3(nslices / 4 + 1), dim3(256), 0, s, n, nslices, row_ptr, col, val,
                       off, sval, scol, scol16, len8);
    return hipGetLastError();
}

} // namespace rpcg
