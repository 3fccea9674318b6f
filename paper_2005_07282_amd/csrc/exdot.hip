// Standalone dot product kernels (exact, expansion-based and plain), the
// rounding of a long accumulator, and the CSR SpMV.
#include "reduce.hpp"

#include <algorithm>

namespace rpcg {

// ---------------------------------------------------------------------------
// Standalone dot product: per-workgroup partials, then a one-workgroup
// finalize that merges them and rounds once.

constexpr int EX_COPIES = 4;
constexpr int EX_PITCH = ACC_DIGITS; // 136 dwords: copies 8 banks apart

template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_exdot_part(long long n, const double *__restrict__ x, const double *__restrict__ y, SlotView sv,
             DotInfo *info, bool ee, bool capture)
{
    __shared__ RedShared sh;
    // lanes add into one of EX_COPIES copies of the long accumulator by
    // lane & (EX_COPIES - 1), so lanes that hit the same word in the same
    // instruction mostly hit different addresses (copies EX_PITCH words
    // apart start in different LDS banks); summed into copy 0 at the end
    __shared__ long long accx[EX_COPIES - 1][EX_PITCH];
    long long *acc = sh.acc[0];
    zero_acc(acc);
    for (int q = threadIdx.x; q < (EX_COPIES - 1) * EX_PITCH; q += blockDim.x) (&accx[0][0])[q] = 0;
    __syncthreads();
    const int cp = threadIdx.x & (EX_COPIES - 1);
    long long *accl = cp ? accx[cp - 1] : acc;

    LaneDot<MODE, P, MODE != MODE_PLAIN> L;
    L.init();
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const bool vec = ((((uintptr_t)x) | ((uintptr_t)y)) & 15) == 0;
    if (vec) {
        const long long n2 = n >> 1;
        const double2 *x2 = reinterpret_cast<const double2 *>(x);
        const double2 *y2 = reinterpret_cast<const double2 *>(y);
        for (long long i = tid; i < n2; i += stride) {
            double2 a = x2[i], b = y2[i];
            L.add(a.x, b.x, accl, ee, capture);
            L.add(a.y, b.y, accl, ee, capture);
        }
        if ((n & 1) && tid == 0) L.add(x[n - 1], y[n - 1], accl, ee, capture);
    } else {
        for (long long i = tid; i < n; i += stride) L.add(x[i], y[i], accl, ee, capture);
    }
    if constexpr (MODE != MODE_PLAIN) {
        __syncthreads();
        for (int q = threadIdx.x; q < ACC_DIGITS; q += blockDim.x) {
            long long v = acc[q];
#pragma unroll
            for (int c = 0; c < EX_COPIES - 1; ++c) v += accx[c][q];
            acc[q] = v;
        }
        __syncthreads();
    }
    block_finish<MODE, P>(L, acc, sv, blockIdx.x, ee, capture, &info->flags, sh);
}

// One workgroup: merges the G slots, rounds, writes *out and the counters;
// or, with digits_out, writes the exact sum as normalized accumulator words.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_exdot_fin(int G, SlotView sv, DotInfo *info, double *out, long long *digits_out, bool ee, bool capture)
{
    __shared__ RedShared sh;
    long long *acc = sh.acc[0];
    if (digits_out) {
        if constexpr (MODE == MODE_EXBLAS) {
            zero_acc(acc);
            __syncthreads();
            for (int k = wave_id(); k < ACC_DIGITS; k += num_waves()) {
                long long s = sum_row(sv.ws.digits + (long long)k * sv.stride, G);
                if (lane_id() == 0) acc[k] = s;
            }
            __syncthreads();
            if (wave_id() == 0) {
                const int l = lane_id();
                long long a = (2 * l < ACC_DIGITS) ? acc[2 * l] : 0;
                long long b = (2 * l + 1 < ACC_DIGITS) ? acc[2 * l + 1] : 0;
                wave_normalize(a, b);
                if (2 * l < ACC_DIGITS) digits_out[2 * l] = a;
                if (2 * l + 1 < ACC_DIGITS) digits_out[2 * l + 1] = b;
            }
        }
        return;
    }
    long long esc = 0;
    int fl = 0;
    double r = merge_slots<MODE, P>(sv, G, ee, capture, acc, &esc, &info->flags, sh, 0);
    if (threadIdx.x == 0) {
        fl = info->flags;
        *out = (fl & FLAG_NONFINITE) ? __builtin_nan("") : r;
        if constexpr (MODE == MODE_FPE) {
            info->escapes += esc;
            if (esc > 0 && capture) info->fallbacks += 1;
        }
    }
}

__global__ void k_acc_round(const long long *digits, double *out)
{
    __shared__ long long acc[ACC_DIGITS];
    for (int k = threadIdx.x; k < ACC_DIGITS; k += blockDim.x) acc[k] = digits[k];
    __syncthreads();
    double r = wave_acc_round(acc);
    if (threadIdx.x == 0) *out = r;
}

// ---------------------------------------------------------------------------
// SpMV on CSR (Section 4.3): y_i = fold over the stored entries of row i, in
// storage order, of acc = fma(a_ik, x[col_k], acc), acc from +0.
//
// A workgroup owns SPMV_R consecutive rows (one per thread); their entries
// form one contiguous range of the CSR arrays. The range is staged through
// LDS in chunks of SPMV_E entries: consecutive threads load consecutive
// values and columns (coalesced, streamed once) and gather the x entries;
// then every thread continues its own row's fma chain over the part of the
// row inside the chunk, reading LDS. The accumulator stays in the row's
// thread across chunks, so a row of any length is one sequential chain in
// storage order, exactly as the definition reads.
// The next chunk's values and columns are loaded under the current chunk's
// chains and its x entries gathered right after them, so rows longer than a
// chunk's share no longer leave the memory idle while their chains run.

#ifndef RPCG_SPMV_R
#define RPCG_SPMV_R 512
#endif
#ifndef RPCG_SPMV_E
#define RPCG_SPMV_E 2048
#endif
constexpr int SPMV_R = RPCG_SPMV_R; // rows per workgroup (= threads)
constexpr int SPMV_E = RPCG_SPMV_E; // chunk of entries staged at a time

template <int R, int E>
__global__ void __launch_bounds__(R)
k_spmv_csr(int n, const int *__restrict__ rp, const int *__restrict__ col, const double *__restrict__ val,
           const double *__restrict__ x, double *__restrict__ y)
{
    constexpr int PER = E / R; // entries each thread stages per chunk
    static_assert(E % R == 0, "chunk shape");
    __shared__ double2 st[E]; // (a_k, x[col_k]) of the chunk's entries
    const int t = threadIdx.x;
    for (long long r0 = (long long)blockIdx.x * R; r0 < n; r0 += (long long)gridDim.x * R) {
        const long long r1 = r0 + R < n ? r0 + R : n;
        const long long i = r0 + t;
        const long long b0 = rp[r0], b1 = rp[r1];
        long long rs = b1, re = b1;
        if (i < r1) { rs = rp[i]; re = rp[i + 1]; }
        double acc = 0.0;
        double a[PER], g[PER];
        int c[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const long long k = b0 + j * R + t;
            const bool in = k < b1;
            a[j] = in ? __builtin_nontemporal_load(val + k) : 0.0;
            c[j] = in ? __builtin_nontemporal_load(col + k) : 0;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) g[j] = x[c[j]];
        for (long long k0 = b0; k0 < b1; k0 += E) {
            if (k0 != b0) __syncthreads(); // the previous chunk has been read
#pragma unroll
            for (int j = 0; j < PER; ++j) st[j * R + t] = make_double2(a[j], g[j]);
            __syncthreads();
            const long long k1 = k0 + E;
            if (k1 < b1) { // the next chunk's values and columns, loaded under this chunk's chains
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const long long k = k1 + j * R + t;
                    const bool in = k < b1;
                    a[j] = in ? __builtin_nontemporal_load(val + k) : 0.0;
                    c[j] = in ? __builtin_nontemporal_load(col + k) : 0;
                }
            }
            const int lo = (int)((rs > k0 ? rs : k0) - k0);
            const int hi = (int)((re < k0 + E ? re : k0 + E) - k0);
            int k = lo;
            for (; k + 4 <= hi; k += 4) {
                const double2 e0 = st[k], e1 = st[k + 1], e2 = st[k + 2], e3 = st[k + 3];
                acc = __builtin_fma(e0.x, e0.y, acc);
                acc = __builtin_fma(e1.x, e1.y, acc);
                acc = __builtin_fma(e2.x, e2.y, acc);
                acc = __builtin_fma(e3.x, e3.y, acc);
            }
            for (; k < hi; ++k) acc = __builtin_fma(st[k].x, st[k].y, acc);
            if (k1 < b1) {
#pragma unroll
                for (int j = 0; j < PER; ++j) g[j] = x[c[j]];
            }
        }
        if (i < r1) y[i] = acc;
        __syncthreads(); // the next block's first chunk overwrites st
    }
}

// ---------------------------------------------------------------------------
// Launch functions

hipError_t launch_exdot(int mode, long long n, const double *x, const double *y, double *out,
                        const DotWs &ws, int stride, DotInfo *info, const LaunchCfg &c)
{
    SlotView sv{ws, stride};
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        k_exdot_part<M, PP><<<c.grid, c.block, 0, c.stream>>>(n, x, y, sv, info, c.early_exit, c.fallback);
        k_exdot_fin<M, PP><<<1, MAX_BLOCK, 0, c.stream>>>(c.grid, sv, info, out, nullptr, c.early_exit,
                                                          c.fallback);
    });
    return hipGetLastError();
}

hipError_t launch_exdot_partial(long long n, const double *x, const double *y, long long *digits,
                                const DotWs &ws, int stride, DotInfo *info, const LaunchCfg &c)
{
    SlotView sv{ws, stride};
    k_exdot_part<MODE_EXBLAS, 4><<<c.grid, c.block, 0, c.stream>>>(n, x, y, sv, info, true, true);
    k_exdot_fin<MODE_EXBLAS, 4><<<1, MAX_BLOCK, 0, c.stream>>>(c.grid, sv, info, nullptr, digits, true, true);
    return hipGetLastError();
}

hipError_t launch_acc_round(const long long *digits, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_acc_round, dim3(1), dim3(64), 0, s, digits, out);
    return hipGetLastError();
}

hipError_t launch_spmv_csr(int n, long long nnz, const int *row_ptr, const int *col, const double *val,
                           const double *x, double *y, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const long long blocks = ((long long)n + SPMV_R - 1) / SPMV_R;
    const unsigned g = (unsigned)std::min<long long>(blocks, 65536);
    // short rows (under 32 entries on average) fill a chunk with many rows:
    // half-size chunks keep more workgroups per CU (measured 160^3: 0.58
    // against 0.56 of 8 TB/s); long rows need the full chunk
    if (nnz < 32ll * n)
        hipLaunchKernelGGL((k_spmv_csr<SPMV_R, SPMV_E / 2>), dim3(g), dim3(SPMV_R), 0, s, n, row_ptr, col, val, x, y);
    else
        hipLaunchKernelGGL((k_spmv_csr<SPMV_R, SPMV_E>), dim3(g), dim3(SPMV_R), 0, s, n, row_ptr, col, val, x, y);
    return hipGetLastError();
}

// Smallest and largest binary exponent (floor(log2 |v|)) over the nonzero
// finite entries of v; *emin / *emax are lowered / raised atomically.
__global__ void k_exp_range(long long n, const double *__restrict__ v, int *emin, int *emax)
{
    int lo = 1 << 20, hi = -(1 << 20);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v[i]) & 0x7FFFFFFFFFFFFFFFull;
        if (b == 0 || (b >> 52) == 0x7FF) continue;
        const int be = (int)(b >> 52);
        const int e = be ? be - 1023 : (63 - __builtin_clzll(b)) - 1074;
        lo = min(lo, e);
        hi = max(hi, e);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off, 64));
        hi = max(hi, __shfl_xor(hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(emin, lo);
        atomicMax(emax, hi);
    }
}

hipError_t launch_exp_range(long long n, const double *v, int *emin, int *emax, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<long long>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_exp_range, dim3(grid), dim3(256), 0, s, n, v, emin, emax);
    return hipGetLastError();
}

} // namespace rpcg
