// Standalone dot product kernels (exact, expansion-only and plain), the
// rounding of a long accumulator, and the CSR SpMV.
#include "reduce.hpp"

namespace rpcg {

// ---------------------------------------------------------------------------
// Standalone dot product

template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_exdot(long long n, const double *__restrict__ x, const double *__restrict__ y, double *out,
        DotWs ws, DotInfo *info, bool ee, bool fallback, bool conditional, long long *digits_out)
{
    __shared__ RedShared sh;
    if (conditional && info->need_fallback == 0) return;
    long long *acc = sh.acc[0];
    if constexpr (MODE == MODE_EXBLAS) zero_acc(acc);
    if (threadIdx.x == 0) sh.flags = 0;
    __syncthreads();

    LaneDot<MODE, P> L;
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
            L.add(a.x, b.x, acc, ee);
            L.add(a.y, b.y, acc, ee);
        }
        if ((n & 1) && tid == 0) L.add(x[n - 1], y[n - 1], acc, ee);
    } else {
        for (long long i = tid; i < n; i += stride) L.add(x[i], y[i], acc, ee);
    }
    block_finish<MODE, P>(L, acc, ws, blockIdx.x, ee, &info->flags, sh);
    if (!arrive_last(&info->ticket, sh)) return;

    long long esc = 0;
    double r;
    if (digits_out) {
        // exact partial: sum the slots into the caller's digit vector, fully normalized
        if constexpr (MODE == MODE_EXBLAS) {
            zero_acc(acc);
            __syncthreads();
            for (int k = 0; k < ACC_DIGITS; ++k) {
                long long s = 0;
                for (int g = threadIdx.x; g < (int)gridDim.x; g += blockDim.x)
                    s += ws.digits[(long long)g * ACC_DIGITS + k];
                s = block_sum_ll(s, sh);
                if (threadIdx.x == 0) acc[k] = s;
            }
            if (threadIdx.x == 0) {
                acc_normalize(acc);
                for (int k = 0; k < ACC_DIGITS; ++k) digits_out[k] = acc[k];
            }
        }
        return;
    }
    r = merge_slots<MODE, P>(ws, gridDim.x, ee, acc, &info->flags, &esc, sh);
    if constexpr (MODE == MODE_FPE) {
        if (threadIdx.x == 0) {
            info->escapes += esc;
            info->need_fallback = (fallback && esc > 0) ? 1 : 0;
            *out = r;
        }
    } else {
        if (threadIdx.x == 0) {
            *out = r;
            if (conditional) { info->need_fallback = 0; info->fallbacks += 1; }
        }
    }
}

__global__ void k_acc_round(const long long *digits, double *out)
{
    __shared__ long long acc[ACC_DIGITS];
    for (int k = threadIdx.x; k < ACC_DIGITS; k += blockDim.x) acc[k] = digits[k];
    __syncthreads();
    if (threadIdx.x == 0) *out = acc_round(acc);
}

// ---------------------------------------------------------------------------
// SpMV on CSR: one lane per row, sequential fma chain in storage order.

__global__ void k_spmv_csr(int n, const int *__restrict__ rp, const int *__restrict__ col,
                           const double *__restrict__ val, const double *__restrict__ x,
                           double *__restrict__ y)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) acc = __builtin_fma(val[k], x[col[k]], acc);
        y[i] = acc;
    }
}

// ---------------------------------------------------------------------------
// Launch functions

hipError_t launch_exdot(int mode, long long n, const double *x, const double *y, double *out,
                        const DotWs &ws, DotInfo *info, const LaunchCfg &c)
{
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        k_exdot<decltype(m)::value, decltype(p)::value><<<c.grid, c.block, 0, c.stream>>>(
            n, x, y, out, ws, info, c.early_exit, c.fallback, false, nullptr);
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (mode == MODE_FPE && c.fallback) {
        hipLaunchKernelGGL((k_exdot<MODE_EXBLAS, 4>), dim3(c.grid), dim3(c.block), 0, c.stream,
                           n, x, y, out, ws, info, true, false, true, nullptr);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_exdot_partial(long long n, const double *x, const double *y, long long *digits,
                                const DotWs &ws, DotInfo *info, const LaunchCfg &c)
{
    hipLaunchKernelGGL((k_exdot<MODE_EXBLAS, 4>), dim3(c.grid), dim3(c.block), 0, c.stream,
                       n, x, y, nullptr, ws, info, true, false, false, digits);
    return hipGetLastError();
}

hipError_t launch_acc_round(const long long *digits, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_acc_round, dim3(1), dim3(64), 0, s, digits, out);
    return hipGetLastError();
}

hipError_t launch_spmv_csr(int n, const int *row_ptr, const int *col, const double *val,
                           const double *x, double *y, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int block = 256;
    long long grid = ((long long)n + block - 1) / block;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_spmv_csr, dim3((unsigned)grid), dim3(block), 0, s, n, row_ptr, col, val, x, y);
    return hipGetLastError();
}

} // namespace rpcg
