// Row-wise CSR product shared by the factored-preconditioner kernels.
#pragma once

#include "reduce.hpp"
#include "sell_spmv.hpp"

namespace rpcg {

// y_i = fold over row i of fma(m_ik, x[col_k], acc) from +0.
__device__ __forceinline__ double csr_row(const int *__restrict__ rp, const int *__restrict__ col,
                                          const double *__restrict__ val, const double *__restrict__ x, long long i)
{
    double acc = 0.0;
    const int k1 = rp[i + 1];
    for (int k = rp[i]; k < k1; ++k) acc = __builtin_fma(val[k], x[col[k]], acc);
    return acc;
}

// t = G^T r (one row per thread).
__global__ void k_fac_gt(int n, FacPre Pr, const double *__restrict__ r, double *__restrict__ t, const PcgState *st);

// z = G t + eps r (and d = z at setup); partials of <z, r>.
template <int MODE, int P, bool SETUP>
__global__ void __launch_bounds__(MAX_BLOCK)
k_fac_z(int n, FacPre Pr, PcgVecs<double> v, const double *__restrict__ t, PcgState *st, SlotView wb, bool ee,
        bool capture)
{
    __shared__ RedShared sh;
    if (!SETUP && wg_read_flag(&st->done, sh)) return;
    zero_acc(sh.acc[0]);
    __syncthreads();
    LaneDot<MODE, P> Lb;
    Lb.init();
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double ri = v.r[i];
        const double zi = __builtin_fma(Pr.eps, ri, csr_row(Pr.g_rp, Pr.g_col, Pr.g_val, t, i));
        v.z[i] = zi;
        if (SETUP) v.d[i] = zi;
        Lb.add(zi, ri, sh.acc[0], ee, capture);
    }
    block_finish<MODE, P>(Lb, sh.acc[0], wb, blockIdx.x, ee, capture, &st->flags, sh);
}

} // namespace rpcg
