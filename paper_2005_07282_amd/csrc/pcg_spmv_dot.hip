// Jacobi-PCG iteration, first kernel: SpMV fused with the first dot (S1, S2).
#include "reduce.hpp"

namespace rpcg {

// K1: w = A d (S1) and delta = <d, w> (S2); the last workgroup sets rho.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_spmv_dot(SellMat A, PcgVecs v, PcgState *st, DotWs ws, bool ee, bool fallback)
{
    __shared__ RedShared sh;
    if (st->done) return;
    long long *acc = sh.acc[0];
    if constexpr (MODE == MODE_EXBLAS) zero_acc(acc);
    __syncthreads();
    LaneDot<MODE, P> L;
    L.init();
    const int lane = lane_id();
    const double *__restrict__ d = v.d;
    const long long wstride = (long long)gridDim.x * num_waves();
    for (long long s = (long long)blockIdx.x * num_waves() + wave_id(); s < A.nslices; s += wstride) {
        long long i = s * 64 + lane;
        if (i < A.n) {
            int len = A.row_ptr[i + 1] - A.row_ptr[i];
            const double *__restrict__ pv = A.val + A.off[s] + lane;
            const int *__restrict__ pc = A.col + A.off[s] + lane;
            double sum = 0.0;
            for (int k = 0; k < len; ++k) sum = __builtin_fma(pv[64 * k], d[pc[64 * k]], sum);
            v.w[i] = sum;
            L.add(d[i], sum, acc, ee);
        }
    }
    block_finish<MODE, P>(L, acc, ws, blockIdx.x, ee, &st->flags, sh);
    if (!arrive_last(&st->ticket[1], sh)) return;

    long long esc;
    double delta = merge_slots<MODE, P>(ws, gridDim.x, ee, acc, &st->flags, &esc, sh);
    if constexpr (MODE == MODE_FPE) {
        if (threadIdx.x == 0) sh.need_fb = fallback && esc > 0;
        __syncthreads();
        if (sh.need_fb) {
            double t = block_exact_dot(A.n, v.d, v.w, acc, &st->flags, sh);
            if (threadIdx.x == 0) { delta = t; st->fallbacks += 1; }
        }
    }
    if (threadIdx.x == 0) {
        st->escapes += esc;
        st->delta = delta;
        if ((st->flags & FLAG_NONFINITE) || !is_finite_bits(delta)) { st->status = -6; st->done = 1; }
        else if (!(delta > 0.0)) { st->status = -5; st->done = 1; }
        else st->rho = st->beta / delta;
    }
}

// ---------------------------------------------------------------------------
// Launch functions

hipError_t launch_pcg_spmv_dot(int mode, const SellMat &A, const PcgVecs &v, PcgState *st,
                               const DotWs &ws, const LaunchCfg &c)
{
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        k_pcg_spmv_dot<decltype(m)::value, decltype(p)::value><<<c.grid, c.block, 0, c.stream>>>(
            A, v, st, ws, c.early_exit, c.fallback);
    });
    return hipGetLastError();
}

} // namespace rpcg
