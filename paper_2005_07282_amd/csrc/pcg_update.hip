// Jacobi-PCG iteration, second and third kernels: vector updates, Jacobi
// preconditioner and the two fused dots (S3-S6, S8), then the search
// direction update (S7).
#include "reduce.hpp"

namespace rpcg {

// K2: x += rho d (S3), r -= rho w (S4), z = dinv r (S5), beta = <z,r> (S6),
// tau = <r,r> (S8); the last workgroup sets gamma, the history and `done`.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_update(int n, PcgVecs v, PcgState *st, DotWs wb, DotWs wt, bool ee, bool fallback)
{
    __shared__ RedShared sh;
    if (st->done) return;
    if constexpr (MODE == MODE_EXBLAS) { zero_acc(sh.acc[0]); zero_acc(sh.acc[1]); }
    __syncthreads();
    const double rho = st->rho;
    LaneDot<MODE, P> Lb, Lt;
    Lb.init(); Lt.init();
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double di = v.d[i], wi = v.w[i];
        v.x[i] = __builtin_fma(rho, di, v.x[i]);
        double ri = __builtin_fma(-rho, wi, v.r[i]);
        double zi = v.dinv[i] * ri;
        v.r[i] = ri;
        v.z[i] = zi;
        Lb.add(zi, ri, sh.acc[0], ee);
        Lt.add(ri, ri, sh.acc[1], ee);
    }
    block_finish<MODE, P>(Lb, sh.acc[0], wb, blockIdx.x, ee, &st->flags, sh);
    block_finish<MODE, P>(Lt, sh.acc[1], wt, blockIdx.x, ee, &st->flags, sh);
    if (!arrive_last(&st->ticket[2], sh)) return;

    long long eb, et;
    double beta = merge_slots<MODE, P>(wb, gridDim.x, ee, sh.acc[0], &st->flags, &eb, sh);
    double tau = merge_slots<MODE, P>(wt, gridDim.x, ee, sh.acc[1], &st->flags, &et, sh);
    if constexpr (MODE == MODE_FPE) {
        if (threadIdx.x == 0) sh.need_fb = fallback && (eb + et) > 0;
        __syncthreads();
        if (sh.need_fb) {
            double t0 = block_exact_dot(n, v.z, v.r, sh.acc[0], &st->flags, sh);
            double t1 = block_exact_dot(n, v.r, v.r, sh.acc[0], &st->flags, sh);
            if (threadIdx.x == 0) { beta = t0; tau = t1; st->fallbacks += 1; }
        }
    }
    if (threadIdx.x == 0) {
        st->escapes += eb + et;
        if ((st->flags & FLAG_NONFINITE) || !is_finite_bits(beta) || !is_finite_bits(tau)) {
            st->status = -6;
            st->done = 1;
        } else {
            st->gamma = beta / st->beta;
            st->beta = beta;
            st->tau = tau;
            int it = st->iter + 1;
            st->iter = it;
            if (v.hist) v.hist[it] = tau;
            if (tau <= st->thr || it >= st->maxit) st->done = 1;
        }
    }
}

// K3: d = gamma d + z (S7).
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_direction(int n, PcgVecs v, const PcgState *st)
{
    if (st->done) return;
    const double gamma = st->gamma;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        v.d[i] = __builtin_fma(gamma, v.d[i], v.z[i]);
}

// ---------------------------------------------------------------------------
// Launch functions

hipError_t launch_pcg_update(int mode, int n, const PcgVecs &v, PcgState *st, const DotWs *ws2,
                             const LaunchCfg &c)
{
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        k_pcg_update<decltype(m)::value, decltype(p)::value><<<c.grid, c.block, 0, c.stream>>>(
            n, v, st, ws2[0], ws2[1], c.early_exit, c.fallback);
    });
    return hipGetLastError();
}

hipError_t launch_pcg_direction(int n, const PcgVecs &v, PcgState *st, const LaunchCfg &c)
{
    hipLaunchKernelGGL(k_pcg_direction, dim3(c.grid), dim3(c.block), 0, c.stream, n, v, st);
    return hipGetLastError();
}

} // namespace rpcg
