// Jacobi-PCG setup kernel: preconditioner, initial residual and dots.
#include "reduce.hpp"

namespace rpcg {

// ---------------------------------------------------------------------------
// Jacobi-PCG kernels (Fig. 2 order; S8 with S6)

__global__ void k_state_init(PcgState *st, int maxit)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    PcgState z = {};
    z.maxit = maxit;
    *st = z;
}

// Setup: dinv = 1/a_ii, r = b - A x0, z = dinv r, d = z, and the dots
// beta = <z,r>, tau = <r,r>, <b,b>; then thr and the stopping test.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_setup(int n, const int *__restrict__ rp, const int *__restrict__ col,
            const double *__restrict__ val, PcgVecs v, PcgState *st, DotWs w0, DotWs w1, DotWs w2,
            double tol, bool ee, bool fallback)
{
    __shared__ RedShared sh;
    if constexpr (MODE == MODE_EXBLAS) { zero_acc(sh.acc[0]); zero_acc(sh.acc[1]); zero_acc(sh.acc[2]); }
    __syncthreads();
    LaneDot<MODE, P> Lb, Lt, Lbb;
    Lb.init(); Lt.init(); Lbb.init();
    int flags = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double acc = 0.0, aii = 0.0;
        bool found = false;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            int c = col[k];
            acc = __builtin_fma(val[k], v.x[c], acc);
            if (c == i) { aii = val[k]; found = true; }
        }
        if (!found || !(aii > 0.0)) flags |= FLAG_NOT_SPD;
        double bi = v.b[i];
        if (!is_finite_bits(bi) || !is_finite_bits(v.x[i])) flags |= FLAG_NONFINITE;
        double di = 1.0 / aii;
        double ri = bi - acc;
        double zi = di * ri;
        v.dinv[i] = di;
        v.r[i] = ri;
        v.z[i] = zi;
        v.d[i] = zi;
        Lb.add(zi, ri, sh.acc[0], ee);
        Lt.add(ri, ri, sh.acc[1], ee);
        Lbb.add(bi, bi, sh.acc[2], ee);
    }
    if (flags) atomicOr(&st->flags, flags);
    block_finish<MODE, P>(Lb, sh.acc[0], w0, blockIdx.x, ee, &st->flags, sh);
    block_finish<MODE, P>(Lt, sh.acc[1], w1, blockIdx.x, ee, &st->flags, sh);
    block_finish<MODE, P>(Lbb, sh.acc[2], w2, blockIdx.x, ee, &st->flags, sh);
    if (!arrive_last(&st->ticket[0], sh)) return;

    long long e0, e1, e2;
    double beta = merge_slots<MODE, P>(w0, gridDim.x, ee, sh.acc[0], &st->flags, &e0, sh);
    double tau = merge_slots<MODE, P>(w1, gridDim.x, ee, sh.acc[1], &st->flags, &e1, sh);
    double bb = merge_slots<MODE, P>(w2, gridDim.x, ee, sh.acc[2], &st->flags, &e2, sh);
    if constexpr (MODE == MODE_FPE) {
        if (threadIdx.x == 0) sh.need_fb = fallback && (e0 + e1 + e2) > 0;
        __syncthreads();
        if (sh.need_fb) {
            double t0 = block_exact_dot(n, v.z, v.r, sh.acc[0], &st->flags, sh);
            double t1 = block_exact_dot(n, v.r, v.r, sh.acc[0], &st->flags, sh);
            double t2 = block_exact_dot(n, v.b, v.b, sh.acc[0], &st->flags, sh);
            if (threadIdx.x == 0) { beta = t0; tau = t1; bb = t2; st->fallbacks += 1; }
        }
    }
    if (threadIdx.x == 0) {
        st->escapes += e0 + e1 + e2;
        int f = st->flags;
        st->beta = beta;
        st->tau = tau;
        st->tau0 = tau;
        st->bb = bb;
        double thr = (tol * tol) * bb;
        st->thr = thr;
        if (v.hist) v.hist[0] = tau;
        st->iter = 0;
        if (f & FLAG_NOT_SPD) { st->status = -4; st->done = 1; }
        else if ((f & FLAG_NONFINITE) || !is_finite_bits(tau) || !is_finite_bits(bb)) { st->status = -6; st->done = 1; }
        else st->done = (tau <= thr || st->maxit <= 0) ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Launch functions

hipError_t launch_pcg_setup(int mode, const SellMat &A, const int *col, const double *val,
                            const PcgVecs &v, PcgState *st, const DotWs *ws3, double tol, int maxit,
                            const LaunchCfg &c)
{
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, c.stream, st, maxit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        k_pcg_setup<decltype(m)::value, decltype(p)::value><<<c.grid, c.block, 0, c.stream>>>(
            A.n, A.row_ptr, col, val, v, st, ws3[0], ws3[1], ws3[2], tol, c.early_exit, c.fallback);
    });
    return hipGetLastError();
}

} // namespace rpcg
