// Jacobi-PCG setup kernels: preconditioner, initial residual and dots
// (Fig. 1/Fig. 2 initialisation; Section 4.3 Jacobi: inverse diagonal once).
#include "reduce.hpp"
#include "sell_spmv.hpp"

namespace rpcg {

__global__ void k_state_init(PcgState *st, int maxit)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    PcgState z = {};
    z.maxit = maxit;
    *st = z;
}

// dinv = RN(1/a_ii), r = RN(b - A x0), z = RN(dinv r), d = z, and the
// workgroup partials of <z,r>, <r,r>, <b,b>. One wavefront per 64-row slice
// of the sliced-ELL copy, as in the iteration's SpMV.
template <int MODE, int P, bool COL16>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_setup(SellMat A, PcgVecs v, PcgState *st, SlotView w0, SlotView w1, SlotView w2, bool ee, bool capture)
{
    __shared__ RedShared sh;
    zero_acc(sh.acc[0]); zero_acc(sh.acc[1]); zero_acc(sh.acc[2]);
    __syncthreads();
    LaneDot<MODE, P> Lb, Lt, Lbb;
    Lb.init(); Lt.init(); Lbb.init();
    int flags = 0;
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(wave_id());
    const long long wstride = (long long)gridDim.x * num_waves();
    for (long long s = (long long)blockIdx.x * num_waves() + wave; s < A.nslices; s += wstride) {
        const long long base = uniform_ll(A.off[s]);
        const int width = __builtin_amdgcn_readfirstlane((int)((A.off[s + 1] - base) >> 6));
        const long long i = s * 64 + lane;
        const int len = sell_len(A, i);
        double aii = 0.0;
        bool found = false;
        const double acc = sell_row<COL16, true>(A, base, width, i, len, v.x, &aii, &found);
        if (i < A.n) {
            if (!found || !(aii > 0.0)) flags |= FLAG_NOT_SPD;
            const double bi = v.b[i];
            if (!is_finite_bits(bi) || !is_finite_bits(v.x[i])) flags |= FLAG_NONFINITE;
            const double di = 1.0 / aii;
            const double ri = bi - acc;
            const double zi = di * ri;
            v.dinv[i] = di;
            v.r[i] = ri;
            v.z[i] = zi;
            v.d[i] = zi;
            Lb.add(zi, ri, sh.acc[0], ee, capture);
            Lt.add(ri, ri, sh.acc[1], ee, capture);
            Lbb.add(bi, bi, sh.acc[2], ee, capture);
        }
    }
    if (flags) atomicOr(&st->flags, flags);
    block_finish<MODE, P>(Lb, sh.acc[0], w0, blockIdx.x, ee, capture, &st->flags, sh);
    block_finish<MODE, P>(Lt, sh.acc[1], w1, blockIdx.x, ee, capture, &st->flags, sh);
    block_finish<MODE, P>(Lbb, sh.acc[2], w2, blockIdx.x, ee, capture, &st->flags, sh);
}

// One workgroup: beta0, tau0, <b,b>; thr = RN(RN(tol*tol) <b,b>); stopping test.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_fin_setup(int G, PcgVecs v, PcgState *st, SlotView w0, SlotView w1, SlotView w2, double tol, bool ee,
                bool capture)
{
    __shared__ RedShared sh;
    long long e0, e1, e2;
    double beta = merge_slots<MODE, P>(w0, G, ee, capture, sh.acc[0], &e0, &st->flags, sh, 0);
    double tau = merge_slots<MODE, P>(w1, G, ee, capture, sh.acc[1], &e1, &st->flags, sh, 1);
    double bb = merge_slots<MODE, P>(w2, G, ee, capture, sh.acc[2], &e2, &st->flags, sh, 2);
    if (threadIdx.x == 0) {
        st->escapes += e0 + e1 + e2;
        if (capture) st->fallbacks += (e0 > 0) + (e1 > 0) + (e2 > 0);
        int f = st->flags;
        v.beta_hist[0] = beta;
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

hipError_t launch_pcg_setup(int mode, const SellMat &A, const PcgVecs &v, PcgState *st, const DotWs *ws3,
                            int stride, double tol, int maxit, const LaunchCfg &c)
{
    SlotView s0{ws3[0], stride}, s1{ws3[1], stride}, s2{ws3[2], stride};
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, c.stream, st, maxit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        if (A.col16)
            k_pcg_setup<M, PP, true><<<c.grid, c.block, 0, c.stream>>>(A, v, st, s0, s1, s2, c.early_exit, c.fallback);
        else
            k_pcg_setup<M, PP, false><<<c.grid, c.block, 0, c.stream>>>(A, v, st, s0, s1, s2, c.early_exit, c.fallback);
        k_pcg_fin_setup<M, PP><<<1, MAX_BLOCK, 0, c.stream>>>(c.grid, v, st, s0, s1, s2, tol, c.early_exit,
                                                              c.fallback);
    });
    return hipGetLastError();
}

} // namespace rpcg
