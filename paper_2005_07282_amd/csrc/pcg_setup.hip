// Jacobi-PCG setup kernels: preconditioner, initial residual and dots
// (Fig. 1/Fig. 2 initialisation; Section 4.3 Jacobi: inverse diagonal once).
// T = double is the paper's solver; T = float the binary32 inner solver of
// the mixed-precision refinement (same steps, every rounding in binary32).
#include "reduce.hpp"
#include "sell_spmv.hpp"

namespace rpcg {

// The setup runs once per solve: its three block partials and three merges go
// through out-of-line calls, which keeps the number of inlined copies (and
// the compile time over all mode and length variants) down.
template <int MODE, int P>
__device__ __noinline__ void setup_block_finish(LaneDot<MODE, P> &L, long long *acc, const SlotView &sv, int g,
                                                bool ee, bool capture, int *gflags, RedShared &sh)
{
    block_finish<MODE, P>(L, acc, sv, g, ee, capture, gflags, sh);
}

template <int MODE, int P, typename T>
__device__ __noinline__ T setup_merge(const SlotView &sv, int G, bool ee, bool capture, long long *acc,
                                      long long *esc_out, int *flags_out, RedShared &sh, int slot_val)
{
    return merge_slots<MODE, P, T>(sv, G, ee, capture, acc, esc_out, flags_out, sh, slot_val);
}

static __global__ void k_state_init(PcgState *st, int maxit)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    PcgState z = {};
    z.maxit = maxit;
    z.ended = 0x7FFFFFFF;
    *st = z;
}

// dinv = RN(1/a_ii), r = RN(b - A x0), z = RN(dinv r), d = z, and the
// workgroup partials of <z,r>, <r,r>, <b,b>. One wavefront per 64-row slice
// of the sliced-ELL copy, as in the iteration's SpMV.
template <int MODE, int P, bool COL16, typename T>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_setup(SellMat<T> A, PcgVecs<T> v, PcgState *st, SlotView w0, SlotView w1, SlotView w2, bool ee, bool capture)
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
        T aii = T(0);
        bool found = false;
        const T acc = sell_row<T, COL16, true>(A, base, width, i, len, v.x, &aii, &found);
        if (i < A.n) {
            if (!found || !(aii > T(0))) flags |= FLAG_NOT_SPD;
            const T bi = v.b[i];
            if (!is_finite_bits((double)bi) || !is_finite_bits((double)v.x[i])) flags |= FLAG_NONFINITE;
            const T di = T(1) / aii;
            const T ri = bi - acc;
            const T zi = di * ri;
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
    setup_block_finish<MODE, P>(Lb, sh.acc[0], w0, blockIdx.x, ee, capture, &st->flags, sh);
    setup_block_finish<MODE, P>(Lt, sh.acc[1], w1, blockIdx.x, ee, capture, &st->flags, sh);
    setup_block_finish<MODE, P>(Lbb, sh.acc[2], w2, blockIdx.x, ee, capture, &st->flags, sh);
}

// One workgroup: beta0, tau0, <b,b>; thr = RN(RN(tol*tol) <b,b>) in T with
// tol rounded to T; stopping test.
template <int MODE, int P, typename T>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_fin_setup(int G, PcgVecs<T> v, PcgState *st, SlotView w0, SlotView w1, SlotView w2, double tol, bool ee,
                bool capture)
{
    __shared__ RedShared sh;
    long long e0, e1, e2;
    const T beta = setup_merge<MODE, P, T>(w0, G, ee, capture, sh.acc[0], &e0, &st->flags, sh, 0);
    const T tau = setup_merge<MODE, P, T>(w1, G, ee, capture, sh.acc[1], &e1, &st->flags, sh, 1);
    const T bb = setup_merge<MODE, P, T>(w2, G, ee, capture, sh.acc[2], &e2, &st->flags, sh, 2);
    if (threadIdx.x == 0) {
        st->escapes += e0 + e1 + e2;
        if (capture) st->fallbacks += (e0 > 0) + (e1 > 0) + (e2 > 0);
        int f = st->flags;
        v.beta_hist[0] = beta;
        st->beta = beta;
        st->tau = tau;
        st->tau0 = tau;
        st->bb = bb;
        const T tolt = (T)tol;
        const T thr = (tolt * tolt) * bb;
        st->thr = thr;
        if (v.hist) v.hist[0] = tau;
        st->iter = 0;
        if (f & FLAG_NOT_SPD) { st->status = -4; st->done = 1; }
        else if ((f & FLAG_NONFINITE) || !is_finite_bits((double)tau) || !is_finite_bits((double)bb)) {
            st->status = -6;
            st->done = 1;
        } else st->done = (tau <= thr || st->maxit <= 0) ? 1 : 0;
        if (st->done) st->ended = 0;
    }
}

template <typename T>
hipError_t launch_pcg_setup(int mode, const SellMat<T> &A, const PcgVecs<T> &v, PcgState *st, const DotWs *ws3,
                            int stride, double tol, int maxit, const LaunchCfg &c)
{
    SlotView s0{ws3[0], stride}, s1{ws3[1], stride}, s2{ws3[2], stride};
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, c.stream, st, maxit);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        if (A.col16)
            k_pcg_setup<M, PP, true, T><<<c.grid, c.block, 0, c.stream>>>(A, v, st, s0, s1, s2, c.early_exit,
                                                                         c.fallback);
        else
            k_pcg_setup<M, PP, false, T><<<c.grid, c.block, 0, c.stream>>>(A, v, st, s0, s1, s2, c.early_exit,
                                                                          c.fallback);
        k_pcg_fin_setup<M, PP, T><<<1, MAX_BLOCK, 0, c.stream>>>(c.grid, v, st, s0, s1, s2, tol, c.early_exit,
                                                                 c.fallback);
    });
    return hipGetLastError();
}

// Built once per value type (the library compiles this file with
// -DRPCG_VALUE_TYPE=double and with -DRPCG_VALUE_TYPE=float).
#ifndef RPCG_VALUE_TYPE
#error "define RPCG_VALUE_TYPE (double or float)"
#endif
template hipError_t launch_pcg_setup<RPCG_VALUE_TYPE>(int, const SellMat<RPCG_VALUE_TYPE> &, const PcgVecs<RPCG_VALUE_TYPE> &, PcgState *,
                                             const DotWs *, int, double, int, const LaunchCfg &);

} // namespace rpcg
