// Setup of the PCG with a factored preconditioner M^-1 = G G^T + eps I
// (Fig. 1 initialisation with the preconditioner step t = G^T r,
// z = G t + eps r). Runs once per solve: its partials and merges go through
// out-of-line calls, which keeps compile time down.
#include "pcg_factored.hpp"

namespace rpcg {

template <int MODE, int P>
__device__ __noinline__ void fac_block_finish(LaneDot<MODE, P> &L, long long *acc, const SlotView &sv, int g, bool ee,
                                              bool capture, int *gflags, RedShared &sh)
{
    block_finish<MODE, P>(L, acc, sv, g, ee, capture, gflags, sh);
}

template <int MODE, int P>
__device__ __noinline__ double fac_merge(const SlotView &sv, int G, bool ee, bool capture, long long *acc,
                                         long long *esc_out, int *flags_out, RedShared &sh, int slot_val)
{
    return merge_slots<MODE, P>(sv, G, ee, capture, acc, esc_out, flags_out, sh, slot_val);
}

static __global__ void k_fac_state_init(PcgState *st, int maxit)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    PcgState z = {};
    z.maxit = maxit;
    *st = z;
}

// r = b - A x0 over the sliced-ELL copy; partials of <r,r> and <b,b>.
template <int MODE, int P, bool COL16>
__global__ void __launch_bounds__(MAX_BLOCK)
k_fac_setup_r(SellMat<double> A, PcgVecs<double> v, PcgState *st, SlotView wt, SlotView wbb, bool ee, bool capture)
{
    __shared__ RedShared sh;
    zero_acc(sh.acc[1]);
    zero_acc(sh.acc[2]);
    __syncthreads();
    LaneDot<MODE, P> Lt, Lbb;
    Lt.init();
    Lbb.init();
    int flags = 0;
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(wave_id());
    const long long wstride = (long long)gridDim.x * num_waves();
    for (long long s = (long long)blockIdx.x * num_waves() + wave; s < A.nslices; s += wstride) {
        const long long base = uniform_ll(A.off[s]);
        const int width = __builtin_amdgcn_readfirstlane((int)((A.off[s + 1] - base) >> 6));
        const long long i = s * 64 + lane;
        const int len = sell_len(A, i);
        const double acc = sell_row<double, COL16, false>(A, base, width, i, len, v.x, nullptr, nullptr);
        if (i < A.n) {
            const double bi = v.b[i];
            if (!is_finite_bits(bi) || !is_finite_bits(v.x[i])) flags |= FLAG_NONFINITE;
            const double ri = bi - acc;
            v.r[i] = ri;
            Lt.add(ri, ri, sh.acc[1], ee, capture);
            Lbb.add(bi, bi, sh.acc[2], ee, capture);
        }
    }
    if (flags) atomicOr(&st->flags, flags);
    fac_block_finish<MODE, P>(Lt, sh.acc[1], wt, blockIdx.x, ee, capture, &st->flags, sh);
    fac_block_finish<MODE, P>(Lbb, sh.acc[2], wbb, blockIdx.x, ee, capture, &st->flags, sh);
}

// One workgroup: beta0, tau0, <b,b>, threshold, stopping test.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK)
k_fac_fin_setup(int G, PcgVecs<double> v, PcgState *st, SlotView w0, SlotView w1, SlotView w2, double tol, bool ee,
                bool capture)
{
    __shared__ RedShared sh;
    long long e0, e1, e2;
    const double beta = fac_merge<MODE, P>(w0, G, ee, capture, sh.acc[0], &e0, &st->flags, sh, 0);
    const double tau = fac_merge<MODE, P>(w1, G, ee, capture, sh.acc[1], &e1, &st->flags, sh, 1);
    const double bb = fac_merge<MODE, P>(w2, G, ee, capture, sh.acc[2], &e2, &st->flags, sh, 2);
    if (threadIdx.x == 0) {
        st->escapes += e0 + e1 + e2;
        if (capture) st->fallbacks += (e0 > 0) + (e1 > 0) + (e2 > 0);
        const int f = __hip_atomic_load(&st->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.beta_hist[0] = beta;
        st->beta = beta;
        st->tau = tau;
        st->tau0 = tau;
        st->bb = bb;
        const double thr = (tol * tol) * bb;
        st->thr = thr;
        if (v.hist) v.hist[0] = tau;
        st->iter = 0;
        if ((f & FLAG_NONFINITE) || !is_finite_bits(tau) || !is_finite_bits(bb) || !is_finite_bits(beta)) {
            st->status = -6;
            st->done = 1;
        } else {
            st->done = (tau <= thr || st->maxit <= 0) ? 1 : 0;
        }
    }
}

hipError_t launch_fac_setup(int mode, const SellMat<double> &A, const FacPre &Pr, const PcgVecs<double> &v, double *t,
                            PcgState *st, const DotWs *ws3, int stride, double tol, int maxit, const LaunchCfg &c)
{
    SlotView s0{ws3[0], stride}, s1{ws3[1], stride}, s2{ws3[2], stride};
    k_fac_state_init<<<1, 64, 0, c.stream>>>(st, maxit);
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        if (A.col16)
            k_fac_setup_r<M, PP, true><<<c.grid, c.block, 0, c.stream>>>(A, v, st, s1, s2, c.early_exit, c.fallback);
        else
            k_fac_setup_r<M, PP, false><<<c.grid, c.block, 0, c.stream>>>(A, v, st, s1, s2, c.early_exit, c.fallback);
        k_fac_gt<<<c.grid, c.block, 0, c.stream>>>(A.n, Pr, v.r, t, st);
        k_fac_z<M, PP, true><<<c.grid, c.block, 0, c.stream>>>(A.n, Pr, v, t, st, s0, c.early_exit, c.fallback);
        k_fac_fin_setup<M, PP><<<1, MAX_BLOCK, 0, c.stream>>>(c.grid, v, st, s0, s1, s2, tol, c.early_exit,
                                                              c.fallback);
    });
    return hipGetLastError();
}

} // namespace rpcg
