// Batched Jacobi-PCG setup (Fig. 1 initialisation, Section 4.3 Jacobi) of
// every system of a batch: state, then dinv, r, z, d and the partials of
// <z,r>, <r,r>, <b,b> per run, then one workgroup per system to merge them.
#include "batch_common.hpp"

namespace rpcg {

__global__ void k_batch_state_init(BatchArgs a, int maxit)
{
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys == 0) *a.active = a.nsys;
    if (sys >= a.nsys) return;
    PcgState z = {};
    z.maxit = maxit;
    z.ended = 0x7FFFFFFF;
    a.st[sys] = z;
}

// The setup runs once per solve: its block partials go through an
// out-of-line call, which keeps the inlined copies (and compile time) down.
template <int MODE, int P>
__device__ __noinline__ void batch_setup_finish(LaneDot<MODE, P> &L, long long *acc, const SlotView &sv, int g,
                                                bool ee, bool capture, int *gflags, RedShared &sh)
{
    block_finish<MODE, P>(L, acc, sv, g, ee, capture, gflags, sh);
}

template <int MODE, int P, bool COL16>
__global__ void __launch_bounds__(MAX_BLOCK)
k_batch_setup(BatchArgs a, SlotView w0, SlotView w1, SlotView w2, bool ee, bool capture)
{
    __shared__ RedShared sh;
    const int lane = lane_id();
    const int W = num_waves();
    const int wave = __builtin_amdgcn_readfirstlane(wave_id());
    for (int ri = a.wg_run[blockIdx.x]; ri < a.wg_run[blockIdx.x + 1]; ++ri) {
        const BatchRun R = a.runs[ri];
        const BatchSys S = a.sys[R.sys];
        const SellMat<double> M = batch_mat(a, S);
        const long long r0 = S.row0;
        __syncthreads();
        zero_acc(sh.acc[0]);
        zero_acc(sh.acc[1]);
        zero_acc(sh.acc[2]);
        __syncthreads();
        LaneDot<MODE, P> Lb, Lt, Lbb;
        Lb.init();
        Lt.init();
        Lbb.init();
        int flags = 0;
        for (long long s = R.s0 + wave; s < R.s1; s += W) {
            const long long base = uniform_ll(M.off[s]);
            const int width = __builtin_amdgcn_readfirstlane((int)((M.off[s + 1] - base) >> 6));
            const long long i = s * 64 + lane;
            const int len = sell_len(M, i);
            double aii = 0.0;
            bool found = false;
            const double acc = sell_row<double, COL16, true>(M, base, width, i, len, a.x + r0, &aii, &found);
            if (i < M.n) {
                const long long g = r0 + i;
                if (!found || !(aii > 0.0)) flags |= FLAG_NOT_SPD;
                const double bi = a.b[g];
                if (!is_finite_bits(bi) || !is_finite_bits(a.x[g])) flags |= FLAG_NONFINITE;
                const double di = 1.0 / aii;
                const double ri = bi - acc;
                const double zi = di * ri;
                a.dinv[g] = di;
                a.r[g] = ri;
                a.z[g] = zi;
                a.d[g] = zi;
                Lb.add(zi, ri, sh.acc[0], ee, capture);
                Lt.add(ri, ri, sh.acc[1], ee, capture);
                Lbb.add(bi, bi, sh.acc[2], ee, capture);
            }
        }
        if (flags) atomicOr(&a.st[R.sys].flags, flags);
        int *gf = &a.st[R.sys].flags;
        batch_setup_finish<MODE, P>(Lb, sh.acc[0], w0, R.slot, ee, capture, gf, sh);
        batch_setup_finish<MODE, P>(Lt, sh.acc[1], w1, R.slot, ee, capture, gf, sh);
        batch_setup_finish<MODE, P>(Lbb, sh.acc[2], w2, R.slot, ee, capture, gf, sh);
    }
}

template <int MODE, int P>
__device__ __noinline__ double batch_setup_merge(const SlotView &sv, int G, bool ee, bool capture, long long *acc,
                                                 long long *esc_out, int *flags_out, RedShared &sh, int slot_val)
{
    return merge_slots<MODE, P>(sv, G, ee, capture, acc, esc_out, flags_out, sh, slot_val);
}

// One workgroup per system: beta0, tau0, <b,b>, thr = RN(RN(tol*tol) <b,b>), stopping test.
template <int MODE, int P>
__global__ void __launch_bounds__(256)
k_batch_fin_setup(BatchArgs a, SlotView w0, SlotView w1, SlotView w2, double tol, bool ee, bool capture)
{
    __shared__ RedShared sh;
    const int sys = blockIdx.x;
    PcgState *st = a.st + sys;
    const BatchSys S = a.sys[sys];
    const int G = S.slot1 - S.slot0;
    long long e0, e1, e2;
    const double beta = batch_setup_merge<MODE, P>(batch_slots<MODE>(w0, S.slot0), G, ee, capture, sh.acc[0], &e0,
                                                   &st->flags, sh, 0);
    const double tau = batch_setup_merge<MODE, P>(batch_slots<MODE>(w1, S.slot0), G, ee, capture, sh.acc[1], &e1,
                                                  &st->flags, sh, 1);
    const double bb = batch_setup_merge<MODE, P>(batch_slots<MODE>(w2, S.slot0), G, ee, capture, sh.acc[2], &e2,
                                                 &st->flags, sh, 2);
    if (threadIdx.x == 0) {
        st->escapes += e0 + e1 + e2;
        if (capture) st->fallbacks += (e0 > 0) + (e1 > 0) + (e2 > 0);
        const int f = batch_flags(st);
        st->beta = beta;
        st->beta_par[0] = beta;
        st->tau = tau;
        st->tau0 = tau;
        st->bb = bb;
        const double thr = (tol * tol) * bb;
        st->thr = thr;
        if (a.hist && a.hist[sys]) a.hist[sys][0] = tau;
        st->iter = 0;
        st->it_cur = 0;
        int done;
        if (f & FLAG_NOT_SPD) { st->status = -4; done = 1; }
        else if ((f & FLAG_NONFINITE) || !is_finite_bits(tau) || !is_finite_bits(bb)) { st->status = -6; done = 1; }
        else done = (tau <= thr || st->maxit <= 0) ? 1 : 0;
        st->done = done;
        if (done) {
            st->ended = 0;
            atomicSub(a.active, 1);
        }
    }
}

hipError_t launch_batch_setup(int mode, bool col16, const BatchArgs &a, int grid, int block, const DotWs *ws3,
                              int stride, double tol, int maxit, const LaunchCfg &c)
{
    SlotView s0{ws3[0], stride}, s1{ws3[1], stride}, s2{ws3[2], stride};
    k_batch_state_init<<<(a.nsys + 63) / 64, 64, 0, c.stream>>>(a, maxit);
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        if (col16) k_batch_setup<M, PP, true><<<grid, block, 0, c.stream>>>(a, s0, s1, s2, c.early_exit, c.fallback);
        else k_batch_setup<M, PP, false><<<grid, block, 0, c.stream>>>(a, s0, s1, s2, c.early_exit, c.fallback);
        k_batch_fin_setup<M, PP><<<a.nsys, 256, 0, c.stream>>>(a, s0, s1, s2, tol, c.early_exit, c.fallback);
    });
    return hipGetLastError();
}

} // namespace rpcg
