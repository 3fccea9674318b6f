// Batched Jacobi-PCG: one iteration of every system of a batch that is not
// done, in five kernels. The three streaming kernels work on runs (slice
// ranges of one system); the two per-system kernels (one workgroup per system)
// merge that system's partials and round them once, so every scalar of a
// system is the rounded exact value of that system's data alone: the results
// do not depend on the other systems, on their order or on the run schedule.
//
// The per-system kernels are the only writers of a system's scalars, iteration
// count and done flag; the streaming kernels only read them. A captured
// sequence of iterations can therefore be replayed unchanged.
#include "batch_common.hpp"

namespace rpcg {

// S1 + partial of S2 (as k_pcg_spmv_dot, per run).
template <int MODE, int P, bool COL16>
__global__ void __launch_bounds__(MAX_BLOCK) k_batch_spmv_dot(BatchArgs a, SlotView sv, bool ee, bool capture)
{
    __shared__ RedShared sh;
    const int lane = lane_id();
    const int W = num_waves();
    const int wave = __builtin_amdgcn_readfirstlane(wave_id());
    for (int ri = a.wg_run[blockIdx.x]; ri < a.wg_run[blockIdx.x + 1]; ++ri) {
        const BatchRun R = a.runs[ri];
        if (a.st[R.sys].done) continue;
        const BatchSys S = a.sys[R.sys];
        const SellMat<double> M = batch_mat(a, S);
        const double *__restrict__ d = a.d + S.row0;
        double *__restrict__ w = a.w + S.row0;
        __syncthreads(); // the previous run's partial is written before the accumulator is reused
        zero_acc(sh.acc[0]);
        __syncthreads();
        LaneDot<MODE, P> L;
        L.init();
        for (long long s = R.s0 + wave; s < R.s1; s += W) {
            const long long base = uniform_ll(M.off[s]);
            const int width = __builtin_amdgcn_readfirstlane((int)((M.off[s + 1] - base) >> 6));
            const long long i = s * 64 + lane;
            const int len = sell_len(M, i);
            const double sum = sell_row<double, COL16, false>(M, base, width, i, len, d, nullptr, nullptr);
            if (i < M.n) {
                w[i] = sum;
                L.add(d[i], sum, sh.acc[0], ee, capture);
            }
        }
        block_finish<MODE, P>(L, sh.acc[0], sv, R.slot, ee, capture, &a.st[R.sys].flags, sh);
    }
}

// S2: delta = <d, w> of one system (one workgroup per system); rho = beta / delta.
template <int MODE, int P>
__global__ void __launch_bounds__(256) k_batch_rho(BatchArgs a, SlotView sd, bool ee, bool capture)
{
    __shared__ RedShared sh;
    const int sys = blockIdx.x;
    PcgState *st = a.st + sys;
    if (st->done) return; // written below by thread 0 only, after every thread has read it
    const BatchSys S = a.sys[sys];
    long long esc = 0;
    const double delta = merge_slots<MODE, P>(batch_slots<MODE>(sd, S.slot0), S.slot1 - S.slot0, ee, capture,
                                              sh.acc[0], &esc, &st->flags, sh, 0);
    if (threadIdx.x == 0) {
        const bool bad = (batch_flags(st) & FLAG_NONFINITE) || !is_finite_bits(delta);
        st->escapes += esc;
        if (capture && esc > 0) st->fallbacks += 1;
        st->delta = delta;
        if (bad || !(delta > 0.0)) {
            st->status = bad ? -6 : -5;
            st->done = 1;
            atomicSub(a.active, 1);
        } else {
            st->rho = st->beta / delta;
        }
    }
}

// S3-S5 and the partials of S6, S8 (as k_pcg_update, per run).
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_batch_update(BatchArgs a, SlotView wb, SlotView wt, bool ee,
                                                            bool capture)
{
    __shared__ RedShared sh;
    for (int ri = a.wg_run[blockIdx.x]; ri < a.wg_run[blockIdx.x + 1]; ++ri) {
        const BatchRun R = a.runs[ri];
        if (a.st[R.sys].done) continue;
        const BatchSys S = a.sys[R.sys];
        const double rho = a.st[R.sys].rho;
        const long long r0 = S.row0;
        const long long i1 = min((long long)R.s1 * 64, (long long)S.n);
        __syncthreads();
        zero_acc(sh.acc[0]);
        zero_acc(sh.acc[1]);
        __syncthreads();
        LaneDot<MODE, P> Lb, Lt;
        Lb.init();
        Lt.init();
        for (long long i = (long long)R.s0 * 64 + threadIdx.x; i < i1; i += blockDim.x) {
            const long long g = r0 + i;
            const double di = a.d[g], wi = a.w[g];
            a.x[g] = __builtin_fma(rho, di, a.x[g]);              // S3
            const double ri = __builtin_fma(-rho, wi, a.r[g]);     // S4
            const double zi = a.dinv[g] * ri;                      // S5
            a.r[g] = ri;
            a.z[g] = zi;
            Lb.add(zi, ri, sh.acc[0], ee, capture);                // S6
            Lt.add(ri, ri, sh.acc[1], ee, capture);                // S8
        }
        block_finish_pair<MODE, P>(Lb, sh.acc[0], wb, Lt, sh.acc[1], wt, R.slot, ee, capture, &a.st[R.sys].flags, sh);
    }
}

// S6, S8 merged per system; the stopping test of Fig. 1; gamma = beta / beta_old.
template <int MODE, int P>
__global__ void __launch_bounds__(256) k_batch_gamma(BatchArgs a, SlotView wb, SlotView wt, bool ee, bool capture)
{
    __shared__ RedShared sh;
    const int sys = blockIdx.x;
    PcgState *st = a.st + sys;
    if (st->done) return;
    const BatchSys S = a.sys[sys];
    const int G = S.slot1 - S.slot0;
    long long eb = 0, et = 0;
    const double beta = merge_slots<MODE, P>(batch_slots<MODE>(wb, S.slot0), G, ee, capture, sh.acc[0], &eb,
                                             &st->flags, sh, 0);
    const double tau = merge_slots<MODE, P>(batch_slots<MODE>(wt, S.slot0), G, ee, capture, sh.acc[1], &et,
                                            &st->flags, sh, 1);
    if (threadIdx.x == 0) {
        const bool bad = (batch_flags(st) & FLAG_NONFINITE) || !is_finite_bits(beta) || !is_finite_bits(tau);
        const int it = st->iter + 1;
        const bool stop = bad || tau <= st->thr || it >= st->maxit;
        st->escapes += eb + et;
        if (capture) st->fallbacks += (eb > 0) + (et > 0);
        if (bad) {
            st->status = -6;
        } else {
            st->gamma = beta / st->beta;
            st->beta = beta;
            st->tau = tau;
            st->iter = it;
            if (a.hist && a.hist[sys]) a.hist[sys][it] = tau;
        }
        if (stop) {
            st->done = 1;
            atomicSub(a.active, 1);
        }
    }
}

// S7 (as k_pcg_direction, per run).
__global__ void __launch_bounds__(MAX_BLOCK) k_batch_direction(BatchArgs a)
{
    for (int ri = a.wg_run[blockIdx.x]; ri < a.wg_run[blockIdx.x + 1]; ++ri) {
        const BatchRun R = a.runs[ri];
        if (a.st[R.sys].done) continue;
        const BatchSys S = a.sys[R.sys];
        const double gamma = a.st[R.sys].gamma;
        const long long i1 = min((long long)R.s1 * 64, (long long)S.n);
        for (long long i = (long long)R.s0 * 64 + threadIdx.x; i < i1; i += blockDim.x) {
            const long long g = S.row0 + i;
            a.d[g] = __builtin_fma(gamma, a.d[g], a.z[g]);
        }
    }
}

hipError_t launch_batch_iteration(int mode, bool col16, const BatchArgs &a, int grid, int block, const DotWs *ws3,
                                  int stride, const LaunchCfg &c)
{
    SlotView s0{ws3[0], stride}, s1{ws3[1], stride}, s2{ws3[2], stride};
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        if (col16) k_batch_spmv_dot<M, PP, true><<<grid, block, 0, c.stream>>>(a, s0, c.early_exit, c.fallback);
        else k_batch_spmv_dot<M, PP, false><<<grid, block, 0, c.stream>>>(a, s0, c.early_exit, c.fallback);
        k_batch_rho<M, PP><<<a.nsys, 256, 0, c.stream>>>(a, s0, c.early_exit, c.fallback);
        k_batch_update<M, PP><<<grid, block, 0, c.stream>>>(a, s1, s2, c.early_exit, c.fallback);
        k_batch_gamma<M, PP><<<a.nsys, 256, 0, c.stream>>>(a, s1, s2, c.early_exit, c.fallback);
    });
    k_batch_direction<<<grid, block, 0, c.stream>>>(a);
    return hipGetLastError();
}

} // namespace rpcg
