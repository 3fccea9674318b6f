// Batched Jacobi-PCG: one iteration of every system of a batch that is not
// done, in three streaming kernels over runs (slice ranges of one system),
// cut at the two global reductions of Fig. 2 as in the single solver:
//   K1 SpMV and the partials of <d, w>;
//   K2 merge of that system's <d, w> partials (every run alike), rho, the
//      residual and Jacobi updates and the partials of <z, r>, <r, r>;
//   K3 merge of those, the stopping test, gamma, the iterate update (S3)
//      and the direction update (S7).
// Each merge sums the integer partials of the run's own system and rounds
// once, so every scalar of a system is the rounded exact value of that
// system's data alone: the results do not depend on the other systems, on
// their order or on the run schedule.
//
// The scalars of a system are written by its lead run (the run holding its
// first slice) and read by every run of the system in later kernels, never
// in the same one: beta alternates between two entries by the parity of the
// iteration, K3 records the new iteration count in iter, and K1 commits it
// to it_cur, which K2 and K3 read. A K3 run returns early only if the system
// ended before its x update of this iteration was owed (ended <= it_cur),
// which the stopping test of the same launch never sets. Nothing depends on
// a launch argument, so a captured sequence of iterations replays unchanged.
#include "batch_common.hpp"

namespace rpcg {

// Workgroup-uniform read of an int another workgroup of the same kernel may
// write (one thread reads, every thread sees its value).
__device__ __forceinline__ int wg_read_int(const int *p, RedShared &sh)
{
    __syncthreads(); // the previous reader's value has been used
    if (threadIdx.x == 0) sh.flag = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return sh.flag;
}

// K1: S1 + partial of S2 (as k_pcg_spmv_dot, per run).
template <int MODE, int P, bool COL16>
__global__ void __launch_bounds__(MAX_BLOCK) k_batch_spmv_dot(BatchArgs a, SlotView sv, bool ee, bool capture)
{
    __shared__ RedShared sh;
    const int lane = lane_id();
    const int W = num_waves();
    const int wave = __builtin_amdgcn_readfirstlane(wave_id());
    for (int ri = a.wg_run[blockIdx.x]; ri < a.wg_run[blockIdx.x + 1]; ++ri) {
        const BatchRun R = a.runs[ri];
        PcgState *st = a.st + R.sys;
        // the lead run commits the iteration count K3 recorded (no workgroup of
        // this kernel reads it_cur; done is not written during this kernel)
        if (R.s0 == 0 && threadIdx.x == 0) st->it_cur = st->iter;
        if (st->done) continue;
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
        block_finish<MODE, P>(L, sh.acc[0], sv, R.slot, ee, capture, &st->flags, sh);
    }
}

// K2: delta = <d, w> of the run's system merged (every run alike), rho =
// beta / delta; S4, S5 and the partials of S6, S8.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_batch_update(BatchArgs a, SlotView sd, SlotView wb, SlotView wt,
                                                            bool ee, bool capture)
{
    __shared__ RedShared sh;
    for (int ri = a.wg_run[blockIdx.x]; ri < a.wg_run[blockIdx.x + 1]; ++ri) {
        const BatchRun R = a.runs[ri];
        PcgState *st = a.st + R.sys;
        if (wg_read_int(&st->done, sh)) continue; // set in this kernel only by a breakdown every run sees
        const BatchSys S = a.sys[R.sys];
        const bool lead = R.s0 == 0;
        const int it = st->it_cur;
        long long esc = 0;
        const double delta = merge_slots<MODE, P>(batch_slots<MODE>(sd, S.slot0), S.slot1 - S.slot0, ee, capture,
                                                  sh.acc[0], &esc, &st->flags, sh, 0);
        const bool bad = (batch_flags(st) & FLAG_NONFINITE) || !is_finite_bits(delta);
        const bool breakdown = !(delta > 0.0);
        if (lead && threadIdx.x == 0) {
            st->escapes += esc;
            if (capture && esc > 0) st->fallbacks += 1;
            st->delta = delta;
            if (bad || breakdown) {
                st->status = bad ? -6 : -5;
                st->ended = it;
                st->done = 1;
                atomicSub(a.active, 1);
            }
        }
        if (bad || breakdown) continue;
        const double rho = st->beta_par[it & 1] / delta;
        if (lead && threadIdx.x == 0) st->rho = rho;
        const long long r0 = S.row0;
        const long long i1 = min((long long)R.s1 * 64, (long long)S.n);
        zero_acc(sh.acc[0]);
        zero_acc(sh.acc[1]);
        __syncthreads();
        LaneDot<MODE, P> Lb, Lt;
        Lb.init();
        Lt.init();
        for (long long i = (long long)R.s0 * 64 + threadIdx.x; i < i1; i += blockDim.x) {
            const long long g = r0 + i;
            const double ri = __builtin_fma(-rho, a.w[g], a.r[g]);    // S4
            const double zi = a.dinv[g] * ri;                         // S5
            a.r[g] = ri;
            a.z[g] = zi;
            Lb.add(zi, ri, sh.acc[0], ee, capture);                   // S6
            Lt.add(ri, ri, sh.acc[1], ee, capture);                   // S8
        }
        block_finish_pair<MODE, P>(Lb, sh.acc[0], wb, Lt, sh.acc[1], wt, R.slot, ee, capture, &st->flags, sh);
    }
}

// K3: beta, tau of the run's system merged; stopping test of Fig. 1; gamma =
// beta / beta_old; S3 and (unless the system stops) S7.
template <int MODE, int P>
__global__ void __launch_bounds__(MAX_BLOCK) k_batch_direction(BatchArgs a, SlotView wb, SlotView wt, bool ee,
                                                               bool capture)
{
    __shared__ RedShared sh;
    for (int ri = a.wg_run[blockIdx.x]; ri < a.wg_run[blockIdx.x + 1]; ++ri) {
        const BatchRun R = a.runs[ri];
        PcgState *st = a.st + R.sys;
        const int it = st->it_cur;
        if (wg_read_int(&st->ended, sh) <= it) continue;
        const BatchSys S = a.sys[R.sys];
        const bool lead = R.s0 == 0;
        const int G = S.slot1 - S.slot0;
        long long eb = 0, et = 0;
        const double beta = merge_slots<MODE, P>(batch_slots<MODE>(wb, S.slot0), G, ee, capture, sh.acc[0], &eb,
                                                 &st->flags, sh, 0);
        const double tau = merge_slots<MODE, P>(batch_slots<MODE>(wt, S.slot0), G, ee, capture, sh.acc[1], &et,
                                                &st->flags, sh, 1);
        const bool bad = (batch_flags(st) & FLAG_NONFINITE) || !is_finite_bits(beta) || !is_finite_bits(tau);
        const bool stop = bad || tau <= st->thr || it + 1 >= st->maxit;
        const double beta_old = st->beta_par[it & 1];
        if (lead && threadIdx.x == 0) {
            st->escapes += eb + et;
            if (capture) st->fallbacks += (eb > 0) + (et > 0);
            if (bad) {
                st->status = -6;
            } else {
                st->gamma = beta / beta_old;
                st->beta = beta;
                st->beta_par[(it + 1) & 1] = beta;
                st->tau = tau;
                st->iter = it + 1;
                if (a.hist && a.hist[R.sys]) a.hist[R.sys][it + 1] = tau;
            }
            if (stop) {
                st->ended = it + 1;
                st->done = 1;
                atomicSub(a.active, 1);
            }
        }
        const double rho = st->rho; // K2's rho of this iteration
        const double gamma = beta / beta_old;
        const long long i1 = min((long long)R.s1 * 64, (long long)S.n);
        for (long long i = (long long)R.s0 * 64 + threadIdx.x; i < i1; i += blockDim.x) {
            const long long g = S.row0 + i;
            const double di = a.d[g];
            a.x[g] = __builtin_fma(rho, di, a.x[g]);                   // S3
            if (!stop) a.d[g] = __builtin_fma(gamma, di, a.z[g]);      // S7
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
        k_batch_update<M, PP><<<grid, block, 0, c.stream>>>(a, s0, s1, s2, c.early_exit, c.fallback);
        k_batch_direction<M, PP><<<grid, block, 0, c.stream>>>(a, s1, s2, c.early_exit, c.fallback);
    });
    return hipGetLastError();
}

} // namespace rpcg
