// Jacobi-PCG iteration, second and third kernels.
//
// K2 starts by merging the SpMV kernel's partials of <d, w> (every workgroup
// alike) into delta and rho = beta / delta (S2), then applies the residual
// update and the Jacobi preconditioner (S4, S5) and forms the partials of
// beta = <z, r> and tau = <r, r> (S6, S8).
// K3 starts by merging those into beta, tau and gamma = beta / beta_old, runs
// the stopping test of Fig. 1, and updates the iterate (S3, with the rho of
// K2) and, unless the solve stops, the search direction (S7). S3 sits in K3
// because K3 loads d anyway: K2 then reads neither d nor x.
//
// The iteration number l is a launch argument, so the beta and tau histories
// one kernel writes for later iterations are never read by another
// workgroup of the same kernel. A workgroup of K3 that starts after the
// first one has run the stopping test must still apply the iteration's S3:
// it returns early only when the solve ended before this iteration's S3 was
// owed (PcgState::ended <= l), which the stopping test of the same launch
// never sets.
#include "reduce.hpp"
#include "sell_spmv.hpp"

namespace rpcg {

template <int MODE, int P, typename T>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_update(int l, int n, PcgVecs<T> v, PcgState *st, SlotView sd, int Gd, SlotView wb, SlotView wt, bool ee,
             bool capture)
{
    __shared__ RedShared sh;
    if (wg_read_flag(&st->done, sh)) return;
    // S2: delta = <d, w> rounded once; rho = beta_l / delta
    long long esc_d = 0;
    const T delta = merge_slots<MODE, P, T>(sd, Gd, ee, capture, sh.acc[0], &esc_d, &st->flags, sh, 0);
    const bool bad = (st->flags & FLAG_NONFINITE) || !is_finite_bits((double)delta);
    const bool breakdown = !(delta > T(0));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->escapes += esc_d;
        if (capture && esc_d > 0) st->fallbacks += 1;
        st->delta = delta;
        if (bad) { st->status = -6; st->done = 1; st->ended = l; }
        else if (breakdown) { st->status = -5; st->done = 1; st->ended = l; }
    }
    if (bad || breakdown) return;
    const T rho = (T)v.beta_hist[l] / delta;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rho = rho;

    zero_acc(sh.acc[0]);
    zero_acc(sh.acc[1]);
    __syncthreads();
    LaneDot<MODE, P> Lb, Lt;
    Lb.init();
    Lt.init();
    // software-pipelined grid-stride loop: the operands of the thread's next
    // element are loaded before the current one is computed, so the loads
    // are in flight while the two exact dots of the current element run
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    T wn = T(0), rn = T(0), qn = T(0);
    if (i < n) { wn = v.w[i]; rn = v.r[i]; qn = v.dinv[i]; }
    for (; i < n; i += stride) {
        const T wi = wn, r0 = rn, qi = qn;
        const long long inext = i + stride;
        if (inext < n) { wn = v.w[inext]; rn = v.r[inext]; qn = v.dinv[inext]; }
        const T ri = fma_t(-rho, wi, r0);                 // S4
        const T zi = qi * ri;                             // S5
        v.r[i] = ri;
        v.z[i] = zi;
        Lb.add(zi, ri, sh.acc[0], ee, capture);           // S6
        Lt.add(ri, ri, sh.acc[1], ee, capture);           // S8
    }
    block_finish_pair<MODE, P>(Lb, sh.acc[0], wb, Lt, sh.acc[1], wt, blockIdx.x, ee, capture, &st->flags, sh);
}

// Elements per thread whose operands K3 loads before merging the dots, so
// the loads are in flight while the merge runs.
constexpr int DIR_PREFETCH = 8;

// Workgroup-uniform value of PcgState::ended (one thread reads it).
__device__ __forceinline__ int wg_read_ended(const int *p, RedShared &sh)
{
    if (threadIdx.x == 0) sh.flag = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return sh.flag;
}

// S3: with S3 set (the Jacobi solver) this kernel also applies the iterate
// update x = fma(rho, d, x) of iteration l; the factored solver's update
// kernel applies it itself.
template <int MODE, int P, typename T, bool S3>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_direction(int l, int n, PcgVecs<T> v, PcgState *st, SlotView wb, SlotView wt, int G, bool ee, bool capture)
{
    __shared__ RedShared sh;
    if constexpr (S3) {
        if (wg_read_ended(&st->ended, sh) <= l) return;
    } else {
        if (wg_read_flag(&st->done, sh)) return;
    }
    const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    T dv[DIR_PREFETCH], zv[DIR_PREFETCH], xv[DIR_PREFETCH];
#pragma unroll
    for (int j = 0; j < DIR_PREFETCH; ++j) {
        const long long i = i0 + j * stride;
        dv[j] = i < n ? v.d[i] : T(0);
        zv[j] = i < n ? v.z[i] : T(0);
        if constexpr (S3) xv[j] = i < n ? v.x[i] : T(0);
    }
    long long eb = 0, et = 0;
    const T beta = merge_slots<MODE, P, T>(wb, G, ee, capture, sh.acc[0], &eb, &st->flags, sh, 0);
    const T tau = merge_slots<MODE, P, T>(wt, G, ee, capture, sh.acc[1], &et, &st->flags, sh, 1);
    const bool bad = (st->flags & FLAG_NONFINITE) || !is_finite_bits((double)beta) || !is_finite_bits((double)tau);
    const int it = l + 1;
    const bool stop = bad || (double)tau <= st->thr || it >= st->maxit;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->escapes += eb + et;
        if (capture) st->fallbacks += (eb > 0) + (et > 0);
        if (bad) {
            st->status = -6;
        } else {
            v.beta_hist[it] = beta;
            st->beta = beta;
            st->tau = tau;
            st->iter = it;
            if (v.hist) v.hist[it] = tau;
        }
        if (stop) {
            st->done = 1;
            if constexpr (S3) st->ended = it;
        }
    }
    if constexpr (S3) {
        const T rho = (T)st->rho; // K2's rho of iteration l
        if (stop) {
#pragma unroll
            for (int j = 0; j < DIR_PREFETCH; ++j) {
                const long long i = i0 + j * stride;
                if (i < n) v.x[i] = fma_t(rho, dv[j], xv[j]);     // S3
            }
            for (long long i = i0 + DIR_PREFETCH * stride; i < n; i += stride)
                v.x[i] = fma_t(rho, v.d[i], v.x[i]);
            return;
        }
        const T gamma = beta / (T)v.beta_hist[l];
        if (blockIdx.x == 0 && threadIdx.x == 0) st->gamma = gamma;
#pragma unroll
        for (int j = 0; j < DIR_PREFETCH; ++j) {
            const long long i = i0 + j * stride;
            if (i < n) {
                v.x[i] = fma_t(rho, dv[j], xv[j]);                 // S3
                v.d[i] = fma_t(gamma, dv[j], zv[j]);               // S7
            }
        }
        for (long long i = i0 + DIR_PREFETCH * stride; i < n; i += stride) {
            const T di = v.d[i];
            v.x[i] = fma_t(rho, di, v.x[i]);
            v.d[i] = fma_t(gamma, di, v.z[i]);
        }
    } else {
        if (stop) return;
        const T gamma = beta / (T)v.beta_hist[l];
        if (blockIdx.x == 0 && threadIdx.x == 0) st->gamma = gamma;
#pragma unroll
        for (int j = 0; j < DIR_PREFETCH; ++j) {
            const long long i = i0 + j * stride;
            if (i < n) v.d[i] = fma_t(gamma, dv[j], zv[j]);   // S7
        }
        for (long long i = i0 + DIR_PREFETCH * stride; i < n; i += stride)
            v.d[i] = fma_t(gamma, v.d[i], v.z[i]);
    }
}

template <typename T>
hipError_t launch_pcg_update(int mode, int l, int n, const PcgVecs<T> &v, PcgState *st, const DotWs &wsd, int Gd,
                             const DotWs *ws2, int stride, const LaunchCfg &c)
{
    SlotView sd{wsd, stride}, sb{ws2[0], stride}, stt{ws2[1], stride};
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        k_pcg_update<M, PP, T><<<c.grid, c.block, 0, c.stream>>>(l, n, v, st, sd, Gd, sb, stt, c.early_exit,
                                                                 c.fallback);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_direction(int mode, int l, int n, const PcgVecs<T> &v, PcgState *st, const DotWs *ws2, int G,
                                int stride, const LaunchCfg &c, bool s3)
{
    SlotView sb{ws2[0], stride}, stt{ws2[1], stride};
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        if (s3)
            k_pcg_direction<M, PP, T, true><<<c.grid, c.block, 0, c.stream>>>(l, n, v, st, sb, stt, G, c.early_exit,
                                                                              c.fallback);
        else
            k_pcg_direction<M, PP, T, false><<<c.grid, c.block, 0, c.stream>>>(l, n, v, st, sb, stt, G,
                                                                               c.early_exit, c.fallback);
    });
    return hipGetLastError();
}

// Built once per value type (the library compiles this file with
// -DRPCG_VALUE_TYPE=double and with -DRPCG_VALUE_TYPE=float).
#ifndef RPCG_VALUE_TYPE
#error "define RPCG_VALUE_TYPE (double or float)"
#endif
template hipError_t launch_pcg_update<RPCG_VALUE_TYPE>(int, int, int, const PcgVecs<RPCG_VALUE_TYPE> &, PcgState *, const DotWs &,
                                              int, const DotWs *, int, const LaunchCfg &);
template hipError_t launch_pcg_direction<RPCG_VALUE_TYPE>(int, int, int, const PcgVecs<RPCG_VALUE_TYPE> &, PcgState *,
                                                 const DotWs *, int, int, const LaunchCfg &, bool);

} // namespace rpcg
