// Jacobi-PCG iteration, first kernel: SpMV fused with the first dot (S1, S2),
// for binary64 (T = double) and the binary32 inner solver (T = float).
#include "reduce.hpp"
#include "sell_spmv.hpp"

namespace rpcg {

// K1: w = A d (S1; Section 4.3: per row a sequential fma chain in storage
// order from +0) and the workgroup partial of <d, w> (S2).
//
// Wavefront -> slice mapping: with xcd_split, the slices are cut into
// `xcd_parts` contiguous ranges and workgroup b works in range b % xcd_parts
// (workgroups are dispatched round-robin over the XCDs), so the rows whose d
// entries an XCD gathers stay together in that XCD's L2.
template <int MODE, int P, bool COL16, typename T>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_spmv_dot(SellMat<T> A, PcgVecs<T> v, PcgState *st, SlotView sv, bool ee, bool capture, int xcd_parts)
{
    __shared__ RedShared sh;
    if (st->done) return;
    long long *acc = sh.acc[0];
    zero_acc(acc);
    __syncthreads();
    LaneDot<MODE, P> L;
    L.init();
    const int lane = lane_id();
    const T *__restrict__ d = v.d;
    const int W = num_waves();
    // range of slices handled by this workgroup's group of workgroups
    const int part = blockIdx.x % xcd_parts;
    const int groups_in_part = (gridDim.x - part + xcd_parts - 1) / xcd_parts;
    const int idx_in_part = blockIdx.x / xcd_parts;
    const long long s_begin = (long long)A.nslices * part / xcd_parts;
    const long long s_end = (long long)A.nslices * (part + 1) / xcd_parts;
    const long long wstride = (long long)groups_in_part * W;
    // the slice index is the same for all lanes of a wavefront: keep it (and
    // what is derived from it) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(wave_id());
    for (long long s = s_begin + (long long)idx_in_part * W + wave; s < s_end; s += wstride) {
        const long long base = uniform_ll(A.off[s]);
        const int width = __builtin_amdgcn_readfirstlane((int)((A.off[s + 1] - base) >> 6));
        const long long i = s * 64 + lane;
        const int len = sell_len(A, i);
        const T sum = sell_row<T, COL16, false>(A, base, width, i, len, d, nullptr, nullptr);
        if (i < A.n) {
            v.w[i] = sum;
            L.add(d[i], sum, acc, ee, capture);
        }
    }
    block_finish<MODE, P>(L, acc, sv, blockIdx.x, ee, capture, &st->flags, sh);
}

template <typename T>
hipError_t launch_pcg_spmv_dot(int mode, const SellMat<T> &A, const PcgVecs<T> &v, PcgState *st,
                               const DotWs &ws, int stride, const LaunchCfg &c)
{
    const int parts = (c.grid >= 64 && c.xcd_parts > 1) ? c.xcd_parts : 1;
    SlotView sv{ws, stride};
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        if (A.col16)
            k_pcg_spmv_dot<M, PP, true, T><<<c.grid, c.block, 0, c.stream>>>(A, v, st, sv, c.early_exit,
                                                                            c.fallback, parts);
        else
            k_pcg_spmv_dot<M, PP, false, T><<<c.grid, c.block, 0, c.stream>>>(A, v, st, sv, c.early_exit,
                                                                             c.fallback, parts);
    });
    return hipGetLastError();
}

// Built once per value type (the library compiles this file with
// -DRPCG_VALUE_TYPE=double and with -DRPCG_VALUE_TYPE=float).
#ifndef RPCG_VALUE_TYPE
#error "define RPCG_VALUE_TYPE (double or float)"
#endif
template hipError_t launch_pcg_spmv_dot<RPCG_VALUE_TYPE>(int, const SellMat<RPCG_VALUE_TYPE> &, const PcgVecs<RPCG_VALUE_TYPE> &, PcgState *,
                                                const DotWs &, int, const LaunchCfg &);

} // namespace rpcg
