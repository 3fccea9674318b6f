// Jacobi-PCG iteration, first kernel: SpMV fused with the first dot (S1, S2).
#include "reduce.hpp"

namespace rpcg {

// Entries of one row loaded per batch: loads of a batch are issued together
// so the wavefront waits for memory once per batch, not once per entry
// (9 divides the 27 entries of an interior 27-point row).
constexpr int SPMV_BATCH = 9;

__device__ __forceinline__ long long uniform_ll(long long v)
{
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xFFFFFFFFll));
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// K1: w = A d (S1; Section 4.3: per row a sequential fma chain in storage
// order from +0) and the workgroup partial of <d, w> (S2).
//
// Wavefront -> slice mapping: with xcd_split, the slices are cut into
// `xcd_parts` contiguous ranges and workgroup b works in range b % xcd_parts
// (workgroups are dispatched round-robin over the XCDs), so the rows whose d
// entries an XCD gathers stay together in that XCD's L2.
// Column of entry k (index kk into the slice arrays): 32-bit absolute, or
// 16-bit offset from min(row, n-1).
template <bool COL16>
__device__ __forceinline__ int sell_col(const SellMat &A, long long kk, int rbase)
{
    if constexpr (COL16) return rbase + (int)A.col16[kk];
    else return A.col[kk];
}

template <int MODE, int P, bool COL16>
__global__ void __launch_bounds__(MAX_BLOCK)
k_pcg_spmv_dot(SellMat A, PcgVecs v, PcgState *st, SlotView sv, bool ee, bool capture, int xcd_parts)
{
    __shared__ RedShared sh;
    if (st->done) return;
    long long *acc = sh.acc[0];
    zero_acc(acc);
    __syncthreads();
    LaneDot<MODE, P> L;
    L.init();
    const int lane = lane_id();
    const double *__restrict__ d = v.d;
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
        const bool row = i < A.n;
        const int rbase = row ? (int)i : A.n - 1;
        const int len = !row ? 0 : (A.len8 ? (int)A.len8[i] : A.row_ptr[i + 1] - A.row_ptr[i]);
        const long long kb = base + lane;
        const double *__restrict__ pv = A.val + kb;
        double sum = 0.0;
        // every position up to the slice width holds a valid column (padding
        // entries and the lanes past the last row point at a row of the
        // matrix), so loads and gathers of a full batch need no branch; the
        // fma applies only to the row's own entries, in storage order
        int k0 = 0;
        for (; k0 + SPMV_BATCH <= width; k0 += SPMV_BATCH) {
            int c[SPMV_BATCH];
            double a[SPMV_BATCH], g[SPMV_BATCH];
#pragma unroll
            for (int u = 0; u < SPMV_BATCH; ++u) c[u] = sell_col<COL16>(A, kb + 64 * (k0 + u), rbase);
#pragma unroll
            for (int u = 0; u < SPMV_BATCH; ++u) a[u] = pv[64 * (k0 + u)];
#pragma unroll
            for (int u = 0; u < SPMV_BATCH; ++u) g[u] = d[c[u]];
#pragma unroll
            for (int u = 0; u < SPMV_BATCH; ++u) {
                const double t = __builtin_fma(a[u], g[u], sum);
                sum = (k0 + u < len) ? t : sum;
            }
        }
        for (; k0 < width; ++k0) {
            const double t = __builtin_fma(pv[64 * k0], d[sell_col<COL16>(A, kb + 64 * k0, rbase)], sum);
            sum = (k0 < len) ? t : sum;
        }
        if (row) {
            v.w[i] = sum;
            L.add(d[i], sum, acc, ee, capture);
        }
    }
    block_finish<MODE, P>(L, acc, sv, blockIdx.x, ee, capture, &st->flags, sh);
}

hipError_t launch_pcg_spmv_dot(int mode, const SellMat &A, const PcgVecs &v, PcgState *st,
                               const DotWs &ws, int stride, const LaunchCfg &c)
{
    const int parts = (c.grid >= 64 && c.xcd_parts > 1) ? c.xcd_parts : 1;
    SlotView sv{ws, stride};
    dispatch(mode, c.fpe_size, [&](auto m, auto p) {
        constexpr int M = decltype(m)::value, PP = decltype(p)::value;
        if (A.col16)
            k_pcg_spmv_dot<M, PP, true><<<c.grid, c.block, 0, c.stream>>>(A, v, st, sv, c.early_exit, c.fallback, parts);
        else
            k_pcg_spmv_dot<M, PP, false><<<c.grid, c.block, 0, c.stream>>>(A, v, st, sv, c.early_exit, c.fallback, parts);
    });
    return hipGetLastError();
}

} // namespace rpcg
