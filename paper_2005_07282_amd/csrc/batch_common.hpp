// Helpers shared by the batched-solve kernels: the per-system view of the
// concatenated matrix copy and of the dot-partial slots.
#pragma once

#include "reduce.hpp"
#include "sell_spmv.hpp"

namespace rpcg {

// The sliced-ELL view of system S (local rows and columns).
__device__ __forceinline__ SellMat<double> batch_mat(const BatchArgs &a, const BatchSys &S)
{
    SellMat<double> M;
    M.n = S.n;
    M.nslices = S.nslices;
    M.off = a.off + S.slice0;
    M.val = a.val;
    M.col = a.col;
    M.row_ptr = S.row_ptr;
    M.len8 = a.len8 ? a.len8 + S.row0 : nullptr;
    M.col16 = a.col16;
    M.cfirst = a.cfirst ? a.cfirst + S.slice0 : nullptr;
    M.val64 = nullptr;
    return M;
}

// Slots [g0, ...) of a workspace seen as slots [0, ...).
template <int MODE>
__device__ __forceinline__ SlotView batch_slots(const SlotView &v, int g0)
{
    SlotView o = v;
    o.ws.digits += g0;
    o.ws.range += 2 * g0;
    o.ws.part += (MODE == MODE_PLAIN) ? (long long)g0 : (long long)g0 * MAX_FPE;
    o.ws.esc += g0;
    return o;
}

// Flags of a system after this workgroup's merges (read from the coherent
// level, not a possibly stale cached copy).
__device__ __forceinline__ int batch_flags(const PcgState *st)
{
    return __hip_atomic_load(&st->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

} // namespace rpcg
