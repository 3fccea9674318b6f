// Host-side context of the C-ABI (private to the library): device
// workspace owned by an rpcg_ctx, and the small helpers every entry point uses.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <map>
#include <vector>

#include "rpcg.h"
#include "kernels.hpp"

namespace rpcg_host {

struct Buffer {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need)
    {
        if (need <= bytes) return hipSuccess;
        if (p) { hipError_t e = hipFree(p); if (e != hipSuccess) return e; p = nullptr; bytes = 0; }
        hipError_t e = hipMalloc(&p, need);
        if (e == hipSuccess) bytes = need;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p); // teardown: nothing to report to
        p = nullptr;
        bytes = 0;
    }
};

} // namespace rpcg_host

struct rpcg_ctx {
    int device = 0;
    int num_cus = 256;
    int ws_groups = 0;        // capacity of the dot workspaces, in workgroups
    rpcg_host::Buffer ws_mem; // 3 dot workspaces
    rpcg::DotWs ws[3];
    rpcg_host::Buffer scalars; // DotInfo + PcgState + IrState
    rpcg::DotInfo *info = nullptr;
    rpcg::PcgState *st = nullptr;
    rpcg::IrState *ist = nullptr;
    rpcg_host::Buffer sell_off, sell_val, sell_val32, sell_col, sell_cfirst, sell_len;
    rpcg_host::Buffer vecs;    // r, z, d, w, dinv of the solver
    rpcg_host::Buffer ir_vecs; // refinement: r (binary64), rf and c (binary32)
    rpcg_host::Buffer beta_hist; // beta of every iteration
    rpcg_host::Buffer scan_scratch; // slice widths of structural checks of extra CSR arguments
    int *host_done = nullptr;  // pinned: polled flags
    rpcg::PcgState *host_state = nullptr;
    rpcg::IrState *host_ir = nullptr;
    std::vector<hipEvent_t> events;
    std::vector<hipEvent_t> ir_events;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    std::map<uint64_t, rpcg_batch_tuning> batch_tunings; // autotuner results by batch signature
};

static_assert(sizeof(rpcg::DotInfo) <= 256 && sizeof(rpcg::PcgState) <= 256 && sizeof(rpcg::IrState) <= 256,
              "scalar layout");

namespace rpcg_host {

inline int hip_status(hipError_t e)
{
    if (e == hipSuccess) return RPCG_OK;
    if (e == hipErrorOutOfMemory) return RPCG_ERR_OOM;
    return RPCG_ERR_HIP;
}

#define RPCG_TRY(expr)                                          \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return rpcg_host::hip_status(_e); \
    } while (0)

inline bool valid_opts(const rpcg_opts &o)
{
    using rpcg::MAX_BLOCK;
    using rpcg::MAX_FPE;
    if (!(o.tol >= 0.0) || o.maxit < 0) return false;
    if (o.fpe_size < 0 || o.fpe_size > MAX_FPE) return false;
    if (o.block_size != 0 && (o.block_size < 64 || o.block_size > MAX_BLOCK || o.block_size % 64)) return false;
    if (o.grid_size < 0 || o.grid_size > 65536) return false;
    if (o.xcd_parts < 0 || o.xcd_parts > 64) return false;
    if (o.spmv_block_size != 0 && (o.spmv_block_size < 64 || o.spmv_block_size > MAX_BLOCK || o.spmv_block_size % 64))
        return false;
    if (o.spmv_grid_size < 0 || o.spmv_grid_size > 65536) return false;
    if (o.timing < 0 || o.timing > 65) return false;
    return true;
}

inline bool valid_csr(const rpcg_csr *A)
{
    if (!A || A->n < 0 || A->nnz < 0) return false;
    if (A->n > 0 && (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))) return false;
    return true;
}

// Expansion length: 0 = auto. FPE mode: 4. EXBLAS mode: 3 (its results do
// not depend on the length; 3 was the fastest on the 27-point workload).
inline int resolve_fpe_size(int p, int mode)
{
    if (p) return p;
    return mode == rpcg::MODE_EXBLAS ? 3 : 4;
}

// Timing events between solver kernels. They carry no system-scope fence:
// the kernels' results stay on the device, and a fence per event would write
// back the caches between kernels and slow the timed loop.
inline int ensure_events(std::vector<hipEvent_t> &evs, size_t need)
{
    while (evs.size() < need) {
        hipEvent_t e;
        RPCG_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        evs.push_back(e);
    }
    return RPCG_OK;
}

inline double ms_since(std::chrono::steady_clock::time_point t)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

} // namespace rpcg_host
