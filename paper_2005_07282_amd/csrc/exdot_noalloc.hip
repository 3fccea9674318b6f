// rpcg_exdot_noalloc: the dot product of rpcg_exdot for callers that cannot
// allocate device memory. The workgroup slots and the call's counters live in
// a file-scope device array instead of a context workspace; the kernels are
// those of rpcg_exdot and take the array's device address as their workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "rpcg.h"
#include "context.hpp"
#include "kernels.hpp"

namespace {

using namespace rpcg;

constexpr int NA_GROUPS = RPCG_NOALLOC_MAX_GROUPS;
constexpr size_t NA_INFO_BYTES = 256;
// per slot: accumulator words, range pair, expansion / partial sum, escape count
constexpr size_t NA_SLOT_BYTES = ACC_WORDS * sizeof(long long) + 2 * sizeof(int) + MAX_FPE * sizeof(double) + sizeof(int);
constexpr size_t NA_BYTES = NA_INFO_BYTES + (size_t)NA_GROUPS * NA_SLOT_BYTES;
static_assert(sizeof(DotInfo) <= NA_INFO_BYTES, "counter record fits its reserved bytes");

// One copy per GPU, held until the process ends. In host code this name is
// only a handle for hipGetSymbolAddress: kernels receive the address that
// call returns.
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_MAX_DEVICES = 64;
struct DevScratch {
    std::once_flag once;
    hipError_t err = hipSuccess;
    unsigned char *ptr = nullptr; // device address of this GPU's copy of scratch
    int num_cus = 256;
};
DevScratch g_dev[NA_MAX_DEVICES];

// Address of the current device's array (looked up once per device, with the
// device current) and its compute-unit count.
hipError_t device_scratch(int dev, unsigned char **ptr, int *cus)
{
    DevScratch &d = g_dev[dev];
    std::call_once(d.once, [&d, dev]() {
        void *p = nullptr;
        d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (d.err == hipSuccess) d.ptr = (unsigned char *)p;
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
            d.num_cus = c;
    });
    *ptr = d.ptr;
    *cus = d.num_cus;
    return d.err;
}

// The counters must start at zero; a fill kernel rather than a memset node,
// so that a captured graph replays it correctly.
__global__ void k_zero_words(unsigned long long *p, int words)
{
    for (int i = threadIdx.x; i < words; i += blockDim.x) p[i] = 0ull;
}

} // namespace

extern "C" int rpcg_exdot_noalloc(rpcg_mode mode_in, int64_t n, const double *x, const double *y, double *out,
                                  const rpcg_opts *opts, rpcg_result *res, void *stream)
{
    using namespace rpcg_host;
    const int mode = (int)mode_in;
    if (n < 0 || (n > 0 && (!x || !y)) || !out) return RPCG_ERR_INVALID;
    if (mode != MODE_PLAIN && mode != MODE_FPE && mode != MODE_EXBLAS) return RPCG_ERR_INVALID;
    rpcg_opts o;
    rpcg_opts_default(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return RPCG_ERR_INVALID;
    if (o.grid_size > NA_GROUPS) return RPCG_ERR_INVALID; // more slots than the static array holds
    o.fpe_size = resolve_fpe_size(o.fpe_size, mode);
    int dev = 0;
    RPCG_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NA_MAX_DEVICES) return RPCG_ERR_INVALID;
    unsigned char *base = nullptr;
    int cus = 256;
    RPCG_TRY(device_scratch(dev, &base, &cus));
    hipStream_t s = (hipStream_t)stream;

    // launch shape of rpcg_exdot, with the grid capped by the slot count
    LaunchCfg cfg;
    cfg.block = o.block_size ? o.block_size : 1024;
    cfg.grid = o.grid_size ? o.grid_size
                           : (int)std::max<int64_t>(1, std::min<int64_t>((n + 8ll * cfg.block - 1) / (8ll * cfg.block),
                                                                         (mode == MODE_PLAIN ? 8ll : 4ll) * cus));
    if (!o.grid_size && mode != MODE_PLAIN)
        cfg.grid = (int)std::max<int64_t>(std::min<int64_t>(cfg.grid, cus),
                                          std::min<int64_t>(cfg.grid, (n + 256ll * cfg.block - 1) / (256ll * cfg.block)));
    cfg.grid = std::min(cfg.grid, NA_GROUPS);
    cfg.early_exit = o.early_exit != 0;
    cfg.fpe_size = o.fpe_size;
    cfg.fallback = o.fpe_fallback != 0;
    cfg.xcd_parts = 1;
    cfg.stream = s;

    // layout of the array: counters, then the slot arrays for NA_GROUPS workgroups
    DotInfo *info = (DotInfo *)base;
    unsigned char *b = base + NA_INFO_BYTES;
    DotWs ws;
    ws.digits = (long long *)b;
    b += (size_t)NA_GROUPS * ACC_WORDS * sizeof(long long);
    ws.part = (double *)b;
    b += (size_t)NA_GROUPS * MAX_FPE * sizeof(double);
    ws.range = (int *)b;
    b += (size_t)NA_GROUPS * 2 * sizeof(int);
    ws.esc = (int *)b;

    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (unsigned long long *)info,
                       (int)(sizeof(DotInfo) / sizeof(unsigned long long)));
    RPCG_TRY(hipGetLastError());
    RPCG_TRY(launch_exdot(mode, n, x, y, out, ws, NA_GROUPS, info, cfg));
    if (res) {
        std::memset(res, 0, sizeof(*res));
        DotInfo inf;
        RPCG_TRY(hipMemcpyAsync(&inf, info, sizeof inf, hipMemcpyDeviceToHost, s));
        RPCG_TRY(hipStreamSynchronize(s));
        res->fpe_escapes = inf.escapes;
        res->fallbacks = inf.fallbacks;
        res->grid_size = cfg.grid;
        res->block_size = cfg.block;
        int st = RPCG_OK;
        if (inf.flags & FLAG_NONFINITE) st = RPCG_ERR_NONFINITE;
        else if (inf.flags & FLAG_INEXACT) st = RPCG_WARN_FPE_INEXACT;
        else if (mode == MODE_FPE && inf.escapes > 0 && !cfg.fallback) st = RPCG_WARN_FPE_INEXACT;
        res->status = st;
        return st;
    }
    return RPCG_OK;
}
