// C-ABI of the reproducible Jacobi-PCG library (declared in include/rpcg.h).
// Host side only: argument checks, workspace, launch configuration and the
// iteration loop. Every arithmetic step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "rpcg.h"
#include "context.hpp"
#include "kernels.hpp"

using namespace rpcg;
using namespace rpcg_host;

static int ensure_ws(rpcg_ctx *c, int groups)
{
    if (groups <= c->ws_groups) return RPCG_OK;
    size_t per = (size_t)groups * (ACC_WORDS * sizeof(long long) + 2 * sizeof(int) +
                                   MAX_FPE * sizeof(double) + sizeof(int));
    RPCG_TRY(c->ws_mem.ensure(3 * per + 256 * 4));
    char *base = (char *)c->ws_mem.p;
    for (int i = 0; i < 3; ++i) {
        char *b = base + i * per;
        c->ws[i].digits = (long long *)b;
        b += (size_t)groups * ACC_WORDS * sizeof(long long);
        c->ws[i].part = (double *)b;
        b += (size_t)groups * MAX_FPE * sizeof(double);
        c->ws[i].range = (int *)b;
        b += (size_t)groups * 2 * sizeof(int);
        c->ws[i].esc = (int *)b;
    }
    c->ws_groups = groups;
    return RPCG_OK;
}

static LaunchCfg make_cfg(const rpcg_ctx *c, const rpcg_opts &o, long long work_items, int block_default,
                          hipStream_t s)
{
    LaunchCfg cfg;
    cfg.block = o.block_size ? o.block_size : block_default;
    long long want = (work_items + cfg.block - 1) / cfg.block;
    long long cap = 8ll * c->num_cus;
    cfg.grid = o.grid_size ? o.grid_size : (int)std::max(1ll, std::min(want, cap));
    cfg.early_exit = o.early_exit != 0;
    cfg.fpe_size = o.fpe_size;
    cfg.fallback = o.fpe_fallback != 0;
    cfg.xcd_parts = o.xcd_parts ? o.xcd_parts : 1;
    cfg.stream = s;
    return cfg;
}

// Vector kernels (setup, K2, K3): 512-thread workgroups, at most two per CU,
// so that the slot merges in the next kernel's prologue stay short.
static LaunchCfg make_vec_cfg(const rpcg_ctx *c, const rpcg_opts &o, long long n, hipStream_t s)
{
    LaunchCfg cfg = make_cfg(c, o, n, 512, s);
    if (!o.grid_size) cfg.grid = (int)std::max(1ll, std::min((n + cfg.block - 1) / cfg.block, 2ll * c->num_cus));
    return cfg;
}

// SpMV kernel: one wavefront per 64-row slice at a time; own overrides. The
// binary32 kernel keeps fewer bytes in flight per wavefront and wants twice
// the workgroups of the binary64 one.
static LaunchCfg make_spmv_cfg(const rpcg_ctx *c, const rpcg_opts &o, long long nslices, hipStream_t s,
                               bool f32 = false)
{
    rpcg_opts q = o;
    q.block_size = o.spmv_block_size;
    q.grid_size = o.spmv_grid_size;
    LaunchCfg cfg = make_cfg(c, q, std::max(1ll, nslices * 64), 256, s);
    const long long cap = (f32 ? 4ll : 2ll) * c->num_cus;
    if (!q.grid_size) cfg.grid = (int)std::max(1ll, std::min((nslices * 64 + cfg.block - 1) / cfg.block, cap));
    return cfg;
}

extern "C" {

void rpcg_opts_default(rpcg_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->maxit = 2000;
    o->fpe_size = 0;
    o->early_exit = 1;
    o->fpe_fallback = 1;
}

const char *rpcg_status_string(int s)
{
    switch (s) {
    case RPCG_OK: return "ok";
    case RPCG_WARN_MAXIT: return "warning: maximum iterations reached";
    case RPCG_WARN_FPE_INEXACT: return "warning: expansion capacity exceeded or product outside the exact domain";
    case RPCG_ERR_INVALID: return "error: invalid argument";
    case RPCG_ERR_HIP: return "error: HIP runtime failure";
    case RPCG_ERR_OOM: return "error: out of device memory";
    case RPCG_ERR_NOT_SPD: return "error: missing or non-positive diagonal entry";
    case RPCG_ERR_BREAKDOWN: return "error: <d, A d> <= 0";
    case RPCG_ERR_NONFINITE: return "error: non-finite value";
    default: return "unknown status";
    }
}

int rpcg_create(rpcg_ctx **out, int device)
{
    if (!out) return RPCG_ERR_INVALID;
    *out = nullptr;
    int count = 0;
    RPCG_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(device));
    rpcg_ctx *c = new (std::nothrow) rpcg_ctx();
    if (!c) return RPCG_ERR_OOM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cus = prop.multiProcessorCount;
    int rc = hip_status(c->scalars.ensure(1024));
    if (rc == RPCG_OK) {
        c->info = (DotInfo *)c->scalars.p;
        c->st = (PcgState *)((char *)c->scalars.p + 256);
        c->ist = (IrState *)((char *)c->scalars.p + 512);
        rc = hip_status(hipMemset(c->scalars.p, 0, 1024));
    }
    if (rc == RPCG_OK) rc = hip_status(hipHostMalloc((void **)&c->host_done, 64 * sizeof(int), hipHostMallocDefault));
    if (rc == RPCG_OK) rc = hip_status(hipHostMalloc((void **)&c->host_state, sizeof(PcgState), hipHostMallocDefault));
    if (rc == RPCG_OK) rc = hip_status(hipHostMalloc((void **)&c->host_ir, sizeof(IrState), hipHostMallocDefault));
    if (rc == RPCG_OK) rc = hip_status(hipEventCreateWithFlags(&c->poll_ev[0], hipEventDisableTiming));
    if (rc == RPCG_OK) rc = hip_status(hipEventCreateWithFlags(&c->poll_ev[1], hipEventDisableTiming));
    if (rc == RPCG_OK) rc = ensure_ws(c, 8 * c->num_cus);
    if (rc != RPCG_OK) { rpcg_destroy(c); return rc; }
    *out = c;
    return RPCG_OK;
}

void rpcg_destroy(rpcg_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device); // teardown reports nothing
    (void)hipDeviceSynchronize();
    c->ws_mem.release();
    c->scalars.release();
    c->sell_off.release();
    c->sell_val.release();
    c->sell_val32.release();
    c->sell_col.release();
    c->sell_cfirst.release();
    c->sell_len.release();
    c->scan_scratch.release();
    c->vecs.release();
    c->ir_vecs.release();
    c->beta_hist.release();
    if (c->host_done) (void)hipHostFree(c->host_done);
    if (c->host_state) (void)hipHostFree(c->host_state);
    if (c->host_ir) (void)hipHostFree(c->host_ir);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ir_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->poll_ev) if (e) (void)hipEventDestroy(e);
    delete c;
}

static int exdot_status(const DotInfo &inf, int mode, bool fallback)
{
    if (inf.flags & FLAG_NONFINITE) return RPCG_ERR_NONFINITE;
    if (inf.flags & FLAG_INEXACT) return RPCG_WARN_FPE_INEXACT;
    if (mode == MODE_FPE && inf.escapes > 0 && !fallback) return RPCG_WARN_FPE_INEXACT;
    return RPCG_OK;
}

static int run_exdot(rpcg_ctx *c, int mode, int64_t n, const double *x, const double *y, double *out,
                     int64_t *digits, const rpcg_opts *opts, rpcg_result *res, void *stream)
{
    if (!c || n < 0 || (n > 0 && (!x || !y)) || (!out && !digits)) return RPCG_ERR_INVALID;
    if (mode != MODE_PLAIN && mode != MODE_FPE && mode != MODE_EXBLAS) return RPCG_ERR_INVALID;
    rpcg_opts o;
    rpcg_opts_default(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return RPCG_ERR_INVALID;
    o.fpe_size = resolve_fpe_size(o.fpe_size, mode);
    RPCG_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    // 1024-thread workgroups; four per CU for the expansion modes, eight for
    // plain (measured at 2^28 elements: 5.2 / 3.8 TB/s exact on narrow / wide
    // data against 4.5 / 3.0 with 256-thread workgroups, eight per CU). The
    // exact modes give a thread at least 256 elements where that still
    // leaves a workgroup per CU: the workgroup's accumulator setup and
    // partial and the lanes' overflow windows are then paid over more data
    // (2^22 to 2^26 elements: 5-25% faster; 2^28 keeps four per CU).
    LaunchCfg cfg = make_cfg(c, o, std::max<int64_t>(1, (n + 7) / 8), 1024, s);
    if (!o.grid_size) {
        cfg.grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 8ll * cfg.block - 1) / (8ll * cfg.block),
                                                               (mode == MODE_PLAIN ? 8ll : 4ll) * c->num_cus));
        if (mode != MODE_PLAIN)
            cfg.grid = (int)std::max<int64_t>(std::min<int64_t>(cfg.grid, c->num_cus),
                                              std::min<int64_t>(cfg.grid, (n + 256ll * cfg.block - 1) / (256ll * cfg.block)));
    }
    int rc = ensure_ws(c, cfg.grid);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipMemsetAsync(c->info, 0, sizeof(DotInfo), s));
    if (digits) RPCG_TRY(launch_exdot_partial(n, x, y, (long long *)digits, c->ws[0], c->ws_groups, c->info, cfg));
    else RPCG_TRY(launch_exdot(mode, n, x, y, out, c->ws[0], c->ws_groups, c->info, cfg));
    if (res) {
        std::memset(res, 0, sizeof(*res));
        DotInfo inf;
        RPCG_TRY(hipMemcpyAsync(&inf, c->info, sizeof inf, hipMemcpyDeviceToHost, s));
        RPCG_TRY(hipStreamSynchronize(s));
        res->fpe_escapes = inf.escapes;
        res->fallbacks = inf.fallbacks;
        res->grid_size = cfg.grid;
        res->block_size = cfg.block;
        res->status = exdot_status(inf, mode, cfg.fallback);
        return res->status;
    }
    return RPCG_OK;
}

int rpcg_exdot(rpcg_ctx *c, rpcg_mode mode, int64_t n, const double *x, const double *y, double *out,
               const rpcg_opts *opts, rpcg_result *res, void *stream)
{
    return run_exdot(c, (int)mode, n, x, y, out, nullptr, opts, res, stream);
}

int rpcg_exdot_partial(rpcg_ctx *c, int64_t n, const double *x, const double *y, int64_t *digits,
                       void *stream)
{
    if (!digits) return RPCG_ERR_INVALID;
    return run_exdot(c, MODE_EXBLAS, n, x, y, nullptr, digits, nullptr, nullptr, stream);
}

int rpcg_acc_round(rpcg_ctx *c, const int64_t *digits, double *out, void *stream)
{
    if (!c || !digits || !out) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(c->device));
    RPCG_TRY(launch_acc_round((const long long *)digits, out, (hipStream_t)stream));
    return RPCG_OK;
}

int rpcg_fpe_size_auto(rpcg_ctx *c, const rpcg_csr *A, const double *b, int32_t *p, int32_t *range_out,
                       void *stream)
{
    if (!c || !valid_csr(A) || (A->n > 0 && !b) || !p) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    int init[2] = {1 << 20, -(1 << 20)};
    int *dev = &c->info->max_len; // two adjacent ints of the scratch record
    static_assert(offsetof(DotInfo, pad1) == offsetof(DotInfo, max_len) + sizeof(int), "adjacent scratch ints");
    RPCG_TRY(hipMemcpyAsync(dev, init, sizeof init, hipMemcpyHostToDevice, s));
    RPCG_TRY(launch_exp_range(A->nnz, A->val, dev, dev + 1, s));
    RPCG_TRY(launch_exp_range(A->n, b, dev, dev + 1, s));
    int got[2];
    RPCG_TRY(hipMemcpyAsync(got, dev, sizeof got, hipMemcpyDeviceToHost, s));
    RPCG_TRY(hipStreamSynchronize(s));
    const int range = got[1] >= got[0] ? got[1] - got[0] : 0;
    // products of two entries span about twice the range; a term holds 53 bits
    *p = std::min(MAX_FPE, 4 + 2 * range / 53);
    if (range_out) *range_out = range;
    return RPCG_OK;
}

int rpcg_spmv(rpcg_ctx *c, const rpcg_csr *A, const double *x, double *y, void *stream)
{
    if (!c || !valid_csr(A) || (A->n > 0 && (!x || !y)) || (A->n > 0 && x == y)) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(c->device));
    RPCG_TRY(launch_spmv_csr(A->n, A->nnz, A->row_ptr, A->col_idx, A->val, x, y, (hipStream_t)stream));
    return RPCG_OK;
}

} // extern "C"

// events per timed iteration: boundaries around K1 | K2 | K3
static const int EV_PER_IT = 4;

// The solver's sliced-ELL copy of a CSR matrix (see SellMat).
struct SellBuilt {
    int nslices = 0;
    bool col16 = false;
    const long long *off = nullptr;
    const double *val64 = nullptr; // binary64 values, if requested
    const float *val32 = nullptr;  // binary32 values, if requested
    const int *col = nullptr;
    const unsigned short *col16p = nullptr;
    const int *cfirst = nullptr;
    const unsigned char *len8 = nullptr;
};

// Device buffers a sliced-ELL copy is built into (the context's for the
// solver, a rpcg_smat's own for prepared matrices).
struct SellBufs {
    rpcg_host::Buffer *off, *val, *val32, *col, *cfirst, *len;
};

static SellBufs ctx_sell_bufs(rpcg_ctx *c)
{
    return {&c->sell_off, &c->sell_val, &c->sell_val32, &c->sell_col, &c->sell_cfirst, &c->sell_len};
}

// One pass over the CSR checks its structure and measures the slices
// (nothing indexes through the matrix before the check has passed), then the
// copy is filled. Source values: v64 or v32; kept as binary64 (out64) and/or
// rounded to binary32 (out32). The interleave is that of the solver's value
// type: two entries for a binary64-only copy, one when binary32 values are
// kept. Waits for the stream.
static int build_sell(rpcg_ctx *c, const SellBufs &bf, int n, int nnz, const int *rp, const int *col,
                      const double *v64, const float *v32, bool out64, bool out32, bool no_col16, hipStream_t s,
                      SellBuilt *out)
{
    const int nslices = (n + 63) / 64;
    const int vec = out32 ? sell_vec<float>() : sell_vec<double>();
    RPCG_TRY(hipMemsetAsync(c->info, 0, sizeof(DotInfo), s));
    RPCG_TRY(bf.off->ensure(sizeof(long long) * (nslices + 1)));
    long long *off = (long long *)bf.off->p;
    RPCG_TRY(hipMemsetAsync(off, 0, sizeof(long long) * (nslices + 1), s));
    RPCG_TRY(launch_csr_scan(n, nnz, rp, col, vec, off + 1, &c->info->flags, &c->info->max_len,
                             &c->info->max_delta, s));
    RPCG_TRY(launch_sell_scan(off, nslices, s));
    long long padded = 0;
    DotInfo scan_info;
    RPCG_TRY(hipMemcpyAsync(&padded, off + nslices, sizeof padded, hipMemcpyDeviceToHost, s));
    RPCG_TRY(hipMemcpyAsync(&scan_info, c->info, sizeof scan_info, hipMemcpyDeviceToHost, s));
    RPCG_TRY(hipStreamSynchronize(s));
    if (scan_info.flags) return RPCG_ERR_INVALID;
    const bool col16 = scan_info.max_delta <= 32767 && !no_col16;
    const size_t np = (size_t)std::max(1ll, padded);
    double *s64 = nullptr;
    float *s32 = nullptr;
    if (out64) { RPCG_TRY(bf.val->ensure(sizeof(double) * np)); s64 = (double *)bf.val->p; }
    if (out32) { RPCG_TRY(bf.val32->ensure(sizeof(float) * np)); s32 = (float *)bf.val32->p; }
    RPCG_TRY(bf.col->ensure((col16 ? sizeof(short) : sizeof(int)) * np));
    int *cfirst = nullptr;
    if (col16) {
        RPCG_TRY(bf.cfirst->ensure(sizeof(int) * (size_t)std::max(1, nslices)));
        cfirst = (int *)bf.cfirst->p;
    }
    unsigned char *len8 = nullptr;
    if (scan_info.max_len < 256) {
        RPCG_TRY(bf.len->ensure((size_t)std::max(1, n)));
        len8 = (unsigned char *)bf.len->p;
    }
    RPCG_TRY(launch_sell_fill(n, rp, col, v64, v32, vec, off, s64, s32, col16 ? nullptr : (int *)bf.col->p,
                              col16 ? (unsigned short *)bf.col->p : nullptr, cfirst, len8, s));
    out->nslices = nslices;
    out->col16 = col16;
    out->off = off;
    out->val64 = s64;
    out->val32 = s32;
    out->col = col16 ? nullptr : (const int *)bf.col->p;
    out->col16p = col16 ? (const unsigned short *)bf.col->p : nullptr;
    out->cfirst = cfirst;
    out->len8 = len8;
    return RPCG_OK;
}

template <typename T>
static SellMat<T> sell_mat(const SellBuilt &B, const T *val, int n, const int *row_ptr)
{
    SellMat<T> M;
    M.n = n;
    M.nslices = B.nslices;
    M.off = B.off;
    M.val = val;
    M.col = B.col;
    M.col16 = B.col16p;
    M.cfirst = B.cfirst;
    M.row_ptr = row_ptr;
    M.len8 = B.len8;
    M.val64 = B.val64;
    return M;
}

struct PcgRun {
    PcgState S;
    int status = 0;
    int launched = 0;
    double setup_ms = 0, loop_ms = 0;
    double k_ms[3] = {0, 0, 0};
    int k_launches = 0;
};

// Jacobi-PCG on a built matrix copy: setup, then batches of K1/K2/K3 with the
// device `done` flag polled one batch behind, so the host never waits on the
// iteration it launches. Waits for the stream.
template <typename T>
static int run_pcg(rpcg_ctx *c, int mode, const SellMat<T> &M, const T *b, T *x, const rpcg_opts &o,
                   const LaunchCfg &cfg_rows, const LaunchCfg &cfg_sl, hipStream_t s, PcgRun *out,
                   const FacPre *fp = nullptr)
{
    constexpr bool F64 = std::is_same<T, double>::value;
    if (fp && !F64) return RPCG_ERR_INVALID;
    auto t0 = std::chrono::steady_clock::now();
    const int n = M.n;
    // five work vectors; the factored preconditioner keeps a second r buffer
    RPCG_TRY(c->vecs.ensure(sizeof(T) * (fp ? 6 : 5) * (size_t)std::max(1, n)));
    T *vb = (T *)c->vecs.p;
    T *r2 = vb + 5 * (size_t)n;
    PcgVecs<T> v;
    v.b = b;
    v.x = x;
    v.r = vb;
    v.z = vb + n;
    v.d = vb + 2 * (size_t)n;
    v.w = vb + 3 * (size_t)n;
    v.dinv = vb + 4 * (size_t)n;
    v.hist = o.tau_history;
    RPCG_TRY(c->beta_hist.ensure(sizeof(double) * ((size_t)o.maxit + 1)));
    v.beta_hist = (double *)c->beta_hist.p;
    const int stride = c->ws_groups;
    T *t = v.dinv; // the factored preconditioner needs no inverse diagonal: t = G^T r lives there
    if constexpr (F64) {
        if (fp) RPCG_TRY(launch_fac_setup(mode, M, *fp, v, t, c->st, c->ws, stride, o.tol, o.maxit, cfg_rows));
        else RPCG_TRY(launch_pcg_setup<T>(mode, M, v, c->st, c->ws, stride, o.tol, o.maxit, cfg_sl));
    } else {
        RPCG_TRY(launch_pcg_setup<T>(mode, M, v, c->st, c->ws, stride, o.tol, o.maxit, cfg_sl));
    }
    RPCG_TRY(hipStreamSynchronize(s));
    out->setup_ms = ms_since(t0);
    auto t1 = std::chrono::steady_clock::now();

    const bool timing = o.timing != 0;
    const bool k1_only = o.timing >= 2;
    const int kstride = k1_only ? o.timing - 1 : 1; // iterations between timed SpMV launches
    const int batch = 8;
    if (timing) {
        int rc = ensure_events(c->events, (size_t)EV_PER_IT * std::max(1, o.maxit));
        if (rc) return rc;
    }
    int launched = 0;
    volatile int *hd = c->host_done;
    hd[0] = hd[1] = 0;
    for (int bidx = 0; launched < o.maxit; ++bidx) {
        int cnt = std::min(batch, o.maxit - launched);
        for (int it = 0; it < cnt; ++it) {
            const int l = launched + it;
            hipEvent_t *ev = (timing && l % kstride == 0) ? &c->events[(size_t)l * EV_PER_IT] : nullptr;
            if (ev) RPCG_TRY(hipEventRecord(ev[0], s));
            RPCG_TRY(launch_pcg_spmv_dot<T>(mode, M, v, c->st, c->ws[0], stride, cfg_sl));
            if (ev) RPCG_TRY(hipEventRecord(ev[1], s));
            if (k1_only) ev = nullptr;
            bool done_fac = false;
            if constexpr (F64) {
                if (fp) {
                    // beta partials in ws[0] (the SpMV's are merged first), tau in ws[1];
                    // r alternates between its buffer and r2
                    PcgVecs<T> vl = v;
                    vl.r = (l & 1) ? r2 : v.r;
                    RPCG_TRY(launch_fac_update(mode, l, n, *fp, vl, (l & 1) ? v.r : r2, t, c->st, c->ws[0],
                                               cfg_sl.grid, c->ws, stride, cfg_rows));
                    if (ev) RPCG_TRY(hipEventRecord(ev[2], s));
                    RPCG_TRY(launch_pcg_direction<T>(mode, l, n, v, c->st, c->ws, cfg_rows.grid, stride, cfg_rows,
                                                     false));
                    done_fac = true;
                }
            }
            if (!done_fac) {
                RPCG_TRY(launch_pcg_update<T>(mode, l, n, v, c->st, c->ws[0], cfg_sl.grid, c->ws + 1, stride,
                                              cfg_rows));
                if (ev) RPCG_TRY(hipEventRecord(ev[2], s));
                RPCG_TRY(launch_pcg_direction<T>(mode, l, n, v, c->st, c->ws + 1, cfg_rows.grid, stride, cfg_rows,
                                                 true));
            }
            if (ev) RPCG_TRY(hipEventRecord(ev[3], s));
        }
        launched += cnt;
        RPCG_TRY(hipMemcpyAsync((void *)&hd[bidx & 1], &c->st->done, sizeof(int), hipMemcpyDeviceToHost, s));
        RPCG_TRY(hipEventRecord(c->poll_ev[bidx & 1], s));
        if (bidx > 0) {
            int pb = (bidx - 1) & 1;
            RPCG_TRY(hipEventSynchronize(c->poll_ev[pb]));
            if (hd[pb]) break;
        }
    }
    RPCG_TRY(hipStreamSynchronize(s));
    out->loop_ms = ms_since(t1);
    RPCG_TRY(hipMemcpy(c->host_state, c->st, sizeof(PcgState), hipMemcpyDeviceToHost));
    const PcgState &S = *c->host_state;
    out->S = S;
    out->launched = launched;
    int status;
    if (S.status < 0) status = S.status;
    else if (!(S.tau <= S.thr)) status = RPCG_WARN_MAXIT;
    else if ((S.flags & FLAG_INEXACT) || (mode == MODE_FPE && S.escapes > 0 && !o.fpe_fallback))
        status = RPCG_WARN_FPE_INEXACT;
    else status = RPCG_OK;
    out->status = status;
    if (timing) {
        // the first L iterations did the work; later launches were no-ops
        const int L = std::min(S.iter, launched);
        int timed = 0;
        for (int i = 0; i < L; i += kstride, ++timed)
            for (int k = 0; k < (k1_only ? 1 : 3); ++k) {
                float ms = 0.f;
                hipEvent_t *ev = &c->events[(size_t)i * EV_PER_IT];
                if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) == hipSuccess) out->k_ms[k] += ms;
            }
        out->k_launches = timed;
    }
    return RPCG_OK;
}

static void fill_result(rpcg_result *res, const PcgRun &run, double build_ms, const LaunchCfg &cfg_rows, bool timing)
{
    if (!res) return;
    const PcgState &S = run.S;
    res->status = run.status;
    res->iterations = S.iter;
    res->tau0 = S.tau0;
    res->tau_final = S.tau;
    res->threshold = S.thr;
    res->fpe_escapes = S.escapes;
    res->fallbacks = S.fallbacks;
    res->setup_ms = build_ms + run.setup_ms;
    res->loop_ms = run.loop_ms;
    res->grid_size = cfg_rows.grid;
    res->block_size = cfg_rows.block;
    if (timing) {
        res->k_spmv_dot_ms = run.k_ms[0];
        res->k_update_ms = run.k_ms[1];
        res->k_direction_ms = run.k_ms[2];
        res->k_launches = run.k_launches;
    }
}

static bool valid_csr_f32(const rpcg_csr_f32 *A)
{
    if (!A || A->n < 0 || A->nnz < 0) return false;
    if (A->n > 0 && (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))) return false;
    return true;
}

// Structural check of a CSR argument on the device (row pointers consistent,
// columns in range), with the scan of the sliced-ELL construction.
static int check_csr(rpcg_ctx *c, const rpcg_csr *E, hipStream_t s)
{
    const int nslices = (E->n + 63) / 64;
    RPCG_TRY(c->scan_scratch.ensure(sizeof(long long) * (nslices + 1)));
    RPCG_TRY(hipMemsetAsync(c->info, 0, sizeof(DotInfo), s));
    RPCG_TRY(launch_csr_scan(E->n, E->nnz, E->row_ptr, E->col_idx, 1, (long long *)c->scan_scratch.p + 1,
                             &c->info->flags, &c->info->max_len, &c->info->max_delta, s));
    DotInfo inf;
    RPCG_TRY(hipMemcpyAsync(&inf, c->info, sizeof inf, hipMemcpyDeviceToHost, s));
    RPCG_TRY(hipStreamSynchronize(s));
    return inf.flags ? RPCG_ERR_INVALID : RPCG_OK;
}

// Common body of the binary64 and binary32 solves.
template <typename T>
static int pcg_solve_any(rpcg_ctx *c, int mode, int n, int nnz, const int *rp, const int *col, const double *v64,
                         const float *v32, const T *b, T *x, const rpcg_opts *opts, rpcg_result *res, void *stream,
                         const FacPre *fp = nullptr, const rpcg_csr *extra0 = nullptr, const rpcg_csr *extra1 = nullptr)
{
    if (mode != MODE_PLAIN && mode != MODE_FPE && mode != MODE_EXBLAS) return RPCG_ERR_INVALID;
    rpcg_opts o;
    rpcg_opts_default(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return RPCG_ERR_INVALID;
    o.fpe_size = resolve_fpe_size(o.fpe_size, mode);
    RPCG_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    const int nslices = (n + 63) / 64;
    constexpr bool F32 = std::is_same<T, float>::value;
    LaunchCfg cfg_rows = make_vec_cfg(c, o, std::max(1, n), s);
    LaunchCfg cfg_sl = make_spmv_cfg(c, o, nslices, s, F32);
    // EXBLAS results do not depend on the lane expansion length. With the
    // default, the binary64 SpMV kernel (and the setup) keep four terms: its
    // <d, w> lanes then flush to the long accumulator less often, while the
    // vector kernels' two dots per element are cheapest with three
    if (!F32 && mode == MODE_EXBLAS && (!opts || opts->fpe_size == 0)) cfg_sl.fpe_size = 4;
    int rc = ensure_ws(c, std::max(cfg_rows.grid, cfg_sl.grid));
    if (rc != RPCG_OK) return rc;
    SellBuilt B;
    rc = build_sell(c, ctx_sell_bufs(c), n, nnz, rp, col, v64, v32, !F32, F32, o.no_col16 != 0, s, &B);
    if (rc != RPCG_OK) return rc;
    for (const rpcg_csr *E : {extra0, extra1}) {
        if (!E) continue;
        rc = check_csr(c, E, s);
        if (rc != RPCG_OK) return rc;
    }
    const double build_ms = ms_since(t0);
    const T *val;
    if constexpr (F32) val = B.val32;
    else val = B.val64;
    SellMat<T> M = sell_mat<T>(B, val, n, rp);
    M.val64 = nullptr;
    PcgRun run;
    rc = run_pcg<T>(c, mode, M, b, x, o, cfg_rows, cfg_sl, s, &run, fp);
    if (rc != RPCG_OK) return rc;
    fill_result(res, run, build_ms, cfg_rows, o.timing != 0);
    return run.status;
}

extern "C" {

int rpcg_pcg_solve(rpcg_ctx *c, rpcg_mode mode, const rpcg_csr *A, const double *b, double *x,
                   const rpcg_opts *opts, rpcg_result *res, void *stream)
{
    if (res) std::memset(res, 0, sizeof(*res));
    if (!c || !valid_csr(A) || (A->n > 0 && (!b || !x))) return RPCG_ERR_INVALID;
    int rc = pcg_solve_any<double>(c, (int)mode, A->n, A->nnz, A->row_ptr, A->col_idx, A->val, nullptr, b, x, opts,
                                   res, stream);
    if (res) res->status = rc;
    return rc;
}

int rpcg_pcg_solve_factored(rpcg_ctx *c, rpcg_mode mode, const rpcg_csr *A, const rpcg_csr *G, const rpcg_csr *Gt,
                            double eps, const double *b, double *x, const rpcg_opts *opts, rpcg_result *res,
                            void *stream)
{
    if (res) std::memset(res, 0, sizeof(*res));
    if (!c || !valid_csr(A) || !valid_csr(G) || !valid_csr(Gt) || (A->n > 0 && (!b || !x))) return RPCG_ERR_INVALID;
    if (G->n != A->n || Gt->n != A->n || !(eps >= 0.0) || !std::isfinite(eps)) return RPCG_ERR_INVALID;
    FacPre fp;
    fp.g_rp = G->row_ptr;
    fp.g_col = G->col_idx;
    fp.g_val = G->val;
    fp.gt_rp = Gt->row_ptr;
    fp.gt_col = Gt->col_idx;
    fp.gt_val = Gt->val;
    fp.eps = eps;
    int rc = pcg_solve_any<double>(c, (int)mode, A->n, A->nnz, A->row_ptr, A->col_idx, A->val, nullptr, b, x, opts,
                                   res, stream, &fp, G, Gt);
    if (res) res->status = rc;
    return rc;
}

int rpcg_pcg_solve_f32(rpcg_ctx *c, rpcg_mode mode, const rpcg_csr_f32 *A, const float *b, float *x,
                       const rpcg_opts *opts, rpcg_result *res, void *stream)
{
    if (res) std::memset(res, 0, sizeof(*res));
    if (!c || !valid_csr_f32(A) || (A->n > 0 && (!b || !x))) return RPCG_ERR_INVALID;
    int rc = pcg_solve_any<float>(c, (int)mode, A->n, A->nnz, A->row_ptr, A->col_idx, nullptr, A->val, b, x, opts,
                                  res, stream);
    if (res) res->status = rc;
    return rc;
}

void rpcg_ir_opts_default(rpcg_ir_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->maxit = 50;
    o->adaptive_inner = 1;
    rpcg_opts_default(&o->inner);
    o->inner.tol = 1e-4;
}

// Residual kernel: two wavefronts per workgroup, at most two workgroups per CU
// (each holds 64 long accumulators per wavefront in LDS).
static LaunchCfg make_res_cfg(const rpcg_ctx *c, long long nslices, hipStream_t s)
{
    LaunchCfg cfg{};
    cfg.block = 128;
    cfg.grid = (int)std::max(1ll, std::min((nslices + 1) / 2, 2ll * c->num_cus));
    cfg.early_exit = true;
    cfg.fpe_size = 3;
    cfg.fallback = true;
    cfg.xcd_parts = 1;
    cfg.stream = s;
    return cfg;
}

static int ir_body(rpcg_ctx *c, int mode, const rpcg_csr *A, const double *b, double *x, const rpcg_ir_opts &io,
                   rpcg_ir_result *res, hipStream_t s)
{
    auto t_start = std::chrono::steady_clock::now();
    const int n = A->n;
    rpcg_opts o = io.inner;
    o.fpe_size = resolve_fpe_size(o.fpe_size, mode);
    const int nslices = (n + 63) / 64;
    LaunchCfg cfg_rows = make_vec_cfg(c, o, std::max(1, n), s);
    LaunchCfg cfg_sl = make_spmv_cfg(c, o, nslices, s, true);
    LaunchCfg cfg_res = make_res_cfg(c, nslices, s);
    rpcg_opts dflt;
    rpcg_opts_default(&dflt);
    dflt.fpe_size = 3;
    LaunchCfg cfg_dot = make_cfg(c, dflt, std::max(1, (n + 7) / 8), 256, s);
    int rc = ensure_ws(c, std::max(std::max(cfg_rows.grid, cfg_sl.grid), std::max(cfg_res.grid, cfg_dot.grid)));
    if (rc != RPCG_OK) return rc;
    SellBuilt B;
    rc = build_sell(c, ctx_sell_bufs(c), n, A->nnz, A->row_ptr, A->col_idx, A->val, nullptr, true, true, o.no_col16 != 0, s,
                    &B);
    if (rc != RPCG_OK) return rc;
    SellMat<float> M = sell_mat<float>(B, B.val32, n, A->row_ptr);
    const size_t nn = (size_t)std::max(1, n);
    RPCG_TRY(c->ir_vecs.ensure(nn * (sizeof(double) + 2 * sizeof(float))));
    double *r = (double *)c->ir_vecs.p;
    float *rf = (float *)(r + nn);
    float *cv = rf + nn;
    const int stride = c->ws_groups;
    IrState *ist = c->ist;
    RPCG_TRY(hipMemsetAsync(ist, 0, sizeof(IrState), s));
    RPCG_TRY(hipMemsetAsync(c->info, 0, sizeof(DotInfo), s));
    RPCG_TRY(launch_exdot(MODE_EXBLAS, n, b, b, &ist->bb, c->ws[0], stride, c->info, cfg_dot));
    RPCG_TRY(hipStreamSynchronize(s));
    const double setup_ms = ms_since(t_start);
    const bool timing = o.timing != 0;
    if (timing) {
        rc = ensure_events(c->ir_events, 2 * ((size_t)io.maxit + 1));
        if (rc) return rc;
    }
    int status = RPCG_OK, outer = 0, inner_its = 0, last_inner = RPCG_OK;
    bool inexact = false;
    long long escapes = 0;
    double inner_ms = 0, outer_ms = 0, kres_ms = 0, kms[3] = {0, 0, 0};
    int klaunch = 0;
    double rr0 = 0;
    IrState *H = c->host_ir;
    for (int k = 0;; ++k) {
        auto to = std::chrono::steady_clock::now();
        hipEvent_t *ev = timing ? &c->ir_events[2 * (size_t)k] : nullptr;
        if (ev) RPCG_TRY(hipEventRecord(ev[0], s));
        RPCG_TRY(launch_ir_residual(M, b, x, r, ist, c->ws[0], stride, cfg_res));
        if (ev) RPCG_TRY(hipEventRecord(ev[1], s));
        RPCG_TRY(launch_ir_prepare(k, io.maxit, io.tol, n, r, rf, cv, io.rr_history, ist, c->ws[0], cfg_res.grid,
                                   stride, cfg_rows));
        RPCG_TRY(hipMemcpyAsync(H, ist, sizeof(IrState), hipMemcpyDeviceToHost, s));
        RPCG_TRY(hipStreamSynchronize(s));
        outer_ms += ms_since(to);
        if (ev) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) kres_ms += ms;
        }
        if (k == 0) rr0 = H->rr;
        if (H->flags & FLAG_INEXACT) inexact = true;
        if (H->stop) { status = H->status; break; }
        auto ti = std::chrono::steady_clock::now();
        // inner tolerance of this step (rr > thr >= 0 here): the reduction the
        // outer residual still needs, with a factor 4 of margin, unless
        // inner.tol asks for more
        rpcg_opts ok = o;
        if (io.adaptive_inner) ok.tol = std::max(o.tol, 0.25 * std::sqrt(H->thr / H->rr));
        PcgRun run;
        rc = run_pcg<float>(c, mode, M, rf, cv, ok, cfg_rows, cfg_sl, s, &run);
        if (rc != RPCG_OK) return rc;
        inner_ms += ms_since(ti);
        inner_its += run.S.iter;
        escapes += run.S.escapes;
        last_inner = run.status;
        for (int j = 0; j < 3; ++j) kms[j] += run.k_ms[j];
        klaunch += run.k_launches;
        if (run.status < 0) { status = run.status; break; }
        if (run.status == RPCG_WARN_FPE_INEXACT) inexact = true;
        auto tu = std::chrono::steady_clock::now();
        RPCG_TRY(launch_ir_update(n, x, cv, ist, cfg_rows));
        RPCG_TRY(hipStreamSynchronize(s));
        outer_ms += ms_since(tu);
        ++outer;
    }
    if (status == RPCG_OK && inexact) status = RPCG_WARN_FPE_INEXACT;
    if (res) {
        res->status = status;
        res->outer = outer;
        res->inner_iterations = inner_its;
        res->last_inner_status = last_inner;
        res->rr0 = rr0;
        res->rr_final = H->rr;
        res->threshold = H->thr;
        res->fpe_escapes = escapes;
        res->setup_ms = setup_ms;
        res->total_ms = ms_since(t_start);
        res->inner_ms = inner_ms;
        res->outer_ms = outer_ms;
        if (timing) {
            res->k_residual_ms = kres_ms;
            res->k_spmv_dot_ms = kms[0];
            res->k_update_ms = kms[1];
            res->k_direction_ms = kms[2];
            res->k_launches = klaunch;
        }
    }
    return status;
}

int rpcg_ir_solve(rpcg_ctx *c, rpcg_mode mode, const rpcg_csr *A, const double *b, double *x,
                  const rpcg_ir_opts *opts, rpcg_ir_result *res, void *stream)
{
    if (res) std::memset(res, 0, sizeof(*res));
    if (!c || !valid_csr(A) || (A->n > 0 && (!b || !x))) return RPCG_ERR_INVALID;
    if ((int)mode != MODE_PLAIN && (int)mode != MODE_FPE && (int)mode != MODE_EXBLAS) return RPCG_ERR_INVALID;
    rpcg_ir_opts io;
    rpcg_ir_opts_default(&io);
    if (opts) io = *opts;
    if (!(io.tol >= 0.0) || io.maxit < 0 || io.inner.tau_history || !valid_opts(io.inner) ||
        (io.adaptive_inner != 0 && io.adaptive_inner != 1))
        return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(c->device));
    int rc = ir_body(c, (int)mode, A, b, x, io, res, (hipStream_t)stream);
    if (res) res->status = rc;
    return rc;
}

} // extern "C"

// A matrix kept in the sliced-ELL layout for repeated products.
struct rpcg_smat {
    int device = 0;
    int num_cus = 256;
    int n = 0;
    rpcg_host::Buffer off, val, val32, col, cfirst, len, rp;
    SellBuilt B;
};

static int smat_build(rpcg_ctx *c, const rpcg_csr *A, rpcg_smat *M, hipStream_t s)
{
    const SellBufs bf{&M->off, &M->val, &M->val32, &M->col, &M->cfirst, &M->len};
    int rc = build_sell(c, bf, A->n, A->nnz, A->row_ptr, A->col_idx, A->val, nullptr, true, false, false, s, &M->B);
    if (rc != RPCG_OK) return rc;
    if (!M->B.len8) { // rows of 256 or more entries: the row lengths come from a copy of row_ptr
        RPCG_TRY(M->rp.ensure(sizeof(int) * ((size_t)A->n + 1)));
        RPCG_TRY(hipMemcpyAsync(M->rp.p, A->row_ptr, sizeof(int) * ((size_t)A->n + 1), hipMemcpyDeviceToDevice, s));
    }
    RPCG_TRY(hipStreamSynchronize(s));
    return RPCG_OK;
}

extern "C" {

int rpcg_smat_create(rpcg_ctx *c, const rpcg_csr *A, rpcg_smat **out, void *stream)
{
    if (out) *out = nullptr;
    if (!c || !out || !valid_csr(A)) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(c->device));
    rpcg_smat *M = new (std::nothrow) rpcg_smat;
    if (!M) return RPCG_ERR_OOM;
    M->device = c->device;
    M->num_cus = c->num_cus;
    M->n = A->n;
    const int rc = A->n > 0 ? smat_build(c, A, M, (hipStream_t)stream) : RPCG_OK;
    if (rc != RPCG_OK) {
        rpcg_smat_destroy(M);
        return rc;
    }
    *out = M;
    return RPCG_OK;
}

int rpcg_smat_spmv(rpcg_smat *M, const double *x, double *y, void *stream)
{
    if (!M || (M->n > 0 && (!x || !y || x == y))) return RPCG_ERR_INVALID;
    if (M->n == 0) return RPCG_OK;
    RPCG_TRY(hipSetDevice(M->device));
    const SellMat<double> A = sell_mat<double>(M->B, M->B.val64, M->n, (const int *)M->rp.p);
    // one workgroup of four wavefronts per four slices, at most two per CU
    const long long want = ((long long)M->B.nslices + 3) / 4;
    const int grid = (int)std::max(1ll, std::min(want, 2ll * M->num_cus));
    RPCG_TRY(launch_sell_spmv(A, x, y, grid, (hipStream_t)stream));
    return RPCG_OK;
}

void rpcg_smat_destroy(rpcg_smat *M)
{
    if (!M) return;
    (void)hipSetDevice(M->device); // teardown: nothing to report to
    for (rpcg_host::Buffer *b : {&M->off, &M->val, &M->val32, &M->col, &M->cfirst, &M->len, &M->rp}) b->release();
    delete M;
}

} // extern "C"
