// C-ABI of the batched solver (declared in include/rpcg.h): the concatenated
// matrix copy, the run schedule of the streaming kernels, the graph of
// captured iterations, the autotuner. Host side only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "rpcg.h"
#include "context.hpp"
#include "kernels.hpp"

using namespace rpcg;
using namespace rpcg_host;

struct rpcg_batch {
    rpcg_ctx *ctx = nullptr;
    int mode = 0;
    rpcg_opts o{};
    int nsys = 0;
    std::vector<BatchSys> sys;         // per system (slot ranges follow the schedule)
    std::vector<long long> off_host;   // concatenated slice offsets
    long long total_rows = 0, total_slices = 0;
    bool col16 = false;
    Buffer off, val, col, cfirst, len8;
    Buffer vecs;                       // b, x, r, z, d, w, dinv
    Buffer st, hist_ptrs, active;
    Buffer dsys, druns, dwg;
    Buffer ws_mem;
    DotWs ws[3];
    int ws_cap = 0;
    int nruns = 0;
    rpcg_batch_tuning tuning{};
    uint64_t signature = 0;
    hipStream_t gs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_valid = false;
    bool graph_hist = false;           // the captured graph writes tau histories
    hipEvent_t ev_in = nullptr, ev_out = nullptr, poll_ev[2] = {nullptr, nullptr}, t_ev[2] = {nullptr, nullptr};
    int *host_active = nullptr;        // pinned, two entries
    std::vector<PcgState> host_st;
    // re-partition between replays: pinned staging of the schedule (two sets,
    // so the next one is written while the previous copy may still be pending)
    PcgState *host_poll_st = nullptr;  // pinned, 2 * nsys
    char *stage[2] = {nullptr, nullptr};
    size_t stage_bytes = 0;
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    int stage_next = 0;
    int slot_cap = 0;                  // slots a schedule of this tuning may use
};

namespace {

bool valid_tuning(const rpcg_batch_tuning &t)
{
    return (t.policy == 0 || t.policy == 1) && t.tile_slices >= 1 && t.grid_size >= 1 && t.grid_size <= 65536 &&
           t.block_size >= 64 && t.block_size <= MAX_BLOCK && t.block_size % 64 == 0 && t.graph_iterations >= 1 &&
           t.graph_iterations <= 64;
}

rpcg_batch_tuning default_tuning(const rpcg_ctx *c)
{
    rpcg_batch_tuning t{};
    t.policy = 0;
    t.tile_slices = 16;
    t.grid_size = 2 * c->num_cus;
    t.block_size = 256;
    t.graph_iterations = 8;
    return t;
}

int ensure_batch_ws(rpcg_batch *B, int groups)
{
    if (groups <= B->ws_cap) return RPCG_OK;
    const size_t per = (size_t)groups * (ACC_WORDS * sizeof(long long) + 2 * sizeof(int) + MAX_FPE * sizeof(double) +
                                         sizeof(int));
    RPCG_TRY(B->ws_mem.ensure(3 * per + 256 * 4));
    char *base = (char *)B->ws_mem.p;
    for (int i = 0; i < 3; ++i) {
        char *p = base + i * per;
        B->ws[i].digits = (long long *)p;
        p += (size_t)groups * ACC_WORDS * sizeof(long long);
        B->ws[i].part = (double *)p;
        p += (size_t)groups * MAX_FPE * sizeof(double);
        B->ws[i].range = (int *)p;
        p += (size_t)groups * 2 * sizeof(int);
        B->ws[i].esc = (int *)p;
    }
    B->ws_cap = groups;
    return RPCG_OK;
}

void drop_graph(rpcg_batch *B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->graph_valid = false;
}

// Runs of the streaming kernels for the current tuning over the systems with
// active[q] != 0 (all when active is null); slots numbered system by system so
// that each system's partials are contiguous.
void compute_schedule(rpcg_batch *B, const std::vector<char> *active, std::vector<BatchRun> &runs,
                      std::vector<int> &wg_run)
{
    const rpcg_batch_tuning &t = B->tuning;
    const int G = t.grid_size;
    auto on = [&](int q) { return !active || (*active)[q]; };
    std::vector<std::vector<BatchRun>> per_wg(G);
    auto add = [&](int g, int sys, int s) {
        std::vector<BatchRun> &v = per_wg[g];
        if (!v.empty() && v.back().sys == sys && v.back().s1 == s) v.back().s1 = s + 1;
        else v.push_back(BatchRun{sys, s, s + 1, -1});
    };
    if (t.policy == 0) {
        // contiguous chunks with equal stored entries (at least one slice of work each)
        long long total = 0;
        for (int q = 0; q < B->nsys; ++q)
            if (on(q)) total += B->off_host[B->sys[q].slice0 + B->sys[q].nslices] - B->off_host[B->sys[q].slice0];
        const long long target = std::max(1ll, (total + G - 1) / G);
        int g = 0;
        long long acc = 0;
        for (int q = 0; q < B->nsys; ++q) {
            if (!on(q)) continue;
            for (int s = 0; s < B->sys[q].nslices; ++s) {
                const long long gsl = B->sys[q].slice0 + s;
                if (acc >= target && g < G - 1) { ++g; acc = 0; }
                add(g, q, s);
                acc += std::max(64ll, B->off_host[gsl + 1] - B->off_host[gsl]);
            }
        }
    } else {
        // tiles of tile_slices slices, systems interleaved, dealt round-robin
        const int T = t.tile_slices;
        long long i = 0;
        int max_tiles = 0;
        for (int q = 0; q < B->nsys; ++q) max_tiles = std::max(max_tiles, (B->sys[q].nslices + T - 1) / T);
        for (int j = 0; j < max_tiles; ++j)
            for (int q = 0; q < B->nsys; ++q) {
                const int s0 = j * T, s1 = std::min(B->sys[q].nslices, s0 + T);
                if (s0 >= s1 || !on(q)) continue;
                const int g = (int)(i++ % G);
                per_wg[g].push_back(BatchRun{q, s0, s1, -1});
            }
    }
    runs.clear();
    wg_run.assign(G + 1, 0);
    for (int g = 0; g < G; ++g) {
        wg_run[g] = (int)runs.size();
        runs.insert(runs.end(), per_wg[g].begin(), per_wg[g].end());
    }
    wg_run[G] = (int)runs.size();
    std::vector<int> order(runs.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        return runs[a].sys != runs[b].sys ? runs[a].sys < runs[b].sys : runs[a].s0 < runs[b].s0;
    });
    for (int q = 0; q < B->nsys; ++q) B->sys[q].slot0 = B->sys[q].slot1 = 0; // no runs: empty slot range
    for (size_t k = 0; k < order.size(); ++k) {
        BatchRun &r = runs[order[k]];
        r.slot = (int)k;
        BatchSys &S = B->sys[r.sys];
        if (k == 0 || runs[order[k - 1]].sys != r.sys) S.slot0 = (int)k;
        S.slot1 = (int)k + 1;
    }
}

size_t schedule_bytes(const rpcg_batch *B, size_t nruns)
{
    return sizeof(BatchSys) * B->nsys + sizeof(BatchRun) * std::max<size_t>(1, nruns) +
           sizeof(int) * (B->tuning.grid_size + 1);
}

// Copy a schedule into the device arrays. With `async` the copies go through
// pinned staging and are only enqueued (used between replays).
int upload_schedule(rpcg_batch *B, const std::vector<BatchRun> &runs, const std::vector<int> &wg_run, bool async)
{
    const int G = B->tuning.grid_size;
    if (!async) {
        RPCG_TRY(hipMemcpyAsync(B->dsys.p, B->sys.data(), sizeof(BatchSys) * B->nsys, hipMemcpyHostToDevice, B->gs));
        if (!runs.empty())
            RPCG_TRY(hipMemcpyAsync(B->druns.p, runs.data(), sizeof(BatchRun) * runs.size(), hipMemcpyHostToDevice,
                                    B->gs));
        RPCG_TRY(hipMemcpyAsync(B->dwg.p, wg_run.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice, B->gs));
        RPCG_TRY(hipStreamSynchronize(B->gs)); // the host vectors are staged before they go out of scope
        return RPCG_OK;
    }
    const int k = B->stage_next;
    B->stage_next ^= 1;
    RPCG_TRY(hipEventSynchronize(B->stage_ev[k])); // the copy that last read this staging set is done
    char *p = B->stage[k];
    const size_t a = sizeof(BatchSys) * B->nsys, r = sizeof(BatchRun) * runs.size(), w = sizeof(int) * (G + 1);
    std::memcpy(p, B->sys.data(), a);
    if (r) std::memcpy(p + a, runs.data(), r);
    std::memcpy(p + a + r, wg_run.data(), w);
    RPCG_TRY(hipMemcpyAsync(B->dsys.p, p, a, hipMemcpyHostToDevice, B->gs));
    if (r) RPCG_TRY(hipMemcpyAsync(B->druns.p, p + a, r, hipMemcpyHostToDevice, B->gs));
    RPCG_TRY(hipMemcpyAsync(B->dwg.p, p + a + r, w, hipMemcpyHostToDevice, B->gs));
    RPCG_TRY(hipEventRecord(B->stage_ev[k], B->gs));
    return RPCG_OK;
}

// Schedule of every system for the current tuning; sizes the slot workspace
// and the staging for any later re-partition over fewer systems.
int build_schedule(rpcg_batch *B)
{
    std::vector<BatchRun> runs;
    std::vector<int> wg_run;
    compute_schedule(B, nullptr, runs, wg_run);
    B->nruns = (int)runs.size();
    // a re-partition over a subset never has more runs: policy 0 makes at most
    // grid + nsys runs, policy 1 a subset of the tiles
    B->slot_cap = std::max(1, B->tuning.policy == 0 ? std::max(B->nruns, B->tuning.grid_size + B->nsys) : B->nruns);
    int rc = ensure_batch_ws(B, B->slot_cap);
    if (rc != RPCG_OK) return rc;
    const size_t maxruns = (size_t)B->slot_cap;
    RPCG_TRY(B->dsys.ensure(sizeof(BatchSys) * B->nsys));
    RPCG_TRY(B->druns.ensure(sizeof(BatchRun) * maxruns));
    RPCG_TRY(B->dwg.ensure(sizeof(int) * (B->tuning.grid_size + 1)));
    const size_t need = schedule_bytes(B, maxruns);
    if (need > B->stage_bytes) {
        RPCG_TRY(hipStreamSynchronize(B->gs));
        for (char *&p : B->stage) {
            if (p) (void)hipHostFree(p);
            p = nullptr;
        }
        B->stage_bytes = 0;
        for (char *&p : B->stage) RPCG_TRY(hipHostMalloc((void **)&p, need, hipHostMallocDefault));
        B->stage_bytes = need;
    }
    rc = upload_schedule(B, runs, wg_run, false);
    if (rc != RPCG_OK) return rc;
    drop_graph(B);
    return RPCG_OK;
}

BatchArgs batch_args(const rpcg_batch *B, bool with_hist)
{
    BatchArgs a;
    a.nsys = B->nsys;
    a.sys = (const BatchSys *)B->dsys.p;
    a.runs = (const BatchRun *)B->druns.p;
    a.wg_run = (const int *)B->dwg.p;
    a.off = (const long long *)B->off.p;
    a.val = (const double *)B->val.p;
    a.col = B->col16 ? nullptr : (const int *)B->col.p;
    a.col16 = B->col16 ? (const unsigned short *)B->col.p : nullptr;
    a.cfirst = B->col16 ? (const int *)B->cfirst.p : nullptr;
    a.len8 = B->len8.p ? (const unsigned char *)B->len8.p : nullptr;
    double *v = (double *)B->vecs.p;
    const size_t T = (size_t)B->total_rows;
    a.b = v;
    a.x = v + T;
    a.r = v + 2 * T;
    a.z = v + 3 * T;
    a.d = v + 4 * T;
    a.w = v + 5 * T;
    a.dinv = v + 6 * T;
    a.st = (PcgState *)B->st.p;
    a.hist = with_hist ? (double *const *)B->hist_ptrs.p : nullptr;
    a.active = (int *)B->active.p;
    return a;
}

LaunchCfg batch_cfg(const rpcg_batch *B)
{
    LaunchCfg c{};
    c.grid = B->tuning.grid_size;
    c.block = B->tuning.block_size;
    c.early_exit = B->o.early_exit != 0;
    c.fpe_size = B->o.fpe_size;
    c.fallback = B->o.fpe_fallback != 0;
    c.xcd_parts = 1;
    c.stream = B->gs;
    return c;
}

// b (and x, or zeros) into the concatenated vectors, then the setup kernels.
int batch_start(rpcg_batch *B, const double *const *b, double *const *x, bool with_hist)
{
    double *v = (double *)B->vecs.p;
    const size_t T = (size_t)B->total_rows;
    for (int q = 0; q < B->nsys; ++q) {
        const BatchSys &S = B->sys[q];
        if (S.n == 0) continue;
        RPCG_TRY(hipMemcpyAsync(v + S.row0, b[q], sizeof(double) * S.n, hipMemcpyDeviceToDevice, B->gs));
        if (x) RPCG_TRY(hipMemcpyAsync(v + T + S.row0, x[q], sizeof(double) * S.n, hipMemcpyDeviceToDevice, B->gs));
    }
    if (!x) RPCG_TRY(hipMemsetAsync(v + T, 0, sizeof(double) * T, B->gs));
    const BatchArgs a = batch_args(B, with_hist);
    RPCG_TRY(launch_batch_setup(B->mode, B->col16, a, B->tuning.grid_size, B->tuning.block_size, B->ws, B->ws_cap,
                                B->o.tol, B->o.maxit, batch_cfg(B)));
    return RPCG_OK;
}

int capture_graph(rpcg_batch *B, bool with_hist)
{
    if (B->graph_valid) return RPCG_OK;
    drop_graph(B);
    const BatchArgs a = batch_args(B, with_hist);
    const LaunchCfg cfg = batch_cfg(B);
    RPCG_TRY(hipStreamBeginCapture(B->gs, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int i = 0; i < B->tuning.graph_iterations && err == hipSuccess; ++i)
        err = launch_batch_iteration(B->mode, B->col16, a, B->tuning.grid_size, B->tuning.block_size, B->ws,
                                     B->ws_cap, cfg);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(B->gs, &g);
    if (err != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hip_status(err); }
    RPCG_TRY(e2);
    B->graph = g;
    RPCG_TRY(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->graph_valid = true;
    return RPCG_OK;
}

uint64_t batch_signature(int mode, const rpcg_opts &o, int nsys, const rpcg_csr *A)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    mix((uint64_t)mode);
    mix((uint64_t)o.fpe_size);
    mix((uint64_t)nsys);
    for (int q = 0; q < nsys; ++q) {
        mix((uint64_t)A[q].n);
        mix((uint64_t)A[q].nnz);
    }
    return h;
}

} // namespace

extern "C" {

void rpcg_batch_destroy(rpcg_batch *B)
{
    if (!B) return;
    (void)hipSetDevice(B->ctx->device); // teardown reports nothing
    if (B->gs) (void)hipStreamSynchronize(B->gs);
    drop_graph(B);
    for (Buffer *b : {&B->off, &B->val, &B->col, &B->cfirst, &B->len8, &B->vecs, &B->st, &B->hist_ptrs, &B->active,
                      &B->dsys, &B->druns, &B->dwg, &B->ws_mem})
        b->release();
    for (hipEvent_t e : {B->ev_in, B->ev_out, B->poll_ev[0], B->poll_ev[1], B->t_ev[0], B->t_ev[1], B->stage_ev[0],
                         B->stage_ev[1]})
        if (e) (void)hipEventDestroy(e);
    if (B->host_active) (void)hipHostFree(B->host_active);
    if (B->host_poll_st) (void)hipHostFree(B->host_poll_st);
    for (char *p : B->stage)
        if (p) (void)hipHostFree(p);
    if (B->gs) (void)hipStreamDestroy(B->gs);
    delete B;
}

static int batch_create_body(rpcg_batch *B, const rpcg_csr *A, hipStream_t caller)
{
    rpcg_ctx *c = B->ctx;
    RPCG_TRY(hipStreamCreateWithFlags(&B->gs, hipStreamNonBlocking));
    for (hipEvent_t *e : {&B->ev_in, &B->ev_out, &B->poll_ev[0], &B->poll_ev[1]})
        RPCG_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    RPCG_TRY(hipEventCreate(&B->t_ev[0]));
    RPCG_TRY(hipEventCreate(&B->t_ev[1]));
    RPCG_TRY(hipHostMalloc((void **)&B->host_active, 2 * sizeof(int), hipHostMallocDefault));
    RPCG_TRY(hipHostMalloc((void **)&B->host_poll_st, 2 * sizeof(PcgState) * B->nsys, hipHostMallocDefault));
    RPCG_TRY(hipEventCreateWithFlags(&B->stage_ev[0], hipEventDisableTiming));
    RPCG_TRY(hipEventCreateWithFlags(&B->stage_ev[1], hipEventDisableTiming));
    // layout: each system's rows start at a multiple of 64, its slices after the previous system's
    B->sys.resize(B->nsys);
    long long row0 = 0, slice0 = 0;
    for (int q = 0; q < B->nsys; ++q) {
        BatchSys &S = B->sys[q];
        S.row0 = row0;
        S.slice0 = slice0;
        S.n = A[q].n;
        S.nslices = (A[q].n + 63) / 64;
        S.slot0 = S.slot1 = 0;
        S.row_ptr = A[q].row_ptr;
        row0 += 64ll * S.nslices;
        slice0 += S.nslices;
    }
    B->total_rows = std::max(64ll, row0);
    B->total_slices = slice0;
    // the caller's matrices may have been written on its stream
    RPCG_TRY(hipEventRecord(B->ev_in, caller));
    RPCG_TRY(hipStreamWaitEvent(B->gs, B->ev_in, 0));
    RPCG_TRY(B->off.ensure(sizeof(long long) * (B->total_slices + 1)));
    long long *off = (long long *)B->off.p;
    RPCG_TRY(hipMemsetAsync(off, 0, sizeof(long long) * (B->total_slices + 1), B->gs));
    RPCG_TRY(hipMemsetAsync(c->info, 0, sizeof(DotInfo), B->gs));
    const int vec = sell_vec<double>();
    for (int q = 0; q < B->nsys; ++q)
        RPCG_TRY(launch_csr_scan(A[q].n, A[q].nnz, A[q].row_ptr, A[q].col_idx, vec, off + B->sys[q].slice0 + 1,
                                 &c->info->flags, &c->info->max_len, &c->info->max_delta, B->gs));
    if (B->total_slices > 0) RPCG_TRY(launch_sell_scan(off, (int)B->total_slices, B->gs));
    B->off_host.resize(B->total_slices + 1);
    DotInfo inf;
    RPCG_TRY(hipMemcpyAsync(B->off_host.data(), off, sizeof(long long) * (B->total_slices + 1),
                            hipMemcpyDeviceToHost, B->gs));
    RPCG_TRY(hipMemcpyAsync(&inf, c->info, sizeof inf, hipMemcpyDeviceToHost, B->gs));
    RPCG_TRY(hipStreamSynchronize(B->gs));
    if (inf.flags) return RPCG_ERR_INVALID;
    B->col16 = inf.max_delta <= 32767;
    const size_t np = (size_t)std::max(1ll, B->off_host[B->total_slices]);
    RPCG_TRY(B->val.ensure(sizeof(double) * np));
    RPCG_TRY(B->col.ensure((B->col16 ? sizeof(short) : sizeof(int)) * np));
    if (B->col16) RPCG_TRY(B->cfirst.ensure(sizeof(int) * (size_t)std::max(1ll, B->total_slices)));
    if (inf.max_len < 256) RPCG_TRY(B->len8.ensure((size_t)B->total_rows));
    for (int q = 0; q < B->nsys; ++q) {
        const BatchSys &S = B->sys[q];
        RPCG_TRY(launch_sell_fill(S.n, A[q].row_ptr, A[q].col_idx, A[q].val, nullptr, vec, off + S.slice0,
                                  (double *)B->val.p, nullptr, B->col16 ? nullptr : (int *)B->col.p,
                                  B->col16 ? (unsigned short *)B->col.p : nullptr,
                                  B->col16 ? (int *)B->cfirst.p + S.slice0 : nullptr,
                                  B->len8.p ? (unsigned char *)B->len8.p + S.row0 : nullptr, B->gs));
    }
    RPCG_TRY(B->vecs.ensure(sizeof(double) * 7 * (size_t)B->total_rows));
    RPCG_TRY(hipMemsetAsync(B->vecs.p, 0, sizeof(double) * 7 * (size_t)B->total_rows, B->gs));
    RPCG_TRY(B->st.ensure(sizeof(PcgState) * B->nsys));
    RPCG_TRY(B->hist_ptrs.ensure(sizeof(double *) * B->nsys));
    RPCG_TRY(B->active.ensure(sizeof(int)));
    B->host_st.resize(B->nsys);
    auto it = c->batch_tunings.find(B->signature);
    B->tuning = it != c->batch_tunings.end() ? it->second : default_tuning(c);
    int rc = build_schedule(B);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipStreamSynchronize(B->gs));
    return RPCG_OK;
}

int rpcg_batch_create(rpcg_ctx *c, rpcg_mode mode, int32_t nsys, const rpcg_csr *A, const rpcg_opts *opts,
                      rpcg_batch **out, void *stream)
{
    if (!out) return RPCG_ERR_INVALID;
    *out = nullptr;
    if (!c || nsys < 1 || !A) return RPCG_ERR_INVALID;
    if ((int)mode != MODE_PLAIN && (int)mode != MODE_FPE && (int)mode != MODE_EXBLAS) return RPCG_ERR_INVALID;
    for (int q = 0; q < nsys; ++q)
        if (!valid_csr(&A[q])) return RPCG_ERR_INVALID;
    rpcg_opts o;
    rpcg_opts_default(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return RPCG_ERR_INVALID;
    o.fpe_size = resolve_fpe_size(o.fpe_size, (int)mode);
    RPCG_TRY(hipSetDevice(c->device));
    rpcg_batch *B = new (std::nothrow) rpcg_batch();
    if (!B) return RPCG_ERR_OOM;
    B->ctx = c;
    B->mode = (int)mode;
    B->o = o;
    B->nsys = nsys;
    B->signature = batch_signature((int)mode, o, nsys, A);
    int rc = batch_create_body(B, A, (hipStream_t)stream);
    if (rc != RPCG_OK) { rpcg_batch_destroy(B); return rc; }
    *out = B;
    return RPCG_OK;
}

int rpcg_batch_get_tuning(const rpcg_batch *B, rpcg_batch_tuning *out)
{
    if (!B || !out) return RPCG_ERR_INVALID;
    *out = B->tuning;
    return RPCG_OK;
}

int rpcg_batch_set_tuning(rpcg_batch *B, const rpcg_batch_tuning *t)
{
    if (!B || !t || !valid_tuning(*t)) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(B->ctx->device));
    B->tuning = *t;
    return build_schedule(B);
}

int rpcg_batch_tune(rpcg_batch *B, const double *const *b, int32_t trial_iterations, rpcg_batch_tuning *chosen,
                    void *stream)
{
    if (!B || !b || trial_iterations < 1 || trial_iterations > 1000) return RPCG_ERR_INVALID;
    for (int q = 0; q < B->nsys; ++q)
        if (B->sys[q].n > 0 && !b[q]) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(B->ctx->device));
    RPCG_TRY(hipEventRecord(B->ev_in, (hipStream_t)stream));
    RPCG_TRY(hipStreamWaitEvent(B->gs, B->ev_in, 0));
    const int cu = B->ctx->num_cus;
    std::vector<rpcg_batch_tuning> cand;
    auto mk = [&](int policy, int tile, int grid, int block) {
        rpcg_batch_tuning t{};
        t.policy = policy;
        t.tile_slices = tile;
        t.grid_size = grid;
        t.block_size = block;
        t.graph_iterations = B->tuning.graph_iterations;
        cand.push_back(t);
    };
    mk(0, 16, cu, 256);
    mk(0, 16, 2 * cu, 256);
    mk(0, 16, 4 * cu, 256);
    mk(0, 16, 2 * cu, 512);
    mk(0, 16, cu, 1024);
    mk(1, 16, 2 * cu, 256);
    mk(1, 64, 2 * cu, 256);
    mk(1, 256, cu, 512);
    const rpcg_batch_tuning keep = B->tuning;
    // two rounds over the candidates, each keeping its faster trial: one
    // short trial per candidate left the choice to run-to-run noise
    for (auto &t : cand) t.ms_per_iteration = 1e300;
    for (int round = 0; round < 2; ++round) {
        for (size_t k = 0; k < cand.size(); ++k) {
            rpcg_batch_tuning t = cand[k];
            B->tuning = t;
            int rc = build_schedule(B);
            if (rc != RPCG_OK) { B->tuning = keep; build_schedule(B); return rc; }
            const BatchArgs a = batch_args(B, false);
            const LaunchCfg cfg = batch_cfg(B);
            const bool warm = round == 0 && k == 0; // the first trial also warms up
            for (int rep = 0; rep < (warm ? 2 : 1); ++rep) {
                rc = batch_start(B, b, nullptr, false);
                if (rc != RPCG_OK) return rc;
                RPCG_TRY(hipEventRecord(B->t_ev[0], B->gs));
                for (int i = 0; i < trial_iterations; ++i)
                    RPCG_TRY(launch_batch_iteration(B->mode, B->col16, a, cfg.grid, cfg.block, B->ws, B->ws_cap, cfg));
                RPCG_TRY(hipEventRecord(B->t_ev[1], B->gs));
                RPCG_TRY(hipEventSynchronize(B->t_ev[1]));
            }
            float ms = 0.f;
            RPCG_TRY(hipEventElapsedTime(&ms, B->t_ev[0], B->t_ev[1]));
            cand[k].ms_per_iteration = std::min(cand[k].ms_per_iteration, (double)ms / trial_iterations);
        }
    }
    int besti = 0;
    for (size_t k = 1; k < cand.size(); ++k)
        if (cand[k].ms_per_iteration < cand[besti].ms_per_iteration) besti = (int)k;
    // the trials run with every system active; later iterations carry fewer
    // systems, where fewer workgroups (fewer slots to merge, less idle
    // launch width) do better: within 1% of the fastest trial, take the
    // candidate with the fewest workgroups
    const double lim = cand[besti].ms_per_iteration * 1.01;
    for (size_t k = 0; k < cand.size(); ++k)
        if (cand[k].ms_per_iteration <= lim && cand[k].grid_size < cand[besti].grid_size) besti = (int)k;
    B->tuning = cand[besti];
    int rc = build_schedule(B);
    if (rc != RPCG_OK) return rc;
    B->ctx->batch_tunings[B->signature] = B->tuning;
    if (chosen) *chosen = B->tuning;
    RPCG_TRY(hipEventRecord(B->ev_out, B->gs));
    RPCG_TRY(hipStreamWaitEvent((hipStream_t)stream, B->ev_out, 0));
    return RPCG_OK;
}

int rpcg_batch_solve(rpcg_batch *B, const double *const *b, double *const *x, double *const *tau_history,
                     rpcg_result *res, rpcg_batch_stats *stats, void *stream)
{
    if (res && B) std::memset(res, 0, sizeof(rpcg_result) * B->nsys);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!B || !b || !x) return RPCG_ERR_INVALID;
    for (int q = 0; q < B->nsys; ++q)
        if (B->sys[q].n > 0 && (!b[q] || !x[q])) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(B->ctx->device));
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t caller = (hipStream_t)stream;
    RPCG_TRY(hipEventRecord(B->ev_in, caller));
    RPCG_TRY(hipStreamWaitEvent(B->gs, B->ev_in, 0));
    const bool with_hist = tau_history != nullptr;
    if (with_hist)
        RPCG_TRY(hipMemcpyAsync(B->hist_ptrs.p, tau_history, sizeof(double *) * B->nsys, hipMemcpyHostToDevice, B->gs));
    int rc = batch_start(B, b, x, with_hist);
    if (rc != RPCG_OK) return rc;
    volatile int *ha = B->host_active;
    RPCG_TRY(hipMemcpyAsync((void *)&ha[0], B->active.p, sizeof(int), hipMemcpyDeviceToHost, B->gs));
    RPCG_TRY(hipStreamSynchronize(B->gs));
    const double setup_ms = ms_since(t0);
    // the graph reaches the histories through B->hist_ptrs; recapture only if their use changed
    if (B->graph_valid && B->graph_hist != with_hist) drop_graph(B);
    B->graph_hist = with_hist;
    rc = capture_graph(B, with_hist);
    if (rc != RPCG_OK) return rc;
    auto t1 = std::chrono::steady_clock::now();
    int launches = 0, repartitions = 0;
    if (ha[0] > 0) {
        const int G = B->tuning.graph_iterations;
        const int max_launch = (B->o.maxit + G - 1) / G;
        const int nsys = B->nsys;
        int scheduled = nsys; // systems the current schedule covers
        std::vector<char> live(nsys);
        std::vector<BatchRun> runs;
        std::vector<int> wg_run;
        for (int k = 0; k < max_launch; ++k) {
            RPCG_TRY(hipGraphLaunch(B->exec, B->gs));
            ++launches;
            RPCG_TRY(hipMemcpyAsync((void *)&ha[k & 1], B->active.p, sizeof(int), hipMemcpyDeviceToHost, B->gs));
            RPCG_TRY(hipMemcpyAsync(B->host_poll_st + (size_t)(k & 1) * nsys, B->st.p, sizeof(PcgState) * nsys,
                                    hipMemcpyDeviceToHost, B->gs));
            RPCG_TRY(hipEventRecord(B->poll_ev[k & 1], B->gs));
            if (k > 0) {
                const int pk = (k - 1) & 1;
                RPCG_TRY(hipEventSynchronize(B->poll_ev[pk]));
                const int left = ha[pk];
                if (left == 0) break;
                // fewer systems left: spread the next replays' work over them
                // (results do not depend on the schedule)
                if (left < scheduled && k + 1 < max_launch) {
                    const PcgState *ps = B->host_poll_st + (size_t)pk * nsys;
                    for (int q = 0; q < nsys; ++q) live[q] = ps[q].done == 0;
                    compute_schedule(B, &live, runs, wg_run);
                    if ((int)runs.size() <= B->slot_cap) {
                        rc = upload_schedule(B, runs, wg_run, true);
                        if (rc != RPCG_OK) return rc;
                        scheduled = left;
                        ++repartitions;
                    }
                }
            }
        }
    }
    RPCG_TRY(hipStreamSynchronize(B->gs));
    const double loop_ms = ms_since(t1);
    if (repartitions) {
        std::vector<BatchRun> runs;
        std::vector<int> wg_run;
        compute_schedule(B, nullptr, runs, wg_run);
        rc = upload_schedule(B, runs, wg_run, false);
        if (rc != RPCG_OK) return rc;
    }
    const double *v = (const double *)B->vecs.p;
    const size_t T = (size_t)B->total_rows;
    for (int q = 0; q < B->nsys; ++q) {
        const BatchSys &S = B->sys[q];
        if (S.n == 0) continue;
        RPCG_TRY(hipMemcpyAsync(x[q], v + T + S.row0, sizeof(double) * S.n, hipMemcpyDeviceToDevice, B->gs));
    }
    RPCG_TRY(hipMemcpyAsync(B->host_st.data(), B->st.p, sizeof(PcgState) * B->nsys, hipMemcpyDeviceToHost, B->gs));
    RPCG_TRY(hipStreamSynchronize(B->gs));
    int worst_err = 0, worst_warn = RPCG_OK;
    long long total_it = 0;
    int max_it = 0;
    for (int q = 0; q < B->nsys; ++q) {
        const PcgState &S = B->host_st[q];
        int status;
        if (S.status < 0) status = S.status;
        else if (!(S.tau <= S.thr)) status = RPCG_WARN_MAXIT;
        else if ((S.flags & FLAG_INEXACT) || (B->mode == MODE_FPE && S.escapes > 0 && !B->o.fpe_fallback))
            status = RPCG_WARN_FPE_INEXACT;
        else status = RPCG_OK;
        if (status < 0) worst_err = std::min(worst_err, status);
        else worst_warn = std::max(worst_warn, status);
        total_it += S.iter;
        max_it = std::max(max_it, S.iter);
        if (res) {
            rpcg_result &r = res[q];
            r.status = status;
            r.iterations = S.iter;
            r.tau0 = S.tau0;
            r.tau_final = S.tau;
            r.threshold = S.thr;
            r.fpe_escapes = S.escapes;
            r.fallbacks = S.fallbacks;
            r.setup_ms = setup_ms;
            r.loop_ms = loop_ms;
            r.grid_size = B->tuning.grid_size;
            r.block_size = B->tuning.block_size;
        }
    }
    const int worst = worst_err < 0 ? worst_err : worst_warn;
    RPCG_TRY(hipEventRecord(B->ev_out, B->gs));
    RPCG_TRY(hipStreamWaitEvent(caller, B->ev_out, 0));
    if (stats) {
        stats->status = worst;
        stats->graph_launches = launches;
        stats->repartitions = repartitions;
        stats->max_iterations = max_it;
        stats->total_iterations = total_it;
        stats->setup_ms = setup_ms;
        stats->loop_ms = loop_ms;
        stats->total_ms = ms_since(t0);
    }
    return worst;
}

} // extern "C"
