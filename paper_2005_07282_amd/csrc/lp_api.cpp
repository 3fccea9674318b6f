// C-ABI of the learned preconditioner (declared in include/rpcg.h): the
// network object, its forward and backward passes, the factor G, the
// training step. Host side only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "rpcg.h"
#include "context.hpp"
#include "kernels.hpp"
#include "lp_factor.hpp"

using namespace rpcg;
using namespace rpcg_host;

static_assert(RPCG_LP_NPARAMS == LP_NPARAMS, "parameter count");

struct rpcg_lpnet {
    rpcg_ctx *ctx = nullptr;
    int N = 0, max_batch = 0;
    long long n = 0;        // N^3
    int gnnz = 0;           // entries of G (and G^T)
    int *bad = nullptr;     // pinned host flag: the generation of the last forward pass that met a bad diagonal
    int gen = 0;            // forward-pass generation
    int step = 0;           // Adam steps taken
    static constexpr int DW_GRID = 1024; // slots of the weight-gradient sums (fixed: fixed order)
    Buffer params, grad, am, av, w1, w2, w3, w2t, w3t;
    Buffer feat, s, h1, h2, o, dob, d2, d1, pw, pb;
    Buffer g_rp, g_col, gt_rp, gt_col, g_val, gt_val, scal;
    // loss over (instance, probe) pairs: v, y, r, q per pair, the exact-dot
    // slots and results, and the matrix / probe pointer table
    Buffer lvec, lws, dots, tab;
    int lws_slots = 0;
    DotWs wu{}, wr{};
    std::vector<unsigned char> tab_host;
};

namespace {

// Structure of G (rows: -z, -y, -x, diagonal) and G^T (rows: diagonal, +x, +y, +z).
void lp_pattern_host(int N, int32_t *grp, int32_t *gcol, int32_t *gtrp, int32_t *gtcol)
{
    const long long n = (long long)N * N * N, NN = (long long)N * N;
    int p = 0, q = 0;
    for (long long i = 0; i < n; ++i) {
        const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / NN);
        grp[i] = p;
        if (z > 0) gcol[p++] = (int32_t)(i - NN);
        if (y > 0) gcol[p++] = (int32_t)(i - N);
        if (x > 0) gcol[p++] = (int32_t)(i - 1);
        gcol[p++] = (int32_t)i;
        gtrp[i] = q;
        gtcol[q++] = (int32_t)i;
        if (x < N - 1) gtcol[q++] = (int32_t)(i + 1);
        if (y < N - 1) gtcol[q++] = (int32_t)(i + N);
        if (z < N - 1) gtcol[q++] = (int32_t)(i + NN);
    }
    grp[n] = p;
    gtrp[n] = q;
}

long long lp_nnz(long long N) { return 4 * N * N * N - 3 * N * N; }

int check_batch(const rpcg_lpnet *L, int nb, const rpcg_csr *A)
{
    if (nb < 1 || nb > L->max_batch || !A) return RPCG_ERR_INVALID;
    for (int k = 0; k < nb; ++k)
        if (!valid_csr(&A[k]) || A[k].n != L->n) return RPCG_ERR_INVALID;
    return RPCG_OK;
}

int lp_prep(rpcg_lpnet *L, hipStream_t s)
{
    RPCG_TRY(launch_lp_prep((const float *)L->params.p, (bf16_t *)L->w1.p, (bf16_t *)L->w2.p, (bf16_t *)L->w3.p,
                            (bf16_t *)L->w2t.p, (bf16_t *)L->w3t.p, s));
    return RPCG_OK;
}

// Forward pass of nb systems: features, three convolutions; the outputs go to
// out (device, [nb][N^3][4]) if given, else to the network's own buffer.
// Waits for completion (the diagonal check).
int lp_forward(rpcg_lpnet *L, int nb, const rpcg_csr *A, float *out, hipStream_t s)
{
    const int gen = L->gen = (L->gen % 0x3FFFFFFF) + 1;
    for (int k0 = 0; k0 < nb; k0 += LP_MAT_ARGS) {
        LpMatSet set{};
        const int m = std::min(LP_MAT_ARGS, nb - k0);
        for (int j = 0; j < m; ++j) set.m[j] = LpMat{A[k0 + j].row_ptr, A[k0 + j].col_idx, A[k0 + j].val};
        RPCG_TRY(launch_lp_features(L->N, m, set, (bf16_t *)L->feat.p + k0 * L->n * 4, (float *)L->s.p + k0 * L->n,
                                    L->bad, gen, s));
    }
    const float *p = (const float *)L->params.p;
    RPCG_TRY(launch_lp_conv(4, 16, EPI_RELU, nb, L->N, (const bf16_t *)L->feat.p, (const bf16_t *)L->w1.p,
                            p + LP_OFF_B1, nullptr, nullptr, (bf16_t *)L->h1.p, s));
    RPCG_TRY(launch_lp_conv(16, 16, EPI_RELU, nb, L->N, (const bf16_t *)L->h1.p, (const bf16_t *)L->w2.p,
                            p + LP_OFF_B2, nullptr, nullptr, (bf16_t *)L->h2.p, s));
    RPCG_TRY(launch_lp_conv(16, 4, EPI_LINEAR, nb, L->N, (const bf16_t *)L->h2.p, (const bf16_t *)L->w3.p,
                            p + LP_OFF_B3, nullptr, out ? out : (float *)L->o.p, nullptr, s));
    RPCG_TRY(hipStreamSynchronize(s));
    if (__atomic_load_n(L->bad, __ATOMIC_ACQUIRE) == gen) return RPCG_ERR_NOT_SPD;
    return RPCG_OK;
}

// G, G^T values of instance k into g_val / gt_val.
int lp_factor_one(rpcg_lpnet *L, int k, double *g_val, double *gt_val, hipStream_t s)
{
    RPCG_TRY(launch_lp_factor(L->N, 1, (const float *)L->o.p + k * L->n * 4, (const float *)L->s.p + k * L->n,
                              (const int *)L->g_rp.p, (const int *)L->gt_rp.p, g_val, gt_val, 0, s));
    return RPCG_OK;
}

// Two exact-dot workspaces of `slots` slots each.
int lp_ensure_dot_ws(rpcg_lpnet *L, int slots)
{
    if (slots <= L->lws_slots) return RPCG_OK;
    const size_t per = (size_t)slots * (ACC_WORDS * sizeof(long long) + MAX_FPE * sizeof(double) +
                                        2 * sizeof(int) + sizeof(int));
    RPCG_TRY(L->lws.ensure(2 * per));
    char *base = (char *)L->lws.p;
    for (DotWs *w : {&L->wu, &L->wr}) {
        char *b = base;
        w->digits = (long long *)b;
        b += (size_t)slots * ACC_WORDS * sizeof(long long);
        w->part = (double *)b;
        b += (size_t)slots * MAX_FPE * sizeof(double);
        w->range = (int *)b;
        b += (size_t)slots * 2 * sizeof(int);
        w->esc = (int *)b;
        base += per;
    }
    L->lws_slots = slots;
    return RPCG_OK;
}

// Loss and dL/do (bfloat16 into dob, binary64 into dout if given) over the
// cached forward pass, for the nb x nu (instance, probe) pairs at once.
int lp_loss_grad(rpcg_lpnet *L, int nb, const rpcg_csr *A, const double *const *u, int nu, double eps, double *loss,
                 double *dout, hipStream_t s)
{
    const long long n = L->n;
    const long long P = (long long)nb * nu;
    if (P > 65535) return RPCG_ERR_INVALID; // pairs index the second grid dimension
    RPCG_TRY(L->lvec.ensure(sizeof(double) * 4 * n * P));
    RPCG_TRY(L->dots.ensure(sizeof(double) * 2 * P));
    int rc = lp_ensure_dot_ws(L, (int)(P * LP_DOT_CHUNKS));
    if (rc != RPCG_OK) return rc;
    // pointer table: A, G, G^T of each instance, then the probe of each pair
    const size_t mat_bytes = sizeof(LpMat) * 3 * nb, tab_bytes = mat_bytes + sizeof(double *) * P;
    RPCG_TRY(L->tab.ensure(tab_bytes));
    L->tab_host.resize(tab_bytes);
    LpMat *hm = (LpMat *)L->tab_host.data();
    const double **hu = (const double **)(L->tab_host.data() + mat_bytes);
    double *G = (double *)L->g_val.p, *Gt = (double *)L->gt_val.p;
    const int *grp = (const int *)L->g_rp.p, *gcol = (const int *)L->g_col.p;
    const int *gtrp = (const int *)L->gt_rp.p, *gtcol = (const int *)L->gt_col.p;
    for (int k = 0; k < nb; ++k) {
        hm[k] = LpMat{A[k].row_ptr, A[k].col_idx, A[k].val};
        hm[nb + k] = LpMat{grp, gcol, G + (long long)k * L->gnnz};
        hm[2 * nb + k] = LpMat{gtrp, gtcol, Gt + (long long)k * L->gnnz};
    }
    for (long long p = 0; p < P; ++p) hu[p] = u[p];
    RPCG_TRY(hipMemcpyAsync(L->tab.p, L->tab_host.data(), tab_bytes, hipMemcpyHostToDevice, s));
    const LpMat *mA = (const LpMat *)L->tab.p, *mG = mA + nb, *mGt = mA + 2 * nb;
    const double *const *ut = (const double *const *)((const char *)L->tab.p + mat_bytes);
    // v, y, r, q: the nu vectors of an instance interleaved ([instance][cell][vector])
    double *v = (double *)L->lvec.p, *y = v + P * n, *r = y + P * n, *q = r + P * n;
    int *flags = (int *)((double *)L->scal.p + 4); // exact-dot flags of the loss (not reported)
    const double scale = 1.0 / (double)P;
    RPCG_TRY(launch_lp_factor(L->N, nb, (const float *)L->o.p, (const float *)L->s.p, grp, gtrp, G, Gt, L->gnnz, s));
    RPCG_TRY(launch_lp_mv(n, nb, nu, mA, ut, nullptr, v, s));                                      // v = A u
    RPCG_TRY(launch_lp_mv(n, nb, nu, mGt, nullptr, v, y, s));                                      // y = G^T v
    RPCG_TRY(launch_lp_resid_dots(n, nb, nu, eps, mG, ut, y, v, r, L->wu, L->wr, L->lws_slots, flags, s)); // r
    RPCG_TRY(launch_lp_dots_merge((int)P, L->wu, L->wr, L->lws_slots, (double *)L->dots.p, flags, s));
    RPCG_TRY(launch_lp_mv(n, nb, nu, mGt, nullptr, r, q, s));                                      // q = G^T r
    RPCG_TRY(launch_lp_dodg_all(L->N, nb, nu, scale, (const double *)L->dots.p, (const float *)L->o.p,
                                (const float *)L->s.p, mG, r, y, v, q, dout, (bf16_t *)L->dob.p,
                                (double *)L->scal.p + 2, s));
    if (loss) {
        RPCG_TRY(hipMemcpyAsync(loss, (double *)L->scal.p + 2, sizeof(double), hipMemcpyDeviceToHost, s));
        RPCG_TRY(hipStreamSynchronize(s));
    }
    return RPCG_OK;
}

// Parameter gradient from the output gradient (bfloat16, in dob) over the cached forward pass.
int lp_backward(rpcg_lpnet *L, int nb, hipStream_t s)
{
    const int N = L->N, G = rpcg_lpnet::DW_GRID;
    float *gr = (float *)L->grad.p, *pw = (float *)L->pw.p, *pb = (float *)L->pb.p;
    // the relu masks of layers 2 and 1 are their stored activations h2, h1
    const bf16_t *mask2 = (const bf16_t *)L->h2.p, *mask1 = (const bf16_t *)L->h1.p;
    // layer 3
    RPCG_TRY(launch_lp_conv_dw(16, 4, nb, N, (const bf16_t *)L->h2.p, (const bf16_t *)L->dob.p, pw, pb, G, s));
    RPCG_TRY(launch_lp_reduce(G, 4, 16, pw, pb, gr + LP_OFF_W3, gr + LP_OFF_B3, s));
    RPCG_TRY(launch_lp_conv(4, 16, EPI_MASK, nb, N, (const bf16_t *)L->dob.p, (const bf16_t *)L->w3t.p, nullptr, mask2,
                            nullptr, (bf16_t *)L->d2.p, s));
    // layer 2
    RPCG_TRY(launch_lp_conv_dw(16, 16, nb, N, (const bf16_t *)L->h1.p, (const bf16_t *)L->d2.p, pw, pb, G, s));
    RPCG_TRY(launch_lp_reduce(G, 16, 16, pw, pb, gr + LP_OFF_W2, gr + LP_OFF_B2, s));
    RPCG_TRY(launch_lp_conv(16, 16, EPI_MASK, nb, N, (const bf16_t *)L->d2.p, (const bf16_t *)L->w2t.p, nullptr, mask1,
                            nullptr, (bf16_t *)L->d1.p, s));
    // layer 1
    RPCG_TRY(launch_lp_conv_dw(4, 16, nb, N, (const bf16_t *)L->feat.p, (const bf16_t *)L->d1.p, pw, pb, G, s));
    RPCG_TRY(launch_lp_reduce(G, 16, 4, pw, pb, gr + LP_OFF_W1, gr + LP_OFF_B1, s));
    return RPCG_OK;
}

int lp_create_body(rpcg_lpnet *L)
{
    const long long cells = L->n * L->max_batch;
    const long long nz = lp_nnz(L->N);
    L->gnnz = (int)nz;
    for (Buffer *b : {&L->params, &L->grad, &L->am, &L->av}) RPCG_TRY(b->ensure(sizeof(float) * LP_NPARAMS));
    RPCG_TRY(L->w1.ensure(sizeof(bf16_t) * LP_TAPS * 16 * 4));
    RPCG_TRY(L->w2.ensure(sizeof(bf16_t) * LP_TAPS * 256));
    RPCG_TRY(L->w3.ensure(sizeof(bf16_t) * LP_TAPS * 256));
    RPCG_TRY(L->w2t.ensure(sizeof(bf16_t) * LP_TAPS * 256));
    RPCG_TRY(L->w3t.ensure(sizeof(bf16_t) * LP_TAPS * 16 * 4));
    RPCG_TRY(L->feat.ensure(sizeof(bf16_t) * 4 * cells));
    RPCG_TRY(L->s.ensure(sizeof(float) * cells));
    RPCG_TRY(L->h1.ensure(sizeof(bf16_t) * 16 * cells));
    RPCG_TRY(L->h2.ensure(sizeof(bf16_t) * 16 * cells));
    RPCG_TRY(L->o.ensure(sizeof(float) * 4 * cells));
    RPCG_TRY(L->dob.ensure(sizeof(bf16_t) * 4 * cells));
    RPCG_TRY(L->d2.ensure(sizeof(bf16_t) * 16 * cells));
    RPCG_TRY(L->d1.ensure(sizeof(bf16_t) * 16 * cells));
    RPCG_TRY(L->pw.ensure(sizeof(float) * rpcg_lpnet::DW_GRID * LP_TAPS * 256));
    RPCG_TRY(L->pb.ensure(sizeof(float) * rpcg_lpnet::DW_GRID * 16));
    RPCG_TRY(L->g_rp.ensure(sizeof(int) * (L->n + 1)));
    RPCG_TRY(L->gt_rp.ensure(sizeof(int) * (L->n + 1)));
    RPCG_TRY(L->g_col.ensure(sizeof(int) * nz));
    RPCG_TRY(L->gt_col.ensure(sizeof(int) * nz));
    RPCG_TRY(L->g_val.ensure(sizeof(double) * nz * L->max_batch));
    RPCG_TRY(L->gt_val.ensure(sizeof(double) * nz * L->max_batch));
    RPCG_TRY(L->scal.ensure(sizeof(double) * 8));
    std::vector<int32_t> grp(L->n + 1), gcol(nz), gtrp(L->n + 1), gtcol(nz);
    lp_pattern_host(L->N, grp.data(), gcol.data(), gtrp.data(), gtcol.data());
    RPCG_TRY(hipMemcpy(L->g_rp.p, grp.data(), sizeof(int) * (L->n + 1), hipMemcpyHostToDevice));
    RPCG_TRY(hipMemcpy(L->gt_rp.p, gtrp.data(), sizeof(int) * (L->n + 1), hipMemcpyHostToDevice));
    RPCG_TRY(hipMemcpy(L->g_col.p, gcol.data(), sizeof(int) * nz, hipMemcpyHostToDevice));
    RPCG_TRY(hipMemcpy(L->gt_col.p, gtcol.data(), sizeof(int) * nz, hipMemcpyHostToDevice));
    RPCG_TRY(hipHostMalloc((void **)&L->bad, sizeof(int), hipHostMallocDefault));
    *L->bad = 0;
    RPCG_TRY(hipMemset(L->params.p, 0, sizeof(float) * LP_NPARAMS));
    RPCG_TRY(hipMemset(L->am.p, 0, sizeof(float) * LP_NPARAMS));
    RPCG_TRY(hipMemset(L->av.p, 0, sizeof(float) * LP_NPARAMS));
    RPCG_TRY(hipDeviceSynchronize());
    return lp_prep(L, nullptr);
}

} // namespace

extern "C" {

int64_t rpcg_lp_pattern_nnz(int32_t N) { return N < 1 ? -1 : lp_nnz(N); }

int rpcg_lp_pattern(int32_t N, int32_t *g_row_ptr, int32_t *g_col, int32_t *gt_row_ptr, int32_t *gt_col)
{
    if (N < 1 || (long long)N * N * N > (1ll << 30) || !g_row_ptr || !g_col || !gt_row_ptr || !gt_col)
        return RPCG_ERR_INVALID;
    lp_pattern_host(N, g_row_ptr, g_col, gt_row_ptr, gt_col);
    return RPCG_OK;
}

void rpcg_lp_destroy(rpcg_lpnet *L)
{
    if (!L) return;
    // teardown reports nothing: release what can be released
    (void)hipSetDevice(L->ctx->device);
    (void)hipDeviceSynchronize();
    for (Buffer *b : {&L->params, &L->grad, &L->am, &L->av, &L->w1, &L->w2, &L->w3, &L->w2t, &L->w3t, &L->feat, &L->s,
                      &L->h1, &L->h2, &L->o, &L->dob, &L->d2, &L->d1, &L->pw, &L->pb,
                      &L->g_rp, &L->g_col, &L->gt_rp, &L->gt_col, &L->g_val, &L->gt_val, &L->scal, &L->lvec,
                      &L->lws, &L->dots, &L->tab})
        b->release();
    if (L->bad) (void)hipHostFree(L->bad);
    delete L;
}

int rpcg_lp_create(rpcg_ctx *c, int32_t N, int32_t max_batch, rpcg_lpnet **out)
{
    if (!out) return RPCG_ERR_INVALID;
    *out = nullptr;
    if (!c || N < 2 || max_batch < 1 || max_batch > 65535 || (long long)N * N * N * max_batch > (1ll << 30))
        return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(c->device));
    rpcg_lpnet *L = new (std::nothrow) rpcg_lpnet();
    if (!L) return RPCG_ERR_OOM;
    L->ctx = c;
    L->N = N;
    L->max_batch = max_batch;
    L->n = (long long)N * N * N;
    int rc = lp_create_body(L);
    if (rc != RPCG_OK) { rpcg_lp_destroy(L); return rc; }
    *out = L;
    return RPCG_OK;
}

int rpcg_lp_set_params(rpcg_lpnet *L, const float *params)
{
    if (!L || !params) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(L->ctx->device));
    RPCG_TRY(hipMemcpy(L->params.p, params, sizeof(float) * LP_NPARAMS, hipMemcpyHostToDevice));
    RPCG_TRY(hipMemset(L->am.p, 0, sizeof(float) * LP_NPARAMS));
    RPCG_TRY(hipMemset(L->av.p, 0, sizeof(float) * LP_NPARAMS));
    L->step = 0;
    int rc = lp_prep(L, nullptr);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipDeviceSynchronize());
    return RPCG_OK;
}

int rpcg_lp_get_params(rpcg_lpnet *L, float *params)
{
    if (!L || !params) return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(L->ctx->device));
    RPCG_TRY(hipMemcpy(params, L->params.p, sizeof(float) * LP_NPARAMS, hipMemcpyDeviceToHost));
    return RPCG_OK;
}

int rpcg_lp_forward(rpcg_lpnet *L, int32_t nb, const rpcg_csr *A, float *o, void *stream)
{
    if (!L) return RPCG_ERR_INVALID;
    int rc = check_batch(L, nb, A);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipSetDevice(L->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    return lp_forward(L, nb, A, o, s);
}

int rpcg_lp_factor(rpcg_lpnet *L, int32_t nb, const rpcg_csr *A, rpcg_csr *G, rpcg_csr *Gt, void *stream)
{
    if (!L || !G || !Gt) return RPCG_ERR_INVALID;
    int rc = check_batch(L, nb, A);
    if (rc != RPCG_OK) return rc;
    for (int k = 0; k < nb; ++k)
        if (G[k].n != L->n || Gt[k].n != L->n || G[k].nnz != L->gnnz || Gt[k].nnz != L->gnnz || !G[k].val || !Gt[k].val)
            return RPCG_ERR_INVALID;
    RPCG_TRY(hipSetDevice(L->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    rc = lp_forward(L, nb, A, nullptr, s);
    if (rc != RPCG_OK) return rc;
    for (int k = 0; k < nb; ++k) {
        rc = lp_factor_one(L, k, (double *)G[k].val, (double *)Gt[k].val, s);
        if (rc != RPCG_OK) return rc;
    }
    RPCG_TRY(hipStreamSynchronize(s));
    return RPCG_OK;
}

int rpcg_lp_loss_grad(rpcg_lpnet *L, int32_t nb, const rpcg_csr *A, const double *const *u, int32_t nu, double eps,
                      double *loss, double *dout, void *stream)
{
    if (!L || !u || nu < 1 || !(eps >= 0.0)) return RPCG_ERR_INVALID;
    int rc = check_batch(L, nb, A);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipSetDevice(L->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    rc = lp_forward(L, nb, A, nullptr, s);
    if (rc != RPCG_OK) return rc;
    rc = lp_loss_grad(L, nb, A, u, nu, eps, loss, dout, s);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipStreamSynchronize(s));
    return RPCG_OK;
}

int rpcg_lp_backward(rpcg_lpnet *L, int32_t nb, const rpcg_csr *A, const double *dout, float *grad, void *stream)
{
    if (!L || !dout || !grad) return RPCG_ERR_INVALID;
    int rc = check_batch(L, nb, A);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipSetDevice(L->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    rc = lp_forward(L, nb, A, nullptr, s);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(launch_lp_to_bf16(4 * L->n * nb, dout, (bf16_t *)L->dob.p, s));
    rc = lp_backward(L, nb, s);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipMemcpyAsync(grad, L->grad.p, sizeof(float) * LP_NPARAMS, hipMemcpyDeviceToDevice, s));
    RPCG_TRY(hipStreamSynchronize(s));
    return RPCG_OK;
}

int rpcg_lp_train_step(rpcg_lpnet *L, int32_t nb, const rpcg_csr *A, const double *const *u, int32_t nu, double eps,
                       float lr, double *loss, void *stream)
{
    if (!L || !u || nu < 1 || !(eps >= 0.0) || !(lr >= 0.f)) return RPCG_ERR_INVALID;
    int rc = check_batch(L, nb, A);
    if (rc != RPCG_OK) return rc;
    RPCG_TRY(hipSetDevice(L->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    rc = lp_forward(L, nb, A, nullptr, s);
    if (rc != RPCG_OK) return rc;
    rc = lp_loss_grad(L, nb, A, u, nu, eps, nullptr, nullptr, s);
    if (rc != RPCG_OK) return rc;
    rc = lp_backward(L, nb, s);
    if (rc != RPCG_OK) return rc;
    L->step += 1;
    RPCG_TRY(launch_lp_adam(LP_NPARAMS, (float *)L->params.p, (const float *)L->grad.p, (float *)L->am.p,
                            (float *)L->av.p, lr, 0.9f, 0.999f, 1e-8f, L->step, s));
    rc = lp_prep(L, s);
    if (rc != RPCG_OK) return rc;
    if (loss) RPCG_TRY(hipMemcpyAsync(loss, (double *)L->scal.p + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    RPCG_TRY(hipStreamSynchronize(s));
    return RPCG_OK;
}

} // extern "C"
