// Learned preconditioner: the training loss and its gradient with respect to
// the network outputs, for every (instance k, probe vector m) pair of a batch
// in a handful of launches.
//
// For pair p = k nu + m with probe u = u_p and the factor G = G_k:
//   v = A u,  y = G^T v,  r = (G y + eps v) - u,  q = G^T r,
//   loss = scale sum_p <r_p, r_p> / <u_p, u_p>,
//   dL/dG_ij = (2 scale / <u, u>) (r_i y_j + v_i q_j) summed over the m of k,
// chained onto the outputs o through G's definition. The products run over
// every instance at once: a matrix row is read once for all nu vectors of its
// instance. <u, u> and <r, r> are exact dots (long accumulator, correctly
// rounded), and every sum over m and over the pairs runs in a fixed order, so
// the loss and the gradient are bit-reproducible.
#include "lp_factor.hpp"
#include "batch_common.hpp"

namespace rpcg {

constexpr int LPL_BLOCK = 256;
constexpr int LPL_ROWCAP = 8; // rows up to this length are held in registers across the nu vectors
constexpr int LPL_MG = 8;     // vectors per pass of the generic (any nu) path
typedef double v4d __attribute__((ext_vector_type(4)));

// The loss's own vectors (v, y, r, q) are interleaved: entry i of the vector
// of pair p = k nu + m sits at X + (k n + i) nu + m, so a gathered column
// brings the nu values of its instance in one run (one 32-byte load for
// nu = 4, the training case). NU = 4 is that case; NU = 0 handles any nu
// with scalar loads. The probes u_p stay where the caller keeps them (a
// pointer per pair). Every product is still one fma chain per row and
// vector, in storage order from zero.

// x value of vector m0 + m at column c: from the caller's probe vectors
// (TAB; xt = the instance's pointers) or from the interleaved xk.
template <bool TAB>
__device__ __forceinline__ double lp_x(const double *__restrict__ xk, const double *const *__restrict__ xt,
                                       long long c, int nu, int m)
{
    if constexpr (TAB) return xt[m][c];
    else return xk[c * nu + m];
}

// One row of M_k (at most LPL_ROWCAP entries held in registers) applied to
// the nu vectors of instance k: acc[m] for m < nu (NU = 4) or for
// m0 <= m < m0 + mg (NU = 0).
template <int NU, bool TAB>
__device__ __forceinline__ void lp_row_apply(const LpMat &M, int b, int len, const double *__restrict__ xk,
                                             const double *const *__restrict__ xt, int nu, int m0, int mg,
                                             double (&acc)[NU ? NU : LPL_MG])
{
    constexpr int A = NU ? NU : LPL_MG;
    const int st = NU ? NU : nu;
#pragma unroll
    for (int m = 0; m < A; ++m) acc[m] = 0.0;
    if (len <= LPL_ROWCAP) {
        double a[LPL_ROWCAP];
        int c[LPL_ROWCAP];
#pragma unroll
        for (int j = 0; j < LPL_ROWCAP; ++j) {
            a[j] = j < len ? M.val[b + j] : 0.0;
            c[j] = j < len ? M.col[b + j] : 0;
        }
#pragma unroll
        for (int j = 0; j < LPL_ROWCAP; ++j) {
            if (j >= len) break;
            if constexpr (NU == 4 && !TAB) {
                const v4d xv = *(const v4d *)(xk + (long long)c[j] * 4);
#pragma unroll
                for (int m = 0; m < 4; ++m) acc[m] = __builtin_fma(a[j], xv[m], acc[m]);
            } else {
#pragma unroll
                for (int m = 0; m < A; ++m)
                    if (NU || m < mg) acc[m] = __builtin_fma(a[j], lp_x<TAB>(xk, xt, c[j], st, m0 + m), acc[m]);
            }
        }
    } else {
        for (int j = 0; j < len; ++j) {
            const double aj = M.val[b + j];
            const long long cj = M.col[b + j];
#pragma unroll
            for (int m = 0; m < A; ++m)
                if (NU || m < mg) acc[m] = __builtin_fma(aj, lp_x<TAB>(xk, xt, cj, st, m0 + m), acc[m]);
        }
    }
}

// Y = M_k X for the nu vectors of instance k = blockIdx.y: X from the probe
// pointers xtab (TAB) or interleaved at xbase; Y interleaved.
template <int NU, bool TAB>
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_mv(long long n, int nu, const LpMat *__restrict__ mats,
                                                     const double *const *__restrict__ xtab,
                                                     const double *__restrict__ xbase, double *__restrict__ ybase)
{
    const int k = blockIdx.y;
    const LpMat M = mats[k];
    const double *__restrict__ xk = TAB ? nullptr : xbase + (long long)k * n * nu;
    const double *const *__restrict__ xt = TAB ? xtab + (long long)k * nu : nullptr;
    double *__restrict__ yk = ybase + (long long)k * n * nu;
    for (long long i = (long long)blockIdx.x * LPL_BLOCK + threadIdx.x; i < n;
         i += (long long)gridDim.x * LPL_BLOCK) {
        const int b = M.rp[i], len = M.rp[i + 1] - b;
        for (int m0 = 0; m0 < nu; m0 += (NU ? NU : LPL_MG)) {
            const int mg = NU ? NU : min(LPL_MG, nu - m0);
            double acc[NU ? NU : LPL_MG];
            lp_row_apply<NU, TAB>(M, b, len, xk, xt, nu, m0, mg, acc);
            if constexpr (NU == 4) {
                *(v4d *)(yk + i * 4) = (v4d){acc[0], acc[1], acc[2], acc[3]};
            } else {
#pragma unroll
                for (int m = 0; m < LPL_MG; ++m)
                    if (m < mg) yk[i * nu + m0 + m] = acc[m];
            }
        }
    }
}

// R = (G_k Y + eps V) - U for instance k = blockIdx.y (U from the probe pointers).
template <int NU>
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_resid(long long n, int nu, double eps,
                                                        const LpMat *__restrict__ gm,
                                                        const double *const *__restrict__ utab,
                                                        const double *__restrict__ ybase,
                                                        const double *__restrict__ vbase, double *__restrict__ rbase)
{
    const int k = blockIdx.y;
    const LpMat G = gm[k];
    const long long o = (long long)k * n * nu;
    for (long long i = (long long)blockIdx.x * LPL_BLOCK + threadIdx.x; i < n;
         i += (long long)gridDim.x * LPL_BLOCK) {
        const int b = G.rp[i], len = G.rp[i + 1] - b;
        for (int m0 = 0; m0 < nu; m0 += (NU ? NU : LPL_MG)) {
            const int mg = NU ? NU : min(LPL_MG, nu - m0);
            double w[NU ? NU : LPL_MG];
            lp_row_apply<NU, false>(G, b, len, ybase + o, nullptr, nu, m0, mg, w);
            if constexpr (NU == 4) {
                const v4d vv = *(const v4d *)(vbase + o + i * 4);
                v4d rr;
#pragma unroll
                for (int m = 0; m < 4; ++m) rr[m] = (w[m] + eps * vv[m]) - utab[k * 4 + m][i];
                *(v4d *)(rbase + o + i * 4) = rr;
            } else {
#pragma unroll
                for (int m = 0; m < LPL_MG; ++m)
                    if (m < mg) {
                        const long long e = o + i * nu + m0 + m;
                        rbase[e] = (w[m] + eps * vbase[e]) - utab[(long long)k * nu + m0 + m][i];
                    }
            }
        }
    }
}

// The exact-dot partials of <u_p, u_p> and <r_p, r_p> into slots p chunks +
// blockIdx.x (grid: chunks x pairs); r_p read from the interleaved R.
template <int P>
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_dots(long long n, int nu, const double *const *__restrict__ utab,
                                                       const double *__restrict__ rbase, SlotView su, SlotView sr,
                                                       int *flags)
{
    __shared__ RedShared sh;
    const int p = blockIdx.y, k = p / nu, m = p % nu;
    const double *__restrict__ u = utab[p];
    const double *__restrict__ r = rbase + (long long)k * n * nu + m;
    zero_acc(sh.acc[0]);
    zero_acc(sh.acc[1]);
    __syncthreads();
    LaneDot<MODE_EXBLAS, P> Lu, Lr;
    Lu.init();
    Lr.init();
    for (long long i = (long long)blockIdx.x * LPL_BLOCK + threadIdx.x; i < n;
         i += (long long)gridDim.x * LPL_BLOCK) {
        const double ui = u[i], ri = r[i * nu];
        Lu.add(ui, ui, sh.acc[0], true, true);
        Lr.add(ri, ri, sh.acc[1], true, true);
    }
    block_finish_pair<MODE_EXBLAS, P>(Lu, sh.acc[0], su, Lr, sh.acc[1], sr, p * gridDim.x + blockIdx.x, true, true,
                                      flags, sh);
}

// dots[2p] = <u_p, u_p>, dots[2p + 1] = <r_p, r_p> from the slots of pair p
// (one workgroup per pair).
template <int P>
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_dots_merge(int chunks, SlotView su, SlotView sr, double *dots,
                                                             int *flags)
{
    __shared__ RedShared sh;
    const int p = blockIdx.x;
    long long esc;
    const double uu = merge_slots<MODE_EXBLAS, P>(batch_slots<MODE_EXBLAS>(su, p * chunks), chunks, true, true,
                                                  sh.acc[0], &esc, flags, sh, 0);
    const double rr = merge_slots<MODE_EXBLAS, P>(batch_slots<MODE_EXBLAS>(sr, p * chunks), chunks, true, true,
                                                  sh.acc[1], &esc, flags, sh, 1);
    if (threadIdx.x == 0) {
        dots[2 * p] = uu;
        dots[2 * p + 1] = rr;
    }
}

// dL/do of instance k = blockIdx.y (summed over its nu pairs in order m = 0,
// 1, ...), rounded to bfloat16 into dob and, if do64 is given, written in
// binary64 there; the loss (pairs in order) by one thread. R, Y, V, Q are
// interleaved.
template <int NU>
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_dodg(int N, int nu_rt, int npairs, double scale,
                                                       const double *__restrict__ dots, const float *__restrict__ o,
                                                       const float *__restrict__ s, const LpMat *__restrict__ gm,
                                                       const double *__restrict__ rbase,
                                                       const double *__restrict__ ybase,
                                                       const double *__restrict__ vbase,
                                                       const double *__restrict__ qbase, double *__restrict__ do64,
                                                       bf16_t *__restrict__ dob, double *loss)
{
    const int nu = NU ? NU : nu_rt;
    const long long n = (long long)N * N * N, NN = (long long)N * N;
    const int k = blockIdx.y;
    if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        double L = 0.0;
        for (int p = 0; p < npairs; ++p) L += scale * dots[2 * p + 1] / dots[2 * p];
        loss[0] = L;
    }
    const LpMat G = gm[k];
    o += (long long)k * n * 4;
    s += (long long)k * n;
    if (do64) do64 += (long long)k * n * 4;
    dob += (long long)k * n * 4;
    const long long off = (long long)k * n * nu;
    const double *__restrict__ R = rbase + off, *__restrict__ Y = ybase + off;
    const double *__restrict__ V = vbase + off, *__restrict__ Q = qbase + off;
    for (long long i = (long long)blockIdx.x * LPL_BLOCK + threadIdx.x; i < n;
         i += (long long)gridDim.x * LPL_BLOCK) {
        const int x = (int)(i % N), yy = (int)((i / N) % N), z = (int)(i / NN);
        const double si = s[i];
        const double gdiag = G.val[G.rp[i + 1] - 1];
        const long long nbr[3] = {x > 0 ? i - 1 : -1, yy > 0 ? i - N : -1, z > 0 ? i - NN : -1};
        double g[4] = {0.0, 0.0, 0.0, 0.0};
        if constexpr (NU == 4) {
            const v4d r4 = *(const v4d *)(R + i * 4), v4 = *(const v4d *)(V + i * 4);
            const v4d y4 = *(const v4d *)(Y + i * 4), q4 = *(const v4d *)(Q + i * 4);
            v4d yn[3], qn[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const long long j = nbr[d] >= 0 ? nbr[d] : i;
                yn[d] = *(const v4d *)(Y + j * 4);
                qn[d] = *(const v4d *)(Q + j * 4);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double c = scale * 2.0 / dots[2 * ((long long)k * 4 + m)];
                g[0] += c * (r4[m] * y4[m] + v4[m] * q4[m]) * gdiag;
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    if (nbr[d] >= 0) g[1 + d] += c * (r4[m] * yn[d][m] + v4[m] * qn[d][m]) * si;
            }
        } else {
            for (int m = 0; m < nu; ++m) {
                const double c = scale * 2.0 / dots[2 * ((long long)k * nu + m)];
                const double ri = R[i * nu + m], vi = V[i * nu + m];
                g[0] += c * (ri * Y[i * nu + m] + vi * Q[i * nu + m]) * gdiag;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const long long j = nbr[d];
                    if (j >= 0) g[1 + d] += c * (ri * Y[j * nu + m] + vi * Q[j * nu + m]) * si;
                }
            }
        }
        if (!(fabsf(o[i * 4]) < LP_OCLAMP)) g[0] = 0.0; // clamped: no gradient through the diagonal output
        if (do64) *(v4d *)(do64 + i * 4) = (v4d){g[0], g[1], g[2], g[3]};
        *(v4s *)(dob + i * 4) = (v4s){(short)f32_to_bf16((float)g[0]), (short)f32_to_bf16((float)g[1]),
                                      (short)f32_to_bf16((float)g[2]), (short)f32_to_bf16((float)g[3])};
    }
}

static unsigned lpl_grid(long long n) { return (unsigned)std::min<long long>(std::max<long long>((n + LPL_BLOCK - 1) / LPL_BLOCK, 1), 2048); }

hipError_t launch_lp_mv(long long n, int nb, int nu, const LpMat *mats, const double *const *xtab, const double *xbase,
                        double *ybase, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 g(lpl_grid(n), nb);
    if (nu == 4 && xtab)
        hipLaunchKernelGGL((k_lp_mv<4, true>), g, dim3(LPL_BLOCK), 0, st, n, nu, mats, xtab, xbase, ybase);
    else if (nu == 4)
        hipLaunchKernelGGL((k_lp_mv<4, false>), g, dim3(LPL_BLOCK), 0, st, n, nu, mats, xtab, xbase, ybase);
    else if (xtab)
        hipLaunchKernelGGL((k_lp_mv<0, true>), g, dim3(LPL_BLOCK), 0, st, n, nu, mats, xtab, xbase, ybase);
    else
        hipLaunchKernelGGL((k_lp_mv<0, false>), g, dim3(LPL_BLOCK), 0, st, n, nu, mats, xtab, xbase, ybase);
    return hipGetLastError();
}

hipError_t launch_lp_resid_dots(long long n, int nb, int nu, double eps, const LpMat *gm, const double *const *utab,
                                const double *y, const double *v, double *r, const DotWs &wu, const DotWs &wr,
                                int stride, int *flags, hipStream_t st)
{
    SlotView su{wu, stride}, sr{wr, stride};
    if (nu == 4)
        hipLaunchKernelGGL(k_lp_resid<4>, dim3(lpl_grid(n), nb), dim3(LPL_BLOCK), 0, st, n, nu, eps, gm, utab, y, v, r);
    else
        hipLaunchKernelGGL(k_lp_resid<0>, dim3(lpl_grid(n), nb), dim3(LPL_BLOCK), 0, st, n, nu, eps, gm, utab, y, v, r);
    hipLaunchKernelGGL(k_lp_dots<LP_DOT_P>, dim3(LP_DOT_CHUNKS, nb * nu), dim3(LPL_BLOCK), 0, st, n, nu, utab, r, su,
                       sr, flags);
    return hipGetLastError();
}

hipError_t launch_lp_dots_merge(int npairs, const DotWs &wu, const DotWs &wr, int stride, double *dots, int *flags,
                                hipStream_t st)
{
    SlotView su{wu, stride}, sr{wr, stride};
    hipLaunchKernelGGL(k_lp_dots_merge<LP_DOT_P>, dim3(npairs), dim3(LPL_BLOCK), 0, st, LP_DOT_CHUNKS, su, sr, dots,
                       flags);
    return hipGetLastError();
}

hipError_t launch_lp_dodg_all(int N, int nb, int nu, double scale, const double *dots, const float *o, const float *s,
                              const LpMat *gm, const double *r, const double *y, const double *v, const double *q,
                              double *do64, bf16_t *dob, double *loss, hipStream_t st)
{
    const long long n = (long long)N * N * N;
    if (nu == 4)
        hipLaunchKernelGGL(k_lp_dodg<4>, dim3(lpl_grid(n), nb), dim3(LPL_BLOCK), 0, st, N, nu, nb * nu, scale, dots, o,
                           s, gm, r, y, v, q, do64, dob, loss);
    else
        hipLaunchKernelGGL(k_lp_dodg<0>, dim3(lpl_grid(n), nb), dim3(LPL_BLOCK), 0, st, N, nu, nb * nu, scale, dots, o,
                           s, gm, r, y, v, q, do64, dob, loss);
    return hipGetLastError();
}

} // namespace rpcg
