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
typedef double v4d __attribute__((ext_vector_type(4)));

// y_p = M_k x_p for p = k nu + m, m < nu (grid.y = k). x_p from the pointer
// table xtab when given, else xbase + p n; y_p = ybase + p n. Each row is an
// fma chain over its entries in storage order from zero.
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_mv(long long n, int nu, const LpMat *__restrict__ mats,
                                                     const double *const *__restrict__ xtab,
                                                     const double *__restrict__ xbase, double *__restrict__ ybase)
{
    const int k = blockIdx.y;
    const LpMat M = mats[k];
    for (long long i = (long long)blockIdx.x * LPL_BLOCK + threadIdx.x; i < n;
         i += (long long)gridDim.x * LPL_BLOCK) {
        const int b = M.rp[i], len = M.rp[i + 1] - b;
        if (len <= LPL_ROWCAP) {
            double a[LPL_ROWCAP];
            int c[LPL_ROWCAP];
#pragma unroll
            for (int j = 0; j < LPL_ROWCAP; ++j) {
                a[j] = j < len ? M.val[b + j] : 0.0;
                c[j] = j < len ? M.col[b + j] : 0;
            }
            for (int m = 0; m < nu; ++m) {
                const long long p = (long long)k * nu + m;
                const double *__restrict__ x = xtab ? xtab[p] : xbase + p * n;
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < LPL_ROWCAP; ++j)
                    if (j < len) acc = __builtin_fma(a[j], x[c[j]], acc);
                ybase[p * n + i] = acc;
            }
        } else {
            for (int m = 0; m < nu; ++m) {
                const long long p = (long long)k * nu + m;
                const double *__restrict__ x = xtab ? xtab[p] : xbase + p * n;
                double acc = 0.0;
                for (int j = 0; j < len; ++j) acc = __builtin_fma(M.val[b + j], x[M.col[b + j]], acc);
                ybase[p * n + i] = acc;
            }
        }
    }
}

// r_p = (G_k y_p + eps v_p) - u_p for the nu pairs of instance k =
// blockIdx.y (a row of G is read once for all of them).
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_resid(long long n, int nu, double eps,
                                                        const LpMat *__restrict__ gm,
                                                        const double *const *__restrict__ utab,
                                                        const double *__restrict__ ybase,
                                                        const double *__restrict__ vbase, double *__restrict__ rbase)
{
    const int k = blockIdx.y;
    const LpMat G = gm[k];
    for (long long i = (long long)blockIdx.x * LPL_BLOCK + threadIdx.x; i < n;
         i += (long long)gridDim.x * LPL_BLOCK) {
        const int b = G.rp[i], len = G.rp[i + 1] - b;
        double a[LPL_ROWCAP];
        int c[LPL_ROWCAP];
#pragma unroll
        for (int j = 0; j < LPL_ROWCAP; ++j) {
            a[j] = j < len ? G.val[b + j] : 0.0;
            c[j] = j < len ? G.col[b + j] : 0;
        }
        for (int m = 0; m < nu; ++m) {
            const long long p = (long long)k * nu + m;
            const double *__restrict__ y = ybase + p * n;
            double w = 0.0;
            if (len <= LPL_ROWCAP) {
#pragma unroll
                for (int j = 0; j < LPL_ROWCAP; ++j)
                    if (j < len) w = __builtin_fma(a[j], y[c[j]], w);
            } else {
                for (int j = 0; j < len; ++j) w = __builtin_fma(G.val[b + j], y[G.col[b + j]], w);
            }
            rbase[p * n + i] = (w + eps * vbase[p * n + i]) - utab[p][i];
        }
    }
}

// The exact-dot partials of <u_p, u_p> and <r_p, r_p> into slots p chunks +
// blockIdx.x (grid: chunks x pairs).
template <int P>
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_dots(long long n, const double *const *__restrict__ utab,
                                                       const double *__restrict__ rbase, SlotView su, SlotView sr,
                                                       int *flags)
{
    __shared__ RedShared sh;
    const int p = blockIdx.y;
    const double *__restrict__ u = utab[p];
    const double *__restrict__ r = rbase + (long long)p * n;
    zero_acc(sh.acc[0]);
    zero_acc(sh.acc[1]);
    __syncthreads();
    LaneDot<MODE_EXBLAS, P> Lu, Lr;
    Lu.init();
    Lr.init();
    for (long long i = (long long)blockIdx.x * LPL_BLOCK + threadIdx.x; i < n;
         i += (long long)gridDim.x * LPL_BLOCK) {
        const double ui = u[i], ri = r[i];
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
// binary64 there; the loss (pairs in order) by one thread.
__global__ void __launch_bounds__(LPL_BLOCK) k_lp_dodg(int N, int nu, int npairs, double scale,
                                                       const double *__restrict__ dots, const float *__restrict__ o,
                                                       const float *__restrict__ s, const LpMat *__restrict__ gm,
                                                       const double *__restrict__ rbase,
                                                       const double *__restrict__ ybase,
                                                       const double *__restrict__ vbase,
                                                       const double *__restrict__ qbase, double *__restrict__ do64,
                                                       bf16_t *__restrict__ dob, double *loss)
{
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
    for (long long i = (long long)blockIdx.x * LPL_BLOCK + threadIdx.x; i < n;
         i += (long long)gridDim.x * LPL_BLOCK) {
        const int x = (int)(i % N), yy = (int)((i / N) % N), z = (int)(i / NN);
        const double si = s[i];
        const double gdiag = G.val[G.rp[i + 1] - 1];
        const long long nbr[3] = {x > 0 ? i - 1 : -1, yy > 0 ? i - N : -1, z > 0 ? i - NN : -1};
        double g[4] = {0.0, 0.0, 0.0, 0.0};
        for (int m = 0; m < nu; ++m) {
            const long long off = ((long long)k * nu + m) * n;
            const double c = scale * 2.0 / dots[2 * ((long long)k * nu + m)];
            const double *__restrict__ r = rbase + off, *__restrict__ y = ybase + off;
            const double *__restrict__ v = vbase + off, *__restrict__ q = qbase + off;
            const double ri = r[i], vi = v[i];
            g[0] += c * (ri * y[i] + vi * q[i]) * gdiag;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const long long j = nbr[d];
                if (j >= 0) g[1 + d] += c * (ri * y[j] + vi * q[j]) * si;
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
    hipLaunchKernelGGL(k_lp_mv, dim3(lpl_grid(n), nb), dim3(LPL_BLOCK), 0, st, n, nu, mats, xtab, xbase, ybase);
    return hipGetLastError();
}

hipError_t launch_lp_resid_dots(long long n, int nb, int nu, double eps, const LpMat *gm, const double *const *utab,
                                const double *y, const double *v, double *r, const DotWs &wu, const DotWs &wr,
                                int stride, int *flags, hipStream_t st)
{
    SlotView su{wu, stride}, sr{wr, stride};
    hipLaunchKernelGGL(k_lp_resid, dim3(lpl_grid(n), nb), dim3(LPL_BLOCK), 0, st, n, nu, eps, gm, utab, y, v, r);
    hipLaunchKernelGGL(k_lp_dots<LP_DOT_P>, dim3(LP_DOT_CHUNKS, nb * nu), dim3(LPL_BLOCK), 0, st, n, utab, r, su, sr,
                       flags);
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
    hipLaunchKernelGGL(k_lp_dodg, dim3(lpl_grid(n), nb), dim3(LPL_BLOCK), 0, st, N, nu, nb * nu, scale, dots, o, s,
                       gm, r, y, v, q, do64, dob, loss);
    return hipGetLastError();
}

} // namespace rpcg
