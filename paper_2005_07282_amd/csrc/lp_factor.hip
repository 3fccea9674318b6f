// Learned preconditioner: per-cell input features from the matrix, the factor
// G (and G^T) from the network outputs, and the training loss's gradient with
// respect to the outputs.
//
// G sits on the lower-triangle pattern of a 7-point operator on an N^3 grid:
// row i holds the -z, -y, -x neighbours and the diagonal (ascending columns);
// G^T row j the diagonal and the +x, +y, +z neighbours. With
// s_i = RN32(1 / sqrt(a_ii)) (in binary64, rounded once):
//   G_ii = RN32(s_i exp(clamp(o_i0, -4, 4))),  G_i,j(k) = RN32(s_i o_ik),
// k = 1, 2, 3 for the -x, -y, -z neighbour, widened to binary64 for the solve.
#include "lp_common.hpp"
#include "lp_factor.hpp"

namespace rpcg {

__device__ __forceinline__ float lp_clamp(float v) { return fminf(fmaxf(v, -LP_OCLAMP), LP_OCLAMP); }

// features: ln(|a_ij| / a_ii) of the -x, -y, -z neighbours (LP_ABSENT if
// missing), (number of absent neighbours) / 6; and s_i. Flags a non-positive
// or missing diagonal.
__global__ void k_lp_features(int N, const int *__restrict__ rp, const int *__restrict__ col,
                              const double *__restrict__ val, bf16_t *__restrict__ feat, float *__restrict__ s,
                              int *bad)
{
    const long long n = (long long)N * N * N;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / ((long long)N * N));
        double aii = 0.0, a[3] = {0.0, 0.0, 0.0};
        const long long nb[3] = {x > 0 ? i - 1 : -1, y > 0 ? i - N : -1, z > 0 ? i - (long long)N * N : -1};
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const long long c = col[k];
            if (c == i) aii = val[k];
            for (int d = 0; d < 3; ++d)
                if (c == nb[d]) a[d] = val[k];
        }
        if (!(aii > 0.0)) atomicOr(bad, 1);
        for (int d = 0; d < 3; ++d) {
            const float f = (nb[d] >= 0 && a[d] != 0.0) ? (float)log(fabs(a[d]) / aii) : LP_ABSENT;
            feat[i * 4 + d] = f32_to_bf16(f);
        }
        feat[i * 4 + 3] = f32_to_bf16((float)((7 - (rp[i + 1] - rp[i])) / 6.0));
        s[i] = (float)(1.0 / sqrt(aii));
    }
}

// G and G^T values at the positions of the structure (lp_pattern).
__global__ void k_lp_factor(int N, const float *__restrict__ o, const float *__restrict__ s,
                            const int *__restrict__ g_rp, const int *__restrict__ gt_rp, double *__restrict__ g_val,
                            double *__restrict__ gt_val)
{
    const long long n = (long long)N * N * N, NN = (long long)N * N;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / NN);
        const float si = s[i];
        // row i of G: -z, -y, -x, diagonal
        int p = g_rp[i];
        if (z > 0) g_val[p++] = (double)(si * o[i * 4 + 3]);
        if (y > 0) g_val[p++] = (double)(si * o[i * 4 + 2]);
        if (x > 0) g_val[p++] = (double)(si * o[i * 4 + 1]);
        g_val[p] = (double)(si * expf(lp_clamp(o[i * 4])));
        // row i of G^T: diagonal, +x, +y, +z (entries G_{i+off, i})
        int q = gt_rp[i];
        gt_val[q++] = (double)(si * expf(lp_clamp(o[i * 4])));
        if (x < N - 1) gt_val[q++] = (double)(s[i + 1] * o[(i + 1) * 4 + 1]);
        if (y < N - 1) gt_val[q++] = (double)(s[i + N] * o[(i + N) * 4 + 2]);
        if (z < N - 1) gt_val[q] = (double)(s[i + NN] * o[(i + NN) * 4 + 3]);
    }
}

// r = (G y + eps v) - u
__global__ void k_lp_resid(long long n, double eps, const double *__restrict__ w, const double *__restrict__ v,
                           const double *__restrict__ u, double *__restrict__ r)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        r[i] = (w[i] + eps * v[i]) - u[i];
}

// do += c (r_i y_j + v_i q_j) dG/do on the pattern, c = scale * 2 / <u,u>;
// loss += scale * <r,r> / <u,u> (thread 0).
__global__ void k_lp_dodg(int N, double scale, const double *__restrict__ uu, const double *__restrict__ rr,
                          const float *__restrict__ o, const float *__restrict__ s, const int *__restrict__ g_rp,
                          const double *__restrict__ g_val, const double *__restrict__ r, const double *__restrict__ y,
                          const double *__restrict__ v, const double *__restrict__ q, double *__restrict__ do64,
                          double *loss)
{
    const long long n = (long long)N * N * N, NN = (long long)N * N;
    const double c = scale * 2.0 / uu[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) loss[0] += scale * rr[0] / uu[0];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % N), yy = (int)((i / N) % N), z = (int)(i / NN);
        const double si = s[i];
        const double gdiag = g_val[g_rp[i + 1] - 1];
        const double d0 = c * (r[i] * y[i] + v[i] * q[i]);
        if (fabsf(o[i * 4]) < LP_OCLAMP) do64[i * 4] += d0 * gdiag;
        const long long nbr[3] = {x > 0 ? i - 1 : -1, yy > 0 ? i - N : -1, z > 0 ? i - NN : -1};
        for (int k = 0; k < 3; ++k) {
            const long long j = nbr[k];
            if (j < 0) continue;
            do64[i * 4 + 1 + k] += c * (r[i] * y[j] + v[i] * q[j]) * si;
        }
    }
}

__global__ void k_lp_to_bf16(long long n, const double *__restrict__ a, bf16_t *__restrict__ b)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = f32_to_bf16((float)a[i]);
}

static int lp_grid(long long n) { return (int)std::min<long long>(std::max<long long>((n + 255) / 256, 1), 4096); }

hipError_t launch_lp_features(int N, const int *rp, const int *col, const double *val, bf16_t *feat, float *s, int *bad,
                              hipStream_t st)
{
    const long long n = (long long)N * N * N;
    k_lp_features<<<lp_grid(n), 256, 0, st>>>(N, rp, col, val, feat, s, bad);
    return hipGetLastError();
}

hipError_t launch_lp_factor(int N, const float *o, const float *s, const int *g_rp, const int *gt_rp, double *g_val,
                            double *gt_val, hipStream_t st)
{
    const long long n = (long long)N * N * N;
    k_lp_factor<<<lp_grid(n), 256, 0, st>>>(N, o, s, g_rp, gt_rp, g_val, gt_val);
    return hipGetLastError();
}

hipError_t launch_lp_resid(long long n, double eps, const double *w, const double *v, const double *u, double *r,
                           hipStream_t st)
{
    k_lp_resid<<<lp_grid(n), 256, 0, st>>>(n, eps, w, v, u, r);
    return hipGetLastError();
}

hipError_t launch_lp_dodg(int N, double scale, const double *uu, const double *rr, const float *o, const float *s,
                          const int *g_rp, const double *g_val, const double *r, const double *y, const double *v,
                          const double *q, double *do64, double *loss, hipStream_t st)
{
    const long long n = (long long)N * N * N;
    k_lp_dodg<<<lp_grid(n), 256, 0, st>>>(N, scale, uu, rr, o, s, g_rp, g_val, r, y, v, q, do64, loss);
    return hipGetLastError();
}

hipError_t launch_lp_to_bf16(long long n, const double *a, bf16_t *b, hipStream_t st)
{
    k_lp_to_bf16<<<lp_grid(n), 256, 0, st>>>(n, a, b);
    return hipGetLastError();
}

} // namespace rpcg
