// Learned preconditioner: per-cell input features from the matrix and the
// factor G (and G^T) from the network outputs.
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
// missing), (number of absent neighbours) / 6; and s_i. A non-positive or
// missing diagonal stores gen into *bad. System k = blockIdx.y.
__global__ void k_lp_features(int N, LpMatSet set, bf16_t *__restrict__ feat, float *__restrict__ s, int *bad, int gen)
{
    const long long n = (long long)N * N * N;
    const int k = blockIdx.y;
    const int *__restrict__ rp = set.m[k].rp;
    const int *__restrict__ col = set.m[k].col;
    const double *__restrict__ val = set.m[k].val;
    feat += (long long)k * n * 4;
    s += (long long)k * n;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / ((long long)N * N));
        double aii = 0.0, a[3] = {0.0, 0.0, 0.0};
        const long long nb[3] = {x > 0 ? i - 1 : -1, y > 0 ? i - N : -1, z > 0 ? i - (long long)N * N : -1};
        const int b = rp[i], e = rp[i + 1];
        for (int q = b; q < e; ++q) {
            const long long c = col[q];
            const double v = val[q];
            if (c == i) aii = v;
            for (int d = 0; d < 3; ++d)
                if (c == nb[d]) a[d] = v;
        }
        if (!(aii > 0.0)) *bad = gen;
        bf16_t f[4];
        for (int d = 0; d < 3; ++d)
            f[d] = f32_to_bf16((nb[d] >= 0 && a[d] != 0.0) ? (float)log(fabs(a[d]) / aii) : LP_ABSENT);
        f[3] = f32_to_bf16((float)((7 - (e - b)) / 6.0));
        *(v4s *)&feat[i * 4] = (v4s){(short)f[0], (short)f[1], (short)f[2], (short)f[3]};
        s[i] = (float)(1.0 / sqrt(aii));
    }
}

// G and G^T values at the positions of the structure (lp_pattern); instance
// k = blockIdx.y reads o, s and writes g_val, gt_val at k times their strides.
__global__ void k_lp_factor(int N, const float *__restrict__ o, const float *__restrict__ s,
                            const int *__restrict__ g_rp, const int *__restrict__ gt_rp, double *__restrict__ g_val,
                            double *__restrict__ gt_val, long long val_stride)
{
    const long long n = (long long)N * N * N, NN = (long long)N * N;
    const int k = blockIdx.y;
    o += (long long)k * n * 4;
    s += (long long)k * n;
    g_val += (long long)k * val_stride;
    gt_val += (long long)k * val_stride;
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

__global__ void k_lp_to_bf16(long long n, const double *__restrict__ a, bf16_t *__restrict__ b)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        b[i] = f32_to_bf16((float)a[i]);
}

static int lp_grid(long long n) { return (int)std::min<long long>(std::max<long long>((n + 255) / 256, 1), 4096); }

hipError_t launch_lp_features(int N, int nb, const LpMatSet &set, bf16_t *feat, float *s, int *bad, int gen,
                              hipStream_t st)
{
    const long long n = (long long)N * N * N;
    if (nb < 1 || nb > LP_MAT_ARGS) return hipErrorInvalidValue;
    k_lp_features<<<dim3(lp_grid(n), nb), 256, 0, st>>>(N, set, feat, s, bad, gen);
    return hipGetLastError();
}

hipError_t launch_lp_factor(int N, int nb, const float *o, const float *s, const int *g_rp, const int *gt_rp,
                            double *g_val, double *gt_val, long long val_stride, hipStream_t st)
{
    const long long n = (long long)N * N * N;
    k_lp_factor<<<dim3(lp_grid(n), nb), 256, 0, st>>>(N, o, s, g_rp, gt_rp, g_val, gt_val, val_stride);
    return hipGetLastError();
}

hipError_t launch_lp_to_bf16(long long n, const double *a, bf16_t *b, hipStream_t st)
{
    k_lp_to_bf16<<<lp_grid(n), 256, 0, st>>>(n, a, b);
    return hipGetLastError();
}

} // namespace rpcg
