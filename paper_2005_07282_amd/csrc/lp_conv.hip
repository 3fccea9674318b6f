// Learned preconditioner: bfloat16 matrix-core convolutions (forward and
// adjoint), weight gradients with fixed-order reductions, weight preparation
// and the Adam update.
#include "lp_common.hpp"

#include <algorithm>

namespace rpcg {

__device__ __forceinline__ void tap_offset(int t, int &dz, int &dy, int &dx)
{
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
}

// Implicit-GEMM convolution on 16x16x16 bfloat16 MFMA. A wavefront computes a
// tile of 16 cells along x (rows M) by 16 output channels (columns N); K runs
// over (tap, input channel) in chunks of 16: one tap per chunk with 16 input
// channels, four taps per chunk with 4. Lane l supplies A[m = l%16][k = 4(l/16)
// + j] and B[k][n = l%16] for j < 4 and receives D[4(l/16) + j][l%16].
template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(256) k_lp_conv(int nb, int N, const bf16_t *__restrict__ in,
                                                 const bf16_t *__restrict__ wt, const float *__restrict__ bias,
                                                 const float *__restrict__ mask, float *__restrict__ pre,
                                                 bf16_t *__restrict__ act)
{
    constexpr int TPC = 16 / CIN;                       // taps per chunk
    constexpr int NCH = (LP_TAPS + TPC - 1) / TPC;      // chunks
    __shared__ bf16_t w[NCH * TPC][16][CIN];
    for (int e = threadIdx.x; e < NCH * TPC * 16 * CIN; e += blockDim.x)
        (&w[0][0][0])[e] = e < LP_TAPS * 16 * CIN ? wt[e] : (bf16_t)0;
    __syncthreads();
    const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
    const int tiles_x = (N + 15) >> 4;
    const long long ntiles = (long long)nb * N * N * tiles_x;
    const long long N3 = (long long)N * N * N;
    const int waves = blockDim.x >> 6;
    for (long long tile = (long long)blockIdx.x * waves + (threadIdx.x >> 6); tile < ntiles;
         tile += (long long)gridDim.x * waves) {
        const int tx = (int)(tile % tiles_x);
        const long long line = tile / tiles_x; // (b, z, y)
        const int y = (int)(line % N), z = (int)((line / N) % N);
        const long long b = line / ((long long)N * N);
        const int x0 = tx * 16;
        const bf16_t *inb = in + b * N3 * CIN;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
        for (int c = 0; c < NCH; ++c) {
            const int t = c * TPC + (CIN == 16 ? 0 : g);
            const int cbase = CIN == 16 ? 4 * g : 0;
            v4s a = {0, 0, 0, 0};
            if (t < LP_TAPS) {
                int dz, dy, dx;
                tap_offset(t, dz, dy, dx);
                const int X = x0 + m + dx, Y = y + dy, Z = z + dz;
                if (x0 + m < N && X >= 0 && X < N && Y >= 0 && Y < N && Z >= 0 && Z < N)
                    a = *(const v4s *)(inb + (((long long)Z * N + Y) * N + X) * CIN + cbase);
            }
            const v4s bw = *(const v4s *)&w[t][m][cbase];
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw, acc, 0, 0, 0);
        }
        const int co = m;
        if (co < COUT) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int x = x0 + 4 * g + j;
                if (x >= N) continue;
                const long long cell = b * N3 + ((long long)z * N + y) * N + x;
                const float v = acc[j];
                if (EPI == EPI_RELU) {
                    const float p = v + bias[co];
                    pre[cell * COUT + co] = p;
                    act[cell * COUT + co] = f32_to_bf16(p > 0.f ? p : 0.f);
                } else if (EPI == EPI_LINEAR) {
                    pre[cell * COUT + co] = v + bias[co];
                } else {
                    act[cell * COUT + co] = f32_to_bf16(mask[cell * COUT + co] > 0.f ? v : 0.f);
                }
            }
        }
    }
}

// Weight gradient dW[t][co][ci] = sum over cells of dout[cell][co] in[cell + off(t)][ci]
// and bias gradient db[co] = sum of dout[cell][co], on 16x16x16 MFMA with
// M = co, N = ci, K = the 16 cells of a tile. Each workgroup sums its waves in
// wave order and writes one slot; the slots are summed in slot order later.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_lp_conv_dw(int nb, int N, const bf16_t *__restrict__ in,
                                                    const bf16_t *__restrict__ dout, float *__restrict__ pw,
                                                    float *__restrict__ pb)
{
    __shared__ float sw[LP_TAPS][16][16];
    __shared__ float sbl[4][4][16]; // [wave][lane group][co]
    const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
    const int wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
    const int tiles_x = (N + 15) >> 4;
    const long long ntiles = (long long)nb * N * N * tiles_x;
    const long long N3 = (long long)N * N * N;
    v4f acc[LP_TAPS];
#pragma unroll
    for (int t = 0; t < LP_TAPS; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (long long tile = (long long)blockIdx.x * waves + wave; tile < ntiles; tile += (long long)gridDim.x * waves) {
        const int tx = (int)(tile % tiles_x);
        const long long line = tile / tiles_x;
        const int y = (int)(line % N), z = (int)((line / N) % N);
        const long long b = line / ((long long)N * N);
        const int x0 = tx * 16;
        // A[m = co][k = cell 4g + j]
        v4s a = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = x0 + 4 * g + j;
            if (m < COUT && x < N) {
                const bf16_t h = dout[(b * N3 + ((long long)z * N + y) * N + x) * COUT + m];
                a[j] = (short)h;
                bsum += bf16_to_f32(h);
            }
        }
#pragma unroll
        for (int t = 0; t < LP_TAPS; ++t) {
            int dz, dy, dx;
            tap_offset(t, dz, dy, dx);
            const int Y = y + dy, Z = z + dz;
            v4s bv = {0, 0, 0, 0};
            if (m < CIN && Y >= 0 && Y < N && Z >= 0 && Z < N) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int xc = x0 + 4 * g + j, X = xc + dx;
                    if (xc < N && X >= 0 && X < N)
                        bv[j] = (short)in[(b * N3 + ((long long)Z * N + Y) * N + X) * CIN + m];
                }
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[t], 0, 0, 0);
        }
    }
    // workgroup sum in wave order; lane l holds dW[t][4g + j][l % 16]
    sbl[wave][g][m] = bsum;
    for (int w = 0; w < waves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < LP_TAPS; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float &dst = sw[t][4 * g + j][m];
                    dst = (w == 0) ? acc[t][j] : dst + acc[t][j];
                }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < LP_TAPS * 256; e += blockDim.x)
        pw[(long long)blockIdx.x * LP_TAPS * 256 + e] = (&sw[0][0][0])[e];
    if (threadIdx.x < 16) {
        float t = 0.f;
        for (int w = 0; w < waves; ++w)
            for (int gg = 0; gg < 4; ++gg) t += sbl[w][gg][threadIdx.x];
        pb[blockIdx.x * 16 + threadIdx.x] = t;
    }
}

// Gradient of one layer from the slots, summed in slot order: weights in the
// layer's layout [27][cout][cin] from the padded [27][16][16] partials, then
// the cout bias entries.
__global__ void k_lp_reduce(int nslots, int cout, int cin, const float *__restrict__ pw, const float *__restrict__ pb,
                            float *__restrict__ gw, float *__restrict__ gb)
{
    const int nw = LP_TAPS * cout * cin;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nw + cout; i += gridDim.x * blockDim.x) {
        float s = 0.f;
        if (i < nw) {
            const int t = i / (cout * cin), o = (i / cin) % cout, c = i % cin;
            const int src = (t * 16 + o) * 16 + c;
            for (int k = 0; k < nslots; ++k) s += pw[(long long)k * LP_TAPS * 256 + src];
            gw[i] = s;
        } else {
            const int o = i - nw;
            for (int k = 0; k < nslots; ++k) s += pb[k * 16 + o];
            gb[o] = s;
        }
    }
}

// Forward weights [27][16][CIN] (outputs padded to 16 with zeros) and the
// adjoint weights of layers 2 and 3: wT[26 - t][ci][co] = W[t][co][ci].
__global__ void k_lp_prep(const float *__restrict__ p, bf16_t *w1, bf16_t *w2, bf16_t *w3, bf16_t *w2t, bf16_t *w3t)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < LP_TAPS * 16 * 16) {
        const int t = e / 256, o = (e / 16) % 16, i = e % 16;
        // layer 2 forward [t][o][i] and adjoint [26 - t][i][o]
        const bf16_t v2 = f32_to_bf16(p[LP_OFF_W2 + (t * LP_HID + o) * LP_HID + i]);
        w2[e] = v2;
        w2t[((LP_TAPS - 1 - t) * 16 + i) * 16 + o] = v2;
        // layer 3 forward [t][o][i], o < 4 (rows 4..15 zero)
        w3[e] = o < LP_COUT ? f32_to_bf16(p[LP_OFF_W3 + (t * LP_COUT + o) * LP_HID + i]) : (bf16_t)0;
    }
    if (e < LP_TAPS * 16 * 4) {
        const int t = e / 64, o = (e / 4) % 16, i = e % 4;
        // layer 1 forward [t][o][i] (4 inputs)
        w1[e] = f32_to_bf16(p[LP_OFF_W1 + (t * LP_HID + o) * LP_CIN + i]);
        // layer 3 adjoint: inputs are its 4 outputs, outputs its 16 inputs: [26 - t][ci = o][co = i]
        w3t[((LP_TAPS - 1 - t) * 16 + o) * 4 + i] = f32_to_bf16(p[LP_OFF_W3 + (t * LP_COUT + i) * LP_HID + o]);
    }
}

// Adam with bias correction (Kingma and Ba, 2015).
__global__ void k_lp_adam(int n, float *__restrict__ p, const float *__restrict__ gr, float *__restrict__ m,
                          float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (__builtin_sqrtf(vi / c2) + eps);
}

hipError_t launch_lp_conv(int cin, int cout, int epi, int nb, int N, const bf16_t *in, const bf16_t *wt,
                          const float *bias, const float *mask, float *pre, bf16_t *act, hipStream_t s)
{
    const long long tiles = (long long)nb * N * N * ((N + 15) / 16);
    const int grid = (int)std::min<long long>((tiles + 3) / 4, 8192);
    if (grid <= 0) return hipSuccess;
    if (cin == 4 && cout == 16 && epi == EPI_RELU)
        k_lp_conv<4, 16, EPI_RELU><<<grid, 256, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else if (cin == 16 && cout == 16 && epi == EPI_RELU)
        k_lp_conv<16, 16, EPI_RELU><<<grid, 256, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else if (cin == 16 && cout == 4 && epi == EPI_LINEAR)
        k_lp_conv<16, 4, EPI_LINEAR><<<grid, 256, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else if (cin == 4 && cout == 16 && epi == EPI_MASK)
        k_lp_conv<4, 16, EPI_MASK><<<grid, 256, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else if (cin == 16 && cout == 16 && epi == EPI_MASK)
        k_lp_conv<16, 16, EPI_MASK><<<grid, 256, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_lp_conv_dw(int cin, int cout, int nb, int N, const bf16_t *in, const bf16_t *dout, float *pw,
                             float *pb, int grid, hipStream_t s)
{
    if (cin == 16 && cout == 4)
        k_lp_conv_dw<16, 4><<<grid, 256, 0, s>>>(nb, N, in, dout, pw, pb);
    else if (cin == 16 && cout == 16)
        k_lp_conv_dw<16, 16><<<grid, 256, 0, s>>>(nb, N, in, dout, pw, pb);
    else if (cin == 4 && cout == 16)
        k_lp_conv_dw<4, 16><<<grid, 256, 0, s>>>(nb, N, in, dout, pw, pb);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_lp_reduce(int nslots, int cout, int cin, const float *pw, const float *pb, float *gw, float *gb,
                            hipStream_t s)
{
    const int len = LP_TAPS * cout * cin + cout;
    k_lp_reduce<<<(len + 255) / 256, 256, 0, s>>>(nslots, cout, cin, pw, pb, gw, gb);
    return hipGetLastError();
}

hipError_t launch_lp_prep(const float *params, bf16_t *w1, bf16_t *w2, bf16_t *w3, bf16_t *w2t, bf16_t *w3t,
                          hipStream_t s)
{
    k_lp_prep<<<(LP_TAPS * 256 + 255) / 256, 256, 0, s>>>(params, w1, w2, w3, w2t, w3t);
    return hipGetLastError();
}

hipError_t launch_lp_adam(int n, float *params, const float *grad, float *m, float *v, float lr, float b1, float b2,
                          float eps, int step, hipStream_t s)
{
    const float c1 = 1.f - __builtin_powf(b1, (float)step), c2 = 1.f - __builtin_powf(b2, (float)step);
    k_lp_adam<<<(n + 255) / 256, 256, 0, s>>>(n, params, grad, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

} // namespace rpcg
