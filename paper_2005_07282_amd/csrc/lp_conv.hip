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
//
// A workgroup of four wavefronts takes a block of 16 x 4 x 1 cells (one
// y-line per wavefront) and first stages the block's inputs with their halo
// (18 x 6 x 3 cells, zeros outside the grid) in LDS with coalesced loads;
// the A operands are then read from LDS, so each input is fetched from
// memory once per block instead of once per tap.
constexpr int CONV_BX = 16, CONV_BY = 4;                       // block of output cells (x, y)
constexpr int CONV_HX = CONV_BX + 2, CONV_HY = CONV_BY + 2, CONV_HZ = 3; // with halo
constexpr int CONV_HCELLS = CONV_HX * CONV_HY * CONV_HZ;

// The staged inputs are kept in groups of four channels: group q of cell c
// is the 8 bytes at tile[(q * P + c) * 4], with a pitch P = 1 (mod 16) cells
// so that the four groups of one cell fall in different LDS banks.
__host__ __device__ constexpr int halo_pitch(int cells) { return cells + (17 - cells % 16) % 16; }

// Stage the inputs of the block of BY y-lines of 16 cells at (x0, y0) of
// system b, with a one-cell halo in x and y, over the HZ planes from z0,
// into cells (zc * (BY + 2) + yc) * 18 + xc of tile (zeros outside the
// grid). 8-byte units; sixteen consecutive threads take one channel group of
// sixteen consecutive cells, so a wavefront reads whole runs of the input
// and writes whole LDS rows.
template <int CIN, int BY, int HZ>
__device__ __forceinline__ void stage_halo(bf16_t *tile, const bf16_t *__restrict__ inb, int N, int x0, int y0, int z0)
{
    constexpr int UPC = CIN / 4, HY = BY + 2, HC = CONV_HX * HY * HZ, P = halo_pitch(HC);
    constexpr int RUNS = (HC + 15) / 16;
    for (int u = threadIdx.x; u < RUNS * 16 * UPC; u += blockDim.x) {
        const int q = (u >> 4) % UPC, cell = (u / (16 * UPC)) * 16 + (u & 15);
        if (cell >= HC) continue;
        const int xc = cell % CONV_HX, yc = (cell / CONV_HX) % HY, zc = cell / (CONV_HX * HY);
        const int X = x0 - 1 + xc, Y = y0 - 1 + yc, Z = z0 + zc;
        v4s v = {0, 0, 0, 0};
        if (X >= 0 && X < N && Y >= 0 && Y < N && Z >= 0 && Z < N)
            v = *(const v4s *)(inb + (((long long)Z * N + Y) * N + X) * CIN + 4 * q);
        *(v4s *)&tile[(q * P + cell) * 4] = v;
    }
}

template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(64 * CONV_BY) k_lp_conv(int nb, int N, const bf16_t *__restrict__ in,
                                                          const bf16_t *__restrict__ wt, const float *__restrict__ bias,
                                                          const float *__restrict__ mask, float *__restrict__ pre,
                                                          bf16_t *__restrict__ act)
{
    constexpr int TPC = 16 / CIN;                       // taps per chunk
    constexpr int NCH = (LP_TAPS + TPC - 1) / TPC;      // chunks
    constexpr int UPC = CIN / 4, P = halo_pitch(CONV_HCELLS);
    // weights by channel group: w[((t * UPC + q) * 16 + co) * 4 + j] = W[t][co][4q + j]
    __shared__ __attribute__((aligned(16))) bf16_t w[NCH * TPC * UPC * 16 * 4];
    __shared__ __attribute__((aligned(16))) bf16_t tile[UPC * P * 4];
    for (int u = threadIdx.x; u < NCH * TPC * UPC * 16; u += blockDim.x) {
        const int co = u & 15, q = (u >> 4) % UPC, t = u / (16 * UPC);
        v4s v = {0, 0, 0, 0};
        if (t < LP_TAPS) v = *(const v4s *)(wt + (t * 16 + co) * CIN + 4 * q);
        *(v4s *)&w[u * 4] = v;
    }
    const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
    const int wave = threadIdx.x >> 6;
    const int tiles_x = (N + CONV_BX - 1) / CONV_BX, tiles_y = (N + CONV_BY - 1) / CONV_BY;
    const long long nblocks = (long long)nb * N * tiles_y * tiles_x;
    const long long N3 = (long long)N * N * N;
    for (long long blk = blockIdx.x; blk < nblocks; blk += gridDim.x) { // workgroup-uniform
        const int tx = (int)(blk % tiles_x);
        long long r = blk / tiles_x;
        const int ty = (int)(r % tiles_y);
        r /= tiles_y;
        const int z = (int)(r % N);
        const long long b = r / N;
        const int x0 = tx * CONV_BX, y0 = ty * CONV_BY;
        const bf16_t *inb = in + b * N3 * CIN;
        __syncthreads(); // the previous block's readers are done (and the weights are in place)
        stage_halo<CIN, CONV_BY, CONV_HZ>(tile, inb, N, x0, y0, z - 1);
        __syncthreads();
        const int y = y0 + wave;
        if (y >= N) continue; // wavefront-uniform; the loop's barrier comes first in the next block
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
        for (int c = 0; c < NCH; ++c) {
            const int t = c * TPC + (CIN == 16 ? 0 : g);
            const int q = CIN == 16 ? g : 0; // channel group
            v4s a = {0, 0, 0, 0};
            if (t < LP_TAPS) {
                int dz, dy, dx;
                tap_offset(t, dz, dy, dx);
                // rows m past the grid's edge read valid LDS cells; their outputs are not stored
                const int hc = ((dz + 1) * CONV_HY + (wave + dy + 1)) * CONV_HX + (m + dx + 1);
                a = *(const v4s *)&tile[(q * P + hc) * 4];
            }
            const v4s bw = *(const v4s *)&w[((t * UPC + q) * 16 + m) * 4];
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
// M = co, N = ci, K = the 16 cells of a tile. The workgroups come in threes
// per slot, one for each dz, so a workgroup keeps the nine tap tiles of its
// dz plane (not all 27), which leaves room for more wavefronts per SIMD. A
// workgroup of DW_BY wavefronts takes blocks of 16 x DW_BY x 1 cells (one
// y-line per wavefront), stages the inputs of its plane with the x and y
// halo in LDS, and each wavefront accumulates its line's nine tap products;
// the B operands come from LDS, six cells per dy serving the three dx taps.
// The three workgroups of a slot take the same blocks in the same order, so
// each tap sums exactly as one workgroup with all 27 taps would. Each
// workgroup sums its waves in wave order and writes its taps of the slot;
// the slots are summed in slot order later.
constexpr int DW_BY = 8;

template <int CIN, int COUT>
__global__ void __launch_bounds__(64 * DW_BY) k_lp_conv_dw(int nb, int N, const bf16_t *__restrict__ in,
                                                          const bf16_t *__restrict__ dout, float *__restrict__ pw,
                                                          float *__restrict__ pb)
{
    constexpr int HY = DW_BY + 2, P = halo_pitch(CONV_HX * HY);
    __shared__ float sw[9][16][16];
    __shared__ float sbl[DW_BY][4][16]; // [wave][lane group][co]
    __shared__ __attribute__((aligned(16))) bf16_t tile[CIN / 4 * P * 4];
    const int lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
    const int wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
    const int dzi = blockIdx.x % 3, slot = blockIdx.x / 3, nslots = gridDim.x / 3; // taps 9 dzi .. 9 dzi + 8
    const int tiles_x = (N + CONV_BX - 1) / CONV_BX, tiles_y = (N + DW_BY - 1) / DW_BY;
    const long long nblocks = (long long)nb * N * tiles_y * tiles_x;
    const long long N3 = (long long)N * N * N;
    v4f acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (long long blk = slot; blk < nblocks; blk += nslots) { // workgroup-uniform
        const int tx = (int)(blk % tiles_x);
        long long r = blk / tiles_x;
        const int ty = (int)(r % tiles_y);
        r /= tiles_y;
        const int z = (int)(r % N);
        const long long b = r / N;
        const int x0 = tx * CONV_BX, y0 = ty * DW_BY;
        __syncthreads(); // the previous block's readers are done
        stage_halo<CIN, DW_BY, 1>(tile, in + b * N3 * CIN, N, x0, y0, z + dzi - 1);
        __syncthreads();
        const int y = y0 + wave;
        if (y >= N) continue; // wavefront-uniform; the loop's barrier comes first in the next block
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
        // B[k = cell 4g + j][n = ci] = in[cell + off(t)][ci]; columns past the
        // row end meet zero A entries, so their (finite) values do not matter
#pragma unroll
        for (int dy3 = 0; dy3 < 3; ++dy3) {
            short v[6] = {0, 0, 0, 0, 0, 0};
            if (m < CIN) {
                const int row = (wave + dy3) * CONV_HX + 4 * g;
#pragma unroll
                for (int i = 0; i < 6; ++i) v[i] = (short)tile[((m >> 2) * P + row + i) * 4 + (m & 3)];
            }
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const v4s bv = {v[dx], v[dx + 1], v[dx + 2], v[dx + 3]};
                acc[dy3 * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[dy3 * 3 + dx], 0, 0, 0);
            }
        }
    }
    // workgroup sum in wave order; lane l holds dW[9 dzi + t][4g + j][l % 16]
    sbl[wave][g][m] = bsum;
    for (int w = 0; w < waves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float &dst = sw[t][4 * g + j][m];
                    dst = (w == 0) ? acc[t][j] : dst + acc[t][j];
                }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < 9 * 256; e += blockDim.x)
        pw[((long long)slot * LP_TAPS + 9 * dzi) * 256 + e] = (&sw[0][0][0])[e];
    if (dzi == 0 && threadIdx.x < 16) {
        float t = 0.f;
        for (int w = 0; w < waves; ++w)
            for (int gg = 0; gg < 4; ++gg) t += sbl[w][gg][threadIdx.x];
        pb[slot * 16 + threadIdx.x] = t;
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
            // the loads run ahead of the adds, which keep the slot order
#pragma unroll 16
            for (int k = 0; k < nslots; ++k) s += pw[(long long)k * LP_TAPS * 256 + src];
            gw[i] = s;
        } else {
            const int o = i - nw;
#pragma unroll 16
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
    const long long blocks = (long long)nb * N * ((N + CONV_BY - 1) / CONV_BY) * ((N + CONV_BX - 1) / CONV_BX);
    const int grid = (int)std::min<long long>(blocks, 8192);
    const int block = 64 * CONV_BY;
    if (grid <= 0) return hipSuccess;
    if (cin == 4 && cout == 16 && epi == EPI_RELU)
        k_lp_conv<4, 16, EPI_RELU><<<grid, block, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else if (cin == 16 && cout == 16 && epi == EPI_RELU)
        k_lp_conv<16, 16, EPI_RELU><<<grid, block, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else if (cin == 16 && cout == 4 && epi == EPI_LINEAR)
        k_lp_conv<16, 4, EPI_LINEAR><<<grid, block, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else if (cin == 4 && cout == 16 && epi == EPI_MASK)
        k_lp_conv<4, 16, EPI_MASK><<<grid, block, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else if (cin == 16 && cout == 16 && epi == EPI_MASK)
        k_lp_conv<16, 16, EPI_MASK><<<grid, block, 0, s>>>(nb, N, in, wt, bias, mask, pre, act);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_lp_conv_dw(int cin, int cout, int nb, int N, const bf16_t *in, const bf16_t *dout, float *pw,
                             float *pb, int grid, hipStream_t s)
{
    const int block = 64 * DW_BY;
    grid *= 3; // one workgroup per slot and dz
    if (cin == 16 && cout == 4)
        k_lp_conv_dw<16, 4><<<grid, block, 0, s>>>(nb, N, in, dout, pw, pb);
    else if (cin == 16 && cout == 16)
        k_lp_conv_dw<16, 16><<<grid, block, 0, s>>>(nb, N, in, dout, pw, pb);
    else if (cin == 4 && cout == 16)
        k_lp_conv_dw<4, 16><<<grid, block, 0, s>>>(nb, N, in, dout, pw, pb);
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
