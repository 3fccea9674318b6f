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

// Implicit-GEMM convolution on gfx950's 16x16x32 bfloat16 MFMA. A wavefront
// computes tiles of 16 cells along x (rows M) by 16 output channels (columns
// N); K runs over (tap, input channel) in chunks of 32: two taps of 16 input
// channels, or eight taps of 4. Lane l supplies A[m = l%16][k = 8(l/16) + j]
// and B[k][n = l%16] for j < 8 and receives D[4(l/16) + j][l%16] for j < 4.
//
// A workgroup of four wavefronts takes a block of 16 x 4 x 2 output cells
// (one y-line and two z-planes per wavefront: two independent accumulator
// chains) and first stages the block's inputs with their halo (18 x 6 x 4
// cells, zeros outside the grid) in LDS with coalesced loads, so each input
// is fetched from memory once per block. The weights are packed once per
// workgroup in the B-operand order, 16 bytes per lane and chunk.
constexpr int CONV_BX = 16, CONV_BY = 4, CONV_BZ = 2;          // block of output cells (x, y, z)
constexpr int CONV_HX = CONV_BX + 2, CONV_HY = CONV_BY + 2, CONV_HZ = CONV_BZ + 2; // with halo
constexpr int CONV_HCELLS = CONV_HX * CONV_HY * CONV_HZ;

template <int CIN>
__host__ __device__ constexpr int conv_chunks() { return CIN == 16 ? 14 : 4; }

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));

// Stage the inputs of the block at (x0, y0, z0) of one system with its
// halo: the 8 channels of group q of halo cell c at tile[(q * HC + c) * 8]
// (CIN = 16, two groups), or the 4 channels of cell c at tile[c * 4] (CIN =
// 4). Consecutive threads take consecutive 16- or 8-byte units along x, so
// a wavefront reads whole runs of the input.
template <int CIN>
__device__ __forceinline__ void stage_block(bf16_t *tile, const bf16_t *__restrict__ inb, int N, int x0, int y0, int z0)
{
    constexpr int Q = CIN == 16 ? 2 : 1, HC = CONV_HCELLS;
    for (int u = threadIdx.x; u < HC * Q; u += blockDim.x) {
        const int q = u % Q, cell = u / Q;
        const int xc = cell % CONV_HX, yc = (cell / CONV_HX) % CONV_HY, zc = cell / (CONV_HX * CONV_HY);
        const int X = x0 - 1 + xc, Y = y0 - 1 + yc, Z = z0 - 1 + zc;
        const bool in = X >= 0 && X < N && Y >= 0 && Y < N && Z >= 0 && Z < N;
        const long long src = (((long long)Z * N + Y) * N + X) * CIN;
        if constexpr (CIN == 16) {
            v8s v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (in) v = *(const v8s *)(inb + src + 8 * q);
            *(v8s *)&tile[(q * HC + cell) * 8] = v;
        } else {
            v4s v = {0, 0, 0, 0};
            if (in) v = *(const v4s *)(inb + src);
            *(v4s *)&tile[cell * 4] = v;
        }
    }
}

// Halo cell of output cell (m, wave line, plane zo) shifted by tap t.
__device__ __forceinline__ int halo_cell(int t, int m, int wave, int zo)
{
    int dz, dy, dx;
    tap_offset(t, dz, dy, dx);
    return ((zo + dz + 1) * CONV_HY + (wave + dy + 1)) * CONV_HX + (m + dx + 1);
}

template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(64 * CONV_BY) k_lp_conv(int nb, int N, const bf16_t *__restrict__ in,
                                                          const bf16_t *__restrict__ wt, const float *__restrict__ bias,
                                                          const bf16_t *__restrict__ mask, float *__restrict__ pre,
                                                          bf16_t *__restrict__ act)
{
    constexpr int NCH = conv_chunks<CIN>();
    // B operands: wp[((c * 4 + kb) * 16 + co) * 8 + j] = W[tap][co][ci] of k = 8 kb + j in chunk c
    __shared__ __attribute__((aligned(16))) bf16_t wp[NCH * 4 * 16 * 8];
    __shared__ __attribute__((aligned(16))) bf16_t tile[CONV_HCELLS * CIN];
    for (int u = threadIdx.x; u < NCH * 4 * 16 * 8; u += blockDim.x) {
        const int j = u & 7, co = (u >> 3) & 15, kb = (u >> 7) & 3, c = u >> 9;
        int t, ci;
        if (CIN == 16) { t = 2 * c + (kb >> 1); ci = 8 * (kb & 1) + j; }
        else { t = 8 * c + 2 * kb + (j >> 2); ci = j & 3; }
        wp[u] = t < LP_TAPS ? wt[(t * 16 + co) * CIN + ci] : (bf16_t)0;
    }
    const int lane = threadIdx.x & 63, kb = lane >> 4, m = lane & 15;
    const int wave = threadIdx.x >> 6;
    const int tiles_x = (N + CONV_BX - 1) / CONV_BX, tiles_y = (N + CONV_BY - 1) / CONV_BY;
    const int tiles_z = (N + CONV_BZ - 1) / CONV_BZ;
    const long long nblocks = (long long)nb * tiles_z * tiles_y * tiles_x;
    const long long N3 = (long long)N * N * N;
    for (long long blk = blockIdx.x; blk < nblocks; blk += gridDim.x) { // workgroup-uniform
        const int tx = (int)(blk % tiles_x);
        long long r = blk / tiles_x;
        const int ty = (int)(r % tiles_y);
        r /= tiles_y;
        const int tz = (int)(r % tiles_z);
        const long long b = r / tiles_z;
        const int x0 = tx * CONV_BX, y0 = ty * CONV_BY, z0 = tz * CONV_BZ;
        __syncthreads(); // the previous block's readers are done (and the weights are in place)
        stage_block<CIN>(tile, in + b * N3 * CIN, N, x0, y0, z0);
        __syncthreads();
        const int y = y0 + wave;
        if (y >= N) continue; // wavefront-uniform; the loop's barrier comes first in the next block
        v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
        for (int c = 0; c < NCH; ++c) {
            const v8bf bw = __builtin_bit_cast(v8bf, *(const v8s *)&wp[((c * 4 + kb) * 16 + m) * 8]);
            v8s a0 = {0, 0, 0, 0, 0, 0, 0, 0}, a1 = a0;
            if constexpr (CIN == 16) {
                const int t = 2 * c + (kb >> 1);
                if (t < LP_TAPS) { // rows m past the grid's edge read valid LDS cells; their outputs are not stored
                    a0 = *(const v8s *)&tile[((kb & 1) * CONV_HCELLS + halo_cell(t, m, wave, 0)) * 8];
                    a1 = *(const v8s *)&tile[((kb & 1) * CONV_HCELLS + halo_cell(t, m, wave, 1)) * 8];
                }
            } else {
                const int t = 8 * c + 2 * kb;
                if (t < LP_TAPS) {
                    const v4s p0 = *(const v4s *)&tile[halo_cell(t, m, wave, 0) * 4];
                    const v4s p1 = *(const v4s *)&tile[halo_cell(t, m, wave, 1) * 4];
                    a0[0] = p0[0]; a0[1] = p0[1]; a0[2] = p0[2]; a0[3] = p0[3];
                    a1[0] = p1[0]; a1[1] = p1[1]; a1[2] = p1[2]; a1[3] = p1[3];
                }
                if (t + 1 < LP_TAPS) {
                    const v4s p0 = *(const v4s *)&tile[halo_cell(t + 1, m, wave, 0) * 4];
                    const v4s p1 = *(const v4s *)&tile[halo_cell(t + 1, m, wave, 1) * 4];
                    a0[4] = p0[0]; a0[5] = p0[1]; a0[6] = p0[2]; a0[7] = p0[3];
                    a1[4] = p1[0]; a1[5] = p1[1]; a1[6] = p1[2]; a1[7] = p1[3];
                }
            }
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a0), bw, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a1), bw, acc1, 0, 0, 0);
        }
        const int co = m;
        if (co < COUT) {
#pragma unroll
            for (int zo = 0; zo < CONV_BZ; ++zo) {
                const int z = z0 + zo;
                if (z >= N) continue;
                const v4f acc = zo ? acc1 : acc0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int x = x0 + 4 * kb + j;
                    if (x >= N) continue;
                    const long long cell = b * N3 + ((long long)z * N + y) * N + x;
                    const float v = acc[j];
                    if (EPI == EPI_RELU) {
                        const float p = v + bias[co];
                        if (pre) pre[cell * COUT + co] = p;
                        act[cell * COUT + co] = f32_to_bf16(p > 0.f ? p : 0.f);
                    } else if (EPI == EPI_LINEAR) {
                        pre[cell * COUT + co] = v + bias[co];
                    } else {
                        // the relu of the forward layer was active where its stored
                        // (bfloat16) activation is nonzero
                        act[cell * COUT + co] = f32_to_bf16(mask[cell * COUT + co] != 0 ? v : 0.f);
                    }
                }
            }
        }
    }
}

// Weight gradients: the staged inputs are kept in groups of four channels: group q of cell c
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
                          const float *bias, const bf16_t *mask, float *pre, bf16_t *act, hipStream_t s)
{
    const long long blocks = (long long)nb * ((N + CONV_BZ - 1) / CONV_BZ) * ((N + CONV_BY - 1) / CONV_BY) *
                             ((N + CONV_BX - 1) / CONV_BX);
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
