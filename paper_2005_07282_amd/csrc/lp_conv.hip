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

// Implicit-GEMM convolution on gfx950's 16x16x32 bfloat16 MFMA, computing
// D[co][cell] = sum_k W[co][k] In[k][cell] for 16 output channels (rows M,
// padded) by 16 cells along x (columns N). Lane l supplies A[m = l%16][k =
// 8(l/16) + j] and B[k][n = l%16] for j < 8 and receives D[4(l/16) + j][l%16]
// for j < 4: four output channels of one cell, stored as one 8-byte unit.
//
// The weights are the A operands and stay in registers for the whole kernel.
// K runs over the taps of one input plane: for each dz, the nine (dy, dx)
// taps go in chunks of 32 = two taps of 16 input channels (five chunks, the
// last half empty) or eight taps of 4 (two chunks). A wavefront owns one
// y-line of 16 cells and a run of CONV_ZR z-planes and streams the input
// planes along z: the B operands of input plane p (read straight from memory,
// zeros outside the grid) feed the three output planes p + 1, p, p - 1
// (dz = -1, 0, +1) with that dz's weights, so each input fragment is loaded
// once per line and used three times; output plane p - 1 is complete after
// plane p and is written. No LDS, no barriers; a plane's loads are issued
// at its start and their latency is covered by the other wavefronts of the
// SIMD (about 110 registers a lane leave room for three or four; loading the
// next plane ahead would double the operand registers and halve that).
constexpr int CONV_BX = 16, CONV_HX = CONV_BX + 2; // cells along x of a line (and with the x halo)
constexpr int CONV_LINES = 4;                      // wavefronts (y-lines) per workgroup
constexpr int CONV_ZR = 16;                        // output planes per wavefront

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));

template <int CIN>
__host__ __device__ constexpr int conv_chunks() { return CIN == 16 ? 5 : 2; }

// Tap (dy, dx) of entry e < 9 of the nine taps of a plane (row-major in dy, dx).
__device__ __forceinline__ int tap9_dy(int e) { return e / 3 - 1; }
__device__ __forceinline__ int tap9_dx(int e) { return e % 3 - 1; }

// Taps of chunk q held by operand lanes of group kb: CIN = 16, tap e =
// 2q + kb/2, channels 8(kb%2) .. + 7; CIN = 4, taps e = 8q + 2kb and
// 8q + 2kb + 1, channels 0 .. 3 of each. e >= 9 is an empty half.
template <int CIN>
__device__ __forceinline__ int chunk_tap(int q, int kb, int h)
{
    return CIN == 16 ? 2 * q + (kb >> 1) : 8 * q + 2 * kb + h;
}

// A operands: W[t][co][ci] of the chunk's taps in the dz plane dzi (0, 1, 2
// for dz = -1, 0, +1), zeros for empty halves.
template <int CIN>
__device__ __forceinline__ v8s load_wchunk(const bf16_t *__restrict__ wt, int dzi, int q, int co, int kb)
{
    v8s a = {0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (CIN == 16) {
        const int e = chunk_tap<16>(q, kb, 0);
        if (e < 9) a = *(const v8s *)(wt + ((9 * dzi + e) * 16 + co) * 16 + 8 * (kb & 1));
    } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = chunk_tap<4>(q, kb, h);
            if (e < 9) {
                const v4s w = *(const v4s *)(wt + ((9 * dzi + e) * 16 + co) * 4);
#pragma unroll
                for (int j = 0; j < 4; ++j) a[4 * h + j] = w[j];
            }
        }
    }
    return a;
}

// B operands of input plane z for the line (x0 + n, y): the chunk's taps at
// (x0 + n + dx, y + dy, z), zeros outside the grid or for empty halves.
template <int CIN>
__device__ __forceinline__ void load_bplane(v8s (&bq)[conv_chunks<CIN>()], const bf16_t *__restrict__ inb, int N,
                                            int x0, int y, int z, int n, int kb)
{
    const bool zin = z >= 0 && z < N;
#pragma unroll
    for (int q = 0; q < conv_chunks<CIN>(); ++q) {
        v8s b = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int h = 0; h < (CIN == 16 ? 1 : 2); ++h) {
            const int e = chunk_tap<CIN>(q, kb, h);
            const int X = x0 + n + tap9_dx(e), Y = y + tap9_dy(e);
            if (e < 9 && zin && X >= 0 && X < N && Y >= 0 && Y < N) {
                const long long cell = ((long long)z * N + Y) * N + X;
                if constexpr (CIN == 16) {
                    b = *(const v8s *)(inb + cell * 16 + 8 * (kb & 1));
                } else {
                    const v4s v = *(const v4s *)(inb + cell * 4);
#pragma unroll
                    for (int j = 0; j < 4; ++j) b[4 * h + j] = v[j];
                }
            }
        }
        bq[q] = b;
    }
}

template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(64 * CONV_LINES) k_lp_conv(int nb, int N, const bf16_t *__restrict__ in,
                                                             const bf16_t *__restrict__ wt,
                                                             const float *__restrict__ bias,
                                                             const bf16_t *__restrict__ mask, float *__restrict__ pre,
                                                             bf16_t *__restrict__ act)
{
    constexpr int NCH = conv_chunks<CIN>();
    const int lane = threadIdx.x & 63, kb = lane >> 4, n = lane & 15;
    const int wave = threadIdx.x >> 6;
    // tiles (system, z-run, x-tile, y-group), y-group fastest; each XCD takes a
    // contiguous range of them when the count allows (neighbours share its L2)
    const int tiles_x = (N + CONV_BX - 1) / CONV_BX, tiles_y = (N + CONV_LINES - 1) / CONV_LINES;
    const int runs = (N + CONV_ZR - 1) / CONV_ZR;
    const long long ntiles = (long long)nb * runs * tiles_x * tiles_y;
    long long tile = blockIdx.x;
    if (ntiles % 8 == 0) tile = (tile % 8) * (ntiles / 8) + tile / 8;
    const int ty = (int)(tile % tiles_y);
    long long r = tile / tiles_y;
    const int tx = (int)(r % tiles_x);
    r /= tiles_x;
    const int zr = (int)(r % runs);
    const long long b = r / runs;
    const int x0 = tx * CONV_BX, y = ty * CONV_LINES + wave, z0 = zr * CONV_ZR;
    const int z1 = min(z0 + CONV_ZR, N);
    if (y >= N) return; // wavefront-uniform; no barriers in this kernel
    const long long N3 = (long long)N * N * N;
    const bf16_t *__restrict__ inb = in + b * N3 * CIN;
    v8bf w[3][NCH];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < NCH; ++q) w[d][q] = __builtin_bit_cast(v8bf, load_wchunk<CIN>(wt, d, q, n, kb));
    float bv[4] = {0.f, 0.f, 0.f, 0.f};
    if (EPI != EPI_MASK && 4 * kb < COUT)
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = bias[4 * kb + j];
    const int x = x0 + n;
    v4f a_prev = {0.f, 0.f, 0.f, 0.f}, a_cur = a_prev, a_next = a_prev; // outputs p - 1, p, p + 1
    for (int p = z0 - 1; p <= z1; ++p) {
        v8s bq[NCH];
        load_bplane<CIN>(bq, inb, N, x0, y, p, n, kb);
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
            const v8bf bb = __builtin_bit_cast(v8bf, bq[q]);
            a_next = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[0][q], bb, a_next, 0, 0, 0); // dz = -1: output p + 1
            a_cur = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[1][q], bb, a_cur, 0, 0, 0);   // dz = 0: output p
            a_prev = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[2][q], bb, a_prev, 0, 0, 0); // dz = +1: output p - 1
        }
        const int z = p - 1; // complete
        if (z >= z0 && x < N && 4 * kb < COUT) {
            const long long cell = b * N3 + ((long long)z * N + y) * N + x;
            if (EPI == EPI_RELU) {
                v4s o;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float v = a_prev[j] + bv[j];
                    o[j] = (short)f32_to_bf16(v > 0.f ? v : 0.f);
                }
                *(v4s *)(act + cell * COUT + 4 * kb) = o;
                if (pre)
                    *(v4f *)(pre + cell * COUT + 4 * kb) =
                        (v4f){a_prev[0] + bv[0], a_prev[1] + bv[1], a_prev[2] + bv[2], a_prev[3] + bv[3]};
            } else if (EPI == EPI_LINEAR) {
                *(v4f *)(pre + cell * COUT + 4 * kb) =
                    (v4f){a_prev[0] + bv[0], a_prev[1] + bv[1], a_prev[2] + bv[2], a_prev[3] + bv[3]};
            } else {
                // the relu of the forward layer was active where its stored
                // (bfloat16) activation is nonzero
                const v4s mk = *(const v4s *)(mask + cell * COUT + 4 * kb);
                v4s o;
#pragma unroll
                for (int j = 0; j < 4; ++j) o[j] = (short)f32_to_bf16(mk[j] != 0 ? a_prev[j] : 0.f);
                *(v4s *)(act + cell * COUT + 4 * kb) = o;
            }
        }
        a_prev = a_cur;
        a_cur = a_next;
        a_next = (v4f){0.f, 0.f, 0.f, 0.f};
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
    const long long tiles = (long long)nb * ((N + CONV_ZR - 1) / CONV_ZR) * ((N + CONV_BX - 1) / CONV_BX) *
                            ((N + CONV_LINES - 1) / CONV_LINES);
    if (tiles <= 0) return hipSuccess;
    if (tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
    const int grid = (int)tiles;
    const int block = 64 * CONV_LINES;
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
