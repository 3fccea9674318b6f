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
constexpr int CONV_BX = 16;    // cells along x of a line
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

// Weight gradient dW[t][co][ci] = sum over cells of dout[cell][co] in[cell + off(t)][ci]
// and bias gradient db[co] = sum of dout[cell][co], on 16x16x32 MFMA with
// M = co, N = ci and K = 32 cells along x: lane l supplies dout at cells
// 8(l/16) + j of channel l%16 (A) and the input at the same cells shifted by
// the tap, channel l%16 (B). A workgroup is three wavefronts, one per dz,
// each holding the nine tap tiles of its plane, and walks its items (system,
// z-run, y-line, 32-cell x-segment) one z-plane at a time. Per plane it
// stages, with 16-byte loads, the dout row of the plane and the three input
// rows y - 1 .. y + 1 of the next plane into a ring of three planes in LDS
// (zeros outside the grid), so every input row is loaded once and read by
// the three wavefronts (dz = -1, 0, +1 read the planes z - 1, z, z + 1); the
// loads of the next plane go to registers under the current plane's
// products and are written to LDS at the start of the next step. The
// operands are then gathered from LDS as 16-bit values: per input row a lane
// reads the ten cells x - 1 .. x + 8 around its eight and forms the three dx
// fragments from them. Every eighth staged cell is followed by a gap of one
// cell (16 channels), so the four k-groups of a gather fall in different
// banks. Each wavefront writes its nine taps to the workgroup's slot; the
// slots are summed in a fixed order later.
constexpr int DW_SEG = 32; // cells along x per item (the K of one product)
constexpr int DW_ZR = 64;  // z-planes per item
constexpr int DW_XC = DW_SEG + 2; // staged input cells per row

// Byte offset of staged cell c in a row of cells of C channels.
template <int C>
__host__ __device__ constexpr int dw_cell(int c) { return C == 16 ? (c + (c >> 3)) * 32 : c * 8; }
template <int C>
__host__ __device__ constexpr int dw_row_bytes(int cells) { return dw_cell<C>(cells); }

// Stage `cells` cells of row (Z, Y) from x = X0 on (zeros outside the grid)
// at dst, with all threads of the workgroup; 16-byte units (8 channels), or
// one 8-byte unit per cell for 4 channels.
template <int C>
__device__ __forceinline__ void dw_stage_row(unsigned char *dst, const bf16_t *__restrict__ src, int N, int Z, int Y,
                                             int X0, int cells, int first, int stride)
{
    constexpr int UPC = C == 16 ? 2 : 1;
    const bool row_in = Z >= 0 && Z < N && Y >= 0 && Y < N;
    for (int u = first; u < cells * UPC; u += stride) {
        const int c = u / UPC, q = u % UPC, X = X0 + c;
        const bool in = row_in && X >= 0 && X < N;
        const long long cell = ((long long)Z * N + Y) * N + X;
        if constexpr (C == 16) {
            v8s v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (in) v = *(const v8s *)(src + cell * 16 + 8 * q);
            *(v8s *)(dst + dw_cell<16>(c) + 16 * q) = v;
        } else {
            v4s v = {0, 0, 0, 0};
            if (in) v = *(const v4s *)(src + cell * 4);
            *(v4s *)(dst + dw_cell<4>(c)) = v;
        }
    }
}

// The same staging in two halves: dw_load_row reads the units thread
// `first` owns (at most K of them) into registers, dw_store_row writes them
// to LDS, so the loads of the next plane can run under the current plane's
// products.
template <int C, int K>
__device__ __forceinline__ void dw_load_row(v8s (&reg)[K], const bf16_t *__restrict__ src, int N, int Z, int Y, int X0,
                                            int cells, int first, int stride)
{
    constexpr int UPC = C == 16 ? 2 : 1;
    const bool row_in = Z >= 0 && Z < N && Y >= 0 && Y < N;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int u = first + k * stride;
        const int c = u / UPC, q = u % UPC, X = X0 + c;
        const bool in = row_in && u < cells * UPC && X >= 0 && X < N;
        const long long cell = ((long long)Z * N + Y) * N + X;
        v8s v = {0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (C == 16) {
            if (in) v = *(const v8s *)(src + cell * 16 + 8 * q);
        } else {
            if (in) {
                const v4s w = *(const v4s *)(src + cell * 4);
                v[0] = w[0]; v[1] = w[1]; v[2] = w[2]; v[3] = w[3];
            }
        }
        reg[k] = v;
    }
}

template <int C, int K>
__device__ __forceinline__ void dw_store_row(unsigned char *dst, const v8s (&reg)[K], int cells, int first, int stride)
{
    constexpr int UPC = C == 16 ? 2 : 1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int u = first + k * stride;
        if (u >= cells * UPC) break;
        const int c = u / UPC, q = u % UPC;
        if constexpr (C == 16) {
            *(v8s *)(dst + dw_cell<16>(c) + 16 * q) = reg[k];
        } else {
            *(v4s *)(dst + dw_cell<4>(c)) = (v4s){reg[k][0], reg[k][1], reg[k][2], reg[k][3]};
        }
    }
}

template <int CIN, int COUT>
__global__ void __launch_bounds__(192) k_lp_conv_dw(int nb, int N, const bf16_t *__restrict__ in,
                                                    const bf16_t *__restrict__ dout, float *__restrict__ pw,
                                                    float *__restrict__ pb)
{
    constexpr int RB = dw_row_bytes<CIN>(DW_XC), DB = dw_row_bytes<COUT>(DW_SEG);
    __shared__ __attribute__((aligned(16))) unsigned char ring[3][3][RB]; // [plane slot][dy][row]
    __shared__ __attribute__((aligned(16))) unsigned char drow[DB];
    const int lane = threadIdx.x & 63, kb = lane >> 4, c16 = lane & 15;
    const int dzi = threadIdx.x >> 6;
    const int segs = (N + DW_SEG - 1) / DW_SEG, runs = (N + DW_ZR - 1) / DW_ZR;
    const long long items = (long long)nb * runs * N * segs;
    const long long N3 = (long long)N * N * N;
    v4f acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) { // workgroup-uniform
        const int seg = (int)(it % segs);
        long long r = it / segs;
        const int y = (int)(r % N);
        r /= N;
        const int zr = (int)(r % runs);
        const long long b = r / runs;
        const int x0 = seg * DW_SEG;
        const bf16_t *__restrict__ Db = dout + b * N3 * COUT;
        const bf16_t *__restrict__ Ib = in + b * N3 * CIN;
        const int z0 = zr * DW_ZR, z1 = min(z0 + DW_ZR, N);
        __syncthreads(); // the previous item's readers are done
        for (int p = z0 - 1; p <= z0; ++p)
            for (int dy = 0; dy < 3; ++dy)
                dw_stage_row<CIN>(ring[(p + 3) % 3][dy], Ib, N, p, y + dy - 1, x0 - 1, DW_XC, threadIdx.x, 192);
        // registers for the next plane's input rows and dout row (loaded one plane ahead)
        constexpr int KI = (DW_XC * (CIN == 16 ? 2 : 1) + 191) / 192, KD = (DW_SEG * (COUT == 16 ? 2 : 1) + 191) / 192;
        v8s ri[3][KI], rd[KD];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) dw_load_row<CIN, KI>(ri[dy], Ib, N, z0 + 1, y + dy - 1, x0 - 1, DW_XC, threadIdx.x, 192);
        dw_load_row<COUT, KD>(rd, Db, N, z0, y, x0, DW_SEG, threadIdx.x, 192);
        for (int z = z0; z < z1; ++z) {
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) dw_store_row<CIN, KI>(ring[(z + 4) % 3][dy], ri[dy], DW_XC, threadIdx.x, 192);
            dw_store_row<COUT, KD>(drow, rd, DW_SEG, threadIdx.x, 192);
            if (z + 1 < z1) {
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
                    dw_load_row<CIN, KI>(ri[dy], Ib, N, z + 2, y + dy - 1, x0 - 1, DW_XC, threadIdx.x, 192);
                dw_load_row<COUT, KD>(rd, Db, N, z + 1, y, x0, DW_SEG, threadIdx.x, 192);
            }
            __syncthreads();
            // A: dout at cells 8 kb + j of channel c16
            v8s a = {0, 0, 0, 0, 0, 0, 0, 0};
            if (c16 < COUT) {
#pragma unroll
                for (int j = 0; j < 8; ++j) a[j] = *(const short *)(drow + dw_cell<COUT>(8 * kb + j) + 2 * c16);
            }
            if (dzi == 1) {
#pragma unroll
                for (int j = 0; j < 8; ++j) bsum += bf16_to_f32((bf16_t)a[j]);
            }
            const v8bf av = __builtin_bit_cast(v8bf, a);
            const unsigned char(*pl)[RB] = ring[(z + dzi + 2) % 3]; // plane z + dz
#pragma unroll
            for (int dyi = 0; dyi < 3; ++dyi) {
                // staged cells 8 kb .. 8 kb + 9 = x - 1 .. x + 8 of channel c16
                short v[10];
#pragma unroll
                for (int m = 0; m < 10; ++m)
                    v[m] = c16 < CIN ? *(const short *)(pl[dyi] + dw_cell<CIN>(8 * kb + m) + 2 * c16) : (short)0;
#pragma unroll
                for (int dxi = 0; dxi < 3; ++dxi) {
                    v8s bq;
#pragma unroll
                    for (int j = 0; j < 8; ++j) bq[j] = v[j + dxi];
                    acc[3 * dyi + dxi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(v8bf, bq),
                                                                                acc[3 * dyi + dxi], 0, 0, 0);
                }
            }
            __syncthreads(); // readers done before the next plane is staged
        }
    }
    // lane l holds dW[9 dzi + t][co = 4(l/16) + j][ci = l%16]
    float *__restrict__ dst = pw + ((long long)blockIdx.x * LP_TAPS + 9 * dzi) * 256;
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) dst[(t * 16 + 4 * kb + j) * 16 + c16] = acc[t][j];
    if (dzi == 1) {
        // lane (co, kb) holds the bias partial of cells 8 kb .. 8 kb + 7: sum over kb in order
        const float p1 = __shfl(bsum, c16 + 16, 64), p2 = __shfl(bsum, c16 + 32, 64), p3 = __shfl(bsum, c16 + 48, 64);
        const float tot = ((bsum + p1) + p2) + p3;
        if (kb == 0) pb[blockIdx.x * 16 + c16] = tot;
    }
}

// Gradient of one layer from the slots in a fixed order: thread group g of
// an element sums the slots g, g + 16, ... in increasing order, then the 16
// group sums are added in group order. Weights in the [tap][out][in] layout
// of the parameters (the slots hold [tap][16][16]), then the bias.
__global__ void __launch_bounds__(256) k_lp_reduce(int nslots, int cout, int cin, const float *__restrict__ pw,
                                                   const float *__restrict__ pb, float *__restrict__ gw,
                                                   float *__restrict__ gb)
{
    __shared__ float part[16][17];
    const int nw = LP_TAPS * cout * cin;
    const int e = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + e;
    float s = 0.f;
    if (i < nw) {
        const int t = i / (cout * cin), o = (i / cin) % cout, c = i % cin;
        const int src = (t * 16 + o) * 16 + c;
#pragma unroll 8
        for (int k = g; k < nslots; k += 16) s += pw[(long long)k * LP_TAPS * 256 + src];
    } else if (i < nw + cout) {
#pragma unroll 8
        for (int k = g; k < nslots; k += 16) s += pb[k * 16 + (i - nw)];
    }
    part[g][e] = s;
    __syncthreads();
    if (g == 0 && i < nw + cout) {
        float tot = 0.f;
        for (int q = 0; q < 16; ++q) tot += part[q][e];
        if (i < nw) gw[i] = tot;
        else gb[i - nw] = tot;
    }
}

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
    const int block = 192; // one wavefront per dz
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
    k_lp_reduce<<<(len + 15) / 16, 256, 0, s>>>(nslots, cout, cin, pw, pb, gw, gb);
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
