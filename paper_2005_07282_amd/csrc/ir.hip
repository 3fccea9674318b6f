// Mixed-precision iterative refinement: the binary64 steps around the
// binary32 inner Jacobi-PCG.
//
// Outer step k: r = b - A x with every row summed exactly and rounded once,
// rr = <r, r> exactly rounded, stop when rr <= RN(RN(tol^2) <b,b>); else the
// inner solve gets rf = RN32(r 2^-s), s = floor(log2(rr) / 2) (a power of
// two, so the scaling is exact and rf has a norm near 1), from c = 0, and
// x = RN(x + c 2^s). The paper's exact dot (Section 3, 4.1) supplies rr and
// <b,b>; its long accumulator, kept per lane, supplies the row sums.
#include "reduce.hpp"
#include "sell_spmv.hpp"

namespace rpcg {

constexpr int IR_BLOCK = 128;            // two wavefronts
constexpr int IR_WAVES = IR_BLOCK / 64;
constexpr int RES_FPE = 4;                // expansion length of the row sums
constexpr int IR_DOT_P = 3;               // expansion length of <r, r>
constexpr int RES_BATCH = 9;              // row entries loaded together

// Each lane sums its row into an expansion (TwoSum, nothing lost: what does
// not fit goes into the lane's own long accumulator in LDS), then adds the
// expansion to that accumulator and rounds once. The accumulators are the
// columns of a [ACC_DIGITS][64] array per wavefront.
template <bool COL16>
__global__ void __launch_bounds__(IR_BLOCK)
k_ir_residual(SellMat<float> A, const double *__restrict__ b, const double *__restrict__ x, double *__restrict__ r,
              IrState *ist, SlotView sv)
{
    __shared__ long long lacc[IR_WAVES][ACC_DIGITS * 64];
    __shared__ RedShared sh;
    for (int k = threadIdx.x; k < IR_WAVES * ACC_DIGITS * 64; k += blockDim.x) (&lacc[0][0])[k] = 0;
    zero_acc(sh.acc[0]);
    __syncthreads();
    LaneDot<MODE_EXBLAS, IR_DOT_P> L;
    L.init();
    int flags = 0;
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(wave_id());
    WindowAcc<64> wa;
    wa.init(&lacc[wave][lane]);
    auto put = [&](double (&e)[RES_FPE], double t) {
        const double left = fpe_accumulate<RES_FPE>(e, t, true);
        if (left != 0.0) {
            if (is_finite_bits(left)) wa.add(left);
            else flags |= FLAG_NONFINITE;
        }
    };
    const long long wstride = (long long)gridDim.x * IR_WAVES;
    for (long long s = (long long)blockIdx.x * IR_WAVES + wave; s < A.nslices; s += wstride) {
        const long long base = uniform_ll(A.off[s]);
        const int width = __builtin_amdgcn_readfirstlane((int)((A.off[s + 1] - base) >> 6));
        const long long i = s * 64 + lane;
        const int len = sell_len(A, i);
        const long long p0 = base + lane; // binary32 layout: no interleave
        int first = 0, cur = 0;
        if constexpr (COL16) first = (i < A.n ? (int)i : A.n - 1) + A.cfirst[s];
        double e[RES_FPE];
#pragma unroll
        for (int j = 0; j < RES_FPE; ++j) e[j] = 0.0;
        if (i < A.n) {
            const double bi = b[i];
            if (!is_finite_bits(bi)) flags |= FLAG_NONFINITE;
            put(e, bi);
        }
        for (int k0 = 0; k0 < width; k0 += RES_BATCH) {
            int c[RES_BATCH];
            double a[RES_BATCH], g[RES_BATCH];
#pragma unroll
            for (int u = 0; u < RES_BATCH; ++u) {
                // positions past the width repeat the last entry (its column decodes unchanged: code 0)
                const int k = min(k0 + u, width - 1);
                if constexpr (COL16) {
                    const unsigned code = k0 + u < width ? __builtin_nontemporal_load(&A.col16[p0 + 64ll * k]) : 0u;
                    cur = (k0 + u == 0) ? first + (int)(short)code : cur + (int)code;
                    c[u] = cur;
                } else {
                    c[u] = __builtin_nontemporal_load(&A.col[p0 + 64ll * k]);
                }
            }
#pragma unroll
            for (int u = 0; u < RES_BATCH; ++u) {
                const int k = min(k0 + u, width - 1);
                a[u] = __builtin_nontemporal_load(&A.val64[p0 + 64ll * k]);
            }
#pragma unroll
            for (int u = 0; u < RES_BATCH; ++u) g[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < RES_BATCH; ++u) {
                if (k0 + u < len) {
                    double ph, pl;
                    two_prod(-a[u], g[u], ph, pl);
                    if (!is_finite_bits(g[u]) || !is_finite_bits(ph)) flags |= FLAG_NONFINITE;
                    else if (__builtin_fabs(ph) < 0x1p-969 && a[u] != 0.0 && g[u] != 0.0) flags |= FLAG_INEXACT;
                    put(e, ph);
                    put(e, pl);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < RES_FPE; ++j) {
            if (e[j] != 0.0) {
                if (is_finite_bits(e[j])) wa.add(e[j]);
                else flags |= FLAG_NONFINITE;
            }
        }
        const double ri = wa.round_and_clear();
        if (i < A.n) {
            r[i] = ri;
            L.add(ri, ri, sh.acc[0], true, true);
        }
    }
    if (flags) atomicOr(&ist->flags, flags);
    block_finish<MODE_EXBLAS, IR_DOT_P>(L, sh.acc[0], sv, blockIdx.x, true, true, &ist->flags, sh);
}

// floor(log2 v) of a positive finite double (subnormals included).
__device__ __forceinline__ int ilog2_pos(double v)
{
    const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
    const int be = (int)((bits >> 52) & 0x7FF);
    if (be) return be - 1023;
    return (63 - __builtin_clzll(bits & 0xFFFFFFFFFFFFFull)) - 1074;
}

// 2^e as a double, -1022 <= e <= 1023.
__device__ __forceinline__ double pow2(int e)
{
    return __builtin_bit_cast(double, (unsigned long long)(e + 1023) << 52);
}

__global__ void __launch_bounds__(MAX_BLOCK)
k_ir_prepare(int k, int maxit, double tol, int n, const double *__restrict__ r, float *__restrict__ rf,
             float *__restrict__ cvec, double *rr_hist, IrState *ist, SlotView sv, int G)
{
    __shared__ RedShared sh;
    if (wg_read_flag(&ist->stop, sh)) return;
    long long esc = 0;
    const double rr = merge_slots<MODE_EXBLAS, IR_DOT_P, double>(sv, G, true, true, sh.acc[0], &esc, &ist->flags,
                                                                 sh, 0);
    const double thr = (tol * tol) * ist->bb;
    const bool bad = (ist->flags & FLAG_NONFINITE) || !is_finite_bits(rr);
    const bool conv = !bad && rr <= thr;
    const bool out = !bad && !conv && k >= maxit;
    const bool stop = bad || conv || out;
    const int sc = (stop || !(rr > 0.0)) ? 0 : (ilog2_pos(rr) >> 1); // floor(e / 2)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ist->rr = rr;
        ist->thr = thr;
        ist->k = k;
        ist->scale = sc;
        if (rr_hist) rr_hist[k] = rr;
        if (bad) ist->status = -6;
        else if (out) ist->status = 1;
        else ist->status = 0;
        ist->stop = stop ? 1 : 0;
    }
    if (stop) return;
    // |s| <= 537, so 2^-s is a normal double and r 2^-s is exact unless it
    // falls below binary64's normal range, far below binary32's
    const double m = pow2(-sc);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        rf[i] = (float)(r[i] * m);
        cvec[i] = 0.0f;
    }
}

__global__ void k_ir_update(int n, double *__restrict__ x, const float *__restrict__ cvec, const IrState *ist)
{
    if (ist->stop) return;
    const double m = pow2(ist->scale);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double ci = (double)cvec[i] * m; // exact
        x[i] = x[i] + ci;
    }
}

hipError_t launch_ir_residual(const SellMat<float> &A, const double *b, const double *x, double *r, IrState *ist,
                              const DotWs &ws, int stride, const LaunchCfg &c)
{
    if (!A.val64 || sell_vec<float>() != 1) return hipErrorInvalidValue;
    SlotView sv{ws, stride};
    if (A.col16) k_ir_residual<true><<<c.grid, IR_BLOCK, 0, c.stream>>>(A, b, x, r, ist, sv);
    else k_ir_residual<false><<<c.grid, IR_BLOCK, 0, c.stream>>>(A, b, x, r, ist, sv);
    return hipGetLastError();
}

hipError_t launch_ir_prepare(int k, int maxit, double tol, int n, const double *r, float *rf, float *cvec,
                             double *rr_hist, IrState *ist, const DotWs &ws, int G, int stride, const LaunchCfg &c)
{
    SlotView sv{ws, stride};
    k_ir_prepare<<<c.grid, c.block, 0, c.stream>>>(k, maxit, tol, n, r, rf, cvec, rr_hist, ist, sv, G);
    return hipGetLastError();
}

hipError_t launch_ir_update(int n, double *x, const float *cvec, const IrState *ist, const LaunchCfg &c)
{
    if (n == 0) return hipSuccess;
    k_ir_update<<<c.grid, c.block, 0, c.stream>>>(n, x, cvec, ist);
    return hipGetLastError();
}

} // namespace rpcg
