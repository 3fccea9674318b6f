// Device-side reduction machinery shared by the kernel translation units:
// per-lane accumulators, workgroup partials, the merge of workgroup partials
// and the correctly rounded conversion of a long accumulator.
//
// Reduction structure (Section 3.2 / 4.3 mapped onto one GPU): each lane
// keeps its own accumulator (an expansion, or a plain sum); the lanes of a
// workgroup combine into one workgroup partial written to a slot: a plain
// sum in a fixed tree, or, in both exact modes, a long accumulator in LDS.
// In EXBLAS mode each wavefront adds its lanes' expansions to it word by
// word as exact integer sums; in FPE mode each wavefront's expansions are
// first merged in a fixed lane tree whose escapes are counted (Section 4.3),
// and the merged expansion is added exactly. The kernel that
// needs the scalar next merges all slots in a fixed order at its start, in
// every workgroup alike, and rounds once; the kernel boundary makes the slots
// visible, so no device-scope fence or atomic ticket is needed inside the
// producing kernel (on multi-XCD gfx950 a per-workgroup release fence writes
// back the XCD's L2 and serialises the workgroups). This replaces the paper's
// MPI_Reduce + Round + MPI_Bcast: every consumer computes the same rounded
// scalar from the same integers.
#pragma once

#include "kernels.hpp"
#include "numerics.hpp"

#include <type_traits>

namespace rpcg {

static_assert(ACC_WORDS == ACC_DIGITS, "accumulator size mismatch");

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ int num_waves() { return blockDim.x >> 6; }

// Lane 0 receives the sum of the wavefront (fixed pairing: lane l adds lane l+off).
template <typename T>
__device__ __forceinline__ T wave_sum_down(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Shared memory of the reduction machinery for up to three dots per kernel.
struct RedShared {
    long long acc[3][ACC_DIGITS]; // long accumulators
    long long red_ll[MAX_WAVES];
    double part[MAX_WAVES];
    int rng[2];
    int rng2[2];
    int flag;
    double val[3];
};

// Workgroup-uniform read of a flag that workgroup 0 of the same kernel may
// set while this workgroup runs: one thread reads, every thread sees its value.
__device__ __forceinline__ bool wg_read_flag(const int *p, RedShared &sh)
{
    if (threadIdx.x == 0) sh.flag = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return sh.flag != 0;
}

__device__ __forceinline__ void acc_add_lds(long long *acc, double v, int &flags)
{
    if (v == 0.0) return;
    if (!is_finite_bits(v)) { flags |= FLAG_NONFINITE; return; }
    AccChunks c = acc_chunks(v);
    if (c.c0) atomicAdd((unsigned long long *)&acc[c.k], (unsigned long long)c.c0);
    if (c.c1) atomicAdd((unsigned long long *)&acc[c.k + 1], (unsigned long long)c.c1);
    if (c.c2) atomicAdd((unsigned long long *)&acc[c.k + 2], (unsigned long long)c.c2);
}

// Exact product x y added to the long accumulator as one integer: the
// 106-bit product of the significands, negated once as a 128-bit two's
// complement value if the signs differ, shifted onto the accumulator's word
// grid and added as four unsigned 32-bit digits and the signed rest above
// them (five adds at most, each below 2^32 in magnitude). It is the same
// exact value as RN(x y) plus its TwoProd error, added with one atomic
// fewer on average. The caller
// ensures RN(x y) is finite and at least 2^-969 in magnitude: then x and y
// are finite and nonzero, TwoProd is exact, and the product's bits lie
// between the accumulator's lowest weight and its top word.
__device__ __forceinline__ void acc_add_product_lds(long long *acc, double x, double y)
{
    const unsigned long long bx = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long by = __builtin_bit_cast(unsigned long long, y);
    int ex = (int)((bx >> 52) & 0x7FF), ey = (int)((by >> 52) & 0x7FF);
    unsigned long long mx = bx & 0xFFFFFFFFFFFFFull, my = by & 0xFFFFFFFFFFFFFull;
    if (ex) mx |= 1ull << 52;
    else ex = 1;
    if (ey) my |= 1ull << 52;
    else ey = 1;
    // x y = mx my 2^(ex + ey - 2150); off = offset of its last bit above 2^ACC_EXP0
    const int off = ex + ey - 2150 - ACC_EXP0;
    const int k = off >> 5, s = off & 31;
    // schoolbook on 32-bit halves (the high halves are below 2^21): four
    // 32 x 32 -> 64 products, the middle sum below 2^55
    const unsigned xl = (unsigned)mx, xh = (unsigned)(mx >> 32), yl = (unsigned)my, yh = (unsigned)(my >> 32);
    const unsigned long long p0 = (unsigned long long)xl * yl;
    unsigned long long mid = (unsigned long long)xl * yh + (p0 >> 32);
    mid += (unsigned long long)xh * yl;
    unsigned long long lo = (p0 & 0xFFFFFFFFull) | (mid << 32);
    unsigned long long hi = (unsigned long long)xh * yh + (mid >> 32); // hi < 2^42
    // the signed product as a 128-bit two's complement value (hi now signed)
    const bool neg = ((bx ^ by) >> 63) != 0;
    if (neg) {
        const unsigned long long nlo = 0ull - lo;
        hi = ~hi + (lo == 0 ? 1ull : 0ull);
        lo = nlo;
    }
    // shifted by s onto the word grid: 32-bit digits of the low 128 bits
    // (unsigned) and the signed rest above them
    const unsigned long long w0 = lo << s;
    const unsigned long long w1 = (hi << s) | (s ? lo >> (64 - s) : 0ull);
    const long long w2 = s ? (long long)hi >> (64 - s) : ((long long)hi >> 63);
    const long long c[5] = {(long long)(w0 & 0xFFFFFFFFull), (long long)(w0 >> 32), (long long)(w1 & 0xFFFFFFFFull),
                            (long long)(w1 >> 32), w2};
#pragma unroll
    for (int i = 0; i < 5; ++i)
        if (c[i]) atomicAdd((unsigned long long *)&acc[k + i], (unsigned long long)c[i]);
}

__device__ __forceinline__ bool product_in_integer_range(double r)
{
    return is_finite_bits(r) && __builtin_fabs(r) >= 0x1p-969;
}

// The same condition decided from the biased exponents alone (sufficient, not
// necessary): for normal x and y, |x y| lies in [2^(ex+ey-2046), 2^(ex+ey-2044)),
// so ex + ey >= 1077 gives |RN(x y)| >= 2^-969 and ex + ey <= 3067 keeps it
// at most 2^1023.
__device__ __forceinline__ bool product_exponents_in_range(double x, double y)
{
    const int ex = (int)((__builtin_bit_cast(unsigned long long, x) >> 52) & 0x7FF);
    const int ey = (int)((__builtin_bit_cast(unsigned long long, y) >> 52) & 0x7FF);
    const int e = ex + ey;
    return ex != 0 && ey != 0 && ex != 0x7FF && ey != 0x7FF && e >= 1077 && e <= 3067;
}

// Per-lane accumulator of one dot product.
//
// EXBLAS (Section 4.1, Listing 1): the TwoProd result and error go into one
// expansion; what an expansion cannot hold is flushed into the workgroup's
// long accumulator, so nothing is lost.
// FPE (Section 4.2): two expansions, results and errors. A nonzero remainder
// after the last level is an "escape" (the capacity warning of Section 4.3);
// it is counted and, with `capture`, added to the long accumulator so the
// result stays exact; without `capture` it is dropped as in the paper.
// PLAIN: an fma running sum.
//
// ADAPT (standalone dot): when the expansion keeps overflowing (wide exponent
// ranges, where nearly every product leaves a remainder), the lane adds
// the exact products straight into the long accumulator for a while and
// skips the expansion arithmetic that would not have absorbed them; one
// window in eight measures the overflow rate again. Either path adds the
// exact products, so the result does not depend on the switching.
constexpr int ADAPT_WINDOW = 32;   // adds per measurement window
constexpr int ADAPT_DIRECT = 7;    // windows in direct mode before measuring again

template <int MODE, int P, bool ADAPT = false>
struct LaneDot {
    double a[P];
    double e[P];
    double s;
    int esc;
    int flags;
    int win, wfl, direct; // ADAPT: adds and flushes in this window, direct windows left

    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int i = 0; i < P; ++i) { a[i] = 0.0; e[i] = 0.0; }
        s = 0.0;
        esc = 0;
        flags = 0;
        win = wfl = direct = 0;
    }

    // ADAPT: end of one add of the measurement window
    __device__ __forceinline__ void adapt_tick()
    {
        if (++win == ADAPT_WINDOW) {
            // more than one flush per add on average: go direct
            direct = direct ? direct - 1 : (wfl > ADAPT_WINDOW ? ADAPT_DIRECT : 0);
            win = wfl = 0;
        }
    }

    __device__ __forceinline__ void add(double x, double y, long long *acc, bool ee, bool capture)
    {
        if constexpr (MODE == MODE_PLAIN) {
            s = __builtin_fma(x, y, s);
        } else if (MODE == MODE_EXBLAS && ADAPT && direct && product_exponents_in_range(x, y)) {
            // direct mode, product in range by its exponents: no TwoProd needed
            acc_add_product_lds(acc, x, y);
            adapt_tick();
        } else {
            double r, t;
            two_prod(x, y, r, t);
            if (__builtin_fabs(r) < 0x1p-969 && x != 0.0 && y != 0.0) flags |= FLAG_INEXACT;
            if constexpr (MODE == MODE_EXBLAS && ADAPT) {
                if (direct) {
                    if (product_in_integer_range(r)) {
                        acc_add_product_lds(acc, x, y);
                    } else {
                        acc_add_lds(acc, r, flags);
                        acc_add_lds(acc, t, flags);
                    }
                } else {
                    double left = fpe_accumulate_all<P>(a, r);
                    if (left != 0.0) { acc_add_lds(acc, left, flags); ++wfl; }
                    left = fpe_accumulate_from<P, (P > 1 ? 1 : 0)>(a, t);
                    if (left != 0.0) { acc_add_lds(acc, left, flags); ++wfl; }
                }
                adapt_tick();
            } else if constexpr (MODE == MODE_EXBLAS) {
                // the TwoProd error is about 2^-53 of the product: it enters
                // the expansion one level down
                double left = fpe_accumulate_all<P>(a, r);
                if (left != 0.0) acc_add_lds(acc, left, flags);
                left = fpe_accumulate_from<P, (P > 1 ? 1 : 0)>(a, t);
                if (left != 0.0) acc_add_lds(acc, left, flags);
            } else if constexpr (ADAPT) {
                // FPE with the fallback: the same switching; what goes to the
                // long accumulator directly counts as escaped (it did not stay
                // in an expansion). Without the fallback the lane never
                // switches, as remainders are then dropped, not kept.
                if (direct) {
                    if (product_in_integer_range(r)) {
                        acc_add_product_lds(acc, x, y);
                    } else {
                        acc_add_lds(acc, r, flags);
                        acc_add_lds(acc, t, flags);
                    }
                    esc += (r != 0.0) + (t != 0.0);
                } else {
                    double left = fpe_accumulate<P>(a, r, ee);
                    if (left != 0.0) { ++esc; ++wfl; if (capture) acc_add_lds(acc, left, flags); }
                    left = fpe_accumulate<P>(e, t, ee);
                    if (left != 0.0) { ++esc; ++wfl; if (capture) acc_add_lds(acc, left, flags); }
                }
                if (++win == ADAPT_WINDOW) {
                    direct = direct ? direct - 1 : (capture && wfl > ADAPT_WINDOW ? ADAPT_DIRECT : 0);
                    win = wfl = 0;
                }
            } else {
                double left = fpe_accumulate<P>(a, r, ee);
                if (left != 0.0) { ++esc; if (capture) acc_add_lds(acc, left, flags); }
                left = fpe_accumulate<P>(e, t, ee);
                if (left != 0.0) { ++esc; if (capture) acc_add_lds(acc, left, flags); }
            }
        }
    }

    // binary32 operands: the product has at most 48 significant bits and an
    // exponent of at least -298, so it is exact in binary64 and enters the
    // expansion as one term (no TwoProd error term).
    __device__ __forceinline__ void add(float x, float y, long long *acc, bool ee, bool capture)
    {
        const double p = (double)x * (double)y;
        if constexpr (MODE == MODE_PLAIN) {
            s += p;
        } else {
            double left = fpe_accumulate<P>(a, p, ee);
            if (left != 0.0) {
                if constexpr (MODE == MODE_FPE) {
                    ++esc;
                    if (capture) acc_add_lds(acc, left, flags);
                } else {
                    acc_add_lds(acc, left, flags);
                }
            }
        }
    }
};

__device__ __forceinline__ void zero_acc(long long *acc)
{
    for (int k = threadIdx.x; k < ACC_DIGITS; k += blockDim.x) acc[k] = 0;
}

// fpesum (Alg. 3) of b into a; each remainder is counted and, with capture,
// kept exactly in the long accumulator.
template <int P>
__device__ __forceinline__ int fpe_sum_capture(double (&a)[P], const double (&b)[P], bool ee, bool capture,
                                               long long *acc, int &flags)
{
    int esc = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        double left = fpe_accumulate<P>(a, b[i], ee);
        if (left != 0.0) { ++esc; if (capture) acc_add_lds(acc, left, flags); }
    }
    return esc;
}

// Exact sum of the lanes' expansions of one wavefront added to the long
// accumulator (EXBLAS): every lane cuts its components into the
// accumulator's 32-bit digit chunks, the wavefront sums each word's chunks
// over its lanes with integer DPP steps (exact: at most 64 * 3 * P chunks
// below 2^32 each), and one lane adds each word sum to the accumulator.
// Integers add exactly in any order, so this is the same value as merging
// the expansions and flushing the remainders; the words are independent,
// so there is no chain of dependent TwoSums. Words outside the wavefront's
// range of chunks hold nothing and are skipped.
// One DPP step of a 64-bit integer (both halves moved by the same lane
// pattern; lanes without a source, or outside the row mask, read 0).
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ long long dpp_i64(long long v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, ROW_MASK, 0xF, true);
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum of a 64-bit integer over the wavefront's 64 lanes, exact, left in lane
// 63: prefix sums within each row of 16 lanes (row shifts by 1, 2, 4, 8),
// then row 0's total broadcast into row 1 and row 2's into row 3, then the
// total of rows 0-1 into rows 2-3. Register moves only, no LDS round trips.
__device__ __forceinline__ long long wave_sum_i64_last(long long v)
{
    v += dpp_i64<0x111>(v);      // row_shr:1
    v += dpp_i64<0x112>(v);      // row_shr:2
    v += dpp_i64<0x114>(v);      // row_shr:4
    v += dpp_i64<0x118>(v);      // row_shr:8
    v += dpp_i64<0x142, 0xA>(v); // row_bcast:15 into rows 1 and 3
    v += dpp_i64<0x143, 0xC>(v); // row_bcast:31 into rows 2 and 3
    return v;
}

// The same sum in every lane (read from lane 63).
__device__ __forceinline__ long long wave_sum_i64_all(long long v)
{
    v = wave_sum_i64_last(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)v, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), 63);
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Minimum / maximum of an int over the wavefront, in every lane: the same
// DPP pattern, lanes without a source keeping the identity.
template <bool MAX>
__device__ __forceinline__ int wave_minmax_i32_all(int v)
{
    constexpr int ID = MAX ? -2147483647 - 1 : 2147483647;
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x111, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x112, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x114, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x118, 0xF, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x142, 0xA, 0xF, false));
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x143, 0xC, 0xF, false));
    return __builtin_amdgcn_readlane(v, 63);
}

template <int P>
__device__ __forceinline__ void wave_flush_exact(const double (&a)[P], long long *acc, int &flags)
{
    int k[P];
    long long c0[P], c1[P], c2[P];
    int lo = ACC_DIGITS, hi = -1;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        k[i] = -8; // matches no word
        c0[i] = c1[i] = c2[i] = 0;
        if (a[i] != 0.0) {
            if (!is_finite_bits(a[i])) {
                flags |= FLAG_NONFINITE;
            } else {
                const AccChunks c = acc_chunks(a[i]);
                k[i] = c.k;
                c0[i] = c.c0;
                c1[i] = c.c1;
                c2[i] = c.c2;
                lo = min(lo, c.k);
                hi = max(hi, c.k + 2);
            }
        }
    }
    lo = wave_minmax_i32_all<false>(lo);
    hi = wave_minmax_i32_all<true>(hi);
    for (int w = lo; w <= hi; ++w) {
        long long v = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int d = w - k[i];
            v += d == 0 ? c0[i] : (d == 1 ? c1[i] : (d == 2 ? c2[i] : 0ll));
        }
        v = wave_sum_i64_last(v);
        if (lane_id() == 63 && v != 0) atomicAdd((unsigned long long *)&acc[w], (unsigned long long)v);
    }
}

// Lane chunks of an expansion (see wave_flush_exact); lo/hi widened to the
// lane's word range.
template <int P>
struct LaneChunks {
    int k[P];
    long long c0[P], c1[P], c2[P];

    __device__ __forceinline__ void cut(const double (&a)[P], int &lo, int &hi, int &flags)
    {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            k[i] = -8; // matches no word
            c0[i] = c1[i] = c2[i] = 0;
            if (a[i] != 0.0) {
                if (!is_finite_bits(a[i])) {
                    flags |= FLAG_NONFINITE;
                } else {
                    const AccChunks c = acc_chunks(a[i]);
                    k[i] = c.k;
                    c0[i] = c.c0;
                    c1[i] = c.c1;
                    c2[i] = c.c2;
                    lo = min(lo, c.k);
                    hi = max(hi, c.k + 2);
                }
            }
        }
    }

    __device__ __forceinline__ long long word(int w) const
    {
        long long v = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int d = w - k[i];
            v += d == 0 ? c0[i] : (d == 1 ? c1[i] : (d == 2 ? c2[i] : 0ll));
        }
        return v;
    }
};

// wave_flush_exact for two dots at once: one loop over the union of their
// word ranges, the two word sums reduced side by side.
template <int P>
__device__ __forceinline__ void wave_flush_exact2(const double (&a0)[P], long long *acc0, int &flags0,
                                                  const double (&a1)[P], long long *acc1, int &flags1)
{
    LaneChunks<P> q0, q1;
    int lo = ACC_DIGITS, hi = -1;
    q0.cut(a0, lo, hi, flags0);
    q1.cut(a1, lo, hi, flags1);
    lo = wave_minmax_i32_all<false>(lo);
    hi = wave_minmax_i32_all<true>(hi);
    for (int w = lo; w <= hi; ++w) {
        const long long v0 = wave_sum_i64_last(q0.word(w)), v1 = wave_sum_i64_last(q1.word(w));
        if (lane_id() == 63) {
            if (v0 != 0) atomicAdd((unsigned long long *)&acc0[w], (unsigned long long)v0);
            if (v1 != 0) atomicAdd((unsigned long long *)&acc1[w], (unsigned long long)v1);
        }
    }
}

// Merge the expansions of one wavefront into lane 0 (fixed tree order).
template <int P>
__device__ __forceinline__ int wave_fpe_merge(double (&a)[P], bool ee, bool capture, long long *acc, int &flags)
{
    int esc = 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double b[P];
#pragma unroll
        for (int i = 0; i < P; ++i) b[i] = __shfl_down(a[i], off, 64);
        if (lane_id() < off) esc += fpe_sum_capture<P>(a, b, ee, capture, acc, flags);
    }
    return esc;
}

// Fixed-order workgroup sum of a double into thread 0.
__device__ inline double block_sum_d(double v, RedShared &sh)
{
    v = wave_sum_down(v);
    if (lane_id() == 0) sh.part[wave_id()] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < num_waves(); ++w) t += sh.part[w];
    __syncthreads();
    return t;
}

// Workgroup sum of an integer into thread 0.
__device__ inline long long block_sum_ll(long long v, RedShared &sh)
{
    v = wave_sum_down(v);
    if (lane_id() == 0) sh.red_ll[wave_id()] = v;
    __syncthreads();
    long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < num_waves(); ++w) t += sh.red_ll[w];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// Slots: one workgroup partial per producing workgroup. Long-accumulator
// words are stored word-major (word k of slot g at digits[k * stride + g]) so
// that the merge reads each word of all slots as one coalesced run.

struct SlotView {
    DotWs ws;
    int stride; // slot capacity (words of one index are `stride` apart)
};

// Write the workgroup partial of one dot into slot g. All threads call.
template <int MODE, int P, bool ADAPT>
__device__ __forceinline__ void block_finish(LaneDot<MODE, P, ADAPT> &L, long long *acc, const SlotView &sv, int g,
                                             bool ee, bool capture, int *gflags, RedShared &sh)
{
    if constexpr (MODE == MODE_PLAIN) {
        double t = block_sum_d(L.s, sh);
        if (threadIdx.x == 0) sv.ws.part[g] = t;
        return;
    } else {
        if constexpr (MODE == MODE_EXBLAS) {
            // the lanes' expansions go into the accumulator word by word, one
            // atomic per word and wavefront
            wave_flush_exact<P>(L.a, acc, L.flags);
        } else {
            // each lane merges its result and error expansions, the
            // wavefront merges its lanes' expansions (fixed tree, escapes
            // counted), and the wavefront's expansion is added exactly to the
            // long accumulator, which already holds whatever escaped on the
            // way: the slot is the exact workgroup partial, merged across
            // workgroups like exblas
            L.esc += fpe_sum_capture<P>(L.a, L.e, ee, capture, acc, L.flags);
            L.esc += wave_fpe_merge<P>(L.a, ee, capture, acc, L.flags);
            if (lane_id() == 0) {
#pragma unroll
                for (int i = 0; i < P; ++i) acc_add_lds(acc, L.a[i], L.flags);
            }
            const long long esc = block_sum_ll(L.esc, sh);
            if (threadIdx.x == 0) sv.ws.esc[g] = (int)esc;
        }
        if (threadIdx.x == 0) { sh.rng[0] = ACC_DIGITS; sh.rng[1] = -1; }
        __syncthreads();
        // one carry step keeps every word below 2^33 in magnitude, so the
        // integer sum over the slots cannot overflow
        for (int k = threadIdx.x; k < ACC_DIGITS; k += blockDim.x) {
            long long v = acc[k];
            long long cin = k ? (acc[k - 1] >> 32) : 0;
            long long o = (k == ACC_DIGITS - 1) ? v + cin : (v & 0xFFFFFFFFll) + cin;
            sv.ws.digits[(long long)k * sv.stride + g] = o;
            if (o != 0) { atomicMin(&sh.rng[0], k); atomicMax(&sh.rng[1], k); }
        }
        __syncthreads();
        if (threadIdx.x == 0) { sv.ws.range[2 * g] = sh.rng[0]; sv.ws.range[2 * g + 1] = sh.rng[1]; }
        if (L.flags) atomicOr(gflags, L.flags);
    }
}

// The partials of two dots into slot g of sv0 and sv1 (as two block_finish
// calls; in EXBLAS mode in one pass, the wavefront word sums of both dots
// side by side and one carry step over both accumulators).
template <int MODE, int P, bool ADAPT>
__device__ __forceinline__ void block_finish_pair(LaneDot<MODE, P, ADAPT> &L0, long long *acc0, const SlotView &sv0,
                                                  LaneDot<MODE, P, ADAPT> &L1, long long *acc1, const SlotView &sv1,
                                                  int g, bool ee, bool capture, int *gflags, RedShared &sh)
{
    if constexpr (MODE != MODE_EXBLAS) {
        block_finish<MODE, P>(L0, acc0, sv0, g, ee, capture, gflags, sh);
        block_finish<MODE, P>(L1, acc1, sv1, g, ee, capture, gflags, sh);
    } else {
        wave_flush_exact2<P>(L0.a, acc0, L0.flags, L1.a, acc1, L1.flags);
        if (threadIdx.x == 0) { sh.rng[0] = ACC_DIGITS; sh.rng[1] = -1; sh.rng2[0] = ACC_DIGITS; sh.rng2[1] = -1; }
        __syncthreads();
        for (int q = threadIdx.x; q < 2 * ACC_DIGITS; q += blockDim.x) {
            const bool second = q >= ACC_DIGITS;
            const int k = second ? q - ACC_DIGITS : q;
            const long long *acc = second ? acc1 : acc0;
            long long v = acc[k];
            long long cin = k ? (acc[k - 1] >> 32) : 0;
            long long o = (k == ACC_DIGITS - 1) ? v + cin : (v & 0xFFFFFFFFll) + cin;
            (second ? sv1 : sv0).ws.digits[(long long)k * (second ? sv1 : sv0).stride + g] = o;
            if (o != 0) {
                int *rng = second ? sh.rng2 : sh.rng;
                atomicMin(&rng[0], k);
                atomicMax(&rng[1], k);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            sv0.ws.range[2 * g] = sh.rng[0];
            sv0.ws.range[2 * g + 1] = sh.rng[1];
            sv1.ws.range[2 * g] = sh.rng2[0];
            sv1.ws.range[2 * g + 1] = sh.rng2[1];
        }
        const int fl = L0.flags | L1.flags;
        if (fl) atomicOr(gflags, fl);
    }
}

// ---------------------------------------------------------------------------
// Correct rounding of a long accumulator by one full wavefront.
//
// Lane l holds words 2l and 2l+1 (lanes past the top hold zeros). Carries
// move up by shuffles until every word below the top is in [0, 2^32); the
// sign is the top word's; the leading word, the 53 bits below the leading
// one and the rounding/sticky information are read with uniform lane
// indices. Same result as acc_round() in numerics.hpp.

constexpr int TOP_LANE = (ACC_DIGITS - 1) / 2; // lane holding the top word (as its odd word)
static_assert(ACC_DIGITS % 2 == 0, "two words per lane");

__device__ __forceinline__ void wave_normalize(long long &a, long long &b)
{
    const int l = lane_id();
    for (int it = 0; it < 2 * ACC_DIGITS; ++it) {
        long long ca = a >> 32;
        a &= 0xFFFFFFFFll;
        b += ca;
        long long cb = 0;
        if (l != TOP_LANE) { cb = b >> 32; b &= 0xFFFFFFFFll; }
        long long cin = __shfl_up(cb, 1, 64);
        if (l == 0) cin = 0;
        a += cin;
        if (__ballot((a >> 32) != 0) == 0) break;
    }
}

__device__ __forceinline__ long long wave_word(long long a, long long b, int k)
{
    if (k < 0 || k >= ACC_DIGITS) return 0;
    long long v = __shfl((k & 1) ? b : a, k >> 1, 64);
    return v;
}

// Rounding format: significand bits, weight of the last bit of the smallest
// subnormal, and the exponent at which values overflow (2^EMAX_INF).
template <typename T> struct Fmt;
template <> struct Fmt<double> { static constexpr int PREC = 53, QMIN = -1074, EMAX_INF = 1024; };
template <> struct Fmt<float> { static constexpr int PREC = 24, QMIN = -149, EMAX_INF = 128; };

// Correctly rounded (nearest, ties to even) value of the accumulator in
// format T, computed by one full wavefront; every lane returns it.
template <typename T = double>
__device__ inline T wave_acc_round(const long long *acc)
{
    constexpr int PREC = Fmt<T>::PREC, QMIN = Fmt<T>::QMIN, EMAX_INF = Fmt<T>::EMAX_INF;
    const int l = lane_id();
    long long a = (2 * l < ACC_DIGITS) ? acc[2 * l] : 0;
    long long b = (2 * l + 1 < ACC_DIGITS) ? acc[2 * l + 1] : 0;
    wave_normalize(a, b);
    const bool neg = __shfl(b, TOP_LANE, 64) < 0;
    if (neg) {
        a = -a;
        b = -b;
        wave_normalize(a, b);
    }
    const unsigned long long mb = __ballot(b != 0), ma = __ballot(a != 0);
    int h = -1;
    if (mb) h = 2 * (63 - __builtin_clzll(mb)) + 1;
    if (ma) h = max(h, 2 * (63 - __builtin_clzll(ma)));
    if (h < 0) return T(0);
    const unsigned long long dh = (unsigned long long)wave_word(a, b, h);
    const int msb = 63 - __builtin_clzll(dh);
    const int B = 32 * h + msb;  // bit index of the leading one
    const int E = B + ACC_EXP0;  // value in [2^E, 2^(E+1))
    if (E >= EMAX_INF) return neg ? -__builtin_inf() : __builtin_inf();
    int q = E - (PREC - 1);
    if (q < QMIN) q = QMIN;
    const int Q = q - ACC_EXP0;  // bit index of the last kept bit
    const int kq = Q >> 5, sq = Q & 31;
    const unsigned long long w0 = (unsigned)wave_word(a, b, kq);
    const unsigned long long w1 = (unsigned)wave_word(a, b, kq + 1);
    const unsigned long long w2 = (unsigned)wave_word(a, b, kq + 2);
    const unsigned long long lo64 = w0 | (w1 << 32);
    const unsigned long long r = (lo64 >> sq) | (sq ? (w2 << (64 - sq)) : 0ull);
    const int len = B - Q + 1; // <= PREC
    unsigned long long I = r & ((1ull << len) - 1);
    // rounding bit Q-1 and sticky bits below it
    const int R = Q - 1, kr = R >> 5, sr = R & 31;
    const unsigned long long wr = (unsigned)wave_word(a, b, kr);
    const bool half = (wr >> sr) & 1ull;
    bool sticky = (wr & ((1ull << sr) - 1)) != 0;
    const bool low = ((2 * l < kr) && a != 0) || ((2 * l + 1 < kr) && b != 0);
    sticky = sticky || (__ballot(low) != 0);
    if (half && (sticky || (I & 1ull))) I += 1;
    // exponent field (q - QMIN) above the significand; a carry of I into the
    // next power of two moves into the exponent field, up to infinity
    if constexpr (PREC == 53) {
        unsigned long long bits = ((unsigned long long)(q - QMIN) << 52) + I;
        if (neg) bits |= 1ull << 63;
        return __builtin_bit_cast(double, bits);
    } else {
        unsigned bits = ((unsigned)(q - QMIN) << 23) + (unsigned)I;
        if (neg) bits |= 1u << 31;
        return __builtin_bit_cast(float, bits);
    }
}

// ---------------------------------------------------------------------------
// Merge of the G slots of one dot, in every workgroup alike. All threads of
// the workgroup call; the result is returned to every thread. `acc` is an
// LDS accumulator the merge may overwrite. *esc_out (thread 0) receives the
// escapes (FPE); flags seen on the way are or-ed into *flags_out.

// Sum of row[0..G) by one wavefront (result in every lane); eight independent
// loads per lane are in flight at a time.
__device__ __forceinline__ long long sum_row(const long long *row, int G)
{
    long long s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int g = lane_id();
    for (; g + 7 * 64 < G; g += 8 * 64) {
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += row[g + 64 * j];
    }
    for (; g < G; g += 64) s[0] += row[g];
    long long t = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    return wave_sum_i64_all(t);
}

template <int MODE, int P, typename T = double>
__device__ __forceinline__ T merge_slots(const SlotView &sv, int G, bool ee, bool capture, long long *acc,
                              long long *esc_out, int *flags_out, RedShared &sh, int slot_val)
{
    *esc_out = 0;
    T r;
    if constexpr (MODE == MODE_PLAIN) {
        // fixed order: wavefront 0 sums the slots lane-strided, then the tree
        if (wave_id() == 0) {
            double s[4] = {0.0, 0.0, 0.0, 0.0};
            int g = lane_id();
            for (; g + 3 * 64 < G; g += 4 * 64) {
#pragma unroll
                for (int j = 0; j < 4; ++j) s[j] += sv.ws.part[g + 64 * j];
            }
            for (; g < G; g += 64) s[0] += sv.ws.part[g];
            double t = wave_sum_down((s[0] + s[1]) + (s[2] + s[3]));
            if (lane_id() == 0) sh.val[slot_val] = t;
        }
        __syncthreads();
        r = (T)sh.val[slot_val];
        __syncthreads();
        return r;
    } else {
        int flags = 0;
        zero_acc(acc);
        if (threadIdx.x == 0) { sh.rng[0] = ACC_DIGITS; sh.rng[1] = -1; }
        __syncthreads();
        // FPE: the slots are exact workgroup partials (expansion included);
        // only the escape counts are summed here
        if constexpr (MODE == MODE_FPE) {
            long long esc_slots = 0;
            for (int g = threadIdx.x; g < G; g += blockDim.x) esc_slots += sv.ws.esc[g];
            long long esc_tot = block_sum_ll(esc_slots, sh);
            if (threadIdx.x == 0) *esc_out = esc_tot;
        }
        // long-accumulator words: global nonzero range, then one word per wavefront
        int kmin = ACC_DIGITS, kmax = -1;
        for (int g = threadIdx.x; g < G; g += blockDim.x) {
            kmin = min(kmin, sv.ws.range[2 * g]);
            kmax = max(kmax, sv.ws.range[2 * g + 1]);
        }
        kmin = wave_minmax_i32_all<false>(kmin);
        kmax = wave_minmax_i32_all<true>(kmax);
        if (lane_id() == 0) { atomicMin(&sh.rng[0], kmin); atomicMax(&sh.rng[1], kmax); }
        __syncthreads();
        const int K0 = sh.rng[0], K1 = sh.rng[1];
        for (int k = K0 + wave_id(); k <= K1; k += num_waves()) {
            long long s = sum_row(sv.ws.digits + (long long)k * sv.stride, G);
            if (lane_id() == 0) atomicAdd((unsigned long long *)&acc[k], (unsigned long long)s);
        }
        __syncthreads();
        if (flags) atomicOr(flags_out, flags);
        if (wave_id() == 0) {
            T v = wave_acc_round<T>(acc);
            if (lane_id() == 0) sh.val[slot_val] = (double)v;
        }
        __syncthreads();
        r = (T)sh.val[slot_val];
        __syncthreads();
        return r;
    }
}

template <int V>
using IC = std::integral_constant<int, V>;

// Call f(IC<mode>, IC<P>) for the runtime mode and expansion length.
template <int M, typename F>
inline void dispatch_p(int p, F &&f)
{
    switch (p) {
    case 1: f(IC<M>{}, IC<1>{}); break;
    case 2: f(IC<M>{}, IC<2>{}); break;
    case 3: f(IC<M>{}, IC<3>{}); break;
    case 4: f(IC<M>{}, IC<4>{}); break;
    case 5: f(IC<M>{}, IC<5>{}); break;
    case 6: f(IC<M>{}, IC<6>{}); break;
    case 7: f(IC<M>{}, IC<7>{}); break;
    default: f(IC<M>{}, IC<8>{}); break;
    }
}

template <typename F>
inline void dispatch(int mode, int p, F &&f)
{
    if (mode == MODE_PLAIN) f(IC<MODE_PLAIN>{}, IC<1>{});
    else if (mode == MODE_FPE) dispatch_p<MODE_FPE>(p, f);
    else dispatch_p<MODE_EXBLAS>(p, f);
}

} // namespace rpcg
