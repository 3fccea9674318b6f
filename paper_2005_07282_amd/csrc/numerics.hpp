// Device numerics of the reproducible dot product: error-free transformations,
// floating-point expansions and the long accumulator.
//
// Everything here is __host__ __device__ so the same source can be exercised
// on the CPU; the atomic LDS variant is device-only.
//
// Compile with -ffp-contract=off: TwoSum and TwoProd rely on every + - *
// being rounded individually, and fma appears only where written.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpcg {

// ---------------------------------------------------------------------------
// Error-free transformations (Section 2)

// Alg. 1 (TwoSum, Knuth): r = RN(a + b) and s with a + b = r + s exactly.
__host__ __device__ __forceinline__ void two_sum(double a, double b, double &r, double &s)
{
    r = a + b;
    double z = r - a;
    s = (a - (r - z)) + (b - z);
}

// Alg. 2 (TwoProd with fma): r = RN(a * b) and s = a*b - r exactly, provided
// the product neither overflows nor falls below 2^-969 (s representable).
__host__ __device__ __forceinline__ void two_prod(double a, double b, double &r, double &s)
{
    r = a * b;
    s = __builtin_fma(a, b, -r);
}

// ---------------------------------------------------------------------------
// Floating-point expansions (Section 2, Section 4.2)

// Alg. 4 (Accumulate): add x into the expansion a[0..P) level by level with
// TwoSum. With early exit (Section 4.2) the propagation stops once the
// carried error is zero, which changes nothing since TwoSum(a, 0) = (a, 0).
// Returns what is left after the last level: nonzero means the expansion
// could not hold every bit (an "escape").
template <int P>
__host__ __device__ __forceinline__ double fpe_accumulate(double (&a)[P], double x, bool early_exit)
{
#pragma unroll
    for (int i = 0; i < P; ++i) {
        if (early_exit && x == 0.0) return 0.0;
        double r, s;
        two_sum(a[i], x, r, s);
        a[i] = r;
        x = s;
    }
    return x;
}

// Alg. 4 without the early exit: all P levels run, branch-free. On a 64-wide
// wavefront a divergent exit saves nothing (the wavefront runs every level
// as long as one lane continues) and costs the exec-mask bookkeeping of each
// branch; the result is the same since TwoSum(a, 0) = (a, 0).
template <int P>
__host__ __device__ __forceinline__ double fpe_accumulate_all(double (&a)[P], double x)
{
#pragma unroll
    for (int i = 0; i < P; ++i) {
        double r, s;
        two_sum(a[i], x, r, s);
        a[i] = r;
        x = s;
    }
    return x;
}

// The same, entering at level L (0 <= L < P): x is added to a[L], the
// remainder carried through a[L+1..P). Any component may receive any value:
// every level is error-free and what is left is returned, so the exact sum
// of the components plus the remainders is unchanged.
template <int P, int L>
__host__ __device__ __forceinline__ double fpe_accumulate_from(double (&a)[P], double x)
{
#pragma unroll
    for (int i = L; i < P; ++i) {
        double r, s;
        two_sum(a[i], x, r, s);
        a[i] = r;
        x = s;
    }
    return x;
}

// Alg. 3 (fpesum): a += b component by component. Returns the number of
// components whose accumulation left a nonzero remainder.
template <int P>
__host__ __device__ __forceinline__ int fpe_sum(double (&a)[P], const double (&b)[P], bool early_exit)
{
    int escapes = 0;
#pragma unroll
    for (int i = 0; i < P; ++i) escapes += fpe_accumulate<P>(a, b[i], early_exit) != 0.0;
    return escapes;
}

// ---------------------------------------------------------------------------
// Long accumulator (Section 2 Kulisch accumulator; Section 4.1, 4.3)
//
// ACC_DIGITS signed 64-bit words; word k holds a digit of weight
// 2^(32 k + ACC_EXP0). Every finite double is an integer multiple of 2^-1074,
// so bit 0 of word 0 (weight 2^-1088) is below any double's last bit, and
// the top words leave room for sums far beyond 2^1024. A double adds at most
// three 32-bit chunks, so each word absorbs 2^31 additions without overflow.

constexpr int ACC_DIGITS = 68;
constexpr int ACC_EXP0 = -1088;

struct AccChunks {
    int k;               // index of the lowest word touched
    long long c0, c1, c2; // signed chunks for words k, k+1, k+2
};

// Decompose a finite nonzero double v = +-m * 2^e into three signed 32-bit
// chunks aligned to the accumulator's words.
__host__ __device__ __forceinline__ AccChunks acc_chunks(double v)
{
    unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
    unsigned be = (unsigned)((bits >> 52) & 0x7FF);
    unsigned long long m = bits & 0xFFFFFFFFFFFFFull;
    if (be) m |= 1ull << 52;
    else be = 1; // subnormal: m * 2^(1 - 1075)
    int off = (int)be - 1075 - ACC_EXP0; // bit offset of m's last bit, >= 14
    int k = off >> 5, s = off & 31;
    unsigned long long lo = m << s;
    unsigned long long hi = s ? (m >> (64 - s)) : 0ull;
    AccChunks c;
    c.k = k;
    c.c0 = (long long)(lo & 0xFFFFFFFFull);
    c.c1 = (long long)(lo >> 32);
    c.c2 = (long long)hi;
    if (bits >> 63) { c.c0 = -c.c0; c.c1 = -c.c1; c.c2 = -c.c2; }
    return c;
}

__host__ __device__ __forceinline__ bool is_finite_bits(double v)
{
    return (__builtin_bit_cast(unsigned long long, v) & 0x7FF0000000000000ull) != 0x7FF0000000000000ull;
}

// Non-atomic add of a double (single owner of the words).
__host__ __device__ __forceinline__ void acc_add(long long *acc, double v)
{
    if (v == 0.0) return;
    AccChunks c = acc_chunks(v);
    acc[c.k] += c.c0;
    acc[c.k + 1] += c.c1;
    acc[c.k + 2] += c.c2;
}

// Carry-propagate so that words 0..D-2 lie in [0, 2^32) and the top word
// carries the sign; the represented value is unchanged.
__host__ __device__ __forceinline__ void acc_normalize(long long *acc)
{
    long long c = 0;
    for (int k = 0; k < ACC_DIGITS - 1; ++k) {
        long long t = acc[k] + c;
        acc[k] = t & 0xFFFFFFFFll;
        c = t >> 32; // arithmetic shift: floor division by 2^32
    }
    acc[ACC_DIGITS - 1] += c;
}

// Bits [pos, pos+len) of a normalized non-negative accumulator, len <= 60.
__host__ __device__ __forceinline__ unsigned long long acc_bits(const long long *acc, int pos, int len)
{
    int k = pos >> 5, s = pos & 31;
    unsigned long long w0 = k < ACC_DIGITS ? (unsigned long long)(unsigned)acc[k] : 0ull;
    unsigned long long w1 = k + 1 < ACC_DIGITS ? (unsigned long long)(unsigned)acc[k + 1] : 0ull;
    unsigned long long w2 = k + 2 < ACC_DIGITS ? (unsigned long long)(unsigned)acc[k + 2] : 0ull;
    unsigned long long lo64 = w0 | (w1 << 32);                  // bits [32k, 32k+64)
    unsigned long long r = (lo64 >> s) | (s ? (w2 << (64 - s)) : 0ull);
    return len >= 64 ? r : (r & ((1ull << len) - 1));
}

// Any bit set in [0, pos) of a normalized non-negative accumulator?
__host__ __device__ __forceinline__ bool acc_any_below(const long long *acc, int pos)
{
    if (pos <= 0) return false;
    int k = pos >> 5, s = pos & 31;
    for (int j = 0; j < k && j < ACC_DIGITS; ++j)
        if (acc[j] != 0) return true;
    if (s && k < ACC_DIGITS) return ((unsigned long long)(unsigned)acc[k] & ((1ull << s) - 1)) != 0;
    return false;
}

// Round the accumulator to the nearest double, ties to even (exblas Round,
// NearSum, Section 4.3). Destroys its argument. Exact zero gives +0; values
// at or above 2^1024 - 2^970 in magnitude give infinity.
__host__ __device__ inline double acc_round(long long *acc)
{
    acc_normalize(acc);
    bool neg = acc[ACC_DIGITS - 1] < 0;
    if (neg) {
        for (int k = 0; k < ACC_DIGITS; ++k) acc[k] = -acc[k];
        acc_normalize(acc);
    }
    int h = ACC_DIGITS - 1;
    while (h >= 0 && acc[h] == 0) --h;
    if (h < 0) return 0.0;
    unsigned long long top = (unsigned long long)acc[h];
    int msb = 63 - __builtin_clzll(top);
    int B = 32 * h + msb;      // bit index of the leading one
    int E = B + ACC_EXP0;      // value in [2^E, 2^(E+1))
    if (E >= 1024) return neg ? -__builtin_inf() : __builtin_inf();
    int q = E - 52;            // weight of the last kept bit
    if (q < -1074) q = -1074;  // subnormal range
    int Q = q - ACC_EXP0;      // its bit index (>= 14)
    unsigned long long I = acc_bits(acc, Q, B - Q + 1);
    bool half = acc_bits(acc, Q - 1, 1) != 0;
    if (half && ((I & 1ull) || acc_any_below(acc, Q - 1))) I += 1; // I <= 2^53
    // normal: exponent field q + 1075 with the leading bit in I; subnormal:
    // field 0; a carry to 2^53 moves into the exponent field (up to infinity).
    unsigned long long bits = ((unsigned long long)(q + 1074) << 52) + I;
    if (neg) bits |= 1ull << 63;
    return __builtin_bit_cast(double, bits);
}

// ---------------------------------------------------------------------------
// Lane-private long accumulator with a tracked window: word k lives at
// w[k * STRIDE] (one column of a [ACC_DIGITS][STRIDE] array, so the lanes of
// a wavefront own neighbouring columns), every word starts at zero, and only
// the words [lo, hi] are touched by additions. Rounding visits the window and
// the few words the carries reach, and leaves every word at zero again.
template <int STRIDE>
struct WindowAcc {
    long long *w;
    int lo, hi;

    __host__ __device__ __forceinline__ void init(long long *col)
    {
        w = col;
        lo = ACC_DIGITS;
        hi = -1;
    }

    // v finite and nonzero
    __host__ __device__ __forceinline__ void add(double v)
    {
        AccChunks c = acc_chunks(v);
        w[c.k * STRIDE] += c.c0;
        w[(c.k + 1) * STRIDE] += c.c1;
        w[(c.k + 2) * STRIDE] += c.c2;
        lo = c.k < lo ? c.k : lo;
        hi = c.k + 2 > hi ? c.k + 2 : hi;
    }

    __host__ __device__ __forceinline__ unsigned long long word(int k) const
    {
        return (k >= 0 && k < ACC_DIGITS) ? (unsigned long long)(unsigned)w[k * STRIDE] : 0ull;
    }

    // Correctly rounded binary64 value (ties to even, +0 for an exact zero,
    // infinity at or above 2^1024 - 2^970 in magnitude; same rule as
    // acc_round), then clear.
    __host__ __device__ inline double round_and_clear()
    {
        if (hi < 0) return 0.0;
        // carry propagation from the lowest touched word; above `hi` the
        // carry settles to 0 (non-negative value) or -1 (negative value)
        long long c = 0;
        int kend = ACC_DIGITS - 1;
        for (int k = lo; k < ACC_DIGITS; ++k) {
            const long long t = w[k * STRIDE] + c;
            w[k * STRIDE] = t & 0xFFFFFFFFll;
            c = t >> 32;
            if (k >= hi && (c == 0 || c == -1)) { kend = k; break; }
        }
        const bool neg = c < 0;
        if (neg) {
            // magnitude = 2^(32 (kend+1)) - U: two's complement of the window
            // (words below lo are zero, so the +1 enters at lo)
            unsigned long long borrow = 1;
            for (int k = lo; k <= kend; ++k) {
                const unsigned long long t = ((~(unsigned long long)w[k * STRIDE]) & 0xFFFFFFFFull) + borrow;
                w[k * STRIDE] = (long long)(t & 0xFFFFFFFFull);
                borrow = t >> 32;
            }
            if (borrow && kend + 1 < ACC_DIGITS) { ++kend; w[kend * STRIDE] = (long long)borrow; }
        }
        int h = kend;
        while (h >= lo && w[h * STRIDE] == 0) --h;
        double result = 0.0;
        if (h >= lo) {
            const int msb = 63 - __builtin_clzll((unsigned long long)w[h * STRIDE]);
            const int B = 32 * h + msb;
            const int E = B + ACC_EXP0;
            if (E >= 1024) {
                result = neg ? -__builtin_inf() : __builtin_inf();
            } else {
                int q = E - 52;
                if (q < -1074) q = -1074;
                const int Q = q - ACC_EXP0;
                const int kq = Q >> 5, sq = Q & 31;
                const unsigned long long lo64 = word(kq) | (word(kq + 1) << 32);
                const unsigned long long r = (lo64 >> sq) | (sq ? (word(kq + 2) << (64 - sq)) : 0ull);
                const int len = B - Q + 1;
                unsigned long long I = r & ((1ull << len) - 1);
                const int R = Q - 1, kr = R >> 5, sr = R & 31;
                const unsigned long long wr = word(kr);
                const bool half = (wr >> sr) & 1ull;
                bool sticky = (wr & ((1ull << sr) - 1)) != 0;
                for (int k = lo; k < kr && !sticky; ++k) sticky = w[k * STRIDE] != 0;
                if (half && (sticky || (I & 1ull))) I += 1;
                unsigned long long bits = ((unsigned long long)(q + 1074) << 52) + I;
                if (neg) bits |= 1ull << 63;
                result = __builtin_bit_cast(double, bits);
            }
        }
        for (int k = lo; k <= kend; ++k) w[k * STRIDE] = 0;
        lo = ACC_DIGITS;
        hi = -1;
        return result;
    }
};

} // namespace rpcg
