// Device-side reduction machinery shared by the kernel translation units:
// per-lane accumulators, workgroup partials, the last-workgroup ticket and
// the merge of workgroup partials.
//
// Reduction structure (Section 3.2 / 4.3 mapped onto one GPU): each lane
// keeps its own accumulator (an expansion, or a plain sum), the lanes of a
// workgroup combine into one workgroup partial (a long accumulator in LDS,
// or an expansion merged in a fixed tree), every workgroup writes its
// partial to a slot, and the last workgroup to arrive (atomic ticket with
// device-scope release/acquire fences) combines the slots and rounds once.
// This replaces the paper's MPI_Reduce + Round + MPI_Bcast: the rounded
// scalar lands in device memory where the next kernel reads it.
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
    long long acc[3][ACC_DIGITS];   // workgroup long accumulators
    long long red_ll[MAX_WAVES];
    double part[MAX_WAVES * MAX_FPE];
    int rng[2];
    int flags;
    int esc;
    int last;
    int need_fb;
    double result[3];
};

__device__ __forceinline__ void acc_add_lds(long long *acc, double v, int &flags)
{
    if (v == 0.0) return;
    if (!is_finite_bits(v)) { flags |= FLAG_NONFINITE; return; }
    AccChunks c = acc_chunks(v);
    if (c.c0) atomicAdd((unsigned long long *)&acc[c.k], (unsigned long long)c.c0);
    if (c.c1) atomicAdd((unsigned long long *)&acc[c.k + 1], (unsigned long long)c.c1);
    if (c.c2) atomicAdd((unsigned long long *)&acc[c.k + 2], (unsigned long long)c.c2);
}

// Per-lane accumulator of one dot product.
template <int MODE, int P>
struct LaneDot {
    double a[P]; // EXBLAS: the lane's expansion; FPE: expansion of the TwoProd results
    double e[P]; // FPE: expansion of the TwoProd errors (Section 4.2: two expansions)
    double s;    // PLAIN: running fma sum
    int esc;
    int flags;

    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int i = 0; i < P; ++i) { a[i] = 0.0; e[i] = 0.0; }
        s = 0.0;
        esc = 0;
        flags = 0;
    }

    __device__ __forceinline__ void add(double x, double y, long long *acc, bool ee)
    {
        if constexpr (MODE == MODE_PLAIN) {
            s = __builtin_fma(x, y, s);
        } else {
            double r, t;
            two_prod(x, y, r, t);
            if (__builtin_fabs(r) < 0x1p-969 && x != 0.0 && y != 0.0) flags |= FLAG_INEXACT;
            if constexpr (MODE == MODE_EXBLAS) {
                // Listing 1: both halves go into the same expansion; what
                // does not fit is flushed into the long accumulator.
                double left = fpe_accumulate<P>(a, r, ee);
                if (left != 0.0) acc_add_lds(acc, left, flags);
                left = fpe_accumulate<P>(a, t, ee);
                if (left != 0.0) acc_add_lds(acc, left, flags);
            } else {
                esc += fpe_accumulate<P>(a, r, ee) != 0.0;
                esc += fpe_accumulate<P>(e, t, ee) != 0.0;
            }
        }
    }
};

__device__ __forceinline__ void zero_acc(long long *acc)
{
    for (int k = threadIdx.x; k < ACC_DIGITS; k += blockDim.x) acc[k] = 0;
}

// Merge the expansions of one wavefront into lane 0 (fixed tree order).
template <int P>
__device__ __forceinline__ int wave_fpe_merge(double (&a)[P], bool ee)
{
    int esc = 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double b[P];
#pragma unroll
        for (int i = 0; i < P; ++i) b[i] = __shfl_down(a[i], off, 64);
        if (lane_id() < off) esc += fpe_sum<P>(a, b, ee);
    }
    return esc;
}

// Merge the expansions of all wavefronts of the workgroup into thread 0's `a`.
// Every thread must call; returns (in thread 0) the escapes of all merges.
template <int P>
__device__ int block_fpe_merge(double (&a)[P], bool ee, RedShared &sh);

__device__ inline int block_sum_i(int v, RedShared &sh);

template <int P>
__device__ int block_fpe_merge(double (&a)[P], bool ee, RedShared &sh)
{
    int esc = block_sum_i(wave_fpe_merge<P>(a, ee), sh); // escapes of every lane, in thread 0
    if (lane_id() == 0) {
#pragma unroll
        for (int i = 0; i < P; ++i) sh.part[wave_id() * MAX_FPE + i] = a[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < num_waves(); ++w) {
            double b[P];
#pragma unroll
            for (int i = 0; i < P; ++i) b[i] = sh.part[w * MAX_FPE + i];
            esc += fpe_sum<P>(a, b, ee);
        }
    }
    __syncthreads();
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

__device__ inline int block_sum_i(int v, RedShared &sh)
{
    return (int)block_sum_ll((long long)v, sh);
}

// Workgroup partial of one dot into slot g of `ws`. All threads call.
template <int MODE, int P>
__device__ void block_finish(LaneDot<MODE, P> &L, long long *acc, const DotWs &ws, int g, bool ee,
                             int *gflags, RedShared &sh)
{
    if constexpr (MODE == MODE_EXBLAS) {
#pragma unroll
        for (int i = 0; i < P; ++i)
            if (L.a[i] != 0.0) acc_add_lds(acc, L.a[i], L.flags);
        if (threadIdx.x == 0) { sh.rng[0] = ACC_DIGITS; sh.rng[1] = -1; }
        __syncthreads();
        // one carry step keeps every word below 2^33 in magnitude, so the
        // integer sum over slots cannot overflow
        for (int k = threadIdx.x; k < ACC_DIGITS; k += blockDim.x) {
            long long v = acc[k];
            long long cin = k ? (acc[k - 1] >> 32) : 0;
            long long o = (k == ACC_DIGITS - 1) ? v + cin : (v & 0xFFFFFFFFll) + cin;
            ws.digits[(long long)g * ACC_DIGITS + k] = o;
            if (o != 0) { atomicMin(&sh.rng[0], k); atomicMax(&sh.rng[1], k); }
        }
        __syncthreads();
        if (threadIdx.x == 0) { ws.range[2 * g] = sh.rng[0]; ws.range[2 * g + 1] = sh.rng[1]; }
    } else if constexpr (MODE == MODE_FPE) {
        L.esc += fpe_sum<P>(L.a, L.e, ee);
        int esc = block_sum_i(L.esc, sh);
        esc += block_fpe_merge<P>(L.a, ee, sh);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int i = 0; i < P; ++i) ws.part[(long long)g * MAX_FPE + i] = L.a[i];
            ws.esc[g] = esc;
        }
    } else {
        double t = block_sum_d(L.s, sh);
        if (threadIdx.x == 0) ws.part[g] = t;
    }
    if (L.flags) atomicOr(gflags, L.flags);
}

// Called by every thread after its slot writes; true in the last workgroup.
__device__ inline bool arrive_last(unsigned *ticket, RedShared &sh)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        sh.last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    bool last = sh.last != 0;
    if (last) {
        __threadfence();
        if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return last;
}

// In the last workgroup: combine the G slots of one dot, round once.
// Result valid in thread 0; *esc_out gets the total escapes (FPE).
template <int MODE, int P>
__device__ double merge_slots(const DotWs &ws, int G, bool ee, long long *acc, int *gflags,
                              long long *esc_out, RedShared &sh)
{
    *esc_out = 0;
    if constexpr (MODE == MODE_EXBLAS) {
        int kmin = ACC_DIGITS, kmax = -1;
        for (int g = threadIdx.x; g < G; g += blockDim.x) {
            kmin = min(kmin, ws.range[2 * g]);
            kmax = max(kmax, ws.range[2 * g + 1]);
        }
        if (threadIdx.x == 0) { sh.rng[0] = ACC_DIGITS; sh.rng[1] = -1; }
        zero_acc(acc);
        __syncthreads();
        atomicMin(&sh.rng[0], kmin);
        atomicMax(&sh.rng[1], kmax);
        __syncthreads();
        int K0 = sh.rng[0], K1 = sh.rng[1];
        for (int k = K0; k <= K1; ++k) {
            long long s = 0;
            for (int g = threadIdx.x; g < G; g += blockDim.x) s += ws.digits[(long long)g * ACC_DIGITS + k];
            s = block_sum_ll(s, sh);
            if (threadIdx.x == 0) acc[k] = s;
        }
        __syncthreads();
        double r = 0.0;
        if (threadIdx.x == 0) {
            int f = __hip_atomic_load(gflags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            r = (f & FLAG_NONFINITE) ? __builtin_nan("") : acc_round(acc);
        }
        __syncthreads();
        return r;
    } else if constexpr (MODE == MODE_FPE) {
        double a[P];
#pragma unroll
        for (int i = 0; i < P; ++i) a[i] = 0.0;
        int esc = 0;
        long long esc_slots = 0;
        for (int g = threadIdx.x; g < G; g += blockDim.x) {
            double b[P];
#pragma unroll
            for (int i = 0; i < P; ++i) b[i] = ws.part[(long long)g * MAX_FPE + i];
            esc += fpe_sum<P>(a, b, ee);
            esc_slots += ws.esc[g];
        }
        long long tot = block_sum_ll(esc_slots + esc, sh);
        int e2 = block_fpe_merge<P>(a, ee, sh);
        double r = 0.0;
        if (threadIdx.x == 0) {
            tot += e2;
            *esc_out = tot;
            for (int k = 0; k < ACC_DIGITS; ++k) acc[k] = 0;
            bool fin = true;
#pragma unroll
            for (int i = 0; i < P; ++i) { fin = fin && is_finite_bits(a[i]); }
            int f = __hip_atomic_load(gflags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!fin || (f & FLAG_NONFINITE)) r = __builtin_nan("");
            else {
#pragma unroll
                for (int i = 0; i < P; ++i) acc_add(acc, a[i]); // NearSum: RN of the exact sum
                r = acc_round(acc);
            }
        }
        __syncthreads();
        return r;
    } else {
        double s = 0.0;
        for (int g = threadIdx.x; g < G; g += blockDim.x) s += ws.part[g];
        return block_sum_d(s, sh);
    }
}

// Exact dot computed by the calling workgroup alone (FPE fallback path).
// All threads call; result in thread 0.
__device__ inline double block_exact_dot(long long n, const double *x, const double *y, long long *acc,
                                  int *gflags, RedShared &sh)
{
    zero_acc(acc);
    __syncthreads();
    LaneDot<MODE_EXBLAS, 4> L;
    L.init();
    for (long long i = threadIdx.x; i < n; i += blockDim.x) L.add(x[i], y[i], acc, true);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (L.a[i] != 0.0) acc_add_lds(acc, L.a[i], L.flags);
    if (L.flags) atomicOr(gflags, L.flags);
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = acc_round(acc);
    __syncthreads();
    return r;
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
