// Host-visible declarations shared by the kernel translation unit and the
// C-ABI implementation: device-side state records, workspace descriptors and
// the launch functions (each kernel is launched only from its own .hip file).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpcg {

enum Mode { MODE_PLAIN = 0, MODE_FPE = 1, MODE_EXBLAS = 2 };

// Flag bits collected on the device.
enum {
    FLAG_NONFINITE = 1, // inf/NaN input, overflowing product or overflowing expansion
    FLAG_INEXACT = 2,   // a nonzero product below 2^-969 (TwoProd error not representable)
    FLAG_NOT_SPD = 4,   // missing or non-positive diagonal entry
};

constexpr int MAX_BLOCK = 1024;
constexpr int MAX_WAVES = MAX_BLOCK / 64;
constexpr int MAX_FPE = 8;
constexpr int ACC_WORDS = 68; // same as ACC_DIGITS in numerics.hpp

// Per-dot reduction workspace for up to `gmax` workgroups (slots).
struct DotWs {
    long long *digits; // [ACC_WORDS][gmax] workgroup accumulator words, word-major
    int *range;        // [gmax][2] nonzero word range of each workgroup accumulator
    double *part;      // [gmax][MAX_FPE] workgroup expansions (fpe) or partial sums (plain)
    int *esc;          // [gmax] escape counts (fpe)
};

// Scalars of one standalone dot call (device memory).
struct DotInfo {
    unsigned pad0;
    int flags;
    int max_len;         // longest row (SELL construction scratch)
    int pad1;
    long long max_delta; // column-code range (SELL construction scratch)
    long long escapes;
    long long fallbacks;
};

// PCG state on the device. Written only by the last workgroup of a kernel
// (or by a single thread of the setup), read by every workgroup of later
// kernels.
struct PcgState {
    double beta;   // beta of the current iteration (Fig. 2)
    double rho;    // rho = beta / <d, w>
    double gamma;  // beta_new / beta_old
    double tau;    // <r, r>
    double thr;    // RN(RN(tol*tol) * <b,b>)
    double delta;  // <d, w>
    double bb;     // <b, b>
    double tau0;
    int iter;      // iterations completed (L)
    int done;      // nonzero: every later kernel is a no-op
    int status;    // rpcg status code
    int maxit;
    int flags;
    int ended;     // the first iteration whose x update (S3) is not owed once the solve has
                   // ended (0 at setup, l at a breakdown in iteration l, l + 1 when the
                   // stopping test of iteration l stops); INT_MAX while running
    int it_cur;    // batched solves: iterations completed, as the kernels of the current
                   // iteration see it (committed by the SpMV kernel from iter)
    int pad2;
    double beta_par[2]; // batched solves: beta of iteration j in beta_par[j & 1]
    long long escapes;
    long long fallbacks;
};

// Sliced-ELL copy of the matrix with slice height 64 (one wavefront) and
// V-entry interleave: entry k of row 64*s + j sits at
//     off[s] + 64*V*(k/V) + V*j + (k%V),
// so lane j reads V consecutive entries of its row with one vector load while
// each load of the wavefront is one contiguous segment. The slice width is
// its longest row; when it is not a multiple of V (V = 2, odd width w) the
// last entry k = w-1 sits alone at off[s] + 64*(w-1) + j, so an odd row
// length costs no padding entry. Rows keep their CSR order and length;
// padding entries hold the value 0 and a valid column. T is the type the solver computes in and V
// = sell_vec<T>() (two for binary64: 16-byte loads; one for binary32).
//
// Columns: with col16 (16-bit column codes), the column of rank 0 of row
// i = 64 s + j is min(i, n-1) + cfirst[s] + (signed) code, and the column of
// rank k >= 1 is the column of rank k-1 plus the (unsigned) code: rows keep
// ascending columns in 16-bit steps and cfirst[s] is the first-column offset
// of the slice's longest row. Padding codes are 0 (the column repeats), and
// rows without entries get a rank-0 code that lands on a valid column.
// Otherwise col holds the columns as 32-bit indices. val64 optionally holds
// the caller's binary64 values in the same layout (used by the refinement's
// residual next to binary32 val).
#ifndef RPCG_SELL_VEC64
#define RPCG_SELL_VEC64 2
#endif
template <typename T>
__host__ __device__ constexpr int sell_vec()
{
    return sizeof(T) == 8 ? RPCG_SELL_VEC64 : 1;
}

template <typename T>
struct SellMat {
    int n;
    int nslices;
    const long long *off; // [nslices + 1]
    const T *val;
    const int *col;
    const int *row_ptr;   // the caller's CSR row pointers (row lengths)
    const unsigned char *len8; // row lengths as bytes when every row has < 256 entries, else null
    const unsigned short *col16; // when non-null: column codes (col unused)
    const int *cfirst;    // with col16: [nslices] first-column offset of each slice
    const double *val64;  // optional binary64 values (same layout), else null
};

struct LaunchCfg {
    int grid;
    int block;
    bool early_exit;
    int fpe_size;
    bool fallback;
    int xcd_parts; // SpMV: number of contiguous slice ranges (one per XCD)
    hipStream_t stream;
};

// ---- launch functions (return hipError_t of the launch) ----
// `stride` is the slot capacity of the dot workspaces (see DotWs).

hipError_t launch_exdot(int mode, long long n, const double *x, const double *y, double *out,
                        const DotWs &ws, int stride, DotInfo *info, const LaunchCfg &cfg);
hipError_t launch_exdot_partial(long long n, const double *x, const double *y, long long *digits,
                                const DotWs &ws, int stride, DotInfo *info, const LaunchCfg &cfg);
hipError_t launch_acc_round(const long long *digits, double *out, hipStream_t s);
// Exponent range (floor(log2 |v|)) of the nonzero finite entries of v, merged into *emin, *emax.
hipError_t launch_exp_range(long long n, const double *v, int *emin, int *emax, hipStream_t s);
// CSR SpMV (nnz = row_ptr[n]): workgroups of 512 rows, one per row block;
// the staging chunk is chosen by the average row length.
hipError_t launch_spmv_csr(int n, long long nnz, const int *row_ptr, const int *col, const double *val,
                           const double *x, double *y, hipStream_t s);

// CSR structural check (*bad set if malformed), slice sizes (64 times the
// slice's longest row, into off_plus1), longest row, and the range of the
// 16-bit column codes (*max_delta <= 32767 iff every code fits), one
// wavefront per 64-row slice.
hipError_t launch_csr_scan(int n, int nnz, const int *row_ptr, const int *col, int vec, long long *off_plus1,
                           int *bad, int *max_len, long long *max_delta, hipStream_t s);

hipError_t launch_sell_scan(long long *off, int nslices, hipStream_t s);
// Fill the sliced-ELL arrays from the CSR. The source values are binary64
// (val64_in) or binary32 (val32_in, exactly one of the two non-null); sval64
// receives them as binary64, sval32 rounded to nearest binary32; either
// output may be null.
hipError_t launch_sell_fill(int n, const int *row_ptr, const int *col, const double *val64_in,
                            const float *val32_in, int vec, const long long *off, double *sval64, float *sval32,
                            int *scol, unsigned short *scol16, int *cfirst, unsigned char *len8, hipStream_t s);
// y = A x on a binary64 sliced-ELL copy (grid workgroups of 256 threads).
hipError_t launch_sell_spmv(const SellMat<double> &A, const double *x, double *y, int grid, hipStream_t s);

template <typename T>
struct PcgVecs {
    const T *b;
    T *x, *r, *z, *d, *w, *dinv;
    double *hist;      // optional [maxit + 1]: tau history (widened to binary64)
    double *beta_hist; // [maxit + 1]: beta of every iteration (widened to binary64)
};

// The PCG launchers exist for T = double (the paper's solver) and T = float
// (the binary32 inner solver of the mixed-precision refinement). Scalars in
// PcgState are held as binary64; binary32 values widen to it exactly.

// Setup (state init, partials, one-workgroup finalize) into ws3[0..2].
template <typename T>
hipError_t launch_pcg_setup(int mode, const SellMat<T> &A, const PcgVecs<T> &v, PcgState *st, const DotWs *ws3,
                            int stride, double tol, int maxit, const LaunchCfg &cfg);
// Iteration l: K1 writes its partials to `ws`; K2 merges them (Gd slots) and
// writes two dots into ws2[0..1]; K3 merges those (G slots).
template <typename T>
hipError_t launch_pcg_spmv_dot(int mode, const SellMat<T> &A, const PcgVecs<T> &v, PcgState *st,
                               const DotWs &ws, int stride, const LaunchCfg &cfg);
template <typename T>
hipError_t launch_pcg_update(int mode, int l, int n, const PcgVecs<T> &v, PcgState *st, const DotWs &wsd, int Gd,
                             const DotWs *ws2, int stride, const LaunchCfg &cfg);
// s3: also apply the iterate update of iteration l (the Jacobi solver; the
// factored solver's update kernel applies it itself).
template <typename T>
hipError_t launch_pcg_direction(int mode, int l, int n, const PcgVecs<T> &v, PcgState *st, const DotWs *ws2, int G,
                                int stride, const LaunchCfg &cfg, bool s3);

// ---- mixed-precision refinement (binary64 outer loop) ----

// Outer-loop state on the device.
struct IrState {
    double rr;      // <r, r> of the current outer step (exact, rounded once)
    double bb;      // <b, b>
    double thr;     // RN(RN(tol*tol) * <b,b>)
    int k;          // outer step whose residual was last formed
    int stop;       // nonzero: converged, out of outer steps or failed
    int status;     // outer status (rpcg codes)
    int scale;      // s of the current correction: inner rhs = RN32(r 2^-s)
    int flags;
    int pad;
    long long escapes;
};

// r = RN(b - A x) with every row summed exactly (binary64 values A.val64 of
// the sliced-ELL copy), and the workgroup partials of <r, r> into ws (exact
// dot, expansion length 3).
hipError_t launch_ir_residual(const SellMat<float> &A, const double *b, const double *x, double *r, IrState *ist,
                              const DotWs &ws, int stride, const LaunchCfg &cfg);
// Merge <r, r> (G slots), record rr_hist[k], decide whether to stop, and for
// a further correction the inner right-hand side rf = RN32(r 2^-s) and c = 0.
hipError_t launch_ir_prepare(int k, int maxit, double tol, int n, const double *r, float *rf, float *c,
                             double *rr_hist, IrState *ist, const DotWs &ws, int G, int stride, const LaunchCfg &cfg);
// x = RN(x + c 2^s).
hipError_t launch_ir_update(int n, double *x, const float *c, const IrState *ist, const LaunchCfg &cfg);


// ---- PCG with a factored preconditioner M^-1 = G G^T + eps I ----

// G and G^T as CSR (device arrays), both n x n.
struct FacPre {
    const int *g_rp, *g_col;
    const double *g_val;
    const int *gt_rp, *gt_col;
    const double *gt_val;
    double eps;
};

// Setup: r = b - A x0, partials of <r,r> (ws3[1]) and <b,b> (ws3[2]); t = G^T r;
// z = G t + eps r, d = z, partials of <z,r> (ws3[0]); merge of the three.
// Every step that writes partials runs on cfg.grid workgroups.
hipError_t launch_fac_setup(int mode, const SellMat<double> &A, const FacPre &P, const PcgVecs<double> &v, double *t,
                            PcgState *st, const DotWs *ws3, int stride, double tol, int maxit, const LaunchCfg &cfg);
// Iteration l after the SpMV kernel (partials of <d,w> in wsd, Gd slots), two
// launches: merge delta, rho; x update; r update read from v.r and written to
// r_new (the caller alternates the two buffers), partials of <r,r> (ws[1]),
// t = G^T r; then z = G t + eps r with partials of <z,r> (ws[0]). The
// direction kernel then merges ws[0] (beta) and ws[1] (tau).
hipError_t launch_fac_update(int mode, int l, int n, const FacPre &P, const PcgVecs<double> &v, double *r_new,
                             double *t, PcgState *st, const DotWs &wsd, int Gd, const DotWs *ws, int stride,
                             const LaunchCfg &cfg);

// ---- batched solves (many independent systems per launch) ----

// Per-system constants of a batch. Rows of system s sit at [row0, row0 + n)
// of the concatenated vectors, its slices at [slice0, slice0 + nslices) of
// the concatenated sliced-ELL copy (slices never span systems), and its
// dot partials in slots [slot0, slot1).
struct BatchSys {
    long long row0;
    long long slice0;
    int n;
    int nslices;
    int slot0;
    int slot1;
    const int *row_ptr; // the caller's CSR row pointers of the system
};

// One run of work: slices [s0, s1) of system `sys`, processed by one
// workgroup, whose dot partials go to slot `slot`.
struct BatchRun {
    int sys;
    int s0;
    int s1;
    int slot;
};

struct BatchArgs {
    int nsys;
    const BatchSys *sys;
    const BatchRun *runs;  // runs of workgroup g: [wg_run[g], wg_run[g + 1])
    const int *wg_run;
    // concatenated sliced-ELL copy (binary64 values, two-entry interleave)
    const long long *off;
    const double *val;
    const int *col;
    const unsigned short *col16;
    const int *cfirst;
    const unsigned char *len8; // indexed by concatenated row
    // concatenated vectors
    const double *b;
    double *x, *r, *z, *d, *w, *dinv;
    PcgState *st;          // [nsys]
    double *const *hist;   // [nsys] tau histories (maxit + 1 each, entries may be null), or null
    int *active;           // number of systems not done
};

// Setup of every system (state, partials of <z,r>, <r,r>, <b,b> into ws3,
// one workgroup per system to merge them).
hipError_t launch_batch_setup(int mode, bool col16, const BatchArgs &a, int grid, int block, const DotWs *ws3,
                              int stride, double tol, int maxit, const LaunchCfg &cfg);
// One iteration of every system not done: SpMV + <d,w> partials (ws[0]),
// per-system rho, updates + <z,r>, <r,r> partials (ws[1], ws[2]), per-system
// stopping test and gamma, direction update.
hipError_t launch_batch_iteration(int mode, bool col16, const BatchArgs &a, int grid, int block, const DotWs *ws3,
                                  int stride, const LaunchCfg &cfg);

} // namespace rpcg
