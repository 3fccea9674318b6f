/*
 * rpcg.h - reproducible Jacobi-preconditioned Conjugate Gradient on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Iakymchuk, Barreda, Graillat, Aliaga, Quintana-Orti,
 * "Reproducibility of Parallel Preconditioned Conjugate Gradient in Hybrid
 * Programming Environments" (arXiv:2005.07282).
 *
 * Problem (Section 3.1): A x = b with A an n x n sparse symmetric positive
 * definite matrix with nnz stored entries, b and x vectors of length n,
 * Jacobi preconditioner M = diag(A), iteration of Fig. 1 in the order of
 * Fig. 2 (S8 computed together with S6, Section 3.2).
 *
 * Reproducibility (Section 4): in the exact modes every dot product is the
 * exact sum of products rounded once to nearest-even (Sections 2, 2.1, 4.3),
 * SpMV rows are sequential fma chains in storage order and the axpy-type
 * updates are single fma operations (Section 4.3). Results are therefore
 * bit-identical for any launch configuration.
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless marked "host". The caller owns all
 *    arrays; the library owns only its context workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Work is enqueued on it in order.
 *  - Return value: 0 ok, > 0 warning (outputs valid), < 0 error (outputs
 *    undefined; device memory given as output may have been written).
 *  - Nothing is thrown across the interface.
 *  - Calls on one context must not overlap (one context per host thread).
 */
#ifndef RPCG_H
#define RPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reduction mode of every dot product (Section 5.2 names the paper's three
 * variants: Regular, Exblas, Opt = FPE8EE).
 *  PLAIN  - ordinary binary64 partial sums in a fixed tree; deterministic for
 *           one launch configuration but not across configurations.
 *  FPE    - per-lane floating-point expansions (two of size fpe_size: result
 *           and error, Section 4.2) updated with TwoSum (Alg. 1, 4) over
 *           TwoProd (Alg. 2), merged by fpesum (Alg. 3) in a fixed order
 *           within each wavefront; each wavefront's expansion is then summed
 *           exactly with the others and rounded once (the value NearSum gives,
 *           Section 4.3); see fpe_fallback for what happens when an expansion
 *           is too short.
 *  EXBLAS - per-lane expansion flushed into a workgroup long accumulator
 *           (Section 2.1 and 4.1), accumulators summed as integers, rounded
 *           once (exblas Round, Section 4.3). */
typedef enum { RPCG_MODE_PLAIN = 0, RPCG_MODE_FPE = 1, RPCG_MODE_EXBLAS = 2 } rpcg_mode;

enum {
    RPCG_OK = 0,
    RPCG_WARN_MAXIT = 1,        /* tau > threshold after maxit iterations */
    RPCG_WARN_FPE_INEXACT = 2,  /* FPE capacity exceeded (Section 4.3 warning) and no
                                   fallback, or a product left the exact domain */
    RPCG_ERR_INVALID = -1,      /* bad argument */
    RPCG_ERR_HIP = -2,          /* a HIP runtime call failed */
    RPCG_ERR_OOM = -3,          /* workspace allocation failed */
    RPCG_ERR_NOT_SPD = -4,      /* a diagonal entry is missing or not > 0 */
    RPCG_ERR_BREAKDOWN = -5,    /* <d, A d> <= 0 inside the loop */
    RPCG_ERR_NONFINITE = -6     /* inf/NaN in the input or an overflowing product */
};

/* Compressed sparse rows, zero-based. row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = nnz; 0 <= col_idx[k] < n. Column order inside a row is the
 * order of the SpMV fma chain (Section 4.3). All three arrays are device
 * memory and are only read. */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
} rpcg_csr;

/* Options. Fill with rpcg_opts_default() first, then change fields. */
typedef struct {
    double tol;            /* stop when <r,r> <= RN(RN(tol*tol) * <b,b>) (Fig. 1 tau_max; default 1e-8, Section 5.1) */
    int32_t maxit;         /* default 2000 */
    int32_t fpe_size;      /* expansion length p, 1..8 (Section 4.2: tunable); 0 = auto (default):
                              4 in FPE mode; in EXBLAS mode (whose result does not depend on
                              it) 3, and 4 in the binary64 solver's SpMV and setup kernels */
    int32_t early_exit;    /* FPE mode: stop propagating zero errors (Section 4.2); default 1.
                              Results do not depend on it. The EXBLAS lane path always runs
                              every level (a divergent exit saves nothing on a 64-wide
                              wavefront) */
    int32_t fpe_fallback;  /* FPE mode: what an expansion cannot hold (an escape, the
                              capacity warning of Section 4.3) is kept exactly in a long
                              accumulator, so the result stays exact (default 1); 0 drops
                              it as the expansion-only variant does (RPCG_WARN_FPE_INEXACT).
                              Escapes arise in the lanes and in the wavefront merges; the
                              sum across wavefronts and workgroups is exact. */
    int32_t block_size;    /* threads per workgroup of the dot and vector kernels:
                              0 = auto, else 64..1024, multiple of 64 */
    int32_t grid_size;     /* workgroups of the dot and vector kernels: 0 = auto, else 1..65536 */
    int32_t timing;        /* 1: bracket every solver kernel with HIP events and report
                              per-kernel times in rpcg_result (solver only); 2..65: bracket
                              only the SpMV+dot kernel, of every (timing-1)-th iteration
                              (iterations 0, timing-1, ...; 2 = every iteration): fewer
                              events in the loop; 0: none (default). Other values:
                              RPCG_ERR_INVALID */
    int32_t xcd_parts;     /* SpMV work split into this many contiguous row ranges, one per
                              XCD (0 = auto = 1, no split). Results do not depend on it. */
    int32_t spmv_block_size; /* solver SpMV kernel: threads per workgroup (0 = auto) */
    int32_t spmv_grid_size;  /* solver SpMV kernel: workgroups (0 = auto) */
    int32_t no_col16;        /* 1: keep 32-bit column indices in the solver's matrix copy even
                                when every |column - row| fits 16 bits (default 0) */
    double *tau_history;   /* optional DEVICE array of maxit+1 doubles: tau^(0..L) */
} rpcg_opts;

/* Host-side result record (host memory). */
typedef struct {
    int32_t status;        /* same value as the return code */
    int32_t iterations;    /* L: loop bodies executed */
    double tau0;           /* <r0, r0> */
    double tau_final;      /* <r_L, r_L> */
    double threshold;      /* RN(RN(tol*tol) * <b,b>) */
    int64_t fpe_escapes;   /* FPE mode: values that did not stay in an expansion (overflow
                              remainders; in the standalone dot also the products that a lane
                              whose expansions keep overflowing adds straight into the long
                              accumulator, which only happens with fpe_fallback set) */
    int64_t fallbacks;     /* FPE mode: dots in which an escape was kept by the long accumulator */
    double setup_ms;       /* wall time of setup (solver) */
    double loop_ms;        /* wall time of the iteration loop (solver) */
    double k_spmv_dot_ms;  /* timing>=1: summed HIP-event time of the SpMV+dot kernel */
    double k_update_ms;    /* timing=1: summed time of the update+two-dot kernel (0 with timing>=2) */
    double k_direction_ms; /* timing=1: summed time of the direction-update kernel (0 with timing>=2) */
    int32_t k_launches;    /* timing>=1: iterations whose kernels were timed */
    int32_t grid_size;     /* launch configuration actually used */
    int32_t block_size;
} rpcg_result;

typedef struct rpcg_ctx rpcg_ctx;

void rpcg_opts_default(rpcg_opts *opts /* host */);
const char *rpcg_status_string(int status);

/* Create a context on HIP device `device` (made current for the calls).
 * *ctx receives a handle owned by the caller until rpcg_destroy. */
int rpcg_create(rpcg_ctx **ctx /* host */, int device);
void rpcg_destroy(rpcg_ctx *ctx);

/* Dot product out[0] = <x, y> over n elements (Section 2.1 exdot; Section 4.1
 * Listing 1 for EXBLAS, Section 4.2 Listing 2 for FPE; Section 4.3 for the
 * final rounding). x, y: device arrays of n doubles; out: device pointer to
 * one double. n >= 0 (n = 0 gives +0). In FPE and EXBLAS mode the result is
 * the exact dot rounded to nearest-even whenever every nonzero product has
 * |x_i y_i| >= 2^-969 (TwoProd exact, Alg. 2) and sum |x_i y_i| < 2^1023
 * (no expansion overflows); a product below 2^-969 gives
 * RPCG_WARN_FPE_INEXACT, an inf/NaN input or an overflow gives
 * RPCG_ERR_NONFINITE with out = NaN.
 * `res` (host, may be NULL): when given, the call waits for the stream and
 * fills status, fpe_escapes and fallbacks; when NULL the call is fully
 * asynchronous and returns RPCG_OK after enqueueing. `opts` may be NULL. */
int rpcg_exdot(rpcg_ctx *ctx, rpcg_mode mode, int64_t n, const double *x, const double *y,
               double *out, const rpcg_opts *opts, rpcg_result *res, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the dot
 * product of rpcg_exdot, same arguments, same kernels and same results,
 * without a context. Its workgroup slots and counters live in a static
 * device array of about 1.3 MB per GPU (allocated when the library is
 * loaded, held until the process ends), so the call allocates nothing; it
 * runs on the current device. It holds at most RPCG_NOALLOC_MAX_GROUPS
 * workgroups: opts->grid_size above that gives RPCG_ERR_INVALID, and the
 * automatic grid is capped there (n itself is unbounded). Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams or host threads) race and give undefined results; calls ordered
 * on one stream are safe. The counters are cleared by a small kernel at the
 * start of each call (no memset node, so the call can be captured into a
 * graph when res is NULL). res: as rpcg_exdot (when given, the call waits
 * for the stream, which a capturing caller must avoid). */
#define RPCG_NOALLOC_MAX_GROUPS 2048
int rpcg_exdot_noalloc(rpcg_mode mode, int64_t n, const double *x, const double *y, double *out,
                       const rpcg_opts *opts, rpcg_result *res, void *stream);

/* y = A x (Section 4.3 SpMV): y_i = fold over the stored entries of row i in
 * order of acc = fma(a_ik, x[col_k], acc), acc starting at +0. A: device CSR
 * (see rpcg_csr; its structure is not checked here, a malformed matrix is
 * undefined behaviour), x: n doubles, y: n doubles (must not alias x).
 * Asynchronous; returns after enqueueing. */
int rpcg_spmv(rpcg_ctx *ctx, const rpcg_csr *A /* host struct */, const double *x, double *y,
              void *stream);

/* A matrix prepared for repeated products (Section 4.3 SpMV): a device copy
 * in the solver's sliced-ELL layout (binary64 values, 16-bit column codes
 * where the columns allow them; about 10 bytes per stored entry plus 9 bytes
 * per row), owned by the handle. Products with it are the same fma chains as
 * rpcg_spmv, so y is bit-identical to rpcg_spmv on the matrix it was made
 * from, at the streaming rate of the solver's own SpMV. */
typedef struct rpcg_smat rpcg_smat;

/* Builds the copy of A (device CSR; its structure is checked on the device,
 * RPCG_ERR_INVALID if row_ptr or a column index is out of range) on ctx's
 * device and waits for the stream. The copy does not refer to A afterwards:
 * A may be freed or changed (the copy keeps the values it was made from).
 * *out receives the handle, or NULL on error (RPCG_ERR_INVALID for NULL
 * ctx, A or out; RPCG_ERR_OOM / RPCG_ERR_HIP if device memory runs out).
 * Uses ctx's scratch memory while it runs: calls on one context must not
 * overlap. */
int rpcg_smat_create(rpcg_ctx *ctx, const rpcg_csr *A /* host struct */, rpcg_smat **out, void *stream);

/* y = A x with a prepared matrix: y_i = fold over the stored entries of row
 * i in order of acc = fma(a_ik, x[col_k], acc) from +0. x, y: n doubles on
 * the matrix's device; y must not alias x (RPCG_ERR_INVALID). Asynchronous;
 * returns after enqueueing. Products on different streams may overlap (the
 * handle is only read). */
int rpcg_smat_spmv(rpcg_smat *M, const double *x, double *y, void *stream);

/* Frees the copy (NULL is ignored). No product with it may be pending. */
void rpcg_smat_destroy(rpcg_smat *M);

/* Expansion length for FPE mode bound to the data's dynamic range (the
 * binding of the FPE length to the dynamic range that Section 7 proposes as
 * future work). With R = largest minus smallest binary exponent over the
 * nonzero finite entries of A and b, *p = min(8, 4 + floor(2R / 53)): 4, the
 * default, on well-scaled data, one more term per 53 bits of the range of
 * the products. The choice affects speed only: with fpe_fallback set,
 * whatever an expansion cannot hold goes to a long accumulator and results
 * stay exact. *range (may be NULL) receives R. Waits for completion.
 * Errors: RPCG_ERR_INVALID for NULL ctx, A, p or (n > 0) b. */
int rpcg_fpe_size_auto(rpcg_ctx *ctx, const rpcg_csr *A /* host struct */, const double *b,
                       int32_t *p /* host */, int32_t *range /* host */, void *stream);

/* Solve A x = b with Jacobi-PCG (Fig. 1 / Fig. 2). b: n doubles; x: n
 * doubles, in: starting guess x^(0), out: final iterate. A must be SPD with a
 * positive stored diagonal entry in every row. The CSR structure is checked
 * on the device first (RPCG_ERR_INVALID if row_ptr or a column index is out
 * of range); the library then keeps a sliced-ELL copy of A for the
 * iteration (same rows, same entry order). Waits for completion; `res`
 * (host, may be NULL) receives iterations, tau, status and timings. The
 * returned status is also written to res->status. */
int rpcg_pcg_solve(rpcg_ctx *ctx, rpcg_mode mode, const rpcg_csr *A /* host struct */,
                   const double *b, double *x, const rpcg_opts *opts, rpcg_result *res,
                   void *stream);

/* Jacobi-PCG with the Jacobi step replaced by a factored preconditioner
 * M^-1 = G G^T + eps I (the form of the learned preconditioner; M^-1 is SPD
 * whenever G is nonsingular or eps > 0). G and its transpose Gt are n x n
 * CSR matrices given separately (Gt must equal G^T; it is not checked), so
 * that S5 of Fig. 1 is three row-wise steps in storage order: t = Gt r,
 * s = G t (fma chains from +0, as the SpMV of Section 4.3), and
 * z_i = fma(eps, r_i, s_i). Everything else is rpcg_pcg_solve; the exact
 * modes give results that are bit-identical for any launch configuration
 * given G. eps: finite, >= 0. The structure of A, G and Gt is checked on the
 * device (RPCG_ERR_INVALID); no diagonal condition applies. */
int rpcg_pcg_solve_factored(rpcg_ctx *ctx, rpcg_mode mode, const rpcg_csr *A /* host struct */,
                            const rpcg_csr *G /* host struct */, const rpcg_csr *Gt /* host struct */,
                            double eps, const double *b, double *x, const rpcg_opts *opts,
                            rpcg_result *res, void *stream);

/* ---- Binary32 solver and mixed-precision refinement ----
 * Extensions of the paper's method (whose solver is binary64 throughout):
 * the same Jacobi-PCG iteration with every value and every rounding in
 * binary32, and an iterative-refinement loop that wraps it in binary64. The
 * reproducible reductions carry over unchanged: the product of two binary32
 * values is exact in binary64, so the exact dot of binary32 vectors is the
 * exact sum of those products rounded once, directly to binary32. */

/* CSR with binary32 values (same conventions as rpcg_csr). */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const float *val;
} rpcg_csr_f32;

/* Jacobi-PCG (Fig. 1 / Fig. 2) entirely in binary32: dinv = RN32(1/a_ii),
 * SpMV rows as binary32 fma chains, the updates as binary32 fma, dots exact
 * and rounded once to binary32, rho, gamma and the stopping threshold
 * RN32(RN32(t*t) <b,b>) with t = RN32(tol) in binary32. b, x: n floats
 * (x: in x^(0), out: final iterate). tau_history (optional, device, maxit+1
 * doubles) and the scalars of `res` hold the binary32 values widened.
 * Options, statuses and waiting behaviour as rpcg_pcg_solve. */
int rpcg_pcg_solve_f32(rpcg_ctx *ctx, rpcg_mode mode, const rpcg_csr_f32 *A /* host struct */,
                       const float *b, float *x, const rpcg_opts *opts, rpcg_result *res,
                       void *stream);

/* Options of the refinement. Fill with rpcg_ir_opts_default() first. */
typedef struct {
    double tol;            /* outer: stop when <r,r> <= RN(RN(tol*tol) <b,b>) with r = b - A x
                              formed in binary64 (default 1e-10) */
    int32_t maxit;         /* outer corrections at most (default 50) */
    int32_t adaptive_inner; /* 1 (default): the inner tolerance of outer step k is
                              max(inner.tol, RN(0.25 * RN(sqrt(RN(thr / rr_k))))), with
                              thr the outer threshold and rr_k = <r,r> of the step, so the
                              last correction aims just below the outer target instead of
                              a full inner.tol reduction past it; 0: inner.tol for every
                              step. Other values: RPCG_ERR_INVALID */
    double *rr_history;    /* optional DEVICE array of maxit+1 doubles: <r,r> of every outer step */
    rpcg_opts inner;       /* the binary32 inner solves: tol (default 1e-4), maxit (default 2000),
                              expansion and launch options; its tau_history must be NULL */
} rpcg_ir_opts;

/* Host-side result record of the refinement. */
typedef struct {
    int32_t status;            /* same value as the return code */
    int32_t outer;             /* corrections applied */
    int32_t inner_iterations;  /* summed over the inner solves */
    int32_t last_inner_status; /* status of the last inner solve */
    double rr0;                /* <r,r> at x^(0) */
    double rr_final;           /* <r,r> at the returned x */
    double threshold;          /* RN(RN(tol*tol) <b,b>) */
    int64_t fpe_escapes;       /* summed over the inner solves (FPE mode) */
    double setup_ms;           /* wall time: matrix copies and <b,b> */
    double total_ms;           /* wall time of the whole call */
    double inner_ms;           /* wall time of the inner solves (their setup included) */
    double outer_ms;           /* wall time of the binary64 steps (residual, scaling, update) */
    double k_residual_ms;      /* HIP-event time of the residual kernels (inner.timing = 1) */
    double k_spmv_dot_ms;      /* inner.timing = 1: summed kernel times of the inner loops */
    double k_update_ms;
    double k_direction_ms;
    int32_t k_launches;        /* inner.timing = 1: inner iterations whose kernels were timed */
    int32_t pad1;
} rpcg_ir_result;

void rpcg_ir_opts_default(rpcg_ir_opts *opts /* host */);

/* Mixed-precision iterative refinement for A x = b. A: binary64 CSR as for
 * rpcg_pcg_solve; the inner solves use its values rounded to nearest
 * binary32. b, x: n doubles (x: in x^(0), out: final iterate).
 * Outer step k = 0, 1, ...: r = b - A x with every row summed exactly (a
 * long accumulator, Section 2.1) and rounded once; rr = <r,r> exact and
 * rounded once (Section 4.1); stop when rr <= RN(RN(tol*tol) <b,b>), or with
 * RPCG_WARN_MAXIT when k = maxit. Otherwise s = floor(e / 2) where
 * rr = m 2^e, 1 <= m < 2; the inner binary32 solve (rpcg_pcg_solve_f32
 * semantics, `mode` selects its dot products) runs on rf = RN32(r 2^-s) from
 * c = 0 to the step's inner tolerance (see adaptive_inner); x = RN(x + c 2^s). An inner solve that stops at its maxit is
 * accepted; an inner error ends the call with that error. The outer dots are
 * always exact (EXBLAS) whatever `mode` is. Waits for completion. */
int rpcg_ir_solve(rpcg_ctx *ctx, rpcg_mode mode, const rpcg_csr *A /* host struct */,
                  const double *b, double *x, const rpcg_ir_opts *opts, rpcg_ir_result *res,
                  void *stream);

/* ---- Batched solves ----
 * Many independent SPD systems solved together (an extension of the paper's
 * method): one concatenated sliced-ELL copy, one launch per kernel step for
 * all systems, iterations captured once into a HIP graph and replayed. In
 * the exact modes every scalar of a system is the rounded exact value of that
 * system's data alone, so each system's iteration count, tau history and
 * solution are bit-identical to rpcg_pcg_solve on that system alone, with the
 * same options, whatever the other systems, their order or the schedule. */

typedef struct rpcg_batch rpcg_batch;

/* Schedule of the streaming kernels: the choice of the autotuner. It changes
 * speed only, never results. */
typedef struct {
    int32_t policy;           /* 0: each workgroup takes one contiguous chunk of the concatenated
                                 slices (equal stored entries per chunk); 1: tiles of tile_slices
                                 slices of one system, systems interleaved, dealt round-robin */
    int32_t tile_slices;      /* policy 1: slices (64 rows each) per tile, >= 1 */
    int32_t grid_size;        /* workgroups of the streaming kernels, 1..65536 */
    int32_t block_size;       /* threads per workgroup: 64..1024, multiple of 64 */
    int32_t graph_iterations; /* iterations captured per graph, 1..64 */
    int32_t pad0;
    double ms_per_iteration;  /* set by rpcg_batch_tune: measured time of one iteration of the batch */
} rpcg_batch_tuning;

/* Aggregate figures of one batched solve (host memory). */
typedef struct {
    int32_t status;           /* most severe per-system status: the lowest error if a system
                                 failed, else the highest warning, else RPCG_OK */
    int32_t graph_launches;   /* graph replays */
    int32_t max_iterations;   /* largest per-system iteration count */
    int32_t repartitions;     /* times the work was re-spread over the systems still running */
    int64_t total_iterations; /* sum of the per-system iteration counts */
    double setup_ms;          /* wall time: copies in, setup kernels */
    double loop_ms;           /* wall time of the replays */
    double total_ms;          /* wall time of the call */
} rpcg_batch_stats;

/* Prepare a batch of nsys >= 1 systems. A: host array of nsys CSR structs
 * (device arrays, as for rpcg_pcg_solve, which must stay valid and unchanged
 * until rpcg_batch_destroy); every row's columns must be valid indices of its
 * own system. opts (may be NULL): tol, maxit, expansion length and fallback
 * for every system (launch fields are ignored: the schedule is the tuning).
 * The structure of every matrix is checked on the device (RPCG_ERR_INVALID);
 * the tuning is taken from the context's autotuner results for the same
 * sizes, else the default. *out receives a handle owned by the caller. */
int rpcg_batch_create(rpcg_ctx *ctx, rpcg_mode mode, int32_t nsys, const rpcg_csr *A /* host array */,
                      const rpcg_opts *opts, rpcg_batch **out /* host */, void *stream);
void rpcg_batch_destroy(rpcg_batch *batch);

int rpcg_batch_get_tuning(const rpcg_batch *batch, rpcg_batch_tuning *out /* host */);
/* Use this schedule from now on (RPCG_ERR_INVALID if a field is out of range). */
int rpcg_batch_set_tuning(rpcg_batch *batch, const rpcg_batch_tuning *tuning /* host */);

/* Autotuner: times trial_iterations (1..1000) iterations of the batch from
 * x = 0 on right-hand sides b (host array of nsys device pointers) for each
 * candidate schedule, twice (the faster trial counts), keeps the fastest for
 * this batch (among those within 1% of it, the one with the fewest
 * workgroups) and records it in the context for batches of the same sizes.
 * *chosen (may be NULL) receives it. */
int rpcg_batch_tune(rpcg_batch *batch, const double *const *b /* host array */, int32_t trial_iterations,
                    rpcg_batch_tuning *chosen /* host */, void *stream);

/* Solve every system: b, x: host arrays of nsys device pointers (n_s
 * doubles each; x: in x^(0), out: final iterate). tau_history (may be NULL,
 * entries may be NULL): host array of device pointers to maxit+1 doubles.
 * res (may be NULL): host array of nsys results (status, iterations, tau0,
 * tau_final, threshold, escapes; the timing fields hold the batch's).
 * stats may be NULL. Waits for completion. Returns the most severe
 * per-system status (as rpcg_batch_stats.status). */
int rpcg_batch_solve(rpcg_batch *batch, const double *const *b, double *const *x,
                     double *const *tau_history, rpcg_result *res, rpcg_batch_stats *stats,
                     void *stream);

/* ---- Learned preconditioner ----
 * An extension of the paper's method: a small convolutional network maps a
 * 7-point operator A on an N^3 grid (rows in z-y-x order) to a sparse factor
 * G on the lower-triangle pattern of A, and PCG runs with M^-1 = G G^T + eps I
 * (rpcg_pcg_solve_factored), which is SPD by construction.
 *
 * Network (per grid cell, zero padding, 3x3x3 kernels, tap t = 9(dz+1) +
 * 3(dy+1) + (dx+1) reading the cell at offset (dz, dy, dx)):
 *   features f: ln(|a_ij| / a_ii) of the -x, -y, -z neighbours (-4 if absent),
 *               (number of absent neighbours) / 6
 *   h1 = relu(conv1(f) + b1), h2 = relu(conv2(h1) + b2)   (16 channels each)
 *   o  = conv3(h2) + b3                                    (4 channels)
 *   G_ii = RN32(s_i exp(clamp(o_0, -4, 4))), G_i,j(k) = RN32(s_i o_k) for the
 *   -x, -y, -z neighbour j(k), s_i = RN32(1 / sqrt(a_ii)); G^T stored too.
 * Weights, features and hidden activations are bfloat16, products accumulate
 * in float32 on the matrix cores. Parameters (float32, RPCG_LP_NPARAMS):
 * W1 [27][16][4], b1 [16], W2 [27][16][16], b2 [16], W3 [27][4][16], b3 [4]
 * (weights [tap][out][in]).
 * Training loss for vectors u of a system: mean |G G^T A u + eps A u - u|^2 /
 * |u|^2; its gradient reaches the parameters through the network's own
 * backward kernels, with weight gradients summed in a fixed order. */
#define RPCG_LP_NPARAMS 10404

typedef struct rpcg_lpnet rpcg_lpnet;

/* Structure of G and G^T for an N^3 grid: rows of G hold the -z, -y, -x
 * neighbours and the diagonal, rows of G^T the diagonal and the +x, +y, +z
 * neighbours (ascending columns); both have rpcg_lp_pattern_nnz(N) =
 * 4 N^3 - 3 N^2 entries. Host arrays of N^3 + 1 and nnz entries. */
int64_t rpcg_lp_pattern_nnz(int32_t N);
int rpcg_lp_pattern(int32_t N, int32_t *g_row_ptr, int32_t *g_col, int32_t *gt_row_ptr, int32_t *gt_col);

/* A network for systems on N^3 grids, batches of up to max_batch systems
 * (device workspace of roughly 230 bytes per cell and system, plus 32 nu
 * bytes per cell and system for the loss vectors, allocated by the first
 * loss or training call with nu vectors). max_batch <= 65535 and
 * N^3 max_batch <= 2^30, else RPCG_ERR_INVALID. Parameters start at zero;
 * set them with rpcg_lp_set_params. Calls on one network must not overlap. */
int rpcg_lp_create(rpcg_ctx *ctx, int32_t N, int32_t max_batch, rpcg_lpnet **out /* host */);
void rpcg_lp_destroy(rpcg_lpnet *net);
/* params: host array of RPCG_LP_NPARAMS floats (layout above). Setting them
 * also resets the optimiser state. */
int rpcg_lp_set_params(rpcg_lpnet *net, const float *params);
int rpcg_lp_get_params(rpcg_lpnet *net, float *params);

/* Network outputs o (device, float32 [nb][N^3][4]; may be NULL to run the
 * pass only) for nb systems A (host array of device CSR 7-point operators on
 * the N^3 grid). RPCG_ERR_NOT_SPD if a diagonal entry is missing or not
 * positive (o is then undefined). Waits for completion (the diagonal check).
 * Every call below runs this forward pass on its own systems first. */
int rpcg_lp_forward(rpcg_lpnet *net, int32_t nb, const rpcg_csr *A, float *o, void *stream);
/* G and G^T of nb systems into caller-allocated device CSR (structure from
 * rpcg_lp_pattern, values written as binary64). Waits for completion. */
int rpcg_lp_factor(rpcg_lpnet *net, int32_t nb, const rpcg_csr *A, rpcg_csr *G, rpcg_csr *Gt, void *stream);
/* Training loss (host, may be NULL) and its gradient with respect to the
 * outputs (device, binary64 [nb][N^3][4], may be NULL), averaged over the nb
 * systems and their nu vectors u (host array of nb * nu device pointers,
 * system-major; nb * nu <= 65535, else RPCG_ERR_INVALID). Waits for
 * completion. */
int rpcg_lp_loss_grad(rpcg_lpnet *net, int32_t nb, const rpcg_csr *A, const double *const *u, int32_t nu,
                      double eps, double *loss, double *dout, void *stream);
/* Parameter gradient (device, float32 RPCG_LP_NPARAMS) for an output gradient
 * dout (device, binary64 [nb][N^3][4], rounded to bfloat16 first), summed in
 * a fixed order (bit-reproducible). Waits for completion. */
int rpcg_lp_backward(rpcg_lpnet *net, int32_t nb, const rpcg_csr *A, const double *dout, float *grad,
                     void *stream);
/* One optimisation step (Adam, beta1 0.9, beta2 0.999, epsilon 1e-8, step
 * size lr) on the loss of nb systems; *loss (host, may be NULL) receives the
 * loss before the step. Waits for completion. */
int rpcg_lp_train_step(rpcg_lpnet *net, int32_t nb, const rpcg_csr *A, const double *const *u, int32_t nu,
                       double eps, float lr, double *loss, void *stream);

/* Long-accumulator interface (Section 4.3, Listing 3: the per-process
 * accumulator that is summed as integers across processes, then rounded).
 * The accumulator is RPCG_ACC_DIGITS signed 64-bit digits; digit k has weight
 * 2^(32 k + RPCG_ACC_EXP0). Any integer sum of such vectors (e.g. an
 * all-reduce over GPUs) represents the sum of the dots exactly as long as
 * fewer than 2^29 vectors are added. */
#define RPCG_ACC_DIGITS 68
#define RPCG_ACC_EXP0 (-1088)

/* digits[0..RPCG_ACC_DIGITS) = exact <x,y> (device array, overwritten).
 * Same domain as rpcg_exdot. Asynchronous. */
int rpcg_exdot_partial(rpcg_ctx *ctx, int64_t n, const double *x, const double *y,
                       int64_t *digits, void *stream);

/* out[0] = the value of `digits` rounded to nearest-even (device arrays).
 * Asynchronous. */
int rpcg_acc_round(rpcg_ctx *ctx, const int64_t *digits, double *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RPCG_H */
