/*
 * CPU oracle for the reproducible Jacobi-PCG hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library links, loads or calls
 * this file; only the tests, the smoke check and the bench's CPU-baseline
 * leg do. It shares no code with the GPU path.
 *
 * It is the plain definition of what the method computes, run slowly:
 *
 *  - exact dot product (Sections 2 and 2.1: the long-accumulator approach,
 *    whose result is rounded once; Section 4.3 "Round"/"NearSum" give the
 *    correctly rounded value): every product x_i*y_i is formed exactly as a
 *    106-bit integer times a power of two, added into a fixed-point big
 *    integer whose least significant bit is 2^-2148 (the smallest possible
 *    product of two binary64 numbers), and the total is rounded once to the
 *    nearest binary64, ties to even (IEEE 754 default rounding, Section 2).
 *    The integer sum does not depend on the order of the terms.
 *  - sparse matrix-vector product (Section 4.3, SpMV paragraph): per row,
 *    sequential fma over the stored entries in CSR order, starting from +0.
 *  - Jacobi-preconditioned CG (Fig. 1 steps S1-S8 in the order of Fig. 2,
 *    S8 merged with S6 as in Section 3.2), axpy-type updates by fma
 *    (Section 4.3), preconditioner by the precomputed inverse diagonal times
 *    the vector (Section 4.3, preconditioner paragraph).
 *
 * Threads (OpenMP): rows of the SpMV and of the exact residual, and the
 * element-wise loops, are split over threads; every element is computed
 * by the same operations whatever thread computes it. The exact dot gives
 * each thread a contiguous range of the terms and its own accumulator, and
 * the accumulators are added as integers, which is exact: the result does
 * not depend on the number of threads (a test compares 1 thread with all).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -mfma -fopenmp -fPIC -shared
 * (-ffp-contract=off: no multiply-add is fused unless fma() is written).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- exact accumulator ------------------------------------------------ */

/* Bit k of the accumulator has weight 2^(k - ORC_BIAS). Products of two
 * finite doubles are integer multiples of 2^-2148 and below 2^2048; 136
 * limbs of 32 bits (4352 bits) leave more than 150 bits of headroom. */
#define ORC_BIAS 2148
#define ORC_LIMBS 136

typedef struct {
    uint32_t pos[ORC_LIMBS]; /* magnitude of the positive terms */
    uint32_t neg[ORC_LIMBS]; /* magnitude of the negative terms */
    int nonfinite;           /* an inf or NaN was seen */
} orc_acc;

static void acc_clear(orc_acc *a) { memset(a, 0, sizeof(*a)); }

/* Split a finite double into (integer mantissa M, exponent E) with v = M*2^E,
 * 0 <= M < 2^53, E >= -1074; the sign is returned separately. */
static void split_double(double v, uint64_t *M, int *E, int *neg)
{
    uint64_t bits;
    memcpy(&bits, &v, sizeof bits);
    *neg = (int)(bits >> 63);
    int be = (int)((bits >> 52) & 0x7FF);
    uint64_t frac = bits & ((UINT64_C(1) << 52) - 1);
    if (be == 0) {          /* zero or subnormal: frac * 2^-1074 */
        *M = frac;
        *E = -1074;
    } else {                /* normal: (2^52 + frac) * 2^(be - 1075) */
        *M = frac | (UINT64_C(1) << 52);
        *E = be - 1075;
    }
}

/* A[] += m * 2^shift, m < 2^128 given as 4 little-endian 32-bit words. */
static void limbs_add_shifted(uint32_t *A, const uint32_t w[4], int shift)
{
    int li = shift / 32, b = shift % 32;
    uint32_t s[5];
    for (int j = 0; j < 5; ++j) {
        uint64_t cur = j < 4 ? w[j] : 0;
        uint64_t prev = j > 0 ? w[j - 1] : 0;
        uint64_t v = (cur << b) | (b ? (prev >> (32 - b)) : 0);
        s[j] = (uint32_t)v;
    }
    uint64_t carry = 0;
    int k = 0;
    for (; k < 5 && li + k < ORC_LIMBS; ++k) {
        uint64_t t = (uint64_t)A[li + k] + s[k] + carry;
        A[li + k] = (uint32_t)t;
        carry = t >> 32;
    }
    for (int j = li + k; carry && j < ORC_LIMBS; ++j) {
        uint64_t t = (uint64_t)A[j] + carry;
        A[j] = (uint32_t)t;
        carry = t >> 32;
    }
}

/* Add the exact product x*y. */
static void acc_add_product(orc_acc *a, double x, double y)
{
    if (!isfinite(x) || !isfinite(y)) { a->nonfinite = 1; return; }
    uint64_t mx, my; int ex, ey, sx, sy;
    split_double(x, &mx, &ex, &sx);
    split_double(y, &my, &ey, &sy);
    if (mx == 0 || my == 0) return;
    unsigned __int128 p = (unsigned __int128)mx * my; /* < 2^106, exact */
    uint32_t w[4];
    for (int j = 0; j < 4; ++j) w[j] = (uint32_t)(p >> (32 * j));
    int shift = ex + ey + ORC_BIAS;                   /* >= 0 */
    limbs_add_shifted((sx ^ sy) ? a->neg : a->pos, w, shift);
}

/* Add the exact value of a double (product with 1). */
static void acc_add_value(orc_acc *a, double v) { acc_add_product(a, v, 1.0); }

static int limbs_cmp(const uint32_t *A, const uint32_t *B)
{
    for (int k = ORC_LIMBS - 1; k >= 0; --k)
        if (A[k] != B[k]) return A[k] > B[k] ? 1 : -1;
    return 0;
}

/* D = A - B, requires A >= B. */
static void limbs_sub(uint32_t *D, const uint32_t *A, const uint32_t *B)
{
    int64_t borrow = 0;
    for (int k = 0; k < ORC_LIMBS; ++k) {
        int64_t t = (int64_t)A[k] - B[k] - borrow;
        borrow = t < 0;
        D[k] = (uint32_t)(t + (borrow ? (INT64_C(1) << 32) : 0));
    }
}

/* A += B (both magnitudes; the headroom above keeps the sum in range). */
static void limbs_add(uint32_t *A, const uint32_t *B)
{
    uint64_t carry = 0;
    for (int k = 0; k < ORC_LIMBS; ++k) {
        uint64_t t = (uint64_t)A[k] + B[k] + carry;
        A[k] = (uint32_t)t;
        carry = t >> 32;
    }
}

/* Exact sum of a[0..n) x b[0..n) products into acc: one accumulator per
 * thread over a contiguous range, then the accumulators added exactly. */
static void acc_add_dot(orc_acc *acc, int64_t n, const double *x, const double *y)
{
    #pragma omp parallel
    {
        orc_acc *t = (orc_acc *)malloc(sizeof(orc_acc));
        acc_clear(t);
        #pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) acc_add_product(t, x[i], y[i]);
        #pragma omp critical
        {
            limbs_add(acc->pos, t->pos);
            limbs_add(acc->neg, t->neg);
            acc->nonfinite |= t->nonfinite;
        }
        free(t);
    }
}

static int limbs_bit(const uint32_t *D, int k)
{
    if (k < 0 || k >= 32 * ORC_LIMBS) return 0;
    return (D[k / 32] >> (k % 32)) & 1;
}

/* Round (-1)^neg * D * 2^-ORC_BIAS to the nearest number with `prec`
 * significant bits, exponents down to a last-bit weight of 2^qmin
 * (subnormals) and overflow to infinity from 2^emax_inf - 2^(emax_inf-prec-1)
 * on (IEEE 754 round to nearest, ties to even). binary64: prec 53, qmin
 * -1074, emax_inf 1024. binary32: prec 24, qmin -149, emax_inf 128.
 * Zero gives +0. The value is returned as a double (exact for binary32). */
static double round_magnitude_fmt(const uint32_t *D, int neg, int prec, int qmin, int emax_inf)
{
    int top = -1;
    for (int k = ORC_LIMBS - 1; k >= 0 && top < 0; --k)
        if (D[k]) for (int b = 31; b >= 0; --b)
            if ((D[k] >> b) & 1) { top = 32 * k + b; break; }
    if (top < 0) return 0.0;
    int emsb = top - ORC_BIAS;               /* value in [2^emsb, 2^(emsb+1)) */
    if (emsb >= emax_inf) return neg ? -INFINITY : INFINITY;
    int q = emsb - (prec - 1);               /* weight of the last kept bit */
    if (q < qmin) q = qmin;                  /* subnormal range */
    int qb = q + ORC_BIAS;                   /* its bit index */
    uint64_t I = 0;
    for (int k = top; k >= qb; --k) I = (I << 1) | (uint64_t)limbs_bit(D, k);
    int half = limbs_bit(D, qb - 1);
    /* sticky: is any bit below the rounding bit (index qb-1) set? */
    int sticky = 0, lim = qb - 1;            /* bits [0, lim) */
    for (int k = 0; k < lim / 32 && !sticky; ++k) sticky = D[k] != 0;
    if (!sticky && lim % 32) sticky = (D[lim / 32] & ((UINT32_C(1) << (lim % 32)) - 1)) != 0;
    if (half && (sticky || (I & 1))) I += 1; /* I <= 2^prec */
    double r = ldexp((double)I, q);          /* exact; 2^emax_inf when rounding up at the top */
    if (r >= ldexp(1.0, emax_inf)) r = INFINITY;
    return neg ? -r : r;
}

static double round_magnitude(const uint32_t *D, int neg)
{
    return round_magnitude_fmt(D, neg, 53, -1074, 1024);
}

static double acc_round_fmt(const orc_acc *a, int prec, int qmin, int emax_inf)
{
    if (a->nonfinite) return NAN;
    uint32_t D[ORC_LIMBS];
    int c = limbs_cmp(a->pos, a->neg);
    if (c == 0) return 0.0;
    if (c > 0) { limbs_sub(D, a->pos, a->neg); return round_magnitude_fmt(D, 0, prec, qmin, emax_inf); }
    limbs_sub(D, a->neg, a->pos);
    return round_magnitude_fmt(D, 1, prec, qmin, emax_inf);
}

static double acc_round(const orc_acc *a) { return acc_round_fmt(a, 53, -1074, 1024); }

/* binary32 rounding of the exact value */
static float acc_round_f32(const orc_acc *a) { return (float)acc_round_fmt(a, 24, -149, 128); }

/* ---- exported API ------------------------------------------------------ */

/* Correctly rounded exact dot product of x and y (length n). NaN if any
 * input is not finite. */
double rpcg_oracle_exdot(int64_t n, const double *x, const double *y)
{
    orc_acc *a = (orc_acc *)malloc(sizeof(orc_acc));
    acc_clear(a);
    acc_add_dot(a, n, x, y);
    double r = acc_round(a);
    free(a);
    return r;
}

/* Exact value of the dot product as a signed fixed-point integer:
 * sum x_i y_i = (-1)^sign * sum_k limbs[k] 2^(32k - 2148). limbs has
 * rpcg_oracle_exact_limbs() entries. Returns 0, or -1 if an input is not
 * finite. */
int rpcg_oracle_exact_limbs(void) { return ORC_LIMBS; }

int rpcg_oracle_exdot_exact(int64_t n, const double *x, const double *y,
                            uint32_t *limbs, int *sign)
{
    orc_acc *a = (orc_acc *)malloc(sizeof(orc_acc));
    acc_clear(a);
    acc_add_dot(a, n, x, y);
    int rc = a->nonfinite ? -1 : 0;
    int c = limbs_cmp(a->pos, a->neg);
    if (c >= 0) { limbs_sub(limbs, a->pos, a->neg); *sign = 0; }
    else        { limbs_sub(limbs, a->neg, a->pos); *sign = 1; }
    free(a);
    return rc;
}

/* Round a signed fixed-point integer (same format as above) to double. */
double rpcg_oracle_round_limbs(const uint32_t *limbs, int sign)
{
    return round_magnitude(limbs, sign);
}

/* y = A x, row by row: acc = +0; acc = fma(val_k, x[col_k], acc) for the
 * stored entries of the row in CSR order. */
void rpcg_oracle_spmv(int32_t n, const int32_t *row_ptr, const int32_t *col,
                      const double *val, const double *x, double *y)
{
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            acc = fma(val[k], x[col[k]], acc);
        y[i] = acc;
    }
}

/* Residual with exact row sums: r_i = RN(b_i - sum_j a_ij x_j), each row
 * accumulated exactly and rounded once. */
void rpcg_oracle_true_residual(int32_t n, const int32_t *row_ptr, const int32_t *col,
                               const double *val, const double *b, const double *x,
                               double *r)
{
    #pragma omp parallel
    {
        orc_acc *a = (orc_acc *)malloc(sizeof(orc_acc));
        #pragma omp for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            acc_clear(a);
            acc_add_value(a, b[i]);
            for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
                acc_add_product(a, -val[k], x[col[k]]);
            r[i] = acc_round(a);
        }
        free(a);
    }
}

/* Jacobi preconditioner apply (Section 4.3): z_i = RN(dinv_i * r_i), with
 * dinv_i = RN(1 / a_ii) formed once at setup. */
static void jacobi_apply(int32_t n, const double *dinv, const double *r, double *z)
{
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
}

/* Status codes shared in value (not in code) with the library's header. */
#define ORC_OK 0
#define ORC_WARN_MAXIT 1
#define ORC_ERR_INVALID (-1)
#define ORC_ERR_NOT_SPD (-4)
#define ORC_ERR_BREAKDOWN (-5)
#define ORC_ERR_NONFINITE (-6)

/*
 * Jacobi-PCG on A x = b (Fig. 1 / Fig. 2).
 *   x      in: starting guess x^(0); out: final iterate
 *   tol    the loop runs while tau > thr, thr = RN(RN(tol*tol) * <b,b>),
 *          tau = <r,r> (both exact dots, rounded once)
 *   hist   optional [maxit+1]: tau^(0..L)
 *   trace_r, trace_d, trace_x optional [(maxit+1)*n]: r, d, x after each
 *          iteration (row l holds iteration l's vectors; d of row l is the
 *          search direction used by iteration l+1)
 *   *iters L, the number of loop bodies executed
 * Returns a status code.
 */
int rpcg_oracle_pcg(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const double *val, const double *b, double *x,
                    double tol, int32_t maxit, double *hist, int32_t *iters,
                    double *trace_r, double *trace_d, double *trace_x)
{
    *iters = 0;
    if (n < 0 || maxit < 0) return ORC_ERR_INVALID;
    double *dinv = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *r = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *z = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *d = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *w = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = ORC_OK;

    /* preconditioner M = diag(A): invert the diagonal once */
    for (int32_t i = 0; i < n && status == ORC_OK; ++i) {
        double aii = 0.0; int found = 0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) { aii = val[k]; found = 1; }
        if (!found || !(aii > 0.0)) status = ORC_ERR_NOT_SPD;
        else dinv[i] = 1.0 / aii;
    }
    for (int32_t i = 0; i < n && status == ORC_OK; ++i)
        if (!isfinite(b[i]) || !isfinite(x[i])) status = ORC_ERR_NONFINITE;
    if (status != ORC_OK) goto out;

    /* r = b - A x0;  z = M^-1 r;  d = z;  beta = <z,r>;  tau = <r,r> */
    rpcg_oracle_spmv(n, row_ptr, col, val, x, w);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
    jacobi_apply(n, dinv, r, z);
    for (int32_t i = 0; i < n; ++i) d[i] = z[i];
    double beta = rpcg_oracle_exdot(n, z, r);
    double tau = rpcg_oracle_exdot(n, r, r);
    double bb = rpcg_oracle_exdot(n, b, b);
    double thr = (tol * tol) * bb;
    if (hist) hist[0] = tau;
    if (trace_r) memcpy(trace_r, r, sizeof(double) * (size_t)n);
    if (trace_d) memcpy(trace_d, d, sizeof(double) * (size_t)n);
    if (trace_x) memcpy(trace_x, x, sizeof(double) * (size_t)n);
    if (!isfinite(tau) || !isfinite(bb)) { status = ORC_ERR_NONFINITE; goto out; }

    int32_t l = 0;
    while (tau > thr && l < maxit) {
        double beta_old = beta;
        rpcg_oracle_spmv(n, row_ptr, col, val, d, w);           /* S1 */
        double delta = rpcg_oracle_exdot(n, d, w);              /* S2 */
        if (!(delta > 0.0)) { status = isfinite(delta) ? ORC_ERR_BREAKDOWN : ORC_ERR_NONFINITE; break; }
        double rho = beta / delta;
        #pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) x[i] = fma(rho, d[i], x[i]);   /* S3 */
        #pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) r[i] = fma(-rho, w[i], r[i]);  /* S4 */
        jacobi_apply(n, dinv, r, z);                            /* S5 */
        beta = rpcg_oracle_exdot(n, z, r);                      /* S6 */
        tau = rpcg_oracle_exdot(n, r, r);                       /* S8 */
        double gamma = beta / beta_old;
        #pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) d[i] = fma(gamma, d[i], z[i]); /* S7 */
        l += 1;
        if (hist) hist[l] = tau;
        if (trace_r) memcpy(trace_r + (size_t)l * n, r, sizeof(double) * (size_t)n);
        if (trace_d) memcpy(trace_d + (size_t)l * n, d, sizeof(double) * (size_t)n);
        if (trace_x) memcpy(trace_x + (size_t)l * n, x, sizeof(double) * (size_t)n);
        if (!isfinite(tau)) { status = ORC_ERR_NONFINITE; break; }
    }
    *iters = l;
    if (status == ORC_OK && tau > thr) status = ORC_WARN_MAXIT;
out:
    free(dinv); free(r); free(z); free(d); free(w);
    return status;
}

/* ---- binary32 routines of the mixed-precision refinement ------------------
 * The inner solver of the refinement runs entirely in binary32: SpMV by fmaf
 * chains, exact dot products rounded once to binary32, fmaf updates, Jacobi
 * with the binary32 inverse diagonal. The outer loop keeps x, b and the
 * residual in binary64: residual rows accumulated exactly and rounded once,
 * exact norms, and the correction added as x + (double)c (scaled by a power
 * of two). */

/* Correctly rounded (binary32) exact dot product of two binary32 vectors. */
float rpcg_oracle_exdot_f32(int64_t n, const float *x, const float *y)
{
    orc_acc *a = (orc_acc *)malloc(sizeof(orc_acc));
    acc_clear(a);
    for (int64_t i = 0; i < n; ++i) acc_add_product(a, (double)x[i], (double)y[i]);
    float r = acc_round_f32(a);
    free(a);
    return r;
}

/* y = A x in binary32: acc = +0; acc = fmaf(val_k, x[col_k], acc) per row. */
void rpcg_oracle_spmv_f32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                          const float *val, const float *x, float *y)
{
    for (int32_t i = 0; i < n; ++i) {
        float acc = 0.0f;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            acc = fmaf(val[k], x[col[k]], acc);
        y[i] = acc;
    }
}

/* Jacobi-PCG in binary32, the loop of rpcg_oracle_pcg with every operation
 * in binary32: thr = RN32(RN32(tol32*tol32) * <b,b>), tol32 = RN32(tol).
 * hist (optional, maxit+1) receives tau^(0..L) widened to double.
 * trace_r, trace_d, trace_x (optional, [(maxit+1)*n] floats) receive r, d
 * and x after each iteration as in rpcg_oracle_pcg; thr_out (optional)
 * receives the threshold. */
int rpcg_oracle_pcg_f32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        const float *val, const float *b, float *x,
                        double tol, int32_t maxit, double *hist, int32_t *iters,
                        float *trace_r, float *trace_d, float *trace_x, float *thr_out)
{
    *iters = 0;
    if (n < 0 || maxit < 0) return ORC_ERR_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    float *dinv = malloc(sizeof(float) * nn), *r = malloc(sizeof(float) * nn);
    float *z = malloc(sizeof(float) * nn), *d = malloc(sizeof(float) * nn);
    float *w = malloc(sizeof(float) * nn);
    int status = ORC_OK;
    for (int32_t i = 0; i < n && status == ORC_OK; ++i) {
        float aii = 0.0f; int found = 0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) { aii = val[k]; found = 1; }
        if (!found || !(aii > 0.0f)) status = ORC_ERR_NOT_SPD;
        else dinv[i] = 1.0f / aii;
    }
    for (int32_t i = 0; i < n && status == ORC_OK; ++i)
        if (!isfinite(b[i]) || !isfinite(x[i])) status = ORC_ERR_NONFINITE;
    if (status != ORC_OK) goto out;
    rpcg_oracle_spmv_f32(n, row_ptr, col, val, x, w);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
    for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    for (int32_t i = 0; i < n; ++i) d[i] = z[i];
    float beta = rpcg_oracle_exdot_f32(n, z, r);
    float tau = rpcg_oracle_exdot_f32(n, r, r);
    float bb = rpcg_oracle_exdot_f32(n, b, b);
    float tol32 = (float)tol;
    float thr = (tol32 * tol32) * bb;
    if (thr_out) *thr_out = thr;
    if (hist) hist[0] = tau;
    if (trace_r) memcpy(trace_r, r, sizeof(float) * (size_t)n);
    if (trace_d) memcpy(trace_d, d, sizeof(float) * (size_t)n);
    if (trace_x) memcpy(trace_x, x, sizeof(float) * (size_t)n);
    if (!isfinite(tau) || !isfinite(bb)) { status = ORC_ERR_NONFINITE; goto out; }
    int32_t l = 0;
    while (tau > thr && l < maxit) {
        float beta_old = beta;
        rpcg_oracle_spmv_f32(n, row_ptr, col, val, d, w);
        float delta = rpcg_oracle_exdot_f32(n, d, w);
        if (!(delta > 0.0f)) { status = isfinite(delta) ? ORC_ERR_BREAKDOWN : ORC_ERR_NONFINITE; break; }
        float rho = beta / delta;
        for (int32_t i = 0; i < n; ++i) x[i] = fmaf(rho, d[i], x[i]);
        for (int32_t i = 0; i < n; ++i) r[i] = fmaf(-rho, w[i], r[i]);
        for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        beta = rpcg_oracle_exdot_f32(n, z, r);
        tau = rpcg_oracle_exdot_f32(n, r, r);
        float gamma = beta / beta_old;
        for (int32_t i = 0; i < n; ++i) d[i] = fmaf(gamma, d[i], z[i]);
        l += 1;
        if (hist) hist[l] = tau;
        if (trace_r) memcpy(trace_r + (size_t)l * n, r, sizeof(float) * (size_t)n);
        if (trace_d) memcpy(trace_d + (size_t)l * n, d, sizeof(float) * (size_t)n);
        if (trace_x) memcpy(trace_x + (size_t)l * n, x, sizeof(float) * (size_t)n);
        if (!isfinite(tau)) { status = ORC_ERR_NONFINITE; break; }
    }
    *iters = l;
    if (status == ORC_OK && tau > thr) status = ORC_WARN_MAXIT;
out:
    free(dinv); free(r); free(z); free(d); free(w);
    return status;
}

/* Power-of-two scale of the residual for the binary32 inner solve: the
 * inner right-hand side is RN32(r * 2^-s) with s = floor(E / 2), where
 * <r,r> = m 2^E, m in [1, 2) (binary64 exponent of rr), so that the scaled
 * residual has a norm near 1. */
int rpcg_oracle_ir_scale(double rr)
{
    int E;
    frexp(rr, &E);                /* rr = f 2^E, f in [0.5, 1) */
    E -= 1;                       /* rr = m 2^E, m in [1, 2) */
    return E >= 0 ? E / 2 : -((-E + 1) / 2);
}

/* Mixed-precision iterative refinement. A is given with binary64 values
 * (val); the inner solves use them rounded to nearest binary32, the outer
 * residual uses them as given.
 *   x: in x0, out: final iterate (binary64)
 *   outer loop k = 0, 1, ...: r = b - A x (rows exact, rounded once);
 *     rr = <r,r> (exact); hist[k] = rr; stop if rr <= RN(RN(tol*tol) <b,b>)
 *     or k = maxit; s = rpcg_oracle_ir_scale(rr);
 *     t = tol_in, or with adaptive = 1 max(tol_in, RN(0.25 RN(sqrt(RN(thr / rr)))))
 *     (the reduction the outer residual still needs, with a margin of 4);
 *     c = PCG32(RN32(A), RN32(r 2^-s), x0 = 0, t, maxit_in);
 *     x = RN(x + (double)c 2^s)
 *   *outer: corrections applied; *inner: total inner iterations;
 *   tin_hist (optional, maxit+1): the inner tolerance t of every correction.
 * Returns the outer status (OK, WARN_MAXIT) or the first inner error. */
int rpcg_oracle_ir(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *val64,
                   const double *b, double *x, double tol, int32_t maxit_out, double tol_in,
                   int32_t maxit_in, int32_t adaptive, double *hist, int32_t *outer, int32_t *inner,
                   double *tin_hist)
{
    *outer = 0; *inner = 0;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t nnz = n > 0 ? row_ptr[n] : 0;
    float *val32 = malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    double *r = malloc(sizeof(double) * nn);
    float *rf = malloc(sizeof(float) * nn), *c = malloc(sizeof(float) * nn);
    for (int32_t k = 0; k < nnz; ++k) val32[k] = (float)val64[k];
    double bb = rpcg_oracle_exdot(n, b, b);
    double thr = (tol * tol) * bb;
    int status = ORC_OK;
    for (int32_t k = 0;; ++k) {
        rpcg_oracle_true_residual(n, row_ptr, col, val64, b, x, r);
        double rr = rpcg_oracle_exdot(n, r, r);
        if (hist) hist[k] = rr;
        if (!isfinite(rr)) { status = ORC_ERR_NONFINITE; break; }
        if (rr <= thr) break;
        if (k == maxit_out) { status = ORC_WARN_MAXIT; break; }
        int sc = rpcg_oracle_ir_scale(rr);
        for (int32_t i = 0; i < n; ++i) rf[i] = (float)ldexp(r[i], -sc);
        for (int32_t i = 0; i < n; ++i) c[i] = 0.0f;
        double t = tol_in;
        if (adaptive) {
            double need = 0.25 * sqrt(thr / rr);
            if (need > t) t = need;
        }
        int32_t it = 0;
        if (tin_hist) tin_hist[k] = t;
        int st = rpcg_oracle_pcg_f32(n, row_ptr, col, val32, rf, c, t, maxit_in, NULL, &it, NULL, NULL, NULL, NULL);
        *inner += it;
        if (st < 0) { status = st; break; }
        for (int32_t i = 0; i < n; ++i) x[i] = x[i] + ldexp((double)c[i], sc);
        *outer = k + 1;
    }
    free(val32); free(r); free(rf); free(c);
    return status;
}

/* ---- PCG with a factored preconditioner M^-1 = G G^T + eps I ----------------
 * The learned preconditioner supplies G (a sparse matrix, in the workload the
 * lower triangle of A's pattern) and G^T explicitly as a second CSR, so that
 * both products are row-wise fma chains in storage order, as the SpMV of
 * Section 4.3. Only the preconditioner step S5 of Fig. 1 changes:
 *   t = G^T r,  s = G t,  z_i = fma(eps, r_i, s_i).
 * Every other step, and the exact dots, are those of rpcg_oracle_pcg,
 * including the optional traces of r, d and x. */
static void factored_apply(int32_t n, const int32_t *g_rp, const int32_t *g_col, const double *g_val,
                           const int32_t *gt_rp, const int32_t *gt_col, const double *gt_val, double eps,
                           const double *r, double *t, double *z)
{
    rpcg_oracle_spmv(n, gt_rp, gt_col, gt_val, r, t);
    rpcg_oracle_spmv(n, g_rp, g_col, g_val, t, z);
    for (int32_t i = 0; i < n; ++i) z[i] = fma(eps, r[i], z[i]);
}

int rpcg_oracle_pcg_factored(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                             const int32_t *g_rp, const int32_t *g_col, const double *g_val,
                             const int32_t *gt_rp, const int32_t *gt_col, const double *gt_val, double eps,
                             const double *b, double *x, double tol, int32_t maxit, double *hist, int32_t *iters,
                             double *trace_r, double *trace_d, double *trace_x)
{
    *iters = 0;
    if (n < 0 || maxit < 0) return ORC_ERR_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *r = malloc(sizeof(double) * nn), *z = malloc(sizeof(double) * nn);
    double *d = malloc(sizeof(double) * nn), *w = malloc(sizeof(double) * nn);
    double *t = malloc(sizeof(double) * nn);
    int status = ORC_OK;
    for (int32_t i = 0; i < n && status == ORC_OK; ++i)
        if (!isfinite(b[i]) || !isfinite(x[i])) status = ORC_ERR_NONFINITE;
    if (status != ORC_OK) goto out;
    rpcg_oracle_spmv(n, row_ptr, col, val, x, w);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
    factored_apply(n, g_rp, g_col, g_val, gt_rp, gt_col, gt_val, eps, r, t, z);
    for (int32_t i = 0; i < n; ++i) d[i] = z[i];
    double beta = rpcg_oracle_exdot(n, z, r);
    double tau = rpcg_oracle_exdot(n, r, r);
    double bb = rpcg_oracle_exdot(n, b, b);
    double thr = (tol * tol) * bb;
    if (hist) hist[0] = tau;
    if (trace_r) memcpy(trace_r, r, sizeof(double) * nn);
    if (trace_d) memcpy(trace_d, d, sizeof(double) * nn);
    if (trace_x) memcpy(trace_x, x, sizeof(double) * nn);
    if (!isfinite(tau) || !isfinite(bb) || !isfinite(beta)) { status = ORC_ERR_NONFINITE; goto out; }
    int32_t l = 0;
    while (tau > thr && l < maxit) {
        double beta_old = beta;
        rpcg_oracle_spmv(n, row_ptr, col, val, d, w);
        double delta = rpcg_oracle_exdot(n, d, w);
        if (!(delta > 0.0)) { status = isfinite(delta) ? ORC_ERR_BREAKDOWN : ORC_ERR_NONFINITE; break; }
        double rho = beta / delta;
        for (int32_t i = 0; i < n; ++i) x[i] = fma(rho, d[i], x[i]);
        for (int32_t i = 0; i < n; ++i) r[i] = fma(-rho, w[i], r[i]);
        factored_apply(n, g_rp, g_col, g_val, gt_rp, gt_col, gt_val, eps, r, t, z);
        beta = rpcg_oracle_exdot(n, z, r);
        tau = rpcg_oracle_exdot(n, r, r);
        double gamma = beta / beta_old;
        for (int32_t i = 0; i < n; ++i) d[i] = fma(gamma, d[i], z[i]);
        l += 1;
        if (hist) hist[l] = tau;
        if (trace_r) memcpy(trace_r + (size_t)l * n, r, sizeof(double) * (size_t)n);
        if (trace_d) memcpy(trace_d + (size_t)l * n, d, sizeof(double) * (size_t)n);
        if (trace_x) memcpy(trace_x + (size_t)l * n, x, sizeof(double) * (size_t)n);
        if (!isfinite(tau) || !isfinite(beta)) { status = ORC_ERR_NONFINITE; break; }
    }
    *iters = l;
    if (status == ORC_OK && tau > thr) status = ORC_WARN_MAXIT;
out:
    free(r); free(z); free(d); free(w); free(t);
    return status;
}

/* ---- threads ------------------------------------------------------------ */

/* Threads used by the parallel loops above (OpenMP); values < 1 select the
 * OpenMP default. Returns the number now in effect. */
int rpcg_oracle_set_threads(int32_t t)
{
    if (t >= 1) omp_set_num_threads(t);
    return omp_get_max_threads();
}

int rpcg_oracle_get_threads(void) { return omp_get_max_threads(); }

/* ---- host comparison loop (not a reference) -----------------------------
 * The iteration of rpcg_oracle_pcg with ordinary binary64 dot products: each
 * thread sums its range of products in order, and OpenMP adds the thread
 * sums in an unspecified order (the paper's Regular variant on a CPU). It
 * computes nothing the tests compare against; the benchmark times it beside
 * the exact loop to give the host's own cost of the exact dots. */
static double plain_dot(int32_t n, const double *x, const double *y)
{
    double s = 0.0;
    #pragma omp parallel for schedule(static) reduction(+:s)
    for (int32_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

int rpcg_cpu_plain_pcg(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *val,
                       const double *b, double *x, double tol, int32_t maxit, int32_t *iters)
{
    *iters = 0;
    if (n < 0 || maxit < 0) return ORC_ERR_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *dinv = malloc(sizeof(double) * nn), *r = malloc(sizeof(double) * nn);
    double *z = malloc(sizeof(double) * nn), *d = malloc(sizeof(double) * nn);
    double *w = malloc(sizeof(double) * nn);
    int status = ORC_OK;
    for (int32_t i = 0; i < n && status == ORC_OK; ++i) {
        double aii = 0.0; int found = 0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (col[k] == i) { aii = val[k]; found = 1; }
        if (!found || !(aii > 0.0)) status = ORC_ERR_NOT_SPD;
        else dinv[i] = 1.0 / aii;
    }
    if (status != ORC_OK) goto out;
    rpcg_oracle_spmv(n, row_ptr, col, val, x, w);
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) { r[i] = b[i] - w[i]; z[i] = dinv[i] * r[i]; d[i] = z[i]; }
    double beta = plain_dot(n, z, r), tau = plain_dot(n, r, r), bb = plain_dot(n, b, b);
    double thr = (tol * tol) * bb;
    int32_t l = 0;
    while (tau > thr && l < maxit) {
        double beta_old = beta;
        rpcg_oracle_spmv(n, row_ptr, col, val, d, w);
        double delta = plain_dot(n, d, w);
        if (!(delta > 0.0)) { status = ORC_ERR_BREAKDOWN; break; }
        double rho = beta / delta;
        #pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            x[i] = fma(rho, d[i], x[i]);
            r[i] = fma(-rho, w[i], r[i]);
            z[i] = dinv[i] * r[i];
        }
        beta = plain_dot(n, z, r);
        tau = plain_dot(n, r, r);
        double gamma = beta / beta_old;
        #pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) d[i] = fma(gamma, d[i], z[i]);
        l += 1;
    }
    *iters = l;
    if (status == ORC_OK && tau > thr) status = ORC_WARN_MAXIT;
out:
    free(dinv); free(r); free(z); free(d); free(w);
    return status;
}
