// Learned preconditioner: launchers of the feature, factor and loss kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "lp_common.hpp"

namespace rpcg {

constexpr float LP_ABSENT = -4.0f; // feature of an absent neighbour
constexpr float LP_OCLAMP = 4.0f;  // clamp of the diagonal output

// A CSR matrix in device memory (32-bit row pointers and column indices).
struct LpMat {
    const int *rp;
    const int *col;
    const double *val;
};
// Up to LP_MAT_ARGS matrices passed by value to one launch.
constexpr int LP_MAT_ARGS = 16;
struct LpMatSet {
    LpMat m[LP_MAT_ARGS];
};

// Features and s of nb <= LP_MAT_ARGS systems (grid.y = system; feat and s of
// system k at k n 4 and k n). A missing or non-positive diagonal stores gen
// into *bad (host-visible memory; plain stores of one value).
hipError_t launch_lp_features(int N, int nb, const LpMatSet &set, bf16_t *feat, float *s, int *bad, int gen,
                              hipStream_t st);
// G, G^T values of nb instances (grid.y = instance): o, s, g_val, gt_val of
// instance k at k times the given strides (in elements).
hipError_t launch_lp_factor(int N, int nb, const float *o, const float *s, const int *g_rp, const int *gt_rp,
                            double *g_val, double *gt_val, long long val_stride, hipStream_t st);
hipError_t launch_lp_to_bf16(long long n, const double *a, bf16_t *b, hipStream_t st);

// ---- loss over a batch of (instance, probe) pairs (lp_loss.hip) ----
constexpr int LP_DOT_P = 3;         // lane expansion length of the exact dots
constexpr int LP_DOT_CHUNKS = 64;   // workgroups (slots) per pair and dot
// The loss's vectors v, y, r, q are interleaved per instance: entry i of the
// vector of pair p = k nu + m at base + (k n + i) nu + m; the probes u_p are
// read through the pointer table utab.
// Y_k = M_k X_k (mats[k], k < nb) for the nu vectors of each instance: X from
// xtab (one pointer per pair) if given, else interleaved at xbase.
hipError_t launch_lp_mv(long long n, int nb, int nu, const LpMat *mats, const double *const *xtab, const double *xbase,
                        double *ybase, hipStream_t st);
// R = (G_k Y + eps V) - U (interleaved; U through utab) and the slot partials
// of <u_p, u_p>, <r_p, r_p> (slots p * LP_DOT_CHUNKS + c of wu, wr; capacity
// stride >= nb nu LP_DOT_CHUNKS).
hipError_t launch_lp_resid_dots(long long n, int nb, int nu, double eps, const LpMat *gm, const double *const *utab,
                                const double *y, const double *v, double *r, const DotWs &wu, const DotWs &wr,
                                int stride, int *flags, hipStream_t st);
// dots[2p] = <u_p, u_p>, dots[2p + 1] = <r_p, r_p>, each correctly rounded.
hipError_t launch_lp_dots_merge(int npairs, const DotWs &wu, const DotWs &wr, int stride, double *dots, int *flags,
                                hipStream_t st);
// dL/do of every instance (bfloat16 into dob; binary64 into do64 unless null)
// and the loss, from the interleaved R, Y, V, Q.
hipError_t launch_lp_dodg_all(int N, int nb, int nu, double scale, const double *dots, const float *o, const float *s,
                              const LpMat *gm, const double *r, const double *y, const double *v, const double *q,
                              double *do64, bf16_t *dob, double *loss, hipStream_t st);

} // namespace rpcg
