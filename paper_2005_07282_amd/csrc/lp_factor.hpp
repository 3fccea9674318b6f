// Learned preconditioner: launchers of the feature, factor and loss kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lp_common.hpp"

namespace rpcg {

constexpr float LP_ABSENT = -4.0f; // feature of an absent neighbour
constexpr float LP_OCLAMP = 4.0f;  // clamp of the diagonal output

hipError_t launch_lp_features(int N, const int *rp, const int *col, const double *val, bf16_t *feat, float *s, int *bad,
                              hipStream_t st);
hipError_t launch_lp_factor(int N, const float *o, const float *s, const int *g_rp, const int *gt_rp, double *g_val,
                            double *gt_val, hipStream_t st);
hipError_t launch_lp_resid(long long n, double eps, const double *w, const double *v, const double *u, double *r,
                           hipStream_t st);
hipError_t launch_lp_dodg(int N, double scale, const double *uu, const double *rr, const float *o, const float *s,
                          const int *g_rp, const double *g_val, const double *r, const double *y, const double *v,
                          const double *q, double *do64, double *loss, hipStream_t st);
hipError_t launch_lp_to_bf16(long long n, const double *a, bf16_t *b, hipStream_t st);

} // namespace rpcg
