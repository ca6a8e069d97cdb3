// Launchers of the curved-element Nystrom correction kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hfmm {

// Constants of the discretisation, in device memory: the six interpolation
// points (u, v) of the reference triangle and their weights, the Lagrange
// coefficients L_i = sum_c mono_c C[c][i] (mono = 1, u, v, u^2, uv, v^2),
// and Gauss-Legendre nodes/weights on [0, 1] for the self rule.
constexpr int kNysMaxGauss = 32;
constexpr int kNysSelfOrder = 10;  // n of the self rule: 6 parts x n^2 points
struct NysConst {
  double uv[12];
  double w[6];
  double lagr[36];
  double gx[kNysMaxGauss], gw[kNysMaxGauss];
  int rule_off[6], rule_cnt[6];  // near rule with 4^L sub-triangles: points [off, off + cnt) of the table
  int max_level;                 // deepest near rule (near_levels)
};

// items: (target point, element, position of its six values in val, -);
// rule: the near rules of 4^0 .. 4^max_level sub-triangles, concatenated;
// k + i ki: the wavenumber (ki >= 0 damps)
void launch_nys_near(int64_t nitems, const int4* items, const double* pts, const double* elem, const NysConst* K,
                     const double* rule, double k, double ki, float2* val, hipStream_t s);
// self6[6 j + i] for every point j (n x n points per Duffy part, n <= kNysMaxGauss)
void launch_nys_self(int64_t npts, const double* pts, const double* elem, const NysConst* K, int n, double k,
                     double ki, double2* self6, hipStream_t s);
void launch_self6_apply_c64(int64_t n, const double2* S, const float2* x, float2* y, hipStream_t s);
// out = (y [+ z in FP32]) + (6 x 6 self blocks) v in FP64
void launch_from_c64_self6(int64_t n, const float2* y, const double2* S, const double2* v, double2* out,
                           hipStream_t s, const float2* z = nullptr);
void launch_plane_wave_pts(int64_t n, const double* pts, double k, double ki, const double* d, double2* b,
                           hipStream_t s);

}  // namespace hfmm
