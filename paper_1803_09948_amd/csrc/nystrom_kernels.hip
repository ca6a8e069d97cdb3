// Locally corrected Nystrom discretisation on curved six-node triangles:
// FP64 correction kernels and their application.
//
// Sec. 2.2, eqs. (8)-(10): the unknown at an element's interpolation point
// is the density times the surface Jacobian, interpolated over the element
// by Lagrange polynomials L_i in the element's parameters (u, v); point
// matching at every interpolation point gives entries
//   Z_(j)(i,e) = integral over the reference triangle of G(r_j, x_e(u,v)) L_i(u,v) du dv,
// the Jacobian cancelling against the surface measure.  The interpolation
// points are the six points of the symmetric degree-4 rule (weights w_i), so
// far entries are w_i G(r_j, r_ie): the FMM over all points with strengths
// w_i I_i.  Two corrections replace that rule where it fails:
//   self element (e = element of j): the weakly singular integral by the
//     Duffy collapse at j's parameter point (Sec. 2.2) over three
//     sub-triangles, with a sinh substitution in the angular variable
//     split at the point of the far edge closest to j;
//   near elements (|r_j - c_e| < eta h_e): 4^L uniform sub-triangles with an
//     n x n collapsed Gauss rule each;
// each minus the rule terms w_i G(r_j, r_ie) the FMM already holds (R > 0).
// The near corrections are stored in complex64, the self blocks in
// complex128 and applied in FP64 inside GMRES.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "nystrom_kernels.h"

namespace hfmm {

namespace {

struct v3 {
  double x, y, z;
};
__device__ inline v3 vsub(v3 a, v3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// Quadratic map of element X (6 nodes v0 v1 v2 m01 m12 m20) at (u, v), and
// its two tangents.
__device__ inline v3 qmap(const double* X, double u, double v) {
  const double l1 = 1.0 - u - v, l2 = u, l3 = v;
  const double N[6] = {l1 * (2 * l1 - 1), l2 * (2 * l2 - 1), l3 * (2 * l3 - 1), 4 * l1 * l2, 4 * l2 * l3,
                       4 * l3 * l1};
  v3 r = {0, 0, 0};
  for (int a = 0; a < 6; ++a) {
    r.x += N[a] * X[3 * a];
    r.y += N[a] * X[3 * a + 1];
    r.z += N[a] * X[3 * a + 2];
  }
  return r;
}
__device__ inline void qtangents(const double* X, double u, double v, v3* xu, v3* xv) {
  const double l1 = 1.0 - u - v, l2 = u, l3 = v;
  const double Nu[6] = {-(4 * l1 - 1), 4 * l2 - 1, 0.0, 4 * (l1 - l2), 4 * l3, -4 * l3};
  const double Nv[6] = {-(4 * l1 - 1), 0.0, 4 * l3 - 1, -4 * l2, 4 * l2, 4 * (l1 - l3)};
  *xu = {0, 0, 0};
  *xv = {0, 0, 0};
  for (int a = 0; a < 6; ++a) {
    xu->x += Nu[a] * X[3 * a];
    xu->y += Nu[a] * X[3 * a + 1];
    xu->z += Nu[a] * X[3 * a + 2];
    xv->x += Nv[a] * X[3 * a];
    xv->y += Nv[a] * X[3 * a + 1];
    xv->z += Nv[a] * X[3 * a + 2];
  }
}

// L_i(u, v) = sum_c mono_c(u, v) C[c][i], mono = (1, u, v, u^2, uv, v^2)
__device__ inline void lagr(const double* C, double u, double v, double* L) {
  const double m[6] = {1.0, u, v, u * u, u * v, v * v};
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
    for (int c = 0; c < 6; ++c) s += m[c] * C[6 * c + i];
    L[i] = s;
  }
}

// G for the wavenumber k + i ki
__device__ inline double2 green(double k, double ki, v3 x, v3 y) {
  const double R = sqrt(vdot(vsub(x, y), vsub(x, y)));
  double s, c;
  sincos(k * R, &s, &c);
  const double f = exp(-ki * R) / (4.0 * M_PI * R);
  return make_double2(c * f, s * f);
}

// Fixed-order sum of 12 doubles over the wave; lane 0 receives the sums.
__device__ inline void wave_sum12(double* acc, double (*red)[64], int lane) {
  for (int c = 0; c < 12; ++c) red[c][lane] = acc[c];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane == 0)
    for (int c = 0; c < 12; ++c) {
      double t = 0.0;
      for (int l = 0; l < 64; ++l) t += red[c][l];
      acc[c] = t;
    }
}

// rule terms w_i G(r_j, r_ie) the FMM holds for element e (R > 0 only)
__device__ inline void subtract_rule(const NysConst* K, const double* X, double k, double ki, v3 x, int skip,
                                     double* acc) {
  for (int i = 0; i < 6; ++i) {
    if (i == skip) continue;
    const v3 y = qmap(X, K->uv[2 * i], K->uv[2 * i + 1]);
    const double2 g = green(k, ki, x, y);
    acc[2 * i] -= K->w[i] * g.x;
    acc[2 * i + 1] -= K->w[i] * g.y;
  }
}

}  // namespace

// Subdivision depth of the near rule for a target at distance >= t h from
// the element (t: centroid distance minus the largest centroid-corner
// distance, over the longest corner-corner distance h): 4^L sub-triangles of
// n x n points keep the relative error of the 1/R integral below about 1e-8
// (measured against the closed form on flat triangles: L = 0 from t = 1,
// L = 1 from t = 0.5, L = 2 from t = 0.25, the deepest rule below).
__device__ inline int near_level(double t, int max_level) {
  const int L = t >= 1.0 ? 0 : t >= 0.5 ? 1 : t >= 0.25 ? 2 : max_level;
  return L < max_level ? L : max_level;
}

// One wave per near pair (target point j, element e); the pair's six values
// go to val[pos .. pos + 5].  Rule: rule[3 q + (0, 1, 2)] = (u, v, weight).
__global__ void __launch_bounds__(256) k_nys_near(int64_t nitems, const int4* __restrict__ items,
                                                  const double* __restrict__ pts, const double* __restrict__ elem,
                                                  const NysConst* __restrict__ K, const double* __restrict__ rule,
                                                  double k, double ki, float2* __restrict__ val) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ double red[4][12][64];
  const int64_t it = (int64_t)blockIdx.x * 4 + wave;
  if (it >= nitems) return;
  const int4 w = items[it];  // (target, element, position, -)
  const v3 x = {pts[3 * (int64_t)w.x], pts[3 * (int64_t)w.x + 1], pts[3 * (int64_t)w.x + 2]};
  const double* X = elem + 18 * (int64_t)w.y;
  int L;
  {
    const v3 c = qmap(X, 1.0 / 3.0, 1.0 / 3.0);
    double re = 0.0, h = 0.0;
    for (int a = 0; a < 3; ++a) {
      const v3 p = {X[3 * a], X[3 * a + 1], X[3 * a + 2]};
      const v3 q = {X[3 * ((a + 1) % 3)], X[3 * ((a + 1) % 3) + 1], X[3 * ((a + 1) % 3) + 2]};
      re = fmax(re, sqrt(vdot(vsub(p, c), vsub(p, c))));
      h = fmax(h, sqrt(vdot(vsub(p, q), vsub(p, q))));
    }
    L = near_level((sqrt(vdot(vsub(x, c), vsub(x, c))) - re) / h, K->max_level);
  }
  const double* R = rule + 3 * (int64_t)K->rule_off[L];
  const int nrule = K->rule_cnt[L];
  double acc[12];
  for (int c = 0; c < 12; ++c) acc[c] = 0.0;
  for (int q = lane; q < nrule; q += 64) {
    const double u = R[3 * q], v = R[3 * q + 1], wq = R[3 * q + 2];
    const double2 g = green(k, ki, x, qmap(X, u, v));
    double L[6];
    lagr(K->lagr, u, v, L);
    for (int i = 0; i < 6; ++i) {
      acc[2 * i] += wq * L[i] * g.x;
      acc[2 * i + 1] += wq * L[i] * g.y;
    }
  }
  wave_sum12(acc, red[wave], lane);
  if (lane == 0) {
    subtract_rule(K, X, k, ki, x, -1, acc);
    for (int i = 0; i < 6; ++i) val[w.z + i] = make_float2((float)acc[2 * i], (float)acc[2 * i + 1]);
  }
}

// One wave per point j: the six self integrals of j's own element (Duffy
// collapse at j's parameter point with the angular sinh map, n x n points per
// part), minus the rule terms of the element's other points.
__global__ void __launch_bounds__(256) k_nys_self(int64_t npts, const double* __restrict__ pts,
                                                  const double* __restrict__ elem, const NysConst* __restrict__ K,
                                                  int n, double k, double ki, double2* __restrict__ self6) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ double red[4][12][64];
  const int64_t j = (int64_t)blockIdx.x * 4 + wave;
  if (j >= npts) return;
  const int jl = (int)(j % 6);
  const double* X = elem + 18 * (j / 6);
  const v3 x = {pts[3 * j], pts[3 * j + 1], pts[3 * j + 2]};
  const double pu = K->uv[2 * jl], pv = K->uv[2 * jl + 1];
  v3 xu, xv;
  qtangents(X, pu, pv, &xu, &xv);
  const double g11 = vdot(xu, xu), g12 = vdot(xu, xv), g22 = vdot(xv, xv);
  auto gnorm2 = [&](double a, double b) { return a * a * g11 + 2.0 * a * b * g12 + b * b * g22; };
  const double cu[3] = {0.0, 1.0, 0.0}, cv[3] = {0.0, 0.0, 1.0};
  double acc[12];
  for (int c = 0; c < 12; ++c) acc[c] = 0.0;
  const int per_part = n * n;
  for (int q = lane; q < 6 * per_part; q += 64) {
    const int part = q / per_part, rem = q % per_part;
    const int sub = part >> 1, side = part & 1;
    const int ia = rem / n, ib = rem % n;
    // sub-triangle (p, corner sub, corner sub + 1): y = p + s (e0 + t e)
    const double e0u = cu[sub] - pu, e0v = cv[sub] - pv;
    const double eu = cu[(sub + 1) % 3] - cu[sub], ev = cv[(sub + 1) % 3] - cv[sub];
    const double det = fabs(e0u * ev - e0v * eu);
    // closest point of the far edge to p in the tangent metric, distance H,
    // edge length B
    const double B2 = gnorm2(eu, ev);
    const double cross_term = e0u * eu * g11 + (e0u * ev + e0v * eu) * g12 + e0v * ev * g22;
    double t0 = -cross_term / B2;
    t0 = fmin(fmax(t0, 0.0), 1.0);
    const double H = sqrt(fmax(gnorm2(e0u + t0 * eu, e0v + t0 * ev), 1e-300));
    const double B = sqrt(B2);
    const double len = side ? 1.0 - t0 : t0;
    if (len <= 1e-15) continue;
    const double mu = asinh(len * B / H);
    const double tau = K->gx[ib], s = K->gx[ia];
    const double sh = sinh(mu * tau), ch = cosh(mu * tau);
    const double t = side ? t0 + (H / B) * sh : t0 - (H / B) * sh;
    const double wt = (H / B) * mu * ch * K->gw[ib];
    const double wq = K->gw[ia] * wt * s * det;
    const double u = pu + s * (e0u + t * eu), v = pv + s * (e0v + t * ev);
    const double2 g = green(k, ki, x, qmap(X, u, v));
    double L[6];
    lagr(K->lagr, u, v, L);
    for (int i = 0; i < 6; ++i) {
      acc[2 * i] += wq * L[i] * g.x;
      acc[2 * i + 1] += wq * L[i] * g.y;
    }
  }
  wave_sum12(acc, red[wave], lane);
  if (lane == 0) {
    subtract_rule(K, X, k, ki, x, jl, acc);
    for (int i = 0; i < 6; ++i) self6[6 * j + i] = make_double2(acc[2 * i], acc[2 * i + 1]);
  }
}

// y_j += sum_i S[j][i] x[6 (j / 6) + i]  (complex64 in/out, FP64 products)
__global__ void k_self6_apply_c64(int64_t n, const double2* __restrict__ S, const float2* __restrict__ x,
                                  float2* __restrict__ y) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t b = 6 * (j / 6);
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < 6; ++i) {
    const double2 a = S[6 * j + i];
    const float2 v = x[b + i];
    sr += a.x * v.x - a.y * v.y;
    si += a.x * v.y + a.y * v.x;
  }
  const float2 o = y[j];
  y[j] = make_float2((float)(o.x + sr), (float)(o.y + si));
}

// out_j = (c128) y_j + sum_i S[j][i] v[6 (j / 6) + i]  (FP64)
__global__ void k_from_c64_self6(int64_t n, const float2* __restrict__ y, const float2* __restrict__ z,
                                 const double2* __restrict__ S, const double2* __restrict__ v,
                                 double2* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t b = 6 * (j / 6);
  float2 yj = y[j];
  if (z) yj = make_float2(yj.x + z[j].x, yj.y + z[j].y);  // the FP32 sum the near apply would form
  double sr = yj.x, si = yj.y;
  for (int i = 0; i < 6; ++i) {
    const double2 a = S[6 * j + i], w = v[b + i];
    sr += a.x * w.x - a.y * w.y;
    si += a.x * w.y + a.y * w.x;
  }
  out[j] = make_double2(sr, si);
}

// b_j = exp(i k d . r_j)
__global__ void k_plane_wave_pts(int64_t n, const double* __restrict__ pts, double k, double ki, double dx,
                                 double dy, double dz, double2* __restrict__ b) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double ph = dx * pts[3 * j] + dy * pts[3 * j + 1] + dz * pts[3 * j + 2];
  double s, c;
  sincos(k * ph, &s, &c);
  const double a = exp(-ki * ph);
  b[j] = make_double2(a * c, a * s);
}

void launch_nys_near(int64_t nitems, const int4* items, const double* pts, const double* elem, const NysConst* K,
                     const double* rule, double k, double ki, float2* val, hipStream_t s) {
  if (nitems > 0) k_nys_near<<<(nitems + 3) / 4, 256, 0, s>>>(nitems, items, pts, elem, K, rule, k, ki, val);
}
void launch_nys_self(int64_t npts, const double* pts, const double* elem, const NysConst* K, int n, double k,
                     double ki, double2* self6, hipStream_t s) {
  if (npts > 0) k_nys_self<<<(npts + 3) / 4, 256, 0, s>>>(npts, pts, elem, K, n, k, ki, self6);
}
void launch_self6_apply_c64(int64_t n, const double2* S, const float2* x, float2* y, hipStream_t s) {
  if (n > 0) k_self6_apply_c64<<<(n + 255) / 256, 256, 0, s>>>(n, S, x, y);
}
void launch_from_c64_self6(int64_t n, const float2* y, const double2* S, const double2* v, double2* out,
                           hipStream_t s, const float2* z) {
  if (n > 0) k_from_c64_self6<<<(n + 255) / 256, 256, 0, s>>>(n, y, z, S, v, out);
}
void launch_plane_wave_pts(int64_t n, const double* pts, double k, double ki, const double* d, double2* b,
                           hipStream_t s) {
  if (n > 0) k_plane_wave_pts<<<(n + 255) / 256, 256, 0, s>>>(n, pts, k, ki, d[0], d[1], d[2], b);
}

}  // namespace hfmm
