// HIP kernels of the boundary-integral layer and of the FP64 GMRES solver.
//
// Discretisation of eq. (7) (Sec. 2.1-2.2) with flat triangles, one unknown
// per triangle, collocation at centroids.  The FMM sums the 3-point interior
// Gauss rule (weights A/3) over ALL panels, the own panel included; two
// corrections make the product equal the collocation matrix:
//   near pairs (j != i, |c_i - c_j| < eta h_j):  Delta_ij = I_ij - 3pt_ij,
//   diagonal:                                    D_i = S_ii - 3pt_ii,
// where I_ij is the panel integral of G(c_i, .) over T_j by a refined rule
// (near-singularity treatment, the near branch of the P2P listing) and S_ii
// the weakly singular self integral (Duffy treatment, Sec. 2.2): the 1/R part
// in closed form, the bounded remainder (e^{ikR}-1)/R by a Duffy-collapsed
// Gauss rule.  All corrections are computed in FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "bie_kernels.h"

namespace hfmm {

struct d3 {
  double x, y, z;
};
__device__ inline d3 mk(double x, double y, double z) { return {x, y, z}; }
__device__ inline d3 sub(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline d3 add(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline d3 scl(d3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline d3 cross(d3 a, d3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline double nrm(d3 a) { return sqrt(dot(a, a)); }

__device__ inline d3 vtx(const double* pan, int i, int v) {
  const double* p = pan + 9 * (size_t)i + 3 * v;
  return {p[0], p[1], p[2]};
}

// G(x, y) = e^{ikR} / (4 pi R) for the wavenumber k + i ki
__device__ inline double2 green64(double k, double ki, d3 x, d3 y) {
  double R = nrm(sub(x, y));
  double s, c;
  sincos(k * R, &s, &c);
  double f = exp(-ki * R) / (4.0 * M_PI * R);
  return make_double2(c * f, s * f);
}

// 3-point interior rule on panel j seen from x: (A/3) sum_g G(x, y_g)
__device__ inline double2 three_point(double k, double ki, d3 x, d3 a, d3 b, d3 c) {
  double area = 0.5 * nrm(cross(sub(b, a), sub(c, a)));
  double2 s = make_double2(0.0, 0.0);
  const double w1 = 2.0 / 3.0, w2 = 1.0 / 6.0;
  d3 g[3] = {add(add(scl(a, w1), scl(b, w2)), scl(c, w2)), add(add(scl(a, w2), scl(b, w1)), scl(c, w2)),
             add(add(scl(a, w2), scl(b, w2)), scl(c, w1))};
  for (int q = 0; q < 3; ++q) {
    double2 v = green64(k, ki, x, g[q]);
    s.x += v.x;
    s.y += v.y;
  }
  return make_double2(s.x * area / 3.0, s.y * area / 3.0);
}

// Closed form of the integral of 1/|x - y| over a flat triangle for x in its
// plane (sum over edges of the perpendicular distance times a log ratio).
__device__ double laplace_inplane(d3 x, d3 a, d3 b, d3 c) {
  d3 n = cross(sub(b, a), sub(c, a));
  n = scl(n, 1.0 / nrm(n));
  d3 P[3] = {a, b, c};
  double tot = 0.0;
  for (int e = 0; e < 3; ++e) {
    d3 p = P[e], q = P[(e + 1) % 3];
    d3 t = sub(q, p);
    t = scl(t, 1.0 / nrm(t));
    d3 u = cross(t, n);
    double P0 = dot(sub(p, x), u);
    double lm = dot(sub(p, x), t), lp = dot(sub(q, x), t);
    double Rm = nrm(sub(p, x)), Rp = nrm(sub(q, x));
    if (fabs(P0) > 0.0) tot += P0 * log((Rp + lp) / (Rm + lm));
  }
  return tot;
}

// Self term D_i = S_ii - 3pt_ii, one thread per panel.
__global__ void k_self(int64_t npan, const double* __restrict__ pan, double k, double ki,
                       const double* __restrict__ gx, const double* __restrict__ gw, int ng,
                       double2* __restrict__ diag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npan) return;
  d3 a = vtx(pan, i, 0), b = vtx(pan, i, 1), c = vtx(pan, i, 2);
  d3 x = scl(add(add(a, b), c), 1.0 / 3.0);
  double lap = laplace_inplane(x, a, b, c) / (4.0 * M_PI);
  // remainder (e^{ikR} - 1) / (4 pi R), Duffy-collapsed at x over the six
  // pieces of (x,a,b), (x,b,c), (x,c,a) cut at the foot of the perpendicular
  // from x onto each edge: along an edge the distance from x is smallest at
  // that foot, sharply so on an elongated panel, and each piece then sees a
  // monotone distance (the rule keeps its accuracy on such panels)
  double sr = 0.0, si = 0.0;
  d3 V[3] = {a, b, c};
  for (int e = 0; e < 6; ++e) {
    const d3 q0 = V[e >> 1], r0 = V[((e >> 1) + 1) % 3];
    const d3 ed = sub(r0, q0);
    const double tf = fmin(fmax(dot(sub(x, q0), ed) / dot(ed, ed), 0.0), 1.0);
    const d3 F = add(q0, scl(ed, tf));
    const d3 q = (e & 1) ? F : q0, r = (e & 1) ? r0 : F;
    double a2 = nrm(cross(sub(q, x), sub(r, x)));  // twice the piece's area
    if (a2 == 0.0) continue;
    for (int iu = 0; iu < ng; ++iu)
      for (int iv = 0; iv < ng; ++iv) {
        double u = gx[iu], v = gx[iv];
        d3 y = add(add(x, scl(sub(q, x), u)), scl(sub(r, q), u * v));
        double R = nrm(sub(y, x));
        double w = gw[iu] * gw[iv] * u * a2 / (4.0 * M_PI * R);
        double s, cc;
        sincos(k * R, &s, &cc);
        // e^{i(k + i ki)R} - 1 = (e^{-ki R} - 1) cos kR + (cos kR - 1) + i e^{-ki R} sin kR,
        // with cos kR - 1 = -2 sin^2(kR/2): no cancellation at small R
        double h = sin(0.5 * k * R);
        sr += w * (expm1(-ki * R) * cc - 2.0 * h * h);
        si += w * exp(-ki * R) * s;
      }
  }
  double2 t3 = three_point(k, ki, x, a, b, c);
  diag[i] = make_double2(lap + sr - t3.x, si - t3.y);
}

// Near corrections: one wave per stored nonzero (i, j): refined integral of
// G(c_i, .) over T_j (4^L uniform sub-triangles, n x n collapsed Gauss rule
// each) minus the 3-point sum.  Values stored as complex64.  L is the
// deepest subdivision; a target at distance >= t h from the panel (t: centroid
// distance minus the largest centroid-corner distance, over the longest
// edge h) takes L = 0 from t = 1, L = 1 from t = 0.5 and L = 2 from t = 0.25,
// which keeps the relative error of the 1/R integral below about 1e-8
// (measured against the closed form).
__global__ void __launch_bounds__(256) k_near(int64_t nnz, const int32_t* __restrict__ rows,
                                              const int32_t* __restrict__ cols,
                                              const double* __restrict__ pan, double k, double ki, int Lmax,
                                              const double* __restrict__ gx,
                                              const double* __restrict__ gw, int ng,
                                              float2* __restrict__ val) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + wave;
  __shared__ double red[4][2][64];
  if (e >= nnz) return;
  const int i = rows[e], j = cols[e];
  d3 x = scl(add(add(vtx(pan, i, 0), vtx(pan, i, 1)), vtx(pan, i, 2)), 1.0 / 3.0);
  d3 a = vtx(pan, j, 0), b = vtx(pan, j, 1), c = vtx(pan, j, 2);
  const double area = 0.5 * nrm(cross(sub(b, a), sub(c, a)));
  int L;
  {
    const d3 cen = scl(add(add(a, b), c), 1.0 / 3.0);
    const double re = fmax(nrm(sub(a, cen)), fmax(nrm(sub(b, cen)), nrm(sub(c, cen))));
    const double h = fmax(nrm(sub(b, a)), fmax(nrm(sub(c, b)), nrm(sub(a, c))));
    const double t = (nrm(sub(x, cen)) - re) / h;
    L = t >= 1.0 ? 0 : t >= 0.5 ? 1 : t >= 0.25 ? 2 : Lmax;
    L = L < Lmax ? L : Lmax;
  }
  const int nsub = 1 << (2 * L);
  const int npt = nsub * ng * ng;
  double sr = 0.0, si = 0.0;
  for (int q = lane; q < npt; q += 64) {
    int s = q / (ng * ng), rem = q % (ng * ng);
    int iu = rem / ng, iv = rem % ng;
    // barycentric vertices of sub-triangle s: descend L levels
    double P0[3] = {1, 0, 0}, P1[3] = {0, 1, 0}, P2[3] = {0, 0, 1};
    for (int lev = 0; lev < L; ++lev) {
      int d = (s >> (2 * lev)) & 3;
      double A0[3], A1[3], A2[3];
      for (int t = 0; t < 3; ++t) {
        double m01 = 0.5 * (P0[t] + P1[t]), m12 = 0.5 * (P1[t] + P2[t]), m20 = 0.5 * (P2[t] + P0[t]);
        if (d == 0) { A0[t] = P0[t]; A1[t] = m01; A2[t] = m20; }
        else if (d == 1) { A0[t] = P1[t]; A1[t] = m12; A2[t] = m01; }
        else if (d == 2) { A0[t] = P2[t]; A1[t] = m20; A2[t] = m12; }
        else { A0[t] = m01; A1[t] = m12; A2[t] = m20; }
      }
      for (int t = 0; t < 3; ++t) {
        P0[t] = A0[t];
        P1[t] = A1[t];
        P2[t] = A2[t];
      }
    }
    double u = gx[iu], v = gx[iv];
    double lam[3];
    for (int t = 0; t < 3; ++t) lam[t] = P0[t] + u * (P1[t] - P0[t]) + u * v * (P2[t] - P1[t]);
    d3 y = add(add(scl(a, lam[0]), scl(b, lam[1])), scl(c, lam[2]));
    double w = gw[iu] * gw[iv] * u * 2.0 * (area / nsub);
    double2 g = green64(k, ki, x, y);
    sr += w * g.x;
    si += w * g.y;
  }
  red[wave][0][lane] = sr;
  red[wave][1][lane] = si;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane == 0) {
    double tr = 0.0, ti = 0.0;
    for (int l = 0; l < 64; ++l) {
      tr += red[wave][0][l];
      ti += red[wave][1][l];
    }
    double2 t3 = three_point(k, ki, x, a, b, c);
    val[e] = make_float2((float)(tr - t3.x), (float)(ti - t3.y));
  }
}

// y_i += sum_j Delta_ij x_j (+ D_i x_i when diag != NULL), FP32, caller order.
// 16 lanes per row: lane g of a row takes nonzeros g, g + 16, ... (adjacent
// lanes read adjacent values), then the 16 partial sums are added by a fixed
// butterfly, so every row sums in the same order on every call.
__global__ void __launch_bounds__(256) k_near_apply(int64_t n, const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ col,
                                                    const float2* __restrict__ val,
                                                    const double2* __restrict__ diag,
                                                    const float2* __restrict__ x, float2* __restrict__ y,
                                                    int overwrite) {
  const int64_t i = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int g = threadIdx.x & 15;
  float sr = 0.f, si = 0.f;
  if (i < n) {
    const int q1 = off[i + 1];
    for (int q = off[i] + g; q < q1; q += 16) {
      const float2 a = val[q], b = x[col[q]];
      sr = fmaf(a.x, b.x, fmaf(-a.y, b.y, sr));
      si = fmaf(a.x, b.y, fmaf(a.y, b.x, si));
    }
  }
  for (int o = 8; o > 0; o >>= 1) {  // within the 16-lane group
    sr += __shfl_xor(sr, o);
    si += __shfl_xor(si, o);
  }
  if (i < n && g == 0) {
    if (diag) {
      const float2 a = make_float2((float)diag[i].x, (float)diag[i].y), b = x[i];
      sr = fmaf(a.x, b.x, fmaf(-a.y, b.y, sr));
      si = fmaf(a.x, b.y, fmaf(a.y, b.x, si));
    }
    if (overwrite) {
      y[i] = make_float2(sr, si);
    } else {
      const float2 o = y[i];
      y[i] = make_float2(o.x + sr, o.y + si);
    }
  }
}

// b_i = exp(i k d . c_i)
__global__ void k_plane_wave(int64_t n, const double* __restrict__ pan, double k, double ki, double dx, double dy,
                             double dz, double2* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  d3 x = scl(add(add(vtx(pan, i, 0), vtx(pan, i, 1)), vtx(pan, i, 2)), 1.0 / 3.0);
  const double ph = dx * x.x + dy * x.y + dz * x.z;
  double s, c;
  sincos(k * ph, &s, &c);
  const double a = exp(-ki * ph);  // e^{i (k + i ki) d.x}
  b[i] = make_double2(a * c, a * s);
}

// ---------------------------------------------------------------------------
// FP64 vector kernels for GMRES
// ---------------------------------------------------------------------------
__global__ void k_to_c64(int64_t n, const double2* __restrict__ a, float2* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// out = (c128) y64 + D .* v  (the self term in FP64)
__global__ void k_from_c64_diag(int64_t n, const float2* __restrict__ y, const float2* __restrict__ z,
                                const double2* __restrict__ diag, const double2* __restrict__ v,
                                double2* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 yi = y[i];
  if (z) yi = make_float2(yi.x + z[i].x, yi.y + z[i].y);  // the FP32 sum the near apply would form
  double2 d = diag[i], x = v[i];
  out[i] = make_double2((double)yi.x + d.x * x.x - d.y * x.y, (double)yi.y + d.x * x.y + d.y * x.x);
}

// partial[b][i] = sum over this block's range of conj(V_i) w, i < nv (nv <= 32)
// V rows have stride ld.  Fixed grid and fixed reduction order: deterministic.
constexpr int kDotBlocks = 240;
__global__ void __launch_bounds__(256) k_mdot(int64_t n, int nv, const double2* __restrict__ V, int64_t ld,
                                              const double2* __restrict__ w, double2* __restrict__ partial) {
  __shared__ double2 sh[8][32];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double2 acc[32];
  for (int v = 0; v < 32; ++v) acc[v] = make_double2(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double2 x = w[e];
    for (int v = 0; v < nv; ++v) {
      double2 a = V[v * ld + e];
      acc[v].x += a.x * x.x + a.y * x.y;
      acc[v].y += a.x * x.y - a.y * x.x;
    }
  }
  for (int v = 0; v < nv; ++v) {
    double2 s = acc[v];
    for (int o = 32; o > 0; o >>= 1) {
      s.x += __shfl_xor(s.x, o);
      s.y += __shfl_xor(s.y, o);
    }
    if (lane == 0) sh[wave][v] = s;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double2 s = make_double2(0.0, 0.0);
    for (int q = 0; q < 4; ++q) {
      s.x += sh[q][threadIdx.x].x;
      s.y += sh[q][threadIdx.x].y;
    }
    partial[(size_t)blockIdx.x * 32 + threadIdx.x] = s;
  }
}

// h[i] (+)= sum_b partial[b][i]; one block of 8 waves, wave w takes
// i = w, w + 8, ...; lane l adds partials l, l + 64, ... in order, then the
// wave adds its lanes by a fixed butterfly (deterministic, all loads of a
// lane in flight together).
__global__ void __launch_bounds__(512) k_mdot_final(int nblk, int nv, const double2* __restrict__ partial,
                                                    double2* __restrict__ h, int accumulate) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = wave; i < nv; i += 8) {
    double sx = 0.0, sy = 0.0;
    for (int b = lane; b < nblk; b += 64) {
      const double2 v = partial[(size_t)b * 32 + i];
      sx += v.x;
      sy += v.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
      sx += __shfl_xor(sx, o);
      sy += __shfl_xor(sy, o);
    }
    if (lane == 0) {
      if (accumulate) {
        h[i].x += sx;
        h[i].y += sy;
      } else {
        h[i] = make_double2(sx, sy);
      }
    }
  }
}

// w -= sum_i V_i h_i   (h from coef, nv entries)
__global__ void k_mupdate(int64_t n, int nv, const double2* __restrict__ V, int64_t ld,
                          const double2* __restrict__ coef, double2* __restrict__ w, double sign) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double2 s = w[e];
  for (int v = 0; v < nv; ++v) {
    double2 a = V[v * ld + e], c = coef[v];
    s.x += sign * (a.x * c.x - a.y * c.y);
    s.y += sign * (a.x * c.y + a.y * c.x);
  }
  w[e] = s;
}

// dst = src * (1 / nrm), nrm = sqrt(re(dotval))
__global__ void k_scale_by_norm(int64_t n, const double2* __restrict__ src, const double2* __restrict__ dotval,
                                double2* __restrict__ dst) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double nr = sqrt(dotval->x);
  double s = nr > 0.0 ? 1.0 / nr : 0.0;
  dst[e] = make_double2(src[e].x * s, src[e].y * s);
}

// r = b - r
__global__ void k_residual(int64_t n, const double2* __restrict__ b, double2* __restrict__ r) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  r[e] = make_double2(b[e].x - r[e].x, b[e].y - r[e].y);
}

__global__ void k_zero_c128(int64_t n, double2* __restrict__ x) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = make_double2(0.0, 0.0);
}

// Arnoldi column j: H[0..j][j] = h, H[j+1][j] = ||w||; apply the previous
// Givens rotations, form rotation j, update g.  One thread.
// Layout: H column-major (m+1) x m; cs, sn: m entries; g: m+1 entries.
// st[0] = |g_{j+1}|, st[1] = H[j+1][j] before rotation.
__global__ void k_givens(int j, int m, const double2* __restrict__ h, const double2* __restrict__ wn,
                         double2* __restrict__ H, double* __restrict__ cs, double2* __restrict__ sn,
                         double2* __restrict__ g, double* __restrict__ st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double2* col = H + (size_t)j * (m + 1);
  for (int i = 0; i <= j; ++i) col[i] = h[i];
  double hn = sqrt(wn->x);
  col[j + 1] = make_double2(hn, 0.0);
  st[1] = hn;
  for (int i = 0; i < j; ++i) {  // [c s; -conj(s) c] applied to (col[i], col[i+1])
    double2 a = col[i], b = col[i + 1];
    double c = cs[i];
    double2 s = sn[i];
    double2 t = make_double2(c * a.x + s.x * b.x - s.y * b.y, c * a.y + s.x * b.y + s.y * b.x);
    double2 u = make_double2(-(s.x * a.x + s.y * a.y) + c * b.x, -(s.x * a.y - s.y * a.x) + c * b.y);
    col[i] = t;
    col[i + 1] = u;
  }
  double2 a = col[j];
  double b = hn;
  double aa = sqrt(a.x * a.x + a.y * a.y);
  double den = sqrt(aa * aa + b * b);
  double c;
  double2 s;
  if (den == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    s = make_double2(1.0, 0.0);
  } else {
    c = aa / den;
    s = make_double2(a.x / aa * b / den, a.y / aa * b / den);  // (a/|a|) conj(b)/den, b real
  }
  cs[j] = c;
  sn[j] = s;
  col[j] = make_double2(c * a.x + s.x * b, c * a.y + s.y * b);
  col[j + 1] = make_double2(0.0, 0.0);
  double2 gj = g[j];
  g[j + 1] = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));  // -conj(s) g_j
  g[j] = make_double2(c * gj.x, c * gj.y);
  st[0] = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
}

// Back substitution R y = g for the leading k x k block; one thread.
__global__ void k_backsolve(int kk, int m, const double2* __restrict__ H, const double2* __restrict__ g,
                            double2* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = kk - 1; i >= 0; --i) {
    double2 s = g[i];
    for (int q = i + 1; q < kk; ++q) {
      double2 r = H[(size_t)q * (m + 1) + i], v = y[q];
      s.x -= r.x * v.x - r.y * v.y;
      s.y -= r.x * v.y + r.y * v.x;
    }
    double2 d = H[(size_t)i * (m + 1) + i];
    double dd = d.x * d.x + d.y * d.y;
    y[i] = make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd);
  }
}

// h += h2 (small vectors)
__global__ void k_vec_add(int n, const double2* __restrict__ a, double2* __restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_double2(b[i].x + a[i].x, b[i].y + a[i].y);
}

// g = (beta, 0, ...), beta = sqrt(re(dotval))
__global__ void k_init_g(int m, const double2* __restrict__ dotval, double2* __restrict__ g) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m) return;
  g[i] = make_double2(i == 0 ? sqrt(dotval->x) : 0.0, 0.0);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_self(int64_t npan, const double* pan, double k, double ki, const double* gx, const double* gw, int ng,
                 double2* diag, hipStream_t s) {
  if (npan > 0) k_self<<<nblk(npan, 128), 128, 0, s>>>(npan, pan, k, ki, gx, gw, ng, diag);
}
void launch_near(int64_t nnz, const int32_t* rows, const int32_t* cols, const double* pan, double k, double ki,
                 int L, const double* gx, const double* gw, int ng, float2* val, hipStream_t s) {
  if (nnz > 0) k_near<<<nblk(nnz, 4), 256, 0, s>>>(nnz, rows, cols, pan, k, ki, L, gx, gw, ng, val);
}
void launch_near_apply(int64_t n, const int32_t* off, const int32_t* col, const float2* val,
                       const double2* diag, const float2* x, float2* y, hipStream_t s, bool overwrite) {
  if (n > 0) k_near_apply<<<nblk(n, 16), 256, 0, s>>>(n, off, col, val, diag, x, y, overwrite ? 1 : 0);
}
void launch_plane_wave(int64_t n, const double* pan, double k, double ki, const double* d, double2* b,
                       hipStream_t s) {
  if (n > 0) k_plane_wave<<<nblk(n, 256), 256, 0, s>>>(n, pan, k, ki, d[0], d[1], d[2], b);
}
void launch_to_c64(int64_t n, const double2* a, float2* b, hipStream_t s) {
  if (n > 0) k_to_c64<<<nblk(n, 256), 256, 0, s>>>(n, a, b);
}
void launch_from_c64_diag(int64_t n, const float2* y, const double2* diag, const double2* v, double2* out,
                          hipStream_t s, const float2* z) {
  if (n > 0) k_from_c64_diag<<<nblk(n, 256), 256, 0, s>>>(n, y, z, diag, v, out);
}
int mdot_blocks() { return kDotBlocks; }
void launch_mdot(int64_t n, int nv, const double2* V, int64_t ld, const double2* w, double2* partial,
                 double2* h, int accumulate, hipStream_t s) {
  k_mdot<<<kDotBlocks, 256, 0, s>>>(n, nv, V, ld, w, partial);
  k_mdot_final<<<1, 512, 0, s>>>(kDotBlocks, nv, partial, h, accumulate);
}
void launch_mupdate(int64_t n, int nv, const double2* V, int64_t ld, const double2* coef, double2* w,
                    double sign, hipStream_t s) {
  if (n > 0) k_mupdate<<<nblk(n, 256), 256, 0, s>>>(n, nv, V, ld, coef, w, sign);
}
void launch_scale_by_norm(int64_t n, const double2* src, const double2* dotval, double2* dst, hipStream_t s) {
  if (n > 0) k_scale_by_norm<<<nblk(n, 256), 256, 0, s>>>(n, src, dotval, dst);
}
void launch_zero_c128(int64_t n, double2* x, hipStream_t s) {
  if (n > 0) k_zero_c128<<<nblk(n, 256), 256, 0, s>>>(n, x);
}
void launch_residual(int64_t n, const double2* b, double2* r, hipStream_t s) {
  if (n > 0) k_residual<<<nblk(n, 256), 256, 0, s>>>(n, b, r);
}
void launch_givens(int j, int m, const double2* h, const double2* wn, double2* H, double* cs, double2* sn,
                   double2* g, double* st, hipStream_t s) {
  k_givens<<<1, 64, 0, s>>>(j, m, h, wn, H, cs, sn, g, st);
}
void launch_backsolve(int kk, int m, const double2* H, const double2* g, double2* y, hipStream_t s) {
  k_backsolve<<<1, 64, 0, s>>>(kk, m, H, g, y);
}
void launch_vec_add(int n, const double2* a, double2* b, hipStream_t s) {
  if (n > 0) k_vec_add<<<(n + 255) / 256, 256, 0, s>>>(n, a, b);
}
void launch_init_g(int m, const double2* dotval, double2* g, hipStream_t s) {
  k_init_g<<<(m + 256) / 256, 256, 0, s>>>(m, dotval, g);
}

}  // namespace hfmm
