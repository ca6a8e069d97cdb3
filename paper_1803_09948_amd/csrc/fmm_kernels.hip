// HIP kernels of the Helmholtz FMM matvec for gfx950 (Sec. 2.3, Listing 1).
//
// Expansion conventions (eqs. (12)-(14)):
//   Y_n^m = N_n^|m| P_n^|m|(cos t) e^{i m p} (no Condon-Shortley phase), so
//   Y_n^{-m} = conj(Y_n^m);  R_n^m(v) = j_n(k|v|) Y_n^m,  S_n^m(v) = h_n(k|v|) Y_n^m;
//   multipole  M_n^m = sum q R_n^{-m}(y - c),  field ik sum M S(x - c);
//   local      L_n^m = sum q S_n^{-m}(y - c),  field ik sum L R(x - c).
// Coefficients are stored scaled per level l to stay inside FP32 range:
//   M = sigma_n Mt,  Lt = sigma_n L,  sigma_n = rho_l^n / (2n+1)!!,
//   rho_l = min(1, k * side_l).
// The translation tables fold these factors in, so the scaling cancels in y.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include <type_traits>

#include "fmm_kernels.h"

namespace hfmm {

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cfma(float2 a, float2 b, float2 c) {  // a*b + c
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
__device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by i^code
__device__ inline float2 mul_ipow(float2 a, int code) {
  switch (code & 3) {
    case 0: return a;
    case 1: return make_float2(-a.y, a.x);
    case 2: return make_float2(-a.x, -a.y);
    default: return make_float2(a.y, -a.x);
  }
}

// Spherical Bessel j_n(x), n < nm <= 2*kMaxP, FP64.  x < 1: power series;
// x > nm: upward recurrence (stable for n < x); otherwise Miller's downward
// recurrence normalised by whichever of j_0, j_1 is larger in magnitude.
__device__ void bessel_j_all(int nm, double x, double* j) {
  if (x < 1.0) {
    double h = -0.5 * x * x, xn = 1.0, df = 1.0;  // x^n, (2n+1)!!
    for (int n = 0; n < nm; ++n) {
      df *= (2.0 * n + 1.0);
      double term = 1.0, sum = 1.0;
      for (int k = 1; k < 30; ++k) {
        term *= h / (k * (2.0 * n + 2.0 * k + 1.0));
        sum += term;
        if (fabs(term) < 1e-17 * fabs(sum)) break;
      }
      j[n] = xn / df * sum;
      xn *= x;
    }
    return;
  }
  double s = sin(x), c = cos(x);
  if (x > (double)nm) {
    j[0] = s / x;
    if (nm > 1) j[1] = s / (x * x) - c / x;
    for (int n = 1; n + 1 < nm; ++n) j[n + 1] = (2.0 * n + 1.0) / x * j[n] - j[n - 1];
    return;
  }
  int N = nm + 16 + (int)x;
  double fp1 = 0.0, f = 1e-30;
  for (int n = N; n >= 1; --n) {  // f = f_n, fp1 = f_{n+1}; step to f_{n-1}
    double fm1 = (2.0 * n + 1.0) / x * f - fp1;
    fp1 = f;
    f = fm1;
    if (n - 1 < nm) j[n - 1] = f;
    if (fabs(f) > 1e250) {
      fp1 *= 1e-250;
      f *= 1e-250;
      for (int m = n - 1; m < nm; ++m) j[m] *= 1e-250;
    }
  }
  double j0 = s / x, j1 = s / (x * x) - c / x;
  double scale = (fabs(j0) >= fabs(j1)) ? j0 / f : j1 / fp1;
  for (int n = 0; n < nm; ++n) j[n] *= scale;
}

// Complex FP64 arithmetic for a complex wavenumber k + i ki (damped waves).
struct zd {
  double re, im;
};
__device__ inline zd zmul(zd a, zd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline zd zscale(zd a, double s) { return {a.re * s, a.im * s}; }
__device__ inline zd zsub(zd a, zd b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline double zabs2(zd a) { return a.re * a.re + a.im * a.im; }
__device__ inline zd zinv(zd a) {
  const double d = 1.0 / zabs2(a);
  return {a.re * d, -a.im * d};
}
__device__ inline zd zsin(zd z) { return {sin(z.re) * cosh(z.im), cos(z.re) * sinh(z.im)}; }
__device__ inline zd zcos(zd z) { return {cos(z.re) * cosh(z.im), -sin(z.re) * sinh(z.im)}; }

// j_n(z), n < nm, complex z (|z| > 0): power series for |z| < 1, else
// Miller's downward recurrence normalised by the larger of j_0, j_1.
__device__ void bessel_j_all_c(int nm, zd z, zd* j) {
  const double az = sqrt(zabs2(z));
  if (az < 1.0) {
    const zd h = zscale(zmul(z, z), -0.5);
    zd zn = {1.0, 0.0};
    double df = 1.0;
    for (int n = 0; n < nm; ++n) {
      df *= (2.0 * n + 1.0);
      zd term = {1.0, 0.0}, sum = {1.0, 0.0};
      for (int k = 1; k < 30; ++k) {
        term = zscale(zmul(term, h), 1.0 / (k * (2.0 * n + 2.0 * k + 1.0)));
        sum = {sum.re + term.re, sum.im + term.im};
        if (zabs2(term) < 1e-34 * zabs2(sum)) break;
      }
      j[n] = zscale(zmul(zn, sum), 1.0 / df);
      zn = zmul(zn, z);
    }
    return;
  }
  const zd iz = zinv(z), sn = zsin(z), cs = zcos(z);
  const zd j0 = zmul(sn, iz), j1 = zmul(zsub(zmul(sn, iz), cs), iz);
  const int N = nm + 16 + (int)az;
  zd fp1 = {0.0, 0.0}, f = {1e-30, 0.0};
  for (int n = N; n >= 1; --n) {
    const zd fm1 = zsub(zscale(zmul(iz, f), 2.0 * n + 1.0), fp1);
    fp1 = f;
    f = fm1;
    if (n - 1 < nm) j[n - 1] = f;
    if (zabs2(f) > 1e300) {
      fp1 = zscale(fp1, 1e-250);
      f = zscale(f, 1e-250);
      for (int m = n - 1; m < nm; ++m) j[m] = zscale(j[m], 1e-250);
    }
  }
  const zd sc = (zabs2(j0) >= zabs2(j1)) ? zmul(j0, zinv(f)) : zmul(j1, zinv(fp1));
  for (int n = 0; n < nm; ++n) j[n] = zmul(j[n], sc);
}

// h_n(z) = j_n + i y_n, n < nm, complex z (|z| > 0), by upward recurrence
// from h_0 = -i e^{iz} / z and h_1 = -e^{iz} (z + i) / z^2.
__device__ void hankel_all_c(int nm, zd z, zd* h) {
  const zd iz = zinv(z);
  const double ea = exp(-z.im);
  const zd eiz = {ea * cos(z.re), ea * sin(z.re)};
  h[0] = zmul({0.0, -1.0}, zmul(eiz, iz));
  if (nm > 1) h[1] = zscale(zmul(eiz, zmul({z.re, z.im + 1.0}, zmul(iz, iz))), -1.0);
  for (int n = 1; n + 1 < nm; ++n) h[n + 1] = zsub(zscale(zmul(iz, h[n]), 2.0 * n + 1.0), h[n - 1]);
}

// ---------------------------------------------------------------------------
// Translation tables.  For operator o and entry (row r = (n',m'), col c=(n,m)):
//   T[o][c][r] = sum_l coef * H_l^{m-m'}(t) * scale(n, n'),
// with H = S (M2L) or R (M2M, L2L) and coef = 4 pi i^{n'+l-n} Gaunt.
// One block per operator; the harmonics of t are built in LDS in FP64.
// XZ: the M2L operators (t in the xz-plane) are stored as the C and S
// blocks of XzDims: C[k][r] = (T[r][(n,m)] + T[r][(n,-m)]) / 2 for m > 0,
// T[r][(n,0)] for m = 0, and S[k][r] = (T[r][(n,m)] - T[r][(n,-m)]) / 2, with
// k = (n, m) and r = (n', m') the C- or S-list entries.
// ---------------------------------------------------------------------------
__device__ inline void store_entry(float2* p, double re, double im) { *p = make_float2((float)re, (float)im); }
__device__ inline void store_entry(double2* p, double re, double im) { *p = make_double2(re, im); }

template <class C2, bool XZ>
__global__ void k_gen_tables(const OpDescDev* __restrict__ ops, int nops, int P, double k, double ki,
                             const int32_t* __restrict__ cp_off, const int32_t* __restrict__ cp_lm,
                             const double2* __restrict__ cp_val, int Kp, int Rp, int stride,
                             C2* __restrict__ tables) {
  const int o = blockIdx.x;
  if (o >= nops) return;
  const int L = 2 * P - 1;
  __shared__ double2 harm[(2 * kMaxP - 1) * (2 * kMaxP - 1)];
  __shared__ double sig_in[kMaxP], sig_out[kMaxP];
  const OpDescDev d = ops[o];
  // an M2L operator in the xz-plane form is built at t turned into the plane
  const bool xzop = XZ && d.kind == 2;
  const double tx = xzop ? sqrt(d.t[0] * d.t[0] + d.t[1] * d.t[1]) : d.t[0], ty = xzop ? 0.0 : d.t[1],
               tz = d.t[2];
  const double r = sqrt(tx * tx + ty * ty + tz * tz);
  if (threadIdx.x == 0) {
    // radial functions
    double jr[2 * kMaxP], yr[2 * kMaxP];
    double x = k * r;
    if (ki != 0.0) {
      // complex argument: (j + i y) or j as complex numbers, split into the
      // real and imaginary parts the angular product below expects
      zd f[2 * kMaxP];
      if (d.kind == 2)
        hankel_all_c(L, {x, ki * r}, f);
      else
        bessel_j_all_c(L, {x, ki * r}, f);
      for (int n = 0; n < L; ++n) {
        jr[n] = f[n].re;
        yr[n] = f[n].im;
      }
    } else if (d.kind == 2) {
      // h_l = j_l + i y_l by upward recurrence: stable for y_l, and the error
      // it leaves in j_l is relative to |h_l|
      double s = sin(x), c = cos(x);
      jr[0] = s / x;
      yr[0] = -c / x;
      if (L > 1) {
        jr[1] = s / (x * x) - c / x;
        yr[1] = -c / (x * x) - s / x;
      }
      for (int n = 1; n + 1 < L; ++n) {
        jr[n + 1] = (2.0 * n + 1.0) / x * jr[n] - jr[n - 1];
        yr[n + 1] = (2.0 * n + 1.0) / x * yr[n] - yr[n - 1];
      }
    } else {
      bessel_j_all(L, x, jr);
      for (int n = 0; n < L; ++n) yr[n] = 0.0;
    }
    // angular part: pbar_l^|mu|(cos theta) e^{i mu phi}
    double ct = (r > 0) ? tz / r : 1.0;
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double ph = atan2(ty, tx);
    double p[(2 * kMaxP - 1) * (2 * kMaxP - 1)];
    for (int i = 0; i < L * L; ++i) p[i] = 0.0;
    p[0] = 1.0 / sqrt(4.0 * M_PI);
    for (int m = 1; m < L; ++m) p[m * m + 2 * m] = sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * p[(m - 1) * (m - 1) + 2 * (m - 1)];
    for (int m = 0; m + 1 < L; ++m) p[(m + 1) * (m + 1) + (m + 1) + m] = sqrt(2.0 * m + 3.0) * ct * p[m * m + 2 * m];
    for (int m = 0; m < L; ++m)
      for (int n = m + 2; n < L; ++n) {
        double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
        double bb = sqrt(((double)(n - 1) * (n - 1) - (double)m * m) / (4.0 * (n - 1) * (n - 1) - 1.0));
        p[n * n + n + m] = a * (ct * p[(n - 1) * (n - 1) + (n - 1) + m] - bb * p[(n - 2) * (n - 2) + (n - 2) + m]);
      }
    for (int n = 0; n < L; ++n)
      for (int m = -n; m <= n; ++m) {
        double pv = p[n * n + n + (m < 0 ? -m : m)];
        double cr = cos(m * ph), si = sin(m * ph);
        double re = jr[n] * pv, im = yr[n] * pv;  // radial (j + i y) times real pbar
        harm[n * n + n + m] = make_double2(re * cr - im * si, re * si + im * cr);
      }
    // scale factors sigma_n(rho) = rho^n / (2n+1)!!
    double df = 1.0, ri = 1.0, ro = 1.0;
    for (int n = 0; n < P; ++n) {
      df *= (2.0 * n + 1.0);
      sig_in[n] = ri / df;
      sig_out[n] = ro / df;
      ri *= d.rho_in;
      ro *= d.rho_out;
    }
  }
  __syncthreads();
  const int P2 = P * P;
  C2* T = tables + (size_t)o * stride;
  // dense entry (row (n',m'), col (n,m)), scaled
  auto dense = [&](int row, int col, double& re, double& im) {
    const int e = row * P2 + col;
    const int n2 = (int)sqrt((double)row), n = (int)sqrt((double)col);
    re = 0.0;
    im = 0.0;
    for (int q = cp_off[e]; q < cp_off[e + 1]; ++q) {
      double2 cv = cp_val[q];
      double2 h = harm[cp_lm[q]];
      re += cv.x * h.x - cv.y * h.y;
      im += cv.x * h.y + cv.y * h.x;
    }
    double sc;
    if (d.kind == 0) sc = sig_in[n] / sig_out[n2];        // M2M
    else if (d.kind == 1) sc = sig_out[n2] / sig_in[n];   // L2L
    else sc = sig_out[n2] * sig_in[n];                    // M2L
    re *= sc;
    im *= sc;
  };
  if (xzop) {
    const XzDims xd = xz_dims(P);
    // azimuth phases e^{i m phi} of t, m < P
    const double phi = atan2(d.t[1], d.t[0]);
    for (int m = threadIdx.x; m < P; m += blockDim.x) store_entry(T + xd.Kx * xd.Rx + m, cos(m * phi), sin(m * phi));
    for (int f = threadIdx.x; f < xd.Kx * xd.Rx; f += blockDim.x) {
      const int kk = f / xd.Rx, r = f % xd.Rx;
      const bool sb = r >= 16 * xd.RTC;
      const int rr = sb ? r - 16 * xd.RTC : r, lim = sb ? xd.S : xd.C;
      if (kk >= lim || rr >= lim) {
        store_entry(T + f, 0.0, 0.0);
        continue;
      }
      int n, m, n2, m2;
      xz_entry(P, kk, &n, &m);
      xz_entry(P, rr, &n2, &m2);
      const int row = n2 * n2 + n2 + m2;
      double ar, ai;
      dense(row, n * n + n + m, ar, ai);
      if (m == 0) {
        store_entry(T + f, ar, ai);
        continue;
      }
      double br, bi;
      dense(row, n * n + n - m, br, bi);
      if (sb)
        store_entry(T + f, 0.5 * (ar - br), 0.5 * (ai - bi));
      else
        store_entry(T + f, 0.5 * (ar + br), 0.5 * (ai + bi));
    }
    return;
  }
  // standard index n^2 + n + m of storage position pos of a multipole (FP32
  // M2M: input and output multipoles are stored in mpos order)
  auto mstd = [&](int pos) {
    for (int n = 0; n < P; ++n)
      for (int m = -n; m <= n; ++m)
        if (mpos(P, n, m) == pos) return n * n + n + m;
    return 0;
  };
  const bool mperm = XZ && d.kind == 0;
  for (int f = threadIdx.x; f < Kp * Rp; f += blockDim.x) {
    const int col = f / Rp, row = f % Rp;  // col (n,m) = input, row (n',m') = output
    if (col >= P2 || row >= P2) {
      store_entry(T + f, 0.0, 0.0);
      continue;
    }
    double re, im;
    if (mperm)
      dense(mstd(row), mstd(col), re, im);
    else
      dense(row, col, re, im);
    store_entry(T + f, re, im);
  }
}

// ---------------------------------------------------------------------------
// Instance-aware kernels.  Every work item names an instance; its pointers
// come from the instance table, so one launch can serve many independent
// problems (a single matvec is a batch of one).
// ---------------------------------------------------------------------------
constexpr int kChunk = 4096;   // elements per block for zero / gather / scatter

// M = L = 0 and the sorted outputs ys = 0 for the listed instances (items:
// instance, element offset over max(ncell P^2, ntgt))
__global__ void k_zero(const int2* __restrict__ items, int n, const InstDev* __restrict__ insts) {
  const int2 it = items[blockIdx.x];
  const InstDev& I = insts[it.x];
  const int64_t e0 = (int64_t)it.y * kChunk;
  const int64_t e1 = min(e0 + kChunk, (int64_t)I.ncellP2);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    I.M[e] = make_float2(0.f, 0.f);
    I.L[e] = make_float2(0.f, 0.f);
  }
  const int64_t t1 = min(e0 + kChunk, I.ntgt);
  for (int64_t e = e0 + threadIdx.x; e < t1; e += blockDim.x) I.ys[e] = make_float2(0.f, 0.f);
}

// q_s = w_s x[unknown_s] in Morton order (items: instance, body offset)
__global__ void k_gather(const int2* __restrict__ items, const InstDev* __restrict__ insts) {
  const int2 it = items[blockIdx.x];
  const InstDev& I = insts[it.x];
  const int64_t e0 = (int64_t)it.y * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.nsrc);
  for (int64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) {
    float2 v = I.x[I.src_idx[i]];
    if (I.src_w) {
      const float s = I.src_w[i];
      v = make_float2(v.x * s, v.y * s);
    }
    I.q[i] = v;
  }
}

// y[perm_i] = ys_i (items: instance, body offset)
__global__ void k_scatter(const int2* __restrict__ items, const InstDev* __restrict__ insts) {
  const int2 it = items[blockIdx.x];
  const InstDev& I = insts[it.x];
  const int64_t e0 = (int64_t)it.y * kChunk;
  const int64_t e1 = min(e0 + kChunk, I.ntgt);
  for (int64_t i = e0 + threadIdx.x; i < e1; i += blockDim.x) I.y[I.tgt_perm[i]] = I.ys[i];
}

// Coefficients of the normalised Legendre recurrences (no Condon-Shortley
// phase), evaluated at compile time:
//   Pb_m^m = f_m (x + iy)/r Pb_{m-1}^{m-1},  f_m = sqrt((2m+1)/(2m)),
//   Pb_{m+1}^m = g_m cos(theta) Pb_m^m,      g_m = sqrt(2m+3),
//   Pb_n^m = a_nm (cos(theta) Pb_{n-1}^m - b_nm Pb_{n-2}^m),
//   a_nm = sqrt((4n^2-1)/(n^2-m^2)),  b_nm = sqrt(((n-1)^2-m^2)/(4(n-1)^2-1)).
constexpr double cx_sqrt(double x) {
  if (x <= 0.0) return 0.0;
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 200; ++i) r = 0.5 * (r + x / r);
  return r;
}
struct YlmTab {
  float a[kMaxP][kMaxP], b[kMaxP][kMaxP], f[kMaxP], g[kMaxP];
};
constexpr YlmTab make_ylm_tab() {
  YlmTab t{};
  for (int n = 0; n < kMaxP; ++n)
    for (int m = 0; m + 2 <= n; ++m) {
      t.a[n][m] = (float)cx_sqrt((4.0 * n * n - 1.0) / (double)(n * n - m * m));
      t.b[n][m] = (float)cx_sqrt((double)((n - 1) * (n - 1) - m * m) / (4.0 * (n - 1) * (n - 1) - 1.0));
    }
  for (int m = 0; m < kMaxP; ++m) {
    t.f[m] = m > 0 ? (float)cx_sqrt((2.0 * m + 1.0) / (2.0 * m)) : 0.f;
    t.g[m] = (float)cx_sqrt(2.0 * m + 3.0);
  }
  return t;
}
__constant__ YlmTab c_ylm = make_ylm_tab();

// Visits Y_n^m (m >= 0, FP32) of the direction (dx, dy, dz)/r in the order
// m = 0..P-1, n = m..P-1, calling f(n, m, Y).  P is a compile-time order, so
// every index is static.
template <int P, class F>
__device__ inline void ylm_visit(float dx, float dy, float dz, float r, F&& f) {
  float c = 1.f, wx = 0.f, wy = 0.f;
  if (r > 0.f) {
    const float ir = 1.f / r;
    c = dz * ir;
    wx = dx * ir;
    wy = dy * ir;
  }
  float2 pmm = make_float2(0.28209479177387814f, 0.f);  // 1/sqrt(4 pi)
#pragma unroll
  for (int m = 0; m < P; ++m) {
    if (m > 0) {
      const float fm = c_ylm.f[m];
      pmm = make_float2(fm * (pmm.x * wx - pmm.y * wy), fm * (pmm.x * wy + pmm.y * wx));
    }
    f(m, m, pmm);
    if (m + 1 < P) {
      const float gm = c_ylm.g[m] * c;
      float2 p2 = pmm, p1 = make_float2(gm * pmm.x, gm * pmm.y);
      f(m + 1, m, p1);
#pragma unroll
      for (int n = m + 2; n < P; ++n) {
        const float an = c_ylm.a[n][m], bn = c_ylm.b[n][m];
        const float2 p = make_float2(an * (c * p1.x - bn * p2.x), an * (c * p1.y - bn * p2.y));
        f(n, m, p);
        p2 = p1;
        p1 = p;
      }
    }
  }
}

// b_n = j_n(x) (2n+1)!! / rho^n, n < P (FP64 recurrences, one division):
// x < 1e-3: the first two terms of the series of j_n; x > P: upward
// recurrence; otherwise Miller's downward recurrence, normalised by j_0 or
// j_1.
template <int P>
__device__ inline void radial_scaled(double x, double rho, float* b) {
  if (x < 1e-3) {
    const double xr = x / rho, x2 = x * x;
    double p = 1.0;
#pragma unroll
    for (int n = 0; n < P; ++n) {
      b[n] = (float)(p * (1.0 - x2 / (4.0 * n + 6.0)));
      p *= xr;
    }
    return;
  }
  double j[P];
  const double ix = 1.0 / x, s = sin(x), c = cos(x);
  const double j0 = s * ix, j1 = (s * ix - c) * ix;
  if (x > (double)P) {
    j[0] = j0;
    if constexpr (P > 1) j[1] = j1;
#pragma unroll
    for (int n = 1; n + 1 < P; ++n) j[n + 1] = (2.0 * n + 1.0) * ix * j[n] - j[n - 1];
  } else {
    // start above P; x >= 1e-3 keeps the values below 1e250 over these steps
    const int N = P + 16 + (int)x;
    double fp1 = 0.0, f = 1e-30;
    for (int n = N; n > P; --n) {
      const double fm1 = (2.0 * n + 1.0) * ix * f - fp1;
      fp1 = f;
      f = fm1;
    }
    // f = f_P, fp1 = f_{P+1}
#pragma unroll
    for (int n = P; n >= 1; --n) {
      const double fm1 = (2.0 * n + 1.0) * ix * f - fp1;
      fp1 = f;
      f = fm1;
      j[n - 1] = f;
    }
    // f = f_0, fp1 = f_1
    const double scale = (fabs(j0) >= fabs(j1)) ? j0 / f : j1 / fp1;
#pragma unroll
    for (int n = 0; n < P; ++n) j[n] *= scale;
  }
  double df = 1.0, rp = 1.0;
#pragma unroll
  for (int n = 0; n < P; ++n) {
    df *= (2.0 * n + 1.0);
    b[n] = (float)(j[n] * df / rp);
    rp *= rho;
  }
}

// The same for a complex argument z = (k + i ki) r: b_n = j_n(z) (2n+1)!! / rho^n.
// |z| < 1e-3: the first two series terms; else Miller's downward recurrence
// normalised by the larger of j_0, j_1.
template <int P>
__device__ inline void radial_scaled_c(double zr, double zi, double rho, float2* b) {
  const zd z = {zr, zi};
  const double az = sqrt(zabs2(z));
  if (az < 1e-3) {
    const zd zr_ = zscale(z, 1.0 / rho), z2 = zmul(z, z);
    zd p = {1.0, 0.0};
#pragma unroll
    for (int n = 0; n < P; ++n) {
      const zd v = zmul(p, {1.0 - z2.re / (4.0 * n + 6.0), -z2.im / (4.0 * n + 6.0)});
      b[n] = make_float2((float)v.re, (float)v.im);
      p = zmul(p, zr_);
    }
    return;
  }
  zd j[P];
  const zd iz = zinv(z), sn = zsin(z), cs = zcos(z);
  const zd j0 = zmul(sn, iz), j1 = zmul(zsub(zmul(sn, iz), cs), iz);
  const int N = P + 16 + (int)az;
  zd fp1 = {0.0, 0.0}, f = {1e-30, 0.0};
  for (int n = N; n > P; --n) {
    const zd fm1 = zsub(zscale(zmul(iz, f), 2.0 * n + 1.0), fp1);
    fp1 = f;
    f = fm1;
  }
#pragma unroll
  for (int n = P; n >= 1; --n) {
    const zd fm1 = zsub(zscale(zmul(iz, f), 2.0 * n + 1.0), fp1);
    fp1 = f;
    f = fm1;
    j[n - 1] = f;
  }
  const zd sc = (zabs2(j0) >= zabs2(j1)) ? zmul(j0, zinv(f)) : zmul(j1, zinv(fp1));
  double df = 1.0, rp = 1.0;
#pragma unroll
  for (int n = 0; n < P; ++n) {
    df *= (2.0 * n + 1.0);
    const zd v = zscale(zmul(j[n], sc), df / rp);
    b[n] = make_float2((float)v.re, (float)v.im);
    rp *= rho;
  }
}

// ---------------------------------------------------------------------------
// P2M: one wave per leaf, up to 32 bodies per pass (keeps the LDS per wave
// small enough for several waves per SIMD).
// Mt_n^m = sum_j q_j b_n(k r_j) conj(Y_n^m(dir_j)), Mt_n^{-m} = sum_j q_j b_n Y_n^m.
// DAMP: complex wavenumber, so b_n is complex and is not conjugated with Y.
// ---------------------------------------------------------------------------
template <int P, bool DAMP>
__global__ void __launch_bounds__(64) k_p2m(const int2* __restrict__ items, const InstDev* __restrict__ insts) {
  constexpr int NY = P * (P + 1) / 2, P2 = P * P;
  const int2 it = items[blockIdx.x];
  const InstDev& I = insts[it.x];
  const int cell = it.y;
  const int4 rg = I.cells[cell];
  const float4 g = I.geo[cell];
  const double rh = I.rho[I.clev[cell]];
  const float k = I.k;
  constexpr int CH = 32;
  __shared__ float2 sa[CH][NY];
  __shared__ float2 sq[CH];
  __shared__ float2 sb[DAMP ? CH : 1][DAMP ? P : 1];
  const int lane = threadIdx.x;
  float2 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = make_float2(0.f, 0.f);
  for (int j0 = rg.x; j0 < rg.y; j0 += CH) {
    const int nj = min(CH, rg.y - j0);
    if (lane < nj) {
      const float4 p = I.spos[j0 + lane];
      const float dx = p.x - g.x, dy = p.y - g.y, dz = p.z - g.z;
      const float r = sqrtf(dx * dx + dy * dy + dz * dz);
      float2* a = sa[lane];
      if constexpr (DAMP) {
        radial_scaled_c<P>((double)k * (double)r, (double)I.ki * (double)r, rh, sb[lane]);
        ylm_visit<P>(dx, dy, dz, r, [&](int n, int m, float2 y) { a[n * (n + 1) / 2 + m] = y; });
      } else {
        float b[P];
        radial_scaled<P>((double)k * (double)r, rh, b);
        ylm_visit<P>(dx, dy, dz, r, [&](int n, int m, float2 y) {
          a[n * (n + 1) / 2 + m] = make_float2(y.x * b[n], y.y * b[n]);
        });
      }
      sq[lane] = I.q[j0 + lane];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t;
      if (e < P2) {
        const int n = (int)sqrtf((float)e + 0.5f);
        const int m = e - n * n - n;
        const int ai = n * (n + 1) / 2 + (m < 0 ? -m : m);
        const float sgn = m >= 0 ? -1.f : 1.f;  // conj for m >= 0
        float2 s = acc[t];
        for (int j = 0; j < nj; ++j) {
          float2 y = sa[j][ai];
          y.y *= sgn;
          if constexpr (DAMP) y = cmul(sb[j][n], y);
          s = cfma(sq[j], y, s);
        }
        acc[t] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = lane + 64 * t;
    if (e < P2) {
      const int n = (int)sqrtf((float)e + 0.5f);
      I.M[(size_t)cell * P2 + mpos(P, n, e - n * n - n)] = acc[t];
    }
  }
}

// ---------------------------------------------------------------------------
// M2L on the matrix cores.  One wave takes up to 16*NCT pairs that share one
// canonical operator: a translation in the xz-plane, held as its C and S
// blocks (XzDims; together about half the P^2 x P^2 complex entries of the
// full operator).  The B matrix (k = input entry, column = pair) is gathered
// straight from the multipoles through the pair's reflection codes and
// turned by the operator's azimuth phase; the table streams from memory as
// the A matrix (row = output entry), with A and B prefetched ahead.  Each
// pair's result goes, in the reflected frame, to the pair's staging slot
// (the reduction maps it back); the LDS holds the code table, the
// operator's phases and one output tile.  Blocks are mapped so that each XCD walks a
// contiguous range of chunks (sorted by operator), keeping an operator's
// table in that XCD's L2 while its chunks run.
//
// MFMA 16x16x4 f32 lane layout: A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k, D[4q + v][j] in lane j + 16q, register v.
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Global-address-space views of pointers read from the instance table (so
// that loads through them are global loads, not flat ones).
typedef float f2v __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) f2v gcfloat2;
typedef __attribute__((address_space(1))) f2v gfloat2;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f4v gfloat4;
typedef int i4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) i4v gcint4;
__device__ inline int4 ld_int4(const int4* p) {
  const i4v v = *(gcint4*)p;
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ inline float2 ld2(gcfloat2* p) {
  const f2v v = *p;
  return make_float2(v.x, v.y);
}
// i^ph (x + iy) for a reflection code (swap bit 16, sign of the real part
// bit 31, of the imaginary part bit 30).
__device__ inline float2 apply_code(float x0, float y0, int e) {
  const bool swap = e & (1 << 16);
  const float x = swap ? y0 : x0, y = swap ? x0 : y0;
  return make_float2(__int_as_float(__float_as_int(x) ^ (e & (int)0x80000000)),
                     __int_as_float(__float_as_int(y) ^ ((e << 1) & (int)0x80000000)));
}

// One wave per item; an item is column group h < sub of chunk item / sub,
// i.e. pairs [16 NCT h, 16 NCT (h + 1)) of the chunk.  The complex product
// uses three real MFMAs per tile and k-step (Gauss):
//   K1 += (Tr + Ti) Br,  K2 += Tr (Bi - Br),  K3 += Ti (Br + Bi),
//   C = (K1 - K3) + i (K1 + K2).
// The RTC C-block tiles take B = u, the RTS S-block tiles B = v, where for
// input (n, m) of the C-list and the operator's azimuth phase p = e^{i m phi}:
//   u = p B[(n,m)] + conj(p) B[(n,-m)],  v = p B[(n,m)] - conj(p) B[(n,-m)]
// with B the reflected multipoles (B[(n,-m)] = 0 for m = 0).  The first KSS
// k-steps feed both blocks, the last KSC - KSS only C.  Outputs: for S-list
// row (n', m'), L^{m'} = conj(p') (A + B) and L^{-m'} = p' (A - B) with
// p' = e^{i m' phi}, A the C-block and B the S-block result; the m' = 0 rows
// are A.
// WPE is the number of waves per SIMD the register budget is sized for.
template <int P, int NCT, int WPE, int CPW, int AD>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE)))
k_m2l_mfma(const int4* __restrict__ chunks, int nitems, int per_xcd, int sub,
           const InstDev* __restrict__ insts, const int32_t* __restrict__ bmap) {
  constexpr XzDims X = xz_dims(P);
  constexpr int P2 = P * P, RT = X.RT, RTC = X.RTC, RTS = X.RTS, KSS = X.KSS, KSC = X.KSC, Kx = X.Kx,
                Rx = X.Rx;
  constexpr int TSTRIDE = xz_table_stride(P);  // table entries per operator
  constexpr int SM = xz_stage_sm(P), ST = xz_stage_st(P);
  constexpr int KXS = xz_code_stride(P), NCODE = 17 * KXS;
  extern __shared__ int smap[];     // [17][KXS] input codes (m2l_xz_codes), then [16 RTS] m' of the S-list rows
  const int b = blockIdx.x;
  const int w = (b & 7) * per_xcd + (b >> 3);
  if (w * CPW >= nitems) return;
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  {  // copy the code table: all loads in flight before the LDS writes (indices
     // are clamped, so a lane past the end copies the last entry again)
    const int4* src = reinterpret_cast<const int4*>(bmap);
    int4* dst = reinterpret_cast<int4*>(smap);
    constexpr int n4 = (NCODE + 16 * RTS) / 4;
    constexpr int U = 8;
    for (int base = 0; base < n4; base += 64 * U) {
      int4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = src[min(base + lane + 64 * u, n4 - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) dst[min(base + lane + 64 * u, n4 - 1)] = v[u];
    }
  }
  __syncthreads();
  const int* mrow = smap + NCODE;
  // the wave runs CPW consecutive items (one operator's table stays hot in
  // L2 and one item's result stores drain while the next item computes)
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int item = w * CPW + c;
    if (item >= nitems) break;
    const int ci = item / sub;
    const int4 ch = chunks[ci];       // (instance, op, pair begin, pair end)
    const InstDev& I = insts[ch.x];
    const int op = ch.y, pb = ch.z + 16 * NCT * (item - ci * sub);
    const int np = min(ch.w - pb, 16 * NCT);
    if (np <= 0) continue;
    // column t of this lane is pair 16 t + li: (target, source, reflection,
    // slot); a column past the item's end reads the all-zero code row 16.
    // The multipoles of column t: a 32-bit byte offset msb[t] beside the
    // wave-uniform base Mb (M of an instance is < 4 GiB)
    const char* Mb = reinterpret_cast<const char*>(I.M);
    uint32_t msb[NCT];
    int goff[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      const int p = 16 * t + li;
      const bool ok = p < np;
      const int4 pr = ld_int4(I.m2l_pairs + pb + (ok ? p : 0));
      msb[t] = (uint32_t)pr.y * (uint32_t)(P2 * sizeof(float2));
      goff[t] = (ok ? pr.z : 16) * KXS + lk;
    }
    // the operator's table ([Kx][Rx], then its phases e^{i m phi}, m < P):
    // the wave-uniform base Tb and this lane's 32-bit byte offset
    const char* Tb = reinterpret_cast<const char*>(I.tables + (size_t)op * TSTRIDE);
    auto lds_sync = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // the operator's phases, copied to LDS (read per k-step and per output row)
    __shared__ float2 sph[kMaxP];
    if (lane < P) sph[lane] = ld2((gcfloat2*)(I.tables + (size_t)op * TSTRIDE + Kx * Rx) + lane);
    lds_sync();
    // B gather: the aligned pair of float2 holding the two reflected
    // multipoles of each column's input (one 16-byte load when P^2 is even,
    // so that every pair is 16-byte aligned and inside the multipole, else
    // two 8-byte loads) and the
    // input's phase (the same for every column: m depends on k only); the
    // loads issue now, codes and phases apply when the step runs
    auto load_b = [&](int k4, float2* rx, float2* ry, float2& rp, int* ce) {
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
        const int e = smap[goff[t] + k4];
        ce[t] = e;
        const uint32_t off = msb[t] + (uint32_t)(e & 0xff) * (uint32_t)sizeof(float2);
        if constexpr (P2 % 2 == 0) {
          const f4v v = *(const __attribute__((address_space(1))) f4v*)(Mb + off);
          rx[t] = make_float2(v.x, v.y);
          ry[t] = make_float2(v.z, v.w);
        } else {
          // odd P^2: the pair of the last (n, 0) entry would end past the
          // multipole; its high half is marked zero, so read the low one again
          rx[t] = ld2((gcfloat2*)(Mb + off));
          ry[t] = ld2((gcfloat2*)(Mb + off + ((e & 0xff) + 1 < P2 ? sizeof(float2) : 0)));
        }
      }
      rp = sph[(ce[0] >> 9) & 15];
    };
    // the Gauss operands of u (C block) and v (S block), from the pair's
    // turned halves lo', hi' (m2l_xz_codes): u = q lo' + conj(q) hi',
    // v = q lo' - conj(q) hi', q = p or conj(p); ZERO: apply the codes' zero
    // marks (needed only where the C-list reaches m = 0 or its end: the
    // columns past a chunk's end are never stored, whatever they compute)
    float uu[NCT], ud[NCT], us[NCT], vu[NCT], vd[NCT], vs[NCT];
    auto finish_b = [&](const float2* rx, const float2* ry, float2 rp, const int* ce, auto zero_tag) {
      constexpr bool ZERO = decltype(zero_tag)::value;
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
        const int e = ce[t], he = e << 3;  // hi's flags sit 3 bits lower
        const float2 l0 = apply_code(rx[t].x, rx[t].y, e);
        const float2 h0 = apply_code(ry[t].x, ry[t].y, he);
        float lr = l0.x, lim = l0.y, hr = h0.x, him = h0.y;
        if constexpr (ZERO) {
          const bool zl = e & (1 << 17), zh = he & (1 << 17);
          lr = zl ? 0.f : lr;
          lim = zl ? 0.f : lim;
          hr = zh ? 0.f : hr;
          him = zh ? 0.f : him;
        }
        const float sr = lr + hr, si = lim + him, dr = lr - hr, di = lim - him;
        const float pr = rp.x, pi = __int_as_float(__float_as_int(rp.y) ^ ((e << 23) & (int)0x80000000));
        const float ur = fmaf(pr, sr, -pi * di), ui = fmaf(pr, si, pi * dr);
        const float wr = fmaf(pr, dr, -pi * si), wi = fmaf(pr, di, pi * sr);
        uu[t] = ur;
        ud[t] = ui - ur;
        us[t] = ur + ui;
        vu[t] = wr;
        vd[t] = wi - wr;
        vs[t] = wr + wi;
      }
    };
    floatx4 k1[NCT][RT], k2[NCT][RT], k3[NCT][RT];
#pragma unroll
    for (int t = 0; t < NCT; ++t)
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        k1[t][r] = floatx4{0.f, 0.f, 0.f, 0.f};
        k2[t][r] = floatx4{0.f, 0.f, 0.f, 0.f};
        k3[t][r] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
    const uint32_t tlane = (uint32_t)li * (uint32_t)sizeof(float2);
    // the table operand (A) is loaded AD k-steps ahead (2 AD register
    // buffers), the gathered multipoles (B) one step ahead into one buffer
    // that each step first turns into its operands; a straight-line loop
    // body of four steps keeps the compiler's wait counts exact
    constexpr int AM = 2 * AD - 1;
    float2 av[2 * AD][RT], bx[NCT], by[NCT], bp;
    int ce[NCT];
    auto load_a = [&](int k, float2* out) {
      const uint32_t off = tlane + (uint32_t)(k * Rx) * (uint32_t)sizeof(float2);
#pragma unroll
      for (int r = 0; r < RT; ++r) out[r] = ld2((gcfloat2*)(Tb + (off + (uint32_t)(16 * r * sizeof(float2)))));
    };
    auto mma = [&](const float2* a, bool joint) {
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        if (r >= RTC && !joint) break;
        const float ar = a[r].x, ai = a[r].y, as = ar + ai;
        const bool sb = r >= RTC;
#pragma unroll
        for (int t = 0; t < NCT; ++t)
          k1[t][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, sb ? vu[t] : uu[t], k1[t][r], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < NCT; ++t)
          k2[t][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, sb ? vd[t] : ud[t], k2[t][r], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < NCT; ++t)
          k3[t][r] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, sb ? vs[t] : us[t], k3[t][r], 0, 0, 0);
      }
    };
    // step s: issue A(s + AD), form step s's B operands, issue B(s + 1),
    // then the MFMAs of step s; the loop runs whole groups of four joint
    // steps and clamps k (redundant in-bounds loads past the end are unused),
    // the remaining steps follow unrolled (joint while s < KSS, then C only).
    // Every step applies the zero marks: a zero-free variant for the steps
    // inside the S-list costs registers (the straight-line remainder grows)
    constexpr int klast = Kx - 4, KS4 = (KSS / 4) * 4;
    using withzero = std::integral_constant<bool, true>;
#pragma unroll
    for (int d = 0; d < AD; ++d)
      if (d < KSC) load_a(4 * d + lk, av[d]);
    load_b(0, bx, by, bp, ce);
    for (int ks = 0; ks < KS4; ks += 4) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        load_a(min(4 * (ks + j + AD), klast) + lk, av[(j + AD) & AM]);
        finish_b(bx, by, bp, ce, withzero{});
        __builtin_amdgcn_sched_barrier(0);  // the raw B registers are free again
        load_b(min(4 * (ks + j + 1), klast), bx, by, bp, ce);
        __builtin_amdgcn_sched_barrier(0);  // loads issue before this step's MFMAs
        // the wave issuing its MFMAs goes first when both waves of the SIMD
        // are ready, so its matrix-core block is not split by the other
        // wave's loads and epilogue
        __builtin_amdgcn_s_setprio(1);
        mma(av[j & AM], true);
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int st = KS4; st < KSC; ++st) {
      if (st + AD < KSC) load_a(4 * (st + AD) + lk, av[(st + AD) & AM]);
      finish_b(bx, by, bp, ce, withzero{});
      __builtin_amdgcn_sched_barrier(0);
      if (st + 1 < KSC) load_b(4 * (st + 1), bx, by, bp, ce);
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_setprio(1);
      mma(av[st & AM], st < KSS);
      __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_sched_barrier(0);
    }
    // each pair owns a staging slot (slots are ordered by target) holding its
    // result in the reflected frame (xz_stage_pos: the pm block, whose
    // 16-byte pairs hold an S-list row's L^{+m'} and L^{-m'}, then the C-only
    // rows); the reduction kernel below maps it back and adds a target's
    // slots in a fixed order.  Lane (j, q) holds rows 4q..4q+3 of every
    // 16-row tile of column j; the results pass through LDS ([column][tile])
    // so that every store instruction writes whole 128-byte lines.
    __shared__ f4v sout[16 * NCT * 17];  // [col][pieces], a column's row padded by one piece (LDS banks)
    // slot of each column (-1 past the chunk's end) and the sign of its S
    // block: -1 when its reflection flips the sign of m (m2l_xz_codes)
    int slots[NCT];
    float ssgn[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      const bool ok = 16 * t + li < np;
      const int4 pr = ld_int4(I.m2l_pairs + pb + (ok ? 16 * t + li : 0));
      slots[t] = ok ? pr.w : -1;
      ssgn[t] = (__builtin_popcount(pr.z & 11) & 1) ? -1.f : 1.f;
    }
    // store NP 16-byte pieces per column from LDS ([col][NP + 1]) to position
    // dst (main array) or, if tail, to position dst - SM of the tail array,
    // pieces past `valid` skipped
    auto store_lds = [&](auto np_tag, int dst, bool tail, int valid) {
      constexpr int NP = decltype(np_tag)::value;
#pragma unroll
      for (int u = 0; u < NP * NCT / 4; ++u) {  // 16 NCT columns x NP pieces over 64 lanes
        const int e = 64 * u + lane, col = e / NP, piece = e % NP;
        int slot = -1;
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
          const int sv = __shfl(slots[t], col & 15);
          if ((col >> 4) == t) slot = sv;
        }
        if (slot < 0 || piece >= valid) continue;
        gfloat4* St = tail ? (gfloat4*)(I.stage_tail + (size_t)slot * ST + (dst - SM))
                           : (gfloat4*)(I.stage + (size_t)slot * SM + dst);
        __builtin_nontemporal_store(sout[col * (NP + 1) + piece], &St[piece]);  // written once, read once
      }
    };
    auto lds_sync2 = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // the pm tiles: row e of tile r gives the piece (L^{+m'}, L^{-m'})
#pragma unroll
    for (int r = 0; r < RTS; ++r) {
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float Ar = k1[t][r][v] - k3[t][r][v], Ai = k1[t][r][v] + k2[t][r][v];
          const int rs = RTC + r;
          const float Br = ssgn[t] * (k1[t][rs][v] - k3[t][rs][v]), Bi = ssgn[t] * (k1[t][rs][v] + k2[t][rs][v]);
          const int e = 16 * r + 4 * lk + v;
          const bool srow = e < X.S;
          const float2 p = srow ? sph[mrow[e]] : make_float2(1.f, 0.f);
          const float sr = Ar + Br, si = Ai + Bi, dr = Ar - Br, di = Ai - Bi;
          // plus: conj(p) (A + B) (A alone past the S-list); minus: p (A - B)
          sout[(16 * t + li) * 17 + 4 * lk + v] =
              f4v{srow ? fmaf(p.x, sr, p.y * si) : Ar, srow ? fmaf(p.x, si, -p.y * sr) : Ai,
                  fmaf(p.x, dr, -p.y * di), fmaf(p.x, di, p.y * dr)};
        }
      }
      lds_sync2();
      store_lds(std::integral_constant<int, 16>{}, 32 * r, false, 16);
      lds_sync2();
    }
    // the C-only tiles: rows of L^{n'0}
#pragma unroll
    for (int r = RTS; r < RTC; ++r) {
#pragma unroll
      for (int t = 0; t < NCT; ++t) {
        float o[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          o[2 * v] = k1[t][r][v] - k3[t][r][v];
          o[2 * v + 1] = k1[t][r][v] + k2[t][r][v];
        }
        const int col = 16 * t + li;
        sout[col * 9 + 2 * lk] = f4v{o[0], o[1], o[2], o[3]};      // rows 4 lk, 4 lk + 1
        sout[col * 9 + 2 * lk + 1] = f4v{o[4], o[5], o[6], o[7]};  // rows 4 lk + 2, 4 lk + 3
      }
      lds_sync2();
      const int first = 16 * (r - RTS), rows = xz_co_rows(P) - first < 16 ? xz_co_rows(P) - first : 16;
      const int dst = xz_stage_pos(P, 16 * r, 1);
      store_lds(std::integral_constant<int, 8>{}, rows == 16 ? dst : SM, rows != 16, (rows + 1) / 2);
      lds_sync2();
    }
  }
}

// ---------------------------------------------------------------------------
// M2M (children -> parent) and L2L (parent -> child) on the matrix cores.
// One wave owns up to 16 destination cells of one instance and level, so
// it writes them directly (no staging, no atomics).  Items: (instance, op,
// first column entry, count).  M2M (MODE 0): a column entry is (parent,
// child of octant 0..7 or -1); op is the level's octant-0 operator and the
// wave runs the 8 octant operators in order, M[parent] = sum_o T_o M[child_o].
// L2L (MODE 1): an entry is (child, parent), all of one octant operator op;
// L[child] += T_op L[parent].  Same tiles and Gauss product as M2L.
// ---------------------------------------------------------------------------
// One row tile per workgroup: workgroup (item, b) computes output tile b,
// so the short operator chains of the coarse levels run on many waves at
// once.  M2M up to P = 11 splits the eight octants over two waves
// (octants 0-3 and 4-7), halving the chain of dependent MFMAs; the second
// wave's sums are added to the first's through LDS, in that fixed order.
// Each operator's A and B loads are issued in groups of 16 k-steps with all
// loads of a group in flight, so a wave waits about once per group instead
// of once per k-step.
constexpr int tr_waves(int RT, int MODE) { return MODE == 0 && RT <= 8 ? 2 : 1; }

template <int RT, int KS, int MODE>
__global__ void __launch_bounds__(64 * tr_waves(RT, MODE))
    __attribute__((amdgpu_waves_per_eu(RT >= 8 ? 1 : 2)))
k_tr_mfma(const int4* __restrict__ items, const int32_t* __restrict__ cols,
          const InstDev* __restrict__ insts, int tstride, int Rp, int P2) {
  constexpr int STRIDE = MODE == 0 ? 9 : 2;
  constexpr int G = KS < 16 ? KS : 16;
  constexpr bool SPLIT = tr_waves(RT, MODE) == 2;
  const int r0 = blockIdx.x % RT;
  const int4 it = items[blockIdx.x / RT];
  const InstDev& I = insts[it.x];
  const int lane = threadIdx.x & 63;
  const int half = SPLIT ? (int)(threadIdx.x >> 6) : 0;  // octants 4 half .. 4 half + 3
  const int li = lane & 15, lk = lane >> 4;
  const bool ok = li < it.w;
  const int32_t* cj = cols + (size_t)(it.z + (ok ? li : 0)) * STRIDE;
  const int dst = cj[0];
  float2* X = MODE == 0 ? I.M : I.L;
  floatx4 k1 = {0.f, 0.f, 0.f, 0.f}, k2 = k1, k3 = k1;
  // Rounds q = 0..R-1: operator o = q / NG of this item (M2M: the children
  // of octant o = 0..7 in order, a column without that child reading zeros;
  // L2L: its one operator) and group q % NG of G k-steps.  The next round's
  // table and operand loads are issued before the current round's MFMAs, so
  // a round's load latency hides under the previous one's matrix-core work;
  // the accumulation order is that of running the rounds one after another.
  // The rounds are unrolled (straight-line code keeps the wait counts exact).
  constexpr int NO = MODE == 0 ? (SPLIT ? 4 : 8) : 1, NG = (KS + G - 1) / G, R = NO * NG;
  const int obase = SPLIT ? 4 * half : 0;  // first octant of this wave
  constexpr int NB = RT <= 8 ? 2 : 1;  // operand buffers
  float2 a[NB][G], bv[NB][G];
  int srcb[NB];
  // the source cells of every operator, read before any operand load (a
  // source index read between rounds would make each round wait for the
  // previous round's loads: the load counter retires in order)
  int srcs[RT <= 8 ? NO : 1];
  if constexpr (RT <= 8) {
#pragma unroll
    for (int o = 0; o < NO; ++o) srcs[o] = ok ? cj[1 + (MODE == 0 ? obase + o : 0)] : -1;
  }
  auto load = [&](int q, int buf) {
    const int o = q / NG, g0 = (q % NG) * G;
    int src;
    if constexpr (RT <= 8)
      src = srcs[o];
    else
      src = ok ? cj[1 + (MODE == 0 ? obase + o : 0)] : -1;
    srcb[buf] = src;
    gcfloat2* T =
        (gcfloat2*)(I.tables + (size_t)(it.y + (MODE == 0 ? obase + o : 0)) * tstride) + li + 16 * r0;
    gcfloat2* B = (gcfloat2*)(X + (size_t)(src < 0 ? 0 : src) * P2);
#pragma unroll
    for (int u = 0; u < G; ++u) {  // steps past KS repeat the last one (unused)
      const int k = 4 * min(g0 + u, KS - 1) + lk;
      a[buf][u] = ld2(T + (size_t)k * Rp);
      bv[buf][u] = ld2(B + min(k, P2 - 1));
    }
  };
  auto compute = [&](int q, int buf) {
    const int g0 = (q % NG) * G;
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (g0 + u < KS) {
        const int k = 4 * (g0 + u) + lk;
        const bool z = srcb[buf] < 0 || k >= P2;
        const float x = z ? 0.f : bv[buf][u].x, y = z ? 0.f : bv[buf][u].y;
        const float ar = a[buf][u].x, ai = a[buf][u].y;
        k1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar + ai, x, k1, 0, 0, 0);
        k2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, y - x, k2, 0, 0, 0);
        k3 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, x + y, k3, 0, 0, 0);
      }
    }
  };
  if constexpr (RT <= 8) {
    load(0, 0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (q + 1 < R) load(q + 1, (q + 1) & 1);
      __builtin_amdgcn_sched_barrier(0);  // the next round's loads go out first
      compute(q, q & 1);
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    // larger orders (P >= 12): the unrolled rounds no longer fit the
    // registers; each round's loads, then its MFMAs
    for (int q = 0; q < R; ++q) {
      load(q, 0);
      __builtin_amdgcn_sched_barrier(0);
      compute(q, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if constexpr (SPLIT) {  // sums of octants 0-3 + sums of octants 4-7
    __shared__ floatx4 part[3][64];
    if (half == 1) {
      part[0][lane] = k1;
      part[1][lane] = k2;
      part[2][lane] = k3;
    }
    __syncthreads();
    if (half == 1) return;
    k1 += part[0][lane];
    k2 += part[1][lane];
    k3 += part[2][lane];
  }
  if (!ok) return;
  float2* D = X + (size_t)dst * P2;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 16 * r0 + 4 * lk + v;
    if (row < P2) {
      float2 val = make_float2(k1[v] - k3[v], k1[v] + k2[v]);
      if (MODE == 1) {
        const float2 old = D[row];
        val.x += old.x;
        val.y += old.y;
      }
      D[row] = val;
    }
  }
}

// L[t] = sum of t's staging slots in slot order (deterministic), each slot's
// result mapped back by the output codes of its pair's reflection.  Items:
// (instance, target cell); the cell's slots are [soff[t], soff[t+1]).  A
// reflection sends the staging positions of (n', m') and (n', -m') onto the
// same two coefficients (straight or exchanged), and those positions are one
// aligned 16-byte pair (xz_stage_pos): thread j < S owns both coefficients of
// S-list entry j and reads the pair with one load, thread S + n' owns
// (n', 0).  C threads, one wave per target up to P = 10.  The slots'
// reflections are staged in LDS per group of kRedGroup slots, and the loads
// of U slots are in flight per thread.
constexpr int kRedGroup = 512;

template <int P>
__global__ void __launch_bounds__(64 * ((xz_dims(P).C + 63) / 64))
k_m2l_reduce(const int2* __restrict__ items, const InstDev* __restrict__ insts, const int32_t* __restrict__ omap,
             int64_t slot_base) {
  constexpr XzDims X = xz_dims(P);
  constexpr int P2 = P * P, SM = xz_stage_sm(P), ST = xz_stage_st(P);
  extern __shared__ int red_lds[];
  int* som = red_lds;              // [16][P2] output codes
  int* sgo = red_lds + 16 * P2;    // [kRedGroup] reflection * P2 of each slot of the group
  const int tid = threadIdx.x, nth = blockDim.x;
  {  // all loads of the code table in flight before the LDS writes (clamped indices)
    const int4* src = reinterpret_cast<const int4*>(omap);
    int4* dst = reinterpret_cast<int4*>(som);
    constexpr int n4 = 4 * P2;
    constexpr int U = 4;
    for (int base = 0; base < n4; base += nth * U) {
      int4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = src[min(base + tid + nth * u, n4 - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) dst[min(base + tid + nth * u, n4 - 1)] = v[u];
    }
  }
  const int2 it = items[blockIdx.x];
  const InstDev& I = insts[it.x];
  const int cell = it.y;
  const int s0 = I.m2l_soff[cell], s1 = I.m2l_soff[cell + 1];
  // this thread's coefficients: c0 = (n', m'), c1 = (n', -m') (none for m' = 0)
  int c0 = -1, c1 = -1;
  if (tid < X.C) {
    int n, m;
    xz_entry(P, tid, &n, &m);
    c0 = n * n + n + m;
    if (m > 0) c1 = n * n + n - m;
  }
  const bool two = c1 >= 0;
  const int c1r = two ? c1 : max(c0, 0);
  float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
  for (int g0 = s0; g0 < s1; g0 += kRedGroup) {
    const int ng = min(kRedGroup, s1 - g0);
    __syncthreads();
    for (int e = tid; e < ng; e += nth) sgo[e] = (int)I.slot_g[g0 + e] * P2;
    __syncthreads();
    if (c0 >= 0) {
      // position r of a slot: main array for r < SM, else the tail
      gcfloat2* S = (gcfloat2*)(I.stage + (size_t)(g0 - slot_base) * SM);
      gcfloat2* T = (gcfloat2*)(I.stage_tail + (size_t)(g0 - slot_base) * ST) - SM;
      auto at = [&](int u, int r) { return r < SM ? S + (size_t)u * SM + r : T + (size_t)u * ST + r; };
      // the aligned 16-byte pair holding position e (main and tail arrays
      // both have an even count of positions per slot); c0 takes its half e
      // & 1, c1 (if any) the other
      auto pair_at = [&](int u, int e) {
        return __builtin_nontemporal_load((const __attribute__((address_space(1))) f4v*)at(u, (e & 0xffff) & ~1));
      };
      auto add = [&](const f4v& w, int e, int f) {
        const bool sw = e & 1;
        const float2 x = apply_code(sw ? w.z : w.x, sw ? w.w : w.y, e);
        const float2 y = apply_code(sw ? w.x : w.z, sw ? w.y : w.w, f);
        ar += x.x;
        ai += x.y;
        br += y.x;  // unused by the (n', 0) threads
        bi += y.y;
      };
      int q = 0;
      constexpr int U = 12;  // slots in flight per thread, added in slot order
      for (; q + U <= ng; q += U, S += U * SM, T += U * ST) {
        int e[U], f[U];
        f4v w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          e[u] = som[sgo[q + u] + c0];
          f[u] = som[sgo[q + u] + c1r];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) w[u] = pair_at(u, e[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) add(w[u], e[u], f[u]);
      }
      for (; q < ng; ++q, S += SM, T += ST) {
        const int e = som[sgo[q] + c0], f = som[sgo[q] + c1r];
        add(pair_at(0, e), e, f);
      }
    }
  }
  if (c0 >= 0) I.L[(size_t)cell * P2 + c0] = make_float2(ar, ai);
  if (two) I.L[(size_t)cell * P2 + c1] = make_float2(br, bi);
}

// ---------------------------------------------------------------------------
// L2P: one wave per leaf, one target per lane;
// phi(x) = ik sum_n b_n(k r) sum_m Lt_n^m Y_n^m(dir), accumulated per degree
// while the harmonics are generated.  Writes (not accumulates) the sorted
// output.
// ---------------------------------------------------------------------------
template <int P, bool DAMP>
__global__ void __launch_bounds__(64) k_l2p(const int2* __restrict__ items, const InstDev* __restrict__ insts) {
  constexpr int P2 = P * P;
  const int2 it = items[blockIdx.x];
  const InstDev& I = insts[it.x];
  const int cell = it.y;
  const int4 rg = I.cells[cell];
  const float4 g = I.geo[cell];
  const double rh = I.rho[I.clev[cell]];
  const float k = I.k;
  __shared__ float2 sl[P2];
  for (int e = threadIdx.x; e < P2; e += blockDim.x) sl[e] = I.L[(size_t)cell * P2 + e];
  __syncthreads();
  for (int i = rg.z + threadIdx.x; i < rg.w; i += 64) {
    const float4 p = I.tpos[i];
    const float dx = p.x - g.x, dy = p.y - g.y, dz = p.z - g.z;
    const float r = sqrtf(dx * dx + dy * dy + dz * dz);
    float b[DAMP ? 1 : P];
    float2 bc[DAMP ? P : 1];
    if constexpr (DAMP)
      radial_scaled_c<P>((double)k * (double)r, (double)I.ki * (double)r, rh, bc);
    else
      radial_scaled<P>((double)k * (double)r, rh, b);
    float2 u[P];
#pragma unroll
    for (int n = 0; n < P; ++n) u[n] = make_float2(0.f, 0.f);
    ylm_visit<P>(dx, dy, dz, r, [&](int n, int m, float2 y) {
      if (m == 0) {
        u[n] = cfma(sl[n * n + n], y, u[n]);
      } else {
        u[n] = cfma(sl[n * n + n + m], y, u[n]);
        u[n] = cfma(sl[n * n + n - m], cconj(y), u[n]);
      }
    });
    float2 s = make_float2(0.f, 0.f);
    if constexpr (DAMP) {
#pragma unroll
      for (int n = 0; n < P; ++n) s = cfma(bc[n], u[n], s);
      // times i (k + i ki) = -ki + i k, added to the near field
      float2 o = I.ys[i];
      o.x = fmaf(-I.ki, s.x, fmaf(-k, s.y, o.x));
      o.y = fmaf(-I.ki, s.y, fmaf(k, s.x, o.y));
      I.ys[i] = o;
    } else {
#pragma unroll
      for (int n = 0; n < P; ++n) {
        s.x = fmaf(b[n], u[n].x, s.x);
        s.y = fmaf(b[n], u[n].y, s.y);
      }
      float2 o = I.ys[i];  // times i k, added to the near field
      o.x = fmaf(-k, s.y, o.x);
      o.y = fmaf(k, s.x, o.y);
      I.ys[i] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// P2P (Listing 1 without the near branch): y_i += sum_j q_j e^{ikR}/(4 pi R),
// R > 0.  One wave per target leaf, its targets taken in blocks of up to 64.
// Each lane owns T targets of a block (T = 1..4, chosen per block so that
// the most lanes are busy) and a residue class of sources (lane = target
// group + ngroup * split).  The source stream of the leaf (its merged source
// intervals) is cut into tiles of L <= 64 sources, L a multiple of the
// number of splits, so every busy lane runs the same number of iterations;
// each tile is staged through LDS while the next one is already being
// loaded into registers.  Coordinates stay unscaled so that the difference
// of two nearby FP32 points is exact; the phase in revolutions is R k/(2 pi).
// Deterministic: each target is owned by one wave and the split partial sums
// are added in a fixed order.
// ---------------------------------------------------------------------------
__device__ inline void p2p_fetch(const int2* __restrict__ ivals, int iv, int ie, int off, int lane,
                                 const float4* __restrict__ spos, const float2* __restrict__ q,
                                 float4& p, float2& w) {
  int pos = off + lane, v = iv;
  while (v < ie) {
    int2 r = ivals[v];
    int len = r.y - r.x;
    if (pos < len) {
      p = spos[r.x + pos];
      w = q[r.x + pos];
      return;
    }
    pos -= len;
    ++v;
  }
  p = make_float4(0.f, 0.f, 0.f, 0.f);
  w = make_float2(0.f, 0.f);
}

// Targets per lane for a block of tc targets: the T in 1..4 with the most
// busy lane slots, tc nsplit / (64 T) with nsplit = floor(64 / ceil(tc / T))
// (ties: the larger T, whose source loads serve more targets).
__device__ inline int p2p_targets_per_lane(int tc) {
  int best = 1;
  int bnum = -1, bden = 1;
  for (int T = 1; T <= 4; ++T) {
    const int ng = (tc + T - 1) / T;
    const int num = tc * (64 / ng), den = 64 * T;
    if (num * bden >= bnum * den) {
      bnum = num;
      bden = den;
      best = T;
    }
  }
  return best;
}

// One pair: a += q G(x, y) up to the 1/(4 pi) applied at the end.
template <bool DAMP>
__device__ inline void p2p_pair(float xx, float xy, float xz, float4 yj, float2 qj, float krev, float kdec,
                                float& ar, float& ai) {
  float dx = xx - yj.x, dy = xy - yj.y, dz = xz - yj.z;
  float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  float rinv = (r2 > 0.f) ? __builtin_amdgcn_rsqf(r2) : 0.f;
  float rev = r2 * rinv * krev;
  float sn = __builtin_amdgcn_sinf(rev), cs = __builtin_amdgcn_cosf(rev);
  if constexpr (DAMP) rinv *= __builtin_amdgcn_exp2f(r2 * rinv * kdec);
  float gr = cs * rinv, gi = sn * rinv;
  ar = fmaf(qj.x, gr, fmaf(-qj.y, gi, ar));
  ai = fmaf(qj.x, gi, fmaf(qj.y, gr, ai));
}

// Targets [t0, t0 + tc) of the leaf against all its sources, T per lane.
// A tile holds TS stages of L sources (lane l < L loads source u L + l of
// stage u); since L is a multiple of the split count, split s still takes
// the sources whose index is s modulo the split count, in increasing order,
// so every TS gives the same sums bit for bit.
template <int T, int TS, bool DAMP>
__device__ inline void p2p_block(const InstDev& I, int4 wk, int total, int t0, int tc, int lane,
                                 float4 (*sp)[64 * TS], float2 (*sq)[64 * TS], float2* red, float krev, float kdec) {
  const int ng = (tc + T - 1) / T;            // target groups
  const int nsplit = 64 / ng;
  const int L = nsplit * (64 / nsplit);       // sources per stage
  const int LT = TS * L;                      // sources per tile
  const int g = lane % ng, s = lane / ng;
  const bool active = s < nsplit;
  float xx[T], xy[T], xz[T], ar[T], ai[T];
#pragma unroll
  for (int i = 0; i < T; ++i) {
    const float4 p = I.tpos[min(t0 + T * g + i, t0 + tc - 1)];
    xx[i] = p.x;
    xy[i] = p.y;
    xz[i] = p.z;
    ar[i] = 0.f;
    ai[i] = 0.f;
  }
  const int2* __restrict__ ivals = I.p2p_ivals;
  int iv = wk.z, off = 0;
  float4 np4[TS];
  float2 nq[TS];
#pragma unroll
  for (int u = 0; u < TS; ++u) {
    np4[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    nq[u] = make_float2(0.f, 0.f);
    if (lane < L) p2p_fetch(ivals, iv, wk.w, off + u * L, lane, I.spos, I.q, np4[u], nq[u]);
  }
  int tile = 0;
  for (int base = 0; base < total; base += LT, ++tile) {
    const int nj = min(LT, total - base);
    const int buf = tile & 1;
    if (lane < L) {
#pragma unroll
      for (int u = 0; u < TS; ++u) {
        sp[buf][u * L + lane] = np4[u];
        sq[buf][u * L + lane] = nq[u];
      }
    }
    off += LT;
    while (iv < wk.w && off >= ivals[iv].y - ivals[iv].x) {
      off -= ivals[iv].y - ivals[iv].x;
      ++iv;
    }
    if (base + LT < total && lane < L) {
#pragma unroll
      for (int u = 0; u < TS; ++u) p2p_fetch(ivals, iv, wk.w, off + u * L, lane, I.spos, I.q, np4[u], nq[u]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (active) {
      const float4* P = sp[buf];
      const float2* Q = sq[buf];
      for (int j = s; j < nj; j += nsplit) {
        const float4 yj = P[j];
        const float2 qj = Q[j];
#pragma unroll
        for (int i = 0; i < T; ++i) p2p_pair<DAMP>(xx[i], xy[i], xz[i], yj, qj, krev, kdec, ar[i], ai[i]);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // target T g + i of this block sums red[(g + ss ng) T + i] over the splits
#pragma unroll
  for (int i = 0; i < T; ++i) red[lane * T + i] = make_float2(ar[i], ai[i]);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane < tc) {
    const int gg = lane / T, ii = lane - T * gg;
    float sr = 0.f, si = 0.f;
    for (int ss = 0; ss < nsplit; ++ss) {
      const float2 v = red[(gg + ss * ng) * T + ii];
      sr += v.x;
      si += v.y;
    }
    const float scale = 0.07957747154594767f;  // 1 / (4 pi)
    float2 o = I.ys[t0 + lane];
    o.x = fmaf(sr, scale, o.x);
    o.y = fmaf(si, scale, o.y);
    I.ys[t0 + lane] = o;
  }
  __builtin_amdgcn_wave_barrier();
}

// DAMP: complex wavenumber k + i ki, G times the decay e^{-ki R} (the
// imaginary wavenumber of the listing's exponential).  W waves per block,
// one leaf block per wave; TS source stages per tile (p2p_block).
template <bool DAMP, int W, int TS>
__global__ void __launch_bounds__(64 * W) k_p2p(const int2* __restrict__ items, int nitems,
                                                const InstDev* __restrict__ insts) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w = blockIdx.x * W + wave;
  __shared__ float4 sp[W][2][64 * TS];
  __shared__ float2 sq[W][2][64 * TS];
  __shared__ float2 red[W][64 * 4];
  if (w >= nitems) return;
  const int2 it = items[w];
  const InstDev& I = insts[it.x];
  const int4 wk = I.p2p_work[it.y];
  const int total = I.p2p_total[it.y];
  const float krev = I.k * 0.15915494309189535f;  // k / (2 pi)
  const float kdec = -I.ki * 1.4426950408889634f;  // -ki log2(e): decay 2^(kdec R)
  for (int t0 = wk.x; t0 < wk.y; t0 += 64) {
    const int tc = min(64, wk.y - t0);
    switch (p2p_targets_per_lane(tc)) {
      case 1: p2p_block<1, TS, DAMP>(I, wk, total, t0, tc, lane, sp[wave], sq[wave], red[wave], krev, kdec); break;
      case 2: p2p_block<2, TS, DAMP>(I, wk, total, t0, tc, lane, sp[wave], sq[wave], red[wave], krev, kdec); break;
      case 3: p2p_block<3, TS, DAMP>(I, wk, total, t0, tc, lane, sp[wave], sq[wave], red[wave], krev, kdec); break;
      default: p2p_block<4, TS, DAMP>(I, wk, total, t0, tc, lane, sp[wave], sq[wave], red[wave], krev, kdec); break;
    }
  }
}

// Per-call caller vectors of each instance.
__global__ void k_set_xy(int count, int base, XYPtrs p, InstDev* __restrict__ insts) {
  const int i = threadIdx.x;
  if (i < count) {
    insts[base + i].x = p.x[i];
    insts[base + i].y = p.y[i];
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
void table_dims(int P, int* Kp, int* Rp) {
  *Kp = 4 * ((P * P + 3) / 4);
  *Rp = 16 * ((P * P + 15) / 16);
}
void stage_dims(int P, int* Sm, int* St) {
  *Sm = xz_stage_sm(P);
  *St = xz_stage_st(P);
}
void launch_gen_tables(const OpDescDev* ops, int nops, int P, double k, double ki, const int32_t* cp_off,
                       const int32_t* cp_lm, const double2* cp_val, float2* tables,
                       hipStream_t s) {
  if (nops <= 0) return;
  int Kp, Rp;
  table_dims(P, &Kp, &Rp);
  k_gen_tables<float2, true><<<nops, 256, 0, s>>>(ops, nops, P, k, ki, cp_off, cp_lm, cp_val, Kp, Rp,
                                                   xz_table_stride(P), tables);
}
void launch_gen_tables64(const OpDescDev* ops, int nops, int P, double k, const int32_t* cp_off,
                         const int32_t* cp_lm, const double2* cp_val, double2* tables, hipStream_t s) {
  if (nops <= 0) return;
  int Kp, Rp;
  table_dims(P, &Kp, &Rp);
  k_gen_tables<double2, false><<<nops, 256, 0, s>>>(ops, nops, P, k, 0.0, cp_off, cp_lm, cp_val, Kp, Rp, Kp * Rp,
                                                    tables);
}
int elem_chunk() { return kChunk; }
void launch_set_xy(int count, int base, const XYPtrs& p, InstDev* insts, hipStream_t s) {
  k_set_xy<<<1, 64, 0, s>>>(count, base, p, insts);
}
void launch_zero(const int2* items, int n, const InstDev* insts, hipStream_t s) {
  if (n > 0) k_zero<<<n, 256, 0, s>>>(items, n, insts);
}
void launch_gather(const int2* items, int n, const InstDev* insts, hipStream_t s) {
  if (n > 0) k_gather<<<n, 256, 0, s>>>(items, insts);
}
void launch_scatter(const int2* items, int n, const InstDev* insts, hipStream_t s) {
  if (n > 0) k_scatter<<<n, 256, 0, s>>>(items, insts);
}
#define HFMM_P_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
void launch_p2m(const int2* items, int n, const InstDev* insts, int P, bool damped, hipStream_t s) {
  if (n <= 0) return;
  switch (P) {
#define X(p)                                                           \
  case p:                                                              \
    if (damped)                                                        \
      k_p2m<p, true><<<n, 64, 0, s>>>(items, insts);                   \
    else                                                               \
      k_p2m<p, false><<<n, 64, 0, s>>>(items, insts);                  \
    break;
    HFMM_P_CASES(X)
#undef X
    default: break;
  }
}
template <int MODE>
static void launch_tr(const int4* items, int n, const int32_t* cols, const InstDev* insts, int P, hipStream_t s) {
  if (n <= 0) return;
  int Kp, Rp;
  table_dims(P, &Kp, &Rp);
  switch (P) {
#define X(p)                                                                                      \
  case p: {                                                                                       \
    constexpr int RT = (p * p + 15) / 16, KS = (p * p + 3) / 4;                                   \
    k_tr_mfma<RT, KS, MODE><<<n * RT, 64 * tr_waves(RT, MODE), 0, s>>>(items, cols, insts,               \
                                                                              xz_table_stride(p), Rp, p * p); \
    break;                                                                                        \
  }
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
    default: break;
  }
}
void launch_m2m(const int4* items, int n, const int32_t* cols, const InstDev* insts, int P, hipStream_t s) {
  launch_tr<0>(items, n, cols, insts, P, s);
}
void launch_l2l(const int4* items, int n, const int32_t* cols, const InstDev* insts, int P, hipStream_t s) {
  launch_tr<1>(items, n, cols, insts, P, s);
}
void launch_l2p(const int2* items, int n, const InstDev* insts, int P, bool damped, hipStream_t s) {
  if (n <= 0) return;
  switch (P) {
#define X(p)                                                           \
  case p:                                                              \
    if (damped)                                                        \
      k_l2p<p, true><<<n, 64, 0, s>>>(items, insts);                   \
    else                                                               \
      k_l2p<p, false><<<n, 64, 0, s>>>(items, insts);                  \
    break;
    HFMM_P_CASES(X)
#undef X
    default: break;
  }
}
void launch_m2l_reduce(const int2* items, int n, const InstDev* insts, const int32_t* omap, int P,
                       int64_t slot_base, hipStream_t s) {
  if (n <= 0) return;
  const size_t lds = (16 * (size_t)P * P + kRedGroup) * sizeof(int);
  switch (P) {
#define X(p)                                                                                    \
  case p:                                                                                       \
    k_m2l_reduce<p><<<n, 64 * ((xz_dims(p).C + 63) / 64), lds, s>>>(items, insts, omap, slot_base); \
    break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
    default: break;
  }
}
// P2P launch shapes (all give the same bits): waves per block and source
// stages per tile.
//   0: 4 waves, 1 stage;  1: 1 wave, 1 stage;  2: 4 waves, 2 stages;
//   3: 1 wave, 2 stages.
int p2p_variant_count() { return 4; }

template <bool DAMP, int W, int TS>
static void launch_p2p_t(const int2* items, int n, const InstDev* insts, hipStream_t s) {
  k_p2p<DAMP, W, TS><<<(n + W - 1) / W, 64 * W, 0, s>>>(items, n, insts);
}

template <bool DAMP>
static void launch_p2p_d(const int2* items, int n, const InstDev* insts, int variant, hipStream_t s) {
  switch (variant) {
    case 1: return launch_p2p_t<DAMP, 1, 1>(items, n, insts, s);
    case 2: return launch_p2p_t<DAMP, 4, 2>(items, n, insts, s);
    case 3: return launch_p2p_t<DAMP, 1, 2>(items, n, insts, s);
    default: return launch_p2p_t<DAMP, 4, 1>(items, n, insts, s);
  }
}

void launch_p2p(const int2* items, int n, const InstDev* insts, bool damped, int variant, hipStream_t s) {
  if (n <= 0) return;
  if (damped)
    launch_p2p_d<true>(items, n, insts, variant, s);
  else
    launch_p2p_d<false>(items, n, insts, variant, s);
}

template <int P, int NCT, int WPE, int CPW, int AD>
static void launch_m2l_t(const int4* chunks, int nchunks, int sub, const InstDev* insts, const int32_t* bmap,
                         hipStream_t s) {
  constexpr XzDims X = xz_dims(P);
  const int nitems = nchunks * sub;
  const int nwaves = (nitems + CPW - 1) / CPW;
  const int per = (nwaves + 7) / 8;
  const size_t lds = (17 * (size_t)xz_code_stride(P) + 16 * (size_t)X.RTS) * sizeof(int);
  k_m2l_mfma<P, NCT, WPE, CPW, AD><<<8 * per, 64, lds, s>>>(chunks, nitems, per, sub, insts, bmap);
}

// Chunks hold 32 pairs while two 16-pair column tiles of three accumulator
// sets fit two waves per SIMD (RTC + RTS <= 7, P <= 10), else 16.
int m2l_pairs_per_chunk(int P) { return xz_dims(P).RT <= 7 ? 32 : 16; }

// Launch shapes (all give the same bits).  With 32-pair chunks:
//   0: one wave per chunk (two column tiles), tables one k-step ahead;
//   1: one wave per 16-pair column tile (smaller register budget, more
//      waves per SIMD), tables one step ahead;
//   2, 3: shapes 0 and 1 with the tables two k-steps ahead.
// (Waves running several chunks each spill registers in the two-tile
// shape.)  With 16-pair chunks: one wave per chunk running 1, 2 or 4
// chunks.
int m2l_variant_count(int P) { return m2l_pairs_per_chunk(P) == 32 ? 4 : 3; }

// waves per SIMD of the one-tile shape: accumulators and A buffers take
// about 16 RT registers
constexpr int m2l_narrow_wpe(int RT) { return RT <= 3 ? 4 : RT <= 7 ? 3 : RT <= 12 ? 2 : 1; }

template <int P>
static void launch_m2l_p(int variant, int sub, const int4* chunks, int nchunks, const InstDev* insts,
                         const int32_t* bmap, hipStream_t s) {
  constexpr int RT = xz_dims(P).RT, NW = m2l_narrow_wpe(RT);
  if constexpr (RT <= 7) {
    if (sub == 2) {
      switch (variant) {
        case 1: return launch_m2l_t<P, 1, NW, 1, 1>(chunks, nchunks, 2, insts, bmap, s);
        case 2: return launch_m2l_t<P, 2, 2, 1, 2>(chunks, nchunks, 1, insts, bmap, s);
        case 3: return launch_m2l_t<P, 1, NW, 1, 2>(chunks, nchunks, 2, insts, bmap, s);
        default: return launch_m2l_t<P, 2, 2, 1, 1>(chunks, nchunks, 1, insts, bmap, s);
      }
    }
  }
  switch (variant) {
    case 1: return launch_m2l_t<P, 1, NW, 2, 1>(chunks, nchunks, sub, insts, bmap, s);
    case 2: return launch_m2l_t<P, 1, NW, 4, 1>(chunks, nchunks, sub, insts, bmap, s);
    default: return launch_m2l_t<P, 1, NW, 1, 1>(chunks, nchunks, sub, insts, bmap, s);
  }
}

void launch_m2l(const int4* chunks, int nchunks, const InstDev* insts, const int32_t* bmap, int P, int variant,
                hipStream_t s) {
  if (nchunks <= 0) return;
  const int sub = m2l_pairs_per_chunk(P) / 16;
  switch (P) {
#define X(p) \
  case p: launch_m2l_p<p>(variant, sub, chunks, nchunks, insts, bmap, s); break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
    default: break;
  }
}

}  // namespace hfmm
