// FP64 variant of the FMM product and an FP64 direct sum.
//
// The variant runs the same tree, interaction lists, translation operators
// (generated in FP64) and expansion order as the FP32 path, with every step
// in double precision, so the difference between the two isolates the FP32
// rounding of the production path from the truncation error of the method
// (eq. 12-14 truncated at P).  It favours plain code over speed: one block
// per cell for the tree passes, one block per M2L chunk accumulating into
// the locals with FP64 atomic adds (no staging buffer, so it scales to large
// N; the summation order, and so the last bits, may vary between runs).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fmm64_kernels.h"

namespace hfmm {

__device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 zfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// i^ph (x + iy) for a reflection code (swap bit 16, sign of the real part
// bit 31, of the imaginary part bit 30)
__device__ inline double2 apply_code64(double2 v, int e) {
  const bool swap = e & (1 << 16);
  double x = swap ? v.y : v.x, y = swap ? v.x : v.y;
  if (e & (int)0x80000000) x = -x;
  if (e & (1 << 30)) y = -y;
  return make_double2(x, y);
}
// i^-ph for the same code: the inverse of a signed swap
__device__ inline double2 apply_code64_inv(double2 v, int e) {
  const bool swap = e & (1 << 16);
  double x = v.x, y = v.y;
  if (swap) {  // v = i^ph u with ph odd: u = (y', x') with the signs moved
    const double nx = (e & (1 << 30)) ? -y : y;
    const double ny = (e & (int)0x80000000) ? -x : x;
    return make_double2(nx, ny);
  }
  if (e & (int)0x80000000) x = -x;
  if (e & (1 << 30)) y = -y;
  return make_double2(x, y);
}

// Normalised Legendre recurrence coefficients (no Condon-Shortley phase),
// compile-time FP64.
constexpr double cx_sqrt64(double x) {
  if (x <= 0.0) return 0.0;
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 200; ++i) r = 0.5 * (r + x / r);
  return r;
}
struct YlmTab64 {
  double a[kMaxP][kMaxP], b[kMaxP][kMaxP], f[kMaxP], g[kMaxP];
};
constexpr YlmTab64 make_ylm_tab64() {
  YlmTab64 t{};
  for (int n = 0; n < kMaxP; ++n)
    for (int m = 0; m + 2 <= n; ++m) {
      t.a[n][m] = cx_sqrt64((4.0 * n * n - 1.0) / (double)(n * n - m * m));
      t.b[n][m] = cx_sqrt64((double)((n - 1) * (n - 1) - m * m) / (4.0 * (n - 1) * (n - 1) - 1.0));
    }
  for (int m = 0; m < kMaxP; ++m) {
    t.f[m] = m > 0 ? cx_sqrt64((2.0 * m + 1.0) / (2.0 * m)) : 0.0;
    t.g[m] = cx_sqrt64(2.0 * m + 3.0);
  }
  return t;
}
__constant__ YlmTab64 c_ylm64 = make_ylm_tab64();

// Visits Y_n^m (m >= 0) of direction d/r, m = 0..P-1, n = m..P-1.
template <int P, class F>
__device__ inline void ylm_visit64(double dx, double dy, double dz, double r, F&& f) {
  double c = 1.0, wx = 0.0, wy = 0.0;
  if (r > 0.0) {
    c = dz / r;
    wx = dx / r;
    wy = dy / r;
  }
  double2 pmm = make_double2(0.28209479177387814, 0.0);  // 1/sqrt(4 pi)
#pragma unroll
  for (int m = 0; m < P; ++m) {
    if (m > 0) {
      const double fm = c_ylm64.f[m];
      pmm = make_double2(fm * (pmm.x * wx - pmm.y * wy), fm * (pmm.x * wy + pmm.y * wx));
    }
    f(m, m, pmm);
    if (m + 1 < P) {
      const double gm = c_ylm64.g[m] * c;
      double2 p2 = pmm, p1 = make_double2(gm * pmm.x, gm * pmm.y);
      f(m + 1, m, p1);
#pragma unroll
      for (int n = m + 2; n < P; ++n) {
        const double an = c_ylm64.a[n][m], bn = c_ylm64.b[n][m];
        const double2 p = make_double2(an * (c * p1.x - bn * p2.x), an * (c * p1.y - bn * p2.y));
        f(n, m, p);
        p2 = p1;
        p1 = p;
      }
    }
  }
}

// b_n = j_n(x) (2n+1)!! / rho^n, n < P, FP64 (as the FP32 path's radial
// factor: two-term series for x < 1e-3, upward recurrence for x > P, else
// Miller's downward recurrence normalised by j_0 or j_1).
template <int P>
__device__ inline void radial_scaled64(double x, double rho, double* b) {
  if (x < 1e-3) {
    const double xr = x / rho, x2 = x * x;
    double p = 1.0;
#pragma unroll
    for (int n = 0; n < P; ++n) {
      b[n] = p * (1.0 - x2 / (4.0 * n + 6.0));
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
    const int N = P + 16 + (int)x;
    double fp1 = 0.0, f = 1e-30;
    for (int n = N; n > P; --n) {
      const double fm1 = (2.0 * n + 1.0) * ix * f - fp1;
      fp1 = f;
      f = fm1;
    }
#pragma unroll
    for (int n = P; n >= 1; --n) {
      const double fm1 = (2.0 * n + 1.0) * ix * f - fp1;
      fp1 = f;
      f = fm1;
      j[n - 1] = f;
    }
    const double scale = (fabs(j0) >= fabs(j1)) ? j0 / f : j1 / fp1;
#pragma unroll
    for (int n = 0; n < P; ++n) j[n] *= scale;
  }
  double df = 1.0, rp = 1.0;
#pragma unroll
  for (int n = 0; n < P; ++n) {
    df *= (2.0 * n + 1.0);
    b[n] = j[n] * df / rp;
    rp *= rho;
  }
}

__global__ void k64_gather(F64Dev D, const double2* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D.nsrc) D.q[i] = x[D.src_idx[i]];
}

__global__ void k64_zero(F64Dev D) {
  const int64_t n = (int64_t)D.ncell * D.P * D.P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    D.M[e] = make_double2(0.0, 0.0);
    D.L[e] = make_double2(0.0, 0.0);
  }
}

// P2M: one block (64 threads) per leaf, 16 or 32 bodies per pass through LDS.
template <int P>
__global__ void __launch_bounds__(64) k64_p2m(F64Dev D, const int32_t* __restrict__ leaves) {
  constexpr int NY = P * (P + 1) / 2, P2 = P * P, CH = NY * 16 * 32 > 48 * 1024 ? 16 : 32;
  const int cell = leaves[blockIdx.x];
  const int4 rg = D.cells[cell];
  const float4 g = D.geo[cell];
  const double rh = D.rho[D.clev[cell]];
  __shared__ double2 sa[CH][NY];
  __shared__ double2 sq[CH];
  const int lane = threadIdx.x;
  double2 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = make_double2(0.0, 0.0);
  for (int j0 = rg.x; j0 < rg.y; j0 += CH) {
    const int nj = min(CH, rg.y - j0);
    if (lane < nj) {
      const float4 p = D.spos[j0 + lane];
      const double dx = (double)p.x - g.x, dy = (double)p.y - g.y, dz = (double)p.z - g.z;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      double b[P];
      radial_scaled64<P>(D.k * r, rh, b);
      double2* a = sa[lane];
      ylm_visit64<P>(dx, dy, dz, r, [&](int n, int m, double2 y) {
        a[n * (n + 1) / 2 + m] = make_double2(y.x * b[n], y.y * b[n]);
      });
      sq[lane] = D.q[j0 + lane];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t;
      if (e < P2) {
        const int n = (int)sqrt((double)e + 0.5);
        const int m = e - n * n - n;
        const int ai = n * (n + 1) / 2 + (m < 0 ? -m : m);
        double2 s = acc[t];
        for (int j = 0; j < nj; ++j) {
          double2 y = sa[j][ai];
          if (m >= 0) y.y = -y.y;  // conj for m >= 0
          s = zfma(sq[j], y, s);
        }
        acc[t] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = lane + 64 * t;
    if (e < P2) D.M[(size_t)cell * P2 + e] = acc[t];
  }
}

// M2M: one block per parent; M[parent] = sum over children of T M[child].
__global__ void __launch_bounds__(256) k64_m2m(F64Dev D, const int32_t* __restrict__ parents) {
  const int cell = parents[blockIdx.x];
  const int4 tp = D.topo[cell];
  const int P2 = D.P * D.P;
  __shared__ double2 sm[kMaxP * kMaxP];
  double2 acc = make_double2(0.0, 0.0);
  const int r = threadIdx.x;
  for (int ch = tp.x; ch < tp.y; ++ch) {
    __syncthreads();
    for (int e = threadIdx.x; e < P2; e += blockDim.x) sm[e] = D.M[(size_t)ch * P2 + e];
    __syncthreads();
    const double2* T = D.tables + (size_t)D.cops[ch].x * D.Kp * D.Rp;
    if (r < P2)
      for (int c = 0; c < P2; ++c) acc = zfma(T[(size_t)c * D.Rp + r], sm[c], acc);
  }
  if (r < P2) D.M[(size_t)cell * P2 + r] = acc;
}

// M2L: one block per chunk (op, up to 32 pairs); the reflected multipoles
// of the chunk sit in LDS; thread r accumulates canonical output row r of
// every pair and adds it, mapped back, into the target's local with FP64
// atomics.
constexpr int kM2L64Pairs = 32;

__global__ void __launch_bounds__(256) k64_m2l(F64Dev D, const int4* __restrict__ chunks) {
  extern __shared__ double2 sb64[];  // [32][Kp]
  const int4 ch = chunks[blockIdx.x];  // (op, pair begin, pair end, -)
  const int np = ch.z - ch.y;
  const int P2 = D.P * D.P, Kp = D.Kp, Rp = D.Rp;
  for (int e = threadIdx.x; e < np * Kp; e += blockDim.x) {
    const int p = e / Kp, k = e - p * Kp;
    const int4 pr = D.m2l_pairs[ch.y + p];
    const int code = D.bmap[pr.z * Kp + k];
    sb64[e] = (code & (1 << 17)) ? make_double2(0.0, 0.0)
                                 : apply_code64(D.M[(size_t)pr.y * P2 + (code & 0xffff)], code);
  }
  __syncthreads();
  const double2* T = D.tables + (size_t)ch.x * Kp * Rp;
  for (int r = threadIdx.x; r < P2; r += blockDim.x) {
    double2 acc[kM2L64Pairs];
#pragma unroll
    for (int p = 0; p < kM2L64Pairs; ++p) acc[p] = make_double2(0.0, 0.0);
    for (int k = 0; k < Kp; ++k) {
      const double2 t = T[(size_t)k * Rp + r];
#pragma unroll
      for (int p = 0; p < kM2L64Pairs; ++p)
        if (p < np) acc[p] = zfma(t, sb64[p * Kp + k], acc[p]);
    }
#pragma unroll
    for (int p = 0; p < kM2L64Pairs; ++p)
      if (p < np) {
        const int4 pr = D.m2l_pairs[ch.y + p];
        const int code = D.bmap[pr.z * Kp + r];  // canonical row r <-> target coefficient
        const double2 v = apply_code64_inv(acc[p], code);
        double* dst = reinterpret_cast<double*>(D.L + (size_t)pr.x * P2 + (code & 0xffff));
        atomicAdd(dst, v.x);
        atomicAdd(dst + 1, v.y);
      }
  }
}

// L2L: one block per child; L[child] += T L[parent].
__global__ void __launch_bounds__(256) k64_l2l(F64Dev D, const int32_t* __restrict__ cells) {
  const int cell = cells[blockIdx.x];
  const int parent = D.topo[cell].z;
  const int P2 = D.P * D.P;
  __shared__ double2 sl[kMaxP * kMaxP];
  for (int e = threadIdx.x; e < P2; e += blockDim.x) sl[e] = D.L[(size_t)parent * P2 + e];
  __syncthreads();
  const double2* T = D.tables + (size_t)D.cops[cell].y * D.Kp * D.Rp;
  const int r = threadIdx.x;
  if (r < P2) {
    double2 s = D.L[(size_t)cell * P2 + r];
    for (int c = 0; c < P2; ++c) s = zfma(T[(size_t)c * D.Rp + r], sl[c], s);
    D.L[(size_t)cell * P2 + r] = s;
  }
}

// L2P: one block per leaf, one target per thread; writes the sorted output.
template <int P>
__global__ void __launch_bounds__(64) k64_l2p(F64Dev D, const int32_t* __restrict__ leaves) {
  constexpr int P2 = P * P;
  const int cell = leaves[blockIdx.x];
  const int4 rg = D.cells[cell];
  const float4 g = D.geo[cell];
  const double rh = D.rho[D.clev[cell]];
  __shared__ double2 sl[P2];
  for (int e = threadIdx.x; e < P2; e += blockDim.x) sl[e] = D.L[(size_t)cell * P2 + e];
  __syncthreads();
  for (int i = rg.z + threadIdx.x; i < rg.w; i += 64) {
    const float4 p = D.tpos[i];
    const double dx = (double)p.x - g.x, dy = (double)p.y - g.y, dz = (double)p.z - g.z;
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double b[P];
    radial_scaled64<P>(D.k * r, rh, b);
    double2 u[P];
#pragma unroll
    for (int n = 0; n < P; ++n) u[n] = make_double2(0.0, 0.0);
    ylm_visit64<P>(dx, dy, dz, r, [&](int n, int m, double2 y) {
      if (m == 0) {
        u[n] = zfma(sl[n * n + n], y, u[n]);
      } else {
        u[n] = zfma(sl[n * n + n + m], y, u[n]);
        u[n] = zfma(sl[n * n + n - m], make_double2(y.x, -y.y), u[n]);
      }
    });
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int n = 0; n < P; ++n) {
      s.x = fma(b[n], u[n].x, s.x);
      s.y = fma(b[n], u[n].y, s.y);
    }
    D.ys[i] = make_double2(-D.k * s.y, D.k * s.x);  // times i k
  }
}

// P2P: one block (64 threads) per target leaf, one target per thread, the
// leaf's merged source intervals read directly; y += sum q e^{ikR}/(4 pi R).
__global__ void __launch_bounds__(64) k64_p2p(F64Dev D) {
  const int4 wk = D.p2p_work[blockIdx.x];  // (tgt begin, tgt end, interval begin, interval end)
  for (int i = wk.x + threadIdx.x; i < wk.y; i += 64) {
    const float4 x = D.tpos[i];
    double sr = 0.0, si = 0.0;
    for (int v = wk.z; v < wk.w; ++v) {
      const int2 iv = D.p2p_ivals[v];
      for (int j = iv.x; j < iv.y; ++j) {
        const float4 y = D.spos[j];
        const double dx = (double)x.x - y.x, dy = (double)x.y - y.y, dz = (double)x.z - y.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 > 0.0) {
          const double R = sqrt(r2);
          double sn, cs;
          sincos(D.k * R, &sn, &cs);
          const double2 q = D.q[j];
          sr += (q.x * cs - q.y * sn) / R;
          si += (q.x * sn + q.y * cs) / R;
        }
      }
    }
    const double sc = 0.07957747154594767;  // 1 / (4 pi)
    D.ys[i].x += sr * sc;
    D.ys[i].y += si * sc;
  }
}

__global__ void k64_scatter(F64Dev D, double2* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D.ntgt) y[D.tgt_perm[i]] = D.ys[i];
}

// Direct sum y_i = sum_{j: R_ij > 0} q_j e^{ikR_ij} / (4 pi R_ij) in FP64:
// one block per target, threads over sources, fixed-order block reduction.
__global__ void __launch_bounds__(256) k64_direct(const float* __restrict__ src, const double2* __restrict__ q,
                                                  int64_t n, const float* __restrict__ tgt, double k,
                                                  double2* __restrict__ y) {
  const int64_t i = blockIdx.x;
  const double tx = tgt[3 * i], ty = tgt[3 * i + 1], tz = tgt[3 * i + 2];
  double sr = 0.0, si = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const double dx = tx - src[3 * j], dy = ty - src[3 * j + 1], dz = tz - src[3 * j + 2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 > 0.0) {
      const double R = sqrt(r2);
      double sn, cs;
      sincos(k * R, &sn, &cs);
      const double2 qj = q[j];
      sr += (qj.x * cs - qj.y * sn) / R;
      si += (qj.x * sn + qj.y * cs) / R;
    }
  }
  __shared__ double rr[256], ri[256];
  rr[threadIdx.x] = sr;
  ri[threadIdx.x] = si;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rr[threadIdx.x] += rr[threadIdx.x + w];
      ri[threadIdx.x] += ri[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) y[i] = make_double2(rr[0] * 0.07957747154594767, ri[0] * 0.07957747154594767);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch64_gather(const F64Dev& D, const double2* x, hipStream_t s) {
  if (D.nsrc > 0) k64_gather<<<(unsigned)((D.nsrc + 255) / 256), 256, 0, s>>>(D, x);
}
void launch64_zero(const F64Dev& D, hipStream_t s) { k64_zero<<<2048, 256, 0, s>>>(D); }
void launch64_p2m(const F64Dev& D, const int32_t* leaves, int n, hipStream_t s) {
  if (n <= 0) return;
  switch (D.P) {
#define X(p) \
  case p: k64_p2m<p><<<n, 64, 0, s>>>(D, leaves); break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
    default: break;
  }
}
void launch64_m2m(const F64Dev& D, const int32_t* parents, int n, hipStream_t s) {
  if (n > 0) k64_m2m<<<n, 256, 0, s>>>(D, parents);
}
void launch64_m2l(const F64Dev& D, const int4* chunks, int n, hipStream_t s) {
  const size_t lds = (size_t)m2l_pairs_per_chunk(D.P) * D.Kp * sizeof(double2);  // <= 64 KiB
  if (n > 0) k64_m2l<<<n, 256, lds, s>>>(D, chunks);
}
void launch64_l2l(const F64Dev& D, const int32_t* cells, int n, hipStream_t s) {
  if (n > 0) k64_l2l<<<n, 256, 0, s>>>(D, cells);
}
void launch64_l2p(const F64Dev& D, const int32_t* leaves, int n, hipStream_t s) {
  if (n <= 0) return;
  switch (D.P) {
#define X(p) \
  case p: k64_l2p<p><<<n, 64, 0, s>>>(D, leaves); break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#undef X
    default: break;
  }
}
void launch64_p2p(const F64Dev& D, int nwork, hipStream_t s) {
  if (nwork > 0) k64_p2p<<<nwork, 64, 0, s>>>(D);
}
void launch64_scatter(const F64Dev& D, double2* y, hipStream_t s) {
  if (D.ntgt > 0) k64_scatter<<<(unsigned)((D.ntgt + 255) / 256), 256, 0, s>>>(D, y);
}
void launch64_direct(const float* src, const double2* q, int64_t n, const float* tgt, int64_t m, double k,
                     double2* y, hipStream_t s) {
  if (m > 0) k64_direct<<<(unsigned)m, 256, 0, s>>>(src, q, n, tgt, k, y);
}

}  // namespace hfmm
