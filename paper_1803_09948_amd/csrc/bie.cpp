// Boundary-integral handles, near/self corrections and the FP64 GMRES driver.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "bie_kernels.h"
#include "nystrom_kernels.h"
#include "hfmm_internal.h"

namespace hfmm {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                \
      return HFMM_EHIP;                                                            \
    }                                                                              \
  } while (0)

// Gauss-Legendre nodes and weights mapped to [0, 1] (Newton on P_n).
static void gl01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // half of the [-1,1] weight
  }
}

constexpr int kSelfOrder = 10;

// Near pattern: j != i with |c_i - c_j| < eta h_j, by a uniform grid hash of
// the centroids with cell size eta * max h.  Rows in caller order, columns
// ascending.
static void near_pattern(const std::vector<double>& cen, const std::vector<double>& h, double eta,
                         std::vector<int32_t>& off, std::vector<int32_t>& col) {
  const int64_t n = (int64_t)h.size();
  double hmax = 0.0, lo[3] = {INFINITY, INFINITY, INFINITY};
  for (int64_t i = 0; i < n; ++i) {
    hmax = std::max(hmax, h[i]);
    for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], cen[3 * i + d]);
  }
  double ext = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) ext = std::max(ext, cen[3 * i + d] - lo[d]);
  // cells no smaller than eta * max h (a larger cell only adds candidates,
  // which the distance test filters), and at most 2^20 of them per axis, so
  // that a cell index plus one and its neighbours fit 21 bits of the key
  const double cs = std::max({eta * hmax, ext / double(1 << 20), 1e-300});
  auto cell = [&](int64_t i, int d) { return (int64_t)std::floor((cen[3 * i + d] - lo[d]) / cs); };
  auto key = [](int64_t a, int64_t b, int64_t c) {  // cells -1 .. 2^20 + 1 -> distinct keys
    return ((uint64_t)(a + 1) << 42) ^ ((uint64_t)(b + 1) << 21) ^ (uint64_t)(c + 1);
  };
  std::unordered_map<uint64_t, std::vector<int32_t>> grid;
  grid.reserve((size_t)n);
  for (int64_t i = 0; i < n; ++i) grid[key(cell(i, 0), cell(i, 1), cell(i, 2))].push_back((int32_t)i);
  off.assign(n + 1, 0);
  col.clear();
  std::vector<int32_t> row;
  for (int64_t i = 0; i < n; ++i) {
    row.clear();
    int64_t ci = cell(i, 0), cj = cell(i, 1), ck = cell(i, 2);
    for (int64_t a = ci - 1; a <= ci + 1; ++a)
      for (int64_t b = cj - 1; b <= cj + 1; ++b)
        for (int64_t c = ck - 1; c <= ck + 1; ++c) {
          auto it = grid.find(key(a, b, c));
          if (it == grid.end()) continue;
          for (int32_t j : it->second) {
            if (j == i) continue;
            double d2 = 0.0;
            for (int d = 0; d < 3; ++d) {
              double t = cen[3 * i + d] - cen[3 * (int64_t)j + d];
              d2 += t * t;
            }
            if (std::sqrt(d2) < eta * h[j]) row.push_back(j);
          }
        }
    std::sort(row.begin(), row.end());
    col.insert(col.end(), row.begin(), row.end());
    off[i + 1] = (int32_t)col.size();
  }
}

int prepare_bie(Tree& t, Plan& pl, hipStream_t s) {
  int rc;
  const int64_t n = t.npanel;
  if (!t.near_ready) {  // set only once every upload below succeeded
    std::vector<int32_t> rows(t.near_col.size());
    for (int64_t i = 0; i < n; ++i)
      for (int q = t.near_off[i]; q < t.near_off[i + 1]; ++q) rows[q] = (int32_t)i;
    std::vector<double> panels(9 * n);
    for (int64_t i = 0; i < n; ++i)
      for (int v = 0; v < 3; ++v)
        for (int d = 0; d < 3; ++d) panels[9 * i + 3 * v + d] = t.verts[3 * (int64_t)t.tris[3 * i + v] + d];
    std::vector<double> gx, gw, sx, sw;
    gl01(t.near_order, gx, gw);
    gl01(kSelfOrder, sx, sw);
    std::vector<double> gl;
    gl.insert(gl.end(), gx.begin(), gx.end());
    gl.insert(gl.end(), gw.begin(), gw.end());
    gl.insert(gl.end(), sx.begin(), sx.end());
    gl.insert(gl.end(), sw.begin(), sw.end());
    if ((rc = upload_vec(t.d_near_off, t.near_off)) || (rc = upload_vec(t.d_near_col, t.near_col)) ||
        (rc = upload_vec(t.d_near_row, rows)) || (rc = upload_vec(t.d_gl, gl)))
      return rc;
    if ((rc = upload_vec(t.d_panels, panels))) return rc;
    t.near_ready = true;
  }
  const int ng = t.near_order;
  const double* gl = t.d_gl.as<double>();
  pl.n_near = (int64_t)t.near_col.size();
  if ((rc = pl.d_near_val.alloc(std::max<size_t>(1, t.near_col.size()) * sizeof(float2))) ||
      (rc = pl.d_diag.alloc((size_t)n * sizeof(double2))))
    return rc;
  // corrections of the chosen treatment (the ablation modes leave zeros)
  if (t.bie_treatment == 0)
    launch_near(pl.n_near, t.d_near_row.as<int32_t>(), t.d_near_col.as<int32_t>(), t.d_panels.as<double>(),
                pl.k, pl.ki, t.near_levels, gl, gl + ng, ng, pl.d_near_val.as<float2>(), s);
  else
    HIP_TRY(hipMemsetAsync(pl.d_near_val.p, 0, pl.d_near_val.bytes, s));
  if (t.bie_treatment <= 1)
    launch_self(n, t.d_panels.as<double>(), pl.k, pl.ki, gl + 2 * ng, gl + 2 * ng + kSelfOrder, kSelfOrder,
                pl.d_diag.as<double2>(), s);
  else
    HIP_TRY(hipMemsetAsync(pl.d_diag.p, 0, pl.d_diag.bytes, s));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return HFMM_OK;
}

// ---------------------------------------------------------------------------
// GMRES(m) in FP64 with two passes of classical Gram-Schmidt (CGS2) and
// complex Givens rotations; the FMM product in FP32, the self term in FP64.
// ---------------------------------------------------------------------------
// Layout of the workspace of one GMRES(m) solve on n unknowns, each array
// 256-byte aligned: Krylov basis V [m+1][n], work vectors w, r (double2) and
// x64, y64 (float2), Hessenberg H [m+1][m], Givens cs, sn, right-hand side
// g, projections h, h2, partial sums, a dot product, status st and the small
// solution yv.  With base == nullptr only the size is computed.
static int64_t gmres_layout(char* base, int64_t n, int m, GmresWork* W) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  GmresWork w{};
  w.V = (double2*)take((int64_t)(m + 1) * n * 16);
  w.w = (double2*)take(n * 16);
  w.r = (double2*)take(n * 16);
  w.x64 = (float2*)take(n * 8);
  w.y64 = (float2*)take(n * 8);
  w.z64 = (float2*)take(n * 8);
  w.H = (double2*)take((int64_t)(m + 1) * m * 16);
  w.cs = (double*)take((int64_t)m * 8);
  w.sn = (double2*)take((int64_t)m * 16);
  w.g = (double2*)take((int64_t)(m + 1) * 16);
  w.h = (double2*)take((int64_t)(m + 32) * 16);
  w.h2 = (double2*)take((int64_t)(m + 32) * 16);
  w.part = (double2*)take((int64_t)mdot_blocks() * 32 * 16);
  w.dot = (double2*)take(16);
  w.st = (double*)take(16);
  w.yv = (double2*)take((int64_t)(m + 1) * 16);
  if (W) *W = w;
  return off;
}

int64_t gmres_workspace_bytes(int64_t n, int m) { return gmres_layout(nullptr, n, m, nullptr); }

GmresWork gmres_carve(void* base, int64_t n, int m) {
  GmresWork w;
  gmres_layout((char*)base, n, m, &w);
  return w;
}

static int gm_workspace(Tree& t, int m, GmresWork* W) {
  if (t.gm_m != m || !t.g_ws.p) {
    t.gm_m = 0;  // not sized for any restart until the buffer is allocated
    int rc = t.g_ws.alloc((size_t)gmres_workspace_bytes(t.npanel, m));
    if (rc) return rc;
    t.gm_m = m;
  }
  *W = gmres_carve(t.g_ws.p, t.npanel, m);
  return HFMM_OK;
}

// Pinned status slots and events of the lagged convergence checks (once per
// handle).
static int gm_lag(Tree& t, GmresLag* lag) {
  if (!t.g_pin) {
    double* p = nullptr;
    HIP_TRY(hipHostMalloc((void**)&p, 4 * sizeof(double), hipHostMallocDefault));
    for (int i = 0; i < 2; ++i) {
      hipError_t e = hipEventCreateWithFlags(&t.g_ev[i], hipEventDisableTiming);
      if (e != hipSuccess) {
        for (int q = 0; q < i; ++q) (void)hipEventDestroy(t.g_ev[q]);
        (void)hipHostFree(p);
        set_error(std::string("hipEventCreateWithFlags: ") + hipGetErrorString(e));
        return HFMM_EHIP;
      }
    }
    t.g_pin = p;
  }
  if (!t.n_stream) {  // the near-correction stream (optional: without it they run after the FMM)
    hipStream_t ns = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&ns, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&e0, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&e1, hipEventDisableTiming) == hipSuccess) {
      t.n_stream = ns;
      t.n_ev[0] = e0;
      t.n_ev[1] = e1;
    } else {
      if (e0) (void)hipEventDestroy(e0);
      if (ns) (void)hipStreamDestroy(ns);
      (void)hipGetLastError();
    }
  }
  lag->pin = t.g_pin;
  lag->ev[0] = t.g_ev[0];
  lag->ev[1] = t.g_ev[1];
  return HFMM_OK;
}

// out = A v (FP64 in/out; FMM and near corrections in FP32, self term in FP64).
// With the handle's near stream, the near corrections (which read only the
// input) run on it beside the FMM into z64, and the conversion adds them to
// the FMM output with the same FP32 add the in-place apply makes: the same
// bits either way.
static int apply_A(Tree& t, Plan& pl, const GmresWork& W, const double2* v, double2* out, hipStream_t s) {
  const int64_t n = t.npanel;
  launch_to_c64(n, v, W.x64, s);
  const int forced = variant_override(kPhaseNear);
  const bool side = t.n_stream != nullptr && (forced >= 0 ? forced == 1 : pl.near_side == 1);
  if (side) {
    HIP_TRY(hipEventRecord(t.n_ev[0], s));
    HIP_TRY(hipStreamWaitEvent(t.n_stream, t.n_ev[0], 0));
    launch_near_apply(n, t.d_near_off.as<int32_t>(), t.d_near_col.as<int32_t>(), pl.d_near_val.as<float2>(),
                      nullptr, W.x64, W.z64, t.n_stream, true);
    HIP_TRY(hipEventRecord(t.n_ev[1], t.n_stream));
  }
  int rc = matvec_impl(t, pl, W.x64, W.y64, s);
  if (rc) return rc;
  if (side) {
    HIP_TRY(hipStreamWaitEvent(s, t.n_ev[1], 0));
  } else {
    launch_near_apply(n, t.d_near_off.as<int32_t>(), t.d_near_col.as<int32_t>(), pl.d_near_val.as<float2>(),
                      nullptr, W.x64, W.y64, s);
  }
  const float2* z = side ? W.z64 : nullptr;
  if (t.nystrom)
    launch_from_c64_self6(n, W.y64, pl.d_self6.as<double2>(), v, out, s, z);
  else
    launch_from_c64_diag(n, W.y64, pl.d_diag.as<double2>(), v, out, s, z);
  HIP_TRY(hipGetLastError());
  return HFMM_OK;
}

// h[0..nv) (+)= V^H w in chunks of 32
static void mdot_all(int64_t n, int nv, const double2* V, const double2* w, double2* part, double2* h,
                     int accumulate, hipStream_t s) {
  for (int c = 0; c < nv; c += 32)
    launch_mdot(n, std::min(32, nv - c), V + (size_t)c * n, n, w, part, h + c, accumulate, s);
}

static int read_doubles(const void* dev, double* host, int cnt, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(host, dev, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return HFMM_OK;
}

// One Arnoldi step j: w = A v_j, two passes of classical Gram-Schmidt
// against V[0..j], the Givens update of column j (its status -- residual
// estimate and breakdown flag -- in W.st) and v_{j+1} = w / ||w||.
static int arnoldi_step(Tree& t, Plan& pl, const GmresWork& W, int m, int j, hipStream_t s) {
  const int64_t n = t.npanel;
  double2* V = W.V;
  int rc = apply_A(t, pl, W, V + (size_t)j * n, W.w, s);
  if (rc) return rc;
  mdot_all(n, j + 1, V, W.w, W.part, W.h, 0, s);
  launch_mupdate(n, j + 1, V, n, W.h, W.w, -1.0, s);
  mdot_all(n, j + 1, V, W.w, W.part, W.h2, 0, s);
  launch_mupdate(n, j + 1, V, n, W.h2, W.w, -1.0, s);
  launch_vec_add(j + 1, W.h2, W.h, s);  // h += h2
  launch_mdot(n, 1, W.w, n, W.w, W.part, W.dot, 0, s);
  launch_givens(j, m, W.h, W.dot, W.H, W.cs, W.sn, W.g, W.st, s);
  launch_scale_by_norm(n, W.w, W.dot, V + (size_t)(j + 1) * n, s);
  HIP_TRY(hipGetLastError());
  return HFMM_OK;
}

int gmres_run(Tree& t, Plan& pl, const GmresWork& W, int m, const double2* b, double2* x, double tol,
              int maxit, hfmm_gmres_info* info, hipStream_t s, const GmresLag* lag) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = t.npanel;
  int rc;
  double2* V = W.V;
  double2* r = W.r;
  double2* part = W.part;
  double2* dotv = W.dot;
  double hv[2];
  // ||b||
  launch_mdot(n, 1, b, n, b, part, dotv, 0, s);
  if ((rc = read_doubles(dotv, hv, 1, s))) return rc;
  const double bnorm = std::sqrt(hv[0]);
  hfmm_gmres_info inf{};
  if (bnorm == 0.0) {
    launch_zero_c128(n, x, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    if (info) *info = inf;
    return HFMM_OK;
  }
  int iters = 0, restarts = 0;
  double est = INFINITY;
  int status = HFMM_ENOTCONV;
  for (;;) {
    // true residual r = b - A x
    if ((rc = apply_A(t, pl, W, x, r, s))) return rc;
    launch_residual(n, b, r, s);
    launch_mdot(n, 1, r, n, r, part, dotv, 0, s);
    if ((rc = read_doubles(dotv, hv, 1, s))) return rc;
    const double beta = std::sqrt(hv[0]);
    inf.resid_true = beta / bnorm;
    if (!std::isfinite(beta)) {
      set_error("GMRES residual is not finite");
      return HFMM_EINTERNAL;
    }
    if (beta / bnorm <= tol) {
      status = HFMM_OK;
      break;
    }
    if (iters >= maxit) break;
    launch_scale_by_norm(n, r, dotv, V, s);
    launch_init_g(m, dotv, W.g, s);
    // Each step's status decides whether the cycle goes on.  Without `lag`
    // the host reads it right after the step; with `lag` the status is
    // copied to a pinned slot and read one step later, after the next step
    // has been queued, so the device never waits for the host.  A step
    // queued past the stopping one is discarded: it changes only H column
    // j, g[j], g[j+1] and V[j+1], which the update of x with `done` columns
    // does not read, so both ways give the same bits.
    int done = 0, decided = 0, queued = 0;
    bool stop = false;
    auto decide = [&](const double* st) -> int {
      ++iters;
      ++decided;
      est = st[0] / bnorm;
      if (!std::isfinite(est)) {
        set_error("GMRES Arnoldi residual estimate is not finite");
        return HFMM_EINTERNAL;
      }
      if (est <= tol || iters >= maxit || st[1] == 0.0) stop = true;
      return HFMM_OK;
    };
    if (!lag) {
      for (int j = 0; j < m && !stop; ++j) {
        if ((rc = arnoldi_step(t, pl, W, m, j, s))) return rc;
        if ((rc = read_doubles(W.st, hv, 2, s)) || (rc = decide(hv))) return rc;
      }
    } else {
      for (int j = 0; j < m && !stop; ++j) {
        if (iters + (queued - decided) >= maxit) break;  // no step beyond maxit products
        if ((rc = arnoldi_step(t, pl, W, m, j, s))) return rc;
        HIP_TRY(hipMemcpyAsync(lag->pin + 2 * (j & 1), W.st, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(lag->ev[j & 1], s));
        ++queued;
        if (queued - decided == 2) {  // step j is queued: decide step j - 1
          const int q = decided;
          HIP_TRY(hipEventSynchronize(lag->ev[q & 1]));
          if ((rc = decide(lag->pin + 2 * (q & 1)))) return rc;
        }
      }
      while (!stop && decided < queued) {
        const int q = decided;
        HIP_TRY(hipEventSynchronize(lag->ev[q & 1]));
        if ((rc = decide(lag->pin + 2 * (q & 1)))) return rc;
      }
      HIP_TRY(hipStreamSynchronize(s));  // a discarded step finishes before its buffers are reused
    }
    done = decided;
    launch_backsolve(done, m, W.H, W.g, W.yv, s);
    launch_mupdate(n, done, V, n, W.yv, x, 1.0, s);
    HIP_TRY(hipGetLastError());
    ++restarts;
  }
  HIP_TRY(hipStreamSynchronize(s));
  inf.iters = iters;
  inf.restarts = restarts;
  inf.resid_est = est;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

// First solve of a plan: time the product with the near corrections beside
// the FMM and after it (a warm-up round, then the best of two rounds of
// three products each, on the workspace's own vectors: their contents do
// not matter) and keep the faster.  Heavy corrections (curved elements)
// gain from the overlap, light ones lose to the extra synchronisation.
static int tune_near(Tree& t, Plan& pl, const GmresWork& W, hipStream_t s) {
  if (pl.near_side >= 0 || variant_override(kPhaseNear) >= 0) return HFMM_OK;
  if (!t.n_stream) {
    pl.near_side = 0;
    return HFMM_OK;
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best[2] = {0.f, 0.f};
  int rc = HFMM_OK;
  for (int rep = 0; rep < 3 && rc == HFMM_OK; ++rep)
    for (int side = 0; side < 2 && rc == HFMM_OK; ++side) {
      pl.near_side = side;
      hipError_t e = hipEventRecord(e0, s);
      for (int i = 0; i < 3 && e == hipSuccess && rc == HFMM_OK; ++i) rc = apply_A(t, pl, W, W.r, W.w, s);
      if (rc) break;
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        set_error(std::string("near-correction timing: ") + hipGetErrorString(e));
        rc = HFMM_EHIP;
        break;
      }
      if (rep == 1 || (rep > 1 && ms < best[side])) best[side] = ms;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  pl.near_side = rc == HFMM_OK && best[1] < best[0] ? 1 : 0;
  return rc;
}

static int gmres(Tree& t, Plan& pl, const double2* b, double2* x, double tol, int m, int maxit,
                 hfmm_gmres_info* info, hipStream_t s) {
  GmresWork W;
  GmresLag lag;
  int rc = gm_workspace(t, m, &W);
  if (rc || (rc = gm_lag(t, &lag)) || (rc = tune_near(t, pl, W, s))) return rc;
  return gmres_run(t, pl, W, m, b, x, tol, maxit, info, s, &lag);
}

}  // namespace hfmm

using namespace hfmm;

extern "C" {

int hfmm_build_bie(const double* verts, int64_t nv, const int32_t* tris, int64_t nt, const hfmm_opts* opts,
                   hfmm_tree** out) {
  try {
    if (!out) return set_error("out is NULL"), HFMM_EINVAL;
    *out = nullptr;
    if (!verts || !tris || nv < 3 || nt < 1 || nt > (int64_t(1) << 28))
      return set_error("need nv >= 3 vertices and 1 <= nt <= 2^28 triangles"), HFMM_EINVAL;
    for (int64_t i = 0; i < 3 * nv; ++i)
      if (!std::isfinite(verts[i])) return set_error("non-finite vertex"), HFMM_EINVAL;
    for (int64_t i = 0; i < 3 * nt; ++i)
      if (tris[i] < 0 || tris[i] >= nv) return set_error("triangle index out of range"), HFMM_EINVAL;
    hfmm_opts d;
    hfmm_default_opts(&d);
    const hfmm_opts* o = opts ? opts : &d;
    if (o->ncrit < 1 || !(o->theta > 0) || !(o->eta > 0) || o->max_level < 0 || o->max_level > kMaxLevel ||
        o->near_levels < 0 || o->near_levels > 5 || o->near_order < 1 || o->near_order > 16 ||
        o->bie_treatment < 0 || o->bie_treatment > 2)
      return set_error("invalid options"), HFMM_EINVAL;
    if (!(o->k_imag >= 0.0) || !std::isfinite(o->k_imag)) return set_error("k_imag must be finite and >= 0"), HFMM_EINVAL;
    auto t = std::make_unique<Tree>();
    t->ncrit = o->ncrit;
    t->max_level = o->max_level;
    t->theta = o->theta;
    t->kappa = o->kappa;
    t->eta = o->eta;
    t->near_levels = o->near_levels;
    t->near_order = o->near_order;
    t->stage_bytes = (int64_t)(o->stage_mb > 0 ? o->stage_mb : 32768) << 20;
    t->bie_treatment = o->bie_treatment;
    t->k_imag = o->k_imag;
    t->bie = true;
    t->npanel = nt;
    t->verts.assign(verts, verts + 3 * nv);
    t->tris.assign(tris, tris + 3 * nt);
    // panel geometry in FP64: centroids, longest edges, 3 interior Gauss points
    std::vector<double> cen(3 * nt), h(nt);
    std::vector<float> src(9 * nt), tgt(3 * nt);
    const double w1 = 2.0 / 3.0, w2 = 1.0 / 6.0;
    for (int64_t i = 0; i < nt; ++i) {
      double P[3][3];
      for (int v = 0; v < 3; ++v)
        for (int dd = 0; dd < 3; ++dd) P[v][dd] = verts[3 * (int64_t)tris[3 * i + v] + dd];
      double e[3] = {0, 0, 0}, cr[3];
      double u[3], ww[3];
      for (int dd = 0; dd < 3; ++dd) {
        u[dd] = P[1][dd] - P[0][dd];
        ww[dd] = P[2][dd] - P[0][dd];
      }
      cr[0] = u[1] * ww[2] - u[2] * ww[1];
      cr[1] = u[2] * ww[0] - u[0] * ww[2];
      cr[2] = u[0] * ww[1] - u[1] * ww[0];
      if (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2] == 0.0)
        return set_error("degenerate triangle"), HFMM_EINVAL;
      for (int dd = 0; dd < 3; ++dd) {
        e[0] += (P[1][dd] - P[0][dd]) * (P[1][dd] - P[0][dd]);
        e[1] += (P[2][dd] - P[1][dd]) * (P[2][dd] - P[1][dd]);
        e[2] += (P[0][dd] - P[2][dd]) * (P[0][dd] - P[2][dd]);
      }
      h[i] = std::sqrt(std::max(e[0], std::max(e[1], e[2])));
      for (int dd = 0; dd < 3; ++dd) {
        cen[3 * i + dd] = (P[0][dd] + P[1][dd] + P[2][dd]) / 3.0;
        tgt[3 * i + dd] = (float)cen[3 * i + dd];
        src[9 * i + 0 + dd] = (float)(w1 * P[0][dd] + w2 * P[1][dd] + w2 * P[2][dd]);
        src[9 * i + 3 + dd] = (float)(w2 * P[0][dd] + w1 * P[1][dd] + w2 * P[2][dd]);
        src[9 * i + 6 + dd] = (float)(w2 * P[0][dd] + w2 * P[1][dd] + w1 * P[2][dd]);
      }
    }
    build_tree(src.data(), 3 * nt, tgt.data(), nt, t->ncrit, t->max_level, t->h);
    t->uid = next_uid();
    near_pattern(cen, h, t->eta, t->near_off, t->near_col);
    *out = reinterpret_cast<hfmm_tree*>(t.release());
    return HFMM_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HFMM_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}

int hfmm_bie_plane_wave(hfmm_tree* tree, double k, const double* dir, void* b, void* stream) {
  try {
    if (!tree || !dir || !b) return set_error("NULL argument"), HFMM_EINVAL;
    Tree& t = *reinterpret_cast<Tree*>(tree);
    if (!t.bie) return set_error("not a BIE handle"), HFMM_EINVAL;
    if (!std::isfinite(k)) return set_error("k must be finite"), HFMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (t.nystrom) {
      if (!t.d_nys_pts.p) {
        int rc = upload_vec(t.d_nys_pts, t.nys_pts);
        if (rc) return rc;
      }
      launch_plane_wave_pts(t.npanel, t.d_nys_pts.as<double>(), k, t.k_imag, dir, (double2*)b, s);
      HIP_TRY(hipGetLastError());
      return HFMM_OK;
    }
    if (!t.d_panels.p) {
      std::vector<double> panels(9 * t.npanel);
      for (int64_t i = 0; i < t.npanel; ++i)
        for (int v = 0; v < 3; ++v)
          for (int d = 0; d < 3; ++d) panels[9 * i + 3 * v + d] = t.verts[3 * (int64_t)t.tris[3 * i + v] + d];
      int rc = upload_vec(t.d_panels, panels);
      if (rc) return rc;
    }
    launch_plane_wave(t.npanel, t.d_panels.as<double>(), k, t.k_imag, dir, (double2*)b, s);
    HIP_TRY(hipGetLastError());
    return HFMM_OK;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}

int hfmm_gmres_solve(hfmm_tree* tree, double k, int32_t P, const void* b, void* x, double tol,
                     int32_t restart, int32_t maxit, hfmm_gmres_info* info, void* stream) {
  try {
    if (!tree || !b || !x) return set_error("NULL argument"), HFMM_EINVAL;
    Tree& t = *reinterpret_cast<Tree*>(tree);
    if (!t.bie) return set_error("GMRES needs a BIE handle"), HFMM_EINVAL;
    int rc = check_kP(k, P);
    if (rc) return rc;
    if (!(tol > 0.0) || restart < 1 || restart > 200 || maxit < 1)
      return set_error("need tol > 0, 1 <= restart <= 200, maxit >= 1"), HFMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Plan* pl;
    if ((rc = prepare(t, k, P, s, &pl))) return rc;
    return gmres(t, *pl, (const double2*)b, (double2*)x, tol, restart, maxit, info, s);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HFMM_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}

}  // extern "C"
