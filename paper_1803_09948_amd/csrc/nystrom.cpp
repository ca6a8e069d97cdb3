// Curved-element Nystrom handles (Sec. 2.2, eqs. (8)-(10); six points per
// curved triangle as in the dataset description of Sec. 5): geometry, the
// near pattern, the quadrature tables and the corrections.  The FMM part is
// the BIE machinery with sources = targets = the points and strengths
// w_i I_i; the corrections are computed by nystrom_kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "hfmm_internal.h"
#include "nystrom_kernels.h"

namespace hfmm {

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                \
      return HFMM_EHIP;                                                            \
    }                                                                              \
  } while (0)

namespace {

// The symmetric degree-4 six-point rule of the reference triangle
// {u, v >= 0, u + v <= 1} (Strang and Fix; Dunavant 1985): barycentric orbits
// (a, b, b) with their weights for a unit-area triangle.
struct Rule6 {
  double u[6], v[6], w[6];
  Rule6() {
    const double orb[2][3] = {{0.816847572980459, 0.091576213509771, 0.109951743655322},
                              {0.108103018168070, 0.445948490915965, 0.223381589678011}};
    int q = 0;
    for (int o = 0; o < 2; ++o) {
      const double a = orb[o][0], b = orb[o][1];
      const double lam[3][3] = {{a, b, b}, {b, a, b}, {b, b, a}};
      for (int p = 0; p < 3; ++p, ++q) {
        u[q] = lam[p][1];
        v[q] = lam[p][2];
        w[q] = 0.5 * orb[o][2];
      }
    }
  }
};
const Rule6& rule6() {
  static const Rule6 r;
  return r;
}

// C = inverse of the 6 x 6 matrix V[k][c] = mono_c(u_k, v_k) (Gauss-Jordan
// with partial pivoting), so L_i = sum_c mono_c C[c][i].
void lagrange_coeffs(double* C) {
  const Rule6& R = rule6();
  double A[6][12];
  for (int k = 0; k < 6; ++k) {
    const double u = R.u[k], v = R.v[k];
    const double m[6] = {1.0, u, v, u * u, u * v, v * v};
    for (int c = 0; c < 6; ++c) A[k][c] = m[c];
    for (int c = 0; c < 6; ++c) A[k][6 + c] = (k == c) ? 1.0 : 0.0;
  }
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    for (int r = col + 1; r < 6; ++r)
      if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
    for (int c = 0; c < 12; ++c) std::swap(A[col][c], A[piv][c]);
    const double d = A[col][col];
    for (int c = 0; c < 12; ++c) A[col][c] /= d;
    for (int r = 0; r < 6; ++r) {
      if (r == col) continue;
      const double f = A[r][col];
      for (int c = 0; c < 12; ++c) A[r][c] -= f * A[col][c];
    }
  }
  for (int c = 0; c < 6; ++c)
    for (int i = 0; i < 6; ++i) C[6 * c + i] = A[c][6 + i];
}

void gauss01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

// (u, v, w) of the reference triangle split into 4^L uniform sub-triangles,
// each with an n x n Gauss rule collapsed at its first corner.
std::vector<double> subdivided_rule(int L, int n) {
  struct T2 {
    double p[3][2];
  };
  std::vector<T2> tris{{{{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}}}};
  for (int l = 0; l < L; ++l) {
    std::vector<T2> nt;
    for (const T2& t : tris) {
      double m[3][2];
      for (int e = 0; e < 3; ++e)
        for (int d = 0; d < 2; ++d) m[e][d] = 0.5 * (t.p[e][d] + t.p[(e + 1) % 3][d]);
      // m[0] = mid(p0,p1), m[1] = mid(p1,p2), m[2] = mid(p2,p0)
      nt.push_back({{{t.p[0][0], t.p[0][1]}, {m[0][0], m[0][1]}, {m[2][0], m[2][1]}}});
      nt.push_back({{{t.p[1][0], t.p[1][1]}, {m[1][0], m[1][1]}, {m[0][0], m[0][1]}}});
      nt.push_back({{{t.p[2][0], t.p[2][1]}, {m[2][0], m[2][1]}, {m[1][0], m[1][1]}}});
      nt.push_back({{{m[0][0], m[0][1]}, {m[1][0], m[1][1]}, {m[2][0], m[2][1]}}});
    }
    tris.swap(nt);
  }
  std::vector<double> gx(n), gw(n), out;
  gauss01(n, gx.data(), gw.data());
  out.reserve(tris.size() * n * n * 3);
  for (const T2& t : tris) {
    const double e0u = t.p[1][0] - t.p[0][0], e0v = t.p[1][1] - t.p[0][1];
    const double eu = t.p[2][0] - t.p[1][0], ev = t.p[2][1] - t.p[1][1];
    const double det = std::fabs(e0u * (t.p[2][1] - t.p[0][1]) - e0v * (t.p[2][0] - t.p[0][0]));
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        const double s = gx[a], tt = gx[b];
        out.push_back(t.p[0][0] + s * e0u + s * tt * eu);
        out.push_back(t.p[0][1] + s * e0v + s * tt * ev);
        out.push_back(gw[a] * gw[b] * s * det);
      }
  }
  return out;
}

void qmap_host(const double* X, double u, double v, double* r, double* jac) {
  const double l1 = 1.0 - u - v, l2 = u, l3 = v;
  const double N[6] = {l1 * (2 * l1 - 1), l2 * (2 * l2 - 1), l3 * (2 * l3 - 1), 4 * l1 * l2, 4 * l2 * l3,
                       4 * l3 * l1};
  const double Nu[6] = {-(4 * l1 - 1), 4 * l2 - 1, 0.0, 4 * (l1 - l2), 4 * l3, -4 * l3};
  const double Nv[6] = {-(4 * l1 - 1), 0.0, 4 * l3 - 1, -4 * l2, 4 * l2, 4 * (l1 - l3)};
  double xu[3] = {0, 0, 0}, xv[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    r[d] = 0.0;
    for (int a = 0; a < 6; ++a) {
      r[d] += N[a] * X[3 * a + d];
      xu[d] += Nu[a] * X[3 * a + d];
      xv[d] += Nv[a] * X[3 * a + d];
    }
  }
  if (jac) {
    const double c0 = xu[1] * xv[2] - xu[2] * xv[1], c1 = xu[2] * xv[0] - xu[0] * xv[2],
                 c2 = xu[0] * xv[1] - xu[1] * xv[0];
    *jac = std::sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  }
}

}  // namespace

float nystrom_weight(int64_t p) { return (float)rule6().w[p % 6]; }

int prepare_nystrom(Tree& t, Plan& pl, hipStream_t s) {
  int rc;
  const int64_t N = t.npanel;
  if (!t.near_ready) {  // set only once every upload below succeeded
    NysConst K{};
    const Rule6& R = rule6();
    for (int i = 0; i < 6; ++i) {
      K.uv[2 * i] = R.u[i];
      K.uv[2 * i + 1] = R.v[i];
      K.w[i] = R.w[i];
    }
    lagrange_coeffs(K.lagr);
    gauss01(kNysSelfOrder, K.gx, K.gw);
    // near rules of 4^0 .. 4^near_levels sub-triangles, one after the other
    std::vector<double> rule;
    K.max_level = t.near_levels;
    for (int L = 0; L <= t.near_levels; ++L) {
      std::vector<double> r = subdivided_rule(L, t.near_order);
      K.rule_off[L] = (int)(rule.size() / 3);
      K.rule_cnt[L] = (int)(r.size() / 3);
      rule.insert(rule.end(), r.begin(), r.end());
    }
    t.nys_nrule = (int)(rule.size() / 3);
    std::vector<NysConst> kv{K};
    std::vector<int32_t> rows(t.near_col.size());
    for (int64_t i = 0; i < N; ++i)
      for (int q = t.near_off[i]; q < t.near_off[i + 1]; ++q) rows[q] = (int32_t)i;
    if ((rc = upload_vec(t.d_nys_K, kv)) || (rc = upload_vec(t.d_nys_rule, rule)) ||
        (rc = upload_vec(t.d_nys_elem, t.nys_elem)) || (rc = upload_vec(t.d_nys_pts, t.nys_pts)) ||
        (rc = upload_vec(t.d_nys_items, t.nys_items)) || (rc = upload_vec(t.d_near_off, t.near_off)) ||
        (rc = upload_vec(t.d_near_col, t.near_col)) || (rc = upload_vec(t.d_near_row, rows)))
      return rc;
    t.near_ready = true;
  }
  pl.n_near = (int64_t)t.near_col.size();
  if ((rc = pl.d_near_val.alloc(std::max<size_t>(1, t.near_col.size()) * sizeof(float2))) ||
      (rc = pl.d_self6.alloc((size_t)N * 6 * sizeof(double2))))
    return rc;
  const NysConst* K = t.d_nys_K.as<NysConst>();
  if (t.bie_treatment == 0)
    launch_nys_near((int64_t)t.nys_items.size(), t.d_nys_items.as<int4>(), t.d_nys_pts.as<double>(),
                    t.d_nys_elem.as<double>(), K, t.d_nys_rule.as<double>(), pl.k, pl.ki,
                    pl.d_near_val.as<float2>(), s);
  else
    HIP_TRY(hipMemsetAsync(pl.d_near_val.p, 0, pl.d_near_val.bytes, s));
  if (t.bie_treatment <= 1)
    launch_nys_self(N, t.d_nys_pts.as<double>(), t.d_nys_elem.as<double>(), K, kNysSelfOrder, pl.k, pl.ki,
                    pl.d_self6.as<double2>(), s);
  else
    HIP_TRY(hipMemsetAsync(pl.d_self6.p, 0, pl.d_self6.bytes, s));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return HFMM_OK;
}

}  // namespace hfmm

using namespace hfmm;

extern "C" {

int hfmm_build_nystrom(const double* nodes, int64_t nn, const int32_t* tri6, int64_t nt, const hfmm_opts* opts,
                       hfmm_tree** out) {
  try {
    if (!out) return set_error("out is NULL"), HFMM_EINVAL;
    *out = nullptr;
    if (!nodes || !tri6 || nn < 6 || nt < 1 || nt > (int64_t(1) << 26))
      return set_error("need nn >= 6 nodes and 1 <= nt <= 2^26 elements"), HFMM_EINVAL;
    for (int64_t i = 0; i < 3 * nn; ++i)
      if (!std::isfinite(nodes[i])) return set_error("non-finite node"), HFMM_EINVAL;
    for (int64_t i = 0; i < 6 * nt; ++i)
      if (tri6[i] < 0 || tri6[i] >= nn) return set_error("element node index out of range"), HFMM_EINVAL;
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
    t->nystrom = true;
    const int64_t N = 6 * nt;
    t->npanel = N;
    t->nys_elem.resize(18 * nt);
    t->nys_pts.resize(3 * N);
    t->nys_jac.resize(N);
    std::vector<double> cen(3 * nt), h(nt);
    std::vector<float> pf(3 * N);
    const Rule6& R = rule6();
    for (int64_t e = 0; e < nt; ++e) {
      double* X = t->nys_elem.data() + 18 * e;
      for (int a = 0; a < 6; ++a)
        for (int dd = 0; dd < 3; ++dd) X[3 * a + dd] = nodes[3 * (int64_t)tri6[6 * e + a] + dd];
      double hm = 0.0;
      for (int a = 0; a < 3; ++a) {
        double d2 = 0.0;
        for (int dd = 0; dd < 3; ++dd) {
          const double q = X[3 * a + dd] - X[3 * ((a + 1) % 3) + dd];
          d2 += q * q;
        }
        hm = std::max(hm, std::sqrt(d2));
      }
      if (!(hm > 0.0)) return set_error("degenerate element"), HFMM_EINVAL;
      h[e] = hm;
      qmap_host(X, 1.0 / 3.0, 1.0 / 3.0, cen.data() + 3 * e, nullptr);
      for (int i = 0; i < 6; ++i) {
        const int64_t p = 6 * e + i;
        double jac;
        qmap_host(X, R.u[i], R.v[i], t->nys_pts.data() + 3 * p, &jac);
        if (!(jac > 0.0)) return set_error("element with a vanishing Jacobian"), HFMM_EINVAL;
        t->nys_jac[p] = jac;
        for (int dd = 0; dd < 3; ++dd) pf[3 * p + dd] = (float)t->nys_pts[3 * p + dd];
      }
    }
    build_tree(pf.data(), N, pf.data(), N, t->ncrit, t->max_level, t->h);
    t->uid = next_uid();
    // near pattern: for each point, elements other than its own whose
    // centroid lies within eta h_e (uniform grid of the centroids)
    double hmax = 0.0, lo[3] = {INFINITY, INFINITY, INFINITY};
    for (int64_t e = 0; e < nt; ++e) {
      hmax = std::max(hmax, h[e]);
      for (int dd = 0; dd < 3; ++dd) lo[dd] = std::min(lo[dd], cen[3 * e + dd]);
    }
    double ext = 0.0;
    for (int64_t e = 0; e < nt; ++e)
      for (int dd = 0; dd < 3; ++dd) ext = std::max(ext, cen[3 * e + dd] - lo[dd]);
    // cells no smaller than eta * max h, at most 2^20 per axis; a point lies
    // within h of its element's centroid, so its cell is at most one outside
    // the centroids' range and its neighbours two: keys of cell + 2 fit 21 bits
    const double cs = std::max({t->eta * hmax, ext / double(1 << 20), 1e-300});
    auto cell = [&](double x, int dd) { return (int64_t)std::floor((x - lo[dd]) / cs); };
    auto key = [](int64_t a, int64_t b, int64_t c) {
      return ((uint64_t)(a + 2) << 42) ^ ((uint64_t)(b + 2) << 21) ^ (uint64_t)(c + 2);
    };
    std::unordered_map<uint64_t, std::vector<int32_t>> grid;
    grid.reserve((size_t)nt);
    for (int64_t e = 0; e < nt; ++e)
      grid[key(cell(cen[3 * e], 0), cell(cen[3 * e + 1], 1), cell(cen[3 * e + 2], 2))].push_back((int32_t)e);
    t->near_off.assign(N + 1, 0);
    t->near_col.clear();
    t->nys_items.clear();
    std::vector<int32_t> row;
    for (int64_t j = 0; j < N; ++j) {
      row.clear();
      const double* x = t->nys_pts.data() + 3 * j;
      const int64_t ci = cell(x[0], 0), cj = cell(x[1], 1), ck = cell(x[2], 2);
      for (int64_t a = ci - 1; a <= ci + 1; ++a)
        for (int64_t b = cj - 1; b <= cj + 1; ++b)
          for (int64_t c = ck - 1; c <= ck + 1; ++c) {
            auto it = grid.find(key(a, b, c));
            if (it == grid.end()) continue;
            for (int32_t e : it->second) {
              if (e == j / 6) continue;
              double d2 = 0.0;
              for (int dd = 0; dd < 3; ++dd) {
                const double q = x[dd] - cen[3 * (int64_t)e + dd];
                d2 += q * q;
              }
              if (std::sqrt(d2) < t->eta * h[e]) row.push_back(e);
            }
          }
      std::sort(row.begin(), row.end());
      for (int32_t e : row) {
        t->nys_items.push_back(make_int4((int)j, e, (int)t->near_col.size(), 0));
        for (int i = 0; i < 6; ++i) t->near_col.push_back(6 * e + i);
      }
      if (t->near_col.size() > (size_t)INT32_MAX) return set_error("near pattern too large"), HFMM_EINVAL;
      t->near_off[j + 1] = (int32_t)t->near_col.size();
    }
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

int hfmm_nystrom_points(const hfmm_tree* tree, double* xyz, double* weight, double* jac) {
  if (!tree) return set_error("tree is NULL"), HFMM_EINVAL;
  const Tree& t = *reinterpret_cast<const Tree*>(tree);
  if (!t.nystrom) return set_error("not a curved-element handle"), HFMM_EINVAL;
  if (xyz) std::memcpy(xyz, t.nys_pts.data(), t.nys_pts.size() * sizeof(double));
  if (weight)
    for (int64_t p = 0; p < t.npanel; ++p) weight[p] = rule6().w[p % 6];
  if (jac) std::memcpy(jac, t.nys_jac.data(), t.nys_jac.size() * sizeof(double));
  return HFMM_OK;
}

}  // extern "C"
