// FP64 variant of the FMM product and the FP64 direct sum (precision
// reference).  The variant reuses the FP32 plan's tree, lists, operator
// descriptors and work lists; it adds FP64 tables and expansions on first
// use and runs the plain FP64 kernels of fmm64_kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fmm64_kernels.h"
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

static int prepare64(Tree& t, Plan& pl, hipStream_t s) {
  if (pl.fp64) return HFMM_OK;
  auto f = std::make_unique<Plan64>();
  const HostTree& h = pl.ct;
  const int P = pl.P, P2 = P * P;
  int Kp, Rp, rc;
  table_dims(P, &Kp, &Rp);
  // tables from the plan's operator descriptors, in FP64
  const Coupling& cp = coupling(P);
  std::vector<double2> cv(cp.re.size());
  for (size_t i = 0; i < cv.size(); ++i) cv[i] = make_double2(cp.re[i], cp.im[i]);
  DevBuf d_off, d_lm, d_val;
  if ((rc = upload_vec(d_off, cp.off)) || (rc = upload_vec(d_lm, cp.lm)) || (rc = upload_vec(d_val, cv)) ||
      (rc = f->d_tables.alloc((size_t)pl.n_ops * Kp * Rp * sizeof(double2))) ||
      (rc = f->d_M.alloc((size_t)h.ncell() * P2 * sizeof(double2))) ||
      (rc = f->d_L.alloc((size_t)h.ncell() * P2 * sizeof(double2))))
    return rc;
  launch_gen_tables64(pl.d_ops.as<OpDescDev>(), (int)pl.n_ops, P, pl.k, d_off.as<int32_t>(), d_lm.as<int32_t>(),
                      d_val.as<double2>(), f->d_tables.as<double2>(), s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  // work lists
  std::vector<int32_t> m2m, l2l;
  const int nlev = (int)pl.m2m_cells.size();
  f->m2m_off.assign(nlev + 1, 0);
  f->l2l_off.assign(nlev + 1, 0);
  for (int l = 0; l < nlev; ++l) {
    f->m2m_off[l] = (int)m2m.size();
    f->l2l_off[l] = (int)l2l.size();
    m2m.insert(m2m.end(), pl.m2m_cells[l].begin(), pl.m2m_cells[l].end());
    if (l < (int)pl.l2l_cells.size()) l2l.insert(l2l.end(), pl.l2l_cells[l].begin(), pl.l2l_cells[l].end());
  }
  f->m2m_off[nlev] = (int)m2m.size();
  f->l2l_off[nlev] = (int)l2l.size();
  std::vector<int4> ch;
  for (const int4& c : pl.m2l_chunks_h) ch.push_back(make_int4(c.x, c.y, c.z, 0));
  f->n_chunks = (int)ch.size();
  if ((rc = upload_vec(f->d_src_leaves, pl.src_leaves)) || (rc = upload_vec(f->d_tgt_leaves, pl.tgt_leaves)) ||
      (rc = upload_vec(f->d_m2m, m2m)) || (rc = upload_vec(f->d_l2l, l2l)) || (rc = upload_vec(f->d_chunks, ch)) ||
      (rc = t.d_q64.ensure((size_t)std::max<int64_t>(1, t.h.nsrc) * sizeof(double2))) ||
      (rc = t.d_ys64.ensure((size_t)std::max<int64_t>(1, t.h.ntgt) * sizeof(double2))))
    return rc;
  pl.fp64 = std::move(f);
  return HFMM_OK;
}

static int matvec64_impl(Tree& t, Plan& pl, const double2* x, double2* y, hipStream_t s) {
  int rc = prepare64(t, pl, s);
  if (rc) return rc;
  Plan64& f = *pl.fp64;
  int Kp, Rp;
  table_dims(pl.P, &Kp, &Rp);
  F64Dev D{};
  D.spos = t.d_src_pos.as<float4>();
  D.tpos = t.d_tgt_pos.as<float4>();
  D.src_idx = t.d_src_idx.as<int32_t>();
  D.tgt_perm = t.d_tgt_perm.as<int32_t>();
  D.cells = pl.d_cells.as<int4>();
  D.geo = pl.d_geo.as<float4>();
  D.clev = pl.d_clev.as<int32_t>();
  D.topo = pl.d_topo.as<int4>();
  D.cops = pl.d_cops.as<int2>();
  D.rho = pl.d_rho.as<double>();
  D.tables = f.d_tables.as<double2>();
  D.M = f.d_M.as<double2>();
  D.L = f.d_L.as<double2>();
  D.q = t.d_q64.as<double2>();
  D.ys = t.d_ys64.as<double2>();
  D.m2l_pairs = pl.d_m2l_pairs.as<int4>();
  D.bmap = pl.d_bmap64.as<int32_t>();
  D.p2p_work = pl.d_p2p_work.as<int4>();
  D.p2p_ivals = pl.d_p2p_ivals.as<int2>();
  D.nsrc = t.h.nsrc;
  D.ntgt = t.h.ntgt;
  D.ncell = pl.ct.ncell();
  D.P = pl.P;
  D.Kp = Kp;
  D.Rp = Rp;
  D.k = pl.k;
  launch64_zero(D, s);
  launch64_gather(D, x, s);
  launch64_p2m(D, f.d_src_leaves.as<int32_t>(), (int)pl.src_leaves.size(), s);
  const int nlev = (int)f.m2m_off.size() - 1;
  for (int l = nlev - 1; l >= 0; --l)
    launch64_m2m(D, f.d_m2m.as<int32_t>() + f.m2m_off[l], f.m2m_off[l + 1] - f.m2m_off[l], s);
  launch64_m2l(D, f.d_chunks.as<int4>(), f.n_chunks, s);
  for (int l = 1; l < nlev; ++l)
    launch64_l2l(D, f.d_l2l.as<int32_t>() + f.l2l_off[l], f.l2l_off[l + 1] - f.l2l_off[l], s);
  launch64_l2p(D, f.d_tgt_leaves.as<int32_t>(), (int)pl.tgt_leaves.size(), s);
  launch64_p2p(D, pl.n_p2p_work, s);
  launch64_scatter(D, y, s);
  HIP_TRY(hipGetLastError());
  return HFMM_OK;
}

}  // namespace hfmm

using namespace hfmm;

extern "C" {

int hfmm_matvec64(hfmm_tree* tree, double k, int32_t P, const void* x_dev, void* y_dev, void* stream) {
  try {
    if (!tree || !x_dev || !y_dev) return set_error("NULL argument"), HFMM_EINVAL;
    if (x_dev == y_dev) return set_error("x and y must not alias"), HFMM_EINVAL;
    int rc = check_kP(k, P);
    if (rc) return rc;
    Tree& t = *reinterpret_cast<Tree*>(tree);
    if (t.bie) return set_error("the FP64 variant takes point-mode handles"), HFMM_EINVAL;
    if (t.k_imag != 0.0) return set_error("the FP64 variant takes a real wavenumber"), HFMM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Plan* pl;
    if ((rc = prepare_operators(t, k, P, s, &pl))) return rc;
    return matvec64_impl(t, *pl, (const double2*)x_dev, (double2*)y_dev, s);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HFMM_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}

int hfmm_direct64(const float* src_dev, const void* q_dev, int64_t n, const float* tgt_dev, int64_t m, double k,
                  void* y_dev, void* stream) {
  if (n < 0 || m < 0) return set_error("negative size"), HFMM_EINVAL;
  if (m == 0) return HFMM_OK;
  if (!tgt_dev || !y_dev || (n > 0 && (!src_dev || !q_dev))) return set_error("NULL argument"), HFMM_EINVAL;
  if (!(k >= 0.0) || !std::isfinite(k)) return set_error("k must be finite and >= 0"), HFMM_EINVAL;
  launch64_direct(src_dev, (const double2*)q_dev, n, tgt_dev, m, k, (double2*)y_dev, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return HFMM_OK;
}

}  // extern "C"
