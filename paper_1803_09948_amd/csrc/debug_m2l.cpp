// Test hook: one M2L translation through the product's own kernels, so the
// matrix-core M2L can be checked coefficient by coefficient.
#include <cmath>
#include <cstring>

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

// `count` columns, column c a pair (target c, source c, reflection g_c) of
// one canonical operator: the table from k_gen_tables, the pair records and
// chunks as a plan lays them out, staging slots in column order, then the
// reduction into out.
static int debug_m2l(int P, double k, double ki, const double* t, double rho_in, double rho_out, int count,
                     const int32_t* refl, const float2* in, float2* out, hipStream_t s) {
  int Sm, St;
  stage_dims(P, &Sm, &St);
  const int P2 = P * P;
  OpDesc d{};
  for (int i = 0; i < 3; ++i) d.t[i] = t[i];
  d.rho_in = rho_in;
  d.rho_out = rho_out;
  d.kind = OP_M2L;
  const Coupling& cp = coupling(P);
  std::vector<double2> cv(cp.re.size());
  for (size_t i = 0; i < cv.size(); ++i) cv[i] = make_double2(cp.re[i], cp.im[i]);
  std::vector<int4> pairs(count), chunks;
  std::vector<uint8_t> slot_g(count);
  std::vector<int32_t> soff(count + 1);
  std::vector<int2> red(count);
  for (int c = 0; c < count; ++c) {
    pairs[c] = make_int4(c, c, refl[c], c);
    slot_g[c] = (uint8_t)refl[c];
    soff[c] = c;
    red[c] = make_int2(0, c);
  }
  soff[count] = count;
  const int CH = m2l_pairs_per_chunk(P);
  for (int b = 0; b < count; b += CH) chunks.push_back(make_int4(0, 0, b, std::min(count, b + CH)));
  std::vector<int32_t> bmap, omap;
  m2l_xz_codes(P, bmap, omap);
  DevBuf d_ops, d_off, d_lm, d_val, d_tab, d_pairs, d_chunks, d_slotg, d_soff, d_red, d_bmap, d_omap, d_stage, d_inst,
      d_min;
  int rc;
  // the product stores multipoles in mpos order: reorder the caller's columns
  std::vector<float2> hin((size_t)count * P2), hperm((size_t)count * P2);
  HIP_TRY(hipMemcpyAsync(hin.data(), in, hin.size() * sizeof(float2), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int c = 0; c < count; ++c)
    for (int n = 0; n < P; ++n)
      for (int m = -n; m <= n; ++m)
        hperm[(size_t)c * P2 + mpos(P, n, m)] = hin[(size_t)c * P2 + n * n + n + m];
  if ((rc = upload_vec(d_min, hperm))) return rc;
  if ((rc = upload_vec(d_ops, std::vector<OpDesc>{d})) || (rc = upload_vec(d_off, cp.off)) ||
      (rc = upload_vec(d_lm, cp.lm)) || (rc = upload_vec(d_val, cv)) || (rc = upload_vec(d_pairs, pairs)) ||
      (rc = upload_vec(d_chunks, chunks)) || (rc = upload_vec(d_slotg, slot_g)) || (rc = upload_vec(d_soff, soff)) ||
      (rc = upload_vec(d_red, red)) || (rc = upload_vec(d_bmap, bmap)) || (rc = upload_vec(d_omap, omap)) ||
      (rc = d_tab.alloc((size_t)xz_table_stride(P) * sizeof(float2))) ||
      (rc = d_stage.alloc((size_t)count * (Sm + St) * sizeof(float2))))
    return rc;
  InstDev I{};
  I.tables = d_tab.as<float2>();
  I.M = d_min.as<float2>();
  I.L = out;
  I.m2l_pairs = d_pairs.as<int4>();
  I.stage = d_stage.as<float2>();
  I.stage_tail = I.stage + (size_t)count * Sm;
  I.slot_g = d_slotg.as<uint8_t>();
  I.m2l_soff = d_soff.as<int32_t>();
  I.ncellP2 = (int64_t)count * P2;
  I.k = (float)k;
  I.ki = (float)ki;
  if ((rc = upload_vec(d_inst, std::vector<InstDev>{I}))) return rc;
  launch_gen_tables(d_ops.as<OpDesc>(), 1, P, k, ki, d_off.as<int32_t>(), d_lm.as<int32_t>(), d_val.as<double2>(),
                    d_tab.as<float2>(), s);
  launch_m2l(d_chunks.as<int4>(), (int)chunks.size(), d_inst.as<InstDev>(), d_bmap.as<int32_t>(), P, 0, s);
  launch_m2l_reduce(d_red.as<int2>(), count, d_inst.as<InstDev>(), d_omap.as<int32_t>(), P, 0, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));  // the local buffers are freed on return
  return HFMM_OK;
}

}  // namespace hfmm

using namespace hfmm;

extern "C" int hfmm_debug_m2l(int32_t P, double k, double k_imag, const double* t_host, double rho_in,
                              double rho_out, int32_t count, const int32_t* refl_host, const void* in_dev,
                              void* out_dev, void* stream) {
  try {
    int rc = check_kP(k, P);
    if (rc) return rc;
    if (!t_host || !refl_host || !in_dev || !out_dev || count < 1 || count > (1 << 20))
      return set_error("need t, refl, in, out and 1 <= count <= 2^20"), HFMM_EINVAL;
    if (!(t_host[0] >= t_host[1] && t_host[1] >= 0.0 && t_host[2] >= 0.0) ||
        !(t_host[0] * t_host[0] + t_host[1] * t_host[1] + t_host[2] * t_host[2] > 0.0))
      return set_error("t must be canonical and nonzero: t0 >= t1 >= 0, t2 >= 0"), HFMM_EINVAL;
    if (!(k_imag >= 0.0) || !std::isfinite(k_imag) || !(rho_in > 0.0 && rho_in <= 1.0) ||
        !(rho_out > 0.0 && rho_out <= 1.0))
      return set_error("need k_imag >= 0 and 0 < rho <= 1"), HFMM_EINVAL;
    for (int c = 0; c < count; ++c)
      if (refl_host[c] < 0 || refl_host[c] > 15) return set_error("reflection codes are 0..15"), HFMM_EINVAL;
    if (in_dev == out_dev) return set_error("in and out must not alias"), HFMM_EINVAL;
    return debug_m2l(P, k, k_imag, t_host, rho_in, rho_out, count, refl_host, (const float2*)in_dev,
                     (float2*)out_dev, (hipStream_t)stream);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HFMM_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}
