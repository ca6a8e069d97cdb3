// Entry points not yet implemented (temporary).
#include "hfmm_internal.h"
using namespace hfmm;
extern "C" {
int hfmm_build_bie(const double*, int64_t, const int32_t*, int64_t, const hfmm_opts*, hfmm_tree** out) {
  if (out) *out = nullptr;
  set_error("not implemented");
  return HFMM_EINTERNAL;
}
int hfmm_gmres_solve(hfmm_tree*, double, int32_t, const void*, void*, double, int32_t, int32_t,
                     hfmm_gmres_info*, void*) {
  set_error("not implemented");
  return HFMM_EINTERNAL;
}
int hfmm_bie_plane_wave(hfmm_tree*, double, const double*, void*, void*) {
  set_error("not implemented");
  return HFMM_EINTERNAL;
}
int hfmm_batch_matvec(int32_t, hfmm_tree* const*, const double*, const int32_t*, const void* const*,
                      void* const*, void*) {
  set_error("not implemented");
  return HFMM_EINTERNAL;
}
}
