// GMRES without device allocation: hfmm_gmres_solve_noalloc runs the same
// solver as hfmm_gmres_solve, with the Krylov workspace taken from a static
// device array instead of library-allocated memory.
#include <cstring>
#include <mutex>

#include "hfmm_internal.h"

namespace hfmm {

// The Krylov workspace of hfmm_gmres_solve_noalloc (see kScratchBytes); each
// device holds its own copy for the life of the process.
constexpr size_t kScratchBytes = size_t(72) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (host code must never pass the array's name itself: on the host
// it is only a stand-in for the device symbol).
static int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return HFMM_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index out of range for the static scratch table");
    return HFMM_EINTERNAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return HFMM_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HFMM_OK;
}

}  // namespace hfmm

using namespace hfmm;

extern "C" int hfmm_gmres_solve_noalloc(hfmm_tree* tree, double k, int32_t P, const void* b, void* x, double tol,
                                        int32_t restart, int32_t maxit, hfmm_gmres_info* info, void* stream) {
  try {
    if (!tree || !b || !x) return set_error("NULL argument"), HFMM_EINVAL;
    Tree& t = *reinterpret_cast<Tree*>(tree);
    if (!t.bie) return set_error("GMRES needs a BIE handle"), HFMM_EINVAL;
    int rc = check_kP(k, P);
    if (rc) return rc;
    if (!(tol > 0.0) || restart < 1 || restart > 200 || maxit < 1)
      return set_error("need tol > 0, 1 <= restart <= 200, maxit >= 1"), HFMM_EINVAL;
    const int64_t need = gmres_workspace_bytes(t.npanel, restart);
    if (need > (int64_t)kScratchBytes)
      return set_error("GMRES workspace of " + std::to_string(need) + " bytes exceeds the static scratch of " +
                       std::to_string(kScratchBytes) + " bytes (fewer unknowns or a smaller restart)"),
             HFMM_ENOMEM;
    // the product must already be prepared: preparing would allocate
    uint64_t kb;
    std::memcpy(&kb, &k, 8);
    auto it = t.plans.find(std::make_pair(kb, (int)P));
    if (it == t.plans.end() || !it->second->device_ready || !it->second->self || !it->second->self->side)
      return set_error("(k, P) is not prepared on this handle: call hfmm_prepare first"), HFMM_EINVAL;
    void* base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    const GmresWork W = gmres_carve(base, t.npanel, restart);
    return gmres_run(t, *it->second, W, restart, (const double2*)b, (double2*)x, tol, maxit, info,
                     (hipStream_t)stream, nullptr);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HFMM_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}
