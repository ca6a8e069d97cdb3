// Continuous-batching server for boundary-integral solves.
//
// Solves are queued with their own BIE handle, wavenumber, right-hand side
// and tolerance.  Each step admits queued solves while slots and the device
// memory budget allow (a solve's footprint is known exactly before anything
// is allocated), then advances every active solve by one GMRES product: one
// fused FMM launch sequence for all of them, followed by each solve's FP64
// Arnoldi work (two-pass classical Gram-Schmidt, Givens update) or residual
// check.  Solves join and leave at these step boundaries; every step ends
// with one host synchronisation that reads all solves' scalars at once.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>

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

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum SolveState : int32_t {
  S_QUEUED = 0, S_ACTIVE = 1, S_CONVERGED = 2, S_NOTCONV = 3, S_STOPPED = 4, S_FAILED = -1
};
enum Phase : int { PH_RESIDUAL = 0, PH_ARNOLDI = 1 };

struct Solve {
  int64_t ticket = 0;
  Tree* t = nullptr;
  Plan* pl = nullptr;
  double k = 0, tol = 1e-4;
  int P = 10, m = 30, maxit = 2000;
  const double2* b = nullptr;
  double2* x = nullptr;
  int64_t bytes = 0;
  int state = S_QUEUED, phase = PH_RESIDUAL, j = 0, iters = 0, restarts = 0;
  double bnorm = 0, est = INFINITY, resid_true = INFINITY;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<double> restart_resid;  // true relative residual at each restart boundary
  DevBuf ws;       // GMRES workspace (one buffer)
  GmresWork W{};   // its parts
};

struct Server {
  int64_t budget = 0, used = 0;
  int max_active = 16;
  int64_t next_ticket = 1;
  std::deque<Solve*> queue;
  std::vector<Solve*> active;
  std::map<int64_t, std::unique_ptr<Solve>> solves;
  std::map<int, std::unique_ptr<Batch>> batches;  // one fused sequence per expansion order P
  bool composition_changed = true;
  // early stop (0 = off): a solve whose true residual has not fallen below
  // stall_factor times its value stall_restarts restarts earlier, or that
  // has run longer than max_seconds since admission, ends in S_STOPPED
  int stall_restarts = 0;
  double stall_factor = 0.5, max_seconds = 0.0;
  double* pinned = nullptr;  // 2 doubles per slot
  int pinned_slots = 0;
  ~Server() {
    if (pinned) (void)hipHostFree(pinned);
  }
};

static int alloc_workspace(Solve& v) {
  int rc = v.ws.alloc((size_t)gmres_workspace_bytes(v.t->npanel, v.m));
  if (rc) return rc;
  v.W = gmres_carve(v.ws.p, v.t->npanel, v.m);
  return HFMM_OK;
}

static void free_workspace(Solve& v) {
  v.ws.reset();
  v.W = GmresWork{};
}

static void mdot_chunks(int64_t n, int nv, const double2* V, const double2* w, double2* part, double2* h,
                        hipStream_t s) {
  for (int c = 0; c < nv; c += 32)
    launch_mdot(n, std::min(32, nv - c), V + (size_t)c * n, n, w, part, h + c, 0, s);
}

static void finish(Server& sv, Solve& v, int state) {
  v.state = state;
  v.t_done = now_s();
  free_workspace(v);
  sv.used -= v.bytes;
  sv.composition_changed = true;
}

// Admits queued solves while slots and memory allow; computes ||b|| for them.
static int admit(Server& sv, hipStream_t s) {
  std::vector<Solve*> fresh;
  while (!sv.queue.empty() && (int)sv.active.size() < sv.max_active) {
    Solve* v = sv.queue.front();
    if (sv.budget > 0 && sv.used + v->bytes > sv.budget && !sv.active.empty()) break;
    sv.queue.pop_front();
    int rc = prepare_device(*v->t, *v->pl, s);
    if (!rc) rc = alloc_workspace(*v);
    if (rc) {
      free_workspace(*v);
      v->state = S_FAILED;
      v->t_done = now_s();
      continue;
    }
    sv.used += v->bytes;
    v->state = S_ACTIVE;
    v->phase = PH_RESIDUAL;
    v->t_admit = now_s();
    sv.active.push_back(v);
    fresh.push_back(v);
    sv.composition_changed = true;
  }
  if (fresh.empty()) return HFMM_OK;
  if (sv.pinned_slots < sv.max_active) {
    if (sv.pinned) (void)hipHostFree(sv.pinned);
    sv.pinned = nullptr;
    HIP_TRY(hipHostMalloc((void**)&sv.pinned, (size_t)sv.max_active * 2 * sizeof(double), hipHostMallocDefault));
    sv.pinned_slots = sv.max_active;
  }
  for (Solve* v : fresh) launch_mdot(v->t->npanel, 1, v->b, v->t->npanel, v->b, v->W.part,
                                     v->W.dot, 0, s);
  for (size_t i = 0; i < fresh.size(); ++i)
    HIP_TRY(hipMemcpyAsync(sv.pinned + 2 * i, fresh[i]->W.dot, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (size_t i = 0; i < fresh.size(); ++i) fresh[i]->bnorm = std::sqrt(sv.pinned[2 * i]);
  for (Solve* v : fresh)
    if (v->bnorm == 0.0) {
      launch_zero_c128(v->t->npanel, v->x, s);
      v->resid_true = 0.0;
      v->est = 0.0;
      finish(sv, *v, S_CONVERGED);
    }
  sv.active.erase(std::remove_if(sv.active.begin(), sv.active.end(), [](Solve* v) { return v->state != S_ACTIVE; }),
                  sv.active.end());
  return HFMM_OK;
}

// Early-stop policy, checked at each restart boundary after the true
// residual is known (and recorded).
static bool stop_early(Server& sv, Solve& v) {
  v.restart_resid.push_back(v.resid_true);
  const int nr = (int)v.restart_resid.size();
  if (sv.stall_restarts > 0 && nr > sv.stall_restarts &&
      !(v.resid_true < sv.stall_factor * v.restart_resid[nr - 1 - sv.stall_restarts]))
    return true;
  return sv.max_seconds > 0.0 && now_s() - v.t_admit > sv.max_seconds;
}

static int step(Server& sv, hipStream_t s) {
  int rc = admit(sv, s);
  if (rc) return rc;
  if (sv.active.empty()) return HFMM_OK;
  // Active solves grouped by expansion order: the kernels of a fused
  // sequence are instantiated for one P, so each P present gets its own
  // sequence (in increasing P, solves in admission order within a group).
  std::map<int, std::vector<Solve*>> groups;
  for (Solve* v : sv.active) groups[v->P].push_back(v);
  if (sv.composition_changed) {
    for (auto it = sv.batches.begin(); it != sv.batches.end();)
      it = groups.count(it->first) ? std::next(it) : sv.batches.erase(it);
    for (auto& kv : groups) {
      std::vector<Tree*> tv;
      std::vector<Plan*> pv;
      for (Solve* v : kv.second) {
        tv.push_back(v->t);
        pv.push_back(v->pl);
      }
      std::unique_ptr<Batch>& b = sv.batches[kv.first];
      if (!b) b = std::make_unique<Batch>();
      if ((rc = build_batch(tv, pv, *b))) {
        sv.batches.clear();
        return rc;
      }
    }
    sv.composition_changed = false;
  }
  // inputs of this step's products: x (residual phase) or v_j (Arnoldi phase)
  for (auto& kv : groups) {
    std::vector<const float2*> xs;
    std::vector<float2*> ys;
    for (Solve* v : kv.second) {
      const double2* in = v->phase == PH_RESIDUAL ? v->x : v->W.V + (size_t)v->j * v->t->npanel;
      launch_to_c64(v->t->npanel, in, v->W.x64, s);
      xs.push_back(v->W.x64);
      ys.push_back(v->W.y64);
    }
    if ((rc = run_batch(*sv.batches[kv.first], xs.data(), ys.data(), s, false, nullptr))) return rc;
  }
  for (size_t i = 0; i < sv.active.size(); ++i) {
    Solve& v = *sv.active[i];
    Tree& t = *v.t;
    Plan& pl = *v.pl;
    const int64_t n = t.npanel;
    const double2* in = v.phase == PH_RESIDUAL ? v.x : v.W.V + (size_t)v.j * n;
    double2* out = v.phase == PH_RESIDUAL ? v.W.r : v.W.w;
    launch_near_apply(n, t.d_near_off.as<int32_t>(), t.d_near_col.as<int32_t>(), pl.d_near_val.as<float2>(),
                      nullptr, v.W.x64, v.W.y64, s);
    if (t.nystrom)  // curved elements: 6 x 6 self blocks in FP64
      launch_from_c64_self6(n, v.W.y64, pl.d_self6.as<double2>(), in, out, s);
    else
      launch_from_c64_diag(n, v.W.y64, pl.d_diag.as<double2>(), in, out, s);
    if (v.phase == PH_RESIDUAL) {
      launch_residual(n, v.b, out, s);
      launch_mdot(n, 1, out, n, out, v.W.part, v.W.dot, 0, s);
      HIP_TRY(hipMemcpyAsync(sv.pinned + 2 * i, v.W.dot, sizeof(double), hipMemcpyDeviceToHost, s));
    } else {
      double2* V = v.W.V;
      double2* w = v.W.w;
      mdot_chunks(n, v.j + 1, V, w, v.W.part, v.W.h, s);
      launch_mupdate(n, v.j + 1, V, n, v.W.h, w, -1.0, s);
      mdot_chunks(n, v.j + 1, V, w, v.W.part, v.W.h2, s);
      launch_mupdate(n, v.j + 1, V, n, v.W.h2, w, -1.0, s);
      launch_vec_add(v.j + 1, v.W.h2, v.W.h, s);
      launch_mdot(n, 1, w, n, w, v.W.part, v.W.dot, 0, s);
      launch_givens(v.j, v.m, v.W.h, v.W.dot, v.W.H, v.W.cs,
                    v.W.sn, v.W.g, v.W.st, s);
      launch_scale_by_norm(n, w, v.W.dot, V + (size_t)(v.j + 1) * n, s);
      HIP_TRY(hipMemcpyAsync(sv.pinned + 2 * i, v.W.st, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    }
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  // decisions (their launches run at the start of the next step, in stream order)
  for (size_t i = 0; i < sv.active.size(); ++i) {
    Solve& v = *sv.active[i];
    const int64_t n = v.t->npanel;
    if (v.phase == PH_RESIDUAL) {
      const double beta = std::sqrt(sv.pinned[2 * i]);
      v.resid_true = beta / v.bnorm;
      if (!std::isfinite(beta)) {
        finish(sv, v, S_FAILED);
      } else if (v.resid_true <= v.tol) {
        finish(sv, v, S_CONVERGED);
      } else if (v.iters >= v.maxit) {
        finish(sv, v, S_NOTCONV);
      } else if (stop_early(sv, v)) {
        finish(sv, v, S_STOPPED);
      } else {
        launch_scale_by_norm(n, v.W.r, v.W.dot, v.W.V, s);
        launch_init_g(v.m, v.W.dot, v.W.g, s);
        v.j = 0;
        v.phase = PH_ARNOLDI;
      }
    } else {
      v.est = sv.pinned[2 * i] / v.bnorm;
      const bool breakdown = sv.pinned[2 * i + 1] == 0.0;
      ++v.iters;
      if (!std::isfinite(v.est)) {
        finish(sv, v, S_FAILED);
      } else if (v.est <= v.tol || v.iters >= v.maxit || breakdown || v.j + 1 == v.m) {
        launch_backsolve(v.j + 1, v.m, v.W.H, v.W.g, v.W.yv, s);
        launch_mupdate(n, v.j + 1, v.W.V, n, v.W.yv, v.x, 1.0, s);
        ++v.restarts;
        v.phase = PH_RESIDUAL;
      } else {
        ++v.j;
      }
    }
  }
  HIP_TRY(hipGetLastError());
  sv.active.erase(std::remove_if(sv.active.begin(), sv.active.end(), [](Solve* v) { return v->state != S_ACTIVE; }),
                  sv.active.end());
  return HFMM_OK;
}

}  // namespace hfmm

using namespace hfmm;

extern "C" {

int hfmm_server_create(int64_t hbm_budget_bytes, int32_t max_active, hfmm_server** out) {
  if (!out || max_active < 1 || max_active > 1024 || hbm_budget_bytes < 0)
    return set_error("need 1 <= max_active <= 1024 and a budget >= 0"), HFMM_EINVAL;
  auto sv = new (std::nothrow) Server();
  if (!sv) return set_error("host allocation failed"), HFMM_ENOMEM;
  sv->budget = hbm_budget_bytes;
  sv->max_active = max_active;
  *out = reinterpret_cast<hfmm_server*>(sv);
  return HFMM_OK;
}

int hfmm_server_set_limits(hfmm_server* server, int32_t stall_restarts, double stall_factor,
                           double max_seconds) {
  if (!server || stall_restarts < 0 || !(stall_factor > 0.0 && stall_factor <= 1.0) || !(max_seconds >= 0.0))
    return set_error("need stall_restarts >= 0, 0 < stall_factor <= 1, max_seconds >= 0"), HFMM_EINVAL;
  Server& sv = *reinterpret_cast<Server*>(server);
  sv.stall_restarts = stall_restarts;
  sv.stall_factor = stall_factor;
  sv.max_seconds = max_seconds;
  return HFMM_OK;
}

int hfmm_server_submit(hfmm_server* server, hfmm_tree* tree, double k, int32_t P, const void* b_dev,
                       void* x_dev, double tol, int32_t restart, int32_t maxit, int64_t* ticket,
                       int64_t* footprint) {
  try {
    if (!server || !tree || !b_dev || !x_dev || !ticket) return set_error("NULL argument"), HFMM_EINVAL;
    Server& sv = *reinterpret_cast<Server*>(server);
    Tree& t = *reinterpret_cast<Tree*>(tree);
    if (!t.bie) return set_error("the server takes BIE handles"), HFMM_EINVAL;
    int rc = check_kP(k, P);
    if (rc) return rc;
    if (!(tol > 0.0) || restart < 1 || restart > 200 || maxit < 1)
      return set_error("need tol > 0, 1 <= restart <= 200, maxit >= 1"), HFMM_EINVAL;
    if (!sv.active.empty() || !sv.queue.empty())
      for (auto& kv : sv.solves)
        if (kv.second->t == &t && (kv.second->state == S_QUEUED || kv.second->state == S_ACTIVE))
          return set_error("this handle already has a solve in flight"), HFMM_EINVAL;
    Plan* pl;
    if ((rc = prepare_host(t, k, P, &pl))) return rc;
    auto v = std::make_unique<Solve>();
    v->ticket = sv.next_ticket++;
    v->t = &t;
    v->pl = pl;
    v->k = k;
    v->P = P;
    v->tol = tol;
    v->m = restart;
    v->maxit = maxit;
    v->b = (const double2*)b_dev;
    v->x = (double2*)x_dev;
    v->bytes = (pl->device_ready ? 0 : pl->est_bytes) + gmres_workspace_bytes(t.npanel, restart);
    if (sv.budget > 0 && v->bytes > sv.budget) return set_error("solve exceeds the memory budget"), HFMM_ENOMEM;
    v->t_submit = now_s();
    *ticket = v->ticket;
    if (footprint) *footprint = v->bytes;
    sv.queue.push_back(v.get());
    sv.solves[v->ticket] = std::move(v);
    return HFMM_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HFMM_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}

int hfmm_server_step(hfmm_server* server, void* stream, int32_t* n_active, int32_t* n_queued) {
  try {
    if (!server) return set_error("NULL server"), HFMM_EINVAL;
    Server& sv = *reinterpret_cast<Server*>(server);
    int rc = step(sv, (hipStream_t)stream);
    if (n_active) *n_active = (int32_t)sv.active.size();
    if (n_queued) *n_queued = (int32_t)sv.queue.size();
    return rc;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HFMM_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}

int hfmm_server_poll(hfmm_server* server, int64_t ticket, int32_t* state, hfmm_gmres_info* info,
                     double* times3) {
  if (!server || !state) return set_error("NULL argument"), HFMM_EINVAL;
  Server& sv = *reinterpret_cast<Server*>(server);
  auto it = sv.solves.find(ticket);
  if (it == sv.solves.end()) return set_error("unknown ticket"), HFMM_EINVAL;
  const Solve& v = *it->second;
  *state = v.state;
  if (info) {
    info->iters = v.iters;
    info->restarts = v.restarts;
    info->resid_est = v.est;
    info->resid_true = v.resid_true;
    info->seconds = v.t_done > 0 ? v.t_done - v.t_admit : 0.0;
  }
  if (times3) {
    times3[0] = v.t_submit;
    times3[1] = v.t_admit;
    times3[2] = v.t_done;
  }
  return HFMM_OK;
}

int hfmm_server_release(hfmm_server* server, int64_t ticket) {
  if (!server) return set_error("NULL server"), HFMM_EINVAL;
  Server& sv = *reinterpret_cast<Server*>(server);
  auto it = sv.solves.find(ticket);
  if (it == sv.solves.end()) return set_error("unknown ticket"), HFMM_EINVAL;
  if (it->second->state == S_QUEUED || it->second->state == S_ACTIVE)
    return set_error("solve still in flight"), HFMM_EINVAL;
  sv.solves.erase(it);
  return HFMM_OK;
}

int hfmm_server_used_bytes(hfmm_server* server, int64_t* used) {
  if (!server || !used) return set_error("NULL argument"), HFMM_EINVAL;
  *used = reinterpret_cast<Server*>(server)->used;
  return HFMM_OK;
}

void hfmm_server_free(hfmm_server* server) { delete reinterpret_cast<Server*>(server); }

}  // extern "C"
