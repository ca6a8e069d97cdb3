// Fused execution of FMM matvecs over one or many instances.
//
// Every kernel is instance-aware: a work item names its instance, whose
// pointers come from a device table.  A batch therefore only concatenates the
// per-instance work lists (cells, M2L chunks, P2P work); tables, bodies and
// expansions stay where each instance's plan put them.  The whole sequence is
// one launch per phase and level for all instances together, and can be
// captured once as a hipGraph and replayed.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

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

Batch::~Batch() {
  for (hipEvent_t e : ev_m2l) (void)hipEventDestroy(e);
  for (hipEvent_t e : ev_red) (void)hipEventDestroy(e);
  if (red) (void)hipStreamDestroy(red);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ev_in) (void)hipEventDestroy(ev_in);
  if (ev_out) (void)hipEventDestroy(ev_out);
  if (stream) (void)hipStreamDestroy(stream);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (side) (void)hipStreamDestroy(side);
}

static InstDev make_inst(Tree& t, Plan& pl) {
  InstDev I{};
  I.spos = t.d_src_pos.as<float4>();
  I.tpos = t.d_tgt_pos.as<float4>();
  I.src_idx = t.d_src_idx.as<int32_t>();
  I.src_w = t.bie ? t.d_src_w.as<float>() : nullptr;
  I.tgt_perm = t.d_tgt_perm.as<int32_t>();
  I.q = t.d_q.as<float2>();
  I.ys = t.d_ys.as<float2>();
  I.cells = pl.d_cells.as<int4>();
  I.geo = pl.d_geo.as<float4>();
  I.clev = pl.d_clev.as<int32_t>();
  I.topo = pl.d_topo.as<int4>();
  I.cops = pl.d_cops.as<int2>();
  I.rho = pl.d_rho.as<double>();
  I.tables = pl.d_tables.as<float2>();
  I.M = pl.d_M.as<float2>();
  I.L = pl.d_L.as<float2>();
  I.m2l_pairs = pl.d_m2l_pairs.as<int4>();
  {
    int Sm, St;
    stage_dims(pl.P, &Sm, &St);
    I.stage = pl.d_stage.as<float2>();  // [slots][Sm], then the tails [slots][St]
    I.stage_tail = I.stage + pl.stage_bufs * std::max<int64_t>(1, pl.max_seg_slots) * Sm;
  }
  I.slot_g = pl.d_slot_g.as<uint8_t>();
  I.m2l_soff = pl.d_m2l_soff.as<int32_t>();
  I.p2p_work = pl.d_p2p_work.as<int4>();
  I.p2p_ivals = pl.d_p2p_ivals.as<int2>();
  I.p2p_total = pl.d_p2p_total.as<int32_t>();
  I.nsrc = pl.ct.nsrc;
  I.ntgt = pl.ct.ntgt;
  I.ncellP2 = (int64_t)pl.ct.ncell() * pl.P * pl.P;
  I.k = (float)pl.k;
  I.ki = (float)pl.ki;
  return I;
}

template <class T>
static int up(DevBuf& b, const std::vector<T>& v) {
  return upload_vec(b, v, true);
}

int build_batch(const std::vector<Tree*>& trees, const std::vector<Plan*>& plans, Batch& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  b.count = (int)trees.size();
  b.P = plans[0]->P;
  // the kernels of one sequence are instantiated for one P, and each
  // instance gathers, accumulates and scatters through its tree's own
  // buffers: differing P or a tree that appears twice cannot share a batch
  for (int i = 0; i < b.count; ++i) {
    if (plans[i]->P != b.P) {
      set_error("all instances of a fused batch need the same P");
      return HFMM_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (trees[j] == trees[i]) {
        set_error("a tree handle appears twice in one fused batch");
        return HFMM_EINVAL;
      }
  }
  b.trees = trees;
  b.plans = plans;
  b.hinst.clear();
  b.damped = false;
  const int ch = elem_chunk();
  std::vector<int2> zero, gather, scatter, p2m, l2p, p2p, red;
  std::vector<int4> m2l;
  b.maxlev = 0;
  for (int i = 0; i < b.count; ++i) {
    Plan& pl = *plans[i];
    b.hinst.push_back(make_inst(*trees[i], pl));
    b.damped = b.damped || pl.ki != 0.0;
    b.maxlev = std::max(b.maxlev, pl.ct.nlevels());
    const InstDev& I = b.hinst.back();
    for (int64_t e = 0; e * ch < std::max<int64_t>(I.ncellP2, I.ntgt); ++e) zero.push_back(make_int2(i, (int)e));
    for (int64_t e = 0; e * ch < I.nsrc; ++e) gather.push_back(make_int2(i, (int)e));
    for (int64_t e = 0; e * ch < I.ntgt; ++e) scatter.push_back(make_int2(i, (int)e));
    for (int c : pl.src_leaves) p2m.push_back(make_int2(i, c));
    for (int c : pl.tgt_leaves) l2p.push_back(make_int2(i, c));
    for (int w = 0; w < pl.n_p2p_work; ++w) p2p.push_back(make_int2(i, w));
  }
  // M2L chunks and reduction items, segment by segment (several staging
  // segments are allowed for a single instance only)
  b.nseg = 1;
  for (int i = 0; i < b.count; ++i) b.nseg = std::max(b.nseg, (int)plans[i]->m2l_segs.size());
  if (b.nseg > 1 && b.count > 1) {
    set_error("an instance whose M2L staging exceeds its budget cannot join a fused batch");
    return HFMM_EINVAL;
  }
  b.m2l_seg_off.assign(b.nseg + 1, 0);
  b.red_seg_off.assign(b.nseg + 1, 0);
  b.seg_slot_base.assign(b.nseg, 0);
  for (int sg = 0; sg < b.nseg; ++sg) {
    b.m2l_seg_off[sg] = (int)m2l.size();
    b.red_seg_off[sg] = (int)red.size();
    for (int i = 0; i < b.count; ++i) {
      const Plan& pl = *plans[i];
      if (sg >= (int)pl.m2l_segs.size()) continue;
      const M2LSeg& S = pl.m2l_segs[sg];
      for (int c = S.chunk_b; c < S.chunk_e; ++c) {
        const int4& ch = pl.m2l_chunks_h[c];
        m2l.push_back(make_int4(i, ch.x, ch.y, ch.z));
      }
      for (int t = S.tgt_b; t < S.tgt_e; ++t) red.push_back(make_int2(i, pl.m2l_targets[t]));
      // the reduction finds slot g of the segment at staging position
      // g - base: the segment's buffer holds its slots from slot_b on
      if (b.count == 1) b.seg_slot_base[sg] = S.slot_b - (int64_t)(sg % pl.stage_bufs) * pl.max_seg_slots;
    }
  }
  b.m2l_seg_off[b.nseg] = (int)m2l.size();
  b.red_seg_off[b.nseg] = (int)red.size();
  // per-level M2M (parents, deepest first) and L2L (children, root first)
  // items: up to 16 destination cells of one instance, level (and, for L2L,
  // octant) per item
  std::vector<int4> m2m, l2l;
  std::vector<int32_t> m2m_cols, l2l_cols;
  b.m2m_off.assign(b.maxlev + 1, 0);
  b.l2l_off.assign(b.maxlev + 1, 0);
  for (int l = 0; l < b.maxlev; ++l) {
    b.m2m_off[l] = (int)m2m.size();
    b.l2l_off[l] = (int)l2l.size();
    for (int i = 0; i < b.count; ++i) {
      Plan& pl = *plans[i];
      const HostTree& h = pl.ct;
      auto octant = [&](int c) {
        return (h.ijk[3 * c] & 1) | ((h.ijk[3 * c + 1] & 1) << 1) | ((h.ijk[3 * c + 2] & 1) << 2);
      };
      if (l < (int)pl.m2m_cells.size() && !pl.m2m_cells[l].empty()) {
        const std::vector<int>& par = pl.m2m_cells[l];
        for (size_t j = 0; j < par.size(); j += 16) {
          const int cnt = (int)std::min<size_t>(16, par.size() - j);
          m2m.push_back(make_int4(i, pl.m2m_base[l + 1], (int)(m2m_cols.size() / 9), cnt));
          for (int u = 0; u < cnt; ++u) {
            const int p = par[j + u];
            int ch[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
            for (int c = h.cb[p]; c < h.ce[p]; ++c) ch[octant(c)] = c;
            m2m_cols.push_back(p);
            m2m_cols.insert(m2m_cols.end(), ch, ch + 8);
          }
        }
      }
      if (l < (int)pl.l2l_cells.size() && !pl.l2l_cells[l].empty()) {
        std::vector<int> by[8];
        for (int c : pl.l2l_cells[l]) by[octant(c)].push_back(c);
        for (int o = 0; o < 8; ++o)
          for (size_t j = 0; j < by[o].size(); j += 16) {
            const int cnt = (int)std::min<size_t>(16, by[o].size() - j);
            l2l.push_back(make_int4(i, pl.l2l_base[l] + o, (int)(l2l_cols.size() / 2), cnt));
            for (int u = 0; u < cnt; ++u) {
              l2l_cols.push_back(by[o][j + u]);
              l2l_cols.push_back(h.parent[by[o][j + u]]);
            }
          }
      }
    }
  }
  b.m2m_off[b.maxlev] = (int)m2m.size();
  b.l2l_off[b.maxlev] = (int)l2l.size();
  int rc;
  if ((rc = up(b.d_inst, b.hinst)) || (rc = up(b.d_zero, zero)) || (rc = up(b.d_gather, gather)) ||
      (rc = up(b.d_scatter, scatter)) || (rc = up(b.d_p2m, p2m)) || (rc = up(b.d_l2p, l2p)) ||
      (rc = up(b.d_p2p, p2p)) || (rc = up(b.d_m2l, m2l)) || (rc = up(b.d_m2m, m2m)) || (rc = up(b.d_l2l, l2l)) ||
      (rc = up(b.d_m2m_cols, m2m_cols)) || (rc = up(b.d_l2l_cols, l2l_cols)) ||
      (rc = up(b.d_red, red)))
    return rc;
  b.n_zero = (int)zero.size();
  b.n_gather = (int)gather.size();
  b.n_scatter = (int)scatter.size();
  b.n_p2m = (int)p2m.size();
  b.n_l2p = (int)l2p.size();
  b.n_p2p = (int)p2p.size();
  b.n_m2l = (int)m2l.size();
  b.n_red = (int)red.size();
  return HFMM_OK;
}

// The fused sequence: zero (M, L and the sorted outputs), gather, P2M, M2M
// (levels up), M2L and its reduction, L2L (levels down) on `s`, with P2P on
// the side stream, forked either right after the gather (beside the whole
// far field) or after the first M2L launch (beside the reduction, which
// leaves the vector units idle); L2P waits for P2P and adds the far field
// to its sums; scatter.  The P2P variant (autotuned) is its launch shape
// and its fork point.  P2P and L2P each add into ys in this order on every
// path.  With `ev`
// (phase timing) everything runs on `s`, one phase after another, and the
// events bracket the phases.  Without `io` the gather from the caller's
// vectors and the scatter into them are left out (the autotuner's runs, which
// may come before any caller vector is bound; every other step reads and
// writes only the batch's own buffers).
static int sequence(Batch& b, hipStream_t s, hipEvent_t* ev, bool io = true) {
  const InstDev* I = b.d_inst.as<InstDev>();
  const int P = b.P;
  const Plan& p0 = *b.plans[0];
  auto mark = [&](int i) -> int {
    if (ev) HIP_TRY(hipEventRecord(ev[i], s));
    return HFMM_OK;
  };
  int rc;
  if ((rc = mark(0))) return rc;
  launch_zero(b.d_zero.as<int2>(), b.n_zero, I, s);
  if (io) launch_gather(b.d_gather.as<int2>(), b.n_gather, I, s);
  const bool fork = !ev;
  const int p2p_v = batch_variant(b, kPhaseP2P), p2p_shape = p2p_v % p2p_variant_count();
  const bool late_fork = p2p_v >= p2p_variant_count();
  auto fork_p2p = [&]() -> int {
    HIP_TRY(hipEventRecord(b.ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(b.side, b.ev_fork, 0));
    launch_p2p(b.d_p2p.as<int2>(), b.n_p2p, I, b.damped, p2p_shape, b.side);
    HIP_TRY(hipEventRecord(b.ev_join, b.side));
    return HFMM_OK;
  };
  if (fork && !late_fork && (rc = fork_p2p())) return rc;
  launch_p2m(b.d_p2m.as<int2>(), b.n_p2m, I, P, b.damped, s);
  if ((rc = mark(1))) return rc;
  for (int l = b.maxlev - 2; l >= 0; --l)
    launch_m2m(b.d_m2m.as<int4>() + b.m2m_off[l], b.m2m_off[l + 1] - b.m2m_off[l], b.d_m2m_cols.as<int32_t>(), I,
               P, s);
  if ((rc = mark(2))) return rc;
  // M2L and its reduction per staging segment (marks 3 and 4 split the two
  // phases when there is one segment; with several, phase 3 holds both).
  // With several segments (and no phase timing) the reduction of segment
  // sg runs on the reduction stream beside the M2L of segment sg + 1; the
  // two staging buffers alternate, so the M2L of segment sg waits for the
  // reduction of segment sg - 2, and the L2L waits for every reduction.
  const bool overlap = fork && b.nseg > 1;
  for (int sg = 0; sg < b.nseg; ++sg) {
    if (overlap && sg >= 2) HIP_TRY(hipStreamWaitEvent(s, b.ev_red[sg - 2], 0));
    launch_m2l(b.d_m2l.as<int4>() + b.m2l_seg_off[sg], b.m2l_seg_off[sg + 1] - b.m2l_seg_off[sg], I,
               p0.d_bmap.as<int32_t>(), P, batch_variant(b, kPhaseM2L), s);
    if (fork && late_fork && sg == 0 && (rc = fork_p2p())) return rc;
    if (b.nseg == 1 && (rc = mark(3))) return rc;
    hipStream_t rs = s;
    if (overlap) {
      HIP_TRY(hipEventRecord(b.ev_m2l[sg], s));
      HIP_TRY(hipStreamWaitEvent(b.red, b.ev_m2l[sg], 0));
      rs = b.red;
    }
    launch_m2l_reduce(b.d_red.as<int2>() + b.red_seg_off[sg], b.red_seg_off[sg + 1] - b.red_seg_off[sg], I,
                      p0.d_omap.as<int32_t>(), P, b.seg_slot_base[sg], rs);
    if (overlap) HIP_TRY(hipEventRecord(b.ev_red[sg], b.red));
  }
  if (overlap)
    for (int sg = std::max(0, b.nseg - 2); sg < b.nseg; ++sg) HIP_TRY(hipStreamWaitEvent(s, b.ev_red[sg], 0));
  if (b.nseg > 1 && (rc = mark(3))) return rc;
  if ((rc = mark(4))) return rc;
  for (int l = 1; l < b.maxlev; ++l)
    launch_l2l(b.d_l2l.as<int4>() + b.l2l_off[l], b.l2l_off[l + 1] - b.l2l_off[l], b.d_l2l_cols.as<int32_t>(), I,
               P, s);
  if ((rc = mark(5))) return rc;
  if (fork) {
    HIP_TRY(hipStreamWaitEvent(s, b.ev_join, 0));
  } else {
    launch_p2p(b.d_p2p.as<int2>(), b.n_p2p, I, b.damped, p2p_shape, s);
  }
  if ((rc = mark(6))) return rc;
  launch_l2p(b.d_l2p.as<int2>(), b.n_l2p, I, P, b.damped, s);
  if ((rc = mark(7))) return rc;
  if (io) launch_scatter(b.d_scatter.as<int2>(), b.n_scatter, I, s);
  HIP_TRY(hipGetLastError());
  return HFMM_OK;
}

// ---------------------------------------------------------------------------
// Autotuner.  Shapes of a phase compute identical results; the first run of
// a batch times every shape of each phase on the batch's own work (eagerly,
// outside any capture) and keeps the fastest.  The M2L shapes are timed
// alone (the M2L only writes its staging slots, which the real sequence
// overwrites).  The P2P runs beside the far field, and a shape that is
// faster alone can share the GPU worse, so its variants (launch shape and
// fork point) are timed inside the whole sequence without the caller's
// vectors (sequence with io off; the real sequence clears what those runs
// wrote).  Choices are cached per
// (phase, P, log2 of the phase's work items), so rebuilt batches of similar
// size do not time again.
// ---------------------------------------------------------------------------
static std::atomic<int> g_override[kNumTunedPhases] = {{-1}, {-1}, {-1}};
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, int> g_tuned;
static bool g_tuned_loaded = false;

int phase_variant_count(int phase, int P) {
  if (P < 1 || P > kMaxP) return 0;
  if (phase == kPhaseM2L) return m2l_variant_count(P);
  if (phase == kPhaseP2P) return 2 * p2p_variant_count();  // launch shape x fork point
  if (phase == kPhaseNear) return 2;                       // near corrections after / beside the FMM
  return 0;
}

// Persistent choices: with HFMM_TUNE_CACHE naming a file, the choices are
// read from it once (lines "phase P log2size variant") and every new choice
// is appended, so later processes skip the timing.  Unreadable or malformed
// lines are ignored.  Call with g_tune_mu held.
static const char* tune_cache_path() {
  const char* p = std::getenv("HFMM_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}
static void tune_cache_load() {
  if (g_tuned_loaded) return;
  g_tuned_loaded = true;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int ph, P, lg, v;
  while (std::fscanf(f, "%d %d %d %d", &ph, &P, &lg, &v) == 4)
    if (ph >= 0 && ph < kNumBatchPhases && v >= 0 && v < phase_variant_count(ph, P))
      g_tuned[std::make_tuple(ph, P, lg)] = v;
  std::fclose(f);
}
static void tune_cache_append(int ph, int P, int lg, int v) {
  const char* path = tune_cache_path();
  if (!path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%d %d %d %d\n", ph, P, lg, v);
    std::fclose(f);
  }
}

int set_variant_override(int phase, int variant) {
  if (phase < 0 || phase >= kNumTunedPhases || variant < -1) return set_error("bad phase or variant"), HFMM_EINVAL;
  g_override[phase].store(variant);
  return HFMM_OK;
}

int variant_override(int phase) { return phase >= 0 && phase < kNumTunedPhases ? g_override[phase].load() : -1; }

int batch_variant(const Batch& b, int phase) {
  if (phase < 0 || phase >= kNumBatchPhases) return 0;
  const int o = g_override[phase].load();
  if (o >= 0 && o < phase_variant_count(phase, b.P)) return o;
  return b.variant[phase] < 0 ? 0 : b.variant[phase];
}

// Times the shapes of one phase (launch(v) enqueues work that runs shape v
// of the phase on s and returns a status): one warm-up round, then `timed`
// rounds, each shape scored by its fastest round; records the fastest shape
// in b.variant[phase].  A timed round runs each shape's work reps times in a
// row, reps sized from the warm-up round so that a round spans about 2 ms
// (short products would otherwise be ranked by launch jitter).
template <class Launch>
static int tune_phase(Batch& b, int phase, int nwork, int timed, Launch launch, hipStream_t s) {
  const int nv = phase_variant_count(phase, b.P);
  if (b.variant[phase] >= 0 || g_override[phase].load() >= 0) return HFMM_OK;
  if (nv <= 1 || nwork == 0) {
    b.variant[phase] = 0;
    return HFMM_OK;
  }
  int lg = 0;
  while ((1 << (lg + 1)) <= nwork) ++lg;
  const auto key = std::make_tuple(phase, b.P, lg);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      b.variant[phase] = it->second;
      return HFMM_OK;
    }
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::vector<float> score(nv, 0.f);
  int rc = HFMM_OK, reps = 1;
  for (int rep = 0; rep <= timed && rc == HFMM_OK; ++rep) {  // the first round warms caches and code
    if (rep == 1) {
      const float fastest = *std::min_element(score.begin(), score.end());
      reps = fastest >= 2.f ? 1 : std::min(64, (int)std::ceil(2.f / std::max(fastest, 0.03f)));
    }
    for (int v = 0; v < nv && rc == HFMM_OK; ++v) {
      hipError_t e = hipEventRecord(e0, s);
      for (int r = 0; r < reps && e == hipSuccess; ++r) {
        if ((rc = launch(v))) break;
        e = hipGetLastError();
      }
      if (rc) break;
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        set_error(std::string("autotuner: ") + hipGetErrorString(e));
        rc = HFMM_EHIP;
        break;
      }
      ms /= (float)reps;
      if (rep <= 1 || ms < score[v]) score[v] = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  int pick = 0;
  for (int v = 1; v < nv; ++v)
    if (score[v] < score[pick]) pick = v;
  b.variant[phase] = pick;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = pick;
  tune_cache_append(phase, b.P, lg, pick);
  return HFMM_OK;
}

static int tune_batch(Batch& b, hipStream_t s) {
  const InstDev* I = b.d_inst.as<InstDev>();
  int rc = tune_phase(
      b, kPhaseM2L, b.n_m2l, 1,
      [&](int v) {
        launch_m2l(b.d_m2l.as<int4>(), b.m2l_seg_off[1], I, b.plans[0]->d_bmap.as<int32_t>(), b.P, v, s);
        return (int)HFMM_OK;
      },
      s);
  if (rc) return rc;
  return tune_phase(
      b, kPhaseP2P, b.n_p2p, 2,
      [&](int v) {
        b.variant[kPhaseP2P] = v;
        const int r = sequence(b, s, nullptr, false);
        b.variant[kPhaseP2P] = -1;
        return r;
      },
      s);
}

int ready_batch(Batch& b, hipStream_t s) {
  if (!b.side) {
    HIP_TRY(hipStreamCreateWithFlags(&b.side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&b.ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&b.ev_join, hipEventDisableTiming));
  }
  if (b.nseg > 1) {
    if (!b.red) HIP_TRY(hipStreamCreateWithFlags(&b.red, hipStreamNonBlocking));
    for (int sg = (int)b.ev_m2l.size(); sg < b.nseg; ++sg) {
      hipEvent_t e1, e2;
      HIP_TRY(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
      b.ev_m2l.push_back(e1);
      HIP_TRY(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
      b.ev_red.push_back(e2);
    }
  }
  return tune_batch(b, s);
}

int run_batch(Batch& b, const float2* const* xs, float2* const* ys, hipStream_t s, bool use_graph,
              Tree* timing) {
  for (int base = 0; base < b.count; base += 64) {
    XYPtrs p{};
    const int n = std::min(64, b.count - base);
    for (int i = 0; i < n; ++i) {
      p.x[i] = xs[base + i];
      p.y[i] = ys[base + i];
    }
    launch_set_xy(n, base, p, b.d_inst.as<InstDev>(), s);
  }
  HIP_TRY(hipGetLastError());
  int rc = ready_batch(b, s);
  if (rc) return rc;
  b.ran = true;
  if (!use_graph) return sequence(b, s, timing ? timing->ev : nullptr);
  if (!b.stream) {
    HIP_TRY(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&b.ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&b.ev_out, hipEventDisableTiming));
  }
  bool stale = false;  // a shape forced since capture
  for (int ph = 0; ph < kNumBatchPhases; ++ph) stale = stale || b.graph_variant[ph] != batch_variant(b, ph);
  if (b.exec && stale) {
    (void)hipGraphExecDestroy(b.exec);
    (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
  }
  if (!b.exec) {
    HIP_TRY(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
    for (int ph = 0; ph < kNumBatchPhases; ++ph) b.graph_variant[ph] = batch_variant(b, ph);
    rc = sequence(b, b.stream, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b.stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) {
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      return HFMM_EHIP;
    }
    b.graph = g;
    HIP_TRY(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
  }
  HIP_TRY(hipEventRecord(b.ev_in, s));
  HIP_TRY(hipStreamWaitEvent(b.stream, b.ev_in, 0));
  HIP_TRY(hipGraphLaunch(b.exec, b.stream));
  HIP_TRY(hipEventRecord(b.ev_out, b.stream));
  HIP_TRY(hipStreamWaitEvent(s, b.ev_out, 0));
  return HFMM_OK;
}

// Batches built by hfmm_batch_matvec, keyed by the instances' (uid, k, P).
static std::mutex g_batch_mu;
static std::map<std::vector<uint64_t>, std::unique_ptr<Batch>> g_batches;

void forget_tree_batches(uint64_t uid) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (auto it = g_batches.begin(); it != g_batches.end();) {
    bool uses = false;
    for (size_t i = 0; i < it->first.size(); i += 3) uses |= it->first[i] == uid;
    it = uses ? g_batches.erase(it) : std::next(it);
  }
}

}  // namespace hfmm

using namespace hfmm;

extern "C" int hfmm_batch_matvec(int32_t count, hfmm_tree* const* trees, const double* ks, const int32_t* Ps,
                                 const void* const* xs, void* const* ys, void* stream) {
  try {
    if (count < 1 || !trees || !ks || !Ps || !xs || !ys) return set_error("bad batch arguments"), HFMM_EINVAL;
    std::vector<uint64_t> key;
    for (int i = 0; i < count; ++i) {
      if (!trees[i] || !xs[i] || !ys[i]) return set_error("NULL instance argument"), HFMM_EINVAL;
      if (xs[i] == ys[i]) return set_error("x and y must not alias"), HFMM_EINVAL;
      int rc = check_kP(ks[i], Ps[i]);
      if (rc) return rc;
      if (Ps[i] != Ps[0]) return set_error("all instances of a batch need the same P"), HFMM_EINVAL;
      Tree& t = *reinterpret_cast<Tree*>(trees[i]);
      if (t.bie) return set_error("batched products take point-mode handles"), HFMM_EINVAL;
      for (int j = 0; j < i; ++j)
        if (trees[j] == trees[i])
          return set_error("a tree handle appears twice in one batch (its instances would share buffers)"),
                 HFMM_EINVAL;
      uint64_t kb;
      std::memcpy(&kb, &ks[i], 8);
      key.push_back(t.uid);
      key.push_back(kb);
      key.push_back((uint64_t)Ps[i]);
    }
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = g_batches.find(key);
    if (it == g_batches.end()) {
      std::vector<Tree*> tv;
      std::vector<Plan*> pv;
      for (int i = 0; i < count; ++i) {
        Tree& t = *reinterpret_cast<Tree*>(trees[i]);
        Plan* pl;
        int rc = prepare_operators(t, ks[i], Ps[i], s, &pl);
        if (rc) return rc;
        tv.push_back(&t);
        pv.push_back(pl);
      }
      auto b = std::make_unique<Batch>();
      int rc = build_batch(tv, pv, *b);
      if (rc) return rc;
      it = g_batches.emplace(key, std::move(b)).first;
    }
    return run_batch(*it->second, (const float2* const*)xs, (float2* const*)ys, s, true, nullptr);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HFMM_ENOMEM;
  } catch (...) {
    set_error("internal error");
    return HFMM_EINTERNAL;
  }
}
