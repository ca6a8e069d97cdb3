// C ABI of the hfmm library: handles, operator preparation and the matvec.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <atomic>
#include <thread>
#include <unordered_map>

#include "bie_kernels.h"
#include "nystrom_kernels.h"
#include "hfmm_internal.h"

namespace hfmm {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static std::atomic<uint64_t> g_uid{1};
uint64_t next_uid() { return g_uid.fetch_add(1); }

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                \
      return HFMM_EHIP;                                                            \
    }                                                                              \
  } while (0)

// Allocation-failure hook for tests of the error paths: when >= 0, the
// countdown reaches the allocation to fail, which then reports ENOMEM
// without calling hipMalloc.
static std::atomic<int64_t> g_fail_alloc{-1};

DevBuf::~DevBuf() { reset(); }
int DevBuf::ensure(size_t n) {
  if (p && bytes >= n) return HFMM_OK;
  return alloc(n);
}
void DevBuf::reset() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}
int DevBuf::alloc(size_t n) {
  if (p) {
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  if (n == 0) n = 16;
  if (g_fail_alloc.load() >= 0 && g_fail_alloc.fetch_sub(1) == 0) {
    set_error(std::string("hipMalloc(") + std::to_string(n) + "): failure injected by hfmm_debug_fail_alloc");
    return HFMM_ENOMEM;
  }
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    set_error(std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e));
    return HFMM_ENOMEM;
  }
  bytes = n;
  return HFMM_OK;
}

template <class T>
static int upload(DevBuf& b, const std::vector<T>& v) {
  int rc = b.alloc(v.size() * sizeof(T));
  if (rc) return rc;
  if (!v.empty()) HIP_TRY(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return HFMM_OK;
}

Tree::~Tree() {
  if (ev_made)
    for (auto& e : ev) (void)hipEventDestroy(e);
  if (g_pin) {
    for (auto& e : g_ev) (void)hipEventDestroy(e);
    (void)hipHostFree(g_pin);
  }
  for (auto& e : n_ev)
    if (e) (void)hipEventDestroy(e);
  if (n_stream) (void)hipStreamDestroy(n_stream);
}

// Device bytes of a handle's resident data: sorted float4 positions, source
// indices, weights (BIE) and target permutation, float2 strengths and sorted
// outputs (what upload_bodies allocates); BIE handles add the near pattern
// (CSR offsets, columns and rows) and the panel geometry (flat: 9 doubles
// per panel; curved: the element nodes, points and near work items).
int64_t body_bytes(const Tree& t) {
  const int64_t ns = t.h.nsrc, nt = t.h.ntgt;
  int64_t b = ns * (16 + 4 + 8) + nt * (16 + 4 + 8);
  if (t.bie) {
    const int64_t nnz = (int64_t)t.near_col.size();
    b += ns * 4 + (t.npanel + 1) * 4 + nnz * 8;
    b += t.nystrom ? t.npanel * (24 + 24) + (int64_t)t.nys_items.size() * 16 + 4096 : t.npanel * 72 + 1024;
  }
  return b;
}

int upload_bodies(Tree& t) {
  const HostTree& h = t.h;
  std::vector<float4> sp(h.nsrc), tp(h.ntgt);
  for (int64_t i = 0; i < h.nsrc; ++i)
    sp[i] = make_float4(h.src_xyz[3 * i], h.src_xyz[3 * i + 1], h.src_xyz[3 * i + 2], 0.f);
  for (int64_t i = 0; i < h.ntgt; ++i)
    tp[i] = make_float4(h.tgt_xyz[3 * i], h.tgt_xyz[3 * i + 1], h.tgt_xyz[3 * i + 2], 0.f);
  int rc;
  if ((rc = upload(t.d_src_pos, sp)) || (rc = upload(t.d_tgt_pos, tp))) return rc;
  std::vector<int32_t> sidx(h.nsrc);
  std::vector<float> sw;
  if (!t.bie) {
    for (int64_t i = 0; i < h.nsrc; ++i) sidx[i] = h.src_perm[i];
  } else if (t.nystrom) {
    // sources are the element points themselves, with their rule weights
    sw.resize(h.nsrc);
    for (int64_t i = 0; i < h.nsrc; ++i) {
      sidx[i] = h.src_perm[i];
      sw[i] = nystrom_weight(h.src_perm[i]);
    }
  } else {
    // sources are the Gauss points 3*panel + g with weight area/3
    sw.resize(h.nsrc);
    for (int64_t i = 0; i < h.nsrc; ++i) {
      int32_t pnl = h.src_perm[i] / 3;
      sidx[i] = pnl;
      const double* v = t.verts.data();
      const int32_t* tr = t.tris.data() + 3 * pnl;
      double u[3], w[3];
      for (int d = 0; d < 3; ++d) {
        u[d] = v[3 * tr[1] + d] - v[3 * tr[0] + d];
        w[d] = v[3 * tr[2] + d] - v[3 * tr[0] + d];
      }
      double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      double area = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      sw[i] = (float)(area / 3.0);
    }
  }
  if ((rc = upload(t.d_src_idx, sidx))) return rc;
  if (t.bie && (rc = upload(t.d_src_w, sw))) return rc;
  if ((rc = upload(t.d_tgt_perm, h.tgt_perm))) return rc;
  if ((rc = t.d_q.alloc((size_t)h.nsrc * sizeof(float2))) || (rc = t.d_ys.alloc((size_t)h.ntgt * sizeof(float2))))
    return rc;
  t.body_bytes = (int64_t)(t.d_src_pos.bytes + t.d_tgt_pos.bytes + t.d_src_idx.bytes + t.d_src_w.bytes +
                           t.d_tgt_perm.bytes + t.d_q.bytes + t.d_ys.bytes);
  t.uploaded = true;
  return HFMM_OK;
}

static int upload_cells(Plan& pl) {
  const HostTree& h = pl.ct;
  int nc = h.ncell();
  std::vector<int4> cells(nc), topo(nc);
  std::vector<float4> geo(nc);
  std::vector<int32_t> clev(nc), sl, tl;
  for (int i = 0; i < nc; ++i) {
    cells[i] = make_int4(h.sb[i], h.se[i], h.tb[i], h.te[i]);
    double c[3];
    h.centre(i, c);
    geo[i] = make_float4((float)c[0], (float)c[1], (float)c[2], (float)h.half(i));
    clev[i] = h.level[i];
    int oct = (h.ijk[3 * i] & 1) | ((h.ijk[3 * i + 1] & 1) << 1) | ((h.ijk[3 * i + 2] & 1) << 2);
    topo[i] = make_int4(h.cb[i], h.ce[i], h.parent[i], oct | (h.level[i] << 3));
    if (h.leaf(i)) {
      if (h.se[i] > h.sb[i]) sl.push_back(i);
      if (h.te[i] > h.tb[i]) tl.push_back(i);
    }
  }
  int rc;
  if ((rc = upload(pl.d_cells, cells)) || (rc = upload(pl.d_geo, geo)) || (rc = upload(pl.d_clev, clev)) ||
      (rc = upload(pl.d_topo, topo)))
    return rc;
  return HFMM_OK;
}

// ---------------------------------------------------------------------------
// Operator preparation for (k, P)
// ---------------------------------------------------------------------------
struct Key128 {
  uint64_t a, b;
  bool operator==(const Key128& o) const { return a == o.a && b == o.b; }
};
struct Key128Hash {
  size_t operator()(const Key128& k) const {
    uint64_t h = k.a * 0x9E3779B97F4A7C15ull ^ (k.b + 0x7F4A7C159E3779B9ull + (k.a << 6) + (k.a >> 2));
    return (size_t)(h ^ (h >> 31));
  }
};

// fn(begin, end) over [0, n) in static contiguous chunks, one per thread
// (chunk t is [t n / T, (t + 1) n / T)); small ranges run inline
static int host_threads(size_t n) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  return (int)std::max<size_t>(1, std::min<size_t>({(size_t)std::min(hw, 16u), n / 65536 + 1}));
}
template <class F>
static void parallel_for(size_t n, int T, F fn) {
  if (T <= 1) {
    fn(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t) th.emplace_back(fn, n * t / T, n * (t + 1) / T, t);
  for (auto& x : th) x.join();
}

double kappa_of(const Tree& t, int P) { return t.kappa < 0 ? 0.4 * P : t.kappa; }

int build_plan_host(Tree& t, double k, int P, Plan& pl) {
  const double kappa = kappa_of(t, P);
  const double kabs = std::hypot(k, t.k_imag);  // wavelength rules on |k + i k_imag|
  build_cells(t.h, t.ncrit, t.max_level, kappa / kabs, pl.ct);
  dual_tree_traversal(pl.ct, kabs, t.theta, kappa, pl.lists);
  int64_t pp = 0;
  for (size_t i = 0; i < pl.lists.p2p_a.size(); ++i) {
    int a = pl.lists.p2p_a[i], b = pl.lists.p2p_b[i];
    pp += int64_t(pl.ct.te[a] - pl.ct.tb[a]) * int64_t(pl.ct.se[b] - pl.ct.sb[b]);
  }
  pl.p2p_body_pairs = pp;
  return HFMM_OK;
}

int prepare_host(Tree& t, double k, int P, Plan** out) {
  uint64_t kb;
  std::memcpy(&kb, &k, 8);
  auto key = std::make_pair(kb, P);
  auto it = t.plans.find(key);
  if (it != t.plans.end()) {
    *out = it->second.get();
    return HFMM_OK;
  }
  int rc;
  auto plp = std::make_unique<Plan>();
  Plan& pl = *plp;
  pl.k = k;
  pl.ki = t.k_imag;
  pl.P = P;
  pl.hd = std::make_unique<HostPlanData>();
  HostPlanData& hd = *pl.hd;
  if ((rc = build_plan_host(t, k, P, pl))) return rc;
  const HostTree& h = pl.ct;
  const int P2 = P * P;
  const int nlev = h.nlevels();
  pl.rho.resize(nlev);
  for (int l = 0; l < nlev; ++l) pl.rho[l] = std::min(1.0, std::hypot(k, t.k_imag) * 2.0 * h.H / double(1 << l));
  // operators: M2M and L2L per child level and octant
  std::vector<OpDesc>& ops = hd.ops;
  pl.m2m_base.assign(nlev, 0);
  pl.l2l_base.assign(nlev, 0);
  for (int l = 1; l < nlev; ++l) {
    double hc = h.H / double(1 << l);
    pl.m2m_base[l] = (int32_t)ops.size();
    for (int o = 0; o < 8; ++o) {
      OpDesc d{};
      for (int dd = 0; dd < 3; ++dd) d.t[dd] = -(2.0 * ((o >> dd) & 1) - 1.0) * hc;
      d.rho_in = pl.rho[l];
      d.rho_out = pl.rho[l - 1];
      d.kind = OP_M2M;
      ops.push_back(d);
    }
    pl.l2l_base[l] = (int32_t)ops.size();
    for (int o = 0; o < 8; ++o) {
      OpDesc d{};
      for (int dd = 0; dd < 3; ++dd) d.t[dd] = (2.0 * ((o >> dd) & 1) - 1.0) * hc;
      d.rho_in = pl.rho[l - 1];
      d.rho_out = pl.rho[l];
      d.kind = OP_L2L;
      ops.push_back(d);
    }
  }
  // M2L: canonical offsets under the 16 reflections.  Each pair's key and
  // reflection are computed in parallel; operators are numbered in the order
  // their key first occurs in the pair list (each chunk lists its new keys in
  // order, the chunks are merged in order), then every pair looks its up.
  const size_t npair = pl.lists.m2l_a.size();
  std::unordered_map<Key128, int32_t, Key128Hash> opmap;
  std::vector<int4> pairs(npair);
  std::vector<Key128> keys(npair);
  int32_t m2l_base = (int32_t)ops.size();
  const int TH = host_threads(npair);
  std::vector<std::vector<Key128>> firsts(TH);
  parallel_for(npair, TH, [&](size_t i0, size_t i1, int tid) {
    std::unordered_map<Key128, char, Key128Hash> seen;
    for (size_t i = i0; i < i1; ++i) {
      int a = pl.lists.m2l_a[i], b = pl.lists.m2l_b[i];
      int la = h.level[a], lb = h.level[b];
      int L = std::max(la, lb);
      int64_t d[3];
      for (int dd = 0; dd < 3; ++dd) {
        int64_t ca = -(int64_t(1) << L) + (2 * (int64_t)h.ijk[3 * a + dd] + 1) * (int64_t(1) << (L - la));
        int64_t cb = -(int64_t(1) << L) + (2 * (int64_t)h.ijk[3 * b + dd] + 1) * (int64_t(1) << (L - lb));
        d[dd] = ca - cb;
      }
      int g = (d[0] < 0 ? 1 : 0) | (d[1] < 0 ? 2 : 0) | (d[2] < 0 ? 4 : 0);
      int64_t w[3] = {std::llabs(d[0]), std::llabs(d[1]), std::llabs(d[2])};
      if (w[0] < w[1]) {
        std::swap(w[0], w[1]);
        g |= 8;
      }
      keys[i] = Key128{(uint64_t)la | ((uint64_t)lb << 8) | ((uint64_t)w[2] << 16),
                       (uint64_t)w[0] | ((uint64_t)w[1] << 32)};
      pairs[i] = make_int4(a, b, g, -1);
      if (seen.find(keys[i]) == seen.end()) {  // look up first: emplace would allocate a node
        seen.emplace(keys[i], 0);
        firsts[tid].push_back(keys[i]);
      }
    }
  });
  for (int tid = 0; tid < TH; ++tid)
    for (const Key128& kk : firsts[tid]) {
      if (opmap.count(kk)) continue;
      const int la = (int)(kk.a & 0xff), lb = (int)((kk.a >> 8) & 0xff), L = std::max(la, lb);
      OpDesc dsc{};
      double u = h.H / double(1 << L);
      dsc.t[0] = (double)(kk.b & 0xffffffffull) * u;
      dsc.t[1] = (double)(kk.b >> 32) * u;
      dsc.t[2] = (double)(kk.a >> 16) * u;
      dsc.rho_in = pl.rho[lb];
      dsc.rho_out = pl.rho[la];
      dsc.kind = OP_M2L;
      opmap.emplace(kk, (int32_t)ops.size());
      ops.push_back(dsc);
    }
  parallel_for(npair, TH, [&](size_t i0, size_t i1, int) {
    for (size_t i = i0; i < i1; ++i) pairs[i].w = opmap.find(keys[i])->second;
  });
  std::vector<Key128>().swap(keys);
  pl.n_tables = (int64_t)ops.size() - m2l_base;
  pl.n_ops = (int64_t)ops.size();
  // staging slots: pairs ordered by (target, source), so each target's
  // slots are contiguous and summed in a fixed order
  int Sm0, St0;
  stage_dims(P, &Sm0, &St0);
  std::vector<int32_t> slot(npair);
  // bytgt: pair indices ordered by (target, source), a counting sort by
  // target and a short sort by source within each target ((target, source)
  // is unique, so the order is total)
  std::vector<int32_t> bytgt(npair);
  {
    std::vector<int64_t> pos(h.ncell() + 1, 0);
    for (size_t i = 0; i < npair; ++i) pos[pairs[i].x + 1]++;
    for (int c = 0; c < h.ncell(); ++c) pos[c + 1] += pos[c];
    std::vector<int64_t> fill(pos.begin(), pos.end() - 1);
    for (size_t i = 0; i < npair; ++i) bytgt[fill[pairs[i].x]++] = (int32_t)i;
    parallel_for((size_t)h.ncell(), host_threads(npair), [&](size_t c0, size_t c1, int) {
      for (size_t c = c0; c < c1; ++c)
        std::sort(bytgt.begin() + pos[c], bytgt.begin() + pos[c + 1],
                  [&](int32_t x, int32_t y) { return pairs[x].y < pairs[y].y; });
    });
  }
  {
    hd.soff.assign(h.ncell() + 1, 0);
    for (size_t r = 0; r < npair; ++r) {
      slot[bytgt[r]] = (int32_t)r;
      hd.soff[pairs[bytgt[r]].x + 1]++;
    }
    for (int c = 0; c < h.ncell(); ++c) {
      if (hd.soff[c + 1] > 0) pl.m2l_targets.push_back(c);
      hd.soff[c + 1] += hd.soff[c];
    }
  }
  // staging segments: runs of consecutive targets whose slots fit the
  // staging budget (a target with more slots than the budget gets its own)
  std::vector<int32_t> seg_of(h.ncell(), 0);
  pl.m2l_segs.clear();
  {
    const int64_t budget = std::max<int64_t>(1, t.stage_bytes / ((int64_t)(Sm0 + St0) * (int64_t)sizeof(float2)));
    M2LSeg cur{};
    for (size_t i = 0; i < pl.m2l_targets.size(); ++i) {
      const int c = pl.m2l_targets[i];
      const int64_t n = hd.soff[c + 1] - hd.soff[c];
      if (cur.slot_e > cur.slot_b && (cur.slot_e - cur.slot_b) + n > budget) {
        pl.m2l_segs.push_back(cur);
        cur = M2LSeg{};
        cur.slot_b = cur.slot_e = hd.soff[c];
        cur.tgt_b = cur.tgt_e = (int)i;
      }
      if (cur.tgt_e == cur.tgt_b) {
        cur.slot_b = hd.soff[c];
        cur.tgt_b = (int)i;
      }
      cur.slot_e = hd.soff[c + 1];
      cur.tgt_e = (int)i + 1;
      seg_of[c] = (int)pl.m2l_segs.size();
    }
    if (cur.tgt_e > cur.tgt_b) pl.m2l_segs.push_back(cur);
  }
  // group pairs by segment, then operator, then target, then source: a
  // stable counting sort by (segment, operator) of the (target, source)
  // order (segments are runs of consecutive targets)
  std::vector<int32_t> order(npair);
  {
    const int64_t nops = (int64_t)ops.size();
    std::vector<int64_t> pos((int64_t)pl.m2l_segs.size() * nops + 1, 0);
    auto key = [&](int32_t i) { return (int64_t)seg_of[pairs[i].x] * nops + pairs[i].w; };
    for (size_t i = 0; i < npair; ++i) pos[key((int32_t)i) + 1]++;
    for (size_t e = 1; e < pos.size(); ++e) pos[e] += pos[e - 1];
    for (size_t r = 0; r < npair; ++r) order[pos[key(bytgt[r])]++] = bytgt[r];
  }
  std::vector<int32_t>().swap(bytgt);
  std::vector<int4>& spairs = hd.spairs;
  spairs.resize(npair);
  std::vector<int4> chunks;
  hd.slot_g.assign(std::max<size_t>(1, npair), 0);
  // With several segments the staging holds two segment buffers, used in
  // turn, so that the reduction of one segment overlaps the M2L of the next.
  pl.max_seg_slots = 0;
  for (const M2LSeg& sgm : pl.m2l_segs) pl.max_seg_slots = std::max<int64_t>(pl.max_seg_slots, sgm.slot_e - sgm.slot_b);
  pl.stage_bufs = pl.m2l_segs.size() > 1 ? 2 : 1;
  parallel_for(npair, TH, [&](size_t i0, size_t i1, int) {
    for (size_t i = i0; i < i1; ++i) {  // slots are local to the pair's segment and its buffer
      const int4& p = pairs[order[i]];
      const int sg = seg_of[p.x];
      const int64_t rel = slot[order[i]] - pl.m2l_segs[sg].slot_b + (sg % pl.stage_bufs) * pl.max_seg_slots;
      spairs[i] = make_int4(p.x, p.y, p.z, (int32_t)rel);
      hd.slot_g[slot[order[i]]] = (uint8_t)p.z;
    }
  });
  const int CH = m2l_pairs_per_chunk(P);
  for (size_t i = 0; i < npair;) {
    size_t j = i;
    const int4& pi = pairs[order[i]];
    const int op = pi.w, sg = seg_of[pi.x];
    if (pl.m2l_segs[sg].chunk_e == 0) pl.m2l_segs[sg].chunk_b = (int)chunks.size();
    while (j < npair && pairs[order[j]].w == op && seg_of[pairs[order[j]].x] == sg && j - i < (size_t)CH) ++j;
    chunks.push_back(make_int4(op, (int)i, (int)j, 0));
    pl.m2l_segs[sg].chunk_e = (int)chunks.size();
    i = j;
  }
  pl.n_m2l_chunks = (int32_t)chunks.size();
  pl.m2l_chunks_h = chunks;
  // per-cell operator indices and per-level work lists
  std::vector<int2>& cops = hd.cops;
  cops.assign(h.ncell(), make_int2(0, 0));
  pl.m2m_cells.assign(nlev, {});
  pl.l2l_cells.assign(nlev, {});
  for (int i = 0; i < h.ncell(); ++i) {
    const int l = h.level[i];
    if (l >= 1) {
      int oct = (h.ijk[3 * i] & 1) | ((h.ijk[3 * i + 1] & 1) << 1) | ((h.ijk[3 * i + 2] & 1) << 2);
      cops[i] = make_int2(pl.m2m_base[l] + oct, pl.l2l_base[l] + oct);
      pl.l2l_cells[l].push_back(i);
    }
    if (!h.leaf(i)) pl.m2m_cells[l].push_back(i);
    else {
      if (h.se[i] > h.sb[i]) pl.src_leaves.push_back(i);
      if (h.te[i] > h.tb[i]) pl.tgt_leaves.push_back(i);
    }
  }
  // P2P work: per target leaf, merged source intervals
  std::vector<int4>& work = hd.work;
  std::vector<int2>& ivals = hd.ivals;
  std::vector<int32_t>& totals = hd.totals;
  {
    const size_t np = pl.lists.p2p_a.size();
    std::vector<int32_t> ord(np);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) {
      int ax = pl.lists.p2p_a[x], ay = pl.lists.p2p_a[y];
      if (ax != ay) return ax < ay;
      return h.sb[pl.lists.p2p_b[x]] < h.sb[pl.lists.p2p_b[y]];
    });
    for (size_t i = 0; i < np;) {
      int a = pl.lists.p2p_a[ord[i]];
      int ib = (int)ivals.size();
      size_t j = i;
      while (j < np && pl.lists.p2p_a[ord[j]] == a) {
        int b = pl.lists.p2p_b[ord[j]];
        int s0 = h.sb[b], s1 = h.se[b];
        if (!ivals.empty() && (int)ivals.size() > ib && ivals.back().y == s0)
          ivals.back().y = s1;
        else
          ivals.push_back(make_int2(s0, s1));
        ++j;
      }
      work.push_back(make_int4(h.tb[a], h.te[a], ib, (int)ivals.size()));
      int tot = 0;
      for (int v = ib; v < (int)ivals.size(); ++v) tot += ivals[v].y - ivals[v].x;
      totals.push_back(tot);
      i = j;
    }
  }
  pl.n_p2p_work = (int32_t)work.size();
  pl.n_ops = (int64_t)ops.size();
  // exact device footprint of this plan (and of the bodies if not yet resident)
  {
    int Kp, Rp, Sm, St;
    table_dims(P, &Kp, &Rp);
    stage_dims(P, &Sm, &St);
    const int64_t nc = h.ncell();
    // cells (int4 bodies, float4 geometry, level, int4 topology, int2 operators)
    pl.bytes_cells = nc * (int64_t)(sizeof(int4) * 2 + sizeof(float4) + sizeof(int32_t) + sizeof(int2));
    // work lists: M2L pair records (int4) and slot reflections (uint8), the
    // per-target slot offsets, P2P work items, source intervals and totals,
    // the reflection code tables
    const XzDims xd = xz_dims(P);
    pl.bytes_lists = (int64_t)spairs.size() * 17 + (nc + 1) * 4 + (int64_t)work.size() * 20 +
                     (int64_t)ivals.size() * 8 + (17 * (int64_t)xz_code_stride(P) + 16 * xd.RTS + 16 * P2) * 4 +
                     17 * (int64_t)Kp * 4;
    // operators (descriptors and padded tables), level scales, M and L, the
    // M2L staging of the largest segment
    pl.bytes_exp = (int64_t)ops.size() * (int64_t)(sizeof(OpDesc) + (size_t)xz_table_stride(P) * sizeof(float2)) +
                   (int64_t)pl.rho.size() * 8 + 2 * nc * P2 * (int64_t)sizeof(float2) +
                   pl.stage_bufs * std::max<int64_t>(1, pl.max_seg_slots) * (int64_t)(Sm + St) *
                       (int64_t)sizeof(float2);
    // BIE corrections: near values (float2) and the self term (double2 per
    // panel, or a 6 x 6 double2 block row per curved-element point)
    pl.bytes_corr = t.bie ? (int64_t)t.near_col.size() * 8 + t.npanel * (t.nystrom ? 96 : 16) : 0;
    pl.est_bytes = pl.bytes_cells + pl.bytes_lists + pl.bytes_exp + pl.bytes_corr +
                   (t.uploaded ? 0 : body_bytes(t));
  }
  t.plans[key] = std::move(plp);
  *out = t.plans[key].get();
  return HFMM_OK;
}

int prepare_device(Tree& t, Plan& pl, hipStream_t s) {
  // device_ready is set only after every step below succeeded: a failed
  // step leaves the plan not ready, and the next call redoes it from the
  // start (each buffer's alloc replaces what an earlier attempt left).
  if (pl.device_ready) return HFMM_OK;
  int rc;
  if (!t.uploaded && (rc = upload_bodies(t))) return rc;
  if ((rc = upload_cells(pl))) return rc;
  HostPlanData& hd = *pl.hd;
  const HostTree& h = pl.ct;
  const int P = pl.P, P2 = P * P;
  const double k = pl.k;
  int Kp, Rp, Sm, St;
  table_dims(P, &Kp, &Rp);
  stage_dims(P, &Sm, &St);
  if ((rc = upload(pl.d_ops, hd.ops)) || (rc = upload(pl.d_rho, pl.rho)) ||
      (rc = upload(pl.d_m2l_pairs, hd.spairs)) || (rc = upload(pl.d_cops, hd.cops)) ||
      (rc = upload(pl.d_m2l_soff, hd.soff)) ||
      (rc = pl.d_stage.alloc((size_t)pl.stage_bufs * (size_t)std::max<int64_t>(1, pl.max_seg_slots) *
                             (size_t)(Sm + St) * sizeof(float2))) ||
      (rc = upload(pl.d_p2p_work, hd.work)) || (rc = upload(pl.d_p2p_ivals, hd.ivals)) ||
      (rc = upload(pl.d_p2p_total, hd.totals)))
    return rc;
  {
    std::vector<int32_t> in, out, din, dout;
    m2l_xz_codes(P, in, out);
    m2l_reflection_codes(P, Kp, din, dout);
    if ((rc = upload(pl.d_bmap, in)) || (rc = upload(pl.d_omap, out)) || (rc = upload(pl.d_bmap64, din)) ||
        (rc = upload(pl.d_slot_g, hd.slot_g)))
      return rc;
  }
  // coupling coefficients and tables
  const Coupling& cp = coupling(P);
  std::vector<double2> cv(cp.re.size());
  for (size_t i = 0; i < cv.size(); ++i) cv[i] = make_double2(cp.re[i], cp.im[i]);
  DevBuf d_off, d_lm, d_val;
  if ((rc = upload(d_off, cp.off)) || (rc = upload(d_lm, cp.lm)) || (rc = upload(d_val, cv)))
    return rc;
  if ((rc = pl.d_tables.alloc((size_t)pl.n_ops * xz_table_stride(P) * sizeof(float2)))) return rc;
  launch_gen_tables(pl.d_ops.as<OpDesc>(), (int)pl.n_ops, P, k, pl.ki, d_off.as<int32_t>(),
                    d_lm.as<int32_t>(), d_val.as<double2>(), pl.d_tables.as<float2>(), s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  if ((rc = pl.d_M.alloc((size_t)h.ncell() * P2 * sizeof(float2))) ||
      (rc = pl.d_L.alloc((size_t)h.ncell() * P2 * sizeof(float2))))
    return rc;
  pl.device_bytes = 0;
  for (DevBuf* b : {&pl.d_cells, &pl.d_geo, &pl.d_clev, &pl.d_topo, &pl.d_ops, &pl.d_tables, &pl.d_rho,
                    &pl.d_m2l_pairs, &pl.d_p2p_work, &pl.d_p2p_ivals, &pl.d_p2p_total, &pl.d_M,
                    &pl.d_L, &pl.d_cops, &pl.d_stage, &pl.d_m2l_soff, &pl.d_bmap, &pl.d_omap,
                    &pl.d_bmap64, &pl.d_slot_g})
    pl.device_bytes += (int64_t)b->bytes;
  if (t.bie && (rc = (t.nystrom ? prepare_nystrom(t, pl, s) : prepare_bie(t, pl, s)))) return rc;
  pl.device_bytes += (int64_t)(pl.d_near_val.bytes + pl.d_diag.bytes);
  pl.hd.reset();
  pl.device_ready = true;
  return HFMM_OK;
}

// Host lists, device operators and (BIE) corrections for (k, P).
int prepare_operators(Tree& t, double k, int P, hipStream_t s, Plan** out) {
  Plan* pl;
  int rc = prepare_host(t, k, P, &pl);
  if (rc) return rc;
  if ((rc = prepare_device(t, *pl, s))) return rc;
  *out = pl;
  return HFMM_OK;
}

// Everything a product on (k, P) needs, so that a product allocates nothing:
// the operators, and the single-instance batch (work lists, launch shape,
// side stream).
int prepare(Tree& t, double k, int P, hipStream_t s, Plan** out) {
  Plan* pl;
  int rc = prepare_operators(t, k, P, s, &pl);
  if (rc) return rc;
  if (!pl->self) {
    pl->self = std::make_unique<Batch>();
    if ((rc = build_batch({&t}, {pl}, *pl->self))) {
      pl->self.reset();
      return rc;
    }
  }
  if ((rc = ready_batch(*pl->self, s))) return rc;
  *out = pl;
  return HFMM_OK;
}

int check_kP(double k, int P) {
  if (!(k > 0.0) || !std::isfinite(k)) {
    set_error("k must be positive and finite");
    return HFMM_EINVAL;
  }
  if (P < 1 || P > kMaxP) {
    set_error("P must be in [1, 16]");
    return HFMM_EINVAL;
  }
  return HFMM_OK;
}

int matvec_impl(Tree& t, Plan& pl, const float2* x, float2* y, hipStream_t s) {
  if (!pl.self) return set_error("internal: product on an unprepared plan"), HFMM_EINVAL;
  const float2* xs[1] = {x};
  float2* ys[1] = {y};
  return run_batch(*pl.self, xs, ys, s, false, t.timing ? &t : nullptr);
}

}  // namespace hfmm

using namespace hfmm;

#define API_GUARD_BEGIN try {
#define API_GUARD_END                          \
  }                                            \
  catch (const std::bad_alloc&) {              \
    set_error("host allocation failed");       \
    return HFMM_ENOMEM;                        \
  }                                            \
  catch (const std::exception& e) {            \
    set_error(e.what());                       \
    return HFMM_EINTERNAL;                     \
  }                                            \
  catch (...) {                                \
    set_error("unknown exception");            \
    return HFMM_EINTERNAL;                     \
  }

extern "C" {

int hfmm_version(void) { return 100; }

int hfmm_debug_fail_alloc(int64_t after) {
  if (after < -1) return set_error("after must be >= -1"), HFMM_EINVAL;
  g_fail_alloc.store(after);
  return HFMM_OK;
}
const char* hfmm_last_error(void) { return g_err.c_str(); }

int hfmm_default_opts(hfmm_opts* o) {
  if (!o) return HFMM_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->ncrit = 64;
  o->max_level = 20;
  o->theta = 0.5;
  o->kappa = -1.0;
  o->eta = 2.0;
  o->near_levels = 3;
  o->near_order = 6;
  o->stage_mb = 32768;
  return HFMM_OK;
}

static int apply_opts(Tree& t, const hfmm_opts* o) {
  hfmm_opts d;
  hfmm_default_opts(&d);
  if (!o) o = &d;
  if (o->ncrit < 1) return set_error("ncrit must be >= 1"), HFMM_EINVAL;
  if (o->max_level < 0 || o->max_level > kMaxLevel) return set_error("max_level in [0, 20]"), HFMM_EINVAL;
  if (!(o->theta > 0.0) || !std::isfinite(o->theta)) return set_error("theta must be > 0"), HFMM_EINVAL;
  if (!(o->eta > 0.0)) return set_error("eta must be > 0"), HFMM_EINVAL;
  if (o->near_levels < 0 || o->near_levels > 5 || o->near_order < 1 || o->near_order > 16)
    return set_error("near_levels in [0,5], near_order in [1,16]"), HFMM_EINVAL;
  if (o->bie_treatment < 0 || o->bie_treatment > 2) return set_error("bie_treatment in [0, 2]"), HFMM_EINVAL;
  if (!(o->k_imag >= 0.0) || !std::isfinite(o->k_imag)) return set_error("k_imag must be finite and >= 0"), HFMM_EINVAL;
  t.ncrit = o->ncrit;
  t.k_imag = o->k_imag;
  t.stage_bytes = (int64_t)(o->stage_mb > 0 ? o->stage_mb : 32768) << 20;
  t.bie_treatment = o->bie_treatment;
  t.max_level = o->max_level;
  t.theta = o->theta;
  t.kappa = o->kappa;
  t.eta = o->eta;
  t.near_levels = o->near_levels;
  t.near_order = o->near_order;
  return HFMM_OK;
}

int hfmm_build_tree(const float* xyz, int64_t n, const hfmm_opts* opts, hfmm_tree** out) {
  API_GUARD_BEGIN
  if (!out) return set_error("out is NULL"), HFMM_EINVAL;
  *out = nullptr;
  if (!xyz || n < 1 || n > (int64_t(1) << 30)) return set_error("need 1 <= n <= 2^30 points"), HFMM_EINVAL;
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) return set_error("non-finite coordinate"), HFMM_EINVAL;
  auto t = std::make_unique<Tree>();
  int rc = apply_opts(*t, opts);
  if (rc) return rc;
  build_tree(xyz, n, nullptr, 0, t->ncrit, t->max_level, t->h);
  t->uid = next_uid();
  *out = reinterpret_cast<hfmm_tree*>(t.release());
  return HFMM_OK;
  API_GUARD_END
}

int hfmm_prepare_host(hfmm_tree* tree, double k, int32_t P, int64_t* footprint) {
  API_GUARD_BEGIN
  if (!tree) return set_error("tree is NULL"), HFMM_EINVAL;
  int rc = check_kP(k, P);
  if (rc) return rc;
  Plan* pl;
  Tree& t = *reinterpret_cast<Tree*>(tree);
  if ((rc = prepare_host(t, k, P, &pl))) return rc;
  if (footprint) *footprint = pl->device_ready ? 0 : pl->est_bytes;
  return HFMM_OK;
  API_GUARD_END
}

int hfmm_tree_plan(hfmm_tree* tree, double k, int32_t P, int32_t restart, hfmm_plan_info* out) {
  API_GUARD_BEGIN
  if (!tree || !out) return set_error("NULL argument"), HFMM_EINVAL;
  int rc = check_kP(k, P);
  if (rc) return rc;
  Tree& t = *reinterpret_cast<Tree*>(tree);
  if (restart < 0 || restart > 200 || (t.bie && restart < 1))
    return set_error("restart in [1, 200] (0 for point handles)"), HFMM_EINVAL;
  Plan* pl;
  if ((rc = prepare_host(t, k, P, &pl))) return rc;
  hfmm_plan_info info{};
  info.n_src = t.h.nsrc;
  info.n_tgt = t.h.ntgt;
  info.n_cell = pl->ct.ncell();
  for (int i = 0; i < pl->ct.ncell(); ++i) info.n_leaf += pl->ct.leaf(i) ? 1 : 0;
  info.n_level = pl->ct.nlevels();
  info.n_m2l = (int64_t)pl->lists.m2l_a.size();
  info.n_p2p = (int64_t)pl->lists.p2p_a.size();
  info.p2p_body_pairs = pl->p2p_body_pairs;
  info.n_tables = pl->n_tables;
  info.n_near = t.bie ? (int64_t)t.near_col.size() : 0;
  info.bytes_tree = body_bytes(t) + pl->bytes_cells;
  info.bytes_lists = pl->bytes_lists;
  info.bytes_expansions = pl->bytes_exp;
  info.bytes_corrections = pl->bytes_corr;
  info.bytes_gmres = t.bie && restart > 0 ? gmres_workspace_bytes(t.npanel, restart) : 0;
  info.bytes_total = info.bytes_tree + info.bytes_lists + info.bytes_expansions + info.bytes_corrections +
                     info.bytes_gmres;
  info.resident = pl->device_ready ? 1 : 0;
  *out = info;
  return HFMM_OK;
  API_GUARD_END
}

int hfmm_prepare(hfmm_tree* tree, double k, int32_t P, void* stream) {
  API_GUARD_BEGIN
  if (!tree) return set_error("tree is NULL"), HFMM_EINVAL;
  int rc = check_kP(k, P);
  if (rc) return rc;
  Plan* pl;
  return prepare(*reinterpret_cast<Tree*>(tree), k, P, (hipStream_t)stream, &pl);
  API_GUARD_END
}

int hfmm_matvec(hfmm_tree* tree, double k, int32_t P, const void* x, void* y, void* stream) {
  API_GUARD_BEGIN
  if (!tree || !x || !y) return set_error("NULL argument"), HFMM_EINVAL;
  if (x == y) return set_error("x and y must not alias"), HFMM_EINVAL;
  int rc = check_kP(k, P);
  if (rc) return rc;
  Tree& t = *reinterpret_cast<Tree*>(tree);
  hipStream_t s = (hipStream_t)stream;
  Plan* pl;
  if ((rc = prepare(t, k, P, s, &pl))) return rc;
  if (t.timing && !t.ev_made) {
    for (auto& e : t.ev) HIP_TRY(hipEventCreate(&e));
    t.ev_made = true;
  }
  if ((rc = matvec_impl(t, *pl, (const float2*)x, (float2*)y, s))) return rc;
  if (t.bie) {
    launch_near_apply(t.npanel, t.d_near_off.as<int32_t>(), t.d_near_col.as<int32_t>(),
                      pl->d_near_val.as<float2>(), t.nystrom ? nullptr : pl->d_diag.as<double2>(),
                      (const float2*)x, (float2*)y, s);
    if (t.nystrom) launch_self6_apply_c64(t.npanel, pl->d_self6.as<double2>(), (const float2*)x, (float2*)y, s);
    HIP_TRY(hipGetLastError());
  }
  if (t.timing) HIP_TRY(hipEventRecord(t.ev[8], s));
  if (t.timing) {
    HIP_TRY(hipEventSynchronize(t.ev[8]));
    float ms;
    // phases: P2M (0-1), M2M (1-2), M2L matrix-core kernel (2-3), M2L
    // reduction (3-4), L2L (4-5), P2P (5-6), L2P (6-7), output scatter and
    // BIE corrections (7-8), total (0-8); reported in the order P2M, M2M,
    // M2L, reduction, L2L, L2P, P2P, scatter
    static const int span[8] = {0, 1, 2, 3, 4, 6, 5, 7};
    for (int i = 0; i < 8; ++i) {
      HIP_TRY(hipEventElapsedTime(&ms, t.ev[span[i]], t.ev[span[i] + 1]));
      t.phase_ms[i] = ms;
    }
    HIP_TRY(hipEventElapsedTime(&ms, t.ev[0], t.ev[8]));
    t.phase_ms[8] = ms;
    t.phase_ms[9] = 0.f;
  }
  return HFMM_OK;
  API_GUARD_END
}

int hfmm_set_timing(hfmm_tree* tree, int32_t on) {
  if (!tree) return set_error("tree is NULL"), HFMM_EINVAL;
  reinterpret_cast<Tree*>(tree)->timing = on != 0;
  return HFMM_OK;
}

int hfmm_phase_times(const hfmm_tree* tree, float* ms10) {
  if (!tree || !ms10) return set_error("NULL argument"), HFMM_EINVAL;
  std::memcpy(ms10, reinterpret_cast<const Tree*>(tree)->phase_ms, 10 * sizeof(float));
  return HFMM_OK;
}

int hfmm_variant_count(int32_t phase, int32_t P) {
  if (phase < 0 || phase >= kNumTunedPhases) return set_error("unknown tuned phase"), HFMM_EINVAL;
  if (P < 1 || P > kMaxP) return set_error("P must be in [1, 16]"), HFMM_EINVAL;
  return phase_variant_count(phase, P);
}

int hfmm_set_variant(int32_t phase, int32_t variant) { return set_variant_override(phase, variant); }

int hfmm_tree_variant(hfmm_tree* tree, double k, int32_t P, int32_t phase, int32_t* variant) {
  if (!tree || !variant) return set_error("NULL argument"), HFMM_EINVAL;
  if (phase < 0 || phase >= kNumTunedPhases) return set_error("unknown tuned phase"), HFMM_EINVAL;
  Tree& t = *reinterpret_cast<Tree*>(tree);
  uint64_t kb;
  std::memcpy(&kb, &k, 8);
  auto it = t.plans.find(std::make_pair(kb, (int)P));
  *variant = -1;
  if (phase == kPhaseNear) {  // the placement the next GMRES product uses
    const int o = variant_override(kPhaseNear);
    if (it != t.plans.end() && t.bie) *variant = o >= 0 ? o : std::max(it->second->near_side, 0);
    if (it != t.plans.end() && t.bie && !t.n_stream) *variant = 0;
    return HFMM_OK;
  }
  if (it != t.plans.end() && it->second->self && it->second->self->ran)
    *variant = batch_variant(*it->second->self, phase);
  return HFMM_OK;
}

int hfmm_tree_stats(hfmm_tree* tree, double k, int32_t P, hfmm_stats* o) {
  API_GUARD_BEGIN
  if (!tree || !o) return set_error("NULL argument"), HFMM_EINVAL;
  Tree& t = *reinterpret_cast<Tree*>(tree);
  std::memset(o, 0, sizeof(*o));
  const HostTree* h = &t.h;
  Plan tmp;
  const Plan* pl = nullptr;
  if (P > 0) {
    int rc = check_kP(k, P);
    if (rc) return rc;
    uint64_t kb;
    std::memcpy(&kb, &k, 8);
    auto it = t.plans.find(std::make_pair(kb, (int)P));
    if (it != t.plans.end()) {
      pl = it->second.get();
    } else {
      build_plan_host(t, k, P, tmp);
      pl = &tmp;
    }
    h = &pl->ct;
  }
  o->n_src = h->nsrc;
  o->n_tgt = h->ntgt;
  o->n_cell = h->ncell();
  int nl = 0;
  for (int i = 0; i < h->ncell(); ++i) nl += h->leaf(i);
  o->n_leaf = nl;
  o->n_level = h->nlevels();
  o->point_mode = h->point_mode ? 1 : 0;
  for (int d = 0; d < 3; ++d) o->centre[d] = h->c[d];
  o->half = h->H;
  o->device_bytes = t.body_bytes;
  if (pl) {
    o->n_m2l = (int64_t)pl->lists.m2l_a.size();
    o->n_p2p = (int64_t)pl->lists.p2p_a.size();
    o->p2p_body_pairs = pl->p2p_body_pairs;
    o->n_tables = pl->n_tables;
    o->n_near = pl->n_near;
    o->device_bytes += pl->device_bytes;
  }
  return HFMM_OK;
  API_GUARD_END
}

int hfmm_tree_export(hfmm_tree* tree, double k, int32_t P, int32_t* src_perm, int32_t* tgt_perm,
                     int32_t* cells) {
  API_GUARD_BEGIN
  if (!tree) return set_error("tree is NULL"), HFMM_EINVAL;
  Tree& t = *reinterpret_cast<Tree*>(tree);
  Plan tmp;
  const HostTree* h = &t.h;
  if (P > 0) {
    int rc = check_kP(k, P);
    if (rc) return rc;
    build_plan_host(t, k, P, tmp);
    h = &tmp.ct;
  }
  if (src_perm) std::memcpy(src_perm, t.h.src_perm.data(), t.h.nsrc * sizeof(int32_t));
  if (tgt_perm) std::memcpy(tgt_perm, t.h.tgt_perm.data(), t.h.ntgt * sizeof(int32_t));
  if (cells)
    for (int i = 0; i < h->ncell(); ++i) {
      int32_t* c = cells + 10 * i;
      c[0] = h->level[i];
      c[1] = h->ijk[3 * i];
      c[2] = h->ijk[3 * i + 1];
      c[3] = h->ijk[3 * i + 2];
      c[4] = h->sb[i];
      c[5] = h->se[i];
      c[6] = h->tb[i];
      c[7] = h->te[i];
      c[8] = h->cb[i];
      c[9] = h->ce[i];
    }
  return HFMM_OK;
  API_GUARD_END
}

int hfmm_lists_export(hfmm_tree* tree, double k, int32_t P, int32_t* m2l, int32_t* p2p) {
  API_GUARD_BEGIN
  if (!tree) return set_error("tree is NULL"), HFMM_EINVAL;
  int rc = check_kP(k, P);
  if (rc) return rc;
  Tree& t = *reinterpret_cast<Tree*>(tree);
  Plan pl;
  build_plan_host(t, k, P, pl);
  for (size_t i = 0; m2l && i < pl.lists.m2l_a.size(); ++i) {
    m2l[2 * i] = pl.lists.m2l_a[i];
    m2l[2 * i + 1] = pl.lists.m2l_b[i];
  }
  for (size_t i = 0; p2p && i < pl.lists.p2p_a.size(); ++i) {
    p2p[2 * i] = pl.lists.p2p_a[i];
    p2p[2 * i + 1] = pl.lists.p2p_b[i];
  }
  return HFMM_OK;
  API_GUARD_END
}

void hfmm_tree_free(hfmm_tree* tree) {
  if (!tree) return;
  forget_tree_batches(reinterpret_cast<Tree*>(tree)->uid);
  delete reinterpret_cast<Tree*>(tree);
}

}  // extern "C"

// Entry points completed in bie.cpp / batch.cpp.
