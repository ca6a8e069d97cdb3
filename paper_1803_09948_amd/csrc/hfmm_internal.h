// Internal structures of the hfmm library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hfmm.h"
#include "fmm_kernels.h"

namespace hfmm {

constexpr int kKeyBits = 21;
constexpr int kMaxLevel = 20;

void set_error(const std::string& msg);

// ---------------------------------------------------------------------------
// Octree over sources and targets (point mode: the same set).
// ---------------------------------------------------------------------------
struct HostTree {
  bool point_mode = true;
  int64_t nsrc = 0, ntgt = 0;
  int ncrit = 64;
  double c[3] = {0, 0, 0};
  double H = 1.0;
  std::vector<int32_t> src_perm, tgt_perm;     // sorted position -> input index
  std::vector<float> src_xyz, tgt_xyz;         // sorted, 3 floats per body
  std::vector<uint64_t> skey, tkey;            // sorted Morton keys (tkey empty in point mode)
  // cells, level by level, Morton order within a level
  std::vector<int32_t> level, ijk, sb, se, tb, te, cb, ce, parent;
  std::vector<int32_t> level_off;              // cells of level l: [off[l], off[l+1])
  int ncell() const { return (int)level.size(); }
  int nlevels() const { return (int)level_off.size() - 1; }
  bool leaf(int i) const { return cb[i] == ce[i]; }
  double half(int i) const { return H / double(1 << level[i]); }
  void centre(int i, double out[3]) const {
    double h = half(i);
    for (int d = 0; d < 3; ++d) out[d] = c[d] - H + (2.0 * ijk[3 * i + d] + 1.0) * h;
  }
};

// Sorts the bodies and builds the base cells.  tgt == nullptr: point mode.
void build_tree(const float* src, int64_t nsrc, const float* tgt, int64_t ntgt,
                int ncrit, int max_level, HostTree& t);
// Cells over the sorted bodies of `b` into `t` (which may be `b`): a cell splits
// when it holds more than ncrit sources, or when it is non-empty and its side
// exceeds split_side.
void build_cells(const HostTree& b, int ncrit, int max_level, double split_side, HostTree& t);

struct Lists {
  std::vector<int32_t> m2l_a, m2l_b;  // (target cell, source cell)
  std::vector<int32_t> p2p_a, p2p_b;  // (target leaf, source leaf)
};

void dual_tree_traversal(const HostTree& t, double k, double theta, double kappa,
                         Lists& out);

// ---------------------------------------------------------------------------
// Translation-operator descriptors (computed on the device in FP64).
// ---------------------------------------------------------------------------
enum OpKind : int32_t { OP_M2M = 0, OP_L2L = 1, OP_M2L = 2 };

using OpDesc = OpDescDev;

// Gaunt coupling in CSR over (row = (n',m'), col = (n,m)) entries:
// coefficient 4 pi i^{n'+l-n} G(n,m;n',m';l) of harmonic index (l, m-m').
struct Coupling {
  int P = 0;
  std::vector<int32_t> off;     // P^4 + 1
  std::vector<int32_t> lm;      // harmonic index l*l + l + mu
  std::vector<double> re, im;   // coefficient
};
const Coupling& coupling(int P);

// Reflection codes of the matrix-core M2L.  A code idx | swap << 16 |
// zero << 17 | neg_im << 30 | neg_re << 31 stands for i^ph v[idx], with
// i^ph (x + iy) = (+-x or +-y) + i (+-y or +-x).  in[g][k], k < Kp (16
// reflections and a 17th all-zero row): input row k of a pair with
// reflection g is B[k] = i^ph M[idx].  out[g][c], c < P^2: output
// coefficient c of such a pair is i^-ph C[idx].
void m2l_reflection_codes(int P, int Kp, std::vector<int32_t>& in, std::vector<int32_t>& out);
void m2l_xz_codes(int P, std::vector<int32_t>& in, std::vector<int32_t>& out);

// ---------------------------------------------------------------------------
// Device-side plan for one (k, P)
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf();
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  int alloc(size_t n);
  int ensure(size_t n);  // grow-only: keeps the buffer if it is large enough
  void reset();
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Host-side results of plan preparation, kept until the device upload.
struct HostPlanData {
  std::vector<OpDesc> ops;
  std::vector<int4> spairs, work;
  std::vector<int2> ivals, cops;
  std::vector<int32_t> totals, soff;
  std::vector<uint8_t> slot_g;    // reflection of the pair of each (global) staging slot
};

// A staging segment of the M2L: targets m2l_targets[tgt_b, tgt_e) own the
// staging slots [slot_b, slot_e) (pair slots are stored relative to slot_b),
// and their pairs form the chunks [chunk_b, chunk_e).
struct M2LSeg {
  int64_t slot_b = 0, slot_e = 0;
  int tgt_b = 0, tgt_e = 0, chunk_b = 0, chunk_e = 0;
};

struct Plan {
  double k = 0;
  int P = 0;
  // BIE handles: whether the GMRES product runs its near corrections on the
  // handle's near stream beside the FMM (1), after it (0), or not yet timed
  // (-1: after it); the same bits either way
  int near_side = -1;
  HostTree ct;                   // cells of this plan (wavenumber-aware splitting)
  Lists lists;
  int64_t n_tables = 0;          // M2L operators
  int64_t n_ops = 0;             // all operators
  int64_t p2p_body_pairs = 0;
  std::vector<double> rho;       // per level
  std::vector<int32_t> m2m_base, l2l_base;  // per child level: op index of octant 0
  // device cells
  DevBuf d_cells;                // int4 (sb, se, tb, te)
  DevBuf d_geo;                  // float4 (cx, cy, cz, half)
  DevBuf d_clev;                 // int32 level
  DevBuf d_topo;                 // int4 (child begin, child end, parent, octant | level << 3)
  // operators and work lists
  DevBuf d_ops, d_tables;        // OpDesc[n_ops]; float2 [n_ops][xz_table_stride(P)]
  DevBuf d_rho;                  // double per level
  DevBuf d_m2l_pairs;            // int4 (target cell, source cell, reflection, staging slot)
  int32_t n_m2l_chunks = 0;
  DevBuf d_p2p_work;             // int4 (tgt begin, tgt end, interval begin, interval end)
  DevBuf d_p2p_ivals;            // int2 (src begin, src end)
  DevBuf d_p2p_total;            // int32 sources per work item
  int32_t n_p2p_work = 0;
  DevBuf d_bmap;                 // int32 [17][Kx] + [16 RTS]: M2L input codes (m2l_xz_codes)
  DevBuf d_omap;                 // int32 [16][P^2]: M2L output codes (m2l_xz_codes)
  DevBuf d_bmap64;               // int32 [17][Kp]: dense input codes (FP64 variant)
  DevBuf d_slot_g;               // uint8 per staging slot: the pair's reflection
  DevBuf d_M, d_L;               // float2 [ncell][P^2]
  DevBuf d_cops;                 // int2 per cell: (M2M op as child, L2L op as child)
  DevBuf d_stage;                // float2 staging, slots of the largest segment ordered by target: [slots][Sm] then [slots][St]
  DevBuf d_m2l_soff;             // int32 [ncell + 1]: first staging slot of each target cell
  std::vector<int32_t> m2l_targets;  // cells that receive M2L
  std::vector<M2LSeg> m2l_segs;      // staging segments (one unless the staging budget is exceeded)
  int64_t max_seg_slots = 0;
  int stage_bufs = 1;                // segment buffers in the staging (2 with several segments)
  // host work lists (cells / chunks of this instance)
  std::vector<int32_t> src_leaves, tgt_leaves;
  std::vector<std::vector<int32_t>> m2m_cells, l2l_cells;  // per level
  std::vector<int4> m2l_chunks_h;                          // (op, pair begin, pair end, 0)
  std::unique_ptr<struct Batch> self;                      // single-instance execution
  std::unique_ptr<struct Plan64> fp64;                     // FP64 variant (allocated on first use)
  // BIE corrections (caller panel order; pattern in the Tree)
  DevBuf d_near_val;                            // float2 per near nonzero
  DevBuf d_diag;                                // double2: self integral - 3-point self sum
  DevBuf d_self6;                               // double2 [points][6]: curved-element self blocks
  double ki = 0.0;                              // imaginary part of the wavenumber
  int64_t n_near = 0;
  int64_t device_bytes = 0;
  int64_t est_bytes = 0;                 // footprint computed before any allocation
  int64_t bytes_cells = 0, bytes_lists = 0, bytes_exp = 0, bytes_corr = 0;  // its parts
  bool device_ready = false;             // prepare_device completed (set last)
  std::unique_ptr<HostPlanData> hd;      // present between host and device preparation
};

// Device data of the FP64 variant of a plan's product.
struct Plan64 {
  DevBuf d_tables, d_M, d_L;               // double2
  DevBuf d_src_leaves, d_tgt_leaves;       // int32
  DevBuf d_m2m, d_l2l;                     // int32 cells, level by level
  std::vector<int> m2m_off, l2l_off;       // per level offsets
  DevBuf d_chunks;                         // int4 (op, pair begin, pair end, 0)
  int n_chunks = 0;
};

// Fused execution of one or more instances (instance-aware kernels).
// Autotuned phases: the M2L matrix-core kernel and the P2P (per fused
// sequence), and where a BIE handle's GMRES product adds its near
// corrections (per plan).
enum { kPhaseM2L = 0, kPhaseP2P = 1, kNumBatchPhases = 2, kPhaseNear = 2, kNumTunedPhases = 3 };

struct Batch {
  int count = 0, P = 0, maxlev = 0;
  bool damped = false;                // some instance has a complex wavenumber
  std::vector<struct Tree*> trees;
  std::vector<Plan*> plans;
  std::vector<InstDev> hinst;
  DevBuf d_inst;
  DevBuf d_zero, d_gather, d_scatter, d_p2m, d_l2p, d_p2p, d_m2l, d_m2m, d_l2l, d_red;
  DevBuf d_m2m_cols, d_l2l_cols;      // M2M / L2L column entries (see launch_m2m / launch_l2l)
  int n_zero = 0, n_gather = 0, n_scatter = 0, n_p2m = 0, n_l2p = 0, n_p2p = 0, n_m2l = 0, n_red = 0;
  std::vector<int> m2m_off, l2l_off;  // per level offsets into d_m2m / d_l2l
  int nseg = 1;                       // M2L staging segments
  std::vector<int> m2l_seg_off, red_seg_off;  // per segment offsets into d_m2l / d_red
  std::vector<int64_t> seg_slot_base;         // first staging slot of each segment
  hipStream_t stream = nullptr;       // private stream for graph capture / replay
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipStream_t side = nullptr;         // P2P, concurrent with the far field
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t red = nullptr;          // M2L reductions of earlier segments beside the M2L of later ones
  std::vector<hipEvent_t> ev_m2l, ev_red;  // per segment: its M2L done, its reduction done
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int variant[kNumBatchPhases] = {-1, -1};        // launch shapes chosen by the autotuner
  int graph_variant[kNumBatchPhases] = {-1, -1};  // shapes captured in the graph
  bool ran = false;                   // has run at least once
  ~Batch();
};

int build_batch(const std::vector<struct Tree*>& trees, const std::vector<Plan*>& plans, Batch& b);
// Launch-shape autotuning: forced shape per phase (-1: tuned), the shape a
// batch uses, and the per-phase shape counts.
int phase_variant_count(int phase, int P);
int set_variant_override(int phase, int variant);
int variant_override(int phase);  // forced variant of a phase, -1 if none
int batch_variant(const Batch& b, int phase);
// First-use setup of a batch: the autotuned launch shapes (times the shapes on
// the batch's own work), the side stream and its events.  run_batch calls it;
// calling it earlier keeps that work out of the first product.
int ready_batch(Batch& b, hipStream_t s);
// Runs the fused FMM sequence; xs/ys are caller vectors per instance.  With
// use_graph the sequence is captured once and replayed on a private stream.
int run_batch(Batch& b, const float2* const* xs, float2* const* ys, hipStream_t s, bool use_graph,
              struct Tree* timing);

struct Tree {
  HostTree h;                   // bodies and base cells
  int ncrit = 64, max_level = 20;
  double theta = 0.5, kappa = -1.0, eta = 2.0;
  double k_imag = 0.0;          // imaginary part of the wavenumber (damping), point handles
  int64_t stage_bytes = int64_t(32) << 30;  // M2L staging budget
  int bie_treatment = 0;        // 0: self + near corrections, 1: self only, 2: none
  int near_levels = 3, near_order = 6;
  // BIE data
  bool bie = false;
  int64_t npanel = 0;
  std::vector<double> verts;    // nv x 3
  std::vector<int32_t> tris;    // nt x 3
  // device bodies
  bool uploaded = false;
  DevBuf d_src_pos, d_tgt_pos;  // float4, sorted
  DevBuf d_src_idx;             // int32 per sorted source: caller unknown index
  DevBuf d_src_w;               // float per sorted source (BIE: area/3)
  DevBuf d_tgt_perm;            // int32 per sorted target: caller index
  DevBuf d_panels;              // double [npanel][9] vertex coordinates (BIE)
  // BIE near pattern (geometry only), caller panel order
  std::vector<int32_t> near_off, near_col;
  DevBuf d_near_off, d_near_row, d_near_col;
  bool near_ready = false;      // near pattern and geometry are on the device
  DevBuf d_gl;                  // Gauss-Legendre nodes/weights on [0,1]: near (n), self (10)
  // curved-element Nystrom handle: unknowns are the six points of each
  // element (npanel = 6 x elements), element-major
  bool nystrom = false;
  std::vector<double> nys_elem;  // [elements][6 nodes][3]
  std::vector<double> nys_pts;   // [points][3]
  std::vector<double> nys_jac;   // [points] surface Jacobian
  std::vector<int4> nys_items;   // near pairs (point, element, value position, -)
  DevBuf d_nys_elem, d_nys_pts, d_nys_K, d_nys_rule, d_nys_items;
  int nys_nrule = 0;
  // GMRES workspace (kept between solves)
  int gm_m = 0;
  DevBuf g_ws;                  // one buffer, carved by gmres_carve
  double* g_pin = nullptr;      // pinned status slots of the lagged checks (4 doubles)
  hipEvent_t g_ev[2] = {};
  // the GMRES product's near corrections run on their own stream beside the
  // FMM (created with the lagged-check slots; absent: they run after it)
  hipStream_t n_stream = nullptr;
  hipEvent_t n_ev[2] = {};
  DevBuf d_q, d_ys;             // float2 per source / target
  DevBuf d_q64, d_ys64;         // double2 per source / target (FP64 variant)
  int64_t body_bytes = 0;
  std::map<std::pair<uint64_t, int>, std::unique_ptr<Plan>> plans;
  bool timing = false;
  float phase_ms[10] = {0};
  hipEvent_t ev[10] = {};
  bool ev_made = false;
  uint64_t uid = 0;
  ~Tree();
};

double kappa_of(const Tree& t, int P);
int build_plan_host(Tree& t, double k, int P, Plan& pl);   // cells + lists (host only)
// Host lists, device operators and (BIE) corrections for (k, P).
int prepare_operators(Tree& t, double k, int P, hipStream_t s, Plan** out);
// prepare_operators plus the execution state of a single product (its work
// lists, autotuned launch shape and side stream): a product then allocates
// nothing.
int prepare(Tree& t, double k, int P, hipStream_t s, Plan** out);
int prepare_host(Tree& t, double k, int P, Plan** out);   // lists, operators, work (host only)
int prepare_device(Tree& t, Plan& pl, hipStream_t s);      // upload and table generation
int matvec_impl(Tree& t, Plan& pl, const float2* x, float2* y, hipStream_t s);
int prepare_bie(Tree& t, Plan& pl, hipStream_t s);
int prepare_nystrom(Tree& t, Plan& pl, hipStream_t s);
// parametric weight of curved-element point p (p mod 6 selects the point)
float nystrom_weight(int64_t p);
int check_kP(double k, int P);
uint64_t next_uid();
void forget_tree_batches(uint64_t uid);
template <class T>
int upload_vec(DevBuf& b, const std::vector<T>& v, bool grow_only = false) {
  int rc = grow_only ? b.ensure(v.size() * sizeof(T)) : b.alloc(v.size() * sizeof(T));
  if (rc) return rc;
  if (!v.empty() && hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("hipMemcpy upload failed");
    return HFMM_EHIP;
  }
  return HFMM_OK;
}
int upload_bodies(Tree& t);
int64_t body_bytes(const Tree& t);
// Device workspace of one GMRES(m) solve on n unknowns: pointers into one
// buffer of gmres_workspace_bytes(n, m) bytes (256-byte aligned parts).
struct GmresWork {
  double2 *V, *w, *r, *H, *sn, *g, *h, *h2, *part, *dot, *yv;
  float2 *x64, *y64, *z64;  // product input, FMM output, near-correction sums
  double *cs, *st;
};
int64_t gmres_workspace_bytes(int64_t n, int m);
GmresWork gmres_carve(void* base, int64_t n, int m);
// Lagged convergence checks of GMRES: two pinned status slots (2 doubles
// each) and their events.
struct GmresLag {
  double* pin = nullptr;
  hipEvent_t ev[2] = {};
};
// Restarted GMRES(m) of a BIE handle on a prepared plan, in workspace W
// (contents on entry do not matter).  Allocates nothing.  With lag, each
// Arnoldi step's status is read one step late (no host wait between
// steps); without, right after the step.  Both give the same bits.
int gmres_run(Tree& t, Plan& pl, const GmresWork& W, int m, const double2* b, double2* x, double tol,
              int maxit, hfmm_gmres_info* info, hipStream_t s, const GmresLag* lag);

}  // namespace hfmm
