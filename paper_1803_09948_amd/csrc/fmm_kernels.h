// Launchers of the HIP kernels (declared for the host code).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hfmm {

constexpr int kMaxP = 16;

struct OpDescDev {         // translation operator descriptor (48 bytes)
  double t[3];             // translation vector
  double rho_in, rho_out;  // scale of the input / output coefficients
  int32_t kind;            // 0: M2M, 1: L2L, 2: M2L
  int32_t pad;
};

// Padded table dimensions: Kp = 4 ceil(P^2/4) inputs, Rp = 16 ceil(P^2/16) outputs.
void table_dims(int P, int* Kp, int* Rp);
// Rows of an M2L staging slot: Sm rows in whole 16-row tiles (whole 128-byte
// lines) and St rows of a partly filled last tile (P^2 mod 16, rounded up to
// even), kept in a separate dense tail array; St = 0 when 16 divides P^2.
void stage_dims(int P, int* Sm, int* St);
// k + i ki: complex wavenumber (ki = 0: real)
void launch_gen_tables(const OpDescDev* ops, int nops, int P, double k, double ki, const int32_t* cp_off,
                       const int32_t* cp_lm, const double2* cp_val, float2* tables,
                       hipStream_t s);
// The same tables in FP64 (precision reference).
void launch_gen_tables64(const OpDescDev* ops, int nops, int P, double k, const int32_t* cp_off,
                         const int32_t* cp_lm, const double2* cp_val, double2* tables, hipStream_t s);
// Pointers of one problem instance, read by every instance-aware kernel.
struct InstDev {
  const float4* spos;       // sorted sources (x, y, z, -)
  const float4* tpos;       // sorted targets
  const int32_t* src_idx;   // sorted source -> caller unknown
  const float* src_w;       // source weights or NULL
  const int32_t* tgt_perm;  // sorted target -> caller index
  const float2* x;          // caller input (set per call)
  float2* y;                // caller output (set per call)
  float2* q;                // sorted source strengths
  float2* ys;               // sorted outputs
  const int4* cells;        // (sb, se, tb, te)
  const float4* geo;        // (cx, cy, cz, half)
  const int32_t* clev;      // level
  const int4* topo;         // (child begin, child end, parent, octant | level << 3)
  const int2* cops;         // per cell: (M2M op as child, L2L op as child)
  const double* rho;        // per level scale
  const float2* tables;     // [op][Kp][Rp]
  float2* M;                // multipoles [ncell][P^2]
  float2* L;                // locals [ncell][P^2]
  const int4* m2l_pairs;    // (target, source, symmetry, staging slot)
  float2* stage;            // M2L staging [slots][Sm] (canonical frame), slots ordered by target
  float2* stage_tail;       // the last St rows of each slot [slots][St] (see stage_dims)
  const uint8_t* slot_g;    // per staging slot: reflection of its pair
  const int32_t* m2l_soff;  // per cell: first staging slot (ncell + 1 entries)
  const int4* p2p_work;     // (tgt begin, tgt end, interval begin, interval end)
  const int2* p2p_ivals;    // (src begin, src end)
  const int32_t* p2p_total; // sources per work item
  int64_t nsrc, ntgt, ncellP2;
  float k;
  float ki;                 // imaginary part of the wavenumber (damping), >= 0
};

struct XYPtrs {
  const float2* x[64];
  float2* y[64];
};

int elem_chunk();
void launch_set_xy(int count, int base, const XYPtrs& p, InstDev* insts, hipStream_t s);
void launch_zero(const int2* items, int n, const InstDev* insts, hipStream_t s);
void launch_gather(const int2* items, int n, const InstDev* insts, hipStream_t s);
void launch_scatter(const int2* items, int n, const InstDev* insts, hipStream_t s);
// damped: some instance has ki != 0 (kernels with the complex radial
// functions / decay factor; they are exact for ki = 0 too)
void launch_p2m(const int2* items, int n, const InstDev* insts, int P, bool damped, hipStream_t s);
// M2M / L2L items: (instance, op, first column entry, count <= 16).  M2M
// column entries are 9 int32 (parent, child of octant 0..7 or -1) and op is
// the octant-0 operator of the child level; L2L entries are 2 int32 (child,
// parent), all children of one item sharing the operator op.
void launch_m2m(const int4* items, int n, const int32_t* cols, const InstDev* insts, int P, hipStream_t s);
void launch_l2l(const int4* items, int n, const int32_t* cols, const InstDev* insts, int P, hipStream_t s);
void launch_l2p(const int2* items, int n, const InstDev* insts, int P, bool damped, hipStream_t s);
void launch_p2p(const int2* items, int n, const InstDev* insts, bool damped, hipStream_t s);
int m2l_pairs_per_chunk(int P);
// chunks: (instance, op, pair begin, pair end), sorted by (instance, op)
// L[t] = sum of the staging slots of t, each mapped back by its reflection's
// output codes omap [16][P^2] (items: instance, target cell)
// slot_base: first staging slot of the segment (the staging buffer holds
// slots [slot_base, ...) of the targets in items)
void launch_m2l_reduce(const int2* items, int n, const InstDev* insts, const int32_t* omap, int P,
                       int64_t slot_base, hipStream_t s);
// per pair: reflected multipoles through the canonical operator into the pair's staging slot
// variant < m2l_variant_count(P) selects the launch shape (results are identical)
int m2l_variant_count(int P);
// bmap: [17][Kp] input codes of the reflections (m2l_input_codes)
void launch_m2l(const int4* chunks, int nchunks, const InstDev* insts, const int32_t* bmap, int P, int variant,
                hipStream_t s);

}  // namespace hfmm
