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

// M2L in the xz-plane frame.  A translation by t with azimuth phi equals
// D^-1 T(t') D, where t' is t turned about the z axis into the xz-plane
// (t'_y = 0) and D = diag(e^{i m phi}) acts on the (n, m) coefficients.  An
// operator with t'_y = 0 commutes with the exchange m <-> -m, so in the
// basis u = M^m + M^-m, v = M^m - M^-m it splits into a block C on the
// entries with m >= 0 and a block S on the entries with m > 0 (the
// translations of eqs. (12)-(14) under the symmetry of the plane y = 0).
// Entry lists, in this order:
//   S-list: (n, m) for n = 1..P-1, m = 1..n          (S = P(P-1)/2 entries)
//   C-list: the S-list, then (n, 0) for n = 0..P-1   (C = S + P entries)
// for inputs (k) and outputs (rows) alike.  The table of an M2L operator is
// [Kx][Rx]: row r < 16 RTC is C-list output r, row 16 RTC + r is S-list
// output r; input k < 4 KSS feeds both blocks (u for C, v for S), inputs
// 4 KSS <= k < Kx only C (zero padded elsewhere).
struct XzDims {
  int S, C, KSS, KSC, Kx, RTS, RTC, RT, Rx;
};
__host__ __device__ constexpr XzDims xz_dims(int P) {
  const int S = P * (P - 1) / 2, C = S + P;
  const int KSS = (S + 3) / 4, KSC = (C + 3) / 4, RTS = (S + 15) / 16, RTC = (C + 15) / 16;
  return XzDims{S, C, KSS, KSC, 4 * KSC, RTS, RTC, RTC + RTS, 16 * (RTC + RTS)};
}
// Storage order of the coefficients of a multipole M in the FP32 path: the
// pairs (n, m), (n, -m) for the S-list entries e = (n, m), m > 0, at 2e and
// 2e + 1, then (n, 0) at 2S + n, so that the M2L reads both members of a
// pair with one 16-byte load (the local expansions L keep the order
// n^2 + n + m).
__host__ __device__ constexpr int mpos(int P, int n, int m) {
  const int S = P * (P - 1) / 2;
  if (m == 0) return 2 * S + n;
  const int a = m > 0 ? m : -m, e = (n - 1) * n / 2 + (a - 1);
  return 2 * e + (m > 0 ? 0 : 1);
}
// Row stride of the M2L input code table ([17][stride] words): at least Kx
// and 4 more than a multiple of 64, so that the 16 reflections x 4 k-lanes of
// one read fall in distinct LDS banks.
__host__ __device__ constexpr int xz_code_stride(int P) {
  const int kx = xz_dims(P).Kx;
  return kx + ((4 - kx) % 64 + 64) % 64;
}
// Entries per operator in the FP32 tables: the dense Kp x Rp operator
// (M2M, L2L), or the [Kx][Rx] blocks of an M2L operator followed by its P
// azimuth phases e^{i m phi} (m < P), whichever is larger (16-entry aligned).
__host__ __device__ constexpr int xz_table_stride(int P) {
  const XzDims d = xz_dims(P);
  const int dense = (4 * ((P * P + 3) / 4)) * (16 * ((P * P + 15) / 16)), xz = d.Kx * d.Rx + 16;
  return dense > xz ? dense : xz;
}
// (n, m) of entry e of the C-list (m >= 0; the S-list is its first S entries)
__host__ __device__ constexpr void xz_entry(int P, int e, int* n, int* m) {
  const int S = P * (P - 1) / 2;
  if (e >= S) {
    *n = e - S;
    *m = 0;
    return;
  }
  int nn = 1, base = 0;
  while (base + nn <= e) {
    base += nn;
    ++nn;
  }
  *n = nn;
  *m = e - base + 1;
}
// Layout of one pair's M2L result in its staging slot (float2 positions).
// First the "pm block": for C-list entry e < 16 RTS, position 2e holds
// L^{+m'} (or L^{n'0} for e >= S) and 2e + 1 holds L^{-m'} (unused for
// e >= S), so that the two outputs of an S-list row are one aligned 16-byte
// pair; RTS whole 32-row tiles.  Then the C-only rows e = 16 RTS..C-1
// (L^{n'0}), in 16-row tiles: the whole ones follow the pm block, a last
// partial one (padded to an even row count) goes to a dense tail array.
// Sm = 32 RTS + 16 (whole C-only tiles) positions per slot in the main array
// (whole 128-byte lines), St in the tail.
__host__ __device__ constexpr int xz_co_rows(int P) {  // C-only rows
  const XzDims d = xz_dims(P);
  return d.C - 16 * d.RTS > 0 ? d.C - 16 * d.RTS : 0;
}
__host__ __device__ constexpr int xz_stage_sm(int P) {
  return 32 * xz_dims(P).RTS + 16 * (xz_co_rows(P) / 16);
}
__host__ __device__ constexpr int xz_stage_st(int P) {
  const int rem = xz_co_rows(P) % 16;
  return 2 * ((rem + 1) / 2);
}
// staging position of C-list entry e's output: sign +1 (L^{+m'}, or L^{n'0}
// for m' = 0) or -1 (L^{-m'}); positions >= Sm are in the tail
__host__ __device__ constexpr int xz_stage_pos(int P, int e, int sign) {
  const XzDims d = xz_dims(P);
  if (e < 16 * d.RTS) return 2 * e + (sign < 0 ? 1 : 0);
  return 32 * d.RTS + (e - 16 * d.RTS);
}
// Positions of an M2L staging slot: Sm in the main array, St in the tail
// (see xz_stage_pos); Sm + St >= P^2.
void stage_dims(int P, int* Sm, int* St);
// k + i ki: complex wavenumber (ki = 0: real).  FP32 tables, xz_table_stride
// entries per operator; the M2L operators (t the canonical offset) are
// stored in the xz-plane form with their azimuth phases.
void launch_gen_tables(const OpDescDev* ops, int nops, int P, double k, double ki, const int32_t* cp_off,
                       const int32_t* cp_lm, const double2* cp_val, float2* tables,
                       hipStream_t s);
// The dense tables in FP64 (precision reference), Kp * Rp entries per operator.
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
  const int4* m2l_pairs;    // (target, source, reflection, staging slot)
  float2* stage;            // M2L staging [slots][Sm] (reflected frame, xz_stage_pos), slots ordered by target
  float2* stage_tail;       // the tail positions of each slot [slots][St] (see stage_dims)
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
// variant < p2p_variant_count() selects the launch shape (results are identical)
int p2p_variant_count();
void launch_p2p(const int2* items, int n, const InstDev* insts, bool damped, int variant, hipStream_t s);
int m2l_pairs_per_chunk(int P);
// chunks: (instance, op, pair begin, pair end), sorted by (instance, op)
// L[t] = sum of the staging slots of t, each mapped back by its reflection's
// output codes omap [16][P^2] (m2l_xz_codes; items: instance, target cell)
// slot_base: first staging slot of the segment (the staging buffer holds
// slots [slot_base, ...) of the targets in items)
void launch_m2l_reduce(const int2* items, int n, const InstDev* insts, const int32_t* omap, int P,
                       int64_t slot_base, hipStream_t s);
// per pair: reflected multipoles through the canonical operator into the pair's staging slot
// variant < m2l_variant_count(P) selects the launch shape (results are identical)
int m2l_variant_count(int P);
// bmap: [17][Kx][2] input codes of the reflections, then the m' of the
// S-list rows (m2l_xz_codes)
void launch_m2l(const int4* chunks, int nchunks, const InstDev* insts, const int32_t* bmap, int P, int variant,
                hipStream_t s);

}  // namespace hfmm
