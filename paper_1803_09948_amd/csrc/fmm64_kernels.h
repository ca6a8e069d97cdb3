// FP64 variant of the FMM product (precision reference) and an FP64 direct
// sum: launchers, declared for the host code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fmm_kernels.h"

namespace hfmm {

// Device pointers of one point-mode instance for the FP64 product; the
// tree, lists and operator descriptors are those of the FP32 plan.
struct F64Dev {
  const float4* spos;        // sorted sources
  const float4* tpos;        // sorted targets
  const int32_t* src_idx;    // sorted source -> caller index
  const int32_t* tgt_perm;   // sorted target -> caller index
  const int4* cells;         // (sb, se, tb, te)
  const float4* geo;         // (cx, cy, cz, half)
  const int32_t* clev;       // level
  const int4* topo;          // (child begin, child end, parent, octant | level << 3)
  const int2* cops;          // per cell: (M2M op as child, L2L op as child)
  const double* rho;         // per level scale
  const double2* tables;     // FP64 translation tables [op][Kp][Rp]
  double2* M;                // multipoles [ncell][P^2]
  double2* L;                // locals [ncell][P^2]
  double2* q;                // sorted strengths
  double2* ys;               // sorted outputs
  const int4* m2l_pairs;     // (target, source, reflection, slot)
  const int32_t* bmap;       // [17][Kp] reflection codes
  const int4* p2p_work;      // (tgt begin, tgt end, interval begin, interval end)
  const int2* p2p_ivals;     // (src begin, src end)
  int64_t nsrc, ntgt;
  int32_t ncell, P, Kp, Rp;
  double k;
};

void launch64_gather(const F64Dev& D, const double2* x, hipStream_t s);
void launch64_zero(const F64Dev& D, hipStream_t s);
void launch64_p2m(const F64Dev& D, const int32_t* leaves, int n, hipStream_t s);
void launch64_m2m(const F64Dev& D, const int32_t* parents, int n, hipStream_t s);
// chunks: (op, pair begin, pair end, -), at most 32 pairs each
void launch64_m2l(const F64Dev& D, const int4* chunks, int n, hipStream_t s);
void launch64_l2l(const F64Dev& D, const int32_t* cells, int n, hipStream_t s);
void launch64_l2p(const F64Dev& D, const int32_t* leaves, int n, hipStream_t s);
void launch64_p2p(const F64Dev& D, int nwork, hipStream_t s);
void launch64_scatter(const F64Dev& D, double2* y, hipStream_t s);
// y[i] = sum_{j: R > 0} q_j e^{ikR}/(4 pi R); src [n][3], tgt [m][3] float, device
void launch64_direct(const float* src, const double2* q, int64_t n, const float* tgt, int64_t m, double k,
                     double2* y, hipStream_t s);

}  // namespace hfmm
