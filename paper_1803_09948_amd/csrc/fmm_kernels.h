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
void launch_gen_tables(const OpDescDev* ops, int nops, int P, double k, const int32_t* cp_off,
                       const int32_t* cp_lm, const double2* cp_val, float2* tables,
                       hipStream_t s);
void launch_gather(int64_t n, const int32_t* idx, const float* w, const float2* x, float2* q,
                   hipStream_t s);
void launch_scatter(int64_t n, const int32_t* perm, const float2* ys, float2* y, hipStream_t s);
void launch_p2m(const int32_t* leaves, int nleaves, const int4* cells, const float4* geo,
                const int32_t* clev, const double* rho, const float4* spos, const float2* q,
                float k, int P, float2* M, hipStream_t s);
void launch_m2m(int c0, int c1, const int4* topo, const int32_t* base, const float2* tables,
                int P, float2* M, hipStream_t s);
void launch_l2l(int c0, int c1, const int4* topo, const int32_t* base, const float2* tables,
                int P, float2* L, hipStream_t s);
void launch_m2l(const int4* chunks, int nchunks, const int4* pairs, const float2* tables,
                const int32_t* symdst, const int32_t* symph, const int32_t* outidx,
                const int32_t* outph, int P, const float2* M, float2* L, hipStream_t s);
void launch_l2p(const int32_t* leaves, int nleaves, const int4* cells, const float4* geo,
                const int32_t* clev, const double* rho, const float4* tpos, float k, int P,
                const float2* L, float2* ys, hipStream_t s);
void launch_p2p(const int4* work, int nwork, const int2* ivals, const int32_t* ivlen_total,
                const float4* tpos, const float4* spos, const float2* q, float k, float2* ys,
                hipStream_t s);
int m2l_chunk_size();
// Matrix-core M2L over padded tables [op][Kp][Rp] (see fmm_kernels.hip).
int m2l_pairs_per_chunk(int P);
void launch_m2l_mfma(const int4* chunks, int nchunks, const int4* pairs, const float2* tables, int P,
                     const int32_t* symdst, const int32_t* symph, const int32_t* outidx,
                     const int32_t* outph, const float2* M, float2* L, hipStream_t s);

}  // namespace hfmm
