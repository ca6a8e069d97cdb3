// Launchers of the boundary-integral and GMRES kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hfmm {

// k + i ki: the wavenumber (ki >= 0 damps)
void launch_self(int64_t npan, const double* pan, double k, double ki, const double* gx, const double* gw, int ng,
                 double2* diag, hipStream_t s);
void launch_near(int64_t nnz, const int32_t* rows, const int32_t* cols, const double* pan, double k, double ki,
                 int L, const double* gx, const double* gw, int ng, float2* val, hipStream_t s);
// y_i += (sum over row i's near entries in a fixed order) in one FP32 add;
// with overwrite, y_i = that sum (the caller adds it later, the same add)
void launch_near_apply(int64_t n, const int32_t* off, const int32_t* col, const float2* val,
                       const double2* diag, const float2* x, float2* y, hipStream_t s, bool overwrite = false);
void launch_plane_wave(int64_t n, const double* pan, double k, double ki, const double* d, double2* b,
                       hipStream_t s);
void launch_to_c64(int64_t n, const double2* a, float2* b, hipStream_t s);
// out = (y [+ z in FP32]) + diag v in FP64
void launch_from_c64_diag(int64_t n, const float2* y, const double2* diag, const double2* v, double2* out,
                          hipStream_t s, const float2* z = nullptr);
int mdot_blocks();
// h[0..nv) (+)= V[0..nv)^H w, nv <= 32, V rows with stride ld
void launch_mdot(int64_t n, int nv, const double2* V, int64_t ld, const double2* w, double2* partial,
                 double2* h, int accumulate, hipStream_t s);
// w += sign * V[0..nv) coef
void launch_mupdate(int64_t n, int nv, const double2* V, int64_t ld, const double2* coef, double2* w,
                    double sign, hipStream_t s);
void launch_scale_by_norm(int64_t n, const double2* src, const double2* dotval, double2* dst, hipStream_t s);
void launch_residual(int64_t n, const double2* b, double2* r, hipStream_t s);
void launch_zero_c128(int64_t n, double2* x, hipStream_t s);  // x[0..n) = 0 (a kernel, capture-safe)
void launch_givens(int j, int m, const double2* h, const double2* wn, double2* H, double* cs, double2* sn,
                   double2* g, double* st, hipStream_t s);
void launch_backsolve(int kk, int m, const double2* H, const double2* g, double2* y, hipStream_t s);
void launch_vec_add(int n, const double2* a, double2* b, hipStream_t s);
void launch_init_g(int m, const double2* dotval, double2* g, hipStream_t s);

}  // namespace hfmm
