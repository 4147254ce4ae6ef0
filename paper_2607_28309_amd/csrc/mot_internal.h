// Internal state and launchers of the MOT-JVIE library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/mot_jvie.h"

namespace motimpl {

// Krylov scalar slots kept in device memory (FP64).
enum Slot {
  S_RHO = 0,
  S_ALPHA,
  S_THETA,
  S_TAU,
  S_ETA,
  S_BETA,
  S_SIGMA,
  S_W2,
  S_RHONEW,
  S_B2,
  S_FLAG,
  S_DCOEF,
  S_R2,
  S_TAU0,
  S_X2,
  S_NSLOT
};

constexpr int RED_BLOCKS = 1024;   // fixed partial count: deterministic reductions
constexpr int RED_THREADS = 256;

// ---- green.hip
hipError_t launch_green(double* out, int nx, int ny, int nz, int k, int alpha, double L, int nq,
                        hipStream_t s);
hipError_t launch_embed(const double* goct, double* E, int comp, int nx, int ny, int nz, hipStream_t s);
int compress_blocks(int nx, int ny, int nz);
// w64 / w32 = 0: [comp][kzc][kyc][kxs] (history lags); > 0: the fused z
// pass's tile layout (motfft::lam_tile_offset) with tiles of that many columns
hipError_t launch_compress(const void* spec, double* lam64, float* lam32, double* imax, int comp, int nx,
                           int ny, int nz, int kxs, double scale, int w64, int w32, hipStream_t s);

// ---- krylov.hip (vectors of length n, element type V = float or double)
// Scalar recurrence applied by the reduction that produced scal[slot].
enum Post { POST_NONE = 0, POST_INIT, POST_ALPHA, POST_HALF0, POST_HALF1, POST_BETA };
hipError_t reduce_post(const double* partials, double* scal, int slot, int post, hipStream_t s);
template <typename V> hipError_t dot_partial(const V* a, const V* b, long long n, double* partials, hipStream_t s);
template <typename V> hipError_t vec_sub(const V* a, const V* b, V* out, long long n, double* partials,
                                         hipStream_t s);  // out = a - b, partials of |out|^2
template <typename V> hipError_t vec_zero(V* a, long long n, hipStream_t s);
hipError_t vec_add64(const double* a, const double* b, double* out, long long n, double* partials,
                     hipStream_t s);  // out = a + b, partials of |out|^2
hipError_t vec_acc_f2d(double* x, const float* d, long long n, hipStream_t s);  // x += d
hipError_t vec_d2f(const double* in, float* out, long long n, double* partials, hipStream_t s);
hipError_t vec_f2d(const float* in, double* out, long long n, hipStream_t s);
hipError_t vec_copy(const double* a, double* out, long long n, hipStream_t s);
template <typename V> hipError_t tfqmr_init(const V* r0, V* w, V* u, V* rt, V* d, V* x, long long n, hipStream_t s);
template <typename V> hipError_t tfqmr_half0(V* u2, const V* u, const V* v, V* w, const V* au, V* d,
                                             const double* scal, long long n, double* partials, hipStream_t s);
template <typename V> hipError_t tfqmr_half1(V* x, V* w, const V* au2, V* d, const V* u2, const double* scal,
                                             long long n, double* partials, hipStream_t s);
template <typename V> hipError_t tfqmr_rho(V* x, const V* d, const V* w, const V* rt, const double* scal,
                                           long long n, double* partials, hipStream_t s);
template <typename V> hipError_t tfqmr_u(V* u, const V* w, const V* u2, const double* scal, long long n,
                                         hipStream_t s);
template <typename V> hipError_t tfqmr_v(V* v, const V* au, const V* au2, const V* rt, const double* scal,
                                         long long n, double* partials, hipStream_t s);
template <typename V> hipError_t tfqmr_v0(V* v, const V* au, const V* rt, long long n, double* partials,
                                          hipStream_t s);

// ---- history.hip: history multiply-accumulate (ring slot t mod nl holds J^_t)
// out = init + sum_{j=1..nrec} Lambda_j J^_{n+1-j}   (init may be null)
hipError_t launch_mac_recent(const void* ring, const void* lamh, const void* init, void* out, int f64, int nl,
                             long long n, int nrec, int nx, int ny, int nz, int kxs, hipStream_t s);
// P_b = sum_{m<nold} Lambda_{m+b} J^_{n0-m}, b = 1..B: P_1 -> out0, P_b -> pblk + (b-2) slots
hipError_t launch_mac_block(const void* ring, const void* lamh, void* out0, void* pblk, int f64, int B, int nl,
                            long long n0, int nold, int nx, int ny, int nz, int kxs, hipStream_t s);

// ---- mot_api.hip: excitation
hipError_t launch_einc(const mot_pulse* p, double t, const double* eps, double* out, int nx, int ny, int nz,
                       hipStream_t s);

}  // namespace motimpl
