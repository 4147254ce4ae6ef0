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
hipError_t launch_compress(const void* spec, double* lam64, float* lam32, double* imax, int comp, int nx,
                           int ny, int nz, int kxs, double scale, hipStream_t s);

// ---- krylov.hip (all vectors FP64, length n)
hipError_t dot_partial(const double* a, const double* b, long long n, double* partials, hipStream_t s);
hipError_t reduce_to(const double* partials, double* scal, int slot, int mode, hipStream_t s);  // mode 0 sum, 1 max
hipError_t vec_add(const double* a, const double* b, double* out, long long n, double* partials,
                   hipStream_t s);  // out = a + b, partials of |out|^2
hipError_t vec_copy_scale(const double* a, double alpha, double* out, long long n, hipStream_t s);
hipError_t vec_sub(const double* a, const double* b, double* out, long long n, double* partials,
                   hipStream_t s);  // out = a - b, partials of |out|^2
hipError_t vec_axpy_inplace(double* x, const double* d, const double* scal, int slot, long long n,
                            hipStream_t s);  // x += scal[slot] d
hipError_t vec_zero(double* a, long long n, hipStream_t s);
hipError_t tfqmr_init(const double* r0, double* w, double* u, double* rt, double* d, double* x, long long n,
                      hipStream_t s);
hipError_t tfqmr_half0(double* x, double* u2, const double* u, const double* v, double* w, const double* au,
                       double* d, const double* scal, bool apply_x, long long n, double* partials,
                       hipStream_t s);
hipError_t tfqmr_half1(double* x, double* w, const double* au2, double* d, const double* u2,
                       const double* scal, long long n, double* partials, hipStream_t s);
hipError_t tfqmr_rho(double* x, const double* d, const double* w, const double* rt, const double* scal,
                     long long n, double* partials, hipStream_t s);
hipError_t tfqmr_u(double* u, const double* w, const double* u2, const double* scal, long long n,
                   hipStream_t s);
hipError_t tfqmr_v(double* v, const double* au, const double* au2, const double* rt, const double* scal,
                   long long n, double* partials, hipStream_t s);
hipError_t tfqmr_v0(double* v, const double* au, const double* rt, long long n, double* partials,
                    hipStream_t s);
hipError_t sc_init(double* scal, hipStream_t s);     // rho = sigma... set from S_B2 etc.
hipError_t sc_alpha(double* scal, hipStream_t s);
hipError_t sc_half(double* scal, bool record_tau0, hipStream_t s);
hipError_t sc_beta(double* scal, hipStream_t s);
hipError_t vec_finite_check(const double* a, long long n, double* partials, hipStream_t s);

// ---- mot_api.hip: history MAC and excitation
hipError_t launch_mac(const void* ring, const void* lamh, void* out, int f64, int nl, int nvalid, int head,
                      int nx, int ny, int nz, int kxs, hipStream_t s);
hipError_t launch_einc(const mot_pulse* p, double t, const double* eps, double* out, int nx, int ny, int nz,
                       hipStream_t s);

}  // namespace motimpl
