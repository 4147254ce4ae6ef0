// C ABI of the MOT-JVIE hot path: context, Z0 product (Eq. 11/12), history
// update, excitation (Eq. 7/8) and the MOT step (Eq. 3) with a
// device-resident TFQMR solve.  See include/mot_jvie.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "fft_core.h"
#include "fft_passes.h"
#include "mot_internal.h"

using motfft::cpx;
using namespace motimpl;

// Tile-variant knobs per compute precision (tune[0] FP32, tune[1] FP64): the
// x passes, the y passes, the history z passes and the fused z pass.
enum { TUNE_X = 0, TUNE_Y, TUNE_Z, TUNE_ZF, TUNE_N };

struct mot_ctx {
  mot_grid grid;
  int nx, ny, nz, px, py, pz, kx, kxs, nl, alpha, nq;
  double L;
  long long N, n3;
  mot_precision prec;
  int ring_f64;
  hipStream_t stream;
  // twiddles: [0] float, [1] double
  void* twx[2];
  void* tw2x[2];
  void* twy[2];
  void* twz[2];
  double* eps;
  bool have_eps, have_spectra;
  // right diagonal scaling of the solver's Z0: rs = 1 / diag(Z0) per voxel,
  // diag(Z0) = eps/2 - (eps - 1) G0(0)_pp (G0(0) is isotropic)
  double g0self;       // G0(0)_xx
  float* rs32;
  float* eps32;  // eps_r rounded to FP32: the epilogues of the FP32 passes
  double* rs64;
  double* lam0_64;
  float* lam0_32;
  void* lamh;          // lags 1..nl, ring precision
  size_t lam_comp;     // elements per component per lag: (nz+1)(ny+1)kxs
  void* wsA;
  void* wsB;
  void* spec;          // MAC output, ring precision, 3*pz*py*kxs complex
  void* ring;
  size_t slot_elems;   // complex elements per ring slot
  int blk_B;           // steps per history block (temporal blocking)
  int mac_wide = 0;    // 1: the block multiply-accumulate takes 64-bit addresses
  long long blk_n0;    // step that started the current block, -1 = none
  void* pblk;          // partial sums P_2..P_B of the current block
  // history scheme: 0 = chosen by the library, 1 = blocked multiply-accumulate
  // over all lags, 2 = far lags by FFTs in time over blocks of TF_S steps
  int hist_scheme;
  bool tf_on;          // the far lags go through FFTs in time
  bool tf_ready;       // tfK holds the transforms of the current spectra
  void* tfK;           // K_m(w), m = 1..M, w = 0..TF_S (FP32 complex)
  void* tfar;          // far parts of the next TF_S right-hand sides
  long long tf_beta;   // time block whose far parts tfar holds, -1 = none
  long long nstep;
  int head;
  double* hrhs;
  double* kv[13];      // FP64 Krylov vectors
  float* kf[11];       // FP32 Krylov vectors (FP32 and refined modes)
  double* partials;
  size_t partials_n;   // entries of partials
  double* scal;
  double* hscal;       // pinned host mirror: [0] for synchronous reads, [1], [2] for the solver's queue
  hipEvent_t ev[3];
  hipEvent_t evq[2];   // the solver's queue: scalars of iteration m copied to bank 1 + (m & 1)
  // TFQMR iterations as graphs: [FP64 vectors][adjoint][with residual check]
  int use_graphs;
  hipStream_t cap_stream;   // capture only; graphs are launched on `stream`
  // mode 2: the refined solve's first sweep as one graph (sg_G gated
  // iterations, FP32 tolerance sg_tol, operator sg_adj); sg_hist: the
  // iterations the last 8 first sweeps needed, sg_need their maximum
  hipGraphExec_t sg_exec;
  int sg_G, sg_adj, sg_need, sg_last, sg_pos, sg_hist[8];
  double sg_tol;
  hipGraphExec_t iter_graph[2][2][2];
  // kernel timing (mot_profile)
  int prof_on, prof_used, prof_cap;
  int prof_mask;       // kinds timed while profiling is on (bit k = kind k)
  hipEvent_t* prof_ev;
  int* prof_cls;
  double prof_ms[MOT_PROF_NCLASS];
  long long prof_cnt[MOT_PROF_NCLASS];
  double spectra_imag;
  void* lam_tile;      // scratch: one history lag in the z-pass layout (gk_matvec)
  int adjoint;         // 1: transposed operators Z_k^T (adjoint march)
  // regularization Z^delta_n = Z_n + dreg[n] diag(eps_r), n = 0, 1, 2 (all
  // zero: the unregularized operator)
  double dreg[3];
  double* jprev2;      // the current pushed before the last one (history term of dreg[2])
  double bd_tol;       // TFQMR near-breakdown tolerance (0: rho or sigma exactly zero)
  double* ffpart;      // scratch: far-field block partials
  size_t ffpart_n;
  int tune[2][TUNE_N]; // tile variants of the FFT passes (0 or 1)
  // initial guess of the refined solve from earlier steps: least squares
  // over the pairs (J_i, Z0 J_i) of the last pred_k steps
  int pred_k;
  int pred_count, pred_head;  // stored pairs; slot of the next one
  bool pred_newrow;           // the newest pair's Gram row is still to be formed
  double* pred_j[PRED_MAX];   // J_i
  double* pred_z[PRED_MAX];   // Z0 J_i
  double pred_G[PRED_MAX][PRED_MAX];  // Gram matrix of the stored Z0 J_i
  double* pred_dots;                  // device: dots of one multidot
  size_t bytes;
  mot_stats last;  // statistics of the last mot_step (host-side values)
  char err[512];
};

namespace {

enum { V_X = 0, V_B, V_W, V_U, V_U2, V_V, V_D, V_AU, V_AU2, V_RT, V_TMP, V_XO, V_RO };

int set_err(mot_ctx* c, int code, const char* fmt, const char* a = "", int line = 0) {
  if (c) snprintf(c->err, sizeof(c->err), fmt, a, line);
  return code;
}
int fail_hip(mot_ctx* c, hipError_t e, const char* what, int line) {
  if (c) snprintf(c->err, sizeof(c->err), "%s failed at line %d: %s", what, line, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? MOT_ENOMEM : MOT_EHIP;
}
#define HT(call)                                                  \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return fail_hip(c, e_, #call, __LINE__); \
  } while (0)
#define TRY(call)          \
  do {                     \
    int r_ = (call);       \
    if (r_ != MOT_OK) return r_; \
  } while (0)

long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

enum Kind { K_XF = 0, K_YF, K_ZFUSED, K_YI, K_XI, K_ZF, K_MAC, K_ZI, K_KRY, K_EINC, K_MACR, K_TFAR };

int prof_flush(mot_ctx* c) {
  if (c->prof_used == 0) return MOT_OK;
  HT(hipEventSynchronize(c->prof_ev[2 * c->prof_used - 1]));
  for (int i = 0; i < c->prof_used; ++i) {
    float ms = 0.f;
    HT(hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]));
    c->prof_ms[c->prof_cls[i]] += ms;
    c->prof_cnt[c->prof_cls[i]] += 1;
  }
  c->prof_used = 0;
  return MOT_OK;
}

// Brackets one launch with an event pair when timing is on.
struct Prof {
  mot_ctx* c;
  int idx = -1;
  Prof(mot_ctx* c_, int kind, bool f64) : c(c_) {
    if (!c->prof_on || !((c->prof_mask >> kind) & 1)) return;
    if (c->prof_used == c->prof_cap && prof_flush(c) != MOT_OK) return;
    idx = c->prof_used++;
    c->prof_cls[idx] = 2 * kind + (f64 ? 1 : 0);
    (void)hipEventRecord(c->prof_ev[2 * idx], c->stream);
  }
  ~Prof() {
    if (idx >= 0) (void)hipEventRecord(c->prof_ev[2 * idx + 1], c->stream);
  }
};
#define PROF(kind, f64) Prof prof_scope_##__LINE__(c, kind, f64)
#define HTP(kind, f64, call) \
  do {                       \
    Prof p_(c, kind, f64);   \
    HT(call);                \
  } while (0)

int nlags_of(const mot_grid* g) {
  if (g->nlags > 0) return g->nlags;
  const long long ax = 2LL * g->nx - 1, ay = 2LL * g->ny - 1, az = 2LL * g->nz - 1;
  if (g->alpha > 0) {
    // least c with (2 c alpha)^2 >= 3 sum (2N_i - 1)^2
    const long long m = 3 * (ax * ax + ay * ay + az * az);
    long long c = (long long)floor(sqrt((double)m) / (2.0 * g->alpha));
    if (c < 0) c = 0;
    while ((2 * c * g->alpha) * (2 * c * g->alpha) < m) ++c;
    while (c > 0 && (2 * (c - 1) * g->alpha) * (2 * (c - 1) * g->alpha) >= m) --c;
    return (int)c + 2;
  }
  const double rmax = 0.5 * sqrt((double)(ax * ax + ay * ay + az * az));
  return (int)ceil(rmax / g->cdt) + 2;
}

bool grid_ok(const mot_grid* g) {
  if (!g || g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || (g->nx & 1)) return false;
  if (g->alpha < 0 || (g->alpha == 0 && !(g->cdt > 0.0))) return false;
  if (g->quad < 0 || g->quad > 32 || g->quad == 1) return false;
  return motfft::length_supported(g->nx) && motfft::length_supported(2 * g->ny) &&
         motfft::length_supported(2 * g->nz);
}

__global__ void k_fill_zero(uint4* p, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

int zero_bytes(mot_ctx* c, void* p, size_t bytes) {
  if (!p || bytes == 0) return MOT_OK;
  hipLaunchKernelGGL(k_fill_zero, dim3(2048), dim3(256), 0, c->stream, (uint4*)p, bytes / 16);
  HT(hipGetLastError());
  return MOT_OK;
}

int dmalloc(mot_ctx* c, void** p, size_t bytes);

// Far lags by FFTs in time: possible with an FP32 ring of at least TF_S
// lags; chosen by default from TF_AUTO_LAGS lags on.  The per-lag
// multiply-accumulate does O(nl) multiply-adds per frequency and step, the
// transforms O(nl / TF_S) blocks of 2 TF_S frequencies, but below ~100 lags
// the blocked pass is as fast on the 96^3 cube (measured history time per
// step: ell 289 0.81 against 1.15 ms, 146 0.59 / 0.71, 74 0.52 / 0.50).
constexpr int TF_AUTO_LAGS = 128;
// (the far kernel addresses one ring slot and one plane of K with 32-bit
// byte offsets)
bool tf_possible(const mot_ctx* c) {
  return !c->ring_f64 && c->nl >= TF_S && c->blk_B == 8 && 8 * c->slot_elems < (1ull << 32) &&
         8 * (TF_S + 1) * c->lam_comp < (1ull << 32);
}

// Resolve the history scheme; allocate its buffers and, once the spectra
// exist, their transforms in time.
int tf_configure(mot_ctx* c) {
  const bool want = c->hist_scheme == 2 || (c->hist_scheme == 0 && tf_possible(c) && c->nl >= TF_AUTO_LAGS);
  c->tf_on = want && tf_possible(c);
  if (!c->tf_on) return MOT_OK;
  if (!c->tfK) {
    const size_t kb = sizeof(float) * 2 * (size_t)tfft_blocks(c->nl) * (TF_S + 1) * 6 * c->lam_comp;
    TRY(dmalloc(c, &c->tfK, kb));
  }
  if (!c->tfar) TRY(dmalloc(c, &c->tfar, sizeof(float) * 2 * c->slot_elems * TF_S));
  if (c->have_spectra && !c->tf_ready) {
    HT(launch_tfft_prep((const float*)c->lamh, c->tfK, c->nl, c->nx, c->ny, c->nz, c->kxs, c->stream));
    c->tf_ready = true;
  }
  return MOT_OK;
}

int dmalloc(mot_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return MOT_OK;
  bytes = (size_t)round_up((long long)bytes, 256);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    snprintf(c->err, sizeof(c->err), "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return MOT_ENOMEM;
  }
  c->bytes += bytes;
  return MOT_OK;
}

// exp(-2 pi i q / M), q = 0..count-1, in both precisions
int make_twiddles(mot_ctx* c, int M, int count, void** out) {
  std::vector<double> d(2 * count);
  std::vector<float> f(2 * count);
  for (int q = 0; q < count; ++q) {
    // angle reduced to [0, pi/4]-accurate evaluation via long double
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)q / (long double)M;
    d[2 * q] = (double)cosl(a);
    d[2 * q + 1] = (double)sinl(a);
    f[2 * q] = (float)cosl(a);
    f[2 * q + 1] = (float)sinl(a);
  }
  TRY(dmalloc(c, &out[0], sizeof(float) * 2 * count));
  TRY(dmalloc(c, &out[1], sizeof(double) * 2 * count));
  HT(hipMemcpy(out[0], f.data(), sizeof(float) * 2 * count, hipMemcpyHostToDevice));
  HT(hipMemcpy(out[1], d.data(), sizeof(double) * 2 * count, hipMemcpyHostToDevice));
  return MOT_OK;
}

// ---------------------------------------------------------------- excitation
__global__ void k_einc(mot_pulse p, double t, const double* __restrict__ eps, double* __restrict__ out, int nx,
                       int ny, int nz) {
  const long long N = (long long)nx * ny * nz;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  double x, y, z;
  voxel_centre(m, nx, ny, nz, x, y, z);
  const double a = (eps[m] - 1.0) * incident_dt(p, t, x, y, z);
  out[m] = a * p.e[0];
  out[N + m] = a * p.e[1];
  out[2 * N + m] = a * p.e[2];
}

// [6][nz+1][ny+1][kxs] -> tile layout of the fused z pass (tiles of w columns)
template <typename T>
__global__ void k_relayout(const T* __restrict__ src, T* __restrict__ dst, int nx, int ny, int nz, int kxs, int w) {
  const long long cnt = 6LL * (nx + 1) * (ny + 1) * (nz + 1);
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= cnt) return;
  const int kx = (int)(id % (nx + 1));
  long long r = id / (nx + 1);
  const int ky = (int)(r % (ny + 1));
  r /= (ny + 1);
  const int kz = (int)(r % (nz + 1)), comp = (int)(r / (nz + 1));
  dst[motfft::lam_tile_offset(kx, ky, kz, comp, nx + 1, nz + 1, w)] =
      src[(((size_t)comp * (nz + 1) + kz) * (ny + 1) + ky) * kxs + kx];
}

// rs = 1 / (w0 eps - (eps - 1) g0), the inverse diagonal of Z0 per voxel
// (w0 = 1/2 + dreg[0])
// (and eps32 = eps rounded to FP32, read by the epilogues of FP32 passes)
__global__ void k_right_scale(const double* __restrict__ eps, double g0, double w0, float* __restrict__ rs32,
                              double* __restrict__ rs64, float* __restrict__ eps32, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = 1.0 / (eps[i] * (w0 - g0) + g0);
  rs64[i] = r;
  rs32[i] = (float)r;
  eps32[i] = (float)eps[i];
}

// fused z pass tile layout of width ws -> the same spectra in width wd
template <typename T>
__global__ void k_retile(const T* __restrict__ src, T* __restrict__ dst, int nx, int ny, int nz, int ws, int wd) {
  const long long cnt = 6LL * (nx + 1) * (ny + 1) * (nz + 1);
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= cnt) return;
  const int kx = (int)(id % (nx + 1));
  long long r = id / (nx + 1);
  const int ky = (int)(r % (ny + 1));
  r /= (ny + 1);
  const int kz = (int)(r % (nz + 1)), comp = (int)(r / (nz + 1));
  dst[motfft::lam_tile_offset(kx, ky, kz, comp, nx + 1, nz + 1, wd)] =
      src[motfft::lam_tile_offset(kx, ky, kz, comp, nx + 1, nz + 1, ws)];
}

}  // namespace

namespace motimpl {
hipError_t launch_einc(const mot_pulse* p, double t, const double* eps, double* out, int nx, int ny, int nz,
                       hipStream_t s) {
  const long long N = (long long)nx * ny * nz;
  hipLaunchKernelGGL(k_einc, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, *p, t, eps, out, nx, ny, nz);
  return hipGetLastError();
}
}  // namespace motimpl

namespace {

// ---------------------------------------------------------------- Green product
// eps_r in the precision of a pass's epilogue
template <typename T> const T* eps_of(const mot_ctx* c);
template <> const double* eps_of<double>(const mot_ctx* c) { return c->eps; }
template <> const float* eps_of<float>(const mot_ctx* c) { return c->eps32; }

struct NoMid {
  int operator()() const { return MOT_OK; }
};

// y = epilogue(J, G J) with spectra `lam` (precision T) through the five passes.
// kf / ki: solver work fused into the x forward / x inverse pass; mid() is
// enqueued between the x forward and the y forward pass.  With kf, J is the
// x forward pass's solver input (see motfft::Krylov) and `Jd` the vector the
// epilogue's diagonal term reads (the product's actual input).
template <typename T, typename IO, typename Mid = NoMid>
int green_product(mot_ctx* c, const IO* J, IO* y, const T* lam, motfft::Epilogue ep, const double* pre = nullptr,
                  motfft::Gate g = motfft::Gate{}, const motfft::Krylov* kf = nullptr,
                  const motfft::Krylov* ki = nullptr, const IO* Jd = nullptr, Mid mid = Mid{}) {
  const int ti = sizeof(T) == 8 ? 1 : 0;
  hipStream_t s = c->stream;
  const int rows = 3 * c->nz * c->ny;
  const bool d = ti == 1;
  const int* tv = c->tune[ti];
  if (!Jd) Jd = J;
  HTP(K_XF, d, (motfft::x_forward<T, IO>(J, c->wsA, c->nx, rows, c->nz * c->ny, 3, c->nx, c->nx / 2, c->kxs,
                                         c->twx[ti], c->tw2x[ti], s, pre, g, tv[TUNE_X], kf)));
  TRY(mid());
  HTP(K_YF, d, motfft::y_pass<T>(c->wsA, c->wsB, c->py, false, c->kx, c->kxs, 3 * c->nz, c->ny, c->ny, c->py, c->py,
                                 c->twy[ti], s, g, tv[TUNE_Y]));
  HTP(K_ZFUSED, d, motfft::z_pass<T>(c->wsB, c->wsB, c->pz, motfft::Z_FUSED, 3, c->kx, c->kxs, c->py, c->nz, c->nz,
                                     c->nz, c->nz, lam, c->twz[ti], s, g, tv[TUNE_ZF]));
  HTP(K_YI, d, motfft::y_pass<T>(c->wsB, c->wsA, c->py, true, c->kx, c->kxs, 3 * c->nz, c->py, c->py, c->ny, c->ny,
                                 c->twy[ti], s, g, tv[TUNE_Y]));
  HTP(K_XI, d, (motfft::x_inverse<T, IO>(c->wsA, y, Jd, eps_of<T>(c), ep, c->nx, rows, c->nz * c->ny, 3, c->nx, c->nx,
                                         c->kxs, c->twx[ti], c->tw2x[ti], s, g, tv[TUNE_X], ki)));
  return MOT_OK;
}

// Epilogues of the products.  D = (1/2 + dreg[0]) eps_r is the diagonal of
// Z0, (1/2 + dreg[1]) eps_r that of Z1 (dreg = 0 without regularization; the
// dreg[2] eps_r J_{n-1} term of the history rides on its epilogue, Epilogue::jp).
motfft::Epilogue ep_z0(const mot_ctx* c) { return {0.5 + c->dreg[0], 0.0, -1.0, 1.0}; }     // D J - X (G J)
const motfft::Epilogue EP_G{0.0, 0.0, 0.0, 1.0};                                             // G J
motfft::Epilogue ep_hist(const mot_ctx* c) { return {-(0.5 + c->dreg[1]), 0.0, 1.0, -1.0}; } // -(diag Z1) J + X (G J)
// transposed operators (contrast on the input, applied by the forward x pass)
motfft::Epilogue ep_z0t(const mot_ctx* c) { return {0.5 + c->dreg[0], 0.0, 0.0, -1.0}; }      // D v - G (X v)
motfft::Epilogue ep_adj_hist(const mot_ctx* c) { return {-(0.5 + c->dreg[1]), 0.0, 0.0, 1.0}; } // -(diag Z1) v + G (X v)

int reduce_sync(mot_ctx* c) {
  HT(hipMemcpyAsync(c->hscal, c->scal, sizeof(double) * S_NSLOT, hipMemcpyDeviceToHost, c->stream));
  HT(hipStreamSynchronize(c->stream));
  return MOT_OK;
}

struct SolveOut {
  int iters = 0, matvecs = 0, matvecs64 = 0;
  double relres = 0.0;
};

// Z0 product in the precision of the vectors: FP64 vectors -> FP64 FFTs,
// FP32 vectors -> FP32 FFTs.
// In an adjoint context the solver's operator is Z0^T.
// With solver hooks: `in` is the x forward pass's solver input, `jd` the
// product's actual input (see green_product).
template <typename Mid = NoMid>
int apply_z0(mot_ctx* c, const double* in, double* out, motfft::Gate g = motfft::Gate{},
             const motfft::Krylov* kf = nullptr, const motfft::Krylov* ki = nullptr, const double* jd = nullptr,
             Mid mid = Mid{}) {
  if (c->adjoint) return green_product<double, double>(c, in, out, c->lam0_64, ep_z0t(c), c->eps, g, kf, ki, jd, mid);
  return green_product<double, double>(c, in, out, c->lam0_64, ep_z0(c), nullptr, g, kf, ki, jd, mid);
}
template <typename Mid = NoMid>
int apply_z0(mot_ctx* c, const float* in, float* out, motfft::Gate g = motfft::Gate{},
             const motfft::Krylov* kf = nullptr, const motfft::Krylov* ki = nullptr, const float* jd = nullptr,
             Mid mid = Mid{}) {
  if (c->adjoint) return green_product<float, float>(c, in, out, c->lam0_32, ep_z0t(c), c->eps, g, kf, ki, jd, mid);
  return green_product<float, float>(c, in, out, c->lam0_32, ep_z0(c), nullptr, g, kf, ki, jd, mid);
}

template <typename V> struct KV;
template <> struct KV<double> {
  static double** get(mot_ctx* c) { return c->kv; }
};
template <> struct KV<float> {
  static float** get(mot_ctx* c) { return c->kf; }
};

// TFQMR for Z0 x = b from x = 0 (b, x: device vectors of type V, distinct from
// the work vectors).  The convergence test runs on the device: the reduction
// that ends an iteration compares the quasi-residual bound with tol ||b|| and
// asks for the true residual, whose reduction declares the solve done (or
// failed).  Every launch of an iteration is gated on those flags, so the host
// stays one iteration ahead: it enqueues iteration m, then waits only for the
// scalars of iteration m-1 (copied to pinned memory behind an event); an
// iteration enqueued after convergence does nothing.
// bound_only: the quasi-residual bound alone ends the solve (no true
// residual products); the pending x update is applied at the end.
// b64 (FP32 solves only): the right-hand side is the FP64 vector b64 rounded
// to FP32, formed by the start kernel itself (b is then not read: the
// rounded copy r~ = r0 stands in for it).  x64 (FP32 solves only): the
// solution goes to x64 (x64_acc: added to it) instead of x.
// fixed > 0: exactly `fixed` iterations are enqueued (each behind the
// convergence gates, max_iter = fixed) with the final x update, and the call
// returns without waiting for the device or reading its scalars (a sequence
// that a graph can capture; the caller reads the outcome).
template <typename V>
int tfqmr(mot_ctx* c, const V* b, V* x, double tol, int max_iter, SolveOut* so, bool bound_only = false,
          const double* b64 = nullptr, double* x64 = nullptr, bool x64_acc = false, int fixed = 0) {
  hipStream_t s = c->stream;
  const long long n = c->n3;
  V** v = KV<V>::get(c);
  double* P = c->partials;
  double* sc = c->scal;
  const bool f64 = sizeof(V) == 8;
  const motfft::Gate RUN{sc + S_DONE, 1}, CHK{sc + S_DONE, 2};
  HTP(K_KRY, f64, solver_setup(sc, tol, max_iter, s, bound_only, c->bd_tol));
  // w = u = r~ = r0 = b, d = 0, x = 0 (also for b = 0)
  if constexpr (sizeof(V) == 4) {
    if (b64) {
      HTP(K_KRY, f64, tfqmr_init_d2f(b64, v[V_W], v[V_U], v[V_RT], v[V_D], x, n, P, s));
      b = v[V_RT];
    }
  }
  if (!b) return set_err(c, MOT_EINVAL, "TFQMR without a right-hand side%s%d");
  if (sizeof(V) == 8 || !b64) {
    HTP(K_KRY, f64, dot_partial<V>(b, b, n, P, s));
    HTP(K_KRY, f64, tfqmr_init<V>(b, v[V_W], v[V_U], v[V_RT], v[V_D], x, n, s));
  }
  HTP(K_KRY, f64, reduce_post(P, sc, S_B2, POST_INIT, s));
  // the solver's operator is Z0 diag(rs) (right scaling by the inverse
  // diagonal of Z0); its solution y gives x = rs y at the end
  const V* rs = f64 ? (const V*)c->rs64 : (const V*)c->rs32;
  motfft::Krylov ks;
  ks.mode = motfft::KRY_SCALE;
  ks.rs = rs;
  TRY(apply_z0(c, v[V_U], v[V_AU], RUN, &ks, &ks));
  HTP(K_KRY, f64, tfqmr_v0<V>(v[V_V], v[V_AU], v[V_RT], n, P, s, RUN));
  HTP(K_KRY, f64, reduce_post(P, sc, S_SIGMA, POST_ALPHA, s, RUN));
  // The iteration's vector work rides on its products (motfft::Krylov): the
  // first half step on the forward x pass of the product of u2, the second
  // on that product's inverse x pass; u = w + beta u2 on the forward x pass
  // and the v update on the inverse x pass of the product of u; the second
  // half step's x update waits in S_ETAP for the next iteration's first
  // product or for the residual check.  The fused sums leave one partial per
  // x-pass workgroup.
  const int rows = 3 * c->nz * c->ny;
  const int xb = motfft::x_pass_blocks(c->nx, f64, c->tune[f64 ? 1 : 0][TUNE_X], rows, c->nz * c->ny, 3);
  if (xb < 1 || 2 * (size_t)xb > c->partials_n) return set_err(c, MOT_EINVAL, "x pass grid outside the partials%s%d");
  motfft::Krylov kb;
  kb.alpha = sc + S_ALPHA;
  kb.beta = sc + S_BETA;
  kb.eta = sc + S_ETA;
  kb.etap = sc + S_ETAP;
  kb.dcoef = sc + S_DCOEF;
  kb.partials = P;
  kb.stride = xb;
  kb.rs = rs;
  // streaming vector accesses once a vector outgrows the caches' share
  kb.stream = (size_t)n * sizeof(V) >= ((size_t)32 << 20) ? 1 : 0;
  motfft::Krylov kh0 = kb, kh1 = kb, ku = kb, kvv = kb, kfix = kb;
  kh0.mode = motfft::KRY_HALF0;  // in = u
  kh0.v = v[V_V];
  kh0.w = v[V_W];
  kh0.au = v[V_AU];
  kh0.d = v[V_D];
  kh0.x = x;
  kh0.out = v[V_U2];
  kh1.mode = motfft::KRY_HALF1;  // J = u2, y = au2
  kh1.x = x;
  kh1.w = v[V_W];
  kh1.d = v[V_D];
  kh1.rt = v[V_RT];
  ku.mode = motfft::KRY_U;  // in = w
  ku.u2 = v[V_U2];
  ku.out = v[V_U];
  kvv.mode = motfft::KRY_V;  // y = au
  kvv.au = v[V_AU2];
  kvv.v = v[V_V];
  kvv.rt = v[V_RT];
  kfix.mode = motfft::KRY_XFIX;  // in = x
  kfix.x = x;
  kfix.d = v[V_D];
  // one iteration's launches on the context stream (gated; see above); its
  // last reduction writes the scalars to the host bank `mirror` (stream
  // launches only: a captured graph keeps one pointer, so graph replays copy
  // the scalars with a memory copy instead)
  double* mirror = nullptr;
  auto enqueue_iter = [&](bool check) -> int {
    hipStream_t st = c->stream;
    auto half0_sum = [&]() -> int {
      HTP(K_KRY, f64, reduce_post(P, sc, S_W2, POST_HALF0, st, RUN, xb));
      return MOT_OK;
    };
    // u2 = u - alpha v and the first half step; au2 = A u2 and the second
    TRY(apply_z0(c, v[V_U], v[V_AU2], RUN, &kh0, &kh1, v[V_U2], half0_sum));
    HTP(K_KRY, f64, reduce_post2(P, sc, S_W2, POST_HALF1, S_RHONEW, POST_BETA, st, RUN, xb, xb));
    // true residual with the solver's own operator, only when asked for (its
    // forward x pass applies the pending x update)
    if (check) {
      TRY(apply_z0(c, x, v[V_TMP], CHK, &kfix, &ks, x));
      HTP(K_KRY, f64, vec_sub<V>(b, v[V_TMP], v[V_TMP], n, P, st, CHK));
      HTP(K_KRY, f64, reduce_post(P, sc, S_R2, POST_RESID, st, CHK));
    }
    // u = w + beta u2; au = A u and v = au + beta (au2 + beta v)
    TRY(apply_z0(c, v[V_W], v[V_AU], RUN, &ku, &kvv, v[V_U]));
    HTP(K_KRY, f64, reduce_post(P, sc, S_SIGMA, POST_ALPHA, st, RUN, xb, mirror));
    return MOT_OK;
  };
  // graph mode: the same launches captured once per (precision, operator,
  // check) on the capture stream and replayed on the context stream; b and x
  // are the context's own vectors, so the captured arguments stay valid
  const bool graphs = c->use_graphs == 1 && !c->prof_on;
  auto launch_iter = [&](bool check) -> int {
    if (!graphs) return enqueue_iter(check);
    hipGraphExec_t& ex = c->iter_graph[f64 ? 1 : 0][c->adjoint ? 1 : 0][check ? 1 : 0];
    if (!ex) {
      if (!c->cap_stream) HT(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      hipStream_t saved = c->stream;
      c->stream = c->cap_stream;
      HT(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
      const int rc = enqueue_iter(check);
      hipGraph_t gr = nullptr;
      const hipError_t ec = hipStreamEndCapture(c->cap_stream, &gr);
      c->stream = saved;
      if (rc != MOT_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
      }
      HT(ec);
      const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (ei != hipSuccess) {
        ex = nullptr;
        HT(ei);
      }
    }
    HT(hipGraphLaunch(ex, c->stream));
    return MOT_OK;
  };
  const double* h = nullptr;
  // host-side screen of the bound test, two iterations late: the true
  // residual is enqueued only once the last known quasi-residual bound is
  // within a factor 1000 of tol ||b|| (the device gate still decides; tau
  // can stall for a half step and then drop by orders of magnitude, so the
  // screen is wide: a check that finds nothing costs a few empty launches, a
  // missed one a whole iteration)
  //
  // The host keeps one iteration enqueued ahead, so a solve that ends in
  // iteration m leaves iteration m + 1 to run empty behind its gates.  When
  // the bound extrapolated from the last two known ones (geometric decrease)
  // says that the iteration in flight will end the solve, the host waits for
  // it before enqueueing the next: a short idle gap instead of a whole empty
  // iteration.
  double tau_last = -1.0, tau_prev = -1.0, tolb = -1.0;
  for (int it = 1; it <= fixed; ++it) TRY(enqueue_iter(!bound_only));
  for (int it = 1; fixed == 0 && it <= max_iter + 1; ++it) {
    if (it >= 3 && tau_last > 0.0 && tau_prev > 0.0 && tolb > 0.0 && tau_last < tau_prev) {
      const double pred = tau_last * (tau_last / tau_prev) * std::sqrt(2.0 * it);
      if (pred <= 1.5 * tolb) {
        HT(hipEventSynchronize(c->evq[(it - 1) & 1]));
        const double* prev = c->hscal + (1 + ((it - 1) & 1)) * S_NSLOT;
        if (prev[S_DONE] != 0.0) {
          h = prev;
          break;
        }
      }
    }
    bool check = !bound_only;
    if (check && tau_last > 0.0 && tolb > 0.0 && it < max_iter)
      check = tau_last * std::sqrt(2.0 * it + 1.0) <= 1e3 * tolb;
    double* bank = c->hscal + (1 + (it & 1)) * S_NSLOT;
    mirror = graphs ? nullptr : bank;
    TRY(launch_iter(check));
    if (graphs) HT(hipMemcpyAsync(bank, sc, sizeof(double) * S_NSLOT, hipMemcpyDeviceToHost, s));
    HT(hipEventRecord(c->evq[it & 1], s));
    if (it >= 2) {
      HT(hipEventSynchronize(c->evq[(it - 1) & 1]));
      const double* prev = c->hscal + (1 + ((it - 1) & 1)) * S_NSLOT;
      if (prev[S_DONE] != 0.0) {
        HT(hipEventSynchronize(c->evq[it & 1]));
        h = bank;
        break;
      }
      // a check the device asked for but the host did not enqueue: enqueue it now
      if (prev[S_CHECK] != 0.0 && !check) {
        TRY(apply_z0(c, x, v[V_TMP], CHK, &kfix, &ks, x));
        HTP(K_KRY, f64, vec_sub<V>(b, v[V_TMP], v[V_TMP], n, P, s, CHK));
        HTP(K_KRY, f64, reduce_post(P, sc, S_R2, POST_RESID, s, CHK));
      }
      tau_prev = tau_last;
      tau_last = prev[S_TAU];
      tolb = prev[S_TOL] * prev[S_BNORM];
    }
    if (it == max_iter + 1) {
      HT(hipEventSynchronize(c->evq[it & 1]));
      h = bank;
    }
  }
  // a solve ended by the bound leaves the second half step's x update
  // pending; the solution is x = rs y
  bool finished = false;
  if constexpr (sizeof(V) == 4) {
    if (x64) {
      HTP(K_KRY, f64, finish_f2d(x, v[V_D], bound_only ? sc + S_ETAP : nullptr, (const float*)rs, x64, c->N,
                                 x64_acc, s));
      finished = true;
    }
  }
  if (!finished) {
    if (bound_only) HTP(K_KRY, f64, vec_axpy_scal<V>(x, v[V_D], sc + S_ETAP, n, s));
    HTP(K_KRY, f64, vec_scale_voxel<V>(x, rs, n, c->N, s));
  }
  if (fixed > 0) return MOT_OK;
  if (!h || h[S_DONE] == 0.0) return set_err(c, MOT_ENOCONV, "TFQMR did not converge in max_iter%s%d");
  so->iters = (int)h[S_ITER];
  so->matvecs += (int)h[S_NMV];
  if (f64) so->matvecs64 += (int)h[S_NMV];
  so->relres = h[S_RELRES];
  switch ((int)h[S_STATUS]) {
    case MOT_OK:
      return MOT_OK;
    case MOT_ENONFINITE:
      return set_err(c, MOT_ENONFINITE, "TFQMR: right-hand side or residual is not finite%s%d");
    case MOT_EBREAKDOWN:
      return set_err(c, MOT_EBREAKDOWN, "TFQMR breakdown (rho or sigma = 0)%s%d");
    default:
      return set_err(c, MOT_ENOCONV, "TFQMR did not converge in max_iter%s%d");
  }
}

// ---------------------------------------------------------------- initial guess
// x0 = sum_i c_i J_i over the stored solutions of earlier steps, with c the
// least-squares fit of b by the stored Z0 J_i, so that r0 = b - Z0 x0 =
// b - sum_i c_i Z0 J_i needs no product (the refined solve computes Z0 J of
// every solution in FP64 for its last residual).  The Gram matrix of the
// Z0 J_i is kept on the host; one pass forms the newest pair's row, the
// dots with b and |b|^2.
static_assert(2 * PRED_MAX + 1 <= S_NSLOT, "the predictor's dots fit a scalar bank");

void pred_clear(mot_ctx* c) {
  c->pred_count = 0;
  c->pred_head = 0;
  c->pred_newrow = false;
}

// Solve the k x k system G c = d by Cholesky with a small diagonal shift;
// false when G is not positive definite even so.
bool pred_solve(int k, const double (*G)[PRED_MAX], const double* d, double* out) {
  double L[PRED_MAX][PRED_MAX] = {};
  double gmax = 0.0;
  for (int i = 0; i < k; ++i) gmax = std::max(gmax, G[i][i]);
  if (!(gmax > 0.0) || !std::isfinite(gmax)) return false;
  const double shift = 1e-12 * gmax;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j <= i; ++j) {
      double a = G[i][j] + (i == j ? shift : 0.0);
      for (int q = 0; q < j; ++q) a -= L[i][q] * L[j][q];
      if (i == j) {
        if (!(a > 0.0)) return false;
        L[i][i] = std::sqrt(a);
      } else {
        L[i][j] = a / L[j][j];
      }
    }
  double y[PRED_MAX];
  for (int i = 0; i < k; ++i) {
    double a = d[i];
    for (int q = 0; q < i; ++q) a -= L[i][q] * y[q];
    y[i] = a / L[i][i];
  }
  for (int i = k - 1; i >= 0; --i) {
    double a = y[i];
    for (int q = i + 1; q < k; ++q) a -= L[q][i] * out[q];
    out[i] = a / L[i][i];
  }
  for (int i = 0; i < k; ++i)
    if (!std::isfinite(out[i])) return false;
  return true;
}

// x0 into x, r0 into r0; bnorm = |b|, rnorm = |r0| (from the Gram data).
int pred_guess(mot_ctx* c, const double* b, double* x, double* r0, double& bnorm, double& rnorm) {
  hipStream_t s = c->stream;
  const int k = c->pred_count, K = c->pred_k;
  const int newest = (c->pred_head + K - 1) % K;
  DotSet ds{};
  ds.u[0] = b;
  ds.u[1] = c->pred_newrow ? c->pred_z[newest] : nullptr;
  ds.nu = c->pred_newrow ? 2 : 1;
  for (int i = 0; i < k; ++i) ds.w[i] = c->pred_z[i];
  ds.nw = k;
  if (!c->pred_dots) TRY(dmalloc(c, (void**)&c->pred_dots, sizeof(double) * (2 * PRED_MAX + 1)));
  HTP(K_KRY, true, multidot(ds, c->n3, c->partials, c->pred_dots, s));
  double* h = c->hscal;
  HT(hipMemcpyAsync(h, c->pred_dots, sizeof(double) * (ds.nu * k + 1), hipMemcpyDeviceToHost, s));
  HT(hipStreamSynchronize(s));
  double d[PRED_MAX], coef[PRED_MAX] = {};
  for (int i = 0; i < k; ++i) d[i] = h[i];
  if (c->pred_newrow) {
    for (int i = 0; i < k; ++i) c->pred_G[newest][i] = c->pred_G[i][newest] = h[k + i];
    c->pred_newrow = false;
  }
  const double bb = h[ds.nu * k];
  bnorm = std::sqrt(bb);
  double rr = bb;
  if (bb > 0.0 && pred_solve(k, c->pred_G, d, coef)) {
    double cd = 0.0, cgc = 0.0;
    for (int i = 0; i < k; ++i) {
      cd += coef[i] * d[i];
      for (int j = 0; j < k; ++j) cgc += coef[i] * c->pred_G[i][j] * coef[j];
    }
    rr = bb - 2.0 * cd + cgc;
    // the fit cannot do worse than x0 = 0; fall back to it if rounding says so
    if (!(rr >= 0.0 && rr <= bb)) {
      for (int i = 0; i < k; ++i) coef[i] = 0.0;
      rr = bb;
    }
  }
  Combo cb{};
  for (int i = 0; i < k; ++i) {
    cb.J[i] = c->pred_j[i];
    cb.Z[i] = c->pred_z[i];
    cb.c[i] = coef[i];
  }
  cb.k = k;
  HTP(K_KRY, true, pred_combine(cb, b, x, r0, c->n3, s));
  rnorm = std::sqrt(rr);
  return MOT_OK;
}

// Store the solution x and zx = Z0 x as the newest pair.
int pred_push(mot_ctx* c, const double* x, const double* zx) {
  const int h = c->pred_head;
  if (!c->pred_j[h]) TRY(dmalloc(c, (void**)&c->pred_j[h], sizeof(double) * c->n3));
  if (!c->pred_z[h]) TRY(dmalloc(c, (void**)&c->pred_z[h], sizeof(double) * c->n3));
  HT(hipMemcpyAsync(c->pred_j[h], x, sizeof(double) * c->n3, hipMemcpyDeviceToDevice, c->stream));
  HT(hipMemcpyAsync(c->pred_z[h], zx, sizeof(double) * c->n3, hipMemcpyDeviceToDevice, c->stream));
  c->pred_head = (h + 1) % c->pred_k;
  c->pred_count = std::min(c->pred_count + 1, c->pred_k);
  c->pred_newrow = true;
  return MOT_OK;
}

// Solve Z0 x = b (FP64 b, x) in the context precision.
//   MOT_F64:         FP64 TFQMR, FP64 FFTs.
//   MOT_F32:         FP32 TFQMR (FP64 inner products), FP32 FFTs.
//   MOT_F32_REFINED: repeated FP32 inner solves of Z0 e = r on the FP64
//                    residual r = b - Z0 x (FP64 FFT product), x += e.
// b2_partials: the reduction partials of |b|^2 are already in c->partials
// (left by the kernel that formed b).
int solve(mot_ctx* c, const double* b, double* x, double tol, int max_iter, mot_stats* st, bool b2_partials = false) {
  SolveOut so;
  int rc = MOT_OK;
  int refinements = 0;
  hipStream_t s = c->stream;
  const long long n = c->n3;
  double* P = c->partials;
  if (c->prec == MOT_F64) {
    rc = tfqmr<double>(c, b, x, tol, max_iter, &so);
  } else if (c->prec == MOT_F32) {
    rc = tfqmr<float>(c, nullptr, c->kf[V_X], tol, max_iter, &so, false, b, x);
  } else {
    double** v = c->kv;
    // without a guess, |b| stays on the device until the first FP64
    // residual comes back (the first inner tolerance does not depend on it;
    // the inner solve itself stops at once on b = 0 or a non-finite b)
    double bnorm = -1.0, rnorm = -1.0;
    const double* r = b;  // residual of the initial x
    const bool guess = c->pred_k > 0 && c->pred_count > 0;
    if (guess) {
      TRY(pred_guess(c, b, x, v[V_RO], bnorm, rnorm));
      r = v[V_RO];
      if (!std::isfinite(bnorm)) return set_err(c, MOT_ENONFINITE, "right-hand side is not finite%s%d");
    } else {
      if (!b2_partials) HTP(K_KRY, true, dot_partial<double>(b, b, n, P, s));
      HTP(K_KRY, true, reduce_post(P, c->scal, S_OB2, POST_NONE, s));
    }
    if (bnorm == 0.0) {
      so.relres = 0.0;
      HTP(K_KRY, true, vec_zero<double>(x, n, s));
    } else {
      const int max_ref = 12;
      // an FP32 TFQMR can stagnate (its recurrence residual keeps falling while
      // the true one stalls): each inner solve gets at most kInnerCap
      // iterations, after which its iterate is kept and the solve restarts
      // from the FP64 residual
      constexpr int kInnerCap = 40;
      // r = b - Z0 x: the product's inverse x pass writes the residual and
      // its partials (the predictor keeps Z0 x itself)
      auto residual64 = [&]() -> int {
        if (c->pred_k > 0) {
          TRY(apply_z0(c, x, v[V_TMP]));
          HTP(K_KRY, true, vec_sub<double>(b, v[V_TMP], v[V_RO], n, P, s));
          HTP(K_KRY, true, reduce_post(P, c->scal, S_R2, POST_NONE, s));
          return MOT_OK;
        }
        const int xb = motfft::x_pass_blocks(c->nx, true, c->tune[1][TUNE_X], 3 * c->nz * c->ny, c->nz * c->ny, 3);
        if (xb < 1 || (size_t)xb > c->partials_n) return set_err(c, MOT_EINVAL, "x pass grid outside the partials%s%d");
        motfft::Krylov kr;
        kr.mode = motfft::KRY_RESID;
        kr.v = (void*)b;
        kr.partials = P;
        kr.stride = xb;
        kr.stream = (size_t)n * sizeof(double) >= ((size_t)32 << 20) ? 1 : 0;
        TRY(apply_z0(c, x, v[V_RO], motfft::Gate{}, nullptr, &kr));
        HTP(K_KRY, true, reduce_post(P, c->scal, S_R2, POST_NONE, s, motfft::Gate{}, xb));
        return MOT_OK;
      };
      // the first sweep's FP32 tolerance (|b| is not known yet)
      const double tin1 = std::max(0.5 * tol, 3e-6);
      // graph mode 2: the first sweep as one graph replay (a fixed number of
      // gated iterations, one more than the most the recent steps needed, and
      // the FP64 residual), then the host reads the outcome as below
      const bool sweep_graph = c->use_graphs == 2 && !(c->prof_on && c->prof_mask) && !guess && c->pred_k == 0 &&
                               c->sg_need > 0 && b == c->kv[V_B] && x == c->kv[V_X] && max_iter >= c->sg_need + 1;
      bool first_done = false;
      if (sweep_graph) {
        const int G = c->sg_need + 1;
        if (c->sg_exec && (c->sg_G != G || c->sg_tol != tin1 || c->sg_adj != c->adjoint)) {
          (void)hipGraphExecDestroy(c->sg_exec);
          c->sg_exec = nullptr;
        }
        if (!c->sg_exec) {
          if (!c->cap_stream) HT(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
          hipStream_t saved = c->stream;
          c->stream = c->cap_stream;
          s = c->cap_stream;
          HT(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
          SolveOut unused;
          int crc = tfqmr<float>(c, nullptr, c->kf[V_X], tin1, G, &unused, true, r, x, false, G);
          if (crc == MOT_OK) crc = residual64();
          hipGraph_t gr = nullptr;
          const hipError_t ec = hipStreamEndCapture(c->cap_stream, &gr);
          c->stream = saved;
          s = saved;
          if (crc != MOT_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return crc;
          }
          HT(ec);
          const hipError_t ei = hipGraphInstantiate(&c->sg_exec, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          if (ei != hipSuccess) {
            c->sg_exec = nullptr;
            HT(ei);
          }
          c->sg_G = G;
          c->sg_tol = tin1;
          c->sg_adj = c->adjoint;
        }
        HT(hipGraphLaunch(c->sg_exec, s));
        TRY(reduce_sync(c));
        const double* h = c->hscal;
        ++refinements;
        so.iters += (int)h[S_ITER];
        so.matvecs += (int)h[S_NMV] + 1;
        so.matvecs64 += 1;
        if ((int)h[S_STATUS] == MOT_ENONFINITE)
          return set_err(c, MOT_ENONFINITE, "TFQMR: right-hand side or residual is not finite%s%d");
        // the iterations the sweep needed (G + 1 when it ran out of them)
        c->sg_last = h[S_DONE] != 0.0 && (int)h[S_STATUS] == MOT_OK ? (int)h[S_ITER] : G + 1;
        first_done = true;
      }
      while (true) {
        if (first_done) {
          first_done = false;
        } else {
          ++refinements;
          double tin = bnorm < 0.0 ? 0.5 * tol : rnorm > 0.0 ? 0.5 * tol * bnorm / rnorm : 1.0;
          // FP32 floor of the inner tolerance: the solve stops on its bound,
          // which sits well above the true residual, and the FP64 residual
          // below decides (a looser floor would risk second sweeps)
          if (tin < 3e-6) tin = 3e-6;
          SolveOut inner;
          const int left = max_iter - so.iters;
          const int cap = left < kInnerCap ? (left > 1 ? left : 1) : kInnerCap;
          // the inner solve (on r rounded to FP32) stops on its quasi-residual
          // bound: the FP64 residual below is its check
          // (x = e on the first sweep from x = 0, else x += e)
          int irc = tfqmr<float>(c, nullptr, c->kf[V_X], tin, cap, &inner, true, r, x, refinements > 1 || guess);
          so.iters += inner.iters;
          so.matvecs += inner.matvecs;
          if (irc != MOT_OK && irc != MOT_ENOCONV && irc != MOT_EBREAKDOWN) return irc;
          if (refinements == 1 && !guess) c->sg_last = irc == MOT_OK ? inner.iters : cap + 1;
          TRY(residual64());
          so.matvecs++;
          so.matvecs64++;
          TRY(reduce_sync(c));
        }
        if (bnorm < 0.0) {
          bnorm = sqrt(c->hscal[S_OB2]);
          if (!std::isfinite(bnorm)) return set_err(c, MOT_ENONFINITE, "right-hand side is not finite%s%d");
        }
        rnorm = sqrt(c->hscal[S_R2]);
        r = v[V_RO];
        if (!std::isfinite(rnorm)) return set_err(c, MOT_ENONFINITE, "refined residual is not finite%s%d");
        if (bnorm == 0.0) {  // b = 0: the inner solve left x = 0
          so.relres = 0.0;
          break;
        }
        so.relres = rnorm / bnorm;
        if (so.relres <= tol) break;
        if (refinements >= max_ref || so.iters >= max_iter) {
          rc = set_err(c, MOT_ENOCONV, "refinement did not reach the tolerance%s%d");
          break;
        }
      }
      // iterations the first sweep of the next graph replay gets: one more
      // than the most any of the last 8 first sweeps needed
      if (c->use_graphs == 2 && !guess && c->sg_last > 0) {
        c->sg_hist[c->sg_pos] = c->sg_last;
        c->sg_pos = (c->sg_pos + 1) % 8;
        int mx = 0;
        for (int k = 0; k < 8; ++k) mx = std::max(mx, c->sg_hist[k]);
        c->sg_need = std::min(mx, kInnerCap);
      }
      // the last residual's product is Z0 x: the pair for later guesses
      if (c->pred_k > 0) TRY(pred_push(c, x, v[V_TMP]));
    }
  }
  if (st) {
    st->iters = so.iters;
    st->matvecs = so.matvecs;
    st->matvecs_f64 = so.matvecs64;
    st->refinements = refinements;
    st->relres = so.relres;
  }
  return rc;
}

template <typename Tr>
int history_update_t(mot_ctx* c, const double* J) {
  const int ti = sizeof(Tr) == 8 ? 1 : 0;
  hipStream_t s = c->stream;
  const int rows = 3 * c->nz * c->ny;
  const int slot = (int)(c->nstep % c->nl);
  cpx<Tr>* dst = (cpx<Tr>*)c->ring + (size_t)slot * c->slot_elems;
  const bool d = ti == 1;
  const int* tv = c->tune[ti];
  // the adjoint march transforms (eps - 1) lam: Z_k^T = T(k) diag(eps) - G_k X
  HTP(K_XF, d, (motfft::x_forward<Tr, double>(J, c->wsA, c->nx, rows, c->nz * c->ny, 3, c->nx, c->nx / 2, c->kxs,
                                              c->twx[ti], c->tw2x[ti], s, c->adjoint ? c->eps : nullptr, {},
                                              tv[TUNE_X])));
  HTP(K_YF, d, motfft::y_pass<Tr>(c->wsA, c->wsB, c->py, false, c->kx, c->kxs, 3 * c->nz, c->ny, c->ny, c->py,
                                  c->py, c->twy[ti], s, {}, tv[TUNE_Y]));
  HTP(K_ZF, d, motfft::z_pass<Tr>(c->wsB, dst, c->pz, motfft::Z_FWD, 3, c->kx, c->kxs, c->py, c->nz, c->nz, c->pz,
                                  c->pz, nullptr, c->twz[ti], s, {}, tv[TUNE_Z]));
  const long long n = c->nstep;
  const size_t bytes_per_slot = (c->ring_f64 ? 16 : 8) * c->slot_elems;
  const bool tf = sizeof(Tr) == 4 && c->tf_on && c->tf_ready;
  if (tf && n % TF_S == 0) {
    // start of a time block: the far lags of its TF_S right-hand sides
    HTP(K_TFAR, d, launch_tfft_far(c->ring, c->tfK, c->tfar, c->nl, n, c->nx, c->ny, c->nz, c->kxs, s));
    c->tf_beta = n / TF_S;
  }
  if (c->blk_n0 < 0 || n - c->blk_n0 >= c->blk_B) {
    // block start: contributions of every slot <= n to the next B right-hand sides
    c->blk_n0 = n;
    const long long r0 = n - (n / TF_S) * TF_S;
    if (tf && c->tf_beta == n / TF_S && r0 + c->blk_B <= TF_S) {
      // the far parts of the time block plus its slots so far (r0 of them)
      HTP(K_MAC, d, launch_mac_block(c->ring, c->lamh, c->spec, c->pblk, (const char*)c->tfar + r0 * bytes_per_slot,
                                     0, c->blk_B, c->nl, n, (int)r0, c->nx, c->ny, c->nz, c->kxs, s, c->mac_wide));
    } else {
      const int nold = (int)(n + 1 < c->nl ? n + 1 : c->nl);
      HTP(K_MAC, d, launch_mac_block(c->ring, c->lamh, c->spec, c->pblk, nullptr, sizeof(Tr) == 8, c->blk_B, c->nl,
                                     n, nold, c->nx, c->ny, c->nz, c->kxs, s, c->mac_wide));
    }
  } else {
    // inside a block: P_{r+1} plus the r = n - n0 newest lags; with B = 8,
    // step n0 + 4 adds the four slots n0+1..n0+4 to P_5..P_8 in one pass and
    // later steps add only the lags newer than n0 + 4
    const int r = (int)(n - c->blk_n0);
    char* pb = (char*)c->pblk;
    if (c->blk_B == 8 && r == 4) {
      HTP(K_MACR, d, launch_mac_block(c->ring, c->lamh, c->spec, pb + 4 * bytes_per_slot, pb + 3 * bytes_per_slot,
                                      sizeof(Tr) == 8, 4, c->nl, n, 4, c->nx, c->ny, c->nz, c->kxs, s,
                                      c->mac_wide));
    } else {
      const int nrec = c->blk_B == 8 && r > 4 ? r - 4 : r;
      HTP(K_MACR, d, launch_mac_recent(c->ring, c->lamh, pb + (size_t)(r - 1) * bytes_per_slot, c->spec,
                                       sizeof(Tr) == 8, c->nl, n, nrec, c->nx, c->ny, c->nz, c->kxs, s));
    }
  }
  HTP(K_ZI, d, motfft::z_pass<Tr>(c->spec, c->wsB, c->pz, motfft::Z_INV, 3, c->kx, c->kxs, c->py, c->pz, c->pz,
                                  c->nz, c->nz, nullptr, c->twz[ti], s, {}, tv[TUNE_Z]));
  HTP(K_YI, d, motfft::y_pass<Tr>(c->wsB, c->wsA, c->py, true, c->kx, c->kxs, 3 * c->nz, c->py, c->py, c->ny,
                                  c->ny, c->twy[ti], s, {}, tv[TUNE_Y]));
  // the d2 eps J_{n-1} part of the regularized history right-hand side, and
  // the hand-over of J_n for the next step, ride on the epilogue
  motfft::Epilogue eh = c->adjoint ? ep_adj_hist(c) : ep_hist(c);
  if (c->dreg[2] != 0.0) {
    eh.jp = c->jprev2;
    eh.cp = c->dreg[2];
  }
  HTP(K_XI, d, (motfft::x_inverse<Tr, double>(c->wsA, c->hrhs, J, eps_of<Tr>(c), eh, c->nx,
                                              rows, c->nz * c->ny, 3,
                                              c->nx, c->nx, c->kxs, c->twx[ti], c->tw2x[ti], s, {},
                                              tv[TUNE_X])));
  c->head = slot;
  c->nstep += 1;
  return MOT_OK;
}

// T{F^-1 S} of the prepared history spectrum S (held in spec until the next
// history update): sum_{k>=1} G_k J_{n-k} for the coming step n, or
// sum_{k>=1} G_k (eps - 1) lam_{n+k} in an adjoint context.
template <typename Tr>
int history_gfield_t(mot_ctx* c, double* out) {
  const int ti = sizeof(Tr) == 8 ? 1 : 0;
  hipStream_t s = c->stream;
  const int rows = 3 * c->nz * c->ny;
  const bool d = ti == 1;
  const int* tv = c->tune[ti];
  HTP(K_ZI, d, motfft::z_pass<Tr>(c->spec, c->wsB, c->pz, motfft::Z_INV, 3, c->kx, c->kxs, c->py, c->pz, c->pz,
                                  c->nz, c->nz, nullptr, c->twz[ti], s, {}, tv[TUNE_Z]));
  HTP(K_YI, d, motfft::y_pass<Tr>(c->wsB, c->wsA, c->py, true, c->kx, c->kxs, 3 * c->nz, c->py, c->py, c->ny,
                                  c->ny, c->twy[ti], s, {}, tv[TUNE_Y]));
  // EP_G ignores its current argument; hrhs is passed as a valid vector
  HTP(K_XI, d, (motfft::x_inverse<Tr, double>(c->wsA, out, c->hrhs, eps_of<Tr>(c), EP_G, c->nx, rows, c->nz * c->ny, 3,
                                              c->nx, c->nx, c->kxs, c->twx[ti], c->tw2x[ti], s, {},
                                              tv[TUNE_X])));
  return MOT_OK;
}

int history_update_impl(mot_ctx* c, const double* J) {
  return c->ring_f64 ? history_update_t<double>(c, J) : history_update_t<float>(c, J);
}

void drop_graphs(mot_ctx* c) {
  if (c->sg_exec) {
    (void)hipGraphExecDestroy(c->sg_exec);
    c->sg_exec = nullptr;
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int k = 0; k < 2; ++k)
        if (c->iter_graph[a][b][k]) {
          (void)hipGraphExecDestroy(c->iter_graph[a][b][k]);
          c->iter_graph[a][b][k] = nullptr;
        }
}

// The solver's right scaling from the current material and G0(0).
int update_right_scale(mot_ctx* c) {
  if (!c->have_eps || !c->have_spectra) return MOT_OK;
  hipLaunchKernelGGL(k_right_scale, dim3((unsigned)((c->N + 255) / 256)), dim3(256), 0, c->stream, c->eps,
                     c->g0self, 0.5 + c->dreg[0], c->rs32, c->rs64, c->eps32, c->N);
  HT(hipGetLastError());
  return MOT_OK;
}

// Rewrite stored Z0 spectra from the fused z pass's tile width ws to wd
// (through the lam_tile scratch, so that the spectra keep their address).
template <typename T>
int retile_lam0(mot_ctx* c, T* lam, int ws, int wd) {
  if (ws == wd) return MOT_OK;
  if (ws <= 0 || wd <= 0) return set_err(c, MOT_EINVAL, "no fused z tile width for this length%s%d");
  if (!c->lam_tile) TRY(dmalloc(c, &c->lam_tile, 6 * c->lam_comp * sizeof(double)));
  const long long cnt = 6LL * (c->nx + 1) * (c->ny + 1) * (c->nz + 1);
  hipLaunchKernelGGL(k_retile<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, c->stream, lam,
                     (T*)c->lam_tile, c->nx, c->ny, c->nz, ws, wd);
  HT(hipGetLastError());
  HT(hipMemcpyAsync(lam, c->lam_tile, sizeof(T) * 6 * c->lam_comp, hipMemcpyDeviceToDevice, c->stream));
  return MOT_OK;
}

// Select tile variant v of one knob; built Z0 spectra follow the fused z
// pass's width, and captured iteration graphs are dropped.
int set_variant(mot_ctx* c, int ti, int knob, int v) {
  if (c->tune[ti][knob] == v) return MOT_OK;
  if (knob == TUNE_ZF && c->have_spectra) {
    const int ws = motfft::z_fused_width(c->pz, ti == 1, c->tune[ti][knob]);
    const int wd = motfft::z_fused_width(c->pz, ti == 1, v);
    TRY(ti == 1 ? retile_lam0(c, c->lam0_64, ws, wd) : retile_lam0(c, c->lam0_32, ws, wd));
  }
  c->tune[ti][knob] = v;
  drop_graphs(c);
  return MOT_OK;
}

// The history z passes alone (forward into the history spectrum buffer and
// back), for timing.
template <typename Tr>
int history_z_passes(mot_ctx* c) {
  const int ti = sizeof(Tr) == 8 ? 1 : 0;
  hipStream_t s = c->stream;
  HT(motfft::z_pass<Tr>(c->wsB, c->spec, c->pz, motfft::Z_FWD, 3, c->kx, c->kxs, c->py, c->nz, c->nz, c->pz, c->pz,
                        nullptr, c->twz[ti], s, {}, c->tune[ti][TUNE_Z]));
  HT(motfft::z_pass<Tr>(c->spec, c->wsB, c->pz, motfft::Z_INV, 3, c->kx, c->kxs, c->py, c->pz, c->pz, c->nz, c->nz,
                        nullptr, c->twz[ti], s, {}, c->tune[ti][TUNE_Z]));
  return MOT_OK;
}

int autotune_impl(mot_ctx* c, int reps, double* ms) {
  double* in = c->kv[V_TMP];
  double* out = c->kv[V_XO];
  TRY(zero_bytes(c, in, sizeof(double) * c->n3));
  // ms per call of fn: the least over three trials of reps calls, after one warm-up call
  auto time_runs = [&](auto&& fn, double* best) -> int {
    TRY(fn());
    *best = 1e300;
    for (int t = 0; t < 3; ++t) {
      HT(hipEventRecord(c->ev[0], c->stream));
      for (int r = 0; r < reps; ++r) TRY(fn());
      HT(hipEventRecord(c->ev[1], c->stream));
      HT(hipEventSynchronize(c->ev[1]));
      float e = 0.f;
      HT(hipEventElapsedTime(&e, c->ev[0], c->ev[1]));
      *best = std::min(*best, (double)e / reps);
    }
    return MOT_OK;
  };
  auto tune_knob = [&](int ti, int knob, auto&& fn) -> int {
    double t[2];
    for (int v = 0; v < 2; ++v) {
      TRY(set_variant(c, ti, knob, v));
      TRY(time_runs(fn, &t[v]));
      if (ms) ms[(ti * TUNE_N + knob) * 2 + v] = t[v];
    }
    // variant 1 replaces the default only when it is faster by more than the
    // run-to-run spread of these timings (about 1%)
    return set_variant(c, ti, knob, t[1] < 0.98 * t[0] ? 1 : 0);
  };
  for (int ti = 1; ti >= 0; --ti) {
    auto product = [&]() -> int {
      return ti == 1 ? green_product<double, double>(c, in, out, c->lam0_64, ep_z0(c))
                     : green_product<float, float>(c, (const float*)in, (float*)out, c->lam0_32, ep_z0(c));
    };
    for (int knob : {TUNE_X, TUNE_Y, TUNE_ZF}) TRY(tune_knob(ti, knob, product));
    if (ti == c->ring_f64) {
      auto hz = [&]() -> int { return ti == 1 ? history_z_passes<double>(c) : history_z_passes<float>(c); };
      TRY(tune_knob(ti, TUNE_Z, hz));
    }
  }
  // the history spectrum buffer held timing data: back to the state of step 0
  const size_t rsz = c->ring_f64 ? sizeof(double) : sizeof(float);
  TRY(zero_bytes(c, c->spec, rsz * 2 * c->slot_elems));
  HT(hipStreamSynchronize(c->stream));
  return MOT_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* mot_strerror(int status) {
  switch (status) {
    case MOT_OK: return "ok";
    case MOT_EINVAL: return "invalid argument";
    case MOT_ENOMEM: return "out of device memory";
    case MOT_EHIP: return "HIP runtime error";
    case MOT_ENOCONV: return "TFQMR did not converge";
    case MOT_EBREAKDOWN: return "TFQMR breakdown";
    case MOT_ENONFINITE: return "non-finite value";
    case MOT_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

const char* mot_last_error(const mot_ctx* ctx) { return ctx ? ctx->err : "no context"; }

int32_t mot_length_supported(int32_t n) { return motfft::length_supported(n) ? 1 : 0; }

int32_t mot_nlags(const mot_grid* grid) {
  if (!grid || grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0) return MOT_EINVAL;
  if (grid->alpha < 0 || (grid->alpha == 0 && !(grid->cdt > 0.0))) return MOT_EINVAL;
  return nlags_of(grid);
}

int64_t mot_zk_nnz(const mot_grid* g, int32_t k) {
  if (!g || g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || k < 0) return MOT_EINVAL;
  if (g->alpha < 0 || (g->alpha == 0 && !(g->cdt > 0.0))) return MOT_EINVAL;
  const double L = g->alpha > 0 ? g->alpha / sqrt(3.0) : g->cdt;
  const long long a2 = (long long)g->alpha * g->alpha;
  int64_t total = 0;
  for (int dz = 0; dz < g->nz; ++dz)
    for (int dy = 0; dy < g->ny; ++dy)
      for (int dx = 0; dx < g->nx; ++dx) {
        bool m;
        if (g->alpha > 0) {
          auto m1 = [](int v) { return (long long)(v > 0 ? 2 * v - 1 : 0); };
          const long long lo = 3 * (m1(dx) * m1(dx) + m1(dy) * m1(dy) + m1(dz) * m1(dz));
          m = lo < 4LL * (k + 1) * (k + 1) * a2;
          if (m && k > 2) {
            const long long hi = 3LL * ((2LL * dx + 1) * (2LL * dx + 1) + (2LL * dy + 1) * (2LL * dy + 1) +
                                        (2LL * dz + 1) * (2LL * dz + 1));
            m = hi > 4LL * (k - 2) * (k - 2) * a2;
          }
        } else {
          const double mx = dx > 0 ? dx - 0.5 : 0.0, my = dy > 0 ? dy - 0.5 : 0.0, mz = dz > 0 ? dz - 0.5 : 0.0;
          const double dmin = sqrt(mx * mx + my * my + mz * mz);
          const double dmax = sqrt((dx + .5) * (dx + .5) + (dy + .5) * (dy + .5) + (dz + .5) * (dz + .5));
          m = dmin < (k + 1) * L && dmax > (k - 2) * L;
        }
        if (!m) continue;
        const int nzc = (dx != 0) + (dy != 0) + (dz != 0);
        static const int w[4] = {3, 3, 5, 9};
        // offsets +-d: each nonzero component doubles the count
        const int64_t mult = (int64_t)(dx ? 2 : 1) * (dy ? 2 : 1) * (dz ? 2 : 1);
        total += mult * w[nzc] * (int64_t)(g->nx - dx) * (g->ny - dy) * (g->nz - dz);
      }
  return total;
}

int mot_create(const mot_grid* grid, mot_precision prec, void* hip_stream, mot_ctx** out) {
  if (!out) return MOT_EINVAL;
  *out = nullptr;
  if (!grid_ok(grid) || (prec != MOT_F64 && prec != MOT_F32 && prec != MOT_F32_REFINED)) return MOT_EINVAL;
  mot_ctx* c = new (std::nothrow) mot_ctx();
  if (!c) return MOT_ENOMEM;
  memset(c, 0, sizeof(*c));
  c->prof_mask = (1 << (MOT_PROF_NCLASS / 2)) - 1;
  c->grid = *grid;
  c->nx = grid->nx;
  c->ny = grid->ny;
  c->nz = grid->nz;
  c->px = 2 * c->nx;
  c->py = 2 * c->ny;
  c->pz = 2 * c->nz;
  c->kx = c->nx + 1;
  c->kxs = (int)round_up(c->kx, 16);
  c->alpha = grid->alpha;
  c->L = grid->alpha > 0 ? grid->alpha / sqrt(3.0) : grid->cdt;
  c->nl = nlags_of(grid);
  c->nq = grid->quad > 0 ? grid->quad : 20;
  c->N = (long long)c->nx * c->ny * c->nz;
  c->n3 = 3 * c->N;
  c->prec = prec;
  c->ring_f64 = prec == MOT_F64 ? 1 : 0;
  c->pred_k = 0;  // the initial guess is opt-in (mot_set_predictor)
  c->stream = (hipStream_t)hip_stream;
  const size_t rsz = c->ring_f64 ? sizeof(double) : sizeof(float);
  c->lam_comp = (size_t)(c->nz + 1) * (c->ny + 1) * c->kxs;
  c->slot_elems = (size_t)3 * c->pz * c->py * c->kxs;
  int rc = MOT_OK;
  auto fail = [&](int r) {
    mot_destroy(c);
    return r;
  };
  if ((rc = make_twiddles(c, c->nx, c->nx, c->twx)) != MOT_OK) return fail(rc);
  if ((rc = make_twiddles(c, 2 * c->nx, c->nx + 1, c->tw2x)) != MOT_OK) return fail(rc);
  if ((rc = make_twiddles(c, c->py, c->py, c->twy)) != MOT_OK) return fail(rc);
  if ((rc = make_twiddles(c, c->pz, c->pz, c->twz)) != MOT_OK) return fail(rc);
  const size_t wsA = (size_t)3 * c->nz * c->ny * c->kxs * 16;
  const size_t wsB = (size_t)3 * c->nz * c->py * c->kxs * 16;
  if ((rc = dmalloc(c, (void**)&c->eps, sizeof(double) * c->N)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, (void**)&c->rs32, sizeof(float) * c->N)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, (void**)&c->eps32, sizeof(float) * c->N)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, (void**)&c->rs64, sizeof(double) * c->N)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, &c->wsA, wsA)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, &c->wsB, wsB)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, (void**)&c->lam0_64, sizeof(double) * 6 * c->lam_comp)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, (void**)&c->lam0_32, sizeof(float) * 6 * c->lam_comp)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, &c->lamh, rsz * 6 * c->lam_comp * c->nl)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, &c->spec, rsz * 2 * c->slot_elems)) != MOT_OK) return fail(rc);
  c->blk_B = 8;
  while (c->blk_B > c->nl) c->blk_B /= 2;
  c->blk_n0 = -1;
  if (c->blk_B > 1 && (rc = dmalloc(c, &c->pblk, rsz * 2 * c->slot_elems * (c->blk_B - 1))) != MOT_OK)
    return fail(rc);
  if ((rc = dmalloc(c, &c->ring, rsz * 2 * c->slot_elems * c->nl)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, (void**)&c->hrhs, sizeof(double) * c->n3)) != MOT_OK) return fail(rc);
  for (int i = 0; i < 13; ++i)
    if ((rc = dmalloc(c, (void**)&c->kv[i], sizeof(double) * c->n3)) != MOT_OK) return fail(rc);
  if (prec != MOT_F64)
    for (int i = 0; i < 11; ++i)
      if ((rc = dmalloc(c, (void**)&c->kf[i], sizeof(float) * c->n3)) != MOT_OK) return fail(rc);
  // the vector kernels' partials, or two sums of one partial per x-pass
  // workgroup (at most one workgroup per row)
  c->partials_n = std::max<size_t>(2 * (size_t)std::max<long long>(RED_BLOCKS, 3LL * c->nz * c->ny),
                                   (size_t)(2 * PRED_MAX + 1) * RED_BLOCKS);
  if ((rc = dmalloc(c, (void**)&c->partials, sizeof(double) * c->partials_n)) != MOT_OK) return fail(rc);
  if ((rc = dmalloc(c, (void**)&c->scal, sizeof(double) * S_NSLOT)) != MOT_OK) return fail(rc);
  if (hipHostMalloc((void**)&c->hscal, sizeof(double) * 3 * S_NSLOT, hipHostMallocDefault) != hipSuccess) {
    c->hscal = nullptr;
    return fail(MOT_ENOMEM);
  }
  for (int i = 0; i < 3; ++i)
    if (hipEventCreate(&c->ev[i]) != hipSuccess) return fail(MOT_EHIP);
  for (int i = 0; i < 2; ++i)
    if (hipEventCreateWithFlags(&c->evq[i], hipEventDisableTiming) != hipSuccess) return fail(MOT_EHIP);
  if ((rc = tf_configure(c)) != MOT_OK) return fail(rc);
  if ((rc = mot_reset(c)) != MOT_OK) return fail(rc);
  if ((rc = zero_bytes(c, c->wsA, wsA)) != MOT_OK) return fail(rc);
  if ((rc = zero_bytes(c, c->wsB, wsB)) != MOT_OK) return fail(rc);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(MOT_EHIP);
  *out = c;
  return MOT_OK;
}

int mot_destroy(mot_ctx* c) {
  if (!c) return MOT_OK;
  (void)hipStreamSynchronize(c->stream);
  void* bufs[] = {c->eps, c->eps32, c->rs32, c->rs64, c->wsA, c->wsB, c->lam0_64, c->lam0_32, c->lamh, c->spec, c->ring, c->hrhs,
                  c->partials, c->scal, c->lam_tile, c->pblk, c->ffpart, c->jprev2, c->tfK, c->tfar};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (int i = 0; i < 13; ++i)
    if (c->kv[i]) (void)hipFree(c->kv[i]);
  for (int i = 0; i < 11; ++i)
    if (c->kf[i]) (void)hipFree(c->kf[i]);
  for (int t = 0; t < 2; ++t) {
    void* tb[] = {c->twx[t], c->tw2x[t], c->twy[t], c->twz[t]};
    for (void* b : tb)
      if (b) (void)hipFree(b);
  }
  for (int i = 0; i < 3; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  for (int i = 0; i < 2; ++i)
    if (c->evq[i]) (void)hipEventDestroy(c->evq[i]);
  for (int i = 0; i < PRED_MAX; ++i) {
    if (c->pred_j[i]) (void)hipFree(c->pred_j[i]);
    if (c->pred_z[i]) (void)hipFree(c->pred_z[i]);
  }
  if (c->pred_dots) (void)hipFree(c->pred_dots);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->hscal) (void)hipHostFree(c->hscal);
  if (c->prof_ev) {
    for (int i = 0; i < 2 * c->prof_cap; ++i) (void)hipEventDestroy(c->prof_ev[i]);
    delete[] c->prof_ev;
    delete[] c->prof_cls;
  }
  delete c;
  return MOT_OK;
}

int mot_info(const mot_ctx* c, int64_t* out, int32_t n) {
  if (!c || !out || n < 7) return MOT_EINVAL;
  out[0] = c->nl;
  out[1] = c->px;
  out[2] = c->py;
  out[3] = c->pz;
  out[4] = c->kxs;
  out[5] = (int64_t)c->bytes;
  out[6] = c->nstep;
  if (n >= 8) out[7] = c->blk_B;
  if (n >= 9) out[8] = c->tf_on ? 2 : 1;
  return MOT_OK;
}

double mot_spectra_imag(const mot_ctx* c) { return c ? c->spectra_imag : -1.0; }

int mot_set_material(mot_ctx* c, const double* eps_r) {
  if (!c || !eps_r) return MOT_EINVAL;
  pred_clear(c);
  HT(hipMemcpyAsync(c->eps, eps_r, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->stream));
  c->have_eps = true;
  return update_right_scale(c);
}

int mot_green_table(mot_ctx* c, int32_t k, double* out) {
  if (!c || !out || k < 0) return MOT_EINVAL;
  HT(launch_green(out, c->nx, c->ny, c->nz, k, c->alpha, c->L, c->nq, c->stream));
  return MOT_OK;
}

int build_green_spectra(mot_ctx* c) {
  if (!c) return MOT_EINVAL;
  pred_clear(c);
  hipStream_t s = c->stream;
  const size_t esz = (size_t)c->px * c->py * c->pz;
  const size_t ssz = (size_t)c->pz * c->py * c->kxs;  // complex elements of one component's spectrum
  const int nblk = compress_blocks(c->nx, c->ny, c->nz);
  double *goct = nullptr, *E = nullptr, *imax = nullptr;
  void *T1 = nullptr, *T2 = nullptr;
  int rc = MOT_OK;
  const size_t before = c->bytes;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    if (goct) (void)hipFree(goct);
    if (E) (void)hipFree(E);
    if (imax) (void)hipFree(imax);
    if (T1) (void)hipFree(T1);
    if (T2) (void)hipFree(T2);
    c->bytes = before;
  };
  if ((rc = dmalloc(c, (void**)&goct, sizeof(double) * 6 * c->N)) != MOT_OK ||
      (rc = dmalloc(c, (void**)&E, sizeof(double) * esz)) != MOT_OK ||
      (rc = dmalloc(c, &T1, 16 * ssz)) != MOT_OK || (rc = dmalloc(c, &T2, 16 * ssz)) != MOT_OK ||
      (rc = dmalloc(c, (void**)&imax, sizeof(double) * nblk)) != MOT_OK) {
    cleanup();
    return rc;
  }
  const double scale = 1.0 / ((double)c->px * c->py * c->pz);
  double imag = 0.0;
  std::vector<double> hmax(nblk);
  for (int k = 0; k <= c->nl && rc == MOT_OK; ++k) {
    hipError_t e = launch_green(goct, c->nx, c->ny, c->nz, k, c->alpha, c->L, c->nq, s);
    // G0(0)_xx (octant entry 0 of component xx) for the solver's scaling
    if (k == 0 && e == hipSuccess)
      if ((e = hipMemcpyAsync(&c->g0self, goct, sizeof(double), hipMemcpyDeviceToHost, s)) == hipSuccess)
        e = hipStreamSynchronize(s);
    for (int comp = 0; comp < 6 && e == hipSuccess; ++comp) {
      if ((e = launch_embed(goct, E, comp, c->nx, c->ny, c->nz, s)) != hipSuccess) break;
      if ((e = motfft::x_forward<double, double>(E, T1, c->nx, c->pz * c->py, c->pz * c->py, 1, c->px, c->nx,
                                                 c->kxs, c->twx[1], c->tw2x[1], s)) != hipSuccess)
        break;
      if ((e = motfft::y_pass<double>(T1, T2, c->py, false, c->kx, c->kxs, c->pz, c->py, c->py, c->py, c->py,
                                      c->twy[1], s)) != hipSuccess)
        break;
      if ((e = motfft::z_pass<double>(T2, T1, c->pz, motfft::Z_FWD, 1, c->kx, c->kxs, c->py, c->pz, c->pz, c->pz,
                                      c->pz, nullptr, c->twz[1], s)) != hipSuccess)
        break;
      // base of lag k (component 0); k_compress adds the component offset
      double* l64 = nullptr;
      float* l32 = nullptr;
      if (k == 0) {
        l64 = c->lam0_64;
        l32 = c->lam0_32;
      } else if (c->ring_f64) {
        l64 = (double*)c->lamh + (size_t)(k - 1) * 6 * c->lam_comp;
      } else {
        l32 = (float*)c->lamh + (size_t)(k - 1) * 6 * c->lam_comp;
      }
      const int w64 = k == 0 ? motfft::z_fused_width(c->pz, true, c->tune[1][TUNE_ZF]) : 0;
      const int w32 = k == 0 ? motfft::z_fused_width(c->pz, false, c->tune[0][TUNE_ZF]) : 0;
      if ((e = launch_compress(T1, l64, l32, imax, comp, c->nx, c->ny, c->nz, c->kxs, scale, w64, w32, s)) !=
          hipSuccess)
        break;
      if ((e = hipMemcpyAsync(hmax.data(), imax, sizeof(double) * nblk, hipMemcpyDeviceToHost, s)) != hipSuccess)
        break;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
      for (double v : hmax) imag = v > imag ? v : imag;
    }
    if (e != hipSuccess) rc = fail_hip(c, e, "spectra build", __LINE__);
  }
  cleanup();
  if (rc != MOT_OK) return rc;
  c->spectra_imag = imag;
  c->have_spectra = true;
  c->tf_ready = false;
  TRY(tf_configure(c));
  return update_right_scale(c);
}

int z0_matvec(mot_ctx* c, const void* J, void* y, mot_precision dtype) {
  if (!c || !J || !y || J == y) return MOT_EINVAL;
  if (!c->have_eps || !c->have_spectra) return set_err(c, MOT_ESTATE, "material or spectra missing%s%d");
  switch (dtype) {
    case MOT_F64:
      return green_product<double, double>(c, (const double*)J, (double*)y, c->lam0_64, ep_z0(c));
    case MOT_F32:
      return green_product<float, float>(c, (const float*)J, (float*)y, c->lam0_32, ep_z0(c));
    case MOT_F32_REFINED:
      return green_product<float, double>(c, (const double*)J, (double*)y, c->lam0_32, ep_z0(c));
    default:
      return MOT_EINVAL;
  }
}

int gk_matvec(mot_ctx* c, int32_t k, const void* J, void* y, mot_precision dtype) {
  if (!c || !J || !y || J == y || k < 0 || k > c->nl) return MOT_EINVAL;
  if (!c->have_eps || !c->have_spectra) return set_err(c, MOT_ESTATE, "material or spectra missing%s%d");
  if (k == 0) {
    if (dtype == MOT_F64) return green_product<double, double>(c, (const double*)J, (double*)y, c->lam0_64, EP_G);
    if (dtype == MOT_F32) return green_product<float, float>(c, (const float*)J, (float*)y, c->lam0_32, EP_G);
    if (dtype == MOT_F32_REFINED)
      return green_product<float, double>(c, (const double*)J, (double*)y, c->lam0_32, EP_G);
    return MOT_EINVAL;
  }
  if (c->ring_f64 ? dtype != MOT_F64 : (dtype != MOT_F32 && dtype != MOT_F32_REFINED)) return MOT_EINVAL;
  // history spectra are stored for the multiply-accumulate; copy lag k into
  // the z-pass layout first
  const size_t off = (size_t)(k - 1) * 6 * c->lam_comp;
  const size_t cnt = (size_t)6 * (c->nx + 1) * (c->ny + 1) * (c->nz + 1);
  // the tile layout pads kx to whole tiles, which never exceeds kxs columns
  if (!c->lam_tile) TRY(dmalloc(c, &c->lam_tile, 6 * c->lam_comp * sizeof(double)));
  dim3 g((unsigned)((cnt + 255) / 256));
  if (c->ring_f64) {
    hipLaunchKernelGGL(k_relayout<double>, g, dim3(256), 0, c->stream, (const double*)c->lamh + off,
                       (double*)c->lam_tile, c->nx, c->ny, c->nz, c->kxs,
                       motfft::z_fused_width(c->pz, true, c->tune[1][TUNE_ZF]));
    HT(hipGetLastError());
    return green_product<double, double>(c, (const double*)J, (double*)y, (const double*)c->lam_tile, EP_G);
  }
  hipLaunchKernelGGL(k_relayout<float>, g, dim3(256), 0, c->stream, (const float*)c->lamh + off,
                     (float*)c->lam_tile, c->nx, c->ny, c->nz, c->kxs,
                     motfft::z_fused_width(c->pz, false, c->tune[0][TUNE_ZF]));
  HT(hipGetLastError());
  if (dtype == MOT_F32)
    return green_product<float, float>(c, (const float*)J, (float*)y, (const float*)c->lam_tile, EP_G);
  return green_product<float, double>(c, (const double*)J, (double*)y, (const float*)c->lam_tile, EP_G);
}

int history_update(mot_ctx* c, const double* J_n) {
  if (!c || !J_n) return MOT_EINVAL;
  if (!c->have_eps || !c->have_spectra) return set_err(c, MOT_ESTATE, "material or spectra missing%s%d");
  return history_update_impl(c, J_n);
}

int mot_get_history_rhs(mot_ctx* c, double* out) {
  if (!c || !out) return MOT_EINVAL;
  HT(hipMemcpyAsync(out, c->hrhs, sizeof(double) * c->n3, hipMemcpyDeviceToDevice, c->stream));
  return MOT_OK;
}

int mot_excitation(mot_ctx* c, const mot_pulse* p, double t, double* out) {
  if (!c || !p || !out) return MOT_EINVAL;
  if (!c->have_eps) return set_err(c, MOT_ESTATE, "material missing%s%d");
  HTP(K_EINC, true, launch_einc(p, t, c->eps, out, c->nx, c->ny, c->nz, c->stream));
  return MOT_OK;
}

int mot_profile(mot_ctx* c, int32_t enable) {
  if (!c) return MOT_EINVAL;
  if (enable && !c->prof_ev) {
    const int cap = 8192;
    c->prof_ev = new (std::nothrow) hipEvent_t[2 * cap];
    c->prof_cls = new (std::nothrow) int[cap];
    if (!c->prof_ev || !c->prof_cls) return MOT_ENOMEM;
    for (int i = 0; i < 2 * cap; ++i) HT(hipEventCreate(&c->prof_ev[i]));
    c->prof_cap = cap;
  }
  if (!enable) TRY(prof_flush(c));
  c->prof_on = enable ? 1 : 0;
  return MOT_OK;
}

int mot_profile_kinds(mot_ctx* c, int32_t kind_mask) {
  if (!c || kind_mask < 0) return MOT_EINVAL;
  c->prof_mask = kind_mask;
  return MOT_OK;
}

int mot_profile_read(mot_ctx* c, double* ms, int64_t* counts, int32_t n) {
  if (!c || !ms || !counts || n < MOT_PROF_NCLASS) return MOT_EINVAL;
  TRY(prof_flush(c));
  for (int i = 0; i < MOT_PROF_NCLASS; ++i) {
    ms[i] = c->prof_ms[i];
    counts[i] = c->prof_cnt[i];
    c->prof_ms[i] = 0.0;
    c->prof_cnt[i] = 0;
  }
  return MOT_OK;
}

int mot_reset(mot_ctx* c) {
  if (!c) return MOT_EINVAL;
  pred_clear(c);
  const size_t rsz = c->ring_f64 ? sizeof(double) : sizeof(float);
  TRY(zero_bytes(c, c->ring, rsz * 2 * c->slot_elems * c->nl));
  TRY(zero_bytes(c, c->hrhs, sizeof(double) * c->n3));
  TRY(zero_bytes(c, c->spec, rsz * 2 * c->slot_elems));
  TRY(zero_bytes(c, c->jprev2, sizeof(double) * c->n3));
  c->nstep = 0;
  c->head = 0;
  c->blk_n0 = -1;
  c->tf_beta = -1;
  return MOT_OK;
}

int mot_set_step(mot_ctx* c, int64_t n) {
  if (!c || n < 0) return MOT_EINVAL;
  pred_clear(c);
  c->nstep = n;
  c->head = (int)((n + c->nl - 1) % c->nl);
  c->blk_n0 = -1;
  c->tf_beta = -1;
  return MOT_OK;
}

int mot_step(mot_ctx* c, const double* einc, double* J_n, double tol, int32_t max_iter, mot_stats* st) {
  if (!c || !einc || !J_n || einc == J_n || !(tol > 0.0) || max_iter < 1) return MOT_EINVAL;
  if (!c->have_eps || !c->have_spectra) return set_err(c, MOT_ESTATE, "material or spectra missing%s%d");
  hipStream_t s = c->stream;
  double* b = c->kv[V_B];
  double* x = c->kv[V_X];
  if (st) HT(hipEventRecord(c->ev[0], s));
  HTP(K_KRY, true, vec_add64(einc, c->hrhs, b, c->n3, c->partials, s));
  // the solve's counts and residual are known on the host when it returns
  c->last = mot_stats{};
  c->last.ms_lhs = c->last.ms_rhs = -1.0;
  int rc = solve(c, b, x, tol, max_iter, &c->last, true);
  if (st) *st = c->last;
  if (rc != MOT_OK && rc != MOT_ENOCONV && rc != MOT_EBREAKDOWN) return rc;
  if (c->prec == MOT_F32_REFINED || rc == MOT_OK || rc == MOT_ENOCONV || rc == MOT_EBREAKDOWN)
    HT(hipMemcpyAsync(J_n, x, sizeof(double) * c->n3, hipMemcpyDeviceToDevice, s));
  if (st) HT(hipEventRecord(c->ev[1], s));
  int hr = history_update_impl(c, J_n);
  if (hr != MOT_OK) return hr;
  if (st) {
    HT(hipEventRecord(c->ev[2], s));
    HT(hipEventSynchronize(c->ev[2]));
    float a = 0.f, bms = 0.f;
    HT(hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
    HT(hipEventElapsedTime(&bms, c->ev[1], c->ev[2]));
    st->ms_lhs = a;
    st->ms_rhs = bms;
    c->last.ms_lhs = a;
    c->last.ms_rhs = bms;
  }
  return rc;
}

int mot_last_stats(const mot_ctx* c, mot_stats* st) {
  if (!c || !st) return MOT_EINVAL;
  *st = c->last;
  return MOT_OK;
}

int mot_step_batch(mot_ctx* const* ctxs, int32_t count, const double* const* einc, double* const* J_n, double tol,
                   int32_t max_iter, mot_stats* stats, int32_t* status, int32_t nthreads) {
  if (!ctxs || !einc || !J_n || !status || count < 1 || nthreads < 1) return MOT_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return MOT_EINVAL;
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) return MOT_EINVAL;  // a context is not thread-safe
  }
  std::atomic<int> next{0};
  // members are stepped without stats (no wait for a member's history
  // update before the thread takes the next one); their statistics are the
  // host-side ones of mot_last_stats
  auto worker = [&]() {
    for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) {
      status[i] = mot_step(ctxs[i], einc[i], J_n[i], tol, max_iter, nullptr);
      if (stats) stats[i] = ctxs[i]->last;
    }
  };
  const int nt = nthreads < count ? nthreads : count;
  std::vector<std::thread> pool;
  pool.reserve(nt > 1 ? nt - 1 : 0);
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  for (int i = 0; i < count; ++i)
    if (status[i] != MOT_OK) return status[i];
  return MOT_OK;
}

int mot_set_predictor(mot_ctx* c, int32_t k) {
  if (!c || k < 0 || k > PRED_MAX || (k > 0 && c->prec != MOT_F32_REFINED)) return MOT_EINVAL;
  c->pred_k = k;
  pred_clear(c);
  return MOT_OK;
}

int mot_set_regularization(mot_ctx* c, double d0, double d1, double d2) {
  if (!c || !std::isfinite(d0) || !std::isfinite(d1) || !std::isfinite(d2) || !(0.5 + d0 > 0.0))
    return MOT_EINVAL;
  if (d0 == c->dreg[0] && d1 == c->dreg[1] && d2 == c->dreg[2]) return MOT_OK;
  if (d2 != 0.0 && !c->jprev2) {
    TRY(dmalloc(c, (void**)&c->jprev2, sizeof(double) * c->n3));
    // the current pushed before the last one is not known here: zero, as
    // after mot_reset (exact for a march started by mot_reset)
    TRY(zero_bytes(c, c->jprev2, sizeof(double) * c->n3));
  }
  c->dreg[0] = d0;
  c->dreg[1] = d1;
  c->dreg[2] = d2;
  // the diagonal of Z0 changed: the right scaling, the captured iteration
  // graphs (their epilogue arguments) and the stored Z0 J_i are stale
  drop_graphs(c);
  pred_clear(c);
  return update_right_scale(c);
}

int mot_set_history_scheme(mot_ctx* c, int32_t scheme) {
  if (!c || scheme < 0 || scheme > 2) return MOT_EINVAL;
  if (scheme == 2 && !tf_possible(c))
    return set_err(c, MOT_EINVAL, "FFTs in time need an FP32 ring of at least 32 lags%s%d");
  c->hist_scheme = scheme;
  // the far parts held now belong to the scheme before: a time block that
  // has begun finishes with the per-lag multiply-accumulate
  c->tf_beta = -1;
  return tf_configure(c);
}

int mot_set_wide_offsets(mot_ctx* c, int32_t on) {
  if (!c || on < 0 || on > 1) return MOT_EINVAL;
  c->mac_wide = on;
  return MOT_OK;
}

int mot_set_breakdown_tolerance(mot_ctx* c, double t) {
  if (!c || !std::isfinite(t) || t < 0.0) return MOT_EINVAL;
  c->bd_tol = t;
  drop_graphs(c);  // a captured first sweep holds the old tolerance
  return MOT_OK;
}

int mot_set_graphs(mot_ctx* c, int32_t on) {
  if (!c || on < 0 || on > 2) return MOT_EINVAL;
  c->use_graphs = on;
  return MOT_OK;
}

int mot_set_adjoint(mot_ctx* c, int32_t on) {
  if (!c || (on != 0 && on != 1)) return MOT_EINVAL;
  if (c->adjoint != on) pred_clear(c);
  c->adjoint = on;
  return MOT_OK;
}

int mot_set_variants(mot_ctx* c, const int32_t* v) {
  if (!c || !v) return MOT_EINVAL;
  for (int i = 0; i < 2 * TUNE_N; ++i)
    if (v[i] != 0 && v[i] != 1) return MOT_EINVAL;
  for (int ti = 0; ti < 2; ++ti)
    for (int k = 0; k < TUNE_N; ++k) TRY(set_variant(c, ti, k, v[ti * TUNE_N + k]));
  return MOT_OK;
}

int mot_get_variants(const mot_ctx* c, int32_t* v) {
  if (!c || !v) return MOT_EINVAL;
  for (int ti = 0; ti < 2; ++ti)
    for (int k = 0; k < TUNE_N; ++k) v[ti * TUNE_N + k] = c->tune[ti][k];
  return MOT_OK;
}

int mot_autotune(mot_ctx* c, int32_t reps, double* ms) {
  if (!c || reps < 0) return MOT_EINVAL;
  if (!c->have_eps || !c->have_spectra) return set_err(c, MOT_ESTATE, "material or spectra missing%s%d");
  if (c->nstep != 0) return set_err(c, MOT_ESTATE, "autotune runs at step 0 (before the march or after a reset)%s%d");
  if (ms)
    for (int i = 0; i < 4 * TUNE_N; ++i) ms[i] = -1.0;
  const int prof = c->prof_on;
  c->prof_on = 0;
  const int rc = autotune_impl(c, reps > 0 ? reps : 20, ms);
  c->prof_on = prof;
  return rc;
}

int z0t_matvec(mot_ctx* c, const void* v, void* y, mot_precision dtype) {
  if (!c || !v || !y || v == y) return MOT_EINVAL;
  if (!c->have_eps || !c->have_spectra) return set_err(c, MOT_ESTATE, "material or spectra missing%s%d");
  switch (dtype) {
    case MOT_F64:
      return green_product<double, double>(c, (const double*)v, (double*)y, c->lam0_64, ep_z0t(c), c->eps);
    case MOT_F32:
      return green_product<float, float>(c, (const float*)v, (float*)y, c->lam0_32, ep_z0t(c), c->eps);
    case MOT_F32_REFINED:
      return green_product<float, double>(c, (const double*)v, (double*)y, c->lam0_32, ep_z0t(c), c->eps);
    default:
      return MOT_EINVAL;
  }
}

int mot_history_gfield(mot_ctx* c, double* out) {
  if (!c || !out || out == c->hrhs) return MOT_EINVAL;
  if (!c->have_eps || !c->have_spectra) return set_err(c, MOT_ESTATE, "material or spectra missing%s%d");
  return c->ring_f64 ? history_gfield_t<double>(c, out) : history_gfield_t<float>(c, out);
}

namespace {
int far_geom(mot_ctx* c, const double* rhat, FarGeom* g) {
  if (!rhat) return MOT_EINVAL;
  const double n2 = rhat[0] * rhat[0] + rhat[1] * rhat[1] + rhat[2] * rhat[2];
  if (!(n2 > 0.0) || !std::isfinite(n2)) return set_err(c, MOT_EINVAL, "far-field direction is zero or not finite%s%d");
  const double inv = 1.0 / std::sqrt(n2);
  for (int i = 0; i < 3; ++i) g->r[i] = rhat[i] * inv;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) g->P[3 * i + k] = (i == k ? 1.0 : 0.0) - g->r[i] * g->r[k];
  g->dt = c->L;
  return MOT_OK;
}
}  // namespace

int mot_farfield(mot_ctx* c, const double* Jhist, int32_t nsteps, const double* rhat, int32_t j0, int32_t nj,
                 double* e, double* energy) {
  if (!c || !Jhist || !e || nsteps < 1 || nj < 1 || nj > 65535) return MOT_EINVAL;
  FarGeom g;
  TRY(far_geom(c, rhat, &g));
  const size_t need = farfield_partials(c->N, nj);
  if (need > c->ffpart_n) {
    if (c->ffpart) {
      HT(hipStreamSynchronize(c->stream));
      HT(hipFree(c->ffpart));
      c->bytes -= sizeof(double) * c->ffpart_n;
      c->ffpart = nullptr;
      c->ffpart_n = 0;
    }
    TRY(dmalloc(c, (void**)&c->ffpart, sizeof(double) * need));
    c->ffpart_n = need;
  }
  HT(launch_farfield(Jhist, nsteps, c->nx, c->ny, c->nz, g, j0, nj, c->ffpart, e, energy, c->stream));
  return MOT_OK;
}

int mot_farfield_static(mot_ctx* c, const double* Jhist, int32_t nsteps, const double* rhat, int32_t j0, int32_t nj,
                        double* e, double* energy) {
  if (!c || !Jhist || !e || nsteps < 1 || nj < 1) return MOT_EINVAL;
  if (nj > FF_NJ_MAX) return set_err(c, MOT_EINVAL, "mot_farfield_static takes at most 1024 samples%s%d");
  FarGeom g;
  TRY(far_geom(c, rhat, &g));
  double* part = nullptr;
  HT(farfield_scratch(&part));
  HT(launch_farfield(Jhist, nsteps, c->nx, c->ny, c->nz, g, j0, nj, part, e, energy, c->stream));
  return MOT_OK;
}

int mot_farfield_adjoint(mot_ctx* c, const double* w, int32_t j0, int32_t nj, const double* rhat, double scale,
                         int64_t n, double* g_n) {
  if (!c || !w || !g_n || nj < 1 || n < 0) return MOT_EINVAL;
  FarGeom g;
  TRY(far_geom(c, rhat, &g));
  HT(launch_farfield_adjoint(w, j0, nj, n, c->nx, c->ny, c->nz, g, scale, g_n, c->stream));
  return MOT_OK;
}

int mot_adjoint_gradient(mot_ctx* c, const mot_pulse* p, double t, const double* lam_n, const double* J_n,
                         const double* J_prev, const double* J_prev2, const double* uh_n, const double* u0_n,
                         double* grad) {
  if (!c || !p || !lam_n || !J_n || !uh_n || !u0_n || !grad) return MOT_EINVAL;
  const double w[3] = {0.5 + c->dreg[0], 0.5 + c->dreg[1], c->dreg[2]};
  HT(launch_adjoint_grad(p, t, lam_n, J_n, J_prev, J_prev2, uh_n, u0_n, grad, w, c->nx, c->ny, c->nz, c->stream));
  return MOT_OK;
}

}  // extern "C"
