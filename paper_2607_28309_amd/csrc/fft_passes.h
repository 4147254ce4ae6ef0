// Launch interface of the FFT passes of the Toeplitz/circulant product
// (Eq. 11): x real-to-complex, y complex, z complex with the spectral
// multiply fused in, and their inverses.  Layout of every spectral buffer:
// [component][plane][row][kxs] complex, kx fastest, kxs = padded Nx+1.
#pragma once

#include <hip/hip_runtime.h>

namespace motfft {

enum ZMode { Z_FWD = 0, Z_INV = 1, Z_FUSED = 2 };

// Epilogue of the inverse x pass:
//   y = (ca*eps + c0) * J + (cb*eps + cb0) * g,    g = the transformed field
// (Eq. 12: ca = 1/2, c0 = 0, cb = -1, cb0 = 1 gives D J - X (G J)).
// Optionally (FP64 output without solver work): y -= cp eps jp with the
// current jp of the previous step, and jp = J afterwards (in place: each
// element is read before its thread writes it).
struct Epilogue {
  double ca, c0, cb, cb0;
  double* jp = nullptr;
  double cp = 0.0;
};

// Optional early exit of a whole launch on device flags, for work enqueued
// ahead of a convergence test: f[0] != 0 means "done", f[1] != 0 "check
// requested".  mode 0: always run; 1: run while not done; 2: run while not
// done and a check is requested.  Every thread of the launch reads the same
// flags, so a closed gate ends every workgroup before its first barrier.
struct Gate {
  const double* f = nullptr;
  int mode = 0;
};
__device__ __forceinline__ bool gate_closed(const Gate& g) {
  if (!g.f || g.mode == 0) return false;
  if (g.f[0] != 0.0) return true;
  return g.mode == 2 && g.f[1] == 0.0;
}

// Solver work fused into the x passes of a Z0 product (TFQMR, Freund): the
// vector updates that go with the product's input or output, done by the
// thread that loads or stores each element, and their inner products as one
// FP64 partial per workgroup (fixed grid and order: deterministic).  Vectors
// are of the product's element type IO (= T); scalars are read from the
// solver's FP64 slots.
//   KRY_HALF0 (x forward; in = u):  x += etap d; u2 = u - alpha v;
//       w -= alpha au; d = u + dcoef d (d before the update in both);
//       the product's input is u2; partial |w|^2.
//   KRY_U (x forward; in = w):  u = w + beta u2, the product's input.
//   KRY_XFIX (x forward; in = x):  x += etap d, the product's input.
//   KRY_HALF1 (x inverse; J = u2, y = au2):  x += eta d; w -= alpha au2;
//       d = u2 + dcoef d; partials |w|^2 and w . rt.
//   KRY_V (x inverse; y = au):  v = au + beta (au2 + beta v); partial v . rt.
//   KRY_SCALE (either pass): no vector work, only the scale below.
//   KRY_RESID (x inverse; y = b - Z0 J with b in `v`): the residual of the
//       product's input, written in place of the product; partial |y|^2.
// rs (optional with every mode but KRY_NONE; per voxel, indexed like the
// epilogue's permittivity): right diagonal scaling of the solver's operator,
// Z0 diag(rs): the product's input (forward pass) and the diagonal term's
// current (inverse pass) are multiplied by rs.
enum KryMode { KRY_NONE = 0, KRY_HALF0, KRY_U, KRY_XFIX, KRY_HALF1, KRY_V, KRY_SCALE, KRY_RESID };
struct Krylov {
  int mode = KRY_NONE;
  const double* alpha = nullptr;  // solver scalars (device)
  const double* beta = nullptr;
  const double* eta = nullptr;
  const double* etap = nullptr;   // pending x update coefficient
  const double* dcoef = nullptr;
  void* x = nullptr;
  void* d = nullptr;
  void* w = nullptr;
  void* v = nullptr;
  void* au = nullptr;   // KRY_HALF0: au; KRY_V: au2
  void* rt = nullptr;
  void* out = nullptr;  // KRY_HALF0: u2; KRY_U: u
  void* u2 = nullptr;   // KRY_U: u2
  double* partials = nullptr;  // partials[b] (and partials[stride + b] for a second sum)
  int stride = 0;
  const void* rs = nullptr;    // right scaling (see above), IO values
  int stream = 0;              // 1: the vectors are read and written with streaming accesses
};

// Precision tags: T = compute type; IO = element type of real vectors.
// Returns hipSuccess or an error; hipErrorInvalidValue for an unsupported length.
// var: tile-shape variant, 0 (default) or 1 (see XCfg, YCfg, ZCfg, ZFCfg); the
// full-length forward forms of the spectra precompute always use variant 0.

// x pass, forward: `nrows` rows of `row_len` reals (row stride row_len) ->
// rows of Nx+1 complex (stride kxs).  M = complex FFT length (= Nx), the
// first n_in complex pairs of each row are read, the rest are zero.  With
// ncomp = 3 the rows are three components of rows_per_comp rows each and a
// workgroup takes the same voxel rows of all three.  pre (optional, n_in =
// M/2 only): per-voxel values indexed like the inverse pass's eps; the input
// is multiplied by (pre - 1) on load.
// kry: solver work fused into the pass (n_in = M/2 only, IO = T).
template <typename T, typename IO>
hipError_t x_forward(const IO* in, void* out, int M, int nrows, int rows_per_comp, int ncomp, int row_len,
                     int n_in, int kxs, const void* tw, const void* tw2, hipStream_t s,
                     const double* pre = nullptr, Gate g = Gate{}, int var = 0, const Krylov* kry = nullptr);

// x pass, inverse with epilogue: rows of M+1 complex -> first n_out reals of
// a length-2M real signal; y/J rows of row_len reals, eps indexed by
// (row mod rows_per_comp) * row_len + x.
template <typename T, typename IO>
hipError_t x_inverse(const void* in, IO* y, const IO* J, const T* eps, Epilogue ep, int M,
                     int nrows, int rows_per_comp, int ncomp, int row_len, int n_out, int kxs,
                     const void* tw, const void* tw2, hipStream_t s, Gate g = Gate{}, int var = 0,
                     const Krylov* kry = nullptr);

// Workgroups of an x pass (forward and inverse alike): the number of partials
// a fused solver sum leaves; 0 for an unsupported length or variant.
int x_pass_blocks(int M, bool f64, int var, int nrows, int rows_per_comp, int ncomp);

// y pass: `planes` planes; input rows_in rows (first n_in read), output
// rows_out rows (first n_out written).
template <typename T>
hipError_t y_pass(const void* in, void* out, int M, bool inverse, int kx, int kxs, int planes,
                  int rows_in, int n_in, int rows_out, int n_out, const void* tw, hipStream_t s,
                  Gate g = Gate{}, int var = 0);

// z pass over `nc` (1 or 3) components; ny = number of ky rows.
// FUSED (nc = 3) multiplies by Lambda between the forward and inverse
// transforms; Lambda is octant-compressed in the tile layout of
// lam_tile_offset with W = z_fused_width(M, T is double, var).
template <typename T>
hipError_t z_pass(const void* in, void* out, int M, int mode, int nc, int kx, int kxs, int ny,
                  int rows_in, int n_in, int rows_out, int n_out, const T* lam, const void* tw,
                  hipStream_t s, Gate g = Gate{}, int var = 0);

bool length_supported(int M);

// kx columns per workgroup of the fused z pass in tile variant var (0 for an
// unsupported length or variant).
int z_fused_width(int M, bool f64, int var = 0);

// Offset of the octant spectrum value of component comp (order xx, yy, zz,
// xy, xz, yz) at (kx, kyc, kzc) in the fused z pass's tile layout
// [kyc][kx / W][kzc][kx % W][comp]: one workgroup's values are one contiguous
// range, a thread reads the six components of a point as one contiguous
// piece, and lanes of consecutive kx read consecutive pieces.
__host__ __device__ inline size_t lam_tile_offset(int kx, int kyc, int kzc, int comp, int kxn, int nzc, int W) {
  const int ntile = (kxn + W - 1) / W;
  return ((((size_t)kyc * ntile + kx / W) * nzc + kzc) * W + kx % W) * 6 + comp;
}

}  // namespace motfft
