// x pass of the circulant-embedded Green product (Eq. 11, Eq. 12): kernels
// and launchers, templated on the tile variant V.
//
// Forward: a real row of length 2M (zero beyond the first n_in pairs) is
//   packed as z[n] = x[2n] + i x[2n+1], transformed with a length-M complex
//   FFT and unpacked to the M+1 non-redundant bins
//   X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) W_{2M}^k (Z[k] - conj Z[M-k]).
// Inverse: Z[k] = (X[k] + conj X[M-k]) + i W_{2M}^{-k} (X[k] - conj X[M-k]),
//   the inverse length-M FFT, and the first M/2 pairs (the physical row) go
//   straight from registers into the diagonal terms of Eq. 12.
//
// Lanes walk along a row (jt fastest), so row loads and stores are coalesced.
#pragma once

#include <type_traits>

#include "fft_impl.h"

namespace motfft {

// Streaming (nontemporal) loads and stores of an element pair.  The solver's
// vectors are read and written once per pass and next touched a whole
// product later; on grids whose vectors far exceed the caches, streaming
// accesses keep them from pushing the data that the next pass reads (this
// pass's output) out of the caches (measured: 79.45 -> 82 steps/s on the
// 320x320x48 pillars).  On small grids everything stays cached and plain
// accesses are faster, so Krylov::stream selects them per launch.
__device__ __forceinline__ float2 load_stream(const float2* p) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v t = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return float2{t.x, t.y};
}
__device__ __forceinline__ double2 load_stream(const double2* p) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  const d2v t = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return double2{t.x, t.y};
}
__device__ __forceinline__ void store_stream(float2* p, float2 v) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<f2v*>(p));
}
__device__ __forceinline__ void store_stream(double2* p, double2 v) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  const d2v t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<d2v*>(p));
}
template <typename V2>
__device__ __forceinline__ V2 load_kv(const V2* p, int stream) {
  return stream ? load_stream(p) : *p;
}
template <typename V2>
__device__ __forceinline__ void store_kv(V2* p, V2 v, int stream) {
  if (stream)
    store_stream(p, v);
  else
    *p = v;
}

// Row of local slot p in this workgroup.  With 3 components a workgroup
// takes G = NP/3 voxel rows in all three components, so the (per-voxel)
// permittivity row read by the epilogue is fetched from HBM once; returns
// nrows (invalid) for slots beyond the data.
template <int NP>
__device__ __forceinline__ int xrow(int p, int ncomp, int rows_per_comp, int nrows) {
  if (ncomp == 3 && NP >= 3) {
    constexpr int G = NP / 3 > 0 ? NP / 3 : 1;
    if (p >= 3 * G) return nrows;
    const int comp = p / G, vr = blockIdx.x * G + (p - comp * G);
    return vr < rows_per_comp ? comp * rows_per_comp + vr : nrows;
  }
  const int r = blockIdx.x * NP + p;
  return r < nrows ? r : nrows;
}

// Deterministic workgroup sums of NV values per thread: out[blockIdx.x]
// (and out[stride + blockIdx.x]), by a tree in LDS `scratch` (2 BLOCK
// doubles, free when called; every thread of the workgroup must call).
template <int BLOCK, int NV>
__device__ __forceinline__ void wg_sums(const double (&val)[NV], double* scratch, double* out, int stride) {
  constexpr int P2 = BLOCK <= 1 ? 1 : 2 * floor_pow2(BLOCK - 1);
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) scratch[k * BLOCK + t] = val[k];
  __syncthreads();
#pragma unroll
  for (int h = P2 / 2; h > 0; h >>= 1) {
    if (t < h && t + h < BLOCK)
#pragma unroll
      for (int k = 0; k < NV; ++k) scratch[k * BLOCK + t] += scratch[k * BLOCK + t + h];
    __syncthreads();
  }
  if (t == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) out[(size_t)k * stride + blockIdx.x] = scratch[k * BLOCK];
}

// pre (optional, per voxel row like the epilogue's permittivity): the input
// is multiplied by (pre - 1) as it is loaded, i.e. the contrast applied on the
// input for the transposed operators.
//
// KM: solver work fused into the loads (see Krylov); the thread that loads a
// pair of elements updates the solver vectors there.
template <typename T, typename IO, int M, bool HIN, int V, int KM>
__global__ __launch_bounds__((XCfg<T, M, V>::BLOCK)) void k_x_forward(const IO* __restrict__ in,
                                                                  cpx<T>* __restrict__ out, int nrows,
                                                                  int rows_per_comp, int ncomp, int row_len,
                                                                  int kxs, const cpx<T>* __restrict__ tw_g,
                                                                  const cpx<T>* __restrict__ tw2_g,
                                                                  const double* __restrict__ pre, Gate gate,
                                                                  Krylov kry) {
  using C = XCfg<T, M, V>;
  constexpr int NP = C::NP, NPS = C::NPS, TJ = C::TJ, E = PlanInfo<M>::E;
  if (gate_closed(gate)) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = lds + (M + 1) * NPS;
  const cpx<T>* tw = C::TWG ? tw_g : twl;
  const cpx<T>* tw2 = C::TWG ? tw2_g : twl + M;
  using V2 = typename io2<IO>::t;
  const int jt = threadIdx.x % TJ, p = threadIdx.x / TJ;
  const int grow = xrow<NP>(p, ncomp, rows_per_comp, nrows);
  const bool valid = grow < nrows;
  const size_t ro = (size_t)(valid ? grow : 0) * row_len + 2 * jt;
  const IO* src = in + ro;
  const double* prow = pre ? pre + (size_t)((valid ? grow : 0) % rows_per_comp) * row_len + 2 * jt : nullptr;
  // right scaling of the solver's operator, per voxel
  const IO* srow = KM != KRY_NONE && kry.rs
                       ? (const IO*)kry.rs + (size_t)((valid ? grow : 0) % rows_per_comp) * row_len + 2 * jt
                       : nullptr;
  IO ka = 0, kb = 0, kep = 0, kdc = 0;
  if constexpr (KM == KRY_HALF0) {
    ka = (IO)*kry.alpha;
    kep = (IO)*kry.etap;
    kdc = (IO)*kry.dcoef;
  }
  if constexpr (KM == KRY_U) kb = (IO)*kry.beta;
  if constexpr (KM == KRY_XFIX) kep = (IO)*kry.etap;
  double acc = 0.0;
  cpx<T> v[E];
  auto contrast = [&](V2 pr, int u) {
    if (prow) {
      const double2 x2 = *reinterpret_cast<const double2*>(prow + 2 * u);
      return cpx<T>{(T)((double)pr.x * (x2.x - 1.0)), (T)((double)pr.y * (x2.y - 1.0))};
    }
    return cpx<T>{(T)pr.x, (T)pr.y};
  };
  if constexpr (KM == KRY_NONE) {
    load_first<T, M, HIN>(v, p, jt,
                          [&](int, int, int u) { return contrast(*reinterpret_cast<const V2*>(src + 2 * u), u); });
  } else {
    // the elements load_first would load (lower half: element jt + u,
    // u = t TJ + r M/R0, register t R0 + r), in chunks of CH: all operand
    // loads of a chunk are issued before its stores
    static_assert(HIN, "solver work rides on the product form");
    constexpr int R0 = PlanInfo<M>::R0, MR = M / R0, HR = R0 / 2, NL = (M / (R0 * TJ)) * HR;
    constexpr int CH = NL < 4 ? NL : 4;
    const IO* kin = KM == KRY_XFIX ? (const IO*)kry.x : in;
#pragma unroll
    for (int l0 = 0; l0 < NL; l0 += CH) {
      V2 a0[CH], a1[CH], a2[CH], a3[CH], a4[CH], a5[CH], sc[CH];
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        const int l = l0 + cc;
        if (l >= NL) break;
        const int u = (l / HR) * TJ + (l % HR) * MR;
        const size_t o = ro + 2 * u;
        a0[cc] = load_kv(reinterpret_cast<const V2*>(kin + o), kry.stream);
        if (srow) sc[cc] = *reinterpret_cast<const V2*>(srow + 2 * u);
        if constexpr (KM == KRY_HALF0) {
          a1[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.v + o), kry.stream);
          a2[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.w + o), kry.stream);
          a3[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.au + o), kry.stream);
          a4[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.d + o), kry.stream);
          a5[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.x + o), kry.stream);
        } else if constexpr (KM == KRY_U) {
          a1[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.u2 + o), kry.stream);
        } else if constexpr (KM == KRY_XFIX) {
          a4[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.d + o), kry.stream);
        }
      }
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        const int l = l0 + cc;
        if (l >= NL) break;
        const int u = (l / HR) * TJ + (l % HR) * MR;
        const size_t o = ro + 2 * u;
        V2 pr;
        if constexpr (KM == KRY_HALF0) {
          // a0 = u, a1 = v, a2 = w, a3 = au, a4 = d, a5 = x
          V2 ww, dd, xx;
          xx.x = a5[cc].x + kep * a4[cc].x;
          xx.y = a5[cc].y + kep * a4[cc].y;
          pr.x = a0[cc].x - ka * a1[cc].x;
          pr.y = a0[cc].y - ka * a1[cc].y;
          ww.x = a2[cc].x - ka * a3[cc].x;
          ww.y = a2[cc].y - ka * a3[cc].y;
          dd.x = a0[cc].x + kdc * a4[cc].x;
          dd.y = a0[cc].y + kdc * a4[cc].y;
          if (valid) {
            store_kv(reinterpret_cast<V2*>((IO*)kry.x + o), xx, kry.stream);
            store_kv(reinterpret_cast<V2*>((IO*)kry.out + o), pr, kry.stream);
            store_kv(reinterpret_cast<V2*>((IO*)kry.w + o), ww, kry.stream);
            store_kv(reinterpret_cast<V2*>((IO*)kry.d + o), dd, kry.stream);
            acc += (double)ww.x * (double)ww.x + (double)ww.y * (double)ww.y;
          }
        } else if constexpr (KM == KRY_U) {  // a0 = w, a1 = u2
          pr.x = a0[cc].x + kb * a1[cc].x;
          pr.y = a0[cc].y + kb * a1[cc].y;
          if (valid) store_kv(reinterpret_cast<V2*>((IO*)kry.out + o), pr, kry.stream);
        } else if constexpr (KM == KRY_XFIX) {  // a0 = x, a4 = d
          pr.x = a0[cc].x + kep * a4[cc].x;
          pr.y = a0[cc].y + kep * a4[cc].y;
          if (valid) store_kv(reinterpret_cast<V2*>((IO*)kry.x + o), pr, kry.stream);
        } else {  // KRY_SCALE
          pr = a0[cc];
        }
        if (srow) {
          pr.x *= sc[cc].x;
          pr.y *= sc[cc].y;
        }
        v[(l / HR) * R0 + (l % HR)] = contrast(pr, u);
      }
    }
  }
  if constexpr (!C::TWG) {
    load_table<cpx<T>, M, C::BLOCK>(twl, tw_g);
    load_table<cpx<T>, M + 1, C::BLOCK>(twl + M, tw2_g);
  }
  run_fft<T, M, false, HIN, false, false, C::SW>(
      v, lds, tw, p, jt, NPS, [&](int pp, int, int u, cpx<T> val) { lds[lslot<C::SW>(jt + u, pp, NPS)] = val; });
  __syncthreads();
  if (valid) {
    // bins k = jt + TJ i of row p (and k = M by lane jt = 0)
    cpx<T>* dst = out + (size_t)grow * kxs + jt;
    auto unpack = [&](cpx<T> zk, cpx<T> zm, cpx<T> w) {
      // E = (zk + conj zm)/2, O = -i/2 (zk - conj zm), X = E + w O
      const cpx<T> ev{(T)0.5 * (zk.x + zm.x), (T)0.5 * (zk.y - zm.y)};
      const cpx<T> od{(T)0.5 * (zk.y + zm.y), (T)-0.5 * (zk.x - zm.x)};
      return cadd(ev, cmul(w, od));
    };
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int k = jt + TJ * i;
      const int m = i == 0 ? (jt == 0 ? 0 : M - jt) : M - k;
      dst[TJ * i] = unpack(lds[lslot<C::SW>(k, p, NPS)], lds[lslot<C::SW>(m, p, NPS)], tw2[k]);
    }
    if (jt == 0) dst[M] = unpack(lds[lslot<C::SW>(0, p, NPS)], lds[lslot<C::SW>(0, p, NPS)], tw2[M]);
  }
  if constexpr (KM == KRY_HALF0) {
    __syncthreads();  // the unpack's LDS reads are done: LDS holds the sums
    const double val[1] = {acc};
    wg_sums<C::BLOCK, 1>(val, reinterpret_cast<double*>(smem_raw), kry.partials, kry.stride);
  }
}

// KM: solver work fused into the stores (see Krylov); the thread that
// writes a pair of y elements updates the solver vectors there.
template <typename T, typename IO, int M, int V, int KM>
__global__ __launch_bounds__((XCfg<T, M, V>::BLOCK)) void k_x_inverse(
    const cpx<T>* __restrict__ in, IO* __restrict__ y, const IO* __restrict__ J,
    const T* __restrict__ eps, Epilogue ep, int nrows, int rows_per_comp, int ncomp, int row_len,
    int kxs, const cpx<T>* __restrict__ tw_g, const cpx<T>* __restrict__ tw2_g, Gate gate, Krylov kry) {
  using C = XCfg<T, M, V>;
  constexpr int NP = C::NP, NPS = C::NPS, TJ = C::TJ, E = PlanInfo<M>::E;
  // swizzled slots only without the solver's vector work: with it the
  // swizzled form was slower (x inverse passes 1.81 -> 1.98 ms per step)
  constexpr int SWI = KM == KRY_NONE ? C::SW : 0;
  if (gate_closed(gate)) return;
  static_assert((M / 2) % TJ == 0, "the kept half of a row is whole columns of the lane layout");
  constexpr int EH = E / 2;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = lds + (M + 1) * NPS;
  const cpx<T>* tw = C::TWG ? tw_g : twl;
  const cpx<T>* tw2 = C::TWG ? tw2_g : twl + M;
  using V2 = typename io2<IO>::t;
  const int jt = threadIdx.x % TJ, p = threadIdx.x / TJ;
  const int grow = xrow<NP>(p, ncomp, rows_per_comp, nrows);
  const bool valid = grow < nrows;
  const int growc = valid ? grow : 0;
  // bins k = jt + TJ i and k = M of row p, all loads issued before any wait
  const cpx<T>* srow = in + (size_t)growc * kxs;
  cpx<T> x[E];
  // the spectrum is read once: past 32 MB with streaming (nontemporal) loads
  const bool big = (size_t)nrows * kxs * sizeof(cpx<T>) >= ((size_t)32 << 20);
  typedef T tv2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int i = 0; i < E; ++i) {
    if (big) {
      const tv2 t = __builtin_nontemporal_load(reinterpret_cast<const tv2*>(srow + jt + TJ * i));
      x[i] = cpx<T>{t.x, t.y};
    } else {
      x[i] = srow[jt + TJ * i];
    }
  }
  const cpx<T> xM = srow[M];
  // epilogue operands of the pairs n = jt + TJ i (i < E/2) this lane writes
  const size_t roff = (size_t)growc * row_len + 2 * jt;
  const size_t eoff = (size_t)(growc % rows_per_comp) * row_len + 2 * jt;
  V2 jv[EH];
  typename io2<T>::t ev[EH];
  // right scaling of the solver's operator: the diagonal term's current is rs J
  constexpr bool SCALED = KM != KRY_NONE && KM != KRY_RESID;
  const IO* rsrow = SCALED && kry.rs ? (const IO*)kry.rs + eoff : nullptr;
  V2 sv[SCALED ? EH : 1];
  V2 bv[KM == KRY_RESID ? EH : 1];  // right-hand side pairs (residual form)
  // the previous step's current (Epilogue::jp), FP64 outputs without solver
  // work; read where it is used (prefetched, it took 40 more registers)
  constexpr bool PREV = KM == KRY_NONE && std::is_same<IO, double>::value;
  const bool prev = PREV && ep.jp != nullptr;
#pragma unroll
  for (int i = 0; i < EH; ++i) {
    jv[i] = *reinterpret_cast<const V2*>(J + roff + 2 * TJ * i);
    ev[i] = *reinterpret_cast<const typename io2<T>::t*>(eps + eoff + 2 * TJ * i);
    if constexpr (SCALED) {
      if (rsrow) sv[i] = *reinterpret_cast<const V2*>(rsrow + 2 * TJ * i);
    }
    if constexpr (KM == KRY_RESID) bv[i] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.v + roff + 2 * TJ * i), kry.stream);
  }
  if constexpr (!C::TWG) {
    load_table<cpx<T>, M, C::BLOCK>(twl, tw_g);
    load_table<cpx<T>, M + 1, C::BLOCK>(twl + M, tw2_g);
  }
#pragma unroll
  for (int i = 0; i < E; ++i) lds[lslot<SWI>(jt + TJ * i, p, NPS)] = x[i];
  if (jt == 0) lds[lslot<SWI>(M, p, NPS)] = xM;
  __syncthreads();
  cpx<T> v[E];
  load_first<T, M, false>(v, p, jt, [&](int, int, int u) {
    const int k = jt + u;
    const cpx<T> xk = lds[lslot<SWI>(k, p, NPS)], xm = lds[lslot<SWI>(M - k, p, NPS)];
    // Z[k] = (Xk + conj Xm) + i W^{-k} (Xk - conj Xm)
    const cpx<T> dk{xk.x - xm.x, xk.y + xm.y};
    const cpx<T> rk = cmulc(dk, tw2[k]);
    return cpx<T>{xk.x + xm.x - rk.y, xk.y - xm.y + rk.x};
  });
  __syncthreads();
  IO* yrow = y + roff;
  IO ka = 0, kb = 0, ke = 0, kdc = 0;
  if constexpr (KM == KRY_HALF1) {
    ka = (IO)*kry.alpha;
    ke = (IO)*kry.eta;
    kdc = (IO)*kry.dcoef;
  }
  if constexpr (KM == KRY_V) kb = (IO)*kry.beta;
  double acc1 = 0.0, acc2 = 0.0;
  V2 yo[KM == KRY_HALF1 || KM == KRY_V ? EH : 1];  // the y pairs this lane wrote (solver forms)
  run_fft<T, M, true, false, true, false, SWI>(v, lds, tw, p, jt, NPS, [&](int, int, int u, cpx<T> z) {
    if (!valid) return;
    const int i = u / TJ;
    const auto e2 = ev[i];
    V2 j2 = jv[i];
    if constexpr (SCALED) {
      if (rsrow) {
        j2.x *= sv[i].x;
        j2.y *= sv[i].y;
      }
    }
    V2 r;
    r.x = (IO)(((T)(ep.ca * e2.x + ep.c0)) * (T)j2.x + ((T)(ep.cb * e2.x + ep.cb0)) * z.x);
    r.y = (IO)(((T)(ep.ca * e2.y + ep.c0)) * (T)j2.y + ((T)(ep.cb * e2.y + ep.cb0)) * z.y);
    if constexpr (KM == KRY_RESID) {
      r.x = bv[i].x - r.x;
      r.y = bv[i].y - r.y;
      acc1 += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
    }
    if constexpr (PREV) {
      if (prev) {
        double2* q = reinterpret_cast<double2*>(ep.jp + roff + 2 * u);
        const double2 pj = *q;
        r.x -= ep.cp * (double)e2.x * pj.x;
        r.y -= ep.cp * (double)e2.y * pj.y;
        *q = double2{(double)jv[i].x, (double)jv[i].y};
      }
    }
    *reinterpret_cast<V2*>(yrow + 2 * u) = r;
    if constexpr (KM == KRY_HALF1 || KM == KRY_V) yo[i] = r;
  });
  if constexpr (KM == KRY_HALF1 || KM == KRY_V) {
    // pairs n = jt + TJ i of the row, in chunks of CH: all operand loads of a
    // chunk are issued before its stores
    constexpr int CH = EH < 4 ? EH : 4;
    if (valid) {
#pragma unroll
      for (int i0 = 0; i0 < EH; i0 += CH) {
        V2 a0[CH], a1[CH], a2[CH], a3[CH];
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          const int i = i0 + cc;
          if (i >= EH) break;
          const size_t o = roff + 2 * TJ * i;
          if constexpr (KM == KRY_HALF1) {
            a0[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.x + o), kry.stream);
            a1[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.w + o), kry.stream);
            a2[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.d + o), kry.stream);
            a3[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.rt + o), kry.stream);
          } else {
            a0[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.au + o), kry.stream);
            a1[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.v + o), kry.stream);
            a3[cc] = load_kv(reinterpret_cast<const V2*>((const IO*)kry.rt + o), kry.stream);
          }
        }
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          const int i = i0 + cc;
          if (i >= EH) break;
          const size_t o = roff + 2 * TJ * i;
          const V2 r = yo[i];
          if constexpr (KM == KRY_HALF1) {  // r = au2, jv = u2; a0 = x, a1 = w, a2 = d, a3 = rt
            V2 xx, ww, dd;
            xx.x = a0[cc].x + ke * a2[cc].x;
            xx.y = a0[cc].y + ke * a2[cc].y;
            ww.x = a1[cc].x - ka * r.x;
            ww.y = a1[cc].y - ka * r.y;
            dd.x = jv[i].x + kdc * a2[cc].x;
            dd.y = jv[i].y + kdc * a2[cc].y;
            store_kv(reinterpret_cast<V2*>((IO*)kry.x + o), xx, kry.stream);
            store_kv(reinterpret_cast<V2*>((IO*)kry.w + o), ww, kry.stream);
            store_kv(reinterpret_cast<V2*>((IO*)kry.d + o), dd, kry.stream);
            acc1 += (double)ww.x * (double)ww.x + (double)ww.y * (double)ww.y;
            acc2 += (double)ww.x * (double)a3[cc].x + (double)ww.y * (double)a3[cc].y;
          } else {  // KRY_V: r = au; a0 = au2, a1 = v, a3 = rt
            V2 vv;
            vv.x = r.x + kb * (a0[cc].x + kb * a1[cc].x);
            vv.y = r.y + kb * (a0[cc].y + kb * a1[cc].y);
            store_kv(reinterpret_cast<V2*>((IO*)kry.v + o), vv, kry.stream);
            acc1 += (double)vv.x * (double)a3[cc].x + (double)vv.y * (double)a3[cc].y;
          }
        }
      }
    }
  }
  // the last stage's exchange ended with a barrier: LDS is free for the sums
  if constexpr (KM == KRY_HALF1) {
    const double val[2] = {acc1, acc2};
    wg_sums<C::BLOCK, 2>(val, reinterpret_cast<double*>(smem_raw), kry.partials, kry.stride);
  } else if constexpr (KM == KRY_V || KM == KRY_RESID) {
    const double val[1] = {acc1};
    wg_sums<C::BLOCK, 1>(val, reinterpret_cast<double*>(smem_raw), kry.partials, kry.stride);
  }
}

template <int NP>
static int x_blocks(int nrows, int rows_per_comp, int ncomp) {
  return (ncomp == 3 && NP >= 3) ? (rows_per_comp + NP / 3 - 1) / (NP / 3) : (nrows + NP - 1) / NP;
}

// Supported forms: n_in = M/2 (product: rows of M reals) or n_in = M (FP64
// only, spectra precompute: rows of 2M reals; tile variant 0 only).  KM != 0
// (solver work, IO = T): the product form only.
template <typename T, typename IO, int V, int KM>
hipError_t x_forward_v(const IO* in, void* out, int M, int nrows, int rows_per_comp, int ncomp, int row_len,
                       int n_in, int kxs, const void* tw, const void* tw2, hipStream_t s, const double* pre,
                       Gate gg, const Krylov& kry) {
  const bool half = 2 * n_in == M;
  if ((!half && n_in != M) || (!half && (sizeof(T) != 8 || V != 0 || KM != KRY_NONE)) || 2 * n_in > row_len ||
      kxs < M + 1 || (pre && !half))
    return hipErrorInvalidValue;
  switch (M) {
#define X(m)                                                                                              \
  case m: {                                                                                               \
    using C = XCfg<T, m, V>;                                                                              \
    const dim3 g(x_blocks<C::NP>(nrows, rows_per_comp, ncomp));                                           \
    if (half)                                                                                             \
      hipLaunchKernelGGL((k_x_forward<T, IO, m, true, V, KM>), g, dim3(C::BLOCK), C::LDS, s, in,           \
                         (cpx<T>*)out, nrows, rows_per_comp, ncomp, row_len, kxs, (const cpx<T>*)tw,        \
                         (const cpx<T>*)tw2, pre, gg, kry);                                               \
    else if constexpr (sizeof(T) == 8 && sizeof(IO) == 8 && V == 0 && KM == KRY_NONE)                    \
      hipLaunchKernelGGL((k_x_forward<T, IO, m, false, V, KM>), g, dim3(C::BLOCK), C::LDS, s, in,          \
                         (cpx<T>*)out, nrows, rows_per_comp, ncomp, row_len, kxs, (const cpx<T>*)tw,        \
                         (const cpx<T>*)tw2, nullptr, gg, kry);                                           \
    return hipGetLastError();                                                                             \
  }
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// Supported form: n_out = M reals (the physical half of the length-2M row).
template <typename T, typename IO, int V, int KM>
hipError_t x_inverse_v(const void* in, IO* y, const IO* J, const T* eps, Epilogue ep, int M, int nrows,
                       int rows_per_comp, int ncomp, int row_len, int n_out, int kxs, const void* tw,
                       const void* tw2, hipStream_t s, Gate gg, const Krylov& kry) {
  if (n_out != M || row_len < M || kxs < M + 1) return hipErrorInvalidValue;
  switch (M) {
#define X(m)                                                                                            \
  case m: {                                                                                             \
    using C = XCfg<T, m, V>;                                                                            \
    const dim3 g(x_blocks<C::NP>(nrows, rows_per_comp, ncomp));                                         \
    hipLaunchKernelGGL((k_x_inverse<T, IO, m, V, KM>), g, dim3(C::BLOCK), C::LDS, s, (const cpx<T>*)in, y, J, \
                       eps, ep, nrows, rows_per_comp, ncomp, row_len, kxs, (const cpx<T>*)tw,             \
                       (const cpx<T>*)tw2, gg, kry);                                                    \
    return hipGetLastError();                                                                           \
  }
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <int V>
int x_pass_blocks_v(int M, bool f64, int nrows, int rows_per_comp, int ncomp) {
  switch (M) {
#define X(m)                                                                                            \
  case m:                                                                                               \
    return f64 ? x_blocks<XCfg<double, m, V>::NP>(nrows, rows_per_comp, ncomp)                          \
               : x_blocks<XCfg<float, m, V>::NP>(nrows, rows_per_comp, ncomp);
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return 0;
  }
}

// Explicit instantiations of one tile variant (each variant, and the solver
// forms, have their own translation units so that they compile in parallel).
#define MOT_X_FWD(T, IO, V, KM)                                                                                \
  template hipError_t x_forward_v<T, IO, V, KM>(const IO*, void*, int, int, int, int, int, int, int,            \
                                                const void*, const void*, hipStream_t, const double*, Gate,     \
                                                const Krylov&);
#define MOT_X_INV(T, IO, V, KM)                                                                                \
  template hipError_t x_inverse_v<T, IO, V, KM>(const void*, IO*, const IO*, const T*, Epilogue, int, int, \
                                                int, int, int, int, int, const void*, const void*,              \
                                                hipStream_t, Gate, const Krylov&);
#define MOT_X_VARIANT(V)                                                                                       \
  MOT_X_FWD(float, float, V, KRY_NONE)                                                                         \
  MOT_X_FWD(float, double, V, KRY_NONE)                                                                        \
  MOT_X_FWD(double, double, V, KRY_NONE)                                                                       \
  MOT_X_INV(float, float, V, KRY_NONE)                                                                         \
  MOT_X_INV(float, double, V, KRY_NONE)                                                                        \
  MOT_X_INV(double, double, V, KRY_NONE)
#define MOT_X_RESID(V) MOT_X_INV(double, double, V, KRY_RESID)
#define MOT_X_SOLVER_T(T, V)                                                                                   \
  MOT_X_FWD(T, T, V, KRY_HALF0)                                                                                \
  MOT_X_FWD(T, T, V, KRY_U)                                                                                    \
  MOT_X_FWD(T, T, V, KRY_XFIX)                                                                                 \
  MOT_X_FWD(T, T, V, KRY_SCALE)                                                                                \
  MOT_X_INV(T, T, V, KRY_HALF1)                                                                                \
  MOT_X_INV(T, T, V, KRY_V)                                                                                    \
  MOT_X_INV(T, T, V, KRY_SCALE)

}  // namespace motfft
