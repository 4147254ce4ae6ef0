// Register-resident Stockham FFT building blocks for gfx950.
//
// A batch of `np` pencils of compile-time length M is transformed by one
// workgroup laid out as (p = tid % np, jt = tid / np): np pencils times TJ
// threads per pencil.  Every thread keeps E = M/TJ complex values in VGPRs;
// each radix stage is a register butterfly followed by one exchange through a
// single LDS buffer laid out element-major, lds[element * np + pencil], so
// that lanes with consecutive pencil indices touch consecutive addresses.
// The first stage's loads and the last stage's stores go through caller
// functors (global memory for strided pencils, LDS for contiguous rows).
// Both receive the element as jt + u with u a compile-time offset, so that
// callers can address memory from one per-thread base.
//
// Zero-padded transforms: with HIN the upper half of the inputs is known to
// be zero (the doubled grid of the circulant embedding) and is neither loaded
// nor added; with HOUT only the lower half of the outputs is stored (the
// truncation back to the physical grid) and the arithmetic that only feeds
// the discarded half is dead code.
//
#pragma once

#include <hip/hip_runtime.h>

namespace motfft {

template <typename T> struct cvec;
template <> struct cvec<float> { using t = float2; };
template <> struct cvec<double> { using t = double2; };
template <typename T> using cpx = typename cvec<T>::t;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { return C{a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C mul_i(C a) {
  return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

// cos/sin of 2 pi j / 8 (j < 4): the rotations of the radix-2 split of a
// length-8 DFT (lengths 6, 10 and 12 use the prime-factor mapping, no rotations)
__host__ __device__ constexpr double rot_cos(int, int j) {
  return j == 0 ? 1.0 : j == 1 ? 0.70710678118654752440 : j == 2 ? 0.0 : -0.70710678118654752440;
}
__host__ __device__ constexpr double rot_sin(int, int j) { return j == 0 ? 0.0 : j == 2 ? 1.0 : 0.70710678118654752440; }

// d * exp(-+2 pi i j / R) for a compile-time j (after unrolling): no
// arithmetic for j = 0, a swap for the quarter turn.
template <int R, bool INV, typename T>
__device__ __forceinline__ cpx<T> rotate(cpx<T> d, int j) {
  if (j == 0) return d;
  if (4 * j == R) return mul_i<INV>(d);
  const T c = (T)rot_cos(R, j);
  const T s = INV ? (T)rot_sin(R, j) : -(T)rot_sin(R, j);
  return cpx<T>{d.x * c - d.y * s, d.x * s + d.y * c};
}

// In-register DFT of length R: v[k] <- sum_j v[j] exp(-+2 pi i jk/R).
// run_half: the same with v[R/2..R-1] = 0 (those registers are not read).
template <int R, bool INV, typename T> struct Dft {
  // radix 8 = 2 x 4: radix-2 split, rotate the odd half, two DFT_4
  static_assert(R == 8, "composite radices: 8 here, 6 and 10 by PfaDft, 12 by its own prime-factor form");
  static constexpr int Q = R / 2;
  static __device__ __forceinline__ void finish(cpx<T>* v, cpx<T>* a, cpx<T>* b) {
    Dft<Q, INV, T>::run(a);
    Dft<Q, INV, T>::run(b);
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      v[2 * m] = a[m];
      v[2 * m + 1] = b[m];
    }
  }
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a[Q], b[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      a[j] = cadd(v[j], v[j + Q]);
      b[j] = rotate<R, INV, T>(csub(v[j], v[j + Q]), j);
    }
    finish(v, a, b);
  }
  static __device__ __forceinline__ void run_half(cpx<T>* v) {
    cpx<T> a[Q], b[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      a[j] = v[j];
      b[j] = rotate<R, INV, T>(v[j], j);
    }
    finish(v, a, b);
  }
};
template <bool INV, typename T> struct Dft<2, INV, T> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  }
  static __device__ __forceinline__ void run_half(cpx<T>* v) { v[1] = v[0]; }
};
template <bool INV, typename T> struct Dft<3, INV, T> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T s = (T)0.86602540378443864676;
    cpx<T> t1 = cadd(v[1], v[2]);
    cpx<T> t2 = csub(v[1], v[2]);
    cpx<T> m = cpx<T>{v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y};
    cpx<T> n = mul_i<INV>(cscale(t2, s));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, n);
    v[2] = csub(m, n);
  }
};
template <bool INV, typename T> struct Dft<4, INV, T> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> t0 = cadd(v[0], v[2]);
    cpx<T> t1 = csub(v[0], v[2]);
    cpx<T> t2 = cadd(v[1], v[3]);
    cpx<T> t3 = mul_i<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
  static __device__ __forceinline__ void run_half(cpx<T>* v) {
    const cpx<T> a = v[0], b = v[1], bi = mul_i<INV>(v[1]);
    v[0] = cadd(a, b);
    v[2] = csub(a, b);
    v[1] = cadd(a, bi);
    v[3] = csub(a, bi);
  }
};
template <bool INV, typename T> struct Dft<5, INV, T> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    cpx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    cpx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    cpx<T> a1 = cpx<T>{v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    cpx<T> a2 = cpx<T>{v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    cpx<T> b1 = cpx<T>{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
    cpx<T> b2 = cpx<T>{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
    b1 = mul_i<INV>(b1);
    b2 = mul_i<INV>(b2);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// Length R = 2Q with Q odd (6, 10) by the prime-factor (Good-Thomas)
// mapping: input n = (Q n1 + 2 n2) mod R, output k = (Q k1 + (Q+1) k2) mod R
// make W_R^{nk} = W_2^{n1 k1} W_Q^{n2 k2}, so Q length-2 DFTs feed two
// length-Q DFTs with no rotations between them (the index maps are resolved
// at compile time).
template <int Q, bool INV, typename T> struct PfaDft {
  static constexpr int R = 2 * Q;
  static __device__ __forceinline__ void finish(cpx<T>* v, cpx<T>* a, cpx<T>* b) {
    Dft<Q, INV, T>::run(a);
    Dft<Q, INV, T>::run(b);
#pragma unroll
    for (int k2 = 0; k2 < Q; ++k2) {
      v[((Q + 1) * k2) % R] = a[k2];
      v[(Q + (Q + 1) * k2) % R] = b[k2];
    }
  }
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a[Q], b[Q];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      const cpx<T> x0 = v[(2 * n2) % R], x1 = v[(Q + 2 * n2) % R];
      a[n2] = cadd(x0, x1);
      b[n2] = csub(x0, x1);
    }
    finish(v, a, b);
  }
  // v[Q..R-1] = 0: of each input pair exactly one index is below Q
  static __device__ __forceinline__ void run_half(cpx<T>* v) {
    cpx<T> a[Q], b[Q];
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) {
      const int i0 = (2 * n2) % R, i1 = (Q + 2 * n2) % R;
      if (i0 < Q) {
        a[n2] = v[i0];
        b[n2] = v[i0];
      } else {
        a[n2] = v[i1];
        b[n2] = cpx<T>{-v[i1].x, -v[i1].y};
      }
    }
    finish(v, a, b);
  }
};
template <bool INV, typename T> struct Dft<6, INV, T> : PfaDft<3, INV, T> {};

// Length 12 = 3 x 4 by the prime-factor mapping: input n = (4 n1 + 3 n2) mod
// 12, output k = (4 k1 + 9 k2) mod 12 give W_12^{nk} = W_3^{n1 k1} W_4^{n2 k2}
// (4 = 1 mod 3, 9 = 1 mod 4), so four length-3 DFTs over n1 feed three
// length-4 DFTs over n2 with no rotations between them.
template <bool INV, typename T> struct Dft<12, INV, T> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a[4][3];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 3; ++n1) a[n2][n1] = v[(4 * n1 + 3 * n2) % 12];
      Dft<3, INV, T>::run(a[n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      cpx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4, INV, T>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[(4 * k1 + 9 * k2) % 12] = b[k2];
    }
  }
};
template <bool INV, typename T> struct Dft<10, INV, T> : PfaDft<5, INV, T> {};

template <int... Rs> struct RadixList {};

template <int A, int B> struct Gcd { static constexpr int value = Gcd<B, A % B>::value; };
template <int A> struct Gcd<A, 0> { static constexpr int value = A; };

// Threads per pencil: gcd over stages of M/R, so every thread owns the same
// number of butterflies in every stage.
template <int M, typename L> struct PlanTJ;
template <int M, int R> struct PlanTJ<M, RadixList<R>> { static constexpr int value = M / R; };
template <int M, int R, int R2, int... Rest> struct PlanTJ<M, RadixList<R, R2, Rest...>> {
  static constexpr int value = Gcd<M / R, PlanTJ<M, RadixList<R2, Rest...>>::value>::value;
};

template <int M, typename L> struct FirstRadix;
template <int M, int R, int... Rest> struct FirstRadix<M, RadixList<R, Rest...>> { static constexpr int value = R; };

// Run the stages of RadixList on registers v (inputs of the first remaining
// stage already loaded).  `store(p, jt, u, value)` receives the outputs of
// the last stage, element jt + u.
//
// SPLIT: the exchanges move the real parts and then the imaginary parts
// through an LDS buffer of M * np reals (half the bytes of a complex buffer,
// so twice the pencils fit a CU's LDS; four barriers per exchange instead of
// two).  The registers a phase reads into hold values already written out.
// LDS slot of element e of pencil p in an exchange buffer of row stride np.
// SW = 1: the pencil index is XOR-swizzled by bit 5 of the element (p ^ 2
// when it is set).  Lanes that step the element by 4 (the scattered writes of
// radix-4 stages) put elements 32 apart on the same banks; the swizzle moves
// one of each such pair to another pencil's banks.  Needs a pencil count that
// is a multiple of 4 (p ^ 2 stays a pencil of the workgroup).
template <int SW>
__device__ __forceinline__ int lslot(int e, int p, int np) {
  return e * np + (SW ? (p ^ (((e >> 5) & 1) << 1)) : p);
}

template <typename T, int M, int TJ, bool INV, int NS, bool HIN, bool HOUT, typename L, bool SPLIT = false,
          int SW = 0>
struct Stages;

template <typename T, int M, int TJ, bool INV, int NS, bool HIN, bool HOUT, int R, int... Rest, bool SPLIT, int SW>
struct Stages<T, M, TJ, INV, NS, HIN, HOUT, RadixList<R, Rest...>, SPLIT, SW> {
  template <typename Store>
  static __device__ __forceinline__ void run(cpx<T>* v, cpx<T>* lds, const cpx<T>* tw, int p, int jt,
                                             int np, Store&& store) {
    constexpr int B = M / (R * TJ);
    constexpr int TWS = M / (NS * R);
    constexpr bool half_in = HIN && NS == 1;
    static_assert(!half_in || R % 2 == 0, "a zero-padded transform needs an even first radix");
#pragma unroll
    for (int t = 0; t < B; ++t) {
      const int j = jt + t * TJ;
      if (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[k * r * TWS];
          v[t * R + r] = INV ? cmulc(v[t * R + r], w) : cmul(v[t * R + r], w);
        }
      }
      if constexpr (half_in)
        Dft<R, INV, T>::run_half(&v[t * R]);
      else
        Dft<R, INV, T>::run(&v[t * R]);
    }
    if constexpr (sizeof...(Rest) == 0) {
      // last stage: NS * R = M, butterfly j < NS, outputs j + r NS
#pragma unroll
      for (int t = 0; t < B; ++t)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int u = t * TJ + r * NS;
          // element jt + u with 0 <= jt < TJ: decided at compile time unless
          // the lane band [u, u + TJ) straddles M/2
          if (HOUT && u >= M / 2) continue;
          if (HOUT && u + TJ > M / 2 && jt + u >= M / 2) continue;
          store(p, jt, u, v[t * R + r]);
        }
    } else {
      constexpr int R2 = FirstRadix<M, RadixList<Rest...>>::value;
      constexpr int B2 = M / (R2 * TJ);
      constexpr int MR2 = M / R2;
      if constexpr (!SPLIT) {
#pragma unroll
        for (int t = 0; t < B; ++t) {
          const int j = jt + t * TJ;
          const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
          for (int r = 0; r < R; ++r) lds[lslot<SW>(base + r * NS, p, np)] = v[t * R + r];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < B2; ++t)
#pragma unroll
          for (int r = 0; r < R2; ++r) v[t * R2 + r] = lds[lslot<SW>(jt + t * TJ + r * MR2, p, np)];
        __syncthreads();
      } else {
        T* ldr = reinterpret_cast<T*>(lds);
#pragma unroll
        for (int part = 0; part < 2; ++part) {
#pragma unroll
          for (int t = 0; t < B; ++t) {
            const int j = jt + t * TJ;
            const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
            for (int r = 0; r < R; ++r)
              ldr[lslot<SW>(base + r * NS, p, np)] = part ? v[t * R + r].y : v[t * R + r].x;
          }
          __syncthreads();
#pragma unroll
          for (int t = 0; t < B2; ++t)
#pragma unroll
            for (int r = 0; r < R2; ++r) {
              const T val = ldr[lslot<SW>(jt + t * TJ + r * MR2, p, np)];
              if (part)
                v[t * R2 + r].y = val;
              else
                v[t * R2 + r].x = val;
            }
          __syncthreads();
        }
      }
      Stages<T, M, TJ, INV, NS * R, false, HOUT, RadixList<Rest...>, SPLIT, SW>::run(v, lds, tw, p, jt, np, store);
    }
  }
};

// Plan of radices per supported length.  Radices are chosen so that every
// M/R shares a large common factor: more threads per pencil, fewer values
// per thread, more waves per CU for the same LDS footprint.
template <int M> struct Plan;
#define MOT_PLAN(M_, ...) \
  template <> struct Plan<M_> { using list = RadixList<__VA_ARGS__>; };
MOT_PLAN(8, 8)
MOT_PLAN(12, 4, 3)
MOT_PLAN(16, 4, 4)
MOT_PLAN(20, 4, 5)
MOT_PLAN(24, 4, 6)
MOT_PLAN(32, 8, 4)
MOT_PLAN(40, 4, 10)
MOT_PLAN(48, 4, 4, 3)
MOT_PLAN(64, 8, 8)
MOT_PLAN(80, 4, 4, 5)
MOT_PLAN(96, 8, 12)
MOT_PLAN(120, 2, 2, 6, 5)
MOT_PLAN(128, 8, 4, 4)
MOT_PLAN(160, 4, 4, 10)
MOT_PLAN(180, 6, 6, 5)
MOT_PLAN(192, 8, 8, 3)
MOT_PLAN(240, 2, 2, 6, 10)
MOT_PLAN(320, 4, 4, 4, 5)
MOT_PLAN(480, 2, 2, 2, 6, 10)
MOT_PLAN(640, 4, 4, 4, 10)
#undef MOT_PLAN

// Supported transform lengths, for host-side dispatch.
#define MOT_FOR_EACH_LEN(X) \
  X(8) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(120) X(128) X(160) X(180) \
  X(192) X(240) X(320) X(480) X(640)

template <int M> struct PlanInfo {
  using list = typename Plan<M>::list;
  static constexpr int TJ = PlanTJ<M, list>::value;
  static constexpr int E = M / TJ;
  static constexpr int R0 = FirstRadix<M, list>::value;
};

// Load the first stage's inputs for pencil p: elem(p, jt, u) returns element
// jt + u.  The elements a thread loads are jt + TJ i, i < E, register
// t R0 + r holding i = t + r M/(R0 TJ).  With HIN only the lower half
// (r < R0/2, exactly the elements below M/2) is loaded.
template <typename T, int M, bool HIN, typename Load>
__device__ __forceinline__ void load_first(cpx<T>* v, int p, int jt, Load&& elem) {
  using PI = PlanInfo<M>;
  constexpr int R = PI::R0;
  constexpr int B = M / (R * PI::TJ);
#pragma unroll
  for (int t = 0; t < B; ++t)
#pragma unroll
    for (int r = 0; r < (HIN ? R / 2 : R); ++r) v[t * R + r] = elem(p, jt, t * PI::TJ + r * (M / R));
}

template <typename T, int M, bool INV, bool HIN, bool HOUT, bool SPLIT = false, int SW = 0, typename Store>
__device__ __forceinline__ void run_fft(cpx<T>* v, cpx<T>* lds, const cpx<T>* tw, int p, int jt, int np,
                                        Store&& store) {
  using PI = PlanInfo<M>;
  Stages<T, M, PI::TJ, INV, 1, HIN, HOUT, typename PI::list, SPLIT, SW>::run(v, lds, tw, p, jt, np, store);
}

}  // namespace motfft
