// Batched 1-D complex FFTs held by groups of lanes of one wavefront (gfx950).
//
// An N-point transform is owned by NT = N / E consecutive lanes of a single
// 64-wide wavefront; lane t of the group holds E complex values.  On entry lane t
// holds x[t + NT * e] in v[e] (e = 0..E-1).  The first Stockham stage is a
// radix-E DFT done in registers; later stages (radices R dividing E, each lane
// doing E/R butterflies) exchange data through the group's private LDS buffer.
// On exit the spectrum is in the LDS buffer in natural order (padded indexing).
// Because a group never spans two wavefronts, the exchanges only need
// wavefront-scope ordering, never a workgroup barrier.
//
// Stockham autosort formulation (decimation in time): at a stage with radix R
// applied after sub-transforms of length Ns, butterfly j (0 <= j < N/R) reads
// in[j + r N/R], multiplies by w_{Ns R}^{r (j mod Ns)}, does an R-point DFT and
// writes out[(j / Ns) Ns R + (j mod Ns) + r Ns].  Twiddles come from one table
// tw[m] = exp(-2 pi i m / N) (host-computed in long double), index
// m = r (j mod Ns) N / (Ns R) < N.
#pragma once

#include <hip/hip_runtime.h>

namespace lm {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> mk(T a, T b) { return cplx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> scale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (DIR = -1, forward) or +i (DIR = +1, inverse)
template <int DIR, typename T>
__device__ __forceinline__ cplx<T> rot90(cplx<T> a) {
  if constexpr (DIR < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

// wavefront-scope ordering of LDS traffic between lanes of one wave
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// padded LDS index: one spare complex slot every 16 spreads strided accesses
// over the banks
__device__ __forceinline__ constexpr int pidx(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 4) + 1; }

// ---------------------------------------------------------------------------
// small DFTs, y_q = sum_r v_r exp(DIR * 2 pi i r q / R)
// ---------------------------------------------------------------------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cplx<T>& a, cplx<T>& b) {
  cplx<T> t = a - b;
  a = a + b;
  b = t;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cplx<T>& v0, cplx<T>& v1, cplx<T>& v2, cplx<T>& v3) {
  cplx<T> t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = rot90<DIR>(v1 - v3);
  v0 = t0 + t2;
  v2 = t0 - t2;
  v1 = t1 + t3;
  v3 = t1 - t3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cplx<T>* v) {
  constexpr T s = T(0.70710678118654752440084436210484903928);
  // even / odd halves
  cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // o_q *= w8^q, w8 = exp(DIR i pi / 4)
  cplx<T> w1 = {s, T(DIR) * s};
  cplx<T> w3 = {-s, T(DIR) * s};
  o1 = cmul(o1, w1);
  o2 = rot90<DIR>(o2) ;
  // rot90 gives multiplication by DIR*i which is w8^2 = exp(DIR i pi/2)
  o3 = cmul(o3, w3);
  v[0] = e0 + o0; v[4] = e0 - o0;
  v[1] = e1 + o1; v[5] = e1 - o1;
  v[2] = e2 + o2; v[6] = e2 - o2;
  v[3] = e3 + o3; v[7] = e3 - o3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cplx<T>* v) {
  constexpr T c1 = T(0.92387953251128675612818318939678828682);  // cos(pi/8)
  constexpr T s1 = T(0.38268343236508977172845998403039886676);  // sin(pi/8)
  constexpr T h = T(0.70710678118654752440084436210484903928);
  // inner radix-4 DFTs over r1 for each r2: X_{r2}[q1] = sum_r1 v[4 r1 + r2] w4^{r1 q1}
  cplx<T> X[16];
#pragma unroll
  for (int r2 = 0; r2 < 4; ++r2) {
    cplx<T> a = v[r2], b = v[4 + r2], c = v[8 + r2], d = v[12 + r2];
    dft4<DIR>(a, b, c, d);
    X[r2 * 4 + 0] = a;
    X[r2 * 4 + 1] = b;
    X[r2 * 4 + 2] = c;
    X[r2 * 4 + 3] = d;
  }
  // twiddle w16^{r2 q1}, w16 = exp(DIR 2 pi i / 16)
  const T sg = T(DIR);
  const cplx<T> w1 = {c1, sg * s1}, w2 = {h, sg * h}, w3 = {s1, sg * c1};
  const cplx<T> w6 = {-h, sg * h}, w9 = {-c1, -sg * s1};
  // r2 = 1: q1 = 1,2,3 -> w1, w2, w3
  X[5] = cmul(X[5], w1);
  X[6] = cmul(X[6], w2);
  X[7] = cmul(X[7], w3);
  // r2 = 2: w2, w4 (= DIR i), w6
  X[9] = cmul(X[9], w2);
  X[10] = rot90<DIR>(X[10]);
  X[11] = cmul(X[11], w6);
  // r2 = 3: w3, w6, w9
  X[13] = cmul(X[13], w3);
  X[14] = cmul(X[14], w6);
  X[15] = cmul(X[15], w9);
  // outer radix-4 over r2: y[q1 + 4 q2] = sum_r2 X_{r2}[q1] w4^{r2 q2}
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1) {
    cplx<T> a = X[q1], b = X[4 + q1], c = X[8 + q1], d = X[12 + q1];
    dft4<DIR>(a, b, c, d);
    v[q1] = a;
    v[q1 + 4] = b;
    v[q1 + 8] = c;
    v[q1 + 12] = d;
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cplx<T>* v) {
  if constexpr (R == 2) {
    dft2<DIR>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    dft8<DIR>(v);
  } else if constexpr (R == 16) {
    dft16<DIR>(v);
  } else {
    static_assert(R == 2 || R == 4 || R == 8 || R == 16, "unsupported radix");
  }
}

// ---------------------------------------------------------------------------
// plans: E values per lane and the radices after the first (radix-E) stage
// ---------------------------------------------------------------------------
template <int N>
struct Plan;
template <> struct Plan<16>   { static constexpr int E = 16; static constexpr int R2 = 1,  R3 = 1; };
template <> struct Plan<32>   { static constexpr int E = 16; static constexpr int R2 = 2,  R3 = 1; };
template <> struct Plan<64>   { static constexpr int E = 16; static constexpr int R2 = 4,  R3 = 1; };
template <> struct Plan<128>  { static constexpr int E = 16; static constexpr int R2 = 8,  R3 = 1; };
template <> struct Plan<256>  { static constexpr int E = 16; static constexpr int R2 = 16, R3 = 1; };
template <> struct Plan<512>  { static constexpr int E = 16; static constexpr int R2 = 16, R3 = 2; };
template <> struct Plan<1024> { static constexpr int E = 16; static constexpr int R2 = 16, R3 = 4; };

template <int N>
struct FFTShape {
  static constexpr int E = Plan<N>::E;
  static constexpr int NT = N / E;          // lanes per transform
  static constexpr int PER_WAVE = 64 / NT;  // transforms per wavefront
  static constexpr int LDS = padded_len(N); // complex slots per transform buffer
  static_assert(NT <= 64, "a transform must fit in one wavefront");
};

// one Stockham stage of radix R after sub-transforms of length Ns (Ns > 1),
// reading and writing the group's LDS buffer
template <typename T, int N, int DIR, int Ns, int R>
__device__ __forceinline__ void stockham_stage(cplx<T>* buf, int t, const cplx<T>* __restrict__ tw) {
  constexpr int E = Plan<N>::E;
  constexpr int NT = N / E;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide E");
  cplx<T> v[E];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + b * NT;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b * R + r] = buf[pidx(j + r * (N / R))];
  }
  wave_sync();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + b * NT;
    const int k = j % Ns;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const cplx<T> w = tw[r * k * (N / (Ns * R))];
      v[b * R + r] = (DIR < 0) ? cmul(v[b * R + r], w) : cmulc(v[b * R + r], w);
    }
    dft<R, DIR>(&v[b * R]);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[pidx(base + r * Ns)] = v[b * R + r];
  }
  wave_sync();
}

// Full transform.  v: lane data x[t + NT e]; buf: the group's LDS buffer.
// DIR = -1: forward (exp(-i...)), DIR = +1: inverse (unnormalised).
template <typename T, int N, int DIR>
__device__ __forceinline__ void fft(cplx<T> (&v)[Plan<N>::E], cplx<T>* buf, int t,
                                    const cplx<T>* __restrict__ tw) {
  constexpr int E = Plan<N>::E;
  dft<E, DIR>(v);
#pragma unroll
  for (int r = 0; r < E; ++r) buf[pidx(t * E + r)] = v[r];
  wave_sync();
  if constexpr (Plan<N>::R2 > 1) stockham_stage<T, N, DIR, E, Plan<N>::R2>(buf, t, tw);
  if constexpr (Plan<N>::R3 > 1) stockham_stage<T, N, DIR, E * Plan<N>::R2, Plan<N>::R3>(buf, t, tw);
}

}  // namespace lm
