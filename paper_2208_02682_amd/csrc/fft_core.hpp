// Batched 1-D complex FFTs held by groups of lanes (gfx950, 64-wide wavefronts).
//
// An N-point transform is owned by NT = N / E consecutive lanes; lane t of the
// group holds E complex values.  On entry lane t holds x[t + NT * e] in v[e]
// (e = 0..E-1).  The first Stockham stage is a radix-E DFT done in registers;
// later stages (radices R dividing E, each lane doing E/R butterflies) exchange
// data through the group's private LDS buffer.  On exit the spectrum is in the
// LDS buffer in natural order (padded indexing).  When a group fits in one
// wavefront (NT <= 64) the exchanges only need wavefront-scope ordering;
// otherwise they use workgroup barriers.
//
// Stockham autosort formulation (decimation in time): at a stage with radix R
// applied after sub-transforms of length Ns, butterfly j (0 <= j < N/R) reads
// in[j + r N/R], multiplies by w_{Ns R}^{r (j mod Ns)}, does an R-point DFT and
// writes out[(j / Ns) Ns R + (j mod Ns) + r Ns], with twiddle w_N^m,
// m = r (j mod Ns) N / (Ns R).  The twiddles (host-computed in long double) are
// stored stage by stage: the block of a stage holds entry (r - 1) Ns + k =
// exp(-2 pi i r k / (Ns R)) for r = 1..R-1, k < Ns, so the lanes of a wavefront
// (consecutive j) read consecutive entries of one block, a few cache lines per
// load instead of one line per lane.
#pragma once

#include <type_traits>

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

// keeps the instruction scheduler from moving work (in particular global loads)
// across phase boundaries, which would keep many loads in flight in registers
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

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

template <int DIR, typename T>
__device__ __forceinline__ void dft3(cplx<T>& a, cplx<T>& b, cplx<T>& c) {
  constexpr T h = T(0.86602540378443864676372317075293618347);  // sqrt(3)/2
  const cplx<T> t1 = b + c;
  const cplx<T> t2 = {a.x - T(0.5) * t1.x, a.y - T(0.5) * t1.y};
  const cplx<T> d = b - c;
  // t3 = DIR i (sqrt 3 / 2) (b - c)
  const cplx<T> t3 = (DIR < 0) ? cplx<T>{h * d.y, -h * d.x} : cplx<T>{-h * d.y, h * d.x};
  a = a + t1;
  b = t2 + t3;
  c = t2 - t3;
}

// 12 = 3 x 4: inner radix-3 DFTs over r1 (r = 4 r1 + r2), twiddles w12^{r2 q1},
// outer radix-4 DFTs over r2, output index q = q1 + 3 q2
template <int DIR, typename T>
__device__ __forceinline__ void dft12(cplx<T>* v) {
  constexpr T c6 = T(0.86602540378443864676372317075293618347);  // cos(pi/6)
  cplx<T> X[12];
#pragma unroll
  for (int r2 = 0; r2 < 4; ++r2) {
    cplx<T> a = v[r2], b = v[4 + r2], c = v[8 + r2];
    dft3<DIR>(a, b, c);
    X[r2 * 3 + 0] = a;
    X[r2 * 3 + 1] = b;
    X[r2 * 3 + 2] = c;
  }
  const T sg = T(DIR);
  const cplx<T> w1 = {c6, sg * T(0.5)}, w2 = {T(0.5), sg * c6}, w4 = {T(-0.5), sg * c6};
  // r2 = 1: q1 = 1, 2 -> w1, w2; r2 = 2: w2, w4; r2 = 3: w3 = DIR i, w6 = -1
  X[4] = cmul(X[4], w1);
  X[5] = cmul(X[5], w2);
  X[7] = cmul(X[7], w2);
  X[8] = cmul(X[8], w4);
  X[10] = rot90<DIR>(X[10]);
  X[11] = {-X[11].x, -X[11].y};
#pragma unroll
  for (int q1 = 0; q1 < 3; ++q1) {
    cplx<T> a = X[q1], b = X[3 + q1], c = X[6 + q1], d = X[9 + q1];
    dft4<DIR>(a, b, c, d);
    v[q1] = a;
    v[q1 + 3] = b;
    v[q1 + 6] = c;
    v[q1 + 9] = d;
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
  } else if constexpr (R == 3) {
    dft3<DIR>(v[0], v[1], v[2]);
  } else if constexpr (R == 12) {
    dft12<DIR>(v);
  } else {
    static_assert(R == 2 || R == 3 || R == 4 || R == 8 || R == 12 || R == 16, "unsupported radix");
  }
}

// ---------------------------------------------------------------------------
// plans: N = E * R2 * R3 * R4 with E values per lane; the first stage is a
// radix-E DFT in registers, the later radices divide E
// ---------------------------------------------------------------------------
struct Radices {
  int R2, R3, R4;
};
__host__ __device__ constexpr Radices plan_of(int n, int e) {
  if (e == 16) {
    switch (n) {
      case 16: return {1, 1, 1};
      case 32: return {2, 1, 1};
      case 64: return {4, 1, 1};
      case 128: return {8, 1, 1};
      case 256: return {16, 1, 1};
      case 512: return {16, 2, 1};
      case 1024: return {16, 4, 1};
      default: break;
    }
  } else if (e == 12) {
    if (n == 192) return {4, 4, 1};
    if (n == 384) return {4, 4, 2};
  }
  return {0, 0, 0};
}
template <int N, int E>
struct Plan {
  static constexpr Radices p = plan_of(N, E);
  static_assert(p.R2 > 0 && E * p.R2 * p.R3 * p.R4 == N, "no FFT plan for this length");
  static constexpr int R2 = p.R2, R3 = p.R3, R4 = p.R4;
};

// offset of stage s (0, 1, 2: the stages of radix R2, R3, R4) in the stage-by-
// stage twiddle table, and the table's length (at most n for every plan)
__host__ __device__ constexpr int tw_offset(int n, int e, int s) {
  const Radices p = plan_of(n, e);
  const int R[3] = {p.R2, p.R3, p.R4};
  int off = 0, ns = e;
  for (int i = 0; i < s; ++i) {
    if (R[i] > 1) off += (R[i] - 1) * ns;
    ns *= R[i];
  }
  return off;
}
__host__ __device__ constexpr int tw_len(int n, int e) { return tw_offset(n, e, 3); }

// values per lane of the column and row passes: 16 for powers of two (a
// 1024-point transform stays inside one wavefront, no workgroup barriers;
// measured on the 1024^2 workload it beats 8 values per lane, which halves the
// registers but needs a barrier per exchange, by about 25% in the row passes),
// 12 for N = 3 * 2^k (first stage radix 12 = 3 x 4)
__host__ __device__ constexpr int fft_E_of(int n) { return (n % 3 == 0) ? 12 : 16; }
template <int N>
__host__ __device__ constexpr int fft_E() { return fft_E_of(N); }

// exchanges of a transform owned by NT lanes: wavefront-scope ordering when the
// transform lives in one wavefront, a workgroup barrier otherwise
template <int NT>
__device__ __forceinline__ void xsync() {
  if constexpr (NT > 64) __syncthreads();
  else wave_sync();
}

// the twiddle table lives in global memory: loads through this pointer type
// are global (not generic) loads, which do not hold up the LDS counter
template <typename T>
using gptr = const __attribute__((address_space(1))) cplx<T>*;

// one Stockham stage of radix R after sub-transforms of length Ns (Ns > 1),
// reading and writing the group's LDS buffer; tw: the stage's twiddle block,
// TW its pointer type
template <typename T, int N, int E, int DIR, int Ns, int R, typename TW>
__device__ __forceinline__ void stockham_stage(cplx<T>* buf, int t, TW tw) {
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
  xsync<NT>();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = t + b * NT;
    const int k = j % Ns;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const cplx<T> w = {tw[(r - 1) * Ns + k].x, tw[(r - 1) * Ns + k].y};
      v[b * R + r] = (DIR < 0) ? cmul(v[b * R + r], w) : cmulc(v[b * R + r], w);
    }
    dft<R, DIR>(&v[b * R]);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[pidx(base + r * Ns)] = v[b * R + r];
  }
  xsync<NT>();
}

// swap of 32-bit words between lane rows (16 lanes) of two registers:
// ROWS = 16: odd rows of a with even rows of b; ROWS = 32: rows 2, 3 of a with
// rows 0, 1 of b (v_permlane16_swap / v_permlane32_swap)
template <int ROWS, typename V>
__device__ __forceinline__ void lane_swap(V& a, V& b) {
  static_assert(sizeof(V) % 4 == 0, "32-bit words");
  constexpr int W = sizeof(V) / 4;
  unsigned wa[W], wb[W];
  __builtin_memcpy(wa, &a, sizeof(V));
  __builtin_memcpy(wb, &b, sizeof(V));
#pragma unroll
  for (int i = 0; i < W; ++i) {
    if constexpr (ROWS == 16) {
      const auto r = __builtin_amdgcn_permlane16_swap(wa[i], wb[i], false, false);
      wa[i] = r[0];
      wb[i] = r[1];
    } else {
      const auto r = __builtin_amdgcn_permlane32_swap(wa[i], wb[i], false, false);
      wa[i] = r[0];
      wb[i] = r[1];
    }
  }
  __builtin_memcpy(&a, wa, sizeof(V));
  __builtin_memcpy(&b, wb, sizeof(V));
}

// The last two stages of N = 256 G (G = 2 or 4; 16 values per lane, NT = 16 G
// lanes, radix 16 then radix G) with the exchange between them done across
// lanes instead of through LDS.  After the radix-16 stage, lane t = c + 16 q
// (c < 16) holds entry 256 q + c + 16 r in x[r]; with r = G a + s that entry is
// element A q + a (A = 16 / G) of lane c + 16 s in the last stage's layout
// (entry t' + NT m in element m of lane t').  So the exchange is a G x G
// transpose over q and s among the lanes c + 16 q, done with row swaps, after
// which x[G a + k] holds element A k + a, which is exactly the last stage's
// input b G + r for b = a, r = k.  The last stage then writes the spectrum to
// buf in natural order, as a Stockham stage would.
template <typename T, int N, int E, int DIR, bool KEEP, typename TW>
__device__ __forceinline__ void stages_16_then_G(cplx<T>* buf, int t, TW tw, cplx<T> (&out)[E]) {
  constexpr int NT = N / E, G = N / 256, A = 16 / G;
  static_assert(E == 16 && (G == 2 || G == 4) && NT == 16 * G, "plan 16 x 16 x G");
  cplx<T> x[16];
  // radix-16 stage after sub-transforms of length 16
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = buf[pidx(t + r * (N / 16))];
  const int k = t % 16;
#pragma unroll
  for (int r = 1; r < 16; ++r) {
    const cplx<T> w = {tw[(r - 1) * 16 + k].x, tw[(r - 1) * 16 + k].y};
    x[r] = (DIR < 0) ? cmul(x[r], w) : cmulc(x[r], w);
  }
  dft<16, DIR>(x);
  // G x G transpose across the lanes c + 16 q
#pragma unroll
  for (int a = 0; a < A; ++a) {
    if constexpr (G == 4) {
      lane_swap<32>(x[4 * a + 0], x[4 * a + 2]);
      lane_swap<32>(x[4 * a + 1], x[4 * a + 3]);
      lane_swap<16>(x[4 * a + 0], x[4 * a + 1]);
      lane_swap<16>(x[4 * a + 2], x[4 * a + 3]);
    } else {
      lane_swap<16>(x[2 * a + 0], x[2 * a + 1]);
    }
  }
  // the buffer is rewritten below: every lane's reads above come first
  xsync<NT>();
  const TW twB = tw + 15 * 16;  // the radix-G stage's twiddle block
  // radix-G stage after sub-transforms of length 256: butterfly b of lane t
  // combines entries j + 256 r, j = t + NT b
#pragma unroll
  for (int b = 0; b < A; ++b) {
    const int j = t + NT * b;
#pragma unroll
    for (int r = 1; r < G; ++r) {
      const cplx<T> w = {twB[(r - 1) * 256 + j].x, twB[(r - 1) * 256 + j].y};
      x[b * G + r] = (DIR < 0) ? cmul(x[b * G + r], w) : cmulc(x[b * G + r], w);
    }
    dft<G, DIR>(&x[b * G]);
    // entry j + 256 r = t + NT (b + A r)
#pragma unroll
    for (int r = 0; r < G; ++r) {
      if constexpr (KEEP) out[b + A * r] = x[b * G + r];
      else buf[pidx(j + 256 * r)] = x[b * G + r];
    }
  }
  xsync<NT>();
}

// whether fft<..., GTW> takes the lane-swap path, which can leave its output in
// the lanes' registers (KEEP) instead of the buffer
template <int N, int E, bool GTW>
__host__ __device__ constexpr bool fft_keeps() {
  return GTW && E == 16 && Plan<N, E>::R2 == 16 && (Plan<N, E>::R3 == 2 || Plan<N, E>::R3 == 4) &&
         Plan<N, E>::R4 == 1;
}

// Full transform of N points held by NT = N / E lanes.  v: lane t holds
// x[t + NT e]; buf: the group's LDS buffer (padded_len(N) slots).  On exit the
// spectrum is in buf in natural order, or, with KEEP (lane-swap plans only), in
// v with lane t holding entry t + NT e.  DIR = -1: forward (exp(-i...)),
// DIR = +1: inverse (unnormalised).  GTW: read the twiddles with global loads
// (else generic ones, which also count against the LDS counter: measured
// faster in the dynamics row pass's forward transforms, slower elsewhere).
template <typename T, int N, int E, int DIR, bool GTW = true, bool KEEP = false>
__device__ __forceinline__ void fft(cplx<T> (&v)[E], cplx<T>* buf, int t, const cplx<T>* __restrict__ tw) {
  using PL = Plan<N, E>;
  constexpr int NT = N / E;
  // a fresh view of the twiddle table for every transform: stops the compiler
  // from keeping twiddles of one transform live until the next one
  asm volatile("" : "+s"(tw));
  using TW = typename std::conditional<GTW, gptr<T>, const cplx<T>*>::type;
  const TW ptw = (TW)tw;
  dft<E, DIR>(v);
#pragma unroll
  for (int r = 0; r < E; ++r) buf[pidx(t * E + r)] = v[r];
  xsync<NT>();
  if constexpr (fft_keeps<N, E, GTW>()) {
    stages_16_then_G<T, N, E, DIR, KEEP>(buf, t, ptw, v);
  } else {
    static_assert(!KEEP, "only the lane-swap plans keep their output in registers");
    if constexpr (PL::R2 > 1) stockham_stage<T, N, E, DIR, E, PL::R2>(buf, t, ptw + tw_offset(N, E, 0));
    if constexpr (PL::R3 > 1)
      stockham_stage<T, N, E, DIR, E * PL::R2, PL::R3>(buf, t, ptw + tw_offset(N, E, 1));
    if constexpr (PL::R4 > 1)
      stockham_stage<T, N, E, DIR, E * PL::R2 * PL::R3, PL::R4>(buf, t, ptw + tw_offset(N, E, 2));
  }
}

}  // namespace lm
