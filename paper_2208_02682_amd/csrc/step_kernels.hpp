// Hot-path kernels of one RK4 stage (templated on the transform precision T and N).
//
// One stage of the coupled system is three launches:
//
//  rows_dyn   per grid row: inverse row transforms of the column-pass outputs to
//             physical u, v, eta = h - H, zeta (zeta = dv/dx - du/dy); stores
//             them interleaved for the gathers; forms zeta v, zeta u,
//             K = (u^2+v^2)/2, eta u, eta v and forward-transforms them along the row.
//
// The physical passes carry the depth anomaly eta = h - H instead of the total
// depth h, and the h accumulators of the three averages integrate eta; H is put
// back exactly where it enters (H u and H v in the flux divergence, H s in the
// accumulators, + H in the float64 outputs).  This is the same arithmetic as the
// total-depth form up to rounding (each average is linear in the averaged field
// and exact for constants) but keeps the full float32 precision for eta.
//  rows_rhs   per grid row and strategy: the Lagrangian-mean right-hand sides
//             in physical space, then forward row transforms:
//               S2: u(x+xi) - w - (w.grad) xi  for both components (eq. (4.5a)),
//                   w = xi/(t-tau), or u/2 at t = tau, and
//                   f(x+xi) - w.grad g-bar, f in {h, zeta}             (eq. (4.5b));
//               S1: f - u.grad g-tilde                                 (eq. (4.1)) and
//                   (t-tau) u - u.grad P  (inverse lift map, eq. (3.9) in P form).
//             u(x+xi) and f(x+xi) are periodic bilinear interpolants.
//  columns    per spectral column kx and prognostic field: forward column
//             transforms, masked spectral assembly of the right-hand side
//             (Coriolis, Bernoulli gradient, flux divergence, -nu8 |k|^8), the
//             classical RK4 update (FP64 for xi and P), and the inverse column
//             transforms of the next stage's input, ready for the next rows pass.
//
// Two real row fields share one complex transform (z = a + i b).
#pragma once

#include <type_traits>

#include "fft_core.hpp"
#include "col_tile.hpp"
#include "layout.hpp"
#include "step_args.hpp"

namespace lm {

constexpr int ROW_WAVES = 4;  // wavefronts per row-kernel block

// row kernels: one lane group of NT = N / E lanes per grid row
template <int N>
struct RowGeo {
  static constexpr int E = fft_E<N>(), NT = N / E;
  static constexpr int RPB = 64 * ROW_WAVES / NT;  // rows per block
  static constexpr int L = padded_len(N);           // LDS slots per row
  static_assert(RPB >= 1 && N % RPB == 0, "row geometry");
};

// group index (uniform per wavefront when a group spans whole wavefronts)
template <int NT>
__device__ __forceinline__ int row_group() {
  if constexpr (NT >= 64) return __builtin_amdgcn_readfirstlane(threadIdx.x / NT);
  else return threadIdx.x / NT;
}

template <int N, int W = 0>
__host__ __device__ constexpr int col_tile() { return col_tile_of(N, W); }
template <int N, int W = 0>
__host__ __device__ constexpr int col_threads() { return col_tile<N, W>() * (N / fft_E<N>()); }

// --------------------------------------------------------------------------
// row helpers
// --------------------------------------------------------------------------

// Build lane registers of the length-N spectrum Z = A' + i B' of two real rows
// from their half spectra A, B (kx = 0..K).  A' = i kx A if DXA (likewise B).
// Index k = t + NT r; negative kx are the conjugate mirror.
template <typename T, int N, bool DXA, bool DXB>
__device__ __forceinline__ void load_pair(cplx<T> (&z)[fft_E<N>()], const cplx<T>* __restrict__ A,
                                          const cplx<T>* __restrict__ B, int t) {
  constexpr int E = fft_E<N>(), NT = N / E, K = kcut<N>();
  sched_fence();
  // branch-free: every lane loads (a clamped index where the mask is empty) and
  // selects, so the unrolled loop has no lane-divergent control flow
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = t + NT * r;
    const bool lo = k <= K, hi = k >= N - K;
    const int kk = min(lo ? k : N - k, K);
    cplx<T> a = A[kk], b = B[kk];
    if (DXA) a = {-T(kk) * a.y, T(kk) * a.x};
    if (DXB) b = {-T(kk) * b.y, T(kk) * b.x};
    const T sy = (kk == 0) ? T(0) : (hi ? T(-1) : T(1));  // real at kx = 0, conjugate mirror
    a.y *= sy;
    b.y *= sy;
    z[r] = (lo || hi) ? cplx<T>{a.x - b.y, a.y + b.x} : cplx<T>{T(0), T(0)};
  }
}

// Inverse-transform a pair and leave lane values p[e] at x = t + NT e.
template <typename T, int N, bool GTW = true>
__device__ __forceinline__ void inverse_row(cplx<T> (&z)[fft_E<N>()], cplx<T>* buf, int t,
                                            const cplx<T>* __restrict__ tw) {
  constexpr int E = fft_E<N>(), NT = N / E;
  if constexpr (fft_keeps<N, E, GTW>()) {
    fft<T, N, E, +1, GTW, true>(z, buf, t, tw);
  } else {
    fft<T, N, E, +1, GTW>(z, buf, t, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = buf[pidx(t + NT * e)];
    xsync<NT>();
  }
  sched_fence();
}

// Forward-transform z = a + i b (lane values at x = t + NT e) and store the
// half spectra of a and b (kx = 0..K) to the row pointers OA and OB.
template <typename T, int N, bool TWO, bool GTW = true>
__device__ __forceinline__ void forward_row(cplx<T> (&z)[fft_E<N>()], cplx<T>* buf, int t,
                                            const cplx<T>* __restrict__ tw,
                                            cplx<T>* __restrict__ OA, cplx<T>* __restrict__ OB) {
  constexpr int E = fft_E<N>(), NT = N / E, K = kcut<N>();
  fft<T, N, E, -1, GTW>(z, buf, t, tw);
#pragma unroll
  for (int r = 0; r < (K + NT) / NT; ++r) {
    const int k = t + NT * r;
    if (k > K) break;
    const cplx<T> zk = buf[pidx(k)];
    const cplx<T> zm = buf[pidx(k == 0 ? 0 : N - k)];
    OA[k] = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    if (TWO) OB[k] = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
  }
  xsync<NT>();
  sched_fence();
}

// i in [-N, 2N) to [0, N): a mask for powers of two, two selects otherwise
template <int N>
__device__ __forceinline__ int wrap2N(int i) {
  if constexpr ((N & (N - 1)) == 0) {
    return i & (N - 1);
  } else {
    i = (i < 0) ? i + N : i;
    return (i >= N) ? i - N : i;
  }
}

// The cell offset floor(o) of a gather (o = displacement / dx) taken
// periodically into [0, N): a finite displacement of any size wraps around the
// torus.  Offsets beyond 2^30 cells and NaN land on cell 0 (their weights are
// non-finite, which the end-of-interval check reports).
template <int N, typename T>
__device__ __forceinline__ int cell_mod(T f) {
  const int i = (fabs(f) < T(1073741824.0)) ? int(f) : 0;
  if constexpr ((N & (N - 1)) == 0) {
    return i & (N - 1);
  } else {
    const int r = i % N;
    return r < 0 ? r + N : r;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Renumber the flattened block index so that every XCD receives a contiguous
// run of logical blocks, and split the logical index with the task (or field
// group) fastest: each XCD then gets an even mix of heavy and light tasks, and
// all tasks of neighbouring rows / column tiles meet in the same L2 (the
// gathers, re-read rows and shared 128-byte lines hit in L2).
constexpr int NUM_XCD = 8;
// remap = 0 keeps the hardware order (logical index = flattened block index).
__device__ __forceinline__ void xcd_split(int nslow, int nfast, int& slow, int& fast, int& z, int remap) {
  const int total = nslow * nfast * gridDim.z;
  const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const int q = total / NUM_XCD, r = total % NUM_XCD;
  const int xcd = b % NUM_XCD;
  const int logical = remap ? xcd * q + min(xcd, r) + b / NUM_XCD : b;
  fast = logical % nfast;
  const int rest = logical / nfast;
  slow = rest % nslow;
  z = rest / nslow;
}

// periodic bilinear interpolation at x + xi of one pair of the interleaved
// physical fields: (u, v) if PAIR == 0, (eta, zeta) if PAIR == 1 (8 bytes per
// corner instead of the whole 16-byte point)
template <typename T, int N, int PAIR>
__device__ __forceinline__ cplx<T> gather2(const P4<T>* __restrict__ F, int x, int y, T xix, T xiy) {
  const T scl = T(double(N) / 6.283185307179586476925286766559);
  T ox = xix * scl, oy = xiy * scl;
  const T fx = floor(ox), fy = floor(oy);
  const T ax = ox - fx, ay = oy - fy;
  // x + (fx mod N) and y + (fy mod N) lie in [0, 2N)
  const int ix0 = wrap2N<N>(x + cell_mod<N>(fx)), iy0 = wrap2N<N>(y + cell_mod<N>(fy));
  const int ix1 = (ix0 + 1 == N) ? 0 : ix0 + 1, iy1 = (iy0 + 1 == N) ? 0 : iy0 + 1;
  // uniform base plus 32-bit byte offsets (the field is far below 4 GiB)
  const char* F2 = reinterpret_cast<const char*>(F) + PAIR * sizeof(cplx<T>);
  constexpr unsigned PT = sizeof(P4<T>), ROW = N * sizeof(P4<T>);
  const unsigned r0 = unsigned(iy0) * ROW, r1 = unsigned(iy1) * ROW;
  const unsigned c0 = unsigned(ix0) * PT, c1 = unsigned(ix1) * PT;
  const cplx<T> f00 = *reinterpret_cast<const cplx<T>*>(F2 + (r0 + c0));
  const cplx<T> f01 = *reinterpret_cast<const cplx<T>*>(F2 + (r0 + c1));
  const cplx<T> f10 = *reinterpret_cast<const cplx<T>*>(F2 + (r1 + c0));
  const cplx<T> f11 = *reinterpret_cast<const cplx<T>*>(F2 + (r1 + c1));
  const T w00 = (T(1) - ax) * (T(1) - ay), w01 = ax * (T(1) - ay);
  const T w10 = (T(1) - ax) * ay, w11 = ax * ay;
  return {w00 * f00.x + w01 * f01.x + w10 * f10.x + w11 * f11.x,
          w00 * f00.y + w01 * f01.y + w10 * f10.y + w11 * f11.y};
}

// periodic tensor-product cubic (4-point Lagrange) interpolation at x + xi of
// one pair of the interleaved physical fields, PAIR as in gather2: with
// o = xi / dx, i0 = floor(o), a = o - i0, the nodes i0-1 .. i0+2 carry
// -a(a-1)(a-2)/6, (a+1)(a-1)(a-2)/2, -(a+1)a(a-2)/2, (a+1)a(a-1)/6
template <typename T, int N, int PAIR>
__device__ __forceinline__ cplx<T> gather2_cubic(const P4<T>* __restrict__ F, int x, int y, T xix, T xiy) {
  const T scl = T(double(N) / 6.283185307179586476925286766559);
  T ox = xix * scl, oy = xiy * scl;
  const T fx = floor(ox), fy = floor(oy);
  const T ax = ox - fx, ay = oy - fy;
  const T wx[4] = {-ax * (ax - T(1)) * (ax - T(2)) / T(6), (ax + T(1)) * (ax - T(1)) * (ax - T(2)) / T(2),
                   -(ax + T(1)) * ax * (ax - T(2)) / T(2), (ax + T(1)) * ax * (ax - T(1)) / T(6)};
  const T wy[4] = {-ay * (ay - T(1)) * (ay - T(2)) / T(6), (ay + T(1)) * (ay - T(1)) * (ay - T(2)) / T(2),
                   -(ay + T(1)) * ay * (ay - T(2)) / T(2), (ay + T(1)) * ay * (ay - T(1)) / T(6)};
  const int bx = wrap2N<N>(x + cell_mod<N>(fx)), by = wrap2N<N>(y + cell_mod<N>(fy));
  const char* F2 = reinterpret_cast<const char*>(F) + PAIR * sizeof(cplx<T>);
  constexpr unsigned PT = sizeof(P4<T>), ROW = N * sizeof(P4<T>);
  unsigned col[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int c = bx + i - 1;
    c = c < 0 ? c + N : (c >= N ? c - N : c);
    col[i] = unsigned(c) * PT;
  }
  cplx<T> out = {T(0), T(0)};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int r = by + j - 1;
    r = r < 0 ? r + N : (r >= N ? r - N : r);
    const unsigned ro = unsigned(r) * ROW;
    cplx<T> row = {T(0), T(0)};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const cplx<T> f = *reinterpret_cast<const cplx<T>*>(F2 + (ro + col[i]));
      row.x += wx[i] * f.x;
      row.y += wx[i] * f.y;
    }
    out.x += wy[j] * row.x;
    out.y += wy[j] * row.y;
  }
  return out;
}

// periodic bilinear interpolation of the interleaved physical fields at x + xi
template <typename T, int N>
__device__ __forceinline__ P4<T> gather4(const P4<T>* __restrict__ F, int x, int y, T xix, T xiy) {
  const T scl = T(double(N) / 6.283185307179586476925286766559);
  T ox = xix * scl, oy = xiy * scl;
  const T fx = floor(ox), fy = floor(oy);
  const T ax = ox - fx, ay = oy - fy;
  const int ix0 = wrap2N<N>(x + cell_mod<N>(fx)), iy0 = wrap2N<N>(y + cell_mod<N>(fy));
  const int ix1 = (ix0 + 1 == N) ? 0 : ix0 + 1, iy1 = (iy0 + 1 == N) ? 0 : iy0 + 1;
  const P4<T> f00 = F[iy0 * N + ix0], f01 = F[iy0 * N + ix1];
  const P4<T> f10 = F[iy1 * N + ix0], f11 = F[iy1 * N + ix1];
  const T w00 = (T(1) - ax) * (T(1) - ay), w01 = ax * (T(1) - ay);
  const T w10 = (T(1) - ax) * ay, w11 = ax * ay;
  P4<T> g;
  g.u = w00 * f00.u + w01 * f01.u + w10 * f10.u + w11 * f11.u;
  g.v = w00 * f00.v + w01 * f01.v + w10 * f10.v + w11 * f11.v;
  g.h = w00 * f00.h + w01 * f01.h + w10 * f10.h + w11 * f11.h;
  g.z = w00 * f00.z + w01 * f01.z + w10 * f10.z + w11 * f11.z;
  return g;
}

// --------------------------------------------------------------------------
// rows_dyn
// --------------------------------------------------------------------------
// value of an averaging slot's field at a point (FieldSel)
template <typename T>
__device__ __forceinline__ T field_value(int fs, const cplx<T>& uv, const cplx<T>& hz, const Phys& ph) {
  switch (fs) {
    case FS_ETA: return hz.x;
    case FS_ZETA: return hz.y;
    case FS_U: return uv.x;
    case FS_V: return uv.y;
    default: return (T(ph.f) + hz.y) / (T(ph.H) + hz.x);  // potential vorticity (f + zeta) / h
  }
}

template <typename T, int N>
__device__ __forceinline__ void rows_dyn_body(const StepPtrs<T>& P, const Dims& d, const Phys& ph, int rowblock,
                                              cplx<T>* lds) {
  using G = RowGeo<N>;
  constexpr int E = G::E, NT = G::NT;
  const int grp = row_group<NT>(), t = threadIdx.x % NT;
  const int y = rowblock * G::RPB + grp;  // the grid covers the rows exactly
  cplx<T>* buf = lds + grp * G::L;
  const size_t rf = d.rowfield_elems();
  const cplx<T>* ICr = P.IC + (size_t)y * d.NKXP;
  constexpr int K = kcut<N>();

  cplx<T> uv[E], hz[E];
  load_pair<T, N, false, false>(uv, ICr + IC_U * rf, ICr + IC_V * rf, t);
  inverse_row<T, N>(uv, buf, t, P.tw);
  // (eta + i zeta): zeta spectrum = i kx C_v - C_uy
  {
    const cplx<T>* Ch = ICr + IC_H * rf;
    const cplx<T>* Cv = ICr + IC_V * rf;
    const cplx<T>* Cuy = ICr + IC_UY * rf;
    sched_fence();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int k = t + NT * r;
      const bool lo = k <= K, hi = k >= N - K;
      const int kk = min(lo ? k : N - k, K);
      cplx<T> a = Ch[kk];
      const cplx<T> cv = Cv[kk], cu = Cuy[kk];
      cplx<T> b = {-T(kk) * cv.y - cu.x, T(kk) * cv.x - cu.y};
      const T sy = (kk == 0) ? T(0) : (hi ? T(-1) : T(1));
      a.y *= sy;
      b.y *= sy;
      hz[r] = (lo || hi) ? cplx<T>{a.x - b.y, a.y + b.x} : cplx<T>{T(0), T(0)};
    }
  }
  inverse_row<T, N>(hz, buf, t, P.tw);

  // u, v and the two averaged fields, interleaved for the gathers
  P4<T>* out = P.uvhz + (size_t)y * N;
  cplx<T>* RSr = P.RS + (size_t)y * d.NKXP;
  cplx<T> z[E];
  if (ph.fs0 == FS_ETA && ph.fs1 == FS_ZETA) {
#pragma unroll
    for (int e = 0; e < E; ++e) out[t + NT * e] = P4<T>{uv[e].x, uv[e].y, hz[e].x, hz[e].y};
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      z[e] = {field_value<T>(ph.fs0, uv[e], hz[e], ph), field_value<T>(ph.fs1, uv[e], hz[e], ph)};
      out[t + NT * e] = P4<T>{uv[e].x, uv[e].y, z[e].x, z[e].y};
    }
    // their spectra, for the Eulerian means
    if (ph.gen) forward_row<T, N, true, false>(z, buf, t, P.tw, RSr + RS_F0 * rf, RSr + RS_F1 * rf);
  }
  if (ph.kin) return;  // prescribed flow: no dynamics


#pragma unroll
  for (int e = 0; e < E; ++e) z[e] = {hz[e].y * uv[e].y, hz[e].y * uv[e].x};  // zeta v, zeta u
  forward_row<T, N, true, false>(z, buf, t, P.tw, RSr + RS_ZV * rf, RSr + RS_ZU * rf);
#pragma unroll
  for (int e = 0; e < E; ++e)
    z[e] = {T(0.5) * (uv[e].x * uv[e].x + uv[e].y * uv[e].y), hz[e].x * uv[e].x};  // K, eta u
  forward_row<T, N, true, false>(z, buf, t, P.tw, RSr + RS_K * rf, RSr + RS_HU * rf);
#pragma unroll
  for (int e = 0; e < E; ++e) z[e] = {hz[e].x * uv[e].y, T(0)};  // eta v
  forward_row<T, N, false, false>(z, buf, t, P.tw, RSr + RS_HV * rf, nullptr);
}

// The dynamics rows pass of float runs: a block of three waves shares one
// group of rows (WR = 64 / NT rows, one per lane group).  Wave 0 inverse-
// transforms (u, v) and wave 1 (eta, zeta) into their LDS buffers; after a
// barrier every wave forms its products from the shared physical values (wave
// 0 also stores them for the gathers) -- wave 0 zeta v, zeta u; wave 1 K,
// eta u; wave 2 eta v and, for other averaged fields, their values -- and
// after a second barrier each forward-transforms its products in its own
// buffer.  Five transforms per row, two deep, instead of five in a row on one
// wave; the products and transforms are the same.
template <typename T, int N>
__device__ __forceinline__ void rows_dyn_coop(const StepPtrs<T>& P, const Dims& d, const Phys& ph, int rowblock,
                                              cplx<T>* lds) {
  using G = RowGeo<N>;
  constexpr int E = G::E, NT = G::NT, L = G::L, WR = 64 / NT;
  constexpr int K = kcut<N>();
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // the wave's role
  const int lane = threadIdx.x % 64;
  const int g = lane / NT, t = lane % NT;
  const int y = rowblock * WR + g;
  cplx<T>* b0 = lds + (0 * WR + g) * L;  // (u, v) after the first phase
  cplx<T>* b1 = lds + (1 * WR + g) * L;  // (eta, zeta)
  cplx<T>* bw = lds + (w * WR + g) * L;  // this wave's transform buffer afterwards
  const size_t rf = d.rowfield_elems();
  const cplx<T>* ICr = P.IC + (size_t)y * d.NKXP;
  cplx<T>* RSr = P.RS + (size_t)y * d.NKXP;
  cplx<T> z[E];
  if (w == 0) {
    load_pair<T, N, false, false>(z, ICr + IC_U * rf, ICr + IC_V * rf, t);
    inverse_row<T, N>(z, b0, t, P.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) b0[pidx(t + NT * e)] = z[e];
  } else if (w == 1) {
    // (eta + i zeta): zeta spectrum = i kx C_v - C_uy
    const cplx<T>* Ch = ICr + IC_H * rf;
    const cplx<T>* Cv = ICr + IC_V * rf;
    const cplx<T>* Cuy = ICr + IC_UY * rf;
    sched_fence();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int k = t + NT * r;
      const bool lo = k <= K, hi = k >= N - K;
      const int kk = min(lo ? k : N - k, K);
      cplx<T> a = Ch[kk];
      const cplx<T> cv = Cv[kk], cu = Cuy[kk];
      cplx<T> b = {-T(kk) * cv.y - cu.x, T(kk) * cv.x - cu.y};
      const T sy = (kk == 0) ? T(0) : (hi ? T(-1) : T(1));
      a.y *= sy;
      b.y *= sy;
      z[r] = (lo || hi) ? cplx<T>{a.x - b.y, a.y + b.x} : cplx<T>{T(0), T(0)};
    }
    inverse_row<T, N>(z, b1, t, P.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) b1[pidx(t + NT * e)] = z[e];
  }
  __syncthreads();
  const bool dyn = !ph.kin;  // a prescribed flow needs the physical fields only
  cplx<T> zf[E];             // wave 2: the averaged fields (other than eta, zeta)
  if (w == 0) {
    // u, v and the two averaged fields, interleaved for the gathers; zeta v, zeta u
    P4<T>* out = P.uvhz + (size_t)y * N;
    const bool plain = (ph.fs0 == FS_ETA && ph.fs1 == FS_ZETA);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cplx<T> uv = b0[pidx(t + NT * e)], hz = b1[pidx(t + NT * e)];
      if (plain) out[t + NT * e] = P4<T>{uv.x, uv.y, hz.x, hz.y};
      else out[t + NT * e] = P4<T>{uv.x, uv.y, field_value<T>(ph.fs0, uv, hz, ph), field_value<T>(ph.fs1, uv, hz, ph)};
      z[e] = {hz.y * uv.y, hz.y * uv.x};
    }
  } else if (w == 1) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cplx<T> uv = b0[pidx(t + NT * e)], hz = b1[pidx(t + NT * e)];
      z[e] = {T(0.5) * (uv.x * uv.x + uv.y * uv.y), hz.x * uv.x};  // K, eta u
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cplx<T> uv = b0[pidx(t + NT * e)], hz = b1[pidx(t + NT * e)];
      z[e] = {hz.x * uv.y, T(0)};  // eta v
      if (ph.gen) zf[e] = {field_value<T>(ph.fs0, uv, hz, ph), field_value<T>(ph.fs1, uv, hz, ph)};
    }
  }
  __syncthreads();
  if (w == 0) {
    if (dyn) forward_row<T, N, true, false>(z, bw, t, P.tw, RSr + RS_ZV * rf, RSr + RS_ZU * rf);
  } else if (w == 1) {
    if (dyn) forward_row<T, N, true, false>(z, bw, t, P.tw, RSr + RS_K * rf, RSr + RS_HU * rf);
  } else {
    // the averaged fields' spectra, for the Eulerian means
    if (ph.gen) forward_row<T, N, true, false>(zf, bw, t, P.tw, RSr + RS_F0 * rf, RSr + RS_F1 * rf);
    if (dyn) forward_row<T, N, false, false>(z, bw, t, P.tw, RSr + RS_HV * rf, nullptr);
  }
}

// Geometry of the dynamics rows pass: float runs take blocks of three waves
// sharing one group of rows; float64 (whose registers leave room for one wave
// per SIMD) blocks of ROW_WAVES waves, one row group each, every product on
// the row's own wave.
template <typename T, int N>
struct DynGeo {
  static constexpr bool COOP = sizeof(T) == 4;
  static constexpr int WR = 64 / RowGeo<N>::NT;  // rows per wave
  static constexpr int THREADS = COOP ? 3 * 64 : 64 * ROW_WAVES;
  static constexpr int RPB = COOP ? WR : RowGeo<N>::RPB;  // rows per block
  static constexpr int LDS = (COOP ? 3 * WR : RowGeo<N>::RPB) * RowGeo<N>::L;
  static_assert(RowGeo<N>::NT <= 64 && 64 % RowGeo<N>::NT == 0, "row groups within a wave");
};

// float: three resident waves per SIMD (at most 168 registers): one block of
// the cooperative form on each
template <typename T>
__host__ __device__ constexpr int dyn_waves() {
  return sizeof(T) == 4 ? 3 : 1;
}

template <typename T, int N>
__global__ void __launch_bounds__((DynGeo<T, N>::THREADS), (dyn_waves<T>())) k_rows_dyn(StepPtrs<T> P, Dims d,
                                                                                       Phys ph, int remap) {
  __shared__ cplx<T> lds[DynGeo<T, N>::LDS];
  int rowblock, unused, z;
  xcd_split(gridDim.x, 1, rowblock, unused, z, remap);
  if constexpr (DynGeo<T, N>::COOP) rows_dyn_coop<T, N>(P, d, ph, rowblock, lds);
  else rows_dyn_body<T, N>(P, d, ph, rowblock, lds);
}

// --------------------------------------------------------------------------
// rows_rhs
// --------------------------------------------------------------------------
// Tasks, one wavefront per row and task.  Float runs of N >= 512 take two:
//   RT_S2  strategy 2: both xi components (eq. (4.5a)) and g-bar of eta and
//          zeta (eq. (4.5b)), from one transform of xi and one gather
//   RT_S1  strategy 1: g-tilde of eta and zeta (eq. (4.1); their sources are
//          added in the column pass) and both P components (eq. (3.9) in P form)
// (each wave holds two output pairs; the rows' 2N waves at two per SIMD run in
// one round).  Smaller grids and float64, where more, shorter waves pay
// better, take four: RT4_XI (xi), RT4_GB (g-bar), RT4_GT (g-tilde), RT4_P (P),
// the two strategy-2 tasks each transforming xi and gathering at x + xi.

// The mean right-hand-side rows pass, two tasks per row.
// Task 0, strategy 2: with w = xi / (t - tau) the partial-mean velocity (u / 2
// at t = tau, SPOS false), the gathered terms at x + xi less w . grad of
// (xi_x, xi_y) and of (g-bar_h, g-bar_zeta): one transform of xi serves both,
// and one gather of the interleaved point serves all four fields.
template <typename T, int N, bool CUB, bool SPOS>
__device__ __forceinline__ void rows_rhs_s2(const StepPtrs<T>& P, const Dims& d, double s, int y, int t,
                                            cplx<T>* buf, cplx<T>* xs) {
  using G = RowGeo<N>;
  constexpr int E = G::E, NT = G::NT;
  const size_t rf = d.rowfield_elems();
  const cplx<T>* ICr = P.IC + (size_t)y * d.NKXP;
  cplx<T>* RSr = P.RS + (size_t)y * d.NKXP;
  const P4<T>* F = P.uvhz;
  const P4<T>* Fr = P.uvhz + (size_t)y * N;
  const T inv_s = SPOS ? T(1.0 / s) : T(0);
  // w at point e from xi
  auto wof = [&](int e, cplx<T> xi) -> cplx<T> {
    if constexpr (SPOS) {
      return {xi.x * inv_s, xi.y * inv_s};
    } else {
      const P4<T> q = Fr[t + NT * e];
      return {T(0.5) * q.u, T(0.5) * q.v};
    }
  };
  cplx<T> a[E], guv[E], ghz[E], b[E];
  // displacement xi, kept in the row's second LDS buffer (xs) after the gathers
  load_pair<T, N, false, false>(a, ICr + IC_XIX * rf, ICr + IC_XIY * rf, t);
  inverse_row<T, N>(a, buf, t, P.tw);
#pragma unroll
  for (int e = 0; e < E; ++e) xs[pidx(t + NT * e)] = a[e];
  // gathered (u, v) less w, and (eta, zeta), at x + xi
  if constexpr (CUB) {
    // cubic gathers: 16 corners per point, one point in flight at a time
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cplx<T> w = wof(e, a[e]);
      const cplx<T> g = gather2_cubic<T, N, 0>(F, t + NT * e, y, a[e].x, a[e].y);
      guv[e] = {g.x - w.x, g.y - w.y};
      ghz[e] = gather2_cubic<T, N, 1>(F, t + NT * e, y, a[e].x, a[e].y);
      sched_fence();
    }
  } else {
    constexpr int GG = 4;  // points with their loads in flight together
    static_assert(E % GG == 0, "gather groups");
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += GG) {
#pragma unroll
      for (int e = e0; e < e0 + GG; ++e) {
        const cplx<T> w = wof(e, a[e]);
        const P4<T> g = gather4<T, N>(F, t + NT * e, y, a[e].x, a[e].y);
        guv[e] = {g.u - w.x, g.v - w.y};
        ghz[e] = {g.h, g.z};
      }
      sched_fence();
    }
  }
  // less w . grad of each component (a rolled loop: unrolled, the compiler
  // interleaves the four transforms and runs out of registers)
#pragma unroll 2
  for (int c = 0; c < 4; ++c) {
    const int f = (c == 0) ? IC_XIX : (c == 1) ? IC_XIY : (c == 2) ? IC_GBH : IC_GBZ;
    load_pair<T, N, true, false>(b, ICr + f * rf, ICr + (f + 1) * rf, t);
    inverse_row<T, N>(b, buf, t, P.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cplx<T> w = wof(e, xs[pidx(t + NT * e)]);
      const T dw = w.x * b[e].x + w.y * b[e].y;
      if (c == 0) guv[e].x = guv[e].x - dw;
      else if (c == 1) guv[e].y = guv[e].y - dw;
      else if (c == 2) ghz[e].x = ghz[e].x - dw;
      else ghz[e].y = ghz[e].y - dw;
    }
    sched_fence();
  }
  forward_row<T, N, true>(guv, buf, t, P.tw, RSr + RS_XIX * rf, RSr + RS_XIY * rf);
  forward_row<T, N, true>(ghz, buf, t, P.tw, RSr + RS_GBH * rf, RSr + RS_GBZ * rf);
}

// Task 1, strategy 1 and the Lagrangian-mean velocity: f - u . grad g-tilde
// and (t - tau) u - u . grad P; the velocity is re-read where it is used.  For
// the default pair (eta, zeta), src = 0: the source f is added in the column
// pass from the stage spectra (as the Eulerian accumulators take it), so that
// only the advection term goes through physical space and float32 rounding;
// other averaged fields (src = 1) take f here.
template <typename T, int N>
__device__ __forceinline__ void rows_rhs_s1(const StepPtrs<T>& P, const Dims& d, double s, int y, int t,
                                            cplx<T>* buf, int src) {
  using G = RowGeo<N>;
  constexpr int E = G::E, NT = G::NT;
  const size_t rf = d.rowfield_elems();
  const cplx<T>* ICr = P.IC + (size_t)y * d.NKXP;
  cplx<T>* RSr = P.RS + (size_t)y * d.NKXP;
  const P4<T>* Fr = P.uvhz + (size_t)y * N;
  const T sT = T(s), fs = src ? T(1) : T(0);
  cplx<T> agt[E], apx[E], b[E];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int f = (c == 0) ? IC_GTH : (c == 1) ? IC_GTZ : (c == 2) ? IC_PX : IC_PY;
    load_pair<T, N, true, false>(b, ICr + f * rf, ICr + (f + 1) * rf, t);
    inverse_row<T, N>(b, buf, t, P.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const P4<T> q = Fr[t + NT * e];
      const T f = (c == 0) ? fs * q.h : (c == 1) ? fs * q.z : (c == 2) ? sT * q.u : sT * q.v;
      const T r = f - (q.u * b[e].x + q.v * b[e].y);
      if (c == 0) agt[e].x = r;
      else if (c == 1) agt[e].y = r;
      else if (c == 2) apx[e].x = r;
      else apx[e].y = r;
    }
    sched_fence();
  }
  forward_row<T, N, true>(agt, buf, t, P.tw, RSr + RS_GTH * rf, RSr + RS_GTZ * rf);
  forward_row<T, N, true>(apx, buf, t, P.tw, RSr + RS_PX * rf, RSr + RS_PY * rf);
}

template <typename T, int N, bool CUB>
__device__ __forceinline__ void rows_rhs_body4(const StepPtrs<T>& P, const Dims& d, double s, int rowblock,
                                              int task, cplx<T>* lds, int src) {
  using G = RowGeo<N>;
  constexpr int E = G::E, NT = G::NT;
  const int grp = row_group<NT>(), t = threadIdx.x % NT;
  const int y = rowblock * G::RPB + grp;  // the grid covers the rows exactly
  cplx<T>* buf = lds + grp * G::L;
  const size_t rf = d.rowfield_elems();
  const cplx<T>* ICr = P.IC + (size_t)y * d.NKXP;
  cplx<T>* RSr = P.RS + (size_t)y * d.NKXP;
  const P4<T>* F = P.uvhz;
  const P4<T>* Fr = P.uvhz + (size_t)y * N;
  constexpr int K = kcut<N>();

  cplx<T> a[E], b[E];
  if (task == RT4_XI || task == RT4_GB) {
    // displacement xi, partial-mean velocity w = xi / (t - tau) (u/2 at t = tau)
    load_pair<T, N, false, false>(a, ICr + IC_XIX * rf, ICr + IC_XIY * rf, t);
    inverse_row<T, N>(a, buf, t, P.tw);
    cplx<T> w[E];
    if (s > 0.0) {
      const T inv_s = T(1.0 / s);
#pragma unroll
      for (int e = 0; e < E; ++e) w[e] = {a[e].x * inv_s, a[e].y * inv_s};
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const P4<T> q = Fr[t + NT * e];
        w[e] = {T(0.5) * q.u, T(0.5) * q.v};
      }
    }
    sched_fence();
    // gathered terms at x + xi, in groups of GG points (bounds loads in flight)
    constexpr int GG = 4;
    static_assert(E % GG == 0, "gather groups");
    const bool xi_task = (task == RT4_XI);
    if constexpr (CUB) {
      // cubic gathers: 16 corners per point, one point in flight at a time
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (xi_task) {
          const cplx<T> g = gather2_cubic<T, N, 0>(F, t + NT * e, y, a[e].x, a[e].y);
          a[e] = {g.x - w[e].x, g.y - w[e].y};
        } else {
          a[e] = gather2_cubic<T, N, 1>(F, t + NT * e, y, a[e].x, a[e].y);
        }
        sched_fence();
      }
    } else if (xi_task) {
#pragma unroll
      for (int e0 = 0; e0 < E; e0 += GG) {
#pragma unroll
        for (int e = e0; e < e0 + GG; ++e) {
          const cplx<T> g = gather2<T, N, 0>(F, t + NT * e, y, a[e].x, a[e].y);
          a[e] = {g.x - w[e].x, g.y - w[e].y};
        }
        sched_fence();
      }
    } else {
#pragma unroll
      for (int e0 = 0; e0 < E; e0 += GG) {
#pragma unroll
        for (int e = e0; e < e0 + GG; ++e) a[e] = gather2<T, N, 1>(F, t + NT * e, y, a[e].x, a[e].y);
        sched_fence();
      }
    }
    // minus w . grad of (xi_x, xi_y) or of (g-bar_h, g-bar_zeta)
    const int f1 = xi_task ? IC_XIX : IC_GBH, f2 = xi_task ? IC_XIY : IC_GBZ;
    load_pair<T, N, true, false>(b, ICr + f1 * rf, ICr + (f1 + 1) * rf, t);
    inverse_row<T, N>(b, buf, t, P.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) a[e].x = a[e].x - (w[e].x * b[e].x + w[e].y * b[e].y);
    load_pair<T, N, true, false>(b, ICr + f2 * rf, ICr + (f2 + 1) * rf, t);
    inverse_row<T, N>(b, buf, t, P.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) a[e].y = a[e].y - (w[e].x * b[e].x + w[e].y * b[e].y);
    const int o = xi_task ? RS_XIX : RS_GBH;
    forward_row<T, N, true>(a, buf, t, P.tw, RSr + o * rf, RSr + (o + 1) * rf);
  } else {
    // f - u . grad g-tilde (f only when src: see rows_rhs_s1), or (t - tau) u - u . grad P
    const bool gt = (task == RT4_GT);
    const T sT = T(s), fs = src ? T(1) : T(0);
    cplx<T> uv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const P4<T> q = Fr[t + NT * e];
      uv[e] = {q.u, q.v};
    }
    const int f1 = gt ? IC_GTH : IC_PX, f2 = gt ? IC_GTZ : IC_PY;
    load_pair<T, N, true, false>(b, ICr + f1 * rf, ICr + (f1 + 1) * rf, t);
    inverse_row<T, N>(b, buf, t, P.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const T f = gt ? fs * Fr[t + NT * e].h : sT * uv[e].x;
      a[e].x = f - (uv[e].x * b[e].x + uv[e].y * b[e].y);
    }
    load_pair<T, N, true, false>(b, ICr + f2 * rf, ICr + (f2 + 1) * rf, t);
    inverse_row<T, N>(b, buf, t, P.tw);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const T f = gt ? fs * Fr[t + NT * e].z : sT * uv[e].y;
      a[e].y = f - (uv[e].x * b[e].x + uv[e].y * b[e].y);
    }
    const int o = gt ? RS_GTH : RS_PX;
    forward_row<T, N, true>(a, buf, t, P.tw, RSr + o * rf, RSr + (o + 1) * rf);
  }
}

template <typename T, int N, bool CUB>
__device__ __forceinline__ void rows_rhs_body(const StepPtrs<T>& P, const Dims& d, double s, int rowblock,
                                              int task, cplx<T>* lds, int src) {
  using G = RowGeo<N>;
  constexpr int NT = G::NT;
  if constexpr (!rhs_merged<T, N>()) {
    rows_rhs_body4<T, N, CUB>(P, d, s, rowblock, task, lds, src);
    return;
  }
  const int grp = row_group<NT>(), t = threadIdx.x % NT;
  const int y = rowblock * G::RPB + grp;  // the grid covers the rows exactly
  cplx<T>* buf = lds + grp * G::L;
  if (task == RT_S2) {
    cplx<T>* xs = lds + (G::RPB + grp) * G::L;
    if (s > 0.0) rows_rhs_s2<T, N, CUB, true>(P, d, s, y, t, buf, xs);
    else rows_rhs_s2<T, N, CUB, false>(P, d, s, y, t, buf, xs);
  } else {
    rows_rhs_s1<T, N>(P, d, s, y, t, buf, src);
  }
}

// two-task form: two resident waves per SIMD, as many as its two LDS buffers
// per row allow, so that every row's two tasks are resident at once
template <typename T, int N>
__host__ __device__ constexpr int rhs_waves() {
  return rhs_merged<T, N>() ? 2 : 1;
}
template <typename T, int N>
__host__ __device__ constexpr int rhs_lds() {
  return (rhs_merged<T, N>() ? 2 : 1) * RowGeo<N>::RPB * RowGeo<N>::L;
}

// CUB: cubic instead of bilinear strategy-2 gathers; src: the strategy-1
// sources are formed here (other averaged fields) rather than in the column pass
template <typename T, int N, bool CUB>
__global__ void __launch_bounds__(64 * ROW_WAVES, (rhs_waves<T, N>())) k_rows_rhs(StepPtrs<T> P, Dims d, double s,
                                                                              int remap, int src) {
  __shared__ cplx<T> lds[rhs_lds<T, N>()];  // transform buffers (and xi, two-task form)
  int rowblock, task, z;
  xcd_split(gridDim.x, gridDim.y, rowblock, task, z, remap);  // grid = (row blocks, tasks)
  rows_rhs_body<T, N, CUB>(P, d, s, rowblock, task, lds, src);
}

// --------------------------------------------------------------------------
// rows_mom: the strategy-2 mean of the momentum 1-form (appendix C, eq. (C.4)
// in the g-bar form of eq. (4.5b)), launched after rows_rhs when requested.
// Component i = x (task 0) or y (task 1):
//   R_i = u_j(x + xi)(delta_ij + d_i xi_j) - w_j d_j g_i - g_j d_i xi_j / s
// (w = xi / s, or u / 2 at s = 0, where g = 0 and the last term is not formed).
// Order of work keeps at most three lane arrays live beside a transform.
// --------------------------------------------------------------------------
template <typename T, int N, bool CUB>
__device__ __forceinline__ void rows_mom_body(const StepPtrs<T>& P, const Dims& d, double s, int rowblock,
                                              int task, cplx<T>* lds) {
  using G = RowGeo<N>;
  constexpr int E = G::E, NT = G::NT;
  const int grp = row_group<NT>(), t = threadIdx.x % NT;
  const int y = rowblock * G::RPB + grp;
  cplx<T>* buf = lds + grp * G::L;
  const size_t rf = d.rowfield_elems();
  const cplx<T>* ICr = P.IC + (size_t)y * d.NKXP;
  cplx<T>* RSr = P.RS + (size_t)y * d.NKXP;
  const P4<T>* F = P.uvhz;
  const P4<T>* Fr = P.uvhz + (size_t)y * N;
  const bool ix = (task == 0);
  cplx<T> a[E], b[E], c[E];
  // d_i xi_x, d_i xi_y: i kx in the row pass for i = x, the column pass's i ky versions for i = y
  if (ix) load_pair<T, N, true, true>(b, ICr + IC_XIX * rf, ICr + IC_XIY * rf, t);
  else load_pair<T, N, false, false>(b, ICr + IC_XIX_Y * rf, ICr + IC_XIY_Y * rf, t);
  inverse_row<T, N>(b, buf, t, P.tw);
  // stretching: a.x = -(g_x d_i xi_x + g_y d_i xi_y) / s
  if (s > 0.0) {
    load_pair<T, N, false, false>(c, ICr + IC_GMX * rf, ICr + IC_GMY * rf, t);
    inverse_row<T, N>(c, buf, t, P.tw);
    const T inv_s = T(1.0 / s);
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = {-(c[e].x * b[e].x + c[e].y * b[e].y) * inv_s, T(0)};
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = {T(0), T(0)};
  }
  // xi (kept until the gathers consume it)
  load_pair<T, N, false, false>(c, ICr + IC_XIX * rf, ICr + IC_XIY * rf, t);
  inverse_row<T, N>(c, buf, t, P.tw);
  // advection: a.x -= w . grad g_i with w = xi / s (u / 2 at s = 0), formed on the fly
  {
    cplx<T> dg[E];
    const int gi = ix ? IC_GMX : IC_GMY;
    load_pair<T, N, true, false>(dg, ICr + gi * rf, ICr + (gi + 1) * rf, t);
    inverse_row<T, N>(dg, buf, t, P.tw);
    if (s > 0.0) {
      const T inv_s = T(1.0 / s);
#pragma unroll
      for (int e = 0; e < E; ++e) a[e].x = a[e].x - (c[e].x * inv_s * dg[e].x + c[e].y * inv_s * dg[e].y);
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const P4<T> q = Fr[t + NT * e];
        a[e].x = a[e].x - (T(0.5) * q.u * dg[e].x + T(0.5) * q.v * dg[e].y);
      }
    }
  }
  // the gathered (u, v) at x + xi and the pulled-back source (consumes xi)
  const T dxi = ix ? T(1) : T(0), dyi = ix ? T(0) : T(1);
  if constexpr (CUB) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const cplx<T> g = gather2_cubic<T, N, 0>(F, t + NT * e, y, c[e].x, c[e].y);
      a[e].x = a[e].x + (g.x * (dxi + b[e].x) + g.y * (dyi + b[e].y));
      sched_fence();
    }
  } else {
    constexpr int GG = 4;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += GG) {
#pragma unroll
      for (int e = e0; e < e0 + GG; ++e) {
        const cplx<T> g = gather2<T, N, 0>(F, t + NT * e, y, c[e].x, c[e].y);
        a[e].x = a[e].x + (g.x * (dxi + b[e].x) + g.y * (dyi + b[e].y));
      }
      sched_fence();
    }
  }
  forward_row<T, N, false>(a, buf, t, P.tw, RSr + (ix ? RS_GMX : RS_GMY) * rf, nullptr);
}

template <typename T, int N, bool CUB>
__global__ void __launch_bounds__(64 * ROW_WAVES) k_rows_mom(StepPtrs<T> P, Dims d, double s, int remap) {
  __shared__ cplx<T> lds[RowGeo<N>::RPB * RowGeo<N>::L];
  int rowblock, task, z;
  xcd_split(gridDim.x, gridDim.y, rowblock, task, z, remap);  // grid = (row blocks, 2 components)
  rows_mom_body<T, N, CUB>(P, d, s, rowblock, task, lds);
}

// --------------------------------------------------------------------------
// columns
// --------------------------------------------------------------------------

template <typename TS>
__device__ __forceinline__ cplx<TS> cadd(cplx<TS> a, cplx<TS> b) { return {a.x + b.x, a.y + b.y}; }

// (hi, lo) + d for a float value carried as two words: Knuth's two-sum of hi
// and d gives the sum and its exact rounding error, which is folded into lo
// before the pair is renormalised (|lo| <= half an ulp of hi).  Contraction to
// fused multiply-adds is off here: the error terms need the plain roundings.
__device__ __forceinline__ void comp_add(float& hi, float& lo, float d) {
#pragma clang fp contract(off)
  const float s = hi + d;
  const float bp = s - hi;
  const float err = (hi - (s - bp)) + (d - bp);
  const float t = lo + err;
  const float h2 = s + t;
  lo = t - (h2 - s);
  hi = h2;
}

// Classical RK4 on one coefficient, in registers: y the state, lo its trailing
// word (compensated float state), a the accumulator of k1 + 2 k2 + 2 k3; k the
// stage's right-hand side.  Returns the next stage input (the new state after
// stage 3) and updates a (stages 0-2) or y and lo (stage 3), which the caller
// stores.  Float state is compensated: y holds the leading word and lo the
// trailing one, so the state itself carries about 48 significant bits and the
// rounding of the state at every step no longer accumulates over a long run.
// Stage inputs, right-hand sides and the accumulator stay float (their rounding
// enters once per step, scaled by dt).  Float64 state ignores lo.
template <typename TS>
__device__ __forceinline__ cplx<TS> rk4v(int stage, cplx<TS>& y, cplx<TS>& lo, cplx<TS>& a, cplx<TS> k,
                                         double dt) {
  if (stage == 0) {
    a = k;
    const TS c = TS(0.5 * dt);
    return {y.x + c * k.x, y.y + c * k.y};
  } else if (stage == 1 || stage == 2) {
    a = {a.x + TS(2) * k.x, a.y + TS(2) * k.y};
    const TS c = TS(stage == 1 ? 0.5 * dt : dt);
    return {y.x + c * k.x, y.y + c * k.y};
  } else {
    const TS c = TS(dt / 6.0);
    if constexpr (std::is_same<TS, float>::value) {
      comp_add(y.x, lo.x, c * (a.x + k.x));
      comp_add(y.y, lo.y, c * (a.y + k.y));
    } else {
      y = {y.x + c * (a.x + k.x), y.y + c * (a.y + k.y)};
    }
    return y;
  }
}

// the words rk4v reads (y always, a from stage 1, lo at stage 3 for float) and
// writes back (a at stages 0-2, y and lo at stage 3)
template <typename TS>
__device__ __forceinline__ void rk4_load(int stage, const cplx<TS>* Yp, const cplx<TS>* Lp, const cplx<TS>* Ap,
                                         cplx<TS>& y, cplx<TS>& lo, cplx<TS>& a) {
  y = *Yp;
  if (stage >= 1) a = *Ap;
  if constexpr (std::is_same<TS, float>::value) {
    if (stage == 3) lo = *Lp;
  }
}
template <typename TS>
__device__ __forceinline__ void rk4_store(int stage, cplx<TS>* Yp, cplx<TS>* Lp, cplx<TS>* Ap, const cplx<TS>& y,
                                          const cplx<TS>& lo, const cplx<TS>& a) {
  if (stage <= 2) {
    *Ap = a;
  } else {
    *Yp = y;
    if constexpr (std::is_same<TS, float>::value) *Lp = lo;
  }
}

template <typename T, int N, int C>
struct ColCtx {
  static constexpr int E = fft_E<N>(), NT = N / E, LC = col_buf(N);
  cplx<T>* lds;     // C buffers of LC
  cplx<T>* buf;     // this group's buffer
  int c, t, kx0, kx;
  bool valid;       // kx <= K
};

// one complex value of a buffer-resource load (8 or 16 bytes)
template <typename T>
__device__ __forceinline__ cplx<T> buffer_cplx(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
  if constexpr (sizeof(cplx<T>) == 8) return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
  else return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
}

// block-wide: rows of a [N][NKXP] field (columns kx0..kx0+C-1) into the C buffers.
// A thread keeps one column c and visits rows y = threadIdx.x / C + NT k.  The
// field is read as one buffer resource: the thread's offset sits in one vector
// register and the row step of each of its E loads in a scalar register, so all
// E loads are in flight at once for the price of their data registers (global
// loads would need an address register pair each).  Columns past K read the
// row's padding and are replaced by zeros.
template <typename T, int N, int C>
__device__ __forceinline__ void tile_load(const ColCtx<T, N, C>& cx, const cplx<T>* __restrict__ src,
                                          const Dims& d) {
  constexpr int LC = ColCtx<T, N, C>::LC, E = fft_E<N>(), NT = N / E;
  const int c = threadIdx.x % C, y0 = threadIdx.x / C;
  const bool in = cx.kx0 + c <= kcut<N>();
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<cplx<T>*>(src), (short)0, (int)(d.rowfield_elems() * sizeof(cplx<T>)), 0x00020000);
  const unsigned voff = ((unsigned)y0 * (unsigned)d.NKXP + (unsigned)(cx.kx0 + c)) * (unsigned)sizeof(cplx<T>);
  const unsigned dy = (unsigned)NT * (unsigned)d.NKXP * (unsigned)sizeof(cplx<T>);
  cplx<T>* dstl = cx.lds + c * LC;
  __syncthreads();
  cplx<T> val[E];
#pragma unroll
  for (int k = 0; k < E; ++k) val[k] = buffer_cplx<T>(rs, voff, (unsigned)k * dy);
#pragma unroll
  for (int k = 0; k < E; ++k) dstl[pidx(y0 + NT * k)] = in ? val[k] : cplx<T>{T(0), T(0)};
  __syncthreads();
}

// block-wide: the C buffers to rows of a [N][NKXP] field (columns kx0..).  The
// block is C * N / E threads, a compile-time count, so the loop unrolls and all
// of a thread's LDS reads are issued before its stores.
template <typename T, int N, int C>
__device__ __forceinline__ void tile_store(const ColCtx<T, N, C>& cx, cplx<T>* __restrict__ dst,
                                           const Dims& d) {
  constexpr int LC = ColCtx<T, N, C>::LC;
  constexpr int NTH = C * (N / fft_E<N>());
  static_assert((N * C) % NTH == 0, "tile store rounds");
  __syncthreads();
#pragma unroll
  for (int i0 = 0; i0 < N * C; i0 += NTH) {
    const int i = i0 + (int)threadIdx.x;
    const int c = i % C, y = i / C;
    const int kx = cx.kx0 + c;
    if (kx <= kcut<N>()) dst[(size_t)y * d.NKXP + kx] = cx.lds[c * LC + pidx(y)];
  }
  __syncthreads();
}

// forward column transform of one row-spectrum field; the spectrum is left in
// the wave's buffer (natural order), unnormalised
template <typename T, int N, int C>
__device__ __forceinline__ void column_forward_lds(const ColCtx<T, N, C>& cx, const cplx<T>* src, const Dims& d,
                                                   const cplx<T>* __restrict__ tw) {
  constexpr int E = fft_E<N>(), NT = N / E;
  tile_load<T, N, C>(cx, src, d);
  cplx<T> v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = cx.buf[pidx(cx.t + NT * r)];
  xsync<NT>();
  fft<T, N, fft_E<N>(), -1>(v, cx.buf, cx.t, tw);
}

// the masked, 1/N^2-normalised right-hand-side value at k = t + NT r from the
// spectrum column_forward_lds left in the buffer
template <typename T, int N, int C>
__device__ __forceinline__ cplx<T> column_value(const ColCtx<T, N, C>& cx, int r) {
  constexpr int NT = N / fft_E<N>();
  const T inv = T(1.0 / (double(N) * double(N)));
  const cplx<T> q = cx.buf[pidx(cx.t + NT * r)];
  return {q.x * inv, q.y * inv};
}

// forward column transform of A - i kx B for two row-spectrum fields: a
// column's kx is fixed, so the x-derivative of B joins A before one transform
// (the transform is linear).  Returns the masked, 1/N^2-normalised values at
// k = t + NT r.
template <typename T, int N, int C>
__device__ __forceinline__ void column_forward_dx(const ColCtx<T, N, C>& cx, const cplx<T>* srcA,
                                                  const cplx<T>* srcB, const Dims& d,
                                                  const cplx<T>* __restrict__ tw, cplx<T> (&out)[fft_E<N>()]) {
  constexpr int E = fft_E<N>(), NT = N / E;
  tile_load<T, N, C>(cx, srcA, d);
  cplx<T> v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = cx.buf[pidx(cx.t + NT * r)];
  tile_load<T, N, C>(cx, srcB, d);  // its opening barrier: every wave has read A
  const T kxT = T(cx.kx);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const cplx<T> b = cx.buf[pidx(cx.t + NT * r)];
    v[r] = {v[r].x + kxT * b.y, v[r].y - kxT * b.x};
  }
  xsync<NT>();
  fft<T, N, fft_E<N>(), -1>(v, cx.buf, cx.t, tw);
#pragma unroll
  for (int r = 0; r < E; ++r) out[r] = column_value<T, N, C>(cx, r);
}

// forward column transform of one row-spectrum field; returns the masked,
// 1/N^2-normalised right-hand-side values at k = t + NT r
template <typename T, int N, int C>
__device__ __forceinline__ void column_forward(const ColCtx<T, N, C>& cx, const cplx<T>* src, const Dims& d,
                                               const cplx<T>* __restrict__ tw, cplx<T> (&out)[fft_E<N>()]) {
  constexpr int E = fft_E<N>();
  column_forward_lds<T, N, C>(cx, src, d, tw);
#pragma unroll
  for (int r = 0; r < E; ++r) out[r] = column_value<T, N, C>(cx, r);
}

// inverse column transform of values S at k = t + NT r (already zero outside
// the mask), optionally times i ky, stored to an intermediate field
template <typename T, int N, int C, typename TS, bool DY>
__device__ __forceinline__ void column_inverse(const ColCtx<T, N, C>& cx, const cplx<TS> (&S)[fft_E<N>()],
                                               cplx<T>* dst, const Dims& d, const cplx<T>* __restrict__ tw) {
  constexpr int E = fft_E<N>(), NT = N / E;
  cplx<T> v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = cx.t + NT * r;
    const int ky = (k <= N / 2) ? k : k - N;
    cplx<T> q = {T(S[r].x), T(S[r].y)};
    if (DY) q = {-T(ky) * q.y, T(ky) * q.x};
    v[r] = q;
  }
  // no barrier: since the last block-wide tile access (which ends with one)
  // only this wavefront has touched its buffer
  fft<T, N, fft_E<N>(), +1>(v, cx.buf, cx.t, tw);
  tile_store<T, N, C>(cx, dst, d);
}

// Fourier coefficient (the stored kx >= 0 half, 1/N^2-normalised) of u, v or h
// (G = CG_U, CG_V, CG_H) of the prescribed flow at time t: a linear Poincare
// plane wave h' = A cos(theta), theta = k.x - omega t + phase, with the linear
// shallow-water polarisation of section 4.2.1, eq. (4.8), in any direction,
//   u' = A (omega kx cos(theta) - f ky sin(theta)) / (H |k|^2),
//   v' = A (omega ky cos(theta) + f kx sin(theta)) / (H |k|^2),
// plus the uniform flow (U0, V0), and the depth H at k = 0.  With
// cos(theta) = (e^{i theta} + e^{-i theta}) / 2 the +k mode's coefficient is
// (A / 2) C e^{i (phase - omega t)}, C = 1, (omega kx + i f ky) / (H |k|^2) or
// (omega ky - i f kx) / (H |k|^2); a stored entry at -k holds its conjugate.
template <int G>
__device__ cplx<double> kin_coef(int kx, int ky, double t, const Phys& ph) {
  cplx<double> c = {0.0, 0.0};
  if (kx == 0 && ky == 0) c.x = (G == CG_U) ? ph.U0 : (G == CG_V) ? ph.V0 : ph.H;
  const int wx = int(ph.kx), wy = int(ph.ky);
  const bool plus = (kx == wx && ky == wy), minus = (kx == -wx && ky == -wy);
  if ((wx == 0 && wy == 0) || !(plus || minus)) return c;
  const double k2 = ph.kx * ph.kx + ph.ky * ph.ky;
  double cr = 1.0, ci = 0.0;
  if (G == CG_U) {
    cr = ph.omega * ph.kx / (ph.H * k2);
    ci = ph.f * ph.ky / (ph.H * k2);
  } else if (G == CG_V) {
    cr = ph.omega * ph.ky / (ph.H * k2);
    ci = -ph.f * ph.kx / (ph.H * k2);
  }
  double sn, cs;
  sincos(ph.phase - ph.omega * t, &sn, &cs);
  const double a = 0.5 * ph.A;
  cplx<double> m = {a * (cr * cs - ci * sn), a * (cr * sn + ci * cs)};
  if (minus) m.y = -m.y;
  c.x += m.x;
  c.y += m.y;
  return c;
}

// stage >= 0: the RK4 stage; stage < 0: the prologue (the current state's
// column-pass outputs only).  t_next: time of the stage input this launch
// prepares (the prescribed flow of a kinematic run is evaluated there).
template <typename T, int N, int C, int G>
__device__ __forceinline__ void column_group(const ColCtx<T, N, C>& cx, const StepPtrs<T>& P, const Dims& d,
                                             const Phys& ph, int stage, double t_next,
                                             const cplx<T>* __restrict__ Ys_in, cplx<T>* __restrict__ Ys_out) {
  constexpr int E = fft_E<N>(), NT = N / E;
  constexpr bool DBL = (G == CG_XIX || G == CG_XIY || G == CG_PX || G == CG_PY);
  constexpr bool DYN = (G == CG_U || G == CG_V || G == CG_H);
  constexpr bool EUL = (G == CG_EF0 || G == CG_EF1);  // Eulerian accumulators of the averaged fields
  using TS = typename std::conditional<DBL, double, T>::type;
  const size_t sp = d.spec_elems();
  const size_t rf = d.rowfield_elems();
  constexpr int K = kcut<N>();
  if constexpr (EUL) {
    if (stage < 0) return;  // not an input of the rows passes
  }

  // right-hand-side inputs of this group
  constexpr int NF = DYN ? 2 : 1;
  constexpr int F0 = (G == CG_U) ? RS_ZV : (G == CG_V) ? RS_ZU : (G == CG_H) ? RS_HU
                   : (G == CG_XIX) ? RS_XIX : (G == CG_XIY) ? RS_XIY : (G == CG_GBH) ? RS_GBH
                   : (G == CG_GBZ) ? RS_GBZ : (G == CG_GTH) ? RS_GTH : (G == CG_GTZ) ? RS_GTZ
                   : (G == CG_PX) ? RS_PX : (G == CG_PY) ? RS_PY : (G == CG_GMX) ? RS_GMX
                   : (G == CG_GMY) ? RS_GMY : (G == CG_EF0) ? RS_F0 : RS_F1;
  constexpr int F1 = (G == CG_U || G == CG_V) ? RS_K : RS_HV;
  // the first input's values in registers; the second one's (dynamics groups)
  // stay in the wave's buffer until the stage update reads them
  cplx<T> r0[E];
  // a kinematic run has no dynamics right-hand sides
  if (stage >= 0 && !(DYN && ph.kin)) {
    if constexpr (G == CG_U) {
      // zeta v - i kx K in one transform
      column_forward_dx<T, N, C>(cx, P.RS + F0 * rf, P.RS + F1 * rf, d, P.tw, r0);
    } else {
      column_forward<T, N, C>(cx, P.RS + F0 * rf, d, P.tw, r0);
      if constexpr (NF == 2) column_forward_lds<T, N, C>(cx, P.RS + F1 * rf, d, P.tw);
    }
  }

  // state of this group
  cplx<TS>* Y;
  cplx<TS>* YL = nullptr;  // trailing words of compensated float state
  cplx<TS>* A;
  if constexpr (DBL) {
    constexpr int sd = (G == CG_XIX) ? SD_XIX : (G == CG_XIY) ? SD_XIY : (G == CG_PX) ? SD_PX : SD_PY;
    Y = P.Yd + sd * sp;
    A = P.Ad + sd * sp;
  } else {
    constexpr int sr = (G == CG_U) ? SF_U : (G == CG_V) ? SF_V : (G == CG_H) ? SF_H : (G == CG_GBH) ? SF_GBH
                     : (G == CG_GBZ) ? SF_GBZ : (G == CG_GTH) ? SF_GTH : (G == CG_GTZ) ? SF_GTZ
                     : (G == CG_GMX) ? SF_GMX : (G == CG_GMY) ? SF_GMY : (G == CG_EF0) ? SF_EH : SF_EZ;
    Y = reinterpret_cast<cplx<TS>*>(P.Yr) + sr * sp;
    if constexpr (std::is_same<TS, float>::value) YL = reinterpret_cast<cplx<TS>*>(P.Yl) + sr * sp;
    A = reinterpret_cast<cplx<TS>*>(P.Ar) + sr * sp;
  }
  const size_t col = (size_t)cx.kx * d.NKY;
  const T fT = T(ph.f), gT = T(ph.g), HT = T(ph.H);

  cplx<TS> S[E];
  if (stage < 0 || (DYN && ph.kin)) {
    // prologue (the current state's transforms) or a prescribed flow
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int k = cx.t + NT * r;
      int ky;
      bool in = true;
      if (k <= K) ky = k;
      else if (k >= N - K) ky = k - N;
      else { ky = 0; in = false; }
      S[r] = {TS(0), TS(0)};
      if (!(in && cx.valid)) continue;
      const size_t j = col + (size_t)(ky + K);
      if constexpr (DYN) {
        if (ph.kin) {
          // the next stage input is the prescribed flow at t_next
          const cplx<double> c = kin_coef<G>(cx.kx, ky, t_next, ph);
          S[r] = {TS(c.x), TS(c.y)};
          Ys_out[(G - CG_U) * sp + j] = S[r];
          continue;
        }
      }
      S[r] = Y[j];
      if constexpr (DYN) Ys_out[(G - CG_U) * sp + j] = S[r];
    }
  } else {
    // RK4 stage.  The coefficients are taken in batches of RB: every load of a
    // batch (stage values, state, accumulator) is issued before its first
    // store, so the batch's loads are in flight together (stores to the state
    // could alias later loads as far as the compiler knows, which would
    // otherwise serialise the coefficients).
    // For the default averaged fields (eta, zeta) the g-tilde groups take their
    // source f from the stage spectra, f = eta (h less H at k = 0) for g-tilde_h
    // and f = i kx v - i ky u for g-tilde_zeta (eq. (4.1): the rows pass formed
    // only - u . grad g-tilde).  The Eulerian accumulators, dE_f/dt = f, the same
    // spectrum with no transform, ride along with the g-tilde groups (even batch
    // positions r, where f is at hand) and the g-bar groups (odd ones), which
    // balances the blocks.  (Other averaged fields: sources in the rows pass,
    // Eulerian means in groups CG_EF0/EF1.)
    constexpr bool EULA = (G == CG_GTH || G == CG_GBH), EULB = (G == CG_GTZ || G == CG_GBZ);
    constexpr bool SRCG = (G == CG_GTH || G == CG_GTZ);
    constexpr int EPAR = SRCG ? 0 : 1;
    const bool eul = (EULA || EULB) && !ph.gen;
    constexpr int RB0 = (DBL || DYN || EULA || EULB) ? 4 : 8;
    constexpr int RB = (E % RB0 == 0) ? RB0 : 4;
    static_assert(E % RB == 0, "coefficient batches");
#pragma unroll
    for (int r0i = 0; r0i < E; r0i += RB) {
      bool ok[RB];
      int kyv[RB];
      cplx<T> su[RB], sv[RB], sh[RB];
      cplx<TS> y[RB], lo[RB], a[RB];
      cplx<T> ey[RB], el[RB], ea[RB];  // Eulerian accumulator
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int k = cx.t + NT * (r0i + q);
        int ky;
        bool in = true;
        if (k <= K) ky = k;
        else if (k >= N - K) ky = k - N;
        else { ky = 0; in = false; }
        ok[q] = in && cx.valid;
        kyv[q] = ky;
        if (!ok[q]) continue;
        const size_t j = col + (size_t)(ky + K);
        if constexpr (DYN) {
          su[q] = Ys_in[0 * sp + j];
          sv[q] = Ys_in[1 * sp + j];
          sh[q] = Ys_in[2 * sp + j];
        }
        rk4_load<TS>(stage, Y + j, YL + j, A + j, y[q], lo[q], a[q]);
        if constexpr (EULA || EULB) {
          const bool acc = (r0i + q) % 2 == EPAR;
          if (eul && (SRCG || acc)) {
            if constexpr (EULA) {
              sh[q] = Ys_in[2 * sp + j];
            } else {
              su[q] = Ys_in[0 * sp + j];
              sv[q] = Ys_in[1 * sp + j];
            }
          }
          if (eul && acc) {
            constexpr int se = EULA ? SF_EH : SF_EZ;
            rk4_load<T>(stage, P.Yr + se * sp + j, P.Yl + se * sp + j, P.Ar + se * sp + j, ey[q], el[q], ea[q]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int r = r0i + q;
        S[r] = {TS(0), TS(0)};
        if (!ok[q]) continue;
        const int ky = kyv[q];
        const size_t j = col + (size_t)(ky + K);
        const T kxT = T(cx.kx), kyT = T(ky);
        cplx<T> fsrc = {T(0), T(0)};  // f = eta or zeta from the stage spectra
        if constexpr (EULA || EULB) {
          // dE_eta/dt = eta (h less H at k = 0), dE_zeta/dt = i kx v - i ky u
          const bool acc = r % 2 == EPAR;
          if (eul && (SRCG || acc)) {
            if constexpr (EULA) {
              fsrc = sh[q];
              if (cx.kx == 0 && ky == 0) fsrc.x -= HT;
            } else {
              fsrc = {-kxT * sv[q].y + kyT * su[q].y, kxT * sv[q].x - kyT * su[q].x};
            }
          }
          if (eul && acc) {
            constexpr int se = EULA ? SF_EH : SF_EZ;
            rk4v<T>(stage, ey[q], el[q], ea[q], fsrc, ph.dt);
            rk4_store<T>(stage, P.Yr + se * sp + j, P.Yl + se * sp + j, P.Ar + se * sp + j, ey[q], el[q], ea[q]);
          }
        }
        const double k2 = double(cx.kx) * cx.kx + double(ky) * ky;
        const T hv = T(ph.nu8 * (k2 * k2) * (k2 * k2));
        cplx<T> R;
        if constexpr (G == CG_U) {
          // (zeta v - i kx K) + f v - i kx g h - nu8 |k|^8 u
          const cplx<T> u = su[q], v = sv[q], h = sh[q];
          const cplx<T> B = {gT * h.x, gT * h.y};
          R = {r0[r].x + fT * v.x + kxT * B.y - hv * u.x, r0[r].y + fT * v.y - kxT * B.x - hv * u.y};
        } else if constexpr (G == CG_V) {
          // -zeta u - f u - i ky (g h + K) - nu8 |k|^8 v
          const cplx<T> u = su[q], v = sv[q], h = sh[q];
          const cplx<T> r1 = column_value<T, N, C>(cx, r);
          const cplx<T> B = {gT * h.x + r1.x, gT * h.y + r1.y};
          R = {-r0[r].x - fT * u.x + kyT * B.y - hv * v.x, -r0[r].y - fT * u.y - kyT * B.x - hv * v.y};
        } else if constexpr (G == CG_H) {
          // -i kx (H u + F(eta u)) - i ky (H v + F(eta v)) - nu8 |k|^8 h
          const cplx<T> u = su[q], v = sv[q], h = sh[q];
          const cplx<T> fx = {HT * u.x + r0[r].x, HT * u.y + r0[r].y};
          const cplx<T> r1 = column_value<T, N, C>(cx, r);
          const cplx<T> fy = {HT * v.x + r1.x, HT * v.y + r1.y};
          R = {kxT * fx.y + kyT * fy.y - hv * h.x, -kxT * fx.x - kyT * fy.x - hv * h.y};
        } else {
          R = r0[r];
          if constexpr (SRCG) R = {R.x + fsrc.x, R.y + fsrc.y};
          (void)hv;
        }
        const cplx<TS> Rk = {TS(R.x), TS(R.y)};
        S[r] = rk4v<TS>(stage, y[q], lo[q], a[q], Rk, ph.dt);
        rk4_store<TS>(stage, Y + j, YL + j, A + j, y[q], lo[q], a[q]);
        if constexpr (DYN) Ys_out[(G - CG_U) * sp + j] = S[r];
      }
    }
  }

  // inverse column transforms of the next stage input
  if constexpr (G == CG_U) {
    column_inverse<T, N, C, TS, false>(cx, S, P.IC + IC_U * rf, d, P.tw);
    column_inverse<T, N, C, TS, true>(cx, S, P.IC + IC_UY * rf, d, P.tw);
  } else if constexpr (G == CG_V) {
    column_inverse<T, N, C, TS, false>(cx, S, P.IC + IC_V * rf, d, P.tw);
  } else if constexpr (G == CG_H) {
    // the rows passes work with eta = h - H: drop H from the mean (k = 0, lane 0)
    if (cx.kx == 0 && cx.t == 0) S[0].x -= TS(ph.H);
    column_inverse<T, N, C, TS, false>(cx, S, P.IC + IC_H * rf, d, P.tw);
  } else if constexpr (!EUL) {
    constexpr int o = (G == CG_XIX) ? IC_XIX : (G == CG_XIY) ? IC_XIY : (G == CG_GBH) ? IC_GBH
                    : (G == CG_GBZ) ? IC_GBZ : (G == CG_GTH) ? IC_GTH : (G == CG_GTZ) ? IC_GTZ
                    : (G == CG_PX) ? IC_PX : (G == CG_PY) ? IC_PY : (G == CG_GMX) ? IC_GMX : IC_GMY;
    column_inverse<T, N, C, TS, false>(cx, S, P.IC + o * rf, d, P.tw);
    column_inverse<T, N, C, TS, true>(cx, S, P.IC + (o + 1) * rf, d, P.tw);
  }
}

// stage >= 0: RK4 stage; stage < 0: only transform the current state (prologue)
template <typename T, int N, int C>
__device__ __forceinline__ void columns_body(const StepPtrs<T>& P, const Dims& d, const Phys& ph, int stage,
                                             double t_next, const cplx<T>* Ys_in, cplx<T>* Ys_out, int tile,
                                             int slot, cplx<T>* lds) {
  constexpr int E = fft_E<N>(), NT = N / E, LC = col_buf(N);
  ColCtx<T, N, C> cx;
  cx.lds = lds;
  cx.c = threadIdx.x / NT;
  cx.t = threadIdx.x % NT;
  cx.buf = lds + cx.c * LC;
  cx.kx0 = tile * C;
  cx.kx = cx.kx0 + cx.c;
  cx.valid = cx.kx <= kcut<N>();
  (void)E;
#define LM_CG(g) \
  case g: column_group<T, N, C, g>(cx, P, d, ph, stage, t_next, Ys_in, Ys_out); break
  switch (col_group_of(ph, slot)) {
    LM_CG(CG_U); LM_CG(CG_V); LM_CG(CG_H); LM_CG(CG_XIX); LM_CG(CG_XIY); LM_CG(CG_GBH); LM_CG(CG_GBZ);
    LM_CG(CG_GTH); LM_CG(CG_GTZ); LM_CG(CG_PX); LM_CG(CG_PY); LM_CG(CG_GMX); LM_CG(CG_GMY);
    LM_CG(CG_EF0); LM_CG(CG_EF1);
    default: break;
  }
#undef LM_CG
}

// float32: ask for 4 resident waves per SIMD (at most 128 registers), which
// every size reaches without spilling more than a few words; float64 is out of
// its reach
template <typename T, int N, bool BATCHED>
__host__ __device__ constexpr int col_waves() {
  return sizeof(T) == 4 ? 4 : 1;
}

// W: column tile width (col_tile<N, W>)
// slot0: the first group slot of this launch (grid = (column tiles, group slots))
template <typename T, int N, int W>
__global__ void __launch_bounds__((col_threads<N, W>()), (col_waves<T, N, false>()))
    k_columns(StepPtrs<T> P, Dims d, Phys ph, int stage, double t_next, const cplx<T>* Ys_in, cplx<T>* Ys_out,
              int remap, int slot0) {
  __shared__ cplx<T> lds[col_tile<N, W>() * col_buf(N)];
  int tile, slot, z;
  xcd_split(gridDim.x, gridDim.y, tile, slot, z, remap);
  columns_body<T, N, col_tile<N, W>()>(P, d, ph, stage, t_next, Ys_in, Ys_out, tile, slot0 + slot, lds);
}

// --------------------------------------------------------------------------
// batched entry points: blockIdx.z selects a run of one (N, precision) group
// --------------------------------------------------------------------------

template <typename T, int N>
__global__ void __launch_bounds__((DynGeo<T, N>::THREADS), (dyn_waves<T>())) k_rows_dyn_b(
    const RunDesc<T>* __restrict__ runs, int remap) {
  __shared__ cplx<T> lds[DynGeo<T, N>::LDS];
  int rowblock, unused, z;
  xcd_split(gridDim.x, 1, rowblock, unused, z, remap);
  if constexpr (DynGeo<T, N>::COOP) rows_dyn_coop<T, N>(runs[z].P, Dims::make(N), runs[z].ph, rowblock, lds);
  else rows_dyn_body<T, N>(runs[z].P, Dims::make(N), runs[z].ph, rowblock, lds);
}

template <typename T, int N, bool CUB>
__global__ void __launch_bounds__(64 * ROW_WAVES, (rhs_waves<T, N>())) k_rows_rhs_b(const RunDesc<T>* __restrict__ runs,
                                                                                int stage, int remap) {
  __shared__ cplx<T> lds[rhs_lds<T, N>()];  // transform buffers (and xi, two-task form)
  int rowblock, task, z;
  xcd_split(gridDim.x, gridDim.y, rowblock, task, z, remap);
  const RunDesc<T>& R = runs[z];
  // time since the interval start, from integers (as the single-run path)
  const double c = (stage == 0) ? 0.0 : ((stage == 3) ? 1.0 : 0.5);
  const double s = (double(*R.counter) + c) * R.ph.dt;
  rows_rhs_body<T, N, CUB>(R.P, Dims::make(N), s, rowblock, task, lds, R.ph.gen);
}

template <typename T, int N, bool CUB>
__global__ void __launch_bounds__(64 * ROW_WAVES) k_rows_mom_b(const RunDesc<T>* __restrict__ runs, int stage, int remap) {
  __shared__ cplx<T> lds[RowGeo<N>::RPB * RowGeo<N>::L];
  int rowblock, task, z;
  xcd_split(gridDim.x, gridDim.y, rowblock, task, z, remap);
  const RunDesc<T>& R = runs[z];
  const double c = (stage == 0) ? 0.0 : ((stage == 3) ? 1.0 : 0.5);
  const double s = (double(*R.counter) + c) * R.ph.dt;
  rows_mom_body<T, N, CUB>(R.P, Dims::make(N), s, rowblock, task, lds);
}

// stage parity selects the stage-value buffers: between steps the current
// stage input is always Ys0 (four swaps per step)
template <typename T, int N, int W>
__global__ void __launch_bounds__((col_threads<N, W>()), (col_waves<T, N, true>()))
    k_columns_b(const RunDesc<T>* __restrict__ runs, int stage, int remap) {
  __shared__ cplx<T> lds[col_tile<N, W>() * col_buf(N)];
  int tile, group, z;
  xcd_split(gridDim.x, gridDim.y, tile, group, z, remap);
  const RunDesc<T>& R = runs[z];
  const cplx<T>* Ys_in = (stage & 1) ? R.Ys1 : R.Ys0;
  cplx<T>* Ys_out = (stage & 1) ? R.Ys0 : R.Ys1;
  // time of the next stage input, from integers (as the single-run path)
  const double cn = (stage <= 1) ? 0.5 : 1.0;
  const double t_next = (double(R.n_tau + *R.counter) + cn) * R.ph.dt;
  columns_body<T, N, col_tile<N, W>()>(R.P, Dims::make(N), R.ph, stage, t_next, Ys_in, Ys_out, tile, group, lds);
}

}  // namespace lm
