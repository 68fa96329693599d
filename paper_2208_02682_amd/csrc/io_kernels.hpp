// Float64 transforms used off the hot loop: physical <-> truncated spectral
// state for set_state / get_state, and the end-of-interval outputs (inverse
// transforms of the accumulators with the division by T in float64).
#pragma once

#include "io_structs.hpp"
#include "step_kernels.hpp"

namespace lm {

template <int N>
__global__ void __launch_bounds__(64 * ROW_WAVES) k_io_row_forward(IoRowFwd J, Dims d, const cplx<double>* tw) {
  using G = RowGeo<N>;
  constexpr int E = G::E, NT = G::NT;
  __shared__ cplx<double> lds[G::RPB * G::L];
  const int grp = row_group<NT>(), t = threadIdx.x % NT;
  const int y = blockIdx.x * G::RPB + grp;
  cplx<double>* buf = lds + grp * G::L;
  const int q = blockIdx.y;
  cplx<double> z[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const size_t i = (size_t)y * N + t + NT * e;
    z[e] = {J.a[q][i], J.b[q] ? J.b[q][i] : 0.0};
  }
  cplx<double>* OA = J.oa[q] + (size_t)y * d.NKXP;
  if (J.b[q]) {
    cplx<double>* OB = J.ob[q] + (size_t)y * d.NKXP;
    forward_row<double, N, true>(z, buf, t, tw, OA, OB);
  } else {
    forward_row<double, N, false>(z, buf, t, tw, OA, nullptr);
  }
}

template <int N>
__global__ void __launch_bounds__(64 * ROW_WAVES) k_io_row_inverse(IoRowInv J, Dims d, const cplx<double>* tw) {
  using G = RowGeo<N>;
  constexpr int E = G::E, NT = G::NT;
  __shared__ cplx<double> lds[G::RPB * G::L];
  const int grp = row_group<NT>(), t = threadIdx.x % NT;
  const int y = blockIdx.x * G::RPB + grp;
  cplx<double>* buf = lds + grp * G::L;
  const int q = blockIdx.y;
  const cplx<double>* A = J.a[q] + (size_t)y * d.NKXP;
  const cplx<double>* B = J.b[q] ? J.b[q] + (size_t)y * d.NKXP : A;
  cplx<double> z[E];
  load_pair<double, N, false, false>(z, A, B, t);
  inverse_row<double, N>(z, buf, t, tw);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const size_t i = (size_t)y * N + t + NT * e;
    J.oa[q][i] = z[e].x * J.sa[q] + J.ca[q];
    if (J.b[q]) J.ob[q][i] = z[e].y * J.sb[q] + J.cb[q];
  }
}

template <int N>
__global__ void __launch_bounds__(col_threads<N>())
    k_io_col_forward(IoColFwd J, Dims d, const cplx<double>* tw) {
  constexpr int C = col_tile<N>();
  constexpr int E = fft_E<N>(), NT = N / E, LC = col_buf(N);
  __shared__ cplx<double> lds[C * LC];
  ColCtx<double, N, C> cx;
  cx.lds = lds;
  cx.c = threadIdx.x / NT;
  cx.t = threadIdx.x % NT;
  cx.buf = lds + cx.c * LC;
  cx.kx0 = blockIdx.x * C;
  cx.kx = cx.kx0 + cx.c;
  cx.valid = cx.kx <= kcut<N>();
  const int q = blockIdx.y;
  cplx<double> out[E];
  column_forward<double, N, C>(cx, J.src[q], d, tw, out);
  if (!cx.valid) return;
  const size_t col = (size_t)cx.kx * d.NKY;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = cx.t + NT * r;
    int ky;
    if (k <= kcut<N>()) ky = k;
    else if (k >= N - kcut<N>()) ky = k - N;
    else continue;
    const size_t j = col + (size_t)(ky + d.K);
    cplx<double> v = out[r];
    if (cx.kx == 0 && ky == 0) v.y = 0.0;
    if (J.dst_f32[q]) {
      const cplx<float> hi = {float(v.x), float(v.y)};
      reinterpret_cast<cplx<float>*>(J.dst[q])[j] = hi;
      if (J.dst_lo[q])
        reinterpret_cast<cplx<float>*>(J.dst_lo[q])[j] = {float(v.x - double(hi.x)), float(v.y - double(hi.y))};
    } else {
      reinterpret_cast<cplx<double>*>(J.dst[q])[j] = v;
    }
  }
}

template <int N>
__global__ void __launch_bounds__(col_threads<N>())
    k_io_col_inverse(IoColInv J, Dims d, const cplx<double>* tw) {
  constexpr int C = col_tile<N>();
  constexpr int E = fft_E<N>(), NT = N / E, LC = col_buf(N);
  __shared__ cplx<double> lds[C * LC];
  ColCtx<double, N, C> cx;
  cx.lds = lds;
  cx.c = threadIdx.x / NT;
  cx.t = threadIdx.x % NT;
  cx.buf = lds + cx.c * LC;
  cx.kx0 = blockIdx.x * C;
  cx.kx = cx.kx0 + cx.c;
  cx.valid = cx.kx <= kcut<N>();
  const int q = blockIdx.y;
  const size_t col = (size_t)cx.kx * d.NKY;
  cplx<double> S[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = cx.t + NT * r;
    int ky;
    S[r] = {0.0, 0.0};
    if (k <= kcut<N>()) ky = k;
    else if (k >= N - kcut<N>()) ky = k - N;
    else continue;
    if (!cx.valid) continue;
    const size_t j = col + (size_t)(ky + d.K);
    if (J.src_f32[q]) {
      const cplx<float> s = reinterpret_cast<const cplx<float>*>(J.src[q])[j];
      S[r] = {double(s.x), double(s.y)};
      if (J.src_lo[q]) {
        const cplx<float> l = reinterpret_cast<const cplx<float>*>(J.src_lo[q])[j];
        S[r] = {S[r].x + double(l.x), S[r].y + double(l.y)};
      }
    } else {
      S[r] = reinterpret_cast<const cplx<double>*>(J.src[q])[j];
    }
  }
  column_inverse<double, N, C, double, false>(cx, S, J.dst[q], d, tw);
}

}  // namespace lm
