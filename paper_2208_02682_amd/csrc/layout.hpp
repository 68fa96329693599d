// Device data layout of one run (one doubly periodic N x N problem).
//
// Spectral state: only the 2/3-rule square |kx|, |ky| <= K, K = floor((N-1)/3),
// is ever non-zero, so each field stores NKX = K+1 columns (kx = 0..K) of
// NKY = 2K+1 entries (ky = -K..K, index ky + K), column-contiguous, complex.
// Coefficients are normalised by 1/N^2 (physical value = plain inverse sum).
//
// Column-pass outputs ("intermediates") and row-pass outputs ("row spectra")
// are [field][y][kx] with y = 0..N-1 and kx = 0..K (row stride NKXP >= NKX,
// padded to 16 complex so row segments are 128-byte aligned).
//
// Physical dynamics fields u, v, h, zeta are stored interleaved per grid point
// (one 4-vector) so that a bilinear gather corner is a single load.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lm {

// prognostic fields, in the order of the per-precision state arrays
enum StateField : int {
  // working precision; the h accumulators (GBH, GTH, EH) integrate eta = h - H
  SF_U = 0, SF_V, SF_H, SF_GBH, SF_GBZ, SF_GTH, SF_GTZ, SF_EH, SF_EZ,
  SF_GMX, SF_GMY,  // strategy-2 g of the momentum 1-form (appendix C; used when requested)
  NSF_R = 11
};
enum StateFieldD : int {
  SD_XIX = 0, SD_XIY, SD_PX, SD_PY,  // always float64 (displacement / position accumulators)
  NSF_D = 4
};

// intermediates: inverse column transforms of the stage state
enum Inter : int {
  IC_U = 0, IC_V, IC_H, IC_UY,                  // u, v, eta = h - H and (i ky u)
  IC_XIX, IC_XIX_Y, IC_XIY, IC_XIY_Y,           // xi components and their (i ky) versions
  IC_GBH, IC_GBH_Y, IC_GBZ, IC_GBZ_Y,           // strategy-2 g
  IC_GTH, IC_GTH_Y, IC_GTZ, IC_GTZ_Y,           // strategy-1 g
  IC_PX, IC_PX_Y, IC_PY, IC_PY_Y,               // strategy-1 position accumulator P
  IC_GMX, IC_GMX_Y, IC_GMY, IC_GMY_Y,           // strategy-2 g of the momentum 1-form
  NIC = 24
};

// row spectra: forward row transforms of the physical right-hand-side terms
enum RowSpec : int {
  RS_ZV = 0, RS_ZU, RS_K, RS_HU, RS_HV,         // zeta v, zeta u, (u^2+v^2)/2, eta u, eta v
  RS_XIX, RS_XIY, RS_GBH, RS_GBZ, RS_GTH, RS_GTZ, RS_PX, RS_PY,
  RS_GMX, RS_GMY,
  RS_F0, RS_F1,      // the two averaged fields themselves (Eulerian means of other fields than h, zeta)
  NRS = 17
};

// column-kernel work groups (one prognostic field each; E_h, E_zeta ride with h)
// (the momentum groups come next and are launched only when requested, then the
// Eulerian-mean groups of averaged fields other than (h, zeta))
enum ColGroup : int {
  CG_U = 0, CG_V, CG_H, CG_XIX, CG_XIY, CG_GBH, CG_GBZ, CG_GTH, CG_GTZ, CG_PX, CG_PY,
  NCG = 11,
  CG_GMX = 11, CG_GMY, NCG_MOM = 13,
  CG_EF0 = 13, CG_EF1
};

// the fields the two averaging slots can hold (f_0, f_1; the default is (eta, zeta))
enum FieldSel : int { FS_ETA = 0, FS_ZETA, FS_U, FS_V, FS_Q /* (f + zeta) / h */ };

// row-kernel tasks of the right-hand-side pass.  Two-task form (float, N >=
// 512): strategy 2 (xi and g-bar), and strategy 1 with the Lagrangian-mean
// velocity (g-tilde and P).  Four-task form: xi, g-bar, g-tilde, P.  The
// momentum rows, when requested, are a kernel of their own with one task per
// component.
enum RowTask : int { RT_S2 = 0, RT_S1 };
enum RowTask4 : int { RT4_XI = 0, RT4_GB, RT4_GT, RT4_P };
template <typename T, int N>
__host__ __device__ constexpr bool rhs_merged() {
  return sizeof(T) == 4 && N >= 512;
}
template <typename T, int N>
__host__ __device__ constexpr int rhs_tasks() {
  return rhs_merged<T, N>() ? 2 : 4;
}

// 2/3-rule cutoff: modes |kx|, |ky| <= K are kept (a compile-time constant of N)
template <int N>
__host__ __device__ constexpr int kcut() { return (N - 1) / 3; }

struct Dims {
  int N, K, NKX, NKY, NKXP;
  __host__ __device__ static Dims make(int N) {
    Dims d;
    d.N = N;
    d.K = (N - 1) / 3;
    d.NKX = d.K + 1;
    d.NKY = 2 * d.K + 1;
    d.NKXP = (d.NKX + 15) / 16 * 16;
    return d;
  }
  __host__ __device__ size_t spec_elems() const { return (size_t)NKX * NKY; }
  __host__ __device__ size_t rowfield_elems() const { return (size_t)N * NKXP; }
};

// physics constants of one run, and what its launches compute
struct Phys {
  double f, g, H, dt, nu8;
  int fs0, fs1;  // FieldSel of averaging slots 0 and 1
  int gen;       // Eulerian means from transforms of the averaged fields (any pair but (eta, zeta))
  int mom;       // the momentum 1-form groups are launched
  int kin;       // u, v, h prescribed: a linear plane wave plus a uniform flow (no dynamics)
  double kx, ky, A, omega, phase, U0, V0;  // kinematic: h' = A cos(kx x + ky y - omega t + phase)
};

// Column groups launched for a run, in slot order: first the groups that need
// only the dynamics rows pass (u, v, h, and the Eulerian groups of fields other
// than (h, zeta)), then those that need the mean right-hand-side rows pass (xi,
// g-bar, g-tilde, P, and the momentum 1-form).  A launch covers a range of slots.
__host__ __device__ inline int col_dyn_groups(const Phys& ph) { return 3 + (ph.gen ? 2 : 0); }
__host__ __device__ inline int col_mean_groups(const Phys& ph) { return 8 + (ph.mom ? 2 : 0); }
__host__ __device__ inline int col_groups(const Phys& ph) { return col_dyn_groups(ph) + col_mean_groups(ph); }
__host__ __device__ inline int col_group_of(const Phys& ph, int slot) {
  if (slot < 3) return CG_U + slot;
  const int nd = col_dyn_groups(ph);
  if (slot < nd) return CG_EF0 + (slot - 3);
  const int j = slot - nd;
  return (j < 8) ? CG_XIX + j : CG_GMX + (j - 8);
}

}  // namespace lm
