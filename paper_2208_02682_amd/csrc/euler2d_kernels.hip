// Two-dimensional incompressible inviscid flow (section 4.1, the test of
// eq. (4.2)) with strategy 1 pseudospectral (eqs. (4.1), (3.9)) and
// semi-Lagrangian (appendix B).  float64.  The 2-D transforms are the
// boundary transforms of io_kernels.hpp; the kernels here are the spectral
// multipliers, the physical products, Heun's stages and the semi-Lagrangian
// update.  Spectral fields use the truncated state layout [kx][ky + K]
// (normalised by 1/N^2), physical fields are N x N row-major.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace lm {

namespace {

__device__ __forceinline__ cplx<double> ik(double k, cplx<double> a) { return {-k * a.y, k * a.x}; }

// floor(o) taken periodically into [0, N): a finite displacement of any size
// wraps around the torus; beyond 2^30 cells, or NaN, cell 0 (non-finite
// weights then reach the outputs)
__device__ __forceinline__ int cell_mod(double f, int N) {
  const int i = (fabs(f) < 1073741824.0) ? int(f) : 0;
  const int r = i % N;
  return r < 0 ? r + N : r;
}

// periodic bilinear interpolant of F at grid point (jx, jy) + (xi_x, xi_y)
// (cells and weights from the small offset xi / dx)
__device__ double bilinear_at(const double* __restrict__ F, int N, int jx, int jy, double xi_x, double xi_y,
                              double dx) {
  const double ox = xi_x / dx, oy = xi_y / dx;
  const double fx = floor(ox), fy = floor(oy);
  const double ax = ox - fx, ay = oy - fy;
  int ix0 = jx + cell_mod(fx, N), iy0 = jy + cell_mod(fy, N);  // in [0, 2N)
  ix0 = ix0 >= N ? ix0 - N : ix0;
  iy0 = iy0 >= N ? iy0 - N : iy0;
  const int ix1 = ix0 + 1 == N ? 0 : ix0 + 1, iy1 = iy0 + 1 == N ? 0 : iy0 + 1;
  return (1.0 - ax) * (1.0 - ay) * F[iy0 * N + ix0] + ax * (1.0 - ay) * F[iy0 * N + ix1] +
         (1.0 - ax) * ay * F[iy1 * N + ix0] + ax * ay * F[iy1 * N + ix1];
}

// periodic tensor-product cubic (4-point Lagrange) interpolant, same conventions
__device__ double cubic_at(const double* __restrict__ F, int N, int jx, int jy, double xi_x, double xi_y,
                           double dx) {
  const double ox = xi_x / dx, oy = xi_y / dx;
  const double fx = floor(ox), fy = floor(oy);
  const double ax = ox - fx, ay = oy - fy;
  const double wx[4] = {-ax * (ax - 1.0) * (ax - 2.0) / 6.0, (ax + 1.0) * (ax - 1.0) * (ax - 2.0) / 2.0,
                        -(ax + 1.0) * ax * (ax - 2.0) / 2.0, (ax + 1.0) * ax * (ax - 1.0) / 6.0};
  const double wy[4] = {-ay * (ay - 1.0) * (ay - 2.0) / 6.0, (ay + 1.0) * (ay - 1.0) * (ay - 2.0) / 2.0,
                        -(ay + 1.0) * ay * (ay - 2.0) / 2.0, (ay + 1.0) * ay * (ay - 1.0) / 6.0};
  int bx = jx + cell_mod(fx, N), by = jy + cell_mod(fy, N);  // in [0, 2N)
  bx = bx >= N ? bx - N : bx;
  by = by >= N ? by - N : by;
  double out = 0.0;
  for (int j = 0; j < 4; ++j) {
    int r = by + j - 1;
    r = r < 0 ? r + N : (r >= N ? r - N : r);
    double row = 0.0;
    for (int i = 0; i < 4; ++i) {
      int c = bx + i - 1;
      c = c < 0 ? c + N : (c >= N ? c - N : c);
      row += wx[i] * F[r * N + c];
    }
    out += wy[j] * row;
  }
  return out;
}

}  // namespace

// spectral inputs of the stage: u, v (from psi = -zeta / |k|^2: u = -dpsi/dy,
// v = dpsi/dx), zeta_x, zeta_y, zeta, and the gradients of g~, P_x, P_y
__global__ void __launch_bounds__(256) k_e2d_spec(Dims d, const cplx<double>* __restrict__ Y,
                                                  cplx<double>* __restrict__ S) {
  const size_t sp = d.spec_elems();
  const size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (j >= sp) return;
  const double kx = double(j / d.NKY), ky = double(int(j % d.NKY) - d.K);
  const double k2 = kx * kx + ky * ky;
  const cplx<double> z = Y[j], g = Y[sp + j], px = Y[2 * sp + j], py = Y[3 * sp + j];
  const double inv = k2 > 0.0 ? 1.0 / k2 : 0.0;
  const cplx<double> psi = {-z.x * inv, -z.y * inv};
  const cplx<double> dpy = ik(ky, psi);
  S[j] = {-dpy.x, -dpy.y};
  S[sp + j] = ik(kx, psi);
  S[2 * sp + j] = ik(kx, z);
  S[3 * sp + j] = ik(ky, z);
  S[4 * sp + j] = z;
  S[5 * sp + j] = ik(kx, g);
  S[6 * sp + j] = ik(ky, g);
  S[7 * sp + j] = ik(kx, px);
  S[8 * sp + j] = ik(ky, px);
  S[9 * sp + j] = ik(kx, py);
  S[10 * sp + j] = ik(ky, py);
}

// products of the stage (physical): -(u.grad zeta) is formed as u zeta_x + v zeta_y
// (the sign goes into the stage update); zeta - u.grad g~; s u - u.grad P_x; s v - u.grad P_y
__global__ void __launch_bounds__(256) k_e2d_products(int nn, const double* __restrict__ PH,
                                                      double* __restrict__ NL, double s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const double u = PH[i], v = PH[nn + i];
  NL[i] = u * PH[2 * nn + i] + v * PH[3 * nn + i];
  NL[nn + i] = PH[4 * nn + i] - (u * PH[5 * nn + i] + v * PH[6 * nn + i]);
  NL[2 * nn + i] = s * u - (u * PH[7 * nn + i] + v * PH[8 * nn + i]);
  NL[3 * nn + i] = s * v - (u * PH[9 * nn + i] + v * PH[10 * nn + i]);
}

// Heun: stage 0: K1 = R, Y1 = Y + dt K1; stage 1: Y = Y + dt/2 (K1 + R)
// (R of the vorticity is the transform of u.grad zeta with the sign flipped here)
__global__ void __launch_bounds__(256) k_e2d_stage(size_t sp, cplx<double>* __restrict__ Y,
                                                   cplx<double>* __restrict__ Y1, cplx<double>* __restrict__ K1,
                                                   const cplx<double>* __restrict__ R, double dt, int stage) {
  const size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (j >= 4 * sp) return;
  const double sg = j < sp ? -1.0 : 1.0;
  const cplx<double> r = {sg * R[j].x, sg * R[j].y};
  if (stage == 0) {
    K1[j] = r;
    Y1[j] = {Y[j].x + dt * r.x, Y[j].y + dt * r.y};
  } else {
    const cplx<double> k = K1[j];
    Y[j] = {Y[j].x + 0.5 * dt * (k.x + r.x), Y[j].y + 0.5 * dt * (k.y + r.y)};
  }
}

// semi-Lagrangian strategy 1 (appendix B, eqs. (B.2), (B.4), (B.5)) after a
// step: departure point Y = X - d, d = dt u(X, t_{n+1}); with m = (t_n - tau)/dt
//   f~_{n+1}(X) = [m f~_n(Y) + (zeta_n(Y) + zeta_{n+1}(X)) / 2] / (m + 1)
//   eta_{n+1}(X) = [m eta_n(Y) + (m + 1/2) d] / (m + 1)
__global__ void __launch_bounds__(256) k_e2d_sl(int N, const double* __restrict__ u, const double* __restrict__ v,
                                                const double* __restrict__ znext, const double* __restrict__ znow,
                                                const double* __restrict__ f_old, const double* __restrict__ ex_old,
                                                const double* __restrict__ ey_old, double* __restrict__ f_new,
                                                double* __restrict__ ex_new, double* __restrict__ ey_new,
                                                double* __restrict__ z_new, double dt, double m, int cubic) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * N) return;
  const int jx = i % N, jy = i / N;
  const double dx = 6.283185307179586476925286766559 / N;
  const double d_x = dt * u[i], d_y = dt * v[i];
  double fY, zY, exY, eyY;
  if (cubic) {
    fY = cubic_at(f_old, N, jx, jy, -d_x, -d_y, dx);
    zY = cubic_at(znow, N, jx, jy, -d_x, -d_y, dx);
    exY = cubic_at(ex_old, N, jx, jy, -d_x, -d_y, dx);
    eyY = cubic_at(ey_old, N, jx, jy, -d_x, -d_y, dx);
  } else {
    fY = bilinear_at(f_old, N, jx, jy, -d_x, -d_y, dx);
    zY = bilinear_at(znow, N, jx, jy, -d_x, -d_y, dx);
    exY = bilinear_at(ex_old, N, jx, jy, -d_x, -d_y, dx);
    eyY = bilinear_at(ey_old, N, jx, jy, -d_x, -d_y, dx);
  }
  const double zn = znext[i];
  f_new[i] = (m * fY + 0.5 * (zY + zn)) / (m + 1.0);
  ex_new[i] = (m * exY + (m + 0.5) * d_x) / (m + 1.0);
  ey_new[i] = (m * eyY + (m + 0.5) * d_y) / (m + 1.0);
  z_new[i] = zn;
}

void launch_e2d_spec(hipStream_t st, const Dims& d, const cplx<double>* Y, cplx<double>* S) {
  const size_t sp = d.spec_elems();
  hipLaunchKernelGGL(k_e2d_spec, dim3((sp + 255) / 256), dim3(256), 0, st, d, Y, S);
}
void launch_e2d_products(hipStream_t st, int nn, const double* PH, double* NL, double s) {
  hipLaunchKernelGGL(k_e2d_products, dim3((nn + 255) / 256), dim3(256), 0, st, nn, PH, NL, s);
}
void launch_e2d_stage(hipStream_t st, size_t sp, cplx<double>* Y, cplx<double>* Y1, cplx<double>* K1,
                      const cplx<double>* R, double dt, int stage) {
  hipLaunchKernelGGL(k_e2d_stage, dim3((4 * sp + 255) / 256), dim3(256), 0, st, sp, Y, Y1, K1, R, dt, stage);
}
void launch_e2d_sl(hipStream_t st, int N, const double* u, const double* v, const double* znext, const double* znow,
                   const double* f_old, const double* ex_old, const double* ey_old, double* f_new, double* ex_new,
                   double* ey_new, double* z_new, double dt, double m, bool cubic) {
  hipLaunchKernelGGL(k_e2d_sl, dim3((N * N + 255) / 256), dim3(256), 0, st, N, u, v, znext, znow, f_old, ex_old,
                     ey_old, f_new, ex_new, ey_new, z_new, dt, m, cubic ? 1 : 0);
}

}  // namespace lm
