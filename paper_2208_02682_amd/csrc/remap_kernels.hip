// Strategy 1 remapped to Lagrangian-mean positions (section 3.1, eq. (3.8)).
//
// For every grid point y, taken as a mean position, the end-of-interval
// position x of its particle solves x - eta(x) = y (eta = x - Xi^{-1}(x) from
// strategy 1, bilinear between grid values); then f-bar^L(y) = f~^L(x) and
// d(y) = x - y.  The equation is solved cell by cell: on the end-position cell
// (ix, iy)..(ix+1, iy+1) the map x -> x - eta(x) is the bilinear patch through
// the four corner mean positions, and every grid point the patch covers is
// located by inverting the patch (closed form, then two Newton steps).  Where
// the mean map folds, the patch of the lowest cell index (iy N + ix) wins, so
// the result does not depend on the order of the threads:
//   pass 1 (claim): every cell takes atomicMin(best[y], cell) for the points it covers;
//   pass 2 (write): the winning cell writes f-bar_h, f-bar_zeta, d_x, d_y and the residual;
//   pass 3: points no patch covers (only through a patch spanning more than
//           max_extent cells, which is skipped) get NaN and an infinite residual.
// float64 throughout, one thread per cell or point.  Grid units inside.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace lm {

namespace {

constexpr double EPS = 1e-12;  // inside-test tolerance in the patch coordinates

struct Patch {
  double ax, ay, bx, by, cx, cy, dx, dy;  // p(s, t) = a + b s + c t + d s t
  int ilo_x, ihi_x, ilo_y, ihi_y;         // grid points in the bounding box
  bool usable;
};

__device__ __forceinline__ int wrapi(long long v, int N) {
  long long r = v % N;
  return int(r < 0 ? r + N : r);
}

__device__ Patch make_patch(int N, int ix, int iy, const double* __restrict__ ex, const double* __restrict__ ey,
                            double h, int max_extent) {
  const int ix1 = ix + 1 == N ? 0 : ix + 1, iy1 = iy + 1 == N ? 0 : iy + 1;
  // corner mean positions (grid units, unwrapped around this cell)
  const double x00 = ix - ex[iy * N + ix] / h, y00 = iy - ey[iy * N + ix] / h;
  const double x10 = (ix + 1) - ex[iy * N + ix1] / h, y10 = iy - ey[iy * N + ix1] / h;
  const double x01 = ix - ex[iy1 * N + ix] / h, y01 = (iy + 1) - ey[iy1 * N + ix] / h;
  const double x11 = (ix + 1) - ex[iy1 * N + ix1] / h, y11 = (iy + 1) - ey[iy1 * N + ix1] / h;
  Patch p;
  p.ax = x00;
  p.ay = y00;
  p.bx = x10 - x00;
  p.by = y10 - y00;
  p.cx = x01 - x00;
  p.cy = y01 - y00;
  p.dx = x11 - x10 - x01 + x00;
  p.dy = y11 - y10 - y01 + y00;
  const bool fin = isfinite(x00) && isfinite(y00) && isfinite(x10) && isfinite(y10) && isfinite(x01) &&
                   isfinite(y01) && isfinite(x11) && isfinite(y11);
  const double lox = ceil(fmin(fmin(x00, x10), fmin(x01, x11)) - EPS);
  const double hix = floor(fmax(fmax(x00, x10), fmax(x01, x11)) + EPS);
  const double loy = ceil(fmin(fmin(y00, y10), fmin(y01, y11)) - EPS);
  const double hiy = floor(fmax(fmax(y00, y10), fmax(y01, y11)) + EPS);
  // the magnitude bound keeps the integer loop bounds in range (only a run that
  // blew up has mean positions millions of cells away)
  p.usable = fin && hix - lox <= max_extent && hiy - loy <= max_extent && fabs(lox) < 1e7 && fabs(hix) < 1e7 &&
             fabs(loy) < 1e7 && fabs(hiy) < 1e7;
  p.ilo_x = p.usable ? int(lox) : 0;
  p.ihi_x = p.usable ? int(hix) : -1;
  p.ilo_y = p.usable ? int(loy) : 0;
  p.ihi_y = p.usable ? int(hiy) : -1;
  return p;
}

__device__ __forceinline__ double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

// patch coordinates (s, t) of the point (Yx, Yy); false if there is none
__device__ bool invert_patch(const Patch& p, double Yx, double Yy, double& s, double& t) {
  const double qx = Yx - p.ax, qy = Yy - p.ay;
  const double A = cross2(p.bx, p.by, p.dx, p.dy);
  const double B = cross2(p.bx, p.by, p.cx, p.cy) - cross2(qx, qy, p.dx, p.dy);
  const double C = -cross2(qx, qy, p.cx, p.cy);
  const bool lin = fabs(A) <= 1e-14 * (fabs(B) + 1e-300);
  const double disc = B * B - 4.0 * A * C;
  const double sq = sqrt(fmax(disc, 0.0));
  const double qq = -0.5 * (B + copysign(sq, B));
  const double r1 = lin ? -C / B : qq / A;
  const double r2 = lin ? -C / B : C / qq;
  auto t_of = [&](double r) {
    const double wx = p.cx + p.dx * r, wy = p.cy + p.dy * r;
    return ((qx - p.bx * r) * wx + (qy - p.by * r) * wy) / (wx * wx + wy * wy);
  };
  const double t1 = t_of(r1), t2 = t_of(r2);
  auto dist = [](double a, double b) { return fmax(fmax(-a, a - 1.0), fmax(-b, b - 1.0)); };
  const bool pick1 = !(dist(r2, t2) < dist(r1, t1));
  s = pick1 ? r1 : r2;
  t = pick1 ? t1 : t2;
  for (int k = 0; k < 2; ++k) {
    const double rx = p.ax + p.bx * s + p.cx * t + p.dx * s * t - Yx;
    const double ry = p.ay + p.by * s + p.cy * t + p.dy * s * t - Yy;
    const double j11 = p.bx + p.dx * t, j12 = p.cx + p.dx * s;
    const double j21 = p.by + p.dy * t, j22 = p.cy + p.dy * s;
    const double det = j11 * j22 - j12 * j21;
    s = s - (j22 * rx - j12 * ry) / det;
    t = t - (-j21 * rx + j11 * ry) / det;
  }
  return isfinite(s) && isfinite(t) && (lin || disc >= 0.0) && s >= -EPS && s <= 1.0 + EPS && t >= -EPS &&
         t <= 1.0 + EPS;
}

}  // namespace

__global__ void __launch_bounds__(256) k_remap_fill(unsigned* __restrict__ best, int nn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) best[i] = 0xffffffffu;
}

__global__ void __launch_bounds__(256) k_remap_claim(int N, const double* __restrict__ ex,
                                                     const double* __restrict__ ey, unsigned* __restrict__ best,
                                                     int max_extent) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N * N) return;
  const int ix = cell % N, iy = cell / N;
  const double h = 6.283185307179586476925286766559 / N;
  const Patch p = make_patch(N, ix, iy, ex, ey, h, max_extent);
  for (int Y = p.ilo_y; Y <= p.ihi_y; ++Y)
    for (int X = p.ilo_x; X <= p.ihi_x; ++X) {
      double s, t;
      if (invert_patch(p, double(X), double(Y), s, t)) atomicMin(&best[wrapi(Y, N) * N + wrapi(X, N)], unsigned(cell));
    }
}

// out: [f-bar_h, f-bar_zeta, d_x, d_y] planes; resid_bits: atomic max of the
// residual |p(s, t) - y| (grid units; non-negative doubles order like their bits)
__global__ void __launch_bounds__(256) k_remap_write(int N, const double* __restrict__ ex,
                                                     const double* __restrict__ ey, const double* __restrict__ fh,
                                                     const double* __restrict__ fz,
                                                     const unsigned* __restrict__ best, double* __restrict__ out,
                                                     int max_extent, unsigned long long* resid_bits) {
  const int nn = N * N;
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  double worst = 0.0;
  if (cell < nn) {
    const int ix = cell % N, iy = cell / N;
    const int ix1 = ix + 1 == N ? 0 : ix + 1, iy1 = iy + 1 == N ? 0 : iy + 1;
    const double h = 6.283185307179586476925286766559 / N;
    const Patch p = make_patch(N, ix, iy, ex, ey, h, max_extent);
    const int c00 = iy * N + ix, c10 = iy * N + ix1, c01 = iy1 * N + ix, c11 = iy1 * N + ix1;
    for (int Y = p.ilo_y; Y <= p.ihi_y; ++Y)
      for (int X = p.ilo_x; X <= p.ihi_x; ++X) {
        double s, t;
        if (!invert_patch(p, double(X), double(Y), s, t)) continue;
        const int tgt = wrapi(Y, N) * N + wrapi(X, N);
        if (best[tgt] != unsigned(cell)) continue;
        const double w0 = (1.0 - s) * (1.0 - t), w1 = s * (1.0 - t), w2 = (1.0 - s) * t, w3 = s * t;
        out[tgt] = w0 * fh[c00] + w1 * fh[c10] + w2 * fh[c01] + w3 * fh[c11];
        out[nn + tgt] = w0 * fz[c00] + w1 * fz[c10] + w2 * fz[c01] + w3 * fz[c11];
        out[2 * nn + tgt] = (ix + s - X) * h;
        out[3 * nn + tgt] = (iy + t - Y) * h;
        const double px = p.ax + p.bx * s + p.cx * t + p.dx * s * t;
        const double py = p.ay + p.by * s + p.cy * t + p.dy * s * t;
        worst = fmax(worst, fmax(fabs(px - X), fabs(py - Y)));
      }
  }
  unsigned long long bits = __double_as_longlong(worst);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(bits, o, 64);
    bits = other > bits ? other : bits;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(resid_bits, bits);
}

__global__ void __launch_bounds__(256) k_remap_uncovered(const unsigned* __restrict__ best, double* __restrict__ out,
                                                         int nn, unsigned long long* resid_bits) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool miss = i < nn && best[i] == 0xffffffffu;
  if (miss) {
    const double nan = __builtin_nan("");
    out[i] = out[nn + i] = out[2 * nn + i] = out[3 * nn + i] = nan;
  }
  if (__any(miss) && (threadIdx.x & 63) == 0) atomicMax(resid_bits, 0x7ff0000000000000ull);  // +inf
}

void launch_remap_s1(RunView& r, const double* fh, const double* fz, const double* ex, const double* ey,
                     double* out, unsigned* best, int max_extent, unsigned long long* resid_bits) {
  const int N = r.d.N, nn = N * N;
  const dim3 g((nn + 255) / 256), b(256);
  hipLaunchKernelGGL(k_remap_fill, g, b, 0, r.stream, best, nn);
  hipLaunchKernelGGL(k_remap_claim, g, b, 0, r.stream, N, ex, ey, best, max_extent);
  hipLaunchKernelGGL(k_remap_write, g, b, 0, r.stream, N, ex, ey, fh, fz, best, out, max_extent, resid_bits);
  hipLaunchKernelGGL(k_remap_uncovered, g, b, 0, r.stream, best, out, nn, resid_bits);
}

}  // namespace lm
