// soma_sq.hpp -- structure factor of the composition field (Sec. 5.6):
// S(q) = N^2 rho0 / (4 V) |F[phi_A - phi_B](q)|^2 with F the Fourier
// transform on the grid, F = dL^3 sum_c psi(c) exp(-i q.r_c), on the
// reciprocal lattice q = 2 pi (mx/Lx, my/Ly, mz/Lz).  With
// phi_t(c) = n_t(c)/(rho0 dL^3) this is S(q) = N^2 |G(q)|^2 / (4 n_beads),
// G the discrete transform of the count difference n_A - n_B.
//
// The 3-D transform is done as three 1-D transforms (x, then y, then z), each
// a direct sum in FP64 with the phase k*x reduced modulo n in integers, so
// every twiddle is exact to one rounding.  This is infrequent analysis work:
// n_cells * (nx + ny + nz) complex multiply-adds.
#pragma once

#include "soma_device.hpp"

namespace soma {

struct SqArgs {
  const void *counts;
  int count64;
  uint32_t nx, ny, nz;
  double2 *a, *b;             // work planes, n_cells complex each
  const double2 *tw[3];       // twiddles exp(-2 pi i k / n) per axis, k < n
};

// tw[k] = exp(-2 pi i k / n) for k < n.
__global__ __launch_bounds__(256) void sq_twiddle_kernel(double2 *tw, uint32_t n) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)n, &s, &c);
  tw[k] = make_double2(c, -s);
}

__device__ __forceinline__ double count_diff(const void *counts, int count64, uint64_t c) {
  if (count64) {
    const unsigned long long w = reinterpret_cast<const unsigned long long *>(counts)[c];
    return (double)(uint32_t)w - (double)(uint32_t)(w >> 32);
  }
  const uint32_t w = reinterpret_cast<const uint32_t *>(counts)[c];
  return (double)(w & 0xFFFFu) - (double)(w >> 16);
}

// Stage 1: a[z][y][k] = sum_x psi(z,y,x) e^{-2 pi i k x / nx}, psi = n_A - n_B.
__global__ __launch_bounds__(256) void sq_dft_x_kernel(const SqArgs a) {
  const uint64_t n = (uint64_t)a.nx * a.ny * a.nz;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = (uint32_t)(i % a.nx);
  const uint64_t row = i - k;
  const double2 *tw = a.tw[0];
  double re = 0.0, im = 0.0;
  uint32_t ph = 0;  // k * x mod nx, advanced by k per step
  for (uint32_t x = 0; x < a.nx; ++x) {
    const double psi = count_diff(a.counts, a.count64, row + x);
    const double2 t = tw[ph];
    re = fma(psi, t.x, re);
    im = fma(psi, t.y, im);
    ph += k;
    if (ph >= a.nx) ph -= a.nx;
  }
  a.a[i] = make_double2(re, im);
}

// Stages 2 and 3: the transform along y (axis 1, stride nx) or z (axis 2,
// stride nx*ny) of `in` into `out`.
__global__ __launch_bounds__(256) void sq_dft_axis_kernel(const double2 *in, double2 *out,
                                                          const double2 *tw, uint32_t nx,
                                                          uint32_t ny, uint32_t nz, int axis) {
  const uint64_t n = (uint64_t)nx * ny * nz;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t y = (uint32_t)((i / nx) % ny);
  const uint32_t z = (uint32_t)(i / ((uint64_t)nx * ny));
  const uint32_t len = axis == 1 ? ny : nz;
  const uint32_t k = axis == 1 ? y : z;
  const uint64_t stride = axis == 1 ? (uint64_t)nx : (uint64_t)nx * ny;
  const uint64_t base = i - (uint64_t)k * stride;
  double re = 0.0, im = 0.0;
  uint32_t ph = 0;
  for (uint32_t j = 0; j < len; ++j) {
    const double2 v = in[base + (uint64_t)j * stride];
    const double2 t = tw[ph];
    re = fma(v.x, t.x, fma(-v.y, t.y, re));
    im = fma(v.x, t.y, fma(v.y, t.x, im));
    ph += k;
    if (ph >= len) ph -= len;
  }
  out[i] = make_double2(re, im);
}

// S(q) = scale |G(q)|^2.
__global__ __launch_bounds__(256) void sq_power_kernel(const double2 *g, double *sq, uint64_t n,
                                                       double scale) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 v = g[i];
  sq[i] = scale * (v.x * v.x + v.y * v.y);
}

}  // namespace soma
