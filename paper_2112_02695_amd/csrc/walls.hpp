// Maxwell diffusive walls (Sec. 2.3) for the one-dimensional space of the
// low-rank and full-tensor steps: the boundary function on the incoming half
// is rho_w M_w, with rho_w set by zero net mass flux through the wall,
//   rho_w = int_{v.n >= 0} (v.n) f dv / int_{v.n < 0} |v.n| M_w dv,
// n the outward normal (-e1 at x_lo = side 0, +e1 at x_hi = side 1) and f the
// distribution leaving the domain.  The midpoint-rule weight dv^d cancels.
#pragma once

#include <hip/hip_runtime.h>

namespace blr {
namespace wall {

// (v.n) on the outgoing half of side `side`, 0 elsewhere (v.n = 0 carries no flux)
__device__ __forceinline__ double out_weight(int side, double v1) {
  return side == 0 ? (v1 <= 0.0 ? -v1 : 0.0) : (v1 >= 0.0 ? v1 : 0.0);
}
// |v.n| on the incoming half (v_1 > 0 at x_lo, v_1 < 0 at x_hi), 0 elsewhere
__device__ __forceinline__ double in_weight(int side, double v1) {
  return side == 0 ? (v1 > 0.0 ? v1 : 0.0) : (v1 < 0.0 ? -v1 : 0.0);
}
__device__ __forceinline__ bool incoming(int side, double v1) {
  return side == 0 ? v1 > 0.0 : v1 < 0.0;
}

// rho_w from the outgoing half of `fadj` (n values) and the wall Maxwellian
// shape M, for a face whose outward normal is sgn e_axis, with v_axis of point
// q = -L + ((q / stride) % N) dv; summed by one block of NT threads in a fixed
// order (strided per-thread sums, wave sums, then the waves in order); every
// thread returns the value.  `red` holds NT / 64 + 1 doubles of shared
// memory.  Ends with a barrier.
template <int NT>
__device__ double density_face(double sgn, const double* __restrict__ fadj,
                               const double* __restrict__ M, int n, double L, double dv,
                               int stride, int N, double* red) {
  constexpr int NW = NT / 64;
  double num = 0.0, den = 0.0;
  for (int q = threadIdx.x; q < n; q += NT) {
    const double vn = sgn * (-L + ((q / stride) % N) * dv);
    if (vn >= 0.0)
      num += vn * fadj[q];
    else
      den -= vn * M[q];
  }
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_down(num, off, 64);
    den += __shfl_down(den, off, 64);
  }
  __shared__ double dred[NW];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = num;
    dred[threadIdx.x >> 6] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < NW; ++w) {
      a += red[w];
      b += dred[w];
    }
    red[NW] = a / b;
  }
  __syncthreads();
  return red[NW];
}

// The x faces of the one-dimensional space: side 0 = x_lo, 1 = x_hi, v_1 of
// point q = -L + (q / plane) dv.
template <int NT>
__device__ double density(int side, const double* __restrict__ fadj,
                          const double* __restrict__ M, int n, double L, double dv, int plane,
                          double* red) {
  return density_face<NT>(side == 0 ? -1.0 : 1.0, fadj, M, n, L, dv, plane, n / plane, red);
}

}  // namespace wall
}  // namespace blr
