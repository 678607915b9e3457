// In-register complex DFTs of compile-time length for gfx950.
//
// dft<T, N, DIR>(re, im) transforms N complex values held in registers:
//   X_k = sum_n x_n exp(DIR * 2 pi i n k / N),   DIR = -1 forward, +1 inverse
// (no normalisation).  N is split as N1 * N2 with N1 in {4, 2, 3} (Cooley-Tukey
// with the twiddles W_N^{n2 k1} between the two stages) until the radix-2/3/4
// butterflies; every index and twiddle is a compile-time constant after
// unrolling, so the whole transform is straight-line FMA code.  Twiddles are
// evaluated at compile time from a Taylor series of sin/cos at the exact
// rational angles 2 pi m / N (|error| < 1e-16).
#pragma once

#include <hip/hip_runtime.h>

namespace blr {
namespace fft {

constexpr double kPi = 3.14159265358979323846264338327950288;

// sin and cos of x for |x| <= pi, from their Taylor series.
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 40; ++k) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 40; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
// angle 2 pi m / N reduced to (-pi, pi]; exact quarter-turns returned exactly
constexpr double cos_frac(int m, int N) {
  m %= N;
  if (m < 0) m += N;
  if (m == 0) return 1.0;
  if (4 * m == N || 4 * m == 3 * N) return 0.0;
  if (2 * m == N) return -1.0;
  double x = 2.0 * kPi * m / N;
  if (x > kPi) x -= 2.0 * kPi;
  return taylor_cos(x);
}
constexpr double sin_frac(int m, int N) {
  m %= N;
  if (m < 0) m += N;
  if (m == 0 || 2 * m == N) return 0.0;
  if (4 * m == N) return 1.0;
  if (4 * m == 3 * N) return -1.0;
  double x = 2.0 * kPi * m / N;
  if (x > kPi) x -= 2.0 * kPi;
  return taylor_sin(x);
}

template <int N>
struct Twiddles {
  double c[N];
  double s[N];
  constexpr Twiddles() : c(), s() {
    for (int m = 0; m < N; ++m) {
      c[m] = cos_frac(m, N);
      s[m] = sin_frac(m, N);
    }
  }
};

template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ void dft(T (&re)[N], T (&im)[N]);

template <typename T, int DIR>
__host__ __device__ __forceinline__ void bfly2(T& ar, T& ai, T& br, T& bi) {
  const T tr = ar - br, ti = ai - bi;
  ar = ar + br;
  ai = ai + bi;
  br = tr;
  bi = ti;
}

template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ void dft(T (&re)[N], T (&im)[N]) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2) {
    bfly2<T, DIR>(re[0], im[0], re[1], im[1]);
  } else if constexpr (N == 3) {
    // w = exp(DIR 2 pi i / 3) = -1/2 + DIR i sqrt(3)/2
    constexpr T h = T(0.86602540378443864676372317075294);
    const T t1r = re[1] + re[2], t1i = im[1] + im[2];
    const T t2r = re[1] - re[2], t2i = im[1] - im[2];
    const T mr = re[0] - T(0.5) * t1r, mi = im[0] - T(0.5) * t1i;
    // DIR * i * h * t2 = DIR * h * (-t2i + i t2r)
    const T sr = T(-DIR) * h * t2i, si = T(DIR) * h * t2r;
    re[0] = re[0] + t1r;
    im[0] = im[0] + t1i;
    re[1] = mr + sr;
    im[1] = mi + si;
    re[2] = mr - sr;
    im[2] = mi - si;
  } else if constexpr (N == 4) {
    const T ar = re[0] + re[2], ai = im[0] + im[2];
    const T br = re[0] - re[2], bi = im[0] - im[2];
    const T cr = re[1] + re[3], ci = im[1] + im[3];
    const T er = re[1] - re[3], ei = im[1] - im[3];
    // w = DIR * i:  w * e = DIR * (-ei + i er)
    const T wr = T(-DIR) * ei, wi = T(DIR) * er;
    re[0] = ar + cr;
    im[0] = ai + ci;
    re[2] = ar - cr;
    im[2] = ai - ci;
    re[1] = br + wr;
    im[1] = bi + wi;
    re[3] = br - wr;
    im[3] = bi - wi;
  } else {
    constexpr int N1 = (N % 4 == 0) ? 4 : ((N % 2 == 0) ? 2 : 3);
    constexpr int N2 = N / N1;
    static_assert(N1 * N2 == N, "length must factor into 2, 3, 4");
    constexpr Twiddles<N> tw{};
    T yr[N1][N2], yi[N1][N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      T ar[N1], ai[N1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) {
        ar[n1] = re[N2 * n1 + n2];
        ai[n1] = im[N2 * n1 + n2];
      }
      dft<T, N1, DIR>(ar, ai);
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) {
        const int m = (n2 * k1) % N;
        const double cd = tw.c[m];
        const double sd = DIR * tw.s[m];
        if (m == 0) {
          yr[k1][n2] = ar[k1];
          yi[k1][n2] = ai[k1];
        } else if (cd == 0.0) {  // multiply by +-i
          yr[k1][n2] = -T(sd) * ai[k1];
          yi[k1][n2] = T(sd) * ar[k1];
        } else {
          const T c = T(cd), s = T(sd);
          yr[k1][n2] = ar[k1] * c - ai[k1] * s;
          yi[k1][n2] = ar[k1] * s + ai[k1] * c;
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      dft<T, N2, DIR>(yr[k1], yi[k1]);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        re[k1 + N1 * k2] = yr[k1][k2];
        im[k1 + N1 * k2] = yi[k1][k2];
      }
    }
  }
}

}  // namespace fft
}  // namespace blr
