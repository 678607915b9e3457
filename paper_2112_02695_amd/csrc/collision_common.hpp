// Shared device helpers of the collision kernels.
#pragma once

#include <algorithm>
#include <cstring>
#include <utility>

#include "fft.hpp"
#include "internal.hpp"

namespace blr {

template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
  using t = float2;
};
template <>
struct Vec2<double> {
  using t = double2;
};

template <typename T>
__host__ __device__ __forceinline__ typename Vec2<T>::t make2(T x, T y) {
  typename Vec2<T>::t v;
  v.x = x;
  v.y = y;
  return v;
}

__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// centred integer mode of a DFT index
template <int N>
__host__ __device__ __forceinline__ int ctr(int k) {
  return k >= N / 2 ? k - N : k;
}

// A tile of the pair products computed by one sigma-reduce launch: basis
// indices (compact numbering) on the left and right, and the output row of
// each (u, v) slot (-1 = not requested).
struct ReduceTile {
  int ni, nj;
  int bi[16];
  int bj[16];
  int out[256];
};

// compact basis and pair list of one call
struct PairPlan {
  std::vector<int> bidx;     // compact basis -> row of V
  std::vector<int> li, lj;   // per distinct pair, compact indices (li <= lj)
  std::vector<int> row;      // per distinct pair, the first output row asking for it
  std::vector<std::pair<int, int>> dup;  // (output row, row it repeats) for repeated pairs
  bool generic_only = false;             // BLR_GENERIC_FFT: no fused kernels
};

// Tiles of the pair products: compact basis indices grouped by G; one tile per
// (group, group) block that holds at least one requested pair.
// Radial nodes whose sigma sums and pair transforms one pass of the general
// path takes together (the products of all of them and their transforms are
// held at once: P n values and P n complex values per node, up to 256 MB).
inline int radial_chunk(int mrho, long P, long n, size_t tbytes) {
  const double per = (double)P * (double)n * 3.0 * (double)tbytes;
  const long c = (long)((256.0 * 1024 * 1024) / per);
  return (int)std::max<long>(1, std::min<long>(mrho, c));
}

inline std::vector<ReduceTile> plan_tiles(int rb, const std::vector<int>& li, const std::vector<int>& lj,
                                          int G, bool& diag_only) {
  std::vector<ReduceTile> tiles;
  const int ng = (rb + G - 1) / G;
  diag_only = (ng == 1);
  for (int g1 = 0; g1 < ng; ++g1)
    for (int g2 = g1; g2 < ng; ++g2) {
      ReduceTile t;
      std::memset(&t, 0, sizeof(t));
      for (int k = 0; k < 256; ++k) t.out[k] = -1;
      t.ni = std::min(G, rb - g1 * G);
      t.nj = std::min(G, rb - g2 * G);
      for (int u = 0; u < t.ni; ++u) t.bi[u] = g1 * G + u;
      for (int v = 0; v < t.nj; ++v) t.bj[v] = g2 * G + v;
      bool any = false;
      for (size_t p = 0; p < li.size(); ++p) {
        int i = std::min(li[p], lj[p]), j = std::max(li[p], lj[p]);
        if (i / G == g1 && j / G == g2) {
          t.out[(i - g1 * G) * G + (j - g2 * G)] = (int)p;
          any = true;
        }
      }
      if (any) tiles.push_back(t);
    }
  return tiles;
}

template <typename T>
void fill(hipStream_t s, T* p, long count, T v);
void timed_begin(const std::string& name, double bytes, hipStream_t s);
void timed_end(hipStream_t s);
bool fast_collision_f32(blr_ctx ctx, const DevTables& tb, const float* V, const PairPlan& pl,
                        const std::vector<int>& prow, float* Q, bool conserve);
bool carleman_filter_f32(blr_ctx ctx, const DevTables& tb, const float2* Vh, float* Sh, int rb);
void basis_spectra_f32(blr_ctx ctx, const DevTables& tb, const float* V, const PairPlan& pl,
                       float2** Vh, float** Vp, float** Lam);

// moment projection parameters
struct MomentArgs {
  double L, dv, w;      // box half width, spacing, dv^d
  double minv[25];      // (C C^T)^-1, (d+2)^2 row-major
  int N, d;
};

}  // namespace blr
