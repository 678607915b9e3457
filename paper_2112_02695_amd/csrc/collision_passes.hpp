// Loaders and storers of the generic pipeline's line passes (collision.hip),
// and the per-thread bodies of its line pass, sigma-reduce and Carleman final
// kernels.  Each loader fills one line of N complex values from a field; each
// storer writes one back.  Host-callable as well, so that the index
// arithmetic can be run and bounds-checked on the CPU.
#pragma once

#include "collision_common.hpp"

namespace blr {

// grid points per block of the moment projection
constexpr int kMomChunk = 2048;

// ------------------------------------------------------------------ loaders
template <typename T>
struct LdComplex {
  static constexpr int bpe = 2;  // algorithmic bytes per element / sizeof(T)
  const typename Vec2<T>::t* p;
  int n;
  template <int N>
  __host__ __device__ void load(long f, int base, int stride, T (&re)[N], T (&im)[N]) const {
    const auto* q = p + f * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const auto v = q[(long)j * stride];
      re[j] = v.x;
      im[j] = v.y;
    }
  }
};

// rows of a matrix picked through an index map (at most 64 rows)
struct Idx64 {
  int v[64];
};

template <typename T>
struct LdRealIdx {
  static constexpr int bpe = 1;  // algorithmic bytes per element / sizeof(T)
  const T* p;
  int n;
  Idx64 idx;
  template <int N>
  __host__ __device__ void load(long f, int base, int stride, T (&re)[N], T (&im)[N]) const {
    const T* q = p + (long)idx.v[f] * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      re[j] = q[(long)j * stride];
      im[j] = T(0);
    }
  }
};

template <typename T>
struct LdReal {
  static constexpr int bpe = 1;  // algorithmic bytes per element / sizeof(T)
  const T* p;
  int n;
  template <int N>
  __host__ __device__ void load(long f, int base, int stride, T (&re)[N], T (&im)[N]) const {
    const T* q = p + f * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      re[j] = q[(long)j * stride];
      im[j] = T(0);
    }
  }
};

// field f < rb: V^_f; field f >= rb: G- V^_(f-rb).  Both inverse transforms
// are real; they are kept in separate fields because |G-| can exceed 1e4 and
// packing the two into one complex transform would leak the rounding of the
// loss field into the projected basis.
template <typename T>
struct LdBasisMode {
  static constexpr int bpe = 2;  // algorithmic bytes per element / sizeof(T)
  const typename Vec2<T>::t* vh;
  const T* gl;
  int n, rb;
  template <int N>
  __host__ __device__ void load(long f, int base, int stride, T (&re)[N], T (&im)[N]) const {
    const bool loss = f >= rb;
    const auto* q = vh + (loss ? f - rb : f) * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const auto v = q[(long)j * stride];
      const T g = loss ? gl[base + j * stride] : T(1);
      re[j] = v.x * g;
      im[j] = v.y * g;
    }
  }
};

// V^_ib (cos x - sin x) for field f = (ib, a, p) of the shift batch
template <typename T, int N, int D>
struct LdShift {
  static constexpr int bpe = 2;  // algorithmic bytes per element / sizeof(T)
  const typename Vec2<T>::t* vh;
  const typename Vec2<T>::t* phase;  // (mrho*nbp) x D x N
  int n, mrho, nbp;
  long f0;
  template <int NN>
  __host__ __device__ void load(long fl, int base, int stride, T (&re)[NN], T (&im)[NN]) const {
    const long f = f0 + fl;
    const int p = (int)(f % nbp);
    const int a = (int)((f / nbp) % mrho);
    const long ib = f / ((long)nbp * mrho);
    const auto* ph = phase + ((long)a * nbp + p) * D * N;
    const auto* q = vh + ib * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int e = base + j * stride;
      typename Vec2<T>::t c;
      if constexpr (D == 3) {
        const int k0 = e / (N * N), k1 = (e / N) % N, k2 = e % N;
        c = cmul(cmul(ph[k0], ph[N + k1]), ph[2 * N + k2]);
      } else {
        const int k0 = e / N, k1 = e % N;
        c = cmul(ph[k0], ph[N + k1]);
      }
      const T fac = c.x + c.y;
      const auto v = q[(long)j * stride];
      re[j] = v.x * fac;
      im[j] = v.y * fac;
    }
  }
};

// Carleman form: V^_ib c_p(k) (complex product) for field f = (ib, p)
template <typename T>
struct LdFilter {
  static constexpr int bpe = 4;  // algorithmic bytes per element / sizeof(T)
  const typename Vec2<T>::t* vh;
  const typename Vec2<T>::t* filt;  // nbp x n
  int n, nbp;
  long f0;
  template <int N>
  __host__ __device__ void load(long fl, int base, int stride, T (&re)[N], T (&im)[N]) const {
    const long f = f0 + fl;
    const int p = (int)(f % nbp);
    const long ib = f / nbp;
    const auto* q = vh + ib * n + base;
    const auto* c = filt + (long)p * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const auto v = q[(long)j * stride];
      const auto w = c[(long)j * stride];
      re[j] = v.x * w.x - v.y * w.y;
      im[j] = v.x * w.y + v.y * w.x;
    }
  }
};

// one pair-product field (real) per complex transform: pairs are not packed
// two to a transform because their magnitudes can differ by orders of
// magnitude and the smaller one would inherit the larger one's rounding.
template <typename T>
struct LdPair1 {
  static constexpr int bpe = 1;  // algorithmic bytes per element / sizeof(T)
  const T* pa;  // P x n
  int n;
  template <int N>
  __host__ __device__ void load(long p, int base, int stride, T (&re)[N], T (&im)[N]) const {
    const T* q = pa + p * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      re[j] = q[(long)j * stride];
      im[j] = T(0);
    }
  }
};

// ------------------------------------------------------------------- storers
template <typename T>
struct StComplex {
  static constexpr int bpe = 2;  // algorithmic bytes per element / sizeof(T)
  typename Vec2<T>::t* p;
  int n;
  template <int N>
  __host__ __device__ void store(long f, int base, int stride, const T (&re)[N], const T (&im)[N]) const {
    auto* q = p + f * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) q[(long)j * stride] = make2<T>(re[j], im[j]);
  }
};

// basis spectrum: scale by 1/n and drop every mode with a Nyquist component
template <typename T, int N, int D>
struct StBasisSpec {
  static constexpr int bpe = 2;  // algorithmic bytes per element / sizeof(T)
  typename Vec2<T>::t* p;
  int n;
  T scale;
  template <int NN>
  __host__ __device__ void store(long f, int base, int stride, const T (&re)[NN], const T (&im)[NN]) const {
    auto* q = p + f * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int e = base + j * stride;
      bool nyq;
      if constexpr (D == 3)
        nyq = (e / (N * N) == N / 2) || ((e / N) % N == N / 2) || (e % N == N / 2);
      else
        nyq = (e / N == N / 2) || (e % N == N / 2);
      q[(long)j * stride] = nyq ? make2<T>(T(0), T(0)) : make2<T>(re[j] * scale, im[j] * scale);
    }
  }
};

template <typename T>
struct StRe {
  static constexpr int bpe = 1;  // algorithmic bytes per element / sizeof(T)
  T* o;
  int n;
  template <int N>
  __host__ __device__ void store(long f, int base, int stride, const T (&re)[N], const T (&im)[N]) const {
#pragma unroll
    for (int j = 0; j < N; ++j) o[f * n + base + (long)j * stride] = re[j];
  }
};

template <typename T>
struct StSplit {
  static constexpr int bpe = 2;  // algorithmic bytes per element / sizeof(T)
  T* o1;
  T* o2;
  int n;
  template <int N>
  __host__ __device__ void store(long f, int base, int stride, const T (&re)[N], const T (&im)[N]) const {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      o1[f * n + base + (long)j * stride] = re[j];
      o2[f * n + base + (long)j * stride] = im[j];
    }
  }
};

// shift batch: field (ib, a, p) -> S(ib, a, b) = re - im, S(ib, a, bbar) = re + im
template <typename T>
struct StShiftSplit {
  static constexpr int bpe = 2;  // algorithmic bytes per element / sizeof(T)
  T* sh;  // (rb*mrho*msig) x n
  const int* bp_b;
  const int* bp_bb;
  int n, mrho, nbp, msig;
  long f0;
  template <int N>
  __host__ __device__ void store(long fl, int base, int stride, const T (&re)[N], const T (&im)[N]) const {
    const long f = f0 + fl;
    const int p = (int)(f % nbp);
    const long iba = f / nbp;  // ib*mrho + a
    T* s1 = sh + (iba * msig + bp_b[p]) * n + base;
    T* s2 = sh + (iba * msig + bp_bb[p]) * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      s1[(long)j * stride] = re[j] - im[j];
      s2[(long)j * stride] = re[j] + im[j];
    }
  }
};

// accumulate w(a, |k|^2) * value into the couple spectrum
template <typename T, int N, int D>
struct StAccumF {
  static constexpr int bpe = 4;  // algorithmic bytes per element / sizeof(T)
  typename Vec2<T>::t* G;
  const T* fw;  // nkk weights of this radial node
  int n;
  template <int NN>
  __host__ __device__ void store(long c, int base, int stride, const T (&re)[NN], const T (&im)[NN]) const {
    auto* g = G + c * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int e = base + j * stride;
      int kk;
      if constexpr (D == 3) {
        const int k0 = ctr<N>(e / (N * N)), k1 = ctr<N>((e / N) % N), k2 = ctr<N>(e % N);
        kk = k0 * k0 + k1 * k1 + k2 * k2;
      } else {
        const int k0 = ctr<N>(e / N), k1 = ctr<N>(e % N);
        kk = k0 * k0 + k1 * k1;
      }
      const T w = fw[kk];
      auto v = g[(long)j * stride];
      v.x += w * re[j];
      v.y += w * im[j];
      g[(long)j * stride] = v;
    }
  }
};

// accumulate tab(k) * value into the couple spectrum (anisotropic kernel:
// the weight depends on the direction of k, one table per radial node and
// antipodal pair)
template <typename T>
struct StAccumTab {
  static constexpr int bpe = 5;  // algorithmic bytes per element / sizeof(T)
  typename Vec2<T>::t* G;
  const T* tab;  // n weights of this (radial node, pair)
  int n;
  template <int N>
  __host__ __device__ void store(long c, int base, int stride, const T (&re)[N], const T (&im)[N]) const {
    auto* g = G + c * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const T w = tab[base + j * stride];
      auto v = g[(long)j * stride];
      v.x += w * re[j];
      v.y += w * im[j];
      g[(long)j * stride] = v;
    }
  }
};

// Q = gain - loss for pair p
template <typename T>
struct StFinal {
  static constexpr int bpe = 5;  // algorithmic bytes per element / sizeof(T)
  T* Q;
  const T* vp;
  const T* lam;
  const int* pi;  // local basis index per pair
  const int* pj;
  const int* prow;  // output row per pair
  int n;
  template <int N>
  __host__ __device__ void store(long p, int base, int stride, const T (&re)[N], const T (&im)[N]) const {
    const long i = pi[p], jj = pj[p];
    T* q = Q + (long)prow[p] * n + base;
    const T* vi = vp + i * n + base;
    const T* vj = vp + jj * n + base;
    const T* li = lam + i * n + base;
    const T* lj = lam + jj * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const long o = (long)j * stride;
      q[o] = re[j] - T(0.5) * (vj[o] * li[o] + vi[o] * lj[o]);
    }
  }
};

// One grid point q of a sigma-reduce tile: basis functions (ni on the left,
// nj on the right, or one set of ni on both sides for a diagonal tile) whose
// pair products are accumulated in registers over the antipodal sphere pairs:
//   P_uv += w_b (S_u(b) S_v(bbar) + S_u(bbar) S_v(b)).
template <typename T, int G, bool DIAG>
__host__ __device__ __forceinline__ void sigma_reduce_point(int q, const T* __restrict__ sh,
                                                            T* __restrict__ pa,
                                                            const ReduceTile& tile,
                                                            const T* __restrict__ wbp,
                                                            const int* __restrict__ bp_b,
                                                            const int* __restrict__ bp_bb, int n,
                                                            int mrho, int msig, int nbp, int a) {
  constexpr int NP = DIAG ? G * (G + 1) / 2 : G * G;
  T acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = T(0);
  for (int bp = 0; bp < nbp; ++bp) {
    const int b = bp_b[bp], bb = bp_bb[bp];
    const T w = wbp[bp];
    T xi[G], yi[G], xj[G], yj[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      T x = T(0), y = T(0);
      if (u < tile.ni) {
        const long fi = ((long)tile.bi[u] * mrho + a) * msig;
        x = sh[(fi + b) * n + q];
        y = sh[(fi + bb) * n + q];
      }
      xi[u] = w * x;
      yi[u] = w * y;
      if constexpr (DIAG) {
        xj[u] = x;
        yj[u] = y;
      } else {
        x = y = T(0);
        if (u < tile.nj) {
          const long fj = ((long)tile.bj[u] * mrho + a) * msig;
          x = sh[(fj + b) * n + q];
          y = sh[(fj + bb) * n + q];
        }
        xj[u] = x;
        yj[u] = y;
      }
    }
    int p = 0;
#pragma unroll
    for (int u = 0; u < G; ++u) {
#pragma unroll
      for (int v = DIAG ? u : 0; v < G; ++v) {
        acc[p] += xi[u] * yj[v] + yi[u] * xj[v];
        ++p;
      }
    }
  }
  int p = 0;
#pragma unroll
  for (int u = 0; u < G; ++u) {
#pragma unroll
    for (int v = DIAG ? u : 0; v < G; ++v) {
      const int row = tile.out[u * G + v];
      if (row >= 0) pa[(long)row * n + q] = acc[p];
      ++p;
    }
  }
}

// The same sum for pair p = (i, i): P_ii = sum_b 2 w_b S_i(b) S_i(bbar).
template <typename T>
__host__ __device__ __forceinline__ void sigma_self_point(int q, int p, const T* __restrict__ sh,
                                                          T* __restrict__ pa,
                                                          const int* __restrict__ pi,
                                                          const T* __restrict__ wbp,
                                                          const int* __restrict__ bp_b,
                                                          const int* __restrict__ bp_bb, int n,
                                                          int mrho, int msig, int nbp, int a) {
  const long fi = ((long)pi[p] * mrho + a) * msig;
  T acc = T(0);
  for (int bp = 0; bp < nbp; ++bp) {
    const T w = wbp[bp];
    const T x = sh[(fi + bp_b[bp]) * n + q];
    const T y = sh[(fi + bp_bb[bp]) * n + q];
    acc += (w * x) * y + (w * y) * x;
  }
  pa[(long)p * n + q] = acc;
}

// Carleman form, point e of pair p: Q = gain - loss with the gain already on
// the grid
template <typename T>
__host__ __device__ __forceinline__ void carleman_final_point(int e, int p, const T* __restrict__ Pa,
                                                              const T* __restrict__ vp,
                                                              const T* __restrict__ lam,
                                                              const int* __restrict__ pi,
                                                              const int* __restrict__ pj,
                                                              const int* __restrict__ prow, int n,
                                                              T* __restrict__ Q) {
  const long i = pi[p], j = pj[p];
  Q[(long)prow[p] * n + e] =
      Pa[(long)p * n + e] - T(0.5) * (vp[j * n + e] * lam[i * n + e] + vp[i * n + e] * lam[j * n + e]);
}

// One thread of a line pass: line t of nlines (fields of D = 2: N lines,
// D = 3: N^2 lines per field) along `axis`, loaded, transformed, stored.
template <typename T, int N, int D, int DIR, class Ld, class St>
__host__ __device__ __forceinline__ void line_pass_thread(long t, const Ld& ld, const St& st,
                                                          int axis) {
  constexpr int lines = (D == 2 ? N : N * N);
  const long f = t / lines;
  const int l = (int)(t % lines);
  const int stride = axis == D - 1 ? 1 : (axis == D - 2 ? N : N * N);
  const int base = (l / stride) * stride * N + (l % stride);
  T re[N], im[N];
  ld.template load<N>(f, base, stride, re, im);
  fft::dft<T, N, DIR>(re, im);
  st.template store<N>(f, base, stride, re, im);
}

// One thread of the last axis of the pair transforms with the radial
// weights: line t of the pairs (P of them) along axis 0, for the na radial
// nodes a0.. in turn: the node's transformed product (field k P + p of tmp,
// k = a - a0) is transformed and accumulated, weighted, into pair p's couple
// spectrum.  Node after node, the same order of accumulation as one pass per
// node.
template <typename T, int N, int D>
__host__ __device__ __forceinline__ void accum_radial_thread(long t,
                                                             const typename Vec2<T>::t* tmp,
                                                             typename Vec2<T>::t* G, const T* fw,
                                                             int nkk, long P, int a0, int na) {
  constexpr int lines = (D == 2 ? N : N * N);
  constexpr int n = (D == 2 ? N * N : N * N * N);
  const long p = t / lines;
  const int base = (int)(t % lines);  // axis 0: stride = lines
  const LdComplex<T> ld{tmp, n};
  for (int k = 0; k < na; ++k) {
    T re[N], im[N];
    ld.template load<N>((long)k * P + p, base, lines, re, im);
    fft::dft<T, N, -1>(re, im);
    const StAccumF<T, N, D> st{G, fw + (size_t)(a0 + k) * nkk, n};
    st.template store<N>(p, base, lines, re, im);
  }
}

}  // namespace blr
