// Pair collisions Q_s(V_i, V_j) on the velocity grid: the generic pipeline.
//
// Steps (for a basis set {V_i} and a list of pairs; T = float or double):
//   1. V^_i = DFT(V_i)/n with the Nyquist modes dropped; from it the projected
//      basis V_i~ = IDFT(V^_i) and the loss field Lam_i = IDFT(G- V^_i).
//   2. shifts S_i(a,b)(v) = V_i~(v - rho_a sigma_b / 2) for every radial node a
//      and sphere node b: for an antipodal pair (b, bbar) one complex inverse
//      transform of V^_i (cos x - sin x), x = theta_a sigma_b . k, yields
//      W with S(b) = Re W - Im W and S(bbar) = Re W + Im W.
//   3. per radial node a and pair (i,j):
//        P_ij,a = sum_b w_b S_i(a,b) S_j(a,bbar)           (pointwise, sigma sum)
//   4. G_ij += w_a rho_a^(d-1) B(rho_a) A_d(theta_a |k|) DFT(P_ij,a)/n
//   5. Q_ij = IDFT(G_ij) - (V_j~ Lam_i + V_i~ Lam_j)/2
//   6. optional FP64 projection removing the d+2 discrete moments.
// Every transform here is done as one kernel per axis ("line pass"): each
// thread holds one line of N complex values in registers (fft.hpp).  This path
// serves every size and both precisions; the fused FP32 kernels in
// collision_fast.hip replace steps 2-5 for the 3D grids when they apply.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "collision_common.hpp"
#include "collision_passes.hpp"

namespace blr {

// Carleman form: Q = gain - loss with the gain already on the grid
template <typename T>
__global__ __launch_bounds__(256) void k_carleman_final(const T* __restrict__ Pa, const T* __restrict__ vp,
                                                        const T* __restrict__ lam,
                                                        const int* __restrict__ pi,
                                                        const int* __restrict__ pj,
                                                        const int* __restrict__ prow, int n,
                                                        T* __restrict__ Q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (e >= n) return;
  carleman_final_point<T>(e, p, Pa, vp, lam, pi, pj, prow, n, Q);
}

// ------------------------------------------------------------ line pass
template <typename T, int N, int D, int DIR, class Ld, class St>
__global__ __launch_bounds__(128) void k_line_pass(Ld ld, St st, int axis, long nlines) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= nlines) return;
  line_pass_thread<T, N, D, DIR>(t, ld, st, axis);
}

// the timer of the context issuing the current launches (set per call)
static thread_local KernelTimer* g_timer = nullptr;
static thread_local const char* g_stage = "";

struct TimedScope {
  hipStream_t s;
  TimedScope(hipStream_t st, const std::string& name, double bytes) : s(st) {
    if (g_timer && g_timer->on) g_timer->begin(s, name, bytes);
  }
  ~TimedScope() {
    if (g_timer && g_timer->on) g_timer->end(s);
  }
};

void timed_begin(const std::string& name, double bytes, hipStream_t s) {
  if (g_timer && g_timer->on) g_timer->begin(s, name, bytes);
}
void timed_end(hipStream_t s) {
  if (g_timer && g_timer->on) g_timer->end(s);
}

template <typename T, int N, int D, int DIR, class Ld, class St>
static void line_pass(hipStream_t s, const Ld& ld, const St& st, int axis, long nfields) {
  constexpr int lines = (D == 2 ? N : N * N);
  const long nl = nfields * lines;
  const int bs = 128;
  const long nb = (nl + bs - 1) / bs;
  constexpr int n = (D == 2 ? N * N : N * N * N);
  TimedScope ts(s, std::string(g_stage) + ".axis" + std::to_string(axis),
                (double)nfields * n * (Ld::bpe + St::bpe) * sizeof(T));
  hipLaunchKernelGGL((k_line_pass<T, N, D, DIR, Ld, St>), dim3((unsigned)nb), dim3(bs), 0, s, ld,
                     st, axis, nl);
  BLR_CHECK_LAUNCH();
}

// The first two axes of a 3D transform in one launch (axis 2 loaded through
// `ld`, axis 1 stored through `st`): each group of N threads takes one plane
// i0 of one field, one line per thread, and the plane passes through LDS
// between the two axes.  The line transforms are those of two line passes;
// only the round trip of the plane through memory is gone.
template <int N>
constexpr int planes_per_block() {
  return 64 / N > 0 ? 64 / N : 1;
}

template <typename T, int N, int DIR, class Ld, class St>
__global__ __launch_bounds__(64) void k_plane_pass(Ld ld, St st, long nplanes) {
  constexpr int PPB = planes_per_block<N>();
  // one component at a time through one array (half the LDS, so that more
  // workgroups fit a CU)
  __shared__ T pl[PPB][N][N + 1];
  const int q = threadIdx.x / N, u = threadIdx.x % N;
  const long g = blockIdx.x * (long)PPB + q;
  const bool ok = g < nplanes;
  const long f = g / N;
  const int i0 = (int)(g % N);
  T re[N], im[N];
  if (ok) {
    // line (i0, i1 = u) along axis 2
    ld.template load<N>(f, (i0 * N + u) * N, 1, re, im);
    fft::dft<T, N, DIR>(re, im);
#pragma unroll
    for (int j = 0; j < N; ++j) pl[q][u][j] = re[j];
  }
  __syncthreads();
  // line (i0, i2 = u) along axis 1
  if (ok) {
#pragma unroll
    for (int j = 0; j < N; ++j) re[j] = pl[q][j][u];
  }
  __syncthreads();
  if (ok) {
#pragma unroll
    for (int j = 0; j < N; ++j) pl[q][u][j] = im[j];
  }
  __syncthreads();
  if (!ok) return;
#pragma unroll
  for (int j = 0; j < N; ++j) im[j] = pl[q][j][u];
  fft::dft<T, N, DIR>(re, im);
  st.template store<N>(f, i0 * N * N + u, N, re, im);
}

template <typename T, int N, int DIR, class Ld, class St>
static void plane_pass(hipStream_t s, const Ld& ld, const St& st, long nfields) {
  constexpr int PPB = planes_per_block<N>();
  const long np = nfields * N;
  const long nb = (np + PPB - 1) / PPB;
  constexpr int n = N * N * N;
  TimedScope ts(s, std::string(g_stage) + ".axis21",
                (double)nfields * n * (Ld::bpe + St::bpe) * sizeof(T));
  hipLaunchKernelGGL((k_plane_pass<T, N, DIR, Ld, St>), dim3((unsigned)nb), dim3(PPB * N), 0, s,
                     ld, st, np);
  BLR_CHECK_LAUNCH();
}

// A whole 2D transform in one launch: each group of N threads takes one
// field, one row (axis 1) per thread, then one column (axis 0) per thread,
// the field passing through LDS in between (one component at a time).  The
// line transforms are those of two line passes.
template <typename T, int N, int DIR, class Ld, class St>
__global__ __launch_bounds__(64) void k_field2d_pass(Ld ld, St st, long nfields) {
  constexpr int PPB = planes_per_block<N>();
  __shared__ T pl[PPB][N][N + 1];
  const int q = threadIdx.x / N, u = threadIdx.x % N;
  const long f = blockIdx.x * (long)PPB + q;
  const bool ok = f < nfields;
  T re[N], im[N];
  if (ok) {
    ld.template load<N>(f, u * N, 1, re, im);  // row u along axis 1
    fft::dft<T, N, DIR>(re, im);
#pragma unroll
    for (int j = 0; j < N; ++j) pl[q][u][j] = re[j];
  }
  __syncthreads();
  if (ok) {
#pragma unroll
    for (int j = 0; j < N; ++j) re[j] = pl[q][j][u];
  }
  __syncthreads();
  if (ok) {
#pragma unroll
    for (int j = 0; j < N; ++j) pl[q][u][j] = im[j];
  }
  __syncthreads();
  if (!ok) return;
#pragma unroll
  for (int j = 0; j < N; ++j) im[j] = pl[q][j][u];
  fft::dft<T, N, DIR>(re, im);  // column u along axis 0
  st.template store<N>(f, u, N, re, im);
}

// every axis of a D-dimensional transform but the last (0): axis D-1 loaded
// through ld, the result stored through st; in 3D the axes 2 and 1 in one
// plane pass
template <typename T, int N, int D, int DIR, class Ld, class St>
static void first_axes(hipStream_t s, const Ld& ld, const St& st, long nfields) {
  if constexpr (D == 3)
    plane_pass<T, N, DIR>(s, ld, st, nfields);
  else
    line_pass<T, N, D, DIR>(s, ld, st, D - 1, nfields);
}

// full D-dimensional transform: first axis (D-1) uses ld, last (0) uses st
template <typename T, int N, int D, int DIR, class Ld, class St>
static void transform(hipStream_t s, const Ld& ld, const St& st, typename Vec2<T>::t* tmp,
                      long nfields) {
  constexpr int n = (D == 2 ? N * N : N * N * N);
  if constexpr (D == 2) {
    // the whole field in one pass
    constexpr int PPB = planes_per_block<N>();
    TimedScope ts(s, std::string(g_stage) + ".axis10",
                  (double)nfields * n * (Ld::bpe + St::bpe) * sizeof(T));
    hipLaunchKernelGGL((k_field2d_pass<T, N, DIR, Ld, St>),
                       dim3((unsigned)((nfields + PPB - 1) / PPB)), dim3(PPB * N), 0, s, ld, st,
                       nfields);
    BLR_CHECK_LAUNCH();
    (void)tmp;
    return;
  }
  StComplex<T> stc{tmp, n};
  LdComplex<T> ldc{tmp, n};
  first_axes<T, N, D, DIR>(s, ld, stc, nfields);
  line_pass<T, N, D, DIR>(s, ldc, st, 0, nfields);
}

// The last axis of the pair transforms of na radial nodes (fields k P + p of
// tmp, k = a - a0), each accumulated with its radial weights into pair p's
// couple spectrum G[p]: one thread per line of a pair, the nodes in turn.
template <typename T, int N, int D>
__global__ __launch_bounds__(128) void k_accum_radial(const typename Vec2<T>::t* __restrict__ tmp,
                                                      typename Vec2<T>::t* __restrict__ G,
                                                      const T* __restrict__ fw, int nkk, long P,
                                                      int a0, int na, long nlines) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= nlines) return;
  accum_radial_thread<T, N, D>(t, tmp, G, fw, nkk, P, a0, na);
}

template <typename T, int N, int D>
static void accum_radial(hipStream_t s, const typename Vec2<T>::t* tmp, typename Vec2<T>::t* G,
                         const T* fw, int nkk, long P, int a0, int na) {
  constexpr int lines = (D == 2 ? N : N * N);
  constexpr int n = (D == 2 ? N * N : N * N * N);
  const long nl = P * lines;
  const int bs = 128;
  TimedScope ts(s, std::string(g_stage) + ".axis0", (double)P * n * na * 6 * sizeof(T));
  hipLaunchKernelGGL((k_accum_radial<T, N, D>), dim3((unsigned)((nl + bs - 1) / bs)), dim3(bs), 0,
                     s, tmp, G, fw, nkk, P, a0, na, nl);
  BLR_CHECK_LAUNCH();
}

// transform of the rows bidx of V: directly when they are the rows 0..rb-1
// (the full-tensor step's cells, up to kMaxSelfRows), else through an index
// map of at most 64 rows
template <typename T, int N, int D, int DIR, class St>
static void transform_rows(hipStream_t s, const T* V, const std::vector<int>& bidx, const St& st,
                           typename Vec2<T>::t* tmp) {
  constexpr int n = (D == 2 ? N * N : N * N * N);
  const int rb = (int)bidx.size();
  bool ident = true;
  for (int ib = 0; ib < rb; ++ib) ident = ident && bidx[ib] == ib;
  if (ident) {
    transform<T, N, D, DIR>(s, LdReal<T>{V, n}, st, tmp, rb);
    return;
  }
  require(rb <= 64, "at most 64 distinct basis functions per call");
  Idx64 idx{};
  for (int ib = 0; ib < rb; ++ib) idx.v[ib] = bidx[ib];
  transform<T, N, D, DIR>(s, LdRealIdx<T>{V, n, idx}, st, tmp, rb);
}

// FP64 sigma sums of the isotropic general path: up to 12 basis functions in
// one diagonal 12-wide tile (one pass over the shifts instead of three 8-wide
// tiles); more functions keep 8-wide tiles (the 12-wide off-diagonal tile
// fits only one wave per SIMD).
inline bool wide_tiles64(int rb) { return rb <= 12; }

// ------------------------------------------------------------- sigma reduce
// One thread per grid point; a tile of basis functions (ni on the left, nj on
// the right, or one set of ni on both sides for a diagonal tile) whose pair
// products are accumulated in registers over the antipodal sphere pairs:
//   P_uv += w_b (S_u(b) S_v(bbar) + S_u(bbar) S_v(b)).
template <typename T, int G, bool DIAG>
__global__ __launch_bounds__(256) void k_sigma_reduce(const T* __restrict__ sh, T* __restrict__ pa,
                                                      ReduceTile tile, const T* __restrict__ wbp,
                                                      const int* __restrict__ bp_b,
                                                      const int* __restrict__ bp_bb, int n,
                                                      int mrho, int msig, int nbp, int a0,
                                                      long pstride) {
  // radial node a0 + blockIdx.y, its products at pa + blockIdx.y pstride
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  sigma_reduce_point<T, G, DIAG>(q, sh, pa + blockIdx.y * pstride, tile, wbp, bp_b, bp_bb, n, mrho,
                                 msig, nbp, a0 + (int)blockIdx.y);
}

// The same sums for pairs (i, i) only (every pair of the full-tensor step):
// one thread per (grid point, pair), P_ii = sum_b 2 w_b S_i(b) S_i(bbar).
template <typename T>
__global__ __launch_bounds__(256) void k_sigma_self(const T* __restrict__ sh, T* __restrict__ pa,
                                                    const int* __restrict__ pi,
                                                    const T* __restrict__ wbp,
                                                    const int* __restrict__ bp_b,
                                                    const int* __restrict__ bp_bb, int n, int mrho,
                                                    int msig, int nbp, int a0, long pstride) {
  // radial node a0 + blockIdx.z, its products at pa + blockIdx.z pstride
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (q >= n) return;
  sigma_self_point<T>(q, p, sh, pa + blockIdx.z * pstride, pi, wbp, bp_b, bp_bb, n, mrho, msig, nbp,
                      a0 + (int)blockIdx.z);
}

// ------------------------------------------------------------ utilities
template <typename T>
__global__ void k_fill(T* p, long count, T v) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

template <typename T>
void fill(hipStream_t s, T* p, long count, T v) {
  if (count <= 0) return;
  const int bs = 256;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((count + bs - 1) / bs)), dim3(bs), 0, s, p, count, v);
  BLR_CHECK_LAUNCH();
}
template void fill<float>(hipStream_t, float*, long, float);
template void fill<double>(hipStream_t, double*, long, double);
template void fill<int>(hipStream_t, int*, long, int);

// FP64 least-squares moment projection of rows of Q: m = C q,
// lambda = (C C^T)^-1 m, q <- q - C^T lambda, with C the rows
// dv^d {1, v_1..v_d, |v|^2}.  Two passes over (chunk, row) blocks: the moments
// of each chunk, then every chunk's block sums its row's partial moments in a
// fixed order and corrects its chunk (deterministic, no atomics).

__device__ inline double grid_coords(int e, const MomentArgs& ma, double (&v)[3]) {
  v[0] = v[1] = v[2] = 0.0;
  int rem = e;
  for (int ax = ma.d - 1; ax >= 0; --ax) {
    v[ax] = -ma.L + (rem % ma.N) * ma.dv;
    rem /= ma.N;
  }
  return v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
}

template <typename T>
__global__ __launch_bounds__(256) void k_moment_part(const T* __restrict__ Q, int n, MomentArgs ma,
                                                     double* __restrict__ part) {
  const int b = blockIdx.x, row = blockIdx.y, nb = gridDim.x;
  const T* q = Q + (long)row * n;
  const int e0 = b * kMomChunk, e1 = min(n, e0 + kMomChunk);
  double acc[5] = {0, 0, 0, 0, 0};
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    double v[3];
    const double v2 = grid_coords(e, ma, v);
    const double val = (double)q[e] * ma.w;
    acc[0] += val;
    for (int ax = 0; ax < ma.d; ++ax) acc[1 + ax] += val * v[ax];
    acc[ma.d + 1] += val * v2;
  }
  __shared__ double red[5][256];
  for (int i = 0; i < 5; ++i) red[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int i = 0; i < 5; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 5) part[((long)row * nb + b) * 5 + threadIdx.x] = red[threadIdx.x][0];
}

template <typename T>
__global__ __launch_bounds__(256) void k_moment_apply(T* __restrict__ Q, int n, MomentArgs ma,
                                                      const double* __restrict__ part) {
  const int b = blockIdx.x, row = blockIdx.y, nb = gridDim.x;
  const int m = ma.d + 2;
  __shared__ double lam[5];
  if (threadIdx.x == 0) {
    double mo[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < nb; ++k)
      for (int i = 0; i < 5; ++i) mo[i] += part[((long)row * nb + k) * 5 + i];
    for (int i = 0; i < 5; ++i) {
      double s = 0.0;
      for (int j = 0; j < m && i < m; ++j) s += ma.minv[i * m + j] * mo[j];
      lam[i] = i < m ? s : 0.0;
    }
  }
  __syncthreads();
  T* q = Q + (long)row * n;
  const int e0 = b * kMomChunk, e1 = min(n, e0 + kMomChunk);
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    double v[3];
    const double v2 = grid_coords(e, ma, v);
    double c = lam[0];
    for (int ax = 0; ax < ma.d; ++ax) c += lam[1 + ax] * v[ax];
    c += lam[ma.d + 1] * v2;
    q[e] = (T)((double)q[e] - ma.w * c);
  }
}

template <typename T>
void conserve_rows(blr_ctx ctx, const HostTables& h, T* Q, int rows) {
  if (rows <= 0) return;
  hipStream_t s = ctx->stream;
  MomentArgs ma{};
  ma.L = h.L;
  ma.dv = h.dv;
  ma.w = std::pow(h.dv, h.d);
  for (size_t i = 0; i < h.minv.size() && i < 25; ++i) ma.minv[i] = h.minv[i];
  ma.N = h.N;
  ma.d = h.d;
  const int nb = (h.n + kMomChunk - 1) / kMomChunk;
  double* part = (double*)ctx->buf("mom.part", (size_t)rows * nb * 5 * sizeof(double));
  TimedScope ts(s, "conserve", 3.0 * rows * h.n * sizeof(T));
  hipLaunchKernelGGL(k_moment_part<T>, dim3(nb, rows), dim3(256), 0, s, Q, h.n, ma, part);
  BLR_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_moment_apply<T>, dim3(nb, rows), dim3(256), 0, s, Q, h.n, ma, part);
  BLR_CHECK_LAUNCH();
}
template void conserve_rows<float>(blr_ctx, const HostTables&, float*, int);
template void conserve_rows<double>(blr_ctx, const HostTables&, double*, int);

// ------------------------------------------------------------ planning
static PairPlan make_plan(int r, const int32_t* pairs, int npairs) {
  PairPlan pl;
  std::vector<int> map(r, -1);
  for (int p = 0; p < npairs; ++p)
    for (int h = 0; h < 2; ++h) {
      const int i = pairs[2 * p + h];
      require(i >= 0 && i < r, "pair index out of range [0, r)");
      map[i] = 1;
    }
  for (int i = 0; i < r; ++i)
    if (map[i] > 0) {
      map[i] = (int)pl.bidx.size();
      pl.bidx.push_back(i);
    }
  // each distinct unordered pair is evaluated once (Q_s is symmetric); a
  // repeated request copies the row of its first occurrence
  std::unordered_map<long, int> first;
  first.reserve(2 * (size_t)npairs);
  for (int p = 0; p < npairs; ++p) {
    const int a = map[pairs[2 * p]], b = map[pairs[2 * p + 1]];
    const int lo = std::min(a, b), hi = std::max(a, b);
    int& f = first.try_emplace((long)lo * r + hi, -1).first->second;
    if (f >= 0) {
      pl.dup.emplace_back(p, f);
      continue;
    }
    f = p;
    pl.li.push_back(lo);
    pl.lj.push_back(hi);
    pl.row.push_back(p);
  }
  return pl;
}

// ------------------------------------------------------------ generic run
template <typename T, int N, int D>
struct Generic {
  static constexpr int n = (D == 2 ? N * N : N * N * N);
  using T2 = typename Vec2<T>::t;

  // every requested pair is (i, i): k_sigma_self instead of the tiles
  static bool self_only(const PairPlan& pl) {
    for (size_t p = 0; p < pl.li.size(); ++p)
      if (pl.li[p] != pl.lj[p]) return false;
    return !pl.li.empty();
  }

  // radial nodes a0 .. a0 + na - 1, node k's products at Pa + k P n
  static void sigma_self(hipStream_t s, const char* name, const T* Sh, T* Pa, const int* dli,
                         const T* wbp, const int* bp_b, const int* bp_bb, int mrho, int msig,
                         int nbp, int a0, int P, int na = 1) {
    TimedScope ts(s, name, (double)n * P * na * (2 * nbp + 1) * sizeof(T));
    hipLaunchKernelGGL(k_sigma_self<T>, dim3((n + 255) / 256, P, na), dim3(256), 0, s, Sh, Pa, dli,
                       wbp, bp_b, bp_bb, n, mrho, msig, nbp, a0, (long)P * n);
    BLR_CHECK_LAUNCH();
  }

  static size_t workspace(const HostTables& h, int rb, int P) {
    const long nc = P;
    const long shift_fields = (long)rb * h.mrho * h.nbp;
    const long batch = std::min<long>(shift_fields, 512);
    size_t b = 0;
    b += (size_t)rb * n * sizeof(T);                       // Vc
    b += (size_t)rb * n * sizeof(T2);                      // Vh
    b += (size_t)2 * rb * n * sizeof(T);                   // Vp, Lam
    b += (size_t)rb * h.mrho * h.msig * n * sizeof(T);     // shifts
    const long cr = (h.carleman || h.aniso_n > 0) ? 1 : radial_chunk(h.mrho, nc, n, sizeof(T));
    b += (size_t)std::max<long>(batch, std::max<long>(cr * nc, 2 * rb)) * n * sizeof(T2);  // tmp
    b += (size_t)cr * P * n * sizeof(T);                   // Pa
    b += (size_t)nc * n * sizeof(T2);                      // G
    return b;
  }

  // step 1 only: compact copy, spectra, projected basis and loss fields
  static void basis(blr_ctx ctx, const DevTables& tb, const T* Vsrc, const PairPlan& pl, T2** pVh,
                    T** pVp, T** pLam) {
    const HostTables& h = tb.h;
    hipStream_t s = ctx->stream;
    const int rb = (int)pl.bidx.size();
    const std::string tag = std::string("bas") + (sizeof(T) == 4 ? "f" : "d");
    T2* Vh = (T2*)ctx->buf(tag + ".Vh", (size_t)rb * n * sizeof(T2));
    T* Vp = (T*)ctx->buf(tag + ".VpLam", (size_t)2 * rb * n * sizeof(T));
    T2* tmp = (T2*)ctx->buf(tag + ".tmp", (size_t)2 * rb * n * sizeof(T2));
    g_stage = "basis";
    transform_rows<T, N, D, -1>(s, Vsrc, pl.bidx, StBasisSpec<T, N, D>{Vh, n, T(1) / T(n)}, tmp);
    transform<T, N, D, +1>(s, LdBasisMode<T>{Vh, (const T*)tb.gloss, n, rb}, StRe<T>{Vp, n}, tmp,
                           2 * rb);
    (void)h;
    *pVh = Vh;
    *pVp = Vp;
    *pLam = Vp + (size_t)rb * n;
  }

  // Carleman form: filtered fields (two per direction pair and basis function,
  // one complex inverse transform each), the direction sums of their pair
  // products (the sigma reduction with weights b0 w), minus the loss.
  static void carleman(blr_ctx ctx, const DevTables& tb, const PairPlan& pl, const T2* Vh,
                       const T* Vp, const T* Lam, T* Sh, T2* tmp, T* Pa, const int* didx, int P,
                       T* Q) {
    const HostTables& h = tb.h;
    hipStream_t s = ctx->stream;
    const int rb = (int)pl.bidx.size();
    const long nfields = (long)rb * h.nbp;
    const long batch = std::min<long>(nfields, 512);
    g_stage = "carl.filter";
    bool fused = false;
    if constexpr (sizeof(T) == 4 && D == 3)
      if (!pl.generic_only) fused = carleman_filter_f32(ctx, tb, (const float2*)Vh, (float*)Sh, rb);
    for (long f0 = 0; !fused && f0 < nfields; f0 += batch) {
      const long nb = std::min(batch, nfields - f0);
      transform<T, N, D, +1>(s, LdFilter<T>{Vh, (const T2*)tb.filt, n, h.nbp, f0},
                             StShiftSplit<T>{Sh, tb.bp_b, tb.bp_bb, n, 1, h.nbp, h.msig, f0}, tmp,
                             nb);
    }
    bool diag_only = false;
    const int Gt = sizeof(T) == 4 ? 12 : 8;
    const bool self = self_only(pl);
    if (self)
      sigma_self(s, "carl.sigma_self", Sh, Pa, didx, (const T*)tb.wbp, tb.bp_b, tb.bp_bb, 1, h.msig,
                 h.nbp, 0, P);
    auto tiles = self ? std::vector<ReduceTile>{} : plan_tiles(rb, pl.li, pl.lj, Gt, diag_only);
    for (const auto& t : tiles) {
      const bool diag = t.bi[0] == t.bj[0];
      const int bs = 64;
      const dim3 grid((n + bs - 1) / bs);
      int nvalid = 0;
      for (int k = 0; k < 256; ++k) nvalid += t.out[k] >= 0;
      const int nload = diag ? 2 * t.ni : 2 * (t.ni + t.nj);
      TimedScope ts(s, "carl.sigma_reduce", (double)n * (nload * h.nbp + nvalid) * sizeof(T));
      if (sizeof(T) == 4) {
        if (diag)
          hipLaunchKernelGGL((k_sigma_reduce<T, 12, true>), grid, dim3(bs), 0, s, Sh, Pa, t,
                             (const T*)tb.wbp, tb.bp_b, tb.bp_bb, n, 1, h.msig, h.nbp, 0, 0L);
        else
          hipLaunchKernelGGL((k_sigma_reduce<T, 12, false>), grid, dim3(bs), 0, s, Sh, Pa, t,
                             (const T*)tb.wbp, tb.bp_b, tb.bp_bb, n, 1, h.msig, h.nbp, 0, 0L);
      } else {
        if (diag)
          hipLaunchKernelGGL((k_sigma_reduce<T, 8, true>), grid, dim3(bs), 0, s, Sh, Pa, t,
                             (const T*)tb.wbp, tb.bp_b, tb.bp_bb, n, 1, h.msig, h.nbp, 0, 0L);
        else
          hipLaunchKernelGGL((k_sigma_reduce<T, 8, false>), grid, dim3(bs), 0, s, Sh, Pa, t,
                             (const T*)tb.wbp, tb.bp_b, tb.bp_bb, n, 1, h.msig, h.nbp, 0, 0L);
      }
      BLR_CHECK_LAUNCH();
    }
    TimedScope ts(s, "carl.final", (double)P * n * 6 * sizeof(T));
    hipLaunchKernelGGL((k_carleman_final<T>), dim3((n + 255) / 256, P), dim3(256), 0, s, Pa, Vp, Lam,
                       didx, didx + P, didx + 2 * P, n, Q);
    BLR_CHECK_LAUNCH();
  }

  // Q rows prow[p] receive Q_s(bidx[li[p]], bidx[lj[p]]) of the compact basis Vc.
  static void run(blr_ctx ctx, const DevTables& tb, const T* Vsrc, const PairPlan& pl,
                  const std::vector<int>& prow, T* Q) {
    const HostTables& h = tb.h;
    hipStream_t s = ctx->stream;
    const int rb = (int)pl.bidx.size();
    const int P = (int)pl.li.size();
    const long nc = P;
    const long shift_fields = (long)rb * h.mrho * h.nbp;
    const long batch = std::min<long>(shift_fields, 512);
    const std::string tag = std::string("gen") + (sizeof(T) == 4 ? "f" : "d");
    T* Sh = (T*)ctx->buf(tag + ".Sh", (size_t)rb * h.mrho * h.msig * n * sizeof(T));
    // the isotropic form keeps the products of a chunk of radial nodes
    const long cr = (h.carleman || h.aniso_n > 0) ? 1 : radial_chunk(h.mrho, nc, n, sizeof(T));
    T2* tmp = (T2*)ctx->buf(
        tag + ".tmp", (size_t)std::max<long>(batch, std::max<long>(cr * nc, 2 * rb)) * n * sizeof(T2));
    T* Pa = (T*)ctx->buf(tag + ".Pa", (size_t)cr * P * n * sizeof(T));
    T2* G = h.carleman ? nullptr : (T2*)ctx->buf(tag + ".G", (size_t)nc * n * sizeof(T2));
    // per-call index arrays (pi, pj, prow) through the pinned stage
    std::vector<int> idx(3 * P);
    for (int p = 0; p < P; ++p) {
      idx[p] = pl.li[p];
      idx[P + p] = pl.lj[p];
      idx[2 * P + p] = prow[p];
    }
    int* didx = (int*)ctx->upload(tag + ".idx", idx.data(), idx.size() * sizeof(int));
    const T2* phase = (const T2*)tb.phase;
    const T* fw = (const T*)tb.fw;
    // 1. spectra, projected basis and loss fields
    T2* Vh;
    T* Vp;
    T* Lam;
    basis(ctx, tb, Vsrc, pl, &Vh, &Vp, &Lam);
    if (h.carleman) {
      carleman(ctx, tb, pl, Vh, Vp, Lam, Sh, tmp, Pa, didx, P, Q);
      return;
    }
    // 2. shifts
    g_stage = "gen.shift";
    for (long f0 = 0; f0 < shift_fields; f0 += batch) {
      const long nb = std::min(batch, shift_fields - f0);
      transform<T, N, D, +1>(s, LdShift<T, N, D>{Vh, phase, n, h.mrho, h.nbp, f0},
                             StShiftSplit<T>{Sh, tb.bp_b, tb.bp_bb, n, h.mrho, h.nbp, h.msig, f0},
                             tmp, nb);
    }
    // 3-4. sigma sums, transforms and radial weights, one radial node at a time
    fill<T>(s, (T*)G, 2 * nc * n, T(0));
    bool diag_only = false;
    const int Gt = (sizeof(T) == 4 || (h.aniso_n == 0 && wide_tiles64(rb))) ? 12 : 8;
    const bool self = self_only(pl);
    auto tiles = self ? std::vector<ReduceTile>{} : plan_tiles(rb, pl.li, pl.lj, Gt, diag_only);
    g_stage = "gen.pairfft";
    if (h.aniso_n > 0) {
      // anisotropic kernel: each antipodal pair's product is transformed and
      // weighted by its own table (the sigma sum happens in Fourier space)
      const T* atab = (const T*)tb.atab;
      for (int a = 0; a < h.mrho; ++a)
        for (int bp = 0; bp < h.nbp; ++bp) {
          if (self)
            sigma_self(s, "gen.sigma_pair", Sh, Pa, didx, (const T*)tb.wbp + bp, tb.bp_b + bp,
                       tb.bp_bb + bp, h.mrho, h.msig, 1, a, P);
          for (const auto& t : tiles) {
            const bool diag = t.bi[0] == t.bj[0];
            const dim3 grid((n + 255) / 256);
            int nvalid = 0;
            for (int k = 0; k < 256; ++k) nvalid += t.out[k] >= 0;
            const int nload = diag ? 2 * t.ni : 2 * (t.ni + t.nj);
            TimedScope ts(s, "gen.sigma_pair", (double)n * (nload + nvalid) * sizeof(T));
            const T* w1 = (const T*)tb.wbp + bp;
            if (sizeof(T) == 4) {
              if (diag)
                hipLaunchKernelGGL((k_sigma_reduce<T, 12, true>), grid, dim3(256), 0, s, Sh, Pa, t,
                                   w1, tb.bp_b + bp, tb.bp_bb + bp, n, h.mrho, h.msig, 1, a, 0L);
              else
                hipLaunchKernelGGL((k_sigma_reduce<T, 12, false>), grid, dim3(256), 0, s, Sh, Pa,
                                   t, w1, tb.bp_b + bp, tb.bp_bb + bp, n, h.mrho, h.msig, 1, a, 0L);
            } else {
              if (diag)
                hipLaunchKernelGGL((k_sigma_reduce<T, 8, true>), grid, dim3(256), 0, s, Sh, Pa, t,
                                   w1, tb.bp_b + bp, tb.bp_bb + bp, n, h.mrho, h.msig, 1, a, 0L);
              else
                hipLaunchKernelGGL((k_sigma_reduce<T, 8, false>), grid, dim3(256), 0, s, Sh, Pa, t,
                                   w1, tb.bp_b + bp, tb.bp_bb + bp, n, h.mrho, h.msig, 1, a, 0L);
            }
            BLR_CHECK_LAUNCH();
          }
          transform<T, N, D, -1>(s, LdPair1<T>{Pa, n},
                                 StAccumTab<T>{G, atab + ((size_t)a * h.nbp + bp) * n, n}, tmp, nc);
        }
    }
    // radial nodes in chunks of ca: the sums of a chunk in one launch per
    // tile, the first axes of its pair transforms in one pass, the last axis
    // with the radial weights node after node in one more
    const int ca = radial_chunk(h.mrho, nc, n, sizeof(T));
    for (int a0 = 0; a0 < h.mrho && h.aniso_n == 0; a0 += ca) {
      const int na = std::min(ca, h.mrho - a0);
      if (self)
        sigma_self(s, "gen.sigma_self", Sh, Pa, didx, (const T*)tb.wbp, tb.bp_b, tb.bp_bb, h.mrho,
                   h.msig, h.nbp, a0, P, na);
      for (const auto& t : tiles) {
        const bool diag = t.bi[0] == t.bj[0];
        const int bs = 64;  // more workgroups than CUs even at 32^3
        const dim3 grid((n + bs - 1) / bs, na);
        const long ps = (long)P * n;
        int nvalid = 0;
        for (int k = 0; k < 256; ++k) nvalid += t.out[k] >= 0;
        const int nload = diag ? 2 * t.ni : 2 * (t.ni + t.nj);
        TimedScope ts(s, "gen.sigma_reduce",
                      (double)n * na * (nload * h.nbp + nvalid) * sizeof(T));
        if (Gt == 12) {
          if (diag)
            hipLaunchKernelGGL((k_sigma_reduce<T, 12, true>), grid, dim3(bs), 0, s, Sh, Pa, t,
                               (const T*)tb.wbp, tb.bp_b, tb.bp_bb, n, h.mrho, h.msig, h.nbp, a0,
                               ps);
          else
            hipLaunchKernelGGL((k_sigma_reduce<T, 12, false>), grid, dim3(bs), 0, s, Sh, Pa, t,
                               (const T*)tb.wbp, tb.bp_b, tb.bp_bb, n, h.mrho, h.msig, h.nbp, a0,
                               ps);
        } else {
          if (diag)
            hipLaunchKernelGGL((k_sigma_reduce<T, 8, true>), grid, dim3(bs), 0, s, Sh, Pa, t,
                               (const T*)tb.wbp, tb.bp_b, tb.bp_bb, n, h.mrho, h.msig, h.nbp, a0,
                               ps);
          else
            hipLaunchKernelGGL((k_sigma_reduce<T, 8, false>), grid, dim3(bs), 0, s, Sh, Pa, t,
                               (const T*)tb.wbp, tb.bp_b, tb.bp_bb, n, h.mrho, h.msig, h.nbp, a0,
                               ps);
        }
        BLR_CHECK_LAUNCH();
      }
      first_axes<T, N, D, -1>(s, LdPair1<T>{Pa, n}, StComplex<T>{tmp, n}, (long)na * nc);
      accum_radial<T, N, D>(s, tmp, G, fw, h.nkk, nc, a0, na);
    }
    // 5. back to velocity space, minus the loss
    g_stage = "gen.final";
    transform<T, N, D, +1>(s, LdComplex<T>{G, n},
                           StFinal<T>{Q, Vp, Lam, didx, didx + P, didx + 2 * P, n}, tmp, nc);
  }
};

// dispatch over (T, N, D)
template <typename T, class F>
static void dispatch_size(int d, int N, F&& f) {
  if (d == 3) {
    switch (N) {
      case 8: f(std::integral_constant<int, 8>{}, std::integral_constant<int, 3>{}); return;
      case 16: f(std::integral_constant<int, 16>{}, std::integral_constant<int, 3>{}); return;
      case 24: f(std::integral_constant<int, 24>{}, std::integral_constant<int, 3>{}); return;
      case 32: f(std::integral_constant<int, 32>{}, std::integral_constant<int, 3>{}); return;
    }
  } else {
    switch (N) {
      case 16: f(std::integral_constant<int, 16>{}, std::integral_constant<int, 2>{}); return;
      case 32: f(std::integral_constant<int, 32>{}, std::integral_constant<int, 2>{}); return;
    }
  }
  throw Error(BLR_ERR_UNSUPPORTED, "velocity grid size not built");
}


// ------------------------------------------------------------ de-aliasing
// Coarse plain-DFT spectra (N per axis) -> fine spectra (2N per axis): the
// modes k with every component in [-N/2 + 1, N/2 - 1] (the Nyquist planes of
// the coarse grid are dropped) keep their value times `scale`, the rest are 0.
template <typename T, int N, int D>
__global__ void k_pad_spec(const typename Vec2<T>::t* __restrict__ cs, typename Vec2<T>::t* __restrict__ fs,
                           int rows, T scale) {
  constexpr int NF = 2 * N;
  constexpr long nf = D == 2 ? (long)NF * NF : (long)NF * NF * NF;
  constexpr long nc = D == 2 ? (long)N * N : (long)N * N * N;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int row = blockIdx.y;
  if (e >= nf || row >= rows) return;
  long rem = e, src = 0, mul = 1;
  bool in = true;
  for (int ax = D - 1; ax >= 0; --ax) {
    const int i = (int)(rem % NF);
    rem /= NF;
    const int k = i < N ? i : i - NF;  // centred fine mode
    if (k <= -N / 2 || k >= N / 2) in = false;
    src += (long)((k + N) % N) * mul;
    mul *= N;
  }
  typename Vec2<T>::t v = make2<T>(T(0), T(0));
  if (in) {
    v = cs[(long)row * nc + src];
    v.x *= scale;
    v.y *= scale;
  }
  fs[(long)row * nf + e] = v;
}

// Fine plain-DFT spectra -> coarse: the coarse modes without a Nyquist
// component take the fine value at the same centred mode times `scale`.
template <typename T, int N, int D>
__global__ void k_restrict_spec(const typename Vec2<T>::t* __restrict__ fs,
                                typename Vec2<T>::t* __restrict__ cs, int rows, T scale) {
  constexpr int NF = 2 * N;
  constexpr long nf = D == 2 ? (long)NF * NF : (long)NF * NF * NF;
  constexpr long nc = D == 2 ? (long)N * N : (long)N * N * N;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int row = blockIdx.y;
  if (e >= nc || row >= rows) return;
  long rem = e, src = 0, mul = 1;
  bool nyq = false;
  for (int ax = D - 1; ax >= 0; --ax) {
    const int i = (int)(rem % N);
    rem /= N;
    const int k = i < N / 2 ? i : i - N;
    if (k == -N / 2) nyq = true;
    src += (long)((k + NF) % NF) * mul;
    mul *= NF;
  }
  typename Vec2<T>::t v = make2<T>(T(0), T(0));
  if (!nyq) {
    v = fs[(long)row * nf + src];
    v.x *= scale;
    v.y *= scale;
  }
  cs[(long)row * nc + e] = v;
}

template <typename T>
__global__ void k_scatter_rows(const T* __restrict__ src, const int* __restrict__ prow, long n,
                               T* __restrict__ dst) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (e < n) dst[(long)prow[p] * n + e] = src[(long)p * n + e];
}

template <typename T>
static void run_pairs(blr_ctx ctx, const DevTables& tb, const T* V, int r, const int32_t* pairs,
                      int npairs, T* Q, uint32_t flags);

__device__ __forceinline__ void sincospi_t(float x, float* sn, float* cs) { sincospif(x, sn, cs); }
__device__ __forceinline__ void sincospi_t(double x, double* sn, double* cs) { sincospi(x, sn, cs); }

// sum of the centred modes k_ax over the axes ax in the bit set s (bit ax set:
// the grid is shifted by half a cell along axis ax; axis 0 outermost)
template <int N, int D>
__device__ __forceinline__ int shifted_mode_sum(int e, int sbits) {
  int m = 0;
#pragma unroll
  for (int ax = D - 1; ax >= 0; --ax) {
    if ((sbits >> ax) & 1) m += ctr<N>(e % N);
    e /= N;
  }
  return m;
}

// V^_f exp(i pi (k.s) / N): the spectrum whose inverse transform samples the
// interpolant at v_q + s dv / 2
template <typename T, int N, int D>
struct LdPhase {
  static constexpr int bpe = 2;  // algorithmic bytes per element / sizeof(T)
  const typename Vec2<T>::t* vh;
  int n, sbits;
  template <int NN>
  __device__ void load(long f, int base, int stride, T (&re)[NN], T (&im)[NN]) const {
    const auto* q = vh + f * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int m = shifted_mode_sum<N, D>(base + j * stride, sbits);
      T sn, cs;
      sincospi_t(T(m) / T(N), &sn, &cs);
      const auto v = q[(long)j * stride];
      re[j] = v.x * cs - v.y * sn;
      im[j] = v.x * sn + v.y * cs;
    }
  }
};

// acc (+)= scale X_k exp(-i pi (k.s) / N); modes with a Nyquist component 0
template <typename T, int N, int D>
struct StDephase {
  static constexpr int bpe = 4;  // algorithmic bytes per element / sizeof(T)
  typename Vec2<T>::t* acc;
  int n, sbits;
  T scale;
  int first;
  template <int NN>
  __device__ void store(long f, int base, int stride, const T (&re)[NN], const T (&im)[NN]) const {
    auto* a = acc + f * n + base;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int e = base + j * stride;
      bool nyq = false;
      int r = e;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        nyq = nyq || (r % N == N / 2);
        r /= N;
      }
      typename Vec2<T>::t v = make2<T>(T(0), T(0));
      if (!nyq) {
        T sn, cs;
        sincospi_t(T(shifted_mode_sum<N, D>(e, sbits)) / T(N), &sn, &cs);
        if (!first) v = a[(long)j * stride];
        v.x += (re[j] * cs + im[j] * sn) * scale;
        v.y += (im[j] * cs - re[j] * sn) * scale;
      }
      a[(long)j * stride] = v;
    }
  }
};

// BLR_DEALIAS from 2^D evaluations on the N-point grid: for every subset s of
// the axes, the pipeline (circular products, no projection) run on the
// samples of the interpolants at v_q + s dv / 2, whose output spectrum, once
// the shift's phase is taken off, holds each exact mode k plus its wraps
// k + jN weighted by (-1)^(j.s).  Two inputs without Nyquist modes give
// products with |k_i| <= N - 2, so every wrap has |j_i| <= 1 and the mean over
// the 2^D subsets keeps j = 0 alone: the exact Galerkin sum over l + m = k,
// without a grid of 2N points.  Then the modes without Nyquist components,
// back to the grid, and the optional projection.
template <typename T, int N, int D>
static void run_dealias_shift(blr_ctx ctx, const DevTables& tb, const T* V, int r,
                              const int32_t* pairs, int npairs, T* Q, uint32_t flags) {
  using T2 = typename Vec2<T>::t;
  constexpr long n = D == 2 ? (long)N * N : (long)N * N * N;
  hipStream_t s = ctx->stream;
  const PairPlan pl = make_plan(r, pairs, npairs);
  const int rb = (int)pl.bidx.size(), P = (int)pl.li.size();
  const std::string tag = std::string("dsh") + (sizeof(T) == 4 ? "f" : "d");
  T2* vh = (T2*)ctx->buf(tag + ".vh", (size_t)rb * n * sizeof(T2));
  T2* tc = (T2*)ctx->buf(tag + ".tc", (size_t)std::max(rb, P) * n * sizeof(T2));
  T2* acc = (T2*)ctx->buf(tag + ".acc", (size_t)P * n * sizeof(T2));
  T* Vs = (T*)ctx->buf(tag + ".Vs", (size_t)rb * n * sizeof(T));
  T* Qs = (T*)ctx->buf(tag + ".Qs", (size_t)P * n * sizeof(T));
  g_stage = "dealias.spec";
  transform_rows<T, N, D, -1>(s, V, pl.bidx, StBasisSpec<T, N, D>{vh, (int)n, T(1) / T(n)}, tc);
  std::vector<int32_t> cp(2 * (size_t)P);
  for (int p = 0; p < P; ++p) {
    cp[2 * p] = pl.li[p];
    cp[2 * p + 1] = pl.lj[p];
  }
  const uint32_t sub = (flags & ~(uint32_t)BLR_DEALIAS) | BLR_NO_CONSERVE;
  const T scale = T(1) / (T(n) * T(1 << D));
  for (int sb = 0; sb < (1 << D); ++sb) {
    g_stage = "dealias.shift";
    transform<T, N, D, +1>(s, LdPhase<T, N, D>{vh, (int)n, sb}, StRe<T>{Vs, (int)n}, tc, rb);
    run_pairs<T>(ctx, tb, Vs, rb, cp.data(), P, Qs, sub);
    g_stage = "dealias.unshift";
    transform<T, N, D, -1>(s, LdReal<T>{Qs, (int)n}, StDephase<T, N, D>{acc, (int)n, sb, scale, sb == 0},
                           tc, P);
  }
  g_stage = "dealias.out";
  transform<T, N, D, +1>(s, LdComplex<T>{acc, (int)n}, StRe<T>{Qs, (int)n}, tc, P);
  int* drow = (int*)ctx->upload(tag + ".row", pl.row.data(), pl.row.size() * sizeof(int));
  hipLaunchKernelGGL((k_scatter_rows<T>), dim3((unsigned)((n + 255) / 256), P), dim3(256), 0, s, Qs,
                     drow, n, Q);
  BLR_CHECK_LAUNCH();
  for (const auto& dp : pl.dup)
    BLR_HIP(hipMemcpyAsync(Q + (size_t)dp.first * n, Q + (size_t)dp.second * n, (size_t)n * sizeof(T),
                           hipMemcpyDeviceToDevice, s));
  if (!(flags & BLR_NO_CONSERVE)) conserve_rows<T>(ctx, tb.h, Q, npairs);
}

// BLR_DEALIAS: the band-limited interpolants of the basis functions on the
// grid of 2N points per axis (same box, same quadrature), the pair operator
// there without the projection (sums of two input modes never wrap on that
// grid, so its circular convolution is the exact Galerkin sum), then the
// output modes of the N-point mode set without Nyquist components.
template <typename T, int N, int D>
static void run_dealias(blr_ctx ctx, const blr_vgrid& vg, int prec, const DevTables& tb, const T* V,
                        int r, const int32_t* pairs, int npairs, T* Q, uint32_t flags) {
  using T2 = typename Vec2<T>::t;
  constexpr int NF = 2 * N;
  constexpr long n = D == 2 ? (long)N * N : (long)N * N * N;
  constexpr long nf = D == 2 ? (long)NF * NF : (long)NF * NF * NF;
  hipStream_t s = ctx->stream;
  const PairPlan pl = make_plan(r, pairs, npairs);
  const int rb = (int)pl.bidx.size(), P = (int)pl.li.size();
  const std::string tag = std::string("dea") + (sizeof(T) == 4 ? "f" : "d");
  T2* cs = (T2*)ctx->buf(tag + ".cs", (size_t)std::max(rb, P) * n * sizeof(T2));
  T2* tc = (T2*)ctx->buf(tag + ".tc", (size_t)std::max(rb, P) * n * sizeof(T2));
  T2* fs = (T2*)ctx->buf(tag + ".fs", (size_t)std::max(rb, P) * nf * sizeof(T2));
  T2* tf = (T2*)ctx->buf(tag + ".tf", (size_t)std::max(rb, P) * nf * sizeof(T2));
  T* Vf = (T*)ctx->buf(tag + ".Vf", (size_t)rb * nf * sizeof(T));
  T* Qf = (T*)ctx->buf(tag + ".Qf", (size_t)P * nf * sizeof(T));
  T* Qc = (T*)ctx->buf(tag + ".Qc", (size_t)P * n * sizeof(T));
  g_stage = "dealias.pad";
  transform_rows<T, N, D, -1>(s, V, pl.bidx, StComplex<T>{cs, (int)n}, tc);
  hipLaunchKernelGGL((k_pad_spec<T, N, D>), dim3((unsigned)((nf + 255) / 256), rb), dim3(256), 0, s,
                     cs, fs, rb, T(1) / T(n));
  BLR_CHECK_LAUNCH();
  transform<T, NF, D, +1>(s, LdComplex<T>{fs, (int)nf}, StRe<T>{Vf, (int)nf}, tf, rb);
  // the pair operator on the fine grid, compact pairs, no projection
  blr_vgrid fg = vg;
  fg.n = NF;
  fg.R = tb.h.R;
  fg.flags = (vg.flags & ~(uint32_t)BLR_DEALIAS) | BLR_NO_CONSERVE;
  std::vector<int32_t> cp(2 * (size_t)P);
  for (int p = 0; p < P; ++p) {
    cp[2 * p] = pl.li[p];
    cp[2 * p + 1] = pl.lj[p];
  }
  const DevTables& tbf = get_tables(ctx, fg, prec);
  run_pairs<T>(ctx, tbf, Vf, rb, cp.data(), P, Qf, fg.flags);
  g_stage = "dealias.restrict";
  transform<T, NF, D, -1>(s, LdReal<T>{Qf, (int)nf}, StComplex<T>{fs, (int)nf}, tf, P);
  hipLaunchKernelGGL((k_restrict_spec<T, N, D>), dim3((unsigned)((n + 255) / 256), P), dim3(256), 0,
                     s, fs, cs, P, T(1) / T(nf));
  BLR_CHECK_LAUNCH();
  transform<T, N, D, +1>(s, LdComplex<T>{cs, (int)n}, StRe<T>{Qc, (int)n}, tc, P);
  int* drow = (int*)ctx->upload(tag + ".row", pl.row.data(), pl.row.size() * sizeof(int));
  hipLaunchKernelGGL((k_scatter_rows<T>), dim3((unsigned)((n + 255) / 256), P), dim3(256), 0, s, Qc,
                     drow, n, Q);
  BLR_CHECK_LAUNCH();
  for (const auto& dp : pl.dup)
    BLR_HIP(hipMemcpyAsync(Q + (size_t)dp.first * n, Q + (size_t)dp.second * n, (size_t)n * sizeof(T),
                           hipMemcpyDeviceToDevice, s));
  if (!(flags & BLR_NO_CONSERVE)) conserve_rows<T>(ctx, tb.h, Q, npairs);
}

template <typename T>
static void run_pairs(blr_ctx ctx, const DevTables& tb, const T* V, int r, const int32_t* pairs,
                      int npairs, T* Q, uint32_t flags) {
  const HostTables& h = tb.h;
  if (npairs == 0) return;
  if (flags & BLR_PLAIN_SCHEDULE) {
    // the baseline schedule: every pair on its own, shifts recomputed per pair
    for (int p = 0; p < npairs; ++p) {
      PairPlan pl = make_plan(r, pairs + 2 * p, 1);
      pl.generic_only = (flags & BLR_GENERIC_FFT) != 0;
      std::vector<int> prow{p};
      dispatch_size<T>(h.d, h.N, [&](auto Nc, auto Dc) {
        Generic<T, decltype(Nc)::value, decltype(Dc)::value>::run(ctx, tb, V, pl, prow, Q);
      });
    }
  } else {
    PairPlan pl = make_plan(r, pairs, npairs);
    pl.generic_only = (flags & BLR_GENERIC_FFT) != 0;
    const std::vector<int>& prow = pl.row;
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (!(flags & BLR_GENERIC_FFT) && !h.carleman && h.aniso_n == 0)
        done = fast_collision_f32(ctx, tb, V, pl, prow, Q, !(flags & BLR_NO_CONSERVE));
    }
    if (!done) {
      dispatch_size<T>(h.d, h.N, [&](auto Nc, auto Dc) {
        Generic<T, decltype(Nc)::value, decltype(Dc)::value>::run(ctx, tb, V, pl, prow, Q);
      });
      if (!(flags & BLR_NO_CONSERVE)) {
        if (pl.dup.empty())
          conserve_rows<T>(ctx, h, Q, npairs);
        else
          for (int p : prow) conserve_rows<T>(ctx, h, Q + (size_t)p * h.n, 1);
      }
    }
    for (const auto& dp : pl.dup)
      BLR_HIP(hipMemcpyAsync(Q + (size_t)dp.first * h.n, Q + (size_t)dp.second * h.n,
                             (size_t)h.n * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
    return;
  }
  if (!(flags & BLR_NO_CONSERVE)) conserve_rows<T>(ctx, h, Q, npairs);
}

static size_t up256(size_t b) { return (std::max<size_t>(b, 256) + 255) / 256 * 256; }

size_t table_bytes(const HostTables& h, int prec) {
  const size_t T = prec == BLR_FP32 ? 4 : 8;
  size_t b = up256(h.phase.size() * T) + up256(h.fw.size() * T) + up256(h.gloss.size() * T) +
             up256((size_t)h.nbp * T) + 2 * up256((size_t)h.nbp * sizeof(int));
  if (h.carleman) b += up256(h.filt.size() * T);
  if (h.aniso_n > 0) b += up256(h.atab.size() * T);
  return b;
}

// Mirrors the buf()/upload() requests of collision_pairs below (basis
// spectra, shifts, products, spectra, index arrays, moment partial sums).
size_t collision_call_bytes(const HostTables& h, int prec, int r, const int32_t* pairs, int npairs,
                            uint32_t flags) {
  if (npairs == 0) return 0;
  const size_t T = prec == BLR_FP32 ? 4 : 8, T2 = 2 * T;
  const size_t n = h.n;
  size_t b = table_bytes(h, prec);
  auto generic = [&](size_t rb, size_t P) {
    size_t g = up256(rb * n * T2) + up256(2 * rb * n * T) + up256(2 * rb * n * T2);  // basis
    const size_t shift_fields = rb * h.mrho * h.nbp;
    const size_t batch = std::min<size_t>(shift_fields, 512);
    g += up256(rb * h.mrho * h.msig * n * T);                                // shifts
    const size_t cr =
        (h.carleman || h.aniso_n > 0) ? 1 : (size_t)radial_chunk(h.mrho, (long)P, (long)n, T);
    g += up256(std::max(batch, std::max(cr * P, 2 * rb)) * n * T2);         // transforms
    g += up256(cr * P * n * T);                                              // products
    if (!h.carleman) g += up256(P * n * T2);                                 // spectra
    return g;
  };
  if (flags & BLR_PLAIN_SCHEDULE) {
    // one pair at a time: one- and two-function calls reuse their slices;
    // every pair uploads its own index array
    b += generic(1, 1) + generic(2, 1) + (size_t)npairs * up256(3 * sizeof(int));
  } else {
    PairPlan pl = make_plan(r, pairs, npairs);
    const size_t rb = pl.bidx.size(), P = pl.li.size();
    const bool fast = prec == BLR_FP32 && !(flags & BLR_GENERIC_FFT) && !h.carleman &&
                      h.aniso_n == 0 && h.d == 3 &&
                      (h.N == 16 || h.N == 24 || h.N == 32) && rb <= 64 && h.msig == 38;
    if (fast) {
      const size_t N = h.N, H = N / 2 + 1;
      b += up256(rb * n * 8) + up256(2 * rb * n * 4) + up256(2 * rb * n * 8);  // basis
      b += up256(rb * h.mrho * h.msig * n * 4);                                // shifts
      b += up256((size_t)h.mrho * P * n * 4);                                  // products
      b += up256(P * h.mrho * N * N * H * 8);  // half spectra: at most one group per node
    } else {
      b += generic(rb, P);
    }
    b += up256(3 * P * sizeof(int));
  }
  if (!(flags & BLR_NO_CONSERVE)) {
    const size_t nb = (n + kMomChunk - 1) / kMomChunk;
    b += up256((size_t)npairs * nb * 5 * sizeof(double));
  }
  return b;
}

static void collision_pairs_impl(blr_ctx ctx, const blr_vgrid& vg, int prec, const void* V, int r,
                                 const int32_t* pairs, int npairs, void* Q);

void collision_pairs(blr_ctx ctx, const blr_vgrid& vg, int prec, const void* V, int r,
                     const int32_t* pairs, int npairs, void* Q) {
  require(r >= 1 && r <= 64, "r must be in [1, 64]");
  collision_pairs_impl(ctx, vg, prec, V, r, pairs, npairs, Q);
}

bool fused_f32_grid(const blr_vgrid& vg) {
  const int ms = vg.m_sigma ? vg.m_sigma : (vg.d == 2 ? 8 : 38);
  return vg.d == 3 && (vg.n == 16 || vg.n == 24 || vg.n == 32) && ms == 38 && vg.aniso_n == 0 &&
         !(vg.flags & (BLR_CARLEMAN | BLR_DEALIAS | BLR_GENERIC_FFT | BLR_PLAIN_SCHEDULE));
}

void collision_batch(blr_ctx ctx, const blr_vgrid& vg, const std::vector<BatchJob>& jobs) {
  const HostTables& h = get_tables(ctx, vg, BLR_FP32).h;
  const size_t n = h.n;
  hipStream_t s = ctx->stream;
  size_t j0 = 0;
  while (j0 < jobs.size()) {
    // the next jobs whose bases and pairs fit one launch sequence
    size_t j1 = j0;
    int rt = 0, pt = 0;
    while (j1 < jobs.size()) {
      const int r = jobs[j1].r, P = (int)jobs[j1].pairs.size() / 2;
      require(r >= 1 && r <= 64 && P >= 1 && P <= 4096, "collision batch: job out of range");
      if (j1 > j0 && (rt + r > 64 || pt + P > 4096)) break;
      rt += r;
      pt += P;
      ++j1;
    }
    float* Vc = (float*)ctx->buf("bat.V", (size_t)rt * n * sizeof(float));
    float* Qc = (float*)ctx->buf("bat.Q", (size_t)pt * n * sizeof(float));
    std::vector<int32_t> pc;
    pc.reserve(2 * (size_t)pt);
    int roff = 0;
    for (size_t j = j0; j < j1; ++j) {
      const BatchJob& b = jobs[j];
      BLR_HIP(hipMemcpyAsync(Vc + (size_t)roff * n, b.V, (size_t)b.r * n * sizeof(float),
                             hipMemcpyDeviceToDevice, s));
      for (size_t k = 0; k < b.pairs.size(); ++k) {
        require(b.pairs[k] >= 0 && b.pairs[k] < b.r, "collision batch: pair index out of range");
        pc.push_back(b.pairs[k] + roff);
      }
      roff += b.r;
    }
    collision_pairs(ctx, vg, BLR_FP32, Vc, rt, pc.data(), pt, Qc);
    int poff = 0;
    for (size_t j = j0; j < j1; ++j) {
      const BatchJob& b = jobs[j];
      const int P = (int)b.pairs.size() / 2;
      BLR_HIP(hipMemcpyAsync(b.Q, Qc + (size_t)poff * n, (size_t)P * n * sizeof(float),
                             hipMemcpyDeviceToDevice, s));
      poff += P;
    }
    j0 = j1;
  }
}

void collision_self(blr_ctx ctx, const blr_vgrid& vg, int prec, const void* V, int rows, void* Q) {
  require(rows >= 1 && rows <= kMaxSelfRows, "collision_self: rows out of range");
  std::vector<int32_t> pairs(2 * (size_t)rows);
  for (int i = 0; i < rows; ++i) pairs[2 * i] = pairs[2 * i + 1] = i;
  collision_pairs_impl(ctx, vg, prec, V, rows, pairs.data(), rows, Q);
}

static void collision_pairs_impl(blr_ctx ctx, const blr_vgrid& vg, int prec, const void* V, int r,
                                 const int32_t* pairs, int npairs, void* Q) {
  g_timer = &ctx->timer;
  require(npairs >= 0 && npairs <= 4096, "npairs must be in [0, 4096]");
  require(npairs == 0 || (pairs && V && Q), "null pointer argument");
  const DevTables& tb = get_tables(ctx, vg, prec);
  if ((vg.flags & BLR_DEALIAS) && npairs > 0) {
    auto go = [&](auto Tc) {
      using T = decltype(Tc);
      if (vg.d == 3 && vg.n == 8)
        run_dealias<T, 8, 3>(ctx, vg, prec, tb, (const T*)V, r, pairs, npairs, (T*)Q, vg.flags);
      else if (vg.d == 3 && vg.n == 16)
        run_dealias<T, 16, 3>(ctx, vg, prec, tb, (const T*)V, r, pairs, npairs, (T*)Q, vg.flags);
      else if (vg.d == 2 && vg.n == 16)
        run_dealias<T, 16, 2>(ctx, vg, prec, tb, (const T*)V, r, pairs, npairs, (T*)Q, vg.flags);
      else
        dispatch_size<T>(vg.d, vg.n, [&](auto Nc, auto Dc) {
          run_dealias_shift<T, decltype(Nc)::value, decltype(Dc)::value>(
              ctx, tb, (const T*)V, r, pairs, npairs, (T*)Q, vg.flags);
        });
    };
    if (prec == BLR_FP32) go(float{});
    else go(double{});
    return;
  }
  if (prec == BLR_FP32)
    run_pairs<float>(ctx, tb, (const float*)V, r, pairs, npairs, (float*)Q, vg.flags);
  else
    run_pairs<double>(ctx, tb, (const double*)V, r, pairs, npairs, (double*)Q, vg.flags);
}

void basis_spectra_f32(blr_ctx ctx, const DevTables& tb, const float* V, const PairPlan& pl,
                       float2** Vh, float** Vp, float** Lam) {
  dispatch_size<float>(tb.h.d, tb.h.N, [&](auto Nc, auto Dc) {
    Generic<float, decltype(Nc)::value, decltype(Dc)::value>::basis(ctx, tb, V, pl, Vh, Vp, Lam);
  });
}

size_t collision_workspace_bytes(const blr_vgrid& vg, int r, int prec) {
  // the estimate needs only the tables' shapes, but building them takes the
  // host a good fraction of a second at 32^3: one build per grid (a server
  // estimates every request it admits)
  static std::mutex mu;
  // d, N, mrho, msig, nbp, carleman, aniso_n
  static std::map<std::string, std::array<int, 7>> shapes;
  std::string key((const char*)&vg, sizeof(vg));
  HostTables h;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = shapes.find(key);
    if (it == shapes.end()) {
      const HostTables t = build_tables(vg);
      it = shapes.emplace(key, std::array<int, 7>{t.d, t.N, t.mrho, t.msig, t.nbp,
                                                  t.carleman ? 1 : 0, t.aniso_n}).first;
    }
    h.d = it->second[0];
    h.N = it->second[1];
    h.mrho = it->second[2];
    h.msig = it->second[3];
    h.nbp = it->second[4];
    h.carleman = it->second[5] != 0;
    h.aniso_n = it->second[6];
  }
  const int P = r * (r + 1) / 2;
  size_t out = 0;
  auto f = [&](auto Tc) {
    using T = decltype(Tc);
    dispatch_size<T>(h.d, h.N, [&](auto Nc, auto Dc) {
      out = Generic<T, decltype(Nc)::value, decltype(Dc)::value>::workspace(h, r, P);
    });
  };
  if (prec == BLR_FP32) f(float{});
  else f(double{});
  return out;
}

}  // namespace blr
