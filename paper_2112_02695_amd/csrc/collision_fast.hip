// Fused FP32 collision kernels for 3D grids n in {16, 24, 32}.
//
// A workgroup of N^2 threads holds one whole N^3 complex field in registers:
// thread t owns one line of N values along the axis being transformed, the
// in-register DFT of fft.hpp transforms it, and the lines are re-dealt between
// the three axis stages through LDS (one real component at a time, rows
// padded to N+1 floats so that both the writes and the reads of every
// exchange are free of bank conflicts).  For N = 32 that is 1024 threads and
// 132 KiB of LDS: one workgroup per CU, the FFT never leaves the CU.
//
// Kernels (same arithmetic as the generic pipeline in collision.hip):
//   k_shift_fused  one antipodal shift pair of one basis function at one
//                  radial node per workgroup iteration: spectrum x
//                  (cos x - sin x) -> 3D inverse DFT W; its real and
//                  imaginary parts (S(b) = Re W - Im W, S(bbar) = Re W + Im W)
//                  written coalesced with streaming stores (the only
//                  HBM-heavy output)
//   k_reduce_diag  sigma sums of all pair products for all radial nodes in
//   k_reduce_all   one launch (thread per grid point, pairs in registers;
//                  the diagonal tile with the sphere pairs in the arguments)
//   k_pair_spec    3D DFTs of one pair product at a group of radial nodes
//                  (two nodes per complex transform), times the radial
//                  weights, summed in registers and written as one half
//                  spectrum (k_2 <= N/2) per group
//   k_final_fused  sum over the groups, 3D inverse DFT from the half
//                  spectrum, minus the loss, FP64 moment projection, store
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "collision_common.hpp"

namespace blr {


namespace fastk {

template <int N>
struct Geo {
  static constexpr int NT = N * N;
  static constexpr int n = N * N * N;
  static constexpr int H = N / 2 + 1;
  static constexpr int LDS = N * N * (N + 1);
};

// element j of the line owned by (u, w) at a stage along axis A
template <int A>
__device__ __forceinline__ void coords(int u, int w, int j, int& i0, int& i1, int& i2) {
  if constexpr (A == 2) {
    i0 = u; i1 = w; i2 = j;
  } else if constexpr (A == 1) {
    i0 = u; i1 = j; i2 = w;
  } else {
    i0 = j; i1 = u; i2 = w;
  }
}

// Ordering of LDS accesses among the lanes of one wavefront (a wave's LDS
// instructions execute in issue order; this keeps the compiler from moving
// them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// An exchange between the stages along axes 1 and 2 stays inside one wave
// when a wave holds whole rows i0 = u (N divides 64: 64 / N values of u per
// wave): both sides then touch only the rows i0 of their own threads.
template <int N, int AF, int AT>
constexpr bool wave_local_exchange() {
  return 64 % N == 0 && AF != 0 && AT != 0;
}

// Re-deal lines from a stage along axis AF to a stage along axis AT.  Across
// waves: a workgroup barrier after the writes and after the reads (the next
// exchange's writes).  Inside a wave: no workgroup barrier; the LDS rows
// written are the wave's own, which no other wave reads or writes between
// the workgroup barriers around them.
template <int N, int AF, int AT>
__device__ __forceinline__ void exchange(float (&v)[N], float* L, int u, int w) {
  constexpr bool local = wave_local_exchange<N, AF, AT>();
#pragma unroll
  for (int j = 0; j < N; ++j) {
    int i0, i1, i2;
    coords<AF>(u, w, j, i0, i1, i2);
    L[(i0 * N + i1) * (N + 1) + i2] = v[j];
  }
  if constexpr (local)
    wave_lds_sync();
  else
    __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) {
    int i0, i1, i2;
    coords<AT>(u, w, j, i0, i1, i2);
    v[j] = L[(i0 * N + i1) * (N + 1) + i2];
  }
  if constexpr (local)
    wave_lds_sync();
  else
    __syncthreads();
}

// ------------------------------------------------------------------ shifts
template <int N>
__global__ __launch_bounds__(N * N) void k_shift_fused(const float2* __restrict__ vh,
                                                       const float2* __restrict__ phase,
                                                       float* __restrict__ sh,
                                                       const int* __restrict__ bp_b,
                                                       const int* __restrict__ bp_bb, int mrho,
                                                       int nbp, int msig, long nfields) {
  __shared__ float L[Geo<N>::LDS];
  constexpr int n = Geo<N>::n;
  const int t = threadIdx.x;
  const int u = t / N, w = t % N;
  // field count < 2^31 (checked by the host): 32-bit index arithmetic
  const int nf = (int)nfields;
  // One workgroup per CU alternates a compute phase (transforms, LDS) with a
  // store phase whose drain the next field's loads wait for; odd workgroups
  // start about 3 us late so that half of the CUs store while the other half
  // compute, instead of all of them storing at once.
  if (blockIdx.x & 1) __builtin_amdgcn_s_sleep(127);
  for (int f = blockIdx.x; f < nf; f += gridDim.x) {
    const int p = f % nbp;
    const int a = (f / nbp) % mrho;
    const int ib = f / (nbp * mrho);
    const float2* ph = phase + (a * nbp + p) * 3 * N;
    // stage along axis 2: thread (k0, k1) = (u, w).  cos x + sin x is the real
    // part of e^{ix} (1 - i): with C = c01 (1 - i), Re(C ph2) = C.x ph2.x - C.y ph2.y
    const float2 c01 = cmul(ph[u], ph[N + w]);
    const float cx = c01.x + c01.y, cy = c01.y - c01.x;
    const float4* src = reinterpret_cast<const float4*>(vh + (long)ib * n + (u * N + w) * N);
    float re[N], im[N];
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const float4 v = src[j];
      const float2 pa = ph[2 * N + 2 * j], pb = ph[2 * N + 2 * j + 1];
      const float fa = cx * pa.x - cy * pa.y, fb = cx * pb.x - cy * pb.y;
      re[2 * j] = v.x * fa;
      im[2 * j] = v.y * fa;
      re[2 * j + 1] = v.z * fb;
      im[2 * j + 1] = v.w * fb;
    }
    fft::dft<float, N, +1>(re, im);
    exchange<N, 2, 1>(re, L, u, w);
    exchange<N, 2, 1>(im, L, u, w);
    fft::dft<float, N, +1>(re, im);
    exchange<N, 1, 0>(re, L, u, w);
    exchange<N, 1, 0>(im, L, u, w);
    fft::dft<float, N, +1>(re, im);
    // thread (i1, i2) = (u, w) holds the line over i0: coalesced stores of
    // Re W into slot b and Im W into slot bbar (read once, by the sigma sums:
    // streaming stores)
    const long base = (((long)ib * mrho + a) * msig) * (long)n + t;
    float* s1 = sh + base + (long)bp_b[p] * n;
    float* s2 = sh + base + (long)bp_bb[p] * n;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      __builtin_nontemporal_store(re[j], s1 + j * N * N);
      __builtin_nontemporal_store(im[j], s2 + j * N * N);
    }
  }
}

// Carleman form: the two filtered fields of one basis function and one
// direction pair per workgroup iteration.  Same transform and stores as
// k_shift_fused; the load multiplies the spectrum by the complex filter
// c_p(k) (table, DFT order) instead of the separable phase factor.
template <int N>
__global__ __launch_bounds__(N * N) void k_filter_fused(const float2* __restrict__ vh,
                                                        const float2* __restrict__ filt,
                                                        float* __restrict__ sh,
                                                        const int* __restrict__ bp_b,
                                                        const int* __restrict__ bp_bb, int nbp,
                                                        int msig, long nfields) {
  __shared__ float L[Geo<N>::LDS];
  constexpr int n = Geo<N>::n;
  const int t = threadIdx.x;
  const int u = t / N, w = t % N;
  const int nf = (int)nfields;  // < 2^31 (checked by the host)
  for (int f = blockIdx.x; f < nf; f += gridDim.x) {
    const int p = f % nbp;
    const int ib = f / nbp;
    const float4* src = reinterpret_cast<const float4*>(vh + (long)ib * n + (u * N + w) * N);
    const float4* cf = reinterpret_cast<const float4*>(filt + (long)p * n + (u * N + w) * N);
    float re[N], im[N];
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const float4 v = src[j];
      const float4 c = cf[j];
      re[2 * j] = v.x * c.x - v.y * c.y;
      im[2 * j] = v.x * c.y + v.y * c.x;
      re[2 * j + 1] = v.z * c.z - v.w * c.w;
      im[2 * j + 1] = v.z * c.w + v.w * c.z;
    }
    fft::dft<float, N, +1>(re, im);
    exchange<N, 2, 1>(re, L, u, w);
    exchange<N, 2, 1>(im, L, u, w);
    fft::dft<float, N, +1>(re, im);
    exchange<N, 1, 0>(re, L, u, w);
    exchange<N, 1, 0>(im, L, u, w);
    fft::dft<float, N, +1>(re, im);
    const long base = ((long)ib * msig) * (long)n + t;
    float* s1 = sh + base + (long)bp_b[p] * n;
    float* s2 = sh + base + (long)bp_bb[p] * n;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      s1[j * N * N] = re[j] - im[j];
      s2[j * N * N] = re[j] + im[j];
    }
  }
}

// ------------------------------------------------------------ sigma sums
// All radial nodes in one launch (blockIdx.y = a); one thread per point.
// The shift kernel leaves x = Re W in slot b and y = Im W in slot bbar of each
// antipodal pair, S(b) = x - y and S(bbar) = x + y, so a pair's term
//   w (S_i(b) S_j(bbar) + S_i(bbar) S_j(b)) = 2 w (x_i x_j - y_i y_j).
template <int G, bool DIAG>
__global__ __launch_bounds__(256) void k_reduce_all(const float* __restrict__ sh,
                                                    float* __restrict__ pa, ReduceTile tile,
                                                    const float* __restrict__ wbp,
                                                    const int* __restrict__ bp_b,
                                                    const int* __restrict__ bp_bb, int n, int mrho,
                                                    int msig, int nbp, int P) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (q >= n) return;
  constexpr int NP = DIAG ? G * (G + 1) / 2 : G * G;
  float acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = 0.f;
  for (int bp = 0; bp < nbp; ++bp) {
    const int b = bp_b[bp], bb = bp_bb[bp];
    const float wt = 2.f * wbp[bp];
    float xi[G], yi[G], xj[G], yj[G];
#pragma unroll
    for (int s = 0; s < G; ++s) {
      float x = 0.f, y = 0.f;
      if (s < tile.ni) {
        const long fi = ((long)tile.bi[s] * mrho + a) * msig;
        x = sh[(fi + b) * n + q];
        y = sh[(fi + bb) * n + q];
      }
      xi[s] = wt * x;
      yi[s] = wt * y;
      if constexpr (DIAG) {
        xj[s] = x;
        yj[s] = y;
      } else {
        x = y = 0.f;
        if (s < tile.nj) {
          const long fj = ((long)tile.bj[s] * mrho + a) * msig;
          x = sh[(fj + b) * n + q];
          y = sh[(fj + bb) * n + q];
        }
        xj[s] = x;
        yj[s] = y;
      }
    }
    int p = 0;
#pragma unroll
    for (int s = 0; s < G; ++s) {
#pragma unroll
      for (int v = DIAG ? s : 0; v < G; ++v) {
        acc[p] += xi[s] * xj[v] - yi[s] * yj[v];
        ++p;
      }
    }
  }
  float* out = pa + (long)a * P * n + q;
  int p = 0;
#pragma unroll
  for (int s = 0; s < G; ++s) {
#pragma unroll
    for (int v = DIAG ? s : 0; v < G; ++v) {
      const int row = tile.out[s * G + v];
      if (row >= 0) out[(long)row * n] = acc[p];
      ++p;
    }
  }
}

// Diagonal tile with the antipodal pairs in the kernel arguments (element
// offsets of the two fields and the weight, uniform registers) and the next
// pair's 2G values loaded while the current pair's products accumulate.
constexpr int kMaxBp = 32;
struct BpArgs {
  int off_b[kMaxBp];
  int off_bb[kMaxBp];
  float w[kMaxBp];
};

template <int G>
__global__ __launch_bounds__(256) void k_reduce_diag(const float* __restrict__ sh,
                                                     float* __restrict__ pa, ReduceTile tile,
                                                     BpArgs bpa, int n, int mrho, int msig,
                                                     int nbp, int P) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (q >= n) return;
  constexpr int NP = G * (G + 1) / 2;
  // field (bi[s], a, sigma) starts at ((bi[s] mrho + a) msig + sigma) n.  Slots
  // s >= ni read basis bi[0]: their sums belong to no output row (out < 0)
  // and are never stored, so no masking is needed.
  const float* base = sh + (long)a * msig * n + q;
  long so[G];
#pragma unroll
  for (int s = 0; s < G; ++s) so[s] = (long)tile.bi[s < tile.ni ? s : 0] * mrho * msig * n;
  float acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = 0.f;
  // the shifted fields are read once: streaming (nontemporal) loads, which
  // measured 15 % faster than cached ones on this launch
  auto load = [&](int b, float(&x)[G], float(&y)[G]) {
#pragma unroll
    for (int s = 0; s < G; ++s) {
      x[s] = __builtin_nontemporal_load(base + so[s] + bpa.off_b[b]);
      y[s] = __builtin_nontemporal_load(base + so[s] + bpa.off_bb[b]);
    }
  };
  auto accum = [&](float wt, const float(&x)[G], const float(&y)[G]) {
    int p = 0;
#pragma unroll
    for (int s = 0; s < G; ++s) {
      const float xs = wt * x[s], ys = wt * y[s];
#pragma unroll
      for (int v = s; v < G; ++v) {
        acc[p] += xs * x[v] - ys * y[v];
        ++p;
      }
    }
  };
  // two register sets alternate (unrolled by two, no copies): the loads of
  // the next sigma pair are in flight while the current one accumulates
  float x0[G], y0[G], x1[G], y1[G];
  load(0, x0, y0);
  int bp = 0;
  for (; bp + 1 < nbp; bp += 2) {
    load(bp + 1, x1, y1);
    accum(bpa.w[bp], x0, y0);
    load(bp + 2 < nbp ? bp + 2 : bp + 1, x0, y0);
    accum(bpa.w[bp + 1], x1, y1);
  }
  if (bp < nbp) accum(bpa.w[bp], x0, y0);
  float* out = pa + (long)a * P * n + q;
  int p = 0;
#pragma unroll
  for (int s = 0; s < G; ++s) {
#pragma unroll
    for (int v = s; v < G; ++v) {
      const int row = tile.out[s * G + v];
      if (row >= 0) out[(long)row * n] = acc[p];
      ++p;
    }
  }
}

// ------------------------------------------------------- pair transforms
// workgroup = (pair p, group g of ga consecutive radial nodes).  Two nodes a,
// b of the group share one complex transform Z = DFT(P_pa + i P_pb); with
// Zc(k) = conj(Z(-k)) (the partner line of thread (-k0, -k1), exchanged
// through LDS) the two real-field spectra are (Z + Zc) / 2 and (Z - Zc) / 2i.
// The two nodes belong to one pair at neighbouring radii, so the magnitudes
// sharing a transform are alike.  w_a(|k|^2)/n times each spectrum is added
// into a register accumulator of the half spectrum k_2 <= N/2, written once
// per group.
template <int N>
__global__ __launch_bounds__(N * N) void k_pair_spec(const float* __restrict__ pa,
                                                     const float* __restrict__ fw,
                                                     float2* __restrict__ wsp, int P, int mrho,
                                                     int nkk, int ga, int ng) {
  constexpr int n = Geo<N>::n, H = Geo<N>::H, NT = Geo<N>::NT;
  // partner exchange: per thread the line elements 0 and N/2 .. N-1 (H values)
  // of both components, rows of 2H + 1 floats (odd: no bank conflicts)
  constexpr int XR = 2 * H + 1;
  constexpr int LSZ = Geo<N>::LDS > NT * XR ? Geo<N>::LDS : NT * XR;
  __shared__ float L[LSZ];
  const int t = threadIdx.x;
  const int u = t / N, w = t % N;
  const int p = blockIdx.x % P;
  const int g = blockIdx.x / P;
  const int a0 = g * ga, a1 = min(mrho, a0 + ga);
  const int k0 = ctr<N>(u), k1 = ctr<N>(w);
  // the thread holding line (-k0, -k1) after the last stage
  const int partner = ((N - u) % N) * N + (N - w) % N;
  float accr[H], acci[H];
#pragma unroll
  for (int j = 0; j < H; ++j) accr[j] = acci[j] = 0.f;
  for (int a = a0; a < a1; a += 2) {
    const bool two = a + 1 < a1;
    // stage along axis 0: thread (i1, i2) = (u, w), coalesced loads
    // uniform field bases, per-thread 32-bit offsets; a lone last node reads
    // its own field twice and drops the copy
    const float* src = pa + ((long)a * P + p) * n;
    const float* src2 = two ? src + (long)P * n : src;
    float re[N], im[N];
    // (the products are read once: streaming loads)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int o = j * N * N + t;
      re[j] = __builtin_nontemporal_load(src + o);
      const float v = __builtin_nontemporal_load(src2 + o);
      im[j] = two ? v : 0.f;
    }
    fft::dft<float, N, -1>(re, im);
    exchange<N, 0, 1>(re, L, u, w);
    exchange<N, 0, 1>(im, L, u, w);
    fft::dft<float, N, -1>(re, im);
    exchange<N, 1, 2>(re, L, u, w);
    exchange<N, 1, 2>(im, L, u, w);
    fft::dft<float, N, -1>(re, im);
    // thread (k0, k1) = (u, w) holds k2 = 0..N-1; keep k2 <= N/2
    // a lone node (im = 0) takes the same path: Zc = Z there, and node b's
    // weight is zero
    const float* fa = fw + (long)a * nkk;
    const float* fb = two ? fa + nkk : fa;
    const float hb = two ? 0.5f : 0.f;
    // Z(-k) for k2 = 0..H-1 is the partner's element (N - j) % N: each thread
    // publishes its elements 0 and N/2 .. N-1 (rows that overlap other
    // waves' rows of the wave-local exchange just done: wait for all waves)
    if constexpr (wave_local_exchange<N, 1, 2>()) __syncthreads();
    float* row = L + t * XR;
    const float* prow = L + partner * XR;
    row[0] = re[0];
    row[H] = im[0];
#pragma unroll
    for (int m = 1; m < H; ++m) {
      row[m] = re[N / 2 + m - 1];
      row[H + m] = im[N / 2 + m - 1];
    }
    __syncthreads();
    float cr[H], ci[H];
    // partner element (N - j) % N sits at slot 0 for j = 0, else N - j - N/2 + 1
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int m = j == 0 ? 0 : N - j - N / 2 + 1;
      cr[j] = prow[m];
      ci[j] = -prow[H + m];
    }
    __syncthreads();
    // weights are fetched here, not during the transform (register pressure)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int k2 = ctr<N>(j);
      const int kk = k0 * k0 + k1 * k1 + k2 * k2;
      const float wa = 0.5f * fa[kk], wb = hb * fb[kk];
      // node a: (Z + Zc) / 2;  node b: (Z - Zc) / 2i = (Im(Z - Zc) - i Re(Z - Zc)) / 2
      const float sr = re[j] + cr[j], si = im[j] + ci[j];
      const float dr = re[j] - cr[j], di = im[j] - ci[j];
      accr[j] += wa * sr + wb * di;
      acci[j] += wa * si - wb * dr;
    }
  }
  float2* dst = wsp + (((long)p * ng + g) * N * N + (long)(u * N + w)) * H;
#pragma unroll
  for (int j = 0; j < H; ++j) dst[j] = make_float2(accr[j], acci[j]);
}

// --------------------------------------------------------------- final
struct FinalArgs {
  double L, dv, w;
  double minv[25];
  int conserve;
};

template <int N>
__global__ __launch_bounds__(N * N) void k_final_fused(const float2* __restrict__ wsp,
                                                       const float* __restrict__ vp,
                                                       const float* __restrict__ lam,
                                                       const int* __restrict__ pidx, float* Q,
                                                       int P, int ng, FinalArgs fa) {
  constexpr int n = Geo<N>::n, H = Geo<N>::H, NT = Geo<N>::NT;
  constexpr int HP = H + 1;  // padded half row
  // two half-spectrum planes during the transform, then one padded real field
  static_assert(N * N * (N + 1) <= 2 * N * N * HP, "gain field must fit the transform buffer");
  __shared__ float LB[2 * N * N * HP];
  __shared__ double red[5][NT / 64];
  __shared__ double lamb[5];
  float* LR = LB;
  float* LI = LB + N * N * HP;
  const int t = threadIdx.x;
  const int p = blockIdx.x;
  const int li = pidx[p], lj = pidx[P + p], row = pidx[2 * P + p];
  // stage A, axis 0 over k0 at fixed (k1, k2h): N*H active lines
  {
    float re[N], im[N];
    const bool act = t < N * H;
    const int k1 = t / H, k2 = t % H;
    if (act) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        re[j] = 0.f;
        im[j] = 0.f;
      }
      // (each group's half spectrum is read once: streaming loads)
      typedef float f2v __attribute__((ext_vector_type(2)));
      for (int g = 0; g < ng; ++g) {
        const f2v* src = reinterpret_cast<const f2v*>(wsp + ((long)p * ng + g) * N * N * H +
                                                      (long)k1 * H + k2);
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const f2v v = __builtin_nontemporal_load(src + (long)j * N * H);
          re[j] += v.x;
          im[j] += v.y;
        }
      }
      fft::dft<float, N, +1>(re, im);
#pragma unroll
      for (int j = 0; j < N; ++j) {  // (i0 = j, k1, k2)
        LR[(j * N + k1) * HP + k2] = re[j];
        LI[(j * N + k1) * HP + k2] = im[j];
      }
    }
    __syncthreads();
    // stage B, axis 1 over k1 at fixed (i0, k2h)
    const int i0 = t / H;
    if (act) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        re[j] = LR[(i0 * N + j) * HP + k2];
        im[j] = LI[(i0 * N + j) * HP + k2];
      }
    }
    __syncthreads();
    if (act) {
      fft::dft<float, N, +1>(re, im);
#pragma unroll
      for (int j = 0; j < N; ++j) {  // (i0, i1 = j, k2)
        LR[(i0 * N + j) * HP + k2] = re[j];
        LI[(i0 * N + j) * HP + k2] = im[j];
      }
    }
    __syncthreads();
  }
  // stage C, axis 2: thread (i0, i1); full Hermitian line from the half
  {
    const int i0 = t / N, i1 = t % N;
    float re[N], im[N];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      re[j] = LR[(i0 * N + i1) * HP + j];
      im[j] = LI[(i0 * N + i1) * HP + j];
    }
#pragma unroll
    for (int j = H; j < N; ++j) {
      re[j] = re[N - j];
      im[j] = -im[N - j];
    }
    fft::dft<float, N, +1>(re, im);
    __syncthreads();  // every half row has been read
    // the gain field back to LDS, rows of N + 1
#pragma unroll
    for (int j = 0; j < N; ++j) LB[(i0 * N + i1) * (N + 1) + j] = re[j];
  }
  __syncthreads();
  // gain - loss with coalesced access: thread t holds the points e = k * NT + t,
  // (i0, i1, i2) = (k, t / N, t % N)
  const int u1 = t / N, u2 = t % N;
  const float* vi = vp + (long)li * n + t;
  const float* vj = vp + (long)lj * n + t;
  const float* lmi = lam + (long)li * n + t;
  const float* lmj = lam + (long)lj * n + t;
  const double v1 = -fa.L + u1 * fa.dv, v2 = -fa.L + u2 * fa.dv;
  const double s12 = v1 * v1 + v2 * v2;
  double m[5] = {0, 0, 0, 0, 0};
  float q[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const long o = (long)k * NT;
    q[k] = LB[(k * N + u1) * (N + 1) + u2] - 0.5f * (vj[o] * lmi[o] + vi[o] * lmj[o]);
    const double v0 = -fa.L + k * fa.dv;
    const double x = (double)q[k];
    m[0] += x;
    m[1] += x * v0;
    m[2] += x * v1;
    m[3] += x * v2;
    m[4] += x * (v0 * v0 + s12);
    // keep the five sums plane by plane (otherwise all N widened values are
    // held at once and spill); at most eight planes of loads in flight
    asm volatile("" : "+v"(m[0]), "+v"(m[1]), "+v"(m[2]), "+v"(m[3]), "+v"(m[4]));
    if (k % 8 == 7) __builtin_amdgcn_sched_barrier(0);
  }
  if (fa.conserve) {
    // deterministic reduction: wave sums then a fixed-order sum of waves
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double x = m[c];
#pragma unroll
      for (int off2 = 32; off2 > 0; off2 >>= 1) x += __shfl_down(x, off2, 64);
      if ((t & 63) == 0) red[c][t >> 6] = x;
    }
    __syncthreads();
    if (t < 5) {
      double s = 0;
      for (int c = 0; c < NT / 64; ++c) s += red[t][c];
      lamb[t] = s * fa.w;
    }
    __syncthreads();
    if (t == 0) {
      double l[5];
      for (int i = 0; i < 5; ++i) {
        l[i] = 0;
        for (int c = 0; c < 5; ++c) l[i] += fa.minv[i * 5 + c] * lamb[c];
      }
      for (int i = 0; i < 5; ++i) red[i][0] = l[i];
    }
    __syncthreads();
    const double l0 = red[0][0], l1 = red[1][0], l2 = red[2][0], l3 = red[3][0], l4 = red[4][0];
    const double base = l0 + l2 * v1 + l3 * v2 + l4 * s12;
    // v0 advanced by dv per plane (not the closed form above), so that the
    // 32 nodes are not kept live in registers across the reduction
    double v0 = -fa.L;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const double c = base + l1 * v0 + l4 * v0 * v0;
      q[k] = (float)((double)q[k] - fa.w * c);
      v0 += fa.dv;
    }
  }
  float* dst = Q + (long)row * n + t;
#pragma unroll
  for (int k = 0; k < N; ++k) dst[(long)k * NT] = q[k];
}

}  // namespace fastk


// Tile width of the sigma sums for a served batch: the candidates (the rule
// of run_fast, 12, 8, 6) timed once on the call's own data when a shape is
// first seen (not while a graph is recorded), the fastest kept per shape.
// Every width computes each pair's sum with the same operations in the same
// order, so the choice changes the time only, never a result.
template <class F>
static int tuned_tile_width(blr_ctx ctx, int N, int rb, const PairPlan& pl, int G0, F&& run) {
  std::string key = std::to_string(N) + ":" + std::to_string(rb) + ":";
  uint64_t hsh = 1469598103934665603ull;
  for (size_t p = 0; p < pl.li.size(); ++p) {
    hsh = (hsh ^ (uint64_t)(pl.li[p] * 131 + pl.lj[p])) * 1099511628211ull;
  }
  key += std::to_string(hsh);
  auto it = ctx->tuned_tile.find(key);
  if (it != ctx->tuned_tile.end()) return it->second;
  if (ctx->capturing) return G0;
  hipStream_t s = ctx->stream;
  std::vector<int> cand{G0};
  for (int g : {12, 8, 6})
    if (std::find(cand.begin(), cand.end(), g) == cand.end()) cand.push_back(g);
  hipEvent_t e0, e1;
  BLR_HIP(hipEventCreate(&e0));
  BLR_HIP(hipEventCreate(&e1));
  int best = G0;
  float best_ms = 1e30f;
  for (int g : cand) {
    run(g);  // warm
    BLR_HIP(hipEventRecord(e0, s));
    run(g);
    BLR_HIP(hipEventRecord(e1, s));
    BLR_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    BLR_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = g;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->tuned_tile[key] = best;
  return best;
}

template <int N>
static void run_fast(blr_ctx ctx, const DevTables& tb, const PairPlan& pl, const std::vector<int>& prow,
                     const float2* Vh, const float* Vp, const float* Lam, float* Q, bool conserve) {
  using namespace fastk;
  const HostTables& h = tb.h;
  hipStream_t s = ctx->stream;
  constexpr int n = Geo<N>::n, H = Geo<N>::H;
  const int rb = (int)pl.bidx.size();
  const int P = (int)pl.li.size();
  const long nfields = (long)rb * h.mrho * h.nbp;
  float* Sh = (float*)ctx->buf("fast.Sh", (size_t)rb * h.mrho * h.msig * n * sizeof(float));
  float* Pa = (float*)ctx->buf("fast.Pa", (size_t)h.mrho * P * n * sizeof(float));
  // radial nodes per pair-transform workgroup: one workgroup fills a CU, so
  // the launch takes about ceil(P * ng / CUs) rounds of ceil(ga / 2)
  // transforms (two nodes per transform); each extra group costs the final
  // kernel one more half-spectrum read
  int ga = 1;
  if (ctx->batch_mode) {
    // served batches: two nodes per transform whatever the pair count, so a
    // pair's sums run in the same order alone and in any batch
    ga = std::min(2, h.mrho);
  } else {
    double best = 1e300;
    for (int g = 1; g <= h.mrho; ++g) {
      const int ngc = (h.mrho + g - 1) / g;
      const double rounds = std::ceil((double)P * ngc / ctx->cu_count());
      const double cost = rounds * ((g + 1) / 2) + 0.1 * ngc;
      if (cost < best - 1e-9) {
        best = cost;
        ga = g;
      }
    }
  }
  const int ng = (h.mrho + ga - 1) / ga;
  float2* Wsp = (float2*)ctx->buf("fast.Wsp", (size_t)P * ng * N * N * H * sizeof(float2));
  std::vector<int> idx(3 * P);
  for (int p = 0; p < P; ++p) {
    idx[p] = pl.li[p];
    idx[P + p] = pl.lj[p];
    idx[2 * P + p] = prow[p];
  }
  int* didx = (int*)ctx->upload("fast.idx", idx.data(), idx.size() * sizeof(int));
  // shifts: persistent-style grid, each workgroup loops over fields
  {
    require(nfields < (1L << 31), "fast collision: too many shift fields");
    // one persistent workgroup per CU (it holds a whole field: all of a CU's
    // registers and 132 KiB of LDS)
    const long grid = std::min<long>(nfields, ctx->cu_count());
    timed_begin("fast.shift", (double)nfields * n * (2 * sizeof(float)), s);
    hipLaunchKernelGGL(k_shift_fused<N>, dim3((unsigned)grid), dim3(N * N), 0, s, Vh,
                       (const float2*)tb.phase, Sh, tb.bp_b, tb.bp_bb, h.mrho, h.nbp, h.msig, nfields);
    BLR_CHECK_LAUNCH();
    timed_end(s);
  }
  // sigma sums for every radial node
  {
    // tile width: the fewest tiles of at most 12 basis functions, each as
    // narrow as possible (a rank-10 basis is one 10-wide tile: no idle slots,
    // 120 VGPRs, four waves per SIMD)
    const int ngr = (rb + 11) / 12, per = (rb + ngr - 1) / ngr;
    int G = std::max(4, per);
    BpArgs bpa{};
    for (int p = 0; p < h.nbp && p < kMaxBp; ++p) {
      bpa.off_b[p] = h.bp_b[p] * n;
      bpa.off_bb[p] = h.bp_bb[p] * n;
      bpa.w[p] = (float)(2.0 * h.wsig[h.bp_b[p]]);  // see k_reduce_all
    }
    // every tile of width Gw over the requested pairs
    auto reduce_all_tiles = [&](int Gw) {
      bool diag_only = false;
      const auto tiles = plan_tiles(rb, pl.li, pl.lj, Gw, diag_only);
      for (const auto& t : tiles) {
        const bool diag = t.bi[0] == t.bj[0];
        int nvalid = 0;
        for (int k = 0; k < 256; ++k) nvalid += t.out[k] >= 0;
        const int nload = diag ? 2 * t.ni : 2 * (t.ni + t.nj);
        timed_begin("fast.reduce.g" + std::to_string(Gw),
                    (double)h.mrho * n * (nload * h.nbp + nvalid) * sizeof(float), s);
        const dim3 grid((n + 255) / 256, h.mrho);
        auto launch = [&](auto Gc) {
          constexpr int Gt = decltype(Gc)::value;
          if (diag && h.nbp <= kMaxBp)
            hipLaunchKernelGGL((k_reduce_diag<Gt>), grid, dim3(256), 0, s, Sh, Pa, t, bpa, n,
                               h.mrho, h.msig, h.nbp, P);
          else if (diag)
            hipLaunchKernelGGL((k_reduce_all<Gt, true>), grid, dim3(256), 0, s, Sh, Pa, t,
                               (const float*)tb.wbp, tb.bp_b, tb.bp_bb, n, h.mrho, h.msig, h.nbp,
                               P);
          else
            hipLaunchKernelGGL((k_reduce_all<Gt, false>), grid, dim3(256), 0, s, Sh, Pa, t,
                               (const float*)tb.wbp, tb.bp_b, tb.bp_bb, n, h.mrho, h.msig, h.nbp,
                               P);
        };
        switch (Gw) {
          case 4: launch(std::integral_constant<int, 4>{}); break;
          case 5: launch(std::integral_constant<int, 5>{}); break;
          case 6: launch(std::integral_constant<int, 6>{}); break;
          case 7: launch(std::integral_constant<int, 7>{}); break;
          case 8: launch(std::integral_constant<int, 8>{}); break;
          case 9: launch(std::integral_constant<int, 9>{}); break;
          case 10: launch(std::integral_constant<int, 10>{}); break;
          case 11: launch(std::integral_constant<int, 11>{}); break;
          default: launch(std::integral_constant<int, 12>{}); break;
        }
        BLR_CHECK_LAUNCH();
        timed_end(s);
      }
    };
    if (ctx->batch_mode) G = tuned_tile_width(ctx, N, rb, pl, G, reduce_all_tiles);
    reduce_all_tiles(G);
  }
  // transforms of the pair products with the radial weights
  timed_begin("fast.pair_spec",
              (double)P * ((double)h.mrho * n * sizeof(float) + (double)ng * N * N * H * sizeof(float2)), s);
  hipLaunchKernelGGL(k_pair_spec<N>, dim3(P * ng), dim3(N * N), 0, s, Pa, (const float*)tb.fw,
                     Wsp, P, h.mrho, h.nkk, ga, ng);
  BLR_CHECK_LAUNCH();
  timed_end(s);
  // radial sum, inverse transform, loss, projection
  FinalArgs fa{};
  fa.L = h.L;
  fa.dv = h.dv;
  fa.w = std::pow(h.dv, 3);
  for (int i = 0; i < 25 && i < (int)h.minv.size(); ++i) fa.minv[i] = h.minv[i];
  fa.conserve = conserve ? 1 : 0;
  timed_begin("fast.final",
              (double)P * ((double)ng * N * N * H * sizeof(float2) + 5.0 * n * sizeof(float)), s);
  hipLaunchKernelGGL(k_final_fused<N>, dim3(P), dim3(N * N), 0, s, Wsp, Vp, Lam, didx, Q, P, ng, fa);
  BLR_CHECK_LAUNCH();
  timed_end(s);
}

// Carleman form, 3D FP32: the filtered fields of rb basis functions (the
// generic path's filter transforms in one fused kernel).  False when the grid
// has no fused kernel.
bool carleman_filter_f32(blr_ctx ctx, const DevTables& tb, const float2* Vh, float* Sh, int rb) {
  using namespace fastk;
  const HostTables& h = tb.h;
  if (h.d != 3 || !h.carleman || (h.N != 16 && h.N != 24 && h.N != 32)) return false;
  hipStream_t s = ctx->stream;
  const long nfields = (long)rb * h.nbp;
  require(nfields < (1L << 31), "carleman filters: too many fields");
  const long grid = std::min<long>(nfields, 2048);
  auto launch = [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    timed_begin("carl.filter_fused", (double)nfields * Geo<N>::n * 4.0 * sizeof(float), s);
    hipLaunchKernelGGL(k_filter_fused<N>, dim3((unsigned)grid), dim3(N * N), 0, s, Vh,
                       (const float2*)tb.filt, Sh, tb.bp_b, tb.bp_bb, h.nbp, h.msig, nfields);
    BLR_CHECK_LAUNCH();
    timed_end(s);
  };
  switch (h.N) {
    case 16: launch(std::integral_constant<int, 16>{}); break;
    case 24: launch(std::integral_constant<int, 24>{}); break;
    case 32: launch(std::integral_constant<int, 32>{}); break;
  }
  return true;
}

// Basis spectra and loss fields come from the generic kernels (collision.hip).

bool fast_collision_f32(blr_ctx ctx, const DevTables& tb, const float* V, const PairPlan& pl,
                        const std::vector<int>& prow, float* Q, bool conserve) {
  const HostTables& h = tb.h;
  if (h.d != 3 || (h.N != 16 && h.N != 24 && h.N != 32)) return false;
  if (pl.bidx.size() > 64 || h.msig != 38) return false;
  float2* Vh;
  float* Vp;
  float* Lam;
  basis_spectra_f32(ctx, tb, V, pl, &Vh, &Vp, &Lam);
  switch (h.N) {
    case 16: run_fast<16>(ctx, tb, pl, prow, Vh, Vp, Lam, Q, conserve); break;
    case 24: run_fast<24>(ctx, tb, pl, prow, Vh, Vp, Lam, Q, conserve); break;
    case 32: run_fast<32>(ctx, tb, pl, prow, Vh, Vp, Lam, Q, conserve); break;
  }
  return true;
}

}  // namespace blr
