// Adaptive dynamical low-rank step on the GPU (FP64 except the pair
// collisions, which are FP32 unless BLR_STEP_FP64_COLLISION).
//
// Physical space is 1D along the first velocity axis; cells x_p, spacing dx;
// inner products <a,b>_x = dx sum_p a_p b_p and <a,b>_v = dv^d sum_q a_q b_q.
// Upwind transport v^+ D_+ (backward difference) and v^- D_- (forward
// difference); ghost values of K from the projected boundary function: at the
// left wall K_j = <f_L 1_{v1>0}, V_j>_v + sum_l K_l(x_0) <1_{v1<=0} V_l V_j>_v,
// at the right wall with f_R, 1_{v1<0} and the last cell.
//
// Layouts (device, FP64): X rows [i][x] (r x nx), V rows [j][q] (r x n),
// S row-major.  All reductions have a fixed order (no atomics), so a step is
// bitwise reproducible.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>

#include "collision_common.hpp"
#include "linalg.hpp"
#include "obstacle.hpp"
#include "walls.hpp"

namespace blr {
namespace dk {

// weight of mode m at velocity point q (v1 = first velocity coordinate)
// (modes from W_V2PLUS on weigh by v_2, the velocity along y of the
// two-dimensional space: its faces y_lo = "bottom" and y_hi = "top")
enum Mode {
  W_ONE = 0, W_VPLUS, W_VMINUS, W_OUT_LEFT, W_OUT_RIGHT, W_IN_LEFT, W_IN_RIGHT,
  W_V2PLUS, W_V2MINUS, W_OUT_BOTTOM, W_OUT_TOP, W_IN_BOTTOM, W_IN_TOP
};

struct VGeo {
  double L, dv;
  int N, d, n;
  __device__ __forceinline__ double v1(int q) const {
    const int q0 = d == 3 ? q / (N * N) : q / N;
    return -L + q0 * dv;
  }
  __device__ __forceinline__ double v2(int q) const {
    const int q1 = d == 3 ? (q / N) % N : q % N;
    return -L + q1 * dv;
  }
};

__device__ __forceinline__ double weight(int mode, double v) {
  switch (mode) {
    case W_VPLUS:
    case W_V2PLUS: return v > 0 ? v : 0.0;
    case W_VMINUS:
    case W_V2MINUS: return v < 0 ? v : 0.0;
    case W_OUT_LEFT:
    case W_OUT_BOTTOM: return v <= 0 ? 1.0 : 0.0;
    case W_OUT_RIGHT:
    case W_OUT_TOP: return v >= 0 ? 1.0 : 0.0;
    case W_IN_LEFT:
    case W_IN_BOTTOM: return v > 0 ? 1.0 : 0.0;
    case W_IN_RIGHT:
    case W_IN_TOP: return v < 0 ? 1.0 : 0.0;
    default: return 1.0;
  }
}
__device__ __forceinline__ double weight(int mode, const VGeo& g, int q) {
  return weight(mode, mode >= W_V2PLUS ? g.v2(q) : g.v1(q));
}

constexpr int GT = 16;  // output tile edge (rows of A x rows of B)

typedef double v4d __attribute__((ext_vector_type(4)));

// A batch of weighted Gram products out = scale * sum_q w(q) A_i(q) B_j(q)
// (ra x rb row-major, ra <= 64), evaluated together: every 16 x 16 output
// tile of every product is one grid row, every velocity chunk one grid
// column; each block writes its tile's chunk sum (waves in order) and a
// second kernel adds the chunks in order.
constexpr int MAXSEG = 8;
struct GramSeg {
  const double* A;
  const void* B;  // double, or float when bfloat
  double* out;
  double scale;
  int ra, rb, mode, bfloat;
  int tile0;  // first grid row of this product
  int ntb;    // tiles along B
  long part0; // offset of its partial sums ([chunk][i][j])
  int out0;   // first flat output index of this product
};
struct GramBatch {
  GramSeg seg[MAXSEG];
  int nseg, ntiles, nout;
};

__global__ __launch_bounds__(256) void k_gram_batch(GramBatch gb, long n, int nchunk, VGeo g,
                                                    double* __restrict__ part) {
  __shared__ double red[4][256];
  const int tile = blockIdx.y;
  int si = 0;
  while (si + 1 < gb.nseg && tile >= gb.seg[si + 1].tile0) ++si;
  const GramSeg sg = gb.seg[si];
  const int tl = tile - sg.tile0;
  const int i0 = (tl / sg.ntb) * GT, j0 = (tl % sg.ntb) * GT;
  const int c = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const long q0 = (long)c * n / nchunk, q1 = (long)(c + 1) * n / nchunk;
  const long len = q1 - q0;
  const long w0 = q0 + len * wv / 4, w1 = q0 + len * (wv + 1) / 4;
  const int ii = lane & 15, kk = lane >> 4;
  const bool arow = i0 + ii < sg.ra, brow = j0 + ii < sg.rb;
  const double* pa = sg.A + (long)(arow ? i0 + ii : 0) * n;
  const double* pbd = (const double*)sg.B + (long)(brow ? j0 + ii : 0) * n;
  const float* pbf = (const float*)sg.B + (long)(brow ? j0 + ii : 0) * n;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (long qb = w0; qb < w1; qb += 32) {
    double xa[8], yb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const long q = qb + 4 * u + kk;
      const bool in = q < w1;
      xa[u] = (in && arow) ? pa[q] * weight(sg.mode, g, (int)q) : 0.0;
      yb[u] = (in && brow) ? (sg.bfloat ? (double)pbf[q] : pbd[q]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], yb[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv][(4 * v + kk) * 16 + ii] = acc[v];
  __syncthreads();
  const int i = t / 16, j = t % 16;
  if (i0 + i < sg.ra && j0 + j < sg.rb)
    part[sg.part0 + ((long)c * sg.ra + i0 + i) * sg.rb + j0 + j] =
        ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// chunk sums of a batch: one wavefront per output, fixed order
__global__ __launch_bounds__(256) void k_gram_batch_finish(GramBatch gb, int nchunk,
                                                           const double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= gb.nout) return;
  int si = 0;
  while (si + 1 < gb.nseg && o >= gb.seg[si + 1].out0) ++si;
  const GramSeg& sg = gb.seg[si];
  const int e = o - sg.out0;
  const long per = (long)sg.ra * sg.rb;
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int c = lane + 64 * k;
    v[k] = c < nchunk ? part[sg.part0 + c * per + e] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += v[k];
  for (int c = lane + 512; c < nchunk; c += 64) s += part[sg.part0 + c * per + e];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) sg.out[e] = sg.scale * s;
}

// K[j][x] = sum_i X[i][x] S[i][j]
__global__ void k_xmul(const double* __restrict__ X, int r, int nx, const double* __restrict__ S,
                       int lds, double* __restrict__ K) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * nx) return;
  const int j = t / nx, x = t % nx;
  double s = 0.0;
  for (int i = 0; i < r; ++i) s += X[(long)i * nx + x] * S[i * lds + j];
  K[t] = s;
}

// ghost values g[0][j] (left), g[1][j] (right) of the columns of K
__global__ void k_ghosts(const double* __restrict__ K, int r, int nx, const double* __restrict__ ginL,
                         const double* __restrict__ ginR, const double* __restrict__ MoL,
                         const double* __restrict__ MoR, double* __restrict__ g) {
  const int j = threadIdx.x;
  if (j >= r) return;
  double sl = ginL[j], sr = ginR[j];
  for (int l = 0; l < r; ++l) {
    sl += K[(long)l * nx + 0] * MoL[l * r + j];
    sr += K[(long)l * nx + nx - 1] * MoR[l * r + j];
  }
  g[j] = sl;
  g[r + j] = sr;
}

__device__ __forceinline__ double dplus(const double* K, const double* g, int l, int x, int nx,
                                        double dx) {
  const double prev = x == 0 ? g[l] : K[(long)l * nx + x - 1];
  return (K[(long)l * nx + x] - prev) / dx;
}
__device__ __forceinline__ double dminus(const double* K, const double* g, int r, int l, int x,
                                         int nx, double dx) {
  const double next = x == nx - 1 ? g[r + l] : K[(long)l * nx + x + 1];
  return (next - K[(long)l * nx + x]) / dx;
}

// K-step: K1 = K + dt (-sum_l A+_{jl} D+K_l - sum_l A-_{jl} D-K_l + sum_p C_{jp} w_p K_m K_n)
__global__ void k_kstep(const double* __restrict__ K, const double* __restrict__ g, int r, int nx,
                        double dx, double dt, const double* __restrict__ Ap,
                        const double* __restrict__ Am, const double* __restrict__ C, int P,
                        const int* __restrict__ pm, const int* __restrict__ pn,
                        double* __restrict__ K1, double* __restrict__ dK) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * nx) return;
  const int j = t / nx, x = t % nx;
  double rhs = 0.0;
  for (int l = 0; l < r; ++l)
    rhs -= Ap[j * r + l] * dplus(K, g, l, x, nx, dx) + Am[j * r + l] * dminus(K, g, r, l, x, nx, dx);
  for (int p = 0; p < P; ++p) {
    const int m = pm[p], nn = pn[p];
    const double w = (m == nn) ? 1.0 : 2.0;
    rhs += C[j * P + p] * w * K[(long)m * nx + x] * K[(long)nn * nx + x];
  }
  const double k1 = K[t] + dt * rhs;
  K1[t] = k1;
  dK[t] = k1 - K[t];
}

// x-side reductions: out[i][c] = dx sum_x X1[i][x] Y_c(x) for
//   c <  r        : Y = D+ K_c
//   c <  2r       : Y = D- K_(c-r)
//   c <  2r + P   : Y = w_p K_m K_n
// (mode 1: Y_c = Z[c][x], a plain matrix with ncols columns).
// One wavefront per output: lanes stride over x, then a shuffle tree.
__global__ __launch_bounds__(256) void k_xreduce(const double* __restrict__ X1, int r, int nx,
                                                 double dx, const double* __restrict__ K,
                                                 const double* __restrict__ g, int P,
                                                 const int* __restrict__ pm,
                                                 const int* __restrict__ pn,
                                                 const double* __restrict__ Z, int zc, int mode,
                                                 double* __restrict__ out, int ncols,
                                                 double* __restrict__ oDp, double* __restrict__ oDm,
                                                 double* __restrict__ oT) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= r * ncols) return;
  const int i = t / ncols, c = t % ncols;
  double s = 0.0;
  for (int x = lane; x < nx; x += 64) {
    double y;
    if (mode == 1) {
      y = Z[(long)c * nx + x];
    } else if (c < r) {
      y = dplus(K, g, c, x, nx, dx);
    } else if (c < 2 * r) {
      y = dminus(K, g, r, c - r, x, nx, dx);
    } else {
      const int p = c - 2 * r;
      const int m = pm[p], nn = pn[p];
      y = ((m == nn) ? 1.0 : 2.0) * K[(long)m * nx + x] * K[(long)nn * nx + x];
    }
    s += X1[(long)i * nx + x] * y;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane != 0) return;
  s *= dx;
  (void)zc;
  if (mode == 1) {
    out[t] = s;
  } else if (c < r) {
    oDp[i * r + c] = s;
  } else if (c < 2 * r) {
    oDm[i * r + c - r] = s;
  } else {
    oT[i * P + c - 2 * r] = s;
  }
}

// L-step on the velocity grid, rows i of this block's chunk of 8:
//   L_i  = sum_l S2_il V_l
//   L1_i = L_i - dt (v+ sum_l Dp_il V_l + v- sum_l Dm_il V_l) + dt sum_p T_ip Q_p
template <typename TQ>
__global__ __launch_bounds__(256) void k_lstep(const double* __restrict__ V, int r, int n,
                                               const double* __restrict__ S2,
                                               const double* __restrict__ Dp,
                                               const double* __restrict__ Dm,
                                               const double* __restrict__ T,
                                               const TQ* __restrict__ Q, int P, double dt, VGeo g,
                                               double* __restrict__ L1, double* __restrict__ dL) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int i0 = blockIdx.y * 8;
  if (q >= n) return;
  double l[8], dp[8], dm[8], cq[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) l[k] = dp[k] = dm[k] = cq[k] = 0.0;
  for (int m = 0; m < r; ++m) {
    const double v = V[(long)m * n + q];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = min(i0 + k, r - 1);
      l[k] += S2[i * r + m] * v;
      dp[k] += Dp[i * r + m] * v;
      dm[k] += Dm[i * r + m] * v;
    }
  }
  for (int p = 0; p < P; ++p) {
    const double qv = (double)Q[(long)p * n + q];
#pragma unroll
    for (int k = 0; k < 8; ++k) cq[k] += T[min(i0 + k, r - 1) * P + p] * qv;
  }
  const double v1 = g.v1(q);
  const double vp = v1 > 0 ? v1 : 0.0, vm = v1 < 0 ? v1 : 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int i = i0 + k;
    if (i < r) {
      const double d = -dt * (vp * dp[k] + vm * dm[k]) + dt * cq[k];
      L1[(long)i * n + q] = l[k] + d;
      dL[(long)i * n + q] = d;
    }
  }
}

// out[i][e] = scale * sum_l M[l * ldm + i] in[l][e]   (combination of rows)
__global__ void k_rows_comb(const double* __restrict__ in, int rin, long len,
                            const double* __restrict__ M, int ldm, int rout, double scale,
                            double* __restrict__ out, long ldo) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (e >= len || i >= rout) return;
  double s = 0.0;
  for (int l = 0; l < rin; ++l) s += M[l * ldm + i] * in[(long)l * len + e];
  out[(long)i * ldo + e] = scale * s;
}

__global__ void k_scale_copy(const double* __restrict__ in, long count, double scale,
                             double* __restrict__ out) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < count) out[e] = scale * in[e];
}



// ---- truncated SVD of a full f0 (state_from_full) ----------------------
constexpr int SFF_BS = 256;

__global__ void k_sff_load(const double* __restrict__ f0, long count, double w,
                           double* __restrict__ Y) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < count) Y[e] = w * f0[e];
}

__global__ void k_sff_eye(double* __restrict__ W, int m) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < (long)m * m) W[e] = (e / m == e % m) ? 1.0 : 0.0;
}

__global__ void k_sff_flag(int* flag, int v) {
  if (threadIdx.x == 0) flag[0] = v;
}

// fixed-order sum of SFF_BS values per component over the block (3 at once)
__device__ __forceinline__ void sff_reduce3(double* sh, double& a, double& b, double& c) {
  const int t = threadIdx.x;
  sh[t] = a;
  sh[SFF_BS + t] = b;
  sh[2 * SFF_BS + t] = c;
  __syncthreads();
  for (int w = SFF_BS / 2; w > 0; w >>= 1) {
    if (t < w) {
      sh[t] += sh[t + w];
      sh[SFF_BS + t] += sh[SFF_BS + t + w];
      sh[2 * SFF_BS + t] += sh[2 * SFF_BS + t + w];
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[SFF_BS];
  c = sh[2 * SFF_BS];
}

// One round of the round-robin schedule on mpad (even) indices: pair slot k
// of round t is (mpad - 1, t) for k = 0 and ((t + k) mod (mpad - 1),
// (t - k) mod (mpad - 1)) otherwise; indices >= m are padding.  The block
// of slot k rotates rows p, q of Y (length n) and of W (length m) so that
// <y_p, y_q> = 0, unless they already are orthogonal to tol.
__global__ __launch_bounds__(SFF_BS) void k_sff_round(double* __restrict__ Y, long n,
                                                      double* __restrict__ W, int m, int mpad,
                                                      int round, double tol, int* flag) {
  __shared__ double sh[3 * SFF_BS];
  const int k = blockIdx.x, M1 = mpad - 1;
  int p, q;
  if (k == 0) {
    p = M1;
    q = round;
  } else {
    p = (round + k) % M1;
    q = (round - k + M1) % M1;
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
  if (q >= m) return;
  double* yp = Y + (long)p * n;
  double* yq = Y + (long)q * n;
  double a = 0.0, b = 0.0, c = 0.0;
  for (long e = threadIdx.x; e < n; e += SFF_BS) {
    const double x = yp[e], y = yq[e];
    a += x * x;
    b += y * y;
    c += x * y;
  }
  sff_reduce3(sh, a, b, c);
  if (!(fabs(c) > tol * sqrt(a) * sqrt(b))) return;
  // rotation angle of one-sided Jacobi: t the smaller root of
  // t^2 + 2 z t - 1 = 0, z = (b - a) / (2 c)
  const double z = (b - a) / (2.0 * c);
  const double t = (z >= 0 ? 1.0 : -1.0) / (fabs(z) + hypot(1.0, z));
  const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
  for (long e = threadIdx.x; e < n; e += SFF_BS) {
    const double x = yp[e], y = yq[e];
    yp[e] = cs * x - sn * y;
    yq[e] = sn * x + cs * y;
  }
  double* wp = W + (long)p * m;
  double* wq = W + (long)q * m;
  for (int e = threadIdx.x; e < m; e += SFF_BS) {
    const double x = wp[e], y = wq[e];
    wp[e] = cs * x - sn * y;
    wq[e] = sn * x + cs * y;
  }
  if (threadIdx.x == 0) flag[0] = 1;
}

__global__ __launch_bounds__(SFF_BS) void k_sff_norms(const double* __restrict__ Y, long n,
                                                      double* __restrict__ nrm) {
  __shared__ double sh[3 * SFF_BS];
  const double* y = Y + (long)blockIdx.x * n;
  double a = 0.0, b = 0.0, c = 0.0;
  for (long e = threadIdx.x; e < n; e += SFF_BS) a += y[e] * y[e];
  sff_reduce3(sh, a, b, c);
  if (threadIdx.x == 0) nrm[blockIdx.x] = sqrt(a);
}

// X_k = W[idx_k] / sqrt(wx), V_k = Y[idx_k] / (sigma_k sqrt(dv^d)), S = diag(sigma)
__global__ void k_sff_store(const double* __restrict__ Y, long n, const double* __restrict__ W,
                            int m, const double* __restrict__ nrm, const int* __restrict__ idx,
                            int r, double sx, double sv, double* __restrict__ X,
                            double* __restrict__ V, double* __restrict__ S, int r_cap) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  const int i = idx[k];
  const double sg = nrm[i];
  if (e < n) V[(long)k * n + e] = Y[(long)i * n + e] * (sv / sg);
  if (e < m) X[(long)k * m + e] = W[(long)i * m + e] * sx;
  if (e < r) S[(long)k * r_cap + e] = (e == k) ? sg : 0.0;
}

// small dense algebra (one block)
// S2 = S1 + dt (Dp Ap^T + Dm Am^T - T C^T);  dS = S2 - S1
__global__ void k_supdate(const double* S1, const double* Dp, const double* Dm, const double* T,
                          const double* Ap, const double* Am, const double* C, int r, int P,
                          double dt, double* S2, double* dS) {
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
  const int i = t / r, j = t % r;
  double s = 0.0;
  for (int l = 0; l < r; ++l) s += Dp[i * r + l] * Ap[j * r + l] + Dm[i * r + l] * Am[j * r + l];
  for (int p = 0; p < P; ++p) s -= T[i * P + p] * C[j * P + p];
  S2[t] = S1[t] + dt * s;
  dS[t] = dt * s;
  }
}

__global__ void k_transpose(const double* A, int r, double* B) {
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) B[(t % r) * r + t / r] = A[t];
}

// err^2 from the pieces; sums written to res[0..5]
__global__ void k_err(const double* dK, long nK, double dx, const double* dS, int r,
                      const double* GdL, const double* kx, const double* lv, double* res) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double s = 0.0;
  for (long e = t; e < nK; e += blockDim.x) s += dK[e] * dK[e];
  red[t] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st) red[t] += red[t + st];
    __syncthreads();
  }
  if (t == 0) {
    const double a = dx * red[0];
    double b = 0.0, c = 0.0, I = 0.0, II = 0.0, III = 0.0;
    for (int e = 0; e < r * r; ++e) {
      b += dS[e] * dS[e];
      I += kx[e] * dS[e];
      II += lv[e] * dS[e];
      III += kx[e] * lv[e];
    }
    for (int i = 0; i < r; ++i) c += GdL[i * r + i];
    res[0] = a + b + c + 2.0 * (I + II + III);
    res[1] = a;
    res[2] = b;
    res[3] = c;
  }
}

// Terms of <f^n, D_keep> for every truncation point: with S^{n+1} = U Sig W^T,
// D_keep = X1 (sum_{s >= keep} sig_s u_s w_s^T) V1 and A_ki = <X^n_k, X1_i>,
// B_lj = <V^n_l, V1_j>,
//   <f^n, D_keep> = sum_{s >= keep} g_s,  g_s = sig_s (A u_s)^T S^n (B w_s).
// One block; g[s] written for s < r.
__global__ __launch_bounds__(256) void k_fnD_terms(const double* S, const double* A,
                                                   const double* U, const double* sig,
                                                   const double* W, const double* B, int r,
                                                   double* g) {
  __shared__ double AU[64 * 64];  // AU[k][s] = sum_i A[k][i] U[i][s]
  __shared__ double BW[64 * 64];  // BW[l][s] = sum_j B[l][j] W[j][s]
  const int t = threadIdx.x;
  for (int e = t; e < r * r; e += blockDim.x) {
    const int k = e / r, q = e % r;
    double au = 0.0, bw = 0.0;
    for (int i = 0; i < r; ++i) {
      au += A[k * r + i] * U[i * r + q];
      bw += B[k * r + i] * W[i * r + q];
    }
    AU[e] = au;
    BW[e] = bw;
  }
  __syncthreads();
  for (int q = t; q < r; q += blockDim.x) {
    double v = 0.0;
    for (int k = 0; k < r; ++k) {
      double sb = 0.0;
      for (int l = 0; l < r; ++l) sb += S[k * r + l] * BW[l * r + q];
      v += AU[k * r + q] * sb;
    }
    g[q] = sig[q] * v;
  }
}

__global__ void k_diag(const double* sig, int r, double* S, int lds) {
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
    const int i = t / r, j = t % r;
    S[i * lds + j] = (i == j) ? sig[i] : 0.0;
  }
}

__global__ void k_copy_S(const double* src, int lds_src, int r, double* dst, int lds_dst) {
  const int t = threadIdx.x + blockIdx.x * blockDim.x;
  if (t >= r * r) return;
  dst[(t / r) * lds_dst + t % r] = src[(t / r) * lds_src + t % r];
}

// Start of a step: S (leading dim lds) -> Sw (leading dim ldw), clear the
// failure flags, and (Fb != 0)
// the boundary rows F_b of the basis augmentation: with K_l = sum_i X_i S_il
// at the two boundary cells, F_b[0] = f_L where v_1 > 0 else K(x_0).V and
// F_b[1] = f_R where v_1 < 0 else K(x_{nx-1}).V (the sums in the order of
// k_xmul).
__global__ __launch_bounds__(256) void k_add_begin(const double* __restrict__ X, int r, int nx,
                                                   const double* __restrict__ S, int lds,
                                                   double* __restrict__ Sw, int ldw,
                                                   int* __restrict__ flag,
                                                   const double* __restrict__ V,
                                                   const double* __restrict__ fL,
                                                   const double* __restrict__ fR, VGeo g,
                                                   double* __restrict__ Fb) {
  __shared__ double kb[2][64];
  const int t = threadIdx.x;
  if (blockIdx.x == 0) {
    for (int e = t; e < r * r; e += blockDim.x) Sw[(e / r) * ldw + e % r] = S[(e / r) * lds + e % r];
    if (t < 2) flag[t] = 0;
  }
  if (!Fb) return;
  if (t < 2 * r) {
    const int side = t / r, l = t % r;
    const int x = side ? nx - 1 : 0;
    double s = 0.0;
    for (int i = 0; i < r; ++i) s += X[(long)i * nx + x] * S[i * lds + l];
    kb[side][l] = s;
  }
  __syncthreads();
  const int q = blockIdx.x * blockDim.x + t;
  if (q >= g.n) return;
  double a = 0.0, b = 0.0;
  for (int l = 0; l < r; ++l) {
    const double v = V[(long)l * g.n + q];
    a += kb[0][l] * v;
    b += kb[1][l] * v;
  }
  const double v1 = g.v1(q);
  Fb[q] = v1 > 0 ? fL[q] : a;
  Fb[g.n + q] = v1 < 0 ? fR[q] : b;
}

// Diffusive walls, boundary rows: k_add_begin leaves the wall Maxwellian's
// shape on the incoming half of a wall's row and the adjacent cell on the
// outgoing half; the incoming half is scaled by rho_w taken from the
// outgoing half.  One block per side.
__global__ __launch_bounds__(1024) void k_wall_rows(double* __restrict__ Fb,
                                                    const double* __restrict__ fL,
                                                    const double* __restrict__ fR, int wl, int wr,
                                                    VGeo g) {
  const int side = blockIdx.x;
  if (!(side == 0 ? wl : wr)) return;
  __shared__ double red[1024 / 64 + 1];
  const double* M = side ? fR : fL;
  double* row = Fb + (long)side * g.n;
  const int plane = g.d == 3 ? g.N * g.N : g.N;
  const double rho = wall::density<1024>(side, row, M, g.n, g.L, g.dv, plane, red);
  for (int q = threadIdx.x; q < g.n; q += 1024)
    if (wall::incoming(side, g.v1(q))) row[q] = rho * M[q];
}

// Diffusive walls, ghost values: rho_w = sum_l K_l(x_b) a_l / den is linear
// in the adjacent cell's K (a_l = sum_q (v.n)_out V_l, den = sum_q
// |v.n|_in M_w), so the ghost
//   g_j = rho_w <M_w 1_in, V_j> + sum_l K_l <1_out V_l V_j>
// is K times (Mo + (a / den) gin^T): the rank-one term is folded into the
// outflow matrix Mo[l r + j] and the inflow vector gin is cleared.  One
// block per side, one wave per sum (lanes strided, fixed order).
__global__ __launch_bounds__(1024) void k_wall_fold(const double* __restrict__ V, int r,
                                                    const double* __restrict__ fL,
                                                    const double* __restrict__ fR, int wl, int wr,
                                                    VGeo g, double* __restrict__ ginL,
                                                    double* __restrict__ ginR,
                                                    double* __restrict__ MoL,
                                                    double* __restrict__ MoR) {
  const int side = blockIdx.x;
  if (!(side == 0 ? wl : wr)) return;
  __shared__ double a[65];
  const double* M = side ? fR : fL;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int l = wv; l <= r; l += 16) {
    double sum = 0.0;
    for (int q = lane; q < g.n; q += 64) {
      const double v1 = g.v1(q);
      sum += l < r ? wall::out_weight(side, v1) * V[(long)l * g.n + q]
                   : wall::in_weight(side, v1) * M[q];
    }
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
    if (lane == 0) a[l] = sum;
  }
  __syncthreads();
  double* Mo = side ? MoR : MoL;
  double* gin = side ? ginR : ginL;
  const double den = a[r];
  for (int e = threadIdx.x; e < r * r; e += 1024) Mo[e] += a[e / r] / den * gin[e % r];
  __syncthreads();
  if (threadIdx.x < r) gin[threadIdx.x] = 0.0;
}

// The added basis rows Vb_i = sum_l Ub[l][i] Fb_l (i < rb, k_rows_comb with
// scale 1), zero rows r .. r+rb-1 of X, and the zero-padded S^ (rk = r + rb).
__global__ __launch_bounds__(256) void k_add_rows(const double* __restrict__ Fb, long n,
                                                  const double* __restrict__ Ub, int rb,
                                                  double* __restrict__ Vb, double* __restrict__ Xz,
                                                  long nxz, const double* __restrict__ Sw, int r,
                                                  double* __restrict__ Shat) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (e < n) {
    double s = 0.0;
    for (int l = 0; l < 2; ++l) s += Ub[l * 2 + i] * Fb[(long)l * n + e];
    Vb[(long)i * n + e] = 1.0 * s;
  }
  if (i == 0) {
    for (long z = e; z < nxz; z += (long)gridDim.x * blockDim.x) Xz[z] = 0.0;
    if (blockIdx.x == 0) {
      const int rk = r + rb;
      for (int t = threadIdx.x; t < rk * rk; t += blockDim.x) {
        const int a = t / rk, b = t % rk;
        Shat[t] = (a < r && b < r) ? Sw[a * r + b] : 0.0;
      }
    }
  }
}

// V (FP64) -> V32, and (src != 0) S^ -> Sw by the first block.
__global__ void k_to_f32_copy_S(const double* __restrict__ in, long count, float* __restrict__ out,
                                const double* __restrict__ src, int rs, double* __restrict__ dst,
                                int lds) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < count) out[e] = (float)in[e];
  if (src && blockIdx.x == 0)
    for (int t = threadIdx.x; t < rs * rs; t += blockDim.x)
      dst[(t / rs) * lds + t % rs] = src[(t / rs) * rs + t % rs];
}

// ------------------------------------------------ FP64 defect correction
// Basis functions the defect correction carries (r_cap bound of the flag).
constexpr int DEFECT_MAX = 32;

// Index of the pair (a, b), a <= b, among the pairs of r functions in the
// step's order (a-major, b from a up).
__device__ __forceinline__ int pair_index(int a, int b, int r) {
  return a * r - a * (a - 1) / 2 + (b - a);
}

// D = Q64 - Q32, element by element (the FP64 defect of the FP32 pairs).
__global__ void k_defect_store(const double* __restrict__ Q64, const float* __restrict__ Q32,
                               long count, double* __restrict__ D) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e < count) D[e] = Q64[e] - (double)Q32[e];
}

// R (r x rr, row-major) into LDS with row stride DM, zeros elsewhere, so
// that the fixed-length loops below read zeros past rr.
template <int DM>
__device__ __forceinline__ void load_rot(double* Rs, const double* __restrict__ R, int r, int rr) {
  for (int i = threadIdx.x; i < DM * DM; i += blockDim.x) {
    const int a = i / DM, m = i % DM;
    Rs[i] = (a < r && m < rr) ? R[a * rr + m] : 0.0;
  }
  __syncthreads();
}

// First half of carrying the kept defect to the step's basis: for every
// velocity point v, T[a][n](v) = sum_m R[a][m] D_mn(v) with D symmetric in
// (m, n) and stored once per pair of the rr kept functions.  One thread per
// (v, n): grid (velocity blocks, rr).
template <int DM>
__global__ __launch_bounds__(64) void k_defect_carry1(const double* __restrict__ D, int rr,
                                                      const double* __restrict__ R, int r, long nv,
                                                      double* __restrict__ T) {
  __shared__ double Rs[DM * DM];
  load_rot<DM>(Rs, R, r, rr);
  const long v = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (v >= nv) return;
  double col[DM];
#pragma unroll
  for (int m = 0; m < DM; ++m)
    col[m] = m < rr ? D[(long)pair_index(m < n ? m : n, m < n ? n : m, rr) * nv + v] : 0.0;
  for (int a = 0; a < r; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < DM; ++m) acc += Rs[a * DM + m] * col[m];
    T[((long)a * rr + n) * nv + v] = acc;
  }
}

// Second half: Q[p](v) = Q32[p](v) + sum_n R[b][n] T[a][n](v) for every pair
// p = (a, b), a <= b, of the step's r functions.  One thread per (v, a):
// grid (velocity blocks, r).
template <int DM>
__global__ __launch_bounds__(64) void k_defect_carry2(const double* __restrict__ T, int rr,
                                                      const double* __restrict__ R, int r, long nv,
                                                      const float* __restrict__ Q32,
                                                      double* __restrict__ Q) {
  __shared__ double Rs[DM * DM];
  load_rot<DM>(Rs, R, r, rr);
  const long v = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (v >= nv) return;
  double row[DM];
#pragma unroll
  for (int n = 0; n < DM; ++n) row[n] = n < rr ? T[((long)a * rr + n) * nv + v] : 0.0;
  for (int b = a; b < r; ++b) {
    const long p = pair_index(a, b, r);
    double acc = 0.0;
#pragma unroll
    for (int n = 0; n < DM; ++n) acc += Rs[b * DM + n] * row[n];
    Q[p * nv + v] = (double)Q32[p * nv + v] + acc;
  }
}

// Commit after the drop decision: X_i = sum_l U[l][i] X1_l and V_i =
// sum_l Wm[l][i] V1_l for i < keep (k_rows_comb), and S = diag(sig) (k_diag),
// in one launch: grid.y = keep, x blocks over max(nx, n).
__global__ __launch_bounds__(256) void k_commit(const double* __restrict__ X1, int r, long nx,
                                                const double* __restrict__ U,
                                                const double* __restrict__ V1, long n,
                                                const double* __restrict__ Wm, int keep,
                                                double* __restrict__ X, double* __restrict__ V,
                                                const double* __restrict__ sig,
                                                double* __restrict__ S, int lds) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (e < nx) {
    double s = 0.0;
    for (int l = 0; l < r; ++l) s += U[l * r + i] * X1[(long)l * nx + e];
    X[(long)i * nx + e] = 1.0 * s;
  }
  if (e < n) {
    double s = 0.0;
    for (int l = 0; l < r; ++l) s += Wm[l * r + i] * V1[(long)l * n + e];
    V[(long)i * n + e] = 1.0 * s;
  }
  if (blockIdx.x == 0 && i == 0)
    for (int t = threadIdx.x; t < keep * keep; t += blockDim.x) {
      const int a = t / keep, b = t % keep;
      S[a * lds + b] = (a == b) ? sig[a] : 0.0;
    }
}


// out = A B^T for r x r row-major A, B
__global__ void k_mul_bt(const double* A, const double* B, int r, double* out) {
  for (int t = threadIdx.x; t < r * r; t += blockDim.x) {
    const int i = t / r, j = t % r;
    double s = 0.0;
    for (int k = 0; k < r; ++k) s += A[i * r + k] * B[j * r + k];
    out[t] = s;
  }
}

// One pass of block Gram-Schmidt with Cholesky normalisation of rb <= 2 new
// rows B (stored right after the r rows of V, row length n) against the r
// rows of V, orthonormal in <.,.>_v.  With G = <B, [V; B]>_v (rb x (r + rb),
// row-major), C = G[:, :r] and M = G[:, r:] - C C^T = L L^T (Cholesky),
//   B <- L^{-1} (B - C V),
// so that [V; B] spans the same space with orthonormal rows.  Two passes give
// orthogonality to rounding as long as each new row keeps a part outside
// span V of relative size above 1e-6; flag[0] is set (pass 0 writes, pass 1
// ors) when a pivot of M is below 1e-12 of the matching diagonal of G or not
// finite, and the caller then orthogonalises by Householder QR instead.
__global__ __launch_bounds__(256) void k_orth_pass(double* __restrict__ V, int r, int rb, long n,
                                                   const double* __restrict__ G, int pass,
                                                   int* __restrict__ flag) {
  __shared__ double C[2 * 64];
  __shared__ double Gb[4];  // G[:, r:]
  __shared__ double Li[4];  // L^{-1}, row-major 2 x 2
  __shared__ int fl;
  const int ld = r + rb;
  for (int e = threadIdx.x; e < rb * r; e += blockDim.x) C[e] = G[(e / r) * ld + e % r];
  if (threadIdx.x < rb * rb) Gb[threadIdx.x] = G[(threadIdx.x / rb) * ld + r + threadIdx.x % rb];
  if (threadIdx.x == 0) fl = (pass == 0 || blockIdx.x != 0) ? 0 : flag[0];
  __syncthreads();
  // M = G[:, r:] - C C^T: wave 0, lanes 16 q + u add the terms j = u, u + 16, ..
  // of entry q = (i, k), then sums over the 16 lanes (butterfly)
  if (threadIdx.x < 64) {
    const int q = threadIdx.x >> 4, u = threadIdx.x & 15;
    const int i = q >> 1, k = q & 1;
    double part = 0.0;
    if (i < rb && k < rb)
      for (int j = u; j < r; j += 16) part += C[i * r + j] * C[k * r + j];
    for (int off = 8; off > 0; off >>= 1) part += __shfl_xor(part, off, 16);
    const double m00 = Gb[0] - __shfl(part, 0, 64);
    const double m10 = rb == 2 ? Gb[2] - __shfl(part, 32, 64) : 0.0;
    const double m11 = rb == 2 ? Gb[3] - __shfl(part, 48, 64) : 1.0;
    if (threadIdx.x == 0) {
      // L = [[l00, 0], [l10, l11]], L^{-1} from reciprocal square roots
      bool bad = !(m00 > 1e-12 * Gb[0]) || !isfinite(m00);
      const double i00 = bad ? 1.0 : rsqrt(m00);
      const double l10 = m10 * i00;
      double i11 = 1.0;
      if (rb == 2) {
        const double piv = m11 - l10 * l10;
        const bool bad1 = !(piv > 1e-12 * Gb[3]) || !isfinite(piv) || !isfinite(l10);
        bad = bad || bad1;
        i11 = bad1 ? 1.0 : rsqrt(piv);
      }
      Li[0] = bad ? 1.0 : i00;
      Li[1] = 0.0;
      Li[2] = bad ? 0.0 : -l10 * i00 * i11;
      Li[3] = bad ? 1.0 : i11;
      if (blockIdx.x == 0) flag[0] = fl | (bad ? 1 : 0);
    }
  }
  __syncthreads();
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double b0 = V[(long)r * n + e];
  double b1 = rb == 2 ? V[(long)(r + 1) * n + e] : 0.0;
  for (int j0 = 0; j0 < r; j0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = j0 + u < r ? V[(long)(j0 + u) * n + e] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (j0 + u < r) {
        b0 -= C[j0 + u] * v[u];
        if (rb == 2) b1 -= C[r + j0 + u] * v[u];
      }
    }
  }
  V[(long)r * n + e] = Li[0] * b0;
  if (rb == 2) V[(long)(r + 1) * n + e] = Li[2] * b0 + Li[3] * b1;
}

// Read-back record of a step: res[0..3], flag[0], sigma_b[0..1], flag[1],
// sigma[0..r), g[0..r)  (absent inputs read as 0).
__global__ void k_pack(const double* res, const int* flag, const double* sb, const double* sg,
                       const double* g, int r, double* out) {
  const int t = threadIdx.x;
  if (t < 4) out[t] = res[t];
  if (t == 4) out[4] = flag ? (double)flag[0] : 0.0;
  if (t == 5 || t == 6) out[t] = sb ? sb[t - 5] : 0.0;
  if (t == 7) out[7] = flag ? (double)flag[1] : 0.0;
  for (int i = t; i < r; i += blockDim.x) {
    out[8 + i] = sg ? sg[i] : 0.0;
    out[8 + r + i] = g ? g[i] : 0.0;
  }
}

// Read-back record of the two-dimensional step: the residual, then (r > 0)
// the singular values of the new S and the drop terms g.
__global__ void k_pack2d(const double* err, const double* sg, const double* g, int r, double* out) {
  const int t = threadIdx.x;
  if (t == 0) out[0] = err[0];
  for (int i = t; i < r; i += blockDim.x) {
    out[1 + i] = sg[i];
    out[1 + r + i] = g[i];
  }
}

// dst[k][i] = src[i][off + k] (r x r, src leading dimension lds)
__global__ void k_gather_T(const double* src, int lds, int off, int r, double* dst) {
  const int t = threadIdx.x + blockIdx.x * blockDim.x;
  if (t >= r * r) return;
  const int k = t / r, i = t % r;
  dst[t] = src[(long)i * lds + off + k];
}

// L-step on the FP64 matrix cores, for r <= 16: each wavefront takes 16
// velocity points q0..q0+15 and forms the 16 x 16 tiles (rows i < 16)
//   l = S2 V,  dp = Dp V,  dm = Dm V   (sum over m < r)
//   cq = T Q                          (sum over pairs p < P)
// with v_mfma_f64_16x16x4f64 (lane l supplies the first operand's element
// (l % 16, l / 16) and the second's (l / 16, l % 16); it holds result
// entries (4v + l / 16, l % 16)), then
//   L1_i = l_i - dt (v1+ dp_i + v1- dm_i) + dt cq_i,  dL_i = L1_i - l_i.
template <typename TQ>
__global__ __launch_bounds__(256) void k_lstep_mfma(const double* __restrict__ V, int r, int n,
                                                    const double* __restrict__ S2,
                                                    const double* __restrict__ Dp,
                                                    const double* __restrict__ Dm,
                                                    const double* __restrict__ T,
                                                    const TQ* __restrict__ Q, int P, double dt,
                                                    VGeo g, double* __restrict__ L1,
                                                    double* __restrict__ dL) {
  const int lane = threadIdx.x & 63;
  const int q0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (q0 >= n) return;
  const int li = lane & 15, lk = lane >> 4;
  const int qq = q0 + li;  // this lane's point in the second operand and the result
  const bool qin = qq < n;
  v4d al = {0.0, 0.0, 0.0, 0.0}, ap = al, am = al, ac = al;
  for (int m0 = 0; m0 < r; m0 += 4) {
    const int m = m0 + lk;
    const double v = (m < r && qin) ? V[(long)m * n + qq] : 0.0;
    const bool rin = li < r && m < r;
    const double s2 = rin ? S2[li * r + m] : 0.0;
    const double dpv = rin ? Dp[li * r + m] : 0.0;
    const double dmv = rin ? Dm[li * r + m] : 0.0;
    al = __builtin_amdgcn_mfma_f64_16x16x4f64(s2, v, al, 0, 0, 0);
    ap = __builtin_amdgcn_mfma_f64_16x16x4f64(dpv, v, ap, 0, 0, 0);
    am = __builtin_amdgcn_mfma_f64_16x16x4f64(dmv, v, am, 0, 0, 0);
  }
  for (int p0 = 0; p0 < P; p0 += 16) {
    double qv[4], tv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = p0 + 4 * u + lk;
      qv[u] = (p < P && qin) ? (double)Q[(long)p * n + qq] : 0.0;
      tv[u] = (p < P && li < r) ? T[li * P + p] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) ac = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[u], qv[u], ac, 0, 0, 0);
  }
  if (!qin) return;
  const double v1 = g.v1(qq);
  const double vp = v1 > 0 ? v1 : 0.0, vm = v1 < 0 ? v1 : 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * v + lk;
    if (i < r) {
      const double d = -dt * (vp * ap[v] + vm * am[v]) + dt * ac[v];
      L1[(long)i * n + qq] = al[v] + d;
      dL[(long)i * n + qq] = d;
    }
  }
}

// ---------------------------------------------- fused x-side kernels --
// For r <= RM <= 16.  K = X S (K_l(x) = sum_i X_i(x) S_il) is formed where
// it is needed instead of being stored; every block computes the ghost
// values of K itself (from K at the two wall cells).

// Loads a row-major r x r matrix into a zero-padded 16 x 16 LDS array.
__device__ __forceinline__ void lds_mat16(double* dst, const double* src, int r, int ld) {
  for (int e = threadIdx.x; e < 256; e += blockDim.x) {
    const int i = e / 16, j = e % 16;
    dst[e] = (i < r && j < r) ? src[i * ld + j] : 0.0;
  }
}

// Ghost values of K = X S at both walls into g[0][j] (left), g[1][j]
// (right); S, MoL, MoR in LDS (16 x 16).  Ends with a barrier.
template <int RM>
__device__ void block_ghosts(const double* X, int r, int nx, const double* Ss, const double* ginL,
                             const double* ginR, const double* MoLs, const double* MoRs,
                             double (*kb)[16], double (*g)[16]) {
  const int t = threadIdx.x;
  if (t < 32) {
    const int side = t / 16, l = t % 16;
    const int x = side ? nx - 1 : 0;
    double xv[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) xv[i] = i < r ? X[(long)i * nx + x] : 0.0;
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < RM; ++i) v += xv[i] * Ss[i * 16 + l];
    kb[side][l] = l < r ? v : 0.0;
  }
  __syncthreads();
  if (t < 32) {
    const int side = t / 16, j = t % 16;
    double v = 0.0;
    if (j < r) {
      v = side ? ginR[j] : ginL[j];
      const double* Mo = side ? MoRs : MoLs;
      for (int l = 0; l < r; ++l) v += kb[side][l] * Mo[l * 16 + j];
    }
    g[side][j] = v;
  }
  __syncthreads();
}

// K = X S for the cells x0 - 1 .. x0 + KB (those outside 0..nx-1 are the
// ghost values) into Ks[l][1 + x - x0]; thread t computes cell x0 - 1 + t.
// S, ghosts in LDS.  Ends with a barrier.
template <int RM, int KB>
__device__ void block_K(const double* X, int r, int nx, int x0, const double* Ss,
                        const double (*g)[16], double (*Ks)[KB + 3]) {
#pragma unroll 1
  for (int t = threadIdx.x; t < KB + 2; t += blockDim.x) {
    const int x = x0 - 1 + t;
    double xv[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) xv[i] = (i < r && x >= 0 && x < nx) ? X[(long)i * nx + x] : 0.0;
    // column loop kept rolled: S is read from LDS per column, not held in registers
#pragma unroll 1
    for (int l = 0; l < RM; ++l) {
      double v = 0.0;
#pragma unroll
      for (int i = 0; i < RM; ++i) v += xv[i] * Ss[i * 16 + l];
      if (x < 0) v = g[0][l];
      else if (x >= nx) v = g[1][l];
      Ks[l][t] = v;
    }
  }
  __syncthreads();
}

// K-step: K = X S, ghosts, and
// K1_j = K_j + dt (-sum_l A+_jl D+K_l - sum_l A-_jl D-K_l + sum_{m<=n} C_j,(mn) w K_m K_n),
// dK = K1 - K; pairs (m, n), m <= n, in row order (index m r - m (m - 1) / 2 + n - m).
// Block (cells x0 .. x0 + 63, outputs j = JB blockIdx.y .. + JB - 1).
constexpr int KSB = 64;
template <int RM>
__global__ __launch_bounds__(KSB) void k_kstep_fused(const double* __restrict__ X,
                                                     const double* __restrict__ S, int r, int nx,
                                                     double dx, double dt, int JB,
                                                     const double* __restrict__ ginL,
                                                     const double* __restrict__ ginR,
                                                     const double* __restrict__ MoL,
                                                     const double* __restrict__ MoR,
                                                     const double* __restrict__ Ap,
                                                     const double* __restrict__ Am,
                                                     const double* __restrict__ C, int P,
                                                     double* __restrict__ K1,
                                                     double* __restrict__ dK) {
  __shared__ double Ss[256], MoLs[256], MoRs[256];
  __shared__ double kb[2][16], g[2][16];
  __shared__ double Ks[16][KSB + 3];
  lds_mat16(Ss, S, r, r);
  lds_mat16(MoLs, MoL, r, r);
  lds_mat16(MoRs, MoR, r, r);
  __syncthreads();
  block_ghosts<RM>(X, r, nx, Ss, ginL, ginR, MoLs, MoRs, kb, g);
  const int x0 = blockIdx.x * KSB;
  block_K<RM, KSB>(X, r, nx, x0, Ss, g, Ks);
  const int t = threadIdx.x, x = x0 + t;
  if (x >= nx) return;
  double kc[RM], dp[RM], dm[RM];
#pragma unroll
  for (int l = 0; l < RM; ++l) {
    const double b = Ks[l][t + 1];
    kc[l] = b;
    dp[l] = (b - Ks[l][t]) / dx;
    dm[l] = (Ks[l][t + 2] - b) / dx;
  }
  const int j0 = blockIdx.y * JB, j1 = min(r, j0 + JB);
  for (int j = j0; j < j1; ++j) {
    double v = 0.0, kj = 0.0;
#pragma unroll
    for (int l = 0; l < RM; ++l) {
      if (l < r) v -= Ap[j * r + l] * dp[l] + Am[j * r + l] * dm[l];
      if (l == j) kj = kc[l];
    }
    // sum_{m <= n} C_j,(mn) w K_m K_n = sum_m K_m (C_j,(mm) K_m + sum_{n > m} C_j,(mn) 2 K_n)
    const double* cj = C + (long)j * P;
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      if (m < r) {
        const int p0 = m * r - m * (m - 1) / 2 - m;
        double tm = cj[p0 + m] * kc[m];
#pragma unroll
        for (int n2 = m + 1; n2 < RM; ++n2)
          if (n2 < r) tm += cj[p0 + n2] * (2.0 * kc[n2]);
        v += kc[m] * tm;
      }
    }
    const double d = dt * v;
    K1[(long)j * nx + x] = kj + d;
    dK[(long)j * nx + x] = d;
  }
}

// x-side inner products out[i][c] = dx sum_x X1_i(x) Y_c(x) with K = X1 S:
//   c < r: D+K_c;  c < 2r: D-K_(c-r);  c < 2r + P: w_p K_m K_n;
//   next r columns (when Zk): Zk rows;  next r (when Zx): Zx rows,
// written to Dp, Dm, T (r x r, r x r, r x P), kx (r x r, kx[i][c]) and
// AadT (Aad[c][i] = <Zx_c, X1_i>).  One block per 16 columns; K of the
// 256-cell chunk in LDS; the sum over x on the FP64 matrix cores (operand
// layout as in k_gram_batch).
template <int RM>
__global__ __launch_bounds__(256) void k_xside(const double* __restrict__ X1, int r, int nx, double dx,
                                               const double* __restrict__ S,
                                               const double* __restrict__ ginL,
                                               const double* __restrict__ ginR,
                                               const double* __restrict__ MoL,
                                               const double* __restrict__ MoR, int P,
                                               const int* __restrict__ pm,
                                               const int* __restrict__ pn,
                                               const double* __restrict__ Zk,
                                               const double* __restrict__ Zx, double* __restrict__ Dp,
                                               double* __restrict__ Dm, double* __restrict__ T,
                                               double* __restrict__ kx, double* __restrict__ Aad) {
  __shared__ double Ss[256], MoLs[256], MoRs[256];
  __shared__ double kb[2][16], g[2][16];
  __shared__ double Ks[16][256 + 3];
  __shared__ double Xs[16][257];
  __shared__ double Ys[16][257];
  __shared__ int pms[136], pns[136];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  lds_mat16(Ss, S, r, r);
  lds_mat16(MoLs, MoL, r, r);
  lds_mat16(MoRs, MoR, r, r);
  for (int e = t; e < P; e += blockDim.x) {
    pms[e] = pm[e];
    pns[e] = pn[e];
  }
  __syncthreads();
  block_ghosts<RM>(X1, r, nx, Ss, ginL, ginR, MoLs, MoRs, kb, g);
  const int nzk = Zk ? r : 0, nzx = Zx ? r : 0;
  const int ncols = 2 * r + P + nzk + nzx;
  const int c0 = blockIdx.x * 16;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int x0 = 0; x0 < nx; x0 += 256) {
    block_K<RM, 256>(X1, r, nx, x0, Ss, g, Ks);
    const int x = x0 + t;
    const bool xin = x < nx;
#pragma unroll
    for (int i = 0; i < 16; ++i) Xs[i][t] = (i < r && xin) ? X1[(long)i * nx + x] : 0.0;
    for (int cc = 0; cc < 16; ++cc) {
      const int c = c0 + cc;
      double y = 0.0;
      if (xin && c < ncols) {
        if (c < r) {
          y = (Ks[c][t + 1] - Ks[c][t]) / dx;
        } else if (c < 2 * r) {
          y = (Ks[c - r][t + 2] - Ks[c - r][t + 1]) / dx;
        } else if (c < 2 * r + P) {
          const int p = c - 2 * r, m = pms[p], n2 = pns[p];
          y = (m == n2 ? 1.0 : 2.0) * Ks[m][t + 1] * Ks[n2][t + 1];
        } else if (c < 2 * r + P + nzk) {
          y = Zk[(long)(c - 2 * r - P) * nx + x];
        } else {
          y = Zx[(long)(c - 2 * r - P - nzk) * nx + x];
        }
      }
      Ys[cc][t] = y;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int xx = 64 * wv + 4 * st + (lane >> 4);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[lane & 15][xx], Ys[lane & 15][xx], acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // four waves' tiles, in order
  double* red = &Xs[0][0];  // 4 x 256 doubles
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv * 256 + (4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc[v];
  __syncthreads();
  const int i = t / 16, c = c0 + t % 16;
  if (i < r && c < ncols) {
    const double o = dx * (((red[t] + red[256 + t]) + red[512 + t]) + red[768 + t]);
    if (c < r) Dp[i * r + c] = o;
    else if (c < 2 * r) Dm[i * r + c - r] = o;
    else if (c < 2 * r + P) T[i * P + c - 2 * r] = o;
    else if (c < 2 * r + P + nzk) kx[i * r + c - 2 * r - P] = o;
    else Aad[(c - 2 * r - P - nzk) * r + i] = o;
  }
}

// S2 = S1 + dt (Dp Ap^T + Dm Am^T - T C^T), dS = S2 - S1, for r <= 16
__global__ __launch_bounds__(256) void k_supdate16(const double* __restrict__ S1,
                                                   const double* __restrict__ Dp,
                                                   const double* __restrict__ Dm,
                                                   const double* __restrict__ T,
                                                   const double* __restrict__ Ap,
                                                   const double* __restrict__ Am,
                                                   const double* __restrict__ C, int r, int P,
                                                   double dt, double* __restrict__ S2,
                                                   double* __restrict__ dS) {
  __shared__ double D1[256], D2[256], A1[256], A2[256];
  __shared__ double Ts[16 * 136], Cs[16 * 136];
  lds_mat16(D1, Dp, r, r);
  lds_mat16(D2, Dm, r, r);
  lds_mat16(A1, Ap, r, r);
  lds_mat16(A2, Am, r, r);
#pragma unroll 4
  for (int e = threadIdx.x; e < r * P; e += blockDim.x) {
    Ts[e] = T[e];
    Cs[e] = C[e];
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= r * r) return;
  const int i = t / r, j = t % r;
  double v = 0.0;
  for (int l = 0; l < r; ++l) v += D1[i * 16 + l] * A1[j * 16 + l] + D2[i * 16 + l] * A2[j * 16 + l];
  for (int p = 0; p < P; ++p) v -= Ts[i * P + p] * Cs[j * P + p];
  S2[t] = S1[t] + dt * v;
  dS[t] = dt * v;
}

// err^2 pieces (as k_err), one block: sum of dK^2 with loads in batches,
// the r x r sums one entry per thread, then fixed-order tree sums.
__global__ __launch_bounds__(256) void k_err16(const double* __restrict__ dK, long nK, double dx,
                                               const double* __restrict__ dS, int r,
                                               const double* __restrict__ GdL,
                                               const double* __restrict__ kx,
                                               const double* __restrict__ lv,
                                               double* __restrict__ res) {
  __shared__ double red[5][256];
  const int t = threadIdx.x;
  double a = 0.0;
  for (long e0 = 0; e0 < nK; e0 += 256 * 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const long e = e0 + k * 256 + t;
      v[k] = e < nK ? dK[e] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) a += v[k] * v[k];
  }
  double b = 0.0, c = 0.0, I = 0.0, II = 0.0, III = 0.0;
  if (t < r * r) {
    const double ds = dS[t], kv = kx[t], lvv = lv[t];
    b = ds * ds;
    I = kv * ds;
    II = lvv * ds;
    III = kv * lvv;
    if (t / r == t % r) c = GdL[t];
  }
  red[0][t] = a;
  red[1][t] = b;
  red[2][t] = c;
  red[3][t] = I;
  red[4][t] = II + III;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st)
      for (int k = 0; k < 5; ++k) red[k][t] += red[k][t + st];
    __syncthreads();
  }
  if (t == 0) {
    const double A = dx * red[0][0];
    res[0] = A + red[1][0] + red[2][0] + 2.0 * (red[3][0] + red[4][0]);
    res[1] = A;
    res[2] = red[1][0];
    res[3] = red[2][0];
  }
}

// <f^n, D_keep> terms (as k_fnD_terms) for r <= 16, inputs staged in LDS
__global__ __launch_bounds__(256) void k_fnD16(const double* S, const double* A, const double* U,
                                               const double* sig, const double* W, const double* B,
                                               int r, double* g) {
  __shared__ double Sm[256], Am_[256], Um[256], Wm[256], Bm[256], AU[256], BW[256];
  lds_mat16(Sm, S, r, r);
  lds_mat16(Am_, A, r, r);
  lds_mat16(Um, U, r, r);
  lds_mat16(Wm, W, r, r);
  lds_mat16(Bm, B, r, r);
  __syncthreads();
  const int t = threadIdx.x, k = t / 16, q = t % 16;
  double au = 0.0, bw = 0.0;
  for (int i = 0; i < r; ++i) {
    au += Am_[k * 16 + i] * Um[i * 16 + q];
    bw += Bm[k * 16 + i] * Wm[i * 16 + q];
  }
  AU[t] = au;
  BW[t] = bw;
  __syncthreads();
  if (t < r) {
    double v = 0.0;
    for (int kk = 0; kk < r; ++kk) {
      double sb = 0.0;
      for (int l = 0; l < r; ++l) sb += Sm[kk * 16 + l] * BW[l * 16 + t];
      v += AU[kk * 16 + t] * sb;
    }
    g[t] = sig[t] * v;
  }
}

// ===================================================== two-dimensional space
// Rectangle with nx x ny cells, cell p = ix ny + iy; arrays over cells are
// rows of nc = nx ny values.  Faces 0 x_lo, 1 x_hi, 2 y_lo, 3 y_hi; the face
// cells of all four faces are numbered b = [x_lo: ny][x_hi: ny][y_lo: nx]
// [y_hi: nx], each face in order of the other coordinate.

__device__ __forceinline__ void face_of(int b, int nx, int ny, int& k, int& c) {
  if (b < ny) {
    k = 0; c = b;
  } else if (b < 2 * ny) {
    k = 1; c = b - ny;
  } else if (b < 2 * ny + nx) {
    k = 2; c = b - 2 * ny;
  } else {
    k = 3; c = b - 2 * ny - nx;
  }
}
__device__ __forceinline__ long face_cell(int k, int c, int nx, int ny) {
  return k == 0 ? c : k == 1 ? (long)(nx - 1) * ny + c : k == 2 ? (long)c * ny
                                                             : (long)c * ny + ny - 1;
}

// Velocity-side pieces of one face: Mo = <1_out V_l V_j> (r x r), gin =
// <f_c 1_in, V_j> (r x rows, rows = 1 or one per face cell).  A diffusive
// wall (wall = 1) also has a_l = sa sum_q (v.n)_out V_l and den_c = sd sum_q
// |v.n|_in f_c, so that rho_w(c) = (sum_l K_l(c) a_l) / den_c.
struct Face2 {
  const double* Mo;
  const double* gin;
  const double* a;
  const double* den;
  int rows, wall;
  double sa, sd;
};
// classes 0..3: the rectangle's faces; 4 + k: obstacle faces of outward normal k
struct Faces2 {
  Face2 f[8];
};

// face b: class cls, the gas cell p next to it and its boundary-function row c
__device__ __forceinline__ void face_at(int b, int nx, int ny, const Obs2& ob, int& cls, long& p,
                                        int& c) {
  if (b < ob.nface) {
    int k;
    face_of(b, nx, ny, k, c);
    cls = k;
    p = face_cell(k, c, nx, ny);
  } else {
    const int i = b - ob.nface;
    p = ob.face[2 * i];
    cls = 4 + ob.face[2 * i + 1];
    c = 0;
  }
}

// Ghost rows of K on every face (the rectangle's face cells, then the
// obstacle's faces; eq. boundary general):
//   G[b][j] = sum_l K_l(c) Mo_lj + (inflow: gin_jc; wall: rho_w(c) gin_jc).
__global__ void k_ghosts2d(const double* __restrict__ K, int r, int nx, int ny, Faces2 fs, Obs2 ob,
                           double* __restrict__ G) {
  const int b = blockIdx.x, j = threadIdx.x;
  if (j >= r) return;
  int cls, c;
  long p;
  face_at(b, nx, ny, ob, cls, p, c);
  const long nc = (long)nx * ny;
  const Face2& F = fs.f[cls];
  const int cr = F.rows > 1 ? c : 0;
  double g = 0.0;
  for (int l = 0; l < r; ++l) g += K[l * nc + p] * F.Mo[l * r + j];
  if (F.wall) {
    double ka = 0.0;
    for (int l = 0; l < r; ++l) ka += K[l * nc + p] * F.a[l];
    g += (F.sa * ka) / (F.sd * F.den[cr]) * F.gin[(long)j * F.rows + cr];
  } else {
    g += F.gin[(long)j * F.rows + cr];
  }
  G[(long)b * r + j] = g;
}

// K_l at the neighbour p + step e_axis (step = -1 or 1), the face ghost where
// that neighbour lies outside or is solid
__device__ __forceinline__ double nb2(const double* K, const double* G, int r, int nx, int ny,
                                      int l, long p, int axis, int step, const Obs2& ob) {
  const long nc = (long)nx * ny;
  const int ix = (int)(p / ny), iy = (int)(p % ny);
  if (axis == 0) {
    const int i = ix + step;
    if (i >= 0 && i < nx) {
      const int b = ob.towards(p, step < 0 ? 0 : 1);
      return b >= 0 ? G[(long)b * r + l] : K[l * nc + p + (long)step * ny];
    }
    return G[(long)(step < 0 ? iy : ny + iy) * r + l];
  }
  const int i = iy + step;
  if (i >= 0 && i < ny) {
    const int b = ob.towards(p, step < 0 ? 2 : 3);
    return b >= 0 ? G[(long)b * r + l] : K[l * nc + p + step];
  }
  return G[(long)(step < 0 ? 2 * ny + ix : 2 * ny + nx + ix) * r + l];
}

// D^a_+- K_l at cell p, k = 0 D1+, 1 D1-, 2 D2+, 3 D2- (backward / forward
// differences along x, then y)
__device__ __forceinline__ double dk2(const double* K, const double* G, int r, int nx, int ny,
                                      int l, long p, int k, double dx, double dy, const Obs2& ob) {
  const double k0 = K[l * (long)nx * ny + p];
  const int axis = k >> 1;
  const double h = axis == 0 ? dx : dy;
  return (k & 1) ? (nb2(K, G, r, nx, ny, l, p, axis, 1, ob) - k0) / h
                 : (k0 - nb2(K, G, r, nx, ny, l, p, axis, -1, ob)) / h;
}

// K-step on the rectangle: K1 = K + dt (-sum_k sum_l A_k[j][l] D_k K_l + sum_p
// C_jp w_p K_m K_n), A = [A1+, A1-, A2+, A2-] (r x r each); dK = K1 - K.
// Solid cells hold no gas: K1 = 0 there.
__global__ void k_kstep2d(const double* __restrict__ K, const double* __restrict__ G, int r, int nx,
                          int ny, double dx, double dy, double dt, const double* __restrict__ A,
                          const double* __restrict__ C, int P, const int* __restrict__ pm,
                          const int* __restrict__ pn, Obs2 ob, double* __restrict__ K1,
                          double* __restrict__ dK) {
  const long nc = (long)nx * ny;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= r * nc) return;
  const int j = (int)(t / nc);
  const long p = t % nc;
  if (ob.is_solid(p)) {
    K1[t] = 0.0;
    dK[t] = -K[t];
    return;
  }
  double rhs = 0.0;
  for (int l = 0; l < r; ++l)
    for (int k = 0; k < 4; ++k)
      rhs -= A[(long)k * r * r + j * r + l] * dk2(K, G, r, nx, ny, l, p, k, dx, dy, ob);
  for (int q = 0; q < P; ++q) {
    const int m = pm[q], nn = pn[q];
    rhs += C[(long)j * P + q] * ((m == nn) ? 1.0 : 2.0) * K[m * nc + p] * K[nn * nc + p];
  }
  const double k1 = K[t] + dt * rhs;
  K1[t] = k1;
  dK[t] = k1 - K[t];
}

// x-side reductions on the rectangle, one wavefront per output (i, c):
//   c < 4r        : oD[c / r][i][c % r] = w sum_p X1_i D_(c/r) K_(c%r)
//   c < 4r + P    : oT[i][c - 4r]      = w sum_p X1_i w_q K_m K_n
//   c < 4r + P + nz: oZ[i][c - 4r - P] = w sum_p X1_i Z_(c-4r-P)
__global__ __launch_bounds__(256) void k_xreduce2d(
    const double* __restrict__ X1, int r, int nx, int ny, double dx, double dy, double w,
    const double* __restrict__ K, const double* __restrict__ G, int P, const int* __restrict__ pm,
    const int* __restrict__ pn, const double* __restrict__ Z, int nz, Obs2 ob,
    double* __restrict__ oD, double* __restrict__ oT, double* __restrict__ oZ) {
  const int lane = threadIdx.x & 63;
  const int ncols = 4 * r + P + nz;
  const long t = blockIdx.x * 4L + (threadIdx.x >> 6);
  if (t >= (long)r * ncols) return;
  const int i = (int)(t / ncols), c = (int)(t % ncols);
  const long nc = (long)nx * ny;
  double s = 0.0;
  for (long p = lane; p < nc; p += 64) {
    double y;
    if (c < 4 * r) {
      y = dk2(K, G, r, nx, ny, c % r, p, c / r, dx, dy, ob);
    } else if (c < 4 * r + P) {
      const int q = c - 4 * r, m = pm[q], nn = pn[q];
      y = ((m == nn) ? 1.0 : 2.0) * K[m * nc + p] * K[nn * nc + p];
    } else {
      y = Z[(long)(c - 4 * r - P) * nc + p];
    }
    s += X1[i * nc + p] * y;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane != 0) return;
  s *= w;
  if (c < 4 * r)
    oD[(long)(c / r) * r * r + i * r + c % r] = s;
  else if (c < 4 * r + P)
    oT[(long)i * P + c - 4 * r] = s;
  else
    oZ[(long)i * nz + c - 4 * r - P] = s;
}

// S2 = S1 + dt (sum_k D_k A_k^T - T C^T), dS = S2 - S1 (r x r row-major)
__global__ void k_supdate2d(const double* __restrict__ S1, int r, const double* __restrict__ D,
                            const double* __restrict__ A, const double* __restrict__ T,
                            const double* __restrict__ C, int P, double dt,
                            double* __restrict__ S2, double* __restrict__ dS) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * r) return;
  const int i = t / r, j = t % r;
  double acc = 0.0;
  for (int k = 0; k < 4; ++k)
    for (int l = 0; l < r; ++l) acc += D[(long)k * r * r + i * r + l] * A[(long)k * r * r + j * r + l];
  for (int q = 0; q < P; ++q) acc -= T[(long)i * P + q] * C[(long)j * P + q];
  const double s2 = S1[t] + dt * acc;
  S2[t] = s2;
  dS[t] = s2 - S1[t];
}

// L-step on the velocity grid: L = S2 V,
//   L1 = L - dt sum_a (v_a^+ sum_l D_a+[i][l] V_l + v_a^- sum_l D_a-[i][l] V_l)
//        + dt sum_p T_ip Q_p,   dL = L1 - L.
template <typename TQ>
__global__ void k_lstep2d(const double* __restrict__ V, int r, int n,
                          const double* __restrict__ S2, const double* __restrict__ D,
                          const double* __restrict__ T, const TQ* __restrict__ Q, int P,
                          double dt, VGeo g, double* __restrict__ L1, double* __restrict__ dL) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)r * n) return;
  const int i = (int)(t / n), q = (int)(t % n);
  const double v1 = g.v1(q), v2 = g.v2(q);
  const double wv[4] = {v1 > 0 ? v1 : 0.0, v1 < 0 ? v1 : 0.0, v2 > 0 ? v2 : 0.0,
                        v2 < 0 ? v2 : 0.0};
  double L = 0.0, tr = 0.0;
  for (int l = 0; l < r; ++l) {
    const double vl = V[(long)l * n + q];
    L += S2[i * r + l] * vl;
    for (int k = 0; k < 4; ++k) tr += wv[k] * D[(long)k * r * r + i * r + l] * vl;
  }
  double col = 0.0;
  for (int p = 0; p < P; ++p) col += T[(long)i * P + p] * (double)Q[(long)p * n + q];
  const double l1 = L - dt * tr + dt * col;
  L1[t] = l1;
  dL[t] = l1 - L;
}

// Sums of squares of a and b (counts na, nb) into part[0 .. 2 gridDim.x):
// block sums (wave sums, waves in order) for a grid-stride split.
__global__ __launch_bounds__(256) void k_sumsq2(const double* __restrict__ a, long na,
                                                const double* __restrict__ b, long nb,
                                                double* __restrict__ part) {
  __shared__ double ws[2][4];
  double sa = 0.0, sb = 0.0;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < na; e += gridDim.x * 256L) sa += a[e] * a[e];
  for (long e = blockIdx.x * 256L + threadIdx.x; e < nb; e += gridDim.x * 256L) sb += b[e] * b[e];
  for (int off = 32; off > 0; off >>= 1) {
    sa += __shfl_down(sa, off, 64);
    sb += __shfl_down(sb, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    ws[0][threadIdx.x >> 6] = sa;
    ws[1][threadIdx.x >> 6] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x] = ((ws[0][0] + ws[0][1]) + ws[0][2]) + ws[0][3];
    part[gridDim.x + blockIdx.x] = ((ws[1][0] + ws[1][1]) + ws[1][2]) + ws[1][3];
  }
}

// err of the step from its pieces (Sec. 5.1):
//   e2 = wx |dK|^2 + |dS|^2 + dvd |dL|^2 + 2 <kx, dS> + 2 <lv, dS> + 2 <kx, lv>
// kx[i][j] = <X1_i, dK_j>, lv[i][j] = <dL_i, V_j> (r x r); one thread.
__global__ void k_err2d(const double* __restrict__ part, int nb, const double* __restrict__ dS,
                        const double* __restrict__ kx, const double* __restrict__ lv, int r,
                        double wx, double dvd, double* __restrict__ err) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double sK = 0.0, sL = 0.0;
  for (int b = 0; b < nb; ++b) {
    sK += part[b];
    sL += part[nb + b];
  }
  double sS = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
  for (int e = 0; e < r * r; ++e) {
    sS += dS[e] * dS[e];
    c1 += kx[e] * dS[e];
    c2 += lv[e] * dS[e];
    c3 += kx[e] * lv[e];
  }
  const double e2 = wx * sK + sS + dvd * sL + 2.0 * c1 + 2.0 * c2 + 2.0 * c3;
  err[0] = std::sqrt(e2 > 0.0 ? e2 : 0.0);
}

// Boundary functions of the four faces; bit k of rows: face k holds one row
// per face cell
struct FaceRows {
  const double* f[4];
  int rows;
  __device__ __forceinline__ const double* row(int k, int c, int n) const {
    return f[k] + (((rows >> k) & 1) ? (long)c * n : 0L);
  }
};

// Boundary rows F_b of the augmentation on the rectangle, one per face b
// (Sec. 3.1 with eq. boundary general): the face's boundary function on its
// incoming half (a wall's shape, scaled by k_wall_rows2d), the adjacent gas
// cell's sum_l K_l V_l on the outgoing half; zero for a solid face cell.
__global__ void k_fb2d(const double* __restrict__ K, int r, int nx, int ny,
                       const double* __restrict__ V, FaceRows fr, Obs2 ob, VGeo g,
                       double* __restrict__ Fb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
  if (q >= g.n) return;
  int cls, c;
  long p;
  face_at(b, nx, ny, ob, cls, p, c);
  const int k = cls & 3;
  const long nc = (long)nx * ny;
  const double va = k < 2 ? g.v1(q) : g.v2(q);
  const bool inc = (k % 2 == 0) ? va > 0 : va < 0;
  double val = 0.0;
  if (cls < 4 && ob.is_solid(p)) {
    val = 0.0;
  } else if (inc) {
    val = cls < 4 ? fr.row(k, c, g.n)[q] : ob.f[q];
  } else {
    for (int l = 0; l < r; ++l) val += K[l * nc + p] * V[(long)l * g.n + q];
  }
  Fb[(long)b * g.n + q] = val;
}

// Diffusive walls: scale the incoming half of each wall row of F_b by rho_w
// from the row's own outgoing half.  One block per face cell.
__global__ __launch_bounds__(1024) void k_wall_rows2d(double* __restrict__ Fb, FaceRows fr,
                                                      int walls, int nx, int ny, Obs2 ob, VGeo g) {
  int cls, c;
  long p;
  face_at(blockIdx.x, nx, ny, ob, cls, p, c);
  const int k = cls & 3;
  if (cls < 4 && (!((walls >> k) & 1) || ob.is_solid(p))) return;
  __shared__ double red[1024 / 64 + 1];
  double* row = Fb + (long)blockIdx.x * g.n;
  const double* M = cls < 4 ? fr.row(k, c, g.n) : ob.f;
  const int stride = k < 2 ? (g.d == 3 ? g.N * g.N : g.N) : (g.d == 3 ? g.N : 1);
  const double rho =
      wall::density_face<1024>((k % 2 == 0) ? -1.0 : 1.0, row, M, g.n, g.L, g.dv, stride, g.N, red);
  for (int q = threadIdx.x; q < g.n; q += 1024) {
    const double va = k < 2 ? g.v1(q) : g.v2(q);
    if ((k % 2 == 0) ? va > 0 : va < 0) row[q] = rho * M[q];
  }
}

// F_b[b] -= sum_l C[b][l] V_l (the rows projected onto V^perp, C = <F_b, V>)
__global__ void k_proj_rows(double* __restrict__ Fb, int nb, long n, const double* __restrict__ C,
                            int r, const double* __restrict__ V) {
  const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (q >= n || b >= nb) return;
  double s = 0.0;
  for (int l = 0; l < r; ++l) s += C[b * r + l] * V[(long)l * n + q];
  Fb[(long)b * n + q] -= s;
}

// S_aug = S^ Rv^T with S^ = [[S, 0], [0, 0]] (r x r block S, leading dim
// lds) and Rv (ra x ra row-major): the state after appending basis rows whose
// QR is V^T = Vq^T Rv
__global__ void k_saug(const double* __restrict__ S, int lds, int r, const double* __restrict__ Rv,
                       int ra, double* __restrict__ Sa) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ra * ra) return;
  const int i = t / ra, j = t % ra;
  double v = 0.0;
  if (i < r)
    for (int l = 0; l < r; ++l) v += S[i * lds + l] * Rv[j * ra + l];
  Sa[t] = v;
}

// S (leading dimension lds) = R^T for an r x r row-major R
__global__ void k_store_RT(const double* __restrict__ R, int r, double* __restrict__ S, int lds) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * r) return;
  const int i = t / r, j = t % r;
  S[i * lds + j] = R[j * r + i];
}

}  // namespace dk

// ------------------------------------------------------------------ host --
namespace {

inline unsigned blocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

struct StepWork {
  blr_ctx ctx;
  hipStream_t s;
  dk::VGeo g;
  int nx, n;
  double dx, dvd;
  double* get(const char* name, size_t count) {
    return (double*)ctx->buf(std::string("dlr.") + name, count * sizeof(double));
  }
};

// Products evaluated by one launch pair (see k_gram_batch).
struct GramJob {
  dk::GramBatch gb{};
  void add(const double* A, int ra, const void* B, int rb, bool bfloat, int mode, double scale,
           double* out) {
    require(gb.nseg < dk::MAXSEG, "gram batch: too many products");
    require(ra >= 1 && ra <= 64 && rb >= 1, "gram batch: bad shape");
    dk::GramSeg& s = gb.seg[gb.nseg++];
    s.A = A;
    s.B = B;
    s.out = out;
    s.scale = scale;
    s.ra = ra;
    s.rb = rb;
    s.mode = mode;
    s.bfloat = bfloat ? 1 : 0;
    s.ntb = (rb + dk::GT - 1) / dk::GT;
    s.tile0 = gb.ntiles;
    gb.ntiles += s.ntb * ((ra + dk::GT - 1) / dk::GT);
    s.out0 = gb.nout;
    gb.nout += ra * rb;
  }
  void run(StepWork& w) {
    if (gb.nseg == 0) return;
    // chunks of 128 points: each wave takes 32 points, one round of eight loads
    const int nchunk = (int)std::max<long>(1, std::min<long>(2048, (long)w.n / 128));
    long off = 0;
    double bytes = 0.0;
    for (int k = 0; k < gb.nseg; ++k) {
      gb.seg[k].part0 = off;
      off += (long)nchunk * gb.seg[k].ra * gb.seg[k].rb;
      bytes += (double)w.n * (gb.seg[k].ra * 8.0 + gb.seg[k].rb * (gb.seg[k].bfloat ? 4.0 : 8.0));
    }
    double* part = w.get("gram.part", (size_t)off);
    timed_begin("dlr.gram", bytes, w.s);
    hipLaunchKernelGGL(dk::k_gram_batch, dim3(nchunk, gb.ntiles), dim3(256), 0, w.s, gb, (long)w.n,
                       nchunk, w.g, part);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_gram_batch_finish, dim3(blocks(gb.nout, 4)), dim3(256), 0, w.s, gb,
                       nchunk, part);
    BLR_CHECK_LAUNCH();
    timed_end(w.s);
  }
};

void validate_problem(const blr_problem* pb, const blr_state* st) {
  require(pb && st, "null problem or state");
  require(pb->nx >= 2 && pb->nx <= (1 << 20), "problem.nx must be in [2, 2^20]");
  require(pb->x_hi > pb->x_lo, "problem.x_hi must exceed x_lo");
  require(pb->f_left && pb->f_right, "null inflow boundary arrays");
  require((pb->wall_left == 0 || pb->wall_left == 1) && (pb->wall_right == 0 || pb->wall_right == 1),
          "problem.wall_left / wall_right must be 0 (inflow) or 1 (diffusive wall)");
  require(pb->ny <= 1, "one-dimensional space expected (problem.ny <= 1)", BLR_ERR_UNSUPPORTED);
  require(pb->face_rows == 0, "problem.face_rows: one-dimensional space takes one row per face");
  validate_vgrid(pb->v);
  require(st->X && st->S && st->V, "null state arrays");
  require(st->r_cap >= 1 && st->r_cap <= 64, "state.r_cap must be in [1, 64]");
  require(st->r >= 1 && st->r <= st->r_cap, "state.r must be in [1, r_cap]");
}

}  // namespace

namespace {

// How the boundary basis is added in one attempt of a step: rb functions,
// orthogonalised against V by two projection passes or by Householder QR.
struct Attempt {
  int rb;
  bool householder;     // boundary functions by Householder QR
  bool householder_qr;  // K- and L-step QRs by Householder QR (else Cholesky QR when r <= 16)
};

// Device-side results of one attempt, the host read-back and the buffers
// the commit reads.
struct Outcome {
  int r = 0;                 // rank after the add
  double res[4] = {0, 0, 0, 0};
  bool orth_failed = false;
  bool qr_failed = false;
  double sb[2] = {0, 0};     // singular values of F_b (when the add ran)
  std::vector<double> sg, g; // singular values of S^{n+1}, err_ada terms (drop only)
  double *X1 = nullptr, *V1 = nullptr, *Snew = nullptr, *U = nullptr, *Wm = nullptr,
         *sgd = nullptr;
  double* hb = nullptr;  // pinned read-back record
  int nrb = 0;           // singular values in it
  bool timed_collision = false;
};

// The device work of one attempt, up to the copy of the read-back record
// into pinned host memory (o.hb); no wait.  Timing events only when
// rec_events (not while a graph is recorded).
void step_enqueue(blr_ctx ctx, const blr_problem* pb, const blr_state* st, const blr_step_params* sp,
                  const HostTables& h, bool add, Attempt at, Outcome& o, bool rec_events) {
  StepWork w{ctx, ctx->stream, {h.L, h.dv, h.N, h.d, h.n}, pb->nx, h.n,
             (pb->x_hi - pb->x_lo) / pb->nx, std::pow(h.dv, h.d)};
  hipStream_t s = w.s;
  const int nx = w.nx, n = w.n;
  const double dx = w.dx, dvd = w.dvd, dt = sp->dt;
  if (rec_events) BLR_HIP(hipEventRecord(ctx->ev[0], s));

  // working copies (rank up to r_cap); the caller's state is written only at commit
  const int rc = st->r_cap;
  // X and V are read in place: the step reads their first r rows only and
  // uses rows r.. (scratch of the state, below r_cap) for the added
  // functions; the Householder variant of the add rewrites every row of V and
  // works on a copy
  double* Xw = st->X;
  double* Vw = st->V;
  double* Sw = w.get("Sw", (size_t)rc * rc);
  int r = st->r;
  if (add && at.rb > 0 && at.householder) {
    Vw = w.get("Vw", (size_t)rc * n);
    BLR_HIP(hipMemcpyAsync(Vw, st->V, (size_t)r * n * 8, hipMemcpyDeviceToDevice, s));
  }
  double* ginL = w.get("ginL", 64);
  double* ginR = w.get("ginR", 64);
  double* MoL = w.get("MoL", 64 * 64);
  double* MoR = w.get("MoR", 64 * 64);
  double* gh = w.get("ghost", 128);
  double* K = w.get("K", (size_t)rc * nx);
  int* flag = (int*)ctx->buf("dlr.flag", 256);  // [0] projection failed, [1] Cholesky QR failed
  // S -> Sw, flags cleared, and the boundary rows F_b of the augmentation
  double* Fb = add ? w.get("Fb", (size_t)2 * n) : nullptr;
  hipLaunchKernelGGL(dk::k_add_begin, dim3(add ? blocks(n, 256) : 1), dim3(256), 0, s, Xw, r, nx,
                     st->S, rc, Sw, r, flag, Vw, pb->f_left, pb->f_right, w.g, Fb);
  BLR_CHECK_LAUNCH();
  const bool walls = pb->wall_left || pb->wall_right;
  if (add && walls) {
    hipLaunchKernelGGL(dk::k_wall_rows, dim3(2), dim3(1024), 0, s, Fb, pb->f_left, pb->f_right,
                       pb->wall_left, pb->wall_right, w.g);
    BLR_CHECK_LAUNCH();
  }
  // S^ still to be copied into Sw (projection variant), done with the FP32 cast
  const double* pend_S = nullptr;
  int pend_r = 0;
  const double* sbd = nullptr;
  // QR of sqrt(w) M with Q scaled back by 1/sqrt(w)
  auto qr = [&](const double* M, long ld, long rows, int rr, double* Qo, double* Ro, const char* tag,
                double w) {
    if (rr <= 16 && !at.householder_qr)
      cholqr(ctx, M, ld, rows, rr, Qo, ld, Ro, tag, std::sqrt(w), 1.0 / std::sqrt(w), flag + 1);
    else
      tsqr(ctx, M, ld, rows, rr, Qo, ld, Ro, tag, std::sqrt(w), 1.0 / std::sqrt(w));
  };

  // ---------------------------------------------------------- add basis
  // F_b = [boundary rows] = U_b Sig_b (right singular vectors); the rb
  // leading right singular vectors are the rows of Sig_b^{-1} U_b^T F_b, and
  // their positive scale does not matter for the orthogonalisation, so the
  // new rows are U_b[:, :rb]^T F_b.  X gains zero rows: with S^ = [[S, 0],
  // [0, 0]] the product X^ S^ (all the step reads of X^n) is unchanged.
  if (add) {
    double* RF = w.get("RF", 4);
    tsqr(ctx, Fb, n, n, 2, nullptr, 0, RF, "qr.fb");
    double* Ub = w.get("Ub", 4);
    double* sb = w.get("sb", 2);
    double* Wb = w.get("Wb", 4);
    // F_b = R_F^T Q_F^T,  R_F^T = U_b Sig_b W_b^T (R_F read transposed)
    svd_small(ctx, RF, 2, Ub, sb, Wb, true);
    sbd = sb;
    const int rb = at.rb;
    if (rb > 0) {
      double* Vb = Vw + (size_t)r * n;
      const int rk = r + rb;
      double* Shat = w.get("Shat", (size_t)rk * rk);
      // Vb = U_b[:, :rb]^T F_b, zero rows of X, S^ = [[S, 0], [0, 0]]
      hipLaunchKernelGGL(dk::k_add_rows, dim3(blocks(n, 256), rb), dim3(256), 0, s, Fb, (long)n, Ub,
                         rb, Vb, Xw + (size_t)r * nx, (long)rb * nx, Sw, r, Shat);
      BLR_CHECK_LAUNCH();
      if (!at.householder) {
        // [V; Vb] with V orthonormal: two projection passes keep V and
        // orthonormalise Vb against it; S^ is unchanged (the triangular
        // factor is [[I, 0], [C, L]] and S^ has zero rows and columns there)
        double* G = w.get("orthG", (size_t)2 * 66);
        for (int pass = 0; pass < 2; ++pass) {
          GramJob gj;
          gj.add(Vb, rb, Vw, rk, false, dk::W_ONE, dvd, G);
          gj.run(w);
          hipLaunchKernelGGL(dk::k_orth_pass, dim3(blocks(n, 256)), dim3(256), 0, s, Vw, r, rb, (long)n,
                             G, pass, flag);
          BLR_CHECK_LAUNCH();
        }
        pend_S = Shat;  // S^ -> Sw before the collisions
        pend_r = rk;
      } else {
        // Householder QR of [V; Vb]^T (weighted): V^ = Sv^T V_q, S <- S^ Sv^T
        double* Sv = w.get("Sv", (size_t)rk * rk);
        tsqr(ctx, Vw, n, n, rk, Vw, n, Sv, "qr.v", std::sqrt(dvd), 1.0 / std::sqrt(dvd));
        hipLaunchKernelGGL(dk::k_mul_bt, dim3(1), dim3(1024), 0, s, Shat, Sv, rk, Sw);
        BLR_CHECK_LAUNCH();
      }
      r = rk;
    }
  }
  o.r = r;

  // ------------------------------------------------------- collisions
  const int P = r * (r + 1) / 2;
  std::vector<int> pidx(2 * P);
  std::vector<int32_t> pairs(2 * P);
  {
    int p = 0;
    for (int m = 0; m < r; ++m)
      for (int nn = m; nn < r; ++nn, ++p) {
        pidx[p] = m;
        pidx[P + p] = nn;
        pairs[2 * p] = m;
        pairs[2 * p + 1] = nn;
      }
  }
  int* dpidx = (int*)ctx->upload("dlr.pidx", pidx.data(), pidx.size() * sizeof(int));
  const bool fp64c = (sp->flags & BLR_STEP_FP64_COLLISION) != 0;
  // FP64 defect correction: a refresh step (FP64 pairs used, the defect kept)
  // or a corrected step (FP32 pairs plus the kept defect); either steps with
  // FP64 pair fields
  const bool refresh = !fp64c && (sp->flags & BLR_STEP_DEFECT_REFRESH) != 0;
  const bool corrected = !fp64c && !refresh && (sp->flags & BLR_STEP_FP64_DEFECT) != 0;
  const bool q64 = fp64c || refresh || corrected;
  void* Qs;
  if (rec_events) BLR_HIP(hipEventRecord(ctx->ev[1], s));
  if (fp64c) {
    if (pend_S) {
      hipLaunchKernelGGL(dk::k_copy_S, dim3(blocks(pend_r * pend_r, 256)), dim3(256), 0, s, pend_S,
                         pend_r, pend_r, Sw, pend_r);
      BLR_CHECK_LAUNCH();
    }
    Qs = w.get("Q64", (size_t)P * n);
    collision_pairs(ctx, pb->v, BLR_FP64, Vw, r, pairs.data(), P, Qs);
  } else {
    float* V32 = (float*)ctx->buf("dlr.V32", (size_t)r * n * sizeof(float));
    hipLaunchKernelGGL(dk::k_to_f32_copy_S, dim3(blocks((long)r * n, 256)), dim3(256), 0, s, Vw,
                       (long)r * n, V32, pend_S, pend_r, Sw, pend_r);
    BLR_CHECK_LAUNCH();
    Qs = ctx->buf("dlr.Q32", (size_t)P * n * sizeof(float));
    if (ctx->collide_hook && ctx->capturing) {
      // recording: the graph ends here, the collisions run between it and the
      // graph of the rest of the step (recorded from here on)
      BLR_HIP(hipStreamEndCapture(ctx->stream, &ctx->split_g1));
      ctx->split_vg = pb->v;
      ctx->split_V = V32;
      ctx->split_r = r;
      ctx->split_pairs = pairs;
      ctx->split_Q = (float*)Qs;
      BLR_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    } else if (ctx->collide_hook)
      ctx->collide_hook->collide(ctx, pb->v, V32, r, pairs, (float*)Qs);
    else
      collision_pairs(ctx, pb->v, BLR_FP32, V32, r, pairs.data(), P, Qs);
    if (refresh) {
      // the same pairs in FP64 drive this step; their difference from the
      // FP32 ones is kept with the basis they were taken on
      const int rc2 = rc * (rc + 1) / 2;
      double* Q64 = w.get("Q64", (size_t)P * n);
      collision_pairs(ctx, pb->v, BLR_FP64, Vw, r, pairs.data(), P, Q64);
      double* Dk = (double*)ctx->buf("dlr.defect.D", (size_t)rc2 * n * 8);
      double* Vk = (double*)ctx->buf("dlr.defect.V", (size_t)rc * n * 8);
      hipLaunchKernelGGL(dk::k_defect_store, dim3(blocks((long)P * n, 256)), dim3(256), 0, s, Q64,
                         (const float*)Qs, (long)P * n, Dk);
      BLR_CHECK_LAUNCH();
      BLR_HIP(hipMemcpyAsync(Vk, Vw, (size_t)r * n * 8, hipMemcpyDeviceToDevice, s));
      Qs = Q64;
    } else if (corrected) {
      const int rr = ctx->defect_r;
      require(rr >= 1 && rr <= dk::DEFECT_MAX && r <= dk::DEFECT_MAX, "defect correction: bad rank");
      const int rc2 = rc * (rc + 1) / 2;
      double* Dk = (double*)ctx->buf("dlr.defect.D", (size_t)rc2 * n * 8);
      double* Vk = (double*)ctx->buf("dlr.defect.V", (size_t)rc * n * 8);
      double* Rk = w.get("defect.R", (size_t)dk::DEFECT_MAX * dk::DEFECT_MAX);
      double* Tk = w.get("defect.T", (size_t)rc * dk::DEFECT_MAX * n);
      double* Qc = w.get("Q64", (size_t)P * n);
      GramJob gj;
      gj.add(Vw, r, Vk, rr, false, dk::W_ONE, dvd, Rk);  // R[a][m] = <W_a, V_m>
      gj.run(w);
      const dim3 g1(blocks(n, 64), rr), g2(blocks(n, 64), r);
      if (rr <= 16 && r <= 16) {
        hipLaunchKernelGGL(dk::k_defect_carry1<16>, g1, dim3(64), 0, s, Dk, rr, Rk, r, (long)n, Tk);
        BLR_CHECK_LAUNCH();
        hipLaunchKernelGGL(dk::k_defect_carry2<16>, g2, dim3(64), 0, s, Tk, rr, Rk, r, (long)n,
                           (const float*)Qs, Qc);
      } else {
        hipLaunchKernelGGL(dk::k_defect_carry1<32>, g1, dim3(64), 0, s, Dk, rr, Rk, r, (long)n, Tk);
        BLR_CHECK_LAUNCH();
        hipLaunchKernelGGL(dk::k_defect_carry2<32>, g2, dim3(64), 0, s, Tk, rr, Rk, r, (long)n,
                           (const float*)Qs, Qc);
      }
      BLR_CHECK_LAUNCH();
      Qs = Qc;
    }
  }
  if (rec_events) BLR_HIP(hipEventRecord(ctx->ev[2], s));
  o.timed_collision = rec_events;

  // velocity-side contractions
  double* Ap = w.get("Ap", (size_t)r * r);
  double* Am = w.get("Am", (size_t)r * r);
  double* Cj = w.get("C", (size_t)r * P);
  {
    GramJob gj;
    gj.add(Vw, r, Vw, r, false, dk::W_VPLUS, dvd, Ap);
    gj.add(Vw, r, Vw, r, false, dk::W_VMINUS, dvd, Am);
    gj.add(Vw, r, Vw, r, false, dk::W_OUT_LEFT, dvd, MoL);
    gj.add(Vw, r, Vw, r, false, dk::W_OUT_RIGHT, dvd, MoR);
    gj.add(Vw, r, Qs, P, !q64, dk::W_ONE, dvd, Cj);
    gj.add(Vw, r, pb->f_left, 1, false, dk::W_IN_LEFT, dvd, ginL);
    gj.add(Vw, r, pb->f_right, 1, false, dk::W_IN_RIGHT, dvd, ginR);
    gj.run(w);
  }
  if (walls) {
    hipLaunchKernelGGL(dk::k_wall_fold, dim3(2), dim3(1024), 0, s, Vw, r, pb->f_left, pb->f_right,
                       pb->wall_left, pb->wall_right, w.g, ginL, ginR, MoL, MoR);
    BLR_CHECK_LAUNCH();
  }

  // ---------------------------------------------------------- K-step
  double* K1 = w.get("K1", (size_t)r * nx);
  double* dK = w.get("dK", (size_t)r * nx);
  double* X1 = w.get("X1", (size_t)r * nx);
  double* S1 = w.get("S1", (size_t)r * r);
  const bool small = r <= 16;  // fused x-side kernels
  auto bucket16 = [&](auto&& f) {
    if (r <= 4) f(std::integral_constant<int, 4>{});
    else if (r <= 8) f(std::integral_constant<int, 8>{});
    else if (r <= 12) f(std::integral_constant<int, 12>{});
    else f(std::integral_constant<int, 16>{});
  };
  if (small) {
    bucket16([&](auto rm) {
      constexpr int RM = decltype(rm)::value;
      const int JB = 2;  // outputs per block
      hipLaunchKernelGGL(dk::k_kstep_fused<RM>, dim3(blocks(nx, dk::KSB), (r + JB - 1) / JB),
                         dim3(dk::KSB), 0, s, Xw, Sw, r, nx, dx, dt, JB, ginL, ginR, MoL, MoR, Ap, Am,
                         Cj, P, K1, dK);
    });
    BLR_CHECK_LAUNCH();
  } else {
    hipLaunchKernelGGL(dk::k_xmul, dim3(blocks((long)r * nx, 256)), dim3(256), 0, s, Xw, r, nx, Sw, r,
                       K);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_ghosts, dim3(1), dim3(64), 0, s, K, r, nx, ginL, ginR, MoL, MoR, gh);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_kstep, dim3(blocks((long)r * nx, 256)), dim3(256), 0, s, K, gh, r, nx, dx,
                       dt, Ap, Am, Cj, P, dpidx, dpidx + P, K1, dK);
    BLR_CHECK_LAUNCH();
  }
  qr(K1, nx, nx, r, X1, S1, "qr.k", dx);

  // ---------------------------------------------------------- S-step
  const int ncols = 2 * r + P;
  double* S2 = w.get("S2", (size_t)r * r);
  double* dS = w.get("dS", (size_t)r * r);
  double* Dp = w.get("Dp", (size_t)r * r);
  double* Dm = w.get("Dm", (size_t)r * r);
  double* T = w.get("T", (size_t)r * P);
  double* kx = w.get("kx", (size_t)r * r);
  double* Aad = w.get("Aad", (size_t)r * r);
  const bool drop_on = (sp->flags & BLR_STEP_DROP) != 0;
  // x-side products of X1 with D+-K, w K_m K_n for K = X1 Sx (and, in the
  // L-step pass, with dK and X^n)
  auto xside = [&](const double* Sx, bool extra) {
    if (small) {
      const int nc = ncols + (extra ? r : 0) + (extra && drop_on ? r : 0);
      bucket16([&](auto rm) {
        constexpr int RM = decltype(rm)::value;
        hipLaunchKernelGGL(dk::k_xside<RM>, dim3(blocks(nc, 16)), dim3(256), 0, s, X1, r, nx, dx, Sx,
                           ginL, ginR, MoL, MoR, P, dpidx, dpidx + P, extra ? dK : nullptr,
                           (extra && drop_on) ? Xw : nullptr, Dp, Dm, T, kx, Aad);
      });
      BLR_CHECK_LAUNCH();
      return;
    }
    hipLaunchKernelGGL(dk::k_xmul, dim3(blocks((long)r * nx, 256)), dim3(256), 0, s, X1, r, nx, Sx, r,
                       K);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_ghosts, dim3(1), dim3(64), 0, s, K, r, nx, ginL, ginR, MoL, MoR, gh);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_xreduce, dim3(blocks((long)r * ncols, 4)), dim3(256), 0, s, X1, r, nx,
                       dx, K, gh, P, dpidx, dpidx + P, nullptr, 0, 0, nullptr, ncols, Dp, Dm, T);
    BLR_CHECK_LAUNCH();
    if (extra) {
      hipLaunchKernelGGL(dk::k_xreduce, dim3(blocks((long)r * r, 4)), dim3(256), 0, s, X1, r, nx, dx,
                         nullptr, nullptr, 0, nullptr, nullptr, dK, r, 1, kx, r, nullptr, nullptr,
                         nullptr);
      BLR_CHECK_LAUNCH();
      if (drop_on) {
        hipLaunchKernelGGL(dk::k_xreduce, dim3(blocks((long)r * r, 4)), dim3(256), 0, s, Xw, r, nx,
                           dx, nullptr, nullptr, 0, nullptr, nullptr, X1, r, 1, Aad, r, nullptr,
                           nullptr, nullptr);
        BLR_CHECK_LAUNCH();
      }
    }
  };
  xside(S1, false);
  if (small)
    hipLaunchKernelGGL(dk::k_supdate16, dim3(1), dim3(256), 0, s, S1, Dp, Dm, T, Ap, Am, Cj, r, P, dt,
                       S2, dS);
  else
    hipLaunchKernelGGL(dk::k_supdate, dim3(1), dim3(1024), 0, s, S1, Dp, Dm, T, Ap, Am, Cj, r, P, dt,
                       S2, dS);
  BLR_CHECK_LAUNCH();

  // ---------------------------------------------------------- L-step
  xside(S2, true);
  double* L1 = w.get("L1", (size_t)r * n);
  double* dL = w.get("dL", (size_t)r * n);
  if (r <= 16) {
    timed_begin("dlr.lstep", (double)n * (r + P + 2 * r) * 8.0, s);
    const dim3 grid(blocks(n, 64));
    if (q64)
      hipLaunchKernelGGL(dk::k_lstep_mfma<double>, grid, dim3(256), 0, s, Vw, r, n, S2, Dp, Dm, T,
                         (const double*)Qs, P, dt, w.g, L1, dL);
    else
      hipLaunchKernelGGL(dk::k_lstep_mfma<float>, grid, dim3(256), 0, s, Vw, r, n, S2, Dp, Dm, T,
                         (const float*)Qs, P, dt, w.g, L1, dL);
    BLR_CHECK_LAUNCH();
    timed_end(s);
  } else {
    const dim3 grid(blocks(n, 256), (r + 7) / 8);
    timed_begin("dlr.lstep", (double)n * (r + P + 2 * r) * 8.0, s);
    if (q64)
      hipLaunchKernelGGL(dk::k_lstep<double>, grid, dim3(256), 0, s, Vw, r, n, S2, Dp, Dm, T,
                         (const double*)Qs, P, dt, w.g, L1, dL);
    else
      hipLaunchKernelGGL(dk::k_lstep<float>, grid, dim3(256), 0, s, Vw, r, n, S2, Dp, Dm, T,
                         (const float*)Qs, P, dt, w.g, L1, dL);
    BLR_CHECK_LAUNCH();
    timed_end(s);
  }
  double* V1 = w.get("V1", (size_t)r * n);
  double* Rl = w.get("Rl", (size_t)r * r);
  double* Snew = w.get("Snew", (size_t)r * r);
  qr(L1, n, n, r, V1, Rl, "qr.l", dvd);
  hipLaunchKernelGGL(dk::k_transpose, dim3(1), dim3(1024), 0, s, Rl, r, Snew);
  BLR_CHECK_LAUNCH();

  // --------------------------------------------------------- residual
  double* lv = w.get("lv", (size_t)r * r);
  double* GdL = w.get("GdL", (size_t)r * r);
  double* res = w.get("res", 8);
  // Gram products of the residual and of err_ada (B = <V^n_l, V1_j>)
  double* Bad = w.get("Bad", (size_t)r * r);
  {
    GramJob gj;
    gj.add(dL, r, Vw, r, false, dk::W_ONE, dvd, lv);
    gj.add(dL, r, dL, r, false, dk::W_ONE, dvd, GdL);
    if (sp->flags & BLR_STEP_DROP) gj.add(Vw, r, V1, r, false, dk::W_ONE, dvd, Bad);
    gj.run(w);
  }
  if (small)
    hipLaunchKernelGGL(dk::k_err16, dim3(1), dim3(256), 0, s, dK, (long)r * nx, dx, dS, r, GdL, kx, lv,
                       res);
  else
    hipLaunchKernelGGL(dk::k_err, dim3(1), dim3(256), 0, s, dK, (long)r * nx, dx, dS, r, GdL, kx, lv,
                       res);
  BLR_CHECK_LAUNCH();

  // ---------------------------------------------- drop ingredients (device)
  double* sg = nullptr;
  double* gterm = nullptr;
  o.X1 = X1;
  o.V1 = V1;
  o.Snew = Snew;
  if (sp->flags & BLR_STEP_DROP) {
    double* U = w.get("U", (size_t)r * r);
    sg = w.get("sig", (size_t)r);
    double* Wm = w.get("W", (size_t)r * r);
    svd_small(ctx, Snew, r, U, sg, Wm);
    // err_ada uses A = <X^n_k, X1_i> (x-side pass of the L-step) and B = <V^n_l, V1_j>
    gterm = w.get("gterm", (size_t)r);
    if (small)
      hipLaunchKernelGGL(dk::k_fnD16, dim3(1), dim3(256), 0, s, Sw, Aad, U, sg, Wm, Bad, r, gterm);
    else
      hipLaunchKernelGGL(dk::k_fnD_terms, dim3(1), dim3(256), 0, s, Sw, Aad, U, sg, Wm, Bad, r, gterm);
    BLR_CHECK_LAUNCH();
    o.U = U;
    o.Wm = Wm;
    o.sgd = sg;
  }

  // ------------------------------------------------------ read-back
  if (rec_events) BLR_HIP(hipEventRecord(ctx->ev[3], s));
  const bool drop = (sp->flags & BLR_STEP_DROP) != 0;
  const int nrb = drop ? r : 0;
  double* pk = w.get("pack", (size_t)8 + 2 * 64);
  hipLaunchKernelGGL(dk::k_pack, dim3(1), dim3(64), 0, s, res, flag, sbd, sg, gterm, nrb, pk);
  BLR_CHECK_LAUNCH();
  const size_t nbytes = (8 + 2 * (size_t)nrb) * sizeof(double);
  double* hb = (double*)ctx->host_readback(nbytes);
  BLR_HIP(hipMemcpyAsync(hb, pk, nbytes, hipMemcpyDeviceToHost, s));
  o.hb = hb;
  o.nrb = nrb;
}

// Host side of the read-back record (after the wait).
void step_parse(Outcome& o) {
  const double* hb = o.hb;
  const int nrb = o.nrb;
  for (int k = 0; k < 4; ++k) o.res[k] = hb[k];
  o.orth_failed = hb[4] != 0.0;
  o.qr_failed = hb[7] != 0.0;
  o.sb[0] = hb[5];
  o.sb[1] = hb[6];
  o.sg.assign(hb + 8, hb + 8 + nrb);
  o.g.assign(hb + 8 + nrb, hb + 8 + 2 * nrb);
}

// Key of a step attempt: every input that shapes the recorded work.
std::string step_key(const blr_problem* pb, const blr_state* st, const blr_step_params* sp, bool add,
                     const Attempt& at, int defect_r) {
  struct {
    int32_t nx;
    double x_lo, x_hi;
    const void *fl, *fr;
    blr_vgrid v;
    int32_t wl, wr;
    int32_t r, r_cap;
    const void *X, *S, *V;
    blr_step_params p;
    int32_t add, rb, hh, hq, dr;
  } k;
  std::memset(&k, 0, sizeof(k));
  k.nx = pb->nx;
  k.x_lo = pb->x_lo;
  k.x_hi = pb->x_hi;
  k.fl = pb->f_left;
  k.fr = pb->f_right;
  k.v = pb->v;
  k.wl = pb->wall_left;
  k.wr = pb->wall_right;
  k.r = st->r;
  k.r_cap = st->r_cap;
  k.X = st->X;
  k.S = st->S;
  k.V = st->V;
  k.p = *sp;
  k.add = add;
  k.rb = at.rb;
  k.hh = at.householder;
  k.hq = at.householder_qr;
  k.dr = defect_r;
  return std::string((const char*)&k, sizeof(k));
}

// One attempt of the step up to the rank decision, one wait.  Unless the
// step is eager or kernels are timed, the device work is recorded as a
// graph the second time a configuration is seen and replayed from then on.
void step_attempt(blr_ctx ctx, const blr_problem* pb, const blr_state* st, const blr_step_params* sp,
                  const HostTables& h, bool add, Attempt at, Outcome& o) {
  hipStream_t s = ctx->stream;
  // (a refresh step runs its FP32 pairs through the collide hook directly,
  // so with a hook it is not recorded)
  const bool graphs = !(sp->flags & BLR_STEP_EAGER) && !ctx->timer.on &&
                      !((sp->flags & BLR_STEP_DEFECT_REFRESH) && ctx->collide_hook);
  auto eager = [&]() {
    step_enqueue(ctx, pb, st, sp, h, add, at, o, true);
    BLR_HIP(hipStreamSynchronize(s));
    step_parse(o);
  };
  if (!graphs) {
    eager();
    return;
  }
  // (with collide_hook the recording is split around the collisions)
  // a corrected step's launches depend on the rank of the kept defect
  const bool corrected = (sp->flags & BLR_STEP_FP64_DEFECT) && !(sp->flags & BLR_STEP_DEFECT_REFRESH);
  const std::string key =
      step_key(pb, st, sp, add, at, corrected ? ctx->defect_r : 0) + (ctx->collide_hook ? "h" : "");
  auto& gs = ctx->graphs;
  size_t gi = gs.size();
  for (size_t k = 0; k < gs.size(); ++k)
    if (gs[k].key == key) gi = k;
  if (gi == gs.size()) {
    if (gs.size() >= 8) {  // forget the oldest
      if (gs.front().exec) (void)hipGraphExecDestroy(gs.front().exec);
      if (gs.front().exec2) (void)hipGraphExecDestroy(gs.front().exec2);
      gs.erase(gs.begin());
    }
    gs.push_back(blr_ctx_t::StepGraph{});
    gi = gs.size() - 1;
    gs[gi].key = key;
  }
  auto& g = gs[gi];
  if (g.gen != ctx->buf_gen) {  // addresses moved: start over
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.exec2) (void)hipGraphExecDestroy(g.exec2);
    g.exec = nullptr;
    g.exec2 = nullptr;
    g.seen = 0;
    g.gen = ctx->buf_gen;
  }
  if (!g.exec && g.seen == 0) {
    eager();
    g.seen = 1;
    g.gen = ctx->buf_gen;
    return;
  }
  if (!g.exec) {
    // record on the capture stream, then replay on the caller's stream
    if (!ctx->cap_stream) BLR_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    const uint64_t gen0 = ctx->buf_gen;
    ctx->stream = ctx->cap_stream;
    ctx->capturing = true;
    ctx->capture_broken = false;
    ctx->split_g1 = nullptr;
    auto drop_split = [&] {
      if (ctx->split_g1) (void)hipGraphDestroy(ctx->split_g1);
      ctx->split_g1 = nullptr;
    };
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        step_enqueue(ctx, pb, st, sp, h, add, at, o, false);
      } catch (const Error&) {
        drop_split();
        // The recording failed: a device-wide operation of another host
        // thread (a device synchronisation, an allocation or free) can
        // invalidate it or make a recorded launch report an error.  The step
        // then runs directly, the same kernels in the same order, where an
        // error of the step's own is reported as usual.
        (void)hipStreamEndCapture(ctx->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        ctx->stream = s;
        ctx->capturing = false;
        (void)hipGetLastError();
        eager();
        g.gen = ctx->buf_gen;
        return;
      } catch (...) {
        drop_split();
        (void)hipStreamEndCapture(ctx->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        ctx->stream = s;
        ctx->capturing = false;
        throw;
      }
      e = hipStreamEndCapture(ctx->cap_stream, &graph);
    }
    ctx->stream = s;
    ctx->capturing = false;
    hipGraphExec_t exec = nullptr, exec2 = nullptr;
    const bool split = ctx->split_g1 != nullptr;
    if (e == hipSuccess && graph && !ctx->capture_broken && ctx->buf_gen == gen0) {
      if (split) {
        e = hipGraphInstantiate(&exec, ctx->split_g1, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphInstantiate(&exec2, graph, nullptr, nullptr, 0);
      } else {
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      }
    }
    if (graph) (void)hipGraphDestroy(graph);
    drop_split();
    if (e != hipSuccess || !exec || (split && !exec2) || (!split && ctx->collide_hook)) {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (exec2) (void)hipGraphExecDestroy(exec2);
      (void)hipGetLastError();
      eager();  // not recordable this time: run it directly
      g.gen = ctx->buf_gen;
      return;
    }
    g.exec = exec;
    g.exec2 = exec2;
    if (split) {
      g.cvg = ctx->split_vg;
      g.cV = ctx->split_V;
      g.cr = ctx->split_r;
      g.cpairs = ctx->split_pairs;
      g.cQ = ctx->split_Q;
    }
    g.gen = ctx->buf_gen;
    g.r = o.r;
    g.nrb = o.nrb;
    g.X1 = o.X1;
    g.V1 = o.V1;
    g.Snew = o.Snew;
    g.U = o.U;
    g.Wm = o.Wm;
    g.sgd = o.sgd;
    g.hb = o.hb;
  } else {
    o.r = g.r;
    o.nrb = g.nrb;
    o.X1 = g.X1;
    o.V1 = g.V1;
    o.Snew = g.Snew;
    o.U = g.U;
    o.Wm = g.Wm;
    o.sgd = g.sgd;
    o.hb = g.hb;
  }
  BLR_HIP(hipEventRecord(ctx->ev[0], s));
  BLR_HIP(hipGraphLaunch(g.exec, s));
  if (g.exec2) {
    ctx->collide_hook->collide(ctx, g.cvg, g.cV, g.cr, g.cpairs, g.cQ);
    BLR_HIP(hipGraphLaunch(g.exec2, s));
  }
  BLR_HIP(hipEventRecord(ctx->ev[3], s));
  BLR_HIP(hipStreamSynchronize(s));
  o.timed_collision = false;
  step_parse(o);
}

}  // namespace


// ----------------------------------------------------- two-dimensional space
// One K -> S -> L step on the rectangle (Sec. 2.2 applied along both axes,
// the boundary of Sec. 2.3 on every face cell), eager, with the adaptivity of
// Sec. 3: the boundary rows of every face cell added first (their SVD from a
// QR of F_b^T and the SVD of its R factor, 2 (nx + ny) <= 64), the rank
// decision on the SVD of the new S last, err_ada from the factors (Sec.
// 5.1).  The substeps: the pair collisions, the velocity-side products (the
// faces' outflow matrices and inflow vectors, at walls the flux sums that
// make rho_w linear in the adjacent cell's K), K, S and L with their QRs, the
// residual from its pieces.  The state is written only at the end, once the
// residual is finite.
static void dlr_step2d(blr_ctx ctx, const blr_problem* pb, blr_state* st,
                       const blr_step_params* sp, blr_step_info* info) {
  require(st && sp, "null state or step params");
  require(pb->nx >= 1 && pb->ny <= (1 << 20) && (long)pb->nx * pb->ny <= (1L << 22),
          "problem.nx >= 1, ny <= 2^20 and nx * ny <= 2^22");
  require(pb->x_hi > pb->x_lo && pb->y_hi > pb->y_lo, "empty rectangle");
  require(pb->f_left && pb->f_right && pb->f_bottom && pb->f_top, "null boundary function");
  const int wl[4] = {pb->wall_left, pb->wall_right, pb->wall_bottom, pb->wall_top};
  for (int k = 0; k < 4; ++k) require(wl[k] == 0 || wl[k] == 1, "wall flags must be 0 or 1");
  require(pb->face_rows >= 0 && pb->face_rows <= 15, "problem.face_rows must be in [0, 15]");
  validate_vgrid(pb->v);
  require(st->X && st->S && st->V, "null state arrays");
  require(st->r_cap >= 1 && st->r_cap <= 64, "state.r_cap must be in [1, 64]");
  require(st->r >= 1 && st->r <= st->r_cap, "state.r must be in [1, r_cap]");
  require(sp->dt > 0 && std::isfinite(sp->dt), "step.dt must be positive");
  require(!(sp->flags & (BLR_STEP_FP64_DEFECT | BLR_STEP_DEFECT_REFRESH)),
          "the FP64 defect correction is for 1D space only", BLR_ERR_UNSUPPORTED);
  const HostTables& h = get_tables(ctx, pb->v, BLR_FP64).h;
  hipStream_t s = ctx->stream;
  const int nx = pb->nx, ny = pb->ny, n = h.n, rc = st->r_cap, r_in = st->r;
  const long nc = (long)nx * ny;
  const double dx = (pb->x_hi - pb->x_lo) / nx, dy = (pb->y_hi - pb->y_lo) / ny;
  const double wx = dx * dy, dvd = std::pow(h.dv, h.d), dt = sp->dt;
  // the rank never exceeds the cell count (the X-side QR needs rows >= r)
  require(r_in <= nc, "state.r must not exceed nx * ny");
  const int r_max = (int)std::min<long>(std::min(sp->r_max > 0 ? sp->r_max : rc, rc), nc);
  // (capped by the gas cells below, once the obstacle is known)
  const bool drop_on = (sp->flags & BLR_STEP_DROP) != 0;
  const int nface = 2 * (nx + ny);
  // the obstacle: its faces follow the rectangle's (one ghost row and one
  // boundary row each); solid cells hold no gas, so the rank is capped by
  // the gas cells
  const ObstacleHost oh = obstacle_host(pb);
  require(!oh.any || pb->f_obstacle, "problem.solid marks a cell: f_obstacle is needed");
  const int nft = nface + oh.nob;
  long gas = nc;
  for (uint8_t b : oh.solid) gas -= b;
  require(gas >= 1, "problem.solid: no gas cell");
  require(r_in <= gas, "state.r must not exceed the gas cells");
  Obs2 ob{nullptr, nullptr, nullptr, pb->f_obstacle, nface, oh.nob};
  if (oh.any) {
    ob.face = (const int*)ctx->upload("d2.ob.face", oh.face.data(), oh.face.size() * sizeof(int));
    ob.nbmap = (const int*)ctx->upload("d2.ob.nb", oh.nbmap.data(), oh.nbmap.size() * sizeof(int));
    ob.solid = (const uint8_t*)ctx->upload("d2.ob.solid", oh.solid.data(), oh.solid.size());
  }
  const int r_max_g = (int)std::min<long>(r_max, gas);
  const int r_min = std::max(1, std::min(sp->r_min, r_max_g));
  const bool add_on = (sp->flags & BLR_STEP_ADD) && r_in < r_max_g;
  if (add_on)
    require(nft <= 64,
            "two-dimensional space: the basis augmentation needs 2 (nx + ny) + obstacle faces <= 64",
            BLR_ERR_UNSUPPORTED);
  StepWork w{ctx, s, {h.L, h.dv, h.N, h.d, h.n}, (int)nc, n, wx, dvd};
  const dk::FaceRows fr{{pb->f_left, pb->f_right, pb->f_bottom, pb->f_top}, pb->face_rows};
  const int walls = wl[0] | (wl[1] << 1) | (wl[2] << 2) | (wl[3] << 3);
  auto dev2host = [&](const double* d, size_t count) {
    std::vector<double> v(count);
    BLR_HIP(hipMemcpyAsync(v.data(), d, count * sizeof(double), hipMemcpyDeviceToHost, s));
    BLR_HIP(hipStreamSynchronize(s));
    return v;
  };

  // ------------------------------------------------ add (Sec. 3.1)
  const double* Xw = st->X;  // working factors: rows of nc / n values
  const double* Sw = st->S;
  const double* Vw = st->V;
  int lsw = rc, r = r_in, r_added = 0;
  if (add_on) {
    double* K = w.get("d2.K", (size_t)r * nc);
    double* Fb = w.get("d2.Fb", (size_t)nft * n);
    double* Rb = w.get("d2.Rb", (size_t)nft * nft);
    double* Ub = w.get("d2.Ub", (size_t)nft * nft);
    hipLaunchKernelGGL(dk::k_xmul, dim3(blocks((long)r * nc, 256)), dim3(256), 0, s, st->X, r,
                       (int)nc, st->S, rc, K);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_fb2d, dim3(blocks(n, 256), nft), dim3(256), 0, s, K, r, nx, ny,
                       st->V, fr, ob, w.g, Fb);
    BLR_CHECK_LAUNCH();
    if (walls || oh.any) {
      hipLaunchKernelGGL(dk::k_wall_rows2d, dim3(nft), dim3(1024), 0, s, Fb, fr, walls, nx, ny, ob,
                         w.g);
      BLR_CHECK_LAUNCH();
    }
    // the rows outnumber the room r_max - r: keep that room for the boundary
    // information not yet in span V (rows projected onto V^perp; the same span
    // as the rows themselves when the cap does not bind)
    {
      double* Cb = w.get("d2.Cb", (size_t)nft * r);
      GramJob gp;
      gp.add(Fb, nft, st->V, r, false, dk::W_ONE, dvd, Cb);
      gp.run(w);
      hipLaunchKernelGGL(dk::k_proj_rows, dim3(blocks(n, 256), nft), dim3(256), 0, s, Fb, nft,
                         (long)n, Cb, r, st->V);
      BLR_CHECK_LAUNCH();
    }
    // F_b^T = Q Rb, F_b = Rb^T Q^T = Ub diag(sig) (Q Wb)^T: the small SVD of
    // Rb^T on the device, its singular values read back for the count
    tsqr(ctx, Fb, n, n, nft, nullptr, n, Rb, "qr2.fb", 1.0, 1.0);   // R only
    double* sbd = w.get("d2.sb", (size_t)nft);
    double* Wb = w.get("d2.Wb", (size_t)nft * nft);
    // Rb = Wq diag(sig) Ub^T, so Ub (the left singular vectors of Rb^T) comes
    // out as the right singular vectors of Rb; they are coordinates over the
    // boundary rows, which change little from step to step, so the rotations
    // start from the previous step's (any orthogonal start gives the same
    // factorisation; a fresh start every 64 steps keeps the start's rounding
    // from piling up).  Only the columns with sig > add_tol are used.
    double* Ww = w.get("d2.Wwarm", (size_t)64 * 64);
    const bool warm = ctx->bsvd_n == nft && ctx->bsvd_age < 64;
    svd_small(ctx, Rb, nft, Wb, sbd, Ub, false, false, warm ? Ww : nullptr);
    BLR_HIP(hipMemcpyAsync(Ww, Ub, (size_t)nft * nft * sizeof(double), hipMemcpyDeviceToDevice, s));
    ctx->bsvd_n = nft;
    ctx->bsvd_age = warm ? ctx->bsvd_age + 1 : 0;
    const std::vector<double> sig = dev2host(sbd, (size_t)nft);
    for (double v : sig)
      if (!std::isfinite(v)) ctx->bsvd_n = 0;  // no start kept from a failed factorisation
    int rb = 0;
    for (int i = 0; i < nft; ++i) rb += sig[i] > sp->add_tol;
    rb = std::min(rb, r_max_g - r);
    if (rb > 0) {
      const int ra = r + rb;
      double* Vh = w.get("d2.Vh", (size_t)ra * n);
      double* Vq = w.get("d2.Vq", (size_t)ra * n);
      double* Rv = w.get("d2.Rv", (size_t)ra * ra);
      double* Sa = w.get("d2.Sa", (size_t)ra * ra);
      double* Xa = w.get("d2.Xa", (size_t)ra * nc);
      BLR_HIP(hipMemcpyAsync(Vh, st->V, (size_t)r * n * sizeof(double), hipMemcpyDeviceToDevice, s));
      // new rows U_b[:, :rb]^T F_b: the leading right singular vectors times sigma
      hipLaunchKernelGGL(dk::k_rows_comb, dim3(blocks(n, 256), rb), dim3(256), 0, s, Fb, nft,
                         (long)n, Ub, nft, rb, 1.0, Vh + (long)r * n, (long)n);
      BLR_CHECK_LAUNCH();
      tsqr(ctx, Vh, n, n, ra, Vq, n, Rv, "qr2.va", std::sqrt(dvd), 1.0 / std::sqrt(dvd));
      hipLaunchKernelGGL(dk::k_saug, dim3(blocks((long)ra * ra, 256)), dim3(256), 0, s, st->S, rc,
                         r, Rv, ra, Sa);
      BLR_CHECK_LAUNCH();
      // X gains zero rows: X^ S^ (all the step reads of X^n) is unchanged
      BLR_HIP(hipMemcpyAsync(Xa, st->X, (size_t)r * nc * sizeof(double), hipMemcpyDeviceToDevice, s));
      fill<double>(s, Xa + (long)r * nc, (long)rb * nc, 0.0);
      Xw = Xa;
      Sw = Sa;
      Vw = Vq;
      lsw = ra;
      r = ra;
      r_added = rb;
    }
  }

  // ------------------------------------------------ pair collisions
  const int P = r * (r + 1) / 2;
  std::vector<int32_t> pairs(2 * P);
  std::vector<int> pidx(2 * P);
  for (int m = 0, q = 0; m < r; ++m)
    for (int nn = m; nn < r; ++nn, ++q) {
      pidx[q] = pairs[2 * q] = m;
      pidx[P + q] = pairs[2 * q + 1] = nn;
    }
  int* dpidx = (int*)ctx->upload("dlr.d2.pidx", pidx.data(), pidx.size() * sizeof(int));
  const bool fp64c = (sp->flags & BLR_STEP_FP64_COLLISION) != 0;
  void* Qs;
  if (fp64c) {
    Qs = w.get("d2.Q64", (size_t)P * n);
    collision_pairs(ctx, pb->v, BLR_FP64, Vw, r, pairs.data(), P, Qs);
  } else {
    float* V32 = (float*)ctx->buf("dlr.d2.V32", (size_t)r * n * sizeof(float));
    hipLaunchKernelGGL(dk::k_to_f32_copy_S, dim3(blocks((long)r * n, 256)), dim3(256), 0, s, Vw,
                       (long)r * n, V32, nullptr, 0, nullptr, 0);
    BLR_CHECK_LAUNCH();
    Qs = ctx->buf("dlr.d2.Q32", (size_t)P * n * sizeof(float));
    collision_pairs(ctx, pb->v, BLR_FP32, V32, r, pairs.data(), P, Qs);
  }
  // ------------------------------------------------ velocity side
  double* A = w.get("d2.A", (size_t)4 * r * r);   // A1+, A1-, A2+, A2-
  double* Mo = w.get("d2.Mo", (size_t)4 * r * r);
  double* C = w.get("d2.C", (size_t)r * P);
  const double* fk[4] = {pb->f_left, pb->f_right, pb->f_bottom, pb->f_top};
  static const int kOut[4] = {dk::W_OUT_LEFT, dk::W_OUT_RIGHT, dk::W_OUT_BOTTOM, dk::W_OUT_TOP};
  static const int kIn[4] = {dk::W_IN_LEFT, dk::W_IN_RIGHT, dk::W_IN_BOTTOM, dk::W_IN_TOP};
  // a_l: (v.n)_out = -v1 (x_lo), v1 (x_hi), -v2 (y_lo), v2 (y_hi) on the outgoing half;
  // den: |v.n|_in = v1 (x_lo), -v1 (x_hi), v2 (y_lo), -v2 (y_hi) on the incoming half
  static const int kA[4] = {dk::W_VMINUS, dk::W_VPLUS, dk::W_V2MINUS, dk::W_V2PLUS};
  static const int kD[4] = {dk::W_VPLUS, dk::W_VMINUS, dk::W_V2PLUS, dk::W_V2MINUS};
  static const double sA[4] = {-1.0, 1.0, -1.0, 1.0}, sD[4] = {1.0, -1.0, 1.0, -1.0};
  static const int kT[4] = {dk::W_VPLUS, dk::W_VMINUS, dk::W_V2PLUS, dk::W_V2MINUS};
  double* ones = nullptr;
  if (walls || oh.any) {
    ones = w.get("d2.ones", (size_t)n);
    fill<double>(s, ones, n, 1.0);
  }
  dk::Faces2 fs{};
  GramJob gj;
  auto add = [&](const double* Aa, int ra, const void* B, int rb, bool bf, int mode, double* out) {
    if (gj.gb.nseg == dk::MAXSEG) {
      gj.run(w);
      gj = GramJob{};
    }
    gj.add(Aa, ra, B, rb, bf, mode, dvd, out);
  };
  for (int k = 0; k < 4; ++k) add(Vw, r, Vw, r, false, kT[k], A + (long)k * r * r);
  add(Vw, r, Qs, P, !fp64c, dk::W_ONE, C);
  for (int k = 0; k < 4; ++k) {
    const int rows = ((pb->face_rows >> k) & 1) ? (k < 2 ? ny : nx) : 1;
    const std::string tag = "d2.face" + std::to_string(k);
    double* gin = w.get((tag + ".gin").c_str(), (size_t)r * rows);
    add(Vw, r, Vw, r, false, kOut[k], Mo + (long)k * r * r);
    add(Vw, r, fk[k], rows, false, kIn[k], gin);
    dk::Face2& F = fs.f[k];
    F.Mo = Mo + (long)k * r * r;
    F.gin = gin;
    F.rows = rows;
    F.wall = wl[k];
    F.sa = sA[k];
    F.sd = sD[k];
    if (wl[k]) {
      double* a = w.get((tag + ".a").c_str(), (size_t)r);
      double* den = w.get((tag + ".den").c_str(), (size_t)rows);
      add(Vw, r, ones, 1, false, kA[k], a);
      add(ones, 1, fk[k], rows, false, kD[k], den);
      F.a = a;
      F.den = den;
    }
  }
  // obstacle faces of outward normal k: the same outgoing-half Gram matrix,
  // the obstacle's Maxwellian on the incoming half, always a diffusive wall
  for (int k = 0; k < 4 && oh.any; ++k) {
    const std::string tag = "d2.obst" + std::to_string(k);
    double* gin = w.get((tag + ".gin").c_str(), (size_t)r);
    double* a = w.get((tag + ".a").c_str(), (size_t)r);
    double* den = w.get((tag + ".den").c_str(), 1);
    add(Vw, r, pb->f_obstacle, 1, false, kIn[k], gin);
    add(Vw, r, ones, 1, false, kA[k], a);
    add(ones, 1, pb->f_obstacle, 1, false, kD[k], den);
    dk::Face2& F = fs.f[4 + k];
    F.Mo = Mo + (long)k * r * r;
    F.gin = gin;
    F.rows = 1;
    F.wall = 1;
    F.sa = sA[k];
    F.sd = sD[k];
    F.a = a;
    F.den = den;
  }
  gj.run(w);
  double* G = w.get("d2.G", (size_t)nft * r);
  auto ghosts = [&](const double* Kx) {
    hipLaunchKernelGGL(dk::k_ghosts2d, dim3(nft), dim3(64), 0, s, Kx, r, nx, ny, fs, ob, G);
    BLR_CHECK_LAUNCH();
  };
  // ------------------------------------------------ K-step
  double* K = w.get("d2.K", (size_t)r * nc);
  double* K1 = w.get("d2.K1", (size_t)r * nc);
  // dK and the working X^n side by side: both are Z rows of the S-pass reduction
  double* Z = w.get("d2.Z", (size_t)2 * r * nc);
  double* dK = Z;
  double* X1 = w.get("d2.X1", (size_t)r * nc);
  double* S1 = w.get("d2.S1", (size_t)r * r);
  hipLaunchKernelGGL(dk::k_xmul, dim3(blocks((long)r * nc, 256)), dim3(256), 0, s, Xw, r, (int)nc,
                     Sw, lsw, K);
  BLR_CHECK_LAUNCH();
  ghosts(K);
  hipLaunchKernelGGL(dk::k_kstep2d, dim3(blocks((long)r * nc, 256)), dim3(256), 0, s, K, G, r, nx,
                     ny, dx, dy, dt, A, C, P, dpidx, dpidx + P, ob, K1, dK);
  BLR_CHECK_LAUNCH();
  tsqr(ctx, K1, nc, nc, r, X1, nc, S1, "qr2.k", std::sqrt(wx), 1.0 / std::sqrt(wx));
  const int nz = drop_on ? 2 * r : r;
  if (drop_on)
    BLR_HIP(hipMemcpyAsync(Z + (long)r * nc, Xw, (size_t)r * nc * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  // ------------------------------------------------ S-step (K = X1 S1)
  double* D = w.get("d2.D", (size_t)4 * r * r);
  double* T = w.get("d2.T", (size_t)r * P);
  double* kz = w.get("d2.kz", (size_t)r * nz);   // [i][j]: <X1_i, dK_j>, then <X1_i, X^n_j>
  double* S2 = w.get("d2.S2", (size_t)r * r);
  double* dS = w.get("d2.dS", (size_t)r * r);
  hipLaunchKernelGGL(dk::k_xmul, dim3(blocks((long)r * nc, 256)), dim3(256), 0, s, X1, r, (int)nc,
                     S1, r, K);
  BLR_CHECK_LAUNCH();
  ghosts(K);
  hipLaunchKernelGGL(dk::k_xreduce2d, dim3(blocks((long)r * (4 * r + P + nz), 4)), dim3(256), 0, s,
                     X1, r, nx, ny, dx, dy, wx, K, G, P, dpidx, dpidx + P, Z, nz, ob, D, T, kz);
  BLR_CHECK_LAUNCH();
  hipLaunchKernelGGL(dk::k_supdate2d, dim3(blocks((long)r * r, 256)), dim3(256), 0, s, S1, r, D, A,
                     T, C, P, dt, S2, dS);
  BLR_CHECK_LAUNCH();
  // kx = <X1_i, dK_j> compact (r x r) for the residual
  double* kx = w.get("d2.kx", (size_t)r * r);
  hipLaunchKernelGGL(dk::k_copy_S, dim3(blocks((long)r * r, 256)), dim3(256), 0, s, kz, nz, r, kx, r);
  BLR_CHECK_LAUNCH();
  // ------------------------------------------------ L-step (K = X1 S2)
  double* Dt = w.get("d2.Dt", (size_t)4 * r * r);
  double* Tt = w.get("d2.Tt", (size_t)r * P);
  double* L1 = w.get("d2.L1", (size_t)r * n);
  double* dL = w.get("d2.dL", (size_t)r * n);
  double* V1 = w.get("d2.V1", (size_t)r * n);
  double* R = w.get("d2.R", (size_t)r * r);
  hipLaunchKernelGGL(dk::k_xmul, dim3(blocks((long)r * nc, 256)), dim3(256), 0, s, X1, r, (int)nc,
                     S2, r, K);
  BLR_CHECK_LAUNCH();
  ghosts(K);
  hipLaunchKernelGGL(dk::k_xreduce2d, dim3(blocks((long)r * (4 * r + P), 4)), dim3(256), 0, s, X1,
                     r, nx, ny, dx, dy, wx, K, G, P, dpidx, dpidx + P, nullptr, 0, ob, Dt, Tt,
                     nullptr);
  BLR_CHECK_LAUNCH();
  if (fp64c)
    hipLaunchKernelGGL(dk::k_lstep2d<double>, dim3(blocks((long)r * n, 256)), dim3(256), 0, s, Vw,
                       r, n, S2, Dt, Tt, (const double*)Qs, P, dt, w.g, L1, dL);
  else
    hipLaunchKernelGGL(dk::k_lstep2d<float>, dim3(blocks((long)r * n, 256)), dim3(256), 0, s, Vw,
                       r, n, S2, Dt, Tt, (const float*)Qs, P, dt, w.g, L1, dL);
  BLR_CHECK_LAUNCH();
  tsqr(ctx, L1, n, n, r, V1, n, R, "qr2.l", std::sqrt(dvd), 1.0 / std::sqrt(dvd));
  // ------------------------------------------------ residual (Sec. 5.1)
  double* lv = w.get("d2.lv", (size_t)r * r);
  double* Bv = w.get("d2.Bv", (size_t)r * r);
  {
    GramJob g2;
    g2.add(dL, r, Vw, r, false, dk::W_ONE, dvd, lv);
    if (drop_on) g2.add(Vw, r, V1, r, false, dk::W_ONE, dvd, Bv);   // <V^n_l, V1_j>
    g2.run(w);
  }
  const int nbp = 256;
  double* part = w.get("d2.part", (size_t)2 * nbp);
  double* err = w.get("d2.err", 1);
  hipLaunchKernelGGL(dk::k_sumsq2, dim3(nbp), dim3(256), 0, s, dK, (long)r * nc, dL, (long)r * n,
                     part);
  BLR_CHECK_LAUNCH();
  hipLaunchKernelGGL(dk::k_err2d, dim3(1), dim3(64), 0, s, part, nbp, dS, kx, lv, r, wx, dvd, err);
  BLR_CHECK_LAUNCH();
  // drop ingredients on the device: the SVD of the new S = R^T and the terms
  // g_c = sigma_c <A U_c, S^n B W_c> of <f^n, D> (A_ki = <X^n_k, X1_i>,
  // B_lj = <V^n_l, V1_j>), read back with the residual in one record
  double* U2 = nullptr;
  double* s2 = nullptr;
  double* W2 = nullptr;
  double* gt = nullptr;
  if (drop_on) {
    U2 = w.get("d2.U2", (size_t)r * r);
    s2 = w.get("d2.s2", (size_t)r);
    W2 = w.get("d2.W2", (size_t)r * r);
    svd_small(ctx, R, r, U2, s2, W2, true);
    double* Sc = w.get("d2.Sc", (size_t)r * r);
    double* Ac = w.get("d2.Ac", (size_t)r * r);
    gt = w.get("d2.gt", (size_t)r);
    hipLaunchKernelGGL(dk::k_copy_S, dim3(blocks((long)r * r, 256)), dim3(256), 0, s, Sw, lsw, r,
                       Sc, r);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_gather_T, dim3(blocks((long)r * r, 256)), dim3(256), 0, s, kz, nz, r, r,
                       Ac);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_fnD_terms, dim3(1), dim3(256), 0, s, Sc, Ac, U2, s2, W2, Bv, r, gt);
    BLR_CHECK_LAUNCH();
  }
  const int nrb = drop_on ? r : 0;
  double* pk = w.get("d2.pack", (size_t)1 + 2 * 64);
  hipLaunchKernelGGL(dk::k_pack2d, dim3(1), dim3(64), 0, s, err, s2, gt, nrb, pk);
  BLR_CHECK_LAUNCH();
  const std::vector<double> rec = dev2host(pk, (size_t)1 + 2 * nrb);
  const double e = rec[0];
  require(std::isfinite(e), "two-dimensional step: non-finite residual", BLR_ERR_NUMERIC);
  blr_step_info inf{};
  inf.r_in = r_in;
  inf.r_added = r_added;
  inf.err = e;
  // ------------------------------------------------ drop (Sec. 3.2) and commit
  if (!drop_on) {
    BLR_HIP(hipMemcpyAsync(st->X, X1, (size_t)r * nc * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(dk::k_store_RT, dim3(blocks((long)r * r, 256)), dim3(256), 0, s, R, r, st->S,
                       rc);
    BLR_CHECK_LAUNCH();
    BLR_HIP(hipMemcpyAsync(st->V, V1, (size_t)r * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    inf.err_ada = e;
    inf.r_out = r;
    st->r = r;
  } else {
    const double* sh = rec.data() + 1;
    const double* g = rec.data() + 1 + r;
    const double drop_tol = sp->c_drop * e;
    int keep = 0;
    for (int i = 0; i < r; ++i) keep += sh[i] >= drop_tol;
    keep = std::max(std::min(std::min(keep, r_max_g), r), std::min(r_min, r));
    // err_ada^2 = err^2 - |Sigma_p|^2 + 2 <f^n, D>,  D = X1 U_p Sigma_p W_p^T V1:
    // <f^n, D> is the sum of g_c over the dropped c
    double sp2 = 0.0, fnD = 0.0;
    for (int c = keep; c < r; ++c) {
      sp2 += sh[c] * sh[c];
      fnD += g[c];
    }
    const double e2 = e * e - sp2 + 2.0 * fnD;
    inf.err_ada = std::sqrt(std::max(e2, 0.0));
    inf.drop_tol = drop_tol;
    inf.r_out = keep;
    // X_i = sum_l U[l][i] X1_l, V_i = sum_l W[l][i] V1_l (i < keep), S = diag(sigma)
    hipLaunchKernelGGL(dk::k_rows_comb, dim3(blocks(nc, 256), keep), dim3(256), 0, s, X1, r, nc, U2,
                       r, keep, 1.0, st->X, nc);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_rows_comb, dim3(blocks(n, 256), keep), dim3(256), 0, s, V1, r, (long)n,
                       W2, r, keep, 1.0, st->V, (long)n);
    BLR_CHECK_LAUNCH();
    hipLaunchKernelGGL(dk::k_diag, dim3(1), dim3(256), 0, s, s2, keep, st->S, rc);
    BLR_CHECK_LAUNCH();
    st->r = keep;
  }
  BLR_HIP(hipStreamSynchronize(s));
  if (info) *info = inf;
}

void dlr_step(blr_ctx ctx, const blr_problem* pb, blr_state* st, const blr_step_params* sp,
              blr_step_info* info) {
  if (pb && pb->ny >= 2) {
    dlr_step2d(ctx, pb, st, sp, info);
    return;
  }
  validate_problem(pb, st);
  require(sp != nullptr, "null step params");
  require(sp->dt > 0 && std::isfinite(sp->dt), "step.dt must be positive");
  const int r_max = std::min(sp->r_max > 0 ? sp->r_max : st->r_cap, st->r_cap);
  const int r_min = std::max(1, std::min(sp->r_min, r_max));
  const HostTables& h = get_tables(ctx, pb->v, BLR_FP64).h;
  hipStream_t s = ctx->stream;
  const int nx = pb->nx, n = h.n, rc = st->r_cap;
  blr_step_info inf{};
  inf.r_in = st->r;

  // FP64 defect correction: refresh when asked, or when the context keeps no
  // defect for this velocity grid
  blr_step_params spx = *sp;
  const bool defect = (sp->flags & BLR_STEP_FP64_DEFECT) != 0;
  require(defect || !(sp->flags & BLR_STEP_DEFECT_REFRESH),
          "BLR_STEP_DEFECT_REFRESH needs BLR_STEP_FP64_DEFECT");
  if (defect) {
    require(!(sp->flags & BLR_STEP_FP64_COLLISION),
            "BLR_STEP_FP64_DEFECT corrects FP32 collisions: not with BLR_STEP_FP64_COLLISION");
    require(rc <= dk::DEFECT_MAX, "BLR_STEP_FP64_DEFECT needs state.r_cap <= 32");
    if (ctx->defect_r == 0 || std::memcmp(&ctx->defect_vg, &pb->v, sizeof(blr_vgrid)) != 0)
      spx.flags |= BLR_STEP_DEFECT_REFRESH;
    // a refresh that does not finish leaves no usable defect
    if (spx.flags & BLR_STEP_DEFECT_REFRESH) ctx->defect_r = 0;
  }
  sp = &spx;

  // The number of boundary functions to add is known only from the singular
  // values of F_b on the device.  The step runs with the count of the
  // previous step (2 at first) and is repeated, from the unchanged state,
  // when the read-back shows another count or a failed projection.
  const bool add = (sp->flags & BLR_STEP_ADD) && st->r < r_max;
  const int room = r_max - st->r;
  Attempt at{add ? std::min(ctx->add_hint < 0 ? 2 : ctx->add_hint, room) : 0,
             (sp->flags & BLR_STEP_HOUSEHOLDER_ADD) != 0, (sp->flags & BLR_STEP_HOUSEHOLDER_QR) != 0};
  Outcome o;
  for (int attempt = 0;; ++attempt) {
    require(attempt < 4, "boundary basis: no consistent attempt", BLR_ERR_NUMERIC);
    o = Outcome{};
    step_attempt(ctx, pb, st, sp, h, add, at, o);
    if (o.qr_failed && !at.householder_qr) {
      at.householder_qr = true;
      continue;
    }
    if (!add) break;
    require(std::isfinite(o.sb[0]) && std::isfinite(o.sb[1]), "non-finite boundary singular value",
            BLR_ERR_NUMERIC);
    int cnt = 0;
    for (double v : o.sb) cnt += v > sp->add_tol ? 1 : 0;
    ctx->add_hint = cnt;
    const int rb = std::min(cnt, room);
    if (rb != at.rb) {
      at = Attempt{rb, at.householder};
      continue;
    }
    if (rb > 0 && o.orth_failed && !at.householder) {
      at.householder = true;
      continue;
    }
    break;
  }
  inf.r_added = at.rb;
  const int r = o.r;
  if (spx.flags & BLR_STEP_DEFECT_REFRESH) {
    ctx->defect_r = r;
    ctx->defect_vg = pb->v;
  }

  const double err = std::sqrt(std::max(o.res[0], 0.0));
  require(std::isfinite(err), "non-finite residual", BLR_ERR_NUMERIC);
  inf.err = err;
  int r_out = r;
  if (sp->flags & BLR_STEP_DROP) {
    for (double v : o.sg) require(std::isfinite(v), "non-finite singular value", BLR_ERR_NUMERIC);
    const double tol = sp->c_drop * err;
    int keep = 0;
    for (double v : o.sg) keep += v >= tol ? 1 : 0;
    keep = std::max(std::min(keep, r_max), std::min(r_min, r));
    double sp2 = 0.0, fnD = 0.0;
    for (int q = keep; q < r; ++q) {
      sp2 += o.sg[q] * o.sg[q];
      fnD += o.g[q];
    }
    inf.drop_tol = tol;
    // err_ada^2 = err^2 - |Sigma_perp|^2 + 2 <f^n, D>
    inf.err_ada = std::sqrt(std::max(err * err - sp2 + 2.0 * fnD, 0.0));
    // commit: rotate and truncate straight into the state
    hipLaunchKernelGGL(dk::k_commit, dim3(blocks(std::max(nx, n), 256), keep), dim3(256), 0, s, o.X1,
                       r, (long)nx, o.U, o.V1, (long)n, o.Wm, keep, st->X, st->V, o.sgd, st->S, rc);
    BLR_CHECK_LAUNCH();
    r_out = keep;
  } else {
    inf.err_ada = err;
    BLR_HIP(hipMemcpyAsync(st->X, o.X1, (size_t)r * nx * 8, hipMemcpyDeviceToDevice, s));
    BLR_HIP(hipMemcpyAsync(st->V, o.V1, (size_t)r * n * 8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(dk::k_copy_S, dim3(blocks(r * r, 256)), dim3(256), 0, s, o.Snew, r, r, st->S, rc);
    BLR_CHECK_LAUNCH();
  }
  // the commit stays queued on the stream; both timed spans ended before the wait
  float ms = 0.f;
  BLR_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[3]));
  inf.ms_step = ms;
  inf.ms_collision = 0.f;
  if (o.timed_collision) {
    BLR_HIP(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
    inf.ms_collision = ms;
  }
  inf.r_out = r_out;
  st->r = r_out;
  st->step += 1;
  if (info) *info = inf;
}

// Truncated SVD of f0 (Sec. 2.4, first paragraph) by one-sided Jacobi on the
// rows of Y = sqrt(wx dv^d) f0 (cells x n, row-major): pairs of rows are
// rotated until every pair is orthogonal to working precision, the same
// rotations accumulated in W (cells x cells, from the identity).  Then
// Y = W A with orthogonal rows, so A = W^T Y: the row norms of Y are the
// singular values, the rows of W the left and the normalised rows of Y the
// right singular vectors.  One-sided Jacobi keeps every singular value to
// high relative accuracy (no Gram matrix is formed).  Each round rotates
// cells/2 disjoint pairs (round-robin schedule, one workgroup per pair); a
// sweep of cells - 1 rounds meets every pair once; sweeps repeat until one
// applies no rotation.
void state_from_full(blr_ctx ctx, const blr_problem* pb, const double* f0, int r, blr_state* st) {
  require(pb && st && f0, "null argument");
  validate_vgrid(pb->v);
  const bool two_d = pb->ny >= 2;
  require(pb->nx >= 1, "nx must be >= 1");
  require(st->r_cap >= 1 && st->r_cap <= 64, "r_cap must be in [1, 64]");
  require(st->r_cap >= r && r >= 1, "r must be in [1, r_cap]");
  const HostTables& h = get_tables(ctx, pb->v, BLR_FP64).h;
  const int cells = pb->nx * (two_d ? pb->ny : 1);
  const long n = h.n;
  require(r <= cells && r <= n, "r must not exceed the number of cells nor of velocity points");
  require(cells <= 8192, "state_from_full: at most 8192 cells", BLR_ERR_UNSUPPORTED);
  const double dx = (pb->x_hi - pb->x_lo) / pb->nx;
  const double wx = two_d ? dx * (pb->y_hi - pb->y_lo) / pb->ny : dx;
  const double dvd = std::pow(h.dv, h.d);
  require(wx > 0, "x_hi must exceed x_lo (and y_hi y_lo)");
  hipStream_t s = ctx->stream;
  auto get = [&](const char* nm, size_t c) {
    return (double*)ctx->buf(std::string("sff.") + nm, c * sizeof(double));
  };
  double* Y = get("Y", (size_t)cells * n);
  double* W = get("W", (size_t)cells * cells);
  double* nrm = get("norm", cells);
  int* flag = (int*)ctx->buf("sff.flag", sizeof(int));
  int* hflag = (int*)ctx->host_readback(sizeof(double) * std::max(cells, 2));
  hipLaunchKernelGGL(dk::k_sff_load, dim3(blocks((long)cells * n, 256)), dim3(256), 0, s, f0,
                     (long)cells * n, std::sqrt(wx * dvd), Y);
  BLR_CHECK_LAUNCH();
  hipLaunchKernelGGL(dk::k_sff_eye, dim3(blocks((long)cells * cells, 256)), dim3(256), 0, s, W,
                     cells);
  BLR_CHECK_LAUNCH();
  if (cells > 1) {
    const int mpad = cells + (cells & 1);
    // rotate while |<y_p, y_q>| > tol |y_p| |y_q|: the rounding level of a dot
    // product of n terms, so that a converged pair is not rotated again
    const double tol = 2.0 * std::sqrt((double)n) * 2.220446049250313e-16;
    bool done = false;
    for (int sweep = 0; sweep < 60 && !done; ++sweep) {
      hipLaunchKernelGGL(dk::k_sff_flag, dim3(1), dim3(64), 0, s, flag, 0);
      BLR_CHECK_LAUNCH();
      for (int round = 0; round < mpad - 1; ++round) {
        hipLaunchKernelGGL(dk::k_sff_round, dim3(mpad / 2), dim3(dk::SFF_BS), 0, s, Y, n, W,
                           cells, mpad, round, tol, flag);
        BLR_CHECK_LAUNCH();
      }
      BLR_HIP(hipMemcpyAsync(hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
      BLR_HIP(hipStreamSynchronize(s));
      done = hflag[0] == 0;
    }
    require(done, "state_from_full: Jacobi SVD did not converge in 60 sweeps", BLR_ERR_NUMERIC);
  }
  hipLaunchKernelGGL(dk::k_sff_norms, dim3(cells), dim3(dk::SFF_BS), 0, s, Y, n, nrm);
  BLR_CHECK_LAUNCH();
  double* hn = (double*)hflag;
  BLR_HIP(hipMemcpyAsync(hn, nrm, sizeof(double) * cells, hipMemcpyDeviceToHost, s));
  BLR_HIP(hipStreamSynchronize(s));
  // the r largest singular values, in descending order (ties by index)
  std::vector<int> order(cells);
  for (int i = 0; i < cells; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hn[a] > hn[b]; });
  for (int k = 0; k < r; ++k)
    require(std::isfinite(hn[order[k]]), "state_from_full: f0 is not finite", BLR_ERR_NUMERIC);
  require(hn[order[r - 1]] > 0.0, "state_from_full: f0 has rank below r", BLR_ERR_NUMERIC);
  int* idx = (int*)ctx->upload("sff.idx", order.data(), sizeof(int) * r);
  hipLaunchKernelGGL(dk::k_sff_store, dim3(blocks(std::max<long>(n, cells), 256), r), dim3(256),
                     0, s, Y, n, W, cells, nrm, idx, r, 1.0 / std::sqrt(wx), 1.0 / std::sqrt(dvd),
                     st->X, st->V, st->S, st->r_cap);
  BLR_CHECK_LAUNCH();
  BLR_HIP(hipStreamSynchronize(s));
  st->r = r;
}

// Repeated steps until err_ada <= res_tol or max_steps (Sec. 5.1).  *info
// holds the steps taken so far also when a step fails (the exception
// propagates) or `cancel` is raised between steps (info->converged = 0).
void steady_solve(blr_ctx ctx, const blr_problem* pb, blr_state* state, const blr_solve_params* p,
                  blr_solve_info* info, const std::atomic<bool>* cancel) {
  require(p != nullptr && info != nullptr, "null solve params");
  require(p->max_steps >= 1, "max_steps must be >= 1");
  require(p->res_tol >= 0, "res_tol must be >= 0");
  *info = blr_solve_info{};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BLR_HIP(hipEventCreate(&e0));
  BLR_HIP(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  // FP64 defect correction: a refresh on the first step and every
  // defect_every steps
  const bool defect = (p->step.flags & BLR_STEP_FP64_DEFECT) != 0;
  const int64_t every = p->defect_every > 0 ? p->defect_every : 4;
  BLR_HIP(hipEventRecord(e0, ctx->stream));
  for (int64_t k = 0; k < p->max_steps; ++k) {
    if (cancel && cancel->load(std::memory_order_relaxed)) break;
    blr_step_info si{};
    blr_step_params spk = p->step;
    if (defect && k % every == 0) spk.flags |= BLR_STEP_DEFECT_REFRESH;
    dlr_step(ctx, pb, state, &spk, &si);
    const int64_t rk = si.r_in + si.r_added;
    info->pair_evals += rk * (rk + 1) / 2;
    info->steps = k + 1;
    info->err_ada = si.err_ada;
    info->r = state->r;
    if (si.err_ada <= p->res_tol) {
      info->converged = 1;
      break;
    }
  }
  BLR_HIP(hipEventRecord(e1, ctx->stream));
  BLR_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  BLR_HIP(hipEventElapsedTime(&ms, e0, e1));
  info->ms_wall = ms;
}

// Device bytes a context holds for solves of this shape: the collision
// workspace at r_cap plus the step's named buffers (velocity-side arrays of
// r_cap rows: working copy, L-step result and update, new basis, QR scratch;
// the pair collisions; x-side arrays).  An estimate used for admission.
size_t solve_workspace_bytes(const blr_vgrid& vg, int nx, int r_cap, bool fp64_collision,
                             bool defect) {
  validate_vgrid(vg);
  require(nx >= 1 && r_cap >= 1 && r_cap <= 64, "bad solve shape");
  const size_t n = (size_t)std::llround(std::pow((double)vg.n, vg.d));
  const size_t P = (size_t)r_cap * (r_cap + 1) / 2;
  size_t b = collision_workspace_bytes(vg, r_cap, fp64_collision ? BLR_FP64 : BLR_FP32);
  b += (size_t)r_cap * n * 8 * 6;
  b += fp64_collision ? P * n * 8 : P * n * 4 + (size_t)r_cap * n * 4;
  b += (size_t)r_cap * nx * 8 * 8 + (size_t)P * r_cap * 8 * 4 + (8u << 20);
  if (defect && !fp64_collision) {
    // FP64 pairs and the FP64 collision workspace; the kept defect and basis;
    // the carried halves
    b += P * n * 8 + collision_workspace_bytes(vg, r_cap, BLR_FP64);
    b += P * n * 8 + (size_t)r_cap * n * 8;
    b += (size_t)r_cap * std::min(r_cap, 32) * n * 8;
  }
  return b;
}

}  // namespace blr

// ------------------------------------------------------------------ C ABI --
template <class F>
static blr_status guarded_dlr(blr_ctx ctx, F&& f) {
  if (!ctx) return BLR_ERR_ARG;
  ctx->err.clear();
  try {
    BLR_HIP(hipSetDevice(ctx->device));
    f();
    return BLR_OK;
  } catch (const blr::Error& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return BLR_ERR_HIP;
  }
}

extern "C" {

blr_status blr_svd_small(blr_ctx ctx, const double* A, int32_t r, int32_t trans, int32_t complete,
                         double* U, double* sig, double* W) {
  return guarded_dlr(ctx, [&] {
    blr::require(A && U && sig && W, "null pointer argument");
    blr::svd_small(ctx, A, r, U, sig, W, trans != 0, complete != 0);
  });
}

blr_status blr_state_from_full(blr_ctx ctx, const blr_problem* pb, const double* f0, int32_t r,
                               blr_state* state) {
  return guarded_dlr(ctx, [&] { blr::state_from_full(ctx, pb, f0, r, state); });
}

blr_status blr_dlr_step(blr_ctx ctx, const blr_problem* pb, blr_state* state,
                        const blr_step_params* sp, blr_step_info* info) {
  return guarded_dlr(ctx, [&] { blr::dlr_step(ctx, pb, state, sp, info); });
}

blr_status blr_steady_solve(blr_ctx ctx, const blr_problem* pb, blr_state* state,
                            const blr_solve_params* p, blr_solve_info* info) {
  blr_solve_info out{};
  const blr_status rc = guarded_dlr(ctx, [&] { blr::steady_solve(ctx, pb, state, p, &out); });
  if (info) *info = out;
  if (rc != BLR_OK) return rc;
  return out.converged ? BLR_OK : BLR_ERR_NOT_CONVERGED;
}

}  // extern "C"
