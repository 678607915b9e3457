// FP64 dense linear algebra of the low-rank step.
//
//   tsqr   Householder QR of a tall-skinny column-major matrix (rows >= 1,
//          1 <= r <= 64) as a reduction tree: blocks of 256 rows are
//          factorised by one wavefront each (up to four rows per lane held in
//          registers, column sums by DPP cross-lane reductions, no barriers;
//          rows padded with zeros to at least r), their R factors are stacked and factorised again until
//          one block remains; Q is formed top-down by applying each level's
//          reflectors to the next level's Q block.  The sign of every row of R
//          is chosen so that diag(R) >= 0 (the top-level Q starts from
//          D = sign(diag R) instead of the identity).  Householder reflections
//          stay orthogonal when the matrix is rank deficient, which the basis-
//          augmentation step produces on purpose (zero block of S).
//   svd    one-sided Jacobi SVD of an r x r matrix (one workgroup), singular
//          values in descending order, zero columns of U completed to an
//          orthonormal set.
#include <cmath>
#include <cstring>

#include "linalg.hpp"

namespace blr {
namespace la {


__device__ __forceinline__ double block_sum(double x, double* red) {
  // deterministic: wave shuffles, then a fixed-order sum of the 4 wave totals
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// One wavefront per block; each lane owns RPL rows of the block in
// registers, so a block covers MBR = 64 * RPL rows.
constexpr int QT = 64;
template <int RM>
struct QRShape {
  // rows per lane: up to 4 for narrow panels, and at least 2 RM / QT so that a
  // block holds twice as many rows as its R factor (each tree level halves
  // the rows; with 64 rows for 64 columns the tree would never shrink)
  static constexpr int RPL0 = (48 / RM) < 1 ? 1 : ((48 / RM) > 4 ? 4 : (48 / RM));
  static constexpr int RMIN = (2 * RM + QT - 1) / QT;
  static constexpr int RPL = RPL0 > RMIN ? RPL0 : RMIN;
  static constexpr int MBR = QT * RPL;  // rows per block
};

// Cross-lane move of a double with a DPP control (two 32-bit moves); lanes
// whose source is outside the row read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes, returned to every lane: quad permutations and row
// rotations sum each row of 16 lanes, two row broadcasts carry the row sums
// into lane 63, whose value is read back as a scalar.  Fixed instruction
// sequence, so the result is reproducible.
__device__ __forceinline__ double wave_allsum(double x) {
  x += dpp_move<0xb1>(x);   // quad_perm [1,0,3,2]
  x += dpp_move<0x4e>(x);   // quad_perm [2,3,0,1]
  x += dpp_move<0x124>(x);  // row_ror:4
  x += dpp_move<0x128>(x);  // row_ror:8
  x += dpp_move<0x142>(x);  // row_bcast:15
  x += dpp_move<0x143>(x);  // row_bcast:31
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Orders the LDS accesses of one wavefront (its DS instructions execute in
// order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sums over the 64 lanes of a one-wavefront block, returned to every lane.
// A few values: DPP sums.  Many (the Householder panels' column products):
// through LDS, lane t writing its NV values as row t of a padded 64 x NV
// table and lane c < NV summing column c in lane order, so the NV sums run
// side by side instead of as NV dependent DPP chains.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double*) {
  if constexpr (NV < 8) {
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = wave_allsum(v[c]);
  } else {
    __shared__ double red[64 * (NV + 1)];
    __shared__ double tot[NV];
    const int t = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < NV; ++c) red[t * (NV + 1) + c] = v[c];
    wave_sync();
    if (t < NV) {
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < 64; ++k) acc += red[k * (NV + 1) + t];
      tot[t] = acc;
    }
    wave_sync();
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = tot[c];
  }
}

// Factor block b of a column-major matrix A (rows x r, leading dim lda),
// scaled by in_scale on load.  Thread t owns rows t, t+QT, .. of the block.
// Writes the Householder vectors (unit diagonal implied) into Y (leading dim
// ldy = padded rows), tau[b*r + k], and R into Rst (stacked column-major,
// leading dim nb*r), rows [b*r, b*r + r).
template <int RM, int RPL = QRShape<RM>::RPL, int MB = QRShape<RM>::MBR>
__global__ __launch_bounds__(QT) void k_qr_block(const double* __restrict__ A, long lda, long rows,
                                                 int r, double in_scale, double* __restrict__ Y,
                                                 long ldy, double* __restrict__ tau,
                                                 double* __restrict__ Rst, long ldr) {
  double* buf = nullptr;
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  const int m = (int)max((long)r, min((long)MB, rows - (long)b * MB));  // active rows (>= r)
  // The pivot column is always a[.][0]: after step k the finished column is
  // written out and the remaining columns shift left, so every register index
  // is static while the column loop stays rolled.
  double a[RPL][RM];
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int i = t + QT * h;
    const long row = (long)b * MB + i;
    const bool live = i < m && row < rows;
#pragma unroll
    for (int c = 0; c < RM; ++c) a[h][c] = (live && c < r) ? in_scale * A[c * lda + row] : 0.0;
  }
#pragma unroll 1
  for (int k = 0; k < r; ++k) {
    double tx[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int i = t + QT * h;
      if (i > k && i < m) tx[0] += a[h][0] * a[h][0];
      if (i == k) tx[1] = a[h][0];
    }
    block_sums<2>(tx, buf);
    const double tail = tx[0], x0 = tx[1];
    double beta, tk, scale;
    if (tail == 0.0) {
      tk = 0.0;
      beta = x0;
      scale = 0.0;
    } else {
      const double nrm = sqrt(x0 * x0 + tail);
      beta = x0 >= 0.0 ? -nrm : nrm;
      tk = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    double vi[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int i = t + QT * h;
      vi[h] = 0.0;
      if (i > k && i < m) {
        a[h][0] *= scale;
        vi[h] = a[h][0];
      } else if (i == k) {
        a[h][0] = beta;
        vi[h] = 1.0;
      }
    }
    // columns past r are zero and stay zero, so no column guard is needed
    double wv[RM - 1];
#pragma unroll
    for (int c = 1; c < RM; ++c) {
      double part = 0.0;
#pragma unroll
      for (int h = 0; h < RPL; ++h) part += vi[h] * a[h][c];
      wv[c - 1] = part;
    }
    block_sums<RM - 1>(wv, buf);
#pragma unroll
    for (int c = 1; c < RM; ++c) {
#pragma unroll
      for (int h = 0; h < RPL; ++h) a[h][c] -= tk * wv[c - 1] * vi[h];
    }
    if (t == 0) tau[(long)b * r + k] = tk;
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int i = t + QT * h;
      Y[k * ldy + (long)b * MB + i] = (i > k && i < m) ? a[h][0] : 0.0;
      if (i < r) Rst[k * ldr + (long)b * r + i] = (i <= k) ? a[h][0] : 0.0;
#pragma unroll
      for (int c = 0; c + 1 < RM; ++c) a[h][c] = a[h][c + 1];
      a[h][RM - 1] = 0.0;
    }
  }
}

// Q block b = out_scale * H_0 .. H_{r-1} [C_b; 0], C_b = rows [b*r, b*r+r) of Cst.
template <int RM, int RPL = QRShape<RM>::RPL, int MB = QRShape<RM>::MBR>
__global__ __launch_bounds__(QT) void k_qr_apply(const double* __restrict__ Y, long ldy, long rows,
                                                 int r, const double* __restrict__ tau,
                                                 const double* __restrict__ Cst, long ldc,
                                                 double out_scale, double* __restrict__ Q,
                                                 long ldq) {
  double* buf = nullptr;
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  const int m = (int)max((long)r, min((long)MB, rows - (long)b * MB));
  double y[RPL][RM];
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int i = t + QT * h;
#pragma unroll
    for (int c = 0; c < RM; ++c) y[h][c] = (i < r && c < r) ? Cst[c * ldc + (long)b * r + i] : 0.0;
  }
#pragma unroll
  for (int k = RM - 1; k >= 0; --k) {
   const double tk = k < r ? tau[(long)b * r + k] : 0.0;
   if (tk != 0.0) {  // uniform across the block
    double v[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
      const int i = t + QT * h;
      v[h] = (i > k && i < m) ? Y[k * ldy + (long)b * MB + i] : (i == k ? 1.0 : 0.0);
    }
    double wv[RM];
#pragma unroll
    for (int c = 0; c < RM; ++c) {
      double part = 0.0;
#pragma unroll
      for (int h = 0; h < RPL; ++h) part += v[h] * y[h][c];
      wv[c] = part;
    }
    block_sums<RM>(wv, buf);
#pragma unroll
    for (int c = 0; c < RM; ++c) {
      if (c < r) {
#pragma unroll
        for (int h = 0; h < RPL; ++h) y[h][c] -= tk * wv[c] * v[h];
      }
    }
   }
  }
#pragma unroll
  for (int h = 0; h < RPL; ++h) {
    const int i = t + QT * h;
    const long row = (long)b * MB + i;
    if (i < m && row < rows) {
#pragma unroll
      for (int c = 0; c < RM; ++c)
        if (c < r) Q[c * ldq + row] = out_scale * y[h][c];
    }
  }
}

// final sign fix: D = sign(diag R) (0 -> +1); R <- D R; C <- D (the top-level
// Q seed, an r x r col-major matrix with leading dimension ldc)
__global__ void k_qr_sign(double* R, long ldr, int r, double* C, long ldc) {
  const int i = threadIdx.x;
  if (i >= r) return;
  const double s = R[i * ldr + i] < 0.0 ? -1.0 : 1.0;
  for (int c = 0; c < r; ++c) {
    R[c * ldr + i] *= s;
    C[c * ldc + i] = (c == i) ? s : 0.0;
  }
}

__global__ void k_copy_R(const double* Rst, long ldr, int r, double* R) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * r) return;
  const int i = t % r, c = t / r;
  R[i * r + c] = Rst[c * ldr + i];  // row-major out
}

// ------------------------------------------------------------------ SVD --
// Sum over aligned groups of lpp in {1, 2, 4, 8} lanes, returned to every lane
// of the group (quad permutations, then the half-row mirror, which pairs
// each lane with one of the other quad).
__device__ __forceinline__ double group_sum(double x, int lpp) {
  if (lpp >= 2) x += dpp_move<0xb1>(x);   // quad_perm [1,0,3,2]
  if (lpp >= 4) x += dpp_move<0x4e>(x);   // quad_perm [2,3,0,1]
  if (lpp >= 8) x += dpp_move<0x141>(x);  // row_half_mirror
  return x;
}


constexpr int SVS = 65;  // LDS column stride of the Jacobi SVD (doubles)

// The end of the Jacobi SVD on one wavefront (lanes t < 64): column norms,
// descending order (ties by index), the outputs, and U's completion.
__device__ void svd_finish(const double* __restrict__ B, double* __restrict__ V,
                           double* __restrict__ nrm, int* __restrict__ order, int r,
                           double* __restrict__ U, double* __restrict__ sig,
                           double* __restrict__ W, int complete, int t) {
  if (t < r) {
    double s = 0;
    for (int i = 0; i < r; ++i) s += B[t * SVS + i] * B[t * SVS + i];
    nrm[t] = sqrt(s);
  }
  wave_sync();
  // descending, ties by index: column t goes to position rank(t)
  if (t < r) {
    const double mine = nrm[t];
    int rank = 0;
    for (int c = 0; c < r; ++c) {
      const double o = nrm[c];
      rank += (o > mine || (o == mine && c < t)) ? 1 : 0;
    }
    order[rank] = t;
  }
  wave_sync();
  // U columns (normalised), W columns, sigma; row-major outputs.  The
  // normalised columns also go to LDS (over V, once W is out) for the
  // completion below.
  double s_mine = 0.0;
  int src = 0;
  if (t < r) {
    src = order[t];
    s_mine = nrm[src];
    sig[t] = s_mine;
    const double inv = s_mine > 0 ? 1.0 / s_mine : 0.0;
    for (int i = 0; i < r; ++i) {
      U[i * r + t] = B[src * SVS + i] * inv;
      W[i * r + t] = V[src * SVS + i];
    }
  }
  // complete U where sigma underflows (tiny or zero columns): each such
  // column j, in order, becomes the normalised part of a unit vector
  // orthogonal to the other (non-small, or earlier completed) columns.  Lane
  // i holds entry i of the candidate; the dot products are wavefront sums.
  const double s0 = __shfl(s_mine, 0, 64);
  const bool small = t < r && !(s_mine > 1e-300 && s_mine > 1e-14 * s0);
  if (!complete || !__any(small)) return;
  wave_sync();
  if (t < r) {
    const double inv = s_mine > 0 ? 1.0 / s_mine : 0.0;
    for (int i = 0; i < r; ++i) V[t * SVS + i] = small ? 0.0 : B[src * SVS + i] * inv;
    nrm[t] = small ? 0.0 : 1.0;  // 1: column t is in the basis
  }
  wave_sync();
  auto wsum = [](double x) { return wave_allsum(x); };
  // part of the unit vector e orthogonal to the basis columns other than j
  // (two Gram-Schmidt passes); returns its norm
  auto orth = [&](int e, int j, double& v) {
    v = (t == e) ? 1.0 : 0.0;
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < r; ++k) {
        if (k == j || nrm[k] == 0.0) continue;
        const double u = t < r ? V[k * SVS + t] : 0.0;
        v -= wsum(u * v) * u;
      }
    return sqrt(wsum(v * v));
  };
  // candidates are tried from the one after the last accepted (the earlier
  // unit vectors are mostly in the span already); the first with a part of
  // norm > 1/2 is taken, else the one with the largest part (at least
  // r^(-1/2): the parts' squared norms over all e sum to at least 1)
  int e_next = 0;
  for (int j = 0; j < r; ++j) {
    if (nrm[j] != 0.0) continue;  // uniform: LDS read by every lane
    double v = 0.0, nn = 0.0, best_nn = -1.0;
    int e = 0, best_e = 0;
    for (int att = 0; att < r; ++att) {
      e = (e_next + att) % r;
      nn = orth(e, j, v);
      if (nn > 0.5) break;
      if (nn > best_nn) {
        best_nn = nn;
        best_e = e;
      }
    }
    if (!(nn > 0.5)) {
      e = best_e;
      nn = orth(e, j, v);
    }
    if (t < r) {
      V[j * SVS + t] = v / nn;
      U[t * r + j] = v / nn;
    }
    wave_sync();
    if (t == 0) nrm[j] = 1.0;
    wave_sync();
    e_next = e + 1;
  }
}

// One-sided Jacobi on the columns of B = A (r x r row-major): B W = U Sigma.
// Columns live in LDS (stride 65 doubles: the column pairs of one round sit
// in different banks).  Each round rotates rr/2 disjoint column pairs
// (circle method, a dummy column when r is odd); a pair is handled by a
// group of lpp lanes, each taking the rows i = sub, sub + lpp, ..; the three
// column sums are completed inside the group by DPP, so every lane of the
// group computes the same rotation.  One wavefront: the rounds are ordered
// by wavefront barriers.
__global__ __launch_bounds__(64) void k_svd_jacobi(const double* __restrict__ A, int r,
                                                   double* __restrict__ U, double* __restrict__ sig,
                                                   double* __restrict__ W, int sweeps, int trans,
                                                   int complete) {
  __shared__ double B[64 * SVS];  // column c: B[c * SVS + i]
  __shared__ double V[64 * SVS];
  __shared__ double nrm[64];
  __shared__ int order[64];
  const int t = threadIdx.x;
  // all r^2 loads in flight at once (lane t: entries t, t + 64, ..)
  double fro2 = 0.0;
  for (int e0 = 0; e0 < r * r; e0 += 64 * 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = e0 + 64 * k + t;
      v[k] = e < r * r ? A[e] : 0.0;
      fro2 += v[k] * v[k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = e0 + 64 * k + t;
      if (e < r * r) {
        // A row-major, or its transpose when trans (A^T[row][c] = A[c][row])
        const int row = trans ? e % r : e / r, c = trans ? e / r : e % r;
        B[c * SVS + row] = v[k];
        V[c * SVS + row] = (row == c) ? 1.0 : 0.0;
      }
    }
  }
  __syncthreads();
  // |A|_F^2; a pair with a column of squared norm below (1e-15 |A|_F)^2 is
  // not rotated.  Such a column ends among the zero singular values (below
  // 1e-14 sigma_1, as sigma_1 >= |A|_F / 8), whose directions the rounding of
  // the other columns' sums keeps turning without end; the other column of
  // the pair would move by less than 1e-15 of its norm.
  fro2 = wave_allsum(fro2);
  const double tiny2 = 1e-30 * fro2;
  // a pair counts as orthogonal once |cos| <= max(1e-15, 4.5e-16 sqrt(r)):
  // the rounding of an r-term column sum of orthogonal columns alone reaches
  // about sqrt(r) 1.1e-16, and a tighter test keeps rotating on it
  const double tol2 = fmax(1e-30, 2e-31 * r);
  const int rr = (r % 2) ? r + 1 : r;
  const int np = rr / 2;
  const int lpp = np <= 8 ? 8 : (np <= 16 ? 4 : 2);
  const int slot = t / lpp, sub = t % lpp;
  // slot's pair in round 0 and the circle-method walk: position k (k >= 1)
  // moves to k + 1 mod (rr - 1) each round, position 0 stays (column rr - 1)
  for (int sw = 0; sw < sweeps; ++sw) {
    int rotated = 0;
    for (int round = 0; round < rr - 1; ++round) {
      int p, q;
      if (slot == 0) {
        p = rr - 1;
        q = round;
      } else {
        p = round + slot;
        if (p >= rr - 1) p -= rr - 1;
        q = round - slot;
        if (q < 0) q += rr - 1;
      }
      if (p > q) {
        const int tmp = p;
        p = q;
        q = tmp;
      }
      const bool live = slot < np && q < r;
      double al = 0, be = 0, ga = 0;
      if (live)
        for (int i = sub; i < r; i += lpp) {
          const double x = B[p * SVS + i], y = B[q * SVS + i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
      al = group_sum(al, lpp);
      be = group_sum(be, lpp);
      ga = group_sum(ga, lpp);
      if (live && al >= tiny2 && be >= tiny2 && fabs(ga) > 1e-300 &&
          ga * ga > tol2 * (al * be)) {
        // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = tau / g2, written
        // without dividing by g2: t = sign(tau) g2 / (|tau| + sqrt(tau^2 + g2^2))
        const double tau = be - al, g2 = 2.0 * ga;
        const double tt = (tau >= 0 ? g2 : -g2) / (fabs(tau) + sqrt(tau * tau + g2 * g2));
        const double c = rsqrt(1.0 + tt * tt), sn = c * tt;
        for (int i = sub; i < r; i += lpp) {
          const double x = B[p * SVS + i], y = B[q * SVS + i];
          B[p * SVS + i] = c * x - sn * y;
          B[q * SVS + i] = sn * x + c * y;
          const double vx = V[p * SVS + i], vy = V[q * SVS + i];
          V[p * SVS + i] = c * vx - sn * vy;
          V[q * SVS + i] = sn * vx + c * vy;
        }
        rotated = 1;
      }
      __syncthreads();
    }
    if (!__any(rotated)) break;
  }
  svd_finish(B, V, nrm, order, r, U, sig, W, complete, t);
}

// Sum over each half (32 lanes) of the wavefront, returned to the lanes of
// that half: row sums as in wave_allsum, then row_bcast:15 adds row 0's sum
// into row 1 and row 2's into row 3, read back from lanes 31 and 63.
__device__ __forceinline__ double half_allsum(double x) {
  x += dpp_move<0xb1>(x);   // quad_perm [1,0,3,2]
  x += dpp_move<0x4e>(x);   // quad_perm [2,3,0,1]
  x += dpp_move<0x124>(x);  // row_ror:4
  x += dpp_move<0x128>(x);  // row_ror:8
  x += dpp_move<0x142>(x);  // row_bcast:15
  const long long b = __double_as_longlong(x);
  const int l0 = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 31);
  const int h0 = __builtin_amdgcn_readlane((int)(b >> 32), 31);
  const int l1 = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int h1 = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  const bool upper = (threadIdx.x & 63) >= 32;
  return __longlong_as_double(((long long)(upper ? h1 : h0) << 32) | (unsigned int)(upper ? l1 : l0));
}

// The same Jacobi SVD for r > 16 on 16 wavefronts: each round's column pairs
// are dealt to groups of GL lanes (a wavefront, GL = 64, or half of one,
// GL = 32; pair slot k to group k mod 1024 / GL), a pair's rows to the lanes
// of its group (64 / GL rows each), its three column sums are group sums;
// the rounds are ordered by workgroup barriers.  The same circle-method
// pairing, rotation and stopping rule as k_svd_jacobi.  With W0 (r x r
// orthogonal, row-major like W) the rotations start from B = A W0, V = W0
// instead of A and the identity: any orthogonal start gives the SVD of A,
// and a start near A's right singular vectors (the previous step's, for a
// matrix that changes little from step to step) leaves few rotations.
template <int GL>
__global__ __launch_bounds__(1024) void k_svd_jacobi_wide(const double* __restrict__ A, int r,
                                                         double* __restrict__ U,
                                                         double* __restrict__ sig,
                                                         double* __restrict__ W, int sweeps,
                                                         int trans, int complete,
                                                         const double* __restrict__ W0) {
  constexpr int NG = 1024 / GL, RPL = 64 / GL;
  __shared__ double B[64 * SVS];  // column c: B[c * SVS + i]
  __shared__ double V[64 * SVS];
  __shared__ double nrm[64];
  __shared__ int order[64];
  __shared__ double part[16];
  const int t = threadIdx.x, wv = t / 64, grp = t / GL, lane = t % GL;
  auto gsum = [](double x) { return GL == 64 ? wave_allsum(x) : half_allsum(x); };
  double fro2 = 0.0;
  for (int e = t; e < r * r; e += blockDim.x) {
    const double v = A[e];
    fro2 += v * v;
    const int row = trans ? e % r : e / r, c = trans ? e / r : e % r;
    B[c * SVS + row] = v;
  }
  for (int e = t; e < r * r; e += blockDim.x) {
    const int row = e / r, c = e % r;
    V[c * SVS + row] = (row == c) ? 1.0 : 0.0;
  }
  fro2 = wave_allsum(fro2);
  if ((t & 63) == 0) part[wv] = fro2;
  __syncthreads();
  fro2 = 0.0;
  for (int k = 0; k < 16; ++k) fro2 += part[k];
  if (W0) {
    // B <- B W0 (through V), then V <- W0
    for (int e = t; e < r * r; e += blockDim.x) {
      const int c = e / r, row = e % r;
      double s = 0.0;
      for (int k = 0; k < r; ++k) s += B[k * SVS + row] * W0[k * r + c];
      V[c * SVS + row] = s;
    }
    __syncthreads();
    for (int e = t; e < r * r; e += blockDim.x) {
      const int c = e / r, row = e % r;
      B[c * SVS + row] = V[c * SVS + row];
      V[c * SVS + row] = W0[row * r + c];
    }
    __syncthreads();
  }
  const double tiny2 = 1e-30 * fro2;  // see k_svd_jacobi
  const double tol2 = fmax(1e-30, 2e-31 * r);
  const int rr = (r % 2) ? r + 1 : r;
  const int np = rr / 2;
  for (int sw = 0; sw < sweeps; ++sw) {
    int rotated = 0;
    for (int round = 0; round < rr - 1; ++round) {
      // every group runs the same number of slots (dead ones with zero
      // columns), so the group sums never see a half-active wavefront
      for (int s0 = 0; s0 < np; s0 += NG) {
        const int slot = s0 + grp;
        int p = 0, q = 0;
        if (slot == 0) {
          p = rr - 1;
          q = round;
        } else {
          p = round + slot;
          if (p >= rr - 1) p -= rr - 1;
          q = round - slot;
          if (q < 0) q += rr - 1;
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        const bool live = slot < np && q < r;  // (q = r: the dummy column of an odd r)
        double x[RPL], y[RPL];
        double sxx = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
          const int i = lane + k * GL;
          x[k] = live && i < r ? B[p * SVS + i] : 0.0;
          y[k] = live && i < r ? B[q * SVS + i] : 0.0;
          sxx += x[k] * x[k];
          syy += y[k] * y[k];
          sxy += x[k] * y[k];
        }
        const double al = gsum(sxx), be = gsum(syy), ga = gsum(sxy);
        if (live && al >= tiny2 && be >= tiny2 && fabs(ga) > 1e-300 && ga * ga > tol2 * (al * be)) {
          const double tau = be - al, g2 = 2.0 * ga;
          const double tt = (tau >= 0 ? g2 : -g2) / (fabs(tau) + sqrt(tau * tau + g2 * g2));
          const double c = rsqrt(1.0 + tt * tt), sn = c * tt;
#pragma unroll
          for (int k = 0; k < RPL; ++k) {
            const int i = lane + k * GL;
            if (i < r) {
              B[p * SVS + i] = c * x[k] - sn * y[k];
              B[q * SVS + i] = sn * x[k] + c * y[k];
              const double vx = V[p * SVS + i], vy = V[q * SVS + i];
              V[p * SVS + i] = c * vx - sn * vy;
              V[q * SVS + i] = sn * vx + c * vy;
            }
          }
          rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
  if (wv == 0) svd_finish(B, V, nrm, order, r, U, sig, W, complete, t);
}

// ------------------------------------------------------- Cholesky QR --
typedef double v4d __attribute__((ext_vector_type(4)));


// Cholesky R^T R = G + shift I of the leading r x r block of G (16 x 16,
// row-major, in LDS; overwritten), on one wavefront, in outer-product form:
// step k subtracts G_ki G_kj / G_kk from the trailing entries (two per lane,
// one wavefront barrier per step); afterwards R_kj = G_kj / sqrt(G_kk) for
// j >= k.  Rows and columns r..15 are completed with the identity.  Writes
// R (r x r row-major, upper; also 16 x 16 to Rl in LDS) and 1 / diag(R).
// flag[0] = 1 when a pivot is not finite or not above pivot_tol times the
// diagonal of G + shift I.
__device__ void chol_wave(double* G, double* Rl, int r, double shift_coef, double pivot_tol,
                          double* __restrict__ Rout, double* __restrict__ dinv_out, int* flag) {
  const int lane = threadIdx.x & 63;
  double tr = 0.0;
  for (int k = 0; k < r; ++k) tr += G[k * 16 + k];
  const double sh = shift_coef * tr;
  wave_sync();
  for (int e = lane; e < 256; e += 64) {
    const int i = e / 16, j = e % 16;
    if (i >= r || j >= r) G[e] = (i == j) ? 1.0 : 0.0;
    else if (i == j) G[e] += sh;
  }
  wave_sync();
  const double dg = lane < 16 ? G[lane * 16 + lane] : 1.0;  // diagonal before elimination
  // lane owns the upper-triangle entries (i, j) = (lane / 16 + 4 m, lane % 16)
  const int cj = lane & 15, i0 = lane >> 4;
  for (int k = 0; k < r; ++k) {
    const double d = G[k * 16 + k];
    const double inv = d != 0.0 ? 1.0 / d : 0.0;
    double upd[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = i0 + 4 * m;
      upd[m] = (i > k && cj >= i) ? G[i * 16 + cj] - G[k * 16 + i] * inv * G[k * 16 + cj] : 0.0;
    }
    wave_sync();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = i0 + 4 * m;
      if (i > k && cj >= i) G[i * 16 + cj] = upd[m];
    }
    wave_sync();
  }
  // G_kk now holds the pivots; R_kj = G_kj / sqrt(G_kk)
  bool bad = false;
  if (lane < 16) {
    const double piv = G[lane * 16 + lane];
    if (lane < r && (!(piv > pivot_tol * dg) || !isfinite(piv))) bad = true;
  }
  double rs[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int i = i0 + 4 * m;
    const double piv = G[i * 16 + i];
    const double q = piv > 0.0 ? rsqrt(piv) : 1.0;
    rs[m] = cj >= i ? G[i * 16 + cj] * q : 0.0;
  }
  wave_sync();
#pragma unroll
  for (int m = 0; m < 4; ++m) Rl[(i0 + 4 * m) * 16 + cj] = rs[m];
  wave_sync();
  if (lane < r) {
    for (int i = 0; i < r; ++i) Rout[i * r + lane] = Rl[i * 16 + lane];
    const double piv = G[lane * 16 + lane];
    dinv_out[lane] = piv > 0.0 ? rsqrt(piv) : 1.0;
  }
  if (__any(bad) && lane == 0) flag[0] = 1;
}

// One pass of the Cholesky QR over the rows of a column-major A (rows x r,
// r <= RM <= 16), tiles of 256 rows: each row a is optionally replaced by
// the solution q of q R_in = scale a (forward substitution with the upper-
// triangular R_in and 1 / diag(R_in); written to Q, which may alias A), and
// with part != null the Gram matrix of the resulting rows is accumulated on
// the FP64 matrix cores.  v_mfma_f64_16x16x4f64 takes a 16x4 and a 4x16
// operand, one double per lane: lane l supplies element (l % 16, l / 16) of
// the first and (l / 16, l % 16) of the second, so the tile entry (row
// 4g + l / 16, column l % 16) is at once the transposed first operand and
// the second, and D += T_g^T T_g; lane l holds D entries (4v + l / 16,
// l % 16).  Each block writes its 16 x 16 sum (waves in order) to part.
template <int RM>
__global__ __launch_bounds__(256) void k_cqr_apply(const double* A, long lda, long rows, int r,
                                                   const double* __restrict__ Rin,
                                                   const double* __restrict__ dinv_in,
                                                   double scale, double* Q, long ldq,
                                                   double* __restrict__ part) {
  __shared__ double tile[256][17];
  __shared__ double rs[16 * 16];
  __shared__ double di[16];
  __shared__ double red[4][256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (Rin) {
    const int ia = t / 16, ib = t % 16;
    rs[t] = (ia < r && ib < r) ? Rin[ia * r + ib] : 0.0;
    if (t < 16) di[t] = t < r ? dinv_in[t] : 0.0;
    __syncthreads();
  }
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (long base = (long)blockIdx.x * 256; base < rows; base += (long)gridDim.x * 256) {
    const long row = base + t;
    double q[RM];
    if (row < rows) {
      double a[RM];
#pragma unroll
      for (int c = 0; c < RM; ++c) a[c] = c < r ? scale * A[c * lda + row] : 0.0;
      if (Rin) {
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
          double v = a[jj];
#pragma unroll
          for (int c = 0; c < jj; ++c) v -= q[c] * rs[c * 16 + jj];
          q[jj] = v * di[jj];
          if (jj < r) Q[jj * ldq + row] = q[jj];
        }
      } else {
#pragma unroll
        for (int c = 0; c < RM; ++c) q[c] = a[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < RM; ++c) q[c] = 0.0;
    }
    if (part) {
#pragma unroll
      for (int c = 0; c < 16; ++c) tile[t][c] = c < RM ? q[c] : 0.0;
      __syncthreads();
#pragma unroll
      for (int gi = 0; gi < 16; ++gi) {
        const double x = tile[64 * wv + 4 * gi + (lane >> 4)][lane & 15];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
      }
      __syncthreads();
    }
  }
  if (!part) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv][(4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc[v];
  __syncthreads();
  part[(long)blockIdx.x * 256 + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// Sum of the nblk partial Gram matrices (block order: thread quarter qd adds
// blocks qd, qd + 4, .., then the quarters in order), times gscale2, then
// chol_wave; with Rp0 != null also Rout = R Rp1 Rp0 (r x r, upper).
__global__ __launch_bounds__(1024) void k_cqr_chol(const double* __restrict__ part, int nblk, int r,
                                                   double gscale2, double shift_coef,
                                                   double pivot_tol, double* __restrict__ Rnew,
                                                   double* __restrict__ dinv_new,
                                                   const double* __restrict__ Rp1,
                                                   const double* __restrict__ Rp0,
                                                   double* __restrict__ Rout, int* flag) {
  __shared__ double q4[4][256];
  __shared__ double G[256];
  __shared__ double P1[256], P0[256], Rl[256];
  const int t = threadIdx.x, e = t & 255, qd = t >> 8;
  double g = 0.0;
  for (int b0 = qd; b0 < nblk; b0 += 64) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int b = b0 + 4 * k;
      v[k] = b < nblk ? part[(long)b * 256 + e] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) g += v[k];
  }
  q4[qd][e] = g;
  if (Rp0 && t < 256) {
    const int i = t / 16, j = t % 16;
    P1[t] = (i < r && j < r) ? Rp1[i * r + j] : 0.0;
    P0[t] = (i < r && j < r) ? Rp0[i * r + j] : 0.0;
  }
  __syncthreads();
  if (t < 256) G[t] = gscale2 * (((q4[0][t] + q4[1][t]) + q4[2][t]) + q4[3][t]);
  __syncthreads();
  if (t < 64) chol_wave(G, Rl, r, shift_coef, pivot_tol, Rnew, dinv_new, flag);
  __syncthreads();
  if (Rp0 && t < r * r) {
    const int i = t / r, j = t % r;
    double v = 0.0;
    for (int k = i; k <= j; ++k) {
      double w = 0.0;
      for (int l = k; l <= j; ++l) w += P1[k * 16 + l] * P0[l * 16 + j];
      v += Rl[i * 16 + k] * w;
    }
    Rout[i * r + j] = v;
  }
}


// The whole shifted Cholesky QR3 of a short matrix (rows <= 256 RPT) in one
// workgroup: thread t keeps rows t + 256 k (k < RPT) of in_scale A in
// registers; each of the three passes forms the Gram matrix on the FP64
// matrix cores (as in k_cqr_apply, one 256-row tile at a time, the four
// waves' sums added in order), factors it with chol_wave (shifted on the
// first pass) and replaces every row a by q with q R = a.  Afterwards
// R = R_2 R_1 R_0 and Q = out_scale q.
template <int RM, int RPT>
__global__ __launch_bounds__(256) void k_cqr_small(const double* A, long lda, long rows, int r,
                                                   double in_scale, double out_scale,
                                                   double shift_coef, double* Q, long ldq,
                                                   double* __restrict__ Rout, int* flag) {
  __shared__ double tile[256][17];
  __shared__ double G[256];
  __shared__ double Rs[3][256];
  __shared__ double di[16];
  __shared__ double red[4][256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double a[RPT][RM];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const long row = t + 256L * k;
#pragma unroll
    for (int c = 0; c < RM; ++c) a[k][c] = (row < rows && c < r) ? in_scale * A[c * lda + row] : 0.0;
  }
  for (int pass = 0; pass < 3; ++pass) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
#pragma unroll
      for (int c = 0; c < 16; ++c) tile[t][c] = c < RM ? a[k][c] : 0.0;
      __syncthreads();
#pragma unroll
      for (int gi = 0; gi < 16; ++gi) {
        const double x = tile[64 * wv + 4 * gi + (lane >> 4)][lane & 15];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wv][(4 * v + (lane >> 4)) * 16 + (lane & 15)] = acc[v];
    if (t < 16) di[t] = 0.0;
    __syncthreads();
    G[t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    __syncthreads();
    if (wv == 0)
      chol_wave(G, Rs[pass], r, pass == 0 ? shift_coef : 0.0, pass == 0 ? 0.0 : 1e-12, nullptr, di,
                flag);
    __syncthreads();
    // q R = a, forward substitution with 1 / diag(R)
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
#pragma unroll
      for (int jj = 0; jj < RM; ++jj) {
        double v = a[k][jj];
#pragma unroll
        for (int c = 0; c < jj; ++c) v -= a[k][c] * Rs[pass][c * 16 + jj];
        a[k][jj] = v * di[jj];
      }
    }
  }
  if (t < r * r) {
    const int i = t / r, j = t % r;
    double v = 0.0;
    for (int k = i; k <= j; ++k) {
      double w = 0.0;
      for (int l = k; l <= j; ++l) w += Rs[1][k * 16 + l] * Rs[0][l * 16 + j];
      v += Rs[2][i * 16 + k] * w;
    }
    Rout[i * r + j] = v;
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const long row = t + 256L * k;
    if (row < rows)
#pragma unroll
      for (int c = 0; c < RM; ++c)
        if (c < r) Q[c * ldq + row] = out_scale * a[k][c];
  }
}
}  // namespace la

// ------------------------------------------------------------------- host --
// column bucket of the QR kernels for rank r
template <class F>
static void qr_bucket(int r, F&& f) {
  if (r <= 4) f(std::integral_constant<int, 4>{});
  else if (r <= 8) f(std::integral_constant<int, 8>{});
  else if (r <= 12) f(std::integral_constant<int, 12>{});
  else if (r <= 16) f(std::integral_constant<int, 16>{});
  else if (r <= 24) f(std::integral_constant<int, 24>{});
  else if (r <= 32) f(std::integral_constant<int, 32>{});
  else f(std::integral_constant<int, 64>{});
}

void tsqr(blr_ctx ctx, const double* A, long lda, long rows, int r, double* Q, long ldq,
          double* R_rowmajor, const std::string& tag, double in_scale, double out_scale) {
  require(r >= 1 && r <= 64, "tsqr: r must be in [1, 64]");
  require(rows >= 1, "tsqr: rows must be >= 1");
  hipStream_t s = ctx->stream;
  struct Level {
    const double* A;
    long lda, rows;
    int nb;
    double *Y, *tau, *Rst;
    long ldy, ldr;
  };
  std::vector<Level> lv;
  const double* cur = A;
  long ld = lda, rws = rows;
  int depth = 0;
  while (true) {
    Level L;
    L.A = cur;
    L.lda = ld;
    L.rows = rws;
    int mbr = 0;
    qr_bucket(r, [&](auto rm) { mbr = la::QRShape<decltype(rm)::value>::MBR; });
    L.nb = (int)((rws + mbr - 1) / mbr);
    L.ldy = (long)L.nb * mbr;
    L.ldr = (long)L.nb * r;
    const std::string t = tag + ".l" + std::to_string(depth);
    L.Y = (double*)ctx->buf(t + ".Y", (size_t)L.ldy * r * sizeof(double));
    L.tau = (double*)ctx->buf(t + ".tau", (size_t)L.nb * r * sizeof(double));
    L.Rst = (double*)ctx->buf(t + ".R", (size_t)L.ldr * r * sizeof(double));
    qr_bucket(r, [&](auto rm) {
      constexpr int RM = decltype(rm)::value;
      hipLaunchKernelGGL(la::k_qr_block<RM>, dim3(L.nb), dim3(la::QT), 0, s, L.A, L.lda, L.rows, r,
                         depth == 0 ? in_scale : 1.0, L.Y, L.ldy, L.tau, L.Rst, L.ldr);
    });
    BLR_CHECK_LAUNCH();
    lv.push_back(L);
    if (L.nb == 1) break;
    cur = L.Rst;
    ld = L.ldr;
    rws = L.ldr;
    ++depth;
    require(depth < 16, "tsqr: too many levels");
  }
  // top: sign fix, seed C = D
  Level& top = lv.back();
  double* C = (double*)ctx->buf(tag + ".C", (size_t)r * r * sizeof(double));
  hipLaunchKernelGGL(la::k_qr_sign, dim3(1), dim3(64), 0, s, top.Rst, top.ldr, r, C, (long)r);
  BLR_CHECK_LAUNCH();
  if (R_rowmajor) {
    hipLaunchKernelGGL(la::k_copy_R, dim3((r * r + 255) / 256), dim3(256), 0, s, top.Rst, top.ldr, r,
                       R_rowmajor);
    BLR_CHECK_LAUNCH();
  }
  if (!Q) return;
  // down the tree
  const double* Cst = C;
  long ldc = r;
  for (int l = (int)lv.size() - 1; l >= 0; --l) {
    Level& L = lv[l];
    double* out;
    long ldo;
    if (l == 0) {
      out = Q;
      ldo = ldq;
    } else {
      out = (double*)ctx->buf(tag + ".q" + std::to_string(l), (size_t)L.rows * r * sizeof(double));
      ldo = L.rows;
    }
    qr_bucket(r, [&](auto rm) {
      constexpr int RM = decltype(rm)::value;
      hipLaunchKernelGGL(la::k_qr_apply<RM>, dim3(L.nb), dim3(la::QT), 0, s, L.Y, L.ldy, L.rows, r, L.tau,
                         Cst, ldc, l == 0 ? out_scale : 1.0, out, ldo);
    });
    BLR_CHECK_LAUNCH();
    Cst = out;
    ldc = ldo;
  }
}

void cholqr(blr_ctx ctx, const double* A, long lda, long rows, int r, double* Q, long ldq,
            double* R_rowmajor, const std::string& tag, double in_scale, double out_scale,
            int* flag) {
  require(r >= 1 && r <= 16, "cholqr: r must be in [1, 16]");
  require(rows >= r, "cholqr: rows must be >= r");
  require(Q && R_rowmajor && flag, "cholqr: null output");
  hipStream_t s = ctx->stream;
  // shift of the first pass: 11 (rows r + r (r + 1)) u ||A||_F^2 (shifted CholeskyQR3)
  const double u53 = std::ldexp(1.0, -53);
  const double shift0 = 11.0 * ((double)rows * r + (double)r * (r + 1)) * u53;
  if (rows <= 1024) {
    // short matrices (up to a 32^2 velocity grid): all three passes in one
    // workgroup
    auto small = [&](auto rm) {
      constexpr int RM = decltype(rm)::value;
      if (rows <= 256)
        hipLaunchKernelGGL((la::k_cqr_small<RM, 1>), dim3(1), dim3(256), 0, s, A, lda, rows, r,
                           in_scale, out_scale, shift0, Q, ldq, R_rowmajor, flag);
      else if (rows <= 512)
        hipLaunchKernelGGL((la::k_cqr_small<RM, 2>), dim3(1), dim3(256), 0, s, A, lda, rows, r,
                           in_scale, out_scale, shift0, Q, ldq, R_rowmajor, flag);
      else
        hipLaunchKernelGGL((la::k_cqr_small<RM, 4>), dim3(1), dim3(256), 0, s, A, lda, rows, r,
                           in_scale, out_scale, shift0, Q, ldq, R_rowmajor, flag);
      BLR_CHECK_LAUNCH();
    };
    if (r <= 4) small(std::integral_constant<int, 4>{});
    else if (r <= 8) small(std::integral_constant<int, 8>{});
    else if (r <= 12) small(std::integral_constant<int, 12>{});
    else small(std::integral_constant<int, 16>{});
    return;
  }
  const int nblk = (int)std::max<long>(1, std::min<long>(128, (rows + 255) / 256));
  double* part = (double*)ctx->buf(tag + ".part", (size_t)nblk * 256 * sizeof(double));
  double* Rk = (double*)ctx->buf(tag + ".rk", (size_t)3 * r * r * sizeof(double));
  double* Dk = (double*)ctx->buf(tag + ".dk", (size_t)3 * 16 * sizeof(double));
  // shift of the first pass: 11 (rows r + r (r + 1)) u ||A||_F^2 (shifted CholeskyQR3)
  const double u = std::ldexp(1.0, -53);
  const double shift = 11.0 * ((double)rows * r + (double)r * (r + 1)) * u;
  auto R = [&](int k) { return Rk + (size_t)k * r * r; };
  auto D = [&](int k) { return Dk + (size_t)k * 16; };
  auto pass = [&](auto rm, int k) {
    constexpr int RM = decltype(rm)::value;
    // k = 0: Gram of in_scale A -> R_0; k = 1, 2: solve with R_{k-1}, Gram -> R_k
    // (k = 2 also forms R = R_2 R_1 R_0); k = 3: solve with R_2, times out_scale
    const double* src = k <= 1 ? A : Q;
    const long ld = k <= 1 ? lda : ldq;
    const double sc = k == 0 ? 1.0 : ((k == 1 ? in_scale : 1.0) * (k == 3 ? out_scale : 1.0));
    hipLaunchKernelGGL(la::k_cqr_apply<RM>, dim3(nblk), dim3(256), 0, s, src, ld, rows, r,
                       k == 0 ? nullptr : R(k - 1), k == 0 ? nullptr : D(k - 1), sc, Q, ldq,
                       k < 3 ? part : nullptr);
    BLR_CHECK_LAUNCH();
    if (k == 3) return;
    hipLaunchKernelGGL(la::k_cqr_chol, dim3(1), dim3(1024), 0, s, part, nblk, r,
                       k == 0 ? in_scale * in_scale : 1.0, k == 0 ? shift : 0.0, k == 0 ? 0.0 : 1e-12,
                       R(k), D(k), k == 2 ? R(1) : nullptr, k == 2 ? R(0) : nullptr,
                       k == 2 ? R_rowmajor : nullptr, flag);
    BLR_CHECK_LAUNCH();
  };
  for (int k = 0; k < 4; ++k) {
    if (r <= 4) pass(std::integral_constant<int, 4>{}, k);
    else if (r <= 8) pass(std::integral_constant<int, 8>{}, k);
    else if (r <= 12) pass(std::integral_constant<int, 12>{}, k);
    else pass(std::integral_constant<int, 16>{}, k);
  }
}

void svd_small(blr_ctx ctx, const double* A, int r, double* U, double* sig, double* W, bool trans,
               bool complete, const double* W0) {
  require(r >= 1 && r <= 64, "svd: r must be in [1, 64]");
  if (r <= 16)
    hipLaunchKernelGGL(la::k_svd_jacobi, dim3(1), dim3(64), 0, ctx->stream, A, r, U, sig, W, 40,
                       trans ? 1 : 0, complete ? 1 : 0);
  else if (r <= 32)
    hipLaunchKernelGGL(la::k_svd_jacobi_wide<64>, dim3(1), dim3(1024), 0, ctx->stream, A, r, U, sig,
                       W, 40, trans ? 1 : 0, complete ? 1 : 0, W0);
  else
    hipLaunchKernelGGL(la::k_svd_jacobi_wide<32>, dim3(1), dim3(1024), 0, ctx->stream, A, r, U, sig,
                       W, 40, trans ? 1 : 0, complete ? 1 : 0, W0);
  BLR_CHECK_LAUNCH();
}

}  // namespace blr
