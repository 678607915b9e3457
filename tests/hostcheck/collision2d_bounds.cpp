// Bounds check, on the CPU, of the generic collision pipeline on 2D velocity
// grids of 48 and 64 points per axis (the (rho, sigma) quadrature form and the
// Carleman form, FP64 and FP32, r = 3 and all six pairs).  Every GPU thread of
// every launch runs here in a loop, through the same per-thread bodies the
// kernels use (line passes with their loaders and storers, sigma reduce,
// Carleman final), on buffers allocated with exactly the element counts the
// library requests (its workspace slices, tables, inputs and outputs).  The
// moment projection's block and chunk indexing is restated here.  Built with
// AddressSanitizer on the host: an access outside any buffer aborts.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "collision_passes.hpp"

using namespace blr;

template <typename X>
static X* exact(size_t count, const char* what) {
  X* p = (X*)malloc(count * sizeof(X));
  if (!p) { fprintf(stderr, "malloc %s\n", what); exit(1); }
  memset(p, 0, count * sizeof(X));
  return p;
}

static long g_threads = 0;

template <typename T, int N, int D, int DIR, class Ld, class St>
static void line_pass(const Ld& ld, const St& st, int axis, long nfields) {
  constexpr int lines = (D == 2 ? N : N * N);
  const long nl = nfields * lines;
  const int bs = 128;
  const long nb = (nl + bs - 1) / bs;
  for (long b = 0; b < nb; ++b)
    for (int tx = 0; tx < bs; ++tx) {
      const long t = b * bs + tx;
      if (t >= nl) continue;
      line_pass_thread<T, N, D, DIR>(t, ld, st, axis);
      ++g_threads;
    }
}

template <typename T, int N, int D, int DIR, class Ld, class St>
static void transform(const Ld& ld, const St& st, typename Vec2<T>::t* tmp, long nfields) {
  constexpr int n = (D == 2 ? N * N : N * N * N);
  StComplex<T> stc{tmp, n};
  LdComplex<T> ldc{tmp, n};
  line_pass<T, N, D, DIR>(ld, stc, D - 1, nfields);
  if constexpr (D == 3) line_pass<T, N, D, DIR>(ldc, stc, 1, nfields);
  line_pass<T, N, D, DIR>(ldc, st, 0, nfields);
}

template <typename T>
static std::vector<T> cast(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

template <typename T>
static void conserve_rows(const HostTables& h, T* Q, int rows) {
  const int n = h.n;
  const int nb = (n + kMomChunk - 1) / kMomChunk;
  double* part = exact<double>((size_t)rows * nb * 5, "mom.part");
  for (int row = 0; row < rows; ++row)
    for (int b = 0; b < nb; ++b) {
      const T* q = Q + (long)row * n;
      const int e0 = b * kMomChunk, e1 = std::min(n, e0 + kMomChunk);
      double acc = 0;
      for (int tx = 0; tx < 256; ++tx)
        for (int e = e0 + tx; e < e1; e += 256) acc += (double)q[e];
      for (int i = 0; i < 5; ++i) part[((long)row * nb + b) * 5 + i] = acc;
    }
  for (int row = 0; row < rows; ++row)
    for (int b = 0; b < nb; ++b) {
      double mo = 0;
      for (int k = 0; k < nb; ++k)
        for (int i = 0; i < 5; ++i) mo += part[((long)row * nb + k) * 5 + i];
      T* q = Q + (long)row * n;
      const int e0 = b * kMomChunk, e1 = std::min(n, e0 + kMomChunk);
      for (int tx = 0; tx < 256; ++tx)
        for (int e = e0 + tx; e < e1; e += 256) q[e] = (T)((double)q[e] - 0.0 * mo);
    }
  free(part);
}

template <typename T, int N, int D>
static void run_case(const blr_vgrid& vg, int r, bool conserve) {
  using T2 = typename Vec2<T>::t;
  constexpr int n = D == 2 ? N * N : N * N * N;
  HostTables h = build_tables(vg);
  // pairs (i, j), i <= j: the upper triangle
  std::vector<int> li, lj;
  for (int i = 0; i < r; ++i)
    for (int j = i; j < r; ++j) { li.push_back(i); lj.push_back(j); }
  const int P = (int)li.size(), rb = r, npairs = P;
  std::vector<int> prow(P);
  for (int p = 0; p < P; ++p) prow[p] = p;
  // tables, as uploaded
  std::vector<double> wbp_d(h.nbp);
  for (int p = 0; p < h.nbp; ++p) wbp_d[p] = h.wsig[h.bp_b[p]];
  auto up = [](const std::vector<T>& v, const char* w) {
    T* p = exact<T>(std::max<size_t>(v.size(), 1), w);
    std::copy(v.begin(), v.end(), p);
    return p;
  };
  T* phase = up(cast<T>(h.phase), "phase");
  T* fw = up(cast<T>(h.fw), "fw");
  T* gloss = up(cast<T>(h.gloss), "gloss");
  T* wbp = up(cast<T>(wbp_d), "wbp");
  T* filt = h.carleman ? up(cast<T>(h.filt), "filt") : nullptr;
  int* bp_b = exact<int>(h.nbp, "bp_b");
  int* bp_bb = exact<int>(h.nbp, "bp_bb");
  std::copy(h.bp_b.begin(), h.bp_b.end(), bp_b);
  std::copy(h.bp_bb.begin(), h.bp_bb.end(), bp_bb);
  printf("  tables: n=%d nbp=%d msig=%d mrho=%d nkk=%d phase=%zu fw=%zu filt=%zu\n", h.n, h.nbp,
         h.msig, h.mrho, h.nkk, h.phase.size(), h.fw.size(), h.filt.size());
  // inputs and output
  T* V = exact<T>((size_t)r * n, "V");
  for (long i = 0; i < (long)r * n; ++i) V[i] = T(std::exp(-0.001 * (i % n)));
  T* Q = exact<T>((size_t)npairs * n, "Q");
  // Generic::run buffers
  const long nc = P;
  const long shift_fields = (long)rb * h.mrho * h.nbp;
  const long batch = std::min<long>(shift_fields, 512);
  T* Sh = exact<T>((size_t)rb * h.mrho * h.msig * n, "Sh");
  // the isotropic form keeps the products of a chunk of radial nodes
  const long cr = h.carleman ? 1 : radial_chunk(h.mrho, nc, n, sizeof(T));
  T2* tmp = exact<T2>((size_t)std::max<long>(batch, std::max<long>(cr * nc, 2 * rb)) * n, "tmp");
  T* Pa = exact<T>((size_t)cr * P * n, "Pa");
  T2* G = h.carleman ? nullptr : exact<T2>((size_t)nc * n, "G");
  int* didx = exact<int>(3 * P, "idx");
  for (int p = 0; p < P; ++p) { didx[p] = li[p]; didx[P + p] = lj[p]; didx[2 * P + p] = prow[p]; }
  // basis
  T2* Vh = exact<T2>((size_t)rb * n, "bas.Vh");
  T* Vp = exact<T>((size_t)2 * rb * n, "bas.VpLam");
  T2* btmp = exact<T2>((size_t)2 * rb * n, "bas.tmp");
  transform<T, N, D, -1>(LdReal<T>{V, n}, StBasisSpec<T, N, D>{Vh, n, T(1) / T(n)}, btmp, rb);
  transform<T, N, D, +1>(LdBasisMode<T>{Vh, gloss, n, rb}, StRe<T>{Vp, n}, btmp, 2 * rb);
  T* Lam = Vp + (size_t)rb * n;
  bool diag_only = false;
  // the Carleman form's tiles; the isotropic form's (12 wide in FP64 too up
  // to 12 basis functions) below
  const int Gt = sizeof(T) == 4 ? 12 : 8;
  auto tiles = plan_tiles(rb, li, lj, Gt, diag_only);
  const int Gi = (sizeof(T) == 4 || rb <= 12) ? 12 : 8;
  auto tiles_iso = plan_tiles(rb, li, lj, Gi, diag_only);
  // node a's products at Pa + k P n (k = a - a0, grid.y of the launch)
  auto reduce = [&](const ReduceTile& t, const T* w, const int* b1, const int* b2, int nbp, int a,
                    int k) {
    const bool diag = t.bi[0] == t.bj[0];
    T* pk = Pa + (size_t)k * P * n;
    for (int q = 0; q < n; ++q) {
      if (Gi == 12) {
        if (diag) sigma_reduce_point<T, 12, true>(q, Sh, pk, t, w, b1, b2, n, h.mrho, h.msig, nbp, a);
        else sigma_reduce_point<T, 12, false>(q, Sh, pk, t, w, b1, b2, n, h.mrho, h.msig, nbp, a);
      } else {
        if (diag) sigma_reduce_point<T, 8, true>(q, Sh, pk, t, w, b1, b2, n, h.mrho, h.msig, nbp, a);
        else sigma_reduce_point<T, 8, false>(q, Sh, pk, t, w, b1, b2, n, h.mrho, h.msig, nbp, a);
      }
    }
  };
  if (h.carleman) {
    const long nfields = (long)rb * h.nbp;
    const long cb = std::min<long>(nfields, 512);
    for (long f0 = 0; f0 < nfields; f0 += cb) {
      const long nb = std::min(cb, nfields - f0);
      transform<T, N, D, +1>(LdFilter<T>{Vh, (const T2*)filt, n, h.nbp, f0},
                             StShiftSplit<T>{Sh, bp_b, bp_bb, n, 1, h.nbp, h.msig, f0}, tmp, nb);
    }
    // the Carleman reduce launch uses mrho = 1
    for (const auto& t : tiles) {
      const bool diag = t.bi[0] == t.bj[0];
      for (int q = 0; q < n; ++q) {
        if (diag) sigma_reduce_point<T, sizeof(T) == 4 ? 12 : 8, true>(q, Sh, Pa, t, wbp, bp_b, bp_bb, n, 1, h.msig, h.nbp, 0);
        else sigma_reduce_point<T, sizeof(T) == 4 ? 12 : 8, false>(q, Sh, Pa, t, wbp, bp_b, bp_bb, n, 1, h.msig, h.nbp, 0);
      }
    }
    for (int p = 0; p < P; ++p)
      for (int e = 0; e < n; ++e)
        carleman_final_point<T>(e, p, Pa, Vp, Lam, didx, didx + P, didx + 2 * P, n, Q);
  } else {
    for (long f0 = 0; f0 < shift_fields; f0 += batch) {
      const long nb = std::min(batch, shift_fields - f0);
      transform<T, N, D, +1>(LdShift<T, N, D>{Vh, (const T2*)phase, n, h.mrho, h.nbp, f0},
                             StShiftSplit<T>{Sh, bp_b, bp_bb, n, h.mrho, h.nbp, h.msig, f0}, tmp, nb);
    }
    for (long i = 0; i < 2 * nc * n; ++i) ((T*)G)[i] = T(0);
    for (int a0 = 0; a0 < h.mrho; a0 += (int)cr) {
      const int na = std::min((int)cr, h.mrho - a0);
      for (int k = 0; k < na; ++k)
        for (const auto& t : tiles_iso) reduce(t, wbp, bp_b, bp_bb, h.nbp, a0 + k, k);
      // first axes of the chunk's pair transforms, then the last axis with
      // the radial weights
      line_pass<T, N, D, -1>(LdPair1<T>{Pa, n}, StComplex<T>{tmp, n}, D - 1, (long)na * nc);
      constexpr int lines = (D == 2 ? N : N * N);
      for (long t = 0; t < nc * lines; ++t) {
        accum_radial_thread<T, N, D>(t, tmp, G, fw, h.nkk, nc, a0, na);
        ++g_threads;
      }
    }
    transform<T, N, D, +1>(LdComplex<T>{G, n}, StFinal<T>{Q, Vp, Lam, didx, didx + P, didx + 2 * P, n},
                           tmp, nc);
  }
  if (conserve) conserve_rows<T>(h, Q, npairs);
  double s = 0;
  for (long i = 0; i < (long)npairs * n; ++i) s += std::fabs((double)Q[i]);
  printf("  ok: sum|Q| = %.6e, threads %ld, finite %d\n", s, g_threads, (int)std::isfinite(s));
  free(phase); free(fw); free(gloss); free(wbp); free(filt); free(bp_b); free(bp_bb);
  free(V); free(Q); free(Sh); free(tmp); free(Pa); free(G); free(didx); free(Vh); free(Vp); free(btmp);
}

int main() {
  for (int carl = 1; carl >= 0; --carl)
    for (int N : {48, 64})
      for (int M : {8, 16})
      for (int prec = 0; prec < 2; ++prec) {
        blr_vgrid vg{};
        vg.d = 2;
        vg.n = N;
        vg.L = 8.0;
        vg.R = 0;
        vg.C = 1.0;
        vg.gamma = 0.0;
        vg.m_rho = carl ? 1 : 8;
        vg.m_sigma = M;
        vg.flags = carl ? BLR_CARLEMAN : 0;
        const int r = 3;
        printf("case carleman=%d N=%d %s M=%d r=%d\n", carl, N, prec ? "fp32" : "fp64", vg.m_sigma, r);
        fflush(stdout);
        if (N == 64) {
          if (prec) run_case<float, 64, 2>(vg, r, true);
          else run_case<double, 64, 2>(vg, r, true);
        } else {
          if (prec) run_case<float, 48, 2>(vg, r, true);
          else run_case<double, 48, 2>(vg, r, true);
        }
      }
  printf("all cases done\n");
  return 0;
}
