/* Direct spectral sum of the discrete collision operator (oracle, C).
 *
 * TEST INFRASTRUCTURE ONLY.  Same sum as oracle/collision.py:qhat_direct,
 * the O(N^{2d}) definition of the Fourier-Galerkin operator
 *
 *   Q^_k  = sum_l [ G+(l, m) - G-(l) ] g^_l f^_m ,      m = wrap(k - l),
 *   Q^+_k = sum_l   G+(l, m)           g^_l f^_m ,
 *   G+(l, m) = sum_a FtW[a][k] * E[a][l - m]
 *
 * where FtW[a][k] = w_a rho_a^{d-1} F(k, rho_a) (real) and E[a][delta] is the sigma
 * sum (real for an antipodally symmetric rule).  All tables are built by the
 * Python oracle and passed in; this file only loops.  Complex arrays are
 * interleaved (re, im) doubles, all indices in DFT order.
 */
#include <stdint.h>
#include <stdlib.h>

static inline int centred(int k, int N) { return k >= N / 2 ? k - N : k; }
static inline int wrapc(int k, int N) {  /* wrap an integer into [-N/2, N/2) */
  int m = ((k + N / 2) % N + N) % N;
  return m - N / 2;
}

int oracle_qhat_direct(int d, int N, int mrho, const double* g, const double* f,
                       const double* FtW, const double* E, const double* Gm,
                       const int64_t* ks, long nk, double* out, double* outp) {
  if (d != 2 && d != 3) return 1;
  const long n = (d == 2) ? (long)N * N : (long)N * N * N;
  const int E1 = 2 * N - 1;
  const long nE = (d == 2) ? (long)E1 * E1 : (long)E1 * E1 * E1;
  int* lc = (int*)malloc(sizeof(int) * 3 * n);
  if (!lc) return 2;
  for (long l = 0; l < n; ++l) {
    long t = l;
    int c[3] = {0, 0, 0};
    for (int ax = d - 1; ax >= 0; --ax) { c[ax] = centred((int)(t % N), N); t /= N; }
    lc[3 * l] = c[0]; lc[3 * l + 1] = c[1]; lc[3 * l + 2] = c[2];
  }
  (void)nE;
#pragma omp parallel for schedule(dynamic, 4)
  for (long t = 0; t < nk; ++t) {
    const long kidx = ks[t];
    const int* kc = lc + 3 * kidx;
    double* H = (double*)calloc((size_t)mrho, sizeof(double) * 2);
    double lr = 0.0, li = 0.0;
    for (long l = 0; l < n; ++l) {
      const int* l3 = lc + 3 * l;
      int m3[3] = {0, 0, 0};
      long midx = 0, eidx = 0;
      for (int ax = 0; ax < d; ++ax) {
        m3[ax] = wrapc(kc[ax] - l3[ax], N);
        midx = midx * N + ((m3[ax] % N) + N) % N;
        eidx = eidx * E1 + (l3[ax] - m3[ax] + N - 1);
      }
      const double gr = g[2 * l], gi = g[2 * l + 1];
      const double fr = f[2 * midx], fi = f[2 * midx + 1];
      const double pr = gr * fr - gi * fi, pi = gr * fi + gi * fr;
      for (int a = 0; a < mrho; ++a) {
        const double e = E[(long)a * nE + eidx];
        H[2 * a] += e * pr;
        H[2 * a + 1] += e * pi;
      }
      lr += Gm[l] * pr;
      li += Gm[l] * pi;
    }
    double qr = 0.0, qi = 0.0;
    for (int a = 0; a < mrho; ++a) {
      const double w = FtW[(long)a * n + kidx];
      qr += w * H[2 * a];
      qi += w * H[2 * a + 1];
    }
    outp[2 * t] = qr; outp[2 * t + 1] = qi;
    out[2 * t] = qr - lr; out[2 * t + 1] = qi - li;
    free(H);
  }
  free(lc);
  return 0;
}
