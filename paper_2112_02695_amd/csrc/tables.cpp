// Host precomputation (FP64) of the quadrature rules and spectral weight
// tables of the Fourier collision solver.
//
// With q = v - v*, rho = |q| and theta_a = pi rho_a / (2L) the gain part of
// the operator is a sum over radial nodes a and sphere nodes b of
//   g(v - rho_a sigma_b / 2) f(v + rho_a sigma_b / 2),
// followed in Fourier space by the weight w_a rho_a^(d-1) B(rho_a) A_d(theta_a |k|),
// where A_d is the exact integral over the direction of q (2 pi J0 in 2D,
// 4 pi sin z / z in 3D).  The loss uses the same sigma rule:
//   G-(k) = |S^(d-1)| sum_a w_a rho_a^(d-1) B(rho_a) sum_b w_b cos(2 theta_a sigma_b . k).
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace blr {

static const double kPi = 3.14159265358979323846;

void gauss_legendre(int m, double R, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration on the Legendre polynomial P_m (three-term recurrence).
  x.assign(m, 0.0);
  w.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (m + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= m; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (m == 1) { p1 = z; p0 = 1.0; }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= m; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (m == 1) { p1 = z; p0 = 1.0; }
    dp = m * (z * p1 - p0) / (z * z - 1.0);
    // node on [-1,1] -> [0,R]
    x[m - 1 - i] = 0.5 * R * (z + 1.0);
    w[m - 1 - i] = 0.5 * R * 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// J0(z) = (1/2pi) int_0^2pi cos(z sin t) dt; the trapezoid rule on the periodic
// integrand converges geometrically once the point count exceeds z.
double bessel_j0(double z) {
  const int M = 64 + 2 * (int)std::ceil(std::fabs(z));
  double s = 0.0;
  for (int j = 0; j < M; ++j) s += std::cos(z * std::sin(2.0 * kPi * j / M));
  return s / M;
}

// J1(z) = (1/2pi) int_0^2pi cos(t - z sin t) dt, same rule as bessel_j0.
static double bessel_j1(double z) {
  const int M = 64 + 2 * (int)std::ceil(std::fabs(z));
  double s = 0.0;
  for (int j = 0; j < M; ++j) {
    const double t = 2.0 * kPi * j / M;
    s += std::cos(t - z * std::sin(t));
  }
  return s / M;
}

// J_n(z) = (1/2pi) int_0^2pi cos(n t - z sin t) dt (trapezoid rule, as above).
static double bessel_jn(int n, double z) {
  const int M = 64 + 2 * (int)std::ceil(std::fabs(z)) + 2 * n;
  double s = 0.0;
  for (int j = 0; j < M; ++j) {
    const double t = 2.0 * kPi * j / M;
    s += std::cos(n * t - z * std::sin(t));
  }
  return s / M;
}

static double legendre_p(int n, double x) {
  double p0 = 1.0, p1 = x;
  if (n == 0) return 1.0;
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Spherical Bessel j_n(z) for even n: ((-1)^(n/2) / 2) int_-1^1 cos(z t) P_n(t) dt,
// by Gauss-Legendre quadrature with more nodes than z (the integrand is
// entire; the rule's error falls faster than geometrically past that).
static double sph_bessel_even(int n, double z) {
  const int M = 48 + (int)std::ceil(std::fabs(z)) + n;
  std::vector<double> x, w;
  gauss_legendre(M, 2.0, x, w);  // nodes on [0, 2] -> t = x - 1
  double s = 0.0;
  for (int i = 0; i < M; ++i) {
    const double t = x[i] - 1.0;
    s += w[i] * std::cos(z * t) * legendre_p(n, t);
  }
  return ((n / 2) % 2 ? -0.5 : 0.5) * s;
}

static void sphere_rule(int d, int msig, std::vector<double>& sig, std::vector<double>& w) {
  sig.clear();
  w.clear();
  if (d == 2) {
    for (int b = 0; b < msig; ++b) {
      const double t = 2.0 * kPi * b / msig;
      sig.push_back(std::cos(t));
      sig.push_back(std::sin(t));
      sig.push_back(0.0);
      w.push_back(2.0 * kPi / msig);
    }
    return;
  }
  // 38-point Lebedev rule: 6 vertices (1/105), 8 cube corners (9/280),
  // 24 points (+-p, +-q, 0) in every placement (1/35); scaled to 4 pi.
  auto add = [&](double a, double b, double c, double wt) {
    sig.push_back(a);
    sig.push_back(b);
    sig.push_back(c);
    w.push_back(4.0 * kPi * wt);
  };
  for (int ax = 0; ax < 3; ++ax)
    for (double s : {1.0, -1.0}) {
      double e[3] = {0, 0, 0};
      e[ax] = s;
      add(e[0], e[1], e[2], 1.0 / 105.0);
    }
  const double c = 1.0 / std::sqrt(3.0);
  for (double sx : {1.0, -1.0})
    for (double sy : {1.0, -1.0})
      for (double sz : {1.0, -1.0}) add(sx * c, sy * c, sz * c, 9.0 / 280.0);
  const double p = 0.4597008433809831, q = std::sqrt(1.0 - p * p);
  for (int z = 0; z < 3; ++z) {
    int o0 = (z == 0) ? 1 : 0, o1 = (z == 2) ? 1 : 2;
    for (int sw = 0; sw < 2; ++sw) {
      const double u = sw ? q : p, v = sw ? p : q;
      for (double su : {1.0, -1.0})
        for (double sv : {1.0, -1.0}) {
          double e[3] = {0, 0, 0};
          e[o0] = su * u;
          e[o1] = sv * v;
          add(e[0], e[1], e[2], 1.0 / 35.0);
        }
    }
  }
}

void validate_vgrid(const blr_vgrid& vg) {
  require(vg.d == 2 || vg.d == 3, "vgrid.d must be 2 or 3");
  if (vg.d == 3)
    require(vg.n == 8 || vg.n == 16 || vg.n == 24 || vg.n == 32,
            "3D vgrid.n must be 8, 16, 24 or 32", BLR_ERR_UNSUPPORTED);
  else
    // 48 and 64 are off: a run of the 2D 64-point FP64 line passes (256 VGPRs
    // plus AGPR spills) faulted the GPU without a cause found in the code
    require(vg.n == 16 || vg.n == 32, "2D vgrid.n must be 16 or 32", BLR_ERR_UNSUPPORTED);
  require(vg.L > 0 && std::isfinite(vg.L), "vgrid.L must be positive");
  require(std::isfinite(vg.C) && std::isfinite(vg.gamma), "vgrid.C/gamma must be finite");
  require(vg.m_rho >= 1 && vg.m_rho <= 64, "vgrid.m_rho must be in [1, 64]");
  const int ms = vg.m_sigma ? vg.m_sigma : (vg.d == 2 ? 8 : 38);
  if (vg.d == 3)
    require(ms == 38, "3D vgrid.m_sigma must be 38 (Lebedev rule)", BLR_ERR_UNSUPPORTED);
  else
    require(ms >= 2 && ms <= 64 && ms % 2 == 0, "2D vgrid.m_sigma must be even in [2, 64]");
  if (vg.flags & BLR_CARLEMAN)
    require(std::fabs(vg.gamma - (vg.d - 2)) < 1e-12,
            "the Carleman form needs gamma = d - 2 (2D Maxwell molecules, 3D hard spheres)");
  require(vg.aniso_n >= 0 && vg.aniso_n <= 5, "vgrid.aniso_n must be in [0, 5]");
  if (vg.aniso_n > 0) {
    require(!(vg.flags & BLR_CARLEMAN), "an anisotropic kernel is not available in the Carleman form");
    for (int i = 0; i < vg.aniso_n; ++i) require(std::isfinite(vg.aniso[i]), "vgrid.aniso must be finite");
  }
}

// (C C^T)^-1 for the moment projection; C rows dv^d {1, v_1..v_d, |v|^2}
static std::vector<double> moment_inverse(const HostTables& t) {
  const int d = t.d, N = t.N, m = d + 2;
  std::vector<double> G(m * m, 0.0);
  const double w = std::pow(t.dv, d);
  for (int q = 0; q < t.n; ++q) {
    double v[3] = {0, 0, 0};
    int rem = q;
    for (int ax = d - 1; ax >= 0; --ax) {
      v[ax] = -t.L + (rem % N) * t.dv;
      rem /= N;
    }
    double phi[5];
    phi[0] = w;
    double v2 = 0;
    for (int ax = 0; ax < d; ++ax) {
      phi[1 + ax] = w * v[ax];
      v2 += v[ax] * v[ax];
    }
    phi[d + 1] = w * v2;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) G[i * m + j] += phi[i] * phi[j];
  }
  // Gauss-Jordan inverse (SPD, small)
  std::vector<double> A(G), I(m * m, 0.0);
  for (int i = 0; i < m; ++i) I[i * m + i] = 1.0;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(A[r * m + c]) > std::fabs(A[piv * m + c])) piv = r;
    for (int j = 0; j < m; ++j) {
      std::swap(A[c * m + j], A[piv * m + j]);
      std::swap(I[c * m + j], I[piv * m + j]);
    }
    const double dgn = A[c * m + c];
    require(std::fabs(dgn) > 0, "singular moment matrix", BLR_ERR_NUMERIC);
    for (int j = 0; j < m; ++j) {
      A[c * m + j] /= dgn;
      I[c * m + j] /= dgn;
    }
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double f = A[r * m + c];
      for (int j = 0; j < m; ++j) {
        A[r * m + j] -= f * A[c * m + j];
        I[r * m + j] -= f * I[c * m + j];
      }
    }
  }
  return I;
}

// Carleman form.  With v' = v + x, v*' = v + y (x orthogonal to y) the kernel
// is the constant b0 = 2^(d-1) C; x = rho e (e on a half sphere, rho in
// [-R, R]) and y in the disc of radius R orthogonal to e give
//   beta(l, m) = b0 int de phi(m.e) psi(l, e),
//   phi(s) = int_{-R}^{R} |rho|^(d-2) exp(i pi rho s / L) d rho,
//   psi    = the same integral over the disc (2D: a segment, phi(l.e_perp)).
// Directions: 2D t_p = p pi / M (weights pi / M), 3D one point per antipodal
// pair of the Lebedev rule with its full-sphere weight.  Each pair of fields
// (f1 -> S(b), f2 -> S(bbar)) is produced by one complex inverse transform of
// V^ ((f1 + f2)/2 + i (f2 - f1)/2); the sigma reduction then yields
//   sum_pairs w (S_i(b) S_j(bbar) + S_i(bbar) S_j(b)) = Q_s+(V_i, V_j).
//   2D: pair p < M/2 is (phi(k.e_p), phi(k.e_{p+M/2})), w = b0 pi / M;
//   3D: pair p is (psi(k, e_p), phi(k.e_p)), w = b0 w_p / 2.
static void carleman_tables(HostTables& t) {
  const int N = t.N, d = t.d, n = t.n;
  const double R = t.R, L = t.L, b0 = std::pow(2.0, d - 1) * t.C;
  auto centred = [N](int k) { return k >= N / 2 ? k - N : k; };
  auto phi = [&](double s) {
    const double a = kPi * s / L;
    if (std::fabs(a) < 1e-12) return d == 2 ? 2.0 * R : R * R;
    if (d == 2) return 2.0 * std::sin(a * R) / a;
    const double h = std::sin(0.5 * a * R);
    return 2.0 * (R * std::sin(a * R) / a - 2.0 * h * h / (a * a));
  };
  auto psi3 = [&](double kperp) {
    const double b = kPi * kperp / L;
    if (b < 1e-12) return kPi * R * R;
    return 2.0 * kPi * R * bessel_j1(b * R) / b;
  };
  std::vector<double> dirs, wdir;  // (nd, 3), nd
  if (d == 2) {
    const int M = t.msig;
    for (int p = 0; p < M; ++p) {
      const double th = kPi * p / M;
      dirs.insert(dirs.end(), {std::cos(th), std::sin(th), 0.0});
      wdir.push_back(kPi / M);
    }
  } else {
    std::vector<double> sig, w;
    sphere_rule(3, 38, sig, w);
    std::vector<int> used(38, 0);
    for (int b = 0; b < 38; ++b) {
      if (used[b]) continue;
      for (int c = 0; c < 38; ++c) {
        const double e = std::fabs(sig[3 * b] + sig[3 * c]) + std::fabs(sig[3 * b + 1] + sig[3 * c + 1]) +
                         std::fabs(sig[3 * b + 2] + sig[3 * c + 2]);
        if (e < 1e-12) {
          used[b] = used[c] = 1;
          break;
        }
      }
      dirs.insert(dirs.end(), {sig[3 * b], sig[3 * b + 1], sig[3 * b + 2]});
      wdir.push_back(w[b]);
    }
  }
  const int nd = (int)wdir.size();
  t.nbp = d == 2 ? nd / 2 : nd;
  t.msig = 2 * t.nbp;
  t.mrho = 1;
  t.rho.assign(1, 0.0);
  t.wrho.assign(1, 1.0);
  t.cw.assign(1, 1.0);
  t.sig.assign((size_t)3 * t.msig, 0.0);
  t.wsig.assign(t.msig, 0.0);
  t.bp_b.clear();
  t.bp_bb.clear();
  for (int p = 0; p < t.nbp; ++p) {
    t.bp_b.push_back(2 * p);
    t.bp_bb.push_back(2 * p + 1);
    const double w = d == 2 ? b0 * wdir[p] : 0.5 * b0 * wdir[p];
    t.wsig[2 * p] = t.wsig[2 * p + 1] = w;
  }
  t.phase.clear();
  t.fw.clear();
  t.nkk = 1;
  t.filt.assign((size_t)t.nbp * n * 2, 0.0);
  t.gloss.assign(n, 0.0);
  for (int q = 0; q < n; ++q) {
    double kc[3] = {0, 0, 0};
    int rem = q;
    for (int ax = d - 1; ax >= 0; --ax) {
      kc[ax] = centred(rem % N);
      rem /= N;
    }
    const double k2 = kc[0] * kc[0] + kc[1] * kc[1] + kc[2] * kc[2];
    double bll = 0.0;
    for (int p = 0; p < t.nbp; ++p) {
      double f1, f2;
      if (d == 2) {
        const double* e1 = &dirs[3 * p];
        const double* e2 = &dirs[3 * (p + nd / 2)];
        f1 = phi(e1[0] * kc[0] + e1[1] * kc[1]);
        f2 = phi(e2[0] * kc[0] + e2[1] * kc[1]);
        bll += 2.0 * b0 * wdir[p] * f1 * f2;  // directions p and p + M/2 give the same term
      } else {
        const double* e = &dirs[3 * p];
        const double ke = e[0] * kc[0] + e[1] * kc[1] + e[2] * kc[2];
        f1 = psi3(std::sqrt(std::max(k2 - ke * ke, 0.0)));
        f2 = phi(ke);
        bll += b0 * wdir[p] * f1 * f2;
      }
      const size_t o = ((size_t)p * n + q) * 2;
      t.filt[o] = 0.5 * (f1 + f2);
      t.filt[o + 1] = 0.5 * (f2 - f1);
    }
    t.gloss[q] = bll;
  }
  t.carleman = true;
}

HostTables build_tables(const blr_vgrid& vg) {
  validate_vgrid(vg);
  HostTables t;
  t.d = vg.d;
  t.N = vg.n;
  t.n = vg.d == 2 ? vg.n * vg.n : vg.n * vg.n * vg.n;
  t.L = vg.L;
  t.R = vg.R > 0 ? vg.R : 4.0 * vg.L / (3.0 + std::sqrt(2.0));
  t.C = vg.C;
  t.gamma = vg.gamma;
  t.dv = 2.0 * vg.L / vg.n;
  t.mrho = vg.m_rho;
  t.msig = vg.m_sigma ? vg.m_sigma : (vg.d == 2 ? 8 : 38);
  if (vg.flags & BLR_CARLEMAN) {
    carleman_tables(t);
    t.minv = moment_inverse(t);
    return t;
  }
  gauss_legendre(t.mrho, t.R, t.rho, t.wrho);
  t.cw.resize(t.mrho);
  for (int a = 0; a < t.mrho; ++a) t.cw[a] = t.wrho[a] * std::pow(t.rho[a], t.d - 1);
  sphere_rule(t.d, t.msig, t.sig, t.wsig);
  // antipodal pairing
  std::vector<int> used(t.msig, 0);
  for (int b = 0; b < t.msig; ++b) {
    if (used[b]) continue;
    int bb = -1;
    for (int c = 0; c < t.msig; ++c) {
      double e = std::fabs(t.sig[3 * b] + t.sig[3 * c]) + std::fabs(t.sig[3 * b + 1] + t.sig[3 * c + 1]) +
                 std::fabs(t.sig[3 * b + 2] + t.sig[3 * c + 2]);
      if (e < 1e-12) { bb = c; break; }
    }
    require(bb >= 0 && bb != b, "sphere rule is not antipodal", BLR_ERR_NUMERIC);
    used[b] = used[bb] = 1;
    t.bp_b.push_back(b);
    t.bp_bb.push_back(bb);
  }
  t.nbp = (int)t.bp_b.size();
  const int N = t.N, d = t.d;
  auto centred = [N](int k) { return k >= N / 2 ? k - N : k; };
  // per-axis phases exp(-i theta_a sigma_{b,ax} k) for the first member b of each pair
  t.phase.assign((size_t)t.mrho * t.nbp * d * N * 2, 0.0);
  for (int a = 0; a < t.mrho; ++a) {
    const double th = kPi * t.rho[a] / (2.0 * t.L);
    for (int p = 0; p < t.nbp; ++p) {
      const int b = t.bp_b[p];
      for (int ax = 0; ax < d; ++ax)
        for (int k = 0; k < N; ++k) {
          const double x = th * t.sig[3 * b + ax] * centred(k);
          const size_t o = ((((size_t)a * t.nbp + p) * d + ax) * N + k) * 2;
          t.phase[o] = std::cos(x);
          t.phase[o + 1] = -std::sin(x);
        }
    }
  }
  // radial weights as a function of |k|^2 (k centred), folded with 1/n
  t.nkk = d * (N / 2) * (N / 2) + 1;
  t.fw.assign((size_t)t.mrho * t.nkk, 0.0);
  const double area = d == 2 ? 2.0 * kPi : 4.0 * kPi;
  for (int a = 0; a < t.mrho; ++a) {
    const double th = kPi * t.rho[a] / (2.0 * t.L);
    const double B = t.C * std::pow(t.rho[a], t.gamma);
    for (int kk = 0; kk < t.nkk; ++kk) {
      const double z = th * std::sqrt((double)kk);
      double A;
      if (d == 2) A = 2.0 * kPi * bessel_j0(z);
      else A = (z == 0.0) ? 4.0 * kPi : 4.0 * kPi * std::sin(z) / z;
      t.fw[(size_t)a * t.nkk + kk] = t.cw[a] * B * A / t.n;
    }
  }
  // loss weight G-(k)
  t.gloss.assign(t.n, 0.0);
  for (int q = 0; q < t.n; ++q) {
    int kc[3] = {0, 0, 0};
    int rem = q;
    for (int ax = d - 1; ax >= 0; --ax) {
      kc[ax] = centred(rem % N);
      rem /= N;
    }
    double g = 0.0;
    for (int a = 0; a < t.mrho; ++a) {
      const double th = kPi * t.rho[a] / (2.0 * t.L);
      const double B = t.C * std::pow(t.rho[a], t.gamma);
      double s = 0.0;
      for (int b = 0; b < t.msig; ++b) {
        const double dot = t.sig[3 * b] * kc[0] + t.sig[3 * b + 1] * kc[1] + t.sig[3 * b + 2] * kc[2];
        s += t.wsig[b] * std::cos(2.0 * th * dot);
      }
      g += t.cw[a] * B * s;
    }
    t.gloss[q] = area * g;
  }
  if (vg.aniso_n > 0) {
    // B(rho, c) = C rho^gamma sum_i aniso[i] Y_i(c): the loss keeps aniso[0];
    // the gain weight of antipodal pair p = (b, bbar) at radial node a is the
    // even part of the Funk-Hecke transform of the angular factor,
    // (F_ab + F_abbar)(k) / 2 = C rho^gamma |S| sum_{i even} aniso[i]
    // (-1)^(i/2) Z_i(theta |k|) Y_i(sigma_b . k^), times cw_a / n.
    t.aniso_n = vg.aniso_n;
    for (int i = 0; i < 5; ++i) t.aniso[i] = i < vg.aniso_n ? vg.aniso[i] : 0.0;
    for (double& g : t.gloss) g *= t.aniso[0];
    // radial factors Z_i(theta_a |k|) by (a, |k|^2)
    std::vector<double> zt((size_t)t.mrho * t.nkk * 5, 0.0);
    for (int a = 0; a < t.mrho; ++a) {
      const double th = kPi * t.rho[a] / (2.0 * t.L);
      for (int k2 = 0; k2 < t.nkk; ++k2) {
        const double z = th * std::sqrt((double)k2);
        for (int i = 0; i < t.aniso_n; i += 2)
          zt[((size_t)a * t.nkk + k2) * 5 + i] = d == 3 ? sph_bessel_even(i, z) : bessel_jn(i, z);
      }
    }
    t.atab.assign((size_t)t.mrho * t.nbp * t.n, 0.0);
    for (int q = 0; q < t.n; ++q) {
      double kc[3] = {0, 0, 0};
      int rem = q;
      for (int ax = d - 1; ax >= 0; --ax) {
        kc[ax] = centred(rem % N);
        rem /= N;
      }
      const int k2 = (int)std::lround(kc[0] * kc[0] + kc[1] * kc[1] + kc[2] * kc[2]);
      const double kk = std::sqrt((double)k2);
      for (int a = 0; a < t.mrho; ++a) {
        const double* zi = &zt[((size_t)a * t.nkk + k2) * 5];
        const double pref = t.cw[a] * t.C * std::pow(t.rho[a], t.gamma) * area / t.n;
        for (int p = 0; p < t.nbp; ++p) {
          const int b = t.bp_b[p];
          const double c = kk > 0 ? (t.sig[3 * b] * kc[0] + t.sig[3 * b + 1] * kc[1] +
                                     t.sig[3 * b + 2] * kc[2]) / kk : 1.0;
          double s = 0.0;
          for (int i = 0; i < t.aniso_n; i += 2) {
            const double y = d == 3 ? legendre_p(i, c) : std::cos(i * std::acos(std::max(-1.0, std::min(1.0, c))));
            s += t.aniso[i] * ((i / 2) % 2 ? -1.0 : 1.0) * zi[i] * y;
          }
          t.atab[((size_t)a * t.nbp + p) * t.n + q] = pref * s;
        }
      }
    }
  }
  t.minv = moment_inverse(t);
  return t;
}

}  // namespace blr
