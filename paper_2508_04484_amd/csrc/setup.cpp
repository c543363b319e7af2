// Host-side set-up: P_N algebra, eigen-split, DG energy operator.
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

namespace dlra {

static const double kPi = 3.14159265358979323846;

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p1 = z, p0 = 1.0;
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute the derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

// Orthonormal associated Legendre functions without the Condon-Shortley
// phase, Pt[l][k] = sqrt((2l+1)/(4pi) (l-k)!/(l+k)!) P_l^k(mu), by the
// standard stable recurrences in l at fixed k.
static void norm_legendre(int N, double mu, std::vector<double> &Pt) {
  Pt.assign((N + 1) * (N + 1), 0.0);
  auto at = [&](int l, int k) -> double & { return Pt[l * (N + 1) + k]; };
  double s = std::sqrt(std::max(0.0, 1.0 - mu * mu));
  at(0, 0) = std::sqrt(1.0 / (4.0 * kPi));
  for (int k = 1; k <= N; ++k) at(k, k) = std::sqrt((2.0 * k + 1.0) / (2.0 * k)) * s * at(k - 1, k - 1);
  for (int k = 0; k < N; ++k) at(k + 1, k) = std::sqrt(2.0 * k + 3.0) * mu * at(k, k);
  for (int k = 0; k <= N; ++k) {
    for (int l = k + 2; l <= N; ++l) {
      double a = std::sqrt((4.0 * l * l - 1.0) / (double(l) * l - double(k) * k));
      double b = std::sqrt((double(l - 1) * (l - 1) - double(k) * k) / (4.0 * (l - 1) * (l - 1) - 1.0));
      at(l, k) = a * (mu * at(l - 1, k) - b * at(l - 2, k));
    }
  }
}

void real_harmonics(int N, double mu, double phi, double *out) {
  std::vector<double> Pt;
  norm_legendre(N, mu, Pt);
  const double r2 = std::sqrt(2.0);
  for (int l = 0; l <= N; ++l) {
    out[l * l + l] = Pt[l * (N + 1)];
    for (int k = 1; k <= l; ++k) {
      double v = r2 * Pt[l * (N + 1) + k];
      out[l * l + l + k] = v * std::cos(k * phi);
      out[l * l + l - k] = v * std::sin(k * phi);
    }
  }
}

void streaming_matrices(int N, std::vector<double> A[3]) {
  const int m = (N + 1) * (N + 1);
  const int nmu = N + 2, nphi = 2 * N + 4;
  std::vector<double> xm, wm;
  gauss_legendre(nmu, xm, wm);
  for (int d = 0; d < 3; ++d) A[d].assign(size_t(m) * m, 0.0);
  std::vector<double> Y(m);
  for (int a = 0; a < nmu; ++a) {
    for (int b = 0; b < nphi; ++b) {
      double phi = 2.0 * kPi * b / nphi;
      double mu = xm[a];
      double w = wm[a] * 2.0 * kPi / nphi;
      real_harmonics(N, mu, phi, Y.data());
      double s = std::sqrt(1.0 - mu * mu);
      double om[3] = {s * std::cos(phi), s * std::sin(phi), mu};
      for (int d = 0; d < 3; ++d) {
        double wd = w * om[d];
        for (int p = 0; p < m; ++p) {
          double yp = wd * Y[p];
          double *row = &A[d][size_t(p) * m];
          for (int q = 0; q < m; ++q) row[q] += yp * Y[q];
        }
      }
    }
  }
  // drop quadrature round-off on structurally zero couplings
  for (int d = 0; d < 3; ++d)
    for (auto &v : A[d])
      if (std::fabs(v) < 1e-14) v = 0.0;
}

// Cyclic two-sided Jacobi for a dense symmetric n x n matrix (row-major, in
// place); V receives the eigenvectors as columns.
static void jacobi_eig(std::vector<double> &a, int n, std::vector<double> &V) {
  V.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double v = a[size_t(i) * n + j] * a[size_t(i) * n + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = a[size_t(p) * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = a[size_t(p) * n + p], aqq = a[size_t(q) * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = a[size_t(k) * n + p], akq = a[size_t(k) * n + q];
          a[size_t(k) * n + p] = c * akp - s * akq;
          a[size_t(k) * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = a[size_t(p) * n + k], aqk = a[size_t(q) * n + k];
          a[size_t(p) * n + k] = c * apk - s * aqk;
          a[size_t(q) * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[size_t(k) * n + p], vkq = V[size_t(k) * n + q];
          V[size_t(k) * n + p] = c * vkp - s * vkq;
          V[size_t(k) * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

void eigen_split(const std::vector<double> &A, int m, std::vector<double> &Ap,
                 std::vector<double> &Am) {
  // connected components of the sparsity graph (union-find)
  std::vector<int> parent(m);
  std::iota(parent.begin(), parent.end(), 0);
  auto root = [&](int x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  for (int p = 0; p < m; ++p)
    for (int q = p + 1; q < m; ++q)
      if (A[size_t(p) * m + q] != 0.0 || A[size_t(q) * m + p] != 0.0) {
        int a = root(p), b = root(q);
        if (a != b) parent[a] = b;
      }
  std::vector<std::vector<int>> comps;
  std::vector<int> cid(m, -1);
  for (int p = 0; p < m; ++p) {
    int r = root(p);
    if (cid[r] < 0) {
      cid[r] = int(comps.size());
      comps.emplace_back();
    }
    comps[cid[r]].push_back(p);
  }
  Ap.assign(size_t(m) * m, 0.0);
  Am.assign(size_t(m) * m, 0.0);
  for (const auto &idx : comps) {
    int n = int(idx.size());
    std::vector<double> a(size_t(n) * n), V;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        a[size_t(i) * n + j] = 0.5 * (A[size_t(idx[i]) * m + idx[j]] + A[size_t(idx[j]) * m + idx[i]]);
    jacobi_eig(a, n, V);
    for (int k = 0; k < n; ++k) {
      double lam = a[size_t(k) * n + k];
      double lp = std::max(lam, 0.0), lm = std::min(lam, 0.0);
      for (int i = 0; i < n; ++i) {
        double vik = V[size_t(i) * n + k];
        for (int j = 0; j < n; ++j) {
          double vv = vik * V[size_t(j) * n + k];
          Ap[size_t(idx[i]) * m + idx[j]] += lp * vv;
          Am[size_t(idx[i]) * m + idx[j]] += lm * vv;
        }
      }
    }
  }
}

void beam_moments(int N, const double dir[3], double *out) {
  double nrm = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  double mu = std::max(-1.0, std::min(1.0, dir[2] / nrm));
  double phi = std::atan2(dir[1] / nrm, dir[0] / nrm);
  real_harmonics(N, mu, phi, out);
}

double interp(const double *e, const double *v, int n, double E) {
  if (E <= e[0]) return v[0];
  if (E >= e[n - 1]) return v[n - 1];
  int j = int(std::upper_bound(e, e + n, E) - e) - 1;
  return v[j] + (E - e[j]) * ((v[j + 1] - v[j]) / (e[j + 1] - e[j]));
}

double interp_slope(const double *e, const double *v, int n, double E) {
  int j = int(std::upper_bound(e, e + n, E) - e) - 1;
  j = std::max(0, std::min(n - 2, j));
  return (v[j + 1] - v[j]) / (e[j + 1] - e[j]);
}

// Legendre polynomials of degree <= 2 on [-1, 1] and their derivatives.
static inline void leg3(double x, double p[3], double dp[3]) {
  p[0] = 1.0;
  p[1] = x;
  p[2] = 1.5 * x * x - 0.5;
  dp[0] = 0.0;
  dp[1] = 1.0;
  dp[2] = 3.0 * x;
}

void energy_operator(double e_cut, double e_max, int G, const double *e, int n_e,
                     const double *S, const double *T, const double *sig,
                     EnergyOperator &op) {
  op.G = G;
  op.e_cut = e_cut;
  op.e_max = e_max;
  const double h = (e_max - e_cut) / G;
  op.h = h;
  op.diag.assign(size_t(G) * 9, 0.0);
  op.up.assign(size_t(G) * 9, 0.0);
  op.lo.assign(size_t(G) * 9, 0.0);
  std::vector<double> xq, wq;
  gauss_legendre(4, xq, wq);
  auto Sstar = [&](double E) { return interp(e, S, n_e, E) + 0.5 * interp_slope(e, T, n_e, E); };
  // volume terms: -int Sig phi_i phi_j - int phi_i' S* phi_j - 1/2 int T phi_i' phi_j'
  for (int g = 0; g < G; ++g) {
    double a = e_cut + h * g;
    double *D = &op.diag[size_t(g) * 9];
    for (int q = 0; q < 4; ++q) {
      double E = a + 0.5 * h * (xq[q] + 1.0);
      double wE = 0.5 * h * wq[q];
      double p[3], dp[3];
      leg3(xq[q], p, dp);
      for (int i = 0; i < 3; ++i) dp[i] *= 2.0 / h;
      double sg = interp(e, sig, n_e, E), ss = Sstar(E), tt = interp(e, T, n_e, E);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          D[i * 3 + j] += wE * (-sg * p[i] * p[j] - ss * dp[i] * p[j] - 0.5 * tt * dp[i] * dp[j]);
    }
  }
  // faces.  phi_i(+1) = 1, phi_i(-1) = (-1)^i; phi_i'(+1) = (0,1,3) 2/h,
  // phi_i'(-1) = (0,1,-3) 2/h.
  const double top[3] = {1.0, 1.0, 1.0}, bot[3] = {1.0, -1.0, 1.0};
  const double dtop[3] = {0.0, 2.0 / h, 6.0 / h}, dbot[3] = {0.0, 2.0 / h, -6.0 / h};
  for (int g = 0; g < G; ++g) {
    double a = e_cut + h * g;
    double *D = &op.diag[size_t(g) * 9];
    // upwind slowing-down flux S*(a) psi_g(a) leaves through the bottom face
    double sa = Sstar(a);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) D[i * 3 + j] -= sa * bot[i] * bot[j];
    if (g + 1 < G) {
      double b = a + h;
      double sb = Sstar(b);
      double *Up = &op.up[size_t(g) * 9];
      // inflow from group g+1 through the top face: + phi_i(+1) S*(b) psi_{g+1}(b)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Up[i * 3 + j] += sb * top[i] * bot[j];
      // SIPG between lower group L = g and upper U = g+1:
      // 1/2 ({T psi'}[v] + {T v'}[psi] - pen [psi][v]), [v] = v_L - v_U
      double Te = interp(e, T, n_e, b);
      double pen = 18.0 * Te / h;
      double jL[3], jU[3], aL[3], aU[3];
      for (int i = 0; i < 3; ++i) {
        jL[i] = top[i];
        jU[i] = -bot[i];
        aL[i] = 0.5 * Te * dtop[i];
        aU[i] = 0.5 * Te * dbot[i];
      }
      double *DU = &op.diag[size_t(g + 1) * 9];
      double *Lo = &op.lo[size_t(g + 1) * 9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          D[i * 3 + j] += 0.5 * (jL[i] * aL[j] + aL[i] * jL[j] - pen * jL[i] * jL[j]);
          Up[i * 3 + j] += 0.5 * (jL[i] * aU[j] + aL[i] * jU[j] - pen * jL[i] * jU[j]);
          Lo[i * 3 + j] += 0.5 * (jU[i] * aL[j] + aU[i] * jL[j] - pen * jU[i] * jL[j]);
          DU[i * 3 + j] += 0.5 * (jU[i] * aU[j] + aU[i] * jU[j] - pen * jU[i] * jU[j]);
        }
    }
  }
}

void project_gaussian(const EnergyOperator &op, double E0, double sE, double *c) {
  std::vector<double> xq, wq;
  gauss_legendre(8, xq, wq);
  const double norm = 1.0 / (std::sqrt(2.0 * kPi) * sE);
  for (int g = 0; g < op.G; ++g) {
    double a = op.e_cut + op.h * g;
    double acc[3] = {0, 0, 0};
    for (int q = 0; q < 8; ++q) {
      double E = a + 0.5 * op.h * (xq[q] + 1.0);
      double f = norm * std::exp(-0.5 * ((E - E0) / sE) * ((E - E0) / sE));
      double p[3], dp[3];
      leg3(xq[q], p, dp);
      for (int i = 0; i < 3; ++i) acc[i] += wq[q] * f * p[i];
    }
    for (int i = 0; i < 3; ++i) c[3 * g + i] = acc[i] * (2.0 * i + 1.0) / 2.0;
  }
}

int step_integral(const EnergyOperator &op, double lo, double hi, int ng, double *w) {
  int g0 = int(std::floor((lo - op.e_cut) / op.h)) - 1;
  g0 = std::max(0, std::min(op.G - ng, g0));
  for (int t = 0; t < ng * 3; ++t) w[t] = 0.0;
  for (int t = 0; t < ng; ++t) {
    int g = g0 + t;
    double a = op.e_cut + op.h * g, b = a + op.h;
    double l = std::max(a, lo), u = std::min(b, hi);
    if (u <= l) continue;
    double x1 = 2.0 * (l - a) / op.h - 1.0, x2 = 2.0 * (u - a) / op.h - 1.0;
    w[3 * t + 0] = 0.5 * op.h * (x2 - x1);
    w[3 * t + 1] = 0.5 * op.h * 0.5 * (x2 * x2 - x1 * x1);
    w[3 * t + 2] = 0.5 * op.h * (0.5 * (x2 * x2 * x2 - x1 * x1 * x1) - 0.5 * (x2 - x1));
  }
  // every group overlapping [lo, hi] must lie in the window
  int gl = int(std::floor((lo - op.e_cut) / op.h)), gh = int(std::ceil((hi - op.e_cut) / op.h)) - 1;
  gl = std::max(gl, 0);
  gh = std::min(gh, op.G - 1);
  if (gl < g0 || gh > g0 + ng - 1) throw std::runtime_error("step integral window too small");
  return g0;
}

void weighted_integral(const EnergyOperator &op, const double *e, const double *f, int n_e,
                       double *w) {
  std::vector<double> xq, wq;
  gauss_legendre(3, xq, wq);
  for (int g = 0; g < op.G; ++g) {
    double a = op.e_cut + op.h * g;
    for (int i = 0; i < 3; ++i) w[3 * g + i] = 0.0;
    for (int q = 0; q < 3; ++q) {
      double E = a + 0.5 * op.h * (xq[q] + 1.0);
      double fv = interp(e, f, n_e, E);
      double p[3], dp[3];
      leg3(xq[q], p, dp);
      for (int i = 0; i < 3; ++i) w[3 * g + i] += 0.5 * op.h * wq[q] * fv * p[i];
    }
  }
}

}  // namespace dlra
