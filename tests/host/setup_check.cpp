// The library's host-side set-up routines (csrc/setup.cpp) run under
// AddressSanitizer and UndefinedBehaviorSanitizer and checked against closed
// forms; built and run by tests/test_host_setup.py (no GPU).
#include "setup.hpp"

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

using namespace dlra;

static int fails = 0;

static void check(bool ok, const char *what, int a = 0) {
  if (!ok) {
    std::printf("FAIL %s (%d)\n", what, a);
    ++fails;
  }
}

static double quad_form(const std::vector<double> &A, int m, const std::vector<double> &x) {
  double s = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) s += x[i] * A[size_t(i) * m + j] * x[j];
  return s;
}

int main() {
  const double pi = std::acos(-1.0);
  std::mt19937_64 rng(11);
  std::normal_distribution<double> nd;

  // Gauss-Legendre with n nodes integrates degree 2n - 1 exactly
  for (int n : {1, 2, 5, 16, 33}) {
    std::vector<double> x, w;
    gauss_legendre(n, x, w);
    double s0 = 0.0, sd = 0.0;
    for (int i = 0; i < n; ++i) {
      s0 += w[i];
      sd += w[i] * std::pow(x[i], 2 * n - 2);
    }
    check(std::fabs(s0 - 2.0) < 1e-13, "Gauss-Legendre weights sum to 2", n);
    check(std::fabs(sd - 2.0 / (2 * n - 1)) < 1e-12, "Gauss-Legendre exact for x^(2n-2)", n);
  }

  for (int N : {0, 1, 3, 7}) {
    const int m = (N + 1) * (N + 1);
    // orthonormality of the real harmonics under a product rule exact for
    // their products (Gauss in mu, uniform in phi)
    std::vector<double> x, w;
    gauss_legendre(N + 1, x, w);
    const int nphi = 2 * N + 2;
    std::vector<double> G(size_t(m) * m, 0.0), y(m);
    for (int i = 0; i <= N; ++i)
      for (int j = 0; j < nphi; ++j) {
        real_harmonics(N, x[i], 2.0 * pi * j / nphi, y.data());
        const double wt = w[i] * 2.0 * pi / nphi;
        for (int p = 0; p < m; ++p)
          for (int q = 0; q < m; ++q) G[size_t(p) * m + q] += wt * y[p] * y[q];
      }
    double err = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = 0; q < m; ++q) err = std::fmax(err, std::fabs(G[size_t(p) * m + q] - (p == q)));
    check(err < 1e-12, "real harmonics orthonormal", N);

    // addition theorem: sum_p m_p(Omega)^2 = (N + 1)^2 / (4 pi)
    for (int t = 0; t < 4; ++t) {
      double d[3] = {nd(rng), nd(rng), nd(rng)};
      const double nrm = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (double &v : d) v /= nrm;
      beam_moments(N, d, y.data());
      double s = 0.0;
      for (int p = 0; p < m; ++p) s += y[p] * y[p];
      check(std::fabs(s - m / (4.0 * pi)) < 1e-12, "addition theorem", N);
    }

    // streaming matrices: symmetric with spectrum in [-1, 1] (Galerkin
    // projections of multiplication by Omega_d); the eigen-split gives
    // A = A+ + A-, A+ >= 0 >= A-, A+ A- = 0
    std::vector<double> A[3];
    streaming_matrices(N, A);
    for (int d = 0; d < 3; ++d) {
      check(A[d].size() == size_t(m) * m, "streaming matrix size", d);
      double asym = 0.0;
      for (int p = 0; p < m; ++p)
        for (int q = 0; q < m; ++q)
          asym = std::fmax(asym, std::fabs(A[d][size_t(p) * m + q] - A[d][size_t(q) * m + p]));
      check(asym < 1e-13, "streaming matrix symmetric", d);
      std::vector<double> Ap, Am;
      eigen_split(A[d], m, Ap, Am);
      double rec = 0.0, prod = 0.0;
      for (int p = 0; p < m; ++p)
        for (int q = 0; q < m; ++q) {
          rec = std::fmax(rec, std::fabs(Ap[size_t(p) * m + q] + Am[size_t(p) * m + q] -
                                         A[d][size_t(p) * m + q]));
          double s = 0.0;
          for (int k = 0; k < m; ++k) s += Ap[size_t(p) * m + k] * Am[size_t(k) * m + q];
          prod = std::fmax(prod, std::fabs(s));
        }
      check(rec < 1e-13, "eigen-split reconstructs A", d);
      check(prod < 1e-12, "A+ A- = 0", d);
      std::vector<double> v(m);
      for (int t = 0; t < 8; ++t) {
        double vv = 0.0;
        for (double &e : v) {
          e = nd(rng);
          vv += e * e;
        }
        const double qp = quad_form(Ap, m, v), qm = quad_form(Am, m, v);
        check(qp >= -1e-13 * vv && qp <= (1.0 + 1e-12) * vv, "0 <= A+ <= 1", d);
        check(qm <= 1e-13 * vv && qm >= -(1.0 + 1e-12) * vv, "-1 <= A- <= 0", d);
      }
    }
  }

  // interpolation: exact on a linear table, clamped outside it
  {
    const double e[4] = {1.0, 2.0, 4.0, 7.0}, v[4] = {3.0, 5.0, 9.0, 15.0};   // 2E + 1
    check(std::fabs(interp(e, v, 4, 3.0) - 7.0) < 1e-14, "interp inside");
    check(interp(e, v, 4, 0.0) == 3.0 && interp(e, v, 4, 10.0) == 15.0, "interp clamps");
    check(std::fabs(interp_slope(e, v, 4, 5.5) - 2.0) < 1e-14, "interp slope");
    check(std::fabs(interp_slope(e, v, 4, 9.0) - 2.0) < 1e-14 &&
              std::fabs(interp_slope(e, v, 4, 0.5) - 2.0) < 1e-14,
          "interp slope beyond the table: the end segments'");
  }

  // DG energy operator of a synthetic material (smooth positive tables) and
  // the integrals the ray tracer's outputs use
  {
    const int n_e = 40, G = 64;
    std::vector<double> e(n_e), S(n_e), T(n_e), sig(n_e);
    for (int i = 0; i < n_e; ++i) {
      e[i] = 0.5 * std::pow(600.0, double(i) / (n_e - 1));   // 0.5 .. 300 MeV
      S[i] = 80.0 / (e[i] + 5.0) + 2.0;
      T[i] = 0.02 + 1e-3 * e[i];
      sig[i] = 0.01 + 1e-5 * e[i];
    }
    EnergyOperator op;
    energy_operator(1.0, 250.0, G, e.data(), n_e, S.data(), T.data(), sig.data(), op);
    bool finite = op.G == G && op.diag.size() == size_t(G) * 9 && op.up.size() == size_t(G) * 9 &&
                  op.lo.size() == size_t(G) * 9;
    for (int t = 0; t < G * 9; ++t)
      finite = finite && std::isfinite(op.diag[t]) && std::isfinite(op.up[t]) &&
               std::isfinite(op.lo[t]);
    check(finite, "energy operator finite");

    // the L2 projection keeps the integral over each whole group, so the
    // projected Gaussian (far inside the range) integrates to 1
    std::vector<double> c(size_t(G) * 3);
    project_gaussian(op, 150.0, 1.5, c.data());
    double total = 0.0;
    for (int g = 0; g < G; ++g) total += op.h * c[3 * g];
    check(std::fabs(total - 1.0) < 1e-10, "projected Gaussian integrates to 1");

    // the step integral over the whole range, and the weighted integral with
    // f = 1, give the same number
    std::vector<double> ws(size_t(G) * 3);
    const int g0 = step_integral(op, op.e_cut, op.e_max, G, ws.data());
    double si = 0.0;
    for (int t = 0; t < 3 * G; ++t) si += ws[t] * c[3 * g0 + t];
    check(g0 == 0 && std::fabs(si - total) < 1e-12, "step integral over the range");
    const double one[2] = {1.0, 1.0}, eo[2] = {0.0, 400.0};
    std::vector<double> wi(size_t(G) * 3);
    weighted_integral(op, eo, one, 2, wi.data());
    double wsum = 0.0;
    for (int t = 0; t < 3 * G; ++t) wsum += wi[t] * c[t];
    check(std::fabs(wsum - total) < 1e-12, "weighted integral with f = 1");
  }

  std::printf("%d failures\n", fails);
  return fails ? 1 : 0;
}
