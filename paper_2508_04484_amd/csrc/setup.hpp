// Host-side set-up of the DLRA proton-transport library: angular P_N algebra,
// per-step coefficients and the DG energy operator of the ray tracer.  Pure
// C++ (FP64); everything here runs once per context in dlra_init.
#pragma once

#include <cstddef>
#include <string>
#include <vector>

namespace dlra {

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);

// Real spherical harmonics m_l^k (Sec. 3.3.1), ordering p = l^2 + l + k, at
// direction (mu, phi): out[p] for p < (N+1)^2.
void real_harmonics(int N, double mu, double phi, double *out);

// Streaming matrices A_d = int m m^T Omega_d dOmega, d = x, y, z (Sec. 3.3.1),
// row-major m x m each, from an exact product quadrature.
void streaming_matrices(int N, std::vector<double> A[3]);

// Eigen-split A = V diag(lambda) V^T -> A^+ = V max(lambda,0) V^T,
// A^- = V min(lambda,0) V^T (Sec. 3.3.2); symmetric Jacobi on the connected
// blocks of A's sparsity pattern.
void eigen_split(const std::vector<double> &A, int m, std::vector<double> &Ap,
                 std::vector<double> &Am);

// T_M = m(Omega_in) for a unit direction.
void beam_moments(int N, const double dir[3], double *out);

// Linear interpolation with clamping at the table ends, and the slope of the
// table segment holding E (the end segments' slopes beyond the table).
double interp(const double *e, const double *v, int n, double E);
double interp_slope(const double *e, const double *v, int n, double E);

// Per-material DG-P2 energy operator of the ray tracer (Sec. 3.2):
// M dpsi/dz = A psi; A is block tridiagonal with 3x3 blocks per group:
//   diag[g], up[g] (couples group g to g+1), lo[g] (couples group g to g-1),
// each row-major 3x3, stored consecutively per group.
struct EnergyOperator {
  int G = 0;
  double e_cut = 0, e_max = 0, h = 0;
  std::vector<double> diag, up, lo;   // G*9 each
};
void energy_operator(double e_cut, double e_max, int G, const double *e, int n_e,
                     const double *S, const double *T, const double *sig,
                     EnergyOperator &op);

// L2 projection of the normalised Gaussian N(E0, sE) onto the DG space.
void project_gaussian(const EnergyOperator &op, double E0, double sE, double *c);

// Exact integral over [lo, hi] of the DG function as weights on the
// coefficients of groups g0 .. g0+ng-1: returns g0, fills w[ng*3].
int step_integral(const EnergyOperator &op, double lo, double hi, int ng, double *w);

// Weights of int f(E) psi dE (3-point Gauss per group) for a tabulated f.
void weighted_integral(const EnergyOperator &op, const double *e, const double *f, int n_e,
                       double *w);

}  // namespace dlra
