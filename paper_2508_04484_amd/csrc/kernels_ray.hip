// Uncollided ray tracer (Sec. 3.2): DG-P2 in energy, Crank-Nicolson in depth.
//
// One thread marches one grid row along the beam axis (all midpoints of a
// row lie on one ray).  Per cell the block-tridiagonal matrix
// M - h/2 A(x), A(x) = sum_i w_i(x) A_i, is factorised once (block Thomas),
// then each substep forms (M + h/2 A) c and solves.  Per-thread state lives in
// a scratch area laid out [element][row] so that a wave's accesses coalesce.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace dlra {

namespace {

__device__ __forceinline__ void inv3(const double a[9], double o[9]) {
  double c00 = a[4] * a[8] - a[5] * a[7];
  double c01 = a[5] * a[6] - a[3] * a[8];
  double c02 = a[3] * a[7] - a[4] * a[6];
  double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  double id = 1.0 / det;
  o[0] = c00 * id;
  o[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  o[3] = c01 * id;
  o[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  o[6] = c02 * id;
  o[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

template <typename T>
__global__ __launch_bounds__(64) void k_raytrace_rows(
    RayParams rp, const int *__restrict__ row_start, const double *__restrict__ row_f,
    const double *__restrict__ w, const double *__restrict__ Adiag,
    const double *__restrict__ Aup, const double *__restrict__ Alo,
    const double *__restrict__ mass, const double *__restrict__ c0,
    const int *__restrict__ step_g0, const double *__restrict__ step_w,
    const double *__restrict__ stop_w, double *__restrict__ scratch, T *__restrict__ psibar,
    double *__restrict__ Du) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rp.n_rows) return;
  const int G = rp.G;
  const int R = rp.n_rows;
  // scratch: c[3G], y[3G], Dinv[9G], E[9G]
  double *c = scratch;
  double *y = scratch + size_t(3) * G * R;
  double *Dinv = scratch + size_t(6) * G * R;
  double *E = scratch + size_t(15) * G * R;
#define SC(base, e) base[size_t(e) * R + row]
  for (int e = 0; e < 3 * G; ++e) SC(c, e) = c0[e];
  const double m0 = mass[0], m1 = mass[1], m2 = mass[2];
  const double h = rp.half / rp.n_half;
  const double hh = 0.5 * h;
  const double f = row_f[row];
  for (int ci = 0; ci < rp.row_len; ++ci) {
    const int cell = rp.sign > 0 ? ci : rp.row_len - 1 - ci;
    const int x = row_start[row] + cell * rp.row_stride;
    double wv[kMaxMat];
    for (int i = 0; i < rp.n_mat; ++i) wv[i] = w[size_t(i) * rp.n + x];
    // factorisation of M - h/2 A for this cell
    double Eprev[9];
    for (int g = 0; g < G; ++g) {
      double D[9], Lg[9], Ug[9];
      for (int t = 0; t < 9; ++t) {
        double ad = 0.0, al = 0.0, au = 0.0;
        for (int i = 0; i < rp.n_mat; ++i) {
          size_t o = (size_t(i) * G + g) * 9 + t;
          ad += wv[i] * Adiag[o];
          al += wv[i] * Alo[o];
          au += wv[i] * Aup[o];
        }
        D[t] = -hh * ad;
        Lg[t] = -hh * al;
        Ug[t] = -hh * au;
      }
      D[0] += m0;
      D[4] += m1;
      D[8] += m2;
      if (g > 0) {
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Lg[i * 3 + k] * Eprev[k * 3 + j];
            D[i * 3 + j] -= s;
          }
      }
      double Di[9];
      inv3(D, Di);
      for (int t = 0; t < 9; ++t) SC(Dinv, g * 9 + t) = Di[t];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double s = 0.0;
          for (int k = 0; k < 3; ++k) s += Di[i * 3 + k] * Ug[k * 3 + j];
          Eprev[i * 3 + j] = s;
        }
      for (int t = 0; t < 9; ++t) SC(E, g * 9 + t) = (g + 1 < G) ? Eprev[t] : 0.0;
    }
    for (int half = 0; half < 2; ++half) {
      for (int sub = 0; sub < rp.n_half; ++sub) {
        // forward sweep: y_g = Dinv_g (rhs_g - L_g y_{g-1}), rhs = (M + h/2 A) c
        double yprev[3] = {0.0, 0.0, 0.0};
        double cprev[3] = {0.0, 0.0, 0.0};
        double cg[3], cnext[3];
        for (int k = 0; k < 3; ++k) cg[k] = SC(c, k);
        for (int g = 0; g < G; ++g) {
          for (int k = 0; k < 3; ++k) cnext[k] = (g + 1 < G) ? SC(c, 3 * (g + 1) + k) : 0.0;
          double rhs[3] = {m0 * cg[0], m1 * cg[1], m2 * cg[2]};
          double Lg[9];
          for (int t = 0; t < 9; ++t) {
            double ad = 0.0, al = 0.0, au = 0.0;
            for (int i = 0; i < rp.n_mat; ++i) {
              size_t o = (size_t(i) * G + g) * 9 + t;
              ad += wv[i] * Adiag[o];
              al += wv[i] * Alo[o];
              au += wv[i] * Aup[o];
            }
            int ii = t / 3, jj = t % 3;
            rhs[ii] += hh * (ad * cg[jj] + al * cprev[jj] + au * cnext[jj]);
            Lg[t] = -hh * al;
          }
          double b[3];
          for (int i = 0; i < 3; ++i)
            b[i] = rhs[i] - (Lg[i * 3 + 0] * yprev[0] + Lg[i * 3 + 1] * yprev[1] +
                             Lg[i * 3 + 2] * yprev[2]);
          double yg[3];
          for (int i = 0; i < 3; ++i)
            yg[i] = SC(Dinv, g * 9 + i * 3 + 0) * b[0] + SC(Dinv, g * 9 + i * 3 + 1) * b[1] +
                    SC(Dinv, g * 9 + i * 3 + 2) * b[2];
          for (int k = 0; k < 3; ++k) {
            SC(y, 3 * g + k) = yg[k];
            yprev[k] = yg[k];
            cprev[k] = cg[k];
            cg[k] = cnext[k];
          }
        }
        // back substitution: c_g = y_g - E_g c_{g+1}
        double cn[3] = {0.0, 0.0, 0.0};
        for (int g = G - 1; g >= 0; --g) {
          double cv[3];
          for (int i = 0; i < 3; ++i)
            cv[i] = SC(y, 3 * g + i) - (SC(E, g * 9 + i * 3 + 0) * cn[0] +
                                        SC(E, g * 9 + i * 3 + 1) * cn[1] +
                                        SC(E, g * 9 + i * 3 + 2) * cn[2]);
          for (int i = 0; i < 3; ++i) {
            SC(c, 3 * g + i) = cv[i];
            cn[i] = cv[i];
          }
        }
      }
      if (half == 0) {
        // midpoint outputs
        for (int k = 0; k < rp.n_steps; ++k) {
          const int g0 = step_g0[k];
          const double *sw = step_w + size_t(k) * rp.ng_step * 3;
          double s = 0.0;
          for (int t = 0; t < rp.ng_step * 3; ++t) s += sw[t] * SC(c, 3 * g0 + t);
          psibar[size_t(k) * rp.n + x] = T(f * s);
        }
        double du = 0.0;
        for (int i = 0; i < rp.n_mat; ++i) {
          const double *sw = stop_w + size_t(i) * 3 * G;
          double s = 0.0;
          for (int e = 0; e < 3 * G; ++e) s += sw[e] * SC(c, e);
          du += wv[i] * s;
        }
        Du[x] = f * du;
      }
    }
  }
#undef SC
}

}  // namespace

template <typename T>
void launch_raytrace_rows(const RayParams &rp, const int *row_start, const double *row_f,
                          const double *w, const double *Adiag, const double *Aup,
                          const double *Alo, const double *mass, const double *c0,
                          const int *step_g0, const double *step_w, const double *stop_w,
                          double *scratch, T *psibar, double *Du, hipStream_t st) {
  if (rp.n_rows <= 0) return;
  k_raytrace_rows<T><<<(rp.n_rows + 63) / 64, 64, 0, st>>>(rp, row_start, row_f, w, Adiag, Aup,
                                                            Alo, mass, c0, step_g0, step_w,
                                                            stop_w, scratch, psibar, Du);
}

template void launch_raytrace_rows<double>(const RayParams &, const int *, const double *,
                                           const double *, const double *, const double *,
                                           const double *, const double *, const double *,
                                           const int *, const double *, const double *,
                                           double *, double *, double *, hipStream_t);
template void launch_raytrace_rows<float>(const RayParams &, const int *, const double *,
                                          const double *, const double *, const double *,
                                          const double *, const double *, const double *,
                                          const int *, const double *, const double *, double *,
                                          float *, double *, hipStream_t);

}  // namespace dlra
