// Uncollided ray tracer (Sec. 3.2): DG-P2 in energy, Crank-Nicolson in depth.
//
// One thread marches one ray.  A ray is either a grid row along an axis-
// aligned beam (every midpoint of the row lies on it; outputs after the first
// half of each cell) or, for an oblique beam, the segment from the domain
// entry to one target cell centre (output at its end).  The path is cut at
// cell faces and, inside every traversed cell, at the foot of the
// perpendicular from that cell's centre; each piece of length L takes
// ceil(L / h_max) equal Crank-Nicolson substeps with the material of its
// cell.  Oblique pieces are generated on the fly by a traversal of the face
// planes in order of the ray parameter, with the plane crossings computed as
// t = (j D_d - x_d) / Omega_d.
//
// Per piece the block-tridiagonal matrix M - h/2 A(x), A(x) = sum_i w_i(x) A_i,
// is factorised once (block LU from the lowest group: Dinv_g, F_g = Dinv_g L_g
// and E_g = Dinv_g U_g).  A substep then solves (M - h/2 A) y = M c and sets
// c <- 2 y - c, which equals (M - h/2 A)^{-1} (M + h/2 A) c, so the mixture
// blocks are not formed again per substep: y_g = Dinv_g M c_g - F_g y_{g-1}
// forward, x_g = y_g - E_g x_{g+1} backward.  Per-ray state lives in a
// scratch area laid out [element][ray] so that a wave's accesses coalesce.
// The sweeps are chains over the groups, and a launch of grid rows has few
// waves, so each sweep keeps the loads of the next kRayAhead groups in flight
// (a ring of registers) to cover the memory latency.
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

constexpr int kRayAhead = 4;   // groups whose loads a sweep keeps in flight

// Per-thread view of the scratch columns of one ray.
struct RayState {
  double *c, *y, *Dinv, *F, *E;
  size_t B;   // rays per scratch row
  __device__ double &C(int e) const { return c[size_t(e) * B]; }
  __device__ double &Y(int e) const { return y[size_t(e) * B]; }
  __device__ double &Di(int e) const { return Dinv[size_t(e) * B]; }
  __device__ double &Ff(int e) const { return F[size_t(e) * B]; }
  __device__ double &Ee(int e) const { return E[size_t(e) * B]; }
};

// factorisation of M - hh A(w) into the ray's Dinv, E
__device__ void factorise(const RayParams &rp, const RayState &s, const double *wv,
                          const double *__restrict__ Adiag, const double *__restrict__ Aup,
                          const double *__restrict__ Alo, const double m[3], double hh) {
  const int G = rp.G;
  double Eprev[9];
  for (int g = 0; g < G; ++g) {
    double D[9], Lg[9], Ug[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      double ad = 0.0, al = 0.0, au = 0.0;
      for (int i = 0; i < rp.n_mat; ++i) {
        const size_t o = (size_t(i) * G + g) * 9 + t;
        ad += wv[i] * Adiag[o];
        al += wv[i] * Alo[o];
        au += wv[i] * Aup[o];
      }
      D[t] = -hh * ad;
      Lg[t] = -hh * al;
      Ug[t] = -hh * au;
    }
    D[0] += m[0];
    D[4] += m[1];
    D[8] += m[2];
    if (g > 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) acc += Lg[i * 3 + k] * Eprev[k * 3 + j];
          D[i * 3 + j] -= acc;
        }
    }
    double Di[9];
    inv3(D, Di);
#pragma unroll
    for (int t = 0; t < 9; ++t) s.Di(g * 9 + t) = Di[t];
    // F_g = Dinv_g L_g (the forward sweep's coupling to group g - 1)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc += Di[i * 3 + k] * Lg[k * 3 + j];
        s.Ff(g * 9 + i * 3 + j) = g > 0 ? acc : 0.0;
      }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc += Di[i * 3 + k] * Ug[k * 3 + j];
        Eprev[i * 3 + j] = acc;
      }
#pragma unroll
    for (int t = 0; t < 9; ++t) s.Ee(g * 9 + t) = (g + 1 < G) ? Eprev[t] : 0.0;
  }
}

// one Crank-Nicolson substep c <- 2 (M - hh A)^{-1} M c - c with the stored
// factorisation; loads run kRayAhead groups ahead of the arithmetic
__device__ void cn_substep(const RayParams &rp, const RayState &s, const double m[3]) {
  constexpr int PD = kRayAhead;
  const int G = rp.G;
  // forward sweep: y_g = Dinv_g M c_g - F_g y_{g-1}
  double fc[PD][3], fd[PD][9], ff[PD][9];
  auto fload = [&](int u, int g) {
    const int gg = min(g, G - 1);   // past the end: clamped, unused
#pragma unroll
    for (int k = 0; k < 3; ++k) fc[u][k] = s.C(3 * gg + k);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      fd[u][t] = s.Di(gg * 9 + t);
      ff[u][t] = s.Ff(gg * 9 + t);
    }
  };
#pragma unroll
  for (int u = 0; u < PD; ++u) fload(u, u);
  double yprev[3] = {0.0, 0.0, 0.0};
  for (int g0 = 0; g0 < G; g0 += PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      const int g = g0 + u;
      if (g < G) {
        const double b[3] = {m[0] * fc[u][0], m[1] * fc[u][1], m[2] * fc[u][2]};
        double v[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
          v[i] = (fd[u][i * 3 + 0] * b[0] + fd[u][i * 3 + 1] * b[1] + fd[u][i * 3 + 2] * b[2]) -
                 (ff[u][i * 3 + 0] * yprev[0] + ff[u][i * 3 + 1] * yprev[1] +
                  ff[u][i * 3 + 2] * yprev[2]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          s.Y(3 * g + i) = v[i];
          yprev[i] = v[i];
        }
      }
      fload(u, g + PD);
    }
  }
  // backward sweep: x_g = y_g - E_g x_{g+1}; c_g <- 2 x_g - c_g
  double by[PD][3], bc[PD][3], be[PD][9];
  auto bload = [&](int u, int g) {
    const int gg = max(g, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      by[u][k] = s.Y(3 * gg + k);
      bc[u][k] = s.C(3 * gg + k);
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) be[u][t] = s.Ee(gg * 9 + t);
  };
#pragma unroll
  for (int u = 0; u < PD; ++u) bload(u, G - 1 - u);
  double xn[3] = {0.0, 0.0, 0.0};
  for (int g0 = G - 1; g0 >= 0; g0 -= PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      const int g = g0 - u;
      if (g >= 0) {
        double xv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
          xv[i] = by[u][i] -
                  (be[u][i * 3 + 0] * xn[0] + be[u][i * 3 + 1] * xn[1] + be[u][i * 3 + 2] * xn[2]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          s.C(3 * g + i) = 2.0 * xv[i] - bc[u][i];
          xn[i] = xv[i];
        }
      }
      bload(u, g - PD);
    }
  }
}

// psibar_k(x) = f (step window k) . c for every step; Du(x) += f sum_i w_i (stop_i . c)
template <typename T>
__device__ void ray_outputs(const RayParams &rp, const RayState &s, int x, double f,
                            const double *wv, const int *__restrict__ step_g0,
                            const double *__restrict__ step_w, const double *__restrict__ stop_w,
                            T *__restrict__ psibar, double *__restrict__ Du) {
  const int G = rp.G;
  for (int k = 0; k < rp.n_steps; ++k) {
    const int g0 = step_g0[k];
    const double *sw = step_w + size_t(k) * rp.ng_step * 3;
    double acc = 0.0;
    for (int t = 0; t < rp.ng_step * 3; ++t) acc += sw[t] * s.C(3 * g0 + t);
    psibar[size_t(k) * rp.n + x] = T(f * acc);
  }
  double du = 0.0;
  for (int i = 0; i < rp.n_mat; ++i) {
    const double *sw = stop_w + size_t(i) * 3 * G;
    double acc = 0.0;
    for (int e = 0; e < 3 * G; ++e) acc += sw[e] * s.C(e);
    du += wv[i] * acc;
  }
  Du[x] += f * du;   // beams of a joint context add up, one launch after the other
}

__device__ __forceinline__ int n_sub_of(double len, double h_max) {
  return max(1, int(ceil(len / h_max - 1e-9)));
}

template <typename T>
__global__ __launch_bounds__(64) void k_raytrace(
    RayParams rp, RayGeom geo, int ray0, int nray, const int *__restrict__ rays,
    const double *__restrict__ ray_f, const double *__restrict__ w,
    const double *__restrict__ Adiag, const double *__restrict__ Aup,
    const double *__restrict__ Alo, const double *__restrict__ mass,
    const double *__restrict__ c0, const int *__restrict__ step_g0,
    const double *__restrict__ step_w, const double *__restrict__ stop_w,
    double *__restrict__ scratch, size_t B, T *__restrict__ psibar, double *__restrict__ Du,
    Ctl *__restrict__ ctl) {
  const int lr = blockIdx.x * blockDim.x + threadIdx.x;   // ray within the batch
  if (lr >= nray) return;
  const int ray = ray0 + lr;
  const int G = rp.G;
  RayState s{scratch + lr, scratch + size_t(3) * G * B + lr, scratch + size_t(6) * G * B + lr,
             scratch + size_t(15) * G * B + lr, scratch + size_t(24) * G * B + lr, B};
  for (int e = 0; e < 3 * G; ++e) s.C(e) = c0[e];
  const double m[3] = {mass[0], mass[1], mass[2]};
  const double f = ray_f[ray];
  double wv[kMaxMat];
  if (rp.axis >= 0) {
    // a grid row: two equal halves per cell, outputs at the midpoints
    const double h = rp.half / rp.n_half, hh = 0.5 * h;
    for (int ci = 0; ci < rp.row_len; ++ci) {
      const int cell = rp.sign > 0 ? ci : rp.row_len - 1 - ci;
      const int x = rays[ray] + cell * rp.row_stride;
      for (int i = 0; i < rp.n_mat; ++i) wv[i] = w[size_t(i) * rp.n + x];
      factorise(rp, s, wv, Adiag, Aup, Alo, m, hh);
      for (int sub = 0; sub < rp.n_half; ++sub) cn_substep(rp, s, m);
      ray_outputs<T>(rp, s, x, f, wv, step_g0, step_w, stop_w, psibar, Du);
      for (int sub = 0; sub < rp.n_half; ++sub) cn_substep(rp, s, m);
    }
    atomicAdd(&ctl->rt_substeps, (unsigned long long)(2 * rp.n_half) * rp.row_len);
    atomicAdd(&ctl->rt_factors, (unsigned long long)rp.row_len);
    return;
  }
  unsigned long long n_cn = 0, n_fac = 0;
  // oblique ray from the domain entry to the centre of its target cell
  const int xt = rays[ray];
  const int n3[3] = {geo.nx, geo.ny, geo.nz};
  const int dims = geo.dim;
  int it[3] = {xt % geo.nx, (xt / geo.nx) % geo.ny, xt / (geo.nx * geo.ny)};
  double xc[3];
  for (int d = 0; d < 3; ++d) xc[d] = (it[d] + 0.5) * geo.D[d];
  if (dims == 2) xc[2] = 0.0;
  double t_in = -1e300;
  for (int d = 0; d < dims; ++d)
    if (geo.om[d] != 0.0) {
      const double t1 = (0.0 - xc[d]) / geo.om[d], t2 = (geo.L[d] - xc[d]) / geo.om[d];
      t_in = fmax(t_in, fmin(t1, t2));
    }
  // index of the next face plane crossed along each axis (planes j D_d, j = 0..n_d)
  int jn[3] = {-1, -1, -1};
  for (int d = 0; d < dims; ++d) {
    if (geo.om[d] == 0.0) continue;
    if (geo.om[d] > 0.0) {
      int j = 0;
      while (j <= n3[d] && (j * geo.D[d] - xc[d]) / geo.om[d] <= t_in) ++j;
      jn[d] = j;
    } else {
      int j = n3[d];
      while (j >= 0 && (j * geo.D[d] - xc[d]) / geo.om[d] <= t_in) --j;
      jn[d] = j;
    }
  }
  double a = t_in;
  int guard = 0;
  const int max_chords = 2 * (geo.nx + geo.ny + geo.nz) + 8;
  while (a < 0.0 && guard++ < max_chords) {
    double b = 0.0;
    for (int d = 0; d < dims; ++d) {
      if (geo.om[d] == 0.0 || jn[d] < 0 || jn[d] > n3[d]) continue;
      const double t = (jn[d] * geo.D[d] - xc[d]) / geo.om[d];
      if (t < b) b = t;
    }
    for (int d = 0; d < dims; ++d) {
      if (geo.om[d] == 0.0 || jn[d] < 0 || jn[d] > n3[d]) continue;
      const double t = (jn[d] * geo.D[d] - xc[d]) / geo.om[d];
      if (t == b) jn[d] += geo.om[d] > 0.0 ? 1 : -1;
    }
    if (b > a) {
      // the chord's cell: the cell of its midpoint (clamped to the grid)
      int ic[3] = {0, 0, 0};
      for (int d = 0; d < dims; ++d) {
        const double p = xc[d] + 0.5 * (a + b) * geo.om[d];
        ic[d] = min(max(int(floor(p / geo.D[d])), 0), n3[d] - 1);
      }
      const int cell = (ic[2] * geo.ny + ic[1]) * geo.nx + ic[0];
      for (int i = 0; i < rp.n_mat; ++i) wv[i] = w[size_t(i) * rp.n + cell];
      double tf = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double cc = d < dims ? (ic[d] + 0.5) * geo.D[d] : 0.0;
        tf += (cc - xc[d]) * geo.om[d];
      }
      double lens[2];
      int np = 1;
      if (a < tf && tf < b) {
        lens[0] = tf - a;
        lens[1] = b - tf;
        np = 2;
      } else {
        lens[0] = b - a;
      }
      for (int q = 0; q < np; ++q) {
        const int ns = n_sub_of(lens[q], rp.h_max);
        const double hh = 0.5 * (lens[q] / ns);
        factorise(rp, s, wv, Adiag, Aup, Alo, m, hh);
        for (int sub = 0; sub < ns; ++sub) cn_substep(rp, s, m);
        n_cn += ns;
        ++n_fac;
      }
    }
    a = b;
  }
  for (int i = 0; i < rp.n_mat; ++i) wv[i] = w[size_t(i) * rp.n + xt];
  ray_outputs<T>(rp, s, xt, f, wv, step_g0, step_w, stop_w, psibar, Du);
  atomicAdd(&ctl->rt_substeps, n_cn);
  atomicAdd(&ctl->rt_factors, n_fac);
}

}  // namespace

template <typename T>
void launch_raytrace(const RayParams &rp, const RayGeom &geo, const int *rays,
                     const double *ray_f, const double *w, const double *Adiag,
                     const double *Aup, const double *Alo, const double *mass, const double *c0,
                     const int *step_g0, const double *step_w, const double *stop_w,
                     double *scratch, size_t batch, T *psibar, double *Du, Ctl *ctl,
                     hipStream_t st) {
  for (int r0 = 0; r0 < rp.n_rays; r0 += int(batch)) {
    const int nr = std::min<int>(int(batch), rp.n_rays - r0);
    k_raytrace<T><<<(nr + 63) / 64, 64, 0, st>>>(rp, geo, r0, nr, rays, ray_f, w, Adiag, Aup,
                                                  Alo, mass, c0, step_g0, step_w, stop_w,
                                                  scratch, batch, psibar, Du, ctl);
  }
}

template void launch_raytrace<double>(const RayParams &, const RayGeom &, const int *,
                                      const double *, const double *, const double *,
                                      const double *, const double *, const double *,
                                      const double *, const int *, const double *,
                                      const double *, double *, size_t, double *, double *,
                                      Ctl *, hipStream_t);
template void launch_raytrace<float>(const RayParams &, const RayGeom &, const int *,
                                     const double *, const double *, const double *,
                                     const double *, const double *, const double *,
                                     const double *, const int *, const double *,
                                     const double *, double *, size_t, float *, double *,
                                     Ctl *, hipStream_t);

}  // namespace dlra
