// Uncollided ray tracer (Sec. 3.2): DG-P2 in energy, Crank-Nicolson in depth.
//
// A ray is either a grid row along an axis-aligned beam (every midpoint of
// the row lies on it; outputs after the first half of each cell) or, for an
// oblique beam, the segment from the domain entry to one target cell centre
// (output at its end).  The path is cut at cell faces and, inside every
// traversed cell, at the foot of the perpendicular from that cell's centre;
// each piece of length L takes ceil(L / h_max) equal Crank-Nicolson substeps
// with the material of its cell.  Oblique pieces are generated on the fly by
// a traversal of the face planes in order of the ray parameter, with the
// plane crossings computed as t = (j D_d - x_d) / Omega_d.
//
// Per piece the block-tridiagonal matrix M - h/2 A(x), A(x) = sum_i w_i(x) A_i,
// is factorised once; a substep then solves (M - h/2 A) y = M c and sets
// c <- 2 y - c, which equals (M - h/2 A)^{-1} (M + h/2 A) c, so the mixture
// blocks are not formed again per substep.
//
// Up to kRayWaveGroups groups one wave marches one ray: lane l holds groups
// 2l and 2l+1.  The odd groups are eliminated inside each lane, then the even
// groups by parallel cyclic reduction across the lanes (level j pairs lanes
// 2^j apart; after ceil(log2(G/2)) levels every equation stands alone).  The
// multipliers of a piece stay on chip (levels 0-1 in registers, 2-5 in the
// wave's LDS rows) and each substep replays them on the right-hand side, so
// a substep touches no global memory.
//
// Beyond that one thread marches one ray with a sequential block LU from the
// lowest group (Dinv_g, F_g = Dinv_g L_g, E_g = Dinv_g U_g): y_g = Dinv_g M c_g
// - F_g y_{g-1} forward, x_g = y_g - E_g x_{g+1} backward, its state in a
// scratch area laid out [element][ray] so that a wave's accesses coalesce, the
// loads of the next kRayAhead groups kept in flight.
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

// Calls piece(cell, length) for every piece of the oblique ray that ends at
// the centre of cell xt, in the order of flight.
template <typename F>
__device__ __forceinline__ void oblique_pieces(const RayGeom &geo, int xt, F &&piece) {
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
      double tf = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double cc = d < dims ? (ic[d] + 0.5) * geo.D[d] : 0.0;
        tf += (cc - xc[d]) * geo.om[d];
      }
      if (a < tf && tf < b) {
        piece(cell, tf - a);
        piece(cell, b - tf);
      } else {
        piece(cell, b - a);
      }
    }
    a = b;
  }
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
  oblique_pieces(geo, xt, [&](int cell, double len) {
    for (int i = 0; i < rp.n_mat; ++i) wv[i] = w[size_t(i) * rp.n + cell];
    const int ns = n_sub_of(len, rp.h_max);
    const double hh = 0.5 * (len / ns);
    factorise(rp, s, wv, Adiag, Aup, Alo, m, hh);
    for (int sub = 0; sub < ns; ++sub) cn_substep(rp, s, m);
    n_cn += ns;
    ++n_fac;
  });
  for (int i = 0; i < rp.n_mat; ++i) wv[i] = w[size_t(i) * rp.n + xt];
  ray_outputs<T>(rp, s, xt, f, wv, step_g0, step_w, stop_w, psibar, Du);
  atomicAdd(&ctl->rt_substeps, n_cn);
  atomicAdd(&ctl->rt_factors, n_fac);
}

// ------------------------------------------------------------ one wave per ray

// v of lane src (ds_bpermute, two 32-bit halves)
__device__ __forceinline__ double lane_read(double v, int src) {
  const int a = src << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// v of lane - 1 (wave_shr:1) or lane + 1 (wave_shl:1) by DPP; 0 at the ends
template <int CTRL>
__device__ __forceinline__ double lane_shift1(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// out = v of lane (lane + delta).  Where that lane is outside the wave the
// value is some finite lane's: every use multiplies it by a coupling block
// that is exactly zero there (no row below group 0 or above group G - 1),
// so no select is needed.  Distance 1 goes through DPP, longer ones through
// ds_bpermute.
template <int N>
__device__ __forceinline__ void from_lane(const double *v, double *out, int lane, int delta) {
  if (delta == -1) {
#pragma unroll
    for (int t = 0; t < N; ++t) out[t] = lane_shift1<0x138>(v[t]);
  } else if (delta == 1) {
#pragma unroll
    for (int t = 0; t < N; ++t) out[t] = lane_shift1<0x130>(v[t]);
  } else {
    const int sl = (lane + delta) & 63;
#pragma unroll
    for (int t = 0; t < N; ++t) out[t] = lane_read(v[t], sl);
  }
}

// 3 x 3 row-major helpers
__device__ __forceinline__ void mul3(const double *A, const double *B, double *C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}
__device__ __forceinline__ void neg_mul3(const double *A, const double *B, double *C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = -(A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j]);
}
__device__ __forceinline__ void sub_mul3(const double *A, const double *B, double *C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] -= A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}
__device__ __forceinline__ void add_mv3(const double *A, const double *x, double *y) {
#pragma unroll
  for (int i = 0; i < 3; ++i) y[i] += A[i * 3] * x[0] + A[i * 3 + 1] * x[1] + A[i * 3 + 2] * x[2];
}

constexpr int kPcrLevels = 6;      // 64 lanes
constexpr int kPcrRegLevels = 2;   // levels whose multipliers stay in registers; the
                                   // rest live in LDS, [level][alpha|gamma][entry][lane]
constexpr int kPcrLdsRows = (kPcrLevels - kPcrRegLevels) * 2 * 9;

// Blocks of row g of M - hh A(w): D (diagonal), L (to g - 1), U (to g + 1);
// rows past the last group are identity rows with no coupling.
__device__ __forceinline__ void form_row(int G, int n_mat, int g, const double *__restrict__ wcell,
                                         size_t wstride, const double *__restrict__ Adiag,
                                         const double *__restrict__ Aup,
                                         const double *__restrict__ Alo, const double m[3],
                                         double hh, double D[9], double L[9], double U[9]) {
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    D[t] = 0.0;
    L[t] = 0.0;
    U[t] = 0.0;
  }
  if (g >= G) {
    D[0] = D[4] = D[8] = 1.0;
    return;
  }
  for (int i = 0; i < n_mat; ++i) {
    const double wi = wcell[size_t(i) * wstride];
    const size_t o = (size_t(i) * G + g) * 9;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      D[t] += wi * Adiag[o + t];
      L[t] += wi * Alo[o + t];
      U[t] += wi * Aup[o + t];
    }
  }
  const bool has_lo = g > 0, has_up = g + 1 < G;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    D[t] = -hh * D[t];
    L[t] = has_lo ? -hh * L[t] : 0.0;
    U[t] = has_up ? -hh * U[t] : 0.0;
  }
  D[0] += m[0];
  D[4] += m[1];
  D[8] += m[2];
}

// The factorisation of one piece, held by each lane for its two groups.
struct WaveLU {
  double a0[9], g0[9];            // even row: multipliers of the odd rows 2l-1 and 2l+1
  double Dio[9], Fo[9], Eo[9];    // odd row 2l+1: inverse, inverse x L, inverse x U
  double al[kPcrRegLevels][9];    // reduction level j: multiplier of lane l - 2^j
  double ga[kPcrRegLevels][9];    //                    multiplier of lane l + 2^j
  double Dif[9];                  // inverse of the fully reduced even row
  double (*lv)[64];               // LDS rows of the levels from kPcrRegLevels on

  // multiplier storage of level j (which: 0 alpha, 1 gamma)
  __device__ __forceinline__ void put(int j, int which, int lane, const double *v) {
    if (j < kPcrRegLevels) {
#pragma unroll
      for (int t = 0; t < 9; ++t) (which ? ga[j] : al[j])[t] = v[t];
    } else {
#pragma unroll
      for (int t = 0; t < 9; ++t) lv[((j - kPcrRegLevels) * 2 + which) * 9 + t][lane] = v[t];
    }
  }
  __device__ __forceinline__ void get(int j, int which, int lane, double *v) const {
    if (j < kPcrRegLevels) {
#pragma unroll
      for (int t = 0; t < 9; ++t) v[t] = (which ? ga[j] : al[j])[t];
    } else {
#pragma unroll
      for (int t = 0; t < 9; ++t) v[t] = lv[((j - kPcrRegLevels) * 2 + which) * 9 + t][lane];
    }
  }

  __device__ __forceinline__ void factorise(int G, int n_mat, int nlev, int lane,
                                            const double *__restrict__ wcell, size_t wstride,
                                            const double *__restrict__ Adiag,
                                            const double *__restrict__ Aup,
                                            const double *__restrict__ Alo, const double m[3],
                                            double hh) {
    double De[9], Le[9], Ue[9], Do[9], Lo[9], Uo[9], t[9], Ln[9], Un[9];
    // odd row 2l+1 couples to the even rows 2l (this lane) and 2l+2 (the next)
    form_row(G, n_mat, 2 * lane + 1, wcell, wstride, Adiag, Aup, Alo, m, hh, Do, Lo, Uo);
    inv3(Do, Dio);
    mul3(Dio, Lo, Fo);
    mul3(Dio, Uo, Eo);
    form_row(G, n_mat, 2 * lane, wcell, wstride, Adiag, Aup, Alo, m, hh, De, Le, Ue);
    // eliminate odd row 2l-1 (previous lane) and 2l+1 from even row 2l
    from_lane<9>(Dio, t, lane, -1);
    neg_mul3(Le, t, a0);
    from_lane<9>(Eo, t, lane, -1);
    sub_mul3(Le, t, De);
    from_lane<9>(Fo, t, lane, -1);
    neg_mul3(Le, t, Ln);
    neg_mul3(Ue, Dio, g0);
    sub_mul3(Ue, Fo, De);
    neg_mul3(Ue, Eo, Un);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      Le[q] = Ln[q];
      Ue[q] = Un[q];
    }
    // cyclic reduction of the even rows: lane l couples to l -+ s
#pragma unroll
    for (int j = 0; j < kPcrLevels; ++j) {
      const int s = 1 << j;
      if (j < nlev) {
        double Di[9], P[9], Q[9];
        inv3(De, Di);
        mul3(Di, Le, P);
        mul3(Di, Ue, Q);
        double mu[9];
        from_lane<9>(Di, t, lane, -s);
        neg_mul3(Le, t, mu);
        put(j, 0, lane, mu);
        from_lane<9>(Q, t, lane, -s);
        sub_mul3(Le, t, De);
        from_lane<9>(P, t, lane, -s);
        neg_mul3(Le, t, Ln);
        from_lane<9>(Di, t, lane, s);
        neg_mul3(Ue, t, mu);
        put(j, 1, lane, mu);
        from_lane<9>(P, t, lane, s);
        sub_mul3(Ue, t, De);
        from_lane<9>(Q, t, lane, s);
        neg_mul3(Ue, t, Un);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          Le[q] = Ln[q];
          Ue[q] = Un[q];
        }
      }
    }
    inv3(De, Dif);
  }

  // c <- 2 (M - hh A)^{-1} M c - c for this lane's rows (ce: 2l, co: 2l+1)
  __device__ __forceinline__ void substep(int nlev, int lane, const double m[3], double ce[3],
                                          double co[3]) const {
    const double ro[3] = {m[0] * co[0], m[1] * co[1], m[2] * co[2]};
    double r[3] = {m[0] * ce[0], m[1] * ce[1], m[2] * ce[2]};
    double t[3], u[3];
    from_lane<3>(ro, t, lane, -1);
    add_mv3(a0, t, r);
    add_mv3(g0, ro, r);
#pragma unroll
    for (int j = 0; j < kPcrLevels; ++j) {
      if (j < nlev) {
        const int s = 1 << j;
        double mu[9];
        from_lane<3>(r, t, lane, -s);
        from_lane<3>(r, u, lane, s);
        get(j, 0, lane, mu);
        add_mv3(mu, t, r);
        get(j, 1, lane, mu);
        add_mv3(mu, u, r);
      }
    }
    double xe[3] = {0.0, 0.0, 0.0}, xo[3] = {0.0, 0.0, 0.0};
    add_mv3(Dif, r, xe);
    from_lane<3>(xe, t, lane, 1);
    add_mv3(Dio, ro, xo);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      xo[i] -= (Fo[i * 3] * xe[0] + Fo[i * 3 + 1] * xe[1] + Fo[i * 3 + 2] * xe[2]) +
               (Eo[i * 3] * t[0] + Eo[i * 3 + 1] * t[1] + Eo[i * 3 + 2] * t[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ce[i] = 2.0 * xe[i] - ce[i];
      co[i] = 2.0 * xo[i] - co[i];
    }
  }
};

// psibar_k(x) = f (step window k) . c for every step (lanes over k) and
// Du(x) += f sum_i w_i (stop_i . c) (wave sum); cl holds 3G doubles of LDS
constexpr int kOutSteps = 4;   // step tables a lane forms at a time

template <typename T>
__device__ __forceinline__ void wave_outputs(const RayParams &rp, int lane, const double ce[3],
                                             const double co[3], int x, double f,
                                             const double *__restrict__ w,
                                             const int *__restrict__ step_g0,
                                             const double *__restrict__ step_w,
                                             const double *__restrict__ stop_w, double *cl,
                                             T *__restrict__ psibar, double *__restrict__ Du) {
  const int G = rp.G, ge = 2 * lane, go = ge + 1;
  double du = 0.0;
  for (int i = 0; i < rp.n_mat; ++i) {
    const double *sw = stop_w + size_t(i) * 3 * G;
    double acc = 0.0;
    if (ge < G) acc += sw[3 * ge] * ce[0] + sw[3 * ge + 1] * ce[1] + sw[3 * ge + 2] * ce[2];
    if (go < G) acc += sw[3 * go] * co[0] + sw[3 * go + 1] * co[1] + sw[3 * go + 2] * co[2];
    du += w[size_t(i) * rp.n + x] * acc;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) du += lane_read(du, lane ^ off);
  if (ge < G)
    for (int k = 0; k < 3; ++k) cl[3 * ge + k] = ce[k];
  if (go < G)
    for (int k = 0; k < 3; ++k) cl[3 * go + k] = co[k];
  __syncthreads();
  // lane l takes the steps l, l + 64, ...: kOutSteps of them at a time, with
  // their window offsets and weights loaded together (same sums as a step at
  // a time: t ascending from zero)
  const int nw = rp.ng_step * 3;
  for (int k0 = 0; k0 < rp.n_steps; k0 += 64 * kOutSteps) {
    const double *sw[kOutSteps];
    const double *cc[kOutSteps];
    double acc[kOutSteps];
#pragma unroll
    for (int u = 0; u < kOutSteps; ++u) {
      const int k = min(k0 + 64 * u + lane, rp.n_steps - 1);
      sw[u] = step_w + size_t(k) * nw;
      cc[u] = cl + 3 * step_g0[k];
      acc[u] = 0.0;
    }
#pragma unroll 4
    for (int t = 0; t < nw; ++t)
#pragma unroll
      for (int u = 0; u < kOutSteps; ++u) acc[u] += sw[u][t] * cc[u][t];
#pragma unroll
    for (int u = 0; u < kOutSteps; ++u) {
      const int k = k0 + 64 * u + lane;
      if (k < rp.n_steps) psibar[size_t(k) * rp.n + x] = T(f * acc[u]);
    }
  }
  if (lane == 0) Du[x] += f * du;   // beams of a joint context add up, one launch after the other
  __syncthreads();
}

// One block of one wave per ray; blocks 8 apart (one XCD) take consecutive rays.
template <typename T>
__global__ __launch_bounds__(64) void k_raytrace_wave(
    RayParams rp, RayGeom geo, int nray, const int *__restrict__ rays,
    const double *__restrict__ ray_f, const double *__restrict__ w,
    const double *__restrict__ Adiag, const double *__restrict__ Aup,
    const double *__restrict__ Alo, const double *__restrict__ mass,
    const double *__restrict__ c0, const int *__restrict__ step_g0,
    const double *__restrict__ step_w, const double *__restrict__ stop_w,
    T *__restrict__ psibar, double *__restrict__ Du, Ctl *__restrict__ ctl) {
  __shared__ double cl[3 * kRayWaveGroups];
  __shared__ double lv[kPcrLdsRows][64];
  const int per = (nray + 7) >> 3;
  const int ray = int(blockIdx.x & 7) * per + int(blockIdx.x >> 3);
  if (ray >= nray) return;   // the whole block
  const int lane = threadIdx.x;
  const int G = rp.G;
  int nlev = 0;
  while ((1 << nlev) < (G + 1) / 2) ++nlev;
  const double m[3] = {mass[0], mass[1], mass[2]};
  const double f = ray_f[ray];
  double ce[3], co[3];
  for (int k = 0; k < 3; ++k) {
    ce[k] = 2 * lane < G ? c0[6 * lane + k] : 0.0;
    co[k] = 2 * lane + 1 < G ? c0[6 * lane + 3 + k] : 0.0;
  }
  WaveLU lu;
  lu.lv = lv;
  if (rp.axis >= 0) {
    // a grid row: two equal halves per cell, outputs at the midpoints
    const double h = rp.half / rp.n_half, hh = 0.5 * h;
    for (int ci = 0; ci < rp.row_len; ++ci) {
      const int cell = rp.sign > 0 ? ci : rp.row_len - 1 - ci;
      const int x = rays[ray] + cell * rp.row_stride;
      lu.factorise(G, rp.n_mat, nlev, lane, w + x, size_t(rp.n), Adiag, Aup, Alo, m, hh);
      for (int sub = 0; sub < rp.n_half; ++sub) lu.substep(nlev, lane, m, ce, co);
      wave_outputs<T>(rp, lane, ce, co, x, f, w, step_g0, step_w, stop_w, cl, psibar, Du);
      for (int sub = 0; sub < rp.n_half; ++sub) lu.substep(nlev, lane, m, ce, co);
    }
    if (lane == 0) {
      atomicAdd(&ctl->rt_substeps, (unsigned long long)(2 * rp.n_half) * rp.row_len);
      atomicAdd(&ctl->rt_factors, (unsigned long long)rp.row_len);
    }
    return;
  }
  unsigned long long n_cn = 0, n_fac = 0;
  const int xt = rays[ray];
  oblique_pieces(geo, xt, [&](int cell, double len) {
    const int ns = n_sub_of(len, rp.h_max);
    const double hh = 0.5 * (len / ns);
    lu.factorise(G, rp.n_mat, nlev, lane, w + cell, size_t(rp.n), Adiag, Aup, Alo, m, hh);
    for (int sub = 0; sub < ns; ++sub) lu.substep(nlev, lane, m, ce, co);
    n_cn += ns;
    ++n_fac;
  });
  wave_outputs<T>(rp, lane, ce, co, xt, f, w, step_g0, step_w, stop_w, cl, psibar, Du);
  if (lane == 0) {
    atomicAdd(&ctl->rt_substeps, n_cn);
    atomicAdd(&ctl->rt_factors, n_fac);
  }
}

}  // namespace

template <typename T>
void launch_raytrace(const RayParams &rp, const RayGeom &geo, const int *rays,
                     const double *ray_f, const double *w, const double *Adiag,
                     const double *Aup, const double *Alo, const double *mass, const double *c0,
                     const int *step_g0, const double *step_w, const double *stop_w,
                     double *scratch, size_t batch, T *psibar, double *Du, Ctl *ctl,
                     hipStream_t st) {
  if (rp.n_rays <= 0) return;
  if (rp.G <= kRayWaveGroups) {
    const int per = (rp.n_rays + 7) / 8;
    k_raytrace_wave<T><<<8 * per, 64, 0, st>>>(rp, geo, rp.n_rays, rays, ray_f, w, Adiag, Aup,
                                                Alo, mass, c0, step_g0, step_w, stop_w, psibar,
                                                Du, ctl);
    return;
  }
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
