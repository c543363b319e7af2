// Kernels over the n cells: K-step stencil stages, stencil projections,
// Gram reductions and tall-skinny updates (gfx950, wave64).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace dlra {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxPartialBlocks = 240;

__device__ __forceinline__ void cell_coords(const GridDev &g, int x, int c[3]) {
  c[0] = x % g.nx;
  int t = x / g.nx;
  c[1] = t % g.ny;
  c[2] = t / g.ny;
}

// second-order one-sided difference of v(x) = s(x) W(x, col) along d
// (zero ghost cells); kind 0: backward (3v_i - 4v_{i-1} + v_{i-2}),
// kind 1: forward (-3v_i + 4v_{i+1} - v_{i+2}), times 1/(2 Delta_d).
template <typename T>
__device__ __forceinline__ T stencil_diff(const GridDev &g, const T *__restrict__ s,
                                          const T *__restrict__ col, int x, const int c[3],
                                          int d, int kind) {
  const int size[3] = {g.nx, g.ny, g.nz};
  const int stride = d == 0 ? 1 : (d == 1 ? g.nx : g.nx * g.ny);
  const T v0 = s[x] * col[x];
  T v1 = T(0), v2 = T(0);
  if (kind == 0) {
    if (c[d] >= 1) v1 = s[x - stride] * col[x - stride];
    if (c[d] >= 2) v2 = s[x - 2 * stride] * col[x - 2 * stride];
    return (T(3) * v0 - T(4) * v1 + v2) * T(g.inv2h[d]);
  }
  if (c[d] + 1 < size[d]) v1 = s[x + stride] * col[x + stride];
  if (c[d] + 2 < size[d]) v2 = s[x + 2 * stride] * col[x + 2 * stride];
  return (T(-3) * v0 + T(4) * v1 - v2) * T(g.inv2h[d]);
}

// ------------------------------------------------------------------ 1/S
template <typename T>
__global__ void k_inverse_stop(GridDev g, const T *__restrict__ w, int n_mat,
                               const double *__restrict__ Si, T *__restrict__ s, Ctl *ctl) {
  int x = blockIdx.x * kBlock + threadIdx.x;
  if (x >= g.n) return;
  double st = 0.0;
  for (int i = 0; i < n_mat; ++i) st += double(w[size_t(i) * g.n + x]) * Si[i];
  if (!(st > 0.0)) {
    atomicOr(&ctl->flags, kFlagStop);
    st = 1.0;
  }
  s[x] = T(1.0 / st);
}

// ------------------------------------------------------------------ K-step stage
constexpr int kTC = 32;   // cells per tile of the reductions

template <typename T, int kTS>
__global__ __launch_bounds__(kBlock) void k_kstep_stage(GridDev g, const T *__restrict__ s,
                                                       const T *__restrict__ W,
                                                       const T *__restrict__ K0,
                                                       T *__restrict__ out, int ld, int r,
                                                       const double *__restrict__ B, int ldb,
                                                       double coef) {
  extern __shared__ unsigned char smem_raw[];
  T *D = reinterpret_cast<T *>(smem_raw);        // [kTS][ndk][r]
  const int ndk = 2 * g.dim;
  const int x0 = blockIdx.x * kTS;
  const int tid = threadIdx.x;
  // phase 1: difference vectors of the tile
  const int total = kTS * ndk * r;
  for (int idx = tid; idx < total; idx += kBlock) {
    int c = idx % kTS;
    int rest = idx / kTS;
    int k = rest % r;
    int dk = rest / r;
    int x = x0 + c;
    T v = T(0);
    if (x < g.n) {
      int cc[3];
      cell_coords(g, x, cc);
      v = stencil_diff(g, s, W + size_t(k) * ld, x, cc, dk >> 1, dk & 1);
    }
    D[(c * ndk + dk) * r + k] = v;
  }
  __syncthreads();
  // phase 2: out(x, j) = K0(x, j) - coef * sum_{dk,k} D(x, dk, k) B_dk(k, j)
  int L = 1;
  while (L < r) L <<= 1;
  const int groups = kBlock / L;
  const int j = tid % L;
  const int grp = tid / L;
  if (j >= r || grp >= groups) return;
  constexpr int kMaxCells = kTS;
  double acc[kMaxCells];
  const int ncell = (kTS + groups - 1 - grp) / groups;
#pragma unroll
  for (int u = 0; u < kMaxCells; ++u) acc[u] = 0.0;
  for (int dk = 0; dk < ndk; ++dk) {
    const double *Bd = B + size_t(dk) * ldb * ldb;
    for (int k = 0; k < r; ++k) {
      const double b = Bd[k + size_t(j) * ldb];
#pragma unroll
      for (int u = 0; u < kMaxCells; ++u) {
        if (u < ncell) {
          int c = grp + u * groups;
          acc[u] += double(D[(c * ndk + dk) * r + k]) * b;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kMaxCells; ++u) {
    if (u < ncell) {
      int x = x0 + grp + u * groups;
      if (x < g.n) {
        size_t o = size_t(j) * ld + x;
        out[o] = T(double(K0[o]) - coef * acc[u]);
      }
    }
  }
}

// ------------------------------------------------------------------ reductions
template <typename Acc, int kMaxOut>
struct OutAcc {
  Acc v[kMaxOut];
};

// Stencil projections: for one dk at a time.
template <typename T, typename Acc>
__global__ __launch_bounds__(kBlock) void k_stencil_projection(GridDev g, const T *__restrict__ s,
                                                              const T *__restrict__ X, int ld,
                                                              int p, double *__restrict__ partial) {
  extern __shared__ unsigned char smem_raw[];
  T *Xs = reinterpret_cast<T *>(smem_raw);   // [kTC][p]
  T *Ds = Xs + kTC * p;                      // [kTC][p]
  const int ndk = 2 * g.dim;
  const int tid = threadIdx.x;
  const int pp = p * p;
  const int nout = (pp + kBlock - 1) / kBlock;
  const int ntile = (g.n + kTC - 1) / kTC;
  for (int dk = 0; dk < ndk; ++dk) {
    Acc acc[40];
    for (int u = 0; u < 40; ++u) acc[u] = Acc(0);
    for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
      const int x0 = t * kTC;
      __syncthreads();
      for (int idx = tid; idx < kTC * p; idx += kBlock) {
        int c = idx % kTC, a = idx / kTC;
        int x = x0 + c;
        T xv = T(0), dv = T(0);
        if (x < g.n) {
          int cc[3];
          cell_coords(g, x, cc);
          xv = X[size_t(a) * ld + x];
          dv = stencil_diff(g, s, X + size_t(a) * ld, x, cc, dk >> 1, dk & 1);
        }
        Xs[c * p + a] = xv;
        Ds[c * p + a] = dv;
      }
      __syncthreads();
      for (int u = 0; u < nout; ++u) {
        int o = tid + u * kBlock;
        if (o < pp) {
          int a = o % p, b = o / p;
          Acc sum = Acc(0);
          for (int c = 0; c < kTC; ++c) sum += Acc(Xs[c * p + a]) * Acc(Ds[c * p + b]);
          acc[u] += sum;
        }
      }
    }
    for (int u = 0; u < nout; ++u) {
      int o = tid + u * kBlock;
      if (o < pp) partial[(size_t(blockIdx.x) * ndk + dk) * pp + o] = double(acc[u]);
    }
  }
}

template <typename T>
struct YMat {
  const T *Y;
  int ld;
  __device__ T operator()(int x, int c) const { return Y[size_t(c) * ld + x]; }
};
template <typename T>
struct YSrc {
  const T *w;
  const T *psi;
  int n;
  __device__ T operator()(int x, int i) const { return w[size_t(i) * n + x] * psi[x]; }
};
template <typename T>
struct WOne {
  __device__ T operator()(int) const { return T(1); }
};
template <typename T>
struct WMatS {
  const T *w;
  const T *s;
  __device__ T operator()(int x) const { return w[x] * s[x]; }
};

// G(a, c) = sum_x X(x, a) wt(x) Y(x, c) partial sums
template <typename T, typename Acc, typename YF, typename WF>
__global__ __launch_bounds__(kBlock) void k_gram(int n, const T *__restrict__ X, int ldx, int p,
                                                YF yf, int q, WF wf,
                                                double *__restrict__ partial) {
  extern __shared__ unsigned char smem_raw[];
  T *Xs = reinterpret_cast<T *>(smem_raw);   // [kTC][p]
  T *Ys = Xs + kTC * p;                      // [kTC][q]
  const int tid = threadIdx.x;
  const int pq = p * q;
  const int nout = (pq + kBlock - 1) / kBlock;
  const int ntile = (n + kTC - 1) / kTC;
  Acc acc[40];
  for (int u = 0; u < 40; ++u) acc[u] = Acc(0);
  for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
    const int x0 = t * kTC;
    __syncthreads();
    for (int idx = tid; idx < kTC * p; idx += kBlock) {
      int c = idx % kTC, a = idx / kTC;
      int x = x0 + c;
      Xs[c * p + a] = x < n ? T(X[size_t(a) * ldx + x] * wf(x)) : T(0);
    }
    for (int idx = tid; idx < kTC * q; idx += kBlock) {
      int c = idx % kTC, b = idx / kTC;
      int x = x0 + c;
      Ys[c * q + b] = x < n ? yf(x, b) : T(0);
    }
    __syncthreads();
    for (int u = 0; u < nout; ++u) {
      int o = tid + u * kBlock;
      if (o < pq) {
        int a = o % p, b = o / p;
        Acc sum = Acc(0);
        for (int c = 0; c < kTC; ++c) sum += Acc(Xs[c * p + a]) * Acc(Ys[c * q + b]);
        acc[u] += sum;
      }
    }
  }
  for (int u = 0; u < nout; ++u) {
    int o = tid + u * kBlock;
    if (o < pq) partial[size_t(blockIdx.x) * pq + o] = double(acc[u]);
  }
}

__global__ void k_reduce_partials(const double *__restrict__ partial, int nblocks, int elems,
                                  double *__restrict__ out) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= elems) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[size_t(b) * elems + e];
  out[e] = s;
}

// scatter a reduced p x q block into a col-major matrix with leading dim ldc
__global__ void k_scatter(const double *__restrict__ src, int p, int q, int nblk,
                          double *__restrict__ dst, int ldc, size_t dst_stride) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  int pq = p * q;
  if (e >= pq * nblk) return;
  int blk = e / pq, o = e % pq;
  int a = o % p, b = o / p;
  dst[blk * dst_stride + a + size_t(b) * ldc] = src[e];
}

template <typename T>
__global__ void k_sumsq(int n, const T *__restrict__ X, int ld, int q, double *partial) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int c = 0; c < q; ++c)
    for (int x = blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
      double v = double(X[size_t(c) * ld + x]);
      acc += v * v;
    }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ updates
constexpr int kUC = 64;   // cells per update tile

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update(int n, const T *__restrict__ X, int ldx, int p,
                                                  const double *__restrict__ G, int ldg,
                                                  double beta, const T *Y, int ldy,
                                                  double alpha, T *Z,
                                                  int ldz, int q, double *__restrict__ dose,
                                                  const double *__restrict__ dc, double dscale,
                                                  const T *__restrict__ sw, int n_mat,
                                                  const T *__restrict__ spsi,
                                                  const double *__restrict__ sC, int ldsc,
                                                  double sdt) {
  extern __shared__ unsigned char smem_raw[];
  T *Xs = reinterpret_cast<T *>(smem_raw);   // [kUC][p + 1]
  __shared__ double dred[kBlock];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * kUC;
  const int ps = p + 1;
  for (int idx = tid; idx < kUC * p; idx += kBlock) {
    int c = idx % kUC, a = idx / kUC;
    int x = x0 + c;
    Xs[c * ps + a] = x < n ? X[size_t(a) * ldx + x] : T(0);
  }
  __syncthreads();
  const int c = tid % kUC;
  const int cg = tid / kUC;
  const int x = x0 + c;
  double dsum = 0.0;
  if (x < n) {
    double src[kMaxMat];
    if (sw != nullptr) {
      double ps_ = double(spsi[x]);
      for (int i = 0; i < n_mat; ++i) src[i] = sdt * double(sw[size_t(i) * n + x]) * ps_;
    }
    for (int col = cg; col < q; col += kBlock / kUC) {
      double acc = 0.0;
      if (Y != nullptr && alpha != 0.0) acc = alpha * double(Y[size_t(col) * ldy + x]);
      const double *Gc = G + size_t(col) * ldg;
      double xg = 0.0;
      for (int a = 0; a < p; ++a) xg += double(Xs[c * ps + a]) * Gc[a];
      acc += beta * xg;
      if (sw != nullptr)
        for (int i = 0; i < n_mat; ++i) acc += src[i] * sC[col + size_t(i) * ldsc];
      T zv = T(acc);
      Z[size_t(col) * ldz + x] = zv;
      if (dose != nullptr) dsum += double(zv) * dc[col];
    }
  }
  if (dose != nullptr) {
    dred[tid] = dsum;
    __syncthreads();
    if (cg == 0 && x < n) {
      double tot = 0.0;
      for (int u = 0; u < kBlock / kUC; ++u) tot += dred[c + u * kUC];
      dose[x] += dscale * tot;
    }
  }
}

template <typename T>
__global__ void k_zero_cols(int n, T *X, int ld, int c0, int c1) {
  int x = blockIdx.x * kBlock + threadIdx.x;
  if (x >= n) return;
  for (int c = c0; c < c1; ++c) X[size_t(c) * ld + x] = T(0);
}

int partial_blocks(int n, int tile) {
  int nt = (n + tile - 1) / tile;
  return nt < kMaxPartialBlocks ? nt : kMaxPartialBlocks;
}

}  // namespace

// ================================================================== launchers

template <typename T>
void launch_inverse_stop(const GridDev &g, const T *w, int n_mat, const double *Si, T *s,
                         Ctl *ctl, hipStream_t st) {
  k_inverse_stop<T><<<(g.n + kBlock - 1) / kBlock, kBlock, 0, st>>>(g, w, n_mat, Si, s, ctl);
}

template <typename T>
void launch_kstep_stage(const GridDev &g, const T *s, const T *W, const T *K0, T *out, int ld,
                        int r, const double *B, int ldb, double coef, hipStream_t st) {
  constexpr int TS = sizeof(T) == 8 ? 16 : 32;
  size_t shm = size_t(TS) * 2 * g.dim * r * sizeof(T);
  k_kstep_stage<T, TS><<<(g.n + TS - 1) / TS, kBlock, shm, st>>>(g, s, W, K0, out, ld, r, B,
                                                                  ldb, coef);
}

template <typename T, typename Acc>
void launch_stencil_projection(const GridDev &g, const T *s, const T *X, int ld, int p,
                               double *C, int ldc, double *partial, size_t partial_elems,
                               hipStream_t st) {
  const int ndk = 2 * g.dim;
  int nb = partial_blocks(g.n, kTC);
  size_t per = size_t(ndk) * p * p;
  if (size_t(nb + 1) * per > partial_elems) nb = int(partial_elems / per) - 1;
  size_t shm = size_t(2) * kTC * p * sizeof(T);
  k_stencil_projection<T, Acc><<<nb, kBlock, shm, st>>>(g, s, X, ld, p, partial);
  // reduce into the first per elements of the partial area's tail
  double *red = partial + size_t(nb) * per;
  k_reduce_partials<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(partial, nb, int(per), red);
  k_scatter<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(red, p, p, ndk, C, ldc,
                                                            size_t(ldc) * ldc);
}

template <typename T, typename Acc>
void launch_gram(int n, const T *X, int ldx, int p, const T *Y, int ldy, int q, const T *wmat,
                 const T *s, double *G, int ldg, double *partial, size_t partial_elems,
                 hipStream_t st) {
  int nb = partial_blocks(n, kTC);
  size_t per = size_t(p) * q;
  if (size_t(nb + 1) * per > partial_elems) nb = int(partial_elems / per) - 1;
  size_t shm = size_t(kTC) * (p + q) * sizeof(T);
  YMat<T> yf{Y, ldy};
  if (wmat != nullptr) {
    k_gram<T, Acc, YMat<T>, WMatS<T>><<<nb, kBlock, shm, st>>>(n, X, ldx, p, yf, q,
                                                              WMatS<T>{wmat, s}, partial);
  } else {
    k_gram<T, Acc, YMat<T>, WOne<T>><<<nb, kBlock, shm, st>>>(n, X, ldx, p, yf, q, WOne<T>{},
                                                             partial);
  }
  double *red = partial + size_t(nb) * per;
  k_reduce_partials<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(partial, nb, int(per), red);
  k_scatter<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(red, p, q, 1, G, ldg, 0);
}

template <typename T, typename Acc>
void launch_xt_source(int n, const T *X, int ld, int p, const T *w, int n_mat, const T *psi,
                      double *H, int ldh, double *partial, size_t partial_elems,
                      hipStream_t st) {
  int nb = partial_blocks(n, kTC);
  size_t per = size_t(p) * n_mat;
  if (size_t(nb + 1) * per > partial_elems) nb = int(partial_elems / per) - 1;
  size_t shm = size_t(kTC) * (p + n_mat) * sizeof(T);
  k_gram<T, Acc, YSrc<T>, WOne<T>><<<nb, kBlock, shm, st>>>(n, X, ld, p, YSrc<T>{w, psi, n},
                                                           n_mat, WOne<T>{}, partial);
  double *red = partial + size_t(nb) * per;
  k_reduce_partials<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(partial, nb, int(per), red);
  k_scatter<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(red, p, n_mat, 1, H, ldh, 0);
}

template <typename T>
void launch_sumsq(int n, const T *X, int ld, int q, double *out, double *partial,
                  size_t partial_elems, hipStream_t st) {
  int nb = partial_blocks(n, kBlock);
  if (size_t(nb) > partial_elems) nb = int(partial_elems);
  k_sumsq<T><<<nb, kBlock, 0, st>>>(n, X, ld, q, partial);
  k_reduce_partials<<<1, kBlock, 0, st>>>(partial, nb, 1, out);
}

template <typename T>
void launch_update(int n, const T *X, int ldx, int p, const double *G, int ldg, double beta,
                   const T *Y, int ldy, double alpha, T *Z, int ldz, int q, double *dose,
                   const double *dc, double dscale, hipStream_t st) {
  size_t shm = size_t(kUC) * (p + 1) * sizeof(T);
  k_update<T><<<(n + kUC - 1) / kUC, kBlock, shm, st>>>(n, X, ldx, p, G, ldg, beta, Y, ldy,
                                                        alpha, Z, ldz, q, dose, dc, dscale,
                                                        nullptr, 0, nullptr, nullptr, 0, 0.0);
}

template <typename T>
void launch_source_k(int n, const T *U, int ld, int r, const double *St, int lds, const T *w,
                     int n_mat, const T *psi, const double *Cg, int ldcg, double dt, T *K,
                     hipStream_t st) {
  size_t shm = size_t(kUC) * (r + 1) * sizeof(T);
  k_update<T><<<(n + kUC - 1) / kUC, kBlock, shm, st>>>(n, U, ld, r, St, lds, 1.0, nullptr, 0,
                                                        0.0, K, ld, r, nullptr, nullptr, 0.0, w,
                                                        n_mat, psi, Cg, ldcg, dt);
}

template <typename T>
void launch_zero_cols(int n, T *X, int ld, int c0, int c1, hipStream_t st) {
  if (c1 <= c0) return;
  k_zero_cols<T><<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(n, X, ld, c0, c1);
}

void launch_reduce_partials(const double *partial, int nblocks, int elems, double *out,
                            hipStream_t st) {
  k_reduce_partials<<<(elems + kBlock - 1) / kBlock, kBlock, 0, st>>>(partial, nblocks, elems,
                                                                      out);
}

#define DLRA_INSTANTIATE(T, Acc)                                                              \
  template void launch_inverse_stop<T>(const GridDev &, const T *, int, const double *, T *,  \
                                       Ctl *, hipStream_t);                                   \
  template void launch_kstep_stage<T>(const GridDev &, const T *, const T *, const T *, T *,  \
                                      int, int, const double *, int, double, hipStream_t);    \
  template void launch_stencil_projection<T, Acc>(const GridDev &, const T *, const T *, int, \
                                                  int, double *, int, double *, size_t,       \
                                                  hipStream_t);                               \
  template void launch_gram<T, Acc>(int, const T *, int, int, const T *, int, int, const T *, \
                                    const T *, double *, int, double *, size_t, hipStream_t); \
  template void launch_xt_source<T, Acc>(int, const T *, int, int, const T *, int, const T *, \
                                         double *, int, double *, size_t, hipStream_t);       \
  template void launch_sumsq<T>(int, const T *, int, int, double *, double *, size_t,         \
                                hipStream_t);                                                 \
  template void launch_update<T>(int, const T *, int, int, const double *, int, double,       \
                                 const T *, int, double, T *, int, int, double *,             \
                                 const double *, double, hipStream_t);                        \
  template void launch_source_k<T>(int, const T *, int, int, const double *, int, const T *,  \
                                   int, const T *, const double *, int, double, T *,          \
                                   hipStream_t);                                              \
  template void launch_zero_cols<T>(int, T *, int, int, int, hipStream_t);

DLRA_INSTANTIATE(double, double)
DLRA_INSTANTIATE(float, float)
template void launch_gram<float, double>(int, const float *, int, int, const float *, int, int,
                                         const float *, const float *, double *, int, double *,
                                         size_t, hipStream_t);

}  // namespace dlra
