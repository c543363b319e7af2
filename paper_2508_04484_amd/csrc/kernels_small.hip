// Small dense FP64 kernels: angular Galerkin products, L- and S-step RK4
// stages, SVD-based truncation, orthonormalisation of augmentations and the
// collided self-scattering solves.  Matrices are column-major double.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace dlra {

namespace {

constexpr int kT = 16;
constexpr int kWG = 512;   // threads of the single-workgroup kernels
typedef double sd4 __attribute__((ext_vector_type(4)));   // f64 MFMA accumulator
constexpr int kTruncLdsDoubles = 19456;   // LDS room of k_truncate (152 KiB)
constexpr size_t kSmallMaxLds = 150 * 1024;   // largest dynamic LDS a small kernel asks for

// ------------------------------------------------------------------ small GEMM
__global__ void k_small_gemm(int ta, int tb, int M, int N, int K, double alpha,
                             const double *__restrict__ A, int lda, size_t sA,
                             const double *__restrict__ B, int ldb, size_t sB, double beta,
                             double *C, int ldc, size_t sC) {
  __shared__ double As[kT][kT + 1];
  __shared__ double Bs[kT][kT + 1];
  const int z = blockIdx.z;
  A += z * sA;
  B += z * sB;
  C += z * sC;
  const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
  const int row = blockIdx.y * kT + tx;   // output row i
  const int col = blockIdx.x * kT + ty;   // output col j
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += kT) {
    // As[i][k] = op(A)(row0 + i, k0 + k)
    {
      int i = blockIdx.y * kT + tx, k = k0 + ty;
      double v = 0.0;
      if (i < M && k < K) v = ta ? A[k + size_t(i) * lda] : A[i + size_t(k) * lda];
      As[tx][ty] = v;
    }
    {
      int k = k0 + tx, j = blockIdx.x * kT + ty;
      double v = 0.0;
      if (k < K && j < N) v = tb ? B[j + size_t(k) * ldb] : B[k + size_t(j) * ldb];
      Bs[tx][ty] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kT; ++k) acc += As[tx][k] * Bs[k][ty];
    __syncthreads();
  }
  if (row < M && col < N) {
    double *c = C + row + size_t(col) * ldc;
    *c = alpha * acc + (beta == 0.0 ? 0.0 : beta * *c);
  }
}

// ------------------------------------------------------------------ block helpers
__device__ double blk_sum(double v, double *red) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// C(p x q) = op(A) op(B) inside one workgroup (global operands), C distinct.
__device__ void blk_gemm(int ta, int tb, int M, int N, int K, double alpha, const double *A,
                         int lda, const double *B, int ldb, double beta, double *C, int ldc) {
  for (int e = threadIdx.x; e < M * N; e += blockDim.x) {
    int i = e % M, j = e / M;
    double s = 0.0;
    for (int k = 0; k < K; ++k) {
      double a = ta ? A[k + size_t(i) * lda] : A[i + size_t(k) * lda];
      double b = tb ? B[j + size_t(k) * ldb] : B[k + size_t(j) * ldb];
      s += a * b;
    }
    double *c = C + i + size_t(j) * ldc;
    *c = alpha * s + (beta == 0.0 ? 0.0 : beta * *c);
  }
  __syncthreads();
}

// x of the lane that the DPP row permutation CTRL names, both 32-bit halves
template <int CTRL>
__device__ inline double dpp_mov(double x) {
  const unsigned long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(v)), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(v >> 32)), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(
      (long long)((unsigned long long)unsigned(hi) << 32 | (unsigned long long)unsigned(lo)));
}

// Sum over each aligned group of 16 lanes (all lanes of the row active): four pairwise
// exchanges (swap neighbours, swap pairs of a quad, mirror each half row,
// mirror the row).  Every step pairs lanes symmetrically, so all 16 lanes end
// with the same bits.
// sum over the 8 lanes of each half of a DPP row
__device__ inline double row8_sum(double x) {
  x += dpp_mov<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += dpp_mov<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += dpp_mov<0x141>(x);   // row_half_mirror
  return x;
}

__device__ inline double row16_sum(double x) {
  x += dpp_mov<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += dpp_mov<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += dpp_mov<0x141>(x);   // row_half_mirror
  x += dpp_mov<0x140>(x);   // row_mirror
  return x;
}

// coef[j] = sum_t Q(t, j) v(t) for j < cnt: 16 lanes (one DPP row) per
// column stride over t and sum across the row (deterministic).  The
// workgroup size is a multiple of 64.
__device__ void blk_coefs(const double *Q, int ldq, int p, int cnt, const double *v,
                          double *coef) {
  const int lane = threadIdx.x & 15, grp = threadIdx.x >> 4, ng = blockDim.x >> 4;
  for (int j = grp; j < cnt; j += ng) {   // uniform within a DPP row
    double s = 0.0;
#pragma unroll 4
    for (int t = lane; t < p; t += 16) s += Q[t + size_t(j) * ldq] * v[t];
    s = row16_sum(s);
    if (lane == 0) coef[j] = s;
  }
  __syncthreads();
}

// Block products on the FP64 matrix cores (16x16x4 f64 MFMA: A lane l holds
// (row l % 16, k l / 16), B lane l holds (k l / 16, column l % 16), register
// v of the accumulator is (row l / 16 + 4 v, column l % 16)).  Each wave owns
// 16 x 16 tiles of C in turn and runs its k-steps in batches of kBlkKB with
// all their loads in flight; operands past the matrix edges are clamped on
// load and zeroed.  Generic pointers (LDS or global); C must not alias A or
// B.  Both end with a barrier.
constexpr int kBlkKB = 8;

// C (M x N) = alpha A^T B for A (K x M, lda) and B (K x N, ldb)
__device__ void blk_mfma_tn(int M, int N, int K, double alpha, const double *A, int lda,
                            const double *B, int ldb, double *C, int ldc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int c = lane & 15, q = lane >> 4;
  const int TM = (M + 15) / 16, TN = (N + 15) / 16, KS = (K + 3) / 4;
  for (int t = w; t < TM * TN; t += nw) {
    const int i0 = 16 * (t % TM), j0 = 16 * (t / TM);
    const double *Ap = A + size_t(min(i0 + c, M - 1)) * lda;
    const double *Bp = B + size_t(min(j0 + c, N - 1)) * ldb;
    sd4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = 0; s0 < KS; s0 += kBlkKB) {
      double a[kBlkKB], b[kBlkKB];
#pragma unroll
      for (int u = 0; u < kBlkKB; ++u) {
        const int k = 4 * (s0 + u) + q, kc = min(k, K - 1);
        const double av = Ap[kc], bv = Bp[kc];
        a[u] = k < K ? av : 0.0;
        b[u] = k < K ? bv : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kBlkKB; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + q + 4 * v, j = j0 + c;
      if (i < M && j < N) C[i + size_t(j) * ldc] = alpha * acc[v];
    }
  }
  __syncthreads();
}

// C (M x N) = beta C + alpha A B for A (M x K, lda) and B (K x N, ldb); C is
// not read when beta == 0
__device__ void blk_mfma_nn(int M, int N, int K, double alpha, const double *A, int lda,
                            const double *B, int ldb, double beta, double *C, int ldc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int c = lane & 15, q = lane >> 4;
  const int TM = (M + 15) / 16, TN = (N + 15) / 16, KS = (K + 3) / 4;
  for (int t = w; t < TM * TN; t += nw) {
    const int i0 = 16 * (t % TM), j0 = 16 * (t / TM);
    const double *Ap = A + min(i0 + c, M - 1);
    const double *Bp = B + size_t(min(j0 + c, N - 1)) * ldb;
    sd4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int s0 = 0; s0 < KS; s0 += kBlkKB) {
      double a[kBlkKB], b[kBlkKB];
#pragma unroll
      for (int u = 0; u < kBlkKB; ++u) {
        const int k = 4 * (s0 + u) + q, kc = min(k, K - 1);
        const double av = Ap[size_t(kc) * lda], bv = Bp[kc];
        a[u] = k < K ? av : 0.0;
        b[u] = k < K ? bv : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kBlkKB; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + q + 4 * v, j = j0 + c;
      if (i < M && j < N) {
        double *o = C + i + size_t(j) * ldc;
        *o = beta == 0.0 ? alpha * acc[v] : beta * *o + alpha * acc[v];
      }
    }
  }
  __syncthreads();
}

// Pair (i, j) with i < j that group k of a round-robin round plays, for qe
// (even) columns: one column stays put, the others rotate.
__device__ inline void rr_pair(int qe, int round, int k, int &i, int &j) {
  // round < qe - 1 and k < qe / 2: one conditional subtraction replaces the
  // modulo qe - 1
  const int n = qe - 1;
  if (k == 0) {
    i = round;
    j = n;
  } else {
    i = round + k;
    i -= i >= n ? n : 0;
    j = round - k + n;
    j -= j >= n ? n : 0;
  }
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
}

// Rounds of the one-sided Jacobi below for p, q <= LP * RPL when the
// workgroup has LP lanes (16 or 8, within one DPP row) for every pair of a
// round: the lanes of a pair hold its two columns of A and of V in registers
// (rows lane, lane + LP, ...), so each round issues all its LDS reads at
// once and sums the three inner products across the LP lanes by DPP.  Same
// ordering, rotation rule and stopping test as the general rounds.
template <int LP, int RPL, bool ACCV>
__device__ void jacobi_rounds_reg(double *A, int lda, int p, int q, double *V, int ldv,
                                  int *flag, double tiny) {
  static_assert(LP == 16 || LP == 8, "a pair's lanes lie in one DPP row");
  const int tid = threadIdx.x;
  const int qe = q + (q & 1);
  const int lane = tid % LP, k = tid / LP;
  const bool active = k < qe / 2;
  for (int sweep = 0; sweep < 80; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < qe - 1; ++round) {
      int i = 0, j = 0;
      if (active) rr_pair(qe, round, k, i, j);
      const bool valid = active && j < q;
      double a[RPL], b[RPL], va[RPL], vb[RPL];
      double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int t = lane + LP * u;
        const bool inA = valid && t < p, inV = valid && t < q;
        a[u] = inA ? A[t + size_t(i) * lda] : 0.0;
        b[u] = inA ? A[t + size_t(j) * lda] : 0.0;
        if constexpr (ACCV) {
          va[u] = inV ? V[t + size_t(i) * ldv] : 0.0;
          vb[u] = inV ? V[t + size_t(j) * ldv] : 0.0;
        }
        al += a[u] * a[u];
        be += b[u] * b[u];
        ga += a[u] * b[u];
      }
      if constexpr (LP == 16) {
        al = row16_sum(al);
        be = row16_sum(be);
        ga = row16_sum(ga);
      } else {
        al = row8_sum(al);
        be = row8_sum(be);
        ga = row8_sum(ga);
      }
      if (valid && al > 0.0 && be > 0.0 && fabs(ga) > 1e-15 * sqrt(al * be) &&
          fabs(ga) > tiny) {
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int r = lane + LP * u;
          if (r < p) {
            A[r + size_t(i) * lda] = c * a[u] - s * b[u];
            A[r + size_t(j) * lda] = s * a[u] + c * b[u];
          }
          if (ACCV && r < q) {
            V[r + size_t(i) * ldv] = c * va[u] - s * vb[u];
            V[r + size_t(j) * ldv] = s * va[u] + c * vb[u];
          }
        }
        if (lane == 0) *flag = 1;
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (!f) break;
  }
}

// One-sided Jacobi: orthogonalise the q columns (length p) of A, accumulating
// the rotations in V (q x q, initialised here) unless V is null.  Parallel round-robin
// ordering; 8 lanes per column pair, or the register rounds above when the
// matrix is at most 128 x 128.  A pair is rotated when its inner
// product is above 1e-15 of the columns' norms and above 1e-30 ||A||_F^2:
// pairs of columns that are both negligible against the matrix (singular
// values below ~1e-15 of the largest) carry only rounding noise, and
// rotating them would keep the sweeps from terminating.
__device__ __attribute__((always_inline)) void blk_jacobi(double *A, int lda, int p, int q, double *V, int ldv, int *flag,
                           double *red) {
  const int tid = threadIdx.x;
  if (V != nullptr)
    for (int e = tid; e < q * q; e += blockDim.x) V[(e % q) + size_t(e / q) * ldv] = (e % q == e / q) ? 1.0 : 0.0;
  double fro = 0.0;
  for (int e = tid; e < p * q; e += blockDim.x) {
    const double a = A[(e % p) + size_t(e / p) * lda];
    fro += a * a;
  }
  const double tiny = 1e-30 * blk_sum(fro, red);
  __syncthreads();
  const int qe = q + (q & 1);
  if (qe < 2) return;
  if (p <= 64 && q <= 64 && (qe / 2) * 16 <= int(blockDim.x) && blockDim.x % 64 == 0) {
    if (V != nullptr) jacobi_rounds_reg<16, 4, true>(A, lda, p, q, V, ldv, flag, tiny);
    else jacobi_rounds_reg<16, 4, false>(A, lda, p, q, V, ldv, flag, tiny);
    return;
  }
  if (p <= 128 && q <= 128 && (qe / 2) * 8 <= int(blockDim.x) && blockDim.x % 64 == 0) {
    if (V != nullptr) jacobi_rounds_reg<8, 16, true>(A, lda, p, q, V, ldv, flag, tiny);
    else jacobi_rounds_reg<8, 16, false>(A, lda, p, q, V, ldv, flag, tiny);
    return;
  }
  const int lane8 = tid & 7;
  const int grp = tid >> 3;
  const int ngrp = blockDim.x >> 3;
  for (int sweep = 0; sweep < 80; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < qe - 1; ++round) {
      for (int k = grp; k < qe / 2; k += ngrp) {
        int i, j;
        rr_pair(qe, round, k, i, j);
        bool valid = j < q;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (valid) {
          for (int t = lane8; t < p; t += 8) {
            double a = A[t + size_t(i) * lda], b = A[t + size_t(j) * lda];
            al += a * a;
            be += b * b;
            ga += a * b;
          }
        }
        for (int o = 4; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 8);
          be += __shfl_xor(be, o, 8);
          ga += __shfl_xor(ga, o, 8);
        }
        if (valid && al > 0.0 && be > 0.0 && fabs(ga) > 1e-15 * sqrt(al * be) &&
            fabs(ga) > tiny) {
          double zeta = (be - al) / (2.0 * ga);
          double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int u = lane8; u < p; u += 8) {
            double a = A[u + size_t(i) * lda], b = A[u + size_t(j) * lda];
            A[u + size_t(i) * lda] = c * a - s * b;
            A[u + size_t(j) * lda] = s * a + c * b;
          }
          if (V != nullptr)
            for (int u = lane8; u < q; u += 8) {
              double a = V[u + size_t(i) * ldv], b = V[u + size_t(j) * ldv];
              V[u + size_t(i) * ldv] = c * a - s * b;
              V[u + size_t(j) * ldv] = s * a + c * b;
            }
          if (lane8 == 0) *flag = 1;
        }
      }
      __syncthreads();
    }
    int f = *flag;
    __syncthreads();
    if (!f) break;
  }
}

// SVD of A (p x q, q <= p <= kSvdMaxP) by one-sided Jacobi with QR
// preconditioning (Householder A = H [R; 0], H = H_0 ... H_{q-1}; Jacobi on
// R^T, whose columns converge in far fewer sweeps than those of a graded A):
// R^T Z = Y with orthogonal columns, sigma_j = ||Y_j||, and then
// A V = H [Z; 0] diag(sigma) for V = Y diag(1 / sigma).  Leaves the same
// outputs as blk_jacobi on A: A <- A V (columns u_j sigma_j), V the right
// singular vectors (a zero column where sigma_j = 0).  Without LEFT the
// rotations are not accumulated and only V and sig[j] = sigma_j are formed (A
// is left as scratch).  X (q x q) and hb (2 q) are scratch; one DPP row of 16 lanes works on one column, and H [Z; 0] is
// formed in registers (a DPP row holds up to kSvdCpg columns, 8 rows a lane),
// so the workgroup needs q <= kSvdCpg * blockDim / 16.
constexpr int kSvdMaxP = 128, kSvdCpg = 4;
// the single-workgroup kernels hold an order-n SVD's A, V, X and 2 n in LDS
inline __host__ __device__ bool svd_qr_fits(int n) {
  return n <= kSvdMaxP && 3 * n * n + 2 * n <= kTruncLdsDoubles;
}
template <bool LEFT>
__device__ __attribute__((always_inline)) void blk_svd_qr(double *A, int p, int q, double *V,
                                                          double *X, double *hb, int *flag,
                                                          double *red, double *sig) {
  const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4, ng = blockDim.x >> 4;
  double *beta = hb, *rdiag = hb + q;
  // Householder QR: reflector k in A[k:, k], R above the diagonal of A
  for (int k = 0; k < q; ++k) {
    double *x = A + k + size_t(k) * p;
    const int len = p - k;
    if (grp == 0) {
      double s2 = 0.0;
#pragma unroll 4
      for (int t = lane; t < len; t += 16) s2 += x[t] * x[t];
      s2 = row16_sum(s2);
      if (lane == 0) {
        const double nrm = sqrt(s2), x0 = x[0];
        if (nrm > 0.0) {
          const double sg = x0 >= 0.0 ? 1.0 : -1.0;
          rdiag[k] = -sg * nrm;
          beta[k] = 1.0 / (nrm * (nrm + fabs(x0)));
          x[0] = x0 + sg * nrm;
        } else {
          rdiag[k] = 0.0;
          beta[k] = 0.0;
        }
      }
    }
    __syncthreads();
    const double bk = beta[k];
    for (int j = k + 1 + grp; j < q; j += ng) {   // uniform within a DPP row
      double *y = A + k + size_t(j) * p;
      double w = 0.0;
#pragma unroll 4
      for (int t = lane; t < len; t += 16) w += x[t] * y[t];
      w = row16_sum(w) * bk;
#pragma unroll 4
      for (int t = lane; t < len; t += 16) y[t] -= w * x[t];
    }
    __syncthreads();
  }
  // X = R^T
  for (int e = tid; e < q * q; e += blockDim.x) {
    const int a = e % q, b = e / q;
    X[e] = b < a ? A[b + size_t(a) * p] : (b == a ? rdiag[a] : 0.0);
  }
  __syncthreads();
  blk_jacobi(X, q, q, q, LEFT ? V : nullptr, q, flag, red);   // X <- Y, V <- Z
  __syncthreads();
  if constexpr (!LEFT) {
    // right singular vectors and singular values only
    for (int j = grp; j < q; j += ng) {   // uniform within a DPP row
      double s2 = 0.0;
#pragma unroll 4
      for (int t = lane; t < q; t += 16) s2 += X[t + size_t(j) * q] * X[t + size_t(j) * q];
      const double sg = sqrt(row16_sum(s2));
#pragma unroll 4
      for (int t = lane; t < q; t += 16)
        V[t + size_t(j) * q] = sg > 0.0 ? X[t + size_t(j) * q] / sg : 0.0;
      if (lane == 0) sig[j] = sg;
    }
    __syncthreads();
    return;
  }
  // B = H [Z; 0] in registers, reflectors applied last to first: DPP row grp
  // owns columns grp + cc ng, its lane the rows lane + 16 u
  constexpr int RPL = kSvdMaxP / 16;
  double y[kSvdCpg][RPL];
#pragma unroll
  for (int cc = 0; cc < kSvdCpg; ++cc) {
    const int j = min(grp + cc * ng, q - 1);
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int t = lane + 16 * u;
      y[cc][u] = t < q ? V[t + size_t(j) * q] : 0.0;
    }
  }
  for (int k = q - 1; k >= 0; --k) {
    double x[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int t = lane + 16 * u;
      x[u] = (t >= k && t < p) ? A[t + size_t(k) * p] : 0.0;
    }
    const double bk = beta[k];
#pragma unroll
    for (int cc = 0; cc < kSvdCpg; ++cc) {
      double w = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) w += x[u] * y[cc][u];
      w = row16_sum(w) * bk;
#pragma unroll
      for (int u = 0; u < RPL; ++u) y[cc][u] -= w * x[u];
    }
  }
  __syncthreads();   // every row has read the reflectors in A
#pragma unroll
  for (int cc = 0; cc < kSvdCpg; ++cc) {
    const int j = grp + cc * ng;
    if (j < q) {   // uniform within a DPP row
      double s2 = 0.0;
#pragma unroll 4
      for (int t = lane; t < q; t += 16) s2 += X[t + size_t(j) * q] * X[t + size_t(j) * q];
      const double sg = sqrt(row16_sum(s2));
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int t = lane + 16 * u;
        if (t < p) A[t + size_t(j) * p] = y[cc][u] * sg;
      }
#pragma unroll 4
      for (int t = lane; t < q; t += 16)
        V[t + size_t(j) * q] = sg > 0.0 ? X[t + size_t(j) * q] / sg : 0.0;
    }
  }
  __syncthreads();
}

// Cholesky-based orthonormalisation of a well-conditioned Gram matrix:
// A = L L^T in place (A: q x q SPD, lower part used and overwritten), then
// T = L^{-T} (q x q upper triangular, leading dimension ldt) so that X T has
// orthonormal columns when A = X^T X.  Returns false (T untouched) when a
// pivot is not above 1e-12 of the largest diagonal entry; the caller then
// falls back to the eigen-decomposition.
__device__ bool blk_chol_orth(double *A, int lda, int q, double *T, int ldt, double *red,
                              int *flag) {
  const int tid = threadIdx.x;
  double dmax = 0.0;
  for (int i = tid; i < q; i += blockDim.x) dmax = fmax(dmax, A[i + size_t(i) * lda]);
  // block maximum (values are >= 0): reduce through red
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  if (tid == 0) *flag = 1;
  __syncthreads();
  dmax = 0.0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) dmax = fmax(dmax, red[w]);
  __syncthreads();
  for (int k = 0; k < q; ++k) {
    if (tid == 0) {
      const double d = A[k + size_t(k) * lda];
      if (!(d > 1e-12 * dmax)) *flag = 0;
      A[k + size_t(k) * lda] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double piv = A[k + size_t(k) * lda];
    for (int i = k + 1 + tid; i < q; i += blockDim.x) A[i + size_t(k) * lda] /= piv;
    __syncthreads();
    const int nt = q - k - 1;
    for (int e = tid; e < nt * nt; e += blockDim.x) {
      const int i = k + 1 + e % nt, j = k + 1 + e / nt;
      if (j <= i) A[i + size_t(j) * lda] -= A[i + size_t(k) * lda] * A[j + size_t(k) * lda];
    }
    __syncthreads();
  }
  if (!*flag) return false;
  // column c of L^{-1} by forward substitution (one thread per column); T = its transpose
  for (int c = tid; c < q; c += blockDim.x) {
    for (int i = 0; i < q; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= A[i + size_t(k) * lda] * T[c + size_t(k) * ldt];
      T[c + size_t(i) * ldt] = i < c ? 0.0 : v / A[i + size_t(i) * lda];
    }
  }
  __syncthreads();
  return true;
}

// column norms of A (p x q) -> sig[q]; order[] = indices sorted by sig descending
// order[] = indices of sig[0 .. q - 1] sorted descending, ranked by counting
// (stable for ties by index)
__device__ void blk_sort_desc(const double *sig, int q, int *order) {
  for (int j = threadIdx.x; j < q; j += blockDim.x) {
    int pos = 0;
    for (int t = 0; t < q; ++t)
      if (sig[t] > sig[j] || (sig[t] == sig[j] && t < j)) ++pos;
    order[pos] = j;
  }
  __syncthreads();
}

__device__ void blk_colnorms_sorted(const double *A, int lda, int p, int q, double *sig,
                                    int *order) {
  for (int j = threadIdx.x; j < q; j += blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < p; ++t) s += A[t + size_t(j) * lda] * A[t + size_t(j) * lda];
    sig[j] = sqrt(s);
  }
  __syncthreads();
  blk_sort_desc(sig, q, order);
}

// Append up to `need` fillers to the orthonormal columns Q[:, 0:cnt) (length p)
// from the unit vectors e_0 .. e_{ncand-1} (ordered, two CGS passes, accepted
// when the residual norm exceeds accept).  Returns the new count.
__device__ int blk_fill(double *Q, int ldq, int p, int cnt, int need, int ncand, double accept,
                        double *v, double *coef, double *red) {
  int added = 0;
  for (int cand = 0; cand < ncand && added < need; ++cand) {
    for (int t = threadIdx.x; t < p; t += blockDim.x) v[t] = (t == cand) ? 1.0 : 0.0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      blk_coefs(Q, ldq, p, cnt, v, coef);
      for (int t = threadIdx.x; t < p; t += blockDim.x) {
        double s = v[t];
#pragma unroll 8
        for (int j = 0; j < cnt; ++j) s -= Q[t + size_t(j) * ldq] * coef[j];
        v[t] = s;
      }
      __syncthreads();
    }
    double nv = 0.0;
    for (int t = threadIdx.x; t < p; t += blockDim.x) nv += v[t] * v[t];
    nv = sqrt(blk_sum(nv, red));
    if (nv > accept) {
      for (int t = threadIdx.x; t < p; t += blockDim.x) Q[t + size_t(cnt) * ldq] = v[t] / nv;
      ++cnt;
      ++added;
    }
    __syncthreads();
  }
  return cnt;
}

// ------------------------------------------------------------------ S-step
// One RK4 stage (Horner form) of dS/dt = -sum_dk C_dk S B_dk:
//   out = S0 - coef sum_dk C_dk (W B_dk)
// on the FP64 matrix cores for P <= 4 NS (NS = 16 or 32 k-steps
// of 4): workgroup (it, jt) owns the 16 x 16 output tile (I, J) = (16 it..,
// 16 jt..), wave dk of it the term dk.  The wave forms T_dk(:, J) = W B_dk(:, J)
// one 16-row tile at a time (A operands: an LDS copy of W, zero padded; B
// operands: B_dk(:, J) in registers) and feeds each tile straight into
// C_dk(I, :) T_dk(:, J) (A operands C_dk(I, :) in registers): the accumulator
// of the first product is already the B operand of the second, so T never
// leaves registers.  The ndk tiles are then summed in order dk = 0, 1, ...
// 16x16x4 f64 MFMA operand layout: A lane l holds (row l % 16, k l / 16), B
// lane l holds (k l / 16, column l % 16), register v of the accumulator is
// (row l / 16 + 4 v, column l % 16) -- for row tile t of T that is the B
// operand of k-step 4 t + v of the second product.
constexpr int kSmMaxDk = 6;

// LDS row stride of the W copy for 16 pt rows: a multiple of 16 doubles with
// 2 * stride = 32 mod 64 banks, so lanes k and k + 1 of an A-operand read
// fall in opposite halves of the banks
inline __host__ __device__ int sstep_lds_stride(int pt) { return 16 * pt + ((pt & 1) ? 0 : 16); }

inline size_t sstep_mfma_lds(int p, int ndk) {
  const int pt = (p + 15) / 16;
  return (size_t(16 * pt) * sstep_lds_stride(pt) + size_t(ndk) * 256) * sizeof(double);
}

constexpr int kSsBatch = 16;   // W staging loads per thread in flight together

template <int NS>
__global__ __launch_bounds__(64 * kSmMaxDk) void k_sstep_mfma(
    int P, int ld, int ndk, const double *__restrict__ Ch, const double *__restrict__ Bh,
    const double *S0, const double *__restrict__ W, double *out, double coef) {
  extern __shared__ double smem_d[];
  // W is staged zero padded to RW x RW, so the k-steps run in whole groups
  // of four (one group per 16 rows of W, guarded once): the group's four
  // LDS reads issue together; the padded k-steps add exact zeros
  const int PT = (P + 15) / 16, RW = 16 * PT, KR = RW;
  const int lw = sstep_lds_stride(PT);
  double *Ws = smem_d;                       // [KR k][lw]: W(i, k) at k * lw + i
  double *Rs = Ws + size_t(KR) * lw;         // [ndk][16][16]
  const int tid = threadIdx.x, lane = tid & 63;
  const int dk = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, q = lane >> 4;
  const int I0 = 16 * blockIdx.x, J0 = 16 * blockIdx.y;
  const double *B = Bh + size_t(dk) * ld * ld, *C = Ch + size_t(dk) * ld * ld;
  // operands of this wave, all loads in flight together (clamped, masked)
  double bop[NS], cop[NS];
  const int jB = min(J0 + c, P - 1), iC = min(I0 + c, P - 1);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int k = 4 * s + q, kc = min(k, P - 1);
    const double bv = B[kc + size_t(jB) * ld];
    const double cv = C[iC + size_t(kc) * ld];
    bop[s] = k < P ? bv : 0.0;
    cop[s] = k < P ? cv : 0.0;
  }
  // this thread's S0 entries of the output tile (at most 2: >= 128 threads)
  double s0v[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = min(tid + u * int(blockDim.x), 255);
    s0v[u] = S0[min(I0 + (e & 15), P - 1) + size_t(min(J0 + (e >> 4), P - 1)) * ld];
  }
  // W into LDS, kSsBatch loads per thread in flight at a time
  const int tot = KR * RW, nthr = blockDim.x;
  for (int e0 = 0; e0 < tot; e0 += kSsBatch * nthr) {
    double wv[kSsBatch];
#pragma unroll
    for (int u = 0; u < kSsBatch; ++u) {
      const int e = min(e0 + u * nthr + tid, tot - 1), i = e % RW, k = e / RW;
      wv[u] = W[min(i, P - 1) + size_t(min(k, P - 1)) * ld];
    }
#pragma unroll
    for (int u = 0; u < kSsBatch; ++u) {
      const int e = e0 + u * nthr + tid, i = e % RW, k = e / RW;
      if (e < tot) Ws[k * lw + i] = (i < P && k < P) ? wv[u] : 0.0;
    }
  }
  __syncthreads();
  sd4 f = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < NS / 4; ++t) {
    if (t < PT) {
      sd4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int g4 = 0; g4 < NS / 4; ++g4) {
        if (g4 < PT) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int s = 4 * g4 + v;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ws[(4 * s + q) * lw + 16 * t + c], bop[s],
                                                       acc, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
        f = __builtin_amdgcn_mfma_f64_16x16x4f64(cop[4 * t + v], acc[v], f, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) Rs[(dk * 16 + q + 4 * v) * 16 + c] = f[v];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * int(blockDim.x);
    const int i = e & 15, j = e >> 4, gi = I0 + i, gj = J0 + j;
    if (e < 256 && gi < P && gj < P) {
      double F = 0.0;
      for (int d = 0; d < ndk; ++d) F -= Rs[(d * 16 + i) * 16 + j];
      out[gi + size_t(gj) * ld] = s0v[u] + coef * F;
    }
  }
}

// One L-step stage in one launch on the FP64 matrix cores:
// out = L0 - coef sum_dk A_dk in C_dk^T (m x r, leading dim m).  Block b owns
// the rows I = 16 b .. 16 b + 15 of out, wave dk the term dk.  The wave forms
// T = A_dk(I, :) in (16 x RB) with A operands straight from A and B operands
// from an LDS copy of in (chunks of kLsKC rows, zero past m and r), parks T in
// LDS and multiplies it by C_dk^T (B operands from C); the ndk partial tiles
// are then summed in order dk = 0, 1, ... .
constexpr int kLsKC = 64;   // rows of in per LDS chunk

// The loads of one chunk (rows l0 .. l0 + kLsKC - 1 of the contraction): this
// lane's A operands and this thread's NST of the tot entries of the in chunk
// (clamped)
template <int NST, int NTHR>
__device__ __forceinline__ void lstep_fetch(int l0, int m, int r, int arow, int q, int tid, int tot,
                                            const double *__restrict__ Ad,
                                            const double *__restrict__ in,
                                            double (&an)[kLsKC / 4], double (&stg)[NST]) {
#pragma unroll
  for (int s = 0; s < kLsKC / 4; ++s) an[s] = Ad[arow + size_t(min(l0 + 4 * s + q, m - 1)) * m];
#pragma unroll
  for (int u = 0; u < NST; ++u) {
    const int e = min(tid + u * NTHR, tot - 1), l = e % kLsKC, k = e / kLsKC;
    stg[u] = in[size_t(min(l0 + l, m - 1)) + size_t(min(k, r - 1)) * m];
  }
}

template <int NKC, int NDK>
__global__ __launch_bounds__(64 * NDK) void k_lstep_mfma(
    int m, int r, const double *__restrict__ A, const double *__restrict__ C, int ldc,
    const double *__restrict__ in, const double *__restrict__ L0, double *__restrict__ out,
    double coef) {
  constexpr int RB = 16 * NKC, IS = RB + 2;   // LDS row stride of the in chunk
  extern __shared__ double smem_d[];
  double *Is = smem_d;                       // [kLsKC][IS]
  double *Ts = Is + kLsKC * IS;              // [NDK][16][RB]: T, then the partial tile
  const int tid = threadIdx.x, lane = tid & 63;
  const int dk = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, q = lane >> 4;
  const int I0 = 16 * blockIdx.x;
  const double *Ad = A + size_t(dk) * m * m;
  const int arow = min(I0 + c, m - 1);       // rows past m: clamped, never stored
  // NST: in-chunk entries per thread; NO: outputs per thread
  constexpr int NTHR = 64 * NDK, NST = (kLsKC * RB + NTHR - 1) / NTHR;
  constexpr int NO = (16 * RB + NTHR - 1) / NTHR;
  const int nthr = NTHR;
  // this thread's L0 entries, read up front
  double l0v[NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int e = min(tid + u * nthr, 16 * RB - 1), i = e % 16, j = e / 16;
    l0v[u] = L0[size_t(min(I0 + i, m - 1)) + size_t(min(j, r - 1)) * m];
  }
  sd4 acc[NKC];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) acc[kc] = sd4{0.0, 0.0, 0.0, 0.0};
  // software pipeline: the loads of chunk l0 + kLsKC are in flight while the
  // matrix cores work on chunk l0
  double an[kLsKC / 4], stg[NST];
  lstep_fetch<NST, NTHR>(0, m, r, arow, q, tid, kLsKC * RB, Ad, in, an, stg);
  for (int l0 = 0; l0 < m; l0 += kLsKC) {
    __syncthreads();   // the previous chunk's readers are done
#pragma unroll
    for (int u = 0; u < NST; ++u) {
      const int e = tid + u * nthr, l = e % kLsKC, k = e / kLsKC;
      if (e < kLsKC * RB) Is[l * IS + k] = (l0 + l < m && k < r) ? stg[u] : 0.0;
    }
    double aop[kLsKC / 4];   // A operands of this chunk (column l0 + 4 s + q)
#pragma unroll
    for (int s = 0; s < kLsKC / 4; ++s) aop[s] = an[s];
    __syncthreads();
    if (l0 + kLsKC < m)
      lstep_fetch<NST, NTHR>(l0 + kLsKC, m, r, arow, q, tid, kLsKC * RB, Ad, in, an, stg);
#pragma unroll
    for (int s = 0; s < kLsKC / 4; ++s)
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc)
        acc[kc] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[s], Is[(4 * s + q) * IS + 16 * kc + c],
                                                       acc[kc], 0, 0, 0);
  }
  // T (row q + 4 v, column 16 kc + c) into this wave's LDS tile
  double *T = Ts + size_t(dk) * 16 * RB;
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
    for (int v = 0; v < 4; ++v) T[(q + 4 * v) * RB + 16 * kc + c] = acc[kc][v];
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's T stores landed
  __builtin_amdgcn_wave_barrier();
  // partial tile (I, J) = T C_dk^T over the RB columns of T; B lane l holds
  // C_dk(j = 16 jt + c, k = 4 s + q) (k past r: T is zero there)
  const double *Cd = C + size_t(dk) * ldc * ldc;
  sd4 f[NKC];
#pragma unroll
  for (int jt = 0; jt < NKC; ++jt) {
    f[jt] = sd4{0.0, 0.0, 0.0, 0.0};
    const int j = min(16 * jt + c, r - 1);
#pragma unroll
    for (int s = 0; s < RB / 4; ++s) {
      const int k = min(4 * s + q, r - 1);
      f[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(T[c * RB + 4 * s + q], Cd[j + size_t(k) * ldc],
                                                   f[jt], 0, 0, 0);
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int jt = 0; jt < NKC; ++jt)
#pragma unroll
    for (int v = 0; v < 4; ++v) T[(q + 4 * v) * RB + 16 * jt + c] = f[jt][v];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    const int e = tid + u * nthr, i = e % 16, j = e / 16;
    if (e < 16 * RB && I0 + i < m && j < r) {
      double F = 0.0;
      for (int d = 0; d < NDK; ++d) F += Ts[(size_t(d) * 16 + i) * RB + j];
      out[size_t(I0 + i) + size_t(j) * m] = l0v[u] - coef * F;
    }
  }
}

// L-step stage combine: out = L0 - coef sum_dk T_dk C_dk^T, T_dk = A_dk in
// (m x r blocks, leading dim m, strided by ts).
__global__ void k_lstep_combine(int m, int r, int ndk, const double *__restrict__ T, size_t ts,
                                const double *__restrict__ C, int ldc,
                                const double *__restrict__ L0, double *__restrict__ out,
                                double coef) {
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= m * r) return;
  int i = e % m, j = e / m;
  double acc = 0.0;
  for (int dk = 0; dk < ndk; ++dk) {
    const double *Td = T + dk * ts;
    const double *Cd = C + size_t(dk) * ldc * ldc;
#pragma unroll 8
    for (int k = 0; k < r; ++k) acc += Td[i + size_t(k) * m] * Cd[j + size_t(k) * ldc];
  }
  out[i + size_t(j) * m] = L0[i + size_t(j) * m] - coef * acc;
}

// ------------------------------------------------------------------ Gram orthonormalisation
__global__ __launch_bounds__(kWG) void k_gram_orth(int q, const double *__restrict__ W,
                                                  double *T, int ldt, double tol2,
                                                  const double *normsq, int *count,
                                                  const int *restrict_count, double *work) {
  __shared__ double red[16];
  __shared__ int flag;
  __shared__ int order[128];
  __shared__ double sig[128];
  extern __shared__ double dyn[];
  const int qq = restrict_count ? *restrict_count : q;
  double *A = dyn;                // qq x qq copy of W (LDS)
  double *V = dyn + q * q;        // eigenvectors (LDS)
  (void)work;
  for (int e = threadIdx.x; e < qq * qq; e += blockDim.x) {
    int i = e % qq, j = e / qq;
    A[i + j * qq] = W[i + j * q];
  }
  for (int e = threadIdx.x; e < q * q; e += blockDim.x) T[(e % q) + size_t(e / q) * ldt] = 0.0;
  __syncthreads();
  if (restrict_count) {
    // second pass on an already orthonormalised block: Cholesky suffices (only
    // the span matters downstream); the eigen path remains the fallback
    if (blk_chol_orth(A, qq, qq, T, ldt, red, &flag)) return;
    for (int e = threadIdx.x; e < qq * qq; e += blockDim.x) {
      int i = e % qq, j = e / qq;
      A[i + j * qq] = W[i + j * q];
    }
    for (int e = threadIdx.x; e < q * q; e += blockDim.x) T[(e % q) + size_t(e / q) * ldt] = 0.0;
    __syncthreads();
  }
  // the QR-preconditioned SVD when its scratch is in the launch's LDS
  // for the PSD W the singular values are its eigenvalues (the column norms
  // of W V)
  if (svd_qr_fits(q)) {
    blk_svd_qr<false>(A, qq, qq, V, dyn + 2 * q * q, dyn + 3 * q * q, &flag, red, sig);
    blk_sort_desc(sig, qq, order);
  } else {
    blk_jacobi(A, qq, qq, qq, V, qq, &flag, red);
    __syncthreads();
    blk_colnorms_sorted(A, qq, qq, qq, sig, order);
  }
  const double thresh = restrict_count ? 0.0 : tol2 * (*normsq);
  int kept = 0;
  for (int t = 0; t < qq; ++t)
    if (sig[order[t]] > thresh && sig[order[t]] > 0.0) ++kept;
  for (int e = threadIdx.x; e < qq * kept; e += blockDim.x) {
    int i = e % qq, c = e / qq;
    int j = order[c];
    T[i + size_t(c) * ldt] = V[i + j * qq] / sqrt(sig[j]);
  }
  if (threadIdx.x == 0 && count != nullptr && restrict_count == nullptr) *count = kept;
}

// ------------------------------------------------------------------ V augmentation
__global__ __launch_bounds__(kWG) void k_vaug(int m, int r, double *Vh, int ldv,
                                             const double *__restrict__ L, double tol, int *count,
                                             double *work) {
  __shared__ double red[16];
  __shared__ int flag;
  __shared__ int order[128];
  __shared__ double sig[128];
  extern __shared__ double dyn[];
  double *R = work;                    // m x r
  double *X = R + size_t(m) * r;       // m x r
  double *G = dyn;                     // r x r (LDS)
  double *W = G + r * r;               // r x r (LDS)
  double *Q = W + r * r;               // r x r (LDS)
  double *Xs = Q + r * r;              // r x r, 2 r: SVD scratch (LDS, r <= 64)
  // ||L||_F^2
  double nl = 0.0;
  for (int e = threadIdx.x; e < m * r; e += blockDim.x) nl += L[e] * L[e];
  nl = blk_sum(nl, red);
  for (int e = threadIdx.x; e < m * r; e += blockDim.x) R[e] = L[e];
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    blk_mfma_tn(r, r, m, 1.0, Vh, ldv, R, m, G, r);                      // G = V^T R
    blk_mfma_nn(m, r, r, -1.0, Vh, ldv, G, r, 1.0, R, m);                // R -= V G
  }
  blk_mfma_tn(r, r, m, 1.0, R, m, R, m, W, r);                           // W = R^T R
  if (r <= 64) {
    blk_svd_qr<false>(W, r, r, Q, Xs, Xs + r * r, &flag, red, sig);
    blk_sort_desc(sig, r, order);
  } else {
    blk_jacobi(W, r, r, r, Q, r, &flag, red);
    __syncthreads();
    blk_colnorms_sorted(W, r, r, r, sig, order);
  }
  const double thresh = tol * tol * nl;
  int kept = 0;
  for (int t = 0; t < r; ++t)
    if (sig[order[t]] > thresh && sig[order[t]] > 0.0) ++kept;
  // X1 = R Q_k diag(lambda^-1/2): the kept eigenvectors, scaled, in G
  for (int e = threadIdx.x; e < r * kept; e += blockDim.x) {
    const int k = e % r, j = order[e / r];
    G[e] = Q[k + j * r] / sqrt(sig[j]);
  }
  __syncthreads();
  blk_mfma_nn(m, kept, r, 1.0, R, m, G, r, 0.0, X, m);
  if (kept > 0) {
    // second pass: project once more against V, then X = X1 Q2 diag(lambda2^-1/2)
    blk_mfma_tn(r, kept, m, 1.0, Vh, ldv, X, m, G, r);
    blk_mfma_nn(m, kept, r, -1.0, Vh, ldv, G, r, 1.0, X, m);
    blk_mfma_tn(kept, kept, m, 1.0, X, m, X, m, W, kept);
    // second pass: Cholesky of the well-conditioned Gram (span unchanged),
    // the eigen-decomposition as the fallback
    if (blk_chol_orth(W, kept, kept, Q, kept, red, &flag)) {
      // Q = L^{-T} is upper triangular with its lower part zero
      blk_mfma_nn(m, kept, kept, 1.0, X, m, Q, kept, 0.0, Vh + size_t(r) * ldv, ldv);
    } else {
      blk_mfma_tn(kept, kept, m, 1.0, X, m, X, m, W, kept);
      blk_jacobi(W, kept, kept, kept, Q, kept, &flag, red);
      __syncthreads();
      blk_colnorms_sorted(W, kept, kept, kept, sig, order);
      for (int e = threadIdx.x; e < kept * kept; e += blockDim.x) {
        const int k = e % kept, j = order[e / kept];
        G[e] = Q[k + j * kept] / sqrt(sig[j]);
      }
      __syncthreads();
      blk_mfma_nn(m, kept, kept, 1.0, X, m, G, kept, 0.0, Vh + size_t(r) * ldv, ldv);
    }
  }
  for (int e = threadIdx.x; e < m * (r - kept); e += blockDim.x) {
    int i = e % m, c = e / m;
    Vh[i + size_t(r + kept + c) * ldv] = 0.0;
  }
  if (threadIdx.x == 0) *count = kept;
}

// ------------------------------------------------------------------ truncation
__global__ __launch_bounds__(kWG) void k_truncate(const double *__restrict__ Sh, int P,
                                                 const int *kU, const int *kV, int r_base,
                                                 TruncOpt opt, double *Pp, double *Qp,
                                                 double *Sp, int lds, Ctl *ctl, double *work) {
  __shared__ double red[16];
  __shared__ int flag;
  __shared__ int order[128];
  __shared__ double sig[128];
  __shared__ double v[128], coef[128];
  extern __shared__ double dyn[];
  const int pU = r_base + (kU ? *kU : 0);
  const int pV = r_base + (kV ? *kV : 0);
  const bool cols = pU >= pV;                 // Jacobi on columns of Sh or of Sh^T
  const int p = cols ? pU : pV, q = cols ? pV : pU;
  // p x q matrix and q x q rotations in LDS when the launch provided room
  const bool in_lds = size_t(P) * P * 2 <= size_t(kTruncLdsDoubles);
  // room for the QR-preconditioned SVD (one more P x P block and 2P)
  const bool pre = svd_qr_fits(P);
  double *A = in_lds ? dyn : work;
  double *V = A + P * P;
  for (int e = threadIdx.x; e < p * q; e += blockDim.x) {
    int i = e % p, j = e / p;
    A[i + j * p] = cols ? Sh[i + j * P] : Sh[j + i * P];
  }
  __syncthreads();
  // the branch lets the LDS case address the matrices as LDS
  if (pre)
    blk_svd_qr<true>(dyn, p, q, dyn + P * P, dyn + 2 * P * P, dyn + 3 * P * P, &flag, red,
                     nullptr);
  else if (in_lds) blk_jacobi(dyn, p, p, q, dyn + P * P, q, &flag, red);
  else blk_jacobi(work, p, p, q, work + P * P, q, &flag, red);
  __syncthreads();
  blk_colnorms_sorted(A, p, p, q, sig, order);
  // rank
  int r1;
  double s1 = q > 0 ? sig[order[0]] : 0.0;
  if (opt.fixed) {
    r1 = opt.r_fixed < q ? opt.r_fixed : q;
  } else {
    double total = 0.0;
    for (int t = 0; t < q; ++t) total += sig[order[t]];
    double tail = 0.0;
    r1 = q;
    // smallest r1 with sum_{t >= r1} sigma_t <= tol * total
    for (int t = q; t >= 0; --t) {
      if (t < q) tail += sig[order[t]];
      if (tail <= opt.trunc_tol * total) r1 = t;
      else break;
    }
    if (r1 < opt.r_min) r1 = opt.r_min;
    if (r1 > opt.r_max) r1 = opt.r_max;
    if (r1 > q) r1 = q;
  }
  int kept = 0;
  if (s1 > 0.0)
    for (int t = 0; t < r1; ++t)
      if (sig[order[t]] > opt.floor_tol * s1) ++kept;
  // singular vectors of the kept directions: left (pU) and right (pV)
  for (int e = threadIdx.x; e < P * r1; e += blockDim.x) {
    Pp[e] = 0.0;
    Qp[e] = 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kept * p; e += blockDim.x) {
    int i = e % p, c = e / p;
    int j = order[c];
    double a = A[i + j * p] / sig[j];
    if (cols) Pp[i + c * P] = a;
    else Qp[i + c * P] = a;
  }
  for (int e = threadIdx.x; e < kept * q; e += blockDim.x) {
    int i = e % q, c = e / q;
    int j = order[c];
    double b = V[i + j * q];
    if (cols) Qp[i + c * P] = b;
    else Pp[i + c * P] = b;
  }
  __syncthreads();
  int cu = blk_fill(Pp, P, pU, kept, r1 - kept, pU, opt.fill_tol, v, coef, red);
  int cv = blk_fill(Qp, P, pV, kept, r1 - kept, pV, opt.fill_tol, v, coef, red);
  for (int e = threadIdx.x; e < r1 * r1; e += blockDim.x) {
    int i = e % r1, j = e / r1;
    Sp[i + j * lds] = (i == j && i < kept) ? sig[order[i]] : 0.0;
  }
  if (threadIdx.x == 0) {
    ctl->r_new = r1;
    if (cu != r1 || cv != r1) atomicOr(&ctl->flags, kFlagCompletion);
    if (!(s1 == s1) || s1 > 1e300) atomicOr(&ctl->flags, kFlagNonFinite);
  }
}

// ------------------------------------------------------------------ collided solves
__global__ __launch_bounds__(256) void k_collided_solve(int N, int m, int r, int n_mat,
                                                       const double *__restrict__ M,
                                                       const double *__restrict__ a, double dt,
                                                       const double *__restrict__ L0,
                                                       double *__restrict__ L1) {
  __shared__ double A[64 * 64];
  const int l = blockIdx.x;
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    int i = e % r, j = e / r;
    double s = (i == j) ? 1.0 : 0.0;
    for (int mi = 0; mi < n_mat; ++mi) s -= dt * a[mi * (N + 1) + l] * M[size_t(mi) * r * r + e];
    A[i + j * 64] = s;
  }
  __syncthreads();
  // Cholesky A = R R^T (lower R in place)
  for (int k = 0; k < r; ++k) {
    if (threadIdx.x == 0) A[k + k * 64] = sqrt(A[k + k * 64]);
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < r; i += blockDim.x) A[i + k * 64] /= A[k + k * 64];
    __syncthreads();
    for (int e = threadIdx.x; e < (r - k - 1) * (r - k - 1); e += blockDim.x) {
      int i = k + 1 + e % (r - k - 1), j = k + 1 + e / (r - k - 1);
      if (j <= i) A[i + j * 64] -= A[i + k * 64] * A[j + k * 64];
    }
    __syncthreads();
  }
  // rows p of degree l: solve R R^T x = L0(p, :)^T
  const int p0 = l * l, np = 2 * l + 1;
  for (int t = threadIdx.x; t < np; t += blockDim.x) {
    const int p = p0 + t;
    double x[64];
    for (int j = 0; j < r; ++j) x[j] = L0[p + size_t(j) * m];
    for (int i = 0; i < r; ++i) {
      double s = x[i];
      for (int k = 0; k < i; ++k) s -= A[i + k * 64] * x[k];
      x[i] = s / A[i + i * 64];
    }
    for (int i = r - 1; i >= 0; --i) {
      double s = x[i];
      for (int k = i + 1; k < r; ++k) s -= A[k + i * 64] * x[k];
      x[i] = s / A[i + i * 64];
    }
    for (int j = 0; j < r; ++j) L1[p + size_t(j) * m] = x[j];
  }
}

// ------------------------------------------------------------------ QR with completion
template <bool QL>
__global__ __launch_bounds__(kWG) void k_qr_complete(int m, int r, const double *__restrict__ L1,
                                                    const double *__restrict__ V, double tol,
                                                    double fill_tol, double *Vt, double *St,
                                                    int lds, Ctl *ctl, double *work) {
  __shared__ double red[16];
  extern __shared__ double dyn[];
  double *v = dyn;                  // m (LDS)
  double *coef = dyn + m;           // r (LDS)
  // the basis being built: in LDS when it fits (copied to Vt at the end)
  double *Q;
  if constexpr (QL) Q = dyn + m + r;
  else Q = Vt;
  (void)work;
  double nl = 0.0;
  for (int e = threadIdx.x; e < m * r; e += blockDim.x) nl += L1[e] * L1[e];
  const double thr = tol * sqrt(blk_sum(nl, red));
  int cnt = 0;
  for (int src = 0; src < 2; ++src) {
    const double *cand = src == 0 ? L1 : V;
    const double accept = src == 0 ? thr : fill_tol;
    for (int c = 0; c < r && cnt < r; ++c) {
      for (int t = threadIdx.x; t < m; t += blockDim.x) v[t] = cand[t + size_t(c) * m];
      __syncthreads();
      for (int pass = 0; pass < 2; ++pass) {
        blk_coefs(Q, m, m, cnt, v, coef);
        for (int t = threadIdx.x; t < m; t += blockDim.x) {
          double s = v[t];
#pragma unroll 8
          for (int j = 0; j < cnt; ++j) s -= Q[t + size_t(j) * m] * coef[j];
          v[t] = s;
        }
        __syncthreads();
      }
      double nv = 0.0;
      for (int t = threadIdx.x; t < m; t += blockDim.x) nv += v[t] * v[t];
      nv = sqrt(blk_sum(nv, red));
      if (nv > accept) {
        for (int t = threadIdx.x; t < m; t += blockDim.x) Q[t + size_t(cnt) * m] = v[t] / nv;
        ++cnt;
      }
      __syncthreads();
    }
  }
  if (cnt != r && threadIdx.x == 0) atomicOr(&ctl->flags, kFlagCompletion);
  if constexpr (QL)
    for (int e = threadIdx.x; e < m * cnt; e += blockDim.x) Vt[e] = Q[e];
  // S~ = L1^T V~
  blk_mfma_tn(r, r, m, 1.0, L1, m, Q, m, St, lds);
}

__global__ void k_check_finite(const double *__restrict__ x, int count, Ctl *ctl) {
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e < count) {
    double v = x[e];
    if (!(v == v) || fabs(v) > 1e300) atomicOr(&ctl->flags, kFlagNonFinite);
  }
}

__global__ void k_min_stop(int n, const double *__restrict__ w, int n_mat,
                           const double *__restrict__ Sk, double *out) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  double mn = 1e300;
  for (int x = threadIdx.x; x < n; x += 256) {
    double s = 0.0;
    for (int i = 0; i < n_mat; ++i) s += w[size_t(i) * n + x] * Sk[k * n_mat + i];
    mn = s < mn ? s : mn;
  }
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = red[0];
}

}  // namespace

void launch_small_gemm(int ta, int tb, int M, int N, int K, double alpha, const double *A,
                       int lda, size_t sA, const double *B, int ldb, size_t sB, double beta,
                       double *C, int ldc, size_t sC, int batch, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  dim3 grid((N + kT - 1) / kT, (M + kT - 1) / kT, batch);
  k_small_gemm<<<grid, kT * kT, 0, st>>>(ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta,
                                         C, ldc, sC);
}

void launch_lstep_stage(int m, int r, int ndk, const double *A, const double *C, int ldc,
                        const double *in, const double *L0, double *out, double coef,
                        double *T, size_t ts, hipStream_t st) {
  if (r <= 64 && (ndk == 4 || ndk == 6)) {   // one wave per term (2D, 3D)
    const int nkc = (r + 15) / 16;
    const size_t shm = (size_t(kLsKC) * (16 * nkc + 2) + size_t(ndk) * 16 * 16 * nkc) * 8;
#define DLRA_LSTEP(NKC, NDK)                                                                 \
  do {                                                                                       \
    auto kern = k_lstep_mfma<NKC, NDK>;                                                      \
    if (shm > 65536)                                                                         \
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),                         \
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));      \
    kern<<<(m + 15) / 16, 64 * NDK, shm, st>>>(m, r, A, C, ldc, in, L0, out, coef);          \
  } while (0)
#define DLRA_LSTEP_NKC(NDK)                  \
  switch (nkc) {                             \
    case 1: DLRA_LSTEP(1, NDK); break;       \
    case 2: DLRA_LSTEP(2, NDK); break;       \
    case 3: DLRA_LSTEP(3, NDK); break;       \
    default: DLRA_LSTEP(4, NDK); break;      \
  }
    if (ndk == 4) {
      DLRA_LSTEP_NKC(4)
    } else {
      DLRA_LSTEP_NKC(6)
    }
#undef DLRA_LSTEP_NKC
#undef DLRA_LSTEP
    return;
  }
  launch_small_gemm(0, 0, m, r, m, 1.0, A, m, size_t(m) * m, in, m, 0, 0.0, T, m, ts, ndk, st);
  k_lstep_combine<<<(m * r + 255) / 256, 256, 0, st>>>(m, r, ndk, T, ts, C, ldc, L0, out, coef);
}

void launch_sstep(int p, int ld, int ndk, const double *Ch, const double *Bh, double *S,
                  double *work, double h, int n_sub, hipStream_t st) {
  static_assert(kSStepMaxP == 4 * 32 && kSStepMaxDk == kSmMaxDk, "S-step limits");
  double *Wa = work, *Wb = work + size_t(ld) * ld;
  const double cf[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
  const size_t shm = sstep_mfma_lds(p, ndk);
  const auto kern = p <= 64 ? k_sstep_mfma<16> : k_sstep_mfma<32>;
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
  const dim3 grid((p + 15) / 16, (p + 15) / 16);
  for (int sub = 0; sub < n_sub; ++sub) {
    const double *in = S;
    double *outs[4] = {Wa, Wb, Wa, S};
    for (int stage = 0; stage < 4; ++stage) {
      kern<<<grid, 64 * ndk, shm, st>>>(p, ld, ndk, Ch, Bh, S, in, outs[stage], cf[stage] * h);
      in = outs[stage];
    }
  }
}

__global__ void k_copy_block(int rows, int cols, const double *__restrict__ src, int lds,
                             double *__restrict__ dst, int ldd, int dst_rows, int dst_cols,
                             double alpha) {
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= dst_rows * dst_cols) return;
  int i = e % dst_rows, j = e / dst_rows;
  double v = 0.0;
  if (i < rows && j < cols && src != nullptr) v = alpha * src[i + size_t(j) * lds];
  dst[i + size_t(j) * ldd] = v;
}

void launch_copy_block(int rows, int cols, const double *src, int lds, double *dst, int ldd,
                       int dst_rows, int dst_cols, double alpha, hipStream_t st) {
  int tot = dst_rows * dst_cols;
  if (tot <= 0) return;
  k_copy_block<<<(tot + 255) / 256, 256, 0, st>>>(rows, cols, src, lds, dst, ldd, dst_rows,
                                                  dst_cols, alpha);
}

void launch_gram_orth(int q, const double *W, double *T, int ldt, double tol2,
                      const double *normsq, int *count, const int *restrict_count, double *work,
                      hipStream_t st) {
  // A, V, and the QR-preconditioned SVD's X (q x q) and 2 q when they fit
  const size_t shm = (svd_qr_fits(q) ? size_t(3) * q * q + 2 * q : size_t(2) * q * q) * sizeof(double);
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_gram_orth),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
  k_gram_orth<<<1, kWG, shm, st>>>(q, W, T, ldt, tol2, normsq, count, restrict_count, work);
}

void launch_vaug(int m, int r, double *Vh, int ldv, const double *L, double tol, int *count,
                 double *work, hipStream_t st) {
  // G, W, Q, and for r <= 64 the QR-preconditioned SVD's scratch (r^2 + 2 r)
  const size_t shm = (r <= 64 ? size_t(4) * r * r + 2 * r : size_t(3) * r * r) * sizeof(double);
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_vaug),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
  k_vaug<<<1, kWG, shm, st>>>(m, r, Vh, ldv, L, tol, count, work);
}

void launch_truncate(const double *Sh, int P, const int *kU, const int *kV, int r_base,
                     TruncOpt opt, double *Pp, double *Qp, double *Sp, int lds, Ctl *ctl,
                     double *work, hipStream_t st) {
  const bool pre = svd_qr_fits(P);
  const size_t shm = pre ? (size_t(P) * P * 3 + 2 * P) * sizeof(double)
                     : size_t(P) * P * 2 <= size_t(kTruncLdsDoubles)
                         ? size_t(P) * P * 2 * sizeof(double)
                         : 0;
  if (shm > 60 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_truncate),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(kTruncLdsDoubles * sizeof(double)));
  k_truncate<<<1, kWG, shm, st>>>(Sh, P, kU, kV, r_base, opt, Pp, Qp, Sp, lds, ctl, work);
}

void launch_collided_solve(int N, int m, int r, int n_mat, const double *M, const double *a,
                           double dt, const double *L0, double *L1, hipStream_t st) {
  k_collided_solve<<<N + 1, 256, 0, st>>>(N, m, r, n_mat, M, a, dt, L0, L1);
}

void launch_qr_complete(int m, int r, const double *L1, const double *V, double tol,
                        double fill_tol, double *Vt, double *St, int lds, Ctl *ctl,
                        double *work, hipStream_t st) {
  const size_t shm = size_t(m + r) * sizeof(double);
  const size_t shm_q = shm + size_t(m) * r * sizeof(double);
  if (shm_q <= kSmallMaxLds) {
    if (shm_q > 64 * 1024)
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_qr_complete<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(kSmallMaxLds));
    k_qr_complete<true><<<1, kWG, shm_q, st>>>(m, r, L1, V, tol, fill_tol, Vt, St, lds, ctl,
                                               work);
  } else {
    k_qr_complete<false><<<1, kWG, shm, st>>>(m, r, L1, V, tol, fill_tol, Vt, St, lds, ctl,
                                              work);
  }
}

void launch_check_finite(const double *x, int count, Ctl *ctl, hipStream_t st) {
  if (count <= 0) return;
  k_check_finite<<<(count + 255) / 256, 256, 0, st>>>(x, count, ctl);
}

void launch_min_stop(int n, const double *w, int n_mat, const double *Sk, int n_steps,
                     double *out, hipStream_t st) {
  k_min_stop<<<n_steps, 256, 0, st>>>(n, w, n_mat, Sk, out);
}

}  // namespace dlra
