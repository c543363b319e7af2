// Kernel launchers of the DLRA proton-transport library (gfx950).
//
// Storage: every n-row matrix ("tall" matrix: U, K, Uhat ...) is column-major
// with leading dimension ld (cells fastest, a multiple of 64), element type T
// (double in FP64 mode, float in mixed mode).  Small matrices (r x r, m x r,
// m x m) are column-major double.  Sizes of tall kernels come from the host;
// small kernels read the data-dependent counts (augmentation ranks) from the
// device control block.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace dlra {

constexpr int kMaxMat = 16;     // base materials per problem
constexpr int kMaxBeams = 64;   // beams of one joint context
constexpr int kMaxSrc = 64;     // source columns n_mat * n_beams of one context
constexpr int kMaxDim = 3;

// Device control block (one per context).
struct Ctl {
  int r;          // current rank
  int kU, kV;     // new directions of the last augmentation
  int r_new;      // rank chosen by the last truncation
  int flags;      // error bits (kFlag*)
  int pad[3];
  double normsq;  // scratch: squared Frobenius norm of the last augmented matrix
  unsigned long long rt_substeps;   // ray tracer: Crank-Nicolson substeps marched
  unsigned long long rt_factors;    // ray tracer: block factorisations
};
constexpr int kFlagNonFinite = 1;
constexpr int kFlagRank = 2;
constexpr int kFlagStop = 4;
constexpr int kFlagCompletion = 8;

struct GridDev {
  int nx, ny, nz, n, dim;
  double inv2h[kMaxDim];   // 1 / (2 Delta_d)
};

// Rank / truncation options passed to the small kernels.
struct TruncOpt {
  int fixed;       // 1: rank r_fixed
  int r_fixed, r_min, r_max;
  double trunc_tol, floor_tol, fill_tol;
};

// ----------------------------------------------------------------- tall kernels
template <typename T>
void launch_inverse_stop(const GridDev &g, const T *w, int n_mat, const double *Si, T *s,
                         Ctl *ctl, hipStream_t st);

// out = K0 + coef * F(W), F(W) = -sum_d [ d^b_d(sW) Bp_d + d^f_d(sW) Bm_d ] (K-step
// right-hand side), on the matrix cores.  Bp: couplings packed by
// launch_pack_couplings, Bp[(dk RB + k) RB + j] = B_dk(k, j), RB = 16 ceil(r/16),
// dk = 2d + {0: +, 1: -}.
template <typename T>
void launch_kstep_stage(const GridDev &g, const T *s, const T *W, const T *K0, T *out, int ld,
                        int r, const T *Bp, double coef, hipStream_t st);
template <typename T>
void launch_pack_couplings(int ndk, int r, const double *B, int ldb, T *Bp, hipStream_t st);

// partial sums of C[dk](a, c) = sum_x X(x,a) d_dk(sY)(x,c), dk = 2d + {0: b, 1: f};
// then reduced into C (2*dim blocks, each p x p col-major, ldc).
template <typename T, typename Acc>
void launch_stencil_projection(const GridDev &g, const T *s, const T *X, int ld, int p,
                               double *C, int ldc, double *partial, size_t partial_elems,
                               hipStream_t st);

// G = X^T diag(wt) Y over the n rows (p x q col-major, ldg).  wt: nullptr (no
// weight), or the product w_mat(x) * s(x) when wmat != nullptr.
template <typename T, typename Acc>
void launch_gram(int n, const T *X, int ldx, int p, const T *Y, int ldy, int q,
                 const T *wmat, const T *s, double *G, int ldg, double *partial,
                 size_t partial_elems, hipStream_t st);

// H(a, b n_mat + i) = sum_x X(x, a) w_i(x) psi_b(x) for i < n_mat, b < n_beams
// (p x n_mat n_beams, ldh); psi_b = psi + b * pstride.
template <typename T, typename Acc>
void launch_xt_source(int n, const T *X, int ld, int p, const T *w, int n_mat, int n_beams,
                      const T *psi, size_t pstride, double *H, int ldh, double *partial,
                      size_t partial_elems, hipStream_t st);

// sum of squares of an n x q tall matrix -> *out (double)
template <typename T>
void launch_sumsq(int n, const T *X, int ld, int q, double *out, double *partial,
                  size_t partial_elems, hipStream_t st);

// Z(x, c) = alpha * Y(x, c) + beta * sum_a X(x, a) G(a, c), c < q (Y may be nullptr
// or alias Z).  When dose != nullptr, also dose[x] += dscale * sum_c Z(x,c) dc[c].
template <typename T>
void launch_update(int n, const T *X, int ldx, int p, const double *G, int ldg, double beta,
                   const T *Y, int ldy, double alpha, T *Z, int ldz, int q, double *dose,
                   const double *dc, double dscale, hipStream_t st);

// K(x, c) = sum_a U(x,a) St(a,c) + dt sum_{b,i} w_i(x) psi_b(x) Cg(c, b n_mat + i)
// (uncollided K; psi_b = psi + b * pstride)
template <typename T>
void launch_source_k(int n, const T *U, int ld, int r, const double *St, int lds,
                     const T *w, int n_mat, int n_beams, const T *psi, size_t pstride,
                     const double *Cg, int ldcg, double dt, T *K, hipStream_t st);

// ----------------------------------------------------------------- small kernels (double)
// C[z] = alpha op(A[z]) op(B[z]) + beta C[z], batched over blockIdx.z with
// strides; op = transpose when ta/tb.
void launch_small_gemm(int ta, int tb, int M, int N, int K, double alpha, const double *A,
                       int lda, size_t sA, const double *B, int ldb, size_t sB, double beta,
                       double *C, int ldc, size_t sC, int batch, hipStream_t st);

// out = L0 + coef * F_L(in), F_L(L) = -sum_dk A_dk L C_dk^T (m x r, ld m);
// T: scratch for the ndk products A_dk in (m x r each, ts apart)
void launch_lstep_stage(int m, int r, int ndk, const double *A, const double *C, int ldc,
                        const double *in, const double *L0, double *out, double coef,
                        double *T, size_t ts, hipStream_t st);

// Throughput probes (roofs.hip): kind 0/1 FP32/FP64 16x16x4 MFMA, 2/3
// FP32/FP64 vector FMA; blocks of 256 threads, out[blocks * 256]
void launch_roof_probe(int kind, int iters, int blocks, double *out, hipStream_t st);
double roof_probe_flops(int kind, int iters, int blocks);

// Horner RK4 of the S-step on the p x p matrix S (leading dim ld, as Ch, Bh
// whose dk-th blocks are ld*ld apart), n_sub substeps.  Requires
// p <= kSStepMaxP and 2 <= ndk <= kSStepMaxDk (one wave per term).
constexpr int kSStepMaxP = 128;
constexpr int kSStepMaxDk = 6;
void launch_sstep(int p, int ld, int ndk, const double *Ch, const double *Bh, double *S,
                  double *work, double h, int n_sub, hipStream_t st);

// dst(0:rows, 0:cols) = alpha * src(0:rows, 0:cols); whole dst (dst_rows x dst_cols) zeroed first
void launch_copy_block(int rows, int cols, const double *src, int lds, double *dst, int ldd,
                       int dst_rows, int dst_cols, double alpha, hipStream_t st);

// eig of the symmetric PSD q x q matrix W (ld q): T = Q_k diag(lambda_k^-1/2)
// for lambda > thresh2 (relative to *normsq when rel); count -> *count.
// When restrict_count != nullptr only the leading *restrict_count rows/cols
// are used and nothing is dropped (second orthonormalisation pass).
void launch_gram_orth(int q, const double *W, double *T, int ldt, double tol2,
                      const double *normsq, int *count, const int *restrict_count,
                      double *work, hipStream_t st);

// V augmentation: Vh(:, r + j) = orth((I - V V^T) L), r columns of V at Vh.
void launch_vaug(int m, int r, double *Vh, int ldv, const double *L, double tol,
                 int *count, double *work, hipStream_t st);

// truncation of Shat (pU x pV, padded ld P): P' (P x r'), Q' (P x r'), S' (r' x r')
void launch_truncate(const double *Sh, int P, const int *pU_extra, const int *pV_extra,
                     int r_base, TruncOpt opt, double *Pp, double *Qp, double *Sp, int lds,
                     Ctl *ctl, double *work, hipStream_t st);

// collided self-scattering L-step: per degree l, (I - dt sum_i a_il M_i) X = L0 rows
void launch_collided_solve(int N, int m, int r, int n_mat, const double *M, const double *a,
                           double dt, const double *L0, double *L1, hipStream_t st);

// V~ = ordered CGS2 over [L1 | V], S~ = L1^T V~ (m x r)
void launch_qr_complete(int m, int r, const double *L1, const double *V, double tol,
                        double fill_tol, double *Vt, double *St, int lds, Ctl *ctl,
                        double *work, hipStream_t st);

// reduction of per-block partial sums: out[e] = sum_b partial[b*elems + e]
// plan objective over beam weights and its gradient (out[0] = J, out[1 + b] =
// dJ/dw_b); work holds plan_objective_work(n, nb) doubles
constexpr int kPlanMaxBeams = 64;
constexpr int kPlanBlocks = 512;
struct PlanWeights {
  double w[kPlanMaxBeams];
};
size_t plan_objective_work(int n, int nb);
void launch_plan_objective(int n, int nb, const double *doses, const PlanWeights &pw,
                           const unsigned char *target, double dhat, double lam, double *work,
                           double *out, hipStream_t st);
// the same in one pass over the doses with only block partials as scratch:
// plan_objective_fused_scratch(nb) doubles, partial rows first; out may lie
// behind them in the same buffer
size_t plan_objective_fused_scratch(int nb);
void launch_plan_objective_fused(int n, int nb, const double *doses, const PlanWeights &pw,
                                 const unsigned char *target, double dhat, double lam,
                                 double *scratch, double *out, hipStream_t st);

// ----------------------------------------------------------------- ray tracer
struct RayParams {
  int G;                 // energy groups
  int n_mat;
  int n_steps;
  int ng_step;           // groups per step-integral window
  int n_rays;            // rays of the beam
  int n;                 // cells
  // grid rows of an axis-aligned beam (axis >= 0): rays[r] is the first cell
  // of row r; oblique beams (axis = -1): rays[r] is the target cell
  int axis, sign;        // beam axis (0, 1, 2) and direction
  int row_len;           // cells per row
  int row_stride;        // cell index stride along the row
  double half;           // half-cell length along the axis
  int n_half;            // CN substeps per half cell
  double h_max;          // longest CN substep (cm)
};
struct RayGeom {
  int nx, ny, nz, dim;
  double D[3];           // cell sizes (cm)
  double L[3];           // box lengths (cm)
  double om[3];          // unit direction of flight
};
// Up to kRayWaveGroups groups a ray is marched by one wave (two groups per
// lane) with no scratch; more groups take one thread per ray, and the scratch
// then holds kRayScratchPerGroup * G * batch doubles (c, y: 3G each; Dinv, F,
// E: 9G each, per ray of a batch).
constexpr int kRayWaveGroups = 128;
constexpr int kRayScratchPerGroup = 33;
// uncollided tables of one beam (scratch and batch unused up to kRayWaveGroups)
template <typename T>
void launch_raytrace(const RayParams &rp, const RayGeom &geo, const int *rays,
                     const double *ray_f, const double *w, const double *Adiag,
                     const double *Aup, const double *Alo, const double *mass, const double *c0,
                     const int *step_g0, const double *step_w, const double *stop_w,
                     double *scratch, size_t batch, T *psibar, double *Du, Ctl *ctl,
                     hipStream_t st);

// min over cells of sum_i w_i S_i(E_k) for every step k
void launch_min_stop(int n, const double *w, int n_mat, const double *Sk, int n_steps,
                     double *out, hipStream_t st);

void launch_check_finite(const double *x, int count, Ctl *ctl, hipStream_t st);

}  // namespace dlra
