// C ABI and host orchestration of one energy step (see include/dlra.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <thread>
#include <mutex>
#include <vector>

#include "dlra.h"
#include "kernels.hpp"
#include "setup.hpp"

using namespace dlra;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw HipError(std::string(#call) + ": " + hipGetErrorString(e_));               \
  } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxRank = 50;      // 2 r_max <= 100 columns in the small kernels
static_assert(2 * kMaxRank <= kSStepMaxP && 2 * 3 <= kSStepMaxDk, "S-step limits");  // ndk = 2 dim
constexpr int kPartialBlocks = 1024;   // partial-sum blocks of a contraction

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ------------------------------------------------------------------ workspace plan
struct Plan {
  size_t bytes = 0;
  size_t take(size_t b) {
    size_t off = bytes;
    bytes += align256(b);
    return off;
  }
  // offsets
  size_t w_t, w_d, s, tall[4], psibar, dose_c, dose_u, Apm, AV, stepS, stepA, stepG, minstop,
      egrid_s, egrid_min;
  size_t S, V, Vn, Bm, Bpk, Cm, Ch, Sh, Pp, Qp, Sp, G1, G2, Wg, T1, T2, Lm, L0, La, Lb, Mi, H, Cg, dc,
      tmp, work, partial, ctl;
  size_t rt_diag, rt_up, rt_lo, rt_mass, rt_c0, rt_g0, rt_sw, rt_stopw, rt_rays, rt_f,
      rt_scratch;
  size_t partial_elems = 0;
};

struct Dims {
  int n, dim, ndk, N, m, n_mat, n_beams, n_src, R, P, ld, n_steps, G, ray_batch;
  size_t tsize;
};

constexpr int kCflIntervals = 4096;   // trapezoid intervals of the CFL energy grid
constexpr int kRayBatch = 32768;      // rays per ray-tracer launch

bool make_dims(const dlra_grid *g, int n_mat, int n_beams, const dlra_options *o, Dims &d,
               std::string &err) {
  if (!g || !o) {
    err = "null grid or options";
    return false;
  }
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0)) {
    err = "grid sizes and spacings must be positive";
    return false;
  }
  if (n_mat < 1 || n_mat > kMaxMat) {
    err = "n_mat must be in [1, 16]";
    return false;
  }
  if (n_beams < 1 || n_beams > kMaxBeams || n_mat * n_beams > kMaxSrc) {
    err = "n_beams must be in [1, 64] with n_mat * n_beams <= 64";
    return false;
  }
  if (o && (o->collision != DLRA_BOLTZMANN && o->collision != DLRA_FOKKER_PLANCK)) {
    err = "collision must be DLRA_BOLTZMANN or DLRA_FOKKER_PLANCK";
    return false;
  }
  if (o && (o->egrid < DLRA_EGRID_UNIFORM || o->egrid > DLRA_EGRID_USER)) {
    err = "egrid must be one of DLRA_EGRID_*";
    return false;
  }
  if (o->pn_degree < 0 || o->pn_degree > 40) {
    err = "pn_degree must be in [0, 40]";
    return false;
  }
  if (o->n_steps < 1) {
    err = "n_steps must be >= 1";
    return false;
  }
  if (o->precision != DLRA_FP64 && o->precision != DLRA_MIXED) {
    err = "precision must be DLRA_FP64 or DLRA_MIXED";
    return false;
  }
  if (o->rank_mode != DLRA_RANK_FIXED && o->rank_mode != DLRA_RANK_ADAPTIVE) {
    err = "rank_mode must be DLRA_RANK_FIXED or DLRA_RANK_ADAPTIVE";
    return false;
  }
  d.N = o->pn_degree;
  d.m = (d.N + 1) * (d.N + 1);
  d.R = o->rank_mode == DLRA_RANK_FIXED ? o->r : o->r_max;
  int r0 = o->rank_mode == DLRA_RANK_FIXED ? o->r : o->r_min;
  if (d.R < 1 || d.R > kMaxRank || r0 < 1 || r0 > d.R || d.R > d.m) {
    err = "ranks must satisfy 1 <= r (r_min) <= r_max <= min(50, (N+1)^2)";
    return false;
  }
  if (o->rank_mode == DLRA_RANK_ADAPTIVE && o->r_min > o->r_max) {
    err = "r_min > r_max";
    return false;
  }
  if (o->n_groups < 4 || o->n_groups > 4096) {
    err = "n_groups must be in [4, 4096]";
    return false;
  }
  long long n = (long long)g->nx * g->ny * g->nz;
  if (n > (1LL << 30)) {
    err = "too many cells";
    return false;
  }
  d.n = int(n);
  d.dim = g->nz == 1 ? 2 : 3;
  d.ndk = 2 * d.dim;
  d.n_mat = n_mat;
  d.n_beams = n_beams;
  d.n_src = n_mat * n_beams;
  d.P = 2 * d.R;
  // columns 64-element aligned, and not a power of two apart: a power-of-two
  // column stride puts the same cell of every column on the same memory
  // channels
  d.ld = (d.n + 63) / 64 * 64 + 64;
  d.n_steps = o->n_steps;
  d.G = o->n_groups;
  d.tsize = o->precision == DLRA_FP64 ? 8 : 4;
  // rays traced together: rows of an axis-aligned beam, or target cells of an
  // oblique one, in batches that bound the per-ray scratch
  d.ray_batch = std::min(d.n, kRayBatch);
  return true;
}

Plan make_plan(const Dims &d) {
  Plan p;
  const size_t T = d.tsize, n = d.n, ld = d.ld, P = d.P, R = d.R, m = d.m;
  p.w_t = p.take(d.n_mat * n * T);
  p.w_d = p.take(d.n_mat * n * 8);
  p.s = p.take(n * T);
  for (int i = 0; i < 4; ++i) p.tall[i] = p.take(ld * P * T);
  p.psibar = p.take(size_t(d.n_beams) * d.n_steps * n * T);
  p.dose_c = p.take(n * 8);
  p.dose_u = p.take(n * 8);
  p.Apm = p.take(d.ndk * m * m * 8);
  p.AV = p.take(d.ndk * m * P * 8);
  p.stepS = p.take(size_t(d.n_steps) * d.n_mat * 8);
  p.stepA = p.take(size_t(d.n_steps) * d.n_mat * (d.N + 1) * 8);
  p.stepG = p.take(size_t(d.n_steps) * m * d.n_src * 8);
  p.minstop = p.take(size_t(d.n_steps) * 8);
  p.egrid_s = p.take(size_t(kCflIntervals + 1) * d.n_mat * 8);
  p.egrid_min = p.take(size_t(kCflIntervals + 1) * 8);
  p.S = p.take(R * R * 8);
  p.V = p.take(m * P * 8);
  p.Vn = p.take(m * P * 8);
  p.Bm = p.take(d.ndk * P * P * 8);
  p.Bpk = p.take(d.ndk * 64 * 64 * 8);
  p.Cm = p.take(d.ndk * P * P * 8);
  p.Ch = p.take(d.ndk * P * P * 8);
  p.Sh = p.take(P * P * 8);
  p.Pp = p.take(P * R * 8);
  p.Qp = p.take(P * R * 8);
  p.Sp = p.take(R * R * 8);
  p.G1 = p.take(P * P * 8);
  p.G2 = p.take(P * P * 8);
  p.Wg = p.take(P * P * 8);
  p.T1 = p.take(P * P * 8);
  p.T2 = p.take(P * P * 8);
  p.Lm = p.take(m * P * 8);
  p.L0 = p.take(m * P * 8);
  p.La = p.take(m * P * 8);
  p.Lb = p.take(m * P * 8);
  p.Mi = p.take(d.n_mat * R * R * 8);
  p.H = p.take(P * kMaxSrc * 8);
  p.Cg = p.take(P * kMaxSrc * 8);
  p.dc = p.take(P * 8);
  p.tmp = p.take(P * 8);
  p.work = p.take((4 * P * P + 3 * m * P + 4 * P + 64) * 8);
  size_t ntile = (n + 31) / 32;
  size_t nb = std::min<size_t>(kPartialBlocks, ntile);
  // partial blocks, their sum and up to 64 segment sums of the reduction
  p.partial_elems = (nb + 1 + 64) * std::max<size_t>({d.ndk * P * P, P * kMaxSrc, 64});
  p.partial = p.take(p.partial_elems * 8);
  p.ctl = p.take(sizeof(Ctl));
  const size_t G = d.G;
  p.rt_diag = p.take(d.n_mat * G * 9 * 8);
  p.rt_up = p.take(d.n_mat * G * 9 * 8);
  p.rt_lo = p.take(d.n_mat * G * 9 * 8);
  p.rt_mass = p.take(3 * 8);
  p.rt_c0 = p.take(size_t(d.n_beams) * 3 * G * 8);
  p.rt_g0 = p.take(size_t(d.n_steps) * 4);
  p.rt_sw = p.take(size_t(d.n_steps) * G * 3 * 8);
  p.rt_stopw = p.take(d.n_mat * 3 * G * 8);
  p.rt_rays = p.take(size_t(d.n_beams) * n * 4);
  p.rt_f = p.take(size_t(d.n_beams) * n * 8);
  p.rt_scratch =
      p.take(G > size_t(kRayWaveGroups) ? size_t(kRayScratchPerGroup) * G * d.ray_batch * 8 : 0);
  return p;
}

}  // namespace

// ==================================================================== context
struct dlra_ctx {
  Dims d;
  Plan plan;
  dlra_grid grid;
  dlra_options opt;
  std::vector<dlra_beam> beams;
  GridDev gdev;
  hipStream_t st = nullptr;
  hipStream_t st2 = nullptr;            // side stream of the L-step (default priority)
  int device = 0;                       // HIP device the context was created on
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_kdone = nullptr;
  hipGraphExec_t graph_exec = nullptr;   // the last dlra_run_graph launch
  hipStream_t st_cap = nullptr;          // dlra_run_graph records on this stream
  char *base = nullptr;
  // host-side state
  int r = 0;
  int step = 0;
  bool traced = false;
  double e_max = 0, e_cut = 0;
  std::vector<double> edges;   // E_0 = E_max > ... > E_n = E_cut
  std::vector<double> dtk;     // dt_k = E_k - E_{k+1}
  std::vector<int> n_sub;
  TruncOpt topt;
  std::vector<int> replay;   // prescribed ranks of the next truncations (test access)
  size_t replay_pos = 0;
  // rays of every beam
  std::vector<RayParams> rps;
  std::vector<RayGeom> rgeo;
  // rotating tall buffers: 0 = Uhat, 1 = K, 2 = Wa, 3 = Wb
  void *tall[4];
  double *V, *Vn;
  // event-based timing
  struct Rec {
    hipEvent_t a, b;
    int ph;
    long long n;   // launches the pair brackets
  };
  int prof = 0;   // 0 off, 1 every phase, 2 light (step and K-step loop only)
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  double prof_ms[DLRA_PH_COUNT] = {};
  long long prof_n[DLRA_PH_COUNT] = {};

  template <typename T>
  T *at(size_t off) {
    return reinterpret_cast<T *>(base + off);
  }
  Ctl *ctl() { return at<Ctl>(plan.ctl); }
  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) throw std::runtime_error("hipEventCreate failed");
    return e;
  }
  void drain() {
    if (pending.empty()) return;
    if (hipStreamSynchronize(st) != hipSuccess) throw std::runtime_error("stream sync failed");
    for (auto &r : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        prof_ms[r.ph] += ms;
        prof_n[r.ph] += r.n;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  ~dlra_ctx() {
    if (st2) {
      (void)hipStreamSynchronize(st2);
      (void)hipStreamDestroy(st2);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_kdone) (void)hipEventDestroy(ev_kdone);
    if (graph_exec) {
      (void)hipStreamSynchronize(st);
      (void)hipGraphExecDestroy(graph_exec);
    }
    if (st_cap) (void)hipStreamDestroy(st_cap);
    if (!pending.empty() || !pool.empty()) {
      (void)hipStreamSynchronize(st);
      for (auto &r : pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
      }
      for (auto e : pool) (void)hipEventDestroy(e);
    }
  }
};

namespace {

// Records an event pair around a phase when timing is on.  An event record
// between two kernels on a stream costs several microseconds of idle device
// time, so the light level (2) records only the pairs marked kLight: the
// whole step and, once per step, the K-step RK4 loop counted as its stage
// launches; the full level (1) records the others.
enum TimerLevel { kFull = 1, kLight = 2, kBoth = 3 };
struct PhaseTimer {
  dlra_ctx *c;
  int ph;
  hipStream_t s;
  long long n;
  hipEvent_t a = nullptr;
  PhaseTimer(dlra_ctx *c_, int ph_, hipStream_t s_ = nullptr, int when = kFull,
             long long n_ = 1)
      : c(c_), ph(ph_), s(s_ ? s_ : c_->st), n(n_) {
    if (c->prof & when) {
      a = c->event();
      (void)hipEventRecord(a, s);
    }
  }
  ~PhaseTimer() {
    if (a) {
      hipEvent_t b = c->event();
      (void)hipEventRecord(b, s);
      c->pending.push_back({a, b, ph, n});
    }
  }
};

void upload(dlra_ctx *c, size_t off, const void *src, size_t bytes) {
  HIPCHK(hipMemcpyAsync(c->base + off, src, bytes, hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
}

template <typename T>
void upload_cast(dlra_ctx *c, size_t off, const double *src, size_t count) {
  std::vector<T> tmp(src, src + count);
  HIPCHK(hipMemcpyAsync(c->base + off, tmp.data(), count * sizeof(T), hipMemcpyHostToDevice,
                        c->st));
  HIPCHK(hipStreamSynchronize(c->st));
}

// Ordered CGS2 with drop over the columns of cand (m x nc, col-major), then
// unit vectors, until r orthonormal columns (initial angular basis).
std::vector<double> initial_angular_basis(const std::vector<double> &g0, int m, int nc, int r,
                                          double tol, double fill_tol) {
  std::vector<double> Q;
  double nrm = 0.0;
  for (double v : g0) nrm += v * v;
  nrm = std::sqrt(nrm);
  int cnt = 0;
  auto try_add = [&](std::vector<double> v, double thr) {
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<double> coef(cnt, 0.0);
      for (int j = 0; j < cnt; ++j)
        for (int t = 0; t < m; ++t) coef[j] += Q[size_t(j) * m + t] * v[t];
      for (int t = 0; t < m; ++t)
        for (int j = 0; j < cnt; ++j) v[t] -= Q[size_t(j) * m + t] * coef[j];
    }
    double nv = 0.0;
    for (double x : v) nv += x * x;
    nv = std::sqrt(nv);
    if (nv > thr) {
      for (double &x : v) x /= nv;
      Q.insert(Q.end(), v.begin(), v.end());
      ++cnt;
    }
  };
  for (int c = 0; c < nc && cnt < r; ++c)
    try_add(std::vector<double>(g0.begin() + size_t(c) * m, g0.begin() + size_t(c + 1) * m),
            tol * nrm);
  for (int c = 0; c < m && cnt < r; ++c) {
    std::vector<double> e(m, 0.0);
    e[c] = 1.0;
    try_add(e, fill_tol);
  }
  if (cnt != r) throw std::runtime_error("initial angular basis: completion failed");
  return Q;
}

// Energy edges E_0 = E_max > ... > E_n = E_cut of the context's grid mode.
// The CFL grid needs S_min(E) = min_x sum_i w_i S_i(E) on kCflIntervals + 1
// energies, taken on the device.
void energy_edges(dlra_ctx *c, const dlra_materials *mat) {
  const Dims &d = c->d;
  const Plan &p = c->plan;
  const int n = d.n_steps;
  std::vector<double> &E = c->edges;
  E.assign(n + 1, 0.0);
  const double e_max = c->e_max, e_cut = c->e_cut;
  switch (c->opt.egrid) {
    case DLRA_EGRID_UNIFORM: {
      const double dt = (e_max - e_cut) / n;
      for (int k = 0; k <= n; ++k) E[k] = e_max - k * dt;
      break;
    }
    case DLRA_EGRID_PROPORTIONAL:
      for (int k = 0; k <= n; ++k) E[k] = e_cut * std::pow(e_max / e_cut, 1.0 - double(k) / n);
      break;
    case DLRA_EGRID_CFL: {
      const int K = kCflIntervals, nm = d.n_mat, ne = mat->n_e;
      const double h = (e_max - e_cut) / K;
      std::vector<double> x(K + 1), Sk(size_t(K + 1) * nm), smin(K + 1);
      for (int j = 0; j <= K; ++j) {
        x[j] = e_cut + h * j;
        for (int i = 0; i < nm; ++i)
          Sk[size_t(j) * nm + i] = interp(mat->e, mat->S + size_t(i) * ne, ne, x[j]);
      }
      upload(c, p.egrid_s, Sk.data(), Sk.size() * 8);
      launch_min_stop(d.n, c->at<double>(p.w_d), nm, c->at<double>(p.egrid_s), K + 1,
                      c->at<double>(p.egrid_min), c->st);
      HIPCHK(hipMemcpyAsync(smin.data(), c->base + p.egrid_min, smin.size() * 8,
                            hipMemcpyDeviceToHost, c->st));
      HIPCHK(hipStreamSynchronize(c->st));
      std::vector<double> R(K + 1, 0.0);
      for (int j = 0; j < K; ++j) {
        if (!(smin[j] > 0) || !(smin[j + 1] > 0))
          throw std::invalid_argument("stopping power must be positive in every cell");
        R[j + 1] = R[j] + 0.5 * h * (1.0 / smin[j] + 1.0 / smin[j + 1]);
      }
      // invert R by linear interpolation (R ascends)
      for (int k = 0; k <= n; ++k) {
        const double t = R[K] * (1.0 - double(k) / n);
        int j = int(std::upper_bound(R.begin(), R.end(), t) - R.begin()) - 1;
        if (j >= K) {
          E[k] = x[K];
          continue;
        }
        j = std::max(j, 0);
        const double slope = (x[j + 1] - x[j]) / (R[j + 1] - R[j]);
        E[k] = x[j] + slope * (t - R[j]);
      }
      break;
    }
    default:
      for (int k = 0; k <= n; ++k) E[k] = c->opt.egrid_points[k];
  }
  if (c->opt.egrid != DLRA_EGRID_USER) {
    E[0] = e_max;
    E[n] = e_cut;
  }
  c->dtk.resize(n);
  for (int k = 0; k < n; ++k) c->dtk[k] = E[k] - E[k + 1];
}

// Per-step collision coefficients from the table differences dg[l] = G_0 - G_l
// at the step midpoint: self-scattering a_l and in-scattering factors gt_l
// (l = 0..N) and the removal rate of the uncollided flux.
//   Boltzmann with the extended transport correction (Sec. 3.3.1):
//     a_l = G_l - G_0, gt_l = G_l - G_{N+1}, removal G_0 - G_{N+1};
//   Fokker-Planck (Sec. 2.1, Sec. 3.1): a_l = gt_l = -xi_1 l (l+1) / 2 with
//     xi_1 = G_0 - G_1, no removal.
void collision_coeffs(int model, int N, const double *dg, double *a, double *gt) {
  if (model == DLRA_FOKKER_PLANCK) {
    for (int l = 0; l <= N; ++l) {
      a[l] = -0.5 * dg[1] * double(l) * double(l + 1);
      gt[l] = a[l];
    }
    return;
  }
  for (int l = 0; l <= N; ++l) {
    a[l] = -dg[l];
    gt[l] = dg[N + 1] - dg[l];
  }
}

template <typename T>
int init_impl(dlra_ctx *c, const dlra_materials *mat) {
  const Dims &d = c->d;
  const Plan &p = c->plan;
  const int n = d.n, m = d.m, N = d.N, nm = d.n_mat, nb = d.n_beams, ns_ = d.n_src;
  HIPCHK(hipMemsetAsync(c->base, 0, p.bytes, c->st));
  // ---- angular algebra
  std::vector<double> A[3];
  streaming_matrices(N, A);
  std::vector<double> Apm(size_t(d.ndk) * m * m);
  for (int dd = 0; dd < d.dim; ++dd) {
    std::vector<double> Ap, Am;
    eigen_split(A[dd], m, Ap, Am);
    // symmetric: row- and column-major coincide
    std::copy(Ap.begin(), Ap.end(), Apm.begin() + size_t(2 * dd) * m * m);
    std::copy(Am.begin(), Am.end(), Apm.begin() + size_t(2 * dd + 1) * m * m);
  }
  upload(c, p.Apm, Apm.data(), Apm.size() * 8);
  std::vector<double> TM(size_t(nb) * m);
  for (int b = 0; b < nb; ++b) beam_moments(N, c->beams[b].dir, TM.data() + size_t(b) * m);
  // ---- materials
  upload(c, p.w_d, mat->w, size_t(nm) * n * 8);
  if (sizeof(T) == 8) {
    upload(c, p.w_t, mat->w, size_t(nm) * n * 8);
  } else {
    upload_cast<T>(c, p.w_t, mat->w, size_t(nm) * n);
  }
  // ---- energy grid and per-step coefficients at the step midpoints
  if (c->opt.egrid == DLRA_EGRID_USER) {
    c->e_max = c->opt.egrid_points[0];
    c->e_cut = c->opt.egrid_points[d.n_steps];
  } else {
    c->e_max = 0.0;
    for (const dlra_beam &bm : c->beams)
      c->e_max = std::max(c->e_max, bm.E0 + c->opt.e_max_sigmas * bm.sigma_E);
    c->e_cut = c->opt.e_cut;
  }
  energy_edges(c, mat);
  std::vector<double> stepS(size_t(d.n_steps) * nm), stepA(size_t(d.n_steps) * nm * (N + 1)),
      stepG(size_t(d.n_steps) * m * ns_);
  const int ne = mat->n_e, nl = mat->n_leg;
  for (int k = 0; k < d.n_steps; ++k) {
    const double E = 0.5 * (c->edges[k] + c->edges[k + 1]);
    for (int i = 0; i < nm; ++i) {
      stepS[size_t(k) * nm + i] = interp(mat->e, mat->S + size_t(i) * ne, ne, E);
      std::vector<double> dg(N + 2), col(ne), a(N + 1), gt(N + 1);
      for (int l = 0; l < N + 2; ++l) {
        for (int e = 0; e < ne; ++e) col[e] = mat->dG[(size_t(i) * ne + e) * nl + l];
        dg[l] = interp(mat->e, col.data(), ne, E);
      }
      collision_coeffs(c->opt.collision, N, dg.data(), a.data(), gt.data());
      for (int l = 0; l <= N; ++l) stepA[(size_t(k) * nm + i) * (N + 1) + l] = a[l];
      // source column b n_mat + i: g_{i,b} = gt_l(p) T_M,b
      for (int b = 0; b < nb; ++b)
        for (int l = 0; l <= N; ++l)
          for (int kk = -l; kk <= l; ++kk) {
            int pidx = l * l + l + kk;
            stepG[(size_t(k) * ns_ + size_t(b) * nm + i) * m + pidx] =
                gt[l] * TM[size_t(b) * m + pidx];
          }
    }
  }
  upload(c, p.stepS, stepS.data(), stepS.size() * 8);
  upload(c, p.stepA, stepA.data(), stepA.size() * 8);
  upload(c, p.stepG, stepG.data(), stepG.size() * 8);
  // ---- RK4 substeps: minimum stopping power per step
  launch_min_stop(n, c->at<double>(p.w_d), nm, c->at<double>(p.stepS), d.n_steps,
                  c->at<double>(p.minstop), c->st);
  std::vector<double> minstop(d.n_steps);
  HIPCHK(hipMemcpyAsync(minstop.data(), c->base + p.minstop, d.n_steps * 8,
                        hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  double nu = c->opt.nu_max > 0 ? c->opt.nu_max : (d.dim == 2 ? 0.45 : 0.35);
  double hmin = d.dim == 2 ? std::min(c->grid.dx, c->grid.dy)
                           : std::min(c->grid.dx, std::min(c->grid.dy, c->grid.dz));
  c->n_sub.resize(d.n_steps);
  for (int k = 0; k < d.n_steps; ++k) {
    if (!(minstop[k] > 0)) return fail(DLRA_E_INVALID, "stopping power must be positive in every cell");
    int ns = std::max(1, int(std::ceil(c->dtk[k] / (nu * minstop[k] * hmin) - 1e-9)));
    if (c->opt.n_sub_max > 0 && ns > c->opt.n_sub_max)
      return fail(DLRA_E_CFL, "energy step " + std::to_string(k) + " needs " +
                                  std::to_string(ns) + " RK4 substeps > n_sub_max");
    c->n_sub[k] = ns;
  }
  // ---- initial state: S = 0, U unit vectors at floor((j+1/2) n / r), V from
  // the source directions of the first step
  const int r0 = c->opt.rank_mode == DLRA_RANK_FIXED ? c->opt.r : c->opt.r_min;
  c->r = r0;
  {
    T one = T(1);
    for (int j = 0; j < r0; ++j) {
      size_t cell = size_t((j + 0.5) * double(n) / r0);
      HIPCHK(hipMemcpyAsync(c->at<T>(p.tall[0]) + size_t(j) * d.ld + cell, &one, sizeof(T),
                            hipMemcpyHostToDevice, c->st));
      HIPCHK(hipStreamSynchronize(c->st));
    }
    std::vector<double> g0(stepG.begin(), stepG.begin() + size_t(m) * ns_);
    std::vector<double> V0 = initial_angular_basis(g0, m, ns_, r0, c->opt.aug_tol, c->opt.fill_tol);
    upload(c, p.V, V0.data(), V0.size() * 8);
  }
  // ---- ray tracer tables (one DG grid on [E_cut, E_max] for all beams)
  {
    const int G = d.G;
    std::vector<double> diag(size_t(nm) * G * 9), up(size_t(nm) * G * 9), lo(size_t(nm) * G * 9);
    std::vector<double> stopw(size_t(nm) * 3 * G);
    EnergyOperator op;
    for (int i = 0; i < nm; ++i) {
      std::vector<double> sig(ne, 0.0), Si(mat->S + size_t(i) * ne, mat->S + size_t(i + 1) * ne),
          Ti(mat->T + size_t(i) * ne, mat->T + size_t(i + 1) * ne);
      if (c->opt.collision == DLRA_BOLTZMANN)
        for (int e = 0; e < ne; ++e) sig[e] = mat->dG[(size_t(i) * ne + e) * nl + N + 1];
      energy_operator(c->e_cut, c->e_max, G, mat->e, ne, Si.data(), Ti.data(), sig.data(), op);
      std::copy(op.diag.begin(), op.diag.end(), diag.begin() + size_t(i) * G * 9);
      std::copy(op.up.begin(), op.up.end(), up.begin() + size_t(i) * G * 9);
      std::copy(op.lo.begin(), op.lo.end(), lo.begin() + size_t(i) * G * 9);
      weighted_integral(op, mat->e, Si.data(), ne, stopw.data() + size_t(i) * 3 * G);
    }
    upload(c, p.rt_diag, diag.data(), diag.size() * 8);
    upload(c, p.rt_up, up.data(), up.size() * 8);
    upload(c, p.rt_lo, lo.data(), lo.size() * 8);
    upload(c, p.rt_stopw, stopw.data(), stopw.size() * 8);
    double mass[3] = {op.h, op.h / 3.0, op.h / 5.0};
    upload(c, p.rt_mass, mass, sizeof(mass));
    std::vector<double> c0(size_t(nb) * 3 * G);
    for (int b = 0; b < nb; ++b)
      project_gaussian(op, c->beams[b].E0, c->beams[b].sigma_E, c0.data() + size_t(b) * 3 * G);
    upload(c, p.rt_c0, c0.data(), c0.size() * 8);
    // step windows: a step of width dt overlaps at most dt/h_E + 2 groups
    double dt_max = 0.0;
    for (double v : c->dtk) dt_max = std::max(dt_max, v);
    const int ng_step = std::min(G, int(std::ceil(dt_max / op.h - 1e-9)) + 3);
    std::vector<int> g0s(d.n_steps);
    std::vector<double> sw(size_t(d.n_steps) * ng_step * 3);
    for (int k = 0; k < d.n_steps; ++k) {
      double hi = c->edges[k], lo_ = c->edges[k + 1];
      g0s[k] = step_integral(op, lo_, hi, ng_step, sw.data() + size_t(k) * ng_step * 3);
      for (int t = 0; t < ng_step * 3; ++t) sw[size_t(k) * ng_step * 3 + t] /= c->dtk[k];
    }
    upload(c, p.rt_g0, g0s.data(), g0s.size() * 4);
    upload(c, p.rt_sw, sw.data(), sw.size() * 8);
    // rays of each beam: the grid rows of an axis-aligned beam, else one ray
    // per target cell; cells beyond beam_cut_sigmas spot sigmas get none
    c->rps.assign(nb, RayParams{});
    c->rgeo.assign(nb, RayGeom{});
    const int nx = c->grid.nx, ny = c->grid.ny, nz = c->grid.nz;
    const double D[3] = {c->grid.dx, c->grid.dy, c->grid.dz};
    for (int b = 0; b < nb; ++b) {
      const dlra_beam &bm = c->beams[b];
      const double *dir = bm.dir;
      int axis = -1, nnz = 0;
      for (int a = 0; a < 3; ++a)
        if (dir[a] != 0.0) {
          axis = a;
          ++nnz;
        }
      if (d.dim == 2 && dir[2] != 0.0) return fail(DLRA_E_INVALID, "2D problems need in-plane beams");
      if (nnz != 1) axis = -1;
      const double sgm = bm.spot_sigma, cut = c->opt.beam_cut_sigmas * sgm;
      // lateral weight f_perp(d_perp) of a cell centre, times the beam weight
      auto lateral = [&](int i, int j, int k, double &f) {
        double xc[3] = {(i + 0.5) * D[0], (j + 0.5) * D[1], d.dim == 3 ? (k + 0.5) * D[2] : 0.0};
        double rel[3], dot = 0.0, nrm2 = 0.0;
        for (int a = 0; a < 3; ++a) rel[a] = xc[a] - bm.pos[a];
        for (int a = 0; a < 3; ++a) dot += rel[a] * dir[a];
        for (int a = 0; a < 3; ++a) {
          double v = rel[a] - dot * dir[a];
          nrm2 += v * v;
        }
        double dp = std::sqrt(nrm2);
        if (dp > cut) return false;
        f = bm.weight * (d.dim == 2 ? std::exp(-0.5 * dp * dp / (sgm * sgm)) / (std::sqrt(2.0 * kPi) * sgm)
                                    : std::exp(-0.5 * dp * dp / (sgm * sgm)) / (2.0 * kPi * sgm * sgm));
        return true;
      };
      std::vector<int> rays;
      std::vector<double> fs;
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) {
            int ijk[3] = {i, j, k};
            if (axis >= 0 && ijk[axis] != 0) continue;   // rows: their first cell
            double f;
            if (!lateral(i, j, k, f)) continue;
            rays.push_back((k * ny + j) * nx + i);
            fs.push_back(f);
          }
      const int n_rays = int(rays.size());
      if (n_rays) {
        upload(c, p.rt_rays + size_t(b) * n * 4, rays.data(), rays.size() * 4);
        upload(c, p.rt_f + size_t(b) * n * 8, fs.data(), fs.size() * 8);
      }
      RayParams &rp = c->rps[b];
      rp.G = G;
      rp.n_mat = nm;
      rp.n_steps = d.n_steps;
      rp.ng_step = ng_step;
      rp.n_rays = n_rays;
      rp.n = n;
      rp.axis = axis;
      rp.h_max = c->opt.ray_h_max;
      if (axis >= 0) {
        rp.sign = dir[axis] > 0 ? 1 : -1;
        rp.row_len = axis == 0 ? nx : (axis == 1 ? ny : nz);
        rp.row_stride = axis == 0 ? 1 : (axis == 1 ? nx : nx * ny);
        rp.half = 0.5 * D[axis];
        rp.n_half = std::max(1, int(std::ceil(rp.half / c->opt.ray_h_max - 1e-9)));
      }
      RayGeom &gm = c->rgeo[b];
      gm.nx = nx;
      gm.ny = ny;
      gm.nz = nz;
      gm.dim = d.dim;
      for (int a = 0; a < 3; ++a) {
        gm.D[a] = D[a];
        gm.L[a] = (a == 0 ? nx : (a == 1 ? ny : nz)) * D[a];
        gm.om[a] = dir[a];
      }
    }
  }
  HIPCHK(hipStreamSynchronize(c->st));
  return DLRA_OK;
}

// ------------------------------------------------------------------ one energy step
template <typename T>
struct Stepper {
  dlra_ctx *c;
  using Acc = T;   // projections accumulate in the storage precision
  const Dims &d() const { return c->d; }
  T *tall(int i) { return reinterpret_cast<T *>(c->tall[i]); }
  double *D(size_t off) { return c->at<double>(off); }

  // Uhat[:, r:2r] <- orth_tau((I - U U^T) K), count -> ctl->kU.  K (tall 1) is consumed.
  // Classical Gram-Schmidt against U twice, then two Gram orthonormalisation
  // (SVQB) passes.  After R = K - U G1 the second projection G2 = U^T R is not
  // applied to R: the Gram of R - U G2 is R^T R - G2^T G2 (U has orthonormal
  // columns) and (R - U G2) T1 = [U | R] [-G2 T1; T1] is formed in one update,
  // one pass over the tall matrices fewer.
  void augment_u(int r, T *K) {
    const Plan &p = c->plan;
    const int n = d().n, ld = d().ld, P = d().P;
    T *U = tall(0);
    T *R = U + size_t(r) * ld;
    Ctl *ctl = c->ctl();
    hipStream_t st = c->st;
    launch_sumsq<T>(n, K, ld, r, &ctl->normsq, D(p.partial), p.partial_elems, st);
    launch_gram<T, double>(n, U, ld, r, K, ld, r, nullptr, nullptr, D(p.G1), P, D(p.partial),
                           p.partial_elems, st);
    launch_update<T>(n, U, ld, r, D(p.G1), P, -1.0, K, ld, 1.0, R, ld, r, nullptr, nullptr, 0,
                     st);
    launch_gram<T, double>(n, U, ld, r, R, ld, r, nullptr, nullptr, D(p.G2), P, D(p.partial),
                           p.partial_elems, st);
    launch_gram<T, double>(n, R, ld, r, R, ld, r, nullptr, nullptr, D(p.Wg), r, D(p.partial),
                           p.partial_elems, st);
    const double *G2 = D(p.G2);   // U^T R
    launch_small_gemm(1, 0, r, r, r, -1.0, G2, P, 0, G2, P, 0, 1.0, D(p.Wg), r, 0, 1, st);
    const double tol = c->opt.aug_tol;
    launch_gram_orth(r, D(p.Wg), D(p.T1), P, tol * tol, &ctl->normsq, &ctl->kU, nullptr,
                     D(p.work), st);
    // coefficients [-G2 T1; T1] (2r x r, ld P) of Uhat for K <- (R - U G2) T1
    launch_small_gemm(0, 0, r, r, r, -1.0, G2, P, 0, D(p.T1), P, 0, 0.0, D(p.G1), P, 0, 1, st);
    launch_copy_block(r, r, D(p.T1), P, D(p.G1) + r, P, r, r, 1.0, st);
    launch_update<T>(n, U, ld, 2 * r, D(p.G1), P, 1.0, nullptr, 0, 0.0, K, ld, r, nullptr,
                     nullptr, 0, st);
    launch_gram<T, double>(n, K, ld, r, K, ld, r, nullptr, nullptr, D(p.Wg), r, D(p.partial),
                           p.partial_elems, st);
    launch_gram_orth(r, D(p.Wg), D(p.T2), P, 0.0, nullptr, nullptr, &ctl->kU, D(p.work), st);
    launch_update<T>(n, K, ld, r, D(p.T2), P, 1.0, nullptr, 0, 0.0, R, ld, r, nullptr, nullptr,
                     0, st);
  }

  // Galerkin angular couplings B_dk = V^T A_dk V over q columns (ld P blocks)
  void angular(int q, double *V) {
    const Plan &p = c->plan;
    const int m = d().m, P = d().P;
    launch_small_gemm(0, 0, m, q, m, 1.0, D(p.Apm), m, size_t(m) * m, V, m, 0, 0.0, D(p.AV), m,
                      size_t(m) * P, d().ndk, c->st);
    launch_small_gemm(1, 0, q, q, m, 1.0, V, m, 0, D(p.AV), m, size_t(m) * P, 0.0, D(p.Bm), P,
                      size_t(P) * P, d().ndk, c->st);
  }

  // truncate Sh, rotate Uhat (+ dose) and Vhat; returns the new rank
  int truncate_rotate(int r, bool with_dose, const int *kU, const int *kV) {
    const Plan &p = c->plan;
    const int n = d().n, ld = d().ld, P = d().P, m = d().m, R = d().R;
    Ctl *ctl = c->ctl();
    hipStream_t st = c->st;
    TruncOpt topt = c->topt;
    int replayed = 0;
    if (c->replay_pos < c->replay.size()) {
      // a prescribed rank (clamped like the rule's) replaces the rank rule
      replayed = std::max(1, std::min(c->replay[c->replay_pos++], std::min(2 * r, R)));
      topt.fixed = 1;
      topt.r_fixed = replayed;
    }
    launch_truncate(D(p.Sh), P, kU, kV, r, topt, D(p.Pp), D(p.Qp), D(p.Sp), R, ctl, D(p.work),
                    st);
    int r1 = r;
    if (replayed || c->opt.rank_mode == DLRA_RANK_ADAPTIVE) {
      Ctl h;
      HIPCHK(hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      r1 = h.r_new;
    } else {
      r1 = c->opt.r;
    }
    double *dcv = nullptr;
    double dscale = 0.0;
    if (with_dose) {
      // dc = S' (Vhat Q')[0, :]^T
      launch_small_gemm(1, 1, r1, 1, 2 * r, 1.0, D(p.Qp), P, 0, c->V, m, 0, 0.0, D(p.tmp), P, 0,
                        1, st);
      launch_small_gemm(0, 0, r1, 1, r1, 1.0, D(p.Sp), R, 0, D(p.tmp), P, 0, 0.0, D(p.dc), P, 0,
                        1, st);
      dcv = D(p.dc);
      dscale = c->dtk[c->step] * std::sqrt(4.0 * kPi);
    }
    launch_update<T>(n, tall(0), ld, 2 * r, D(p.Pp), P, 1.0, nullptr, 0, 0.0, tall(2), ld, r1,
                     with_dose ? D(p.dose_c) : nullptr, dcv, dscale, st);
    std::swap(c->tall[0], c->tall[2]);
    launch_small_gemm(0, 0, m, r1, 2 * r, 1.0, c->V, m, 0, D(p.Qp), P, 0, 0.0, c->Vn, m, 0, 1,
                      st);
    std::swap(c->V, c->Vn);
    launch_copy_block(r1, r1, D(p.Sp), R, D(p.S), R, R, R, 1.0, st);
    return r1;
  }

  void run() {
    const Plan &p = c->plan;
    const Dims &dd = d();
    const int n = dd.n, ld = dd.ld, P = dd.P, m = dd.m, R = dd.R, N = dd.N, nm = dd.n_mat;
    const int nb = dd.n_beams, nsrc = dd.n_src;
    const int k = c->step;
    const int ns = c->n_sub[k];
    const double dt = c->dtk[k], h = dt / ns;
    hipStream_t st = c->st;
    Ctl *ctl = c->ctl();
    int r = c->r;
    T *s = c->at<T>(p.s);
    PhaseTimer t_step(c, DLRA_PH_STEP, nullptr, kBoth);
    // coefficients
    launch_inverse_stop<T>(c->gdev, c->at<T>(p.w_t), nm, D(p.stepS) + size_t(k) * nm, s, ctl, st);
    // ---------------- streaming (augmented BUG, RK4)
    angular(r, c->V);
    {
      PhaseTimer t(c, DLRA_PH_PROJECTION);
      launch_stencil_projection<T, Acc>(c->gdev, s, tall(0), ld, r, D(p.Cm), P, D(p.partial),
                                        p.partial_elems, st);
    }
    const double cf[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};   // Horner coefficients of RK4
    // L-step: L0 = V S^T, Horner RK4 (m x r), on the side stream beside the
    // K-step: it reads only V, S and this projection's couplings C (the
    // S-step's projection writes its own buffer), one small launch per stage
    double *Lk = D(p.L0), *La = D(p.La), *Lb = D(p.Lb);
    HIPCHK(hipEventRecord(c->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(c->st2, c->ev_fork, 0));
    {
      hipStream_t s2 = c->st2;
      PhaseTimer t(c, DLRA_PH_LSTEP, s2);
      launch_small_gemm(0, 1, m, r, r, 1.0, c->V, m, 0, D(p.S), R, 0, 0.0, Lk, m, 0, 1, s2);
      for (int sub = 0; sub < ns; ++sub) {
        double *in = Lk;
        double *outs[2] = {La, Lb};
        for (int stg = 0; stg < 4; ++stg) {
          double *out = outs[stg & 1];
          launch_lstep_stage(m, r, dd.ndk, D(p.Apm), D(p.Cm), P, in, Lk, out, cf[stg] * h,
                             D(p.AV), size_t(m) * P, s2);
          in = out;
        }
        std::swap(Lk, Lb);
      }
    }
    // K-step: K0 = U S, Horner RK4
    launch_pack_couplings<T>(dd.ndk, r, D(p.Bm), P, c->at<T>(p.Bpk), st);
    launch_update<T>(n, tall(0), ld, r, D(p.S), R, 1.0, nullptr, 0, 0.0, tall(1), ld, r, nullptr,
                     nullptr, 0, st);
    {
      PhaseTimer t_kloop(c, DLRA_PH_KSTAGE, nullptr, kLight, 4LL * ns);
      for (int sub = 0; sub < ns; ++sub) {
        T *K0 = tall(1);
        T *in = K0;
        T *outs[2] = {tall(2), tall(3)};
        for (int stg = 0; stg < 4; ++stg) {
          T *out = outs[stg & 1];
          PhaseTimer t(c, DLRA_PH_KSTAGE);
          launch_kstep_stage<T>(c->gdev, s, in, K0, out, ld, r, c->at<T>(p.Bpk), cf[stg] * h,
                                st);
          in = out;
        }
        std::swap(c->tall[1], c->tall[3]);
      }
    }
    // The V-side augmentation (V and L1 only) waits for the end of the K-step
    // and runs beside the U-side one: the K-step's stages hold one block per
    // CU for the whole launch, so a long single-workgroup kernel on one CU
    // would stretch a whole stage.
    HIPCHK(hipEventRecord(c->ev_kdone, st));
    HIPCHK(hipStreamWaitEvent(c->st2, c->ev_kdone, 0));
    {
      PhaseTimer t(c, DLRA_PH_AUGMENT, c->st2);
      launch_vaug(m, r, c->V, m, Lk, c->opt.aug_tol, &ctl->kV, D(p.work), c->st2);
    }
    HIPCHK(hipEventRecord(c->ev_join, c->st2));
    // augmentation
    {
      PhaseTimer t(c, DLRA_PH_AUGMENT);
      augment_u(r, tall(1));
    }
    // S-step on the augmented bases
    {
      PhaseTimer t(c, DLRA_PH_PROJECTION);
      launch_stencil_projection<T, Acc>(c->gdev, s, tall(0), ld, 2 * r, D(p.Ch), P, D(p.partial),
                                        p.partial_elems, st);
    }
    HIPCHK(hipStreamWaitEvent(st, c->ev_join, 0));
    {
      PhaseTimer t(c, DLRA_PH_SSTEP);
      angular(2 * r, c->V);
      launch_copy_block(r, r, D(p.S), R, D(p.Sh), P, P, P, 1.0, st);
      launch_sstep(2 * r, P, dd.ndk, D(p.Ch), D(p.Bm), D(p.Sh), D(p.work), h, ns, st);
    }
    {
      PhaseTimer t(c, DLRA_PH_TRUNCATE);
      r = truncate_rotate(r, false, &ctl->kU, &ctl->kV);
    }
    // ---------------- collided self-scattering (L-step, implicit Euler)
    {
      PhaseTimer t(c, DLRA_PH_COLLIDED);
      for (int i = 0; i < nm; ++i)
        launch_gram<T, Acc>(n, tall(0), ld, r, tall(0), ld, r, c->at<T>(p.w_t) + size_t(i) * n,
                            s, D(p.Mi) + size_t(i) * r * r, r, D(p.partial), p.partial_elems, st);
      launch_small_gemm(0, 1, m, r, r, 1.0, c->V, m, 0, D(p.S), R, 0, 0.0, D(p.L0), m, 0, 1, st);
      launch_collided_solve(N, m, r, nm, D(p.Mi), D(p.stepA) + size_t(k) * nm * (N + 1), dt,
                            D(p.L0), D(p.La), st);
      launch_qr_complete(m, r, D(p.La), c->V, c->opt.aug_tol, c->opt.fill_tol, c->Vn, D(p.S), R,
                         ctl, D(p.work), st);
      std::swap(c->V, c->Vn);
    }
    // ---------------- uncollided in-scattering source (explicit Euler K, L, S)
    // beam b's table of step k: psi + b * pstride
    const T *psi = c->at<T>(p.psibar) + size_t(k) * n;
    const size_t pstride = size_t(dd.n_steps) * n;
    const double *gk = D(p.stepG) + size_t(k) * m * nsrc;
    {
      PhaseTimer t(c, DLRA_PH_SOURCE);
      launch_xt_source<T, Acc>(n, tall(0), ld, r, c->at<T>(p.w_t), nm, nb, psi, pstride, D(p.H),
                               P, D(p.partial), p.partial_elems, st);
      launch_small_gemm(1, 0, r, nsrc, m, 1.0, c->V, m, 0, gk, m, 0, 0.0, D(p.Cg), P, 0, 1, st);
      launch_source_k<T>(n, tall(0), ld, r, D(p.S), R, c->at<T>(p.w_t), nm, nb, psi, pstride,
                         D(p.Cg), P, dt, tall(1), st);
      launch_small_gemm(0, 1, m, r, r, 1.0, c->V, m, 0, D(p.S), R, 0, 0.0, D(p.Lm), m, 0, 1, st);
      launch_small_gemm(0, 1, m, r, nsrc, dt, gk, m, 0, D(p.H), P, 0, 1.0, D(p.Lm), m, 0, 1, st);
    }
    // V-side augmentation on the side stream beside the U-side one
    HIPCHK(hipEventRecord(c->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(c->st2, c->ev_fork, 0));
    {
      PhaseTimer t(c, DLRA_PH_AUGMENT, c->st2);
      launch_vaug(m, r, c->V, m, D(p.Lm), c->opt.aug_tol, &ctl->kV, D(p.work), c->st2);
    }
    HIPCHK(hipEventRecord(c->ev_join, c->st2));
    {
      PhaseTimer t(c, DLRA_PH_AUGMENT);
      augment_u(r, tall(1));
    }
    HIPCHK(hipStreamWaitEvent(st, c->ev_join, 0));
    {
      PhaseTimer t(c, DLRA_PH_SOURCE);
      launch_xt_source<T, Acc>(n, tall(0), ld, 2 * r, c->at<T>(p.w_t), nm, nb, psi, pstride,
                               D(p.H), P, D(p.partial), p.partial_elems, st);
      launch_small_gemm(1, 0, 2 * r, nsrc, m, 1.0, c->V, m, 0, gk, m, 0, 0.0, D(p.Cg), P, 0, 1,
                        st);
      launch_copy_block(r, r, D(p.S), R, D(p.Sh), P, P, P, 1.0, st);
      launch_small_gemm(0, 1, 2 * r, 2 * r, nsrc, dt, D(p.H), P, 0, D(p.Cg), P, 0, 1.0, D(p.Sh),
                        P, 0, 1, st);
    }
    {
      PhaseTimer t(c, DLRA_PH_TRUNCATE);
      r = truncate_rotate(r, true, &ctl->kU, &ctl->kV);
    }
    launch_check_finite(D(p.S), R * R, ctl, st);
    c->r = r;
    c->step = k + 1;
  }
};

// Waits for the context's streams and reports (then clears) the error flags
// its kernels raised.
int sync_flags(dlra_ctx *c) {
  Ctl h;
  HIPCHK(hipStreamSynchronize(c->st2));
  HIPCHK(hipMemcpyAsync(&h, c->ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (h.flags) {
    const int zero = 0;
    HIPCHK(hipMemcpyAsync(&c->ctl()->flags, &zero, sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
  }
  if (h.flags & kFlagNonFinite) return fail(DLRA_E_NUMERIC, "non-finite value in the low-rank state");
  if (h.flags & kFlagStop) return fail(DLRA_E_NUMERIC, "non-positive stopping power");
  if (h.flags & kFlagCompletion) return fail(DLRA_E_RANK, "basis completion failed");
  if (h.flags) return fail(DLRA_E_NUMERIC, "error flag raised by a kernel");
  return DLRA_OK;
}

void clear_flags(dlra_ctx *c) {
  const int zero = 0;
  HIPCHK(hipMemcpyAsync(&c->ctl()->flags, &zero, sizeof(int), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
}

__global__ void k_dose_out(int n, int n_mat, const double *__restrict__ Du,
                           const double *__restrict__ Dc, const double *__restrict__ w, int flags,
                           double *__restrict__ out) {
  int x = blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
  double v = 0.0;
  if (flags & 1) v += Du[x];
  if (flags & 2) v += Dc[x];
  if (flags & 4) {
    double rho = 0.0;
    for (int i = 0; i < n_mat; ++i) rho += w[size_t(i) * n + x];
    v = rho > 0.0 ? v / rho : 0.0;
  }
  if (flags & 8) out[x] += v;
  else out[x] = v;
}

template <typename T>
int get_state_impl(dlra_ctx *c, double *U, double *S, double *V) {
  const Dims &d = c->d;
  const int r = c->r;
  HIPCHK(hipStreamSynchronize(c->st));
  if (U) {
    std::vector<T> col(d.n);
    for (int j = 0; j < r; ++j) {
      HIPCHK(hipMemcpy(col.data(), reinterpret_cast<T *>(c->tall[0]) + size_t(j) * d.ld,
                       d.n * sizeof(T), hipMemcpyDeviceToHost));
      for (int x = 0; x < d.n; ++x) U[size_t(x) * r + j] = double(col[x]);
    }
  }
  if (S) {
    std::vector<double> h(size_t(d.R) * d.R);
    HIPCHK(hipMemcpy(h.data(), c->base + c->plan.S, h.size() * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < r; ++j) S[i * r + j] = h[i + size_t(j) * d.R];
  }
  if (V) {
    std::vector<double> h(size_t(d.m) * r);
    HIPCHK(hipMemcpy(h.data(), c->V, h.size() * 8, hipMemcpyDeviceToHost));
    for (int p = 0; p < d.m; ++p)
      for (int j = 0; j < r; ++j) V[size_t(p) * r + j] = h[p + size_t(j) * d.m];
  }
  return DLRA_OK;
}

template <typename T>
int set_state_impl(dlra_ctx *c, const double *U, const double *S, const double *V, int r) {
  const Dims &d = c->d;
  HIPCHK(hipStreamSynchronize(c->st));
  HIPCHK(hipMemset(c->tall[0], 0, size_t(d.ld) * d.P * sizeof(T)));
  std::vector<T> col(d.n);
  for (int j = 0; j < r; ++j) {
    for (int x = 0; x < d.n; ++x) col[x] = T(U[size_t(x) * r + j]);
    HIPCHK(hipMemcpy(reinterpret_cast<T *>(c->tall[0]) + size_t(j) * d.ld, col.data(),
                     d.n * sizeof(T), hipMemcpyHostToDevice));
  }
  std::vector<double> hs(size_t(d.R) * d.R, 0.0);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) hs[i + size_t(j) * d.R] = S[i * r + j];
  HIPCHK(hipMemcpy(c->base + c->plan.S, hs.data(), hs.size() * 8, hipMemcpyHostToDevice));
  std::vector<double> hv(size_t(d.m) * d.P, 0.0);
  for (int p = 0; p < d.m; ++p)
    for (int j = 0; j < r; ++j) hv[p + size_t(j) * d.m] = V[size_t(p) * r + j];
  HIPCHK(hipMemcpy(c->V, hv.data(), hv.size() * 8, hipMemcpyHostToDevice));
  c->r = r;
  clear_flags(c);
  return DLRA_OK;
}

// ------------------------------------------------------------------ checkpoints
struct SaveHeader {
  unsigned long long magic;
  int version, n, m, R, tsize, n_beams, n_steps, r, step;
};
constexpr unsigned long long kSaveMagic = 0x31544b4344524c44ULL;   // "DLRCDKT1"

size_t save_bytes(const dlra_ctx *c) {
  const Dims &d = c->d;
  return sizeof(SaveHeader) + size_t(d.n) * d.R * d.tsize + size_t(d.R) * d.R * 8 +
         size_t(d.m) * d.R * 8 + size_t(d.n) * 8;
}

// header, then U (r columns of n values in the storage precision), S (r x r,
// column-major, leading dimension R), V (m x r, column-major), collided dose
void save_impl(dlra_ctx *c, char *buf) {
  const Dims &d = c->d;
  SaveHeader h{kSaveMagic, 1, d.n, d.m, d.R, int(d.tsize), d.n_beams, d.n_steps, c->r, c->step};
  std::memcpy(buf, &h, sizeof(h));
  char *q = buf + sizeof(h);
  for (int j = 0; j < c->r; ++j) {
    HIPCHK(hipMemcpy(q, static_cast<char *>(c->tall[0]) + size_t(j) * d.ld * d.tsize,
                     size_t(d.n) * d.tsize, hipMemcpyDeviceToHost));
    q += size_t(d.n) * d.tsize;
  }
  HIPCHK(hipMemcpy(q, c->base + c->plan.S, size_t(d.R) * d.R * 8, hipMemcpyDeviceToHost));
  q += size_t(d.R) * d.R * 8;
  HIPCHK(hipMemcpy(q, c->V, size_t(d.m) * c->r * 8, hipMemcpyDeviceToHost));
  q += size_t(d.m) * c->r * 8;
  HIPCHK(hipMemcpy(q, c->base + c->plan.dose_c, size_t(d.n) * 8, hipMemcpyDeviceToHost));
}

int load_impl(dlra_ctx *c, const char *buf, size_t bytes) {
  const Dims &d = c->d;
  SaveHeader h;
  if (bytes < sizeof(h)) return fail(DLRA_E_INVALID, "checkpoint too short");
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kSaveMagic || h.version != 1)
    return fail(DLRA_E_INVALID, "not a checkpoint of this library");
  if (h.n != d.n || h.m != d.m || h.R != d.R || h.tsize != int(d.tsize) ||
      h.n_beams != d.n_beams || h.n_steps != d.n_steps)
    return fail(DLRA_E_INVALID, "checkpoint of a different problem");
  if (h.r < 1 || h.r > d.R || h.step < 0 || h.step > d.n_steps)
    return fail(DLRA_E_INVALID, "checkpoint rank or step out of range");
  const size_t need = sizeof(h) + size_t(d.n) * h.r * d.tsize + size_t(d.R) * d.R * 8 +
                      size_t(d.m) * h.r * 8 + size_t(d.n) * 8;
  if (bytes < need) return fail(DLRA_E_INVALID, "checkpoint truncated");
  HIPCHK(hipStreamSynchronize(c->st));
  HIPCHK(hipStreamSynchronize(c->st2));
  const char *q = buf + sizeof(h);
  HIPCHK(hipMemset(c->tall[0], 0, size_t(d.ld) * d.P * d.tsize));
  for (int j = 0; j < h.r; ++j) {
    HIPCHK(hipMemcpy(static_cast<char *>(c->tall[0]) + size_t(j) * d.ld * d.tsize, q,
                     size_t(d.n) * d.tsize, hipMemcpyHostToDevice));
    q += size_t(d.n) * d.tsize;
  }
  HIPCHK(hipMemcpy(c->base + c->plan.S, q, size_t(d.R) * d.R * 8, hipMemcpyHostToDevice));
  q += size_t(d.R) * d.R * 8;
  HIPCHK(hipMemset(c->V, 0, size_t(d.m) * d.P * 8));
  HIPCHK(hipMemcpy(c->V, q, size_t(d.m) * h.r * 8, hipMemcpyHostToDevice));
  q += size_t(d.m) * h.r * 8;
  HIPCHK(hipMemcpy(c->base + c->plan.dose_c, q, size_t(d.n) * 8, hipMemcpyHostToDevice));
  c->r = h.r;
  c->step = h.step;
  clear_flags(c);
  return DLRA_OK;
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// Device memory of dlra_plan_objective_noalloc: the block partials of its
// reduction and the result row, for up to kPlanMaxBeams beams.  Each GPU the
// library runs on holds its own copy until the process ends; calls on one GPU
// share it.
constexpr size_t kNoallocDoubles = size_t(kPlanBlocks + 64 + 1) * (kPlanMaxBeams + 1) +
                                   (kPlanMaxBeams + 1);
static __device__ __align__(256) double scratch[kNoallocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// Device address of the static scratch on the current device, looked up once
// per device (the array's name is only a host-side stand-in).
static int noalloc_scratch(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(DLRA_E_HIP, "no current HIP device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(DLRA_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return DLRA_OK;
}

// ==================================================================== C ABI
extern "C" {

int dlra_workspace_size(const dlra_grid *grid, int n_mat, int n_beams, const dlra_options *opt,
                        size_t *bytes) {
  Dims d;
  std::string err;
  if (!bytes) return fail(DLRA_E_INVALID, "bytes is NULL");
  if (!make_dims(grid, n_mat, n_beams, opt, d, err)) return fail(DLRA_E_INVALID, err);
  *bytes = make_plan(d).bytes;
  return DLRA_OK;
}

int dlra_init(const dlra_grid *grid, const dlra_materials *mat, int n_beams,
              const dlra_beam *beams, const dlra_options *opt, void *workspace,
              size_t workspace_bytes, void *stream, dlra_ctx **out) {
  if (!out) return fail(DLRA_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!mat || !beams || !workspace) return fail(DLRA_E_INVALID, "null materials, beams or workspace");
  Dims d;
  std::string err;
  if (!make_dims(grid, mat->n_mat, n_beams, opt, d, err)) return fail(DLRA_E_INVALID, err);
  if (!mat->w || !mat->e || !mat->S || !mat->T || !mat->dG || mat->n_e < 2)
    return fail(DLRA_E_INVALID, "material tables missing");
  if (mat->n_leg < d.N + 2) return fail(DLRA_E_INVALID, "n_leg must be >= pn_degree + 2");
  for (int e = 1; e < mat->n_e; ++e)
    if (!(mat->e[e] > mat->e[e - 1])) return fail(DLRA_E_INVALID, "table energies must ascend");
  for (size_t t = 0; t < size_t(mat->n_mat) * d.n; ++t)
    if (!(mat->w[t] >= 0.0) || !std::isfinite(mat->w[t]))
      return fail(DLRA_E_INVALID, "partial densities must be finite and >= 0");
  double e_cut = opt->e_cut;
  if (opt->egrid == DLRA_EGRID_USER) {
    const double *E = opt->egrid_points;
    if (!E) return fail(DLRA_E_INVALID, "egrid_points is NULL");
    for (int k = 0; k <= opt->n_steps; ++k)
      if (!std::isfinite(E[k]) || !(E[k] > 0.0) || (k > 0 && !(E[k] < E[k - 1])))
        return fail(DLRA_E_INVALID, "egrid_points must be n_steps + 1 descending energies > 0");
    e_cut = E[opt->n_steps];
  }
  for (int b = 0; b < n_beams; ++b) {
    const dlra_beam &bm = beams[b];
    double dn = std::sqrt(bm.dir[0] * bm.dir[0] + bm.dir[1] * bm.dir[1] + bm.dir[2] * bm.dir[2]);
    if (!(std::fabs(dn - 1.0) < 1e-9)) return fail(DLRA_E_INVALID, "beam direction must be a unit vector");
    if (!(bm.sigma_E > 0) || !(bm.spot_sigma > 0) || !(e_cut > 0) || !(bm.E0 > e_cut))
      return fail(DLRA_E_INVALID, "need sigma_E > 0, spot_sigma > 0 and E0 > e_cut > 0");
    if (!std::isfinite(bm.weight)) return fail(DLRA_E_INVALID, "beam weight must be finite");
  }
  if (!(opt->aug_tol > 0) || !(opt->fill_tol > 0) || !(opt->fill_tol < 0.1) || !(opt->floor_tol >= 0) ||
      !(opt->ray_h_max > 0) || !(opt->beam_cut_sigmas > 0) || !(opt->e_max_sigmas > 0))
    return fail(DLRA_E_INVALID, "tolerances out of range");
  if (opt->rank_mode == DLRA_RANK_ADAPTIVE && !(opt->trunc_tol > 0))
    return fail(DLRA_E_INVALID, "trunc_tol must be > 0 in adaptive mode");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(DLRA_E_INVALID, "workspace must be 256-byte aligned");
  Plan plan = make_plan(d);
  if (workspace_bytes < plan.bytes)
    return fail(DLRA_E_NOMEM, "workspace too small: need " + std::to_string(plan.bytes) + " bytes");
  dlra_ctx *c = new dlra_ctx();
  c->d = d;
  c->plan = plan;
  c->grid = *grid;
  c->opt = *opt;
  c->opt.egrid_points = nullptr;   // copied into c->edges during init
  c->beams.assign(beams, beams + n_beams);
  c->st = reinterpret_cast<hipStream_t>(stream);
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  if (hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_kdone, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return fail(DLRA_E_HIP, "creating the side stream or its events failed");
  }
  c->base = reinterpret_cast<char *>(workspace);
  c->gdev.nx = grid->nx;
  c->gdev.ny = grid->ny;
  c->gdev.nz = grid->nz;
  c->gdev.n = d.n;
  c->gdev.dim = d.dim;
  c->gdev.inv2h[0] = 1.0 / (2.0 * grid->dx);
  c->gdev.inv2h[1] = 1.0 / (2.0 * grid->dy);
  c->gdev.inv2h[2] = 1.0 / (2.0 * grid->dz);
  c->topt.fixed = opt->rank_mode == DLRA_RANK_FIXED;
  c->topt.r_fixed = opt->r;
  c->topt.r_min = opt->r_min;
  c->topt.r_max = opt->r_max;
  c->topt.trunc_tol = opt->trunc_tol;
  c->topt.floor_tol = opt->floor_tol;
  c->topt.fill_tol = opt->fill_tol;
  for (int i = 0; i < 4; ++i) c->tall[i] = c->base + plan.tall[i];
  c->V = c->at<double>(plan.V);
  c->Vn = c->at<double>(plan.Vn);
  int rc;
  try {
    if (opt->egrid == DLRA_EGRID_USER) c->opt.egrid_points = opt->egrid_points;
    rc = d.tsize == 8 ? init_impl<double>(c, mat) : init_impl<float>(c, mat);
    c->opt.egrid_points = nullptr;
  } catch (const std::invalid_argument &e) {
    rc = fail(DLRA_E_INVALID, e.what());
  } catch (const std::exception &e) {
    rc = fail(DLRA_E_HIP, e.what());
  }
  if (rc != DLRA_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return DLRA_OK;
}

int uncollided_raytrace(dlra_ctx *c) {
  if (!c) return fail(DLRA_E_INVALID, "ctx is NULL");
  try {
    const Plan &p = c->plan;
    const Dims &d = c->d;
    HIPCHK(hipMemsetAsync(c->base + p.psibar, 0, size_t(d.n_beams) * d.n_steps * d.n * d.tsize,
                          c->st));
    HIPCHK(hipMemsetAsync(c->base + p.dose_u, 0, size_t(d.n) * 8, c->st));
    HIPCHK(hipMemsetAsync(&c->ctl()->rt_substeps, 0, 2 * sizeof(unsigned long long), c->st));
    auto go = [&](int b, auto *psib) {
      using T = std::remove_pointer_t<decltype(psib)>;
      launch_raytrace<T>(c->rps[b], c->rgeo[b], c->at<int>(p.rt_rays) + size_t(b) * d.n,
                         c->at<double>(p.rt_f) + size_t(b) * d.n, c->at<double>(p.w_d),
                         c->at<double>(p.rt_diag), c->at<double>(p.rt_up),
                         c->at<double>(p.rt_lo), c->at<double>(p.rt_mass),
                         c->at<double>(p.rt_c0) + size_t(b) * 3 * d.G, c->at<int>(p.rt_g0),
                         c->at<double>(p.rt_sw), c->at<double>(p.rt_stopw),
                         c->at<double>(p.rt_scratch), size_t(d.ray_batch),
                         psib + size_t(b) * d.n_steps * d.n, c->at<double>(p.dose_u), c->ctl(),
                         c->st);
    };
    PhaseTimer t(c, DLRA_PH_RAYTRACE, nullptr, kBoth);
    for (int b = 0; b < d.n_beams; ++b) {
      if (d.tsize == 8) go(b, c->at<double>(p.psibar));
      else go(b, c->at<float>(p.psibar));
    }
    HIPCHK(hipGetLastError());
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  c->traced = true;
  return DLRA_OK;
}

int dlra_step(dlra_ctx *c, int *rank_out) {
  if (!c) return fail(DLRA_E_INVALID, "ctx is NULL");
  if (!c->traced) return fail(DLRA_E_STATE, "uncollided_raytrace must precede dlra_step");
  if (c->step >= c->d.n_steps) return fail(DLRA_E_STATE, "all energy steps done");
  try {
    if (c->d.tsize == 8) Stepper<double>{c}.run();
    else Stepper<float>{c}.run();
    HIPCHK(hipGetLastError());
    if (rank_out) {
      int rc = sync_flags(c);
      if (rc != DLRA_OK) return rc;
      *rank_out = c->r;
    }
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  return DLRA_OK;
}

int dlra_run_graph(dlra_ctx *c, int count) {
  if (!c) return fail(DLRA_E_INVALID, "ctx is NULL");
  if (!c->traced) return fail(DLRA_E_STATE, "uncollided_raytrace must precede dlra_run_graph");
  if (count < 1 || count > c->d.n_steps - c->step)
    return fail(DLRA_E_INVALID, "count outside [1, steps left]");
  if (c->opt.rank_mode != DLRA_RANK_FIXED || c->prof != 0 || c->replay_pos < c->replay.size())
    return fail(DLRA_E_STATE, "graph runs need fixed rank, profiling off and no rank replay");
  // host state the recording advances; restored if the capture fails.  The
  // steps are recorded on a private stream (the caller's may be the legacy
  // default stream, which cannot be captured) and the graph is launched on
  // the caller's.
  const int step0 = c->step, r0 = c->r;
  void *tall0[4] = {c->tall[0], c->tall[1], c->tall[2], c->tall[3]};
  double *V0 = c->V, *Vn0 = c->Vn;
  hipStream_t user = c->st;
  auto restore = [&]() {
    c->st = user;
    c->step = step0;
    c->r = r0;
    for (int i = 0; i < 4; ++i) c->tall[i] = tall0[i];
    c->V = V0;
    c->Vn = Vn0;
  };
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  try {
    // the previous graph (if any) has finished before it is released
    if (c->graph_exec) {
      HIPCHK(hipStreamSynchronize(c->st));
      HIPCHK(hipGraphExecDestroy(c->graph_exec));
      c->graph_exec = nullptr;
    }
    if (!c->st_cap) HIPCHK(hipStreamCreateWithFlags(&c->st_cap, hipStreamNonBlocking));
    c->st = c->st_cap;
    HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeRelaxed));
    try {
      for (int i = 0; i < count; ++i) {
        if (c->d.tsize == 8) Stepper<double>{c}.run();
        else Stepper<float>{c}.run();
      }
    } catch (...) {
      (void)hipStreamEndCapture(c->st, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(c->st, &g));
    c->st = user;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      throw std::runtime_error("graph instantiation failed");
    }
    (void)hipGraphDestroy(g);
    if (hipGraphLaunch(ge, c->st) != hipSuccess) {
      (void)hipGraphExecDestroy(ge);
      throw std::runtime_error("graph launch failed");
    }
    c->graph_exec = ge;   // released after the stream has passed it
  } catch (const std::exception &e) {
    restore();
    (void)hipGetLastError();
    return fail(DLRA_E_HIP, e.what());
  }
  return DLRA_OK;
}

int dose_deposit(dlra_ctx *c, double *dose, int flags) {
  if (!c || !dose) return fail(DLRA_E_INVALID, "null ctx or dose");
  if (flags & ~15) return fail(DLRA_E_INVALID, "unknown flag bits");
  try {
    int rc = sync_flags(c);
    if (rc != DLRA_OK) return rc;
    const Plan &p = c->plan;
    k_dose_out<<<(c->d.n + 255) / 256, 256, 0, c->st>>>(c->d.n, c->d.n_mat,
                                                        c->at<double>(p.dose_u),
                                                        c->at<double>(p.dose_c),
                                                        c->at<double>(p.w_d), flags, dose);
    HIPCHK(hipGetLastError());
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  return DLRA_OK;
}

int dlra_get_state(dlra_ctx *c, double *U, double *S, double *V, int *rank, int *step) {
  if (!c) return fail(DLRA_E_INVALID, "ctx is NULL");
  if (rank) *rank = c->r;
  if (step) *step = c->step;
  try {
    return c->d.tsize == 8 ? get_state_impl<double>(c, U, S, V) : get_state_impl<float>(c, U, S, V);
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
}

int dlra_set_state(dlra_ctx *c, const double *U, const double *S, const double *V, int rank,
                   int step) {
  if (!c || !U || !S || !V) return fail(DLRA_E_INVALID, "null argument");
  if (rank < 1 || rank > c->d.R) return fail(DLRA_E_INVALID, "rank outside [1, r_max]");
  if (step < 0 || step > c->d.n_steps) return fail(DLRA_E_INVALID, "step outside [0, n_steps]");
  try {
    int rc = c->d.tsize == 8 ? set_state_impl<double>(c, U, S, V, rank)
                             : set_state_impl<float>(c, U, S, V, rank);
    if (rc == DLRA_OK) c->step = step;
    return rc;
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
}

int dlra_get_uncollided(dlra_ctx *c, double *psibar, double *Du) {
  if (!c) return fail(DLRA_E_INVALID, "ctx is NULL");
  if (!c->traced) return fail(DLRA_E_STATE, "uncollided_raytrace has not run");
  try {
    const Dims &d = c->d;
    HIPCHK(hipStreamSynchronize(c->st));
    if (psibar) {
      size_t cnt = size_t(d.n_beams) * d.n_steps * d.n;
      if (d.tsize == 8) {
        HIPCHK(hipMemcpy(psibar, c->base + c->plan.psibar, cnt * 8, hipMemcpyDeviceToHost));
      } else {
        std::vector<float> h(cnt);
        HIPCHK(hipMemcpy(h.data(), c->base + c->plan.psibar, cnt * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < cnt; ++i) psibar[i] = h[i];
      }
    }
    if (Du) HIPCHK(hipMemcpy(Du, c->base + c->plan.dose_u, size_t(d.n) * 8, hipMemcpyDeviceToHost));
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  return DLRA_OK;
}

int dlra_set_uncollided(dlra_ctx *c, int beam, int step, const double *psibar, const double *Du) {
  if (!c) return fail(DLRA_E_INVALID, "ctx is NULL");
  const Dims &d = c->d;
  if (psibar && (beam < 0 || beam >= d.n_beams || step < 0 || step >= d.n_steps))
    return fail(DLRA_E_INVALID, "beam or step out of range");
  try {
    HIPCHK(hipStreamSynchronize(c->st));
    if (psibar) {
      char *dst = c->base + c->plan.psibar + (size_t(beam) * d.n_steps + step) * d.n * d.tsize;
      if (d.tsize == 8) {
        HIPCHK(hipMemcpy(dst, psibar, size_t(d.n) * 8, hipMemcpyHostToDevice));
      } else {
        std::vector<float> h(psibar, psibar + d.n);
        HIPCHK(hipMemcpy(dst, h.data(), size_t(d.n) * 4, hipMemcpyHostToDevice));
      }
    }
    if (Du) HIPCHK(hipMemcpy(c->base + c->plan.dose_u, Du, size_t(d.n) * 8, hipMemcpyHostToDevice));
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  c->traced = true;
  return DLRA_OK;
}

int dlra_save(dlra_ctx *c, void *buf, size_t *bytes) {
  if (!c || !bytes) return fail(DLRA_E_INVALID, "null ctx or bytes");
  const size_t need = save_bytes(c);
  if (!buf) {
    *bytes = need;
    return DLRA_OK;
  }
  if (*bytes < need) return fail(DLRA_E_INVALID, "buffer smaller than the checkpoint");
  try {
    int rc = sync_flags(c);
    if (rc != DLRA_OK) return rc;
    save_impl(c, static_cast<char *>(buf));
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  *bytes = need;
  return DLRA_OK;
}

int dlra_load(dlra_ctx *c, const void *buf, size_t bytes) {
  if (!c || !buf) return fail(DLRA_E_INVALID, "null ctx or buffer");
  try {
    return load_impl(c, static_cast<const char *>(buf), bytes);
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
}

int dlra_raytrace_work(dlra_ctx *c, long long *substeps, long long *factorizations,
                       long long *rays) {
  if (!c || !substeps || !factorizations || !rays) return fail(DLRA_E_INVALID, "null argument");
  if (!c->traced) return fail(DLRA_E_STATE, "uncollided_raytrace has not run");
  try {
    Ctl h;
    HIPCHK(hipMemcpyAsync(&h, c->ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    *substeps = (long long)h.rt_substeps;
    *factorizations = (long long)h.rt_factors;
    long long nr = 0;
    for (const RayParams &rp : c->rps) nr += rp.n_rays;
    *rays = nr;
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  return DLRA_OK;
}

int dlra_replay_ranks(dlra_ctx *c, int count, const int *ranks) {
  if (!c || count < 0 || (count > 0 && !ranks)) return fail(DLRA_E_INVALID, "bad arguments");
  for (int i = 0; i < count; ++i)
    if (ranks[i] < 1 || ranks[i] > c->d.R) return fail(DLRA_E_INVALID, "rank outside [1, r_max]");
  c->replay.assign(ranks, ranks + count);
  c->replay_pos = 0;
  return DLRA_OK;
}

int dlra_substeps(dlra_ctx *c, int k, int *n_sub) {
  if (!c || !n_sub) return fail(DLRA_E_INVALID, "null argument");
  if (k < 0 || k >= c->d.n_steps) return fail(DLRA_E_INVALID, "k outside [0, n_steps)");
  *n_sub = c->n_sub[k];
  return DLRA_OK;
}

int dlra_sync(dlra_ctx *c) {
  if (!c) return fail(DLRA_E_INVALID, "ctx is NULL");
  try {
    return sync_flags(c);
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
}

int dlra_profile(dlra_ctx *c, int on) {
  if (!c) return fail(DLRA_E_INVALID, "ctx is NULL");
  if (on < 0 || on > 2) return fail(DLRA_E_INVALID, "profile level must be 0, 1 or 2");
  try {
    c->drain();
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  if (on) {
    for (int i = 0; i < DLRA_PH_COUNT; ++i) {
      c->prof_ms[i] = 0.0;
      c->prof_n[i] = 0;
    }
  }
  c->prof = on;
  return DLRA_OK;
}

int dlra_profile_read(dlra_ctx *c, int phase, double *total_ms, long long *count) {
  if (!c || !total_ms || !count) return fail(DLRA_E_INVALID, "null argument");
  if (phase < 0 || phase >= DLRA_PH_COUNT) return fail(DLRA_E_INVALID, "unknown phase");
  try {
    c->drain();
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  *total_ms = c->prof_ms[phase];
  *count = c->prof_n[phase];
  return DLRA_OK;
}

void dlra_destroy(dlra_ctx *c) { delete c; }

size_t dlra_plan_objective_work(int n_cells, int n_beams) {
  if (n_cells <= 0 || n_beams < 1 || n_beams > kPlanMaxBeams) return 0;
  return plan_objective_work(n_cells, n_beams);
}

int dlra_plan_objective(int n_cells, int n_beams, const double *doses, const double *weights,
                        const unsigned char *target, double dhat, double lam, double *work,
                        size_t work_doubles, void *stream, double *J, double *grad) {
  if (n_cells <= 0 || n_beams < 1 || n_beams > kPlanMaxBeams)
    return fail(DLRA_E_INVALID, "n_cells must be positive and n_beams in [1, 64]");
  if (!doses || !weights || !target || !work || !J || !grad)
    return fail(DLRA_E_INVALID, "null argument");
  if (!(lam >= 0.0) || !std::isfinite(lam) || !std::isfinite(dhat))
    return fail(DLRA_E_INVALID, "lam must be finite and >= 0, dhat finite");
  if (work_doubles < plan_objective_work(n_cells, n_beams))
    return fail(DLRA_E_INVALID, "work space smaller than dlra_plan_objective_work()");
  PlanWeights pw{};
  for (int b = 0; b < n_beams; ++b) {
    if (!std::isfinite(weights[b])) return fail(DLRA_E_INVALID, "non-finite weight");
    pw.w[b] = weights[b];
  }
  try {
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *out = work + plan_objective_work(n_cells, n_beams) - size_t(n_beams + 1);
    launch_plan_objective(n_cells, n_beams, doses, pw, target, dhat, lam, work, out, st);
    HIPCHK(hipGetLastError());
    std::vector<double> h(size_t(n_beams) + 1);
    HIPCHK(hipMemcpyAsync(h.data(), out, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *J = h[0];
    for (int b = 0; b < n_beams; ++b) grad[b] = h[1 + b];
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  return DLRA_OK;
}

int dlra_plan_objective_noalloc(int n_cells, int n_beams, const double *doses,
                                const double *weights, const unsigned char *target, double dhat,
                                double lam, void *stream, double *J, double *grad) {
  if (n_cells <= 0 || n_beams < 1 || n_beams > kPlanMaxBeams)
    return fail(DLRA_E_INVALID, "n_cells must be positive and n_beams in [1, 64] (the static "
                                "scratch holds the partial sums of at most 64 beams)");
  if (!doses || !weights || !target || !J || !grad) return fail(DLRA_E_INVALID, "null argument");
  if (!(lam >= 0.0) || !std::isfinite(lam) || !std::isfinite(dhat))
    return fail(DLRA_E_INVALID, "lam must be finite and >= 0, dhat finite");
  if (plan_objective_fused_scratch(n_beams) + size_t(n_beams + 1) > kNoallocDoubles)
    return fail(DLRA_E_INVALID, "static scratch too small");
  PlanWeights pw{};
  for (int b = 0; b < n_beams; ++b) {
    if (!std::isfinite(weights[b])) return fail(DLRA_E_INVALID, "non-finite weight");
    pw.w[b] = weights[b];
  }
  double *buf = nullptr;
  int rc = noalloc_scratch(&buf);
  if (rc != DLRA_OK) return rc;
  try {
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *out = buf + plan_objective_fused_scratch(n_beams);
    launch_plan_objective_fused(n_cells, n_beams, doses, pw, target, dhat, lam, buf, out, st);
    HIPCHK(hipGetLastError());
    double h[kPlanMaxBeams + 1];
    HIPCHK(hipMemcpyAsync(h, out, size_t(n_beams + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *J = h[0];
    for (int b = 0; b < n_beams; ++b) grad[b] = h[1 + b];
  } catch (const std::exception &e) {
    return fail(DLRA_E_HIP, e.what());
  }
  return DLRA_OK;
}

int dlra_run_batch(dlra_ctx *const *ctxs, int n_ctx, int n_steps, int n_threads) {
  if (!ctxs || n_ctx < 0 || n_steps < 0) return fail(DLRA_E_INVALID, "bad batch arguments");
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctxs[i]) return fail(DLRA_E_INVALID, "ctx is NULL");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(DLRA_E_INVALID, "a context appears twice in the batch");
  }
  if (n_ctx == 0) return DLRA_OK;
  const int nt = n_threads <= 0 ? n_ctx : std::min(n_threads, n_ctx);
  std::atomic<bool> stop{false};
  std::mutex mu;
  int first_rc = DLRA_OK;
  std::string first_msg;
  auto record = [&](int rc) {
    std::lock_guard<std::mutex> lk(mu);
    if (first_rc == DLRA_OK) {
      first_rc = rc;
      first_msg = g_err;   // this worker's message
    }
    stop = true;
  };
  // worker t drives contexts t, t + nt, ...: ray trace, then the energy
  // steps interleaved across its contexts, then a wait on their streams
  auto worker = [&](int t) {
    if (hipSetDevice(ctxs[t]->device) != hipSuccess) {
      g_err = "hipSetDevice failed";
      record(DLRA_E_HIP);
      return;
    }
    for (int i = t; i < n_ctx && !stop; i += nt)
      if (!ctxs[i]->traced) {
        const int rc = uncollided_raytrace(ctxs[i]);
        if (rc != DLRA_OK) return record(rc);
      }
    for (int k = 0; k < n_steps && !stop; ++k)
      for (int i = t; i < n_ctx && !stop; i += nt)
        if (ctxs[i]->step < ctxs[i]->d.n_steps) {
          const int rc = dlra_step(ctxs[i], nullptr);
          if (rc != DLRA_OK) return record(rc);
        }
    for (int i = t; i < n_ctx; i += nt) {
      const int rc = dlra_sync(ctxs[i]);
      if (rc != DLRA_OK) return record(rc);
    }
  };
  std::vector<std::thread> pool;
  pool.reserve(nt);
  for (int t = 0; t < nt; ++t) pool.emplace_back(worker, t);
  for (auto &th : pool) th.join();
  if (first_rc != DLRA_OK) g_err = first_msg;
  return first_rc;
}

int dlra_roof_probe(int kind, int iters, double *tflops) {
  if (kind < 0 || kind > 3 || iters < 1 || tflops == nullptr)
    return fail(DLRA_E_INVALID, "dlra_roof_probe: kind 0..3, iters >= 1 and tflops required");
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      n_cu <= 0)
    return fail(DLRA_E_HIP, "dlra_roof_probe: no device");
  const int blocks = 4 * n_cu;
  double *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    if (out != nullptr) (void)hipFree(out);
    if (e0 != nullptr) (void)hipEventDestroy(e0);
    if (e1 != nullptr) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&out, size_t(blocks) * 256 * sizeof(double)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    release();
    return fail(DLRA_E_HIP, "dlra_roof_probe: buffer or events");
  }
  launch_roof_probe(kind, std::min(iters, 64), blocks, out, nullptr);   // warm-up
  hipError_t err = hipEventRecord(e0, nullptr);
  if (err == hipSuccess) launch_roof_probe(kind, iters, blocks, out, nullptr);
  if (err == hipSuccess) err = hipEventRecord(e1, nullptr);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  if (err == hipSuccess) err = hipGetLastError();
  release();
  if (err != hipSuccess) return fail(DLRA_E_HIP, std::string("dlra_roof_probe: ") + hipGetErrorString(err));
  if (!(ms > 0.0f)) return fail(DLRA_E_HIP, "dlra_roof_probe: no elapsed time");
  *tflops = roof_probe_flops(kind, iters, blocks) / (double(ms) * 1e-3) / 1e12;
  return DLRA_OK;
}

const char *dlra_last_error(void) { return g_err.c_str(); }

}  // extern "C"
