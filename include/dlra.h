/*
 * dlra.h -- C ABI of the MI355X dynamical low-rank proton transport library.
 *
 * The library advances the collided proton flux of a pencil beam through a
 * voxel phantom with the rank-adaptive augmented basis-update & Galerkin
 * integrator (paper Sec. 2.2, eq. KLS), energy acting as pseudo-time
 * (Sec. 3.3), and feeds it with the uncollided flux of a ray tracer
 * (Sec. 3.2).  A context holds one pencil beam, or several beams whose
 * uncollided fluxes source one joint collided solve (the two-beam case of
 * Sec. 4.3).  All compute runs in HIP kernels on the stream given at
 * initialisation.
 *
 * Conventions
 *   - Cells are ordered x fastest: cell = (k*ny + j)*nx + i (Sec. 3.3.2).
 *   - Units: cm, MeV, g/cm^3.  Deposited energy is MeV/cm^3 per source proton
 *     (per cm of depth out of plane in 2D).
 *   - Host arrays passed in are copied during the call; the caller may free
 *     them afterwards.  Device memory: the caller owns the workspace passed to
 *     dlra_init and every device output buffer; the library never allocates
 *     device memory and keeps pointers into the workspace until dlra_destroy.
 *   - Calls enqueue work on the context's stream and return without waiting,
 *     unless stated otherwise.  Calls on one context must not overlap;
 *     different contexts are independent.
 *   - Every call returns DLRA_OK (0) or a negative error code; the message of
 *     the last error on the calling thread is available from dlra_last_error.
 *     Invalid arguments are rejected before anything is enqueued.
 */
#ifndef DLRA_H
#define DLRA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DLRA_OK = 0,
  DLRA_E_INVALID = -1,   /* bad argument, size or pointer; nothing enqueued */
  DLRA_E_NOMEM = -2,     /* workspace smaller than dlra_workspace_size */
  DLRA_E_HIP = -3,       /* a HIP runtime call failed */
  DLRA_E_NUMERIC = -4,   /* non-finite value detected in the low-rank state */
  DLRA_E_CFL = -5,       /* RK4 substeps needed exceed the configured maximum */
  DLRA_E_RANK = -6,      /* rank outside [1, r_max] */
  DLRA_E_STATE = -7      /* call out of order (e.g. step before raytrace) */
};

enum { DLRA_RANK_FIXED = 0, DLRA_RANK_ADAPTIVE = 1 };
enum { DLRA_FP64 = 0, DLRA_MIXED = 1 };
/* Collision operator (Sec. 2.1, Sec. 3.1): Boltzmann with the extended
 * transport correction, or Fokker-Planck (eigenvalues -xi_1 l (l+1) / 2 of the
 * scaled Laplace-Beltrami operator, xi_1 = G_0 - G_1; no removal of the
 * uncollided flux, Gamma_out = 0, which sources the whole operator). */
enum { DLRA_BOLTZMANN = 0, DLRA_FOKKER_PLANCK = 1 };
/* Pseudo-time (energy) grid E_0 = E_max > E_1 > ... > E_n = E_cut; step k
 * spans [E_{k+1}, E_k] and takes its coefficients at the midpoint.
 *   UNIFORM       equal steps (the paper's experiments)
 *   PROPORTIONAL  E_k = E_cut (E_max / E_cut)^(1 - k/n): short steps at low
 *                 energy, where the flux changes fastest (the non-uniform
 *                 grid proposed in Sec. 6)
 *   CFL           equal steps of residual range in the least-stopping voxel,
 *                 R(E_k) = (1 - k/n) R(E_max), R(E) = int_{E_cut}^E dE'/S_min,
 *                 S_min(E) = min_x S(x, E) (trapezoid rule on 4096 equal
 *                 intervals, inverted by linear interpolation): every step
 *                 takes the same number of RK4 substeps
 *   USER          the n_steps + 1 descending energies of egrid_points */
enum { DLRA_EGRID_UNIFORM = 0, DLRA_EGRID_PROPORTIONAL = 1, DLRA_EGRID_CFL = 2,
       DLRA_EGRID_USER = 3 };

/* Structured grid (Sec. 3.3.2).  nz == 1 selects the 2D problem (streaming in
 * x and y only).  Spacings in cm. */
typedef struct {
  int nx, ny, nz;
  double dx, dy, dz;
} dlra_grid;

/* Mixture model (Sec. 2.1, eq. mixXS): per-voxel partial densities of n_mat
 * base materials (1 <= n_mat <= 16; the paper's decomposition has twelve
 * elements) and per-material energy tables, interpolated linearly in E.
 *   w   [n_mat][n_cells]     partial density of material i in the cell, g/cm^3
 *   e   [n_e]                ascending table energies, MeV
 *   S   [n_mat][n_e]         mass stopping power, MeV cm^2/g
 *   T   [n_mat][n_e]         mass straggling coefficient, MeV^2 cm^2/g
 *   dG  [n_mat][n_e][n_leg]  G_0 - G_l of the Legendre moments
 *                            G_l = 2 pi int P_l(mu) Sigma_s dmu (Sec. 3.3.1),
 *                            cm^2/g; n_leg >= pn_degree + 2, dG[..][..][0] = 0.
 * The transport-corrected operator only uses differences of moments
 * (Sec. 3.3.1, extended transport correction), hence this form. */
typedef struct {
  int n_mat;
  int n_e;
  int n_leg;
  const double *w;
  const double *e;
  const double *S;
  const double *T;
  const double *dG;
} dlra_materials;

/* Pencil beam (Sec. 4): Gaussian energy spectrum N(E0, sigma_E) and Gaussian
 * lateral profile of standard deviation spot_sigma around the axis through
 * pos along the unit vector dir.  weight scales the beam's source (protons
 * per unit of the plan); the deposited energy is linear in it. */
typedef struct {
  double E0, sigma_E, spot_sigma, weight;
  double pos[3];
  double dir[3];
} dlra_beam;

/* Method options.
 *   pn_degree     N of the real spherical-harmonics expansion, m = (N+1)^2
 *   n_steps       energy steps on [e_cut, E_max], E_max = the largest
 *                 E0 + e_max_sigmas*sigma_E of the context's beams
 *   rank_mode     DLRA_RANK_FIXED (rank r) or DLRA_RANK_ADAPTIVE
 *                 (relative L1 singular-value tail <= trunc_tol, rank clamped
 *                 to [r_min, r_max], initial rank r_min) (Sec. 2.2)
 *   precision     DLRA_FP64, or DLRA_MIXED: FP32 storage, stencil and
 *                 projections with FP32 accumulation; QR, SVD and the rank
 *                 decisions in FP64
 *   aug_tol       drop tolerance of basis augmentation, relative to ||K||_F
 *   floor_tol     singular values <= floor_tol * sigma_1 keep no direction;
 *                 their slots are filled from the previous basis
 *   fill_tol      acceptance threshold of filler directions
 *   nu_max        CFL number of the RK4 substep rule (0: 0.45 in 2D, 0.35 in 3D)
 *   n_sub_max     upper bound on RK4 substeps per energy step (DLRA_E_CFL)
 *   ray_h_max     maximal Crank-Nicolson step of the ray tracer, cm (Sec. 3.2)
 *   n_groups      DG energy groups of the ray tracer (Sec. 3.2)
 *   beam_cut_sigmas  rays are traced for cells within this many spot sigmas
 *   collision     DLRA_BOLTZMANN or DLRA_FOKKER_PLANCK
 *   egrid         DLRA_EGRID_*; egrid_points: host [n_steps + 1] strictly
 *                 descending energies > 0 for DLRA_EGRID_USER (then E_max and
 *                 e_cut are its first and last entries), else ignored */
typedef struct {
  int pn_degree;
  int n_steps;
  int rank_mode;
  int r, r_min, r_max;
  int precision;
  int n_groups;
  int n_sub_max;
  double e_cut;
  double e_max_sigmas;
  double trunc_tol;
  double aug_tol;
  double floor_tol;
  double fill_tol;
  double nu_max;
  double ray_h_max;
  double beam_cut_sigmas;
  int collision;
  int egrid;
  const double *egrid_points;
} dlra_options;

typedef struct dlra_ctx dlra_ctx;

/* Bytes of device workspace dlra_init needs for this grid, material count,
 * beam count and options. */
int dlra_workspace_size(const dlra_grid *grid, int n_mat, int n_beams, const dlra_options *opt,
                        size_t *bytes);

/* Validates the problem, copies the tables to the device, builds the P_N
 * streaming matrices A_d = int m m^T Omega_d and their eigen-split A_d^{+-}
 * (Sec. 3.3.1-3.3.2), the energy grid, the per-step coefficients at the step
 * midpoints, the RK4 substep counts and the initial low-rank state (S = 0).
 *   n_beams     1 <= n_beams <= 64 beams (host array beams[n_beams]); with
 *               more than one, their weighted uncollided fluxes source one
 *               joint collided solve, sum_b sum_i (w_i psi_b) g_{i,b}^T
 *               (Sec. 4.3), with n_mat * n_beams <= 64
 *   workspace   device memory of at least dlra_workspace_size bytes, 256-byte
 *               aligned, owned by the caller and kept until dlra_destroy
 *   stream      hipStream_t to enqueue on (NULL: the null stream)
 * On success *out receives the context.  Synchronises the stream once.
 * DLRA_E_CFL when a step needs more than n_sub_max RK4 substeps. */
int dlra_init(const dlra_grid *grid, const dlra_materials *mat, int n_beams,
              const dlra_beam *beams, const dlra_options *opt, void *workspace,
              size_t workspace_bytes, void *stream, dlra_ctx **out);

/* Ray tracer for the uncollided flux (Sec. 3.2): for every beam and every
 * cell within beam_cut_sigmas of the beam axis marches a DG-in-energy /
 * Crank-Nicolson ray from the domain entry to the cell centre and stores the
 * step-averaged uncollided flux of every energy step (times the beam weight)
 * and the weighted uncollided deposited energy.  Must precede the first
 * dlra_step (or be replaced by dlra_set_uncollided). */
int uncollided_raytrace(dlra_ctx *ctx);

/* One energy (pseudo-time) step k -> k+1 of the collided flux (Sec. 3.3.3):
 * streaming by the augmented BUG integrator with RK4 substeps (eq. KLS),
 * collided self-scattering (implicit Euler L-step), uncollided in-scattering
 * (explicit Euler K, L, S steps), rank truncation, and accumulation of the
 * collided deposited energy.
 *   rank_out  nullable host pointer; if given, receives the rank after the
 *             step, and the call synchronises the stream and reports
 *             DLRA_E_NUMERIC / DLRA_E_RANK raised by the step's kernels. */
int dlra_step(dlra_ctx *ctx, int *rank_out);

/* The next `count` energy steps, exactly as `count` dlra_step calls would
 * compute them (bitwise), recorded once into a HIP graph (both streams of the
 * context) and launched as one graph: the per-launch host overhead of the
 * small kernels is paid once.  A fixed-rank context only (the adaptive rank
 * rule decides on the host after each truncation), with profiling off and no
 * rank replay pending; otherwise DLRA_E_STATE and nothing runs.  count in
 * [1, steps left].  Asynchronous like dlra_step; a failed capture leaves the
 * context as it was and returns DLRA_E_HIP. */
int dlra_run_graph(dlra_ctx *ctx, int count);

/* Deposited energy of the context's (weighted) beams into the caller's device
 * buffer dose[n_cells] (FP64).  The paper states the quantity (deposited
 * energy, Sec. 4) but not its formula; the library takes the energy lost by
 * the collided flux, int int psi~ dOmega dE over each energy step by the
 * right-endpoint rule, sqrt(4 pi) sum_k dt_k u_0^{k+1}(x) (m_0^0 = 1/sqrt(4 pi)),
 * plus that of the uncollided flux, int S(x, E) psi_u(E, x) dE.
 *   flags bit 0  the uncollided part, bit 1  the collided part,
 *   bit 2  divide by the local density (dose per mass, 0 where it is 0),
 *   bit 3  add into dose instead of overwriting it (summing the separately
 *          solved beams of a plan).
 * Synchronises the stream first and returns DLRA_E_NUMERIC / DLRA_E_RANK if
 * a kernel raised an error flag (then nothing is written). */
int dose_deposit(dlra_ctx *ctx, double *dose, int flags);

/* Test and checkpoint access (host buffers, FP64, synchronous).
 *   dlra_get_state: U [n_cells][r] row-major, S [r][r], V [m][r]; *rank and
 *                   *step receive the current rank and energy-step index;
 *                   any of U, S, V may be NULL (then only sizes are returned).
 *   dlra_set_state: replaces the state by (U, S, V) of rank r at step index
 *                   step (0 <= step <= n_steps); the collided dose is kept. */
int dlra_get_state(dlra_ctx *ctx, double *U, double *S, double *V, int *rank, int *step);
int dlra_set_state(dlra_ctx *ctx, const double *U, const double *S, const double *V,
                   int rank, int step);

/* Uncollided tables after uncollided_raytrace, host FP64:
 *   psibar [n_beams][n_steps][n_cells] step-averaged uncollided flux (times
 *   the beam weight), Du [n_cells] the weighted uncollided deposited energy;
 *   either may be NULL. */
int dlra_get_uncollided(dlra_ctx *ctx, double *psibar, double *Du);

/* Test access: overwrite the uncollided table of one beam and energy step
 * with host FP64 psibar[n_cells] (NULL: leave it), and the uncollided
 * deposited energy with Du[n_cells] (NULL: leave it).  Marks the context as
 * traced (tables never set read as zero).  Synchronous. */
int dlra_set_uncollided(dlra_ctx *ctx, int beam, int step, const double *psibar,
                        const double *Du);

/* Checkpoint of the collided state (rank, step, U, S, V, collided dose) as a
 * byte buffer in host memory.  dlra_save with buf == NULL stores the size
 * needed in *bytes; otherwise *bytes is the buffer's size on input and the
 * bytes written on output (DLRA_E_INVALID if too small).  dlra_load restores
 * a buffer written by dlra_save of a context with the same grid, moments,
 * rank bound, precision, beam count and step count (DLRA_E_INVALID
 * otherwise); the uncollided tables are not part of it.  A run resumed from a
 * checkpoint reproduces the uninterrupted run bitwise.  Both synchronise the
 * stream; dlra_save first reports pending error flags like dlra_sync. */
int dlra_save(dlra_ctx *ctx, void *buf, size_t *bytes);
int dlra_load(dlra_ctx *ctx, const void *buf, size_t bytes);

/* Work of the last uncollided_raytrace (measurement support): Crank-Nicolson
 * substeps marched and block factorisations of M - h/2 A, summed over all
 * rays, and the number of rays.  Synchronous. */
int dlra_raytrace_work(dlra_ctx *ctx, long long *substeps, long long *factorizations,
                       long long *rays);

/* Test access (rank replay): the next `count` truncations take the ranks
 * ranks[0..count) instead of the rank rule, two per energy step (after the
 * streaming step, then after the uncollided source step), clamped to
 * [1, min(2r, r_max)]; count = 0 clears the schedule.  In adaptive mode the
 * rank rule's decisions can flip under rounding-level input changes (a tail
 * sum at the threshold); replaying another implementation's ranks makes the
 * two comparable step by step. */
int dlra_replay_ranks(dlra_ctx *ctx, int count, const int *ranks);

/* Number of RK4 substeps of energy step k (host-side, from dlra_init). */
int dlra_substeps(dlra_ctx *ctx, int k, int *n_sub);

/* Waits for the context's stream, then reports errors raised by its kernels
 * since the last report: DLRA_E_NUMERIC (a non-finite value in the low-rank
 * state, or a non-positive stopping power), DLRA_E_RANK (basis completion
 * failed).  The flags are cleared once reported. */
int dlra_sync(dlra_ctx *ctx);

/* Batched beams.  The paper treats one pencil beam per solve; a treatment
 * plan has many independent beams (Sec. 1, Sec. 4).  This entry point
 * advances several contexts (one beam each, each on its own stream) at once so
 * that the kernels of different beams overlap on the device: host thread t of
 * n_threads (n_threads <= 0: one thread per context) drives contexts t,
 * t + n_threads, ...; each context that has not yet traced its uncollided
 * flux does so first, then up to n_steps energy steps follow, interleaved
 * across the thread's contexts (a context stops at its last step), and
 * finally every stream is waited for.  The result of every context is the
 * one dlra_step alone would give (no data is shared between contexts).
 *   ctxs      host array of n_ctx distinct contexts, not used by other
 *             threads during the call; n_ctx >= 0, n_steps >= 0
 *   returns   DLRA_OK, or the first error raised in any context (the other
 *             workers stop at their next step; the message is available
 *             from dlra_last_error() in the calling thread). */
int dlra_run_batch(dlra_ctx *const *ctxs, int n_ctx, int n_steps, int n_threads);

/* Treatment-plan objective over beam weights and its exact gradient.  The
 * transport equations are linear in the incoming flux (Sec. 3.2, Sec. 3.3),
 * so the dose of a plan is D = sum_b w_b D_b with D_b the dose of beam b at
 * unit weight.  For
 *   J(w) = sum_{x in T} (D(x) - dhat)^2 + lam sum_{x not in T} D(x)^2
 * the gradient is dJ/dw_b = sum_x g(x) D_b(x), g = dJ/dD: the adjoint of the
 * linear dose map, which needs no reverse sweep through the integrator.
 * (Gradients with respect to voxel densities are not provided.)
 *   doses    device, [n_beams][n_cells] FP64, cells x-fastest (dose_deposit)
 *   weights  host, [n_beams]; target: device, [n_cells], nonzero = in T
 *   dhat     prescription level; lam >= 0 weight of the dose outside T
 *   work     device, >= dlra_plan_objective_work(n_cells, n_beams) doubles,
 *            owned by the caller
 *   stream   HIP stream (NULL: the default stream); the call synchronises it
 *   J, grad  host outputs: the objective and [n_beams] gradient entries
 * Sums are taken in a fixed order (identical results on every call).
 * DLRA_E_INVALID for n_cells <= 0, n_beams outside [1, 64], null pointers,
 * a too small work space, lam < 0 or non-finite inputs. */
size_t dlra_plan_objective_work(int n_cells, int n_beams);
int dlra_plan_objective(int n_cells, int n_beams, const double *doses, const double *weights,
                        const unsigned char *target, double dhat, double lam, double *work,
                        size_t work_doubles, void *stream, double *J, double *grad);

/* Allocation-free form of dlra_plan_objective, for callers that cannot
 * allocate device memory or pass a work space (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments and results as dlra_plan_objective without work / work_doubles;
 * the partial sums of its reduction live in a static device array of the
 * library (about 300 KB, one per GPU, held until the process ends) instead
 * of a caller work space, and the residual g(x) is formed per cell inside a
 * single pass instead of being stored, so n_cells is not limited.  The call
 * allocates nothing on the device.  Limit: n_beams <= 64 (DLRA_E_INVALID
 * beyond).  Calls that overlap on one GPU share the array and race; the
 * call synchronises its stream before it returns. */
int dlra_plan_objective_noalloc(int n_cells, int n_beams, const double *doses,
                                const double *weights, const unsigned char *target, double dhat,
                                double lam, void *stream, double *J, double *grad);

/* Timing of the library's own work with HIP events recorded on the context's
 * stream (measurement support).  Every event record between two kernels
 * leaves the device idle for a few microseconds.
 *   dlra_profile(ctx, on): on = 1 records every phase (one event pair per
 *                          timed launch or phase); on = 2 records only the
 *                          whole step (DLRA_PH_STEP), the ray tracer and, once
 *                          per step, the K-step RK4 loop, whose duration goes
 *                          to DLRA_PH_KSTAGE counted as its 4 n_sub stage
 *                          launches (the launch gaps inside the loop
 *                          included); 0 stops.  Counters are reset when
 *                          recording starts.  DLRA_E_INVALID for another on.
 *   dlra_profile_read(ctx, phase, total_ms, count): synchronises and returns
 *                          the summed duration and number of recorded launches
 *                          of one phase (DLRA_PH_*). */
enum {
  DLRA_PH_KSTAGE = 0,      /* one RK4 stage of the K-step stencil kernel */
  DLRA_PH_PROJECTION = 1,  /* stencil projections U^T d(sU) */
  DLRA_PH_LSTEP = 2,       /* L-step RK4 (all substeps of one step) */
  DLRA_PH_AUGMENT = 3,     /* basis augmentation (U and V, both BUG parts) */
  DLRA_PH_SSTEP = 4,       /* S-step RK4 */
  DLRA_PH_TRUNCATE = 5,    /* SVD truncation and basis rotation */
  DLRA_PH_COLLIDED = 6,    /* collided self-scattering L-step and QR */
  DLRA_PH_SOURCE = 7,      /* uncollided source products */
  DLRA_PH_STEP = 8,        /* a whole dlra_step */
  DLRA_PH_RAYTRACE = 9,    /* uncollided_raytrace */
  DLRA_PH_COUNT = 10
};
int dlra_profile(dlra_ctx *ctx, int on);
int dlra_profile_read(dlra_ctx *ctx, int phase, double *total_ms, long long *count);

/* Achievable throughput of the current device for one probe (measurement
 * only: the achievable roofs quoted beside the vendor peaks; nothing of the
 * transport path calls it).  kind 0: FP32 matrix cores (16x16x4 MFMA), 1:
 * FP64 matrix cores (16x16x4 MFMA), 2: FP32 vector FMA, 3: FP64 vector FMA;
 * iters >= 1 loop iterations of independent chains (four accumulators a
 * wave, or eight FMA chains a lane) on 4 blocks of 4 waves per CU.  One
 * warm-up and one timed launch on the legacy default stream; *tflops (host)
 * receives the rate of the timed one.  Allocates and frees a small device
 * buffer.  DLRA_E_INVALID for another kind, iters < 1 or a null tflops;
 * DLRA_E_HIP when a HIP call fails. */
int dlra_roof_probe(int kind, int iters, double *tflops);

/* Releases the context (not the caller's workspace). */
void dlra_destroy(dlra_ctx *ctx);

/* Message of the last failed call on the calling thread. */
const char *dlra_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DLRA_H */
