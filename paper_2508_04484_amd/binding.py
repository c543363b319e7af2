"""ctypes binding of libdlra.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch provides the device
workspace and the stream.  Importing this module does not need a GPU; creating
a solver does, and fails loudly when the library or the GPU is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdlra.so")

DLRA_OK = 0
ERRORS = {-1: "DLRA_E_INVALID", -2: "DLRA_E_NOMEM", -3: "DLRA_E_HIP", -4: "DLRA_E_NUMERIC",
          -5: "DLRA_E_CFL", -6: "DLRA_E_RANK", -7: "DLRA_E_STATE"}
RANK_FIXED, RANK_ADAPTIVE = 0, 1
FP64, MIXED = 0, 1
COLLISION = {"boltzmann": 0, "fokker_planck": 1}
EGRID = {"uniform": 0, "proportional": 1, "cfl": 2, "user": 3}
DOSE_UNCOLLIDED, DOSE_COLLIDED, DOSE_PER_MASS, DOSE_ACCUMULATE = 1, 2, 4, 8

EXPORTS = ["dlra_workspace_size", "dlra_init", "uncollided_raytrace", "dlra_step",
           "dlra_run_graph",
           "dose_deposit", "dlra_get_state", "dlra_set_state", "dlra_get_uncollided",
           "dlra_set_uncollided", "dlra_save", "dlra_load",
           "dlra_substeps", "dlra_raytrace_work", "dlra_replay_ranks", "dlra_sync", "dlra_profile", "dlra_profile_read", "dlra_run_batch",
           "dlra_plan_objective", "dlra_plan_objective_work", "dlra_plan_objective_noalloc",
           "dlra_roof_probe", "dlra_destroy", "dlra_last_error"]
PHASES = ["kstage", "projection", "lstep", "augment", "sstep", "truncate", "collided", "source",
          "step", "raytrace"]


class DlraError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class Materials(C.Structure):
    _fields_ = [("n_mat", C.c_int), ("n_e", C.c_int), ("n_leg", C.c_int),
                ("w", C.POINTER(C.c_double)), ("e", C.POINTER(C.c_double)),
                ("S", C.POINTER(C.c_double)), ("T", C.POINTER(C.c_double)),
                ("dG", C.POINTER(C.c_double))]


class Beam(C.Structure):
    _fields_ = [("E0", C.c_double), ("sigma_E", C.c_double), ("spot_sigma", C.c_double),
                ("weight", C.c_double), ("pos", C.c_double * 3), ("dir", C.c_double * 3)]


class Options(C.Structure):
    _fields_ = [("pn_degree", C.c_int), ("n_steps", C.c_int), ("rank_mode", C.c_int),
                ("r", C.c_int), ("r_min", C.c_int), ("r_max", C.c_int),
                ("precision", C.c_int), ("n_groups", C.c_int), ("n_sub_max", C.c_int),
                ("e_cut", C.c_double), ("e_max_sigmas", C.c_double),
                ("trunc_tol", C.c_double), ("aug_tol", C.c_double),
                ("floor_tol", C.c_double), ("fill_tol", C.c_double),
                ("nu_max", C.c_double), ("ray_h_max", C.c_double),
                ("beam_cut_sigmas", C.c_double), ("collision", C.c_int), ("egrid", C.c_int),
                ("egrid_points", C.POINTER(C.c_double))]


_lib = None
_lib_path = None


def load(path: str = LIB_PATH):
    """Load libdlra.so (once per process: contexts belong to the copy that made
    them); raises when it has not been built, or when another path is asked
    for after one has been loaded."""
    global _lib, _lib_path
    if _lib is not None:
        if os.path.realpath(path) != _lib_path:
            raise RuntimeError(f"{_lib_path} is already loaded in this process; "
                               f"{path} can only be used from another process")
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2508_04484_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(path)
    _lib_path = os.path.realpath(path)
    P, I, D, V = C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_void_p
    lib.dlra_workspace_size.argtypes = [C.POINTER(Grid), I, I, C.POINTER(Options),
                                        C.POINTER(C.c_size_t)]
    lib.dlra_init.argtypes = [C.POINTER(Grid), C.POINTER(Materials), I, C.POINTER(Beam),
                              C.POINTER(Options), V, C.c_size_t, V, C.POINTER(P)]
    lib.uncollided_raytrace.argtypes = [P]
    lib.dlra_step.argtypes = [P, C.POINTER(I)]
    lib.dlra_run_graph.argtypes = [P, I]
    lib.dlra_roof_probe.argtypes = [I, I, C.POINTER(C.c_double)]
    lib.dose_deposit.argtypes = [P, V, I]
    lib.dlra_get_state.argtypes = [P, D, D, D, C.POINTER(I), C.POINTER(I)]
    lib.dlra_set_state.argtypes = [P, D, D, D, I, I]
    lib.dlra_get_uncollided.argtypes = [P, D, D]
    lib.dlra_set_uncollided.argtypes = [P, I, I, D, D]
    lib.dlra_save.argtypes = [P, V, C.POINTER(C.c_size_t)]
    lib.dlra_load.argtypes = [P, V, C.c_size_t]
    lib.dlra_substeps.argtypes = [P, I, C.POINTER(I)]
    lib.dlra_raytrace_work.argtypes = [P] + [C.POINTER(C.c_longlong)] * 3
    lib.dlra_replay_ranks.argtypes = [P, I, C.POINTER(I)]
    lib.dlra_sync.argtypes = [P]
    lib.dlra_profile.argtypes = [P, I]
    lib.dlra_profile_read.argtypes = [P, I, D, C.POINTER(C.c_longlong)]
    lib.dlra_run_batch.argtypes = [C.POINTER(P), I, I, I]
    lib.dlra_plan_objective.argtypes = [I, I, V, D, V, C.c_double, C.c_double, V, C.c_size_t, V,
                                        D, D]
    lib.dlra_plan_objective_work.argtypes = [I, I]
    lib.dlra_plan_objective_noalloc.argtypes = [I, I, V, D, V, C.c_double, C.c_double, V, D, D]
    lib.dlra_destroy.argtypes = [P]
    lib.dlra_destroy.restype = None
    lib.dlra_last_error.restype = C.c_char_p
    for name in EXPORTS[:-2]:
        getattr(lib, name).restype = C.c_int
    lib.dlra_plan_objective_work.restype = C.c_size_t
    _lib = lib
    return lib


def check(rc: int):
    if rc != DLRA_OK:
        raise DlraError(rc, load().dlra_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_grid(g) -> Grid:
    return Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz)


def make_options(o):
    """(Options, keep-alive) for a workloads Options; the second item holds the
    user energy grid the struct points to."""
    pts = np.ascontiguousarray(getattr(o, "egrid_points", ()) or (), dtype=np.float64)
    egrid = EGRID[getattr(o, "egrid", "uniform")]
    opts = Options(o.pn_degree, o.n_steps,
                   RANK_FIXED if o.rank_mode == "fixed" else RANK_ADAPTIVE,
                   o.r, o.r_min, o.r_max, FP64 if o.precision == "fp64" else MIXED,
                   o.n_groups, getattr(o, "n_sub_max", 0), o.e_cut, o.e_max_sigmas,
                   o.trunc_tol, o.aug_tol, o.floor_tol, o.fill_tol, o.nu_max, o.ray_h_max,
                   o.beam_cut_sigmas, COLLISION[getattr(o, "collision", "boltzmann")], egrid,
                   _dptr(pts) if pts.size else None)
    return opts, pts


def make_beam(b, weight=None) -> Beam:
    return Beam(b.E0, b.sigma_E, b.spot_sigma, b.weight if weight is None else weight,
                (C.c_double * 3)(*b.pos), (C.c_double * 3)(*b.dir))


ROOF_PROBES = ("fp32_mfma", "fp64_mfma", "fp32_fma", "fp64_fma")


def roof_probe(kind: str, iters: int) -> float:
    """Achievable TFLOP/s of one throughput probe on the current device
    (dlra_roof_probe): kind is one of ROOF_PROBES."""
    lib = load()
    out = C.c_double(0.0)
    check(lib.dlra_roof_probe(ROOF_PROBES.index(kind), int(iters), C.byref(out)))
    return out.value


def workspace_size(problem, n_beams: int = 1) -> int:
    lib = load()
    out = C.c_size_t(0)
    opts, _keep = make_options(problem.options)
    check(lib.dlra_workspace_size(C.byref(make_grid(problem.grid)), problem.materials.n_mat,
                                  int(n_beams), C.byref(opts), C.byref(out)))
    return int(out.value)


class Solver:
    """A context of the library on the current CUDA (HIP) device: one beam of a
    problem, or several beams in one joint collided solve.

      beams        indices into problem.beams (default: all of them)
      unit_weight  solve at unit beam weight (the single-beam dose) instead of
                   the beams' own weights

    Usage: s = Solver(problem); s.raytrace(); s.run(); dose = s.dose()."""

    def __init__(self, problem, beams=None, unit_weight=False, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the DLRA library needs a GPU (torch.cuda.is_available() is False)")
        self.lib = load()
        self.problem = problem
        idx = list(range(len(problem.beams))) if beams is None else list(beams)
        self.beams = [problem.beams[b] for b in idx]
        self.n_beams = len(self.beams)
        self.torch = torch
        size = workspace_size(problem, self.n_beams)
        self._ws = torch.empty(size + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._ws.record_stream(self.stream)
        mat = problem.materials
        self._arrays = [np.ascontiguousarray(a, dtype=np.float64)
                        for a in (mat.w, mat.e, mat.S, mat.T, mat.dG)]
        w, e, S, T, dG = self._arrays
        m = Materials(mat.n_mat, e.size, dG.shape[-1], _dptr(w), _dptr(e), _dptr(S), _dptr(T),
                      _dptr(dG))
        barr = (Beam * self.n_beams)(*[make_beam(b, 1.0 if unit_weight else None)
                                       for b in self.beams])
        opts, _keep = make_options(problem.options)
        ctx = C.c_void_p(0)
        check(self.lib.dlra_init(C.byref(make_grid(problem.grid)), C.byref(m), self.n_beams,
                                 barr, C.byref(opts), C.c_void_p(self._ws_ptr), C.c_size_t(size),
                                 C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self.n = problem.grid.n
        self.m = problem.m

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            # the library syncs its streams before releasing the context; the
            # workspace goes back to torch only after that
            rc = self.lib.dlra_sync(self.ctx)
            self.lib.dlra_destroy(self.ctx)
            self.ctx = None
            self.stream.synchronize()
            check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def raytrace(self):
        check(self.lib.uncollided_raytrace(self.ctx))

    def step(self, sync: bool = False):
        if sync:
            r = C.c_int(0)
            check(self.lib.dlra_step(self.ctx, C.byref(r)))
            return r.value
        check(self.lib.dlra_step(self.ctx, None))
        return None

    def run_graph(self, count: int):
        """The next `count` steps recorded and launched as one HIP graph
        (fixed rank only); bitwise the same as `count` step() calls."""
        check(self.lib.dlra_run_graph(self.ctx, count))

    def run(self, n_steps=None):
        n_steps = self.problem.options.n_steps if n_steps is None else n_steps
        for _ in range(n_steps):
            self.step()
        self.sync()

    def sync(self):
        check(self.lib.dlra_sync(self.ctx))

    def dose(self, flags=DOSE_UNCOLLIDED | DOSE_COLLIDED, out=None):
        """Deposited energy (torch float64 on the GPU); with out given and
        flags containing DOSE_ACCUMULATE it is added into out."""
        if out is None:
            out = self.torch.empty(self.n, dtype=self.torch.float64, device="cuda")
        check(self.lib.dose_deposit(self.ctx, C.c_void_p(out.data_ptr()), flags))
        self.sync()
        return out

    def profile(self, on=True, light=False):
        """Event timing: every phase, or (light) only the step, the ray tracer
        and the K-step RK4 loop once per step."""
        check(self.lib.dlra_profile(self.ctx, (2 if light else 1) if on else 0))

    def profile_read(self):
        """{phase: (total_ms, launches)} of the event timings recorded so far."""
        out = {}
        for i, name in enumerate(PHASES):
            ms, cnt = C.c_double(0.0), C.c_longlong(0)
            check(self.lib.dlra_profile_read(self.ctx, i, C.byref(ms), C.byref(cnt)))
            out[name] = (ms.value, cnt.value)
        return out

    def replay_ranks(self, ranks):
        """Prescribe the ranks of the next truncations (two per energy step)."""
        arr = (C.c_int * max(len(ranks), 1))(*[int(r) for r in ranks])
        check(self.lib.dlra_replay_ranks(self.ctx, len(ranks), arr))

    def raytrace_work(self):
        """(Crank-Nicolson substeps, block factorisations, rays) of the last ray trace."""
        a, b, c = C.c_longlong(0), C.c_longlong(0), C.c_longlong(0)
        check(self.lib.dlra_raytrace_work(self.ctx, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def substeps(self, k):
        v = C.c_int(0)
        check(self.lib.dlra_substeps(self.ctx, k, C.byref(v)))
        return v.value

    def state(self):
        r, k = C.c_int(0), C.c_int(0)
        check(self.lib.dlra_get_state(self.ctx, None, None, None, C.byref(r), C.byref(k)))
        U = np.zeros((self.n, r.value))
        S = np.zeros((r.value, r.value))
        V = np.zeros((self.m, r.value))
        check(self.lib.dlra_get_state(self.ctx, _dptr(U), _dptr(S), _dptr(V), C.byref(r),
                                      C.byref(k)))
        return U, S, V, k.value

    def set_state(self, U, S, V, step):
        U = np.ascontiguousarray(U, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        check(self.lib.dlra_set_state(self.ctx, _dptr(U), _dptr(S), _dptr(V), U.shape[1], step))

    def uncollided(self):
        """(psibar, Du): psibar [n_steps, n] for one beam, [n_beams, n_steps, n]
        for several."""
        ps = np.zeros((self.n_beams, self.problem.options.n_steps, self.n))
        Du = np.zeros(self.n)
        check(self.lib.dlra_get_uncollided(self.ctx, _dptr(ps), _dptr(Du)))
        return (ps[0] if self.n_beams == 1 else ps), Du

    def set_uncollided(self, beam, step, psibar=None, Du=None):
        ps = None if psibar is None else np.ascontiguousarray(psibar, dtype=np.float64)
        du = None if Du is None else np.ascontiguousarray(Du, dtype=np.float64)
        check(self.lib.dlra_set_uncollided(self.ctx, int(beam), int(step),
                                           None if ps is None else _dptr(ps),
                                           None if du is None else _dptr(du)))

    def save(self) -> bytes:
        """Checkpoint of the collided state as bytes (dlra_save)."""
        need = C.c_size_t(0)
        check(self.lib.dlra_save(self.ctx, None, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        check(self.lib.dlra_save(self.ctx, buf, C.byref(need)))
        return buf.raw[:need.value]

    def load(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        check(self.lib.dlra_load(self.ctx, buf, len(data)))


class BeamSolver(Solver):
    """One pencil beam of a problem at unit weight (the single-beam solve)."""

    def __init__(self, problem, beam_index: int = 0, stream=None):
        super().__init__(problem, [beam_index], unit_weight=True, stream=stream)
        self.beam = self.beams[0]


def run_batch(solvers, n_steps=None, n_threads=0):
    """Advance several solvers (each on its own stream) together through the
    library's batch scheduler: ray traces first where missing, then n_steps
    energy steps (default: all), concurrently; returns when all are done."""
    if not solvers:
        return
    lib = solvers[0].lib
    n_steps = max(s.problem.options.n_steps for s in solvers) if n_steps is None else n_steps
    arr = (C.c_void_p * len(solvers))(*[s.ctx.value for s in solvers])
    check(lib.dlra_run_batch(arr, len(solvers), int(n_steps), int(n_threads)))


def batch_solvers(problem, beam_indices=None):
    """One BeamSolver per beam, each on a stream of its own (default priority)."""
    import torch
    idx = range(len(problem.beams)) if beam_indices is None else beam_indices
    return [BeamSolver(problem, b, stream=torch.cuda.Stream()) for b in idx]


def plan_objective(doses, weights, target, dhat, lam, stream=None):
    """Plan objective J and its gradient over the beam weights (the library's
    dlra_plan_objective).  doses: torch float64 CUDA tensor [n_beams, n_cells];
    target: torch uint8 CUDA tensor [n_cells]; weights: host sequence.
    Returns (J, grad as a numpy array)."""
    import torch
    lib = load()
    nb, n = int(doses.shape[0]), int(doses.shape[1])
    if doses.dtype != torch.float64 or not doses.is_cuda or not doses.is_contiguous():
        raise ValueError("doses must be a contiguous float64 CUDA tensor")
    if target.dtype != torch.uint8 or not target.is_cuda or target.numel() != n:
        raise ValueError("target must be a uint8 CUDA tensor of n_cells entries")
    w = np.ascontiguousarray(weights, dtype=np.float64)
    if w.shape != (nb,):
        raise ValueError("one weight per beam")
    nwork = lib.dlra_plan_objective_work(n, nb)
    if nwork == 0:
        check(lib.dlra_plan_objective(n, nb, None, None, None, 0.0, 0.0, None, 0, None,
                                      None, None))
    work = torch.empty(nwork, dtype=torch.float64, device=doses.device)
    st = torch.cuda.current_stream(doses.device) if stream is None else stream
    J = C.c_double(0.0)
    grad = np.zeros(nb)
    check(lib.dlra_plan_objective(n, nb, C.c_void_p(doses.data_ptr()), _dptr(w),
                                  C.c_void_p(target.data_ptr()), float(dhat), float(lam),
                                  C.c_void_p(work.data_ptr()), nwork, C.c_void_p(st.cuda_stream),
                                  C.byref(J), _dptr(grad)))
    return J.value, grad


def batch_group_size(problem, reserve=0.1):
    """Beams of a problem whose work spaces fit the free device memory at once
    (keeping `reserve` of it free), at least 1."""
    import torch
    free, _ = torch.cuda.mem_get_info()
    per = workspace_size(problem.single_beam(0), 1)
    return max(1, min(len(problem.beams), int(free * (1.0 - reserve)) // max(per, 1)))


def solve(problem, n_steps=None, joint=False, batch=1):
    """Deposited energy of all beams of a problem at their weights (torch
    float64 on the GPU): one joint collided solve (joint=True), or every beam
    solved on its own and its weighted dose added into one buffer by the
    library (dose_deposit with DOSE_ACCUMULATE).  With batch > 1 (0: as many
    as fit the free device memory) the separate beams run in groups through
    the library's batch scheduler, each on a stream of its own; the doses are
    added in beam order, so the result is bitwise the one-by-one solve's."""
    import torch
    if joint:
        s = Solver(problem)
        s.raytrace()
        s.run(n_steps)
        d = s.dose()
        s.close()
        return d
    total = torch.zeros(problem.grid.n, dtype=torch.float64, device="cuda")
    torch.cuda.current_stream().synchronize()   # the solvers' streams add into it
    nb = len(problem.beams)
    group = batch_group_size(problem) if batch == 0 else max(1, int(batch))
    for b0 in range(0, nb, group):
        idx = list(range(b0, min(nb, b0 + group)))
        if len(idx) == 1:
            solvers = [Solver(problem, idx)]
            solvers[0].raytrace()
            solvers[0].run(n_steps)
        else:
            solvers = [Solver(problem, [b], stream=torch.cuda.Stream()) for b in idx]
            run_batch(solvers, n_steps)
        for s in solvers:
            s.dose(DOSE_UNCOLLIDED | DOSE_COLLIDED | DOSE_ACCUMULATE, out=total)
            s.close()
    return total
