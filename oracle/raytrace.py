"""Uncollided ray tracer (Sec. 3.2).

Along a ray of depth z the uncollided flux obeys (Sec. 3.2)
  d psi/dz + Sig~ psi = d/dE (S* psi) + 1/2 d/dE (T d psi/dE),  S* = S + 1/2 dT/dE,
with Sig~ = G_0 - G_{N+1} (removal with the extended transport correction).
Energy: discontinuous Galerkin on n_groups equal groups of [E_cut, E_max],
Legendre polynomials of degree <= 2 per group (3 dof), Lax-Friedrichs flux
for slowing down with alpha = S* (pure upwind from higher energy), SIPG for
straggling with penalty 2 (p+1)^2 T / h_E, no inflow at E_max, free outflow and
zero diffusive flux at E_cut, coefficients at 4 Gauss points per group.  The
semi-discrete system M_E dpsi/dz = A psi (A = -G of Sec. 3.2) is linear in the
mixture weights, A(x) = sum_i w_i(x) A_i, and is advanced with Crank-Nicolson,
(M - h/2 A) psi+ = (M + h/2 A) psi, with substeps no longer than 0.01 cm.

Rays (Sec. 3.2, one per target cell): the line through the cell centre along
the beam direction, from its entry into the domain to the centre.  The path is
cut at cell faces and, inside each traversed cell, at the foot of the
perpendicular from that cell's centre; each piece of length L takes
ceil(L / h_max) equal substeps with the material of its cell.  For beams along
a grid axis the rays of one grid row coincide, and one march along the row
yields every midpoint.  psi_u(E, x) = f_perp(d_perp) phi(E) with a lateral
Gaussian normalised to one proton (per cm^2 in 3D, per cm in 2D); cells with
d_perp beyond beam_cut_sigmas spot sigmas get no ray.

Outputs per energy step k: psibar_k(x) = (1/dt) int_{E_{k+1}}^{E_k} psi_u dE
(exact integral of the DG polynomials), and the uncollided deposited energy
D_u(x) = int S(x, E) psi_u(E, x) dE (3-point Gauss per group).
"""
from __future__ import annotations

import math

import numpy as np

from .coeffs import energy_edges


def _slope_table(e_tab, v_tab, E):
    j = np.clip(np.searchsorted(e_tab, E, side="right") - 1, 0, e_tab.size - 2)
    return (v_tab[j + 1] - v_tab[j]) / (e_tab[j + 1] - e_tab[j])


class EnergyDG:
    def __init__(self, e_cut, e_max, n_groups, nq=4):
        self.e_cut, self.e_max, self.G = e_cut, e_max, n_groups
        self.h = (e_max - e_cut) / n_groups
        self.lo = e_cut + self.h * np.arange(n_groups)
        self.nq = nq
        self.mass = np.tile(self.h * np.array([1.0, 1.0 / 3.0, 1.0 / 5.0]), n_groups)

    # Legendre values on [-1, 1]
    @staticmethod
    def _phi(x):
        return np.array([np.ones_like(x), x, 0.5 * (3.0 * x * x - 1.0)])

    @staticmethod
    def _dphi(x):
        return np.array([np.zeros_like(x), np.ones_like(x), 3.0 * x])

    def operator(self, e_tab, S_tab, T_tab, sig_tab):
        """A for one base material (mass coefficients), dense (3G x 3G)."""
        G, h = self.G, self.h
        A = np.zeros((3 * G, 3 * G))
        xq, wq = np.polynomial.legendre.leggauss(self.nq)
        ph, dph = self._phi(xq), self._dphi(xq) * (2.0 / h)
        for g in range(G):
            a = self.lo[g]
            E = a + 0.5 * h * (xq + 1.0)
            wE = 0.5 * h * wq
            S = np.interp(E, e_tab, S_tab)
            T = np.interp(E, e_tab, T_tab)
            dT = _slope_table(e_tab, T_tab, E)
            Ss = S + 0.5 * dT
            Sig = np.interp(E, e_tab, sig_tab)
            blk = (-(ph * (wE * Sig)) @ ph.T          # - int Sig phi_i phi_j
                   - (dph * (wE * Ss)) @ ph.T          # - int phi_i' S* phi_j
                   - 0.5 * (dph * (wE * T)) @ dph.T)   # - 1/2 int T phi_i' phi_j'
            A[3 * g:3 * g + 3, 3 * g:3 * g + 3] += blk
        one = np.ones(3)
        alt = np.array([1.0, -1.0, 1.0])           # phi_i(-1)
        d_top = np.array([0.0, 1.0, 3.0]) * (2.0 / h)   # phi_i'(+1)
        d_bot = np.array([0.0, 1.0, -3.0]) * (2.0 / h)  # phi_i'(-1)
        for g in range(G):
            # bottom face of group g: outflow flux S*(a) psi_g(a)
            ea = self.lo[g]
            Sa = np.interp(ea, e_tab, S_tab) + 0.5 * _slope_table(e_tab, T_tab, ea)
            A[3 * g:3 * g + 3, 3 * g:3 * g + 3] -= Sa * np.outer(alt, alt)
            if g + 1 < G:
                # top face: inflow S*(b) psi_{g+1}(b) from the group above
                eb = self.lo[g] + h
                Sb = np.interp(eb, e_tab, S_tab) + 0.5 * _slope_table(e_tab, T_tab, eb)
                A[3 * g:3 * g + 3, 3 * (g + 1):3 * (g + 1) + 3] += Sb * np.outer(one, alt)
                # SIPG on the interior face between L = g and U = g+1
                Te = np.interp(eb, e_tab, T_tab)
                pen = 18.0 * Te / h
                jump = {0: one, 1: -alt}               # [v] = v_L - v_U
                avgd = {0: 0.5 * Te * d_top, 1: 0.5 * Te * d_bot}   # {T v'}
                cells = {0: g, 1: g + 1}
                for X in (0, 1):
                    for Y in (0, 1):
                        blk = 0.5 * (np.outer(jump[X], avgd[Y]) + np.outer(avgd[X], jump[Y])
                                     - pen * np.outer(jump[X], jump[Y]))
                        cx, cy = cells[X], cells[Y]
                        A[3 * cx:3 * cx + 3, 3 * cy:3 * cy + 3] += blk
        return A

    def project(self, f, nq=8):
        """L2 projection of f(E) onto the DG space."""
        xq, wq = np.polynomial.legendre.leggauss(nq)
        ph = self._phi(xq)
        c = np.zeros(3 * self.G)
        for g in range(self.G):
            E = self.lo[g] + 0.5 * self.h * (xq + 1.0)
            c[3 * g:3 * g + 3] = (ph @ (wq * f(E))) * (np.arange(3) * 2 + 1) / 2.0
        return c

    def integral(self, c, lo, hi):
        """int_lo^hi psi dE for coefficients c (exact)."""
        total = 0.0
        g0 = max(int(math.floor((lo - self.e_cut) / self.h)) - 1, 0)
        g1 = min(int(math.ceil((hi - self.e_cut) / self.h)) + 1, self.G)
        for g in range(g0, g1):
            a = self.lo[g]
            b = a + self.h
            l, u = max(a, lo), min(b, hi)
            if u <= l:
                continue
            x1 = 2.0 * (l - a) / self.h - 1.0
            x2 = 2.0 * (u - a) / self.h - 1.0
            ints = np.array([x2 - x1, 0.5 * (x2**2 - x1**2),
                             0.5 * (x2**3 - x1**3) - 0.5 * (x2 - x1)])
            total += 0.5 * self.h * ints @ c[3 * g:3 * g + 3]
        return total

    def weighted_integral(self, c, fun):
        """int fun(E) psi(E) dE with 3-point Gauss per group."""
        xq, wq = np.polynomial.legendre.leggauss(3)
        ph = self._phi(xq)
        E = (self.lo[:, None] + 0.5 * self.h * (xq[None, :] + 1.0))
        vals = c.reshape(self.G, 3) @ ph                 # (G, 3)
        return float(np.sum(0.5 * self.h * wq[None, :] * fun(E) * vals))

    def functional(self, f):
        """Row vector l with l @ c = f(c) for a linear functional f of the coefficients."""
        eye = np.eye(3 * self.G)
        return np.array([f(eye[j]) for j in range(3 * self.G)])


def removal_table(problem, i):
    """Tabulated removal rate of the uncollided flux for material i:
    G_0 - G_{N+1} (Boltzmann with the extended transport correction), or zero
    (Fokker-Planck: Gamma_out = 0, Sec. 3.1)."""
    mat = problem.materials
    if getattr(problem.options, "collision", "boltzmann") == "fokker_planck":
        return np.zeros_like(mat.e)
    return mat.dG[i, :, problem.options.pn_degree + 1]


def material_operators(problem, dg):
    mat = problem.materials
    return [dg.operator(mat.e, mat.S[i], mat.T[i], removal_table(problem, i))
            for i in range(mat.n_mat)]


# ------------------------------------------------------------------ geometry

def _box(grid):
    L = [grid.nx * grid.dx, grid.ny * grid.dy, grid.nz * grid.dz]
    n = [grid.nx, grid.ny, grid.nz]
    D = [grid.dx, grid.dy, grid.dz]
    return L, n, D


def cell_of_point(grid, p):
    L, n, D = _box(grid)
    idx = [min(max(int(math.floor(p[d] / D[d])), 0), n[d] - 1) for d in range(3)]
    if grid.dim == 2:
        idx[2] = 0
    return (idx[2] * grid.ny + idx[1]) * grid.nx + idx[0]


def ray_pieces(grid, xc, omega):
    """[(cell, length)] from the domain entry to xc along omega."""
    L, n, D = _box(grid)
    dims = 2 if grid.dim == 2 else 3
    t_in = -math.inf
    for d in range(dims):
        if omega[d] != 0.0:
            t1 = (0.0 - xc[d]) / omega[d]
            t2 = (L[d] - xc[d]) / omega[d]
            t_in = max(t_in, min(t1, t2))
    ts = [t_in, 0.0]
    for d in range(dims):
        if omega[d] != 0.0:
            for j in range(n[d] + 1):
                t = (j * D[d] - xc[d]) / omega[d]
                if t_in < t < 0.0:
                    ts.append(t)
    ts = sorted(ts)
    chords = []
    for a, b in zip(ts[:-1], ts[1:]):
        if b <= a:
            continue
        mid = [xc[d] + 0.5 * (a + b) * omega[d] for d in range(3)]
        chords.append((cell_of_point(grid, mid), a, b))
    centers = grid.centers()
    pieces = []
    for cell, a, b in chords:
        tf = float(np.dot(centers[cell] - np.asarray(xc), omega))
        if a < tf < b:
            pieces += [(cell, tf - a), (cell, b - tf)]
        else:
            pieces.append((cell, b - a))
    return pieces


def n_substeps(length, h_max):
    return max(1, math.ceil(length / h_max - 1e-9))


def lateral(grid, beam, xc):
    """(f_perp, d_perp) for the cell centre xc."""
    om = np.asarray(beam.dir, dtype=np.float64)
    rel = np.asarray(xc) - np.asarray(beam.pos, dtype=np.float64)
    perp = rel - np.dot(rel, om) * om
    d = float(np.linalg.norm(perp))
    s = beam.spot_sigma
    if grid.dim == 2:
        f = math.exp(-0.5 * d * d / (s * s)) / (math.sqrt(2.0 * math.pi) * s)
    else:
        f = math.exp(-0.5 * d * d / (s * s)) / (2.0 * math.pi * s * s)
    return f, d


# ------------------------------------------------------------------ tracing

class Tracer:
    def __init__(self, problem, beam, edges=None):
        """edges: the run's energy grid E_0 > ... > E_n (default: the beam's own)."""
        o = problem.options
        self.problem, self.beam = problem, beam
        self.edges = energy_edges(problem, [beam]) if edges is None else np.asarray(edges)
        self.e_max, self.e_cut = float(self.edges[0]), float(self.edges[-1])
        self.dg = EnergyDG(self.e_cut, self.e_max, o.n_groups)
        self.ops = material_operators(problem, self.dg)
        self._cache = {}
        mat = problem.materials
        # linear functionals of the DG coefficients: step integrals and, per
        # material, int S_i(E) psi dE
        E = self.edges
        self.step_int = np.stack([
            self.dg.functional(lambda c, k=k: self.dg.integral(c, E[k + 1], E[k]))
            / (E[k] - E[k + 1]) for k in range(o.n_steps)])
        self.stop_int = np.stack([
            self.dg.functional(lambda c, i=i: self.dg.weighted_integral(
                c, lambda E: np.interp(E, mat.e, mat.S[i])))
            for i in range(mat.n_mat)])
        E0, sE = beam.E0, beam.sigma_E
        self.c0 = self.dg.project(
            lambda E: np.exp(-0.5 * ((E - E0) / sE) ** 2) / (math.sqrt(2.0 * math.pi) * sE))

    def propagator(self, cell, length):
        o = self.problem.options
        ns = n_substeps(length, o.ray_h_max)
        h = length / ns
        w = self.problem.materials.w[:, cell]
        key = (w.tobytes(), h)
        if key not in self._cache:
            A = sum(w[i] * self.ops[i] for i in range(len(self.ops)))
            M = np.diag(self.dg.mass)
            self._cache[key] = np.linalg.solve(M - 0.5 * h * A, M + 0.5 * h * A)
        return self._cache[key], ns

    def march(self, pieces):
        c = self.c0.copy()
        for cell, length in pieces:
            P, ns = self.propagator(cell, length)
            for _ in range(ns):
                c = P @ c
        return c

    def outputs(self, c, cell, f):
        """(psibar[k] for all steps, D_u) for DG coefficients c at cell."""
        w = self.problem.materials.w[:, cell]
        return f * (self.step_int @ c), f * float(w @ (self.stop_int @ c))

    def axis(self):
        om = np.asarray(self.beam.dir, dtype=np.float64)
        nz = np.flatnonzero(om != 0.0)
        return int(nz[0]) if nz.size == 1 else None

    def trace(self, rowwise=True, rows=None, cells=None):
        """Return (psibar (n_steps, n), D_u (n,)) for the beam.  For a beam
        along a grid axis, rows (indices into grid_rows()) restricts the march
        to those rows; otherwise cells restricts the per-cell rays to those
        target cells.  The other cells stay zero."""
        g = self.problem.grid
        o = self.problem.options
        if g.dim == 2 and self.beam.dir[2] != 0.0:
            raise ValueError("2D problems need in-plane beams")
        n = g.n
        psibar = np.zeros((o.n_steps, n))
        Du = np.zeros(n)
        centers = g.centers()
        cut = o.beam_cut_sigmas * self.beam.spot_sigma
        ax = self.axis() if rowwise else None
        if ax is not None:
            self._trace_rows(ax, centers, cut, psibar, Du, rows)
            return psibar, Du
        if rows is not None:
            raise ValueError("a row subset needs a beam along a grid axis")
        om = tuple(float(v) for v in self.beam.dir)
        for cell in (range(n) if cells is None else (int(c) for c in cells)):
            f, d = lateral(g, self.beam, centers[cell])
            if d > cut:
                continue
            c = self.march(ray_pieces(g, centers[cell], om))
            psibar[:, cell], Du[cell] = self.outputs(c, cell, f)
        return psibar, Du

    def grid_rows(self):
        """Cell indices of the grid rows along the beam axis, one row per
        line, in the order the row march takes them (before the beam's sign)."""
        g = self.problem.grid
        shape = (g.nz, g.ny, g.nx)
        idx = np.arange(g.n).reshape(shape)
        np_ax = (2, 1, 0)[self.axis()]
        return np.moveaxis(idx, np_ax, -1).reshape(-1, shape[np_ax])

    def _trace_rows(self, ax, centers, cut, psibar, Du, only=None):
        g = self.problem.grid
        sign = 1 if self.beam.dir[ax] > 0 else -1
        rows = self.grid_rows()
        if only is not None:
            rows = rows[np.asarray(only, dtype=np.int64)]
        D = (g.dx, g.dy, g.dz)[ax]
        for row in rows:
            cells = row if sign > 0 else row[::-1]
            f, d = lateral(g, self.beam, centers[cells[0]])
            if d > cut:
                continue
            c = self.c0.copy()
            for cell in cells:
                for half in (0, 1):
                    P, ns = self.propagator(int(cell), 0.5 * D)
                    for _ in range(ns):
                        c = P @ c
                    if half == 0:
                        psibar[:, cell], Du[cell] = self.outputs(c, int(cell), f)
