"""Literal micro-oracle: Eq. (1) discretised on a full space-time grid.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every term of Eq. (1) is evaluated at the centre (x_c, t_c) of the square being
solved, in physical coordinates, exactly as the paper states it:
  * the line-1 terms (d/dt, d/dx, W psi and the delay term) by the "square"
    of Eq. (3): averages over the four corners of a square of side Delta;
  * the source terms of lines 2-3 by the "bar" of Eq. (4): the average of two
    points Delta apart at the same time;
  * the drive (line 4) analytically at the centre.
The unknown top-right corner is found by evaluating the square's left-hand
side at two trial values (it is affine in the unknown), so no hand algebra
of the update enters.  Pure Python loops: tiny grids only.

Read modes (the paper reads its own marched values wherever they are stored):
  "hybrid"     x <= -a is read from the exact solution; x > -a is marched.
  "paper_diag" `diag_cols` extra columns left of -a are marched too, and only
               x left of them is read from the exact solution (the paper's
               test 1 compares these columns with the exact solution).
"""
from __future__ import annotations

import math

import numpy as np


class Micro:
    """E and phi: the one-excitation amplitude on the rows and the packet.
    Two different photons (Sec. 2 case (c)): phi and E are photon 1's packet
    and e0^(1), phi2 and E2 photon 2's; then chi(x1, x2, 0) =
    (A/sqrt 2)[phi(x1) phi2(x2) + phi(x2) phi2(x1)] and, in x <= -a,
    psi = A [phi(x-t) E2(t) + phi2(x-t) E(t)], with A of Eq. (11)."""

    def __init__(self, inst, E: np.ndarray, phi, *, mode: str = "hybrid", diag_cols: int = 0,
                 phi2=None, E2: np.ndarray | None = None):
        d = inst if isinstance(inst, dict) else inst.as_dict()
        self.Nx, self.D, self.Nt = int(d["Nx"]), int(d["D"]), int(d["Nt"])
        self.dl = float(d["Delta"])
        self.a = 0.5 * self.D * self.dl
        self.G = float(d["Gamma"])
        self.W = 1j * float(d["omega0"]) + self.G / 2.0
        self.incident = int(d["incident"])
        self.theta_ph = float(d.get("phase", 0.0))
        self.E = np.asarray(E, dtype=np.complex128)
        self.phi = phi                     # callable: phi(x) for scalar x
        self.mode = mode
        self.lo = 1 if mode == "hybrid" else 1 - int(diag_cols)   # first marched column
        self.psi = np.zeros((self.Nt + 1, self.Nx - self.lo + 1), np.complex128)
        self.done_row = 0                  # rows <= done_row are complete
        self.cur = (0, 0)                  # cell being solved (row, col)
        self.c_ex = 1.0 if self.incident == 2 else math.sqrt(2.0) * complex(math.cos(self.theta_ph), math.sin(self.theta_ph))
        self.phi2 = phi2
        self.E2 = None if E2 is None else np.asarray(E2, dtype=np.complex128)
        if phi2 is not None:
            k1, k2 = float(d["k1"]), float(d["k2"])
            a1, a2 = float(d["alpha1"]), float(d["alpha2"])
            num = 4 * (k1 - k2) ** 2 + ((a1 + a2) * self.G) ** 2
            self.A = math.sqrt(num / (num + 4 * a1 * a2 * self.G ** 2))
            self.c_ex = self.A * complex(math.cos(self.theta_ph), math.sin(self.theta_ph))

    # ---- grid <-> coordinates -------------------------------------------
    def col(self, x: float) -> int:
        q = (x + self.a) / self.dl
        i = int(round(q))
        assert abs(q - i) < 1e-6, f"x={x} is off the grid"
        return i

    def row(self, t: float) -> int:
        q = t / self.dl
        r = int(round(q))
        assert abs(q - r) < 1e-6, f"t={t} is off the grid"
        return r

    # ---- the solution at a grid point -----------------------------------
    def exact(self, i: int, r: int) -> complex:
        x = -self.a + i * self.dl
        t = r * self.dl
        if self.phi2 is not None:
            return self.c_ex * (self.phi(x - t) * self.E2[r] + self.phi2(x - t) * self.E[r])
        return self.c_ex * self.phi(x - t) * self.E[r]

    def value(self, x: float, t: float) -> complex:
        if t < -1e-9 * self.dl:
            return 0.0
        i, r = self.col(x), self.row(t)
        if i < self.lo:
            return self.exact(i, r)
        assert i <= self.Nx, "read right of the box"
        cr, ci = self.cur
        assert r < cr or (r == cr and i < ci), f"read of ({i},{r}) before it is solved (at {ci},{cr})"
        return self.psi[r, i - self.lo]

    def chi0(self, x1: float, x2: float) -> complex:
        if self.incident == 2:
            return 0.0
        ph = complex(math.cos(self.theta_ph), math.sin(self.theta_ph))
        if self.phi2 is not None:
            return ph * self.A / math.sqrt(2.0) * (self.phi(x1) * self.phi2(x2) + self.phi(x2) * self.phi2(x1))
        return ph * self.phi(x1) * self.phi(x2)

    # ---- Eq. (3) and Eq. (4) --------------------------------------------
    def square(self, X: float, T: float) -> complex:
        h = 0.5 * self.dl
        return 0.25 * (self.value(X - h, T - h) + self.value(X + h, T - h)
                       + self.value(X - h, T + h) + self.value(X + h, T + h))

    def bar(self, X: float, T: float) -> complex:
        h = 0.5 * self.dl
        return 0.5 * (self.value(X - h, T) + self.value(X + h, T))

    @staticmethod
    def step(y: float, tol: float) -> float:
        """theta(y) with theta(0) = 1"""
        return 1.0 if y > -tol else 0.0

    # ---- one square ------------------------------------------------------
    def solve(self, i: int, r: int) -> complex:
        dl, a, G, W = self.dl, self.a, self.G, self.W
        h = 0.5 * dl
        tol = 1e-6 * dl
        xc = -a + i * dl - h
        tc = r * dl - h
        self.cur = (r, i)
        bl = self.value(xc - h, tc - h)
        br = self.value(xc + h, tc - h)
        tl = self.value(xc - h, tc + h)

        def lhs(tr):
            dt = (0.5 * (tl + tr) - 0.5 * (bl + br)) / dl          # Eq. (3a)
            dx = (0.5 * (tr + br) - 0.5 * (bl + tl)) / dl          # Eq. (3b)
            av = 0.25 * (tr + br + tl + bl)                        # Eq. (3c)
            return dt + dx + W * av

        rhs = 0.0
        if tc - 2 * a > 0:
            rhs += (G / 2.0) * self.square(xc - 2 * a, tc - 2 * a)
        s1 = (self.bar(-xc - 2 * a, tc - xc - a) - self.bar(-xc, tc - xc - a)) \
            if (xc + a > 0 and self.step(tc - xc - a, tol)) else 0.0
        s2 = (self.bar(2 * a - xc, tc - xc + a) - self.bar(-xc, tc - xc + a)) \
            if (xc - a > 0 and self.step(tc - xc + a, tol)) else 0.0
        rhs -= (G / 2.0) * (s1 + s2)
        rhs += math.sqrt(G) * (self.chi0(xc - tc, -a - tc) - self.chi0(xc - tc, a - tc))
        b0 = lhs(0.0)
        a1 = lhs(1.0) - b0
        return (rhs - b0) / a1

    def run(self, rows: int | None = None):
        rows = self.Nt if rows is None else rows
        for r in range(self.done_row + 1, rows + 1):
            for i in range(self.lo, self.Nx + 1):
                self.psi[r, i - self.lo] = self.solve(i, r)
            self.done_row = r
        self.cur = (self.done_row + 1, -10**9)
        return self

    # ---- readouts --------------------------------------------------------
    def at(self, i: int, r: int) -> complex:
        """psi at column i, row r (exact left of the marched region)."""
        if r < 0:
            return 0.0
        if i < self.lo:
            return self.exact(i, r)
        return self.psi[r, i - self.lo]

    def chi(self, x1: float, x2: float, t: float, half_step: bool = False) -> complex:
        """chi(x1, x2, t) by Eq. (2); half_step=True takes theta(0) = 1/2 on the
        lines x = -a and x = a (for quadratures over the plane)."""
        a, G = self.a, self.G
        tol = 1e-6 * self.dl

        def th(y):
            if half_step and abs(y) <= tol:
                return 0.5
            return 1.0 if y > tol else 0.0

        def ps(x, s):
            if s < -tol:
                return 0.0
            return self.at(self.col(x), self.row(s))

        def part(u, v):
            out = 0.0
            if th(v + a) and t - v - a > -tol:
                out += th(v + a) * ps(u - v - a, t - v - a)
            if th(v - a) and t - v + a > -tol:
                out -= th(v - a) * ps(u - v + a, t - v + a)
            return out

        return self.chi0(x1 - t, x2 - t) - math.sqrt(G) / 2.0 * (part(x1, x2) + part(x2, x1))

    def exact_mass(self, r: int, x_edge: float, depth: float) -> float:
        """int_{x_edge - depth}^{x_edge} |psi_exact(x, t_r)|^2 dx by composite
        20-point Gauss-Legendre (for states without a closed form at hand)."""
        t = r * self.dl
        xg, wg = np.polynomial.legendre.leggauss(20)
        edges = np.linspace(x_edge - depth, x_edge, 401)
        tot = 0.0
        for u, v in zip(edges[:-1], edges[1:]):
            for xq, wq in zip(0.5 * (u + v) + 0.5 * (v - u) * xg, wg):
                y = xq - t
                val = self.c_ex * (self.phi(y) * self.E2[r] + self.phi2(y) * self.E[r])
                tot += 0.5 * (v - u) * wq * abs(val) ** 2
        return tot

    def pe(self, r: int, phi_mass_below) -> float:
        """int |psi(x, t_r)|^2 dx: the exact part left of the marched columns in
        closed form (|c E|^2 times the packet's mass), plus the trapezoid rule
        over the columns from the first marched one's left neighbour to Nx.
        Two different photons: phi_mass_below is the depth of the quadrature
        of the exact part instead (see exact_mass)."""
        t = r * self.dl
        x_edge = -self.a + (self.lo - 1) * self.dl
        if self.phi2 is not None:
            ex = self.exact_mass(r, x_edge, float(phi_mass_below))
        else:
            ex = abs(self.c_ex * self.E[r]) ** 2 * phi_mass_below(x_edge - t)
        vals = [self.at(i, r) for i in range(self.lo - 1, self.Nx + 1)]
        m2 = np.abs(np.asarray(vals)) ** 2
        return ex + self.dl * (m2.sum() - 0.5 * m2[0] - 0.5 * m2[-1])
