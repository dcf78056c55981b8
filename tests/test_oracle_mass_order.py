"""Pins of the oracle's exact part of P_e, its grid E table, the scheme's
order under grid refinement and its amplification factor.

* The mass of the packet below y, int_{-inf}^{y} |phi|^2 (the exact part of
  P_e: App. D's trapezoid over the box plus this closed form for x <= -a), against composite
  Gauss-Legendre quadrature of |phi|^2 at points across the packet, for the
  Gaussian and the exponential packet of Eq. (7).  A wrong scale of the
  Gaussian's erf argument (w or 2w instead of sqrt(2) w) moves the value at
  y = x0 + w by more than 0.05.
* E on the grid (the delay series assembled from J_n at T = q Delta, each
  value serving two rows) against the same series evaluated row by row, and
  against the closed forms of Eqs. (6), (9) and (13).
* P9: P_e(t) and chi of Eq. (2) under grid refinement (Delta, Delta/2,
  Delta/4 at fixed physical parameters): observed order about 2 for the
  Gaussian packet (P_e) and at least 1 where the data are not smooth (the
  exponential packet's front at -a; chi's first detector at a + Delta moves
  with Delta).
* P6: App. A's amplification factor, Eq. (A.1), of the square scheme for
  the free equation d/dt + d/dx + W: the literal micro-oracle (Eq. 1 term by
  term) advances a Fourier mode by exactly that factor, whose modulus is at
  most 1 for Re W > 0 and equals 1 at k Delta = pi.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.micro import Micro
from paper_1707_05943_amd import workloads as W


def _gl_mass(inst, y, lo, panels=400):
    """int_lo^y |phi(x)|^2 dx by composite 20-point Gauss-Legendre."""
    xg, wg = np.polynomial.legendre.leggauss(20)
    edges = np.linspace(lo, y, panels + 1)
    tot = 0.0
    for u, v in zip(edges[:-1], edges[1:]):
        x = 0.5 * (u + v) + 0.5 * (v - u) * xg
        tot += 0.5 * (v - u) * float(np.sum(wg * np.abs(oracle.phi(inst, x)) ** 2))
    return tot


def _gauss_inst(width=0.7, D=20, Delta=0.05):
    inst = W.tiny_gauss(D=D, Nx=40, Nt=40, Delta=Delta, width=width, seed=4)
    inst.x0 = -inst.a - 3.0 * width
    return inst


def test_gaussian_mass_below_against_quadrature():
    inst = _gauss_inst()
    w, x0, a = inst.width, inst.x0, inst.a
    ys = [x0 - 3 * w, x0 - w, x0 - 0.3 * w, x0, x0 + w, x0 + 2 * w, -a]
    got = oracle.phi_mass_below(inst, ys)
    for y, g in zip(ys, got):
        ref = _gl_mass(inst, y, x0 - 14 * w)
        assert abs(g - ref) < 1e-13, (y, g, ref)
    # the packet is normalised over the real line (its mass beyond -a is e^{-4.5}-small
    # here, and the mass below +inf equals 1 with the truncation lifted)
    assert abs(_gl_mass(inst, -a, x0 - 14 * w) + 0.5 * math.erfc(3.0 / math.sqrt(2.0)) - 1.0) < 1e-13
    # a scale of w or 2 w in the erf argument would miss the quadrature by > 0.05 one width
    # from the centre (the bound above is 1e-13)
    ref = _gl_mass(inst, x0 + w, x0 - 14 * w)
    for wrong in (w, 2 * w):
        assert abs(0.5 * math.erfc((x0 - (x0 + w)) / wrong) - ref) > 0.05


@pytest.mark.parametrize("alpha,k", [(0.5, 2.0), (1.7, -1.3)])
def test_exponential_mass_below_against_quadrature(alpha, k):
    inst = W.Instance(name="m", Nx=10, D=8, Nt=10, Delta=0.05, omega0=2.0, Gamma=1.3,
                      incident=W.INC_EXP2, k=k, alpha=alpha)
    a = inst.a
    dec = alpha * inst.Gamma
    ys = [-a, -a - 0.1 / dec, -a - 1.0 / dec, -a - 3.0 / dec]
    got = oracle.phi_mass_below(inst, ys)
    for y, g in zip(ys, got):
        ref = _gl_mass(inst, y, y - 60.0 / dec, panels=600)
        assert abs(g - ref) < 1e-13, (y, g, ref)
    assert abs(got[0] - 1.0) < 1e-15          # Eq. (7) is normalised on x <= -a


def _einst(incident, **kw):
    base = dict(name="e", Nx=10, D=20, Nt=160, Delta=0.05, omega0=3.0, Gamma=1.0, incident=incident,
                k=2.5, alpha=0.0, x0=0.0, width=1.0, phase=0.0)
    base.update(kw)
    return W.Instance(**base)


E_CASES = {
    "plane": _einst(W.INC_PLANE, k=2.5),
    "exp2": _einst(W.INC_EXP2, alpha=0.7),
    "exp2_re_z_neg": _einst(W.INC_EXP2, alpha=1.6, k=3.0),
    "exp1": _einst(W.INC_EXP1, alpha=0.5),
    "gauss": W.tiny_gauss(D=20, Nx=10, Nt=160, Delta=0.05, width=0.6),
}
E_CASES["gauss"].x0 = -E_CASES["gauss"].a - 4 * 0.6


@pytest.mark.parametrize("name", list(E_CASES))
def test_E_on_the_grid_equals_E_row_by_row(name):
    inst = E_CASES[name]
    grid = oracle.E_table(inst, mode=1)
    rows = oracle.E_table(inst, mode=2)
    scale = max(1.0, float(np.max(np.abs(rows))))
    assert np.max(np.abs(grid - rows)) < 1e-14 * scale
    if inst.incident != W.INC_GAUSS2:
        # against the closed forms (Eqs. 6, 9, 13 times e^{-ika}) at every row
        closed = oracle.E_table(inst, mode=0)
        assert np.max(np.abs(grid - closed)) < 1e-12 * scale
    assert np.max(np.abs(rows)) > 0.05                   # a non-trivial table


def _refine_case(incident, D):
    """The same physical problem on grid step 0.5/D (2a = 0.5, T = 4, box 5)."""
    dl = 0.5 / D
    if incident == W.INC_GAUSS2:
        inst = W.tiny_gauss(D=D, Nx=int(round(5.0 / dl)), Nt=int(round(4.0 / dl)), Delta=dl, width=0.5,
                            seed=8, k0a=0.5 * math.pi)
        inst.x0 = -inst.a - 4.0 * inst.width
        return inst
    return W.Instance(name=f"exp_{D}", Nx=int(round(5.0 / dl)), D=D, Nt=int(round(4.0 / dl)), Delta=dl,
                      omega0=2 * math.pi, Gamma=1.0, incident=W.INC_EXP2, k=2 * math.pi, alpha=0.8)


def _observed_order(incident):
    pes, chis = [], []
    n_tau = 9
    for D in (10, 20, 40):
        inst = _refine_case(incident, D)
        res = oracle.march(inst, oracle.E_table(inst), chi_rows=[inst.Nt], n_tau=(n_tau - 1) * D // 10 + 1,
                           want_ring=False)
        stride = D // 10
        pes.append(res["pe"][::stride])                  # t = 0, 0.05, ..., 4 on every grid
        chis.append(res["chi"][0][::stride])             # tau = 0, 0.05, ..., 0.4 at t = 4
    e1 = np.max(np.abs(pes[0] - pes[1]))
    e2 = np.max(np.abs(pes[1] - pes[2]))
    c1 = np.max(np.abs(chis[0] - chis[1]))
    c2 = np.max(np.abs(chis[1] - chis[2]))
    return math.log2(e1 / e2), math.log2(c1 / c2), pes, chis


def test_refinement_order_gaussian():
    p_pe, p_chi, pes, chis = _observed_order(W.INC_GAUSS2)
    assert np.max(pes[2]) > 0.05 and np.max(np.abs(chis[2])) > 0.01     # a non-trivial signal
    assert 1.7 < p_pe < 2.4, p_pe
    assert p_chi > 0.9, p_chi


def test_refinement_order_exponential_front():
    p_pe, p_chi, pes, _ = _observed_order(W.INC_EXP2)
    assert np.max(pes[2]) > 0.05
    assert p_pe > 0.9, p_pe
    assert p_chi > 0.9, p_chi


def _xi_A1(kd, Wc, dl):
    e = np.exp(1j * kd)
    return ((1 / dl - Wc / 4) - (Wc / 4) * e) / ((1 / dl + Wc / 4) + (Wc / 4) / e) / e


@pytest.mark.parametrize("omega0,Gamma,dl", [(2.0, 1.0, 0.05), (30.0, 0.2, 0.01), (0.0, 5.0, 0.1)])
def test_amplification_factor_of_the_micro_oracle(omega0, Gamma, dl):
    """Row 0 set to e^{i k x}; before the delay (t < 2a) and right of the
    mirror's light cone the march is the free scheme, so each row multiplies
    the mode by xi(k) of Eq. (A.1)."""
    D, Nx = 40, 110
    inst = W.Instance(name="xi", Nx=Nx, D=D, Nt=3, Delta=dl, omega0=omega0, Gamma=Gamma,
                      incident=W.INC_GAUSS2, width=1.0, x0=-1e9)
    Wc = 1j * omega0 + Gamma / 2
    for kd in (0.3, 1.1, 2.0, 2.9, math.pi):
        m = Micro(inst, np.zeros(inst.Nt + 1, complex), lambda x: 0.0)
        x = -inst.a + dl * np.arange(1, Nx + 1)
        m.psi[0, :] = np.exp(1j * (kd / dl) * x)
        m.run()
        # columns j >= D + 15: right of the mirror's light cone x = a + t (source 2 is off) by
        # more than the recurrence's reach; psi[r, i] holds column i + 1
        cols = slice(D + 14, Nx)
        ratio = m.psi[3, cols] / m.psi[2, cols]
        xi = _xi_A1(kd, Wc, dl)
        assert np.max(np.abs(ratio - xi)) < 1e-12, (kd, ratio[:3], xi)
        assert abs(xi) <= 1.0 + 1e-15
        if kd == math.pi:
            assert abs(abs(xi) - 1.0) < 1e-14          # the grid-scale mode is not damped
    # |xi| <= 1 over the whole band for Re W > 0 (App. A)
    ks = np.linspace(-math.pi, math.pi, 2001)
    assert np.max(np.abs(_xi_A1(ks, Wc, dl))) <= 1.0 + 1e-14
