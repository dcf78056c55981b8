"""Pins of the oracle's two-photon exponential family with different photons
(Sec. 2 case (c): photon i is the packet of Eq. (7) with (k_i, alpha_i)).

* The incident state chi(x1, x2, 0) = (A/sqrt 2)[phi1(x1) phi2(x2) +
  phi1(x2) phi2(x1)] with A of Eq. (11) has unit norm (2-D Gauss-Legendre
  quadrature over x1, x2 <= -a) and is symmetric.
* With k1 = k2 and alpha1 = alpha2 the family reduces to identical photons
  (Eq. 12 becomes sqrt 2 phi(x-t) e0(t)): the march, P_e and chi equal the
  identical-photon path's.
* Exchanging the photons leaves every output unchanged.
* The C oracle equals the literal micro-oracle (Eq. 1 term by term, its own
  A and a quadrature of the exact part of P_e) on a small grid.
* The paper's test 1 for this family: with the columns left of -a marched
  as well (the micro-oracle's reads of its own values), Eq. (1) itself
  converges there to Eq. (12)'s psi = A [phi1(x-t) e0^(2) + phi2(x-t) e0^(1)]
  at second order.  (Pairing each packet with its own e0 instead leaves an
  error of 0.3 that does not shrink: checked on the CPU.)
* Total probability int |psi|^2 + iint |chi|^2 (chi from Eq. 2) tends to 1
  as Delta -> 0 (first order: the packets' fronts at -a are jumps).
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle.micro import Micro
from paper_1707_05943_amd import workloads as W


def _two(**kw):
    base = dict(name="two", Nx=60, D=8, Nt=100, Delta=0.05, omega0=2.0, Gamma=1.0, incident=W.INC_EXP2,
                identical_photons=0, k1=2.3, k2=1.6, alpha1=0.8, alpha2=1.5, phase=0.4)
    base.update(kw)
    return W.Instance(**base)


def test_incident_state_is_normalised_and_symmetric():
    inst = _two(Gamma=1.3, k1=2.9, k2=0.7, alpha1=0.6, alpha2=2.2)
    a = inst.a
    # |phi_i|^2 decays as e^{alpha_i G (x + a)}: cover 45 e-folds of the slower one
    depth = 45.0 / (min(inst.alpha1, inst.alpha2) * inst.Gamma)
    xg, wg = np.polynomial.legendre.leggauss(24)
    edges = np.linspace(-a - depth, -a, 161)
    xs = np.concatenate([0.5 * (u + v) + 0.5 * (v - u) * xg for u, v in zip(edges[:-1], edges[1:])])
    ws = np.concatenate([0.5 * (v - u) * wg for u, v in zip(edges[:-1], edges[1:])])
    X1, X2 = np.meshgrid(xs, xs, indexing="ij")
    c = oracle.chi0(inst, X1.ravel(), X2.ravel()).reshape(X1.shape)
    norm = float(np.einsum("i,j,ij->", ws, ws, np.abs(c) ** 2))
    assert abs(norm - 1.0) < 1e-12, norm
    ct = oracle.chi0(inst, X2.ravel(), X1.ravel()).reshape(X1.shape)
    assert np.max(np.abs(c - ct)) < 1e-15
    # with A = 1 the norm would be 1 + |<phi1|phi2>|^2 instead
    A = oracle.two_photon_A(inst)
    assert A < 0.99 and abs(1.0 / A ** 2 - 1.0) > 1e-3


def _identical_pair(two):
    one = dataclasses.replace(two, identical_photons=1, k=two.k1, alpha=two.alpha1)
    return one


@pytest.mark.parametrize("k,alpha", [(2.3, 0.8), (2.0, 1.6)])
def test_identical_limit(k, alpha):
    two = _two(k1=k, k2=k, alpha1=alpha, alpha2=alpha)
    one = _identical_pair(two)
    E2 = oracle.E_table(two)
    E1 = oracle.E_table(one)
    n = two.Nt + 1
    assert np.max(np.abs(E2[:n] - E1)) == 0.0 and np.max(np.abs(E2[n:] - E1)) == 0.0
    kw = dict(chi_rows=[50, 100], n_tau=20, snap_rows=[30, 70])
    r2 = oracle.march(two, E2, **kw)
    r1 = oracle.march(one, E1, **kw)
    scale = np.abs(r1["ring"]).max()
    assert abs(oracle.two_photon_A(two) - 1.0 / math.sqrt(2.0)) < 1e-15
    assert np.max(np.abs(r2["ring"] - r1["ring"])) < 1e-14 * scale
    assert np.max(np.abs(r2["snaps"] - r1["snaps"])) < 1e-14 * scale
    assert np.max(np.abs(r2["chi"] - r1["chi"])) < 1e-14 * np.abs(r1["chi"]).max()
    assert np.max(np.abs(r2["pe"] - r1["pe"])) < 1e-14


def test_photon_exchange_symmetry():
    two = _two()
    swp = dataclasses.replace(two, k1=two.k2, k2=two.k1, alpha1=two.alpha2, alpha2=two.alpha1)
    kw = dict(chi_rows=[60, 100], n_tau=20, snap_rows=[40])
    a = oracle.march(two, oracle.E_table(two), **kw)
    b = oracle.march(swp, oracle.E_table(swp), **kw)
    scale = np.abs(a["ring"]).max()
    assert scale > 1e-3
    assert np.max(np.abs(a["ring"] - b["ring"])) < 1e-14 * scale
    assert np.max(np.abs(a["chi"] - b["chi"])) < 1e-14 * np.abs(a["chi"]).max()
    assert np.max(np.abs(a["pe"] - b["pe"])) < 1e-14


def _phis(inst):
    p1 = dataclasses.replace(inst, identical_photons=1, k=inst.k1, alpha=inst.alpha1)
    p2 = dataclasses.replace(inst, identical_photons=1, k=inst.k2, alpha=inst.alpha2)
    return (lambda x: complex(oracle.phi(p1, x)[0])), (lambda x: complex(oracle.phi(p2, x)[0]))


def test_c_oracle_equals_literal_micro_oracle():
    inst = _two(Nx=40, D=6, Nt=80)
    E = oracle.E_table(inst)
    n = inst.Nt + 1
    rows = [20, 45, inst.Nt]
    res = oracle.march(inst, E, chi_rows=[40, inst.Nt], n_tau=12, snap_rows=rows)
    f1, f2 = _phis(inst)
    m = Micro(inst, E[:n], f1, phi2=f2, E2=E[n:]).run()
    for q, r in enumerate(rows):
        b = np.array([m.at(i, r) for i in range(0, inst.Nx + 1)])
        assert np.linalg.norm(res["snaps"][q] - b) <= 1e-13 * np.linalg.norm(b), r
    for q, r in enumerate([40, inst.Nt]):
        t = r * inst.Delta
        b = np.array([m.chi(inst.a + inst.Delta, inst.a + (1 + k) * inst.Delta, t) for k in range(12)])
        assert np.linalg.norm(res["chi"][q] - b) <= 1e-13 * np.linalg.norm(b)
    # P_e: the oracle's closed-form exact part (with the cross term of the two
    # packets) against the micro-oracle's quadrature of |psi_exact|^2
    depth = 50.0 / (min(inst.alpha1, inst.alpha2) * inst.Gamma)
    for r in (0, 10, 33, 61, inst.Nt):
        assert abs(res["pe"][r] - m.pe(r, depth)) < 1e-13, r


def test_paper_test1_left_of_minus_a():
    errs = []
    for D in (10, 20, 40):
        dl = 1.0 / D
        Nt = int(round(2.0 / dl))
        inst = _two(Nx=D, D=D, Nt=Nt, Delta=dl, Gamma=1.0, k1=1.0, k2=3.5, alpha1=0.9, alpha2=2.0, omega0=2.5,
                    phase=0.3)
        E = oracle.E_table(inst)
        n = inst.Nt + 1
        f1, f2 = _phis(inst)
        m = Micro(inst, E[:n], f1, phi2=f2, E2=E[n:], mode="paper_diag", diag_cols=Nt).run()
        errs.append(max(abs(m.at(i, Nt) - m.exact(i, Nt)) for i in range(m.lo, 1)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
    assert errs[2] < 2e-3, errs


def _conservation_defect(D):
    """norm0 - int |psi|^2 - iint |chi|^2 at t = 6 on the grid Delta = 1/D (2a = 0.5)"""
    dl = 1.0 / D
    T = 6.0
    Nt = int(round(T / dl))
    inst = _two(Nx=Nt + 4, D=D // 2, Nt=Nt, Delta=dl, Gamma=1.0, k1=2.0, k2=3.1, alpha1=1.6, alpha2=2.4,
                omega0=2.5, phase=0.0)
    E = oracle.E_table(inst)
    n = inst.Nt + 1
    f1, f2 = _phis(inst)
    m = Micro(inst, E[:n], f1, phi2=f2, E2=E[n:]).run()
    t = Nt * dl
    a = inst.a
    # the incoming packets' mass left of -a - 2 is below e^{-1.6 (t + 2)}
    iL = int(math.floor(-2.0 / dl))
    xs = [-a + i * dl for i in range(iL, Nt + 3)]
    nn = len(xs)
    chi = np.zeros((nn, nn), complex)
    for p_, x1 in enumerate(xs):
        for q in range(p_, nn):
            chi[p_, q] = chi[q, p_] = m.chi(x1, xs[q], t, half_step=True)
    w = np.ones(nn)
    w[0] = w[-1] = 0.5
    chi2 = dl * dl * np.einsum("i,j,ij->", w, w, np.abs(chi) ** 2)
    pe = m.pe(Nt, 40.0)
    return 1.0 - pe - chi2


def test_two_excitation_probability_converges():
    d = [_conservation_defect(D) for D in (8, 16, 32)]
    assert abs(d[0]) / abs(d[1]) > 1.8 and abs(d[1]) / abs(d[2]) > 1.8, d
    assert abs(d[2]) < 0.1, d
