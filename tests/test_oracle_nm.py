"""Pins of the oracle's non-Markovian measures (App. D): the photon field of
the one-excitation problem conserves that problem's probability, mu at t = 0
is the quadrature of |phi_in|^2 e1(0), and without coupling mu(t) is the free
phase e^{-i omega0 t} and lambda(t) the total probability."""
import dataclasses

import numpy as np
import pytest

from oracle import nm
from paper_1707_05943_amd import workloads as W


def _inst(Delta, Gamma=1.5, alpha=0.5, T=12.0, L=30.0):
    D = int(round(0.48 / Delta))
    D += D % 2
    return W.Instance(name="nm", Nx=int(round(L / Delta)), D=D, Nt=int(round(T / Delta)), Delta=Delta,
                      omega0=2.0, Gamma=Gamma, incident=W.INC_EXP1, k=2.3, alpha=alpha)


def test_one_excitation_probability_is_conserved():
    """int |phi(x,t)|^2 dx + |e0(t)|^2 = 1 up to the trapezoid rule's O(Delta)
    error at the field's jumps (x = -a, x = +a): a wrong sign of either
    emission term breaks it by O(1)."""
    errs = []
    for dl in (0.02, 0.01):
        inst = _inst(dl)
        e0 = nm.e0_table(inst)
        err = max(abs(nm.one_excitation_norm(inst, e0, r) - 1.0) for r in range(0, inst.Nt + 1, inst.Nt // 6))
        assert err <= 0.6 * dl, (dl, err)
        errs.append(err)
    assert errs[1] < 0.6 * errs[0]


def test_mu_and_lambda_at_t0():
    """At t = 0 psi = phi = phi_in (in x <= -a), so mu(0) is the exact mass 1
    plus the trapezoid's endpoint term Delta/2 |phi_in(-a)|^2 = Delta alpha G / 2
    (e1(0) = 1), and lambda(0) = P_e(0) since e0(0) = 0."""
    inst = _inst(0.02, T=2.0)
    m = nm.measures(inst, [0, 5])
    assert abs(m["mu"][0] - (1.0 + 0.5 * inst.Delta * inst.alpha * inst.Gamma)) <= 1e-13
    assert abs(m["e0"][0]) <= 1e-15
    assert abs(m["lambda"][0] - m["pe"][0]) <= 1e-15


@pytest.mark.parametrize("dl,bound", [(0.02, 0.05), (0.01, 0.02)])
def test_uncoupled_limit(dl, bound):
    """Gamma -> 0 (alpha Gamma fixed): the packet moves freely with the
    emitter's phase, psi = phi_in(x-t) e^{-i omega0 t} and phi = phi_in(x-t),
    so mu(t) e^{i omega0 t} -> 1 and lambda(t) -> 1, to the scheme's
    discretisation error (which shrinks with Delta)."""
    inst = _inst(dl, Gamma=1e-5, alpha=1e5)
    rows = [inst.Nt // 3, inst.Nt]
    m = nm.measures(inst, rows)
    for mu, r in zip(m["mu"], m["rows"]):
        assert abs(mu * np.exp(1j * inst.omega0 * r * inst.Delta) - 1.0) <= bound
    assert np.all(np.abs(m["lambda"] - 1.0) <= bound)


def test_n_geo_of_closed_forms():
    """N_geo is the integral of the positive part of d|det|/dt: zero for a
    decaying |det|, the total rise for |det| = |cos t| on [0, 2 pi] (two rises
    of 1), and for det = e^{-t} (1 + 0.5 sin 3t) the sum of the rises of the
    continuous function between its critical points, to the sampling error."""
    t = np.linspace(0.0, 2.0 * np.pi, 20001)
    assert nm.n_geo(np.exp(-0.25 * t), np.ones_like(t)) == 0.0
    assert abs(nm.n_geo(np.ones_like(t), np.cos(t)) - 2.0) <= 1e-12
    # |mu|^2 lambda with mu = e^{-t/2} e^{i t}, lambda = 1 + 0.5 sin 3t
    f = lambda x: np.exp(-x) * (1.0 + 0.5 * np.sin(3.0 * x))
    mu = np.exp(-0.5 * t + 1j * t)
    got = nm.n_geo(mu, 1.0 + 0.5 * np.sin(3.0 * t))
    # critical points: f' = e^{-x} (1.5 cos 3x - 1 - 0.5 sin 3x) = 0
    from scipy.optimize import brentq
    g = lambda x: 1.5 * np.cos(3.0 * x) - 1.0 - 0.5 * np.sin(3.0 * x)
    xs = np.linspace(0.0, 2.0 * np.pi, 4001)
    crit = [brentq(g, a, b) for a, b in zip(xs[:-1], xs[1:]) if g(a) * g(b) < 0]
    pts = np.concatenate(([0.0], crit, [2.0 * np.pi]))
    ref = sum(max(0.0, f(b) - f(a)) for a, b in zip(pts[:-1], pts[1:]))
    assert ref > 0.05
    assert abs(got - ref) <= 2e-7       # extrema missed by the samples: O(h^2 f'') each
