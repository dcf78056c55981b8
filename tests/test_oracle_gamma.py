"""Pins of the oracle's P(n, z) = gamma(n, z)/(n-1)! (App. C).

* against mpmath's lower incomplete gamma at 40 digits, over the regimes the
  paper's map distinguishes (its Fig. 9 is missing; the oracle's split is
  series |z| < n+1, continued fraction beyond, and the gamma-star series or
  the Poincare-type sum next to the negative real axis);
* against the power series sum_j (-1)^j z^{n+j} / (j! (n+j)) summed in exact
  rational arithmetic on tiny inputs, with a rigorous tail bound;
* against the recurrence gamma(n+1, z) = n gamma(n, z) - z^n e^{-z}.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

mp = pytest.importorskip("mpmath")


def _mp_P(n, z):
    """P(n, z) for integer n from its definition 1 - e^{-z} sum_{k<n} z^k/k!,
    in enough decimal digits to absorb the cancellation (mpmath's own
    gammainc recurses without end on part of this grid)."""
    az = abs(z)
    digits = 40 + int(n * max(0.0, math.log10(max(1.0, n) / max(az, 1e-300)))) + int(az / 2.0)
    with mp.workdps(digits):
        zz = mp.mpc(z.real, z.imag)
        s = mp.mpf(0)
        term = mp.mpf(1)
        for k in range(n):
            if k:
                term = term * zz / k
            s += term
        return complex(1 - mp.exp(-zz) * s)


GRID = []
for n in (1, 2, 3, 5, 8, 13, 21, 40, 100):
    for mod in (1e-3, 0.3, 1.0, 3.0, 10.0, 30.0, 100.0, 300.0):
        for ang in (0.0, 0.5 * math.pi, -0.5 * math.pi, 0.75 * math.pi, -0.75 * math.pi, 0.25 * math.pi,
                    math.pi, math.pi - 1e-13, -math.pi + 1e-13):
            z = mod * complex(math.cos(ang), math.sin(ang))
            GRID.append((n, z))


def test_gamma_against_mpmath():
    ns = np.array([g[0] for g in GRID], np.int32)
    zs = np.array([g[1] for g in GRID], np.complex128)
    vals, reg, ok = oracle.gamma_P(ns, zs)
    worst = 0.0
    seen = set()
    for (n, z), v, r, c in zip(GRID, vals, reg, ok):
        ref = _mp_P(n, z)
        if not np.isfinite(ref.real) or abs(ref) > 1e300:
            continue
        if abs(ref) < 1e-280:          # below double range: only require a tiny result
            assert abs(v) < 1e-270, (n, z, v)
            continue
        assert c == 1, (n, z)
        seen.add(int(r))
        # relative to the size of the result or of the 1 in P = 1 - Q,
        # whichever is larger (the regimes computing 1 - Q lose relative
        # accuracy where P is tiny against 1)
        scale = max(abs(ref), 1.0) if r in (1, 4) else abs(ref)
        err = abs(v - ref) / scale
        worst = max(worst, err)
        assert err < 5e-13, (n, z, r, v, ref)
    assert seen == {1, 2, 3, 4}, f"every regime must be exercised, saw {seen}"
    assert worst < 5e-13


def test_each_regime_agrees_where_valid():
    # (b) and (c) are both convergent series: they agree for small |z|
    n = np.array([1, 2, 4, 7], np.int32)
    z = np.array([0.3 + 0.2j, -1.5 + 0.5j, 2.0 - 1.0j, -0.7 + 0j])
    b = oracle.gamma_P_regime(n, z, 2)
    c = oracle.gamma_P_regime(n, z, 3)
    assert np.max(np.abs(b - c) / np.abs(b)) < 1e-14
    # (d) + its exact 1 equals (c) on the negative axis for integer n
    n = np.array([1, 3, 6, 10], np.int32)
    z = np.array([-2.0, -8.0, -25.0, -40.0], np.complex128)
    c = oracle.gamma_P_regime(n, z, 3)
    d = oracle.gamma_P_regime(n, z, 4)
    assert np.max(np.abs(c - d) / np.abs(c)) < 1e-12


def _exact_gamma_series(n, zr: Fraction, zi: Fraction, terms: int):
    """sum_{j<terms} (-1)^j z^{n+j} / (j! (n+j)) in exact rationals, plus a
    bound on the tail."""
    # complex power by repeated multiplication
    pr, pi_ = Fraction(1), Fraction(0)
    for _ in range(n):
        pr, pi_ = pr * zr - pi_ * zi, pr * zi + pi_ * zr
    sr, si = Fraction(0), Fraction(0)
    fact = 1
    for j in range(terms):
        if j > 0:
            fact *= j
        sgn = -1 if j % 2 else 1
        den = fact * (n + j)
        sr += sgn * pr / den
        si += sgn * pi_ / den
        pr, pi_ = pr * zr - pi_ * zi, pr * zi + pi_ * zr
    az = math.hypot(float(zr), float(zi))
    tail = az ** (n + terms) / (math.factorial(terms) * (n + terms)) / (1 - az / (terms + 1))
    return complex(float(sr), float(si)), tail


@pytest.mark.parametrize("n", [1, 2, 3, 5])
@pytest.mark.parametrize("zz", [(Fraction(1, 2), Fraction(1, 3)), (Fraction(-3, 2), Fraction(1, 4)),
                                (Fraction(2), Fraction(-1)), (Fraction(-1), Fraction(0)),
                                (Fraction(1, 8), Fraction(7, 4))])
def test_gamma_exact_rational_series(n, zz):
    zr, zi = zz
    ref, tail = _exact_gamma_series(n, zr, zi, 60)
    assert tail < 1e-30
    v, reg, ok = oracle.gamma_P(n, complex(float(zr), float(zi)))
    g = v[0] * math.factorial(n - 1)
    assert abs(g - ref) <= 2e-15 * max(abs(ref), 1e-3) + tail


def test_gamma_recurrence():
    rng = np.random.default_rng(7)
    for _ in range(200):
        n = int(rng.integers(1, 60))
        z = complex(rng.uniform(-40, 80), rng.uniform(-80, 80))
        if z.real < 0 and abs(z) > 30:
            continue
        v1 = oracle.gamma_P(n, z)[0][0] * math.gamma(n)
        v2 = oracle.gamma_P(n + 1, z)[0][0] * math.gamma(n + 1)
        rhs = n * v1 - np.exp(n * np.log(z) - z)
        scale = max(abs(v2), abs(n * v1), abs(np.exp(n * np.log(z) - z)))
        assert abs(v2 - rhs) <= 1e-12 * scale, (n, z)
