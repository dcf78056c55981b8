"""Pins of the oracle's march with the paper's own reads (march_diag): the
columns x <= -a are marched too and every read of a marched point takes the
marched value, as the paper's program does (Sec. 3); only points left of the
marched columns take the exact solution (the paper's boundary region).

* It equals the literal micro-oracle's paper_diag mode cell for cell on small
  grids (Eq. 1 term by term, no shared code), for the one-packet families
  including stimulated emission (whose row 0 is non-zero left of -a).
* Its P_e is the exact part below -a plus the trapezoid over columns 0..Nx
  of the marched values (column 0 included).
* The paper's test 1: in x <= -a the marched values converge to the exact
  solution c phi(x - t) E(t) at second order (the scheme is O(Delta^2),
  Sec. 3).
* Right of -a both read modes solve the same equation: their difference
  shrinks at second order too.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.micro import Micro
from paper_1707_05943_amd import workloads as W


def _inst(incident, **kw):
    base = dict(name="diag", Nx=24, D=6, Nt=40, Delta=0.05, omega0=2.0, Gamma=1.0, incident=incident, k=2.3,
                alpha=0.8, phase=0.4)
    base.update(kw)
    if incident == W.INC_GAUSS2:
        a = 0.5 * base["D"] * base["Delta"]
        base.update(width=0.3, x0=-a - 1.2, k=1.7)
    return W.Instance(**base)


FAMILIES = {"exp2": _inst(W.INC_EXP2), "gauss2": _inst(W.INC_GAUSS2), "plane": _inst(W.INC_PLANE, k=1.9),
            "exp1": _inst(W.INC_EXP1, alpha=0.6)}


@pytest.mark.parametrize("name", list(FAMILIES))
def test_equals_the_micro_oracle(name):
    inst = FAMILIES[name]
    dc = 11
    E = oracle.E_table(inst)
    rows = [0, 7, 23, inst.Nt]
    res = oracle.march_diag(inst, dc, E, snap_rows=rows)
    phi = lambda x: complex(oracle.phi(inst, x)[0])
    m = Micro(inst, E, phi, mode="paper_diag", diag_cols=dc)
    # row 0 of the micro-oracle: the exact solution in x <= -a
    for i in range(m.lo, 1):
        m.psi[0, i - m.lo] = m.exact(i, 0)
    m.run()
    assert res["lo"] == m.lo
    for q, r in enumerate(rows):
        b = np.array([m.at(i, r) for i in range(m.lo, inst.Nx + 1)])
        scale = max(np.linalg.norm(b), 1e-3)
        assert np.linalg.norm(res["snaps"][q] - b) <= 1e-13 * scale, (name, r)
    if name == "exp1":
        assert np.abs(res["snaps"][0][: 1 - m.lo]).max() > 0.1     # the excited emitter's row 0 is not zero
    if name == "plane":
        return                                   # the plane wave has no finite P_e
    # P_e: exact part below -a and the trapezoid over columns 0..Nx, column 0 marched
    ex = oracle.exact_part(inst, E)
    for r in (3, 19, inst.Nt):
        v = np.abs(np.array([m.at(i, r) for i in range(0, inst.Nx + 1)])) ** 2
        want = ex[r] + inst.Delta * (v.sum() - 0.5 * v[0] - 0.5 * v[-1])
        assert abs(res["pe"][r] - want) <= 1e-13 * max(1.0, want), (name, r)


def _test1(D, T=4.0, L=5.0, two_a=2.0, incident=W.INC_PLANE):
    """max |marched - exact| over x in [-a - L, -a] at t = T, and the largest
    |difference| of the two read modes right of -a, on the grid Delta = 2a/D"""
    dl = two_a / D
    Nt = int(round(T / dl))
    dc = int(round(L / dl)) + 1
    inst = W.Instance(name="t1", Nx=D + 2, D=D, Nt=Nt, Delta=dl, omega0=math.pi / 2, Gamma=math.pi / 4,
                      incident=incident, k=math.pi / 2, alpha=0.7, phase=0.0)
    E = oracle.E_table(inst)
    res = oracle.march_diag(inst, dc, E, snap_rows=[Nt])
    lo = res["lo"]
    cols = np.arange(lo, 1)
    phi = oracle.phi(inst, -inst.a + (cols - Nt) * dl)
    c_ex = math.sqrt(2.0) if incident != W.INC_EXP1 else 1.0
    exact = c_ex * phi * E[Nt]
    got = res["snaps"][0][: 1 - lo]
    e_left = np.abs(got - exact).max() / np.abs(exact).max()
    hyb = oracle.march(inst, E, snap_rows=[Nt], want_ring=False, want_pe=False)["snaps"][0]
    e_right = np.abs(res["snaps"][0][1 - lo:] - hyb[1:]).max() / np.abs(hyb).max()
    return e_left, e_right


@pytest.mark.parametrize("incident", [W.INC_PLANE, W.INC_EXP2])
def test_paper_test1_second_order(incident):
    errs = [_test1(D, incident=incident) for D in (20, 40, 80)]
    left = [e[0] for e in errs]
    right = [e[1] for e in errs]
    assert left[0] / left[1] > 3.3 and left[1] / left[2] > 3.5, left
    assert right[0] / right[1] > 3.0 and right[1] / right[2] > 3.3, right
    assert left[2] < 3e-3 and right[2] < 3e-3, (left, right)
