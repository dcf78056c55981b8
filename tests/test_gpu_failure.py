"""Failure detection of the march, forced from the host.

* Read-before-write: after the boundary is set, every ring slot except row
  0's and every entry of the strip's diagonal copy except row 0's is filled
  with NaN (rows before t = 0 are never read from memory: their terms are
  dropped by the row tests).  A read of any value before the march has
  written it would carry a NaN into the compared rows; the march must match
  the oracle as with a cleared workspace, and report no non-finite value.
* Non-finite values: a NaN planted in row 0 (the initial condition) spreads
  through the march; fdtd_sync and readouts into host memory report
  FDTD_ERANGE, and a new boundary clears the report.
Every kernel runs to its normal end in both cases.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1707_05943_amd import fdtd
from paper_1707_05943_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12
FLOOR = 0.01


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gauss(D, Nx, Nt, Delta, width, seed, x0w=6.0, k0a=0.5 * math.pi):
    inst = W.tiny_gauss(D=D, Nx=Nx, Nt=Nt, Delta=Delta, width=width, seed=seed, k0a=k0a)
    inst.x0 = -inst.a - x0w * width
    return inst


CASES = {
    "gauss_D10_Nx2600": _gauss(10, 2600, 300, 0.02, 0.5, 11),
    "gauss_D1200_Nx3100": _gauss(1200, 3100, 2600, 0.0025, 0.5, 14),   # several strip workgroups and the cone
    "exp1_D24": W.Instance(name="exp1_D24", Nx=1500, D=24, Nt=400, Delta=0.02, omega0=2.0, Gamma=1.5,
                           incident=W.INC_EXP1, k=2.3, alpha=0.5),
}


def _views(sol, inst):
    """the ring (R x (Nx+1)) and the diagonal copy (R x (D+1)) inside the
    solver's workspace, as float64 pairs (the workspace's first two buffers)"""
    import torch
    R = fdtd.describe(inst)["ring_rows"]
    C = inst.Nx + 1
    ring_bytes = R * C * 16
    md_off = (ring_bytes + 255) // 256 * 256
    ring = sol.ws[:ring_bytes].view(torch.float64).view(R, C, 2)
    md = sol.ws[md_off:md_off + R * (inst.D + 1) * 16].view(torch.float64).view(R, inst.D + 1, 2)
    return R, ring, md


@pytest.mark.parametrize("name", list(CASES))
def test_poisoned_workspace_gives_the_same_march(name):
    import torch
    inst = CASES[name]
    _say(f"[failure] poisoned ring and diagonal copy: {name}")
    E = oracle.E_table(inst)
    pre = oracle.march(inst, E, want_ring=False)["pe"]
    peak = max(1, int(np.argmax(pre)))
    rows = sorted({inst.Nt // 3, peak, inst.Nt})
    ref = oracle.march(inst, E, snap_rows=rows)
    sol = fdtd.Solver(inst).set_boundary(E)
    R, ring, md = _views(sol, inst)
    ring[1:] = float("nan")                      # row 0 sits in slot 0
    md[:] = float("nan")
    c = torch.arange(1, inst.D + 1, device=md.device)
    md[inst.D - c, c] = 0.0                      # psi(c, 0) = 0 at row D - c of the copy
    torch.cuda.synchronize()
    scale = max(np.linalg.norm(v) for v in ref["snaps"])
    for q, r in enumerate(rows):
        sol.march(r - sol.row)
        got = sol.row_values(r)
        e = np.linalg.norm(got - ref["snaps"][q]) / max(np.linalg.norm(ref["snaps"][q]), FLOOR * scale)
        assert np.isfinite(got).all() and e <= TOL, (name, r, e)
    sol.sync()                                   # no non-finite value reported
    e = np.linalg.norm(sol.pe() - ref["pe"]) / np.linalg.norm(ref["pe"])
    assert e <= TOL, e
    if inst.incident == W.INC_EXP1:
        assert np.isfinite(sol.mu()).all() and np.isfinite(sol.lam()).all()
    sol.close()


def test_nan_in_the_march_is_reported():
    import torch
    inst = CASES["gauss_D10_Nx2600"]
    _say("[failure] NaN planted in row 0")
    sol = fdtd.Solver(inst).set_boundary()
    R, ring, md = _views(sol, inst)
    ring[0, 1500, 0] = float("nan")             # psi(1500, 0): the initial condition
    torch.cuda.synchronize()
    sol.march(inst.Nt)
    with pytest.raises(fdtd.FdtdError) as e:
        sol.sync()
    assert e.value.code == -5 and "non-finite" in str(e.value)
    with pytest.raises(fdtd.FdtdError) as e:
        sol.pe()
    assert e.value.code == -5
    # a new boundary (which also rewrites row 0) clears the report
    sol.set_boundary()
    sol.march(inst.Nt)
    sol.sync()
    assert np.isfinite(sol.pe()).all()
    sol.close()
