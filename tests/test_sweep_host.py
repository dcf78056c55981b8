"""Host-side logic of the sweep pipeline (no GPU): target plans, the coarse
grids of the a-posteriori check, the P_e window."""
import math

import numpy as np

from paper_1707_05943_amd import sweep as SW
from paper_1707_05943_amd import workloads as W


def test_chi_plan_is_inside_the_grid():
    for inst in W.sweep_draw(64, 3):
        row, stride = SW.chi_plan(inst)
        assert 1 <= row <= inst.Nt and stride >= 1
        # the free packet's centre reaches x1 = a + Delta at t* = x1 - x0
        assert abs(row * inst.Delta - (inst.a + inst.Delta - inst.x0)) <= inst.Delta or row == inst.Nt


def test_coarse_grids_keep_the_physics_and_the_box():
    """coarse grids keep a and the box's right edge exactly (the box a
    multiple of 2a) and cover the window; unboxed instances are refused"""
    n = 0
    for inst in SW.draw(64, 4):
        assert inst.Nx % inst.D == 0 and inst.Nx >= 2 * inst.D
        for f in (2, 4, 8):
            c = SW.coarse(inst, f)
            if c is None:
                continue
            n += 1
            assert c.D % 2 == 0 and 2 <= c.D < inst.D
            assert math.isclose(c.a, inst.a, rel_tol=1e-14)              # the same emitter-mirror distance
            assert math.isclose(c.Nx * c.Delta, inst.Nx * inst.Delta, rel_tol=1e-13)   # the same box
            assert c.Nt * c.Delta >= SW.pe_window(inst) - 1e-9            # the window is covered
            assert c.Delta >= 0.6 * f * inst.Delta
    assert n >= 150
    raw = next(i for i in W.sweep_draw(64, 4) if i.Nx % i.D)
    try:
        SW.coarse(raw, 2)
    except ValueError:
        pass
    else:
        raise AssertionError("an instance whose box is not a multiple of 2a has no coarse grid of the same box")


def test_box_leaves_the_march_of_its_columns_unchanged():
    """box() only drops columns (D, Delta, Nt and the packet stay), and the
    march of the columns it keeps is the same bit for bit (the oracle on a
    small grid: no column depends on columns to its right)"""
    for inst in W.sweep_draw(32, 8):
        b = SW.box(inst)
        assert b.Nx <= inst.Nx < b.Nx + inst.D
        assert (b.D, b.Delta, b.Nt, b.x0, b.width, b.k) == (inst.D, inst.Delta, inst.Nt, inst.x0, inst.width, inst.k)
    import oracle
    small = W.gaussian_instance("box", Gamma=1.0, two_a=0.24, Delta=0.01, k0a=1.1, width=0.3, Nx=131, Nt=260,
                                seed=3)
    b = SW.box(small)
    assert b.Nx == 120 and small.D == 24
    rows = [50, 140, 260]
    full = oracle.march(small, oracle.E_table(small), snap_rows=rows)["snaps"]
    cut = oracle.march(b, oracle.E_table(b), snap_rows=rows)["snaps"]
    assert np.abs(full).max() > 1e-3
    assert np.array_equal(full[:, :b.Nx + 1], cut)


def test_pe_window_inside_the_march():
    for inst in W.sweep_draw(64, 6):
        T_s = SW.pe_window(inst)
        assert 0 < T_s <= inst.Nt * inst.Delta + 1e-12
        # the box is sized so that the window holds the packet and its decay
        assert T_s >= min(inst.Nt * inst.Delta, 16 * inst.width)
