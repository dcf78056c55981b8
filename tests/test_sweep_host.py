"""Host-side logic of the sweep pipeline (no GPU): target plans, the coarse
grids of the a-posteriori check, the input encoding."""
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


def test_coarse_grid_keeps_the_physics():
    for inst in W.sweep_draw(64, 4):
        c = SW.coarse(inst, 4)
        if c is None:
            continue
        assert c.D % 2 == 0 and c.D >= 2
        assert math.isclose(c.a, inst.a, rel_tol=1e-12)              # the same emitter-mirror distance
        assert c.Nt * c.Delta >= inst.Nt * inst.Delta - 1e-9          # the window is covered
        assert c.Nx * c.Delta >= inst.Nx * inst.Delta - 1e-9          # and the box
        assert c.Delta >= 2.5 * inst.Delta or c.D == 2


def test_features_encode_the_profile():
    import torch
    insts = W.sweep_draw(3, 5)
    x = SW.features(insts, "cpu").numpy()
    assert x.shape == (3, SW.N_SAMPLES, SW.C_IN)
    # the envelope peaks at sigma = 8 w (the packet centre), value 1
    env = np.hypot(x[:, :, 0], x[:, :, 1])
    p = np.argmax(env, axis=1)
    assert np.all(np.abs(p - (SW.N_SAMPLES - 1) / 2) <= 1) and np.allclose(env.max(axis=1), 1.0, atol=1e-3)
    for b, inst in enumerate(insts):
        assert np.allclose(x[b, :, 5], inst.Delta / 0.01)
        assert np.allclose(x[b, :, 2], inst.Gamma * 2 * inst.a / 10.0, atol=1e-7)


def test_pe_window_inside_the_march():
    for inst in W.sweep_draw(64, 6):
        T_s = SW.pe_window(inst)
        assert 0 < T_s <= inst.Nt * inst.Delta + 1e-12
        # the box is sized so that the window holds the packet and its decay
        assert T_s >= min(inst.Nt * inst.Delta, 16 * inst.width)
