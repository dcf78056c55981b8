"""GPU checks of the sweep pipeline: the batched targets against one-instance
solves; the library's input encoding and a-posteriori check against plain
numpy evaluations of their formulas; the trained network against the method
without it (FP64 solves on coarser grids at matched cost); the soundness of
the check on audited points."""
import math
import sys
import time

import numpy as np
import pytest

from paper_1707_05943_amd import fdtd
from paper_1707_05943_amd import surrogate as S
from paper_1707_05943_amd import sweep as SW
from paper_1707_05943_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _small_draw(n, seed):
    """sweep draws cut to short windows so the checks stay quick, boxes cut
    to multiples of 2a"""
    out = []
    for inst in W.sweep_draw(n, seed):
        out.append(SW.box(W.with_sizes(inst, Nx=min(inst.Nx, 2048 if inst.D < 1000 else inst.Nx),
                                       Nt=min(inst.Nt, 3000), name=inst.name)))
    return [i for i in out if i.Nx >= i.D + 1]


@pytest.fixture(scope="module")
def solver():
    return SW.Solver()


def test_targets_match_one_instance_solves(solver):
    insts = _small_draw(6, 41)
    pe, chi, mask = solver.solve(insts)
    pe, chi, mask = pe.cpu().numpy(), chi.cpu().numpy(), mask.cpu().numpy()
    for i, inst in enumerate(insts[:3]):
        row, stride = SW.chi_plan(inst)
        sol = fdtd.Solver(inst).set_boundary()
        sol.march(row)
        navail = inst.Nx - inst.D
        c = sol.chi(min(navail, SW.N_SAMPLES * stride))[::stride] * np.exp(-1j * inst.phase)
        want = np.zeros(SW.N_SAMPLES, complex)
        want[:c.size] = c
        e_chi = np.linalg.norm(chi[i] - want) / np.linalg.norm(want)
        assert np.array_equal(mask[i] > 0, np.arange(SW.N_SAMPLES) < c.size)
        sol.march(inst.Nt - row)
        full = sol.pe()
        pos = np.arange(SW.N_SAMPLES) * (SW.pe_window(inst) / inst.Delta) / (SW.N_SAMPLES - 1)
        e_pe = np.linalg.norm(pe[i] - np.interp(pos, np.arange(inst.Nt + 1), full)) / np.linalg.norm(full)
        _say(f"[sweep] {inst.name}: D={inst.D} Nx={inst.Nx} chi {e_chi:.2e}, P_e {e_pe:.2e}")
        assert e_chi <= 1e-12 and e_pe <= 1e-12
        sol.close()


def test_encoding_matches_its_formula():
    """sur_encode against the same encoding in float64 numpy (rounded to float32)"""
    insts = W.sweep_draw(5, 5)
    x = SW.features(insts, "cuda:0").cpu().numpy()
    n = SW.N_SAMPLES
    p = np.arange(n) / (n - 1)
    for b, i in enumerate(insts):
        u = 8.0 - 16.0 * p
        env = np.exp(-0.25 * u * u)
        ph = i.k * i.width * u
        want = np.stack([env * np.cos(ph), env * np.sin(ph), np.full(n, i.Gamma * 2 * i.a / 10.0),
                         np.full(n, i.k * i.a / (2 * math.pi)), np.full(n, math.log(i.width) / math.log(5.0)),
                         np.full(n, i.Delta / 0.01), np.full(n, math.log(i.Gamma * SW.pe_window(i)) / math.log(1000.0)),
                         p], axis=1)
        assert np.max(np.abs(x[b] - want.astype(np.float32))) <= 2e-7 * max(1.0, np.abs(want).max())
        # the packet's envelope peaks at its centre, sigma = 8 w, with value 1
        env_got = np.hypot(x[b, :, 0], x[b, :, 1])
        assert abs(int(np.argmax(env_got)) - (n - 1) / 2) <= 1


def test_check_matches_its_formula():
    """sur_check against the same formulas in numpy, on random profiles:
    points in and out of the asymptotic range, a point without coarse grids"""
    import torch
    rng = np.random.default_rng(7)
    B, n = 12, SW.N_SAMPLES
    P = rng.random((B, n)) + 0.5
    K = rng.standard_normal((B, n))
    h = np.array([[0.01, 0.02, 0.04, 0.08]] * B)
    h[5] = [0.005, 0.0101, 0.0198, 0.0412]                 # grid steps not exactly in the ratio 2
    P2, P4 = P + K * h[:, 1:2] ** 2, P + K * h[:, 2:3] ** 2
    # the 8x solve in the asymptotic range, except for points 1, 4, 7 (ratio off by 40%)
    P8 = P + K * h[:, 3:4] ** 2
    for b in (1, 4, 7):
        P8[b] = P4[b] + 1.4 * (P8[b] - P4[b])
    Sx = P2 + 10.0 ** rng.uniform(-5, -1, (B, 1)) * rng.standard_normal((B, n))
    valid = np.ones(B, np.int32)
    valid[3] = 0
    T = lambda a: torch.tensor(a, device="cuda:0")
    tol, safety, rtol = 3e-3, 2.0, 0.25
    de, acc = S.check(T(Sx), T(P2), T(P4), T(P8), T(h), T(valid), tol, safety, rtol)
    de, acc = de.cpu().numpy(), acc.cpu().numpy()
    nrm = np.linalg.norm(P2, axis=1)
    dist = np.linalg.norm(Sx - P2, axis=1) / nrm
    h0, h2, h4, h8 = h.T
    est = safety * np.abs((h2 ** 2 - h0 ** 2) / (h4 ** 2 - h2 ** 2)) * np.linalg.norm(P4 - P2, axis=1) / nrm
    rho = (h8 ** 2 - h4 ** 2) / (h4 ** 2 - h2 ** 2)
    q = np.linalg.norm(P8 - P4, axis=1) / np.linalg.norm(P4 - P2, axis=1) / rho
    assert np.allclose(de[:, 0], dist, rtol=1e-13) and np.allclose(de[:, 1], est, rtol=1e-13)
    assert np.allclose(de[:, 2], q, rtol=1e-12)
    inr = (valid > 0) & (np.abs(q - 1) <= rtol)
    assert np.array_equal(inr, ~np.isin(np.arange(B), [1, 3, 4, 7]))
    assert np.array_equal(acc[:, 0], inr & (dist + est <= tol))
    assert np.array_equal(acc[:, 1], inr & (est <= tol))
    assert acc[:, 1].sum() > 0 and acc[:, 0].sum() > 0 and (acc[:, 1] & ~acc[:, 0]).sum() > 0
    # the estimate is exact (up to safety) in the asymptotic range: the fine
    # solve is P + K h0^2
    true = np.linalg.norm(P2 - (P + K * h[:, 0:1] ** 2), axis=1) / nrm
    assert np.allclose(est[inr] / safety, true[inr], rtol=1e-9)


@pytest.fixture(scope="module")
def trained(solver):
    train_set = _small_draw(256, 42)
    val_set = _small_draw(48, 43)
    x, t, m = SW.make_dataset(train_set, solver, log=_say)
    for c in range(3):
        v = t[:, :, c]
        _say(f"[sweep] target channel {c}: mean |.| {float(v.abs().mean()):.3e}, max {float(v.abs().max()):.3e}")
    net = SW.train(x, t, m, steps=1500, batch=32, lr=1e-3, log=_say)
    return net, (x, t, m), val_set


def test_trained_network_beats_an_input_blind_predictor(trained, solver):
    """validation error of the network against the mean training trajectory"""
    import torch
    net, (x, t, m), val = trained
    xv, tv, mv = SW.make_dataset(val, solver)
    pred = SW.predict_pe(net, xv)
    truth = tv[:, :, 0].to(torch.float64)
    e_net = SW.rel_err(pred, truth)
    mean = t[:, :, 0].to(torch.float64).mean(dim=0, keepdim=True).expand_as(truth)
    e_mean = SW.rel_err(mean, truth)
    _say(f"[sweep] validation P_e rel-L2: network median {e_net.median():.3e}, input-blind {e_mean.median():.3e}")
    assert float(e_net.median()) < 0.6 * float(e_mean.median())


def test_network_against_coarser_grids_at_matched_cost(trained, solver):
    """The method without the network: FP64 solves of the same window on
    grids 2, 4, 8 and 16 times coarser.  Cost per point (inference, solves)
    and median relative L2 error of P_e against the fine solve; the network
    is compared with the coarse grids whose cost is closest to its own (all
    are reported)."""
    import torch
    net, _, val = trained
    fine, _, _ = solver.solve(val, with_chi=False)
    x = SW.features(val, solver.device)
    SW.predict_pe(net, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = SW.predict_pe(net, x)
    torch.cuda.synchronize()
    cost_net = (time.perf_counter() - t0) / len(val)
    e_net = float(SW.rel_err(pred, fine).median())
    rows = []
    for f in (2, 4, 8, 16):
        SW.coarse_pe(val, solver, f)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc, vc, _ = SW.coarse_pe(val, solver, f)
        torch.cuda.synchronize()
        cost = (time.perf_counter() - t0) / len(val)
        e = float(SW.rel_err(pc[vc], fine[vc]).median()) if bool(vc.any()) else float("nan")
        rows.append((f, cost, e, int(vc.sum())))
        _say(f"[sweep] {f}x coarser grid: {cost * 1e3:.3f} ms per point, median error {e:.2e} ({int(vc.sum())} points)")
    _say(f"[sweep] network: {cost_net * 1e3:.3f} ms per point, median error {e_net:.2e}")
    # the solves are all valid and more accurate the finer the grid
    assert all(r[3] > 0 for r in rows[:2])
    assert rows[0][2] < rows[1][2]
    assert cost_net < rows[-1][1]                 # inference is cheaper than even the coarsest solve


def test_sweep_check_is_sound(trained, solver):
    """Points the check accepts are within tol of the fine solve (audited
    against the fine solve of every point); the network path accepts a
    subset of what the coarse solve alone does; rejected points carry the
    fine solve bit for bit.  At tol = 1e-3 and at a loose tol = 0.5, where
    this small network's answers get accepted too."""
    import torch
    net = trained[0]
    pts = _small_draw(64, 44)
    fine, _, _ = solver.solve(pts, with_chi=False)
    for tol in (1e-3, 0.5):
        out_s, out_c, acc, de, info = SW.sweep(pts, net, solver, tol=tol, log=_say)
        e_s = SW.rel_err(out_s, fine)
        e_c = SW.rel_err(out_c, fine)
        a_s, a_c = acc[:, 0], acc[:, 1]
        _say(f"[sweep] tol {tol}: accepted network {int(a_s.sum())}, coarse {int(a_c.sum())}; worst accepted error "
             f"network {float(e_s[a_s].max()) if bool(a_s.any()) else 0:.2e}, "
             f"coarse {float(e_c[a_c].max()) if bool(a_c.any()) else 0:.2e}")
        assert bool((~a_s | a_c).all())
        assert bool((e_s[a_s] <= tol).all()) and bool((e_c[a_c] <= tol).all())
        assert torch.equal(out_s[~a_s], fine[~a_s]) and torch.equal(out_c[~a_c], fine[~a_c])
        if tol > 0.1:
            assert int(a_s.sum()) > 0             # the loose tolerance exercises the network's acceptance
        assert int(a_c.sum()) > 0
