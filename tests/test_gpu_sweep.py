"""GPU checks of the sweep pipeline: the batched targets against one-instance
solves, the fallback logic of the surrogate sweep, and what the trained
network gains over a predictor that ignores the inputs."""
import sys

import numpy as np
import pytest

from paper_1707_05943_amd import fdtd
from paper_1707_05943_amd import sweep as SW
from paper_1707_05943_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _small_draw(n, seed):
    """sweep draws cut to short windows so the checks stay quick"""
    out = []
    for inst in W.sweep_draw(n, seed):
        out.append(W.with_sizes(inst, Nx=min(inst.Nx, 2048 if inst.D < 1000 else inst.Nx), Nt=min(inst.Nt, 3000),
                                name=inst.name))
    return [i for i in out if i.Nx >= i.D + 1]


@pytest.fixture(scope="module")
def solver():
    return SW.Solver()


def test_targets_match_one_instance_solves(solver):
    import torch
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


@pytest.fixture(scope="module")
def trained(solver):
    train_set = _small_draw(256, 42)
    val_set = _small_draw(32, 43)
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


def test_sweep_fallback_logic(trained, solver):
    import torch
    net = trained[0]
    pts = _small_draw(12, 44)
    plain, _, _ = solver.solve(pts, with_chi=False)
    # nothing accepted: every point is re-solved, bitwise the plain solve
    out, ok, info = SW.sweep(pts, net, solver, tol=1e-3, accept=-1.0)
    assert not bool(ok.any()) and info["fallback"] == len(pts)
    assert torch.equal(out, plain)
    # everything accepted: the surrogate's answer
    out, ok, info = SW.sweep(pts, net, solver, tol=1e-3, accept=1e30)
    have = [SW.coarse(p, 4) is not None for p in pts]
    assert ok.tolist() == have
    pred = SW.predict_pe(net, SW.features(pts, solver.device))
    sel = torch.tensor(have, device=out.device)
    assert torch.equal(out[sel], pred[sel]) and torch.equal(out[~sel], plain[~sel])


def test_corrected_sweep_logic(solver):
    """the corrector network on a small training set: its accepted points are
    coarse + correction, the others the fine solve bitwise; the errors of the
    coarse solve, the corrected one and the Richardson estimate are reported"""
    import torch
    train_set = _small_draw(128, 45)
    xc, tc, mc, cscale = SW.make_corrector_dataset(train_set, solver, log=_say)
    cnet = SW.train(xc, tc, mc, steps=600, batch=32, lr=1e-3, log=_say, weights=(1.0,), seed=6)
    cnet.corr_scale = cscale
    pts = _small_draw(24, 46)
    plain, _, _ = solver.solve(pts, with_chi=False)
    out, ok, info, rich = SW.sweep_corrected(pts, cnet, solver, tol=1e-3, log=_say)
    fb = ~ok
    assert torch.equal(out[fb], plain[fb])
    c4, v4, _ = SW.coarse_pe(pts, solver, 4)
    pred = SW.predict_pe(cnet, SW.corrector_inputs(pts, c4, solver.device)) / cscale
    if bool(ok.any()):
        assert torch.equal(out[ok], (c4 + pred)[ok])
    e_c = SW.rel_err(c4[v4], plain[v4])
    e_n = SW.rel_err((c4 + pred)[v4], plain[v4])
    rv = ~torch.isnan(rich[:, 0])
    e_r = SW.rel_err(rich[rv], plain[rv])
    _say(f"[sweep] median rel-L2 of P_e: coarse {e_c.median():.2e}, coarse + network {e_n.median():.2e}, "
         f"coarse + Richardson {e_r.median():.2e}; accepted {int(ok.sum())}/{len(pts)}")
    # accepted points meet the tolerance the check was set for
    e_out = SW.rel_err(out, plain)
    assert float(e_out[ok].max()) <= 1e-3 if bool(ok.any()) else True
