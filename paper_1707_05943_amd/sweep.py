"""Parameter sweeps over the batched solver, the surrogate's data and
training, and the surrogate-with-fallback sweep.

Orchestration only: the solves run in the HIP march (fdtd.Batch), the network
in the HIP surrogate library (surrogate.Net).  Torch device tensors carry the
data between them; the input encoding and the packing of targets are
element-wise torch operations on the device.

Targets of an instance (n = 1024 samples each):
  * P_e(t_k), t_k = k T_s / (n-1) over T_s = min(Nt Delta, 16 w + 2a + 10/Gamma),
    the span in which the packet (16 w long) has reached the emitter and the
    response has decayed over a few round trips; the box of the instance is
    sized for that span, and later P_e is the slow leak of the box;
  * chi_out(tau_k) e^{-i theta}: chi of Eq. (2) at the detectors x1 = a + Delta,
    x2 = x1 + tau_k, taken at the row nearest t* = x1 - x0 (when the free
    packet's centre reaches x1), tau_k = k s Delta with the integer stride
    s = max(1, round(L / (1023 Delta))), L = min(6 w + 2a, x_R - x1), x_R the
    box's right edge; samples beyond the box are masked.  The global phase
    theta multiplies chi as a whole and is removed.
Input encoding (8 channels at n points sigma_p = 16 w p/(n-1)): the incident
profile phi(-a - sigma) without its normalisation (real, imaginary), then
Gamma 2a / 10, k0 a / 2 pi, ln w / ln 5, Delta / 0.01, ln(Gamma T_s) / ln 1000
(the window the P_e samples span) and p / (n-1).
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import fdtd
from . import surrogate as S
from . import sur_inputs as SI
from . import workloads as W

N_SAMPLES = 1024
C_IN = 8
C_OUT = 3


def pe_window(inst) -> float:
    """T_s, the end of the P_e target window"""
    return min(inst.Nt * inst.Delta, 16.0 * inst.width + 2.0 * inst.a + 10.0 / inst.Gamma)


def chi_plan(inst) -> tuple[int, int]:
    """(snapshot row, detector stride) of the chi target"""
    a, d = inst.a, inst.Delta
    x1 = a + d
    row = int(round((x1 - inst.x0) / d))
    row = min(max(row, 1), inst.Nt)
    x_r = -a + inst.Nx * d
    L = min(6.0 * inst.width + 2.0 * a, x_r - x1)
    stride = max(1, int(round(L / ((N_SAMPLES - 1) * d))))
    return row, stride


def features(insts, device):
    """(B, n, 8) float32 input encoding on the device"""
    import torch
    n = N_SAMPLES
    w = torch.tensor([i.width for i in insts], dtype=torch.float64, device=device)[:, None]
    k0 = torch.tensor([i.k for i in insts], dtype=torch.float64, device=device)[:, None]
    a = torch.tensor([i.a for i in insts], dtype=torch.float64, device=device)[:, None]
    G = torch.tensor([i.Gamma for i in insts], dtype=torch.float64, device=device)[:, None]
    dl = torch.tensor([i.Delta for i in insts], dtype=torch.float64, device=device)[:, None]
    T = torch.tensor([pe_window(i) for i in insts], dtype=torch.float64, device=device)[:, None]
    p = torch.arange(n, dtype=torch.float64, device=device)[None, :] / (n - 1)
    # phi(-a - sigma) with x0 = -a - 8w: x - x0 = 8w - sigma
    u = 8.0 - 16.0 * p
    env = torch.exp(-0.25 * u * u)
    ph = k0 * w * u
    ones = torch.ones_like(p)
    x = torch.stack([env * torch.cos(ph), env * torch.sin(ph), (G * 2 * a / 10.0) * ones,
                     (k0 * a / (2 * math.pi)) * ones, (torch.log(w) / math.log(5.0)) * ones,
                     (dl / 0.01) * ones, (torch.log(G * T) / math.log(1000.0)) * ones,
                     p.expand(len(insts), n)], dim=-1)
    return x.to(torch.float32).contiguous()


def coarse(inst, factor: int):
    """the same physical problem on a grid about `factor` times coarser: D_c
    even and a kept exactly (so Delta_c = 2a / D_c), the box and the window
    covered"""
    D_c = max(2, 2 * int(round(inst.D / (2.0 * factor))))
    d_c = 2.0 * inst.a / D_c
    Nx_c = max(D_c + 1, int(math.ceil(inst.Nx * inst.Delta / d_c)))
    Nt_c = int(math.ceil(inst.Nt * inst.Delta / d_c - 1e-9))
    c = W.Instance(**{**inst.as_dict(), "D": D_c, "Delta": d_c, "Nx": Nx_c, "Nt": Nt_c,
                      "name": f"{inst.name}_c{factor}"})
    try:
        fdtd.workspace_size(c)           # the coarse grid must still be a valid instance
    except fdtd.FdtdError:
        return None
    return c


class Solver:
    """Batched FP64 solves of lists of instances, reusing one workspace."""

    def __init__(self, device="cuda:0", opts=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.opts = opts if opts is not None else fdtd.batch_opts()
        self.ws = None

    def _workspace(self, insts):
        need = fdtd.batch_workspace_size(insts, self.opts)
        if self.ws is None or self.ws.numel() < need:
            self.ws = None
            self.torch.cuda.empty_cache()
            self.ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self.ws

    def solve(self, insts, with_chi=True, t_end=None):
        """P_e samples (B, n) float64 over [0, t_end[i]] (default: each
        instance's pe_window) and, with_chi, chi_out e^{-i theta} samples
        (B, n) complex128 and their mask (B, n) on the device"""
        torch = self.torch
        B = len(insts)
        pe = torch.empty(B, N_SAMPLES, dtype=torch.float64, device=self.device)
        bat = fdtd.Batch(insts, self.opts, device=str(self.device), workspace=self._workspace(insts))
        chi = mask = None
        if with_chi:
            plans = [chi_plan(i) for i in insts]
            chi = torch.zeros(B, N_SAMPLES, dtype=torch.complex128, device=self.device)
            bat.set_chi([p[0] for p in plans], [p[1] for p in plans], N_SAMPLES, chi)
            avail = torch.tensor([(i.Nx - i.D + p[1] - 1) // p[1] for i, p in zip(insts, plans)],
                                 device=self.device)
            mask = (torch.arange(N_SAMPLES, device=self.device)[None, :] < avail[:, None]).to(torch.float32)
        if t_end is None:
            t_end = [pe_window(i) for i in insts]
        te = torch.tensor(t_end, dtype=torch.float64, device=self.device)
        bat.set_boundary().march()
        bat.sample_pe(N_SAMPLES, pe, te)
        torch.cuda.current_stream(self.device).synchronize()
        bat.close()
        if with_chi:
            theta = torch.tensor([i.phase for i in insts], dtype=torch.float64, device=self.device)
            chi = chi * torch.exp(-1j * theta)[:, None]
        return pe, chi, mask


def targets(pe, chi, mask):
    """(B, n, 3) float32 targets and mask"""
    import torch
    t = torch.stack([pe, chi.real, chi.imag], dim=-1).to(torch.float32).contiguous()
    m = torch.stack([torch.ones_like(mask), mask, mask], dim=-1).contiguous()
    return t, m


def make_dataset(insts, solver: Solver, chunk=512, log=None):
    """inputs, targets and masks of `insts`, solved in batches of `chunk`"""
    import torch
    xs, ts, ms = [], [], []
    for s in range(0, len(insts), chunk):
        part = insts[s:s + chunk]
        t0 = time.perf_counter()
        pe, chi, mask = solver.solve(part)
        t, m = targets(pe, chi, mask)
        xs.append(features(part, solver.device))
        ts.append(t)
        ms.append(m)
        if log:
            log(f"[sweep] solved {s + len(part)}/{len(insts)} instances ({time.perf_counter() - t0:.1f} s)")
    return torch.cat(xs), torch.cat(ts), torch.cat(ms)


# channel weights of the loss: P_e counts most (the sweep's accuracy is on P_e)
LOSS_WEIGHTS = (4.0, 1.0, 1.0)


def surrogate_cfg(max_batch=32, c_in=C_IN, c_out=C_OUT):
    return S.cfg(n_points=N_SAMPLES, c_in=c_in, width=64, modes=64, layers=4, proj=128, c_out=c_out,
                 max_batch=max_batch)


def train(x, t, m, steps=2000, batch=32, lr=1e-3, seed=5, net=None, log=None, weights=LOSS_WEIGHTS):
    """Adam on random mini-batches of (x, t, m); returns the network (its
    input and output channels are those of x and t)"""
    import torch
    dev = x.device
    if net is None:
        c = surrogate_cfg(batch, c_in=x.shape[2], c_out=t.shape[2])
        theta = SI.init_params(SI.cfg_dict(c), seed)
        net = S.Net(c, torch.from_numpy(theta).to(dev), device=str(dev))
    wo = torch.tensor(weights, dtype=torch.float32, device=dev)
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    n = x.shape[0]
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(dev)
        xb, tb, mb = x[idx].contiguous(), t[idx].contiguous(), m[idx].contiguous()
        step_lr = lr if it < steps // 2 else lr * 0.5 ** (1 + 4 * (it - steps // 2) // steps)
        loss = net.train_step(xb, tb, wo, mb, lr=step_lr)
        if log and (it % 500 == 0 or it == steps - 1):
            log(f"[sweep] step {it}: loss {float(loss.cpu()[0]):.3e} ({(time.perf_counter() - t0) / (it + 1) * 1e3:.2f} "
                f"ms per step)")
    return net


def predict_pe(net, x, batch=None):
    """surrogate P_e (B, n) float64 for inputs x"""
    import torch
    B = x.shape[0]
    mb = batch or net.cfg.max_batch
    out = torch.empty(B, N_SAMPLES, dtype=torch.float64, device=x.device)
    for s in range(0, B, mb):
        y = net.forward(x[s:s + mb].contiguous())
        out[s:s + mb] = y[:, :, 0].to(torch.float64)
    return out


def rel_err(a, b):
    """relative L2 error per row"""
    import torch
    return torch.linalg.norm(a - b, dim=1) / torch.clamp(torch.linalg.norm(b, dim=1), min=1e-300)


def sweep(insts, net, solver: Solver, tol=1e-3, accept=None, factor=4, chunk=512, log=None):
    """Surrogate with a-posteriori check and FP64 fallback, for P_e.

    For each point: the surrogate's P_e; a coarse FP64 solve (grid `factor`
    times coarser, same physical window); the surrogate is accepted where its
    relative L2 distance to the coarse solve is at most `accept` (default
    tol / 2), otherwise the point is re-solved on its own grid.  Returns the
    P_e of every point, the accepted mask and timings."""
    import torch
    accept = tol / 2 if accept is None else accept
    dev = solver.device
    t0 = time.perf_counter()
    x = torch.cat([features(insts[s:s + chunk], dev) for s in range(0, len(insts), chunk)])
    s_pe = predict_pe(net, x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # coarse solves of the points that have a valid coarse grid (the others fall back)
    cs = [coarse(i, factor) for i in insts]
    have = [i for i, c in enumerate(cs) if c is not None]
    ok = torch.zeros(len(insts), dtype=torch.bool, device=dev)
    for s in range(0, len(have), chunk):
        ids = have[s:s + chunk]
        pe, _, _ = solver.solve([cs[i] for i in ids], with_chi=False, t_end=[pe_window(insts[i]) for i in ids])
        idx = torch.tensor(ids, device=dev)
        ok[idx] = rel_err(s_pe[idx], pe) <= accept
    t2 = time.perf_counter()
    out = s_pe.clone()
    fb = [i for i, a in enumerate(ok.tolist()) if not a]
    for s in range(0, len(fb), chunk):
        ids = fb[s:s + chunk]
        pe, _, _ = solver.solve([insts[i] for i in ids], with_chi=False)
        out[torch.tensor(ids, device=dev)] = pe
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    if log:
        log(f"[sweep] {len(insts)} points: surrogate {t1 - t0:.2f} s, check {t2 - t1:.2f} s, "
            f"fallback {len(fb)} points {t3 - t2:.2f} s")
    return out, ok, {"surrogate_s": t1 - t0, "check_s": t2 - t1, "fallback_s": t3 - t2, "total_s": t3 - t0,
                     "fallback": len(fb), "points": len(insts)}


# ---------------------------------------------------------------------------
# Corrected sweep: a network predicts the difference between the fine solve's
# P_e and that of a 4x coarser FP64 solve; the a-posteriori check compares the
# prediction with the Richardson estimate of the same difference from a
# second, 8x coarser solve (the scheme is second order:
# P_h = P + K h^2, so P_fine - P_4 = (P_8 - P_4)(Delta^2 - h_4^2)/(h_8^2 - h_4^2)).
# ---------------------------------------------------------------------------
CORR_SCALE = 100.0          # default scale of the difference seen by the network (set from the data)


def coarse_pe(insts, solver: Solver, factor: int, chunk=512):
    """P_e of each point on its `factor`-coarser grid, sampled on the point's
    own window; (pe (B, n), valid (B,) bool, grid steps (B,))"""
    import torch
    dev = solver.device
    cs = [coarse(i, factor) for i in insts]
    have = [i for i, c in enumerate(cs) if c is not None]
    pe = torch.zeros(len(insts), N_SAMPLES, dtype=torch.float64, device=dev)
    for s in range(0, len(have), chunk):
        ids = have[s:s + chunk]
        p, _, _ = solver.solve([cs[i] for i in ids], with_chi=False, t_end=[pe_window(insts[i]) for i in ids])
        pe[torch.tensor(ids, device=dev)] = p
    valid = torch.zeros(len(insts), dtype=torch.bool, device=dev)
    if have:
        valid[torch.tensor(have, device=dev)] = True
    h = torch.tensor([c.Delta if c is not None else float("nan") for c in cs], dtype=torch.float64, device=dev)
    return pe, valid, h


def corrector_inputs(insts, c4, device):
    """the surrogate's encoding plus the coarse solve's P_e as a ninth channel"""
    import torch
    return torch.cat([features(insts, device), c4.to(torch.float32)[:, :, None]], dim=2).contiguous()


def make_corrector_dataset(insts, solver: Solver, chunk=512, log=None, fine=None):
    """inputs and targets (P_fine - P_4) x CORR_SCALE of the points whose
    coarse grid is valid (`fine`: the points' fine P_e samples, if at hand)"""
    import torch
    if fine is None:
        fine = torch.cat([solver.solve(insts[s:s + chunk], with_chi=False)[0] for s in range(0, len(insts), chunk)])
    fine = fine.to(torch.float64)
    c4, v4, _ = coarse_pe(insts, solver, 4, chunk)
    keep = [i for i, v in enumerate(v4.tolist()) if v]
    idx = torch.tensor(keep, device=solver.device)
    x = corrector_inputs([insts[i] for i in keep], c4[idx], solver.device)
    d = fine[idx] - c4[idx]
    scale = 1.0 / max(float(torch.sqrt(torch.mean(d * d))), 1e-300)     # unit RMS targets
    t = (d * scale).to(torch.float32)[:, :, None].contiguous()
    m = torch.ones_like(t)
    if log:
        log(f"[sweep] corrector data: {len(keep)} of {len(insts)} points have a coarse grid, "
            f"difference RMS {1.0 / scale:.3e}")
    return x, t, m, scale


def sweep_corrected(insts, net, solver: Solver, tol=1e-3, accept=None, chunk=512, log=None):
    """P_e of every point: coarse solve + network correction where the check
    passes (the two estimates of the correction agree within tol/4 relative),
    the fine FP64 solve elsewhere.  Returns (P_e, accepted, info,
    Richardson-only estimate)."""
    import torch
    accept = tol / 4 if accept is None else accept
    dev = solver.device
    t0 = time.perf_counter()
    c4, v4, h4 = coarse_pe(insts, solver, 4, chunk)
    c8, v8, h8 = coarse_pe(insts, solver, 8, chunk)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x = corrector_inputs(insts, c4, dev)
    d_nn = predict_pe(net, x) / getattr(net, "corr_scale", CORR_SCALE)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    hf = torch.tensor([i.Delta for i in insts], dtype=torch.float64, device=dev)
    w = ((hf ** 2 - h4 ** 2) / (h8 ** 2 - h4 ** 2))[:, None]
    d_r = (c8 - c4) * w
    scale = torch.clamp(torch.linalg.norm(c4, dim=1), min=1e-300)
    ok = v4 & v8 & (torch.linalg.norm(d_nn - d_r, dim=1) / scale <= accept)
    out = c4 + d_nn
    rich = torch.where((v4 & v8)[:, None], c4 + d_r, torch.full_like(c4, float("nan")))
    fb = [i for i, a in enumerate(ok.tolist()) if not a]
    for s in range(0, len(fb), chunk):
        ids = fb[s:s + chunk]
        pe, _, _ = solver.solve([insts[i] for i in ids], with_chi=False)
        out[torch.tensor(ids, device=dev)] = pe
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    if log:
        log(f"[sweep] corrected, {len(insts)} points: coarse solves {t1 - t0:.2f} s, network {t2 - t1:.2f} s, "
            f"fallback {len(fb)} points {t3 - t2:.2f} s")
    return out, ok, {"coarse_s": t1 - t0, "network_s": t2 - t1, "fallback_s": t3 - t2, "total_s": t3 - t0,
                     "fallback": len(fb), "points": len(insts)}, rich
