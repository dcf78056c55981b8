"""Parameter sweeps over the batched solver, the surrogate's data and
training, and the surrogate-with-fallback sweep.

Orchestration only: the solves run in the HIP march (fdtd.Batch), the network
and its input encoding in the HIP surrogate library (surrogate.Net,
surrogate.encode), the a-posteriori check in the library too
(surrogate.check).  Torch device tensors carry the data between them.

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


def params_array(insts, device):
    """(B, 6) float64 device tensor of (w, k0, a, Gamma, Delta, T_s) per instance"""
    import torch
    return torch.tensor([[i.width, i.k, i.a, i.Gamma, i.Delta, pe_window(i)] for i in insts], dtype=torch.float64,
                        device=device)


def features(insts, device):
    """(B, n, 8) float32 input encoding on the device (the library's sur_encode)"""
    return S.encode(params_array(insts, device), N_SAMPLES)


def params_from_arrays(d, lo, hi, device):
    """params_array of points lo..hi-1 of a workloads.sweep_draw_arrays draw"""
    import torch
    sl = slice(lo, hi)
    w, a, dl = d["width"][sl], d["a"][sl], d["Delta"][sl]
    ts = np.minimum(d["Nt"][sl] * dl, 16.0 * w + 2.0 * a + 10.0)
    par = np.stack([w, d["k0"][sl], a, np.ones_like(w), dl, ts], axis=1)
    return torch.from_numpy(np.ascontiguousarray(par)).to(device)


def box(inst):
    """the instance with its box cut to the largest multiple of the round
    trip 2a inside it (Nx = floor(Nx / D) D): the box's right edge is then a
    node of every grid that keeps a exactly, so the P_e of a coarser grid
    (exact part plus the box integral) is the same physical quantity.  The
    march of columns 0..Nx does not depend on columns beyond Nx."""
    Nx = (inst.Nx // inst.D) * inst.D
    return inst if Nx == inst.Nx else W.Instance(**{**inst.as_dict(), "Nx": Nx})


def draw(n: int, seed: int):
    """workloads.sweep_draw with each box cut by box()"""
    return [box(i) for i in W.sweep_draw(n, seed)]


def coarse(inst, factor: int):
    """the same physical problem on a grid about `factor` times coarser: D_c
    even and a kept exactly (so Delta_c = 2a / D_c), the same box (the
    instance's box must be a multiple of 2a, see box()) and the time window
    covered; None where no such grid exists"""
    if inst.Nx % inst.D:
        raise ValueError(f"{inst.name}: the box (Nx = {inst.Nx}) is not a multiple of D = {inst.D}")
    D_c = max(2, 2 * int(round(inst.D / (2.0 * factor))))
    if D_c >= inst.D:
        return None
    d_c = 2.0 * inst.a / D_c
    Nx_c = (inst.Nx // inst.D) * D_c
    Nt_c = int(math.ceil(inst.Nt * inst.Delta / d_c - 1e-9))
    c = W.Instance(**{**inst.as_dict(), "D": D_c, "Delta": d_c, "Nx": Nx_c, "Nt": Nt_c,
                      "name": f"{inst.name}_c{factor}"})
    try:
        fdtd.workspace_size(c)           # the coarse grid must still be a valid instance
    except fdtd.FdtdError:
        return None
    return c


class Solver:
    """Batched FP64 solves of lists of instances, reusing one workspace (by
    default in two concurrently marched groups, the autotuner's pick for the
    512-instance sweep draw)."""

    def __init__(self, device="cuda:0", opts=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.opts = opts if opts is not None else fdtd.batch_opts(groups=2)
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


def coarse_pe(insts, solver: Solver, factor: int, chunk=512):
    """P_e of each point on its `factor`-coarser grid, sampled on the point's
    own window; (pe (B, n), valid (B,) bool, grid steps (B,) as a list).
    Batches hold chunk * factor^2 points (about the cells and the memory of
    `chunk` points on their own grids)."""
    import torch
    dev = solver.device
    cs = [coarse(i, factor) for i in insts]
    have = [i for i, c in enumerate(cs) if c is not None]
    pe = torch.zeros(len(insts), N_SAMPLES, dtype=torch.float64, device=dev)
    step = min(chunk * factor * factor, 16384)
    for s in range(0, len(have), step):
        ids = have[s:s + step]
        p, _, _ = solver.solve([cs[i] for i in ids], with_chi=False, t_end=[pe_window(insts[i]) for i in ids])
        pe[torch.tensor(ids, device=dev)] = p
    valid = torch.zeros(len(insts), dtype=torch.bool, device=dev)
    if have:
        valid[torch.tensor(have, device=dev)] = True
    return pe, valid, [c.Delta if c is not None else float("nan") for c in cs]


SAFETY = 2.0        # the check's factor on the leading-order estimate of the coarse solve's error
RATIO_TOL = 0.25    # the check's band on the observed/expected ratio of successive coarse differences


def sweep(insts, net, solver: Solver, tol=1e-3, safety=SAFETY, ratio_tol=RATIO_TOL, chunk=512, log=None):
    """Surrogate with an a-posteriori check and FP64 fallback, for P_e, next
    to the same check without the network.  Points must have boxes that are
    multiples of 2a (box()).

    Each point: the network's P_e (S); FP64 solves of the same window and box
    on grids about 2x, 4x and 8x coarser (P2, P4, P8).  In the scheme's
    asymptotic range (checked: successive differences in the ratio the grid
    steps give, within ratio_tol) the fine solve differs from P2 by about
    (P4 - P2)(h2^2 - h^2)/(h4^2 - h2^2); with that estimate (times `safety`)
    the network's answer is within tol of the fine solve when |S - P2|/|P2| +
    est <= tol, and P2 itself is when est <= tol; points that fail are solved
    on their own grid.  Whenever the first holds, so does the second: under a
    check that bounds the true error, the network path accepts a subset of
    what the coarse solve alone does, at the check's cost plus inference.
    Returns (P_e of the network path, P_e of the coarse path, accepted (B, 2)
    bool: network, coarse; (dist, est, q) (B, 3); timings and P2)."""
    import torch
    dev = solver.device
    t0 = time.perf_counter()
    x = torch.cat([features(insts[s:s + chunk], dev) for s in range(0, len(insts), chunk)])
    s_pe = predict_pe(net, x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p2, v2, h2 = coarse_pe(insts, solver, 2, chunk)
    p4, v4, h4 = coarse_pe(insts, solver, 4, chunk)
    p8, v8, h8 = coarse_pe(insts, solver, 8, chunk)
    h = torch.tensor([[i.Delta, a, b, c] for i, a, b, c in zip(insts, h2, h4, h8)], dtype=torch.float64, device=dev)
    h = torch.nan_to_num(h, nan=1.0)
    de, acc = S.check(s_pe, p2, p4, p8, h, (v2 & v4 & v8).to(torch.int32), tol, safety, ratio_tol)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # fallback: the coarse path rejects a subset of what the network path rejects
    rej_c = [i for i, a in enumerate(acc[:, 1].tolist()) if not a]
    rej_s_only = [i for i, (a, b) in enumerate(acc.tolist()) if b and not a]
    fine = {}
    t_parts = []
    for group in (rej_c, rej_s_only):
        tg = time.perf_counter()
        for s in range(0, len(group), chunk):
            ids = group[s:s + chunk]
            pe, _, _ = solver.solve([insts[i] for i in ids], with_chi=False)
            for k, i in enumerate(ids):
                fine[i] = pe[k]
        torch.cuda.synchronize()
        t_parts.append(time.perf_counter() - tg)
    out_s = s_pe.clone()
    out_c = p2.clone()
    in_c = set(rej_c)
    for i, v in fine.items():
        out_s[i] = v
        if i in in_c:
            out_c[i] = v
    t3 = time.perf_counter()
    info = {"points": len(insts), "inference_s": t1 - t0, "check_s": t2 - t1,
            "fallback_coarse_path_s": t_parts[0], "fallback_network_path_s": t_parts[0] + t_parts[1],
            "accepted_network": int(acc[:, 0].sum()), "accepted_coarse": int(acc[:, 1].sum()),
            "network_path_s": (t1 - t0) + (t2 - t1) + t_parts[0] + t_parts[1],
            "coarse_path_s": (t2 - t1) + t_parts[0], "assemble_s": t3 - t2 - sum(t_parts), "p2": p2}
    if log:
        log(f"[sweep] {len(insts)} points: inference {t1 - t0:.2f} s, check {t2 - t1:.2f} s; accepted network "
            f"{info['accepted_network']}, coarse alone {info['accepted_coarse']}")
    return out_s, out_c, acc, de, info
