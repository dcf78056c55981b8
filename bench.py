"""Benchmark: FP64 FDTD march of the 1+1D delay PDE on one MI355X.

One step = the whole hot path over one instance: the boundary tables
(gamma-function delay series for E(t_r)), the march over every row, and the
readouts (P_e(t_r) for all rows, chi at the detectors).  Inputs are synthetic
and already resident (the workspace lives in HBM before timing starts).

Prints one JSON line.  `value` is cell updates per second of the whole step;
`roofline` is the dominant kernel (the march) against the HBM peak, its
duration measured with events on the stream it runs on; `cpu_baseline` is the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FDTD cell-updates/s + % HBM roofline; sweep points/s at 1e-3 err (surrogate vs plain)"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0          # dense bf16 MFMA


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["large", "small", "batch", "nm", "sweep"], default="large")
    ap.add_argument("--batch", type=int, default=512, help="instances of the batched sweep")
    ap.add_argument("--batch-seed", type=int, default=7)
    ap.add_argument("--no-batch", action="store_true", help="leave the batched sweep out of the default line")
    ap.add_argument("--no-sweep", action="store_true", help="leave the surrogate sweep out of the default line")
    ap.add_argument("--sweep-train", type=int, default=20000, help="training instances of the surrogate")
    ap.add_argument("--sweep-steps", type=int, default=6000, help="Adam steps of the surrogate")
    ap.add_argument("--sweep-points", type=int, default=1000000, help="points of the surrogate sweep")
    ap.add_argument("--sweep-sub", type=int, default=10000,
                    help="points of the sweep on which the check, the fallback and the plain solver run")
    ap.add_argument("--no-nm", action="store_true",
                    help="leave the stimulated-emission march with the measures of App. D out of the default line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c0", action="store_true", help="leave the D=100, Nx=4000, Nt=4000 instance out")
    ap.add_argument("--cpu-rows", type=int, default=600, help="rows past D in the oracle's sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only the library's streaming copy of 21 GB each way (3 times): copy bandwidth and "
                         "the scale of the HBM byte counters")
    return ap.parse_args()


PROFILE = os.path.join(ROOT, "profiles", "k_block_gauss_D10000_Nx262144.md")
KERNEL_SOURCES = ["paper_1707_05943_amd/csrc/march_block.hip", "paper_1707_05943_amd/csrc/fdtd_common.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per k_block launch from the FETCH_SIZE / WRITE_SIZE counters
    recorded in the profile summary (scaled by a plain copy's counters), or
    None when the summary is for another workload or an older kernel."""
    if workload != "large" or not os.path.exists(PROFILE):
        return None
    vals = {}
    with open(PROFILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, _, v = line.partition(":")
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy():
    """The library's streaming copy (fdtd_stream_copy) of 21 GB each way, about
    the ring's size, three times: its kernel-trace duration gives the copy
    bandwidth, and its FETCH_SIZE / WRITE_SIZE counters, divided by the bytes
    moved, give the counters' scale."""
    import torch

    from paper_1707_05943_amd import fdtd
    n = 21 * 10**9 // 16 * 16
    src = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ms = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fdtd.stream_copy(dst, src)
        b.record(s)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    print(json.dumps({"calibrate_copy_bytes_each_way": n, "copies": 3, "ms": ms,
                      "GBps": [2.0 * n / (t * 1e-3) / 1e9 for t in ms]}), flush=True)


def cpu_baseline(inst, extra_rows: int) -> dict:
    """The oracle as it stands, single-threaded, on a column window of the
    same instance (columns 0..2D+1100, rows 1..D+extra_rows)."""
    import oracle
    from paper_1707_05943_amd import workloads as W
    win = W.with_sizes(inst, Nx=min(inst.Nx, 2 * inst.D + 1100), Nt=min(inst.Nt, inst.D + extra_rows))
    t0 = time.perf_counter()
    E = oracle.E_table(win)
    t1 = time.perf_counter()
    oracle.march(win, E, want_ring=False)
    t2 = time.perf_counter()
    cells = win.Nx * win.Nt
    return {"value": cells / (t2 - t1), "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "host": host_cpu(),
            "sample": f"march of columns 1..{win.Nx} over rows 1..{win.Nt} of {inst.name} "
                      f"({cells:.3g} cells, {t2 - t1:.1f} s; boundary table {t1 - t0:.1f} s not counted)"}


def run_batch(n: int, seed: int, steps: int, warmup: int) -> dict:
    """The batched sweep: n seed-drawn heterogeneous instances (Gamma 2a in
    [0.1, 10], k0 a in [0, 2 pi), width log-uniform in [0.2, 5], Delta in
    {0.01, 0.005, 0.002}, Nx 1024..16384, Nt = 4 Nx) marched together.  One
    step = boundary tables of every instance, the march of every row of every
    instance (graph replay), and P_e of every instance into device memory."""
    import torch

    from paper_1707_05943_amd import fdtd
    from paper_1707_05943_amd import workloads as W

    insts = W.sweep_draw(n, seed)
    dev = torch.device("cuda:0")
    need = max(fdtd.batch_workspace_size(insts, fdtd.batch_opts(t, w)) for t in (32, 16, 8) for w in (0, 768))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    best, rate = fdtd.autotune(insts, probe_rows=1024, workspace=ws)
    t_tune = time.perf_counter() - t0
    print(f"[bench] batch autotune: tmax={best.tmax} wmax={best.wmax} groups={best.groups} probe rate {rate:.3g} cells/s "
          f"({t_tune:.1f} s)", file=sys.stderr, flush=True)
    bat = fdtd.Batch(insts, best, workspace=ws)
    stream = torch.cuda.current_stream(dev)
    pe_dev = [torch.empty(i.Nt + 1, dtype=torch.float64, device=dev) for i in insts]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step(record=False):
        if record:
            ev[0].record(stream)
        bat.set_boundary()
        if record:
            ev[1].record(stream)
        bat.march()
        if record:
            ev[2].record(stream)
        for i, inst in enumerate(insts):
            bat.readout_device(i, fdtd.RO_PE, 0, pe_dev[i], inst.Nt + 1)
        if record:
            ev[3].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tb = tm = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        step(record=True)
        torch.cuda.synchronize()
        tb += ev[0].elapsed_time(ev[1])
        tm += ev[1].elapsed_time(ev[2])
    t1 = time.perf_counter()
    cells = float(sum(i.Nx * i.Nt for i in insts))
    sec = (t1 - t0) / steps
    info = bat.info()
    bat.close()
    del ws
    torch.cuda.empty_cache()
    # algorithmic HBM bytes of the march: per cell 16 B written and 16 B of the
    # delay row read, plus 32 B per strip cell of mirror reads
    hbm = float(sum(32.0 * (i.Nx + i.D) * i.Nt for i in insts))
    gbs = hbm / (tm / steps * 1e-3) / 1e9
    return {"instances": n, "seed": seed, "cells": cells, "s_per_step": sec, "cell_updates_per_s": cells / sec,
            "march_algorithmic_GBps": gbs, "march_hbm_frac": gbs / HBM_PEAK_GBS,
            "instances_per_s": n / sec, "march_ms": tm / steps, "boundary_ms": tb / steps,
            "march_cell_updates_per_s": cells / (tm / steps * 1e-3), "launches": info["launches"],
            "max_workgroups_per_launch": info["max_workgroups"],
            "autotune": {"tmax": best.tmax, "wmax": best.wmax, "groups": best.groups, "graph": bool(best.use_graph),
                         "probe_rate": rate, "seconds": t_tune},
            "ring_GB": sum((i.D + 2 * best.tmax + 2) * (i.Nx + 1) * 16 for i in insts) / 1e9}


def run_nm(steps: int, warmup: int, base_march_ms: float | None = None) -> dict:
    """The stimulated-emission instance on the large grid, marched with the
    non-Markovian measures of App. D: mu's row sums follow every march launch
    (k_mu_rows); mu(t_r) and lambda(t_r) for every row and N_geo are read into
    device memory after the march.  k_block does the same work as for the Gaussian
    on this grid (same plan), so the march time minus the Gaussian's is the
    cost of k_mu_rows: 16 B per cell of row r inside the photon field's
    support, columns j <= min(Nx, r + D), read once more from HBM."""
    import numpy as np
    import torch

    from paper_1707_05943_amd import fdtd
    from paper_1707_05943_amd import workloads as W

    inst = W.large_stimulated()
    dev = torch.device("cuda:0")
    sol = fdtd.Solver(inst, device=str(dev))
    stream = torch.cuda.current_stream(dev)
    mu_dev = torch.empty(2 * (inst.Nt + 1), dtype=torch.float64, device=dev)
    lam_dev = torch.empty(inst.Nt + 1, dtype=torch.float64, device=dev)
    ngeo_dev = torch.empty(1, dtype=torch.float64, device=dev)
    lib = sol.lib

    def step(ev=None):
        sol._check(lib.fdtd_set_boundary(sol.ctx))
        if ev is not None:
            ev[0].record(stream)
        sol._check(lib.fdtd_march(sol.ctx, inst.Nt))
        if ev is not None:
            ev[1].record(stream)
        sol._check(lib.fdtd_readout(sol.ctx, fdtd.RO_MU, 0, ctypes.c_void_p(mu_dev.data_ptr()), inst.Nt + 1, 1))
        sol._check(lib.fdtd_readout(sol.ctx, fdtd.RO_LAMBDA, 0, ctypes.c_void_p(lam_dev.data_ptr()),
                                    inst.Nt + 1, 1))
        sol._check(lib.fdtd_readout(sol.ctx, fdtd.RO_NGEO, inst.Nt, ctypes.c_void_p(ngeo_dev.data_ptr()), 1, 1))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    march_ms = sum(a.elapsed_time(b) for a, b in evs) / steps
    mu = mu_dev.view(-1, 2).cpu().numpy()
    lam = lam_dev.cpu().numpy()
    r = np.arange(1, inst.Nt + 1, dtype=np.float64)
    mu_bytes = 16.0 * float(np.sum(np.minimum(inst.Nx + 1, r + inst.D + 1)))
    out = {"workload": inst.name, "ms_per_step": ms_step, "march_ms": march_ms,
           "cell_updates_per_s": inst.Nx * inst.Nt / (ms_step * 1e-3),
           "mu_end": [float(mu[-1, 0]), float(mu[-1, 1])], "lambda_end": float(lam[-1]),
           "n_geo": float(ngeo_dev.cpu()[0]), "k_mu_rows_bytes_per_step": mu_bytes}
    if base_march_ms is not None and march_ms > base_march_ms:
        mu_ms = march_ms - base_march_ms
        out["mu_ms"] = mu_ms
        gbs = mu_bytes / (mu_ms * 1e-3) / 1e9
        out["k_mu_rows_achieved_GBps"] = gbs
        out["k_mu_rows_hbm_frac"] = gbs / HBM_PEAK_GBS
    sol.close()
    del sol
    torch.cuda.empty_cache()
    return out


def run_sweep(n_train: int, n_pts: int, n_sub: int, steps: int, tol: float = 1e-3) -> dict:
    """The learned part at its configurations.  Training: n_train seed-drawn
    instances of the batched sweep's distribution solved in FP64 by the
    batched solver (P_e and chi_out, 1024 samples each), then Adam on the
    network.  Sweep: n_pts points of the same distribution; the network's
    P_e for every point (input encoding and inference, timed); on a random
    subsample of n_sub points the a-posteriori check (FP64 solves on grids
    2x and 4x coarser, the check kernel) and the FP64 fallback of the points
    it rejects, timed, next to the plain batched solver on the same points,
    whose answers also audit every accepted point.  Rates of the full draw
    are the subsample's per-point costs (plus the full draw's measured
    inference per point) extrapolated; the method without the network (the
    coarse solve under the same check) is reported beside it."""
    import numpy as np
    import torch

    from paper_1707_05943_amd import surrogate as S
    from paper_1707_05943_amd import sweep as SW
    from paper_1707_05943_amd import workloads as W

    log = lambda m: print(m, file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    solver = SW.Solver()
    t0 = time.perf_counter()
    train_set = SW.draw(n_train, 101)
    x, t, m = SW.make_dataset(train_set, solver, chunk=512, log=log)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    train_cells = float(sum(i.Nx * i.Nt for i in train_set))
    net = SW.train(x, t, m, steps=steps, batch=32, lr=1e-3, log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del x, t, m, train_set
    torch.cuda.empty_cache()
    fl = S.gemm_flops(net.cfg)

    # the network on every point of the draw
    d = W.sweep_draw_arrays(n_pts, 202)
    ib = 512
    inet = S.Net(SW.surrogate_cfg(max_batch=ib), net.params, device=str(dev))
    pe_all = torch.empty(n_pts, SW.N_SAMPLES, dtype=torch.float64, device=dev)
    chunk = 8192
    x = torch.empty(chunk, SW.N_SAMPLES, SW.C_IN, dtype=torch.float32, device=dev)
    par = SW.params_from_arrays(d, 0, n_pts, dev)
    torch.cuda.synchronize()
    ti = time.perf_counter()
    for s0 in range(0, n_pts, chunk):
        nb = min(chunk, n_pts - s0)
        S.encode(par[s0:s0 + nb], SW.N_SAMPLES, x[:nb])
        pe_all[s0:s0 + nb] = SW.predict_pe(inet, x[:nb])
        if (s0 // chunk) % 32 == 0:
            log(f"[sweep] inference {s0 + nb}/{n_pts}")
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - ti
    inet.close()
    del x

    # the subsample: plain, the check, the fallbacks
    rng = np.random.default_rng(404)
    idx = np.sort(rng.choice(n_pts, size=min(n_sub, n_pts), replace=False))
    sub = [SW.box(W.sweep_point(d, int(i))) for i in idx]
    cells_sub = float(sum(i.Nx * i.Nt for i in sub))
    torch.cuda.synchronize()
    ta = time.perf_counter()
    plain = torch.cat([solver.solve(sub[s0:s0 + 512], with_chi=False)[0] for s0 in range(0, len(sub), 512)])
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - ta
    log(f"[sweep] plain: {len(sub)} points in {t_plain:.1f} s")
    out_s, out_c, acc, de, info = SW.sweep(sub, net, solver, tol=tol, log=log)
    e_s = SW.rel_err(out_s, plain).cpu().numpy()
    e_c = SW.rel_err(out_c, plain).cpu().numpy()
    a_s, a_c = acc[:, 0].cpu().numpy(), acc[:, 1].cpu().numpy()
    e_net = SW.rel_err(pe_all[torch.from_numpy(idx).to(dev)], plain).cpu().numpy()
    e_p2 = SW.rel_err(info["p2"], plain).cpu().numpy()
    est = de[:, 1].cpu().numpy()
    ok2 = np.isfinite(est)
    ns = len(sub)
    c_plain = t_plain / ns
    c_check = info["check_s"] / ns
    c_net = t_inf / n_pts + c_check + info["fallback_network_path_s"] / ns
    c_coarse = c_check + info["fallback_coarse_path_s"] / ns
    solver.ws = None
    del pe_all
    torch.cuda.empty_cache()
    q = lambda v, p: float(np.quantile(v, p)) if v.size else None
    return {
        "tol": tol, "safety": SW.SAFETY,
        "training": {"instances": n_train, "seed": 101, "cells": train_cells, "data_s": t1 - t0,
                     "data_cell_updates_per_s": train_cells / (t1 - t0), "steps": steps, "batch": 32,
                     "train_s": t2 - t1, "ms_per_step": (t2 - t1) / steps * 1e3,
                     "gemm_flops_per_sample": {"forward": fl[0], "backward": fl[1]},
                     "gemm_TFLOPs": (fl[0] + fl[1]) * 32 * steps / (t2 - t1) / 1e12,
                     "frac_of_bf16_mfma_peak": (fl[0] + fl[1]) * 32 * steps / (t2 - t1) / 1e12 / BF16_PEAK_TFLOPS},
        "draw": {"points": n_pts, "seed": 202, "subsample": ns, "subsample_seed": 404,
                 "mean_cells_per_point": float(np.mean(d["Nx"] * d["Nt"]))},
        "inference": {"points": n_pts, "s": t_inf, "points_per_s": n_pts / t_inf, "batch": ib,
                      "gemm_TFLOPs": fl[0] * n_pts / t_inf / 1e12,
                      "frac_of_bf16_mfma_peak": fl[0] * n_pts / t_inf / 1e12 / BF16_PEAK_TFLOPS},
        "points_per_s": {"plain": 1.0 / c_plain, "network_with_check": 1.0 / c_net,
                         "coarse_with_check": 1.0 / c_coarse, "network_alone_unchecked": n_pts / t_inf},
        "extrapolated_s_for_draw": {"plain": c_plain * n_pts, "network_with_check": c_net * n_pts,
                                    "coarse_with_check": c_coarse * n_pts},
        "subsample_s": {"plain": t_plain, "check": info["check_s"],
                        "fallback_network_path": info["fallback_network_path_s"],
                        "fallback_coarse_path": info["fallback_coarse_path_s"],
                        "inference_of_subsample": info["inference_s"]},
        "accepted": {"network": int(a_s.sum()), "coarse": int(a_c.sum()),
                     "network_not_coarse": int((a_s & ~a_c).sum())},
        "audit": {"accepted_network_true_err_above_tol": int(((e_s > tol) & a_s).sum()),
                  "accepted_coarse_true_err_above_tol": int(((e_c > tol) & a_c).sum()),
                  "audited_points": ns, "max_err_network_path": float(e_s.max()),
                  "max_err_coarse_path": float(e_c.max()),
                  "estimate_covers_coarse_error": float(np.mean(est[ok2] >= e_p2[ok2])) if ok2.any() else None},
        "errors_vs_fp64": {"network_median": q(e_net, 0.5), "network_p10": q(e_net, 0.1),
                           "network_within_tol": float(np.mean(e_net <= tol)),
                           "coarse2x_median": q(e_p2[ok2], 0.5), "coarse2x_within_tol": float(np.mean(e_p2[ok2] <= tol))},
        "reason": ("the check bounds the network's error by its distance to the 2x-coarser FP64 solve plus that "
                   "solve's own estimated error, so every point it accepts is one the coarse solve alone passes "
                   "too: the network adds inference to the coarse path and cannot raise its acceptance"),
    }


def run_single(inst, steps: int, warmup: int) -> dict:
    """One instance: a step is the boundary tables, the march of every row,
    and P_e of every row and chi at 1024 detector separations into device
    memory.  Events on the march's stream bracket the boundary and the march."""
    import numpy as np
    import torch

    from paper_1707_05943_amd import fdtd
    dev = torch.device("cuda:0")
    sol = fdtd.Solver(inst, device=str(dev))
    stream = torch.cuda.current_stream(dev)
    n_tau = 1024
    pe_dev = torch.empty(inst.Nt + 1, dtype=torch.float64, device=dev)
    chi_dev = torch.empty(2 * n_tau, dtype=torch.float64, device=dev)
    lib = sol.lib

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        sol._check(lib.fdtd_set_boundary(sol.ctx))
        if ev is not None:
            ev[1].record(stream)
        sol._check(lib.fdtd_march(sol.ctx, inst.Nt))
        if ev is not None:
            ev[2].record(stream)
        sol._check(lib.fdtd_readout(sol.ctx, fdtd.RO_PE, 0, ctypes.c_void_p(pe_dev.data_ptr()),
                                    inst.Nt + 1, 1))
        sol._check(lib.fdtd_readout(sol.ctx, fdtd.RO_CHI, 0, ctypes.c_void_p(chi_dev.data_ptr()),
                                    min(n_tau, inst.Nx - inst.D), 1))

    print(f"[bench] {inst.name}: warmup {warmup}", file=sys.stderr, flush=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    print(f"[bench] {inst.name}: timing {steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sol.sync()                                   # reports a non-finite value in the march
    ms_step = (t1 - t0) * 1e3 / steps
    boundary_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / steps
    march_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / steps
    # the march kernel (k_block): one launch per block of T rows plus one to
    # start the strip a block ahead; algorithmic bytes per launch are
    # 32 (Nx + D) T: per cell 16 B written and 16 B of the delay row read,
    # plus 32 B per strip cell for the mirror reads
    plan = fdtd.describe(inst)
    T = plan["T"]
    launches = (inst.Nt + T - 1) // T + 1
    bytes_per_launch = 32.0 * (inst.Nx + inst.D) * T
    avg_launch_s = march_ms * 1e-3 / launches
    pe = pe_dev.cpu().numpy()
    sol.close()
    del sol
    torch.cuda.empty_cache()
    return {"ms_per_step": ms_step, "march_ms": march_ms, "boundary_ms": boundary_ms, "plan": plan,
            "launches": launches, "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_launch_s * 1e6,
            "march_algorithmic_GBps": bytes_per_launch / avg_launch_s / 1e9, "pe_max": float(np.max(pe)),
            "ring_GB": plan["ring_rows"] * (inst.Nx + 1) * 16 / 1e9}


def copy_peak(traffic_bytes: float) -> dict:
    """The HBM bandwidth a plain copy attains: the library's streaming copy
    (fdtd_stream_copy) of half the given traffic each way, best of three."""
    import torch

    from paper_1707_05943_amd import fdtd
    n = int(traffic_bytes / 2) // 16 * 16
    src = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    best = float("inf")
    s = torch.cuda.current_stream()
    for _ in range(4):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fdtd.stream_copy(dst, src)
        b.record(s)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": 2.0 * n / (best * 1e-3) / 1e9,
            "note": f"library streaming copy of {n / 1e9:.1f} GB each way ({2 * n / 1e9:.1f} GB of traffic), "
                    f"best of 4: {best:.2f} ms"}


def host_cpu() -> dict:
    """The host the oracle ran on: cores visible to the process and the CPU model (lscpu)."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                             "CPU max MHz"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    return info


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is "
              "designed (column blocks per GPU, halos over xGMI) but not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1707_05943_amd import fdtd
    from paper_1707_05943_amd import workloads as W

    if args.workload == "nm":
        nm = run_nm(args.steps, args.warmup)
        print(json.dumps({"metric": METRIC, "value": nm["cell_updates_per_s"], "unit": "cell-updates/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": nm["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": nm["workload"]}, "nm": nm}), flush=True)
        return

    if args.workload == "sweep":
        sw = run_sweep(args.sweep_train, args.sweep_points, args.sweep_sub, args.sweep_steps)
        pps = sw["points_per_s"]
        print(json.dumps({"metric": METRIC, "value": pps["network_with_check"],
                          "unit": "points/s", "n_gpus": 1, "steps": 1, "warmup": 0,
                          "ms_per_step": sw["extrapolated_s_for_draw"]["network_with_check"] * 1e3,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": f"sweep of {args.sweep_points} points"},
                          "sweep": sw}), flush=True)
        return

    if args.workload == "batch":
        b = run_batch(args.batch, args.batch_seed, args.steps, args.warmup)
        print(json.dumps({"metric": METRIC, "value": b["cell_updates_per_s"], "unit": "cell-updates/s",
                          "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "ms_per_step": b["s_per_step"] * 1e3, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": f"batched sweep of {args.batch} instances"}, "batch": b}),
              flush=True)
        return

    inst = W.large_gauss() if args.workload == "large" else W.small_gauss()
    one = run_single(inst, args.steps, args.warmup)
    ms_step = one["ms_per_step"]
    cells = inst.Nx * inst.Nt
    value = cells / (ms_step * 1e-3)
    achieved = one["march_algorithmic_GBps"]
    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": inst.name, "D": inst.D, "Nx": inst.Nx, "Nt": inst.Nt, "Delta": inst.Delta,
                   "incident": "gaussian two-photon", "ring_GB": one["ring_GB"],
                   "march_ms": one["march_ms"], "boundary_ms": one["boundary_ms"], "pe_max": one["pe_max"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "k_block", "bytes_per_launch": one["bytes_per_launch"],
                     "avg_launch_us": one["avg_launch_us"], "launches_per_step": one["launches"],
                     "plan": one["plan"]},
    }
    import torch
    torch.cuda.empty_cache()
    try:
        cp = copy_peak(one["ring_GB"] * 1e9)
        out["roofline"]["copy_peak_GBps"] = cp["GBps"]
        out["roofline"]["frac_of_copy_peak"] = achieved / cp["GBps"]
        out["roofline"]["copy_peak_note"] = cp["note"]
    except Exception as e:                                  # the headline line is printed regardless
        out["roofline"]["copy_peak_GBps"] = None
        out["roofline"]["copy_peak_note"] = f"{type(e).__name__}: {e}"
    if args.workload == "large" and not args.no_c0:
        print("[bench] D=100, Nx=4000, Nt=4000 instance", file=sys.stderr, flush=True)
        try:
            c0 = W.small_gauss()
            r0 = run_single(c0, max(args.steps, 3), max(args.warmup, 1))
            out["c0"] = {"workload": c0.name, "ms_per_step": r0["ms_per_step"],
                         "cell_updates_per_s": c0.Nx * c0.Nt / (r0["ms_per_step"] * 1e-3),
                         "march_ms": r0["march_ms"], "boundary_ms": r0["boundary_ms"],
                         "boundary_share": r0["boundary_ms"] / r0["ms_per_step"],
                         "avg_launch_us": r0["avg_launch_us"], "launches": r0["launches"],
                         "note": "ring of 11 MB: cache-resident, the march is latency-bound by construction"}
        except Exception as e:
            out["c0"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_rows)
    if args.workload == "large" and not args.no_nm:
        print("[bench] stimulated emission with the measures of App. D", file=sys.stderr, flush=True)
        try:
            out["nm"] = run_nm(args.steps, args.warmup, one["march_ms"])
        except Exception as e:
            out["nm"] = {"error": f"{type(e).__name__}: {e}"}
    if args.workload == "large" and not args.no_batch:
        print(f"[bench] batched sweep of {args.batch} instances", file=sys.stderr, flush=True)
        try:
            out["batch"] = run_batch(args.batch, args.batch_seed, max(1, args.steps - 1), 1)
        except Exception as e:                                  # the headline line is printed regardless
            out["batch"] = {"error": f"{type(e).__name__}: {e}"}
    if args.workload == "large" and not args.no_sweep:
        print("[bench] surrogate sweep", file=sys.stderr, flush=True)
        try:
            out["sweep"] = run_sweep(args.sweep_train, args.sweep_points, args.sweep_sub, args.sweep_steps)
        except Exception as e:
            out["sweep"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
