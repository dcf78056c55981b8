"""GPU parity of the batched march: many heterogeneous instances in one
launch sequence, against the CPU oracle per instance, with and without the
captured HIP graph, and after the autotuner's choice."""
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


def _gauss(D, Nx, Nt, Delta, width, seed, k0a=0.5 * math.pi, x0w=6.0):
    inst = W.tiny_gauss(D=D, Nx=Nx, Nt=Nt, Delta=Delta, width=width, seed=seed, k0a=k0a)
    inst.x0 = -inst.a - x0w * width
    return inst


def batch_cases():
    """different D (and so different rows per block), widths, lengths and
    families; the instances finish after different numbers of launches; the
    boundary of every other instance comes from the delay equation (one
    batched launch for those), the rest from the delay series"""
    cases = [
        _gauss(10, 2600, 300, 0.02, 0.5, 31),                 # T = 8, several workgroups
        _gauss(40, 1025, 200, 0.025, 0.6, 32),                # T = 32
        _gauss(2, 3, 50, 0.1, 0.4, 33),                       # Nx = D + 1, T = 2
        _gauss(1200, 3100, 1400, 0.0025, 0.5, 34),            # strip wider than a workgroup
        _gauss(24, 700, 900, 0.02, 0.7, 35, k0a=2.0),         # longest march
        W.Instance(name="exp2_b", Nx=1500, D=24, Nt=400, Delta=0.02, omega0=2.0, Gamma=1.0,
                   incident=W.INC_EXP2, k=2.3, alpha=0.8, x0=0.0, width=1.0, phase=0.9),
        W.Instance(name="coarse_b", Nx=1500, D=24, Nt=300, Delta=0.5, omega0=4.5, Gamma=1.0,
                   incident=W.INC_GAUSS2, k=4.5, x0=-6.0 - 8 * 3.0, width=3.0, phase=0.3),
    ]
    for i, c in enumerate(cases):
        c.boundary = i % 2
    return cases


def _oracle(inst):
    """the oracle's run of `inst` with the row at the peak of P_e kept: rows
    that have decayed below 1% of that row are measured against 1% of it
    (their own rounding noise, ~1e-16 of the peak per row, is what remains)"""
    E = oracle.E_table(inst)
    pre = oracle.march(inst, E, want_ring=False)["pe"]
    rp = int(np.argmax(pre)) if np.all(np.isfinite(pre)) else inst.Nt // 2
    ref = oracle.march(inst, E, snap_rows=[max(1, rp)])
    ref["scale"] = max([np.linalg.norm(ref["snaps"][0])] + [np.linalg.norm(v) for v in ref["ring"]])
    return ref


def _compare_instance(bat, i, inst, ref, label):
    """last D+2 rows and P_e of instance i against the oracle run `ref`"""
    scale = ref["scale"]
    R = inst.D + 2
    worst = own = 0.0
    for q in range(R):
        rho = inst.Nt - (R - 1) + q
        if rho < 0:
            continue
        got = bat.row_values(i, rho)
        d, n = np.linalg.norm(got - ref["ring"][q]), np.linalg.norm(ref["ring"][q])
        e = d / max(n, FLOOR * scale, 1e-300)
        worst = max(worst, e)
        own = max(own, d / n if n > 0 else 0.0)
        assert e <= TOL, (label, inst.name, "row", rho, e)
    if inst.incident != W.INC_PLANE:
        pe = bat.pe(i)
        e = np.linalg.norm(pe - ref["pe"]) / np.linalg.norm(ref["pe"])
        assert e <= TOL, (label, inst.name, "P_e", e)
        worst = max(worst, e)
    _say(f"[batch] {label} {inst.name}: worst row error against its own norm {own:.2e}")
    return worst


@pytest.fixture(scope="module")
def oracle_runs():
    cases = batch_cases()
    return cases, [_oracle(inst) for inst in cases]


@pytest.mark.parametrize("use_graph,groups", [(False, 1), (True, 1), (False, 2), (True, 2)])
def test_batch_vs_oracle(oracle_runs, use_graph, groups):
    cases, refs = oracle_runs
    _say(f"[batch] {len(cases)} instances, graph={use_graph}, groups={groups}")
    bat = fdtd.Batch(cases, fdtd.batch_opts(use_graph=use_graph, groups=groups)).set_boundary().march()
    _say(f"[batch] launches {bat.info()}")
    for i, inst in enumerate(cases):
        w = _compare_instance(bat, i, inst, refs[i], f"graph={use_graph} groups={groups}")
        _say(f"[batch] {inst.name}: worst {w:.2e}")
    bat.close()


@pytest.mark.parametrize("groups", [2, 4])
def test_groups_match_one_group(groups):
    """groups on their own streams run the same kernels on the same instances:
    rows, P_e and the chi snapshots (taken per group) are bitwise those of one
    group, over graph replays with other device work in between"""
    import torch
    cases = batch_cases()
    n_tau = 24
    rows = [max(1, inst.Nt // 2) for inst in cases]
    rows[1] = -1
    strides = [1 + (i % 2) for i in range(len(cases))]

    def run(groups, reps):
        out = torch.zeros(len(cases), n_tau, dtype=torch.complex128, device="cuda:0")
        bat = fdtd.Batch(cases, fdtd.batch_opts(use_graph=True, groups=groups))
        bat.set_chi(rows, strides, n_tau, out)
        res = []
        x = torch.ones(1 << 18, dtype=torch.float64, device="cuda:0")
        for rep in range(reps):
            _say(f"[batch] groups={groups} replay {rep}")
            bat.set_boundary().march()
            x = x * 1.0001 + 1.0
            torch.cuda.synchronize()
            res.append(([bat.pe(i) for i in range(len(cases))],
                        [bat.row_values(i, cases[i].Nt) for i in range(len(cases))], out.cpu().numpy().copy()))
        _say(f"[batch] groups={groups}: launches, workgroups {bat.info()}")
        bat.close()
        return res

    want = run(1, 1)[0]
    for rep, got in enumerate(run(groups, 3)):
        for i in range(len(cases)):
            assert np.array_equal(got[0][i], want[0][i]), (rep, i, "P_e")
            assert np.array_equal(got[1][i], want[1][i]), (rep, i, "row")
        assert np.array_equal(got[2], want[2]), (rep, "chi")
    assert np.abs(want[2]).max() > 0


def test_graph_replays_match_plain_launches():
    """the captured graph, replayed several times with other device work and
    synchronisations in between, gives bitwise the plain launches' result"""
    import torch
    cases = batch_cases()
    plain = fdtd.Batch(cases, fdtd.batch_opts(use_graph=False)).set_boundary().march()
    want = [(plain.pe(i), plain.row_values(i, cases[i].Nt)) for i in range(len(cases))]
    plain.close()
    g = fdtd.Batch(cases, fdtd.batch_opts(use_graph=True))
    x = torch.ones(1 << 20, dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        _say(f"[batch] graph replay {rep}")
        g.set_boundary().march()
        x = x * 1.0001 + 1.0            # unrelated eager work on the same device
        torch.cuda.synchronize()
        for i in range(len(cases)):
            assert np.array_equal(g.pe(i), want[i][0]), (rep, i)
            assert np.array_equal(g.row_values(i, cases[i].Nt), want[i][1]), (rep, i)
    g.close()


def test_batch_matches_single_instance_march():
    """the batch's wider workgroups change only the truncation of the
    within-row recurrence, far below the parity bar"""
    cases = batch_cases()[:3]
    bat = fdtd.Batch(cases).set_boundary().march()
    for i, inst in enumerate(cases):
        one = fdtd.Solver(inst).set_boundary().march(inst.Nt)
        a, b = bat.row_values(i, inst.Nt), one.row_values(inst.Nt)
        assert np.linalg.norm(a - b) <= 1e-13 * max(np.linalg.norm(b), 1e-300), inst.name
        assert np.linalg.norm(bat.pe(i) - one.pe()) <= 1e-13 * np.linalg.norm(one.pe())
        one.close()
    bat.close()


def test_autotune_then_parity(oracle_runs):
    cases, refs = oracle_runs
    best, rate = fdtd.autotune(cases, probe_rows=64)
    _say(f"[batch] autotune: tmax={best.tmax} wmax={best.wmax} graph={best.use_graph} rate={rate:.3g}")
    assert best.use_graph == 1 and best.tmax in (8, 16, 32) and best.wmax in (768, 1536) and rate > 0
    bat = fdtd.Batch(cases, best).set_boundary().march()
    for i, inst in enumerate(cases):
        _compare_instance(bat, i, inst, refs[i], "autotuned")
    bat.close()


def test_batch_state_errors():
    cases = batch_cases()[:2]
    bat = fdtd.Batch(cases)
    with pytest.raises(fdtd.FdtdError) as e:
        bat.march()                            # before the boundary
    assert e.value.code == -3
    bat.set_boundary().march()
    with pytest.raises(fdtd.FdtdError) as e:
        bat.march()                            # twice without a new boundary
    assert e.value.code == -3
    with pytest.raises(fdtd.FdtdError) as e:
        bat.pe(5)                              # no such instance
    assert e.value.code == -1
    bat.close()


def test_chi_snapshots_and_pe_samples(oracle_runs):
    """chi taken during the (graph-captured) batched march at a row of each
    instance, with a detector stride, and P_e sampled on a fixed grid of each
    instance's window, against the oracle"""
    import torch
    cases = batch_cases()
    n_tau, ns = 40, 257
    # at the peak of P_e, where the field is alive
    rows = [max(1, int(np.argmax(oracle_runs[1][i]["pe"]))) for i in range(len(cases))]
    rows[2] = -1                                             # no snapshot for this one
    strides = [1 + (i % 3) for i in range(len(cases))]
    out = torch.zeros(len(cases), n_tau, dtype=torch.complex128, device="cuda:0")
    pes = torch.zeros(len(cases), ns, dtype=torch.float64, device="cuda:0")
    bat = fdtd.Batch(cases, fdtd.batch_opts(use_graph=True))
    bat.set_chi(rows, strides, n_tau, out)
    for rep in range(2):                                     # the graph replays the snapshots too
        bat.set_boundary().march()
        bat.sample_pe(ns, pes)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        got_pe = pes.cpu().numpy()
        for i, inst in enumerate(cases):
            ref_pe = oracle_runs[1][i]["pe"]
            pos = np.arange(ns) * inst.Nt / (ns - 1)
            want_pe = np.interp(pos, np.arange(inst.Nt + 1), ref_pe)
            if inst.incident != W.INC_PLANE:
                e = np.linalg.norm(got_pe[i] - want_pe) / np.linalg.norm(want_pe)
                assert e <= TOL, (rep, inst.name, "P_e samples", e)
            if rows[i] < 0:
                assert np.all(got[i] == 0)
                continue
            navail = min(n_tau * strides[i], inst.Nx - inst.D)
            ref = oracle.march(inst, oracle.E_table(inst), chi_rows=[rows[i]], n_tau=navail, want_ring=False)
            want = np.zeros(n_tau, dtype=complex)
            sel = np.arange(n_tau) * strides[i]
            ok = sel < navail
            want[ok] = ref["chi"][0][sel[ok]]
            e = np.linalg.norm(got[i] - want) / max(np.linalg.norm(want), 1e-300)
            _say(f"[batch] chi snapshot {inst.name} row {rows[i]} stride {strides[i]}: {e:.2e}")
            assert e <= TOL, (rep, inst.name, "chi", e)
    bat.close()


def test_batch_lambda_of_stimulated_emission():
    """lambda(t_r) of App. D for stimulated-emission instances of a batch
    (series and delay-equation boundaries) against the oracle; batches keep
    mu of row 0 only."""
    from oracle import nm
    exp1 = dict(Nx=1500, D=24, Nt=400, Delta=0.02, omega0=2.0, Gamma=1.5, incident=W.INC_EXP1, k=2.3, alpha=0.5)
    cases = [W.Instance(name="exp1_series", **exp1), _gauss(10, 2600, 300, 0.02, 0.5, 36),
             W.Instance(name="exp1_ode", **dict(exp1, D=40, Nt=520))]
    cases[2].boundary = 1
    _say("[batch] lambda of stimulated emission")
    bat = fdtd.Batch(cases).set_boundary().march()
    for i in (0, 2):
        inst = cases[i]
        ref = nm.measures(inst, range(inst.Nt + 1))
        lam = bat.lam(i)
        e = np.linalg.norm(lam - ref["lambda"]) / np.linalg.norm(ref["lambda"])
        assert e <= TOL, (inst.name, e)
        assert abs(bat.mu(i, 1)[0] - ref["mu"][0]) <= TOL
        with pytest.raises(fdtd.FdtdError) as err:
            bat.mu(i, 2)
        assert err.value.code == -3
    with pytest.raises(fdtd.FdtdError) as err:
        bat.lam(1)
    assert err.value.code == -1
    bat.close()


# Instances of the 512-instance sweep draw (seed 7) checked inside the full,
# autotuned batch, as the benchmark runs it: (index, rows compared).  The
# oracle's E (direct quadrature of the delay series) costs O(Nt^2 / D), so
# the extremes with long windows are compared on a row prefix (P_e and E of
# rows 0..prefix depend on nothing later); two mid-range instances in full
# (their last D+2 rows as well).
SWEEP_PICKS = [
    (205, 1024),        # smallest D (18), Nx 1024, boundary over 57 round trips
    (144, 2048),        # largest |alpha| (0.084): the recurrence's longest horizon
    (179, 2 * 4960 + 600),   # largest D (4960), Nx 16384: the widest instance
    (139, 2 * 4084 + 600),   # largest D/Nx (0.4985)
    (300, None),        # D 894, Nx 2048, Nt 8192: in full
    (100, None),        # D 942, Nx 4096, Nt 16384: in full
]


def test_sweep_draw_instances_in_the_full_batch():
    """The benchmark's batched sweep -- 512 seed-drawn instances, autotuned
    tiles, one captured graph -- and six of its instances against the oracle
    (the batch's E comes from the delay equation, the oracle's from the
    quadrature of the delay series)."""
    import torch
    insts = W.sweep_draw(512, 7)
    refs = {}
    for k, prefix in SWEEP_PICKS:
        inst = insts[k]
        ref_inst = inst if prefix is None else W.with_sizes(inst, Nt=prefix)
        _say(f"[batch] oracle for sweep instance {k}: D={inst.D} Nx={inst.Nx} Nt={inst.Nt} rows {ref_inst.Nt}")
        refs[k] = (ref_inst, _oracle(ref_inst) if prefix is None else
                   oracle.march(ref_inst, oracle.E_table(ref_inst), want_ring=False))
    dev = torch.device("cuda:0")
    need = max(fdtd.batch_workspace_size(insts, fdtd.batch_opts(t, w)) for t in (32, 16, 8) for w in (0, 768))
    _say(f"[batch] autotune over the 512 instances ({need / 1e9:.0f} GB workspace)")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    best, rate = fdtd.autotune(insts, probe_rows=256, workspace=ws)
    _say(f"[batch] autotuned tmax={best.tmax} wmax={best.wmax}; marching the batch")
    bat = fdtd.Batch(insts, best, workspace=ws).set_boundary().march()
    bat.sync()
    for k, prefix in SWEEP_PICKS:
        inst = insts[k]
        ref_inst, ref = refs[k]
        n = ref_inst.Nt + 1
        c = math.sqrt(2.0) * np.exp(1j * inst.phase)
        got_E = bat.E(k)[:n] / c
        eE = np.max(np.abs(got_E - ref["E"])) / np.max(np.abs(ref["E"]))
        pe = bat.pe(k)[:n]
        ePe = np.linalg.norm(pe - ref["pe"]) / np.linalg.norm(ref["pe"])
        _say(f"[batch] sweep instance {k}: E {eE:.2e}, P_e over rows 0..{n - 1} {ePe:.2e}")
        assert eE <= TOL and ePe <= TOL, (k, eE, ePe)
        if prefix is None:
            w = _compare_instance(bat, k, inst, ref, "sweep draw")
            assert w <= TOL
    bat.close()
    del ws
    torch.cuda.empty_cache()


def test_one_instance_batch_with_more_groups_than_instances():
    """a batch of one instance asked for four groups marches as one group and
    gives bitwise the single-group batch"""
    inst = batch_cases()[0]
    one = fdtd.Batch([inst], fdtd.batch_opts(groups=1)).set_boundary().march()
    four = fdtd.Batch([inst], fdtd.batch_opts(groups=4)).set_boundary().march()
    assert four.info() == one.info()
    assert np.array_equal(four.pe(0), one.pe(0))
    assert np.array_equal(four.row_values(0, inst.Nt), one.row_values(0, inst.Nt))
    one.close()
    four.close()

