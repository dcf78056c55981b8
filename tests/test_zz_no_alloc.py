"""The allocation-free entry point (fdtd_solve_noalloc) against the
allocating one (fdtd_init + fdtd_set_boundary + fdtd_march + readouts into
device memory): same kernels, so the same values bit for bit.  Two calls in a
row share the library's device array, the second with a smaller instance; a
third instance that does not fit is refused before anything is enqueued."""
import sys

import numpy as np
import pytest

from paper_1707_05943_amd import fdtd
from paper_1707_05943_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cases():
    big = W.with_sizes(W.small_gauss(), Nt=1500)          # D=100, Nx=4000: about 16 MB of workspace
    small = W.tiny_gauss(D=10, Nx=1500, Nt=240, Delta=0.05, width=0.5, seed=21)
    small.x0 = -small.a - 6 * small.width
    stim = W.Instance(name="stim_small", Nx=1200, D=24, Nt=500, Delta=0.02, omega0=2.0, Gamma=1.5,
                      incident=W.INC_EXP1, k=2.3, alpha=0.5)
    return [(big, 1500), (small, 240), (stim, 333)]


def _reference(inst, n_rows):
    sol = fdtd.Solver(inst).set_boundary()
    sol.march(n_rows)
    pe, row = sol.pe(n_rows + 1), sol.row_values(n_rows)
    sol.close()
    return pe, row


def test_noalloc_matches_the_allocating_entry_points():
    import torch
    dev = torch.device("cuda:0")
    cases = _cases()
    for inst, _ in cases:
        assert fdtd.workspace_size(inst) <= fdtd.NOALLOC_MAX_BYTES
    refs = []
    for inst, n in cases:
        _say(f"[noalloc] reference (allocating path): {inst.name} D={inst.D} Nx={inst.Nx} rows={n}")
        refs.append(_reference(inst, n))
    # consecutive calls, each on the array the previous one left behind
    for (inst, n), (pe_ref, row_ref) in zip(cases, refs):
        _say(f"[noalloc] fdtd_solve_noalloc: {inst.name} rows={n}")
        pe = torch.full((n + 1,), float("nan"), dtype=torch.float64, device=dev)
        row = torch.full((2 * (inst.Nx + 1),), float("nan"), dtype=torch.float64, device=dev)
        fdtd.solve_noalloc(inst, n, pe, row)
        torch.cuda.synchronize()
        got_pe = pe.cpu().numpy()
        got_row = row.cpu().numpy().view(np.complex128)
        assert np.array_equal(got_pe, pe_ref), (inst.name, np.max(np.abs(got_pe - pe_ref)))
        assert np.array_equal(got_row, row_ref), (inst.name, np.max(np.abs(got_row - row_ref)))
        assert np.isfinite(got_pe).all() and np.max(np.abs(got_row)) > 0


def test_noalloc_refuses_what_does_not_fit():
    big = W.large_gauss()
    assert fdtd.workspace_size(big) > fdtd.NOALLOC_MAX_BYTES
    with pytest.raises(fdtd.FdtdError) as e:
        fdtd.solve_noalloc(big, 10)
    assert e.value.code == -2 and "allocation-free" in str(e.value)
    with pytest.raises(fdtd.FdtdError) as e:
        fdtd.solve_noalloc(_cases()[1][0], 10**6)
    assert e.value.code == -1
