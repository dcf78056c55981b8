"""GPU checks of the surrogate network: the bf16 matrix-core product against
float64 products of the same bf16-rounded operands, and the network's
forward pass, gradients, loss and Adam step against the float64 CPU
reference (oracle/fno_ref.py) on the same seeded parameters and inputs.

Tolerances.  The products round their operands to bf16 (unit roundoff
u = 2^-9): a single product carries a relative error of about u, and a
forward pass chains about a dozen of them, so the network's outputs and
gradients are compared in relative L2 with bars of 2e-2 and 5e-2.  The bare
product, fed operands already rounded the same way, is exact up to fp32
accumulation (K 2^-24 relative to sum |a b|).
"""
import sys

import numpy as np
import pytest

from oracle import fno_ref as F
from paper_1707_05943_amd import sur_inputs as SI
from paper_1707_05943_amd import surrogate as S

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def bf16_round(a):
    """round fp32 to the nearest bf16 (ties to even), kept in fp32"""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (100, 70, 45), (1, 3, 7), (130, 129, 257)])
@pytest.mark.parametrize("tA,tB", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_layouts(M, N, K, tA, tB):
    import torch
    rng = np.random.Generator(np.random.PCG64(M * 1000 + N * 10 + K + 7 * tA + 3 * tB))
    batch = 3
    A = rng.standard_normal((batch, K, M) if tA else (batch, M, K)).astype(np.float32)
    B = rng.standard_normal((batch, N, K) if tB else (batch, K, N)).astype(np.float32)
    C0 = rng.standard_normal((batch, M, N)).astype(np.float32)
    alpha, beta = 1.3, 0.7
    dA, dB, dC = (torch.from_numpy(v).cuda() for v in (A, B, C0))
    S.gemm(dA, dB, dC, transA=tA, transB=tB, alpha=alpha, beta=beta, M=M, N=N, K=K, lda=A.shape[2],
           ldb=B.shape[2], ldc=N, sA=A[0].size, sB=B[0].size, sC=M * N, batch=batch)
    got = dC.cpu().numpy()
    Ar, Br = bf16_round(A).astype(np.float64), bf16_round(B).astype(np.float64)
    opA = np.transpose(Ar, (0, 2, 1)) if tA else Ar
    opB = np.transpose(Br, (0, 2, 1)) if tB else Br
    want = alpha * (opA @ opB) + beta * C0.astype(np.float64)
    scale = alpha * (np.abs(opA) @ np.abs(opB)) + beta * np.abs(C0)
    err = np.max(np.abs(got - want) / (scale + 1e-30))
    assert err <= (K + 2) * 2.0 ** -23, err


SMALL = {"n_points": 64, "c_in": 7, "width": 16, "modes": 8, "layers": 2, "proj": 32, "c_out": 3}
FULL = {"n_points": 1024, "c_in": 7, "width": 64, "modes": 64, "layers": 4, "proj": 128, "c_out": 3}


def _theta(cfg, seed):
    theta = SI.init_params(cfg, seed)
    # spectral weights large enough that the Fourier path matters in the check
    lay = F.layout(cfg)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    for k in ("Rr", "Ri"):
        o, s = lay[k]
        theta[o:o + int(np.prod(s))] = (rng.standard_normal(int(np.prod(s))) / cfg["width"]).astype(np.float32)
    return theta


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("cfg,B", [(SMALL, 3), (FULL, 2)])
def test_forward_and_gradients_match_reference(cfg, B):
    import torch
    theta = _theta(cfg, 11)
    x, t, mask, wo = SI.random_batch(cfg, B, 12)
    c = S.cfg(max_batch=B, **cfg)
    net = S.Net(c, torch.from_numpy(theta).cuda())
    dx, dt, dm, dw = (torch.from_numpy(v).cuda() for v in (x, t, mask, wo))
    y = net.forward(dx)
    loss, dy = net.loss(y, dt, dw, dm)
    g = net.backward(dx, dy).cpu().numpy()
    torch.cuda.synchronize()
    yr, cache = F.forward(cfg, theta.astype(np.float64), x.astype(np.float64))
    lr, dyr = F.loss(yr, t.astype(np.float64), wo.astype(np.float64), mask.astype(np.float64))
    gr = F.backward(cfg, theta.astype(np.float64), x.astype(np.float64), cache, dyr)
    ey = _rel(y.cpu().numpy(), yr)
    el = abs(float(loss.cpu()[0]) - lr) / lr
    _say(f"[surrogate] n={cfg['n_points']} forward rel-L2 {ey:.2e}, loss {el:.2e}")
    assert ey <= 2e-2 and el <= 2e-2
    lay = F.layout(cfg)
    for name, (o, s) in ((k, v) for k, v in lay.items() if k != "_n"):
        n = int(np.prod(s))
        e = _rel(g[o:o + n], gr[o:o + n])
        _say(f"[surrogate]   grad {name}: rel-L2 {e:.2e}")
        assert e <= 5e-2, (name, e)
    net.close()


def test_backward_needs_matching_forward():
    import torch
    c = S.cfg(max_batch=4, **SMALL)
    net = S.Net(c, torch.from_numpy(_theta(SMALL, 3)).cuda())
    x = torch.zeros(2, SMALL["n_points"], SMALL["c_in"], device="cuda")
    dy = torch.zeros(2, SMALL["n_points"], SMALL["c_out"], device="cuda")
    with pytest.raises(S.SurError) as e:
        net.backward(x, dy)
    assert e.value.code == -3
    with pytest.raises(S.SurError):
        net.forward(torch.zeros(5, SMALL["n_points"], SMALL["c_in"], device="cuda"))   # above max_batch
    net.close()


def test_adam_step_matches_formula():
    import torch
    c = S.cfg(max_batch=1, **SMALL)
    theta = _theta(SMALL, 4)
    net = S.Net(c, torch.from_numpy(theta.copy()).cuda())
    rng = np.random.Generator(np.random.PCG64(9))
    m = np.zeros_like(theta, dtype=np.float64)
    v = np.zeros_like(theta, dtype=np.float64)
    p = theta.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(theta.size).astype(np.float32)
        net.grad.copy_(torch.from_numpy(g))
        net.adam(lr=1e-2)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g.astype(np.float64) ** 2
        p = p - 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    got = net.params.cpu().numpy()
    assert np.max(np.abs(got - p)) <= 1e-5
    net.close()


def test_training_reduces_the_loss():
    """a student network fits a fixed teacher network's outputs"""
    import torch
    cfg = SMALL
    B = 8
    c = S.cfg(max_batch=B, **cfg)
    x, _, _, wo = SI.random_batch(cfg, B, 21, with_mask=False)
    teacher, _ = F.forward(cfg, _theta(cfg, 22).astype(np.float64), x.astype(np.float64))
    net = S.Net(c, torch.from_numpy(SI.init_params(cfg, 23)).cuda())
    dx = torch.from_numpy(x).cuda()
    dt = torch.from_numpy(teacher.astype(np.float32)).cuda()
    dw = torch.from_numpy(np.ones(cfg["c_out"], np.float32)).cuda()
    first = float(net.train_step(dx, dt, dw, lr=3e-3).cpu()[0])
    for _ in range(200):
        last = net.train_step(dx, dt, dw, lr=3e-3)
    last = float(last.cpu()[0])
    _say(f"[surrogate] training loss {first:.3e} -> {last:.3e}")
    assert last < 0.2 * first
    net.close()
