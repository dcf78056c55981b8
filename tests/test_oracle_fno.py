"""Pins of the CPU reference of the surrogate network (oracle/fno_ref.py)."""
import numpy as np
import pytest

from oracle import fno_ref as F
from paper_1707_05943_amd import sur_inputs as SI

TINY = {"n_points": 16, "c_in": 3, "width": 4, "modes": 3, "layers": 2, "proj": 5, "c_out": 2}


def _setup(seed=1, B=2):
    theta = SI.init_params(TINY, seed).astype(np.float64)
    # larger spectral weights than the initialisation, so that they matter
    lay = F.layout(TINY)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    for k in ("Rr", "Ri"):
        o, s = lay[k]
        theta[o:o + int(np.prod(s))] = 0.5 * rng.standard_normal(int(np.prod(s)))
    x, t, mask, wo = SI.random_batch(TINY, B, seed)
    return theta, x.astype(np.float64), t.astype(np.float64), mask.astype(np.float64), wo.astype(np.float64)


def test_gradient_matches_finite_differences():
    theta, x, t, mask, wo = _setup()
    y, cache = F.forward(TINY, theta, x)
    _, dy = F.loss(y, t, wo, mask)
    g = F.backward(TINY, theta, x, cache, dy)
    lay = F.layout(TINY)
    rng = np.random.Generator(np.random.PCG64(5))
    h = 1e-6
    for name in ("W0", "b0", "Rr", "Ri", "W", "b", "W1", "b1", "W2", "b2"):
        o, s = lay[name]
        for idx in rng.choice(int(np.prod(s)), size=min(6, int(np.prod(s))), replace=False):
            e = np.zeros_like(theta)
            e[o + idx] = h
            lp = F.loss(F.forward(TINY, theta + e, x)[0], t, wo, mask)[0]
            lm = F.loss(F.forward(TINY, theta - e, x)[0], t, wo, mask)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[o + idx]) <= 1e-7 * max(1.0, abs(fd)), (name, idx, fd, g[o + idx])


def test_fourier_layer_keeps_modes_below_the_cut():
    """with R = identity, W = 0, b = 0 a layer maps cos(2 pi m p / n) to itself
    for m < modes and to zero for m >= modes"""
    n, M, C = 16, 3, 4
    R = np.broadcast_to(np.eye(C, dtype=complex), (M, C, C))
    p = np.arange(n)
    for m in range(n // 2):
        u = np.cos(2 * np.pi * m * p / n)[None, :, None] * np.ones((1, n, C))
        s, _ = F.spectral(u, R, M)
        want = u if m < M else np.zeros_like(u)
        assert np.max(np.abs(s - want)) < 1e-13, m


def test_gelu_closed_form():
    v = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    phi = 0.5 * (1 + np.array([-0.9973002039367398, -0.6826894921370859, 0.0, 0.38292492254802624,
                                0.9544997361036416]))        # P(|Z| < |v|) signs: Phi(v) = (1 + erf(v/sqrt2))/2
    assert np.allclose(F.gelu(v), v * phi, atol=1e-15)
    # derivative by central differences
    h = 1e-6
    assert np.allclose((F.gelu(v + h) - F.gelu(v - h)) / (2 * h), F.gelu_d(v), atol=1e-8)


def test_pack_roundtrip_and_order():
    lay = F.layout(TINY)
    theta = np.arange(lay["_n"], dtype=np.float64)
    parts = F.unpack(TINY, theta)
    assert np.array_equal(F.pack(TINY, parts), theta)
    # the same block order and sizes as the input generator (and the library header)
    off = 0
    for name, shape, _ in SI.param_blocks(TINY):
        assert lay[name] == (off, shape)
        off += int(np.prod(shape))
