"""Seeded inputs of the surrogate network: initial parameters and random
batches (numpy PCG64).  Holds none of the network's arithmetic; the GPU
library and the CPU reference both take what this module draws."""
from __future__ import annotations

import numpy as np


def cfg_dict(c) -> dict:
    names = ("n_points", "c_in", "width", "modes", "layers", "proj", "c_out")
    return {k: int(getattr(c, k)) if not isinstance(c, dict) else int(c[k]) for k in names}


def param_blocks(cfg: dict):
    """(name, shape, fan_in or None) in the library's parameter order"""
    C, M, L, P = cfg["width"], cfg["modes"], cfg["layers"], cfg["proj"]
    return [("W0", (cfg["c_in"], C), cfg["c_in"]), ("b0", (C,), cfg["c_in"]),
            ("Rr", (L, M, C, C), None), ("Ri", (L, M, C, C), None),
            ("W", (L, C, C), C), ("b", (L, C), C), ("W1", (C, P), C), ("b1", (P,), C),
            ("W2", (P, cfg["c_out"]), P), ("b2", (cfg["c_out"],), P)]


def init_params(cfg: dict, seed: int) -> np.ndarray:
    """Dense weights and biases uniform in +-1/sqrt(fan_in); the spectral
    matrices uniform in [0, 1/width^2) (real and imaginary parts)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for name, shape, fan in param_blocks(cfg):
        if fan is None:
            v = rng.random(shape) / (cfg["width"] ** 2)
        else:
            bound = 1.0 / np.sqrt(fan)
            v = rng.uniform(-bound, bound, shape)
        out.append(v.ravel())
    return np.concatenate(out).astype(np.float32)


def random_batch(cfg: dict, B: int, seed: int, with_mask: bool = True):
    """x ~ N(0,1) of shape (B, n, c_in); targets t ~ N(0, 0.1); a mask with
    about 10% zeros; channel weights wo in [0.5, 1.5)"""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, ci, co = cfg["n_points"], cfg["c_in"], cfg["c_out"]
    x = rng.standard_normal((B, n, ci)).astype(np.float32)
    t = (0.1 * rng.standard_normal((B, n, co))).astype(np.float32)
    mask = (rng.random((B, n, co)) > 0.1).astype(np.float32) if with_mask else None
    wo = (0.5 + rng.random(co)).astype(np.float32)
    return x, t, mask, wo
