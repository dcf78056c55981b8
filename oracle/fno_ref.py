"""CPU reference of the surrogate network (float64 numpy).

TEST INFRASTRUCTURE ONLY: the test-suite may use this module; the product
path never does.  It shares no code with the GPU kernels: the Fourier layers
use numpy's FFT (the GPU side multiplies by DFT matrices), and every gradient
is written out from the chain rule below.  What pins it
(tests/test_oracle_fno.py): central finite differences of the loss for every
parameter group, a single Fourier mode below the cut passing a layer whose
mixing matrix is the identity unchanged and one above the cut being removed,
and the closed form of gelu.

Network (sizes in `cfg`: n_points, c_in, width, modes, layers, proj, c_out):
    u0 = x W0 + b0
    z_l = irfft(pad(rfft(u_l)[:modes] R_l)) + u_l W_l + b_l,  u_{l+1} = gelu(z_l)
          (identity instead of gelu after the last layer)
    y = gelu(u_L W1 + b1) W2 + b2
with R_l one complex width x width matrix per kept mode, applied as a row
vector times the matrix; gelu(v) = v (1 + erf(v / sqrt 2)) / 2.  The loss is
sum wo[o] mask (y - t)^2 / (B n_points).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def layout(cfg: dict) -> dict:
    """offsets of each parameter block in the flat parameter vector"""
    C, M, L, P = cfg["width"], cfg["modes"], cfg["layers"], cfg["proj"]
    shapes = [("W0", (cfg["c_in"], C)), ("b0", (C,)), ("Rr", (L, M, C, C)), ("Ri", (L, M, C, C)),
              ("W", (L, C, C)), ("b", (L, C)), ("W1", (C, P)), ("b1", (P,)), ("W2", (P, cfg["c_out"])),
              ("b2", (cfg["c_out"],))]
    out, off = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = (off, shp)
        off += n
    out["_n"] = off
    return out


def unpack(cfg: dict, theta: np.ndarray) -> dict:
    lay = layout(cfg)
    return {k: theta[v[0]:v[0] + int(np.prod(v[1]))].reshape(v[1]) for k, v in lay.items() if k != "_n"}


def pack(cfg: dict, parts: dict) -> np.ndarray:
    lay = layout(cfg)
    theta = np.zeros(lay["_n"])
    for k, v in lay.items():
        if k != "_n":
            o, s = v
            theta[o:o + int(np.prod(s))] = np.asarray(parts[k], dtype=np.float64).ravel()
    return theta


def gelu(v):
    return 0.5 * v * (1.0 + erf(v / np.sqrt(2.0)))


def gelu_d(v):
    return 0.5 * (1.0 + erf(v / np.sqrt(2.0))) + v * np.exp(-0.5 * v * v) / np.sqrt(2.0 * np.pi)


def spectral(u, R, modes):
    """irfft of the first `modes` modes of rfft(u) along the points, each mode's
    channel vector times its complex matrix"""
    n = u.shape[1]
    X = np.fft.rfft(u, axis=1)[:, :modes, :]                 # (B, modes, C)
    Y = np.einsum("bmc,mcd->bmd", X, R)
    full = np.zeros((u.shape[0], n // 2 + 1, u.shape[2]), dtype=complex)
    full[:, :modes, :] = Y
    return np.fft.irfft(full, n=n, axis=1), X


def forward(cfg: dict, theta: np.ndarray, x: np.ndarray):
    """returns y and the intermediate values the backward pass needs"""
    p = unpack(cfg, theta)
    L, M = cfg["layers"], cfg["modes"]
    R = p["Rr"] + 1j * p["Ri"]
    u = x @ p["W0"] + p["b0"]
    us, zs, Xs = [u], [], []
    for l in range(L):
        s, X = spectral(u, R[l], M)
        z = s + u @ p["W"][l] + p["b"][l]
        u = gelu(z) if l < L - 1 else z
        us.append(u)
        zs.append(z)
        Xs.append(X)
    zh = u @ p["W1"] + p["b1"]
    h = gelu(zh)
    y = h @ p["W2"] + p["b2"]
    return y, {"us": us, "zs": zs, "Xs": Xs, "zh": zh, "h": h}


def loss(y, t, wo, mask=None):
    m = np.ones_like(y) if mask is None else mask
    B, n = y.shape[0], y.shape[1]
    e = y - t
    val = np.sum(wo * m * e * e) / (B * n)
    dy = 2.0 * wo * m * e / (B * n)
    return val, dy


def backward(cfg: dict, theta: np.ndarray, x: np.ndarray, cache: dict, dy: np.ndarray) -> np.ndarray:
    """gradient of the loss with respect to theta, given dloss/dy"""
    p = unpack(cfg, theta)
    L, M = cfg["layers"], cfg["modes"]
    n = x.shape[1]
    R = p["Rr"] + 1j * p["Ri"]
    g = {k: np.zeros_like(v) for k, v in p.items()}
    rows = lambda a: a.reshape(-1, a.shape[-1])                     # (B n) x channels
    # projection
    g["W2"] = rows(cache["h"]).T @ rows(dy)
    g["b2"] = rows(dy).sum(axis=0)
    dzh = (dy @ p["W2"].T) * gelu_d(cache["zh"])
    g["W1"] = rows(cache["us"][L]).T @ rows(dzh)
    g["b1"] = rows(dzh).sum(axis=0)
    du = dzh @ p["W1"].T
    # Fourier layers
    cm = np.full(M, 2.0)
    cm[0] = 1.0
    for l in range(L - 1, -1, -1):
        dz = du * gelu_d(cache["zs"][l]) if l < L - 1 else du
        ul = cache["us"][l]
        g["b"][l] = rows(dz).sum(axis=0)
        g["W"][l] = rows(ul).T @ rows(dz)
        # z's spectral part is irfft of Y: its adjoint takes (c_m / n) rfft(dz)
        dY = (cm[None, :, None] / n) * np.fft.rfft(dz, axis=1)[:, :M, :]
        X = cache["Xs"][l]
        dR = np.einsum("bmc,bmd->mcd", np.conj(X), dY)
        g["Rr"][l] = dR.real
        g["Ri"][l] = dR.imag
        dX = np.einsum("bmd,mcd->bmc", dY, np.conj(R[l]))
        # X is the first modes of rfft(u): its adjoint is Re sum_m dX_m e^{2 pi i m p / n}
        full = np.zeros((x.shape[0], n, ul.shape[2]), dtype=complex)
        full[:, :M, :] = dX
        du_spec = np.real(np.fft.ifft(full, axis=1)) * n
        du = dz @ p["W"][l].T + du_spec
    g["W0"] = rows(x).T @ rows(du)
    g["b0"] = rows(du).sum(axis=0)
    return pack(cfg, g)
