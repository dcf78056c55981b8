"""Python binding of include/surrogate.h (argument marshalling only).

The network's forward and backward passes, its loss and Adam run in the HIP
library; this module allocates parameters and workspace with PyTorch and
passes pointers.  There is no fallback: without the library, `load()` raises.
"""
from __future__ import annotations

import ctypes

from . import fdtd

SUR_STATUS = {0: "SUR_OK", -1: "SUR_EINVAL", -2: "SUR_ESIZE", -3: "SUR_ESTATE", -4: "SUR_EDEVICE"}
EXPORTS = ("sur_sizes", "sur_init", "sur_forward", "sur_backward", "sur_loss", "sur_adam", "sur_reset_moments",
           "sur_gemm", "sur_destroy", "sur_last_error", "sur_encode", "sur_check")


class SurCfg(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_points", ctypes.c_int32), ("c_in", ctypes.c_int32),
                ("width", ctypes.c_int32), ("modes", ctypes.c_int32), ("layers", ctypes.c_int32),
                ("proj", ctypes.c_int32), ("c_out", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class SurError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{SUR_STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    lib = fdtd.load()
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    C = ctypes.POINTER(SurCfg)
    lib.sur_sizes.argtypes = [C, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)]
    lib.sur_init.argtypes = [C, vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.sur_forward.argtypes = [vp, i32, vp, vp]
    lib.sur_backward.argtypes = [vp, i32, vp, vp, vp]
    lib.sur_loss.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.sur_adam.argtypes = [vp, vp, f32, f32, f32, f32, i64]
    lib.sur_reset_moments.argtypes = [vp]
    lib.sur_gemm.argtypes = [i32, i32, i32, i32, i32, f32, vp, i32, i64, vp, i32, i64, f32, vp, i32, i64, i32, vp]
    lib.sur_destroy.argtypes = [vp]
    lib.sur_encode.argtypes = [vp, i32, i32, vp, vp]
    lib.sur_check.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double, vp,
                              vp, vp]
    lib.sur_last_error.argtypes = [vp]
    lib.sur_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def cfg(n_points=1024, c_in=7, width=64, modes=64, layers=4, proj=128, c_out=3, max_batch=32) -> SurCfg:
    return SurCfg(struct_size=ctypes.sizeof(SurCfg), n_points=n_points, c_in=c_in, width=width, modes=modes,
                  layers=layers, proj=proj, c_out=c_out, max_batch=max_batch)


def sizes(c: SurCfg):
    lib = load()
    n = ctypes.c_int64(0)
    b = ctypes.c_size_t(0)
    rc = lib.sur_sizes(ctypes.byref(c), ctypes.byref(n), ctypes.byref(b))
    if rc:
        raise SurError(rc, lib.sur_last_error(None).decode())
    return int(n.value), int(b.value)


def gemm_flops(c: SurCfg) -> tuple[int, int]:
    """(forward, backward) flops per sample of the GEMMs sur_forward and
    sur_backward issue: lift, per layer the DFT to 2*modes rows, the per-mode
    complex mixing (4 real C x C products), the inverse DFT and the pointwise
    C x C product, the two projection layers; the backward has the data and
    the weight gradient of each."""
    Np, C, M2, P, m = c.n_points, c.width, 2 * c.modes, c.proj, c.modes
    fwd = 2 * Np * c.c_in * C + c.layers * (2 * M2 * C * Np + 8 * C * C * m + 2 * Np * C * M2 + 2 * Np * C * C) \
        + 2 * Np * C * P + 2 * Np * P * c.c_out
    bwd = 4 * Np * P * c.c_out + 4 * Np * C * P \
        + c.layers * (4 * Np * C * C + 4 * M2 * C * Np + 16 * C * C * m) + 2 * c.c_in * C * Np
    return fwd, bwd


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def gemm(A, B, C, transA=False, transB=False, alpha=1.0, beta=0.0, M=None, N=None, K=None, lda=None, ldb=None,
         ldc=None, sA=0, sB=0, sC=0, batch=1, stream=None):
    """C = alpha op(A) op(B) + beta C on the library's bf16 matrix cores (torch fp32 device tensors)."""
    import torch
    lib = load()
    M = M if M is not None else (A.shape[-1] if transA else A.shape[-2])
    K = K if K is not None else (A.shape[-2] if transA else A.shape[-1])
    N = N if N is not None else (B.shape[-2] if transB else B.shape[-1])
    lda = lda if lda is not None else A.shape[-1]
    ldb = ldb if ldb is not None else B.shape[-1]
    ldc = ldc if ldc is not None else C.shape[-1]
    st = stream if stream is not None else torch.cuda.current_stream(C.device)
    rc = lib.sur_gemm(int(transA), int(transB), int(M), int(N), int(K), float(alpha), _p(A), int(lda), int(sA),
                      _p(B), int(ldb), int(sB), float(beta), _p(C), int(ldc), int(sC), int(batch),
                      ctypes.c_void_p(st.cuda_stream))
    if rc:
        raise SurError(rc, lib.sur_last_error(None).decode())
    return C


def encode(par, n, x=None, stream=None):
    """sur_encode: par (B, 6) float64 device tensor of (w, k0, a, Gamma, Delta, T) -> x (B, n, 8) float32"""
    import torch
    lib = load()
    B = par.shape[0]
    if x is None:
        x = torch.empty(B, n, 8, dtype=torch.float32, device=par.device)
    st = stream if stream is not None else torch.cuda.current_stream(par.device)
    rc = lib.sur_encode(_p(par), int(B), int(n), _p(x), ctypes.c_void_p(st.cuda_stream))
    if rc:
        raise SurError(rc, "sur_encode")
    return x


def check(S, P2, P4, P8, h, valid, tol, safety, ratio_tol, stream=None):
    """sur_check: (dist, est, q) (B, 3) float64 and accepted (B, 2) bool (network, coarse alone)"""
    import torch
    lib = load()
    B, n = S.shape
    out = torch.empty(B, 3, dtype=torch.float64, device=S.device)
    acc = torch.empty(B, 2, dtype=torch.int32, device=S.device)
    st = stream if stream is not None else torch.cuda.current_stream(S.device)
    rc = lib.sur_check(_p(S), _p(P2), _p(P4), _p(P8), _p(h), _p(valid), int(B), int(n), float(tol), float(safety),
                       float(ratio_tol), _p(out), _p(acc), ctypes.c_void_p(st.cuda_stream))
    if rc:
        raise SurError(rc, "sur_check")
    return out, acc.bool()


class Net:
    """The surrogate network bound to a torch parameter tensor and workspace."""

    def __init__(self, c: SurCfg, params=None, device: str = "cuda:0"):
        import torch
        self.lib = load()
        self.cfg = c
        self.n_params, nbytes = sizes(c)
        self.device = torch.device(device)
        if params is None:
            params = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        assert params.numel() == self.n_params and params.dtype == torch.float32
        self.params = params
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.grad = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p(0)
        rc = self.lib.sur_init(ctypes.byref(c), _p(self.params), _p(self.ws), nbytes,
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            raise SurError(rc, self.lib.sur_last_error(None).decode())
        self.h = h
        self.step = 0

    def _check(self, rc):
        if rc:
            raise SurError(rc, self.lib.sur_last_error(self.h).decode())

    def forward(self, x, y=None):
        import torch
        B = x.shape[0]
        if y is None:
            y = torch.empty(B, self.cfg.n_points, self.cfg.c_out, dtype=torch.float32, device=self.device)
        self._check(self.lib.sur_forward(self.h, B, _p(x), _p(y)))
        return y

    def backward(self, x, dy):
        self._check(self.lib.sur_backward(self.h, x.shape[0], _p(x), _p(dy), _p(self.grad)))
        return self.grad

    def loss(self, y, t, wo, mask=None, dy=None, out=None):
        import torch
        if dy is None:
            dy = torch.empty_like(y)
        if out is None:
            out = torch.empty(1, dtype=torch.float32, device=self.device)
        self._check(self.lib.sur_loss(self.h, y.shape[0], _p(y), _p(t), _p(mask) if mask is not None else None,
                                      _p(wo), _p(dy), _p(out)))
        return out, dy

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        self._check(self.lib.sur_adam(self.h, _p(self.grad), float(lr), float(beta1), float(beta2), float(eps),
                                      self.step))

    def train_step(self, x, t, wo, mask=None, lr=1e-3):
        """forward, loss, backward and Adam on one batch; returns the loss tensor (device)"""
        y = self.forward(x)
        loss, dy = self.loss(y, t, wo, mask)
        self.backward(x, dy)
        self.adam(lr)
        return loss

    def close(self):
        if getattr(self, "h", None):
            self.lib.sur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
