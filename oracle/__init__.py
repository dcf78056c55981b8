"""CPU oracle for the FDTD march of the 1+1D delay PDE (arXiv:1707.05943).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may use this package; the product path never does.  It
shares no code with the GPU path: its arithmetic lives in `fdtd_oracle.c`
(plain C99, double precision, single thread) and in `micro.py` (a literal
pure-Python transcription of Eq. (1) on a full space-time grid for tiny
cases).  The only module both sides read is the seeded workload generator.

Parity status of each part (what pins it, see tests/test_oracle_*.py):
  * P(n, z), App. C            -- mpmath and exact rational series
  * E(t) closed forms (6),(9),(13) -- the delay equation itself, and the
    independent quadrature of the delay series
  * E(t) Gaussian (quadrature) -- the delay equation, conservation of the
    one-excitation probability, and the plane-wave superposition
  * march (HYBRID reads)       -- the literal micro-oracle; the micro-oracle in
    turn converges to the exact solution in x <= -a (paper's test 1) and
    conserves the two-excitation probability as Delta -> 0; the rounding of
    long FP64 marches against the same source built in long double
    (`march(..., long_double=True)`)
  * march with the paper's own reads (march_diag) -- the micro-oracle's
    paper_diag mode; second-order convergence to the exact solution in
    x <= -a (the paper's test 1) and to the hybrid march right of -a
  * chi readout, Eq. (2)       -- the micro-oracle's full-grid Eq. (2)
  * mu, lambda, App. D (nm.py) -- conservation of the one-excitation sector,
    the exact value at t = 0, the uncoupled limit
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdtd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_PATH_LD = os.path.join(_HERE, "liboracle_ld.so")
_lib = None
_lib_ld = None


def build(force: bool = False) -> str:
    """Compile the oracle's C source with gcc (no FMA contraction, no
    fast-math): the FP64 library, and the same source with its arithmetic in
    long double (-DORC_LONG_DOUBLE; the arrays passed stay double)."""
    for path, extra in ((_LIB_PATH, []), (_LIB_PATH_LD, ["-DORC_LONG_DOUBLE"])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            tmp = path + ".tmp"
            subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", *extra,
                            "-o", tmp, _SRC, "-lm"], check=True)
            os.replace(tmp, path)
    return _LIB_PATH


class OrcParams(ctypes.Structure):
    _fields_ = [("Nx", ctypes.c_int64), ("D", ctypes.c_int64), ("Nt", ctypes.c_int64),
                ("Delta", ctypes.c_double), ("omega0", ctypes.c_double), ("Gamma", ctypes.c_double),
                ("incident", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("k", ctypes.c_double), ("alpha", ctypes.c_double),
                ("x0", ctypes.c_double), ("width", ctypes.c_double),
                ("phase", ctypes.c_double), ("identical", ctypes.c_int32), ("pad1", ctypes.c_int32),
                ("k1", ctypes.c_double), ("k2", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("alpha2", ctypes.c_double)]


def _load(long_double: bool = False):
    global _lib, _lib_ld
    if long_double and _lib_ld is not None:
        return _lib_ld
    if not long_double and _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH_LD if long_double else _LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.orc_gamma_P_arr.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.orc_gamma_P_regime_arr.argtypes = [i64, vp, vp, ctypes.c_int32, vp]
    lib.orc_E_closed_arr.argtypes = [P(OrcParams), i64, vp, vp]
    lib.orc_E_quad_arr.argtypes = [P(OrcParams), i64, vp, vp]
    lib.orc_Jn_quad_arr.argtypes = [P(OrcParams), ctypes.c_int, i64, vp, vp]
    lib.orc_phi_arr.argtypes = [P(OrcParams), i64, vp, vp]
    lib.orc_march_diag.argtypes = [P(OrcParams), vp, i64, vp, vp, i64, vp]
    lib.orc_phi_mass_below_arr.argtypes = [P(OrcParams), i64, vp, vp]
    lib.orc_E_table.argtypes = [P(OrcParams), ctypes.c_int, vp]
    lib.orc_march.argtypes = [P(OrcParams), vp, vp, vp, vp, i64, i64, vp, vp, i64, vp]
    lib.orc_march.restype = ctypes.c_int
    lib.orc_chi0_arr.argtypes = [P(OrcParams), i64, vp, vp, vp]
    lib.orc_exact_part_arr.argtypes = [P(OrcParams), vp, vp]
    lib.orc_two_photon_A.argtypes = [P(OrcParams)]
    lib.orc_two_photon_A.restype = ctypes.c_double
    if long_double:
        _lib_ld = lib
    else:
        _lib = lib
    return lib


def params(inst) -> OrcParams:
    """Oracle parameter block from a workload instance (or a dict of the same keys)."""
    d = inst if isinstance(inst, dict) else inst.as_dict()
    return OrcParams(Nx=int(d["Nx"]), D=int(d["D"]), Nt=int(d["Nt"]), Delta=float(d["Delta"]),
                     omega0=float(d["omega0"]), Gamma=float(d["Gamma"]), incident=int(d["incident"]),
                     pad0=0, k=float(d.get("k", 0.0)), alpha=float(d.get("alpha", 0.0)),
                     x0=float(d.get("x0", 0.0)), width=float(d.get("width", 1.0)),
                     phase=float(d.get("phase", 0.0)), identical=int(d.get("identical_photons", 1)), pad1=0,
                     k1=float(d.get("k1", 0.0)), k2=float(d.get("k2", 0.0)),
                     alpha1=float(d.get("alpha1", 0.0)), alpha2=float(d.get("alpha2", 0.0)))


def two_photons(inst) -> bool:
    """two different exponential photons (Sec. 2 case (c) with identical_photons = 0)"""
    d = inst if isinstance(inst, dict) else inst.as_dict()
    return int(d["incident"]) == 3 and int(d.get("identical_photons", 1)) == 0


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def gamma_P(n, z):
    """P(n, z) = gamma(n, z)/(n-1)! (App. C); returns (values, regime, converged)."""
    lib = _load()
    z = np.ascontiguousarray(np.atleast_1d(np.asarray(z, dtype=np.complex128)))
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(n, dtype=np.int32), z.shape)).copy()
    out = np.empty_like(z)
    reg = np.empty(z.shape, np.int32)
    ok = np.empty(z.shape, np.int32)
    lib.orc_gamma_P_arr(z.size, _ptr(n), _ptr(z), _ptr(out), _ptr(reg), _ptr(ok))
    return out, reg, ok


def gamma_P_regime(n, z, regime: int):
    lib = _load()
    z = np.ascontiguousarray(np.atleast_1d(np.asarray(z, dtype=np.complex128)))
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(n, dtype=np.int32), z.shape)).copy()
    out = np.empty_like(z)
    lib.orc_gamma_P_regime_arr(z.size, _ptr(n), _ptr(z), int(regime), _ptr(out))
    return out


def _tarr(t):
    return np.ascontiguousarray(np.atleast_1d(np.asarray(t, dtype=np.float64)))


def E_closed(inst, t):
    lib = _load()
    p = params(inst)
    t = _tarr(t)
    out = np.empty(t.shape, np.complex128)
    lib.orc_E_closed_arr(ctypes.byref(p), t.size, _ptr(t), _ptr(out))
    return out


def E_quad(inst, t):
    lib = _load()
    p = params(inst)
    t = _tarr(t)
    out = np.empty(t.shape, np.complex128)
    lib.orc_E_quad_arr(ctypes.byref(p), t.size, _ptr(t), _ptr(out))
    return out


def Jn_quad(inst, n: int, T):
    lib = _load()
    p = params(inst)
    T = _tarr(T)
    out = np.empty(T.shape, np.complex128)
    lib.orc_Jn_quad_arr(ctypes.byref(p), int(n), T.size, _ptr(T), _ptr(out))
    return out


def phi(inst, x):
    lib = _load()
    p = params(inst)
    x = _tarr(x)
    out = np.empty(x.shape, np.complex128)
    lib.orc_phi_arr(ctypes.byref(p), x.size, _ptr(x), _ptr(out))
    return out


def phi_mass_below(inst, y):
    lib = _load()
    p = params(inst)
    y = _tarr(y)
    out = np.empty(y.shape, np.float64)
    lib.orc_phi_mass_below_arr(ctypes.byref(p), y.size, _ptr(y), _ptr(out))
    return out


def E_table(inst, mode: int = 0) -> np.ndarray:
    """E(t_r) for r = 0..Nt.  mode 0: closed form where the paper gives one,
    quadrature of the delay series for the Gaussian; mode 1: quadrature on the
    grid for every family; mode 2: quadrature evaluated row by row.  Two
    different photons: e0^(1)(t_r) followed by e0^(2)(t_r) (2 (Nt+1) values)."""
    lib = _load()
    p = params(inst)
    out = np.empty((2 if two_photons(inst) else 1) * (int(p.Nt) + 1), np.complex128)
    lib.orc_E_table(ctypes.byref(p), int(mode), _ptr(out))
    return out


def march(inst, E: np.ndarray | None = None, *, chi_rows=(), n_tau: int = 0, snap_rows=(),
          want_ring: bool = True, want_pe: bool = True, long_double: bool = False) -> dict:
    """Run the oracle march over rows 1..Nt (HYBRID reads: x <= -a from the
    exact solution); long_double: the same source with its arithmetic in
    long double (the inputs and results are double).  Returns a dict with
      E    : the boundary table used, E(t_r)
      pe   : P_e(t_r), r = 0..Nt
      ring : rows Nt-D-1 .. Nt (oldest first), columns 0..Nx
      chi  : chi at detectors x1 = a + Delta, x2 = x1 + k Delta (k < n_tau), per chi row
      snaps: full rows at snap_rows
    """
    lib = _load(long_double)
    p = params(inst)
    if E is None:
        E = E_table(inst)
    E = np.ascontiguousarray(E, dtype=np.complex128)
    assert E.shape == ((2 if two_photons(inst) else 1) * (p.Nt + 1),)
    C = p.Nx + 1
    R = p.D + 2
    pe = np.empty(p.Nt + 1, np.float64) if want_pe else None
    ring = np.empty((R, C), np.complex128) if want_ring else None
    cr = np.ascontiguousarray(np.asarray(chi_rows, dtype=np.int64))
    chi = np.empty((len(cr), n_tau), np.complex128)
    sr = np.ascontiguousarray(np.asarray(snap_rows, dtype=np.int64))
    snaps = np.empty((len(sr), C), np.complex128)
    nul = ctypes.c_void_p(0)
    rc = lib.orc_march(ctypes.byref(p), _ptr(E), _ptr(pe) if pe is not None else nul,
                       _ptr(ring) if ring is not None else nul,
                       _ptr(cr) if len(cr) else nul, len(cr), int(n_tau), _ptr(chi) if len(cr) else nul,
                       _ptr(sr) if len(sr) else nul, len(sr), _ptr(snaps) if len(sr) else nul)
    if rc != 0:
        raise RuntimeError(f"oracle march failed ({rc}): a read broke the ring's lag bound")
    return {"E": E, "pe": pe, "ring": ring, "chi": chi, "snaps": snaps}


def march_diag(inst, diag_cols: int, E: np.ndarray | None = None, *, snap_rows=(), want_pe: bool = True) -> dict:
    """The march with the paper's own reads: diag_cols columns left of and at
    x = -a (columns 1-diag_cols..0) are marched too and read back wherever
    Eq. (1) reaches them; only points left of them take the exact solution.
    Every row is kept (memory (Nt+1)(Nx+diag_cols)16 B).  Returns a dict
    with lo (the first marched column), pe (P_e(t_r), column 0 marched) and
    snaps (columns lo..Nx of the listed rows)."""
    lib = _load()
    p = params(inst)
    if E is None:
        E = E_table(inst)
    E = np.ascontiguousarray(E, dtype=np.complex128)
    assert E.shape == (p.Nt + 1,)
    lo = 1 - int(diag_cols)
    W = p.Nx - lo + 1
    pe = np.empty(p.Nt + 1, np.float64) if want_pe else None
    sr = np.ascontiguousarray(np.asarray(snap_rows, dtype=np.int64))
    snaps = np.empty((len(sr), W), np.complex128)
    nul = ctypes.c_void_p(0)
    rc = lib.orc_march_diag(ctypes.byref(p), _ptr(E), int(diag_cols), _ptr(pe) if pe is not None else nul,
                            _ptr(sr) if len(sr) else nul, len(sr), _ptr(snaps) if len(sr) else nul)
    if rc != 0:
        raise RuntimeError(f"oracle diag march failed ({rc})")
    return {"E": E, "lo": lo, "pe": pe, "snaps": snaps}


def chi0(inst, x1, x2):
    """the initial two-photon state chi(x1, x2, 0), global phase included"""
    lib = _load()
    p = params(inst)
    x1, x2 = np.broadcast_arrays(_tarr(x1), _tarr(x2))
    x1, x2 = np.ascontiguousarray(x1), np.ascontiguousarray(x2)
    out = np.empty(x1.shape, np.complex128)
    lib.orc_chi0_arr(ctypes.byref(p), x1.size, _ptr(x1), _ptr(x2), _ptr(out))
    return out


def exact_part(inst, E) -> np.ndarray:
    """int_{-inf}^{-a} |psi(x, t_r)|^2 dx of the exact solution, r = 0..Nt"""
    lib = _load()
    p = params(inst)
    E = np.ascontiguousarray(E, dtype=np.complex128)
    out = np.empty(int(p.Nt) + 1, np.float64)
    lib.orc_exact_part_arr(ctypes.byref(p), _ptr(E), _ptr(out))
    return out


def two_photon_A(inst) -> float:
    """the normalisation constant A of Eq. (11)"""
    return float(_load().orc_two_photon_A(ctypes.byref(params(inst))))
