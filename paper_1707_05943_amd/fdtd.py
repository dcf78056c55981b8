"""Python binding of the C ABI in include/fdtd.h (argument marshalling only).

Every step of the march runs in the HIP library; this module allocates the
device workspace with PyTorch, passes pointers and sizes, and copies results
back.  There is no fallback: if the library is missing or cannot be loaded,
`load()` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")

FDTD_ABI_VERSION = 3
INC_PLANE, INC_EXP1, INC_EXP2, INC_GAUSS2 = 1, 2, 3, 4
RO_ROW, RO_PE, RO_CHI, RO_E, RO_MU, RO_LAMBDA, RO_NGEO, RO_LEFT = 1, 2, 3, 4, 5, 6, 7, 8
READ_EXACT, READ_PAPER_DIAG = 0, 1
E_SERIES, E_DELAY_ODE = 0, 1
STATUS = {0: "FDTD_OK", -1: "FDTD_EINVAL", -2: "FDTD_ESIZE", -3: "FDTD_ESTATE", -4: "FDTD_EDEVICE",
          -5: "FDTD_ERANGE"}

# every symbol include/fdtd.h declares
EXPORTS = ("fdtd_workspace_size", "fdtd_init", "fdtd_set_boundary", "fdtd_set_boundary_tables",
           "fdtd_march", "fdtd_current_row", "fdtd_readout", "fdtd_sync", "fdtd_destroy",
           "fdtd_checkpoint_size", "fdtd_checkpoint", "fdtd_restore",
           "fdtd_describe", "fdtd_strerror", "fdtd_last_error",
           "fdtd_batch_workspace_size", "fdtd_batch_init", "fdtd_batch_set_boundary", "fdtd_batch_march",
           "fdtd_batch_readout", "fdtd_batch_info", "fdtd_batch_sync", "fdtd_batch_destroy",
           "fdtd_batch_last_error", "fdtd_batch_autotune", "fdtd_batch_set_chi", "fdtd_batch_sample_pe",
           "fdtd_solve_noalloc", "fdtd_stream_copy")

# bytes of the library's own workspace for fdtd_solve_noalloc (FDTD_NOALLOC_MAX_BYTES)
NOALLOC_MAX_BYTES = 64 << 20


class FdtdParams(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("struct_size", ctypes.c_uint32),
                ("Nx", ctypes.c_int64), ("D", ctypes.c_int64), ("Nt", ctypes.c_int64),
                ("Delta", ctypes.c_double), ("omega0", ctypes.c_double), ("Gamma", ctypes.c_double),
                ("incident", ctypes.c_int32), ("boundary", ctypes.c_int32),
                ("k", ctypes.c_double), ("alpha", ctypes.c_double), ("x0", ctypes.c_double),
                ("width", ctypes.c_double), ("phase", ctypes.c_double),
                ("identical_photons", ctypes.c_int32), ("read_mode", ctypes.c_int32),
                ("k1", ctypes.c_double), ("k2", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("alpha2", ctypes.c_double), ("diag_cols", ctypes.c_int64)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("tmax", ctypes.c_int32), ("wmax", ctypes.c_int64),
                ("use_graph", ctypes.c_int32), ("groups", ctypes.c_int32)]


def batch_opts(tmax: int = 0, wmax: int = 0, use_graph: bool = True, groups: int = 1) -> BatchOpts:
    return BatchOpts(struct_size=ctypes.sizeof(BatchOpts), tmax=int(tmax), wmax=int(wmax),
                     use_graph=1 if use_graph else 0, groups=int(groups))


class FdtdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FdtdError(-4, f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    # One HIP runtime per process: torch ships its own libamdhip64 under the
    # same soname, which its libraries load by file name.  Loading torch first
    # makes this library bind to that copy; loaded the other way round the
    # process would hold two runtimes and one of them would see no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    P = ctypes.POINTER(FdtdParams)
    lib.fdtd_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.fdtd_init.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.fdtd_set_boundary.argtypes = [vp]
    lib.fdtd_set_boundary_tables.argtypes = [vp, vp, i64]
    lib.fdtd_march.argtypes = [vp, i64]
    lib.fdtd_current_row.argtypes = [vp, ctypes.POINTER(i64)]
    lib.fdtd_readout.argtypes = [vp, i32, i64, vp, i64, i32]
    lib.fdtd_sync.argtypes = [vp]
    lib.fdtd_checkpoint_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.fdtd_checkpoint.argtypes = [vp, vp, ctypes.c_size_t]
    lib.fdtd_restore.argtypes = [vp, vp, ctypes.c_size_t]
    lib.fdtd_destroy.argtypes = [vp]
    lib.fdtd_describe.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
    lib.fdtd_strerror.argtypes = [ctypes.c_int]
    lib.fdtd_strerror.restype = ctypes.c_char_p
    lib.fdtd_last_error.argtypes = [vp]
    lib.fdtd_last_error.restype = ctypes.c_char_p
    BO = ctypes.POINTER(BatchOpts)
    lib.fdtd_batch_workspace_size.argtypes = [P, i32, BO, ctypes.POINTER(ctypes.c_size_t)]
    lib.fdtd_batch_init.argtypes = [P, i32, BO, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.fdtd_batch_set_boundary.argtypes = [vp]
    lib.fdtd_batch_march.argtypes = [vp]
    lib.fdtd_batch_readout.argtypes = [vp, i32, i32, i64, vp, i64, i32]
    lib.fdtd_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.fdtd_batch_sync.argtypes = [vp]
    lib.fdtd_batch_destroy.argtypes = [vp]
    lib.fdtd_batch_last_error.argtypes = [vp]
    lib.fdtd_batch_last_error.restype = ctypes.c_char_p
    lib.fdtd_batch_autotune.argtypes = [P, i32, vp, ctypes.c_size_t, vp, i64, BO, ctypes.POINTER(ctypes.c_double)]
    lib.fdtd_batch_set_chi.argtypes = [vp, vp, vp, i64, vp]
    lib.fdtd_batch_sample_pe.argtypes = [vp, i64, vp, vp]
    lib.fdtd_solve_noalloc.argtypes = [P, i64, vp, vp, vp]
    lib.fdtd_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    _lib = lib
    return lib


def params(inst) -> FdtdParams:
    d = inst if isinstance(inst, dict) else inst.as_dict()
    return FdtdParams(abi_version=FDTD_ABI_VERSION, struct_size=ctypes.sizeof(FdtdParams),
                      Nx=int(d["Nx"]), D=int(d["D"]), Nt=int(d["Nt"]), Delta=float(d["Delta"]),
                      omega0=float(d["omega0"]), Gamma=float(d["Gamma"]), incident=int(d["incident"]),
                      boundary=int(d.get("boundary", 0)), k=float(d.get("k", 0.0)), alpha=float(d.get("alpha", 0.0)),
                      x0=float(d.get("x0", 0.0)), width=float(d.get("width", 1.0)),
                      phase=float(d.get("phase", 0.0)), identical_photons=int(d.get("identical_photons", 1)),
                      read_mode=int(d.get("read_mode", 0)), k1=float(d.get("k1", 0.0)), k2=float(d.get("k2", 0.0)),
                      alpha1=float(d.get("alpha1", 0.0)), alpha2=float(d.get("alpha2", 0.0)),
                      diag_cols=int(d.get("diag_cols", 0)))


def workspace_size(inst) -> int:
    lib = load()
    p = params(inst)
    n = ctypes.c_size_t(0)
    rc = lib.fdtd_workspace_size(ctypes.byref(p), ctypes.byref(n))
    if rc:
        raise FdtdError(rc, lib.fdtd_last_error(None).decode())
    return int(n.value)


def describe(inst) -> dict:
    """The work decomposition the library uses for this instance."""
    import json
    lib = load()
    p = params(inst)
    buf = ctypes.create_string_buffer(1024)
    rc = lib.fdtd_describe(ctypes.byref(p), buf, 1024)
    if rc:
        raise FdtdError(rc, lib.fdtd_last_error(None).decode())
    return json.loads(buf.value.decode())


def solve_noalloc(inst, n_rows: int, pe_out=None, row_out=None, stream=None) -> None:
    """fdtd_solve_noalloc: boundary, march of n_rows rows and the readouts of
    P_e (into the float64 device tensor pe_out, n_rows+1 values) and of row
    n_rows (into the device tensor row_out, Nx+1 complex values) in the
    library's own device workspace; enqueued on `stream` (torch's current
    stream by default).  Raises FdtdError on failure."""
    import torch
    lib = load()
    p = params(inst)
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = lib.fdtd_solve_noalloc(ctypes.byref(p), int(n_rows),
                                ctypes.c_void_p(pe_out.data_ptr()) if pe_out is not None else None,
                                ctypes.c_void_p(row_out.data_ptr()) if row_out is not None else None,
                                ctypes.c_void_p(stream.cuda_stream))
    if rc:
        raise FdtdError(rc, lib.fdtd_last_error(None).decode())


def stream_copy(dst, src, stream=None) -> None:
    """fdtd_stream_copy: the library's streaming copy of the device tensor src
    into dst (same byte size, a multiple of 16), on `stream` (torch's current
    stream by default)."""
    import torch
    lib = load()
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("dst and src differ in size")
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = lib.fdtd_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), n,
                              ctypes.c_void_p(stream.cuda_stream))
    if rc:
        raise FdtdError(rc, "fdtd_stream_copy: misaligned or empty arguments")


class Solver:
    """One instance of the march on one GPU (a context bound to a torch stream)."""

    def __init__(self, inst, device: str = "cuda:0", stream=None):
        import torch
        self.lib = load()
        self.inst = inst
        self.p = params(inst)
        self.device = torch.device(device)
        self.torch = torch
        nbytes = workspace_size(inst)
        # 256-byte aligned workspace owned by this object (torch's allocator aligns to 512)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p(0)
        rc = self.lib.fdtd_init(ctypes.byref(self.p), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc:
            raise FdtdError(rc, self.lib.fdtd_last_error(None).decode())
        self.ctx = ctx

    def _check(self, rc):
        if rc:
            raise FdtdError(rc, self.lib.fdtd_last_error(self.ctx).decode())

    def set_boundary(self, E: np.ndarray | None = None):
        if E is None:
            self._check(self.lib.fdtd_set_boundary(self.ctx))
        else:
            E = np.ascontiguousarray(E, dtype=np.complex128)
            self._check(self.lib.fdtd_set_boundary_tables(self.ctx, E.ctypes.data_as(ctypes.c_void_p), E.size))
        return self

    def march(self, n_rows: int):
        self._check(self.lib.fdtd_march(self.ctx, int(n_rows)))
        return self

    @property
    def row(self) -> int:
        r = ctypes.c_int64(0)
        self._check(self.lib.fdtd_current_row(self.ctx, ctypes.byref(r)))
        return int(r.value)

    def _ro(self, what, arg, count, dtype):
        out = np.empty(count, dtype=dtype)
        self._check(self.lib.fdtd_readout(self.ctx, what, int(arg), out.ctypes.data_as(ctypes.c_void_p),
                                          int(count), 0))
        return out

    def checkpoint(self) -> np.ndarray:
        """the march's state as bytes (host memory)"""
        n = ctypes.c_size_t(0)
        self._check(self.lib.fdtd_checkpoint_size(self.ctx, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self.lib.fdtd_checkpoint(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.size))
        return buf

    def restore(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.fdtd_restore(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.size))
        return self

    def row_values(self, rho: int) -> np.ndarray:
        return self._ro(RO_ROW, rho, self.p.Nx + 1, np.complex128)

    def pe(self, count: int | None = None) -> np.ndarray:
        return self._ro(RO_PE, 0, self.row + 1 if count is None else count, np.float64)

    def left_values(self, rho: int) -> np.ndarray:
        """READ_PAPER_DIAG: the marched columns 1-diag_cols..0 of row rho"""
        return self._ro(RO_LEFT, rho, int(self.p.diag_cols), np.complex128)

    def chi(self, count: int) -> np.ndarray:
        return self._ro(RO_CHI, 0, count, np.complex128)

    def mu(self, count: int | None = None) -> np.ndarray:
        """mu(t_r) of App. D (stimulated-emission instances)"""
        return self._ro(RO_MU, 0, self.row + 1 if count is None else count, np.complex128)

    def lam(self, count: int | None = None) -> np.ndarray:
        """lambda(t_r) of App. D (stimulated-emission instances)"""
        return self._ro(RO_LAMBDA, 0, self.row + 1 if count is None else count, np.float64)

    def n_geo(self, row: int | None = None) -> float:
        """the geometric measure N_geo of App. D over [0, t_row] (default: the current row)"""
        return float(self._ro(RO_NGEO, self.row if row is None else row, 1, np.float64)[0])

    def E(self, photon: int = 0) -> np.ndarray:
        """the boundary table c E(t_r); two different photons: photon 0 -> A e^{i theta} e0^(1),
        photon 1 -> A e^{i theta} e0^(2)"""
        return self._ro(RO_E, photon, self.p.Nt + 1, np.complex128)

    def sync(self):
        self._check(self.lib.fdtd_sync(self.ctx))

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.fdtd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _param_array(instances):
    arr = (FdtdParams * len(instances))()
    for i, inst in enumerate(instances):
        arr[i] = params(inst)
    return arr


def batch_workspace_size(instances, opts: BatchOpts | None = None) -> int:
    lib = load()
    arr = _param_array(instances)
    n = ctypes.c_size_t(0)
    rc = lib.fdtd_batch_workspace_size(arr, len(instances), ctypes.byref(opts) if opts else None, ctypes.byref(n))
    if rc:
        raise FdtdError(rc, lib.fdtd_batch_last_error(None).decode())
    return int(n.value)


def autotune(instances, probe_rows: int = 1024, device: str = "cuda:0", workspace=None):
    """Run the library's autotuner on this batch; returns (BatchOpts, cell updates/s of the winner)."""
    import torch
    lib = load()
    arr = _param_array(instances)
    dev = torch.device(device)
    if workspace is None:
        need = max(batch_workspace_size(instances, batch_opts(t, w)) for t in (32, 16, 8) for w in (0, 768))
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    best = BatchOpts()
    rate = ctypes.c_double(0.0)
    rc = lib.fdtd_batch_autotune(arr, len(instances), ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                 ctypes.c_void_p(stream.cuda_stream), int(probe_rows), ctypes.byref(best),
                                 ctypes.byref(rate))
    if rc:
        raise FdtdError(rc, lib.fdtd_batch_last_error(None).decode())
    return best, float(rate.value)


class Batch:
    """Many instances marched together (one launch per row block for the whole batch)."""

    def __init__(self, instances, opts: BatchOpts | None = None, device: str = "cuda:0", stream=None,
                 workspace=None):
        import torch
        self.lib = load()
        self.instances = list(instances)
        self.n = len(self.instances)
        self.arr = _param_array(self.instances)
        self.opts = opts if opts is not None else batch_opts()
        self.device = torch.device(device)
        nbytes = batch_workspace_size(self.instances, self.opts)
        if workspace is not None and workspace.numel() >= nbytes:
            self.ws = workspace
        else:
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p(0)
        rc = self.lib.fdtd_batch_init(self.arr, self.n, ctypes.byref(self.opts), ctypes.c_void_p(self.ws.data_ptr()),
                                      self.ws.numel(), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            raise FdtdError(rc, self.lib.fdtd_batch_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc:
            raise FdtdError(rc, self.lib.fdtd_batch_last_error(self.h).decode())

    def set_boundary(self):
        self._check(self.lib.fdtd_batch_set_boundary(self.h))
        return self

    def march(self):
        self._check(self.lib.fdtd_batch_march(self.h))
        return self

    def set_chi(self, rows, strides, n_tau: int, out):
        """chi snapshots at rows[i] with detector stride strides[i] into the device
        tensor `out` (complex128, n x n_tau); rows=None switches them off"""
        if rows is None:
            self._check(self.lib.fdtd_batch_set_chi(self.h, None, None, 0, None))
            return self
        self._rows = np.ascontiguousarray(rows, dtype=np.int64)
        self._strides = np.ascontiguousarray(strides, dtype=np.int64)
        self._check(self.lib.fdtd_batch_set_chi(self.h, self._rows.ctypes.data_as(ctypes.c_void_p),
                                                self._strides.ctypes.data_as(ctypes.c_void_p), int(n_tau),
                                                ctypes.c_void_p(out.data_ptr())))
        return self

    def sample_pe(self, n_samples: int, out, t_end=None):
        """P_e at n_samples equally spaced times of each instance's window (or of
        [0, t_end[i]], a float64 device tensor) into the device tensor `out`
        (float64, n x n_samples)"""
        te = ctypes.c_void_p(t_end.data_ptr()) if t_end is not None else None
        self._check(self.lib.fdtd_batch_sample_pe(self.h, int(n_samples), te, ctypes.c_void_p(out.data_ptr())))
        return out

    def info(self) -> dict:
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self.lib.fdtd_batch_info(self.h, ctypes.byref(a), ctypes.byref(b)))
        return {"launches": int(a.value), "max_workgroups": int(b.value)}

    def _ro(self, i, what, arg, count, dtype):
        out = np.empty(count, dtype=dtype)
        self._check(self.lib.fdtd_batch_readout(self.h, int(i), what, int(arg), out.ctypes.data_as(ctypes.c_void_p),
                                                int(count), 0))
        return out

    def readout_device(self, i, what, arg, dst, count):
        """readout into a device tensor (enqueued on the batch's stream)"""
        self._check(self.lib.fdtd_batch_readout(self.h, int(i), what, int(arg), ctypes.c_void_p(dst.data_ptr()),
                                                int(count), 1))

    def _p(self, i):
        # out-of-range indices go to the library, which reports them
        return self.arr[i] if 0 <= i < self.n else FdtdParams(Nx=0, Nt=0)

    def row_values(self, i: int, rho: int) -> np.ndarray:
        return self._ro(i, RO_ROW, rho, self._p(i).Nx + 1, np.complex128)

    def pe(self, i: int, count: int | None = None) -> np.ndarray:
        return self._ro(i, RO_PE, 0, self._p(i).Nt + 1 if count is None else count, np.float64)

    def chi(self, i: int, count: int) -> np.ndarray:
        return self._ro(i, RO_CHI, 0, count, np.complex128)

    def E(self, i: int) -> np.ndarray:
        return self._ro(i, RO_E, 0, self._p(i).Nt + 1, np.complex128)

    def lam(self, i: int, count: int | None = None) -> np.ndarray:
        """lambda(t_r) of App. D for a stimulated-emission instance (mu is not tracked in batches)"""
        return self._ro(i, RO_LAMBDA, 0, self._p(i).Nt + 1 if count is None else count, np.float64)

    def mu(self, i: int, count: int) -> np.ndarray:
        return self._ro(i, RO_MU, 0, count, np.complex128)

    def sync(self):
        self._check(self.lib.fdtd_batch_sync(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.lib.fdtd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
