"""MI355X (gfx950) FDTD solver for the 1+1D delay PDE of waveguide QED
(Fang, arXiv:1707.05943).

The compute path is the HIP library `libfdtd.so` behind the C ABI of
`include/fdtd.h`; `fdtd.py` marshals arguments to it with ctypes and uses
PyTorch only for device memory and streams.  Importing this package loads
nothing; the library is loaded on first use and its absence is an error.
"""
__all__ = ["fdtd", "workloads"]
