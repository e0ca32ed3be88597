"""MI355X (gfx950) implementation of the autoencoder-compressed adjoint
gradient and Gauss-Newton Hessian-vector product of the acoustic
velocity-strain inverse problem (Wittmer, Badger, Sundar, Bui-Thanh,
arXiv 2304.04781).

The computation lives in the HIP library libwavecomp.so (C ABI declared in
include/wavecomp.h). `_lib` binds it with ctypes under the same names,
`solver.WaveSolver` manages a context and its device buffers with torch,
and `autograd.WaveMisfit` exposes J(c), its gradient and Hv to
torch.autograd. PyTorch only provides device memory and streams.
"""
from . import _lib  # noqa: F401

__all__ = ["_lib"]
