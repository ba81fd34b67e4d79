"""Lattice box-spline evaluation on MI355X (gfx950).

Fast evaluation of the lattice convolution sum f(x) = sum_n c_n phi(x - n)
with the scheme of Horacsek & Alim, "Automatic Generation of Interpolants
for Lattice Samplings: Part I" (Sec. 4, Algorithm 1), as hand-written HIP
kernels behind a C ABI (include/lsp.h).  This module is the thin Python
layer: it marshals torch device tensors and the current HIP stream into the
C calls; PyTorch only provides memory and streams.
"""

from . import _lib
from ._lib import LSP_BF16, LSP_F16, LSP_F32, LSP_F64, LspError  # noqa: F401
from .api import LatticeSpline, Volume  # noqa: F401
from .autograd import lattice_spline  # noqa: F401

__all__ = ["LatticeSpline", "Volume", "lattice_spline", "LspError"]
