"""MI355X (gfx950) implementation of the implicit regularized enthalpy
lattice Boltzmann method (IREBM) for the two-phase Stefan problem
(Luddens, Lothode, Danaila, arXiv 2505.13097).

The compute path is the C ABI of liblbm_stefan.so (include/lbm_stefan.h);
this package only marshals arguments, with PyTorch supplying device
memory and streams.  There is no CPU fallback: if the library is not
built, using it raises LibraryMissing.
"""
from ._lib import LbmError, LibraryMissing  # noqa: F401
from .stefan import (HotWallFront, Stefan, StefanBatch, make_params,  # noqa: F401
                     step_noalloc, variant_names,
                     workspace_bytes)

__version__ = "0.1.0"
