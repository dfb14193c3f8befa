"""MI355X (gfx950) implementation of the hot path of FEWHA, the Finite Element
Wavelet Hybrid Algorithm for MCAO atmospheric tomography (Stadler & Ramlau,
arXiv 2202.11945): the matrix-free operator of the wavelet-domain MAP system
inside a fixed-iteration Jacobi-preconditioned CG, warm restart and open-loop
control, as hand-written HIP kernels behind a C ABI (include/fewha.h).

Importing the package loads ``lib/libfewha.so``; if it is not built the
import fails (``python paper_2202_11945_amd/build.py`` builds it).
"""

from . import _abi  # noqa: F401  (loads the library or raises)
from ._abi import FewhaError  # noqa: F401
from .fewha import Batch, Context  # noqa: F401
