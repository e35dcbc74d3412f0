"""MI355X-native TRT-R D2Q9 lattice Boltzmann hot path (arXiv:2312.10316).

``lbm`` is the ctypes binding of the C ABI in ``include/lbm.h``; ``Solver`` wraps one context.
The HIP library is loaded on first use and is required: there is no CPU path.
"""
from . import lbm
from .solver import Solver

__all__ = ["lbm", "Solver"]
