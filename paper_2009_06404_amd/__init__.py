"""MI355X (gfx950) implementation of the D2Q9 single-relaxation-time lattice
Boltzmann step for elastic waves (Escande, Kolluru, Cleon & Sagaut, arXiv
2009.06404): hand-written HIP kernels behind the C ABI of include/lbm.h
(liblbm.so), with a thin ctypes binding (``_lib``) and a ``Solver`` that owns
the torch tensors the library borrows."""
from . import _lib
from ._lib import LBMError
from .solver import Solver
from .autograd import ShotTraces, shot_traces

__all__ = ["Solver", "LBMError", "ShotTraces", "shot_traces", "_lib"]
