"""lmag: MI355X-native differentiable Lindblad-Magnus pulse propagator.

The compute path is the HIP library liblmag.so (C ABI in include/lmag.h);
this package is its Python binding. Build with
``python -m paper_2511_13330_amd.build``.
"""
from ._lib import LmagError, lib, LIB_PATH
from .system import System, PulseFidelity, spin_chain_system
from .spin import chain_operators
from .hubbard import hubbard_operators, hubbard_system

__all__ = ["LmagError", "lib", "LIB_PATH", "System", "PulseFidelity",
           "spin_chain_system", "chain_operators", "hubbard_operators", "hubbard_system"]
