"""MI355X-native D2Q9 multi-relaxation-time lattice Boltzmann library.

The compute path is the HIP library ``liblbm.so`` (C ABI in include/lbm.h);
this package is its Python binding.  Importing the package does not load the
library; the first call does, and fails loudly if it has not been built.
"""
from . import _lib  # noqa: F401

__all__ = ["Lattice", "load_library"]


def load_library():
    return _lib.load()


def __getattr__(name):
    if name == "Lattice":
        from .lattice import Lattice
        return Lattice
    raise AttributeError(name)
