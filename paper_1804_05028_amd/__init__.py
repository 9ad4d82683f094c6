"""MI355X-native symmetry-sector exact diagonalisation (sublattice coding).

The hot path -- basis build, representative search, index lookup, bond-loop
H.v, Lanczos and its adjoint -- runs in the HIP kernels of ``libed.so``
behind the C ABI in ``include/ed.h``; this package only marshals arguments.
"""
from . import _lib  # noqa: F401
from ._lib import EDError  # noqa: F401

__all__ = ["_lib", "EDError", "ed"]


def __getattr__(name):
    if name == "ed":
        import importlib
        return importlib.import_module(__name__ + ".ed")
    raise AttributeError(name)
