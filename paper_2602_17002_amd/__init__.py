"""MI355X-native (gfx950) Total Lagrangian internal force, adjoint and tangent kernels.

The computation lives in the HIP library ``libtlfea.so`` behind the C ABI of
``include/tlfea.h``; this package only marshals arguments.  Importing
``Mesh`` or ``TLInternalForce`` loads the library and fails loudly if it has
not been built.
"""
from ._lib import AUTOTUNE, BATCHED, H8, KEEP_ORDER, MR, NH, PLAIN, Q27, SVK, T10, TlfeaError  # noqa: F401

__all__ = ["Mesh", "TLInternalForce", "internal_force", "TlfeaError",
           "T10", "H8", "Q27", "SVK", "MR", "NH", "PLAIN", "BATCHED", "AUTOTUNE", "KEEP_ORDER"]


def __getattr__(name):
    if name == "Mesh":
        from .mesh import Mesh
        return Mesh
    if name in ("TLInternalForce", "internal_force"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
