"""MI355X (gfx950) mortar coupling operators: search, segment-based
integration of D, M and the weighted gap, CSR assembly, reverse-mode
gradients and batched evaluation, as a HIP library behind a C ABI
(include/mortar_mi355x.h) with a thin ctypes binding."""

from . import _capi  # noqa: F401
from ._capi import MortarError, lib  # noqa: F401

__all__ = ["MortarError", "lib", "MortarInterface", "MortarFunction", "default_params", "build"]


def build():
    from .build_lib import build as _b
    return _b()


def __getattr__(name):
    if name in ("MortarInterface", "MortarFunction", "default_params"):
        from . import interface
        return getattr(interface, name)
    if name in ("MortarBatch",):
        from . import batch
        return getattr(batch, name)
    raise AttributeError(name)
