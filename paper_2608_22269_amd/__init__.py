"""MI355X (gfx950) implementation of the well-balanced WCSPH hot path.

The computation lives in the HIP library ``lib/libwbsph.so`` (C ABI in
``include/wbsph.h``); this package only marshals arguments to it.
"""
from . import _lib  # noqa: F401

__all__ = ["Simulation", "build"]


def build():
    from .buildlib import build as _build
    return _build()


def __getattr__(name):
    if name == "Simulation":
        from .sim import Simulation
        return Simulation
    raise AttributeError(name)
