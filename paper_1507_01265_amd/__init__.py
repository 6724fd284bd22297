"""MI355X (gfx950) MPDATA time step behind a C ABI (include/mpdata.h).

Submodules are imported on use: ``inputs`` (seeded synthetic fields, numpy
only), ``solver`` (single-grid solver on torch tensors), ``_lib`` (ctypes
binding of libmpdata.so) and ``build`` (hipcc build of the library).
"""
import importlib

__all__ = ["inputs", "solver", "build", "Solver"]


def __getattr__(name):
    if name in ("inputs", "solver", "build", "_lib"):
        return importlib.import_module(f"{__name__}.{name}")
    if name == "Solver":
        return importlib.import_module(f"{__name__}.solver").Solver
    raise AttributeError(name)
