"""MI355X-native open-boundary RPY mobility (the N-body solver of libMobility).

The compute path is the HIP library ``librpy.so`` (gfx950) behind the C
interface ``include/rpy.h``; this package only marshals torch device tensors
into it.  Importing the package loads the library and raises ImportError
when it has not been built.
"""
from . import _lib
from ._lib import NotConvergedError, RpyError, Status

_lib.load()

from .solver import AdamsBashforth, Batch, Solver, mdot  # noqa: E402

NBody = Solver

__all__ = ["Solver", "NBody", "Batch", "AdamsBashforth", "mdot", "RpyError", "NotConvergedError", "Status"]
