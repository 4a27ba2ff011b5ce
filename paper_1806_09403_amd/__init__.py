"""MI355X (gfx950) library for the boundary-thickening direct-forcing
immersed-boundary lattice Boltzmann method (Jiang & Liu, arXiv 1806.09403).

The compute lives in ``libbtdf.so`` (HIP kernels behind the C ABI of
include/btdf.h); ``api`` exposes each C call under its own name and ``Sim``
wraps one simulation with torch-owned device memory and stream.
"""
from ._lib import (BtdfError, BtdfUnstable, COS4, LINEAR2, PESKIN4, ROMA3, PERIODIC, VELOCITY_INLET,
                   ZERO_GRADIENT_OUTLET, BOUNCEBACK_WALL, FREE_SLIP_WALL, CONVECTIVE_OUTLET, load)
from .sim import BatchSim, Sim

__all__ = ["Sim", "BatchSim", "BtdfError", "BtdfUnstable", "load", "COS4", "LINEAR2", "PESKIN4", "ROMA3",
           "PERIODIC", "VELOCITY_INLET", "ZERO_GRADIENT_OUTLET", "BOUNCEBACK_WALL", "FREE_SLIP_WALL",
           "CONVECTIVE_OUTLET"]
