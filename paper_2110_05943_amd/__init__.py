"""MI355X (gfx950) porous-media cascaded lattice Boltzmann solver.

The coupled D2Q9/D2Q5 cascaded LB time step of Feng, Liu & He
(arXiv:2110.05943) in hand-written HIP (libclb.so, C ABI in include/clb.h),
with a thin ctypes binding.  PyTorch supplies device memory and streams.
"""
from ._binding import (EAST, INLET, NORTH, OUTLET, PERIODIC, SOUTH, STORE_F16,  # noqa: F401
                       STORE_F32, STORE_MIXED, WALL_ADIABATIC, WALL_T, WEST, CLBError, DivergedError,
                       Solver, derive, make_params)
from . import inputs  # noqa: F401
