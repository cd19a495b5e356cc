"""FP64 CPU oracle of the porous-media cascaded lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
benchmark's cpu_baseline leg may import this package.  It shares no code with
the GPU library (paper_2110_05943_amd) and never imports it.
"""
from . import params  # noqa: F401
from .oracle import (EAST, NORTH, SOUTH, WEST, Lattice, feq, geq, lib, matrix, meq,  # noqa: F401
                     mteq, neq, Sraw, St)
