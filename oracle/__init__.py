"""CPU oracle of the HDM pseudopotential lattice Boltzmann step (TEST INFRASTRUCTURE).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg may
import this module.  The GPU library never uses it; the two share no code.
The arithmetic lives in ``lbm_oracle.cpp``; this file only marshals numpy
arrays through ctypes.
"""
from .oracle import *  # noqa: F401,F403
