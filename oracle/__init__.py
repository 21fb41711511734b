"""FP64 CPU oracle for the equilibrium projection of voxelized stress fields.

TEST INFRASTRUCTURE ONLY.  This package is the checker: the tests, the smoke
check and the benchmark's CPU-baseline leg call it; the library never does, and
it shares no code with the HIP implementation.  See ``oracle.equilibrium``.
"""
from .equilibrium import *  # noqa: F401,F403
from .equilibrium import __all__  # noqa: F401
