"""CPU FP64 oracle for the completed double-layer Stokes system.

TEST INFRASTRUCTURE ONLY: it may be imported by the tests, by the entry-point
smoke check and by the CPU-baseline leg of the benchmark, and by nothing
else.  It shares no code with the GPU path; the two meet only in the seeded
input generators of ``stokes_inputs``.
"""
from . import dlp, solve  # noqa: F401
