"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds only input generation: a SplitMix64 stream, FCC lattice
coordinates, optional jitter and initial velocities.  It contains none of the
simulation arithmetic (no distances, cells, forces or integration), so both
the CPU oracle and the HIP path can consume its arrays without sharing any of
the method's code.
"""

from .lattice import (  # noqa: F401
    SplitMix64,
    fcc_lattice_constant,
    fcc_positions,
    md_system,
    batched_box_specs,
    MDInput,
    SDInput,
    sd_system,
    sd_half_domain,
)
