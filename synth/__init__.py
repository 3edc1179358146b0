"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This package only generates inputs (particle positions and momenta); it holds
none of the particle-mesh step's arithmetic and imports neither the oracle nor
the HIP binding.
"""
from .ics import (  # noqa: F401
    Cosmology, lattice_positions, zeldovich_ics, uniform_particles,
    clustered_particles, edge_particles, power_eh, power_law, sigma_r,
)
