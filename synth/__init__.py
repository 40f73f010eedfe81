"""Seeded synthetic devices shared by the GPU path's tests/bench and the CPU oracle.

This module only produces inputs: tight-binding Hamiltonians (CSR), site
coordinates, contact site lists with their lead parameters, and energy grids.
It holds none of the solver's arithmetic (no self-energies, no Green's
functions).  Everything is deterministic given the seed.
"""
from .devices import (  # noqa: F401
    Device,
    cuboid,
    orbital_cuboid,
    random_graph_device,
    dna_ladder,
    chain,
    trilayer,
    energy_grid,
    config0_device,
    config1_device,
    config2_devices, config2_sizes,
    config3_device,
    learned_grid_device,
)
