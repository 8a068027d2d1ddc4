"""Seeded synthetic inputs for the multigrid-ISDF exchange path.

This package only *describes* systems: cell, atoms, uncontracted Gaussian
shells, grid ladders, thresholds and a random closed-shell density matrix.
It holds none of the ISDF arithmetic (no grids are evaluated, no points are
selected, no Coulomb metric is formed), so both the FP64 oracle and the GPU
path may import it without sharing any of the method.
"""
from .diamond import (  # noqa: F401
    BOHR_PER_ANGSTROM,
    System,
    config,
    diamond_system,
    tiny_system,
    periodic_overlap,
    random_density,
    level_bounds,
    batched_cells,
    primitive_norm,
    LARGE_SHELLS,
    bond_orbitals,
)
from .selector_init import initial_weights  # noqa: F401
