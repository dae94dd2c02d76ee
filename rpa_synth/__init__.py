"""Seeded synthetic inputs (geometry, LRI coefficients, Green's functions, grids,
Coulomb matrices) shared by the oracle and the GPU path.  Holds no step of the
chi0 build, the transforms or the correlation energy."""
from .configs import Cell, config, MASTER_SEED, SPECIES_TABLE  # noqa: F401
from .inputs import Inputs, LRIBlocks, make_inputs, SPIN_FACTOR  # noqa: F401
