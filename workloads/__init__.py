"""Seeded synthetic inputs for the SPH particle update.

This package only builds initial particle sets and parameter records (geometry,
lattices, seeded jitter, the nondimensional Re/We mapping). It holds none of the
per-step arithmetic of the method; both the HIP library and the CPU oracle are
fed from here.
"""
from .scenarios import (  # noqa: F401
    FLUID,
    WALL,
    PISTON,
    INACTIVE,
    WENDLAND,
    CUBIC,
    System,
    Batch,
    dam_break,
    rest_tank,
    jet,
    paper_jet,
    batch_sweep,
    circle,
    sinusoid,
    flat_slab,
    random_cloud,
    lattice_block,
    round_for_dtype,
    hydrostatic_density,
)
from . import scenarios, groups  # noqa: F401
