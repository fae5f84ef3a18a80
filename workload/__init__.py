"""Seeded synthetic suspensions of active spring dumbbells.

This package is shared by the CPU oracle tests and the GPU path. It draws the
initial conditions only (positions, phases, system sizes). It holds none of the
method's arithmetic: no forces, no mobility, no integrator.
"""
from .suspensions import (  # noqa: F401
    Params,
    Suspension,
    Ensemble,
    PRESETS,
    make_single,
    make_ensemble,
    make_preset,
    place_dumbbells,
)
from .arrays import (  # noqa: F401
    fig1_params,
    lattice_array,
    array_runs,
    rotation_pair,
    rotation_pairs,
    checkerboard_phases,
)
