"""Seeded synthetic workloads shared by the oracle and the GPU path.

This package only draws random numbers and lays out gate lists (names, qubit
positions, parameters).  It holds none of the simulation arithmetic: no gate
matrices, no amplitudes.  Both the CPU oracle and the HIP library turn these
gate lists into matrices with their own, independent gate tables.
"""
from .circuits import (  # noqa: F401
    Gate,
    grid_rqc,
    ladder_rqc,
    ansatz_circuit,
    ansatz_observable,
    trajectory_batch,
    config_circuit,
    GRID_CONFIGS,
)
