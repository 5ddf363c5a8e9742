"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package builds particle states only (lattices, a single sine mode,
Zel'dovich initial conditions) and converts them between float cell
coordinates and 32-bit fixed point.  It contains none of the particle-mesh
step's arithmetic (no deposit, Poisson solve, quantum pressure, gradient,
interpolation or time integration).
"""

from .ics import (  # noqa: F401
    State,
    lattice_cells,
    sine_mode_state,
    zeldovich_state,
    to_fixed,
    from_fixed,
    quantize_state,
    hbar_over_m_mpc_kms,
    comoving_code_params,
    growth_factor,
    growth_rate,
    transfer_cdm_eh98,
    transfer_fdm_hu2000,
)
