"""FP64 CPU oracle for the fuzzy-dark-matter particle-mesh step.

TEST INFRASTRUCTURE ONLY.  This package is the independent, deliberately
slow and plain reference that the GPU path is checked against.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product library never does, and it shares no code with the
HIP kernels or their host library.

Every function follows a passage of Veltmaat & Niemeyer (2016),
"Cosmological particle-in-cell simulations with ultralight axion dark
matter" (arXiv:1608.00802); the passage is cited in each docstring.
"""

from .pm import (  # noqa: F401
    Params,
    cic_index_weights,
    deposit,
    green_discrete,
    poisson,
    qpot,
    grad_central,
    interp_cic,
    fields,
    forces,
    hubble,
    kick_factors,
    drift_factor,
    step_factors,
    kdk_step,
    run,
    energies,
    gradient_energy,
    kinetic_split,
    density_rms_diff,
    layzer_irvine_error,
    omega_max,
    timestep,
    power_spectrum,
    spline_w,
    spline_dw,
    spline_deposit,
    spline_qforce,
    spline_kinetic_rho,
    spline_forces,
    spline_run,
    spline_energies,
)
