"""MI355X-native particle-mesh step for fuzzy dark matter (arXiv:1608.00802).

The compute path is the HIP library libfdmpm.so (C ABI in include/fdmpm.h);
this package holds its ctypes binding, the build script and the serving loop.
"""

from ._lib import (  # noqa: F401
    EXPORTED,
    PM_BATCH_GRAPH,
    PM_CONTINUE,
    PM_FIXED32,
    PM_FP32,
    PM_SORT_AUTO,
    PM_SORT_EVERY,
    PMBatch,
    PMContext,
    PMError,
    PMParams,
    load_library,
    make_params,
    pm_batch_step,
    pm_deposit,
    pm_destroy,
    pm_density_rms_diff,
    pm_energy,
    pm_force,
    pm_init,
    pm_kinetic_split,
    pm_poisson,
    pm_power_spectrum,
    pm_qpot,
    pm_sort,
    pm_spline_density,
    pm_spline_qforce,
    pm_spline_step,
    pm_spline_energy,
    pm_step,
    pm_step_energies,
    pm_timing_enable,
    pm_timing_read,
    pm_workspace_bytes,
)
