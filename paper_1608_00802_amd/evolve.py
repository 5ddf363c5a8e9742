"""Advance a comoving context's state under the time-step condition of
Sec. II A: no particle moves farther than one mesh cell in a step, and the
quantum-pressure force stays resolved (omega_max dt <= 1/2, omega_max =
1.1155 (hbar/m)/(a^2 dx^2) for the 7-point Q with central-difference
gradients on the particle lattice).

The step sizes are planned on the host in chunks: before each chunk the
largest canonical momentum component of the state is read back and doubled
(momenta grow inside a chunk), and every step of the chunk is bounded by it
at the step's start, where the bound is tightest in the matter era.  The
steps themselves are pm_step calls (continued calls keep the merged kicks).
"""

from __future__ import annotations

import math

from .fdm_vs_cdm import plan_chunk


def evolve(ctx, pos, vel, a_start: float, a_end: float, hm_cells: float, omega_m: float,
           chunk: int = 10, safety: float = 2.0, dlna_max: float = math.log(100.0) / 150.0,
           flags: int = 0, continued: bool = False, max_steps: int = 100000) -> list:
    """Step (pos, vel) of context ``ctx`` from a_start to a_end.

    hm_cells: hbar/m in cells^2 H0; flags: extra pm_step flags (a sort
    mode).  continued: the context's fields are those of pos already.
    Returns the schedule of scale factors taken (a_start first, a_end last).
    """
    from ._lib import PM_CONTINUE
    times = [float(a_start)]
    cont = continued
    while times[-1] < a_end:
        if len(times) - 1 >= max_steps:
            raise RuntimeError(f"evolve: more than {max_steps} steps before a = {a_end}")
        vmax = safety * float(vel.abs().max().item())
        nxt = plan_chunk(times[-1], chunk, hm_cells, vmax, omega_m, a_end=a_end,
                         dlna_max=dlna_max)
        ctx.step(pos, vel, [times[-1]] + nxt, flags=flags | (PM_CONTINUE if cont else 0))
        cont = True
        times.extend(nxt)
    return times


def plan(a_start: float, count: int, hm_cells: float, vmax: float, omega_m: float,
         dlna_max: float = math.log(100.0) / 500.0) -> list:
    """``count`` further steps after a_start under the same bounds (for a
    timed run of fixed length that starts from an evolved state; no end)."""
    return [float(a_start)] + plan_chunk(a_start, count, hm_cells, vmax, omega_m,
                                         a_end=math.inf, dlna_max=dlna_max)
