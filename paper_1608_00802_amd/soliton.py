"""A single solitonic core in a static periodic box (Sec. II B, the test of
Fig. 1): the ground state of the Schroedinger-Poisson system sampled with
equal-mass particles at rest, evolved with the paper's spline coupling
(pm_spline_step, h = 4 cells) or with cloud-in-cell (pm_step), recording the
kinetic energy K_v, the gradient energy K_rho, the gravitational energy W_g
and their sum E.  The paper reports E conserved to better than 1e-2 and a
stable oscillation of the profile about the ground state, K_rho and W_g
exchanging energy with the quasinormal period.

Units are those of the ground state (hbar/m = 1, 4 pi G = 1, central
amplitude psi0 = 1); the core is scaled so that r95 (the radius holding 95%
of its mass) spans r95_cells mesh cells (18.6 in the paper, with N = 1e6
particles).  The box's mean density enters the Poisson equation's
background (4 pi G rho_bar = M / L^3).  Energies are in the library's units
(mean density as mass unit, cells as length unit); only their changes
relative to |E| are reported.

Steps obey the static-box form of the Sec. II A condition (no particle moves
more than c_x cells in a step) and omega_max dt <= c_q with the quantum
pressure's largest frequency on the mesh, 1.1155 (hbar/m)/dx^2 (a bound the
spline kernel's smoothing only lowers).

    python -m paper_1608_00802_amd.soliton --coupling spline --t-end 60
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from .serve import OMEGA_MAX_COEF


def run(n: int = 128, npart: int = 10 ** 6, r95_cells: float = 18.6, coupling: str = "spline",
        h: float = 4.0, t_end: float = 60.0, seed: int = 1, chunk: int = 20,
        c_x: float = 1.0, c_q: float = 0.5, device=None, progress=None) -> dict:
    import torch

    import paper_1608_00802_amd as pm
    from synth.soliton import soliton_state

    if coupling not in ("spline", "cic"):
        raise ValueError("coupling: 'spline' or 'cic'")
    dev = torch.device(device if device is not None else "cuda:0")
    st, u = soliton_state(n, npart, r95_cells, seed)
    hm_cells = u["hbar_m"] / u["dx"] ** 2
    params = pm.make_params(n, npart, u["box"], precision=pm.PM_FIXED32, comoving=False,
                            four_pi_G_rhobar=u["four_pi_G_rhobar"], hbar_over_m=u["hbar_m"],
                            rho_floor=1e-6, rho_fp64_below=1e-3)
    ctx = pm.PMContext(params, device=dev)
    pos = torch.from_numpy(np.ascontiguousarray(st.pos_fixed.view(np.int32))).to(dev)
    vel = torch.from_numpy(np.ascontiguousarray(st.vel32)).to(dev)
    dt_q = c_q / (OMEGA_MAX_COEF * hm_cells)

    def energy():
        if coupling == "spline":
            return ctx.spline_energy(pos, vel, 1.0, h)
        return ctx.energy(pos, vel, 1.0)

    t = 0.0
    series = {"t": [0.0], "K_v": [], "K_rho": [], "W_g": [], "E": []}

    def record(e):
        series["K_v"].append(e["K"])
        series["K_rho"].append(e["U"])
        series["W_g"].append(e["W"])
        series["E"].append(e["E"])

    record(energy())
    steps = 0
    flags = pm.PM_SORT_AUTO
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while t < t_end * (1.0 - 1e-12):
        vmax = 2.0 * float(vel.abs().max().item())
        dt = dt_q if vmax == 0.0 else min(dt_q, c_x / vmax)
        k = max(1, min(chunk, int(math.ceil((t_end - t) / dt))))
        times = [t + i * dt for i in range(k + 1)]
        times[-1] = min(times[-1], t_end)
        if coupling == "spline":
            ctx.sort(pos, vel)
            ctx.spline_step(pos, vel, times, h)
            series["t"].append(times[-1])
            record(energy())
        else:
            # energies of every step from the step's own kernels (row 0 is
            # the previous call's last row)
            rows = torch.empty((k + 1, 4), dtype=torch.float64, device=dev)
            ctx.step_energies(pos, vel, times, rows, flags=flags)
            flags = pm.PM_SORT_AUTO | pm.PM_CONTINUE
            for tt_, r in zip(times[1:], rows[1:].cpu().numpy()):
                series["t"].append(tt_)
                record({"K": r[0], "W": r[1], "U": r[2], "E": r[3]})
        t = times[-1]
        steps += k
        if progress is not None:
            progress(f"t = {t:.3f} after {steps} steps, dE/|E0| = "
                     f"{(series['E'][-1] - series['E'][0]) / abs(series['E'][0]):+.3e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e = np.asarray(series["E"])
    w = np.asarray(series["W_g"])
    tt = np.asarray(series["t"])
    out = {"n": n, "npart": npart, "r95_cells": r95_cells, "coupling": coupling,
           "h_cells": h if coupling == "spline" else None, "t_end": t, "steps": steps,
           "dt_quantum_bound": dt_q, "wall_s": wall, "units": {k: v for k, v in u.items()
                                                              if k != "ground_state"},
           "max_rel_energy_change": float(np.max(np.abs(e - e[0])) / abs(e[0])),
           "period_W_g": oscillation_period(tt, w),
           "finite": bool(torch.isfinite(vel).all().item()), "series": series}
    ctx.close()
    return out


def oscillation_period(t, y) -> float | None:
    """Mean spacing of successive upward crossings of the series' mean after
    the first quarter of the run (the breathing period), or None."""
    t = np.asarray(t)
    y = np.asarray(y)
    keep = t >= t[-1] / 4
    t, y = t[keep], y[keep] - np.mean(y[keep])
    up = np.nonzero((y[:-1] < 0) & (y[1:] >= 0))[0]
    if up.size < 2:
        return None
    tc = t[up] - y[up] * (t[up + 1] - t[up]) / (y[up + 1] - y[up])
    return float(np.mean(np.diff(tc)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--npart", type=int, default=10 ** 6)
    ap.add_argument("--r95-cells", type=float, default=18.6)
    ap.add_argument("--coupling", default="spline", choices=("spline", "cic"))
    ap.add_argument("--h", type=float, default=4.0)
    ap.add_argument("--t-end", type=float, default=60.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--series", action="store_true", help="print the energy series too")
    args = ap.parse_args(argv)
    res = run(args.n, args.npart, args.r95_cells, args.coupling, args.h, args.t_end, args.seed,
              progress=lambda s: print(s, file=sys.stderr, flush=True))
    if not args.series:
        res.pop("series")
    print(json.dumps(res))


if __name__ == "__main__":
    main()
