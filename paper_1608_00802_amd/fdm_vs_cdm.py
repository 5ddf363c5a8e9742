"""FDM against CDM from identical initial conditions (Sec. III).

Zel'dovich initial conditions at z = 100 (first test: CDM transfer function,
to z = 18.5; second test: the FDM transfer function of the boson mass, to
z = 2.38) are evolved twice: once with quantum pressure (boson mass m, comoving
Q of Eq. (18)) and once without (hbar/m = 0), on one step schedule.  The
power spectra of both runs are then compared shell by shell, (P_FDM -
P_CDM) / P_CDM, beside the quantum Jeans wavenumber k_J(a) of Eq. (19) at the
start and at the end: growth is suppressed above k_J and unchanged well below
it.  Every step and every spectrum runs through the library (pm_step,
pm_power_spectrum, pm_density_rms_diff); this module only plans the steps and
reports.

With the cloud-in-cell deposit and mesh gradients (--coupling cic) the FDM
run also develops growth near the grid scale (k above about half the mesh
Nyquist wavenumber) on fine meshes, and the velocity bound then shortens the
steps, hence the step cap; the paper's own spline coupling (--coupling
spline) stays stable there.

Units follow the library's comoving convention: lengths in Mpc/h, time in
1/H0, hbar/m in (Mpc/h)^2 H0.  The paper's box of L = 2 Mpc is 1.4 Mpc/h at
h = 0.7; its cosmology is Omega_m = 0.25, Omega_Lambda = 0.75.

    python -m paper_1608_00802_amd.fdm_vs_cdm --n 256
    python -m paper_1608_00802_amd.fdm_vs_cdm --ics fdm --box 1.75 --z-end 2.38 --n 512 \
        --coupling spline
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from .serve import OMEGA_MAX_COEF, hbar_over_m

A_START = 1.0 / 101.0     # z = 100
A_END = 1.0 / 19.5        # z = 18.5


def jeans_k(a: float, hm: float, omega_m: float) -> float:
    """Eq. (19) in comoving units: k_J = (16 pi G rho_bar a)^(1/4) (m/hbar)^(1/2)
    with 4 pi G rho_bar = (3/2) Omega_m H0^2, so k_J = (6 Omega_m a)^(1/4) /
    sqrt(hbar/m) for hbar/m in (Mpc/h)^2 H0; returns h/Mpc."""
    return (6.0 * omega_m * a) ** 0.25 / math.sqrt(hm)


def plan_chunk(a: float, count: int, hm_cells: float, vmax: float, omega_m: float,
               a_end: float = A_END, c_q: float = 0.5, c_x: float = 1.0,
               dlna_max: float = 0.02) -> list:
    """Up to `count` further scale factors after a, each step bounded as in
    Sec. II A (no particle moves more than c_x cells: dx/dt = p/a^2 with p
    at most vmax cells H0) and by the quantum-pressure stability bound
    omega_max dt <= c_q, omega_max = 1.1155 (hbar/m)/(a^2 dx^2); both taken
    at the step's start, where they are tightest in the matter era."""
    out = []
    while len(out) < count and a < a_end:
        hub = math.sqrt(omega_m / a ** 3 + 1.0 - omega_m)
        d = dlna_max
        if hm_cells > 0:
            d = min(d, c_q * hub * a * a / (OMEGA_MAX_COEF * hm_cells))
        if vmax > 0:
            d = min(d, c_x * a * a * hub / vmax)
        nxt = a * math.exp(d)
        if nxt >= a_end * (1.0 - 1e-12):
            nxt = a_end
        out.append(nxt)
        a = nxt
    return out


def run(n: int = 256, box: float = 1.4, m_ev: float = 2.5e-22, seed: int = 1,
        omega_m: float = 0.25, h: float = 0.7, a_start: float = A_START, a_end: float = A_END,
        chunk: int = 10, device=None, keep_states: bool = False, max_steps: int = 4000,
        progress=None, ics: str = "cdm", coupling: str = "cic", h_spline: float = 3.5) -> dict:
    """ics = "cdm": initial power with the CDM transfer function (the first
    test); "fdm": with the FDM transfer function of the same boson mass
    (the second test, Fig. 6), both runs still starting from one state.
    coupling = "cic": the fused cloud-in-cell step (pm_step); "spline": the
    paper's own coupling (pm_spline_step, smoothing length h_spline cells),
    the particles re-sorted by tile every chunk."""
    import torch

    import paper_1608_00802_amd as pm
    from synth import zeldovich_state

    dev = device if device is not None else torch.device("cuda:0")
    if ics not in ("cdm", "fdm"):
        raise ValueError("ics: 'cdm' or 'fdm'")
    if coupling not in ("cic", "spline"):
        raise ValueError("coupling: 'cic' or 'spline'")
    st = zeldovich_state(n, box, a_start, seed, m_ev=m_ev if ics == "fdm" else None, om=omega_m,
                         h=h)
    hm = hbar_over_m(m_ev, h)
    hm_cells = hm / (box / n) ** 2

    def params(hbar_m):
        return pm.make_params(n, n ** 3, box, precision=pm.PM_FIXED32, comoving=True,
                              omega_m=omega_m, omega_l=1.0 - omega_m, h0=1.0,
                              hbar_over_m=hbar_m, rho_floor=1e-6, rho_fp64_below=1e-3)

    ctx_f = pm.PMContext(params(hm), device=dev)
    ctx_c = pm.PMContext(params(0.0), device=dev)
    pos0 = torch.from_numpy(np.ascontiguousarray(st.pos_fixed.view(np.int32))).to(dev)
    vel0 = torch.from_numpy(np.ascontiguousarray(st.vel32)).to(dev)
    pos_f, vel_f = pos0.clone(), vel0.clone()
    pos_c, vel_c = pos0.clone(), vel0.clone()
    k, p_start, counts = ctx_c.power_spectrum(pos0)
    times = [a_start]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flags = pm.PM_SORT_AUTO
    while times[-1] < a_end and len(times) - 1 < max_steps:
        # velocity bound of both runs, with room for a doubling within the chunk
        vmax = 2.0 * max(float(vel_f.abs().max().item()), float(vel_c.abs().max().item()))
        nxt = plan_chunk(times[-1], chunk, hm_cells, vmax, omega_m, a_end)
        seg = [times[-1]] + nxt
        if coupling == "spline":
            for ctx, p_, v_ in ((ctx_f, pos_f, vel_f), (ctx_c, pos_c, vel_c)):
                ctx.sort(p_, v_)
                ctx.spline_step(p_, v_, seg, h_spline)
        else:
            ctx_f.step(pos_f, vel_f, seg, flags=flags)
            ctx_c.step(pos_c, vel_c, seg, flags=flags)
        flags = pm.PM_SORT_AUTO | pm.PM_CONTINUE
        times += nxt
        if progress is not None and (len(times) - 1) % (10 * chunk) < chunk:
            progress(f"a = {times[-1]:.5f} after {len(times) - 1} steps, |p|max = {vmax / 2:.4g}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, p_f, _ = ctx_f.power_spectrum(pos_f)
    _, p_c, _ = ctx_c.power_spectrum(pos_c)
    rms, cells = ctx_c.density_rms_diff(pos_f, pos_c)
    p_f, p_c, p_start = np.asarray(p_f), np.asarray(p_c), np.asarray(p_start)
    out = {
        "n": n, "box_mpch": box, "m_ev": m_ev, "hbar_over_m": hm, "omega_m": omega_m,
        "ics": ics, "coupling": coupling,
        "seed": seed, "a_start": a_start, "a_end": times[-1], "steps": len(times) - 1,
        "reached_a_end": times[-1] >= a_end,
        "wall_s": wall, "finite": bool(torch.isfinite(vel_f).all().item()
                                       and torch.isfinite(vel_c).all().item()),
        "k": list(k), "modes": list(counts), "P_start": list(p_start),
        "P_cdm": list(p_c), "P_fdm": list(p_f), "rel_diff": list((p_f - p_c) / p_c),
        "k_J_start": jeans_k(a_start, hm, omega_m), "k_J_end": jeans_k(times[-1], hm, omega_m),
        "rms_rel_density_diff": rms, "rms_cells": cells, "times": times,
    }
    if keep_states:
        out["states"] = {"pos0": pos0, "vel0": vel0, "pos_fdm": pos_f, "pos_cdm": pos_c}
    ctx_f.close()
    ctx_c.close()
    return out


def summary(res: dict) -> dict:
    """Largest and smallest relative difference with their k; mean relative
    difference well below k_J(start), between the two Jeans scales, and
    above twice k_J(end)."""
    k = np.asarray(res["k"])
    rd = np.asarray(res["rel_diff"])
    lo = k < 0.5 * res["k_J_start"]
    mid = (k >= res["k_J_start"]) & (k <= res["k_J_end"])
    hi = k > 2.0 * res["k_J_end"]
    pick = lambda m: float(rd[m].mean()) if m.any() else None  # noqa: E731
    top = int(np.argmax(rd))
    return {"max_rel_diff": float(rd[top]), "k_at_max": float(k[top]),
            "min_rel_diff": float(rd.min()), "k_at_min": float(k[int(np.argmin(rd))]),
            "below_half_kJ_start": pick(lo), "between_kJ": pick(mid),
            "above_2kJ_end": pick(hi),
            "growth_cdm_above_2kJ_end": float(np.mean(np.asarray(res["P_cdm"])[hi] /
                                                      np.asarray(res["P_start"])[hi]))
            if hi.any() else None,
            "growth_fdm_above_2kJ_end": float(np.mean(np.asarray(res["P_fdm"])[hi] /
                                                      np.asarray(res["P_start"])[hi]))
            if hi.any() else None}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--box", type=float, default=1.4, help="box side in Mpc/h")
    ap.add_argument("--m-ev", type=float, default=2.5e-22)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--ics", choices=("cdm", "fdm"), default="cdm",
                    help="transfer function of the initial power (first or second test)")
    ap.add_argument("--z-end", type=float, default=1.0 / A_END - 1.0)
    ap.add_argument("--coupling", choices=("cic", "spline"), default="cic",
                    help="fused cloud-in-cell step, or the paper's spline kernel (h = 3.5 cells)")
    ap.add_argument("--max-steps", type=int, default=4000,
                    help="stop there (the velocity bound shortens the steps of a run gone unstable)")
    args = ap.parse_args(argv)
    res = run(args.n, args.box, args.m_ev, args.seed, a_end=1.0 / (1.0 + args.z_end),
              max_steps=args.max_steps, ics=args.ics, coupling=args.coupling,
              progress=lambda msg: print(msg, file=sys.stderr, flush=True))
    res.pop("times")
    res["summary"] = summary(res)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
