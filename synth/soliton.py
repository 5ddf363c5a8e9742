"""Solitonic core initial conditions (Sec. II B, the static-box test of a
single core): the ground state of the Schroedinger-Poisson system and
particles sampled from its density.

The ground state is the nodeless, spherically symmetric stationary solution
Psi = psi(r) exp(-i gamma t) of the two equations of Sec. II A.  In units
hbar/m = 1 and 4 pi G = 1, with rho = psi^2 and U = V - gamma:

    psi'' + (2/r) psi' = 2 U psi,        U'' + (2/r) U' = psi^2,

psi'(0) = U'(0) = 0, psi(0) = psi0, psi -> 0 without nodes.  For psi0 = 1
the central value U(0) is found by bisection (shooting): too low a U(0)
makes psi cross zero, too high makes it turn up again.  Other psi0 follow
from the scale symmetry of Eq. (16) (psi -> lambda^2 psi, r -> r / lambda),
which the tests check against a direct solve.  The potential with V -> 0 at
infinity follows from the enclosed mass, V'(r) = M(<r) / (4 pi r^2), and
gamma = V(0) - U(0).

This module builds inputs only: it holds none of the particle-mesh step's
arithmetic.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.integrate import cumulative_trapezoid, solve_ivp

from .ics import quantize_state


def _rhs(r, y):
    psi, dpsi, u, du = y
    if r == 0.0:
        return [dpsi, 2.0 * u * psi / 3.0, du, psi * psi / 3.0]
    return [dpsi, 2.0 * u * psi - 2.0 * dpsi / r, du, psi * psi - 2.0 * du / r]


def _shoot(u0: float, psi0: float, r_max: float):
    """Integrate outwards from a small radius (series start); returns (-1 if
    psi crossed zero, +1 if it turned upwards, 0 otherwise) and the solution."""
    r0 = 1e-6 / math.sqrt(psi0)
    # series: psi = psi0 (1 + u0 r^2 / 3), U = u0 + psi0^2 r^2 / 6
    y0 = [psi0 * (1.0 + u0 * r0 * r0 / 3.0), 2.0 * psi0 * u0 * r0 / 3.0,
          u0 + psi0 * psi0 * r0 * r0 / 6.0, psi0 * psi0 * r0 / 3.0]

    def crosses(r, y):
        return y[0]
    crosses.terminal = True

    def turns(r, y):
        return y[1]
    turns.terminal = True
    sol = solve_ivp(_rhs, (r0, r_max), y0, events=[crosses, turns], rtol=1e-12, atol=1e-15,
                    dense_output=True)
    if sol.t_events[0].size:
        return -1, sol
    if sol.t_events[1].size:
        return 1, sol
    return 0, sol


def ground_state(psi0: float = 1.0, n_r: int = 40001) -> dict:
    """The nodeless ground state with central amplitude psi0 (units hbar/m = 1,
    4 pi G = 1).  Returns the radial grid and psi, V (zero at infinity), the
    eigenvalue gamma, the mass M, the enclosed mass, the radius r95 holding 95%
    of the mass, K = (1/2) int |grad psi|^2 (= K_rho of Eq. (6)) and
    W = (1/2) int rho V (the gravitational energy W_g)."""
    r_max = 14.0 / math.sqrt(psi0)
    lo, hi = -4.0 * psi0, -0.01 * psi0          # psi crosses at lo, turns up at hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid in (lo, hi):
            break
        s, _ = _shoot(mid, psi0, r_max)
        if s < 0:
            lo = mid
        else:
            hi = mid
    _, sol = _shoot(lo, psi0, r_max)
    r_end = float(sol.t[-1])
    r = np.linspace(0.0, r_end, n_r)
    y = sol.sol(np.maximum(r, sol.t[0]))
    psi, dpsi = y[0].copy(), y[1].copy()
    # beyond the smallest |psi| the shooting solution departs from the bound
    # state (exponentially growing branch): the tail is set to zero there
    cut = int(np.argmin(np.abs(psi)))
    psi[cut:] = 0.0
    dpsi[cut:] = 0.0
    rho = psi * psi
    menc = cumulative_trapezoid(4.0 * np.pi * r * r * rho, r, initial=0.0)
    mass = float(menc[-1])
    # V(r) = -int_r^inf M(<r') / (4 pi r'^2) dr', the mass being complete at r_end
    g = np.zeros_like(r)
    g[1:] = menc[1:] / (4.0 * np.pi * r[1:] ** 2)
    inner = cumulative_trapezoid(g, r, initial=0.0)
    v = -(inner[-1] - inner) - mass / (4.0 * np.pi * r_end)
    gamma = float(v[0] - lo)
    kin = 0.5 * float(np.trapezoid(4.0 * np.pi * r * r * dpsi * dpsi, r))
    pot = 0.5 * float(np.trapezoid(4.0 * np.pi * r * r * rho * v, r))
    r95 = float(np.interp(0.95 * mass, menc, r))
    return {"r": r, "psi": psi, "dpsi": dpsi, "V": v, "U0": lo, "gamma": gamma, "M": mass,
            "M_enc": menc, "r95": r95, "K": kin, "W": pot, "psi0": psi0}


def soliton_state(n_mesh: int, npart: int, r95_cells: float, seed: int, gs: dict | None = None):
    """npart equal-mass particles sampled from the ground-state density
    (radius by the inverse of the enclosed-mass fraction, direction uniform on
    the sphere), centred in a periodic box of n_mesh cells, at rest (the ground
    state's phase is uniform in space, so its velocity field is zero).  The
    core is scaled so that r95 spans r95_cells mesh cells.

    Returns (state, units) with units: dx (box length per cell in the
    ground-state units of psi0 = 1), box, hbar_m (1), four_pi_G_rhobar
    (M / box^3: the box's mean density, 4 pi G = 1) and the ground state."""
    if gs is None:
        gs = ground_state()
    dx = gs["r95"] / r95_cells
    box = n_mesh * dx
    rng = np.random.default_rng(seed)
    frac = rng.random(npart)
    rad = np.interp(frac * gs["M"], gs["M_enc"], gs["r"])
    cost = 2.0 * rng.random(npart) - 1.0
    phi = 2.0 * np.pi * rng.random(npart)
    sint = np.sqrt(1.0 - cost * cost)
    xyz = np.stack([rad * sint * np.cos(phi), rad * sint * np.sin(phi), rad * cost], axis=1)
    pos = (xyz / dx + 0.5 * n_mesh) % n_mesh
    st = quantize_state(pos, np.zeros_like(pos), n_mesh,
                        {"kind": "soliton", "r95_cells": r95_cells, "seed": seed})
    units = {"dx": dx, "box": box, "hbar_m": 1.0, "four_pi_G_rhobar": gs["M"] / box ** 3,
             "ground_state": gs}
    return st, units
