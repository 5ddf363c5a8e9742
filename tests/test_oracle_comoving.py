"""Pins of the FP64 oracle in an expanding (comoving) box, Sec. III.

Closed forms for the Einstein-de Sitter kick and drift factors, linear growth
of a single lattice mode against the ODE that the discrete scheme implies,
and the Layzer-Irvine energy budget.
"""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from oracle import Params
from synth import lattice_cells


def _eds(n=16, hbar_m=0.0):
    return Params(n=n, box=float(n), S=1.5, hbar_m=hbar_m, comoving=True,
                  omega_m=1.0, omega_l=0.0, h0=1.0)


def test_kick_drift_factors_eds_closed_form():
    p = _eds()
    for a0, a1 in ((0.01, 0.02), (0.3, 0.31), (0.5, 1.0)):
        fg, fq = oracle.kick_factors(a0, a1, p)
        # H = a^-3/2: int a^-1/2 da and int a^-3/2 da
        assert abs(fg - 2 * (math.sqrt(a1) - math.sqrt(a0))) < 1e-12 * fg
        assert abs(fq - 2 * (1 / math.sqrt(a0) - 1 / math.sqrt(a1))) < 1e-12 * fq
        assert abs(oracle.drift_factor(a0, a1, p) - fq) < 1e-12 * fq


def test_kick_factors_lcdm_additive():
    p = Params(n=8, box=8.0, S=0.45, hbar_m=0.0, comoving=True)
    a0, am, a1 = 0.1, 0.2, 0.4
    f01 = oracle.kick_factors(a0, a1, p)
    f0m = oracle.kick_factors(a0, am, p)
    fm1 = oracle.kick_factors(am, a1, p)
    for i in range(2):
        assert abs(f01[i] - f0m[i] - fm1[i]) < 1e-13 * f01[i]


def _mode_amp(pos, n, mode=1):
    q = lattice_cells(n, n)
    disp = (pos[:, 0] - q[:, 0] + n / 2) % n - n / 2
    basis = np.sin(2 * np.pi * mode * q[:, 0] / n)
    return float(disp @ basis / (basis @ basis))


def test_linear_growth_eds_cdm():
    """CDM in Einstein-de Sitter: the lattice mode feels S cos^2(k dx/2) xi
    (discrete linear response of CIC deposit, 7-point Green's function,
    central gradient and CIC interpolation), so xi ~ a^alpha with
    alpha^2 + alpha/2 - 3/2 cos^2(k dx/2) = 0 (alpha = 1 in the continuum)."""
    n = 16
    p = _eds(n)
    c2 = math.cos(math.pi / n) ** 2
    alpha = (-0.5 + math.sqrt(0.25 + 6 * c2)) / 2
    a0, a1, steps = 0.1, 1.0, 200
    q = lattice_cells(n, n)
    eps = 1e-4
    xi = eps * np.sin(2 * np.pi * q[:, 0] / n)
    pos = q.copy()
    pos[:, 0] += xi
    vel = np.zeros_like(pos)
    vel[:, 0] = alpha * math.sqrt(a0) * xi    # p = a^2 dxi/dt = alpha H0 sqrt(a) xi
    times = np.exp(np.linspace(math.log(a0), math.log(a1), steps + 1))
    x, v = oracle.run(pos, vel, p, times)
    ratio = _mode_amp(x, n) / eps
    assert abs(ratio - 10 ** alpha) < 2e-4 * 10 ** alpha
    assert abs(10 ** alpha - 10.0) > 0.1   # the discrete exponent is visibly not 1


def test_linear_mode_fdm_lcdm_against_ode():
    """Flat LCDM with quantum pressure: the same lattice mode obeys
    dxi/da = p/(a^3 H), dp/da = [S C2/(a^2 H) - (hbar/m)^2 (K^2)^2 C2/4/(a^3 H)] xi,
    which crosses the quantum Jeans scale during the run (Eq. (19): k_J grows
    as a^(1/4)).  Integrated to 1e-12 with an adaptive ODE solver."""
    n = 16
    om = 0.3
    p = Params(n=n, box=float(n), S=1.5 * om, hbar_m=1.0, comoving=True, omega_m=om,
               omega_l=1 - om, h0=1.0)
    kdx = 2 * math.pi * 2 / n
    k2 = 4 * math.sin(kdx / 2) ** 2
    c2 = math.cos(kdx / 2) ** 2

    def hub(a):
        return math.sqrt(om / a ** 3 + 1 - om)

    def rhs(a, y, hm=p.hbar_m):
        xi, pp = y
        h = hub(a)
        return [pp / (a ** 3 * h), (p.S * c2 / (a * a * h) - hm ** 2 * k2 * k2 * c2 / 4 / (a ** 3 * h)) * xi]

    a0, a1, steps = 0.05, 0.5, 400
    eps = 1e-4
    sol = solve_ivp(rhs, (a0, a1), [eps, 0.0], rtol=1e-12, atol=1e-20)
    cdm = solve_ivp(lambda a, y: rhs(a, y, 0.0), (a0, a1), [eps, 0.0], rtol=1e-12, atol=1e-20)
    q = lattice_cells(n, n)
    pos = q.copy()
    pos[:, 0] += eps * np.sin(2 * np.pi * 2 * q[:, 0] / n)
    times = np.exp(np.linspace(math.log(a0), math.log(a1), steps + 1))
    x, _ = oracle.run(pos, np.zeros_like(pos), p, times)
    got = _mode_amp(x, n, mode=2)
    want = sol.y[0, -1]
    # the Q term matters: without it the mode grows several times more
    assert cdm.y[0, -1] > 2 * abs(want)
    assert abs(got - want) < 2e-3 * eps, (got, want, cdm.y[0, -1])


def _li_cdm_modes(n):
    """EdS, CDM, eight explicit Fourier modes in Zel'dovich growing-mode form
    (x = q + a psi, p = a^(3/2) psi), the same physical field at every n."""
    rng = np.random.default_rng(3)
    q = lattice_cells(n, n) / n
    psi = np.zeros_like(q)
    for m in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, -1, 1), (2, 1, 0)]:
        k = 2 * np.pi * np.array(m, float)
        ph = rng.random() * 2 * np.pi
        amp = 0.3 * rng.standard_normal()
        psi += amp * np.outer(np.cos(q @ k + ph), k / (k @ k))
    a_vals = np.exp(np.linspace(math.log(0.02), math.log(0.2), 61))
    pos = ((q + a_vals[0] * psi) % 1.0) * n
    vel = a_vals[0] ** 1.5 * psi * n
    p = Params(n=n, box=float(n), S=1.5, hbar_m=0.0, comoving=True, omega_m=1.0, omega_l=0.0)
    return p, pos, vel, a_vals


def _li_fdm_mode(n):
    """Flat LCDM with quantum pressure, one linear lattice mode, steps from
    the time-step rule (omega_max dt <= 0.5, d ln a <= 0.02)."""
    om = 0.3
    p = Params(n=n, box=float(n), S=1.5 * om, hbar_m=0.006 * n * n, comoving=True,
               omega_m=om, omega_l=1 - om)
    q = lattice_cells(n, n)
    pos = q.copy()
    pos[:, 0] += 1e-3 * n / 16 * np.sin(2 * np.pi * q[:, 0] / n)
    a = 0.1
    a_vals = [a]
    while a < 0.5:
        a = min(0.5, oracle.timestep(p, a, 0.0, c_q=0.5, dlna_max=0.02))
        a_vals.append(a)
    return p, pos, np.zeros_like(pos), np.array(a_vals)


def _li_run(setup, n):
    p, x, v, a_vals = setup(n)
    series = [oracle.energies(x, v, p, a_vals[0])]
    acc = None
    for a0, a1 in zip(a_vals[:-1], a_vals[1:]):
        x, v, acc = oracle.kdk_step(x, v, p, a0, a1, acc)
        series.append(oracle.energies(x, v, p, a1))
    return a_vals, series


@pytest.mark.slow
@pytest.mark.parametrize("setup", [_li_cdm_modes, _li_fdm_mode])
def test_layzer_irvine_second_order(setup):
    """Layzer-Irvine budget dE/da = -(2K + W + 2U)/a.  The paper has no
    cosmic-energy test (its sub-percent figure is for a static soliton).  As
    for the static energy, the mesh-gradient force is conjugate to W and U
    only to O((k dx)^2): the residual must fall about 4x per mesh doubling
    for the same physical field, and be near or below 1e-2 at 32^3.  A wrong
    power of a in any energy term destroys the budget."""
    a16, s16 = _li_run(setup, 16)
    a32, s32 = _li_run(setup, 32)
    e16 = np.max(oracle.layzer_irvine_error(a16, s16))
    e32 = np.max(oracle.layzer_irvine_error(a32, s32))
    assert e32 < 1.6e-2, (e16, e32)
    assert 3.3 < e16 / e32 < 5.5, (e16, e32)
    assert abs(s32[-1]["W"]) > 0.9 * abs(s32[0]["W"])
    term = "U" if setup is _li_fdm_mode else "K"
    wrong = [dict(e, **{term: e[term] * a}) for e, a in zip(s32, a32)]
    for e in wrong:
        e["E"] = e["K"] + e["W"] + e["U"]
    assert np.max(oracle.layzer_irvine_error(a32, wrong)) > 5 * e32


def test_timestep_rule():
    p = Params(n=32, box=32.0, S=0.45, hbar_m=0.1, comoving=True)
    a = 0.1
    a1 = oracle.timestep(p, a, vmax=0.0)
    assert a1 > a
    # displacement limit: p/a^2 * dt <= 0.5 cell
    a1v = oracle.timestep(p, a, vmax=1e3)
    dt = math.log(a1v / a) / oracle.hubble(a, p)
    assert 1e3 / a ** 2 * dt <= 0.5 + 1e-9
    ps = Params(n=16, box=1.0, S=1.0, hbar_m=0.01)
    dts = oracle.timestep(ps, 0.0, vmax=0.0)
    assert abs(dts * oracle.omega_max(ps) - 0.5) < 1e-12
