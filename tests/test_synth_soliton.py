"""Pins of the solitonic-core initial conditions (Sec. II B): the ground
state of the Schroedinger-Poisson system must satisfy relations that the
shooting solve does not impose.

* virial: a stationary self-gravitating state has 2 K + W = 0 (K the
  gradient energy K_rho of Eq. (6) -- the velocity field is zero -- and W the
  gravitational energy);
* eigenvalue: multiplying the stationary equation by psi and integrating gives
  gamma M = K + 2 W (with V -> 0 at infinity), so gamma = -3 K / M;
* scale symmetry, Eq. (16): the solve at psi0 = 4 (lambda = 2) gives
  r95 / 2, 2 M, 8 K, 8 W and a central potential 4 U(0);
* the residual of both radial equations on the output grid is small and
  psi has no node.
"""

import math

import numpy as np
import pytest

from synth.soliton import ground_state, soliton_state


@pytest.fixture(scope="module")
def gs():
    return ground_state()


def test_virial_and_eigenvalue(gs):
    assert abs(2 * gs["K"] + gs["W"]) < 1e-6 * abs(gs["W"])
    assert abs(gs["gamma"] * gs["M"] - (gs["K"] + 2 * gs["W"])) < 1e-5 * gs["K"]
    assert math.isclose(gs["gamma"], -3 * gs["K"] / gs["M"], rel_tol=1e-5)


def test_scale_symmetry_eq16(gs):
    g2 = ground_state(4.0)
    assert math.isclose(g2["r95"], gs["r95"] / 2, rel_tol=1e-6)
    assert math.isclose(g2["M"], 2 * gs["M"], rel_tol=1e-6)
    assert math.isclose(g2["K"], 8 * gs["K"], rel_tol=1e-6)
    assert math.isclose(g2["W"], 8 * gs["W"], rel_tol=1e-6)
    assert math.isclose(g2["U0"], 4 * gs["U0"], rel_tol=1e-6)
    assert math.isclose(g2["gamma"], 4 * gs["gamma"], rel_tol=1e-6)


def test_ode_residual_and_shape(gs):
    r, psi, v = gs["r"], gs["psi"], gs["V"]
    h = r[1] - r[0]
    keep = (r > 0.05) & (r < 0.8 * gs["r95"] * 2)
    i = np.nonzero(keep)[0]
    d2psi = (psi[i + 1] - 2 * psi[i] + psi[i - 1]) / h ** 2
    dpsi = (psi[i + 1] - psi[i - 1]) / (2 * h)
    u = v[i] - gs["gamma"]
    res = d2psi + 2 * dpsi / r[i] - 2 * u * psi[i]
    assert np.max(np.abs(res)) < 1e-5
    d2v = (v[i + 1] - 2 * v[i] + v[i - 1]) / h ** 2
    dv = (v[i + 1] - v[i - 1]) / (2 * h)
    assert np.max(np.abs(d2v + 2 * dv / r[i] - psi[i] ** 2)) < 1e-5
    nz = psi[psi != 0.0]
    assert np.all(nz > 0) and np.all(np.diff(nz) <= 0)        # nodeless, decreasing
    assert gs["psi0"] == 1.0 and abs(psi[0] - 1.0) < 1e-9


def test_sampled_particles(gs):
    st, units = soliton_state(64, 20000, 9.3, seed=4, gs=gs)
    x = st.pos - 32.0
    r = np.sqrt((x * x).sum(axis=1)) * units["dx"]
    # enclosed-mass fractions of the sample follow the profile
    for q in (0.25, 0.5, 0.95):
        rq = float(np.interp(q * gs["M"], gs["M_enc"], gs["r"]))
        assert abs(np.mean(r < rq) - q) < 0.02
    assert math.isclose(units["box"], 64 * gs["r95"] / 9.3)
    assert np.all(st.vel32 == 0.0)
    assert math.isclose(units["four_pi_G_rhobar"], gs["M"] / units["box"] ** 3)
