"""Checks of the seeded input generators (not part of the step itself)."""

import math

import numpy as np

import oracle
from oracle import Params
from synth import (comoving_code_params, from_fixed, growth_factor, growth_rate,
                   hbar_over_m_mpc_kms, lattice_cells, sine_mode_state, to_fixed,
                   transfer_cdm_eh98, transfer_fdm_hu2000, zeldovich_state)


def test_fixed_point_round_trip_and_wrap():
    rng = np.random.default_rng(0)
    for n in (32, 256, 512):
        pos = rng.random((1000, 3)) * n
        f = to_fixed(pos, n)
        assert f.dtype == np.uint32 and f.shape == (3, 1000)
        back = from_fixed(f, n)
        d = (back - pos + n / 2) % n - n / 2
        assert np.max(np.abs(d)) <= 0.5 * n / 2 ** 32 + 1e-12
    # a position equal to the box side wraps to zero
    assert to_fixed(np.array([[32.0, 0.0, 31.999999999999]]), 32)[0, 0] == 0


def test_hbar_over_m_value():
    # 1e-22 eV: hbar c^2 / (m c^2) = 0.0191715 Mpc km/s
    assert abs(hbar_over_m_mpc_kms(1e-22) - 0.0191715) < 2e-7
    cp = comoving_code_params(10.0, 256, 1e-22, 0.7)
    # (Mpc/h)^2 H0 = 100/h Mpc km/s; dx = 10/256 Mpc/h
    assert abs(cp["hbar_m_cells"] - 0.0191715 * 0.7 / 100 / (10 / 256) ** 2) < 1e-5


def test_growth_eds_and_lcdm():
    assert abs(growth_factor(0.3, 1.0, 0.0) - 0.3) < 1e-10
    assert abs(growth_rate(0.3, 1.0, 0.0) - 1.0) < 1e-9
    # LCDM: early times matter dominated, later suppressed; f ~ Om(a)^0.55
    assert abs(growth_factor(1e-3, 0.3, 0.7) / 1e-3 - 1.0) < 1e-3
    om_a = 0.3 / (0.3 + 0.7)
    assert abs(growth_rate(1.0, 0.3, 0.7) - om_a ** 0.55) < 0.01


def test_transfer_functions_limits():
    assert abs(transfer_cdm_eh98(1e-5, 0.3, 0.7) - 1.0) < 1e-3
    t = transfer_cdm_eh98(np.logspace(-3, 2, 50), 0.3, 0.7)
    assert np.all(np.diff(t) < 0)
    assert abs(transfer_fdm_hu2000(0.0, 1e-22, 0.7) - 1.0) < 1e-15
    # cut-off: beyond x ~ 2 the FDM transfer is below 1e-2
    kcut = 2.0 * 9.0 / 1.61 / 0.7
    assert abs(transfer_fdm_hu2000(kcut, 1e-22, 0.7)) < 1e-2


def test_sine_mode_state():
    st = sine_mode_state(32, 2, 1e-3)
    q = lattice_cells(32, 32)
    d = st.pos - q
    assert np.allclose(d[:, 1:], 0.0)
    s = np.sin(2 * np.pi * 2 * q[:, 0] / 32)
    assert np.max(np.abs(d[:, 0] - 1e-3 * s)) <= 0.5 * 32 / 2 ** 32 + 1e-15  # half a fixed-point unit


def test_zeldovich_linear_density():
    """Deposit of Zel'dovich positions at small amplitude reproduces
    -div(psi) computed from the same displacement (first order), and the
    measured P(k) grows as D^2 between two scale factors."""
    n = 32
    st1 = zeldovich_state(n, 10.0, 0.01, seed=5, m_ev=1e-22)
    st2 = zeldovich_state(n, 10.0, 0.01, seed=5, m_ev=1e-22, a_eval=0.02)
    p = Params(n=n, box=float(n), S=1.0, hbar_m=0.0)
    d1 = oracle.deposit(st1.pos, p) - 1
    d2 = oracle.deposit(st2.pos, p) - 1
    _, p1, _ = oracle.power_spectrum(d1, 10.0)
    _, p2, _ = oracle.power_spectrum(d2, 10.0)
    g = growth_factor(0.02, 0.3, 0.7) / growth_factor(0.01, 0.3, 0.7)
    ratio = p2[1:8] / p1[1:8]
    assert np.all(np.abs(ratio / g ** 2 - 1) < 0.02)
    # momenta: p = a^2 H f D psi, so p / (x - q) = a^2 E(a) f(a) for every particle
    q = lattice_cells(n, n)
    disp = (st1.pos - q + n / 2) % n - n / 2
    e = math.sqrt(0.3 / 0.01 ** 3 + 0.7)
    k = 0.01 ** 2 * e * growth_rate(0.01, 0.3, 0.7)
    big = np.abs(disp) > 1e-3
    assert np.allclose(st1.vel[big] / disp[big], k, rtol=1e-3)


def test_power_spectrum_estimator_sine():
    n, box = 16, 5.0
    x = np.arange(n)
    amp = 0.1
    delta = amp * np.cos(2 * np.pi * 3 * x / n)[:, None, None] * np.ones((1, n, n))
    k, pk, cnt = oracle.power_spectrum(delta, box)
    # a real cosine of amplitude A has |delta_k|^2 = (A n^3 / 2)^2 in two modes
    expect_total = 2 * (amp * n ** 3 / 2) ** 2 * box ** 3 / n ** 6
    assert abs(pk[2] * cnt[2] - expect_total) < 1e-12 * expect_total
    assert np.all(pk[np.arange(len(pk)) != 2] < 1e-25)
