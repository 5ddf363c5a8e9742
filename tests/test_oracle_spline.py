"""Pins of the oracle's spline-kernel functions (Sec. II A: density from
particles with the kernel of Eq. (15), Eq. (9); quantum force by the kernel
gradient, Eq. (14)).

Against: the kernel's normalisation as a continuous integral and its
continuity, a numerical derivative of W, a brute-force double loop with the
periodic minimum image, the uniform density of a node lattice, and -- the
strongest pin -- the force as minus the particle derivative of the discrete
energy K_rho of Eq. (11) (finite differences of the energy, which also fixes
the sign read for Eq. (14) and its dx^3 and m factors).  CPU only.
"""

import math

import numpy as np
from scipy import integrate

import oracle
from oracle import Params


def test_s1_kernel_normalisation_and_continuity():
    for h in (1.0, 3.5, 4.0):
        tot, _ = integrate.quad(lambda r: 4 * math.pi * r * r * float(oracle.spline_w(r, h)),
                                0.0, h, points=[0.5 * h], epsabs=1e-14, epsrel=1e-13)
        assert abs(tot - 1.0) < 1e-12
        e = 1e-9 * h
        assert abs(oracle.spline_w(0.5 * h - e, h) - oracle.spline_w(0.5 * h + e, h)) < 1e-7
        assert abs(oracle.spline_dw(0.5 * h - e, h) - oracle.spline_dw(0.5 * h + e, h)) < 1e-6
        assert oracle.spline_w(h, h) == 0.0 and oracle.spline_w(1.2 * h, h) == 0.0
        assert math.isclose(oracle.spline_w(0.0, h), 8.0 / (math.pi * h ** 3), rel_tol=1e-15)


def test_s2_derivative_matches_w():
    h = 3.5
    r = np.linspace(0.05, 3.45, 40)
    d = 1e-6
    num = (oracle.spline_w(r + d, h) - oracle.spline_w(r - d, h)) / (2 * d)
    assert np.allclose(oracle.spline_dw(r, h), num, rtol=1e-6, atol=1e-10)


def test_s3_brute_force_density():
    rng = np.random.default_rng(3)
    p = Params(n=8, box=4.0, S=1.0, hbar_m=0.0)
    h = 2.5 * p.dx
    pos = rng.random((5, 3)) * p.box
    mp = p.box ** 3 / 5
    want = np.zeros((8, 8, 8))
    for q in pos:
        for j in range(8):
            for k in range(8):
                for l in range(8):
                    d = np.array([j, k, l]) * p.dx - q
                    d -= p.box * np.round(d / p.box)       # minimum image
                    want[j, k, l] += mp * float(oracle.spline_w(math.sqrt(d @ d), h))
    got = oracle.spline_deposit(pos, p, h)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15)


def test_s4_node_lattice_is_uniform_and_mass_is_kept():
    n = 16
    p = Params(n=n, box=float(n), S=1.0, hbar_m=0.0)
    g = np.arange(n, dtype=np.float64)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    lat = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    rho = oracle.spline_deposit(lat, p, 3.5)
    assert np.ptp(rho) < 1e-12 * rho.mean()
    # the discrete sum of W over nodes approximates its unit integral
    assert abs(rho.mean() - 1.0) < 2e-3
    rng = np.random.default_rng(4)
    rho = oracle.spline_deposit(rng.random((3000, 3)) * n, p, 3.5)
    assert abs(rho.mean() - 1.0) < 2e-3


def test_s5_force_is_minus_energy_gradient():
    # a jittered lattice keeps rho well above the floor, so Q of the oracle
    # is exactly the node derivative of K_rho (forward differences)
    n = 16
    p = Params(n=n, box=float(n), S=1.0, hbar_m=0.7)
    h = 3.5
    rng = np.random.default_rng(5)
    g = np.arange(n, dtype=np.float64) + 0.5
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) + 0.3 * rng.standard_normal((n ** 3, 3))
    pos %= n
    rho = oracle.spline_deposit(pos, p, h)
    assert rho.min() > 0.1
    q = oracle.qpot(rho, p)
    acc = oracle.spline_qforce(pos, q, p, h)
    npart = pos.shape[0]
    d = 1e-4
    for i in (77, 1234):
        for ax in range(3):
            pp, pm_ = pos.copy(), pos.copy()
            pp[i, ax] += d
            pm_[i, ax] -= d
            de = (oracle.spline_kinetic_rho(pp, p, h) - oracle.spline_kinetic_rho(pm_, p, h)) / (2 * d)
            want = -(npart / p.box ** 3) * de
            assert abs(acc[i, ax] - want) <= 1e-6 * np.abs(acc).max() + 1e-5 * abs(want), \
                (i, ax, acc[i, ax], want)


def test_s6_spline_leapfrog_conserves_the_discrete_energy():
    # Sec. II A: the kernel-gradient force conserves K_v + K_rho of Eqs. (8),
    # (11) by construction, so the leapfrog's energy error (gravity off) falls
    # as dt^2: a factor near 4 per halving of the step
    n = 12
    p = Params(n=n, box=float(n), S=0.0, hbar_m=0.8)
    h = 3.5
    rng = np.random.default_rng(6)
    g = np.arange(n, dtype=np.float64) + 0.5
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = (np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
           + 0.25 * rng.standard_normal((n ** 3, 3))) % n
    vel = np.zeros_like(pos)
    mp = p.box ** 3 / pos.shape[0]

    def energy(xx, vv):
        return 0.5 * mp * float(np.sum(vv * vv)) + oracle.spline_kinetic_rho(xx, p, h)

    e0 = energy(pos, vel)
    errs = []
    for steps in (4, 8):
        t = np.linspace(0.0, 1.2, steps + 1)
        xx, vv = oracle.spline_run(pos, vel, p, t, h)
        errs.append(abs(energy(xx, vv) - e0))
    # the run converts a sizeable part of K_rho into motion
    assert 0.5 * mp * float(np.sum(vv * vv)) > 0.05 * e0
    assert 3.0 < errs[0] / errs[1] < 5.5, errs


def test_s7_spline_energies_terms():
    # U is the K_rho whose particle gradient the force is (pinned above); W
    # vanishes without gravity and equals the CIC form's expression on the
    # spline density; K is Eq. (8)
    n = 16
    rng = np.random.default_rng(7)
    pos = rng.random((3000, 3)) * n
    vel = rng.standard_normal((3000, 3))
    p0 = Params(n=n, box=float(n), S=0.0, hbar_m=0.6)
    e = oracle.spline_energies(pos, vel, p0, 3.5)
    assert e["W"] == 0.0
    assert np.isclose(e["U"], oracle.spline_kinetic_rho(pos, p0, 3.5), rtol=1e-13)
    assert np.isclose(e["K"], 0.5 * (n ** 3 / 3000) * np.sum(vel * vel), rtol=1e-13)
    p1 = Params(n=n, box=float(n), S=1.0, hbar_m=0.6)
    e1 = oracle.spline_energies(pos, vel, p1, 3.5, a=1.0)
    delta = oracle.spline_deposit(pos, p1, 3.5) - 1.0
    assert e1["W"] < 0.0
    assert np.isclose(e1["W"], 0.5 * np.sum(delta * oracle.poisson(delta, p1)), rtol=1e-12)
