"""Pins of the oracle's grid diagnostics: the bulk/dispersion split of the
kinetic energy (Sec. II B, Eq. (17)) and the RMS relative density difference
per cell (Sec. III).

Each test checks against something other than the oracle's own formula:
special states whose split is known in closed form, invariants (Galilean
boosts, the Cauchy-Schwarz bound), a brute-force evaluation of Eq. (17)
particle by particle, and lattice states whose density difference is
counted by hand.  None of these calls a GPU.
"""

import math

import numpy as np

import oracle
from oracle import Params


def _p(n=8, box=8.0):
    return Params(n=n, box=box, S=1.0, hbar_m=0.0)


def _rand_state(rng, npart, box, vscale=1.0):
    return rng.random((npart, 3)) * box, rng.normal(scale=vscale, size=(npart, 3))


# ------------------------------------------------------------ kinetic split

def test_d1_common_velocity_has_no_dispersion():
    # every particle moves with one velocity: v(x) is that velocity at every
    # node with mass, so the whole of K is bulk motion
    rng = np.random.default_rng(1)
    p = _p()
    pos, _ = _rand_state(rng, 700, p.box)
    vel = np.tile(np.array([0.3, -1.7, 0.9]), (700, 1))
    for a in (1.0, 0.25):
        s = oracle.kinetic_split(pos, vel, p, a=a)
        k = 0.5 * (p.box ** 3 / 700) * 700 * float(vel[0] @ vel[0]) / a ** 2
        assert math.isclose(s["K"], k, rel_tol=1e-13)
        assert math.isclose(s["K_bulk"], k, rel_tol=1e-12)
        assert abs(s["K_disp"]) < 1e-12 * k


def test_d2_counter_streaming_pairs_are_pure_dispersion():
    # coincident pairs with opposite velocities: the mass-weighted mean
    # velocity vanishes at every node, so K_bulk = 0 and K_disp = K
    rng = np.random.default_rng(2)
    p = _p()
    half, _ = _rand_state(rng, 300, p.box)
    u = rng.normal(size=(300, 3))
    pos = np.concatenate([half, half])
    vel = np.concatenate([u, -u])
    s = oracle.kinetic_split(pos, vel, p)
    assert abs(s["K_bulk"]) < 1e-12 * s["K"]
    assert math.isclose(s["K_disp"], s["K"], rel_tol=1e-12)


def test_d3_dispersion_is_galilean_invariant():
    # a uniform boost u adds u.P_tot + M u^2/2 to both K and K_bulk (the CIC
    # weights of each particle sum to one), so K_disp does not change
    rng = np.random.default_rng(3)
    p = _p(n=8, box=5.0)
    pos, vel = _rand_state(rng, 900, p.box)
    s0 = oracle.kinetic_split(pos, vel, p)
    s1 = oracle.kinetic_split(pos, vel + np.array([4.0, -2.5, 1.0]), p)
    assert not math.isclose(s0["K"], s1["K"], rel_tol=1e-3)
    assert math.isclose(s0["K_disp"], s1["K_disp"], rel_tol=1e-10)


def test_d4_bulk_is_bounded_by_total():
    # Cauchy-Schwarz per node: |sum w p|^2 <= (sum w) (sum w p^2)
    rng = np.random.default_rng(4)
    for n, npart in ((4, 50), (8, 400), (16, 5000)):
        p = _p(n=n, box=float(n))
        pos, vel = _rand_state(rng, npart, p.box)
        s = oracle.kinetic_split(pos, vel, p)
        assert 0.0 < s["K_bulk"] < s["K"]
        assert s["K_disp"] > 0.0


def test_d5_brute_force_eq17():
    # Eq. (17) evaluated particle by particle and node by node: the velocity
    # field at each node from the kernel sums, then sum rho |v|^2 dx^3 / 2
    rng = np.random.default_rng(5)
    p = Params(n=4, box=2.0, S=1.0, hbar_m=0.0)
    npart = 7
    pos, vel = _rand_state(rng, npart, p.box)
    mp = p.box ** 3 / npart
    dx = p.box / p.n
    num = {}
    den = {}
    for q, v in zip(pos, vel):
        u = q / dx
        base = [int(math.floor(x)) for x in u]
        frac = [x - b for x, b in zip(u, base)]
        for cx in (0, 1):
            for cy in (0, 1):
                for cz in (0, 1):
                    w = ((frac[0] if cx else 1 - frac[0]) * (frac[1] if cy else 1 - frac[1])
                         * (frac[2] if cz else 1 - frac[2]))
                    node = ((base[0] + cx) % p.n, (base[1] + cy) % p.n, (base[2] + cz) % p.n)
                    num[node] = num.get(node, np.zeros(3)) + mp * w * v / dx ** 3
                    den[node] = den.get(node, 0.0) + mp * w / dx ** 3
    bulk = 0.0
    for node, rho in den.items():
        if rho > 0.0:
            vx = num[node] / rho
            bulk += 0.5 * rho * float(vx @ vx) * dx ** 3
    for a in (1.0, 0.5):
        s = oracle.kinetic_split(pos, vel, p, a=a)
        assert math.isclose(s["K_bulk"], bulk / a ** 2, rel_tol=1e-12)
        assert math.isclose(s["K"], 0.5 * mp * float(np.sum(vel * vel)) / a ** 2, rel_tol=1e-13)


def test_d6_particle_on_node_and_split_components():
    # one particle on a node and one at a cell centre with orthogonal
    # velocities in separate cells: every node sees one velocity, so the
    # split is all bulk, component by component
    p = _p()
    pos = np.array([[1.0, 2.0, 3.0], [5.5, 5.5, 5.5]])
    vel = np.array([[2.0, 0.0, 0.0], [0.0, 0.0, -3.0]])
    s = oracle.kinetic_split(pos, vel, p)
    assert math.isclose(s["K_bulk"], s["K"], rel_tol=1e-14)
    # move the second particle onto the first one's node: that node now
    # holds the mean velocity (1, 0, -1.5) of mass 2 m
    pos[1] = pos[0]
    s = oracle.kinetic_split(pos, vel, p)
    mp = p.box ** 3 / 2
    assert math.isclose(s["K_bulk"], 0.5 * 2 * mp * (1.0 + 2.25), rel_tol=1e-14)
    assert math.isclose(s["K"], 0.5 * mp * (4.0 + 9.0), rel_tol=1e-14)


# ------------------------------------------------------ density difference

def _lattice(n, box):
    g = (np.arange(n) * (box / n))
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def test_d7_identical_states_have_zero_difference():
    rng = np.random.default_rng(7)
    p = _p()
    pos, _ = _rand_state(rng, 2000, p.box)
    rms, cnt = oracle.density_rms_diff(pos, pos.copy(), p)
    assert rms == 0.0 and cnt == p.n ** 3


def test_d8_one_particle_moved_on_a_lattice():
    # b: one particle on every node (rho_b = 1).  a: the same, with one
    # particle moved onto a neighbour's node: one node at 0, one at 2, so
    # two nodes have |rel| = 1 and rms = sqrt(2 / n^3)
    p = _p(n=8, box=4.0)
    b = _lattice(p.n, p.box)
    a = b.copy()
    a[10] = a[11]
    rms, cnt = oracle.density_rms_diff(a, b, p)
    assert cnt == p.n ** 3
    assert math.isclose(rms, math.sqrt(2.0 / p.n ** 3), rel_tol=1e-12)


def test_d9_empty_reference_nodes_are_left_out():
    # b: eight particles on each node of the even sublattice (x, y, z even),
    # nothing elsewhere; a: one particle on every node.  Only the n^3/8
    # even nodes count, each with rho_a = 1/8 of rho_b, rel = -7/8
    n = 8
    p = _p(n=n, box=8.0)
    a = _lattice(n, p.box)
    even = a[np.all((np.rint(a).astype(int) % 2) == 0, axis=1)]
    b = np.concatenate([even] * 8)
    assert b.shape == a.shape
    rms, cnt = oracle.density_rms_diff(a, b, p)
    assert cnt == n ** 3 // 8
    assert math.isclose(rms, 7.0 / 8.0, rel_tol=1e-12)
    # and swapped: every node of a has mass; the odd ones of b are -1 off
    rms2, cnt2 = oracle.density_rms_diff(b, a, p)
    assert cnt2 == n ** 3
    rel = np.full(n ** 3, -1.0)
    rel[: n ** 3 // 8] = 7.0
    assert math.isclose(rms2, math.sqrt(float(np.mean(rel * rel))), rel_tol=1e-12)



# ------------------------------------------------------------ power spectrum

def test_d10_power_of_a_z_cosine_counts_its_conjugate():
    # a cosine along z lives at m_z = +-3; the stored half spectrum holds only
    # m_z = 3, which must count twice, giving the same total as along x
    n, box, amp = 16, 5.0, 0.1
    z = np.arange(n)
    delta = amp * np.cos(2 * np.pi * 3 * z / n)[None, None, :] * np.ones((n, n, 1))
    k, pk, cnt = oracle.power_spectrum(delta, box)
    expect_total = 2 * (amp * n ** 3 / 2) ** 2 * box ** 3 / n ** 6
    assert abs(pk[2] * cnt[2] - expect_total) < 1e-12 * expect_total
    assert np.all(pk[np.arange(len(pk)) != 2] < 1e-25)
    assert np.allclose(k, 2 * np.pi * np.arange(1, n // 2 + 1) / box)


def test_d11_shell_counts_by_enumeration():
    # every integer vector of the full n^3 spectrum with |m| in [b - 1/2,
    # b + 1/2) is counted once, whichever half stores it
    n = 12
    delta = np.random.default_rng(0).standard_normal((n, n, n))
    _, _, cnt = oracle.power_spectrum(delta, 1.0)
    m = np.fft.fftfreq(n, 1.0 / n)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    mag = np.sqrt(mx ** 2 + my ** 2 + mz ** 2).ravel()
    for b in range(1, n // 2 + 1):
        assert cnt[b - 1] == np.count_nonzero((mag >= b - 0.5) & (mag < b + 0.5))


def test_d12_power_of_white_noise_is_its_variance():
    # Parseval: for white noise the mean |delta_m|^2 over all modes is
    # n^3 var, so every shell's P is near var * box^3 / n^3
    n, box = 32, 7.0
    rng = np.random.default_rng(1)
    delta = rng.standard_normal((n, n, n)) * 0.3
    _, pk, cnt = oracle.power_spectrum(delta, box)
    expect = 0.09 * box ** 3 / n ** 3
    big = cnt > 500
    assert np.all(np.abs(pk[big] / expect - 1) < 0.15)
