"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Sizes span several tiles and ragged particle counts; tolerances are the
stated targets: relative L2 error below 1e-5 on rho, phi and Q, position
drift below 1e-4 cell after 100 steps of the static single-mode problem.
"""

import math

import numpy as np
import pytest

import oracle
from synth import lattice_cells, sine_mode_state, to_fixed, quantize_state, zeldovich_state

from gpu_helpers import (TWO40, cosmo_setup, mass_mesh, periodic_diff, positions_cells, rel_l2,
                         single_mode_setup, to_device)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm(gpu):
    import paper_1608_00802_amd as pm_mod
    pm_mod.load_library()
    return pm_mod


def _ctx(pm, lp, gpu):
    return pm.PMContext(lp, device=gpu)


def _clustered_state(n, npart, seed, nclumps=6, width=1.5):
    """Particles in a few Gaussian clumps plus a sparse background, so that
    many cells are empty or nearly empty (exercises the floor and the FP64
    path)."""
    rng = np.random.default_rng(seed)
    centres = rng.random((nclumps, 3)) * n
    k = rng.integers(0, nclumps, npart)
    pos = centres[k] + width * rng.standard_normal((npart, 3))
    bg = rng.random(npart) < 0.15
    pos[bg] = rng.random((int(bg.sum()), 3)) * n
    pos %= n
    vel = 0.01 * rng.standard_normal((npart, 3))
    return quantize_state(pos, vel, n, {"kind": "clumps"})


# ------------------------------------------------------------------ deposit

@pytest.mark.parametrize("n,npart", [(16, 3001), (32, 32 ** 3), (64, 40 ** 3 + 17),
                                     (128, 100003), (256, 1 << 20), (512, 1 << 20)])
def test_deposit_exact_mass_and_parity(pm, gpu, n, npart):
    import torch
    rng = np.random.default_rng(n)
    st = quantize_state(rng.random((npart, 3)) * n, np.zeros((npart, 3)), n, {})
    lp = pm.make_params(n, npart, float(n))
    ctx = _ctx(pm, lp, gpu)
    pos, _ = to_device(st, gpu)
    delta = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.deposit(pos, delta)
    torch.cuda.synchronize()
    m = mass_mesh(ctx)
    assert int(m.astype(np.int64).sum()) == npart * 2 ** 40      # exact, integer
    assert m.min() >= 0
    op = oracle.Params(n=n, box=float(n), S=1.0, hbar_m=0.0)
    rho = oracle.deposit(st.pos, op)
    mbar = npart * TWO40 / n ** 3
    # integer weights are rounded to 2^-40 of a particle: <= 4 units per corner
    assert np.max(np.abs(m / mbar - rho)) <= 8 * 4.0 / mbar + 1e-15
    d = delta.cpu().numpy().reshape(n, n, n)
    assert rel_l2(1.0 + d, rho) < 1e-7
    assert rel_l2(d, rho - 1.0) < 1e-6


def test_deposit_bitwise_order_independent(pm, gpu):
    import torch
    n = 32
    st = zeldovich_state(n, 10.0, 0.5, seed=3, m_ev=1e-22)
    lp = pm.make_params(n, st.npart, float(n))
    ctx = _ctx(pm, lp, gpu)
    pos, _ = to_device(st, gpu)
    ctx.deposit(pos)
    m0 = mass_mesh(ctx).copy()
    ctx.deposit(pos)
    assert np.array_equal(mass_mesh(ctx), m0)
    perm = torch.from_numpy(np.random.default_rng(1).permutation(st.npart)).to(gpu)
    ctx.deposit(pos[:, perm].contiguous())
    assert np.array_equal(mass_mesh(ctx), m0)


# ------------------------------------------------------------------ Poisson

@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512])
def test_poisson_sine_closed_form(pm, gpu, n):
    import torch
    lp = pm.make_params(n, n ** 3, float(n), four_pi_G_rhobar=1.7)
    ctx = _ctx(pm, lp, gpu)
    x = np.arange(n)
    m = (1, 2, 3) if n > 16 else (1, 2, 1)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    arg = 2 * np.pi * (m[0] * X + m[1] * Y + m[2] * Z) / n
    d = (0.2 * np.sin(arg)).astype(np.float32)
    phi = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.poisson(torch.from_numpy(d.ravel()).to(gpu), phi)
    k2 = sum(4 * math.sin(math.pi * mm / n) ** 2 for mm in m)
    expect = -1.7 * d.astype(np.float64) / k2
    assert rel_l2(phi.cpu().numpy().reshape(n, n, n), expect) < 2e-6


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512])
def test_poisson_random_vs_oracle(pm, gpu, n):
    import torch
    rng = np.random.default_rng(100 + n)
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    lp = pm.make_params(n, n ** 3, float(n), four_pi_G_rhobar=0.9)
    ctx = _ctx(pm, lp, gpu)
    phi = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.poisson(torch.from_numpy(d.ravel()).to(gpu), phi)
    op = oracle.Params(n=n, box=float(n), S=0.9, hbar_m=0.0)
    dd = d.astype(np.float64)
    ref = oracle.poisson(dd - dd.mean(), op)
    assert rel_l2(phi.cpu().numpy().reshape(n, n, n), ref) < 1e-5


# ------------------------------------------------------------------ Q

@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("precision", [1, 0])
def test_qpot_vs_oracle_smooth(pm, gpu, precision, n):
    """Q of a Zel'dovich state against the oracle's Q of the same density."""
    import torch
    st = zeldovich_state(n, 10.0, 0.3, seed=7, m_ev=1e-22)
    lp, op = cosmo_setup(n, 10.0, 1e-22, precision=precision)
    ctx = _ctx(pm, lp, gpu)
    pos, _ = to_device(st, gpu, fp32_positions=(precision == 0))
    q = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.deposit(pos)
    ctx.qpot(None, q)
    rho = oracle.deposit(positions_cells(pos, n, precision == 0), op)
    ref = oracle.qpot(rho, op)
    err = rel_l2(q.cpu().numpy().reshape(n, n, n), ref)
    assert err < (1e-5 if precision == 1 else 1e-3), err


@pytest.mark.parametrize("n,npart,width", [(32, 20000, 1.5), (128, 200000, 6.0)])
def test_qpot_near_empty_cells_fp64_path(pm, gpu, n, npart, width):
    import torch
    st = _clustered_state(n, npart, seed=5, width=width)
    lp, op = cosmo_setup(n, 5.0, 1e-22)
    lp.n_part = st.npart
    ctx = _ctx(pm, lp, gpu)
    pos, _ = to_device(st, gpu)
    q = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.deposit(pos)
    ctx.qpot(None, q)
    rho = oracle.deposit(st.pos, op)
    ref = oracle.qpot(rho, op)
    got = q.cpu().numpy().reshape(n, n, n)
    low = rho < 1e-3
    assert low.sum() > 100 and (rho == 0).sum() > 10
    assert rel_l2(got, ref) < 1e-5
    assert rel_l2(got[~low], ref[~low]) < 1e-5
    assert rel_l2(got[low], ref[low]) < 1e-5


# ------------------------------------------------------------------ force, one step

def test_force_vs_oracle(pm, gpu):
    import torch
    n = 64
    st = zeldovich_state(n, 10.0, 0.2, seed=11, m_ev=1e-22)
    lp, op = cosmo_setup(n, 10.0, 1e-22)
    ctx = _ctx(pm, lp, gpu)
    pos, _ = to_device(st, gpu)
    acc = torch.empty((3, st.npart), dtype=torch.float32, device=gpu)
    a = 0.2
    ctx.deposit(pos)
    ctx.poisson()
    ctx.qpot()
    ctx.force(pos, acc, a)
    gphi, gq = oracle.forces(st.pos, op)
    ref = gphi / a + gq / a ** 2
    assert rel_l2(acc.cpu().numpy().T, ref) < 1e-5


@pytest.mark.parametrize("a0,precision", [(0.01, 1), (0.3, 1), (0.3, 0)])
def test_one_step_vs_oracle(pm, gpu, a0, precision):
    import torch
    n = 64
    st = zeldovich_state(n, 10.0, a0, seed=1, m_ev=1e-22)
    lp, op = cosmo_setup(n, 10.0, 1e-22, precision=precision)
    ctx = _ctx(pm, lp, gpu)
    fp32 = precision == 0
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    a1 = a0 * math.exp(math.log(100.0) / 500)
    ctx.step(pos, vel, [a0, a1])
    torch.cuda.synchronize()
    x0 = positions_cells(torch.from_numpy(st.pos_f32) if fp32 else
                         torch.from_numpy(st.pos_fixed.view(np.int32)), n, fp32)
    x1, v1 = oracle.kdk_step(x0, st.vel, op, a0, a1)[:2]
    xg = positions_cells(pos, n, fp32)
    vg = vel.cpu().numpy().T.astype(np.float64)
    dx = np.max(np.abs(periodic_diff(xg, x1, n)))
    assert dx < (1e-5 if precision == 1 else 2e-4), dx
    assert rel_l2(vg, v1) < (1e-5 if precision == 1 else 1e-3)
    # fields at the new positions: the GPU's own x1 through the GPU, the
    # same x1 through the oracle (kernel parity at x1)
    dl = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ph = torch.empty_like(dl)
    qq = torch.empty_like(dl)
    ctx.deposit(pos, dl)
    ctx.poisson(None, ph)
    ctx.qpot(None, qq)
    rho, delta, phi, q = oracle.fields(xg, op)
    tol = 1e-5 if precision == 1 else 1e-3
    assert rel_l2(1.0 + dl.cpu().numpy().reshape(n, n, n), rho) < tol
    assert rel_l2(ph.cpu().numpy().reshape(n, n, n), phi) < tol
    assert rel_l2(qq.cpu().numpy().reshape(n, n, n), q) < tol


def test_step_continue_equals_single_call(pm, gpu):
    import torch
    n = 32
    st = zeldovich_state(n, 10.0, 0.05, seed=2, m_ev=1e-22)
    lp, _ = cosmo_setup(n, 10.0, 1e-22)
    times = list(0.05 * np.exp(np.arange(11) * 0.01))
    ctx = _ctx(pm, lp, gpu)
    p1, v1 = to_device(st, gpu)
    ctx.step(p1, v1, times)
    p2, v2 = to_device(st, gpu)
    ctx.step(p2, v2, times[:6])
    ctx.step(p2, v2, times[5:], flags=pm.PM_CONTINUE)
    torch.cuda.synchronize()
    # the only difference: the split call closes and reopens the kick at a_5
    # in two float adds instead of one -- positions agree to rounding
    d = periodic_diff(positions_cells(p1, n), positions_cells(p2, n), n)
    assert np.max(np.abs(d)) < 1e-6
    assert rel_l2(v2.cpu().numpy(), v1.cpu().numpy()) < 1e-6


# ------------------------------------------------------------------ static box, 100 steps

@pytest.mark.parametrize("precision", [1, 0])
def test_single_mode_drift_100_steps(pm, gpu, precision):
    import torch
    st = sine_mode_state(32, 2, 1e-3)
    lp, op = single_mode_setup(precision)
    ctx = _ctx(pm, lp, gpu)
    fp32 = precision == 0
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    times = list(np.arange(101) * 0.01)
    ctx.step(pos, vel, times)
    torch.cuda.synchronize()
    x0 = positions_cells(torch.from_numpy(st.pos_f32) if fp32 else
                         torch.from_numpy(st.pos_fixed.view(np.int32)), 32, fp32)
    xo, vo = oracle.run(x0, st.vel, op, times)
    xg = positions_cells(pos, 32, fp32)
    drift = np.max(np.abs(periodic_diff(xg, xo, 32)))
    if precision == 1:
        assert drift < 1e-4, drift
    # linear theory: amplitude ratio 1.486711 (discrete dispersion + KDK)
    q = lattice_cells(32, 32)
    basis = np.sin(2 * np.pi * 2 * q[:, 0] / 32)
    amp = periodic_diff(xg[:, 0], q[:, 0], 32) @ basis / (basis @ basis)
    amp0 = periodic_diff(x0[:, 0], q[:, 0], 32) @ basis / (basis @ basis)
    if precision == 1:
        assert abs(amp / amp0 - 1.486711) < 1e-4
    else:
        # the plain FP32 form: 1.1e-5 cell of drift measured (inside the 1e-4
        # budget), the growth 2.3e-3 below linear theory (the 1e-3-cell mode is
        # resolved to ~1e-6 cell by FP32 positions near 16 cells)
        assert drift < 5e-5, drift
        assert abs(amp / amp0 - 1.486711) < 5e-3
    print(f"single mode precision={precision}: drift vs oracle {drift:.3e} cell, growth {amp / amp0:.7f}")


# ------------------------------------------------------------------ energies

@pytest.mark.parametrize("n", [32, 128])
def test_energy_vs_oracle(pm, gpu, n):
    st = zeldovich_state(n, 2.0, 0.1, seed=4, m_ev=2.5e-22)
    lp, op = cosmo_setup(n, 2.0, 2.5e-22)
    ctx = _ctx(pm, lp, gpu)
    pos, vel = to_device(st, gpu)
    a = 0.1
    e = ctx.energy(pos, vel, a)
    ref = oracle.energies(st.pos, st.vel, op, a)
    for k in ("K", "W", "U"):
        assert abs(e[k] - ref[k]) < 1e-5 * abs(ref[k]), (k, e[k], ref[k])


def test_fixed_point_wrap_across_boundary(pm, gpu):
    """Particles drifting through the box faces wrap exactly (fixed point)."""
    import torch
    n = 16
    q = lattice_cells(n, n)
    vel = np.zeros_like(q)
    vel[:, 0] = 3.0      # 3 cells per time unit along x
    vel[:, 2] = -1.25
    st = quantize_state(q, vel, n, {})
    lp = pm.make_params(n, n ** 3, float(n), four_pi_G_rhobar=0.0)
    ctx = _ctx(pm, lp, gpu)
    pos, v = to_device(st, gpu)
    ctx.step(pos, v, [0.0, 1.0, 2.0, 3.0, 4.0])
    torch.cuda.synchronize()
    got = pos.cpu().numpy().view(np.uint32)
    expect = to_fixed((q + 4.0 * vel) % n, n)
    assert np.array_equal(got, expect)


def test_comoving_20_steps_vs_oracle(pm, gpu):
    """Twenty merged-kick comoving steps from a = 0.01 (10 Mpc/h cell size,
    m = 1e-22 eV) against the oracle stepping the same schedule."""
    import torch
    n = 64
    box = 10.0 * n / 256
    st = zeldovich_state(n, box, 0.01, seed=1, m_ev=1e-22)
    lp, op = cosmo_setup(n, box, 1e-22)
    ctx = _ctx(pm, lp, gpu)
    pos, vel = to_device(st, gpu)
    times = list(0.01 * np.exp(np.arange(21) * math.log(100.0) / 500))
    ctx.step(pos, vel, times)
    torch.cuda.synchronize()
    xo, vo = oracle.run(st.pos, st.vel, op, times)
    xg = positions_cells(pos, n)
    assert np.max(np.abs(periodic_diff(xg, xo, n))) < 1e-5
    assert rel_l2(vel.cpu().numpy().T, vo) < 1e-5


def test_full_size_256_fields_and_step(pm, gpu):
    """The benchmark workload at full size (10 Mpc/h, 256^3 particles and
    mesh, m = 1e-22 eV, Zel'dovich ICs at a = 0.01) in the launch
    configuration the benchmark times: delta, phi, Q and the force at the
    initial state, then positions and velocities after one step."""
    import torch
    n = 256
    st = zeldovich_state(n, 10.0, 0.01, seed=1, m_ev=1e-22)
    lp, op = cosmo_setup(n, 10.0, 1e-22)
    ctx = _ctx(pm, lp, gpu)
    pos, vel = to_device(st, gpu)
    d = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ph = torch.empty_like(d)
    qq = torch.empty_like(d)
    acc = torch.empty((3, st.npart), dtype=torch.float32, device=gpu)
    a0 = 0.01
    ctx.deposit(pos, d)
    ctx.poisson(None, ph)
    ctx.qpot(None, qq)
    ctx.force(pos, acc, a0)
    torch.cuda.synchronize()
    rho, delta, phi, q = oracle.fields(st.pos, op)
    assert rel_l2(1.0 + d.cpu().numpy().reshape(n, n, n), rho) < 1e-5
    assert rel_l2(d.cpu().numpy().reshape(n, n, n), delta) < 1e-5
    assert rel_l2(ph.cpu().numpy().reshape(n, n, n), phi) < 1e-5
    assert rel_l2(qq.cpu().numpy().reshape(n, n, n), q) < 1e-5
    gphi = oracle.interp_cic(oracle.grad_central(phi, op), st.pos, op)
    gq = oracle.interp_cic(oracle.grad_central(q, op), st.pos, op)
    assert rel_l2(acc.cpu().numpy().T, gphi / a0 + gq / a0 ** 2) < 1e-5
    del rho, delta, phi, q
    a1 = a0 * math.exp(math.log(100.0) / 500)
    ctx.step(pos, vel, [a0, a1])
    torch.cuda.synchronize()
    x1, v1, _ = oracle.kdk_step(st.pos, st.vel, op, a0, a1, (gphi, gq))
    assert np.max(np.abs(periodic_diff(positions_cells(pos, n), x1, n))) < 1e-5
    assert rel_l2(vel.cpu().numpy().T, v1) < 1e-5


# ------------------------------------------------------------------ sort + tiled kernels

def test_sort_is_permutation_by_tile(pm, gpu):
    import torch
    n = 64
    st = zeldovich_state(n, 10.0, 0.5, seed=8, m_ev=1e-22)
    lp, _ = cosmo_setup(n, 10.0, 1e-22)
    ctx = _ctx(pm, lp, gpu)
    pos, vel = to_device(st, gpu)
    ids = torch.arange(st.npart, dtype=torch.int32, device=gpu)
    ctx.sort(pos, vel, ids)
    torch.cuda.synchronize()
    idn = ids.cpu().numpy()
    assert np.array_equal(np.sort(idn), np.arange(st.npart))
    assert np.array_equal(pos.cpu().numpy(), st.pos_fixed.view(np.int32)[:, idn])
    assert np.array_equal(vel.cpu().numpy(), st.vel32[:, idn])
    cell = pos.cpu().numpy().view(np.uint32) >> (32 - 6)
    key = ((cell[0] >> 3) * (n // 8) + (cell[1] >> 3)) * (n // 32) + (cell[2] >> 5)
    assert np.all(np.diff(key.astype(np.int64)) >= 0)


@pytest.mark.parametrize("precision", [1, 0])
def test_tiled_deposit_equals_direct(pm, gpu, precision):
    """Tiled (LDS) deposit after a sort, with some particles moved out of
    their tiles afterwards, against the direct deposit of the same particles:
    bitwise equal in the integer form, to rounding in the float form."""
    import torch
    n = 64
    st = zeldovich_state(n, 10.0, 0.5, seed=9, m_ev=1e-22)
    lp, _ = cosmo_setup(n, 10.0, 1e-22, precision=precision)
    fp32 = precision == 0
    ctx_t = _ctx(pm, lp, gpu)
    ctx_d = _ctx(pm, lp, gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    ctx_t.sort(pos, vel)
    # move every 7th particle by 9.3 cells along y: out of its 8x8x32 tile
    sel = torch.arange(0, st.npart, 7, device=gpu)
    if fp32:
        pos[1, sel] = torch.remainder(pos[1, sel] + 9.3, float(n))
    else:
        shift = int(9.3 * 2 ** 32 / n)
        u = (pos[1, sel].to(torch.int64) & 0xffffffff) + shift
        u = u & 0xffffffff
        pos[1, sel] = torch.where(u >= 2 ** 31, u - 2 ** 32, u).to(torch.int32)
    d_t = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    d_d = torch.empty_like(d_t)
    ctx_t.deposit(pos, d_t)
    ctx_d.deposit(pos, d_d)
    torch.cuda.synchronize()
    if precision == 1:
        assert np.array_equal(mass_mesh(ctx_t), mass_mesh(ctx_d))
    else:
        assert rel_l2(d_t.cpu().numpy(), d_d.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("n", [16, 32, 64])
def test_sorted_steps_vs_oracle(pm, gpu, n):
    """Twenty steps with a sort before each half (tiled deposit and gather)
    against the oracle, matched through the permuted ids; at 16^3 and 32^3
    the 8 x 8 x 32 tile is clamped to the mesh along z (one tile row, and at
    16^3 tile windows that wrap onto themselves)."""
    import torch
    box = 10.0 * n / 256
    st = zeldovich_state(n, box, 0.01, seed=1, m_ev=1e-22)
    lp, op = cosmo_setup(n, box, 1e-22)
    ctx = _ctx(pm, lp, gpu)
    pos, vel = to_device(st, gpu)
    ids = torch.arange(st.npart, dtype=torch.int32, device=gpu)
    times = list(0.01 * np.exp(np.arange(21) * math.log(100.0) / 500))
    ctx.sort(pos, vel, ids)
    ctx.step(pos, vel, times[:11])
    ctx.sort(pos, vel, ids)
    ctx.step(pos, vel, times[10:], flags=pm.PM_CONTINUE)
    torch.cuda.synchronize()
    xo, vo = oracle.run(st.pos, st.vel, op, times)
    idn = ids.cpu().numpy()
    xg = positions_cells(pos, n)
    assert np.max(np.abs(periodic_diff(xg, xo[idn], n))) < 1e-5
    assert rel_l2(vel.cpu().numpy().T, vo[idn]) < 1e-5


@pytest.mark.parametrize("precision", [1, 0])
def test_step_sort_every_flag(pm, gpu, precision):
    """PM_SORT_EVERY inside pm_step evolves the same particle set as the
    unsorted run: order-independent comparisons (density field of the final
    positions, sums of velocity moments).  Three sorts in the call leave the
    particles in the workspace copies, so the closing kick writes them back."""
    import torch
    n = 32
    st = zeldovich_state(n, 10.0, 0.05, seed=2, m_ev=1e-22)
    lp, _ = cosmo_setup(n, 10.0, 1e-22, precision=precision)
    times = list(0.05 * np.exp(np.arange(9) * 0.01))
    fp32 = precision == 0
    c1 = _ctx(pm, lp, gpu)
    p1, v1 = to_device(st, gpu, fp32_positions=fp32)
    c1.step(p1, v1, times)
    c2 = _ctx(pm, lp, gpu)
    p2, v2 = to_device(st, gpu, fp32_positions=fp32)
    c2.step(p2, v2, times, flags=pm.PM_SORT_EVERY(3))
    torch.cuda.synchronize()
    d1 = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    d2 = torch.empty_like(d1)
    c1.deposit(p1, d1)
    c2.deposit(p2, d2)
    torch.cuda.synchronize()
    # the float deposit sums in a different order after a sort
    tol = 1e-5 if fp32 else 1e-6
    assert rel_l2(d2.cpu().numpy(), d1.cpu().numpy()) < tol
    a = v1.cpu().numpy().astype(np.float64)
    b = v2.cpu().numpy().astype(np.float64)
    for k in (1, 2):
        assert abs((b ** k).sum() - (a ** k).sum()) < tol * np.abs(a ** k).sum()


def _blob_state(n, frac=0.6, sigma=1.5, seed=21, vsig=0.05):
    """A dense Gaussian blob (frac of the particles, width sigma cells) on a
    uniform background: tiles of the blob hold many chunks of particles."""
    rng = np.random.default_rng(seed)
    npart = n ** 3
    nb = int(frac * npart)
    centre = np.array([n / 2 - 0.3, n / 4 + 0.2, n / 2 + 0.1])   # straddles tile faces
    x = np.concatenate([centre + sigma * rng.standard_normal((nb, 3)),
                        n * rng.random((npart - nb, 3))]) % n
    v = vsig * rng.standard_normal((npart, 3))
    return quantize_state(x, v, n, {"kind": "blob"})


def _lex(pos, vel):
    a = np.concatenate([pos.view(np.uint32).astype(np.float64), vel.astype(np.float64)], axis=0)
    return a[:, np.lexsort(a[::-1])]


@pytest.mark.parametrize("precision", [1, 0])
def test_multi_chunk_tiles_deposit(pm, gpu, precision):
    """Tiles holding many chunks (partial windows summed by the reduce
    kernel) against the direct deposit of the same particles."""
    import torch
    n = 64
    st = _blob_state(n)
    lp, _ = cosmo_setup(n, 10.0, 1e-22, precision=precision)
    fp32 = precision == 0
    ctx_t = _ctx(pm, lp, gpu)
    ctx_d = _ctx(pm, lp, gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    ctx_t.sort(pos, vel)
    d_t = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    d_d = torch.empty_like(d_t)
    ctx_t.deposit(pos, d_t)
    ctx_d.deposit(pos, d_d)
    torch.cuda.synchronize()
    # the blob's tiles really hold several chunks of 4096
    cell = positions_cells(pos, n, fp32).astype(np.int64)
    tile = ((cell[:, 0] >> 3) * (n // 8) + (cell[:, 1] >> 3)) * (n // 32) + (cell[:, 2] >> 5)
    assert np.bincount(tile).max() > 4 * 4096
    if precision == 1:
        assert np.array_equal(mass_mesh(ctx_t), mass_mesh(ctx_d))
        assert mass_mesh(ctx_t).sum() == st.npart * 2 ** 40
    else:
        # float atomics sum the blob's cells (thousands of particles each) in
        # another order: rounding grows like sqrt(terms) * 6e-8
        assert rel_l2(d_t.cpu().numpy(), d_d.cpu().numpy()) < 1e-5


def test_multi_chunk_tiles_fused_steps(pm, gpu):
    """Steps with a sort before every step (tiled gather with the fused
    deposit over multi-chunk tiles) evolve bitwise the same particle set as
    unsorted steps (direct gather and deposit)."""
    import torch
    n = 64
    st = _blob_state(n, seed=22)
    lp, _ = cosmo_setup(n, 10.0, 1e-22)
    times = [0.5 * math.exp(0.01 * k) for k in range(4)]
    c1 = _ctx(pm, lp, gpu)
    p1, v1 = to_device(st, gpu)
    c1.step(p1, v1, times)
    c2 = _ctx(pm, lp, gpu)
    p2, v2 = to_device(st, gpu)
    c2.step(p2, v2, times, flags=pm.PM_SORT_EVERY(1))
    torch.cuda.synchronize()
    assert np.array_equal(mass_mesh(c1), mass_mesh(c2))
    assert np.array_equal(_lex(p1.cpu().numpy(), v1.cpu().numpy()),
                          _lex(p2.cpu().numpy(), v2.cpu().numpy()))


def test_sort_auto_equals_unsorted(pm, gpu):
    """PM_SORT_AUTO (sort interval chosen from sampled stray counts) evolves
    bitwise the same particle set as unsorted steps, over calls that sort
    at different ages; the FP32 form rejects it."""
    import torch
    n = 64
    st = _blob_state(n, seed=23)
    lp, _ = cosmo_setup(n, 10.0, 1e-22)
    times = [0.5 * math.exp(0.02 * k) for k in range(13)]
    c1 = _ctx(pm, lp, gpu)
    p1, v1 = to_device(st, gpu)
    # the same two calls (a call boundary splits the merged half-kicks)
    c1.step(p1, v1, times[:5])
    c1.step(p1, v1, times[4:], flags=pm.PM_CONTINUE)
    c2 = _ctx(pm, lp, gpu)
    p2, v2 = to_device(st, gpu)
    c2.step(p2, v2, times[:5], flags=pm.PM_SORT_AUTO)
    c2.step(p2, v2, times[4:], flags=pm.PM_SORT_AUTO | pm.PM_CONTINUE)
    torch.cuda.synchronize()
    assert np.array_equal(mass_mesh(c1), mass_mesh(c2))
    assert np.array_equal(_lex(p1.cpu().numpy(), v1.cpu().numpy()),
                          _lex(p2.cpu().numpy(), v2.cpu().numpy()))
    lf, _ = cosmo_setup(n, 10.0, 1e-22, precision=0)
    c3 = _ctx(pm, lf, gpu)
    p3, v3 = to_device(st, gpu, fp32_positions=True)
    with pytest.raises(pm.PMError):
        c3.step(p3, v3, times[:3], flags=pm.PM_SORT_AUTO)


def test_sort_auto_streaming_equals_unsorted(pm, gpu):
    """Fast particles (about 0.3 cells per step): the adaptive interval turns
    short and steps after the first since a sort use the wider gather and
    deposit windows; the evolved particle set and mesh stay bitwise those of
    unsorted steps."""
    import torch
    n = 64
    st = _blob_state(n, seed=29, vsig=6.0)
    lp, _ = cosmo_setup(n, 10.0, 1e-22)
    times = [0.5 * math.exp(0.02 * k) for k in range(17)]
    c1 = _ctx(pm, lp, gpu)
    p1, v1 = to_device(st, gpu)
    c1.step(p1, v1, times[:9])
    c1.step(p1, v1, times[8:], flags=pm.PM_CONTINUE)
    c2 = _ctx(pm, lp, gpu)
    p2, v2 = to_device(st, gpu)
    c2.step(p2, v2, times[:9], flags=pm.PM_SORT_AUTO)
    c2.step(p2, v2, times[8:], flags=pm.PM_SORT_AUTO | pm.PM_CONTINUE)
    torch.cuda.synchronize()
    assert np.array_equal(mass_mesh(c1), mass_mesh(c2))
    assert np.array_equal(_lex(p1.cpu().numpy(), v1.cpu().numpy()),
                          _lex(p2.cpu().numpy(), v2.cpu().numpy()))
