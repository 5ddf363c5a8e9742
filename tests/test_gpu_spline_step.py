"""pm_spline_step (KDK with the paper's spline coupling, Sec. II A) against
the oracle's spline_run on the same state and schedule, through the C ABI.

The library works in FP32 (forces, velocities) on fixed-point or float
positions; after 6-8 steps positions agree with the FP64 oracle to 1e-4
cell and velocities to a relative 1e-4 (written below).
"""

import numpy as np
import pytest

import oracle
from synth import quantize_state, zeldovich_state

from gpu_helpers import cosmo_setup, periodic_diff, positions_cells, rel_l2, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm(gpu):
    import paper_1608_00802_amd as pm_mod
    pm_mod.load_library()
    return pm_mod


def _jittered(n, seed, sigma=0.3):
    rng = np.random.default_rng(seed)
    g = np.arange(n, dtype=np.float64) + 0.5
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    pos = (pos + sigma * rng.standard_normal(pos.shape)) % n
    vel = 0.05 * rng.standard_normal(pos.shape)
    return quantize_state(pos, vel, n, {"kind": "jittered"})


def _compare(pos_t, vel_t, x_ref, v_ref, n, fp32):
    import torch
    torch.cuda.synchronize()
    d = periodic_diff(positions_cells(pos_t, n, fp32), x_ref, n)
    assert np.max(np.abs(d)) < 1e-4, np.max(np.abs(d))
    assert rel_l2(vel_t.cpu().numpy().T, v_ref) < 1e-4


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("hm,S", [(0.8, 1.0), (0.0, 1.0), (0.8, 0.0)])
def test_static_spline_steps_vs_oracle(pm, gpu, precision, hm, S):
    n = 16
    st = _jittered(n, 1)
    fp32 = precision == 0
    lp = pm.make_params(n, n ** 3, float(n), precision=precision, four_pi_G_rhobar=S,
                        hbar_over_m=hm, rho_floor=1e-6, rho_fp64_below=0.0)
    op = oracle.Params(n=n, box=float(n), S=S, hbar_m=hm, rho_floor=1e-6)
    ctx = pm.PMContext(lp, device=gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    x0 = positions_cells(pos, n, fp32)
    v0 = vel.cpu().numpy().T.astype(np.float64)
    times = list(np.linspace(0.0, 0.8, 9))
    ctx.spline_step(pos, vel, times, 3.5)
    x, v = oracle.spline_run(x0, v0, op, times, 3.5)
    _compare(pos, vel, x, v, n, fp32)


@pytest.mark.parametrize("precision", [1, 0])
def test_comoving_spline_steps_vs_oracle(pm, gpu, precision):
    n = 32
    st = zeldovich_state(n, 2.0, 0.05, seed=9, m_ev=2.5e-22)
    lp, op = cosmo_setup(n, 2.0, 2.5e-22, precision=precision, rho_fp64_below=0.0)
    fp32 = precision == 0
    ctx = pm.PMContext(lp, device=gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    x0 = positions_cells(pos, n, fp32)
    v0 = vel.cpu().numpy().T.astype(np.float64)
    times = list(0.05 * np.exp(np.arange(7) * 0.01))
    ctx.spline_step(pos, vel, times[:4], 3.5)
    ctx.spline_step(pos, vel, times[3:], 3.5)
    x, v = oracle.spline_run(x0, v0, op, times, 3.5)
    _compare(pos, vel, x, v, n, fp32)


@pytest.mark.parametrize("precision", [1, 0])
def test_spline_energy_vs_oracle(pm, gpu, precision):
    n = 32
    st = _jittered(n, 2)
    fp32 = precision == 0
    lp = pm.make_params(n, n ** 3, float(n), precision=precision, four_pi_G_rhobar=1.0,
                        hbar_over_m=0.5, rho_floor=1e-6, rho_fp64_below=0.0)
    op = oracle.Params(n=n, box=float(n), S=1.0, hbar_m=0.5, rho_floor=1e-6)
    ctx = pm.PMContext(lp, device=gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    got = ctx.spline_energy(pos, vel, 1.0, 3.5)
    ref = oracle.spline_energies(positions_cells(pos, n, fp32),
                                 vel.cpu().numpy().T.astype(np.float64), op, 3.5)
    for key in ("K", "W", "U"):
        assert abs(got[key] - ref[key]) <= 1e-5 * abs(ref[key]), (key, got[key], ref[key])


def test_spline_step_conserves_the_discrete_energy(pm, gpu):
    # Sec. II A: with gravity off the kernel-gradient force conserves K + U of
    # the spline density by construction; the leapfrog's error falls as dt^2
    import torch
    n = 16
    st = _jittered(n, 6, sigma=0.25)
    lp = pm.make_params(n, n ** 3, float(n), precision=1, four_pi_G_rhobar=0.0,
                        hbar_over_m=0.8, rho_floor=1e-6, rho_fp64_below=0.0)
    errs = []
    for steps in (4, 8):
        ctx = pm.PMContext(lp, device=gpu)
        pos, vel = to_device(st, gpu)
        vel.zero_()
        e0 = ctx.spline_energy(pos, vel, 1.0, 3.5)["E"]
        ctx.spline_step(pos, vel, list(np.linspace(0.0, 1.2, steps + 1)), 3.5)
        e1 = ctx.spline_energy(pos, vel, 1.0, 3.5)
        errs.append(abs(e1["E"] - e0) / e0)
        assert e1["K"] > 0.05 * e0
        torch.cuda.synchronize()
    assert errs[1] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.5, errs


@pytest.mark.parametrize("precision", [1, 0])
def test_sorted_spline_steps_with_strays_vs_oracle(pm, gpu, precision):
    """A context sorted first (tiled LDS deposit), then stepped with fast
    particles (about half a cell per step) so that many leave their tile
    windows: the deposit mixes tiled and direct additions; positions and
    velocities against the oracle's spline leapfrog."""
    import torch
    n = 32
    st = _jittered(n, 9)
    rng = np.random.default_rng(10)
    fp32 = precision == 0
    lp = pm.make_params(n, n ** 3, float(n), precision=precision, four_pi_G_rhobar=1.0,
                        hbar_over_m=0.8, rho_floor=1e-6, rho_fp64_below=1e-3)
    op = oracle.Params(n=n, box=float(n), S=1.0, hbar_m=0.8, rho_floor=1e-6)
    ctx = pm.PMContext(lp, device=gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    vel.copy_(torch.from_numpy((5.0 * rng.standard_normal((3, n ** 3))).astype(np.float32)))
    ctx.sort(pos, vel)
    torch.cuda.synchronize()
    x0 = positions_cells(pos, n, fp32)
    v0 = vel.cpu().numpy().T.astype(np.float64)
    times = list(np.linspace(0.0, 0.8, 9))      # 0.1 per step: ~0.5 cell per step
    ctx.spline_step(pos, vel, times, 3.5)
    x, v = oracle.spline_run(x0, v0, op, times, 3.5)
    _compare(pos, vel, x, v, n, fp32)
