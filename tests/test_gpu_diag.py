"""Parity of the grid diagnostics (pm_kinetic_split, pm_density_rms_diff)
with the FP64 oracle, through the C ABI.

Tolerances: the fixed-point form deposits with integer 2^-40 weights (exact
fractions to 2^-41 of a particle) and sums node momenta in FP64, so results
agree with the oracle to about 1e-12; 1e-9 is asserted.  The plain FP32 form
takes its CIC weights and mass sums in float (rounding 6e-8 per weight);
3e-6 is asserted.  K_disp = K - K_bulk is checked against K's scale, since
it is a difference.
"""

import numpy as np
import pytest

import oracle
from synth import quantize_state, zeldovich_state

from gpu_helpers import TWO40, cosmo_setup, mass_mesh, positions_cells, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm(gpu):
    import paper_1608_00802_amd as pm_mod
    pm_mod.load_library()
    return pm_mod


def _tol(precision):
    return 1e-9 if precision == 1 else 3e-6


def _clumps(n, npart, seed, vsig=0.3):
    """Gaussian clumps on a sparse background: many empty nodes, and
    velocities with both a coherent part and a dispersion."""
    rng = np.random.default_rng(seed)
    centres = rng.random((5, 3)) * n
    k = rng.integers(0, 5, npart)
    pos = centres[k] + 1.2 * rng.standard_normal((npart, 3))
    bg = rng.random(npart) < 0.1
    pos[bg] = rng.random((int(bg.sum()), 3)) * n
    pos %= n
    vel = vsig * rng.standard_normal((npart, 3)) + 0.5 * np.sin(2 * np.pi * pos / n)
    return quantize_state(pos, vel, n, {"kind": "clumps"})


def _oracle_inputs(pos_t, vel_t, n, fp32):
    return positions_cells(pos_t, n, fp32), vel_t.cpu().numpy().T.astype(np.float64)


def _ctx_for(pm, n, npart, precision, comoving=True):
    if comoving:
        lp, op = cosmo_setup(n, 2.0, 2.5e-22, precision=precision)
        lp.n_part = npart
    else:
        lp = pm.make_params(n, npart, float(n), precision=precision, four_pi_G_rhobar=1.0)
        op = oracle.Params(n=n, box=float(n), S=1.0, hbar_m=0.0)
    return lp, op


def _check_split(got, ref, tol):
    assert abs(got["K"] - ref["K"]) <= tol * ref["K"], (got, ref)
    assert abs(got["K_bulk"] - ref["K_bulk"]) <= tol * ref["K_bulk"], (got, ref)
    assert abs(got["K_disp"] - ref["K_disp"]) <= tol * ref["K"], (got, ref)


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("n", [32, 64])
def test_kinetic_split_zeldovich(pm, gpu, precision, n):
    st = zeldovich_state(n, 2.0, 0.1, seed=11, m_ev=2.5e-22)
    lp, op = cosmo_setup(n, 2.0, 2.5e-22, precision=precision)
    fp32 = precision == 0
    ctx = pm.PMContext(lp, device=gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    a = 0.1
    got = ctx.kinetic_split(pos, vel, a)
    x, v = _oracle_inputs(pos, vel, n, fp32)
    ref = oracle.kinetic_split(x, v, op, a)
    _check_split(got, ref, _tol(precision))
    # K is Eq. (8) exactly as pm_energy reports it
    e = ctx.energy(pos, vel, a)
    assert abs(e["K"] - got["K"]) <= 1e-12 * got["K"]


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("npart", [40000, 70001])
def test_kinetic_split_clumps_ragged(pm, gpu, precision, npart):
    # empty nodes, particle counts that fill no whole block, static box
    n = 32
    st = _clumps(n, npart, seed=npart)
    lp, op = _ctx_for(pm, n, npart, precision, comoving=False)
    fp32 = precision == 0
    ctx = pm.PMContext(lp, device=gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    got = ctx.kinetic_split(pos, vel)
    x, v = _oracle_inputs(pos, vel, n, fp32)
    ref = oracle.kinetic_split(x, v, op)
    assert ref["K_disp"] > 0.1 * ref["K"]
    _check_split(got, ref, _tol(precision))


@pytest.mark.parametrize("precision", [1, 0])
def test_kinetic_split_sorted_with_strays(pm, gpu, precision):
    # a sorted context takes the tiled LDS path; after the sort the particles
    # are moved by up to 2.5 cells, so some leave their tile's window and add
    # to the mesh directly
    import torch
    from synth import to_fixed
    n = 32
    npart = 70001
    st = _clumps(n, npart, seed=8)
    lp, op = _ctx_for(pm, n, npart, precision, comoving=False)
    fp32 = precision == 0
    ctx = pm.PMContext(lp, device=gpu)
    pos, vel = to_device(st, gpu, fp32_positions=fp32)
    ctx.sort(pos, vel)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    x = (positions_cells(pos, n, fp32) + rng.uniform(-2.5, 2.5, (npart, 3))) % n
    if fp32:
        xf = np.ascontiguousarray(x.T.astype(np.float32))
        xf[xf >= np.float32(n)] = 0.0
        pos.copy_(torch.from_numpy(xf))
    else:
        pos.copy_(torch.from_numpy(to_fixed(x, n).view(np.int32)))
    got = ctx.kinetic_split(pos, vel)
    xo, v = _oracle_inputs(pos, vel, n, fp32)
    ref = oracle.kinetic_split(xo, v, op)
    _check_split(got, ref, _tol(precision))


def test_kinetic_split_full_size_properties(pm, gpu):
    # 256^3 particles on a 256^3 mesh: one common velocity is all bulk
    # motion; Zel'dovich velocities give 0 <= K_bulk <= K and the K of
    # pm_energy
    import torch
    n = 256
    st = zeldovich_state(n, 10.0, 0.01, seed=1, m_ev=1e-22)
    lp, _ = cosmo_setup(n, 10.0, 1e-22)
    ctx = pm.PMContext(lp, device=gpu)
    pos, vel = to_device(st, gpu)
    got = ctx.kinetic_split(pos, vel, 0.01)
    e = ctx.energy(pos, vel, 0.01)
    assert abs(e["K"] - got["K"]) <= 1e-12 * got["K"]
    assert 0.0 <= got["K_bulk"] <= got["K"] * (1 + 1e-12)
    assert got["K_disp"] >= -1e-12 * got["K"]
    common = torch.tensor([0.25, -1.5, 0.75], device=gpu).view(3, 1).expand(3, n ** 3)
    common = common.contiguous()
    got = ctx.kinetic_split(pos, common, 0.01)
    assert abs(got["K_bulk"] - got["K"]) <= 1e-12 * got["K"]
    assert abs(got["K_disp"]) <= 1e-12 * got["K"]


@pytest.mark.parametrize("precision", [1, 0])
def test_density_rms_diff_vs_oracle(pm, gpu, precision):
    import torch
    n = 32
    st_b = zeldovich_state(n, 2.0, 0.1, seed=12, m_ev=None)
    rng = np.random.default_rng(3)
    xa = (st_b.pos + 0.4 * rng.standard_normal(st_b.pos.shape)) % n
    st_a = quantize_state(xa, st_b.vel, n, {"kind": "displaced"})
    lp, op = cosmo_setup(n, 2.0, 2.5e-22, precision=precision)
    fp32 = precision == 0
    ctx = pm.PMContext(lp, device=gpu)
    pa, _ = to_device(st_a, gpu, fp32_positions=fp32)
    pb, _ = to_device(st_b, gpu, fp32_positions=fp32)
    rms, cells = ctx.density_rms_diff(pa, pb)
    ref_rms, ref_cells = oracle.density_rms_diff(positions_cells(pa, n, fp32),
                                                 positions_cells(pb, n, fp32), op)
    assert cells == ref_cells
    assert abs(rms - ref_rms) <= _tol(precision) * ref_rms, (rms, ref_rms)
    # a state against itself: exactly zero in fixed point (integer deposit);
    # the FP32 form's float atomics sum in a varying order (rounding 1e-7)
    rms0, cells0 = ctx.density_rms_diff(pb, pb)
    assert cells0 == ref_cells
    assert rms0 == 0.0 if precision == 1 else rms0 < 1e-6
    if precision == 1:
        # the mass mesh is left at the last state deposited
        torch.cuda.synchronize()
        assert int(mass_mesh(ctx).sum()) == n ** 3 * int(TWO40)


@pytest.mark.parametrize("precision", [1, 0])
def test_density_rms_diff_empty_reference_nodes(pm, gpu, precision):
    # b: a ragged number of particles sitting exactly on a random subset of
    # nodes (exact weights: every other node is exactly empty and left out);
    # a: uniform random positions.  Nodes that hold only a sliver of a
    # particle are avoided on purpose: there the weights' own quantisation
    # (2^-41 of a particle in fixed point, float rounding in FP32) is large
    # relative to the node mass, a property of the representation
    n = 32
    npart = 50001
    rng = np.random.default_rng(9)
    nodes = rng.choice(n ** 3, size=12000, replace=False)
    idx = nodes[rng.integers(0, nodes.size, npart)]
    xb = np.stack([idx // (n * n), (idx // n) % n, idx % n], axis=1).astype(np.float64)
    vel = np.zeros((npart, 3))
    st_b = quantize_state(xb, vel, n, {"kind": "on nodes"})
    st_a = quantize_state(rng.random((npart, 3)) * n, vel, n, {"kind": "uniform"})
    lp, op = _ctx_for(pm, n, npart, precision, comoving=False)
    fp32 = precision == 0
    ctx = pm.PMContext(lp, device=gpu)
    pa, _ = to_device(st_a, gpu, fp32_positions=fp32)
    pb, _ = to_device(st_b, gpu, fp32_positions=fp32)
    rms, cells = ctx.density_rms_diff(pa, pb)
    ref_rms, ref_cells = oracle.density_rms_diff(positions_cells(pa, n, fp32),
                                                 positions_cells(pb, n, fp32), op)
    assert ref_cells == np.unique(idx).size < n ** 3
    assert cells == ref_cells
    assert abs(rms - ref_rms) <= _tol(precision) * ref_rms, (rms, ref_rms)


@pytest.mark.parametrize("m_ev", [2.5e-22, None])
def test_steps_after_diagnostics_are_unchanged(pm, gpu, m_ev):
    # the diagnostics use the field area as scratch: the next call recomputes
    # every field, as it does after pm_energy, and gives bit-identical
    # particles (fixed point)
    import torch
    n = 32
    st = zeldovich_state(n, 2.0, 0.05, seed=6, m_ev=m_ev)
    lp, _ = cosmo_setup(n, 2.0, m_ev)
    times = list(0.05 * np.exp(np.arange(6) * 0.01))
    ctx1 = pm.PMContext(lp, device=gpu)
    p1, v1 = to_device(st, gpu)
    ctx1.step(p1, v1, times[:3])
    ctx1.energy(p1, v1, times[2])
    ctx1.step(p1, v1, times[2:], flags=pm.PM_CONTINUE)
    ctx2 = pm.PMContext(lp, device=gpu)
    p2, v2 = to_device(st, gpu)
    p3, _ = to_device(st, gpu)
    ctx2.step(p2, v2, times[:3])
    ctx2.kinetic_split(p2, v2, times[2])
    ctx2.density_rms_diff(p3, p2)
    ctx2.step(p2, v2, times[2:], flags=pm.PM_CONTINUE)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2)
    assert torch.equal(v1, v2)


# ------------------------------------------------------------ power spectrum

def _oracle_power(pos_t, n, op, fp32, nbins=None):
    x = positions_cells(pos_t, n, fp32)
    delta = oracle.deposit(x, op) - 1.0
    return oracle.power_spectrum(delta, op.box, nbins)


def _check_power(got, ref, tol):
    # relative tolerance per shell, with a floor at 1e-9 of the largest shell
    # for the float FFT's rounding where the spectrum has fallen far below it
    k, p, c = (np.asarray(a) for a in got)
    rk, rp, rc = ref
    assert np.array_equal(c, rc)
    assert np.allclose(k, rk, rtol=1e-14, atol=0)
    err = np.abs(p - rp)
    assert np.all(err <= tol * rp + 1e-9 * rp.max()), np.max(err / rp)


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("n", [16, 32, 64])
def test_power_spectrum_vs_oracle(pm, gpu, precision, n):
    # CDM initial conditions (no FDM cutoff): power in every shell
    st = zeldovich_state(n, 2.0, 0.1, seed=13, m_ev=None)
    lp, op = cosmo_setup(n, 2.0, 2.5e-22, precision=precision)
    fp32 = precision == 0
    ctx = pm.PMContext(lp, device=gpu)
    pos, _ = to_device(st, gpu, fp32_positions=fp32)
    got = ctx.power_spectrum(pos)
    _check_power(got, _oracle_power(pos, n, op, fp32), 2e-5 if precision == 1 else 2e-4)
    # fewer bins: the same leading shells (a new deposit: in FP32 its float
    # atomics add in another order)
    got5 = ctx.power_spectrum(pos, 5)
    assert got5[2] == got[2][:5]
    assert np.allclose(got5[1], got[1][:5], rtol=1e-12 if precision == 1 else 1e-6)


def test_power_spectrum_single_mode_along_z(pm, gpu):
    # a lattice displaced along z by one sine mode: its power sits in shell
    # `mode` at m_z = +-mode (stored once, counted for its conjugate)
    from synth import sine_mode_state
    n = 32
    st = sine_mode_state(n, mode=3, amp_cells=1e-2, axis=2)
    lp, op = cosmo_setup(n, 2.0, 2.5e-22)
    ctx = pm.PMContext(lp, device=gpu)
    pos, _ = to_device(st, gpu)
    k, p, c = ctx.power_spectrum(pos)
    rk, rp, rc = _oracle_power(pos, n, op, False)
    assert np.array_equal(np.asarray(c), rc)
    assert abs(p[2] - rp[2]) <= 1e-5 * rp[2]
    assert p[2] > 1e6 * max(p[b] for b in range(len(p)) if b != 2)


def test_power_spectrum_full_size(pm, gpu):
    # 256^3 particles on a 256^3 mesh (the benchmark box), every shell
    n = 256
    st = zeldovich_state(n, 10.0, 0.05, seed=1, m_ev=None)
    lp, op = cosmo_setup(n, 10.0, 1e-22)
    ctx = pm.PMContext(lp, device=gpu)
    pos, _ = to_device(st, gpu)
    got = ctx.power_spectrum(pos)
    _check_power(got, _oracle_power(pos, n, op, False), 2e-5)


def test_power_spectrum_rejects_bad_bins(pm, gpu):
    n = 16
    lp, _ = cosmo_setup(n, 2.0, 2.5e-22)
    ctx = pm.PMContext(lp, device=gpu)
    st = zeldovich_state(n, 2.0, 0.1, seed=1, m_ev=2.5e-22)
    pos, _ = to_device(st, gpu)
    for nb in (0, n // 2 + 1):
        with pytest.raises(pm.PMError):
            ctx.power_spectrum(pos, nb)
