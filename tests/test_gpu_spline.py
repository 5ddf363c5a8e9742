"""Parity of the spline-kernel steps (pm_spline_density, pm_spline_qforce;
Sec. II A, Eqs. (9), (14), (15)) with the FP64 oracle, through the C ABI.

Tolerances: the density is an integer sum of about 180 kernel values per
particle, each rounded once to 2^-40 of a particle after an FP32 evaluation
(relative error a few 1e-7): rel-L2 below 1e-5, on near-empty nodes too, and
the integer mesh is bitwise the same in every order and launch form.  The force sums
about 180 terms Q_j grad W in float whose total is a small difference of
large terms for smooth Q: rel-L2 below 1e-4.  The composed chain (density,
then the library's Q from float delta, then the force) is held to 5e-4.
"""

import numpy as np
import pytest

import oracle
from synth import quantize_state

from gpu_helpers import mass_mesh, positions_cells, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm(gpu):
    import paper_1608_00802_amd as pm_mod
    pm_mod.load_library()
    return pm_mod


def _jittered(n, seed, sigma=0.35):
    rng = np.random.default_rng(seed)
    g = np.arange(n, dtype=np.float64) + 0.5
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    pos = (pos + sigma * rng.standard_normal(pos.shape)) % n
    return quantize_state(pos, np.zeros_like(pos), n, {"kind": "jittered"})


def _clumps(n, npart, seed):
    rng = np.random.default_rng(seed)
    c = rng.random((4, 3)) * n
    pos = c[rng.integers(0, 4, npart)] + 2.0 * rng.standard_normal((npart, 3))
    bg = rng.random(npart) < 0.3
    pos[bg] = rng.random((int(bg.sum()), 3)) * n
    return quantize_state(pos % n, np.zeros((npart, 3)), n, {"kind": "clumps"})


def _setup(pm, gpu, n, npart, precision, hm=0.5):
    lp = pm.make_params(n, npart, float(n), precision=precision, four_pi_G_rhobar=1.0,
                        hbar_over_m=hm, rho_floor=1e-6, rho_fp64_below=0.0)
    op = oracle.Params(n=n, box=float(n), S=1.0, hbar_m=hm, rho_floor=1e-6)
    return pm.PMContext(lp, device=gpu), op


def _positions(st, gpu, fp32):
    import torch
    if fp32:
        return torch.from_numpy(st.pos_f32.copy()).to(gpu)
    return torch.from_numpy(st.pos_fixed.view(np.int32).copy()).to(gpu)


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("case", ["lattice", "clumps"])
@pytest.mark.parametrize("h", [3.5, 4.0, 2.0])
def test_spline_density_and_force_vs_oracle(pm, gpu, precision, case, h):
    import torch
    n = 32
    st = _jittered(n, 1) if case == "lattice" else _clumps(n, 20001, 2)
    ctx, op = _setup(pm, gpu, n, st.npart, precision)
    fp32 = precision == 0
    pos = _positions(st, gpu, fp32)
    delta = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.spline_density(pos, delta, h)
    x = positions_cells(pos, n, fp32)
    rho = oracle.spline_deposit(x, op, h)
    torch.cuda.synchronize()
    got = 1.0 + delta.cpu().numpy().astype(np.float64).reshape(n, n, n)
    assert rel_l2(got, rho) < 1e-5
    # force from one Q for both sides (the oracle's Q rounded to float)
    q32 = oracle.qpot(rho, op).astype(np.float32)
    qd = torch.from_numpy(q32.ravel().copy()).to(gpu)
    acc = torch.empty(3, st.npart, dtype=torch.float32, device=gpu)
    ctx.spline_qforce(pos, qd, acc, h)
    ref = oracle.spline_qforce(x, q32.astype(np.float64), op, h)
    torch.cuda.synchronize()
    assert rel_l2(acc.cpu().numpy().T, ref) < 1e-4


@pytest.mark.parametrize("precision", [1, 0])
def test_spline_chain_vs_oracle(pm, gpu, precision):
    # density -> pm_qpot -> force, against the oracle's chain (n = 32)
    import torch
    n = 32
    st = _jittered(n, 3)
    ctx, op = _setup(pm, gpu, n, st.npart, precision)
    fp32 = precision == 0
    pos = _positions(st, gpu, fp32)
    delta = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    q = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    acc = torch.empty(3, st.npart, dtype=torch.float32, device=gpu)
    ctx.spline_density(pos, delta, 3.5)
    ctx.qpot(delta, q)
    ctx.spline_qforce(pos, q, acc, 3.5)
    x = positions_cells(pos, n, fp32)
    rho = oracle.spline_deposit(x, op, 3.5)
    ref = oracle.spline_qforce(x, oracle.qpot(rho, op), op, 3.5)
    torch.cuda.synchronize()
    assert rel_l2(q.cpu().numpy().reshape(n, n, n), oracle.qpot(rho, op)) < 5e-4
    assert rel_l2(acc.cpu().numpy().T, ref) < 5e-4


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("h", [3.5, 4.0])
def test_spline_density_sorted_with_strays(pm, gpu, precision, h):
    # a sorted context takes the tiled LDS paths; particles moved by up to
    # 3 cells after the sort leave their tile and use the mesh directly
    import torch
    from synth import to_fixed
    n = 32
    st = _clumps(n, 60001, 7)
    ctx, op = _setup(pm, gpu, n, st.npart, precision)
    fp32 = precision == 0
    pos = _positions(st, gpu, fp32)
    vel = torch.zeros(3, st.npart, dtype=torch.float32, device=gpu)
    ctx.sort(pos, vel)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    x = (positions_cells(pos, n, fp32) + rng.uniform(-3.0, 3.0, (st.npart, 3))) % n
    if fp32:
        xf = np.ascontiguousarray(x.T.astype(np.float32))
        xf[xf >= np.float32(n)] = 0.0
        pos.copy_(torch.from_numpy(xf))
    else:
        pos.copy_(torch.from_numpy(to_fixed(x, n).view(np.int32)))
    delta = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.spline_density(pos, delta, h)
    xs = positions_cells(pos, n, fp32)
    rho = oracle.spline_deposit(xs, op, h)
    torch.cuda.synchronize()
    got = 1.0 + delta.cpu().numpy().astype(np.float64).reshape(n, n, n)
    assert rel_l2(got, rho) < 1e-5
    # the tiled force (Q staged per tile chunk in LDS), strays from the mesh
    q32 = oracle.qpot(rho, op).astype(np.float32)
    qd = torch.from_numpy(q32.ravel().copy()).to(gpu)
    acc = torch.empty(3, st.npart, dtype=torch.float32, device=gpu)
    ctx.spline_qforce(pos, qd, acc, h)
    ref = oracle.spline_qforce(xs, q32.astype(np.float64), op, h)
    torch.cuda.synchronize()
    assert rel_l2(acc.cpu().numpy().T, ref) < 1e-4


def test_spline_full_size_sampled(pm, gpu):
    # 256^3 particles on a 256^3 mesh: mean density one to the kernel's
    # discretisation, and the force of 400 sampled particles against the
    # oracle on the library's own Q (the force step checked on its inputs)
    import torch
    n = 256
    st = _jittered(n, 4, sigma=0.6)
    ctx, op = _setup(pm, gpu, n, st.npart, 1)
    pos = _positions(st, gpu, False)
    delta = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    q = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    acc = torch.empty(3, st.npart, dtype=torch.float32, device=gpu)
    ctx.spline_density(pos, delta, 3.5)
    ctx.qpot(delta, q)
    ctx.spline_qforce(pos, q, acc, 3.5)
    torch.cuda.synchronize()
    assert abs(float(delta.double().mean().item())) < 2e-3
    rng = np.random.default_rng(0)
    pick = rng.choice(st.npart, 400, replace=False)
    x = positions_cells(pos, n)[pick]
    ref = oracle.spline_qforce(x, q.cpu().numpy().astype(np.float64), op, 3.5)
    assert rel_l2(acc.cpu().numpy().T[pick], ref) < 1e-4


def test_spline_rejects_bad_h(pm, gpu):
    import torch
    n = 16
    st = _jittered(n, 5)
    ctx, _ = _setup(pm, gpu, n, st.npart, 1)
    pos = _positions(st, gpu, False)
    delta = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    for h in (0.1, 1.5, 1.99, 8.0, float("nan")):
        with pytest.raises(pm.PMError):
            ctx.spline_density(pos, delta, h)
    # the smallest accepted h: every particle deposits its mass to 0.2 %
    ctx.spline_density(pos, delta, 2.0)
    torch.cuda.synchronize()
    total = mass_mesh(ctx).astype(np.float64).sum() / (st.npart * 2.0 ** 40)
    assert abs(total - 1.0) < 2e-3


@pytest.mark.parametrize("precision", [1, 0])
def test_spline_density_bitwise_order_free(pm, gpu, precision):
    """The integer spline density is bitwise the same on repeated calls, for a
    permuted particle order and from the tiled (sorted) and direct forms."""
    import torch
    n = 32
    st = _clumps(n, 30001, 11)
    ctx, _ = _setup(pm, gpu, n, st.npart, precision)
    fp32 = precision == 0
    pos = _positions(st, gpu, fp32)
    delta = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.spline_density(pos, delta, 3.5)
    m0 = mass_mesh(ctx).copy()
    ctx.spline_density(pos, delta, 3.5)
    assert np.array_equal(mass_mesh(ctx), m0)
    perm = torch.from_numpy(np.random.default_rng(2).permutation(st.npart)).to(gpu)
    ctx.spline_density(pos[:, perm].contiguous(), delta, 3.5)
    assert np.array_equal(mass_mesh(ctx), m0)
    ctx2, _ = _setup(pm, gpu, n, st.npart, precision)
    p2 = pos.clone()
    vel = torch.zeros(3, st.npart, dtype=torch.float32, device=gpu)
    ctx2.sort(p2, vel)
    ctx2.spline_density(p2, delta, 3.5)
    assert np.array_equal(mass_mesh(ctx2), m0)


@pytest.mark.parametrize("n,width", [(32, 1.2), (64, 2.0)])
def test_spline_q_near_empty_nodes_fp64(pm, gpu, n, width):
    """Q of the spline density in a box with voids (clumps, no background):
    the fixed-point form takes Q from the integer density in FP64 on nodes
    below 1e-3 of the mean; all, low and other nodes against the oracle."""
    import torch
    rng = np.random.default_rng(n)
    c = rng.random((3, 3)) * n
    npart = 40000
    x = (c[rng.integers(0, 3, npart)] + width * rng.standard_normal((npart, 3))) % n
    st = quantize_state(x, np.zeros((npart, 3)), n, {"kind": "voids"})
    hm = 0.5
    lp = pm.make_params(n, npart, float(n), four_pi_G_rhobar=1.0, hbar_over_m=hm,
                        rho_floor=1e-6, rho_fp64_below=1e-3)
    op = oracle.Params(n=n, box=float(n), S=1.0, hbar_m=hm, rho_floor=1e-6)
    ctx = pm.PMContext(lp, device=gpu)
    pos = _positions(st, gpu, False)
    delta = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    q = torch.empty(n ** 3, dtype=torch.float32, device=gpu)
    ctx.spline_density(pos, delta, 3.5)
    ctx.qpot(None, q)
    torch.cuda.synchronize()
    rho = oracle.spline_deposit(st.pos, op, 3.5)
    ref = oracle.qpot(rho, op)
    got = q.cpu().numpy().astype(np.float64).reshape(n, n, n)
    low = (rho < 1e-3) & (rho > 0.0)
    errs = (rel_l2(got, ref), rel_l2(got[low], ref[low]), rel_l2(got[~low], ref[~low]))
    print(f"spline Q with voids {n}^3: {int(low.sum())} nodes in (0, 1e-3), "
          f"{int((rho == 0).sum())} empty; rel-L2 all / low / other {errs}", flush=True)
    assert low.sum() > 100
    assert max(errs) < 1e-5
