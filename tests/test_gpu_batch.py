"""Batched runs (one launch per kernel for all active slots) against the
same runs stepped alone, and against the oracle."""

import math

import numpy as np
import pytest

import oracle
from synth import comoving_code_params, zeldovich_state

from gpu_helpers import periodic_diff, positions_cells, rel_l2

pytestmark = pytest.mark.gpu

N = 32
RUNS = [  # (box Mpc/h, m eV, seed, a0)
    (2.0, 2.5e-22, 11, 0.01),
    (5.0, 1e-22, 12, 0.02),
    (8.0, 1e-23, 13, 0.01),
    (3.0, 1e-21, 14, 0.05),
]


@pytest.fixture(scope="module")
def pm(gpu):
    import paper_1608_00802_amd as pm_mod
    pm_mod.load_library()
    return pm_mod


def _params(pm, box, m_ev):
    hm = comoving_code_params(box, N, m_ev, 0.7)["hbar_m_cells"] * (box / N) ** 2
    return pm.make_params(N, N ** 3, box, comoving=True, omega_m=0.3, omega_l=0.7, h0=1.0,
                          hbar_over_m=hm), hm


def _sched(a0, nsteps, dlna=0.01):
    return [a0 * math.exp(k * dlna) for k in range(nsteps + 1)]


def _states():
    return [zeldovich_state(N, box, a0, seed=seed, m_ev=m) for box, m, seed, a0 in RUNS]


def _lex(pos, vel):
    """Rows (x, y, z, vx, vy, vz) sorted lexicographically (order-free view)."""
    a = np.concatenate([pos.astype(np.float64), vel.astype(np.float64)], axis=0)
    idx = np.lexsort(a[::-1])
    return a[:, idx]


@pytest.mark.parametrize("flags_sort", [0, 5])
def test_batch_equals_runs_alone(pm, gpu, flags_sort):
    import torch
    states = _states()
    nsteps = 12
    lp0, _ = _params(pm, 1.0, 1e-22)
    batch = pm.PMBatch(lp0, 6, device=gpu)
    slots = [4, 0, 2, 5]   # not in order, and two slots left idle
    for s, st, (box, m, seed, a0) in zip(slots, states, RUNS):
        _, hm = _params(pm, box, m)
        batch.load(s, torch.from_numpy(st.pos_fixed.view(np.int32).copy()).to(gpu),
                   torch.from_numpy(st.vel32.copy()).to(gpu), box, hm)
    flags = pm.PM_SORT_EVERY(flags_sort) if flags_sort else 0
    times = [_sched(a0, nsteps) for (_, _, _, a0) in RUNS]
    batch.step(slots[:2], times[:2], flags)               # a partial batch first
    batch.step(slots[2:], times[2:], flags)
    torch.cuda.synchronize()
    for s, st, (box, m, seed, a0), t in zip(slots, states, RUNS, times):
        lp, _ = _params(pm, box, m)
        ctx = pm.PMContext(lp, device=gpu)
        pos = torch.from_numpy(st.pos_fixed.view(np.int32).copy()).to(gpu)
        vel = torch.from_numpy(st.vel32.copy()).to(gpu)
        ctx.step(pos, vel, t, flags=flags)
        torch.cuda.synchronize()
        bp, bv = batch.pos[s].cpu().numpy(), batch.vel[s].cpu().numpy()
        ap, av = pos.cpu().numpy(), vel.cpu().numpy()
        if flags_sort:
            assert np.array_equal(_lex(bp.view(np.uint32), bv), _lex(ap.view(np.uint32), av))
        else:
            assert np.array_equal(bp, ap) and np.array_equal(bv, av)
        # the mass meshes left by the last deposit are bitwise equal
        m_b = batch.mass_mesh(s).cpu().numpy()
        m_a = ctx.workspace[: 8 * N ** 3].view(torch.int64).cpu().numpy()
        assert np.array_equal(m_b, m_a)
        ctx.close()
    # idle slots were not touched
    assert not batch.pos[1].any() and not batch.pos[3].any()


def _cic_moments(x, v, n):
    """CIC deposits of mass and momentum (order-free, continuous in x)."""
    op = oracle.Params(n=n, box=float(n), S=1.0, hbar_m=0.0)
    i, f = oracle.cic_index_weights(x, op)
    out = np.zeros((4, n ** 3))
    for c in range(8):
        cx, cy, cz = c >> 2, (c >> 1) & 1, c & 1
        w = np.ones(x.shape[0])
        for d, cc in enumerate((cx, cy, cz)):
            w = w * (f[:, d] if cc else 1.0 - f[:, d])
        idx = (((i[:, 0] + cx) % n) * n + (i[:, 1] + cy) % n) * n + (i[:, 2] + cz) % n
        out[0] += np.bincount(idx, weights=w, minlength=n ** 3)
        for d in range(3):
            out[1 + d] += np.bincount(idx, weights=w * v[:, d], minlength=n ** 3)
    return out


def test_batch_slot_vs_oracle_and_continue(pm, gpu):
    """One slot of a batch across two calls against the oracle: element by
    element without sorting; with a sort every 4 steps (particles permuted)
    through CIC deposits of mass and momentum."""
    import torch
    st = _states()[1]
    box, m, seed, a0 = RUNS[1]
    lp, hm = _params(pm, box, m)
    op = oracle.Params(n=N, box=float(N), S=0.45, hbar_m=hm / (box / N) ** 2, comoving=True)
    t = _sched(a0, 16)
    xo, vo = oracle.run(st.pos, st.vel, op, t)
    for sort in (0, 4):
        batch = pm.PMBatch(lp, 3, device=gpu)
        batch.load(1, torch.from_numpy(st.pos_fixed.view(np.int32).copy()).to(gpu),
                   torch.from_numpy(st.vel32.copy()).to(gpu), box, hm)
        f = pm.PM_SORT_EVERY(sort) if sort else 0
        batch.step([1], [t[:9]], f)
        batch.step([1], [t[8:]], pm.PM_CONTINUE | f)
        torch.cuda.synchronize()
        xg = positions_cells(batch.pos[1], N)
        vg = batch.vel[1].cpu().numpy().T.astype(np.float64)
        if sort == 0:
            assert np.max(np.abs(periodic_diff(xg, xo, N))) < 1e-5
            assert rel_l2(vg, vo) < 1e-5
        else:
            mg, mo = _cic_moments(xg, vg, N), _cic_moments(xo, vo, N)
            assert rel_l2(mg[0], mo[0]) < 1e-6 and rel_l2(mg[1:], mo[1:]) < 1e-5
    # continuing a slot whose fields are stale is refused
    batch.load(2, batch.pos[1].clone(), batch.vel[1].clone(), box, hm)
    with pytest.raises(pm.PMError):
        batch.step([2], [t[:3]], pm.PM_CONTINUE)


@pytest.mark.parametrize("flags_sort", [0, 3])
def test_batch_graph_replay_equals_eager(pm, gpu, flags_sort):
    """PM_BATCH_GRAPH: calls captured into HIP graphs and replayed (same shape,
    other slots and schedules) give bitwise the states of uncaptured calls;
    eager work and synchronisations run between the replays."""
    import torch
    states = _states()
    lp0, _ = _params(pm, 1.0, 1e-22)
    streams = [torch.cuda.Stream(gpu), torch.cuda.Stream(gpu)]
    batches = []
    for sm in streams:
        with torch.cuda.stream(sm):
            b = pm.PMBatch(lp0, 4, device=gpu, stream=sm)
        for s, st, (box, m, seed, a0) in zip(range(4), states, RUNS):
            _, hm = _params(pm, box, m)
            b.load(s, torch.from_numpy(st.pos_fixed.view(np.int32).copy()).to(gpu),
                   torch.from_numpy(st.vel32.copy()).to(gpu), box, hm)
        batches.append(b)
    torch.cuda.synchronize()
    sort = pm.PM_SORT_EVERY(flags_sort) if flags_sort else 0
    k = [0, 0, 0, 0]
    # pairs of slots of the same count: the graphs of the first calls are
    # replayed for the other pair and for later calls
    plan = [[0, 1], [2, 3], [0, 1], [2, 3], [0, 1], [2, 3], [1, 2], [0, 3], [1, 2], [0, 3]]
    started = [False] * 4
    for call, sl in enumerate(plan):
        cont = all(started[s] for s in sl)
        times = [_sched(RUNS[s][3] * math.exp(0.01 * k[s]), 3) for s in sl]
        for b, g in zip(batches, (0, pm.PM_BATCH_GRAPH)):
            b.step(sl, times, sort | (pm.PM_CONTINUE if cont else 0) | g)
        for s in sl:
            k[s] += 3
            started[s] = True
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device=gpu).sum().item()      # eager work between
        assert math.isfinite(junk)
        for s in range(4):
            if flags_sort:
                # a sort orders particles inside a tile by device atomics:
                # compare the particle sets
                a = _lex(batches[0].pos[s].cpu().numpy().view(np.uint32),
                         batches[0].vel[s].cpu().numpy())
                g = _lex(batches[1].pos[s].cpu().numpy().view(np.uint32),
                         batches[1].vel[s].cpu().numpy())
                assert np.array_equal(a, g), (call, s)
            else:
                assert torch.equal(batches[0].pos[s], batches[1].pos[s]), (call, s)
                assert torch.equal(batches[0].vel[s], batches[1].vel[s]), (call, s)
    # replays queued back to back (no synchronisation between calls: the host
    # refills the staging buffers while earlier calls are still queued)
    for call in range(6):
        sl = [0, 1] if call % 2 == 0 else [2, 3]
        times = [_sched(RUNS[s][3] * math.exp(0.01 * k[s]), 3) for s in sl]
        for b, g in zip(batches, (0, pm.PM_BATCH_GRAPH)):
            b.step(sl, times, sort | pm.PM_CONTINUE | g)
        for s in sl:
            k[s] += 3
    torch.cuda.synchronize()
    for s in range(4):
        a = _lex(batches[0].pos[s].cpu().numpy().view(np.uint32), batches[0].vel[s].cpu().numpy())
        g = _lex(batches[1].pos[s].cpu().numpy().view(np.uint32), batches[1].vel[s].cpu().numpy())
        assert np.array_equal(a, g), ("queued", s)
    assert all(started)
    # the default stream cannot be captured
    b0 = pm.PMBatch(lp0, 1, device=gpu)
    if b0.stream.cuda_stream == 0:
        with pytest.raises(pm.PMError):
            b0.step([0], [_sched(0.01, 2)], pm.PM_BATCH_GRAPH)
