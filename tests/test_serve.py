"""Request loop on the CPU: scheduling, admission by footprint, slot reuse,
failure handling and the per-request time-step schedule, against a
virtual-clock executor (no GPU)."""

import math

import numpy as np

import oracle
from paper_1608_00802_amd.serve import (A_END, A_START, OMEGA_MAX_COEF, FakeExecutor, Request,
                                        Scheduler, VirtualClock, dlna_step, extend_times,
                                        hbar_over_m, make_trace, schedule, summarize)
from synth import comoving_code_params, zeldovich_state


def _req(rid, n=32, arrival=0.0, nsteps=50, box=5.0, m_ev=1e-21):
    return Request(rid=rid, n=n, box=box, m_ev=m_ev, seed=rid, nsteps=nsteps, arrival=arrival)


def _serve(trace, ex_kw=None, scale=1.0, chunk=10, ics=None):
    vc = VirtualClock()
    ex = FakeExecutor(vc.now, **(ex_kw or {}))
    sch = Scheduler(ex, chunk=chunk)
    res = sch.run(trace, ics or (lambda r: None), clock=vc.now, sleep=vc.sleep,
                  time_scale=scale)
    return res, ex, sch


# ------------------------------------------------------------------ trace and schedule

def test_trace_shape():
    tr = make_trace(400, rate=4.0, seed=2026)
    t = np.array([r.arrival for r in tr])
    assert np.all(np.diff(t) > 0)
    # Poisson process: mean gap 1/rate within a few standard errors
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.25) < 4 * 0.25 / math.sqrt(len(gaps))
    assert {r.n for r in tr} == {32, 64, 128, 256}
    assert all(r.seed == r.rid for r in tr)
    assert all(50 <= r.nsteps <= 200 and 1.0 <= r.box <= 10.0 for r in tr)
    assert all(1e-23 <= r.m_ev <= 1e-21 for r in tr)
    assert make_trace(400, seed=2026) == tr


def test_hbar_over_m_matches_ic_units():
    for box, n, m in [(2.0, 128, 2.5e-22), (7.5, 32, 1e-23)]:
        dx = box / n
        want = comoving_code_params(box, n, m, 0.7)["hbar_m_cells"]
        assert abs(hbar_over_m(m) / dx ** 2 / want - 1) < 1e-12


def test_schedule_uniform_when_stable():
    # heavy boson, coarse cells: the quantum-pressure bound never binds
    r = _req(0, n=32, box=10.0, m_ev=1e-21, nsteps=80)
    a = schedule(r)
    assert len(a) == 81 and a[0] == A_START and a[-1] == A_END
    d = np.diff(np.log(a))
    assert np.allclose(d, math.log(100.0) / 80, rtol=1e-9)


def test_schedule_clamped_stops_short_and_is_stable():
    # light boson, fine cells: the bound binds early and the run stops short
    r = _req(0, n=256, box=1.0, m_ev=1e-23, nsteps=200)
    a = np.array(schedule(r))
    assert len(a) == 201 and a[-1] < A_END
    dx = r.box / r.n
    hm = hbar_over_m(r.m_ev) / dx ** 2
    p = oracle.Params(n=r.n, box=float(r.n), S=0.45, hbar_m=hm, comoving=True)
    for a0, a1 in zip(a[:-1], a[1:]):
        hub = math.sqrt(0.3 / a0 ** 3 + 0.7)
        # omega_max dt <= 0.5, dt = d ln a / H, with the oracle's omega_max
        assert oracle.omega_max(p, a0) * math.log(a1 / a0) / hub <= 0.5 * (1 + 1e-9)
    assert abs(OMEGA_MAX_COEF * hm / oracle.omega_max(p, 1.0) - 1) < 1e-4


def test_displacement_bound_and_chunked_schedule():
    """With a velocity bound no particle moves more than a cell per step;
    planning chunk by chunk with the same bound gives the same schedule as
    planning it whole."""
    r = _req(0, n=128, box=2.0, m_ev=1e-21, nsteps=200)
    vmax = 3.0                                           # cells * H0, canonical momentum
    a = np.array(schedule(r, vmax))
    for a0, a1 in zip(a[:-1], a[1:]):
        hub = math.sqrt(0.3 / a0 ** 3 + 0.7)
        # displacement vmax / a^2 * dt, dt = d ln a / H
        assert vmax / a0 ** 2 * math.log(a1 / a0) / hub <= 1.0 * (1 + 1e-9)
    assert a[-1] < schedule(r)[-1]                        # a tighter bound gets less far
    times = [A_START]
    while extend_times(r, times, 7, vmax):
        pass
    assert times == list(a)
    assert dlna_step(r, 0.5, 0.0) == math.log(100.0) / 200


def test_schedule_short_only_where_the_bound_binds():
    tr = make_trace(2000, seed=2026)
    short = 0
    for r in tr:
        a = schedule(r)
        clamped = np.any(np.diff(np.log(a)) < math.log(100.0) / r.nsteps * (1 - 1e-9))
        if a[-1] < A_END:
            short += 1
            assert clamped and len(a) == r.nsteps + 1
        else:
            assert a[-1] == A_END
    # light bosons in small, fine boxes: a minority of the trace
    assert 0.05 < short / len(tr) < 0.25, short / len(tr)


# ------------------------------------------------------------------ loop

def test_all_requests_served_fifo_within_size():
    tr = [_req(i, n=[32, 64, 128, 256][i % 4], arrival=0.01 * i, nsteps=20 + i) for i in range(24)]
    res, ex, sch = _serve(tr, {"pool_slots": {32: 2, 64: 2}, "max_large": 2})
    assert [r.rid for r in res] == list(range(24))
    assert all(r.status == "ok" for r in res)
    assert all(r.steps == len(schedule(q)) - 1 for r, q in zip(res, tr))
    admits = [rid for _, what, rid in sch.events if what == "admit"]
    for n in (32, 64, 128, 256):
        ids = [rid for rid in admits if tr[rid].n == n]
        assert ids == sorted(ids)
    assert all(r.finished >= r.admitted >= r.arrival for r in res)


def test_slot_reuse_and_memory_budget():
    # six 32^3 requests at once, a pool of two slots: at most two run together
    tr = [_req(i, n=32, arrival=0.0, nsteps=30) for i in range(6)]
    res, ex, sch = _serve(tr, {"pool_slots": {32: 2}})
    assert all(r.status == "ok" for r in res)
    assert ex.peak_active == 2
    # large runs under a tight budget: never more resident than fits
    tr = [_req(i, n=128, arrival=0.0, nsteps=30) for i in range(5)]
    budget = int(2.5 * 50 * 128 ** 3)
    res, ex, sch = _serve(tr, {"budget_bytes": budget, "max_large": 8})
    assert all(r.status == "ok" for r in res)
    assert ex.peak_used <= budget and ex.peak_active == 2


def test_refused_when_it_can_never_fit():
    tr = [_req(0, n=256), _req(1, n=32, arrival=0.1)]
    res, ex, sch = _serve(tr, {"budget_bytes": 50 * 128 ** 3})
    assert res[0].status == "refused" and res[1].status == "ok"


def test_idle_pool_memory_is_reclaimed_for_large_runs():
    # a pool fills most of the budget; once idle it is freed for a 128^3 run
    tr = [_req(0, n=64, arrival=0.0, nsteps=20), _req(1, n=128, arrival=0.5, nsteps=20)]
    budget = 50 * 128 ** 3 + 2 * 50 * 64 ** 3 + 1000
    res, ex, sch = _serve(tr, {"budget_bytes": budget, "pool_slots": {64: 8}})
    assert [r.status for r in res] == ["ok", "ok"]
    assert 64 not in ex.pools


def test_failed_run_frees_its_slot():
    tr = [_req(i, n=32, arrival=0.0, nsteps=20) for i in range(5)]
    res, ex, sch = _serve(tr, {"pool_slots": {32: 1}, "fail": {1, 3}})
    assert [r.status for r in res] == ["ok", "failed", "ok", "failed", "ok"]
    assert ex.pools[32]["free"] == [0]


def test_allocation_failure_is_reported_and_loop_continues():
    tr = [_req(i, n=128, arrival=0.0, nsteps=20) for i in range(3)]
    res, ex, sch = _serve(tr, {"oom": {1}})
    assert [r.status for r in res] == ["ok", "failed", "ok"]
    assert ex.used == 0


def test_time_compression_raises_load():
    tr = make_trace(60, rate=4.0, seed=7)
    kw = {"base": 2e-3, "per_particle": 2e-9, "max_large": 2}
    _, s1 = (lambda r: (r[0], summarize(r[0], tr)))(_serve(tr, kw, scale=1.0))
    _, s100 = (lambda r: (r[0], summarize(r[0], tr)))(_serve(tr, kw, scale=100.0))
    assert s1["ok"] == s100["ok"] == 60
    assert s100["p50_s"] > s1["p50_s"]
    assert s100["makespan_s"] < s1["makespan_s"]
    assert s100["particle_updates"] == s1["particle_updates"]


# ------------------------------------------------------------------ results routed to their requests

def _oracle_compute(req, state, times):
    """Final state of a request by the oracle (tiny meshes only)."""
    pos0, vel0, st = state
    dx = req.box / req.n
    hm = hbar_over_m(req.m_ev) / dx ** 2
    p = oracle.Params(n=req.n, box=float(req.n), S=1.5 * 0.3, hbar_m=hm, comoving=True,
                      omega_m=0.3, omega_l=0.7, h0=1.0, rho_floor=1e-6)
    x, v = oracle.run(st.pos, st.vel, p, times)
    return x, v


def test_results_alone_equal_results_in_the_mix():
    reqs = [Request(rid=i, n=8, box=[1.0, 3.0, 6.0][i % 3], m_ev=[1e-21, 1e-22, 1e-23][i % 3],
                    seed=100 + i, nsteps=12 + i, arrival=0.002 * i) for i in range(6)]
    states = {r.rid: (None, None, zeldovich_state(r.n, r.box, A_START, r.seed, m_ev=r.m_ev))
              for r in reqs}
    kw = {"batch_max_n": 8, "pool_slots": {8: 3}, "compute": _oracle_compute}
    mix, _, _ = _serve(reqs, kw, ics=lambda r: states[r.rid])
    for r in reqs:
        alone, _, _ = _serve([r], kw, ics=lambda q: states[q.rid])
        assert mix[r.rid].status == alone[0].status == "ok"
        assert np.array_equal(mix[r.rid].pos, alone[0].pos)
        assert np.array_equal(mix[r.rid].vel, alone[0].vel)
    # distinct requests give distinct results (no state mixed up)
    assert not np.array_equal(mix[0].pos, mix[1].pos)


def test_summary_counts():
    tr = [_req(i, n=32, arrival=0.0, nsteps=10) for i in range(4)] + [_req(4, n=256)]
    res, _, _ = _serve(tr, {"budget_bytes": 50 * 128 ** 3, "fail": {2}})
    s = summarize(res, tr)
    assert (s["ok"], s["failed"], s["refused"]) == (3, 1, 1)
    assert s["particle_updates"] == 3 * 32 ** 3 * 10
    assert s["p99_s"] >= s["p50_s"] > 0
