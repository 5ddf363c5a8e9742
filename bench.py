#!/usr/bin/env python
"""Throughput of one full particle-mesh step on one MI355X.

A step is one pass of the whole hot path over the particle set: CIC deposit
(integer, fixed-point), forward real FFT, Green's function, inverse FFT,
quantum-pressure stencil and the fused gather-kick-drift (merged half-kicks).
Workload: comoving box of 10 Mpc/h, 256^3 particles on a 256^3 mesh, boson
mass 1e-22 eV, Omega_m = 0.3, h = 0.7, Zel'dovich initial conditions at
a = 0.01 (seed 1), 32-bit fixed-point positions, FP32 FFT and stencils.
Inputs are resident in HBM before the timed region.

Prints one JSON line.  Also measured: the same step with the energies of
every synchronised time formed inside its kernels, the same box evolved to
a = 0.5 (a nonlinear, clustered state), the plain FP32 form of the step,
per-kernel times from HIP events on the library's stream, a short served
trace of independent requests (batched and one at a time), and the FP64
oracle on the host as a CPU baseline (whose fields also give both forms'
errors at the initial state).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s per full PM step at 256^3; p50/p99 run latency (served)"
HBM_PEAK_GBS = 8000.0
DLNA = math.log(100.0) / 500.0


def alg_bytes(n: int, npart: int, steps: int = 20) -> dict:
    """Algorithmic HBM bytes per launch of each kernel family (fixed form),
    averaged over the launches of one continued call of `steps` steps.

    cells: N^3; spectrum: (N/2+1) N^2 complex64.  Each byte that a kernel
    must read or write once: positions 12 B/particle (uint32 x3), velocities
    12 B/particle, int64 mass 8 B/cell, float meshes 4 B/cell.  Inside a call
    the Q stencil reads delta and phi and writes psi = F_g phi + F_q Q, and
    the next gather reads psi alone; the last stencil launch of a call writes
    Q and the first gather of a continued call reads phi and Q.
    """
    cells = n ** 3
    spec = 8 * (n // 2 + 1) * n * n
    k = max(1, steps)
    return {
        "fill_zero": 8 * cells,
        "deposit": 12 * npart + 16 * cells,         # read positions, read+write mass once
        "r2c_z": 8 * cells + 4 * cells + spec,      # mass in, delta and spectrum out
        "fft_y": 2 * spec,
        "fft_x_green": 2 * spec,
        "fft_y_inv": 2 * spec,
        "c2r_z": spec + 4 * cells,
        # delta and phi in, psi out (k - 1 launches); delta in, Q out (one)
        "qpot": (12 * (k - 1) + 8) * cells // k,
        # pos+vel in/out, psi once (phi and Q in the first launch), and the
        # fused deposit of the drifted particles (read+write of the int64
        # mass mesh once)
        "gather_kick_drift": 48 * npart + (4 * (k - 1) + 8) * cells // k + 16 * cells,
        # closing half-kick of a call: phi and Q in; on a sorted context it
        # also copies the positions from the workspace copies back
        "kick": 48 * npart + 8 * cells,
        "sort_count": 12 * npart + 8 * npart,        # positions in, key and rank out
        "sort_scatter": 8 * npart + 48 * npart,      # key, rank, pos+vel in, copies out
        "sort_copy": 48 * npart,
    }


def make_state(n, box):
    from synth import zeldovich_state
    return zeldovich_state(n, box, 0.01, seed=1, m_ev=1e-22)


EVOLVE_DLNA = math.log(100.0) / 150.0


def run_gpu(st, n, steps, warmup, a_start, kernel_pass=True, sort_every=10, fp32=False,
            evolve_to=None, box=10.0, diag=False, energies=False):
    """Time `steps` steps (after `warmup`) from a_start; with evolve_to, the
    state is first stepped (untimed) from a_start to evolve_to under the
    time-step condition of Sec. II A (no particle moves more than one cell
    per step; quantum-pressure bound; d ln a at most ln(100)/150), and the
    timed steps follow the same condition (d ln a at most ln(100)/500)."""
    import numpy as np
    import torch

    import paper_1608_00802_amd as pm
    from paper_1608_00802_amd.evolve import evolve, plan
    from synth import comoving_code_params

    dev = torch.device("cuda:0")
    hm = comoving_code_params(box, n, 1e-22, 0.7)["hbar_m_cells"] * (box / n) ** 2
    lp = pm.make_params(n, st.npart, box, precision=pm.PM_FP32 if fp32 else pm.PM_FIXED32,
                        comoving=True, omega_m=0.3, omega_l=0.7, h0=1.0, hbar_over_m=hm,
                        rho_floor=1e-6, rho_fp64_below=1e-3)
    ctx = pm.PMContext(lp, device=dev)
    p0 = st.pos_f32 if fp32 else st.pos_fixed.view(np.int32)
    pos = torch.from_numpy(p0.copy()).to(dev)
    vel = torch.from_numpy(st.vel32.copy()).to(dev)
    # sort_every < 0: adaptive interval (PM_SORT_AUTO); 0: never; k: every k steps
    # (the FP32 form has no adaptive interval: it sorts every 10 steps then)
    if sort_every < 0:
        sort_flag = pm.PM_SORT_EVERY(10) if fp32 else pm.PM_SORT_AUTO
    else:
        sort_flag = pm.PM_SORT_EVERY(sort_every) if sort_every else 0
    flags0 = 0
    evolve_steps = 0
    total = warmup + steps + (steps if kernel_pass else 0)
    hm_cells = comoving_code_params(box, n, 1e-22, 0.7)["hbar_m_cells"]
    if evolve_to is not None:
        ev = evolve(ctx, pos, vel, a_start, evolve_to, hm_cells, 0.3, flags=sort_flag,
                    dlna_max=EVOLVE_DLNA)
        evolve_steps = len(ev) - 1
        a_start = ev[-1]
        flags0 = pm.PM_CONTINUE
        vmax = 2.0 * float(vel.abs().max().item())
        times = plan(a_start, total, hm_cells, vmax, 0.3, dlna_max=DLNA)
    else:
        times = [a_start * math.exp(i * DLNA) for i in range(total + 1)]
    torch.cuda.synchronize()
    ctx.step(pos, vel, times[: warmup + 1], flags=sort_flag | flags0)
    torch.cuda.synchronize()
    stream = ctx.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # with energies: K, W, U, E of every synchronised time, formed inside the
    # step's kernels (pm_step_energies), into a device array
    rows = torch.empty((steps + 1, 4), dtype=torch.float64, device=dev) if energies else None

    def timed_call(seg):
        if energies:
            ctx.step_energies(pos, vel, seg, rows, flags=pm.PM_CONTINUE | sort_flag)
        else:
            ctx.step(pos, vel, seg, flags=pm.PM_CONTINUE | sort_flag)

    t0 = time.perf_counter()
    ev0.record(stream)
    timed_call(times[warmup: warmup + steps + 1])
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    out = {"wall_s": wall, "event_ms": ev_ms, "np": st.npart, "evolve_steps": evolve_steps,
           "a_timed": a_start, "a_timed_end": times[warmup + steps]}
    if energies:
        r = rows.cpu().numpy()
        out["energy_rows"] = {"first": [float(v) for v in r[1]], "last": [float(v) for v in r[-1]]}
    if kernel_pass:
        ctx.timing(True)
        timed_call(times[warmup + steps: warmup + 2 * steps + 1])
        out["kernels"] = ctx.timing_read()
        ctx.timing(False)
    if diag:
        out["diag"] = diag_pass(ctx, pos, vel, p0, times[-1] if kernel_pass else
                                times[warmup + steps])
    ok = bool(torch.isfinite(vel).all().item())
    out["finite"] = ok
    ctx.close()
    return out


def spline_section(st, n, box, steps=5, warmup=2, h=3.5):
    """The step with the paper's own coupling (pm_spline_step, h = 3.5 cells)
    on the same Zel'dovich box, sorted by tile first; wall time of `steps`
    steps after `warmup`, and its per-kernel times."""
    import numpy as np
    import torch

    import paper_1608_00802_amd as pm
    from synth import comoving_code_params

    dev = torch.device("cuda:0")
    hm = comoving_code_params(box, n, 1e-22, 0.7)["hbar_m_cells"] * (box / n) ** 2
    lp = pm.make_params(n, st.npart, box, precision=pm.PM_FIXED32, comoving=True, omega_m=0.3,
                        omega_l=0.7, h0=1.0, hbar_over_m=hm, rho_floor=1e-6, rho_fp64_below=1e-3)
    ctx = pm.PMContext(lp, device=dev)
    pos = torch.from_numpy(st.pos_fixed.view(np.int32).copy()).to(dev)
    vel = torch.from_numpy(st.vel32.copy()).to(dev)
    ctx.sort(pos, vel)
    times = [0.01 * math.exp(i * DLNA) for i in range(warmup + 2 * steps + 1)]
    ctx.spline_step(pos, vel, times[: warmup + 1], h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.spline_step(pos, vel, times[warmup: warmup + steps + 1], h)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.timing(True)
    ctx.spline_step(pos, vel, times[warmup + steps:], h)
    kern = ctx.timing_read()
    ctx.timing(False)
    out = {"form": "pm_spline_step: spline density (h = 3.5 cells) for gravity and Q, "
                   "kernel-gradient Q force, unfused KDK",
           "value": st.npart * steps / wall, "ms_per_step": wall * 1e3 / steps,
           "finite": bool(torch.isfinite(vel).all().item()),
           "kernels": {k: {"launches": v[0], "avg_ms": round(v[1] / v[0], 4)}
                       for k, v in kern.items()}}
    ctx.close()
    return out


def diag_pass(ctx, pos, vel, p0, a, reps=3):
    """Grid diagnostics of the state left by the timed steps (after the timed
    region), sorted by tile first so that the momentum deposit takes its
    tiled path without strays: the bulk/dispersion split of K, the RMS
    relative density difference against the initial state and the power
    spectrum, each timed as a blocking call."""
    import torch
    pos0 = torch.from_numpy(p0.copy()).to(pos.device)
    ctx.sort(pos, vel)
    ctx.kinetic_split(pos, vel, a)          # warm-up
    ctx.timing(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ks = ctx.kinetic_split(pos, vel, a)
    t1 = time.perf_counter()
    for _ in range(reps):
        rms, cells = ctx.density_rms_diff(pos, pos0)
    t2 = time.perf_counter()
    for _ in range(reps):
        _, pk, _ = ctx.power_spectrum(pos)
    t3 = time.perf_counter()
    # the paper's spline coupling (h = 3.5 cells): density, Q, kernel-gradient force
    n = ctx.n
    dl = torch.empty(n ** 3, dtype=torch.float32, device=pos.device)
    qq = torch.empty_like(dl)
    acc = torch.empty(3, ctx.np, dtype=torch.float32, device=pos.device)
    ctx.spline_density(pos, dl, 3.5)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(reps):
        ctx.spline_density(pos, dl, 3.5)
        ctx.qpot(dl, qq)
        ctx.spline_qforce(pos, qq, acc, 3.5)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    kern = ctx.timing_read()
    ctx.timing(False)
    np_ = ctx.np
    out = {"a": a, "state": "sorted by tile just before", "K_disp_over_K": ks["K_disp"] / ks["K"],
           "rms_rel_diff_vs_initial": rms,
           "cells": cells, "kinetic_split_ms": (t1 - t0) * 1e3 / reps,
           "density_rms_diff_ms": (t2 - t1) * 1e3 / reps,
           "power_spectrum_ms": (t3 - t2) * 1e3 / reps, "power_shells": len(pk),
           "spline_chain_ms": (t5 - t4) * 1e3 / reps}
    for name in ("momentum_deposit", "diag_nodes", "fft_x_power", "spline_deposit",
                 "spline_qforce"):
        if name in kern:
            launches, total_ms = kern[name]
            out[name] = {"launches": launches, "avg_ms": round(total_ms / launches, 5)}
    for name in ("spline_deposit", "spline_qforce"):
        if name in out:
            # nodes inside the support of h = 3.5 cells: 4/3 pi h^3 = 179.6 per particle
            out[name]["kernel_evals_per_s"] = 179.6 * np_ / (out[name]["avg_ms"] * 1e-3)
    if "momentum_deposit" in out:
        out["momentum_deposit"]["fp64_atomics_per_s"] = 8 * np_ / (
            out["momentum_deposit"]["avg_ms"] * 1e-3)
    return out


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling HBM byte counters."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


# rocprofv3 kernel name of each kernel family in the traffic summary, for
# log2 N = {ln} (inside a call the gather reads psi alone and the stencil
# writes psi)
TRAFFIC_KERNEL = {"gather_kick_drift": "k_gather_tiled<{ln}, true, false, 1, true, 0, false>",
                  "deposit": "k_deposit_tiled<{ln}, true>",
                  "qpot": "k_qpot_tiled<{ln}, true, 2>", "r2c_z": "k_r2c_z<{ln}, 0>",
                  "fft_y": "k_fft_y_reg<{ln}, false>", "fft_x_green": "k_fft_x_green_reg<{ln}>",
                  "fft_y_inv": "k_fft_y_reg<{ln}, true>", "c2r_z": "k_c2r_z<{ln}>",
                  "fill_zero": "k_fill_zero16"}


# the sources each kernel family is built from (its counters go stale when one changes)
TRAFFIC_SOURCES = {"gather_kick_drift": ("gather.hip", "cic.h", "internal.h"),
                   "deposit": ("deposit.hip", "cic.h", "internal.h"),
                   "qpot": ("stencil.hip", "internal.h")}
for _k in ("r2c_z", "fft_y", "fft_x_green", "fft_y_inv", "c2r_z"):
    TRAFFIC_SOURCES[_k] = ("fft.hip", "internal.h")
TRAFFIC_SOURCES["fill_zero"] = ("deposit.hip", "internal.h")


def measured_traffic(kernel: str, n: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none for this kernel and size or if a source the kernel
    is built from changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pm_step_{n}_traffic.json")
    if not os.path.exists(path) or kernel not in TRAFFIC_KERNEL:
        return None
    with open(path) as fh:
        rec = json.load(fh)
    deps = TRAFFIC_SOURCES.get(kernel, ())
    for f, h in rec.get("source_sha256_16", {}).items():
        if f not in deps:
            continue
        src = os.path.join(ROOT, "paper_1608_00802_amd", "csrc", f)
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != h:
            return None
    k = rec["kernels"].get(TRAFFIC_KERNEL[kernel].format(ln=n.bit_length() - 1))
    if k is None:
        return None
    return int(k["fetch_bytes"] + k["write_bytes"])


def kernel_table(kern, n, npart, steps):
    ab = alg_bytes(n, npart, steps)
    rows = {}
    for name, (launches, ms) in kern.items():
        avg = ms / launches
        row = {"launches": launches, "avg_ms": round(avg, 5)}
        if name in ab:
            row["alg_bytes"] = ab[name]
            row["alg_GBs"] = round(ab[name] / (avg * 1e-3) / 1e9, 1)
        rows[name] = row
    return rows


def gpu_fields(st, n, box, fp32):
    """delta, phi, Q_c and the acceleration of the initial state (a = 0.01)
    through the library in one precision, as float64 host arrays (outside
    every timed region)."""
    import numpy as np
    import torch

    import paper_1608_00802_amd as pm
    from synth import comoving_code_params

    dev = torch.device("cuda:0")
    hm = comoving_code_params(box, n, 1e-22, 0.7)["hbar_m_cells"] * (box / n) ** 2
    lp = pm.make_params(n, st.npart, box, precision=pm.PM_FP32 if fp32 else pm.PM_FIXED32,
                        comoving=True, omega_m=0.3, omega_l=0.7, h0=1.0, hbar_over_m=hm,
                        rho_floor=1e-6, rho_fp64_below=1e-3)
    ctx = pm.PMContext(lp, device=dev)
    pos = torch.from_numpy((st.pos_f32 if fp32 else st.pos_fixed.view(np.int32)).copy()).to(dev)
    d = torch.empty(n ** 3, dtype=torch.float32, device=dev)
    ph = torch.empty_like(d)
    qq = torch.empty_like(d)
    acc = torch.empty((3, st.npart), dtype=torch.float32, device=dev)
    ctx.deposit(pos, d)
    ctx.poisson(None, ph)
    ctx.qpot(None, qq)
    ctx.force(pos, acc, 0.01)
    torch.cuda.synchronize()
    out = {"delta": d.cpu().numpy().astype(np.float64).reshape(n, n, n),
           "phi": ph.cpu().numpy().astype(np.float64).reshape(n, n, n),
           "Q": qq.cpu().numpy().astype(np.float64).reshape(n, n, n),
           "force": acc.cpu().numpy().T.astype(np.float64)}
    ctx.close()
    del pos, d, ph, qq, acc
    return out


def cpu_baseline(st, n, box, gpu_sets=None):
    """FP64 oracle, one steady-state kick-drift-kick step on the full workload.

    The oracle's fields and forces at the initial state, computed on the way
    (untimed), also give the relative L2 error of each precision form of the
    library (gpu_sets: {form: gpu_fields(...)}) on rho, phi, Q and the force."""
    import numpy as np

    import oracle
    from synth import comoving_code_params
    hm = comoving_code_params(box, n, 1e-22, 0.7)["hbar_m_cells"]
    p = oracle.Params(n=n, box=float(n), S=1.5 * 0.3, hbar_m=hm, comoving=True,
                      omega_m=0.3, omega_l=0.7, h0=1.0, rho_floor=1e-6)
    a0 = 0.01
    a1 = a0 * math.exp(DLNA)
    # opening forces, untimed
    rho, delta, phi, q = oracle.fields(st.pos, p)
    gphi = oracle.interp_cic(oracle.grad_central(phi, p), st.pos, p)
    gq = oracle.interp_cic(oracle.grad_central(q, p), st.pos, p)
    errors = {}

    def rel(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    for form, g in (gpu_sets or {}).items():
        errors[form] = {"rho": rel(1.0 + g["delta"], rho), "phi": rel(g["phi"], phi),
                        "Q": rel(g["Q"], q),
                        "force": rel(g["force"], gphi / a0 + gq / a0 ** 2)}
    del rho, delta, phi, q
    t0 = time.perf_counter()
    oracle.kdk_step(st.pos, st.vel, p, a0, a1, (gphi, gq))
    dt = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count()
    out = {"value": st.npart / dt, "unit": "particle-updates/s", "cores": 1,
           "cores_available": cores, "kind": "oracle",
           "sample": f"one steady-state KDK step (force evaluation at the drifted positions, "
                     f"both half-kicks, drift) of the FP64 NumPy oracle on the full {n}^3 "
                     f"workload, single-threaded NumPy; {dt:.1f} s"}
    if errors:
        out["gpu_rel_l2_at_a0"] = errors
    return out


def batch_launch_section(n=32, slots=64, steps=10, calls=6):
    """Launch cost of batched small boxes: one batch of `slots` runs of n^3
    (every kernel launched once for all slots) stepped `calls` times by
    `steps` steps, call by call and replayed from captured HIP graphs
    (PM_BATCH_GRAPH); ms per step of the whole batch, and the GPU time of the
    kernels alone from HIP events around each call."""
    import numpy as np
    import torch

    import paper_1608_00802_amd as pm
    from paper_1608_00802_amd import serve
    from synth import zeldovich_state

    dev = torch.device("cuda:0")
    out = {"batch": f"{slots} runs of {n}^3 particles on {n}^3 meshes, {steps} steps per call"}
    states = [zeldovich_state(n, 2.0 + 0.1 * i, 0.01, seed=100 + i, m_ev=1e-22)
              for i in range(slots)]
    for mode, flag in (("eager", 0), ("graph", pm.PM_BATCH_GRAPH)):
        stream = torch.cuda.Stream(dev)
        lp = pm.make_params(n, n ** 3, 2.0, comoving=True, omega_m=0.3, omega_l=0.7, h0=1.0)
        with torch.cuda.stream(stream):
            b = pm.PMBatch(lp, slots, device=dev, stream=stream)
        for i, st in enumerate(states):
            box = 2.0 + 0.1 * i
            hm = serve.hbar_over_m(1e-22)
            b.load(i, torch.from_numpy(st.pos_fixed.view(np.int32).copy()).to(dev),
                   torch.from_numpy(st.vel32.copy()).to(dev), box, hm)
        sl = list(range(slots))
        a = [0.01] * slots

        def call(first):
            times = []
            for i in range(slots):
                t = [a[i] * math.exp(k * DLNA) for k in range(steps + 1)]
                a[i] = t[-1]
                times.append(t)
            b.step(sl, times, pm.PM_SORT_EVERY(10) | flag | (0 if first else pm.PM_CONTINUE))

        call(True)
        call(False)                       # captures the continued shape
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(calls):
            call(False)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[mode] = {"ms_per_step": round(wall * 1e3 / (calls * steps), 4),
                     "event_ms_per_step": round(e0.elapsed_time(e1) / (calls * steps), 4),
                     "particle_updates_per_s": slots * n ** 3 * calls * steps / wall}
        b.close()
    out["speedup_graph_vs_eager"] = round(out["eager"]["ms_per_step"] /
                                          out["graph"]["ms_per_step"], 3)
    return out


def serve_section(trace, ics):
    """Served trace: batched at a compressed arrival rate, and one request at
    a time (fixed point, plain FP32) with every request queued at once."""
    from paper_1608_00802_amd import serve
    out = {"requests": len(trace), "trace": "Poisson arrivals (4/s, seed 2026) of independent "
           "runs: N in {32,64,128,256}, box U[1,10] Mpc/h, m log-uniform [1e-23,1e-21] eV, "
           "50-200 steps from a = 0.01, Zel'dovich ICs built on the host before the clock"}
    for rec in serve.run_modes(trace, ics, scales=(100.0,), serial=True, emit=lambda d: None,
                               eager=True):
        rec = dict(rec)
        rec.pop("per_size", None)
        name = rec.pop("mode") + ("" if rec.get("time_scale") is None else "_x100")
        rec.pop("time_scale", None)
        out[name] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in rec.items()}
    b = out.get("batched_x100", {}).get("particle_updates_per_s")
    be = out.get("batched_eager_x100", {}).get("particle_updates_per_s")
    s1 = out.get("serial_fixed", {}).get("particle_updates_per_s")
    s2 = out.get("serial_fp32", {}).get("particle_updates_per_s")
    if b and s1 and s2:
        out["speedup_batched_vs_serial_fixed"] = round(b / s1, 3)
        out["speedup_batched_vs_serial_fp32"] = round(b / s2, 3)
    if b and be:
        out["speedup_graphs_vs_eager_batched"] = round(b / be, 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--box", type=float, default=10.0, help="box side in Mpc/h")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-evolved", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-energies", action="store_true",
                    help="skip the timed step with per-step energies")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-spline", action="store_true",
                    help="skip the step with the spline kernel")
    ap.add_argument("--no-diag", action="store_true",
                    help="skip the grid diagnostics after the evolved run")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--evolved-only", action="store_true",
                    help="profiling aid: time only the evolved (a = 0.5) state, print a short "
                         "line instead of the benchmark line")
    ap.add_argument("--no-kernel-pass", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--sort-every", type=int, default=-1,
                    help="sort particles by tile every k steps inside the timed steps (0: never, "
                         "-1: adaptive interval from sampled stray counts, the default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the single-GPU box is the whole measured job)", file=sys.stderr)
        sys.exit(2)
    n = args.n
    # host-side inputs first, before this process touches the GPU
    st = make_state(n, args.box)
    trace = ics = None
    if not args.no_serve:
        from paper_1608_00802_amd import serve
        trace = serve.make_trace(args.serve_requests)
        try:
            workers = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:  # pragma: no cover
            workers = 8
        ics = serve.generate_ics(trace, workers)
    if args.copy_calibration:
        copy_calibration()
    if args.evolved_only:
        # profiling aid: only the evolved state's steps (no JSON line)
        re_ = run_gpu(st, n, args.steps, args.warmup, 0.01, kernel_pass=not args.no_kernel_pass,
                      sort_every=args.sort_every, evolve_to=0.5, box=args.box)
        print(json.dumps({"evolved_only": True, "a": re_["a_timed"], "evolve_steps":
                          re_["evolve_steps"], "ms_per_step": re_["wall_s"] * 1e3 / args.steps}),
              flush=True)
        return
    res = run_gpu(st, n, args.steps, args.warmup, 0.01, kernel_pass=not args.no_kernel_pass,
                  sort_every=args.sort_every, box=args.box)
    value = res["np"] * args.steps / res["wall_s"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: Zel'dovich initial conditions from a seeded Gaussian field",
        "config": {
            "workload": f"comoving {args.box:g} Mpc/h box, {n}^3 particles on a {n}^3 mesh, "
                        "m = 1e-22 eV, Omega_m = 0.3, h = 0.7, Zel'dovich ICs at a = 0.01, "
                        "fixed-point uint32 positions, FP32 FFT/stencils, int64 deposit",
            "n_mesh": n,
            "n_part": res["np"],
            "a_start": 0.01,
            "dlna_per_step": DLNA,
            "event_ms_per_step": res["event_ms"] / args.steps,
            "sort_every": "adaptive" if args.sort_every < 0 else args.sort_every,
        },
    }
    if "kernels" in res:
        table = kernel_table(res["kernels"], n, res["np"], args.steps)
        line["kernels"] = table
        timed = {k: v for k, v in table.items() if "alg_bytes" in v}
        dom = max(timed, key=lambda k: timed[k]["avg_ms"] * timed[k]["launches"])
        ach = timed[dom]["alg_GBs"]
        line["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                            "traffic": measured_traffic(dom, n),
                            "alg_bytes": timed[dom]["alg_bytes"]}
        ab = alg_bytes(n, res["np"], args.steps)
        per_step = ("fill_zero", "r2c_z", "fft_y", "fft_x_green", "fft_y_inv", "c2r_z",
                    "qpot", "gather_kick_drift")
        step_bytes = sum(ab[k] for k in per_step)
        line["step_alg_bytes"] = step_bytes
        line["step_alg_GBs"] = round(step_bytes / (res["wall_s"] / args.steps) / 1e9, 1)
    if not args.no_energies:
        rn = run_gpu(st, n, args.steps, args.warmup, 0.01, kernel_pass=not args.no_kernel_pass,
                     sort_every=args.sort_every, box=args.box, energies=True)
        line["with_energies"] = {
            "form": "pm_step_energies: the same step with K (gather, at the synchronised "
                    "time), W and U (Q stencil) partial sums and one reduction kernel per step",
            "value": rn["np"] * args.steps / rn["wall_s"],
            "ms_per_step": rn["wall_s"] * 1e3 / args.steps,
            "rows_K_W_U_E": rn["energy_rows"]}
        if "kernels" in rn:
            line["with_energies"]["kernels"] = kernel_table(rn["kernels"], n, rn["np"],
                                                            args.steps)
    if not args.no_fp32:
        rf = run_gpu(st, n, args.steps, args.warmup, 0.01, kernel_pass=False,
                     sort_every=args.sort_every, fp32=True, box=args.box)
        vf = rf["np"] * args.steps / rf["wall_s"]
        line["plain_fp32"] = {
            "form": "float32 positions, float atomics deposit, sqrt(rho) formed directly for Q, "
                    "same FFT/stencil/gather kernels",
            "value": vf, "ms_per_step": rf["wall_s"] * 1e3 / args.steps,
            "speedup_fixed_vs_fp32": round(value / vf, 3)}
    if not args.no_evolved:
        re_ = run_gpu(st, n, args.steps, args.warmup, 0.01, kernel_pass=not args.no_kernel_pass,
                      sort_every=args.sort_every, evolve_to=0.5, box=args.box,
                      diag=not args.no_diag)
        line["evolved"] = {
            "state": f"the same box stepped from a = 0.01 to a = 0.5 ({re_['evolve_steps']} "
                     f"steps, untimed) under the time-step condition of Sec. II A (no particle "
                     f"moves more than one cell per step, quantum-pressure bound, d ln a <= "
                     f"ln(100)/150), then timed from a = {re_['a_timed']:.4f} to "
                     f"{re_['a_timed_end']:.4f} under the same condition: nonlinear, clustered",
            "value": re_["np"] * args.steps / re_["wall_s"],
            "ms_per_step": re_["wall_s"] * 1e3 / args.steps,
            "finite": re_["finite"],
        }
        if "kernels" in re_:
            line["evolved"]["kernels"] = kernel_table(re_["kernels"], n, re_["np"], args.steps)
        if "diag" in re_:
            line["evolved"]["diagnostics"] = re_["diag"]
    if not args.no_spline:
        line["spline_form"] = spline_section(st, n, args.box)
    if not args.no_serve:
        line["batch_launch"] = batch_launch_section()
    if trace is not None:
        line["serving"] = serve_section(trace, ics)
        del ics
    if not args.no_cpu_baseline:
        sets = {"fixed": gpu_fields(st, n, args.box, False)}
        if not args.no_fp32:
            sets["plain_fp32"] = gpu_fields(st, n, args.box, True)
        line["cpu_baseline"] = cpu_baseline(st, n, args.box, sets)
        del sets
        errs = line["cpu_baseline"].get("gpu_rel_l2_at_a0", {})
        if "plain_fp32" in line and "plain_fp32" in errs:
            # the speedup counts as one at equal accuracy only where the plain
            # form meets the same 1e-5 bound on every field
            worst = max(errs["plain_fp32"].values())
            line["plain_fp32"]["rel_l2_vs_oracle_at_a0"] = errs["plain_fp32"]
            line["plain_fp32"]["fixed_rel_l2_vs_oracle_at_a0"] = errs["fixed"]
            line["plain_fp32"]["equal_accuracy"] = bool(worst < 1e-5)
            if worst >= 1e-5:
                line["plain_fp32"]["note"] = (
                    "unequal accuracy: the plain FP32 form misses the 1e-5 bound that the "
                    "fixed-point form meets, so the speedup compares a more accurate step "
                    "with a less accurate one")
    line["finite"] = res["finite"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
