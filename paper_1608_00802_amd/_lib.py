"""ctypes binding of libfdmpm (C ABI in include/fdmpm.h).

Argument marshalling and host-side validation only: every step of the
particle-mesh path runs in the HIP kernels of the shared library.  PyTorch
supplies device memory and the stream.  If the library has not been built
the import of this module fails loudly; there is no fallback path.
"""

from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdmpm.so")

PM_OK, PM_EINVAL, PM_ENOMEM, PM_EDEVICE, PM_EUNSUPPORTED, PM_ESTATE = 0, -1, -2, -3, -4, -5
PM_FP32, PM_FIXED32 = 0, 1
PM_CONTINUE = 1
PM_SORT_AUTO = 1 << 24
PM_BATCH_GRAPH = 1 << 25


def PM_SORT_EVERY(k: int) -> int:
    return (int(k) & 0xffff) << 8

EXPORTED = ("pm_workspace_bytes", "pm_init", "pm_deposit", "pm_poisson", "pm_qpot",
            "pm_force", "pm_step", "pm_step_energies", "pm_sort", "pm_energy", "pm_kinetic_split",
            "pm_density_rms_diff", "pm_power_spectrum", "pm_spline_density",
            "pm_spline_qforce", "pm_spline_step", "pm_spline_energy", "pm_timing_enable", "pm_timing_read",
            "pm_batch_workspace_bytes", "pm_batch_init", "pm_batch_slot_offset",
            "pm_batch_set_slot", "pm_batch_step", "pm_batch_destroy", "pm_poisson_static",
            "pm_destroy", "pm_strerror")
PM_BATCH_MAX_STEPS = 256


class PMParams(ctypes.Structure):
    _fields_ = [
        ("n_mesh", c_int32),
        ("precision", c_int32),
        ("n_part", c_int64),
        ("box", c_double),
        ("comoving", c_int32),
        ("reserved0", c_int32),
        ("four_pi_G_rhobar", c_double),
        ("omega_m", c_double),
        ("omega_l", c_double),
        ("h0", c_double),
        ("hbar_over_m", c_double),
        ("rho_floor", c_double),
        ("rho_fp64_below", c_double),
    ]


class PMEnergies(ctypes.Structure):
    _fields_ = [("K", c_double), ("W", c_double), ("U", c_double), ("E", c_double)]


class PMKineticParts(ctypes.Structure):
    _fields_ = [("K", c_double), ("K_bulk", c_double), ("K_disp", c_double)]


class PMKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_int64), ("total_ms", c_double)]


class PMSlotParams(ctypes.Structure):
    _fields_ = [("box", c_double), ("hbar_over_m", c_double)]


class PMError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {strerror(status)} (status {status})")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfdmpm.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: call __graft_entry__.build() or "
                          "python -m paper_1608_00802_amd.build")
    # torch first: the library must bind to the HIP runtime that owns torch's
    # streams and allocations (torch ships its own); loaded before torch, it
    # would bring up a second runtime and every call on torch's memory fails
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = POINTER
    sig = {
        "pm_workspace_bytes": ([P(PMParams), P(c_size_t)], c_int32),
        "pm_init": ([P(PMParams), c_void_p, c_size_t, c_void_p, P(c_void_p)], c_int32),
        "pm_deposit": ([c_void_p, c_void_p, c_void_p], c_int32),
        "pm_poisson": ([c_void_p, c_void_p, c_void_p], c_int32),
        "pm_qpot": ([c_void_p, c_void_p, c_void_p], c_int32),
        "pm_force": ([c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_double], c_int32),
        "pm_step": ([c_void_p, c_void_p, c_void_p, P(c_double), c_int32, c_int32], c_int32),
        "pm_step_energies": ([c_void_p, c_void_p, c_void_p, P(c_double), c_int32, c_int32,
                              c_void_p], c_int32),
        "pm_sort": ([c_void_p, c_void_p, c_void_p, c_void_p], c_int32),
        "pm_energy": ([c_void_p, c_void_p, c_void_p, c_double, P(PMEnergies)], c_int32),
        "pm_kinetic_split": ([c_void_p, c_void_p, c_void_p, c_double, P(PMKineticParts)],
                             c_int32),
        "pm_density_rms_diff": ([c_void_p, c_void_p, c_void_p, P(c_double), P(c_int64)], c_int32),
        "pm_power_spectrum": ([c_void_p, c_void_p, c_int32, P(c_double), P(c_double),
                               P(c_double)], c_int32),
        "pm_spline_density": ([c_void_p, c_void_p, c_double, c_void_p], c_int32),
        "pm_spline_qforce": ([c_void_p, c_void_p, c_void_p, c_double, c_void_p], c_int32),
        "pm_spline_step": ([c_void_p, c_void_p, c_void_p, P(c_double), c_int32, c_double],
                           c_int32),
        "pm_spline_energy": ([c_void_p, c_void_p, c_void_p, c_double, c_double, P(PMEnergies)],
                             c_int32),
        "pm_timing_enable": ([c_void_p, c_int32], c_int32),
        "pm_timing_read": ([c_void_p, P(PMKernelTime), c_int32, P(c_int32)], c_int32),
        "pm_batch_workspace_bytes": ([P(PMParams), c_int32, P(c_size_t)], c_int32),
        "pm_batch_init": ([P(PMParams), c_int32, c_void_p, c_size_t, c_void_p, P(c_void_p)],
                          c_int32),
        "pm_batch_slot_offset": ([c_void_p, c_int32, P(c_size_t)], c_int32),
        "pm_batch_set_slot": ([c_void_p, c_int32, P(PMSlotParams)], c_int32),
        "pm_batch_step": ([c_void_p, c_void_p, c_void_p, c_int32, P(c_int32), P(c_double),
                           c_int32, c_int32], c_int32),
        "pm_batch_destroy": ([c_void_p], c_int32),
        "pm_poisson_static": ([c_int32, c_double, c_void_p, c_void_p, c_void_p], c_int32),
        "pm_destroy": ([c_void_p], c_int32),
        "pm_strerror": ([c_int32], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def strerror(status: int) -> str:
    try:
        return load_library().pm_strerror(status).decode()
    except ImportError:
        return f"status {status}"


def _check(status: int, where: str) -> None:
    if status != PM_OK:
        raise PMError(status, where)


def make_params(n_mesh: int, n_part: int, box: float, *, precision: int = PM_FIXED32,
                comoving: bool = False, four_pi_G_rhobar: float = 1.0, omega_m: float = 0.3,
                omega_l: float = 0.7, h0: float = 1.0, hbar_over_m: float = 0.0,
                rho_floor: float = 1e-6, rho_fp64_below: float = 1e-3) -> PMParams:
    return PMParams(int(n_mesh), int(precision), int(n_part), float(box), int(bool(comoving)), 0,
                    float(four_pi_G_rhobar), float(omega_m), float(omega_l), float(h0),
                    float(hbar_over_m), float(rho_floor), float(rho_fp64_below))


# ------------------------------------------------------------------ same-named C calls

def pm_workspace_bytes(params: PMParams) -> int:
    n = c_size_t(0)
    _check(load_library().pm_workspace_bytes(byref(params), byref(n)), "pm_workspace_bytes")
    return n.value


def pm_init(params: PMParams, workspace_ptr: int, nbytes: int, stream_ptr: int) -> int:
    ctx = c_void_p(None)
    _check(load_library().pm_init(byref(params), c_void_p(workspace_ptr), nbytes,
                                  c_void_p(stream_ptr), byref(ctx)), "pm_init")
    return ctx.value


def pm_deposit(ctx: int, pos_ptr: int, delta_ptr: int | None) -> None:
    _check(load_library().pm_deposit(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(delta_ptr)),
           "pm_deposit")


def pm_poisson(ctx: int, delta_ptr: int | None, phi_ptr: int | None) -> None:
    _check(load_library().pm_poisson(c_void_p(ctx), c_void_p(delta_ptr), c_void_p(phi_ptr)),
           "pm_poisson")


def pm_qpot(ctx: int, delta_ptr: int | None, q_ptr: int | None) -> None:
    _check(load_library().pm_qpot(c_void_p(ctx), c_void_p(delta_ptr), c_void_p(q_ptr)),
           "pm_qpot")


def pm_force(ctx: int, phi_ptr: int | None, q_ptr: int | None, pos_ptr: int, acc_ptr: int,
             a: float) -> None:
    _check(load_library().pm_force(c_void_p(ctx), c_void_p(phi_ptr), c_void_p(q_ptr),
                                   c_void_p(pos_ptr), c_void_p(acc_ptr), float(a)), "pm_force")


def pm_step(ctx: int, pos_ptr: int, vel_ptr: int, times, flags: int = 0) -> None:
    t = [float(v) for v in times]
    arr = (c_double * len(t))(*t)
    _check(load_library().pm_step(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(vel_ptr), arr,
                                  len(t) - 1, int(flags)), "pm_step")


def pm_step_energies(ctx: int, pos_ptr: int, vel_ptr: int, times, flags: int,
                     energies_ptr: int) -> None:
    t = [float(v) for v in times]
    arr = (c_double * len(t))(*t)
    _check(load_library().pm_step_energies(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(vel_ptr),
                                           arr, len(t) - 1, int(flags), c_void_p(energies_ptr)),
           "pm_step_energies")


def pm_sort(ctx: int, pos_ptr: int, vel_ptr: int, ids_ptr: int | None) -> None:
    _check(load_library().pm_sort(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(vel_ptr),
                                  c_void_p(ids_ptr)), "pm_sort")


def pm_energy(ctx: int, pos_ptr: int, vel_ptr: int, a: float) -> dict:
    out = PMEnergies()
    _check(load_library().pm_energy(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(vel_ptr),
                                    float(a), byref(out)), "pm_energy")
    return {"K": out.K, "W": out.W, "U": out.U, "E": out.E}


def pm_kinetic_split(ctx: int, pos_ptr: int, vel_ptr: int, a: float) -> dict:
    out = PMKineticParts()
    _check(load_library().pm_kinetic_split(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(vel_ptr),
                                           float(a), byref(out)), "pm_kinetic_split")
    return {"K": out.K, "K_bulk": out.K_bulk, "K_disp": out.K_disp}


def pm_density_rms_diff(ctx: int, pos_a_ptr: int, pos_b_ptr: int) -> tuple:
    rms = c_double()
    cells = c_int64()
    _check(load_library().pm_density_rms_diff(c_void_p(ctx), c_void_p(pos_a_ptr),
                                              c_void_p(pos_b_ptr), byref(rms), byref(cells)),
           "pm_density_rms_diff")
    return rms.value, cells.value


def pm_power_spectrum(ctx: int, pos_ptr: int, nbins: int) -> tuple:
    """(k, P, counts) as three lists of nbins floats."""
    nb = int(nbins)
    k = (c_double * max(nb, 1))()
    p = (c_double * max(nb, 1))()
    cnt = (c_double * max(nb, 1))()
    _check(load_library().pm_power_spectrum(c_void_p(ctx), c_void_p(pos_ptr), nb, k, p, cnt),
           "pm_power_spectrum")
    return list(k)[:nb], list(p)[:nb], list(cnt)[:nb]


def pm_spline_density(ctx: int, pos_ptr: int, h: float, delta_ptr: int) -> None:
    _check(load_library().pm_spline_density(c_void_p(ctx), c_void_p(pos_ptr), float(h),
                                            c_void_p(delta_ptr)), "pm_spline_density")


def pm_spline_qforce(ctx: int, pos_ptr: int, q_ptr: int, h: float, acc_ptr: int) -> None:
    _check(load_library().pm_spline_qforce(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(q_ptr),
                                           float(h), c_void_p(acc_ptr)), "pm_spline_qforce")


def pm_spline_step(ctx: int, pos_ptr: int, vel_ptr: int, times, h: float) -> None:
    t = [float(x) for x in times]
    arr = (c_double * len(t))(*t)
    _check(load_library().pm_spline_step(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(vel_ptr),
                                         arr, len(t) - 1, float(h)), "pm_spline_step")


def pm_spline_energy(ctx: int, pos_ptr: int, vel_ptr: int, h: float, a: float) -> dict:
    out = PMEnergies()
    _check(load_library().pm_spline_energy(c_void_p(ctx), c_void_p(pos_ptr), c_void_p(vel_ptr),
                                           float(h), float(a), byref(out)), "pm_spline_energy")
    return {"K": out.K, "W": out.W, "U": out.U, "E": out.E}


def pm_timing_enable(ctx: int, on: bool) -> None:
    _check(load_library().pm_timing_enable(c_void_p(ctx), int(bool(on))), "pm_timing_enable")


def pm_timing_read(ctx: int) -> dict:
    """{kernel family: (launches, total ms)} since the last pm_timing_enable."""
    buf = (PMKernelTime * 32)()
    n = c_int32(0)
    _check(load_library().pm_timing_read(c_void_p(ctx), buf, 32, byref(n)), "pm_timing_read")
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(n.value)}


def pm_destroy(ctx: int) -> None:
    _check(load_library().pm_destroy(c_void_p(ctx)), "pm_destroy")


# ------------------------------------------------------------------ torch-facing wrapper

class PMContext:
    """One particle-mesh problem bound to a torch device and stream.

    The workspace is a torch uint8 tensor owned by this object.  Particle
    arrays are torch tensors: positions [3, Np] uint32 (fixed point, stored
    as int32 bit patterns) or float32 (cells), velocities [3, Np] float32.
    Shapes, dtypes, devices and contiguity are checked here before any call.
    """

    def __init__(self, params: PMParams, device=None, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device if device is not None else "cuda:0")
        if self.device.type != "cuda":
            raise ValueError("PMContext needs a GPU device")
        self.params = params
        self.n = params.n_mesh
        self.np = params.n_part
        self.fixed = params.precision == PM_FIXED32
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nbytes = pm_workspace_bytes(params)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.ctx = pm_init(params, self.workspace.data_ptr(), self.nbytes,
                               self.stream.cuda_stream)

    # -- validation
    def _mesh(self, t, name):
        torch = self.torch
        if t is None:
            return None
        if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous() \
                or t.numel() != self.n ** 3:
            raise ValueError(f"{name}: need contiguous float32 [{self.n}]^3 on {self.device}")
        return t.data_ptr()

    def _pos(self, t):
        torch = self.torch
        want = torch.int32 if self.fixed else torch.float32
        if t.dtype not in ((torch.int32, torch.uint32) if self.fixed else (torch.float32,)) \
                or t.device != self.device or not t.is_contiguous() \
                or tuple(t.shape) != (3, self.np):
            raise ValueError(f"positions: need contiguous {want} [3, {self.np}] on {self.device}")
        return t.data_ptr()

    def _vec(self, t, name):
        torch = self.torch
        if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous() \
                or tuple(t.shape) != (3, self.np):
            raise ValueError(f"{name}: need contiguous float32 [3, {self.np}] on {self.device}")
        return t.data_ptr()

    # -- calls
    def deposit(self, pos, delta_out=None):
        pm_deposit(self.ctx, self._pos(pos), self._mesh(delta_out, "delta_out"))

    def poisson(self, delta=None, phi_out=None):
        pm_poisson(self.ctx, self._mesh(delta, "delta"), self._mesh(phi_out, "phi_out"))

    def qpot(self, delta=None, q_out=None):
        pm_qpot(self.ctx, self._mesh(delta, "delta"), self._mesh(q_out, "q_out"))

    def force(self, pos, acc_out, a=1.0, phi=None, q=None):
        pm_force(self.ctx, self._mesh(phi, "phi"), self._mesh(q, "q"), self._pos(pos),
                 self._vec(acc_out, "acc_out"), a)

    def step(self, pos, vel, times, flags=0):
        if len(times) < 2 or any(not math.isfinite(float(t)) for t in times):
            raise ValueError("times: need at least two finite values")
        pm_step(self.ctx, self._pos(pos), self._vec(vel, "vel"), times, flags)

    def step_energies(self, pos, vel, times, energies, flags=0):
        """pm_step_energies; energies: float64 [len(times), 4] on the device
        (rows K, W, U, E per synchronised time)."""
        torch = self.torch
        if len(times) < 2 or any(not math.isfinite(float(t)) for t in times):
            raise ValueError("times: need at least two finite values")
        if energies.dtype != torch.float64 or energies.device != self.device \
                or not energies.is_contiguous() or tuple(energies.shape) != (len(times), 4):
            raise ValueError(f"energies: need contiguous float64 [{len(times)}, 4] on "
                             f"{self.device}")
        pm_step_energies(self.ctx, self._pos(pos), self._vec(vel, "vel"), times, flags,
                         energies.data_ptr())

    def sort(self, pos, vel, ids=None):
        torch = self.torch
        ip = None
        if ids is not None:
            if ids.dtype != torch.int32 or ids.device != self.device or not ids.is_contiguous() \
                    or tuple(ids.shape) != (self.np,):
                raise ValueError(f"ids: need contiguous int32 [{self.np}] on {self.device}")
            ip = ids.data_ptr()
        pm_sort(self.ctx, self._pos(pos), self._vec(vel, "vel"), ip)

    def energy(self, pos, vel, a=1.0):
        return pm_energy(self.ctx, self._pos(pos), self._vec(vel, "vel"), a)

    def kinetic_split(self, pos, vel, a=1.0):
        return pm_kinetic_split(self.ctx, self._pos(pos), self._vec(vel, "vel"), a)

    def density_rms_diff(self, pos_a, pos_b):
        return pm_density_rms_diff(self.ctx, self._pos(pos_a), self._pos(pos_b))

    def power_spectrum(self, pos, nbins=None):
        return pm_power_spectrum(self.ctx, self._pos(pos), self.n // 2 if nbins is None else nbins)

    def spline_density(self, pos, delta_out, h=3.5):
        pm_spline_density(self.ctx, self._pos(pos), h, self._mesh(delta_out, "delta_out"))

    def spline_qforce(self, pos, q, acc_out, h=3.5):
        pm_spline_qforce(self.ctx, self._pos(pos), self._mesh(q, "q"), h,
                         self._vec(acc_out, "acc_out"))

    def spline_step(self, pos, vel, times, h=3.5):
        if len(times) < 2 or any(not math.isfinite(float(t)) for t in times):
            raise ValueError("times: need at least two finite values")
        pm_spline_step(self.ctx, self._pos(pos), self._vec(vel, "vel"), times, h)

    def spline_energy(self, pos, vel, a=1.0, h=3.5):
        return pm_spline_energy(self.ctx, self._pos(pos), self._vec(vel, "vel"), h, a)

    def timing(self, on: bool):
        pm_timing_enable(self.ctx, on)

    def timing_read(self) -> dict:
        return pm_timing_read(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            pm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ batched runs

def pm_batch_workspace_bytes(params: PMParams, slots: int) -> int:
    n = c_size_t(0)
    _check(load_library().pm_batch_workspace_bytes(byref(params), int(slots), byref(n)),
           "pm_batch_workspace_bytes")
    return n.value


def pm_batch_init(params: PMParams, slots: int, workspace_ptr: int, nbytes: int,
                  stream_ptr: int) -> int:
    out = c_void_p(None)
    _check(load_library().pm_batch_init(byref(params), int(slots), c_void_p(workspace_ptr), nbytes,
                                        c_void_p(stream_ptr), byref(out)), "pm_batch_init")
    return out.value


def pm_batch_slot_offset(batch: int, slot: int) -> int:
    n = c_size_t(0)
    _check(load_library().pm_batch_slot_offset(c_void_p(batch), int(slot), byref(n)),
           "pm_batch_slot_offset")
    return n.value


def pm_batch_set_slot(batch: int, slot: int, box: float, hbar_over_m: float) -> None:
    sp = PMSlotParams(float(box), float(hbar_over_m))
    _check(load_library().pm_batch_set_slot(c_void_p(batch), int(slot), byref(sp)),
           "pm_batch_set_slot")


def pm_batch_step(batch: int, pos_ptr: int, vel_ptr: int, slots, times, flags: int = 0) -> None:
    """slots: list of slot indices; times: one schedule (nsteps + 1 values) per slot."""
    ns = len(slots)
    nsteps = len(times[0]) - 1
    if any(len(t) != nsteps + 1 for t in times) or len(times) != ns:
        raise ValueError("times: one schedule of equal length per listed slot")
    sl = (c_int32 * ns)(*[int(s) for s in slots])
    flat = [float(v) for t in times for v in t]
    tt = (c_double * len(flat))(*flat)
    _check(load_library().pm_batch_step(c_void_p(batch), c_void_p(pos_ptr), c_void_p(vel_ptr),
                                        ns, sl, tt, nsteps, int(flags)), "pm_batch_step")


def pm_batch_destroy(batch: int) -> None:
    _check(load_library().pm_batch_destroy(c_void_p(batch)), "pm_batch_destroy")


class PMBatch:
    """Independent runs of one mesh size stepped together (torch-owned memory).

    Owns the workspace and the particle arrays pos [slots, 3, Np] and
    vel [slots, 3, Np]; load() copies a run into a slot, fetch() returns
    copies of a slot's state.
    """

    def __init__(self, params: PMParams, slots: int, device=None, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device if device is not None else "cuda:0")
        self.params = params
        self.slots = int(slots)
        self.n = params.n_mesh
        self.np = params.n_part
        self.fixed = params.precision == PM_FIXED32
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nbytes = pm_batch_workspace_bytes(params, slots)
        pdt = torch.int32 if self.fixed else torch.float32
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.pos = torch.zeros((self.slots, 3, self.np), dtype=pdt, device=self.device)
            self.vel = torch.zeros((self.slots, 3, self.np), dtype=torch.float32,
                                   device=self.device)
            self.batch = pm_batch_init(params, slots, self.workspace.data_ptr(), self.nbytes,
                                       self.stream.cuda_stream)

    def load(self, slot: int, pos, vel, box: float, hbar_over_m: float):
        """Copy a run's state (tensors [3, Np], any device) into a slot, on the batch stream."""
        torch = self.torch
        want = torch.int32 if self.fixed else torch.float32
        if tuple(pos.shape) != (3, self.np) or tuple(vel.shape) != (3, self.np) \
                or pos.dtype != want or vel.dtype != torch.float32:
            raise ValueError(f"load: need pos {want} and vel float32 of shape [3, {self.np}]")
        with torch.cuda.stream(self.stream):
            self.pos[slot].copy_(pos, non_blocking=True)
            self.vel[slot].copy_(vel, non_blocking=True)
        pm_batch_set_slot(self.batch, slot, box, hbar_over_m)

    def step(self, slots, times, flags: int = 0):
        pm_batch_step(self.batch, self.pos.data_ptr(), self.vel.data_ptr(), slots, times, flags)

    def mass_mesh(self, slot: int):
        off = pm_batch_slot_offset(self.batch, slot)
        n3 = self.n ** 3
        return self.workspace[off: off + 8 * n3].view(self.torch.int64)

    def close(self):
        if getattr(self, "batch", None):
            pm_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
