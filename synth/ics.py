"""Synthetic particle states in mesh-cell coordinates.

Conventions shared by every consumer:

* positions are in cells, u in [0, n_mesh); the fixed-point form stores
  u * 2^32 / n_mesh as uint32, structure-of-arrays [3][Np];
* velocities are in cells per unit time (static box) or canonical momentum
  a^2 du/dt in cells * H0 (comoving box, time unit 1/H0), float32 [3][Np];
* particles are in lattice order (ix, iy, iz), iz fastest, Lagrangian
  positions at cell centres u = i + 1/2 when n_side == n_mesh;
* the float64 views (``pos``, ``vel``) are the exact values of the quantised
  arrays, so every consumer starts from bit-identical states.

Zel'dovich initial conditions follow Sec. III of the paper (initial
conditions in the Zel'dovich approximation, CDM transfer function of
Eisenstein & Hu 1998, FDM transfer function of Hu, Barkana & Gruzinov 2000),
generated here instead of with the external code the paper used.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import integrate

TWO32 = 4294967296.0

# physical constants for the hbar/m conversion
HBAR_EV_S = 6.582119569e-16
C_KM_S = 299792.458
MPC_KM = 3.0856775814913673e19
T_CMB = 2.7255


@dataclasses.dataclass
class State:
    n_mesh: int
    pos_fixed: np.ndarray   # uint32 [3, Np]
    vel32: np.ndarray       # float32 [3, Np]
    meta: dict

    @property
    def npart(self) -> int:
        return self.pos_fixed.shape[1]

    @property
    def pos(self) -> np.ndarray:
        """float64 (Np, 3) cells, exact dequantisation of ``pos_fixed``."""
        return from_fixed(self.pos_fixed, self.n_mesh)

    @property
    def pos_f32(self) -> np.ndarray:
        """float32 [3, Np] cells (input of the plain FP32 form)."""
        p = from_fixed(self.pos_fixed, self.n_mesh).T.astype(np.float32)
        p[p >= np.float32(self.n_mesh)] = 0.0
        return np.ascontiguousarray(p)

    @property
    def vel(self) -> np.ndarray:
        """float64 (Np, 3), exact widening of ``vel32``."""
        return self.vel32.T.astype(np.float64)


# ---------------------------------------------------------------- fixed point

def to_fixed(pos_cells, n_mesh: int) -> np.ndarray:
    """(Np, 3) float cells -> uint32 [3, Np]; round to nearest, wrap mod 2^32."""
    u = np.asarray(pos_cells, dtype=np.float64) * (TWO32 / n_mesh)
    q = np.rint(u).astype(np.int64) % (1 << 32)
    return np.ascontiguousarray(q.T.astype(np.uint32))


def from_fixed(pos_fixed, n_mesh: int) -> np.ndarray:
    """uint32 [3, Np] -> (Np, 3) float64 cells (exact)."""
    return (np.asarray(pos_fixed, dtype=np.float64) * (n_mesh / TWO32)).T.copy()


def quantize_state(pos_cells, vel, n_mesh: int, meta: dict) -> State:
    vel32 = np.ascontiguousarray(np.asarray(vel, dtype=np.float64).T.astype(np.float32))
    return State(n_mesh, to_fixed(pos_cells, n_mesh), vel32, meta)


# ---------------------------------------------------------------- lattices

def lattice_cells(n_side: int, n_mesh: int, offset: float = 0.5) -> np.ndarray:
    """Cubic lattice of n_side^3 particles at (i + offset) * n_mesh / n_side."""
    g = (np.arange(n_side, dtype=np.float64) + offset) * (n_mesh / n_side)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def sine_mode_state(n: int = 32, mode: int = 2, amp_cells: float = 1e-3,
                    axis: int = 0) -> State:
    """Half-offset lattice displaced by amp * sin(2 pi mode (i + 1/2) / n)
    along one axis, at rest (single-mode linear test of a static box)."""
    q = lattice_cells(n, n)
    pos = q.copy()
    pos[:, axis] += amp_cells * np.sin(2.0 * np.pi * mode * q[:, axis] / n)
    pos %= n
    vel = np.zeros_like(pos)
    return quantize_state(pos, vel, n, {"kind": "sine", "n": n, "mode": mode,
                                        "amp_cells": amp_cells, "axis": axis})


# ---------------------------------------------------------------- cosmology inputs

def hbar_over_m_mpc_kms(m_ev: float) -> float:
    """hbar/m in Mpc km/s for a boson mass m in eV/c^2."""
    return HBAR_EV_S * C_KM_S ** 2 / m_ev / MPC_KM


def comoving_code_params(box_mpch: float, n_mesh: int, m_ev: float, h: float):
    """Cell-unit constants of a comoving box (length: cell, time: 1/H0).

    Returns dict with hbar_m (cells^2 H0) and dx (Mpc/h per cell).
    1 (Mpc/h)^2 H0 = 100/h Mpc km/s.
    """
    dx = box_mpch / n_mesh
    hm_mpch2_h0 = hbar_over_m_mpc_kms(m_ev) * h / 100.0
    return {"dx_mpch": dx, "hbar_m_cells": hm_mpch2_h0 / dx ** 2}


def _e_of_a(a, om, ol):
    return np.sqrt(om / a ** 3 + ol)


def growth_factor(a: float, om: float, ol: float) -> float:
    """Linear growth D(a) = 5/2 Om E(a) int_0^a da'/(a' E(a'))^3 (flat)."""
    val = integrate.quad(lambda x: (x * _e_of_a(x, om, ol)) ** -3, 0.0, a,
                         epsabs=0.0, epsrel=1e-12, limit=200)[0]
    return 2.5 * om * _e_of_a(a, om, ol) * val


def growth_rate(a: float, om: float, ol: float) -> float:
    """f = dlnD/dlna for the same D(a)."""
    e = _e_of_a(a, om, ol)
    val = integrate.quad(lambda x: (x * _e_of_a(x, om, ol)) ** -3, 0.0, a,
                         epsabs=0.0, epsrel=1e-12, limit=200)[0]
    return -1.5 * om / (a ** 3 * e * e) + 1.0 / (a * a * e ** 3 * val)


def transfer_cdm_eh98(k_hmpc, om: float, h: float) -> np.ndarray:
    """Eisenstein & Hu (1998) zero-baryon transfer function.

    The paper's cosmology has all matter in the axion field, so the baryon
    fraction is zero and the fitting formula reduces to
    T = L0/(L0 + C0 q^2), L0 = ln(2e + 1.8 q), C0 = 14.2 + 731/(1 + 62.5 q),
    q = k Theta^2 / (Om h^2), k in 1/Mpc, Theta = T_CMB/2.7 K.
    """
    k = np.asarray(k_hmpc, dtype=np.float64) * h
    theta = T_CMB / 2.7
    q = k * theta ** 2 / (om * h * h)
    l0 = np.log(2.0 * math.e + 1.8 * q)
    c0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
    return l0 / (l0 + c0 * q * q)


def transfer_fdm_hu2000(k_hmpc, m_ev: float, h: float) -> np.ndarray:
    """T(k) = cos(x^3)/(1 + x^8), x = 1.61 m22^(1/18) k / k_Jeq (Sec. III,
    Eq. (21)); k_Jeq = 9 m22^(1/2) / Mpc (Hu, Barkana & Gruzinov 2000; the
    paper does not print the value)."""
    m22 = m_ev / 1e-22
    k = np.asarray(k_hmpc, dtype=np.float64) * h
    kjeq = 9.0 * math.sqrt(m22)
    x = 1.61 * m22 ** (1.0 / 18.0) * k / kjeq
    return np.cos(x ** 3) / (1.0 + x ** 8)


def _power_shape(k_hmpc, om, h, m_ev, ns):
    t = transfer_cdm_eh98(k_hmpc, om, h)
    if m_ev is not None:
        t = t * transfer_fdm_hu2000(k_hmpc, m_ev, h)
    return np.asarray(k_hmpc, dtype=np.float64) ** ns * t * t


def _sigma_r(amp, r, om, h, m_ev, ns):
    def integrand(lnk):
        k = math.exp(lnk)
        x = k * r
        w = 3.0 * (math.sin(x) - x * math.cos(x)) / x ** 3 if x > 1e-4 else 1.0 - x * x / 10.0
        return k ** 3 * amp * float(_power_shape(k, om, h, m_ev, ns)) * w * w / (2.0 * math.pi ** 2)
    val = integrate.quad(integrand, math.log(1e-5), math.log(5e2), limit=400)[0]
    return math.sqrt(val)


def zeldovich_state(n: int, box_mpch: float, a_init: float, seed: int,
                    m_ev: float | None = 2.5e-22, om: float = 0.3, h: float = 0.7,
                    sigma8: float = 0.8, ns: float = 0.96, a_eval: float | None = None) -> State:
    """Zel'dovich initial conditions, n^3 particles on an n^3 mesh.

    Gaussian field with P(k) = A k^ns T_CDM^2 T_FDM^2 normalised to sigma_8 at
    a = 1, real-space white noise from numpy's default_rng(seed).  Displacement
    psi_k = i k delta_k / k^2 (Nyquist planes zeroed); x = q + D psi,
    p = a^2 E(a) f(a) D(a) psi in cells and cells*H0.  ``a_eval`` (default
    a_init) evaluates the same field at a later scale factor (a stand-in for
    an evolved, more clustered state).  m_ev None gives a pure CDM spectrum.
    """
    ol = 1.0 - om
    a = a_init if a_eval is None else a_eval
    amp = (sigma8 / _sigma_r(1.0, 8.0, om, h, m_ev, ns)) ** 2
    vol = box_mpch ** 3
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(white)
    del white
    kf = 2.0 * np.pi / box_mpch
    mfull = np.fft.fftfreq(n) * n
    mhalf = np.fft.rfftfreq(n) * n
    kx = (kf * mfull)[:, None, None]
    ky = (kf * mfull)[None, :, None]
    kz = (kf * mhalf)[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    pk = amp * _power_shape(np.sqrt(k2), om, h, m_ev, ns)
    pk[0, 0, 0] = 0.0
    dk = wk * np.sqrt(pk * n ** 3 / vol)
    del wk, pk
    nyq = n // 2
    growth = growth_factor(a, om, ol) / growth_factor(1.0, om, ol)
    fgrowth = growth_rate(a, om, ol)
    e = math.sqrt(om / a ** 3 + ol)
    dx = box_mpch / n
    q = lattice_cells(n, n)
    pos = np.empty_like(q)
    mom = np.empty_like(q)
    for d, kd in enumerate((kx, ky, kz)):
        psik = 1j * kd * dk / k2
        psik[0, 0, 0] = 0.0
        psik[nyq, :, :] = 0.0
        psik[:, nyq, :] = 0.0
        psik[:, :, nyq] = 0.0
        psi = np.fft.irfftn(psik, s=(n, n, n), axes=(0, 1, 2)).ravel() / dx   # cells, at a = 1
        del psik
        pos[:, d] = q[:, d] + growth * psi
        mom[:, d] = a * a * e * fgrowth * growth * psi
        del psi
    pos %= n
    meta = {"kind": "zeldovich", "n": n, "box_mpch": box_mpch, "a": a, "seed": seed,
            "m_ev": m_ev, "omega_m": om, "h": h, "sigma8": sigma8, "ns": ns}
    return quantize_state(pos, mom, n, meta)
