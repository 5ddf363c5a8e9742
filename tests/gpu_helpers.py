"""Shared helpers of the GPU parity tests (import only inside GPU tests)."""

import math

import numpy as np

import oracle
from synth import comoving_code_params, from_fixed

TWO40 = float(2 ** 40)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def periodic_diff(a, b, n):
    return (np.asarray(a) - np.asarray(b) + n / 2) % n - n / 2


def to_device(st, device, fp32_positions=False):
    import torch
    if fp32_positions:
        pos = torch.from_numpy(st.pos_f32.copy()).to(device)
    else:
        pos = torch.from_numpy(st.pos_fixed.view(np.int32).copy()).to(device)
    vel = torch.from_numpy(st.vel32.copy()).to(device)
    return pos, vel


def positions_cells(pos_t, n, fp32_positions=False):
    """(Np, 3) float64 cells from a device position tensor."""
    a = pos_t.cpu().numpy()
    if fp32_positions:
        return a.T.astype(np.float64)
    return from_fixed(a.view(np.uint32), n)


def mass_mesh(ctx):
    """The deposited int64 mass mesh (first 8 N^3 workspace bytes)."""
    import torch
    n = ctx.n
    return ctx.workspace[: 8 * n ** 3].view(torch.int64).cpu().numpy().reshape(n, n, n)


def cosmo_setup(n, box_mpch, m_ev, h=0.7, om=0.3, precision=1, rho_fp64_below=1e-3):
    """(library params, oracle params) of a comoving box in cell units."""
    from paper_1608_00802_amd import make_params
    hm = comoving_code_params(box_mpch, n, m_ev, h)["hbar_m_cells"] if m_ev else 0.0
    lp = make_params(n, n ** 3, float(n), precision=precision, comoving=True, omega_m=om,
                     omega_l=1 - om, h0=1.0, hbar_over_m=hm, rho_floor=1e-6,
                     rho_fp64_below=rho_fp64_below)
    op = oracle.Params(n=n, box=float(n), S=1.5 * om, hbar_m=hm, comoving=True, omega_m=om,
                       omega_l=1 - om, h0=1.0, rho_floor=1e-6)
    return lp, op


def single_mode_setup(precision=1):
    """Static box of the single-mode test: L = 1, 4 pi G rho = 1, hbar/m at
    half the quantum Jeans wavenumber of mode 2 (Eq. (19))."""
    from paper_1608_00802_amd import make_params
    n = 32
    hm_box = 1.0 / (32 * math.pi ** 2)
    lp = make_params(n, n ** 3, 1.0, precision=precision, comoving=False, four_pi_G_rhobar=1.0,
                     hbar_over_m=hm_box, rho_floor=1e-6, rho_fp64_below=1e-3)
    op = oracle.Params(n=n, box=float(n), S=1.0, hbar_m=hm_box * n * n, rho_floor=1e-6)
    return lp, op
