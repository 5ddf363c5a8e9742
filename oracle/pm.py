"""Plain FP64 NumPy particle-mesh step: the oracle.

TEST INFRASTRUCTURE ONLY -- imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Paper: Veltmaat & Niemeyer, arXiv:1608.00802.  Equation numbers follow the
order of the displayed equations in the paper:

  Eq. (4)  Euler equation, acceleration -grad(Q + V)        (Sec. II A)
  Eq. (5)  quantum pressure Q = -(hbar^2/2m^2) lap(sqrt rho)/sqrt rho
  Eq. (6)  K = K_v + K_rho
  Eq. (8)  discrete K_v = sum_i m_i qdot_i^2 / 2
  Eq. (9)  density from particles with an assignment kernel W
  Eq. (11) discrete K_rho with central differences on the mesh
  Eq. (14) equation of motion: quantum force by the kernel gradient
  Eq. (15) cubic spline smoothing kernel
  Eq. (16) scale symmetry                                     (Sec. II B)
  Eq. (17) bulk velocity field of the particles on the mesh   (Sec. II B)
  Eq. (18) comoving Q carries an extra 1/a^2                  (Sec. III)
  Sec. III  RMS relative FDM-CDM density difference per cell

Readings where the paper is silent or where the hot path departs from the
paper's own discretisation (all deliberate, all listed in the design notes):

  * assignment kernel: cloud-in-cell (trilinear) instead of the paper's SPH
    cubic spline, for both the deposit and the force interpolation;
  * force: central-difference gradient of (phi + Q) on the mesh, then CIC
    interpolation, instead of the paper's kernel-gradient convolution;
  * gravity: FFT Poisson solve with the Green's function of the compact
    7-point Laplacian, -1/K^2, K^2 = sum_d (2/dx)^2 sin^2(k_d dx/2); the
    k = 0 mode is zero; no window deconvolution;
  * Q: the compact 7-point Laplacian of sqrt(R), R = max(rho, floor), with
    the floor in units of the mean density;
  * mesh values live on nodes x_j = j*dx; a position equal to the box side
    wraps to 0;
  * comoving integrator: kick-drift-kick in canonical momentum
    p = a^2 dx/dt with kick factors int da/(a^2 H) (gravity) and
    int da/(a^3 H) (quantum pressure and drift), half-kicks split at the
    geometric mid-point sqrt(a0 a1).

Units: any consistent set.  ``box`` is the side length, positions lie in
[0, box), densities are in units of the mean, ``S`` is 4 pi G rho_bar in a
static box and (3/2) Omega_m H0^2 in a comoving one, ``hbar_m`` is hbar/m in
length^2/time.  The particle mass is box^3/Np (mean density one), so all
three energies share one mass unit.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import integrate


@dataclasses.dataclass(frozen=True)
class Params:
    """Problem definition (Sec. II A and Sec. III)."""

    n: int                      # mesh cells per side
    box: float                  # side length L
    S: float                    # static: 4 pi G rho_bar; comoving: 1.5 Omega_m H0^2
    hbar_m: float               # hbar/m; 0 switches quantum pressure off (CDM)
    comoving: bool = False
    omega_m: float = 0.3
    omega_l: float = 0.7
    h0: float = 1.0             # H0 in inverse time units (comoving only)
    rho_floor: float = 1e-6     # floor on rho/rho_bar inside Q and U

    @property
    def dx(self) -> float:
        return self.box / self.n


# ---------------------------------------------------------------- deposit

def cic_index_weights(pos, p: Params):
    """Cell-in-cloud base index and fractional offset per particle.

    Mesh nodes sit at x_j = j*dx.  u = x/dx, i = floor(u), f = u - i; the
    particle touches nodes i and i+1 (mod n) along each axis with linear
    weights 1-f and f.  Returns (i as int64 in [0, n), f in [0, 1]).
    """
    u = np.asarray(pos, dtype=np.float64) / p.dx
    i = np.floor(u)
    f = u - i
    return i.astype(np.int64) % p.n, f


def _corners():
    for cx in (0, 1):
        for cy in (0, 1):
            for cz in (0, 1):
                yield cx, cy, cz


def _corner_weight(f, c):
    w = np.ones(f.shape[0])
    for d in range(3):
        w = w * (f[:, d] if c[d] else 1.0 - f[:, d])
    return w


def _corner_index(i, c, n):
    ix = (i[:, 0] + c[0]) % n
    iy = (i[:, 1] + c[1]) % n
    iz = (i[:, 2] + c[2]) % n
    return (ix * n + iy) * n + iz


def deposit(pos, p: Params) -> np.ndarray:
    """rho/rho_bar on the mesh, Eq. (9) with a cloud-in-cell kernel.

    Each particle carries mass box^3/Np; its mass is split over the 8
    surrounding nodes with trilinear weights, then divided by dx^3 and by the
    mean density.  Layout: C order [ix][iy][iz].
    """
    n = p.n
    npart = pos.shape[0]
    i, f = cic_index_weights(pos, p)
    rho = np.zeros(n ** 3)
    for c in _corners():
        rho += np.bincount(_corner_index(i, c, n), weights=_corner_weight(f, c),
                           minlength=n ** 3)
    return rho.reshape(n, n, n) * (n ** 3 / npart)


# ---------------------------------------------------------------- Poisson

def _mode_numbers(n):
    """Integer frequencies along a full axis and along the half (rfft) axis."""
    full = np.fft.fftfreq(n) * n
    half = np.fft.rfftfreq(n) * n
    return full, half


def green_discrete(p: Params) -> np.ndarray:
    """-S / K^2(k) on the rfft half-spectrum, with the k = 0 mode zero.

    K^2 = sum_d (2/dx)^2 sin^2(k_d dx / 2), k_d = 2 pi m_d / box: the symbol of
    the compact 7-point Laplacian, so the FFT solve equals a converged 7-point
    solve.  The paper reuses the gravity solver of its host code (Sec. II A)
    without naming it; this is the reading taken.
    """
    full, half = _mode_numbers(p.n)
    s2 = lambda m: (2.0 / p.dx) ** 2 * np.sin(np.pi * m / p.n) ** 2  # noqa: E731
    k2 = (s2(full)[:, None, None] + s2(full)[None, :, None]
          + s2(half)[None, None, :])
    g = np.zeros_like(k2)
    nz = k2 > 0
    g[nz] = -p.S / k2[nz]
    return g


def poisson(delta, p: Params) -> np.ndarray:
    """phi with lap(phi) = S * delta on the periodic mesh (Sec. II A)."""
    dk = np.fft.rfftn(delta)
    return np.fft.irfftn(dk * green_discrete(p), s=delta.shape, axes=(0, 1, 2))


# ---------------------------------------------------------------- Q

def qpot(rho, p: Params) -> np.ndarray:
    """Quantum pressure on the mesh, Eq. (5), static-box form.

    R = max(rho, floor); Q = -(hbar/m)^2/2 * L7[sqrt R] / (dx^2 sqrt R) with L7
    the compact 7-point stencil sum_{+-d} s_{j+-e_d} - 6 s_j (Sec. II A names
    the seven-point stencil).  The comoving Q of Eq. (18) is this divided by
    a^2; callers apply that factor.
    """
    s = np.sqrt(np.maximum(rho, p.rho_floor))
    lap = -6.0 * s
    for ax in range(3):
        lap = lap + np.roll(s, 1, axis=ax) + np.roll(s, -1, axis=ax)
    return -(p.hbar_m ** 2 / 2.0) * lap / (p.dx ** 2 * s)


# ---------------------------------------------------------------- force

def grad_central(field, p: Params) -> np.ndarray:
    """-grad(field) by 2-point central differences, shape (3, n, n, n).

    Central differences are the ones the paper uses for K_rho, Eq. (11).
    """
    out = np.empty((3,) + field.shape)
    for ax in range(3):
        out[ax] = -(np.roll(field, -1, axis=ax) - np.roll(field, 1, axis=ax)) / (2.0 * p.dx)
    return out


def interp_cic(vec_field, pos, p: Params) -> np.ndarray:
    """Interpolate a (3, n, n, n) mesh vector field to particles, (Np, 3).

    Same trilinear weights and nodes as :func:`deposit`.
    """
    n = p.n
    i, f = cic_index_weights(pos, p)
    flat = vec_field.reshape(3, -1)
    out = np.zeros((pos.shape[0], 3))
    for c in _corners():
        idx = _corner_index(i, c, n)
        w = _corner_weight(f, c)
        out += w[:, None] * flat[:, idx].T
    return out


def fields(pos, p: Params):
    """rho, delta, phi and Q_c on the mesh for one particle state.

    Principal steps (i) and (ii) of Sec. II A plus the gravity solve on the
    same density.
    """
    rho = deposit(pos, p)
    delta = rho - 1.0
    phi = poisson(delta, p)
    q = qpot(rho, p) if p.hbar_m != 0.0 else np.zeros_like(rho)
    return rho, delta, phi, q


def forces(pos, p: Params):
    """(g_phi, g_Q): -grad(phi) and -grad(Q_c) interpolated to the particles.

    Step (iii) of Sec. II A in the mesh-gradient form; Euler equation Eq. (4)
    fixes the sign (acceleration is minus the gradient of Q + V).
    """
    _, _, phi, q = fields(pos, p)
    g_phi = interp_cic(grad_central(phi, p), pos, p)
    g_q = interp_cic(grad_central(q, p), pos, p) if p.hbar_m != 0.0 else np.zeros_like(g_phi)
    return g_phi, g_q


# ---------------------------------------------------------------- time integration

def hubble(a, p: Params) -> float:
    """H(a) = H0 sqrt(Omega_m a^-3 + Omega_L) (flat background, Sec. III)."""
    return p.h0 * math.sqrt(p.omega_m / a ** 3 + p.omega_l)


def kick_factors(a0, a1, p: Params):
    """(F_g, F_q) = (int da/(a^2 H), int da/(a^3 H)) from a0 to a1.

    Canonical momentum p = a^2 dx/dt obeys dp/dt = -grad(phi_c)/a -
    grad(Q_c)/a^2 (Eq. (18) gives the 1/a^2 of Q); with dt = da/(aH) the two
    terms integrate to these factors.  Adaptive quadrature in FP64.
    """
    fg = integrate.quad(lambda a: 1.0 / (a * a * hubble(a, p)), a0, a1,
                        epsabs=0.0, epsrel=1e-13, limit=200)[0]
    fq = integrate.quad(lambda a: 1.0 / (a ** 3 * hubble(a, p)), a0, a1,
                        epsabs=0.0, epsrel=1e-13, limit=200)[0]
    return fg, fq


def drift_factor(a0, a1, p: Params) -> float:
    """int da/(a^3 H): dx = p dt / a^2 with dt = da/(aH)."""
    return integrate.quad(lambda a: 1.0 / (a ** 3 * hubble(a, p)), a0, a1,
                          epsabs=0.0, epsrel=1e-13, limit=200)[0]


def step_factors(t0, t1, p: Params):
    """((F_g, F_q) first half-kick, F_drift, (F_g, F_q) second half-kick).

    Static box: time t, both half-kicks dt/2, drift dt.  Comoving: scale
    factor a, halves split at a_m = sqrt(a0 a1).
    """
    if not p.comoving:
        dt = t1 - t0
        return (0.5 * dt, 0.5 * dt), dt, (0.5 * dt, 0.5 * dt)
    am = math.sqrt(t0 * t1)
    return kick_factors(t0, am, p), drift_factor(t0, t1, p), kick_factors(am, t1, p)


def _wrap(x, box):
    x = np.mod(x, box)
    return np.where(x >= box, x - box, x)


def kdk_step(pos, vel, p: Params, t0, t1, acc0=None):
    """One kick-drift-kick leapfrog step (Sec. II A, leapfrog with the added
    quantum-pressure force).

    pos: (Np, 3) in [0, box); vel: (Np, 3) velocity (static) or canonical
    momentum a^2 dx/dt (comoving).  ``acc0`` may carry (g_phi, g_Q) at pos.
    Returns (pos1, vel1, acc1) with acc1 = (g_phi, g_Q) at pos1.
    """
    (fg0, fq0), fd, (fg1, fq1) = step_factors(t0, t1, p)
    g_phi, g_q = forces(pos, p) if acc0 is None else acc0
    v = vel + g_phi * fg0 + g_q * fq0
    x = _wrap(pos + v * fd, p.box)
    g_phi, g_q = forces(x, p)
    v = v + g_phi * fg1 + g_q * fq1
    return x, v, (g_phi, g_q)


def run(pos, vel, p: Params, times):
    """Advance through the schedule ``times`` (len = steps + 1)."""
    acc = None
    x, v = pos, vel
    for t0, t1 in zip(times[:-1], times[1:]):
        x, v, acc = kdk_step(x, v, p, t0, t1, acc)
    return x, v


# ---------------------------------------------------------------- energies

def energies(pos, vel, p: Params, a: float = 1.0) -> dict:
    """K, W, U and E at a synchronised state.

    K: Eq. (8) with canonical momentum, sum m p^2 / (2 a^2).
    W: 1/(2a) sum_j delta_j phi_j dx^3 (mean density one).
    U: gradient energy K_rho of Eq. (6); 'U' uses forward differences (the
       exact conjugate of the compact Laplacian used for Q) and 'U_central'
       the central differences of Eq. (11); both carry 1/a^2 from Eq. (18).
    """
    npart = pos.shape[0]
    mp = p.box ** 3 / npart
    rho, delta, phi, _ = fields(pos, p)
    kin = 0.5 * mp * float(np.sum(vel * vel)) / a ** 2
    wg = 0.5 * float(np.sum(delta * phi)) * p.dx ** 3 / a
    u_f, u_c = gradient_energy(rho, p, a)
    return {"K": kin, "W": wg, "U": u_f, "U_central": u_c, "E": kin + wg + u_f}


def gradient_energy(rho, p: Params, a: float = 1.0):
    """(forward, central) discretisations of K_rho, Eq. (6), on the mesh
    density rho (units of the mean), with the 1/a^2 of Eq. (18).

    central: Eq. (11) as printed, (hbar^2/2m^2) (dx/4) sum_j sum_d
    (s_{j+e_d} - s_{j-e_d})^2; forward: (hbar^2/2m^2) dx sum_j sum_d
    (s_{j+e_d} - s_j)^2, whose variation with respect to rho_j is the
    7-point Q.  s = sqrt(max(rho, floor)); the volume element dx^3 and the
    1/dx^2 of the squared difference quotient leave one power of dx.
    """
    s = np.sqrt(np.maximum(rho, p.rho_floor))
    fwd = 0.0
    cen = 0.0
    for ax in range(3):
        fwd += float(np.sum((np.roll(s, -1, axis=ax) - s) ** 2))
        cen += float(np.sum((np.roll(s, -1, axis=ax) - np.roll(s, 1, axis=ax)) ** 2))
    pref = p.hbar_m ** 2 / 2.0 / a ** 2
    return pref * p.dx * fwd, pref * (p.dx / 4.0) * cen


def layzer_irvine_error(a_values, series):
    """Layzer-Irvine residual |E(a) - E(a0) + int (2K + W + 2U) da/a| / |W(a)|.

    From the Hamiltonian sum p^2/(2 m a^2) + W_c/a + U_c/a^2: dE/da =
    -(2K + W + 2U)/a.  Trapezoid rule over the recorded states.  Returns the
    array of residuals, one per recorded a.
    """
    a = np.asarray(a_values, dtype=np.float64)
    k = np.array([e["K"] for e in series])
    w = np.array([e["W"] for e in series])
    u = np.array([e["U"] for e in series])
    e = k + w + u
    rate = (2.0 * k + w + 2.0 * u) / a
    integral = np.concatenate([[0.0], np.cumsum(0.5 * (rate[1:] + rate[:-1]) * np.diff(a))])
    return np.abs(e - e[0] + integral) / np.abs(w)


# ---------------------------------------------------------------- time-step rule

def omega_max(p: Params, a: float = 1.0) -> float:
    """Largest linear quantum-pressure frequency on the mesh (G = 0).

    Linearising the discrete scheme around a uniform lattice gives, per mode,
    omega = 2 (hbar/m)/(a^2 dx^2) * prod_d cos(theta_d) * sum_d sin^2(theta_d),
    theta_d = k_d dx/2; its maximum over the Brillouin zone is found here by
    a dense scan of the symmetric diagonal theta_x = theta_y = theta_z.
    """
    th = np.linspace(0.0, np.pi / 2, 200001)
    f = np.cos(th) ** 3 * 3.0 * np.sin(th) ** 2
    return 2.0 * p.hbar_m / (a * a * p.dx * p.dx) * float(f.max())


def timestep(p: Params, t_or_a: float, vmax: float, c_x: float = 0.5,
             c_q: float = 0.5, dlna_max: float = math.log(100.0) / 500.0):
    """Next step size: no particle moves more than c_x * dx (Sec. II A, the
    modified time-step condition) and omega_max * dt <= c_q.

    Static box: returns dt.  Comoving: returns the next scale factor a1,
    additionally capping d ln a at ``dlna_max``.
    """
    if not p.comoving:
        dt = np.inf
        if vmax > 0:
            dt = c_x * p.dx / vmax
        if p.hbar_m > 0:
            dt = min(dt, c_q / omega_max(p))
        return dt
    a = t_or_a
    h = hubble(a, p)
    dlna = dlna_max
    if vmax > 0:  # dx/dt = p/a^2, dt = dlna / H
        dlna = min(dlna, c_x * p.dx * a * a / vmax * h)
    if p.hbar_m > 0:
        dlna = min(dlna, c_q / omega_max(p, a) * h)
    return a * math.exp(dlna)


# ---------------------------------------------------------------- diagnostics

def power_spectrum(delta, box: float, nbins: int | None = None):
    """Shell-averaged P(k) = <|delta_k|^2> V / n^6 in bins of |m| (integer
    mode number, bin width 1, shells m in [b-0.5, b+0.5)).  Used only to
    report errors, never on the step path.  Returns (k, P, counts).
    """
    n = delta.shape[0]
    dk = np.fft.rfftn(delta)
    full, half = _mode_numbers(n)
    mm = np.sqrt(full[:, None, None] ** 2 + full[None, :, None] ** 2 + half[None, None, :] ** 2)
    # modes with 0 < m_z < n/2 stand for two complex-conjugate modes
    wgt = np.full(mm.shape, 2.0)
    wgt[:, :, 0] = 1.0
    if n % 2 == 0:
        wgt[:, :, -1] = 1.0
    power = np.abs(dk) ** 2 * box ** 3 / float(n) ** 6
    b = np.floor(mm + 0.5).astype(np.int64)
    nb = nbins if nbins is not None else n // 2
    keep = (b >= 1) & (b <= nb)
    cnt = np.bincount(b[keep], weights=wgt[keep], minlength=nb + 1)[1:]
    tot = np.bincount(b[keep], weights=(wgt * power)[keep], minlength=nb + 1)[1:]
    with np.errstate(invalid="ignore", divide="ignore"):
        pk = tot / cnt
    k = 2.0 * np.pi * np.arange(1, nb + 1) / box
    return k, pk, cnt


def kinetic_split(pos, vel, p: Params, a: float = 1.0) -> dict:
    """K_v split into grid-scale bulk motion and velocity dispersion.

    Sec. II B, Eq. (17): the bulk velocity field on the mesh is the
    kernel-weighted, mass-weighted mean of the particle velocities,
    v(x) = sum_i m qdot_i W(x - q_i) / rho(x), with the deposit's kernel W
    (cloud-in-cell here).  Its kinetic energy on the mesh is
    K_bulk = sum_x rho(x) |v(x)|^2 dx^3 / 2, with the 1/a^2 of canonical
    momentum as in K; nodes without mass hold no velocity and add nothing.
    The rest of Eq. (8)'s K is the velocity dispersion: K_disp = K - K_bulk.
    With node sums M(x) = rho(x) dx^3 and P(x) = sum_i m W_i(x) p_i this is
    K_bulk = sum_x |P(x)|^2 / (2 M(x) a^2).
    """
    n = p.n
    npart = pos.shape[0]
    mp = p.box ** 3 / npart
    i, f = cic_index_weights(pos, p)
    mass = np.zeros(n ** 3)
    mom = np.zeros((3, n ** 3))
    for c in _corners():
        idx = _corner_index(i, c, n)
        w = _corner_weight(f, c)
        mass += np.bincount(idx, weights=mp * w, minlength=n ** 3)
        for d in range(3):
            mom[d] += np.bincount(idx, weights=mp * w * vel[:, d], minlength=n ** 3)
    has = mass > 0.0
    bulk = 0.5 * float(np.sum(np.sum(mom[:, has] ** 2, axis=0) / mass[has])) / a ** 2
    kin = 0.5 * mp * float(np.sum(vel * vel)) / a ** 2
    return {"K": kin, "K_bulk": bulk, "K_disp": kin - bulk}


def density_rms_diff(pos_a, pos_b, p: Params):
    """RMS over mesh nodes of the relative density difference
    (rho_a - rho_b) / rho_b of two particle states on the same mesh.

    Sec. III compares the FDM run (a) with the CDM run (b) from the same
    initial conditions by this number per numerical cell.  Reading: nodes
    where rho_b is zero have no relative difference and are left out.
    Returns (rms, number of nodes used); no node gives (0, 0).
    """
    ra = deposit(pos_a, p).ravel()
    rb = deposit(pos_b, p).ravel()
    keep = rb > 0.0
    cnt = int(np.count_nonzero(keep))
    if cnt == 0:
        return 0.0, 0
    rel = (ra[keep] - rb[keep]) / rb[keep]
    return math.sqrt(float(np.mean(rel * rel))), cnt


# ---------------------------------------------------------------- spline kernel (the paper's own)

def spline_w(r, h):
    """Eq. (15): the cubic spline smoothing kernel of support h,
    W = 8/(pi h^3) [1 - 6 q^2 + 6 q^3] for q = r/h <= 1/2, 8/(pi h^3) 2 (1 - q)^3
    for 1/2 < q <= 1, zero beyond."""
    q = np.asarray(r, dtype=np.float64) / h
    c = 8.0 / (math.pi * h ** 3)
    inner = 1.0 - 6.0 * q ** 2 + 6.0 * q ** 3
    outer = 2.0 * (1.0 - q) ** 3
    return c * np.where(q <= 0.5, inner, np.where(q <= 1.0, outer, 0.0))


def spline_dw(r, h):
    """dW/dr of Eq. (15)."""
    q = np.asarray(r, dtype=np.float64) / h
    c = 8.0 / (math.pi * h ** 3) / h
    inner = -12.0 * q + 18.0 * q ** 2
    outer = -6.0 * (1.0 - q) ** 2
    return c * np.where(q <= 0.5, inner, np.where(q <= 1.0, outer, 0.0))


def _spline_offsets(h_cells):
    m = int(math.ceil(h_cells)) + 1
    return range(-m, m + 1)


def spline_deposit(pos, p: Params, h: float) -> np.ndarray:
    """rho/rho_bar on the mesh nodes from Eq. (9) with the kernel of Eq. (15):
    rho(x_j) = sum_i m W(|x_j - q_i|, h), m = box^3/Np.  Every node within h of
    a particle is visited (a cube of offsets around its cell)."""
    n = p.n
    npart = pos.shape[0]
    dx = p.dx
    u = np.asarray(pos, dtype=np.float64) / dx
    base = np.floor(u).astype(np.int64)
    rho = np.zeros(n ** 3)
    mp = p.box ** 3 / npart
    offs = list(_spline_offsets(h / dx))
    for ox in offs:
        for oy in offs:
            for oz in offs:
                node = base + np.array([ox, oy, oz])
                r = np.sqrt(np.sum(((node - u) * dx) ** 2, axis=1))
                w = spline_w(r, h)
                idx = ((node[:, 0] % n) * n + node[:, 1] % n) * n + node[:, 2] % n
                rho += np.bincount(idx, weights=mp * w, minlength=n ** 3)
    return rho.reshape(n, n, n)          # mean density is one: rho/rho_bar


def spline_qforce(pos, q, p: Params, h: float) -> np.ndarray:
    """Acceleration from the quantum potential on the nodes by the kernel
    gradient, Eq. (14): a_i = dx^3 sum_j Q_j grad W(x_j - q_i), the sign taken
    so that a = -grad Q (reading R3); it is minus the q_i-derivative of the
    mesh energy whose node variation is Q (see spline_kinetic_rho)."""
    n = p.n
    dx = p.dx
    u = np.asarray(pos, dtype=np.float64) / dx
    base = np.floor(u).astype(np.int64)
    qf = np.asarray(q, dtype=np.float64).ravel()
    acc = np.zeros((pos.shape[0], 3))
    offs = list(_spline_offsets(h / dx))
    for ox in offs:
        for oy in offs:
            for oz in offs:
                node = base + np.array([ox, oy, oz])
                d = (node - u) * dx
                r = np.sqrt(np.sum(d ** 2, axis=1))
                g = np.where(r > 0.0, spline_dw(r, h) / np.where(r > 0.0, r, 1.0), 0.0)
                idx = ((node[:, 0] % n) * n + node[:, 1] % n) * n + node[:, 2] % n
                acc += (qf[idx] * g)[:, None] * d
    return acc * dx ** 3


def spline_kinetic_rho(pos, p: Params, h: float) -> float:
    """K_rho of Eq. (11) on the spline density per unit mass density
    (rho in units of the mean), with forward differences, the exact
    conjugate of the 7-point Laplacian in Q; no floor (rho > 0 assumed)."""
    s = np.sqrt(spline_deposit(pos, p, h))
    tot = 0.0
    for ax in range(3):
        tot += float(np.sum((np.roll(s, -1, axis=ax) - s) ** 2))
    return p.hbar_m ** 2 / 2.0 * p.dx * tot


def spline_forces(pos, p: Params, h: float):
    """(g_phi, g_Q) with the paper's own coupling (Sec. II A): the density of
    Eq. (9) with the spline of Eq. (15) feeds both the gravity solve and Q;
    gravity is -grad(phi) interpolated by cloud-in-cell (the host code's PM
    interpolation), the quantum force is the kernel gradient of Eq. (14)."""
    rho = spline_deposit(pos, p, h)
    phi = poisson(rho - 1.0, p)
    g_phi = interp_cic(grad_central(phi, p), pos, p)
    if p.hbar_m != 0.0:
        g_q = spline_qforce(pos, qpot(rho, p), p, h)
    else:
        g_q = np.zeros_like(g_phi)
    return g_phi, g_q


def spline_run(pos, vel, p: Params, times, h: float):
    """kdk_step's leapfrog with spline_forces, through the schedule ``times``."""
    x, v = pos, vel
    acc = spline_forces(x, p, h)
    for t0, t1 in zip(times[:-1], times[1:]):
        (fg0, fq0), fd, (fg1, fq1) = step_factors(t0, t1, p)
        v = v + acc[0] * fg0 + acc[1] * fq0
        x = _wrap(x + v * fd, p.box)
        acc = spline_forces(x, p, h)
        v = v + acc[0] * fg1 + acc[1] * fq1
    return x, v


def spline_energies(pos, vel, p: Params, h: float, a: float = 1.0) -> dict:
    """energies() with the density of Eq. (9) and the spline of Eq. (15):
    K of Eq. (8), W = 1/(2a) sum delta phi dx^3, and U the forward-difference
    K_rho of Eq. (11) of sqrt(max(rho, floor)) with the 1/a^2 of Eq. (18)."""
    npart = pos.shape[0]
    mp = p.box ** 3 / npart
    rho = spline_deposit(pos, p, h)
    delta = rho - 1.0
    phi = poisson(delta, p)
    kin = 0.5 * mp * float(np.sum(vel * vel)) / a ** 2
    wg = 0.5 * float(np.sum(delta * phi)) * p.dx ** 3 / a
    s = np.sqrt(np.maximum(rho, p.rho_floor))
    fwd = 0.0
    for ax in range(3):
        fwd += float(np.sum((np.roll(s, -1, axis=ax) - s) ** 2))
    u_f = p.hbar_m ** 2 / 2.0 / a ** 2 * p.dx * fwd
    return {"K": kin, "W": wg, "U": u_f, "E": kin + wg + u_f}
