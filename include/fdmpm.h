/*
 * fdmpm.h -- C ABI of the MI355X (gfx950) particle-mesh step for fuzzy dark
 * matter (Veltmaat & Niemeyer, arXiv:1608.00802).
 *
 * One step of the method: cloud-in-cell mass deposit of the particles on a
 * periodic mesh, FFT Poisson solve for the gravitational potential, the
 * quantum pressure Q = -(hbar^2/2m^2) lap(sqrt rho)/sqrt rho on the same mesh
 * (Sec. II A, Eq. (5); comoving form Sec. III, Eq. (18)), central-difference
 * gradients of both, CIC interpolation back to the particles, and a
 * kick-drift-kick leapfrog (static box, or comoving in canonical momentum).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units.  Particle coordinates and the mesh use CELL units: positions
 *   u in [0, N), the mesh spacing is 1.  Time is the caller's time unit
 *   (static box) or 1/H0 (comoving box).  Velocities are du/dt in cells per
 *   time unit (static) or canonical momentum p = a^2 du/dt in cells*H0
 *   (comoving).  Densities are in units of the mean.  ``box`` converts the
 *   caller's hbar/m (length^2/time) into cells^2/time.
 * Layout.  Meshes are C-order [ix][iy][iz] (iz fastest), N^3 contiguous
 *   float.  Particles are structure-of-arrays: positions [3][Np] (x block,
 *   then y block, then z block) and velocities / accelerations [3][Np] float.
 *   Fixed-point positions (PM_FIXED32) store u * 2^32 / N as uint32, so the
 *   periodic wrap is the natural wrap of 32-bit arithmetic; PM_FP32 positions
 *   store u as float in [0, N).
 * Memory ownership.  The caller owns every device buffer: the workspace
 *   passed to pm_init (size from pm_workspace_bytes, 256-byte aligned) and all
 *   particle and mesh arrays.  The library never allocates device memory;
 *   pm_destroy frees only the host-side context.
 * Workspace contents.  Bytes [0, 8 N^3) of the workspace hold the deposited
 *   mass mesh after pm_deposit, pm_step or pm_energy: int64 in units of 2^-40
 *   particle masses (PM_FIXED32; exactly 2^40 per particle in total) or float
 *   sums of CIC weights (PM_FP32, first 4 N^3 bytes); after pm_spline_density,
 *   pm_spline_step or pm_spline_energy, the int64 spline density in the same
 *   units (both precisions).  Everything else in the workspace is private.
 * Asynchrony.  All calls except pm_workspace_bytes, pm_energy,
 *   pm_kinetic_split, pm_density_rms_diff, pm_power_spectrum, pm_spline_energy
 *   and pm_destroy only enqueue work on the context's HIP stream and return.  Argument errors
 *   are reported synchronously; a kernel launch error is reported as
 *   PM_EDEVICE.  A context is bound to one stream and is not thread-safe;
 *   distinct contexts on distinct workspaces are independent.
 * Devices.  All device pointers must belong to the device that was current
 *   when pm_init was called; calls must be made with that device current.
 */
#ifndef FDMPM_H
#define FDMPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PM_OK = 0,
  PM_EINVAL = -1,        /* bad argument: null pointer, out-of-range value */
  PM_ENOMEM = -2,        /* workspace smaller than pm_workspace_bytes */
  PM_EDEVICE = -3,       /* a HIP runtime call or kernel launch failed */
  PM_EUNSUPPORTED = -4,  /* mesh size not a power of two in [16, 512] */
  PM_ESTATE = -5         /* call needs state that is not there yet */
} pm_status;

typedef enum {
  PM_FP32 = 0,     /* float positions, float atomics, direct sqrt(rho) for Q */
  PM_FIXED32 = 1   /* uint32 fixed-point positions, exact integer deposit,
                      FP32 FFT/stencils, FP64 for near-empty cells */
} pm_precision;

/* Problem definition (Sec. II A static box; Sec. III comoving box). */
typedef struct {
  int32_t n_mesh;            /* N: cells per side, power of two, 16..512 */
  int32_t precision;         /* pm_precision */
  int64_t n_part;            /* particle count (equal masses), >= 1; PM_FIXED32
                                needs n_part <= 8 N^3 (a cell then holds up to
                                2^20 times the mean mass) */
  double box;                /* side length L in the caller's length unit */
  int32_t comoving;          /* 0: static box (a == 1); 1: flat comoving box */
  int32_t reserved0;         /* must be 0 */
  double four_pi_G_rhobar;   /* static box: 4 pi G rho_bar (1/time^2) */
  double omega_m;            /* comoving: matter density parameter */
  double omega_l;            /* comoving: cosmological constant */
  double h0;                 /* comoving: H0 in 1/time (use 1 for time in 1/H0) */
  double hbar_over_m;        /* hbar/m in length^2/time; 0 disables quantum pressure */
  double rho_floor;          /* floor on rho/rho_bar inside Q, > 0 (1e-6 typical) */
  double rho_fp64_below;     /* PM_FIXED32: cells with rho/rho_bar below this
                                compute sqrt(rho) and Q in FP64 from the exact
                                integer mass; 0 disables (1e-3 typical) */
} pm_params;

/* Energies in cell units with the mean density as mass unit (mass per cell
 * 1, per particle N^3/Np):
 *   K = sum_p (N^3/Np) |p|^2 / (2 a^2)                    (Eq. (8))
 *   W = 1/(2a) sum_j delta_j phi_j                        (potential energy)
 *   U = (hbar/m)^2/(2 a^2) sum_j sum_d (s_{j+e_d} - s_j)^2, s = sqrt(max(rho, floor))
 *       (gradient energy K_rho of Eq. (6), forward differences)
 *   E = K + W + U.  Multiply by rho_bar dx^5/time^2 for physical units. */
typedef struct {
  double K, W, U, E;
} pm_energies;

typedef struct pm_ctx pm_ctx;

/* Flags of pm_step. */
#define PM_CONTINUE 1  /* phi and Q held by the context are those of the
                          positions passed in (left by the previous pm_step
                          on this context, with unchanged positions): skip
                          the opening force evaluation */
/* Sort the particles by tile (as pm_sort, without ids) before every k-th
 * step of the call, starting with the first; k in 1..65535.  A sort is
 * skipped when the particles have not moved since the last one.  A
 * fixed-point context that has never sorted sorts before the opening force
 * evaluation as well, with this flag or PM_SORT_AUTO, so that its deposit
 * runs from tiles.  Particle order
 * then changes; use pm_sort with an id array between calls to track
 * particles. */
#define PM_SORT_EVERY(k) ((((int32_t)(k)) & 0xffff) << 8)
/* Sort by tile at an interval the context adapts to how fast particles
 * leave their tiles (fixed-point form only; PM_EUNSUPPORTED otherwise).
 * At the end of each interval the context samples the count of particles
 * whose deposit left their tile's window into pinned host memory (allocated
 * on first use, freed by pm_destroy) and reads it once it has arrived,
 * without waiting; the interval starts at 32 steps, shortens where that
 * count calls for it and doubles after an interval without such particles.
 * The interval, and so the particle order, may depend on timing, never the
 * state as a set of particles.  Where that count is high (clustered
 * states), steps after the first since a sort use larger tile windows and
 * the interval is one step longer; results do not depend on the windows.
 * Overrides PM_SORT_EVERY. */
#define PM_SORT_AUTO (1 << 24)

/* Bytes of device workspace a context with these parameters needs.  Pure
 * host function, no device access.  Returns PM_EINVAL / PM_EUNSUPPORTED for
 * parameters pm_init would reject. */
pm_status pm_workspace_bytes(const pm_params* params, size_t* bytes);

/* Create a context.  d_workspace: device buffer of at least
 * pm_workspace_bytes bytes, 256-byte aligned, owned by the caller and used
 * exclusively by this context until pm_destroy.  hip_stream: a hipStream_t
 * (NULL = default stream).  Enqueues the upload of small constant tables.
 * *out receives the context on PM_OK and is untouched otherwise. */
pm_status pm_init(const pm_params* params, void* d_workspace, size_t bytes,
                  void* hip_stream, pm_ctx** out);

/* Step (i) of Sec. II A with the cloud-in-cell kernel: deposit the particles
 * at d_pos (uint32 or float [3][Np] per the precision) into the context's
 * mass mesh and form delta = rho/rho_bar - 1 in the context.  If d_delta is
 * not NULL, delta (float [N^3]) is also written there. */
pm_status pm_deposit(pm_ctx* ctx, const void* d_pos, float* d_delta);

/* Gravity (Sec. II A, Eq. (2): the Poisson equation of the potential V,
 * solved on the mesh that carries the density of step (i)): phi with
 * lap(phi) = S delta, S = four_pi_G_rhobar (static) or 1.5 omega_m h0^2
 * (comoving, the a-independent potential phi_c of Sec. III), through the FFT
 * with the Green's function of the 7-point Laplacian, zero mean (the k = 0
 * mode of a periodic box carries no force).
 * d_delta NULL uses the context's delta from pm_deposit.  The result stays
 * in the context (for pm_force and pm_step) and is also written to d_phi
 * (float [N^3]) if not NULL. */
pm_status pm_poisson(pm_ctx* ctx, const float* d_delta, float* d_phi);

/* Step (ii) of Sec. II A: Q_c = -(hbar/m)^2/2 L7[sqrt R]/sqrt R with
 * R = max(rho, rho_floor) and L7 the 7-point stencil, in cells^2/time^2
 * (the comoving Q of Eq. (18) is Q_c / a^2).  d_delta NULL uses the
 * context's delta and enables the FP64 path for near-empty cells; an
 * explicit d_delta is used as given (FP32 path only).  The result stays in
 * the context and is also written to d_q (float [N^3]) if not NULL. */
pm_status pm_qpot(pm_ctx* ctx, const float* d_delta, float* d_q);

/* Step (iii) in mesh-gradient form: acceleration at the particles,
 * acc = -grad(phi)/a - grad(Q)/a^2 (a = 1 in a static box), central
 * differences on the mesh and CIC interpolation with the deposit's weights.
 * d_phi / d_q NULL use the context's fields.  d_acc: float [3][Np]. */
pm_status pm_force(pm_ctx* ctx, const float* d_phi, const float* d_q,
                   const void* d_pos, float* d_acc, double a);

/* The leapfrog of Sec. II A with the quantum force added to gravity
 * (principal steps (i)-(iii) at every force evaluation; comoving form with
 * the 1/a^2 of Q from Eq. (18), Sec. III).  Kick-drift-kick over the
 * schedule times[0..nsteps] (host array:
 * times in a static box, scale factors in a comoving box, strictly
 * increasing).  Positions and velocities are synchronised on entry and on
 * return; kicks between steps are merged, so each step costs one deposit,
 * one Poisson solve, one Q evaluation and one fused gather-kick-drift.
 * Comoving kick factors int da/(a^2 H) (gravity) and int da/(a^3 H) (Q,
 * drift) are computed on the host in FP64; half-kicks split at sqrt(a0 a1).
 * flags: PM_CONTINUE or 0.  On return the context's phi and Q are those of
 * the final positions.  PM_FIXED32 drifts are exact (the displacement in
 * fixed-point units rounded to nearest, ties to even, wrapped modulo 2^32)
 * for displacements below 2^51 units (2^19 box lengths) per step. */
pm_status pm_step(pm_ctx* ctx, void* d_pos, float* d_vel, const double* times,
                  int32_t nsteps, int32_t flags);

/* pm_step that also records the energies of Sec. II A and II B (as
 * pm_energy: K of Eq. (8), W = W_g, U = K_rho of Eq. (6) by the forward
 * differences of Eq. (11)'s mesh sum, E = K + W + U) at every synchronised
 * time of the call.  d_energies: device array of (nsteps + 1) x 4 doubles;
 * row s receives K, W, U, E at times[s] (a = times[s] in a comoving box).
 * The partial sums are formed inside the step's own kernels: the Q stencil
 * adds up delta phi and the squared forward differences per block, the fused
 * gather splits each merged kick at the synchronised time and adds up |p|^2
 * there; a one-block kernel per row sums the partials in a fixed order, so
 * the rows are deterministic.  With PM_CONTINUE on a context whose fields
 * are those of the positions, row 0 is left untouched (it is the last row of
 * the previous call).  Enqueues only.  The trajectory equals pm_step's up to
 * the rounding of the split kick (closing and opening halves added one after
 * the other instead of as one merged factor). */
pm_status pm_step_energies(pm_ctx* ctx, void* d_pos, float* d_vel, const double* times,
                           int32_t nsteps, int32_t flags, double* d_energies);

/* Reorder the particles in place by mesh tile (8 x 8 x 32 cells; counting
 * sort, order inside a tile unspecified) and remember the tile ranges.
 * Afterwards the deposit and the gather stage each tile's mesh window in
 * LDS.  Positions and velocities are permuted together; d_ids (int32 [Np],
 * may be NULL) is permuted alongside so callers can track particles.  No
 * result depends on the order: particles that leave their tile later are
 * handled by a direct path, and the integer deposit is order-independent.
 * Call again every few steps as particles move. */
pm_status pm_sort(pm_ctx* ctx, void* d_pos, float* d_vel, int32_t* d_ids);

/* The energies of Sec. II A and II B for the synchronised state (d_pos,
 * d_vel) at scale factor a (1 in a static box): K = K_v of Eq. (8), U = K_rho
 * of Eq. (6) discretised on the mesh as in Eq. (11) (forward differences, the
 * exact conjugate of the 7-point Laplacian in Q), W = W_g the gravitational
 * potential energy (the energy of Eq. (16)'s scale symmetry); definitions
 * and units at pm_energies.  Recomputes delta and phi; blocks until done.
 * Leaves the context's delta, phi and Q at d_pos. */
pm_status pm_energy(pm_ctx* ctx, const void* d_pos, const float* d_vel,
                    double a, pm_energies* out);

/* Grid diagnostics (not part of a step).  Both block until done, use the
 * workspace's field area as scratch (delta, phi and Q must be recomputed
 * afterwards, which pm_step, pm_force and pm_energy do by themselves) and
 * leave the mass mesh of the last state deposited.
 *
 * pm_kinetic_split: the kinetic energy K of Eq. (8) (as in pm_energies) split
 * into the grid-scale bulk motion and the velocity dispersion inside cells
 * (Sec. II B, Eq. (17)).  The bulk velocity at a mesh node is the mean of
 * the particle velocities weighted by mass and by the deposit's CIC kernel;
 * K_bulk = sum over nodes with mass of |P|^2 / (2 M a^2), with M = sum_i m W_i
 * and P = sum_i m W_i p_i at the node; K_disp = K - K_bulk >= 0 up to
 * rounding.  Node momenta are FP64 atomic sums, so the last digits of K_bulk
 * may differ between runs.  a as for pm_energy (1 in a static box). */
typedef struct {
  double K;       /* total kinetic energy, sum m p^2 / (2 a^2) */
  double K_bulk;  /* kinetic energy of the node velocity field */
  double K_disp;  /* K - K_bulk: velocity dispersion below the mesh scale */
} pm_kinetic_parts;

pm_status pm_kinetic_split(pm_ctx* ctx, const void* d_pos, const float* d_vel,
                           double a, pm_kinetic_parts* out);

/* RMS over mesh nodes of the relative density difference
 * (rho_a - rho_b) / rho_b of two particle states of this context's size and
 * precision (Sec. III: an FDM run, a, against the CDM run, b, from the same
 * initial conditions).  Nodes where rho_b is zero are left out; *cells
 * receives the number of nodes used and *rms is 0 when it is 0.  In the
 * fixed-point form the numerator is the exact integer mass difference (a
 * state against itself gives exactly 0); the PM_FP32 deposit sums float
 * atomics in a varying order, so there it carries rounding of order 1e-7. */
pm_status pm_density_rms_diff(pm_ctx* ctx, const void* d_pos_a,
                              const void* d_pos_b, double* rms, int64_t* cells);

/* Shell-averaged power spectrum of the density contrast of the state d_pos
 * (Sec. III measures the FDM suppression as the relative difference of the
 * FDM and CDM spectra).  delta comes from the CIC deposit (no window
 * deconvolution), its forward 3-D FFT is unnormalised, and shell b = 1 ..
 * nbins (nbins <= N/2) holds the modes whose integer mode number |m| lies in
 * [b - 1/2, b + 1/2).  Host arrays of nbins doubles receive
 *   k_out[b-1]      = 2 pi b / box (caller's length units),
 *   p_out[b-1]      = box^3 / N^6 * mean of |delta_m|^2 over the shell,
 *   counts_out[b-1] = number of modes in the shell (of the full spectrum:
 *                     the stored half counts modes with 0 < m_z < N/2 twice).
 * Blocks until done, like the other diagnostics (same scratch use).
 * PM_EINVAL for null pointers or nbins outside [1, N/2]. */
pm_status pm_power_spectrum(pm_ctx* ctx, const void* d_pos, int32_t nbins,
                            double* k_out, double* p_out, double* counts_out);

/* The paper's own coupling of particles and mesh (Sec. II A), as two
 * composable steps (the step loop of pm_step keeps cloud-in-cell):
 *
 * pm_spline_density: d_delta (float [N^3], caller-owned) receives
 * rho/rho_bar - 1 at the mesh nodes from Eq. (9) with the cubic spline of
 * Eq. (15), smoothing length h in cells (the paper uses 3.5 to 4):
 * rho(x_j) = sum_i m W(|x_j - q_i|, h), m = N^3 / Np mean densities.  Each
 * kernel value is rounded once to 2^-40 of a particle mass and summed as a
 * 64-bit integer into the workspace's mass mesh (bytes [0, 8 N^3), the
 * units of the fixed-point CIC deposit, in both precisions): the sums are
 * bitwise reproducible and independent of particle order, and delta is
 * formed by the exact subtraction of the mean.  The context's delta is the
 * spline density's afterwards: pm_qpot(ctx, NULL, d_q) gives Q on it, with
 * the FP64 path below rho_fp64_below in the fixed-point form.
 *
 * pm_spline_qforce: d_acc ([3][Np] float) receives the quantum acceleration of
 * every particle by the kernel gradient, Eq. (14): a_i = sum_j Q_j
 * grad W(x_j - q_i) (cell units, dx = 1), with the sign that makes it
 * -grad Q, i.e. minus the particle derivative of the discrete K_rho of
 * Eq. (11) whose node derivative is Q.  d_q is float [N^3] as from pm_qpot.
 *
 * Both enqueue only.  PM_EINVAL for null pointers or h outside
 * [2, 16] (below two cells the lattice sum of W, a particle's deposited
 * mass, varies with its position by more than 0.2 %) or so wide that
 * 2 floor(h) + 2 > N. */
pm_status pm_spline_density(pm_ctx* ctx, const void* d_pos, double h, float* d_delta);
pm_status pm_spline_qforce(pm_ctx* ctx, const void* d_pos, const float* d_q, double h,
                           float* d_acc);

/* nsteps kick-drift-kick steps through times[0..nsteps] (as pm_step) with the
 * paper's own coupling (Sec. II A): every force evaluation deposits the
 * spline density (pm_spline_density), solves gravity on it (FFT Poisson,
 * -grad phi interpolated by cloud-in-cell, as the host code's PM does) and
 * takes Q on it with the kernel-gradient force (pm_spline_qforce), with the
 * FP64 near-empty path of the fixed-point form.  Comoving factors as pm_step
 * (Q's kick carries 1/a^3, gravity's 1/a^2).  Unfused: separate deposit,
 * Poisson, Q, force, kick and drift kernels, no merged half-kicks, two extra
 * [3][Np] float arrays in the workspace's particle buffers.  The particle
 * order is the caller's; on a context sorted by pm_sort the deposit runs
 * from the tiles' LDS windows (particles that left their tile since the sort
 * add directly; the result does not depend on it).  Enqueues only;
 * positions and velocities are synchronised on entry and on return.  Leaves
 * no cloud-in-cell field valid (later calls recompute them). */
pm_status pm_spline_step(pm_ctx* ctx, void* d_pos, float* d_vel, const double* times,
                         int32_t nsteps, double h);

/* K, W, U, E as pm_energy, with the density of pm_spline_density (smoothing
 * length h cells) in place of cloud-in-cell: the energy that the kernel-
 * gradient force of pm_spline_step conserves (with gravity off) up to the
 * leapfrog's second-order error (Sec. II A).  U takes forward differences
 * of sqrt(max(rho, floor)), W = sum delta phi / 2a.  Blocks until done;
 * uses the field area as scratch like the other diagnostics. */
pm_status pm_spline_energy(pm_ctx* ctx, const void* d_pos, const float* d_vel, double h,
                           double a, pm_energies* out);

/* Per-kernel timing (observability).  While enabled, every kernel the
 * context launches is bracketed by two HIP events recorded on its stream.
 * pm_timing_enable(ctx, 1) clears the counters and starts recording;
 * (ctx, 0) stops.  pm_timing_read synchronises the stream, folds all
 * recorded events into per-kernel totals and writes up to max entries
 * (*count receives the number written).  Event objects come from the HIP
 * runtime and are reused; no device buffer is allocated. */
typedef struct {
  char name[32];      /* kernel family, e.g. "deposit", "fft_x_green" */
  int64_t launches;   /* launches recorded since enable */
  double total_ms;    /* summed event-to-event time */
} pm_kernel_time;

pm_status pm_timing_enable(pm_ctx* ctx, int32_t on);
pm_status pm_timing_read(pm_ctx* ctx, pm_kernel_time* out, int32_t max, int32_t* count);

/* ---------------------------------------------------------------------
 * Batched runs (serving many independent boxes of one mesh size).
 *
 * A batch holds `slots` independent runs that share n_mesh, n_part,
 * precision, cosmology (or four_pi_G_rhobar) and floors; each slot has its
 * own box size and hbar/m.  Every kernel of a step is launched once for all
 * active slots (the launch grid's second dimension enumerates them), so a
 * step of B small boxes costs one set of launches instead of B.
 *
 * Memory: the caller passes one workspace of pm_batch_workspace_bytes bytes;
 * particle arrays of all slots are contiguous: positions [slots][3][Np]
 * (uint32 or float), velocities [slots][3][Np] float.  Slot s of the
 * workspace has the layout of a single context, so bytes [0, 8 N^3) of slot
 * s hold its mass mesh; slot s starts at pm_batch_slot_offset(batch, s).
 * ------------------------------------------------------------------- */
typedef struct pm_batch pm_batch;

typedef struct {
  double box;           /* side length of this run, caller's length unit */
  double hbar_over_m;   /* hbar/m of this run (length^2/time), >= 0 */
} pm_slot_params;

/* Largest number of steps one pm_batch_step call may take. */
#define PM_BATCH_MAX_STEPS 256
/* Flag of pm_batch_step: capture the call's kernels in a HIP graph the first
 * time a call of its shape is made -- shape: the number of listed slots,
 * nsteps, the other flags and whether every listed slot was sorted on entry
 * -- and replay the graph for later calls of the same shape (up to 64 graphs
 * per batch, freed by pm_batch_destroy); the upload of the call's slot list
 * and kick/drift table precedes the graph on the stream as in an uncaptured
 * call.
 * The slot identities and the time-step factors are data of the uploaded
 * table, so a replay advances whichever slots are listed along their own
 * schedules; results equal those of the uncaptured call bitwise.  Needs a
 * non-default stream (PM_EINVAL on the NULL stream). */
#define PM_BATCH_GRAPH (1 << 25)

/* Workspace of a batch: params as for pm_workspace_bytes (box and
 * hbar_over_m are ignored: they are per slot), slots >= 1. */
pm_status pm_batch_workspace_bytes(const pm_params* params, int32_t slots, size_t* bytes);

/* Create a batch on a caller-owned workspace (256-byte aligned) and stream.
 * All slots start with box = params->box and hbar_over_m =
 * params->hbar_over_m.  The batch allocates two pinned host buffers (the
 * per-call slot list and kick/drift table are staged through them, so a
 * call never waits for steps still queued); PM_EDEVICE if that fails. */
pm_status pm_batch_init(const pm_params* params, int32_t slots, void* d_workspace, size_t bytes,
                        void* hip_stream, pm_batch** out);

/* Byte offset of slot s's region inside the batch workspace. */
pm_status pm_batch_slot_offset(const pm_batch* batch, int32_t slot, size_t* offset);

/* Set the box size and hbar/m of one slot (host only; takes effect at the
 * next pm_batch_step that lists the slot).  Marks the slot's fields stale. */
pm_status pm_batch_set_slot(pm_batch* batch, int32_t slot, const pm_slot_params* sp);

/* Advance the listed slots (host array slots[0..nactive), distinct, in
 * range) by nsteps kick-drift-kick steps each, slot slots[i] along its own
 * schedule times[i * (nsteps + 1) .. i * (nsteps + 1) + nsteps] (host array,
 * strictly increasing; scale factors in a comoving batch).  State in and out
 * is synchronised, as for pm_step.  flags: PM_CONTINUE (every listed slot's
 * fields are those of its positions, left by the previous pm_batch_step),
 * PM_SORT_EVERY(k) and PM_BATCH_GRAPH.  1 <= nsteps <= PM_BATCH_MAX_STEPS. */
pm_status pm_batch_step(pm_batch* batch, void* d_pos, float* d_vel, int32_t nactive,
                        const int32_t* slots, const double* times, int32_t nsteps,
                        int32_t flags);

/* Wait for the batch's queued uploads, then free its host-side object and
 * pinned staging buffers (the caller's workspace is untouched). */
pm_status pm_batch_destroy(pm_batch* batch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): the Poisson solve
 * of pm_poisson without a context or workspace.  d_phi (float [N^3])
 * receives phi with lap(phi) = S delta (S in 1/time^2, cell units: the S of
 * pm_poisson), zero mean, from d_delta (float [N^3], its mean ignored), both
 * C-order device arrays owned by the caller; enqueued on hip_stream (NULL =
 * default stream).  The spectrum and the FFT's constant tables live in a
 * device array of the library, one per GPU, held until the process ends:
 * 8.5 MB, enough for N <= 128.  Calls that overlap on one GPU (concurrent
 * streams, threads) share it and race; serialise them.  Nothing is cleared
 * between calls (every pass writes all it reads).  PM_EINVAL for null
 * pointers or a non-finite S, PM_EUNSUPPORTED for N not a power of two >= 16,
 * PM_ENOMEM for N above 128 (the array's size), PM_EDEVICE for HIP errors.
 * No hipMalloc, hipFree or allocating library call is made. */
pm_status pm_poisson_static(int32_t n_mesh, double S, const float* d_delta, float* d_phi,
                            void* hip_stream);

/* Free the host-side context (no device memory is owned). */
pm_status pm_destroy(pm_ctx* ctx);

/* Static, NUL-terminated description of a status code. */
const char* pm_strerror(pm_status status);

#ifdef __cplusplus
}
#endif

#endif /* FDMPM_H */
