/*
 * nspnp.h -- C ABI of the MI355X (gfx950) solver for the coupled
 * Navier-Stokes / Poisson-Nernst-Planck equations of sheared electrolyte
 * between two sliding charged walls (plane Couette flow), after
 * Ostilla-Monico & Lee, arXiv:1701.02005.
 *
 * What is solved (Sec. II, Eqs. (1)-(4)), in units of the half gap h, the
 * wall speed U, the bulk concentration c0 and the thermal voltage V_T:
 *   du/dt + div(u u) = -grad p + Re^-1 lap u + sF K (c+ - c-) grad Phi
 *   div u = 0
 *   dc+-/dt + div(u c+-) = (Re Sc)^-1 div(grad c+- +- c+- grad Phi)
 *   lap phi = -(c+ - c-) / (2 lam^2),  Phi = (vhat/2) y + phi,  phi(+-1) = 0
 * K = beta / (2 Sc Re^2 lam^2), lam = lambda_D / h.  Walls y = -1, +1 move at
 * u_bot, u_top; no slip, no penetration, zero ion flux through the walls
 * (Fig. 1 caption), wall potentials -vhat/2, +vhat/2 (Phi_0 = V y / h,
 * Sec. II).  x (length lx) and z (length lz) are periodic.
 *
 * Discretisation (Sec. II, Fig. 1): second-order central differences on a
 * staggered mesh, tanh-stretched in y; p, c+-, phi at cell centres, velocity
 * components and ion fluxes on the cell faces.  One call of nspnp_step with
 * n = 1 advances one Runge-Kutta substep: explicit advection, horizontal
 * diffusion, Coulomb force and migration; implicit (Crank-Nicolson) wall-
 * normal diffusion of u, v, w, c+, c- as batched tridiagonal systems; the
 * pressure projection and the potential solve, each by FFT in x and z plus a
 * tridiagonal (Thomas) solve in y per Fourier mode (Sec. II).
 *
 * Memory and ownership.  All field memory is ONE device buffer owned by the
 * caller (size from nspnp_workspace_bytes); the library owns only the small
 * host handle.  Every field is stored as a contiguous array of
 * nx * nz * (ny - 1) values indexed x + nx * (z + nz * j), x fastest, j the
 * cell row across the gap.  v is stored at the bottom face of each row (row 0
 * is the bottom wall and holds 0; the top wall face is implicit).  u sits on
 * the x-face at x = i*lx/nx, w on the z-face at z = k*lz/nz.  Work is queued
 * on the caller's HIP stream and is asynchronous unless stated otherwise.
 *
 * Errors.  Every int-returning call returns NSPNP_OK (0) or a negative code;
 * nothing throws or aborts across the ABI.  nspnp_last_error() gives a
 * message for the calling thread.  A device-side failure (HIP error) is
 * reported by the call that detects it.
 */
#ifndef NSPNP_H
#define NSPNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* symbols of this header are the only ones the shared library exports */
#if defined(__GNUC__) || defined(__clang__)
#define NSPNP_API __attribute__((visibility("default")))
#else
#define NSPNP_API
#endif

#define NSPNP_OK 0
#define NSPNP_ERR_INVALID (-1)     /* bad argument or configuration                 */
#define NSPNP_ERR_SIZE (-2)        /* unsupported size (see nspnp_config)            */
#define NSPNP_ERR_HIP (-3)         /* a HIP runtime call failed                      */
#define NSPNP_ERR_NONFINITE (-4)   /* NaN/Inf or negative concentration detected     */
#define NSPNP_ERR_WORKSPACE (-5)   /* workspace missing, too small or misaligned     */

#define NSPNP_PREC_FP64 0  /* every field and every operation in FP64              */
#define NSPNP_PREC_MIXED 1 /* FP32 state, stencils and transport; FP64 elliptic
                              solves, tridiagonal eliminations and reductions */

/* field ids for get/set */
#define NSPNP_FIELD_U 0
#define NSPNP_FIELD_V 1
#define NSPNP_FIELD_W 2
#define NSPNP_FIELD_CP 3   /* cation concentration c+            */
#define NSPNP_FIELD_CM 4   /* anion concentration c-             */
#define NSPNP_FIELD_PHI 5  /* potential perturbation phi         */
#define NSPNP_FIELD_P 6    /* pressure                           */

/*
 * Configuration.  Sizes: nx, nz of the form 2^a 3^b, even, 4..1024; ny (the
 * number of wall-normal NODES, so ny - 1 cell rows) within 5..513, and
 * nx * nz * (ny - 1) below 2^31.  Lengths in
 * units of h.  stretch is the tanh clustering factor g of the y nodes
 * y_j = tanh(g xi_j)/tanh(g), xi_j uniform on [-1, 1] (g = 0: uniform).
 * force_sign sF: -1 is the physical Coulomb force rho E = -rho grad Phi,
 * +1 the sign printed in Eq. (1).  dt > 0 fixes the full Runge-Kutta step;
 * dt <= 0 selects the adaptive step min(cfl / max(|u|/dx + |v|/dy + |w|/dz),
 * 2 lam^2 Re Sc / max(c+ + c-), min(Re, Re Sc) / (4/dx^2 + 4/dz^2)),
 * recomputed at the first stage of every step.  Initial state (init_state):
 * linear Couette profile plus seeded uniform noise of amplitude u_noise on
 * every velocity unknown, concentrations 1 plus seeded noise of amplitude
 * c_noise with the volume mean removed, one projection, phi from the charge,
 * p = 0.  The noise is SplitMix64 (Steele, Lea & Flood 2014) output number
 * (field << 40) + index + 1 for the given seed, mapped to [-1, 1).
 */
typedef struct nspnp_config {
    int32_t nx, ny, nz;
    int32_t precision; /* NSPNP_PREC_FP64 or NSPNP_PREC_MIXED */
    double lx, lz, stretch;
    double re, sc, beta, debye, vhat;
    double u_top, u_bot, force_sign;
    double dt, cfl;
    uint64_t seed;
    double u_noise, c_noise;
    /* 1: diffusion implicit in x and z as well as y, by the three-direction
     * tridiagonal approximate factorisation of the base solver (Sec. II):
     * (I - b L_x)(I - b L_y)(I - b L_z) delta = r, b = alpha dt nu / 2, the
     * x/z diffusion leaving H for the implicit part, the pressure update
     * using the full Laplacian of psi and the dt rule dropping its explicit
     * diffusion limit.  0: only the wall-normal diffusion is implicit. */
    int32_t implicit_xz;
    /* Face value of c in the migration flux.  0: the mean of the two cells
     * (the second-order central form of Sec. II), whose stationary cell
     * ratio (1 - z dPhi/2)/(1 + z dPhi/2) turns negative once the potential
     * difference dPhi across a face exceeds 2 thermal volts.  1: hybrid, the
     * cell the species' drift comes from (upwind) on faces with |dPhi| >= 2,
     * the mean elsewhere; its stationary ratios 1/(1 + z dPhi) and 1 + |dPhi|
     * stay positive (first order on those faces only).  2: as 1, and the
     * face value of c in the advective flux limited as well: the upwind cell
     * of the face velocity plus the van Leer slope a b / (a + b) (a, b the
     * differences across the upwind cell and across the face; c_U alone when
     * a b <= 0 or when the upwind cell is a wall row), so that a profile advected
     * at cell Peclet numbers Re Sc |u| h >> 2 forms no new extrema; equal to
     * the mean on a linear profile of equal spacings.  Applies to the update
     * and to the flux diagnostics alike.  Other values: NSPNP_ERR_INVALID. */
    int32_t migration_face;
} nspnp_config;

typedef struct nspnp_state nspnp_state;

/* Bytes of device memory the caller must provide for this configuration
 * (0 if the configuration is invalid).  The buffer must be 256-byte aligned. */
NSPNP_API size_t nspnp_workspace_bytes(const nspnp_config *cfg);

/* Build the grid and operator tables, lay the fields out in dev_workspace
 * and compute the seeded initial state (Sec. II geometry and boundary
 * conditions).  hip_stream is a hipStream_t (NULL: the null stream).  The
 * workspace must stay allocated until nspnp_destroy.  Synchronises the
 * stream before returning.  On success *out receives the handle. */
NSPNP_API int nspnp_init_state(const nspnp_config *cfg, void *dev_workspace, size_t bytes, void *hip_stream,
                     nspnp_state **out);

/* Host-only: the ny wall-normal node coordinates yn and the ny-1 cell-centre
 * coordinates yc of this configuration (caller-owned host arrays). */
NSPNP_API int nspnp_grid(const nspnp_config *cfg, double *yn, double *yc);

/* Advance n_substeps Runge-Kutta substeps (stage = substep count mod 3, three
 * substeps make one full step dt).  Asynchronous.
 * Health check: at the first stage of every step a device reduction (the
 * one that also evaluates the adaptive dt rule) looks at every cell and sets
 * a sticky flag when a field value or the step is not finite or a
 * concentration is negative.  The flag is copied back behind the queued
 * work; nspnp_step returns NSPNP_ERR_NONFINITE, with a message naming the
 * fault, from the first call that starts after the copy has landed, and
 * nspnp_sync, which waits for the copy, from its next call.  The run stays
 * flagged until
 * nspnp_set_clock (or a new init).  The same check records the largest
 * potential difference across one cell face (nspnp_diagnostics out[5]). */
NSPNP_API int nspnp_step(nspnp_state *s, int32_t n_substeps);

/* Solve the elliptic problem of the pressure projection (kind 0) or of the
 * potential (kind 1) on this grid (Sec. II): (Lxx + Lzz + Lyy) out = rhs with
 * three-point periodic Lxx, Lzz and the finite-volume Lyy across the gap;
 * kind 0 has zero-flux walls and a zero volume-mean solution (rhs must have
 * zero volume mean), kind 1 has out = 0 on the walls.  rhs and out are
 * caller-owned FP64 device arrays of nx*nz*(ny-1) cell values; they may
 * alias.  Asynchronous. */
NSPNP_API int nspnp_poisson_solve(nspnp_state *s, int32_t kind, const double *dev_rhs, double *dev_out);

/* Mean wall shear stress in units of rho_w U^2 (Sec. II, tau_w = eta d<u_x>/dy):
 * the plane-averaged viscous flux through the bottom and top wall faces,
 * Re^-1 (<u>_0 - u_bot)/(dy_0/2) and Re^-1 (u_top - <u>_last)/(dy_last/2).
 * Host FP64 outputs.  Synchronises the stream. */
NSPNP_API int nspnp_wall_shear_stress(nspnp_state *s, double *tau_bottom, double *tau_top);

/* Plane-averaged total wall-normal flux of each ion species (advection +
 * diffusion + migration) at the ny y-nodes, exactly zero on the two walls
 * (Fig. 1 caption); and the total ion contents sum(c Omega).  jy_plus and
 * jy_minus are caller-owned host arrays of ny doubles.  Synchronises. */
NSPNP_API int nspnp_ion_flux(nspnp_state *s, double *jy_plus, double *jy_minus, double *mass_plus,
                   double *mass_minus);

/* ---- extras used by drivers and tests -------------------------------- */

/* Copy a field to / from a caller-owned FP64 device array of nx*nz*(ny-1)
 * values (converted to / from FP32 in the mixed form).  Asynchronous.
 * Setting u, v, w, c+- does not re-solve phi; call nspnp_refresh_potential. */
NSPNP_API int nspnp_get_field(nspnp_state *s, int32_t field, double *dev_out);
NSPNP_API int nspnp_set_field(nspnp_state *s, int32_t field, const double *dev_in);

/* Re-solve phi from the current c+-.  Asynchronous. */
NSPNP_API int nspnp_refresh_potential(nspnp_state *s);

/* Explicit right-hand sides H (advection, horizontal diffusion, Coulomb force,
 * migration) of u, v, w, c+, c- for the current state, written to five
 * caller-owned FP64 device arrays out[0..4].  Asynchronous. */
NSPNP_API int nspnp_explicit_terms(nspnp_state *s, double *const dev_out[5]);

/* Scalar diagnostics, FP64, synchronising: out[0] kinetic energy
 * 1/2 sum(|u|^2 Omega), out[1] max |div u| over the cells, out[2] min c+,
 * out[3] min c-, out[4] max(c+ + c-), out[5] the largest difference of the
 * total potential Phi across an interior cell face (x, z or y).  out[5] is
 * the cell Peclet number of migration: the central face value of c in the
 * migration flux (Sec. II) keeps concentrations positive at equilibrium only
 * while it stays below 2.  Returns NSPNP_ERR_NONFINITE if any is not
 * finite. */
NSPNP_API int nspnp_diagnostics(nspnp_state *s, double out[6]);

/* Simulation clock: time, current full step dt, next stage (0..2), substeps
 * taken.  get synchronises; set is used to restart from saved fields and
 * clears the health flag (see nspnp_step). */
NSPNP_API int nspnp_get_clock(nspnp_state *s, double *t, double *dt, int32_t *stage, int64_t *substeps);
NSPNP_API int nspnp_set_clock(nspnp_state *s, double t, double dt, int32_t stage, int64_t substeps);

/* Arbitrary wall potential (the model admits spatially and temporally varying
 * wall potentials, Sec. II and Sec. V): the walls are at -vhat/2 + g_bot(x, z)
 * and +vhat/2 + g_top(x, z) thermal volts.  g is the wall value of the
 * potential perturbation phi, so the potential solve becomes the
 * inhomogeneous Dirichlet problem lap phi = -(c+ - c-)/(2 lam^2),
 * phi = g on the walls (at the half-cell distance, like the zero value of the
 * uniform case).  dev_bot / dev_top: device arrays of nx * nz doubles, x
 * fastest (the cell columns of one plane), copied into the workspace; NULL
 * sets that wall's g to zero; both NULL restore uniform walls.  Asynchronous
 * on the solver's stream; used from the next potential solve on (every
 * substep, or nspnp_refresh_potential to make phi consistent at once).  A
 * time-varying wall potential is set again between calls of nspnp_step.
 * Not part of checkpoints (set it again after nspnp_load); single runs only.
 * nspnp_poisson_solve keeps zero wall values. */
NSPNP_API int nspnp_set_wall_potential(nspnp_state *s, const double *dev_bot, const double *dev_top);

/* Run statistics: the time averages behind the mean and RMS profiles and
 * the friction coefficient of the turbulent runs (Sec. III).  Every sample
 * adds, for each of the M = ny - 1 rows, the plane (x-z) means of
 * u, v, w, c+, c-, phi, p and of their squares, weighted by the time elapsed
 * since the previous sample (or since nspnp_stats_begin).  Cell rows for all
 * fields except v, whose row j is its node row j (the lower face of cell
 * row j); phi is the potential perturbation (Phi = phi + vhat y / 2).
 *
 * nspnp_stats_begin(s, every): every > 0 clears the statistics, takes the
 * current time as the start and samples at the end of every substep whose
 * count (after it) is a multiple of every; every = 0 stops sampling and
 * keeps the sums.  Asynchronous.  nspnp_set_clock does not touch the
 * statistics: call nspnp_stats_begin again after a clock change.
 *
 * nspnp_stats_read: *time (NULL allowed) receives the averaged time span,
 * *samples (NULL allowed) the number of samples, and out (NULL or
 * 14 * M doubles) the averages as out[q * M + j], q = 0..6 the means of
 * u, v, w, c+, c-, phi, p and q = 7..13 the means of their squares (all 0
 * before the first sample).  RMS profiles are sqrt(out[7+q] - out[q]^2).
 * Synchronises. */
NSPNP_API int nspnp_stats_begin(nspnp_state *s, int32_t every);
NSPNP_API int nspnp_stats_read(nspnp_state *s, double *time, int64_t *samples, double *out);

/* Friction quantities and wall units of the run statistics (Sec. II
 * definitions: wall shear stress tau_w = eta d<u_x>/dy in units of rho U^2,
 * c_f = tau_w / (rho U^2 / 2), Re_tau = u_tau h / nu with u_tau = sqrt(tau_w
 * / rho)), applied to the time-averaged plane-mean velocity of the run
 * statistics.  out[0] tau at the bottom wall and out[1] at the top wall (the
 * viscous flux through the wall face over the half cell next to it, as in
 * nspnp_wall_shear_stress), out[2] their mean tau, out[3] c_f = 2 tau,
 * out[4] Re_tau = Re sqrt(|tau|), out[5] u_tau = sqrt(|tau_bottom|) of the
 * lower wall.  rms (NULL or 7 * M doubles, M = ny - 1): the RMS profiles
 * sqrt(max(<q^2> - <q>^2, 0)) of u, v, w, c+, c-, phi, p as rms[q * M + j].
 * y_plus, u_plus (NULL or M doubles each): the lower wall's wall units of the
 * rows, y+ = (1 + y_j) Re u_tau and u+ = (<u>_j - u_bot) / u_tau (y_j the
 * cell centres).  Before the first sample every output is NaN.
 * Synchronises. */
NSPNP_API int nspnp_stats_derived(nspnp_state *s, double out[6], double *rms, double *y_plus, double *u_plus);

/* Kinetic-energy budget of the semi-discrete momentum equation (Sec. II,
 * Eq. (1)): dKE/dt = out[0] - out[1] + out[2] with out[0] the power of the
 * moving walls against the viscous wall stress, sum over the wall faces of
 * u_wall Re^-1 (u_wall - u_next)/(dy/2) dA; out[1] the viscous dissipation
 * Re^-1 sum |grad u|^2 Omega over every difference of the staggered velocity
 * components (with the half cells next to the walls); out[2] the work of the
 * Coulomb force, sum u . f Omega.  Convection and the pressure gradient do no
 * work on a discretely divergence-free field.  FP64 host outputs.
 * Synchronises. */
NSPNP_API int nspnp_energy_budget(nspnp_state *s, double out[3]);

/* Checkpoint of a run: the seven fields and the five explicit-term buffers
 * H (kept between the stages of a Runge-Kutta step) in the storage type,
 * the clock, the substep count and the run statistics with their sampling
 * interval, written to the file at path as a small header followed by raw
 * little-endian arrays.  nspnp_load restores it into a handle initialised
 * with the same configuration (seed and noise amplitudes may differ); the
 * run, and its statistics, then continue bit for bit as the saved one
 * would have.  Time statistics of ensembles are not part of it.  Both
 * synchronise; NSPNP_ERR_INVALID for an unreadable, foreign or mismatching
 * file. */
NSPNP_API int nspnp_save(nspnp_state *s, const char *path);
NSPNP_API int nspnp_load(nspnp_state *s, const char *path);

/* Choose this run's launch shapes as nspnp_ensemble_autotune does for a
 * size class (same candidates, cache format and key, with member count 1).
 * Trials advance the run by trial_substeps (a multiple of 3) per candidate;
 * the shapes never change a result beyond the rounding order of the CN
 * method.  tiles_out (NULL or 8 ints) receives the choice.  Synchronises. */
NSPNP_API int nspnp_autotune(nspnp_state *s, const char *cache_path, int32_t trial_substeps, int32_t *tiles_out);

/* Read / set this run's launch shapes (8 ints in the order of
 * nspnp_ensemble_autotune's tiles_out).  set validates every entry
 * (NSPNP_ERR_INVALID when out of range) and synchronises. */
NSPNP_API int nspnp_get_tiles(const nspnp_state *s, int32_t *tiles_out);
NSPNP_API int nspnp_set_tiles(nspnp_state *s, const int32_t *tiles);

/* Kernel timing with HIP events recorded on the solver's stream around every
 * kernel launch (off by default).  enable(1) clears the totals and starts
 * recording; read() synchronises, folds the recorded events into per-kernel
 * totals and reports, for each of *count kernel classes, its name (static
 * strings), the accumulated milliseconds and the number of launches.  names,
 * total_ms and launches may be NULL or arrays of at least 16 entries. */
NSPNP_API int nspnp_profile_enable(nspnp_state *s, int32_t on);
NSPNP_API int nspnp_profile_read(nspnp_state *s, int32_t *count, const char **names, double *total_ms,
                                 int64_t *launches);

/* ---- ensembles of independent runs ----------------------------------- */

/*
 * An ensemble advances n independent runs together, each with its own
 * configuration (Re, Sc, beta, Debye length, voltage, walls, seed, noise, dt
 * rule).  Runs with the same grid (nx, ny, nz, lx, lz, stretch, precision,
 * fixed-or-adaptive dt) share every kernel launch; each run keeps its own
 * adaptive dt and clock, and gives the same result as a single run of the
 * same configuration.  The caller owns one device workspace of
 * nspnp_ensemble_workspace_bytes(); members are numbered as in cfgs.
 */
typedef struct nspnp_ensemble nspnp_ensemble;

NSPNP_API size_t nspnp_ensemble_workspace_bytes(const nspnp_config *cfgs, int32_t n);
/* Initialise every member as nspnp_init_state does.  hip_stream must not be
 * the legacy null stream if nspnp_ensemble_capture is used.  Synchronises. */
NSPNP_API int nspnp_ensemble_init(const nspnp_config *cfgs, int32_t n, void *dev_workspace, size_t bytes,
                                  void *hip_stream, nspnp_ensemble **out);
/* Advance every member n_substeps substeps (replaying the captured graph for
 * whole multiples of its length when one exists).  Asynchronous.  Health
 * checks as for nspnp_step; the message names the first flagged member.
 * A flagged ensemble stays flagged. */
NSPNP_API int nspnp_ensemble_step(nspnp_ensemble *e, int32_t n_substeps);
/* Wait for the queued work of every member; NSPNP_ERR_NONFINITE if a health
 * check has flagged a member. */
NSPNP_API int nspnp_ensemble_sync(nspnp_ensemble *e);
/* Capture substeps_per_replay substeps (a multiple of 3, from the start of a
 * Runge-Kutta step) of all members into one hipGraph, replayed by step().
 * Nothing is executed by the capture itself. */
NSPNP_API int nspnp_ensemble_capture(nspnp_ensemble *e, int32_t substeps_per_replay);
/* on = 1: clear and start accumulating, after every substep, the plane means
 * of u, c+ - c- and phi of every cell row, weighted by the substep duration;
 * on = 0: stop.  Asynchronous. */
NSPNP_API int nspnp_ensemble_stats(nspnp_ensemble *e, int32_t on);
/* Time means since statistics were switched on of member's plane-averaged
 * u, c+ - c-, phi per cell row (host arrays of ny-1 doubles) and the
 * averaging time.  Synchronises. */
NSPNP_API int nspnp_ensemble_profiles(nspnp_ensemble *e, int32_t member, double *u, double *rho, double *phi,
                                      double *time_weight);
/* Single-run diagnostics of one member (see the single-run calls). */
NSPNP_API int nspnp_ensemble_get_field(nspnp_ensemble *e, int32_t member, int32_t field, double *dev_out);
NSPNP_API int nspnp_ensemble_set_field(nspnp_ensemble *e, int32_t member, int32_t field, const double *dev_in);
NSPNP_API int nspnp_ensemble_refresh_potential(nspnp_ensemble *e, int32_t member);
NSPNP_API int nspnp_ensemble_diagnostics(nspnp_ensemble *e, int32_t member, double out[6]);
NSPNP_API int nspnp_ensemble_wall_shear_stress(nspnp_ensemble *e, int32_t member, double *tau_bottom,
                                               double *tau_top);
NSPNP_API int nspnp_ensemble_ion_flux(nspnp_ensemble *e, int32_t member, double *jy_plus, double *jy_minus,
                                      double *mass_plus, double *mass_minus);
NSPNP_API int nspnp_ensemble_clock(nspnp_ensemble *e, int32_t member, double *t, double *dt, int64_t *substeps);
/* Choose the launch shapes of every size class (threads per block of the
 * stencil, Crank-Nicolson, mode-Thomas and correction kernels, points per
 * block of the x and z transforms) by timing trial_substeps substeps (a
 * multiple of 3) per candidate, coordinate by coordinate; also the rows
 * one block of the stencil kernel marches.  Results are read from /
 * appended to the text cache at cache_path (NULL: no cache), one line per
 * (arch, grid, precision, members) key.  Trials advance the members (the
 * launch shape does not change any result); on return every member has
 * advanced by the same number of substeps.  tiles_out (NULL or 8 ints per
 * class) receives the choice: explicit-kernel threads, CN threads (64 to
 * 256: tiles of 16 columns; 512: tiles of 32 columns), x and z
 * transform points, modes per tile of the mode solves, correction threads,
 * explicit-kernel and correction slab rows, and the CN method (0: lane
 * scans over whole columns; 16 or 32: row slabs of that height, three
 * passes).
 * Synchronises. */
NSPNP_API int nspnp_ensemble_autotune(nspnp_ensemble *e, const char *cache_path, int32_t trial_substeps,
                                      int32_t *tiles_out);
/* Number of size classes. */
NSPNP_API int32_t nspnp_ensemble_classes(const nspnp_ensemble *e);
NSPNP_API void nspnp_ensemble_destroy(nspnp_ensemble *e);

/* ---- warm-start surrogate network ------------------------------------- */

/*
 * A fully connected network x -> GELU(x W_0 + b_0) -> ... -> x W_L + b_L
 * (GELU in erf form on every hidden layer) trained by mean-squared error and
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8) with FP32 master weights.  All
 * matrix products run on the matrix cores in BF16 with FP32 accumulation;
 * activations are rounded to BF16 between layers.  n_layers weight layers
 * map sizes[0] inputs to sizes[n_layers] outputs; max_rows bounds the rows
 * of one call.  Parameters cross the ABI as FP32 host arrays ordered
 * W_0 [sizes[0] x sizes[1]] row-major, b_0 [sizes[1]], W_1, b_1, ...; inputs
 * [rows x sizes[0]] and targets / outputs [rows x sizes[n_layers]] are
 * caller-owned FP32 device arrays.
 */
typedef struct nspnp_mlp nspnp_mlp;

NSPNP_API size_t nspnp_mlp_workspace_bytes(int32_t n_layers, const int32_t *sizes, int32_t max_rows);
NSPNP_API int nspnp_mlp_init(int32_t n_layers, const int32_t *sizes, int32_t max_rows, const float *host_params,
                             void *dev_workspace, size_t bytes, void *hip_stream, nspnp_mlp **out);
NSPNP_API int nspnp_mlp_set_params(nspnp_mlp *h, const float *host_params);
/* FP32 master parameters and / or the gradients of the last gradients() or
 * train_step() call, in the parameter order above (either may be NULL). */
NSPNP_API int nspnp_mlp_get_params(nspnp_mlp *h, float *host_params, float *host_grads);
/* Network outputs for rows inputs.  Asynchronous. */
NSPNP_API int nspnp_mlp_forward(nspnp_mlp *h, const float *dev_x, int32_t rows, float *dev_y);
/* Loss and gradients without updating the parameters; *loss (host, may be
 * NULL) receives the mean squared error.  Synchronises when loss != NULL. */
NSPNP_API int nspnp_mlp_gradients(nspnp_mlp *h, const float *dev_x, const float *dev_y, int32_t rows, float *loss);
/* One full-batch Adam step with learning rate lr; the loss before the step is
 * written to dev_loss (device FP32, may be NULL).  Asynchronous. */
NSPNP_API int nspnp_mlp_train_step(nspnp_mlp *h, const float *dev_x, const float *dev_y, int32_t rows, float lr,
                                   float *dev_loss);
NSPNP_API int nspnp_mlp_sync(nspnp_mlp *h);
NSPNP_API void nspnp_mlp_destroy(nspnp_mlp *h);

/* ---- elliptic solve without device allocation ------------------------- */

/* Bytes of the fixed device scratch of nspnp_poisson_solve_noalloc. */
#define NSPNP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of nspnp_poisson_solve (same kinds, operators, layouts and kernels) on the
 * grid of cfg (nx, ny, nz, lx, lz, stretch; the other fields are checked but
 * not used), with no handle and no workspace.  rhs and out are caller-owned
 * FP64 device arrays of nx*nz*(ny-1) cell values (may alias); hip_stream is
 * a hipStream_t (NULL: the null stream); the current device is used.
 * Scratch: a fixed array of NSPNP_NOALLOC_SCRATCH_BYTES in device memory,
 * one per GPU, held from the library's first use on that GPU until the
 * process ends; it takes the grid tables, the Thomas pivots of both
 * operators and one half spectrum, 48 (nx/2+1) nz (ny-1) bytes plus the
 * tables, and a grid needing more is refused with NSPNP_ERR_SIZE.  The call
 * allocates no device memory.  The first call on a GPU, and any call whose
 * grid differs from the previous call's on that GPU, writes the tables and
 * pivots into the scratch and synchronises the stream (do it outside a
 * graph capture); later calls with the same grid only queue the solve
 * kernels (asynchronous).  Every call on a GPU shares that GPU's scratch:
 * calls whose work overlaps on one GPU (other streams, other host threads
 * before the earlier work has finished) race and give wrong results.
 */
NSPNP_API int nspnp_poisson_solve_noalloc(const nspnp_config *cfg, int32_t kind, const double *dev_rhs,
                                          double *dev_out, void *hip_stream);

/* Wait for all queued work of this state. */
NSPNP_API int nspnp_sync(nspnp_state *s);

/* Release the host handle (the workspace stays the caller's). */
NSPNP_API void nspnp_destroy(nspnp_state *s);

/* Message of the last failed call on this thread ("" if none). */
NSPNP_API const char *nspnp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NSPNP_H */
