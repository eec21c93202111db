/*
 * nspnp_oracle.c -- plain FP64 CPU reference solver for the coupled
 * Navier-Stokes / Poisson-Nernst-Planck (NS-PNP) plane-Couette problem of
 * Ostilla-Monico & Lee, "Controlling turbulent drag across electrolytes using
 * electric fields" (arXiv:1701.02005).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It is slow on purpose: every operator is a plain loop
 * nest that follows the paper's statement of the equations (Sec. II,
 * Eqs. (1)-(4)), its staggered arrangement (Fig. 1) and its elliptic solver
 * (Sec. II: Fourier transform in the two periodic directions, Thomas
 * algorithm across the gap).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the GPU library.
 *
 * Nondimensional equations (scales h, U, h/U, c0, V_T, rho_w U^2), derived
 * from Eqs. (1)-(4) with the control groups of Sec. II (Debye length, beta,
 * Sc, Vhat, Re):
 *     du/dt + div(u u) = -grad p + Re^-1 lap u + sF*K*(c+ - c-) grad Phi
 *     div u = 0
 *     dc+-/dt + div(u c+-) = (Re Sc)^-1 div(grad c+- +- c+- grad Phi)
 *     lap phi = -(c+ - c-)/(2 lam^2),  phi(+-1) = 0,  Phi = (Vhat/2) y + phi
 * with K = beta/(2 Sc Re^2 lam^2) and lam = lambda_D/h.  sF = -1 gives the
 * physical Coulomb force rho*E = -rho grad Phi; sF = +1 follows the sign as
 * printed in Eq. (1).  Walls at y = -1 (velocity u_bot) and y = +1 (u_top);
 * no-slip, no-penetration, zero total ion flux (Fig. 1 caption), fixed
 * potential +-Vhat/2 (Phi_0 = V y / h, Sec. II).
 *
 * Discretisation (Sec. II, Fig. 1): second-order central differences on a
 * staggered mesh.  Cell (i,j,k), i < nx, j < M = ny-1, k < nz.  p, c+-, phi
 * at cell centres; u on x-faces (x = i dx), v on y-nodes (y = yn[j], j < M;
 * v[j=0] is the bottom wall and stays 0, the top wall node M is implicit 0),
 * w on z-faces (z = k dz); ion fluxes on the faces of the matching direction.
 * Arrays are [j][k][i] with i fastest.  x and z are periodic and uniform; y
 * nodes are tanh-stretched: yn[j] = tanh(g xi_j)/tanh(g), xi_j = -1 + 2j/M.
 *
 * Time integration (Sec. II): low-storage three-stage Runge-Kutta for the
 * explicit terms with coefficients gamma = (8/15, 5/12, 3/4),
 * zeta = (0, -17/60, -5/12), alpha = gamma + zeta; wall-normal diffusion of
 * velocity and ions is implicit (Crank-Nicolson) and solved as tridiagonal
 * systems; incompressibility by an incremental projection-correction; the
 * potential perturbation is solved after the ion update of every substep.
 */
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* configuration and state                                              */
/* ------------------------------------------------------------------ */

typedef struct {
    double lx, lz;        /* periodic lengths in units of h                */
    double stretch;       /* tanh clustering factor g of the y nodes       */
    double re, sc, beta;  /* Reynolds, Schmidt, dielectric coupling        */
    double debye;         /* lam = lambda_D / h                            */
    double vhat;          /* 2 V / V_T: wall potentials are +-vhat/2       */
    double u_top, u_bot;  /* wall velocities                               */
    double force_sign;    /* sF, -1 physical, +1 as printed                */
    double dt;            /* > 0: fixed full RK step; <= 0: adaptive       */
    double cfl;           /* CFL number for the adaptive step              */
    int32_t nx, ny, nz;   /* ny = number of wall-normal NODES              */
    int32_t implicit_xz;  /* 1: diffusion implicit in x and z too, by the
                             three-direction approximate factorisation    */
    int32_t migration_face; /* face value of c in the migration flux:
                               0 the unweighted mean of the two cells,
                               1 hybrid: the upwind cell of the species'
                               drift on faces whose potential difference
                               is at least 2, the mean elsewhere;
                               2 as 1, and the advective face value of c
                               limited (or_adv_face)                      */
} or_config;

enum { F_U = 0, F_V, F_W, F_CP, F_CM, F_PHI, F_P, F_NFIELD };

typedef struct {
    or_config cfg;
    int nx, nz, M, ny;
    double dx, dz;
    double *yn, *yc, *dn, *dc;  /* dc[0..M]: centre-to-centre distance at node j */
    double *f[F_NFIELD];        /* state fields, each M*nz*nx                    */
    double *hold[5];            /* H^{k-1} of u, v, w, c+, c-                    */
    double t, dt;
    int stage;                  /* 0,1,2: next RK stage                          */
    long long substeps;
    double *phiw[2];            /* wall values of phi (lower, upper wall), nz*nx
                                   each, x fastest; NULL: zero (uniform walls)  */
} or_solver;

#define IDX(s, i, j, k) ((size_t)(i) + (size_t)(s)->nx * ((size_t)(k) + (size_t)(s)->nz * (size_t)(j)))

static const double RK_GAMMA[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
static const double RK_ZETA[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

static double or_alpha(int k) { return RK_GAMMA[k] + RK_ZETA[k]; }

size_t or_ncell(const or_solver *s) { return (size_t)s->nx * s->nz * s->M; }

/* ------------------------------------------------------------------ */
/* grid                                                                 */
/* ------------------------------------------------------------------ */

static void or_build_grid(or_solver *s) {
    int M = s->M;
    double g = s->cfg.stretch;
    for (int j = 0; j <= M; j++) {
        double xi = -1.0 + 2.0 * (double)j / (double)M;
        s->yn[j] = (g > 0.0) ? tanh(g * xi) / tanh(g) : xi;
    }
    s->yn[0] = -1.0;
    s->yn[M] = 1.0;
    for (int j = 0; j < M; j++) {
        s->yc[j] = 0.5 * (s->yn[j] + s->yn[j + 1]);
        s->dn[j] = s->yn[j + 1] - s->yn[j];
    }
    s->dc[0] = s->yc[0] - s->yn[0];
    for (int j = 1; j < M; j++) s->dc[j] = s->yc[j] - s->yc[j - 1];
    s->dc[M] = s->yn[M] - s->yc[M - 1];
}

or_solver *or_create(const or_config *cfg) {
    if (cfg->nx < 1 || cfg->nz < 1 || cfg->ny < 3) return NULL;
    or_solver *s = (or_solver *)calloc(1, sizeof(or_solver));
    s->cfg = *cfg;
    s->nx = cfg->nx;
    s->nz = cfg->nz;
    s->ny = cfg->ny;
    s->M = cfg->ny - 1;
    s->dx = cfg->lx / cfg->nx;
    s->dz = cfg->lz / cfg->nz;
    s->yn = (double *)calloc(s->M + 1, sizeof(double));
    s->yc = (double *)calloc(s->M, sizeof(double));
    s->dn = (double *)calloc(s->M, sizeof(double));
    s->dc = (double *)calloc(s->M + 1, sizeof(double));
    size_t n = or_ncell(s);
    for (int q = 0; q < F_NFIELD; q++) s->f[q] = (double *)calloc(n, sizeof(double));
    for (int q = 0; q < 5; q++) s->hold[q] = (double *)calloc(n, sizeof(double));
    or_build_grid(s);
    s->dt = cfg->dt;
    return s;
}

void or_destroy(or_solver *s) {
    if (!s) return;
    free(s->yn); free(s->yc); free(s->dn); free(s->dc);
    for (int q = 0; q < F_NFIELD; q++) free(s->f[q]);
    for (int q = 0; q < 5; q++) free(s->hold[q]);
    free(s->phiw[0]); free(s->phiw[1]);
    free(s);
}

double *or_field(or_solver *s, int id) { return (id >= 0 && id < F_NFIELD) ? s->f[id] : NULL; }
double *or_hold(or_solver *s, int id) { return (id >= 0 && id < 5) ? s->hold[id] : NULL; }
const double *or_yn(const or_solver *s) { return s->yn; }
const double *or_yc(const or_solver *s) { return s->yc; }
const double *or_dn(const or_solver *s) { return s->dn; }
const double *or_dc(const or_solver *s) { return s->dc; }
double or_time(const or_solver *s) { return s->t; }
double or_get_dt(const or_solver *s) { return s->dt; }
int or_stage(const or_solver *s) { return s->stage; }
void or_set_clock(or_solver *s, double t, double dt, int stage) { s->t = t; s->dt = dt; s->stage = stage; }

/* Coulomb coupling K = beta / (2 Sc Re^2 lam^2): Eq. (1) scaled by rho_w U^2/h
 * with e c0 = eps V_T / (2 lambda_D^2) (Debye length definition, Sec. II),
 * eps V_T^2 = beta eta D (beta definition) and D = eta/(rho_w Sc). */
double or_coulomb_k(const or_config *c) {
    return c->beta / (2.0 * c->sc * c->re * c->re * c->debye * c->debye);
}

/* ------------------------------------------------------------------ */
/* counter-based random numbers: SplitMix64 (Steele, Lea & Flood,       */
/* OOPSLA 2014).  The n-th output for seed s is mix(s + n*golden).      */
/* ------------------------------------------------------------------ */

static uint64_t or_splitmix(uint64_t seed, uint64_t n) {
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* raw n-th output, exported for the published test vector */
uint64_t or_splitmix_raw(uint64_t seed, uint64_t n) { return or_splitmix(seed, n); }

/* uniform in [-1, 1) for (field id, linear index) */
double or_noise(uint64_t seed, int field, uint64_t lin) {
    uint64_t n = ((uint64_t)field << 40) + lin + 1ULL;
    double u01 = (double)(or_splitmix(seed, n) >> 11) * (1.0 / 9007199254740992.0);
    return 2.0 * u01 - 1.0;
}

/* ------------------------------------------------------------------ */
/* FFT: textbook recursive mixed-radix Cooley-Tukey (decimation in      */
/* time), radices 2 and 3, direct DFT for any other factor.  The        */
/* twiddle table holds W^m = exp(sign 2 pi i m / n) of the top length n; */
/* a sub-transform of length n/ts reads it with stride ts.              */
/* sign = -1 forward, +1 inverse (unnormalised).                        */
/* ------------------------------------------------------------------ */

static void or_fft_rec(int n, int stride, const double *xr, const double *xi, double *yr, double *yi,
                       const double *wr, const double *wi, int ts, double *tr, double *ti) {
    int ntop = n * ts;
    if (n == 1) { yr[0] = xr[0]; yi[0] = xi[0]; return; }
    int p = (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : n;
    int m = n / p;
    if (m == 1) { /* direct DFT of length p */
        for (int k = 0; k < n; k++) {
            double sr = 0.0, si = 0.0;
            for (int r = 0; r < n; r++) {
                int e = (int)(((long long)k * r % n) * ts % ntop);
                double ar = xr[(size_t)r * stride], ai = xi[(size_t)r * stride];
                sr += ar * wr[e] - ai * wi[e];
                si += ar * wi[e] + ai * wr[e];
            }
            yr[k] = sr; yi[k] = si;
        }
        return;
    }
    /* sub-transforms Y_r of the p decimated sequences x[p q + r], into t */
    for (int r = 0; r < p; r++)
        or_fft_rec(m, stride * p, xr + (size_t)r * stride, xi + (size_t)r * stride, tr + (size_t)r * m,
                   ti + (size_t)r * m, wr, wi, ts * p, yr, yi);
    /* combine: X[k] = sum_r W_n^{r k} Y_r[k mod m] */
    for (int k = 0; k < n; k++) {
        double sr = 0.0, si = 0.0;
        for (int r = 0; r < p; r++) {
            int e = (int)(((long long)r * k % n) * ts % ntop);
            double ar = tr[(size_t)r * m + k % m], ai = ti[(size_t)r * m + k % m];
            sr += ar * wr[e] - ai * wi[e];
            si += ar * wi[e] + ai * wr[e];
        }
        yr[k] = sr; yi[k] = si;
    }
}

typedef struct { int n; double *wr, *wi, *xr, *xi, *yr, *yi, *tr, *ti; } or_fft_plan;

static void or_fft_plan_init(or_fft_plan *pl, int n, int sign) {
    pl->n = n;
    pl->wr = (double *)malloc(8 * (size_t)n * sizeof(double));
    pl->wi = pl->wr + n; pl->xr = pl->wi + n; pl->xi = pl->xr + n;
    pl->yr = pl->xi + n; pl->yi = pl->yr + n; pl->tr = pl->yi + n; pl->ti = pl->tr + n;
    for (int m = 0; m < n; m++) {
        pl->wr[m] = cos(2.0 * M_PI * m / n);
        pl->wi[m] = sign * sin(2.0 * M_PI * m / n);
    }
}

static void or_fft_plan_free(or_fft_plan *pl) { free(pl->wr); }

/* in-place complex transform of one line */
static void or_fft_line(or_fft_plan *pl, double *re, double *im) {
    int n = pl->n;
    memcpy(pl->xr, re, n * sizeof(double));
    memcpy(pl->xi, im, n * sizeof(double));
    or_fft_rec(n, 1, pl->xr, pl->xi, pl->yr, pl->yi, pl->wr, pl->wi, 1, pl->tr, pl->ti);
    memcpy(re, pl->yr, n * sizeof(double));
    memcpy(im, pl->yi, n * sizeof(double));
}

/* exported for tests: complex DFT of one line */
void or_fft(int n, double *re, double *im, int sign) {
    or_fft_plan pl;
    or_fft_plan_init(&pl, n, sign);
    or_fft_line(&pl, re, im);
    or_fft_plan_free(&pl);
}

/* ------------------------------------------------------------------ */
/* Thomas algorithm (no pivoting) for a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j,
 * real coefficients, complex right-hand side.  a[0], c[n-1] are ignored.   */
/* ------------------------------------------------------------------ */

void or_thomas(int n, const double *a, const double *b, const double *c, double *dr, double *di) {
    double *cp = (double *)malloc(n * sizeof(double));
    double den = b[0];
    cp[0] = c[0] / den;
    dr[0] /= den; di[0] /= den;
    for (int j = 1; j < n; j++) {
        den = b[j] - a[j] * cp[j - 1];
        cp[j] = (j < n - 1) ? c[j] / den : 0.0;
        dr[j] = (dr[j] - a[j] * dr[j - 1]) / den;
        di[j] = (di[j] - a[j] * di[j - 1]) / den;
    }
    for (int j = n - 2; j >= 0; j--) {
        dr[j] -= cp[j] * dr[j + 1];
        di[j] -= cp[j] * di[j + 1];
    }
    free(cp);
}

/* ------------------------------------------------------------------ */
/* wall-normal second-difference operator L_y (finite-volume form)      */
/* ------------------------------------------------------------------ */

/* Coefficients of L_y on cell-centred data, row j < M:
 *   L_y q_j = lo_j q_{j-1} + di_j q_j + up_j q_{j+1} (+ wall terms)
 * bc = 0: Neumann (zero flux through the wall faces)  -- c+-, pressure
 * bc = 1: Dirichlet, wall value at distance dc[0] / dc[M] -- u, w, phi  */
static void or_ly_centre(const or_solver *s, int bc, double *lo, double *di, double *up) {
    int M = s->M;
    for (int j = 0; j < M; j++) {
        double a = 1.0 / (s->dn[j] * s->dc[j]);
        double c = 1.0 / (s->dn[j] * s->dc[j + 1]);
        lo[j] = (j > 0) ? a : 0.0;
        up[j] = (j < M - 1) ? c : 0.0;
        di[j] = -(lo[j] + up[j]);
        if (bc == 1 && j == 0) di[j] -= a;
        if (bc == 1 && j == M - 1) di[j] -= c;
    }
}

/* Coefficients of L_y on node data v_j, j = 1..M-1 (v_0 = v_M = 0),
 * stored at row index j (rows 0 unused). */
static void or_ly_node(const or_solver *s, double *lo, double *di, double *up) {
    int M = s->M;
    lo[0] = di[0] = up[0] = 0.0;
    for (int j = 1; j < M; j++) {
        double a = 1.0 / (s->dc[j] * s->dn[j - 1]);
        double c = 1.0 / (s->dc[j] * s->dn[j]);
        lo[j] = (j > 1) ? a : 0.0;
        up[j] = (j < M - 1) ? c : 0.0;
        di[j] = -(a + c);
    }
}

/* L_y of a cell-centred field with wall values (qbot, qtop) for bc = 1 */
static void or_apply_ly_centre(const or_solver *s, const double *q, int bc, double qbot, double qtop, double *out) {
    int M = s->M;
#pragma omp parallel for
    for (int j = 0; j < M; j++) {
        for (int k = 0; k < s->nz; k++) {
            for (int i = 0; i < s->nx; i++) {
                double qj = q[IDX(s, i, j, k)];
                double fb, ft; /* diffusive fluxes through the bottom / top faces */
                if (j > 0) fb = (qj - q[IDX(s, i, j - 1, k)]) / s->dc[j];
                else fb = (bc == 1) ? (qj - qbot) / s->dc[0] : 0.0;
                if (j < M - 1) ft = (q[IDX(s, i, j + 1, k)] - qj) / s->dc[j + 1];
                else ft = (bc == 1) ? (qtop - qj) / s->dc[M] : 0.0;
                out[IDX(s, i, j, k)] = (ft - fb) / s->dn[j];
            }
        }
    }
}

/* L_y of node field v (v_0 = v_M = 0); out at rows 1..M-1, row 0 set 0 */
static void or_apply_ly_node(const or_solver *s, const double *v, double *out) {
    int M = s->M;
#pragma omp parallel for
    for (int j = 0; j < M; j++) {
        for (int k = 0; k < s->nz; k++) {
            for (int i = 0; i < s->nx; i++) {
                if (j == 0) { out[IDX(s, i, 0, k)] = 0.0; continue; }
                double vj = v[IDX(s, i, j, k)];
                double vb = (j > 1) ? v[IDX(s, i, j - 1, k)] : 0.0;
                double vt = (j < M - 1) ? v[IDX(s, i, j + 1, k)] : 0.0;
                double ft = (vt - vj) / s->dn[j];
                double fb = (vj - vb) / s->dn[j - 1];
                out[IDX(s, i, j, k)] = (ft - fb) / s->dc[j];
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* explicit terms                                                       */
/* ------------------------------------------------------------------ */

#define PX(i) (((i) + 1) % s->nx)
#define MX(i) (((i) - 1 + s->nx) % s->nx)
#define PZ(k) (((k) + 1) % s->nz)
#define MZ(k) (((k) - 1 + s->nz) % s->nz)

/* Momentum convection C(u) = div(u u) in divergence form on the staggered
 * mesh: the flux through each face of a velocity control volume is the
 * face-area-weighted advecting velocity, the advected velocity is the
 * unweighted mean of the two neighbouring control volumes.  For a discretely
 * divergence-free field this makes sum(u . C(u) Omega) = 0 (energy-neutral
 * convection; Verstappen & Veldman, J. Comput. Phys. 187 (2003)). */
void or_convection(const or_solver *s, const double *u, const double *v, const double *w,
                   double *cu, double *cv, double *cw) {
    int M = s->M;
    double dx = s->dx, dz = s->dz;
#pragma omp parallel for
    for (int j = 0; j < M; j++) {
        for (int k = 0; k < s->nz; k++) {
            for (int i = 0; i < s->nx; i++) {
                int ip = PX(i), im = MX(i), kp = PZ(k), km = MZ(k);
                size_t c0 = IDX(s, i, j, k);
                /* ---- u at (x_i face, row j, z-cell k) ---- */
                {
                    double uu_r = 0.5 * (u[IDX(s, ip, j, k)] + u[c0]);
                    double uu_l = 0.5 * (u[c0] + u[IDX(s, im, j, k)]);
                    double cx = (uu_r * uu_r - uu_l * uu_l) / dx;
                    double vt = (j + 1 < M) ? 0.5 * (v[IDX(s, i, j + 1, k)] + v[IDX(s, im, j + 1, k)]) : 0.0;
                    double vb = (j > 0) ? 0.5 * (v[c0] + v[IDX(s, im, j, k)]) : 0.0;
                    double ut = (j + 1 < M) ? 0.5 * (u[IDX(s, i, j + 1, k)] + u[c0]) : 0.0;
                    double ub = (j > 0) ? 0.5 * (u[c0] + u[IDX(s, i, j - 1, k)]) : 0.0;
                    double cy = (vt * ut - vb * ub) / s->dn[j];
                    double wf = 0.5 * (w[IDX(s, i, j, kp)] + w[IDX(s, im, j, kp)]);
                    double wb = 0.5 * (w[c0] + w[IDX(s, im, j, k)]);
                    double cz = (wf * 0.5 * (u[IDX(s, i, j, kp)] + u[c0]) - wb * 0.5 * (u[c0] + u[IDX(s, i, j, km)])) / dz;
                    cu[c0] = cx + cy + cz;
                }
                /* ---- w at (x-cell i, row j, z_k face) ---- */
                {
                    double ww_f = 0.5 * (w[IDX(s, i, j, kp)] + w[c0]);
                    double ww_b = 0.5 * (w[c0] + w[IDX(s, i, j, km)]);
                    double cz = (ww_f * ww_f - ww_b * ww_b) / dz;
                    double ur = 0.5 * (u[IDX(s, ip, j, k)] + u[IDX(s, ip, j, km)]);
                    double ul = 0.5 * (u[c0] + u[IDX(s, i, j, km)]);
                    double cx = (ur * 0.5 * (w[IDX(s, ip, j, k)] + w[c0]) - ul * 0.5 * (w[c0] + w[IDX(s, im, j, k)])) / dx;
                    double vt = (j + 1 < M) ? 0.5 * (v[IDX(s, i, j + 1, k)] + v[IDX(s, i, j + 1, km)]) : 0.0;
                    double vb = (j > 0) ? 0.5 * (v[c0] + v[IDX(s, i, j, km)]) : 0.0;
                    double wt = (j + 1 < M) ? 0.5 * (w[IDX(s, i, j + 1, k)] + w[c0]) : 0.0;
                    double wb = (j > 0) ? 0.5 * (w[c0] + w[IDX(s, i, j - 1, k)]) : 0.0;
                    double cy = (vt * wt - vb * wb) / s->dn[j];
                    cw[c0] = cx + cy + cz;
                }
                /* ---- v at (x-cell i, node j, z-cell k), j >= 1 ---- */
                if (j == 0) {
                    cv[c0] = 0.0;
                } else {
                    double dcj = s->dc[j];
                    double vj = v[c0];
                    double vtop = (j + 1 < M) ? v[IDX(s, i, j + 1, k)] : 0.0;
                    double vbot = (j - 1 > 0) ? v[IDX(s, i, j - 1, k)] : 0.0;
                    double vv_t = 0.5 * (vtop + vj), vv_b = 0.5 * (vj + vbot);
                    double cy = (vv_t * vv_t - vv_b * vv_b) / dcj;
                    double wl = s->dn[j - 1], wu = s->dn[j];
                    /* volume-weighted advecting velocities on the v control volume faces */
                    double ur = (u[IDX(s, ip, j - 1, k)] * wl + u[IDX(s, ip, j, k)] * wu) / (2.0 * dcj);
                    double ul = (u[IDX(s, i, j - 1, k)] * wl + u[c0] * wu) / (2.0 * dcj);
                    double cx = (ur * 0.5 * (v[IDX(s, ip, j, k)] + vj) - ul * 0.5 * (vj + v[IDX(s, im, j, k)])) / dx;
                    double wf = (w[IDX(s, i, j - 1, kp)] * wl + w[IDX(s, i, j, kp)] * wu) / (2.0 * dcj);
                    double wb = (w[IDX(s, i, j - 1, k)] * wl + w[c0] * wu) / (2.0 * dcj);
                    double cz = (wf * 0.5 * (v[IDX(s, i, j, kp)] + vj) - wb * 0.5 * (vj + v[IDX(s, i, j, km)])) / dz;
                    cv[c0] = cx + cy + cz;
                }
            }
        }
    }
}

/* Horizontal (x, z) Laplacian, periodic three-point */
void or_lap_xz(const or_solver *s, const double *q, double *out) {
    double ix2 = 1.0 / (s->dx * s->dx), iz2 = 1.0 / (s->dz * s->dz);
#pragma omp parallel for
    for (int j = 0; j < s->M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                double q0 = q[IDX(s, i, j, k)];
                out[IDX(s, i, j, k)] = (q[IDX(s, PX(i), j, k)] - 2.0 * q0 + q[IDX(s, MX(i), j, k)]) * ix2 +
                                       (q[IDX(s, i, j, PZ(k))] - 2.0 * q0 + q[IDX(s, i, j, MZ(k))]) * iz2;
            }
}

/* Coulomb body force sF K rho grad(Phi) at the velocity points, with
 * rho = c+ - c- averaged (unweighted) to the face and the total potential
 * Phi = (vhat/2) y + phi differenced across it (Eq. (1), Sec. II). */
void or_coulomb(const or_solver *s, const double *cp, const double *cm, const double *phi,
                double *fu, double *fv, double *fw) {
    double kf = s->cfg.force_sign * or_coulomb_k(&s->cfg);
    double e0 = 0.5 * s->cfg.vhat; /* d Phi_0 / dy */
#pragma omp parallel for
    for (int j = 0; j < s->M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k), cxm = IDX(s, MX(i), j, k), czm = IDX(s, i, j, MZ(k));
                double r0 = cp[c0] - cm[c0];
                fu[c0] = kf * 0.5 * (r0 + cp[cxm] - cm[cxm]) * (phi[c0] - phi[cxm]) / s->dx;
                fw[c0] = kf * 0.5 * (r0 + cp[czm] - cm[czm]) * (phi[c0] - phi[czm]) / s->dz;
                if (j == 0) fv[c0] = 0.0;
                else {
                    size_t cym = IDX(s, i, j - 1, k);
                    double ey = e0 + (phi[c0] - phi[cym]) / s->dc[j];
                    fv[c0] = kf * 0.5 * (r0 + cp[cym] - cm[cym]) * ey;
                }
            }
}

/* Face value of c in the migration flux of a species of valence zs across a
 * face with potential difference dphi = Phi_R - Phi_L (cell R on the side of
 * increasing index).  Sec. II gives second-order central differences, whose
 * face value is the mean of the two cells.  At equilibrium that value makes
 * the cell ratio c_R / c_L = (1 - zs dphi / 2) / (1 + zs dphi / 2), which is
 * negative once |dphi| > 2 (the cell Peclet number of migration).  The hybrid
 * rule takes, on such faces, the cell the drift comes from: the drift
 * velocity of the species is -zs (Re Sc)^-1 grad Phi, so the upwind cell is R
 * when zs dphi > 0 and L otherwise; its equilibrium ratio 1 / (1 + zs dphi)
 * or 1 + |dphi| stays positive. */
static double or_mig_face(const or_solver *s, double cL, double cR, double dphi, double zs) {
    if (s->cfg.migration_face >= 1 && fabs(dphi) >= 2.0) return (zs * dphi > 0.0) ? cR : cL;
    return 0.5 * (cL + cR);
}

/* Advective face value of c.  Sec. II's central differences take the mean of
 * the two cells; at the ions' cell Peclet numbers of a turbulent run
 * (Re Sc |u| dx ~ 10^2) that value lets a transported profile overshoot, and
 * steep near-wall layers go negative.  The limited value (migration_face 2)
 * starts from the upwind cell U of the face velocity and adds the van Leer
 * slope: with a = c_U - c_UU and b = c_D - c_U (D the downwind cell, UU the
 * cell beyond U), c_face = c_U + a b / (a + b) when a b > 0, else c_U.  On a
 * linear profile of equal spacings a = b and this is the mean; at an extremum
 * it is the upwind value, so no new extrema form.  vel_up: the face velocity
 * is >= 0 (U on the low-index side).  have_uu = 0 (U is a wall row): the
 * cell beyond the wall is taken as an image of U (zero gradient, as the
 * wall's zero normal flux has it), so a = 0 and the face value is c_U. */
static double or_adv_face(const or_solver *s, double cL, double cR, double cUU, int vel_up, int have_uu) {
    if (s->cfg.migration_face != 2) return 0.5 * (cL + cR);
    double cU = vel_up ? cL : cR, cD = vel_up ? cR : cL;
    if (!have_uu) return cU;
    double a = cU - cUU, b = cD - cU;
    return (a * b > 0.0) ? cU + a * b / (a + b) : cU;
}

/* Ion transport terms for one species of valence zs = +1 / -1 except the
 * implicit wall-normal diffusion:
 *   -div(u c) + (Re Sc)^-1 [ (Lxx + Lzz) c + zs div(c_face grad Phi) ]
 * Migration fluxes live on the cell faces (Fig. 1) and are exactly zero on
 * the two wall faces, as are the advective fluxes (v = 0 there). */
void or_ion_explicit(const or_solver *s, const double *u, const double *v, const double *w, const double *c,
                     const double *phi, double zs, double *out) {
    int M = s->M;
    double dx = s->dx, dz = s->dz;
    double kd = 1.0 / (s->cfg.re * s->cfg.sc);
    double e0 = 0.5 * s->cfg.vhat;
#pragma omp parallel for
    for (int j = 0; j < M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                int ip = PX(i), im = MX(i), kp = PZ(k), km = MZ(k);
                size_t c0 = IDX(s, i, j, k);
                double cc = c[c0];
                double cxp = c[IDX(s, ip, j, k)], cxm = c[IDX(s, im, j, k)];
                double czp = c[IDX(s, i, j, kp)], czm = c[IDX(s, i, j, km)];
                double cxp2 = c[IDX(s, PX(ip), j, k)], cxm2 = c[IDX(s, MX(im), j, k)];
                double czp2 = c[IDX(s, i, j, PZ(kp))], czm2 = c[IDX(s, i, j, MZ(km))];
                /* advection: face velocity times face value (the mean, or the
                 * limited upwind value; periodic in x and z) */
                double uR = u[IDX(s, ip, j, k)], uL = u[c0];
                double wF = w[IDX(s, i, j, kp)], wB = w[c0];
                double ax = (uR * or_adv_face(s, cc, cxp, uR >= 0.0 ? cxm : cxp2, uR >= 0.0, 1) -
                             uL * or_adv_face(s, cxm, cc, uL >= 0.0 ? cxm2 : cxp, uL >= 0.0, 1)) / dx;
                double az = (wF * or_adv_face(s, cc, czp, wF >= 0.0 ? czm : czp2, wF >= 0.0, 1) -
                             wB * or_adv_face(s, czm, cc, wB >= 0.0 ? czm2 : czp, wB >= 0.0, 1)) / dz;
                double vt = 0.0, vb = 0.0, ft = 0.0, fb = 0.0;
                /* potential differences across the faces (y: applied field
                 * e0 over the centre distance plus the perturbation) */
                if (j + 1 < M) {
                    size_t cu = IDX(s, i, j + 1, k);
                    double cup = c[cu];
                    double dpy = e0 * s->dc[j + 1] + (phi[cu] - phi[c0]);
                    int up = v[cu] >= 0.0;  /* U = row j (UU = j - 1), else U = j + 1 (UU = j + 2) */
                    int have = up ? (j > 0) : (j + 2 < M);
                    double cuu = have ? c[IDX(s, i, up ? j - 1 : j + 2, k)] : 0.0;
                    vt = v[cu] * or_adv_face(s, cc, cup, cuu, up, have);
                    ft = or_mig_face(s, cc, cup, dpy, zs) * (e0 + (phi[cu] - phi[c0]) / s->dc[j + 1]);
                }
                if (j > 0) {
                    size_t cd = IDX(s, i, j - 1, k);
                    double cdn = c[cd];
                    double dpy = e0 * s->dc[j] + (phi[c0] - phi[cd]);
                    int up = v[c0] >= 0.0;  /* U = row j - 1 (UU = j - 2), else U = j (UU = j + 1) */
                    int have = up ? (j > 1) : (j + 1 < M);
                    double cuu = have ? c[IDX(s, i, up ? j - 2 : j + 1, k)] : 0.0;
                    vb = v[c0] * or_adv_face(s, cdn, cc, cuu, up, have);
                    fb = or_mig_face(s, cdn, cc, dpy, zs) * (e0 + (phi[c0] - phi[cd]) / s->dc[j]);
                }
                double ay = (vt - vb) / s->dn[j];
                /* migration: face concentration times face potential gradient */
                double dpxp = phi[IDX(s, ip, j, k)] - phi[c0], dpxm = phi[c0] - phi[IDX(s, im, j, k)];
                double dpzp = phi[IDX(s, i, j, kp)] - phi[c0], dpzm = phi[c0] - phi[IDX(s, i, j, km)];
                double mx = (or_mig_face(s, cc, cxp, dpxp, zs) * dpxp / dx -
                             or_mig_face(s, cxm, cc, dpxm, zs) * dpxm / dx) / dx;
                double mz = (or_mig_face(s, cc, czp, dpzp, zs) * dpzp / dz -
                             or_mig_face(s, czm, cc, dpzm, zs) * dpzm / dz) / dz;
                double my = (ft - fb) / s->dn[j];
                double dxx = (cxp - 2.0 * cc + cxm) / (dx * dx) + (czp - 2.0 * cc + czm) / (dz * dz);
                if (s->cfg.implicit_xz) dxx = 0.0; /* treated implicitly (or_substep) */
                out[c0] = -(ax + ay + az) + kd * (dxx + zs * (mx + my + mz));
            }
}

/* All explicit right-hand sides H of one RK stage */
void or_explicit_terms(const or_solver *s, double *hu, double *hv, double *hw, double *hcp, double *hcm) {
    size_t n = or_ncell(s);
    const double *u = s->f[F_U], *v = s->f[F_V], *w = s->f[F_W];
    const double *cp = s->f[F_CP], *cm = s->f[F_CM], *phi = s->f[F_PHI];
    double *lu = (double *)malloc(3 * n * sizeof(double)), *lv = lu + n, *lw = lv + n;
    double *fu = (double *)malloc(3 * n * sizeof(double)), *fv = fu + n, *fw = fv + n;
    double ire = 1.0 / s->cfg.re;
    or_convection(s, u, v, w, hu, hv, hw);
    or_lap_xz(s, u, lu);
    or_lap_xz(s, v, lv);
    or_lap_xz(s, w, lw);
    or_coulomb(s, cp, cm, phi, fu, fv, fw);
    /* with the three-direction factorisation the x/z diffusion is implicit */
    double ixz = s->cfg.implicit_xz ? 0.0 : ire;
    for (size_t q = 0; q < n; q++) {
        hu[q] = -hu[q] + ixz * lu[q] + fu[q];
        hw[q] = -hw[q] + ixz * lw[q] + fw[q];
        hv[q] = -hv[q] + ixz * lv[q] + fv[q];
    }
    /* v on the bottom wall node is not an unknown */
    for (int k = 0; k < s->nz; k++)
        for (int i = 0; i < s->nx; i++) hv[IDX(s, i, 0, k)] = 0.0;
    or_ion_explicit(s, u, v, w, cp, phi, +1.0, hcp);
    or_ion_explicit(s, u, v, w, cm, phi, -1.0, hcm);
    free(lu);
    free(fu);
}

/* ------------------------------------------------------------------ */
/* divergence and gradient                                              */
/* ------------------------------------------------------------------ */

void or_divergence(const or_solver *s, const double *u, const double *v, const double *w, double *out) {
    int M = s->M;
#pragma omp parallel for
    for (int j = 0; j < M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k);
                double vt = (j + 1 < M) ? v[IDX(s, i, j + 1, k)] : 0.0;
                double vb = (j > 0) ? v[c0] : 0.0;
                out[c0] = (u[IDX(s, PX(i), j, k)] - u[c0]) / s->dx + (vt - vb) / s->dn[j] +
                          (w[IDX(s, i, j, PZ(k))] - w[c0]) / s->dz;
            }
}

/* velocity -= scale * grad(psi) at the staggered points; v on the wall untouched */
static void or_sub_gradient(or_solver *s, const double *psi, double scale) {
    double *u = s->f[F_U], *v = s->f[F_V], *w = s->f[F_W];
#pragma omp parallel for
    for (int j = 0; j < s->M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k);
                u[c0] -= scale * (psi[c0] - psi[IDX(s, MX(i), j, k)]) / s->dx;
                w[c0] -= scale * (psi[c0] - psi[IDX(s, i, j, MZ(k))]) / s->dz;
                if (j > 0) v[c0] -= scale * (psi[c0] - psi[IDX(s, i, j - 1, k)]) / s->dc[j];
            }
}

/* ------------------------------------------------------------------ */
/* elliptic solver (Sec. II): DFT in x and z, Thomas in y                */
/* ------------------------------------------------------------------ */

/* Solve (Lxx + Lzz + L_y) out = rhs.
 * kind 0: pressure-type, zero-flux walls; the singular (0,0) mode is pinned
 *         at its first row and the result is shifted to zero volume mean.
 * kind 1: potential-type, zero value on the walls (one-sided half cell).
 * Lxx, Lzz are the periodic three-point operators, whose Fourier symbols are
 * -(2 - 2 cos(2 pi m / N)) / d^2. */
void or_poisson(const or_solver *s, int kind, const double *rhs, double *out) {
    int nx = s->nx, nz = s->nz, M = s->M;
    size_t n = or_ncell(s);
    double *re = (double *)malloc(n * sizeof(double));
    double *im = (double *)calloc(n, sizeof(double));
    memcpy(re, rhs, n * sizeof(double));
    /* forward transform along x, then along z */
#pragma omp parallel
    {
        or_fft_plan px, pz;
        or_fft_plan_init(&px, nx, -1);
        or_fft_plan_init(&pz, nz, -1);
        int nmax = nx > nz ? nx : nz;
        double *lr = (double *)malloc(2 * (size_t)nmax * sizeof(double)), *li = lr + nmax;
#pragma omp for
        for (int jk = 0; jk < M * nz; jk++) {
            int j = jk / nz, k = jk % nz;
            for (int i = 0; i < nx; i++) { lr[i] = re[IDX(s, i, j, k)]; li[i] = im[IDX(s, i, j, k)]; }
            or_fft_line(&px, lr, li);
            for (int i = 0; i < nx; i++) { re[IDX(s, i, j, k)] = lr[i]; im[IDX(s, i, j, k)] = li[i]; }
        }
#pragma omp for
        for (int ji = 0; ji < M * nx; ji++) {
            int j = ji / nx, i = ji % nx;
            for (int k = 0; k < nz; k++) { lr[k] = re[IDX(s, i, j, k)]; li[k] = im[IDX(s, i, j, k)]; }
            or_fft_line(&pz, lr, li);
            for (int k = 0; k < nz; k++) { re[IDX(s, i, j, k)] = lr[k]; im[IDX(s, i, j, k)] = li[k]; }
        }
        or_fft_plan_free(&px);
        or_fft_plan_free(&pz);
        free(lr);
    }
    /* tridiagonal solve in y for every (kx, kz) mode */
    double *lo = (double *)malloc(3 * M * sizeof(double)), *di = lo + M, *up = di + M;
    or_ly_centre(s, kind == 0 ? 0 : 1, lo, di, up);
#pragma omp parallel
    {
        double *b = (double *)malloc(M * sizeof(double));
        double *a = (double *)malloc(M * sizeof(double));
        double *c = (double *)malloc(M * sizeof(double));
        double *dr = (double *)malloc(M * sizeof(double)), *dim = (double *)malloc(M * sizeof(double));
#pragma omp for
        for (int ki = 0; ki < nx * nz; ki++) {
            int k = ki / nx, i = ki % nx;
            double kx2 = (2.0 - 2.0 * cos(2.0 * M_PI * i / nx)) / (s->dx * s->dx);
            double kz2 = (2.0 - 2.0 * cos(2.0 * M_PI * k / nz)) / (s->dz * s->dz);
            for (int j = 0; j < M; j++) {
                a[j] = lo[j];
                c[j] = up[j];
                b[j] = di[j] - kx2 - kz2;
                dr[j] = re[IDX(s, i, j, k)];
                dim[j] = im[IDX(s, i, j, k)];
            }
            if (kind == 0 && i == 0 && k == 0) { /* pin the undetermined constant */
                b[0] = 1.0; c[0] = 0.0; dr[0] = 0.0; dim[0] = 0.0;
            }
            or_thomas(M, a, b, c, dr, dim);
            for (int j = 0; j < M; j++) { re[IDX(s, i, j, k)] = dr[j]; im[IDX(s, i, j, k)] = dim[j]; }
        }
        free(a); free(b); free(c); free(dr); free(dim);
    }
    free(lo);
    /* inverse transforms, z then x */
#pragma omp parallel
    {
        or_fft_plan px, pz;
        or_fft_plan_init(&px, nx, +1);
        or_fft_plan_init(&pz, nz, +1);
        int nmax = nx > nz ? nx : nz;
        double *lr = (double *)malloc(2 * (size_t)nmax * sizeof(double)), *li = lr + nmax;
#pragma omp for
        for (int ji = 0; ji < M * nx; ji++) {
            int j = ji / nx, i = ji % nx;
            for (int k = 0; k < nz; k++) { lr[k] = re[IDX(s, i, j, k)]; li[k] = im[IDX(s, i, j, k)]; }
            or_fft_line(&pz, lr, li);
            for (int k = 0; k < nz; k++) { re[IDX(s, i, j, k)] = lr[k]; im[IDX(s, i, j, k)] = li[k]; }
        }
#pragma omp for
        for (int jk = 0; jk < M * nz; jk++) {
            int j = jk / nz, k = jk % nz;
            for (int i = 0; i < nx; i++) { lr[i] = re[IDX(s, i, j, k)]; li[i] = im[IDX(s, i, j, k)]; }
            or_fft_line(&px, lr, li);
            for (int i = 0; i < nx; i++) { re[IDX(s, i, j, k)] = lr[i]; im[IDX(s, i, j, k)] = li[i]; }
        }
        or_fft_plan_free(&px);
        or_fft_plan_free(&pz);
        free(lr);
    }
    double scale = 1.0 / ((double)nx * (double)nz);
    for (size_t q = 0; q < n; q++) out[q] = re[q] * scale;
    if (kind == 0) { /* zero volume-weighted mean */
        double sum = 0.0, vol = 0.0;
        for (int j = 0; j < M; j++)
            for (int k = 0; k < nz; k++)
                for (int i = 0; i < nx; i++) { sum += out[IDX(s, i, j, k)] * s->dn[j]; vol += s->dn[j]; }
        double mean = sum / vol;
        for (size_t q = 0; q < n; q++) out[q] -= mean;
    }
    free(re);
    free(im);
}

/* ------------------------------------------------------------------ */
/* potential                                                            */
/* ------------------------------------------------------------------ */

/* phi from lap phi = -(c+ - c-)/(2 lam^2) (Sec. II).  The wall potential is
 * -+vhat/2 (the uniform field carried by Phi_0) plus, where set, a wall
 * value g(x, z) of phi itself: the arbitrary (spatially or temporally
 * varying) wall potential the model admits (Sec. II, Sec. V).  With the wall
 * value at the half-cell distance dc, L_y phi at the first row is the
 * homogeneous operator plus g / (dn_0 dc_0) (last row: g / (dn_{M-1} dc_M)),
 * so the homogeneous solve takes rhs - that term. */
void or_solve_potential(or_solver *s) {
    size_t n = or_ncell(s);
    double *rhs = (double *)malloc(n * sizeof(double));
    double sc = -1.0 / (2.0 * s->cfg.debye * s->cfg.debye);
    for (size_t q = 0; q < n; q++) rhs[q] = sc * (s->f[F_CP][q] - s->f[F_CM][q]);
    int M = s->M;
    for (int w = 0; w < 2; w++) {
        if (!s->phiw[w]) continue;
        int j = w == 0 ? 0 : M - 1;
        double coef = w == 0 ? 1.0 / (s->dn[0] * s->dc[0]) : 1.0 / (s->dn[M - 1] * s->dc[M]);
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) rhs[IDX(s, i, j, k)] -= coef * s->phiw[w][(size_t)k * s->nx + i];
    }
    or_poisson(s, 1, rhs, s->f[F_PHI]);
    free(rhs);
}

/* Wall values of phi on the lower and upper wall (nz*nx each, x fastest);
 * NULL clears a wall to zero.  Takes effect at the next potential solve. */
void or_set_wall_potential(or_solver *s, const double *bot, const double *top) {
    const double *src[2] = {bot, top};
    size_t np = (size_t)s->nx * s->nz;
    for (int w = 0; w < 2; w++) {
        free(s->phiw[w]);
        s->phiw[w] = NULL;
        if (src[w]) {
            s->phiw[w] = (double *)malloc(np * sizeof(double));
            memcpy(s->phiw[w], src[w], np * sizeof(double));
        }
    }
}

/* ------------------------------------------------------------------ */
/* time step rule                                                       */
/* ------------------------------------------------------------------ */

/* min of: CFL / max(|u|/dx + |v|/dy + |w|/dz) with velocities averaged to
 * cell centres; the Debye charge-relaxation limit 2 lam^2 Re Sc / max(c+ + c-)
 * of the explicit migration term; the explicit horizontal diffusion limit. */
double or_compute_dt(const or_solver *s) {
    const double *u = s->f[F_U], *v = s->f[F_V], *w = s->f[F_W], *cp = s->f[F_CP], *cm = s->f[F_CM];
    int M = s->M;
    double rate = 0.0, cmax = 0.0;
    for (int j = 0; j < M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k);
                double uc = 0.5 * (u[c0] + u[IDX(s, PX(i), j, k)]);
                double vt = (j + 1 < M) ? v[IDX(s, i, j + 1, k)] : 0.0;
                double vc = 0.5 * (v[c0] + vt);
                double wc = 0.5 * (w[c0] + w[IDX(s, i, j, PZ(k))]);
                double r = fabs(uc) / s->dx + fabs(vc) / s->dn[j] + fabs(wc) / s->dz;
                if (r > rate) rate = r;
                double ct = cp[c0] + cm[c0];
                if (ct > cmax) cmax = ct;
            }
    double re = s->cfg.re, rs = s->cfg.re * s->cfg.sc;
    double dt = 1e30;
    if (rate > 0.0) dt = s->cfg.cfl / rate;
    if (cmax > 0.0) { double d = 2.0 * s->cfg.debye * s->cfg.debye * rs / cmax; if (d < dt) dt = d; }
    double nu_min = (re < rs) ? re : rs;
    double d2 = nu_min / (4.0 / (s->dx * s->dx) + 4.0 / (s->dz * s->dz));
    if (!s->cfg.implicit_xz && d2 < dt) dt = d2; /* no explicit diffusion limit when implicit */
    return dt;
}

/* ------------------------------------------------------------------ */
/* one Runge-Kutta substep                                              */
/* ------------------------------------------------------------------ */

/* Solve (I - beta L_y) x = r column by column, L_y given by (lo, di, up)
 * over rows [j0, M). */
static void or_cn_solve(const or_solver *s, const double *lo, const double *di, const double *up, double beta,
                        int j0, double *r) {
    int M = s->M, n = M - j0;
#pragma omp parallel
    {
        double *a = (double *)malloc(n * sizeof(double)), *b = (double *)malloc(n * sizeof(double));
        double *c = (double *)malloc(n * sizeof(double)), *dr = (double *)malloc(n * sizeof(double));
        double *dz = (double *)calloc(n, sizeof(double));
#pragma omp for
        for (int ki = 0; ki < s->nx * s->nz; ki++) {
            int k = ki / s->nx, i = ki % s->nx;
            for (int q = 0; q < n; q++) {
                int j = j0 + q;
                a[q] = -beta * lo[j];
                b[q] = 1.0 - beta * di[j];
                c[q] = -beta * up[j];
                dr[q] = r[IDX(s, i, j, k)];
                dz[q] = 0.0;
            }
            or_thomas(n, a, b, c, dr, dz);
            for (int q = 0; q < n; q++) r[IDX(s, i, j0 + q, k)] = dr[q];
        }
        free(a); free(b); free(c); free(dr); free(dz);
    }
}

/* Solve (I - beta L_d) x = r along every periodic line of direction d
 * (0: x, 1: z), L_d the three-point operator (q_{+1} - 2 q + q_{-1}) / h^2.
 * The matrix is circulant, so each Fourier mode m of a line is divided by
 * 1 + beta (2 - 2 cos(2 pi m / N)) / h^2 (the three-point symbol). */
void or_xz_solve(const or_solver *s, int d, double beta, double *r) {
    int N = d == 0 ? s->nx : s->nz;
    double h = d == 0 ? s->dx : s->dz;
    int nlines = s->M * (d == 0 ? s->nz : s->nx);
#pragma omp parallel
    {
        or_fft_plan pf, pb;
        or_fft_plan_init(&pf, N, -1);
        or_fft_plan_init(&pb, N, +1);
        double *lr = (double *)malloc(2 * (size_t)N * sizeof(double)), *li = lr + N;
#pragma omp for
        for (int L = 0; L < nlines; L++) {
            int j = L / (d == 0 ? s->nz : s->nx), o = L % (d == 0 ? s->nz : s->nx);
            for (int m = 0; m < N; m++) {
                size_t c = d == 0 ? IDX(s, m, j, o) : IDX(s, o, j, m);
                lr[m] = r[c];
                li[m] = 0.0;
            }
            or_fft_line(&pf, lr, li);
            for (int m = 0; m < N; m++) {
                double sym = 1.0 + beta * (2.0 - 2.0 * cos(2.0 * M_PI * m / N)) / (h * h);
                lr[m] /= sym;
                li[m] /= sym;
            }
            or_fft_line(&pb, lr, li);
            for (int m = 0; m < N; m++) {
                size_t c = d == 0 ? IDX(s, m, j, o) : IDX(s, o, j, m);
                r[c] = lr[m] / N;
            }
        }
        or_fft_plan_free(&pf);
        or_fft_plan_free(&pb);
        free(lr);
    }
}

void or_substep(or_solver *s) {
    int k = s->stage, M = s->M;
    size_t n = or_ncell(s);
    if (k == 0 && s->cfg.dt <= 0.0) s->dt = or_compute_dt(s);
    double dt = s->dt, gam = RK_GAMMA[k], zet = RK_ZETA[k], alp = or_alpha(k);
    double re = s->cfg.re, rs = s->cfg.re * s->cfg.sc;

    /* (ii) explicit right-hand sides H^k */
    double *h[5];
    for (int q = 0; q < 5; q++) h[q] = (double *)malloc(n * sizeof(double));
    or_explicit_terms(s, h[0], h[1], h[2], h[3], h[4]);

    /* (iii) Crank-Nicolson right-hand sides
     *   r = dt [gam H^k + zet H^{k-1} - alp G p^k + alp nu L_y q^k]  */
    double *ly = (double *)malloc(n * sizeof(double));
    double *r = (double *)malloc(n * sizeof(double));
    int imp = s->cfg.implicit_xz;
    double *lxz = imp ? (double *)malloc(n * sizeof(double)) : NULL;
    double *p = s->f[F_P];
    double *lo = (double *)malloc(3 * M * sizeof(double)), *di = lo + M, *up = di + M;
    for (int q = 0; q < 5; q++) {
        double *fq = s->f[q];
        double nu = (q < 3) ? 1.0 / re : 1.0 / rs;
        if (q == F_U) or_apply_ly_centre(s, fq, 1, s->cfg.u_bot, s->cfg.u_top, ly);
        else if (q == F_W) or_apply_ly_centre(s, fq, 1, 0.0, 0.0, ly);
        else if (q == F_V) or_apply_ly_node(s, fq, ly);
        else or_apply_ly_centre(s, fq, 0, 0.0, 0.0, ly);
        /* three-direction factorisation: the x/z diffusion joins the implicit part */
        if (imp) {
            or_lap_xz(s, fq, lxz);
            for (size_t c0 = 0; c0 < n; c0++) ly[c0] += lxz[c0];
            if (q == F_V)
                for (int kk = 0; kk < s->nz; kk++)
                    for (int i = 0; i < s->nx; i++) ly[IDX(s, i, 0, kk)] = 0.0;
        }
        for (int j = 0; j < M; j++)
            for (int kk = 0; kk < s->nz; kk++)
                for (int i = 0; i < s->nx; i++) {
                    size_t c0 = IDX(s, i, j, kk);
                    double gp = 0.0;
                    if (q == F_U) gp = (p[c0] - p[IDX(s, MX(i), j, kk)]) / s->dx;
                    if (q == F_W) gp = (p[c0] - p[IDX(s, i, j, MZ(kk))]) / s->dz;
                    if (q == F_V) gp = (j > 0) ? (p[c0] - p[IDX(s, i, j - 1, kk)]) / s->dc[j] : 0.0;
                    double hold = (k > 0) ? s->hold[q][c0] : 0.0;
                    r[c0] = dt * (gam * h[q][c0] + zet * hold - alp * gp + alp * nu * ly[c0]);
                }
        /* implicit wall-normal diffusion: (I - alp dt nu / 2 L_y) delta = r;
         * factorised: (I - beta L_x)(I - beta L_y)(I - beta L_z) delta = r */
        double beta = 0.5 * alp * dt * nu;
        if (imp) or_xz_solve(s, 0, beta, r);
        if (q == F_V) {
            or_ly_node(s, lo, di, up);
            or_cn_solve(s, lo, di, up, beta, 1, r);
            for (int kk = 0; kk < s->nz; kk++)
                for (int i = 0; i < s->nx; i++) r[IDX(s, i, 0, kk)] = 0.0;
        } else {
            or_ly_centre(s, (q == F_CP || q == F_CM) ? 0 : 1, lo, di, up);
            or_cn_solve(s, lo, di, up, beta, 0, r);
        }
        if (imp) or_xz_solve(s, 1, beta, r);
        for (size_t c0 = 0; c0 < n; c0++) fq[c0] += r[c0];
    }
    free(lo);

    /* (vi) keep H^k for the next stage */
    for (int q = 0; q < 5; q++) { memcpy(s->hold[q], h[q], n * sizeof(double)); free(h[q]); }

    /* (iv) projection: D G psi = D u_hat / (alp dt);  u -= alp dt G psi;
     *      p += psi - (alp dt / (2 Re)) L_y psi */
    or_divergence(s, s->f[F_U], s->f[F_V], s->f[F_W], r);
    for (size_t c0 = 0; c0 < n; c0++) r[c0] /= (alp * dt);
    double *psi = (double *)malloc(n * sizeof(double));
    or_poisson(s, 0, r, psi);
    or_sub_gradient(s, psi, alp * dt);
    or_apply_ly_centre(s, psi, 0, 0.0, 0.0, ly);
    if (imp) { /* the pressure update follows the implicit operator: full Laplacian */
        or_lap_xz(s, psi, lxz);
        for (size_t c0 = 0; c0 < n; c0++) ly[c0] += lxz[c0];
    }
    for (size_t c0 = 0; c0 < n; c0++) p[c0] += psi[c0] - 0.5 * alp * dt / re * ly[c0];
    free(psi);
    free(lxz);
    free(ly);
    free(r);

    /* (v) potential from the updated concentrations */
    or_solve_potential(s);

    s->t += alp * dt;
    s->stage = (k + 1) % 3;
    s->substeps++;
}

void or_run(or_solver *s, int nsub) {
    for (int q = 0; q < nsub; q++) or_substep(s);
}

/* ------------------------------------------------------------------ */
/* initial state                                                        */
/* ------------------------------------------------------------------ */

/* Linear Couette profile plus seeded uniform noise of amplitude u_noise on
 * every velocity unknown; concentrations 1 plus seeded noise of amplitude
 * c_noise with its volume mean removed; one projection without pressure;
 * phi solved from the initial charge; p = 0. */
void or_init(or_solver *s, uint64_t seed, double u_noise, double c_noise) {
    int M = s->M;
    size_t n = or_ncell(s);
    double ut = s->cfg.u_top, ub = s->cfg.u_bot;
    for (int j = 0; j < M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k);
                double ulin = 0.5 * (ut + ub) + 0.5 * (ut - ub) * s->yc[j];
                s->f[F_U][c0] = ulin + u_noise * or_noise(seed, 0, c0);
                s->f[F_V][c0] = (j > 0) ? u_noise * or_noise(seed, 1, c0) : 0.0;
                s->f[F_W][c0] = u_noise * or_noise(seed, 2, c0);
                s->f[F_CP][c0] = c_noise * or_noise(seed, 3, c0);
                s->f[F_CM][c0] = c_noise * or_noise(seed, 4, c0);
                s->f[F_P][c0] = 0.0;
            }
    for (int q = F_CP; q <= F_CM; q++) {
        double sum = 0.0, vol = 0.0;
        for (int j = 0; j < M; j++)
            for (int k = 0; k < s->nz; k++)
                for (int i = 0; i < s->nx; i++) { sum += s->f[q][IDX(s, i, j, k)] * s->dn[j]; vol += s->dn[j]; }
        double mean = sum / vol;
        for (size_t c0 = 0; c0 < n; c0++) s->f[q][c0] = 1.0 + (s->f[q][c0] - mean);
    }
    double *div = (double *)malloc(n * sizeof(double)), *psi = (double *)malloc(n * sizeof(double));
    or_divergence(s, s->f[F_U], s->f[F_V], s->f[F_W], div);
    or_poisson(s, 0, div, psi);
    or_sub_gradient(s, psi, 1.0);
    free(div);
    free(psi);
    or_solve_potential(s);
    for (int q = 0; q < 5; q++) memset(s->hold[q], 0, n * sizeof(double));
    s->t = 0.0;
    s->stage = 0;
    s->substeps = 0;
    s->dt = (s->cfg.dt > 0.0) ? s->cfg.dt : 0.0;
}

/* Recompute phi from the current concentrations (used after fields are set
 * directly by a test). */
void or_refresh_potential(or_solver *s) { or_solve_potential(s); }

/* ------------------------------------------------------------------ */
/* diagnostics (Sec. II: tau_w = eta d<u_x>/dy, c_f, Re_tau)             */
/* ------------------------------------------------------------------ */

/* plane mean of a field at row j */
static double or_plane_mean(const or_solver *s, const double *q, int j) {
    double sum = 0.0;
    for (int k = 0; k < s->nz; k++)
        for (int i = 0; i < s->nx; i++) sum += q[IDX(s, i, j, k)];
    return sum / ((double)s->nx * s->nz);
}

/* Wall shear stress, in units of rho_w U^2, as the viscous flux through the
 * wall faces: Re^-1 (<u>_0 - u_bot)/dc_0 and Re^-1 (u_top - <u>_{M-1})/dc_M. */
void or_wall_shear(const or_solver *s, double *tau_bot, double *tau_top) {
    double ire = 1.0 / s->cfg.re;
    *tau_bot = ire * (or_plane_mean(s, s->f[F_U], 0) - s->cfg.u_bot) / s->dc[0];
    *tau_top = ire * (s->cfg.u_top - or_plane_mean(s, s->f[F_U], s->M - 1)) / s->dc[s->M];
}

/* Plane-averaged total wall-normal ion flux (advective + diffusive +
 * migration) at the ny nodes, zero on the two wall nodes (Fig. 1), and the
 * total ion contents sum(c Omega). */
void or_ion_flux(const or_solver *s, double *jp, double *jm, double *mp, double *mm) {
    int M = s->M;
    double kd = 1.0 / (s->cfg.re * s->cfg.sc), e0 = 0.5 * s->cfg.vhat;
    const double *v = s->f[F_V], *phi = s->f[F_PHI];
    for (int sp = 0; sp < 2; sp++) {
        const double *c = s->f[sp == 0 ? F_CP : F_CM];
        double zs = (sp == 0) ? 1.0 : -1.0;
        double *jo = (sp == 0) ? jp : jm;
        jo[0] = 0.0;
        jo[M] = 0.0;
        for (int j = 1; j < M; j++) {
            double sum = 0.0;
            for (int k = 0; k < s->nz; k++)
                for (int i = 0; i < s->nx; i++) {
                    size_t c0 = IDX(s, i, j, k), cd = IDX(s, i, j - 1, k);
                    int up = v[c0] >= 0.0, have = up ? (j > 1) : (j + 1 < M);
                    double cuu = have ? c[IDX(s, i, up ? j - 2 : j + 1, k)] : 0.0;
                    double cf = or_adv_face(s, c[cd], c[c0], cuu, up, have);
                    double ey = e0 + (phi[c0] - phi[cd]) / s->dc[j];
                    double cmig = or_mig_face(s, c[cd], c[c0], e0 * s->dc[j] + (phi[c0] - phi[cd]), zs);
                    sum += v[c0] * cf - kd * ((c[c0] - c[cd]) / s->dc[j] + zs * cmig * ey);
                }
            jo[j] = sum / ((double)s->nx * s->nz);
        }
        double mass = 0.0;
        for (int j = 0; j < M; j++)
            for (int k = 0; k < s->nz; k++)
                for (int i = 0; i < s->nx; i++) mass += c[IDX(s, i, j, k)] * s->dx * s->dn[j] * s->dz;
        if (sp == 0) *mp = mass; else *mm = mass;
    }
}

/* kinetic energy 1/2 sum(u^2 Omega_u + v^2 Omega_v + w^2 Omega_w) */
double or_kinetic_energy(const or_solver *s) {
    const double *u = s->f[F_U], *v = s->f[F_V], *w = s->f[F_W];
    double e = 0.0;
    for (int j = 0; j < s->M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k);
                double vol = s->dx * s->dn[j] * s->dz;
                e += 0.5 * (u[c0] * u[c0] + w[c0] * w[c0]) * vol;
                if (j > 0) e += 0.5 * v[c0] * v[c0] * s->dx * s->dc[j] * s->dz;
            }
    return e;
}

/* max |D u| over the cells */
double or_max_divergence(const or_solver *s) {
    size_t n = or_ncell(s);
    double *d = (double *)malloc(n * sizeof(double));
    or_divergence(s, s->f[F_U], s->f[F_V], s->f[F_W], d);
    double m = 0.0;
    for (size_t q = 0; q < n; q++) if (fabs(d[q]) > m) m = fabs(d[q]);
    free(d);
    return m;
}

/* Kinetic-energy budget terms of the semi-discrete equations:
 *   dKE/dt = (wall work) - (viscous dissipation) + (Coulomb work)
 * The wall work (power of the two moving walls against the viscous wall
 * stress) and the dissipation are the boundary and volume terms of the
 * summation by parts of Re^-1 sum(u . L u Omega); convection does no work
 * and the pressure gradient does none on a divergence-free field. */
void or_energy_terms(const or_solver *s, double *wall_work, double *dissipation, double *force_work) {
    size_t n = or_ncell(s);
    int M = s->M;
    const double *u = s->f[F_U], *v = s->f[F_V], *w = s->f[F_W];
    double ire = 1.0 / s->cfg.re;
    double dx = s->dx, dz = s->dz;
    /* dissipation: Re^-1 sum over all velocity differences squared / spacing * face area */
    double dis = 0.0;
    for (int j = 0; j < M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k);
                size_t xp = IDX(s, PX(i), j, k), zp = IDX(s, i, j, PZ(k));
                double dn = s->dn[j];
                /* u: x, z differences over the u control volumes, y differences across centre rows */
                double gux = (u[xp] - u[c0]) / dx, guz = (u[zp] - u[c0]) / dz;
                double gwx = (w[xp] - w[c0]) / dx, gwz = (w[zp] - w[c0]) / dz;
                dis += (gux * gux + guz * guz + gwx * gwx + gwz * gwz) * dx * dn * dz;
                if (j + 1 < M) {
                    size_t yp = IDX(s, i, j + 1, k);
                    double guy = (u[yp] - u[c0]) / s->dc[j + 1], gwy = (w[yp] - w[c0]) / s->dc[j + 1];
                    dis += (guy * guy + gwy * gwy) * dx * s->dc[j + 1] * dz;
                }
                if (j > 0) {
                    double dcj = s->dc[j];
                    double gvx = (v[xp] - v[c0]) / dx, gvz = (v[zp] - v[c0]) / dz;
                    dis += (gvx * gvx + gvz * gvz) * dx * dcj * dz;
                }
                /* v: y differences over cell rows j (nodes j, j+1) */
                {
                    double vb = (j > 0) ? v[c0] : 0.0;
                    double vt = (j + 1 < M) ? v[IDX(s, i, j + 1, k)] : 0.0;
                    double gvy = (vt - vb) / dn;
                    dis += gvy * gvy * dx * dn * dz;
                }
            }
    /* wall half-cells of u, w */
    for (int k = 0; k < s->nz; k++)
        for (int i = 0; i < s->nx; i++) {
            size_t b = IDX(s, i, 0, k), t = IDX(s, i, M - 1, k);
            double gub = (u[b] - s->cfg.u_bot) / s->dc[0], gut = (s->cfg.u_top - u[t]) / s->dc[M];
            double gwb = w[b] / s->dc[0], gwt = -w[t] / s->dc[M];
            dis += (gub * gub + gwb * gwb) * dx * s->dc[0] * dz + (gut * gut + gwt * gwt) * dx * s->dc[M] * dz;
        }
    *dissipation = ire * dis;
    /* wall work: the wall moves with u_top / u_bot and exerts the viscous flux */
    double ww = 0.0;
    for (int k = 0; k < s->nz; k++)
        for (int i = 0; i < s->nx; i++) {
            size_t b = IDX(s, i, 0, k), t = IDX(s, i, M - 1, k);
            ww += s->cfg.u_top * ire * (s->cfg.u_top - u[t]) / s->dc[M] * dx * dz;
            ww -= s->cfg.u_bot * ire * (u[b] - s->cfg.u_bot) / s->dc[0] * dx * dz;
        }
    *wall_work = ww;
    double *fu = (double *)malloc(3 * n * sizeof(double)), *fv = fu + n, *fw = fv + n;
    or_coulomb(s, s->f[F_CP], s->f[F_CM], s->f[F_PHI], fu, fv, fw);
    double fwk = 0.0;
    for (int j = 0; j < M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k);
                double vol = dx * s->dn[j] * dz;
                fwk += (u[c0] * fu[c0] + w[c0] * fw[c0]) * vol;
                if (j > 0) fwk += v[c0] * fv[c0] * dx * s->dc[j] * dz;
            }
    *force_work = fwk;
    free(fu);
}

/* exported helpers for operator-level tests */
void or_apply_ly(const or_solver *s, const double *q, int kind, double qbot, double qtop, double *out) {
    if (kind == 2) or_apply_ly_node(s, q, out);
    else or_apply_ly_centre(s, q, kind, qbot, qtop, out);
}

void or_gradient(const or_solver *s, const double *psi, double *gx, double *gy, double *gz) {
    for (int j = 0; j < s->M; j++)
        for (int k = 0; k < s->nz; k++)
            for (int i = 0; i < s->nx; i++) {
                size_t c0 = IDX(s, i, j, k);
                gx[c0] = (psi[c0] - psi[IDX(s, MX(i), j, k)]) / s->dx;
                gz[c0] = (psi[c0] - psi[IDX(s, i, j, MZ(k))]) / s->dz;
                gy[c0] = (j > 0) ? (psi[c0] - psi[IDX(s, i, j - 1, k)]) / s->dc[j] : 0.0;
            }
}

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
