// api.hip -- the C ABI declared in include/nspnp.h: configuration checks,
// workspace layout, grid and operator tables, initial state, the substep
// sequence and the host side of the diagnostics.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.h"

using namespace nspnp;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(NSPNP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Low-storage three-stage Runge-Kutta (Sec. II): gamma, zeta, alpha = gamma + zeta

bool smooth_size(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

FftPlan make_plan(int n) {
    FftPlan p{};
    p.n = n;
    int m = n, s = 0;
    // radix-8 passes for lines of 512 points and more (fewer passes through
    // LDS: 512 = 8 8 8 runs 5-13% faster than radix 4); shorter lines keep
    // radix 4, whose passes give twice the threads work (256 = 8 8 4 was
    // measured 2-5% slower than 4 4 4 4)
    if (n >= 512)
        while (m % 8 == 0) { p.radix[s++] = 8; m /= 8; }
    while (m % 4 == 0) { p.radix[s++] = 4; m /= 4; }
    while (m % 2 == 0) { p.radix[s++] = 2; m /= 2; }
    while (m % 3 == 0) { p.radix[s++] = 3; m /= 3; }
    p.nstages = s;
    return p;
}

int check_config(const nspnp_config *c) {
    if (!c) return fail(NSPNP_ERR_INVALID, "config is NULL");
    if (c->precision != NSPNP_PREC_FP64 && c->precision != NSPNP_PREC_MIXED)
        return fail(NSPNP_ERR_INVALID, "precision must be 0 (FP64) or 1 (mixed)");
    for (int n : {c->nx, c->nz}) {
        if (n < 4 || n > 1024 || n % 2 != 0 || !smooth_size(n))
            return fail(NSPNP_ERR_SIZE, "nx and nz must be even, of the form 2^a 3^b, and within 4..1024");
    }
    if (c->ny < 5 || c->ny > kMaxRows + 1)
        return fail(NSPNP_ERR_SIZE, "ny (wall-normal nodes) must be within 5.." + std::to_string(kMaxRows + 1) +
                                        " (cell rows staged in 64 KB of LDS)");
    if ((int64_t)c->nx * c->nz * (c->ny - 1) > 2147483647LL)
        return fail(NSPNP_ERR_SIZE, "nx * nz * (ny - 1) must stay below 2^31 cells (32-bit cell indices)");
    const double pos[] = {c->lx, c->lz, c->re, c->sc, c->debye};
    for (double v : pos)
        if (!(v > 0.0) || !std::isfinite(v)) return fail(NSPNP_ERR_INVALID, "lx, lz, re, sc, debye must be > 0");
    if (!(c->stretch >= 0.0) || !std::isfinite(c->beta) || !std::isfinite(c->vhat) || !std::isfinite(c->u_top) ||
        !std::isfinite(c->u_bot) || !std::isfinite(c->force_sign) || !std::isfinite(c->dt))
        return fail(NSPNP_ERR_INVALID, "non-finite configuration value");
    if (c->dt <= 0.0 && !(c->cfl > 0.0)) return fail(NSPNP_ERR_INVALID, "adaptive dt needs cfl > 0");
    if (c->implicit_xz != 0 && c->implicit_xz != 1) return fail(NSPNP_ERR_INVALID, "implicit_xz must be 0 or 1");
    if (c->migration_face < 0 || c->migration_face > 2)
        return fail(NSPNP_ERR_INVALID,
                    "migration_face must be 0 (mean), 1 (hybrid) or 2 (hybrid + limited advective face values)");
    return NSPNP_OK;
}

struct Layout {
    size_t off_f[7], off_h[5], off_r[5], off_psi, off_spec, off_fac, off_coef, off_clock, off_phys, off_stats,
        off_rstats, off_phiw, off_cyc, off_red, off_tab, off_cpv, off_mu;
    size_t ntab, nred, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(const nspnp_config *c) {
    Layout L{};
    const int64_t M = c->ny - 1, nxh = c->nx / 2 + 1;
    const int64_t n = (int64_t)c->nx * c->nz * M;
    const size_t ws = c->precision == NSPNP_PREC_FP64 ? 8 : 4;
    size_t o = 0;
    for (int q = 0; q < 7; ++q) { L.off_f[q] = o; o = align256(o + n * ws); }
    for (int q = 0; q < 5; ++q) { L.off_h[q] = o; o = align256(o + n * ws); }
    for (int q = 0; q < 5; ++q) { L.off_r[q] = o; o = align256(o + n * ws); }
    L.off_psi = o; o = align256(o + n * 8);
    const int64_t nspec = nxh * c->nz * M;
    L.off_spec = o; o = align256(o + 2 * nspec * 16);
    L.off_fac = o; o = align256(o + 2 * nspec * 16);  // [kind][mode][row] pivots
    L.off_cpv = o; o = align256(o + 2 * nspec * 8);   // [kind][row][mode] c' (fused y-march)
    L.off_mu = o; o = align256(o + 2 * 16);           // pinned-mode volume means
    L.off_coef = o; o = align256(o + 3 * cn_stage_stride((int)M) * 8);  // 3 stages: rows, slab products, n products
    L.off_clock = o; o = align256(o + kClockSlots * 8);
    L.off_phys = o; o = align256(o + sizeof(Phys));
    L.off_stats = o; o = align256(o + (3 * M + 2) * 8);
    L.off_rstats = o; o = align256(o + (kRunStatsQ * M + kRunStatsTail) * 8);
    L.off_phiw = o; o = align256(o + 2 * (int64_t)c->nx * c->nz * 8);
    L.off_cyc = o; o = align256(o + cyc_block_doubles(c->nx, c->nz) * kCycBlocks * 8);
    L.nred = std::max<int64_t>({(int64_t)kDtParts * dt_max_blocks((int64_t)c->nx * c->nz), M * kPlaneQ,
                                 M * (int64_t)run_stats_chunks((int)M) * kRunStatsQ});
    L.off_red = o; o = align256(o + L.nred * 8);
    L.ntab = 11 * M + 2 + nxh + c->nz + 2 * c->nx + 2 * c->nz;
    L.off_tab = o; o = align256(o + L.ntab * 8);
    L.total = o;
    return L;
}

size_t table_count(int M, int nx, int nz) { return 11 * (size_t)M + 2 + (nx / 2 + 1) + nz + 2 * nx + 2 * nz; }

// Host tables: tanh-stretched y nodes, finite-volume L_y coefficients and
// reciprocals, modified wavenumbers of the three-point x/z Laplacians, FFT
// twiddles.  All FP64; the layout is a sequence of named arrays.
void build_tables(nspnp_state *s, double *dev_tab) {
    const nspnp_config &c = s->cfg;
    const int M = s->d.M, nx = c.nx, nz = c.nz, nxh = s->d.nxh;
    double yn[kMaxRows + 1];  // (no heap use: the allocation-free solve builds tables too)
    for (int j = 0; j <= M; ++j) {
        const double xi = -1.0 + 2.0 * j / (double)M;
        yn[j] = (c.stretch > 0.0) ? std::tanh(c.stretch * xi) / std::tanh(c.stretch) : xi;
    }
    yn[0] = -1.0;
    yn[M] = 1.0;
    std::vector<double> &t = s->host_tables;
    t.assign(table_count(M, nx, nz), 0.0);
    size_t off = 0;
    auto take = [&](size_t len, const double **dev) {
        double *h = t.data() + off;
        *dev = dev_tab + off;
        off += len;
        return h;
    };
    double *yc = take(M, &s->tb.yc), *dn = take(M, &s->tb.dn), *dc = take(M + 1, &s->tb.dc);
    double *lyc_lo = take(M, &s->tb.lyc_lo), *lyc_up = take(M, &s->tb.lyc_up);
    double *lyn_lo = take(M, &s->tb.lyn_lo), *lyn_up = take(M, &s->tb.lyn_up);
    double *idn = take(M, &s->tb.idn), *idc = take(M + 1, &s->tb.idc);
    double *vwl = take(M, &s->tb.vwl), *vwu = take(M, &s->tb.vwu);
    double *kx2 = take(nxh, &s->tb.kx2), *kz2 = take(nz, &s->tb.kz2);
    const double *twx_dev, *twz_dev;
    double *twx = take(2 * nx, &twx_dev), *twz = take(2 * nz, &twz_dev);
    s->tb.twx = (const double2 *)twx_dev;
    s->tb.twz = (const double2 *)twz_dev;
    for (int j = 0; j < M; ++j) {
        yc[j] = 0.5 * (yn[j] + yn[j + 1]);
        dn[j] = yn[j + 1] - yn[j];
    }
    dc[0] = yc[0] - yn[0];
    for (int j = 1; j < M; ++j) dc[j] = yc[j] - yc[j - 1];
    dc[M] = yn[M] - yc[M - 1];
    for (int j = 0; j < M; ++j) {
        lyc_lo[j] = 1.0 / (dn[j] * dc[j]);
        lyc_up[j] = 1.0 / (dn[j] * dc[j + 1]);
        lyn_lo[j] = (j > 0) ? 1.0 / (dc[j] * dn[j - 1]) : 0.0;
        lyn_up[j] = (j > 0) ? 1.0 / (dc[j] * dn[j]) : 0.0;
        idn[j] = 1.0 / dn[j];
        vwl[j] = (j > 0) ? dn[j - 1] / (2.0 * dc[j]) : 0.0;
        vwu[j] = (j > 0) ? dn[j] / (2.0 * dc[j]) : 0.0;
    }
    for (int j = 0; j <= M; ++j) idc[j] = 1.0 / dc[j];
    const double dx = s->d.dx, dz = s->d.dz;
    const double twopi = 6.283185307179586476925286766559;
    for (int m = 0; m < nxh; ++m) kx2[m] = (2.0 - 2.0 * std::cos(twopi * m / nx)) / (dx * dx);
    for (int m = 0; m < nz; ++m) kz2[m] = (2.0 - 2.0 * std::cos(twopi * m / nz)) / (dz * dz);
    // FFT twiddles in pass order (the plan of make_plan): pass after pass,
    // [r - 1][k] = exp(-2 pi i r k ts / N) for k < Ns, 0 < r < R, ts = N / (Ns R)
    // (N - 1 entries; the last slot is unused), so that a pass's lanes read
    // consecutive entries
    auto pass_twiddles = [twopi](int n, double *tw) {
        const FftPlan pl = make_plan(n);
        int Ns = 1, off = 0;
        for (int q = 0; q < pl.nstages; ++q) {
            const int R = pl.radix[q], ts = n / (Ns * R);
            for (int r = 1; r < R; ++r)
                for (int k = 0; k < Ns; ++k) {
                    const int m = r * k * ts, e = off + (r - 1) * Ns + k;
                    tw[2 * e] = std::cos(twopi * m / n);
                    tw[2 * e + 1] = -std::sin(twopi * m / n);
                }
            off += Ns * (R - 1);
            Ns *= R;
        }
        tw[2 * (n - 1)] = 0.0;
        tw[2 * (n - 1) + 1] = 0.0;
    };
    pass_twiddles(nx, twx);
    pass_twiddles(nz, twz);
}

const double *host_dn(const nspnp_state *s) { return s->host_tables.data() + s->d.M; }
const double *host_dc(const nspnp_state *s) { return s->host_tables.data() + 2 * s->d.M; }

int plane_reduce(nspnp_state *s, std::vector<double> &host) {
    HIP_TRY(launch_plane_sums(s, 0, s->red));
    host.resize((size_t)s->d.M * kPlaneQ);
    HIP_TRY(hipMemcpyAsync(host.data(), s->red, host.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return NSPNP_OK;
}

PoissonSrc div_source(nspnp_state *s, double alp, double fixed) {
    return PoissonSrc{SRC_DIV, s->f[0], s->f[1], s->f[2], fixed, alp};
}

PoissonSrc charge_source(nspnp_state *s) {
    return PoissonSrc{SRC_CHARGE, s->f[3], s->f[4], nullptr, 0.0, 0.0, s->phiw_on ? s->phiw : nullptr};
}

// A batch over the members of this handle (member stride) or over caller
// arrays for member 0 (stride 0).
PoissonBatch make_batch(nspnp_state *s, bool members) {
    PoissonBatch b{};
    b.ms = members ? s->mstride : 0;
    b.phys = s->d_phys;
    return b;
}

// phi from the current c+- (potential-type solve straight into the state)
int solve_potential(nspnp_state *s) {
    PoissonBatch b = make_batch(s, true);
    b.nprob = 1;
    b.kind[0] = 1;
    b.src[0] = charge_source(s);
    b.out[0] = s->f[5];
    b.out_state[0] = 1;
    HIP_TRY(launch_poisson_batch(s, b));
    return NSPNP_OK;
}

}  // namespace

namespace nspnp {

int fail_code(int code, const std::string &msg) { return fail(code, msg); }

void fill_tables(nspnp_state *s, double *dev_tab) { build_tables(s, dev_tab); }

size_t tables_len(int M, int nx, int nz) { return table_count(M, nx, nz); }

int check(const nspnp_config *c) { return check_config(c); }

size_t layout_bytes(const nspnp_config *c) { return make_layout(c).total; }

Phys make_phys(const nspnp_config *cfg) {
    Phys ph{};
    ph.re = cfg->re;
    ph.ire = 1.0 / cfg->re;
    ph.kd = 1.0 / (cfg->re * cfg->sc);
    ph.kf = cfg->force_sign * cfg->beta / (2.0 * cfg->sc * cfg->re * cfg->re * cfg->debye * cfg->debye);
    ph.e0 = 0.5 * cfg->vhat;
    ph.ch = -1.0 / (2.0 * cfg->debye * cfg->debye);
    ph.u_top = cfg->u_top;
    ph.u_bot = cfg->u_bot;
    ph.debye = cfg->debye;
    ph.cfl = cfg->cfl;
    ph.adaptive = cfg->dt > 0.0 ? 0.0 : 1.0;
    ph.implicit_xz = cfg->implicit_xz ? 1.0 : 0.0;
    ph.hybrid = cfg->migration_face ? 1.0 : 0.0;
    ph.limited = cfg->migration_face == 2 ? 1.0 : 0.0;
    return ph;
}

// Sizes, constants, FFT plans, default launch shapes and the device's LDS
// limit of a handle on this configuration (no device memory touched).
void setup_common(nspnp_state *s, const nspnp_config *cfg, int nmem, hipStream_t stream) {
    s->cfg = *cfg;
    s->stream = stream;
    s->fp64 = cfg->precision == NSPNP_PREC_FP64;
    s->wsize = s->fp64 ? 8 : 4;
    Dims &d = s->d;
    d.nx = cfg->nx;
    d.nz = cfg->nz;
    d.M = cfg->ny - 1;
    d.nxh = cfg->nx / 2 + 1;
    d.plane = (int64_t)cfg->nx * cfg->nz;
    d.n = d.plane * d.M;
    d.dx = cfg->lx / cfg->nx;
    d.dz = cfg->lz / cfg->nz;
    s->ph = make_phys(cfg);
    s->nmem = nmem;
    s->mstride = 0;
    s->planx = make_plan(cfg->nx);
    s->planz = make_plan(cfg->nz);
    // the tuner's choices at 256 x 193 x 256 (the mixed form takes 32-column
    // Crank-Nicolson tiles: whole 128-byte lines of FP32 per row)
    s->tiles = Tiles{256, cfg->precision == NSPNP_PREC_FP64 ? 256 : 512, 512, 1024, 16, 128, 16, 0};
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
            s->lds_max = lds;
    }
}

// Handle over nmem members of one size class: member m's workspace starts at
// base + m * layout_bytes(cfg); pointers refer to member 0.
void setup_handle(nspnp_state *s, const nspnp_config *cfg, char *base, int nmem, hipStream_t stream) {
    const Layout L = make_layout(cfg);
    setup_common(s, cfg, nmem, stream);
    s->mstride = nmem > 1 ? L.total : 0;
    for (int q = 0; q < 7; ++q) s->f[q] = base + L.off_f[q];
    for (int q = 0; q < 5; ++q) s->h[q] = base + L.off_h[q];
    for (int q = 0; q < 5; ++q) s->r[q] = base + L.off_r[q];
    s->psi = (double *)(base + L.off_psi);
    s->spec = (double2 *)(base + L.off_spec);
    s->fac = (double2 *)(base + L.off_fac);
    s->cpv = (double *)(base + L.off_cpv);
    s->mu = (double2 *)(base + L.off_mu);
    s->cn_coef = (double *)(base + L.off_coef);
    s->clock = (double *)(base + L.off_clock);
    s->d_phys = (Phys *)(base + L.off_phys);
    s->stats = (double *)(base + L.off_stats);
    s->rstats = (double *)(base + L.off_rstats);
    s->rstats_every = 0;
    s->phiw = (double *)(base + L.off_phiw);
    s->cyc = (double *)(base + L.off_cyc);
    s->phiw_on = false;
    s->red = (double *)(base + L.off_red);
    s->nred = L.nred;
    s->tab_base = base + L.off_tab;
    build_tables(s, (double *)(base + L.off_tab));
    s->substeps = 0;
    s->stats_on = false;
}

int upload_tables(nspnp_state *s) {
    HIP_TRY(hipMemcpyAsync(s->tab_base, s->host_tables.data(), s->host_tables.size() * sizeof(double),
                           hipMemcpyHostToDevice, s->stream));
    return NSPNP_OK;
}

// A single-member handle for member m of a class handle (same tables).
nspnp_state *member_view(const nspnp_state *cls, int m, const nspnp_config *cfg) {
    nspnp_state *v = new nspnp_state(*cls);
    v->prof = Profiler{};
    const size_t off = (size_t)m * cls->mstride;
    auto sh = [off](auto *p) { return (decltype(p))((char *)p + off); };
    for (int q = 0; q < 7; ++q) v->f[q] = sh(cls->f[q]);
    for (int q = 0; q < 5; ++q) { v->h[q] = sh(cls->h[q]); v->r[q] = sh(cls->r[q]); }
    v->psi = sh(cls->psi);
    v->spec = sh(cls->spec);
    v->fac = sh(cls->fac);
    v->cpv = sh(cls->cpv);
    v->mu = sh(cls->mu);
    v->cn_coef = sh(cls->cn_coef);
    v->clock = sh(cls->clock);
    v->d_phys = sh(cls->d_phys);
    v->stats = sh(cls->stats);
    v->rstats = sh(cls->rstats);
    v->phiw = sh(cls->phiw);
    v->cyc = sh(cls->cyc);
    v->red = sh(cls->red);
    v->nmem = 1;
    v->mstride = 0;
    v->host_health = cls->host_health ? cls->host_health + 2 * (size_t)m : nullptr;
    v->owns_host_health = false;
    if (cfg) {
        v->cfg = *cfg;
        v->ph = make_phys(cfg);
    }
    return v;
}

// Seeded initial state of a single-member handle (Sec. II geometry and
// boundary conditions; noise recipe in include/nspnp.h).
int init_member(nspnp_state *s) {
    const Dims &d = s->d;
    const double clock0[kClockSlots] = {0.0, s->cfg.dt > 0.0 ? s->cfg.dt : 0.0, 0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(s->clock, clock0, sizeof(clock0), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->d_phys, &s->ph, sizeof(Phys), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(launch_run_stats_begin(s));  // empty statistics, start time 0
    HIP_TRY(launch_init_fields(s));
    // remove the volume mean of the concentration noise
    std::vector<double> ps;
    int rc = plane_reduce(s, ps);  // synchronises: the stack clock0 is consumed
    if (rc) return rc;
    double sp = 0.0, sm = 0.0, vol = 0.0;
    for (int j = 0; j < d.M; ++j) {
        const double dn = host_dn(s)[j];
        sp += ps[j * kPlaneQ + PQ_SUM_CP] * dn;
        sm += ps[j * kPlaneQ + PQ_SUM_CM] * dn;
        vol += dn * (double)d.plane;
    }
    HIP_TRY(launch_shift_conc(s, sp / vol, sm / vol));
    HIP_TRY(launch_thomas_factors(s));
    // project the initial velocity (no pressure), then the initial potential
    PoissonBatch b = make_batch(s, true);
    b.nprob = 1;
    b.kind[0] = 0;
    b.src[0] = div_source(s, 0.0, 1.0);
    b.out[0] = s->psi;
    b.out_state[0] = 0;
    HIP_TRY(launch_poisson_batch(s, b));
    HIP_TRY(launch_correct(s, Stage{0, 0, 0, 0}, false, 1.0, false));
    return solve_potential(s);
}

// n Runge-Kutta substeps of every member of the handle.
int step_handle(nspnp_state *s, int n) {
    for (int it = 0; it < n; ++it) {
        const int k = (int)(s->substeps % 3);
        const Stage st{kRkGam[k], kRkZet[k], kRkAlp[k], k};
        if (k == 0) HIP_TRY(launch_dt(s));  // dt rule (adaptive runs) and health check
        HIP_TRY(launch_explicit(s, st, true));
        HIP_TRY(launch_cn_solve(s, st));
        // pressure projection and potential depend only on the updated
        // fields, so both elliptic solves share one batched pipeline
        PoissonBatch b = make_batch(s, true);
        b.nprob = 2;
        b.kind[0] = 0;
        b.src[0] = div_source(s, st.alp, 0.0);
        b.out[0] = s->psi;
        b.out_state[0] = 0;
        b.kind[1] = 1;
        b.src[1] = charge_source(s);
        b.out[1] = s->f[5];
        b.out_state[1] = 1;
        HIP_TRY(launch_poisson_batch(s, b));
        HIP_TRY(launch_correct(s, st, true, 0.0, true));
        if (s->stats_on) HIP_TRY(launch_stats_accum(s, st.alp));
        if (s->rstats_every > 0 && (s->substeps + 1) % s->rstats_every == 0) HIP_TRY(launch_run_stats(s));
        s->substeps++;
    }
    return NSPNP_OK;
}

int health_error(int bits, int member) {
    std::string m = "run";
    if (member >= 0) m += " (ensemble member " + std::to_string(member) + ")";
    if (bits & kHealthNonFinite) m += " produced a non-finite value";
    if (bits & kHealthNegative) m += std::string((bits & kHealthNonFinite) ? " and" : "") + " a negative concentration";
    return fail(NSPNP_ERR_NONFINITE, m + "; the state is invalid until it is reset (nspnp_set_clock or a new init)");
}

// Pinned host mirror of the health slots of every member of a handle.
int alloc_host_health(nspnp_state *s) {
    void *p = nullptr;
    HIP_TRY(hipHostMalloc(&p, 2 * sizeof(double) * (size_t)s->nmem, hipHostMallocDefault));
    s->host_health = (double *)p;
    s->owns_host_health = true;
    for (int q = 0; q < 2 * s->nmem; ++q) s->host_health[q] = 0.0;
    return NSPNP_OK;
}

// Health of the last check whose copy has landed (member ids from first_id).
int check_health(const nspnp_state *s, int first_id) {
    if (!s->host_health) return NSPNP_OK;
    for (int m = 0; m < s->nmem; ++m) {
        const int bits = (int)s->host_health[2 * m];
        if (bits) return health_error(bits, first_id < 0 ? -1 : first_id + m);
    }
    return NSPNP_OK;
}

// Queue the copy of every member's [health, max |dPhi|] to the host mirror.
int queue_health_copy(nspnp_state *s) {
    if (!s->host_health) return NSPNP_OK;
    const size_t w = 2 * sizeof(double);
    HIP_TRY(hipMemcpy2DAsync(s->host_health, w, s->clock + 2, s->nmem > 1 ? s->mstride : w, w, (size_t)s->nmem,
                             hipMemcpyDeviceToHost, s->stream));
    return NSPNP_OK;
}

}  // namespace nspnp

nspnp_state::~nspnp_state() {
    for (hipEvent_t e : prof.ev) (void)hipEventDestroy(e);
    if (owns_host_health && host_health) (void)hipHostFree(host_health);
}

namespace {
const char *const kKernelNames[K_NKERNEL] = {
    "dt", "explicit_rhs", "cn_tridiag", "fft_x_r2c", "fft_z_fwd", "thomas_modes",
    "fft_z_inv", "fft_x_c2r", "correct", "stats"};
}

extern "C" {

const char *nspnp_last_error(void) { return g_last_error.c_str(); }

int nspnp_profile_enable(nspnp_state *s, int32_t on) {
    if (!s) return fail(NSPNP_ERR_INVALID, "state is NULL");
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->prof.on = on != 0;
    s->prof.used = 0;
    s->prof.ids.clear();
    for (int k = 0; k < K_NKERNEL; ++k) {
        s->prof.total_ms[k] = 0.0;
        s->prof.launches[k] = 0;
    }
    return NSPNP_OK;
}

int nspnp_profile_read(nspnp_state *s, int32_t *count, const char **names, double *total_ms, int64_t *launches) {
    if (!s || !count) return fail(NSPNP_ERR_INVALID, "bad profile_read arguments");
    HIP_TRY(hipStreamSynchronize(s->stream));
    Profiler &p = s->prof;
    const size_t pairs = std::min(p.ids.size(), p.used / 2);
    for (size_t q = 0; q < pairs; ++q) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.ev[2 * q], p.ev[2 * q + 1]));
        p.total_ms[p.ids[q]] += ms;
        p.launches[p.ids[q]] += 1;
    }
    p.used = 0;
    p.ids.clear();
    *count = K_NKERNEL;
    for (int k = 0; k < K_NKERNEL; ++k) {
        if (names) names[k] = kKernelNames[k];
        if (total_ms) total_ms[k] = p.total_ms[k];
        if (launches) launches[k] = p.launches[k];
    }
    return NSPNP_OK;
}

size_t nspnp_workspace_bytes(const nspnp_config *cfg) {
    if (check_config(cfg) != NSPNP_OK) return 0;
    return make_layout(cfg).total;
}

int nspnp_init_state(const nspnp_config *cfg, void *dev_workspace, size_t bytes, void *hip_stream,
                     nspnp_state **out) {
    if (!out) return fail(NSPNP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    const size_t need = layout_bytes(cfg);
    if (!dev_workspace || bytes < need)
        return fail(NSPNP_ERR_WORKSPACE, "workspace missing or smaller than nspnp_workspace_bytes()");
    if (((uintptr_t)dev_workspace & 255) != 0) return fail(NSPNP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    nspnp_state *s = new nspnp_state();
    setup_handle(s, cfg, (char *)dev_workspace, 1, (hipStream_t)hip_stream);
    if ((rc = alloc_host_health(s)) || (rc = upload_tables(s)) || (rc = init_member(s))) {
        delete s;
        return rc;
    }
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        delete s;
        return fail(NSPNP_ERR_HIP, std::string("init sync: ") + hipGetErrorString(e));
    }
    *out = s;
    return NSPNP_OK;
}

int nspnp_grid(const nspnp_config *cfg, double *yn, double *yc) {
    int rc = check_config(cfg);
    if (rc) return rc;
    if (!yn || !yc) return fail(NSPNP_ERR_INVALID, "grid: NULL output");
    nspnp_state tmp;
    tmp.cfg = *cfg;
    tmp.d.M = cfg->ny - 1;
    tmp.d.nxh = cfg->nx / 2 + 1;
    tmp.d.dx = cfg->lx / cfg->nx;
    tmp.d.dz = cfg->lz / cfg->nz;
    std::vector<double> dev_dummy(table_count(tmp.d.M, cfg->nx, cfg->nz));
    build_tables(&tmp, dev_dummy.data());
    const int M = tmp.d.M;
    const double *hyc = tmp.host_tables.data(), *hdn = hyc + M;
    yn[0] = -1.0;
    for (int j = 0; j < M; ++j) {
        yc[j] = hyc[j];
        yn[j + 1] = yn[j] + hdn[j];
    }
    yn[M] = 1.0;
    return NSPNP_OK;
}

int nspnp_step(nspnp_state *s, int32_t n_substeps) {
    if (!s || n_substeps < 0) return fail(NSPNP_ERR_INVALID, "bad state or substep count");
    int rc = check_health(s, -1);
    if (rc) return rc;
    // a check runs at every substep of stage 0 among the ones queued here
    const int r = (int)(s->substeps % 3);
    const bool checks = n_substeps > 0 && (r == 0 || r + n_substeps > 3);
    if ((rc = step_handle(s, n_substeps))) return rc;
    return checks ? queue_health_copy(s) : NSPNP_OK;
}

int nspnp_poisson_solve(nspnp_state *s, int32_t kind, const double *dev_rhs, double *dev_out) {
    if (!s || !dev_rhs || !dev_out || (kind != 0 && kind != 1)) return fail(NSPNP_ERR_INVALID, "bad poisson_solve arguments");
    PoissonBatch b = make_batch(s, false);
    b.nprob = 1;
    b.kind[0] = kind;
    b.src[0] = PoissonSrc{SRC_REAL, dev_rhs, nullptr, nullptr, 0.0, 0.0};
    b.out[0] = dev_out;
    b.out_state[0] = 0;
    HIP_TRY(launch_poisson_batch(s, b));
    return NSPNP_OK;
}

int nspnp_wall_shear_stress(nspnp_state *s, double *tau_bottom, double *tau_top) {
    if (!s || !tau_bottom || !tau_top) return fail(NSPNP_ERR_INVALID, "bad wall_shear_stress arguments");
    std::vector<double> ps;
    int rc = plane_reduce(s, ps);
    if (rc) return rc;
    const int M = s->d.M;
    const double pl = (double)s->d.plane;
    const double *dc = host_dc(s);
    *tau_bottom = s->ph.ire * (ps[PQ_SUM_U] / pl - s->cfg.u_bot) / dc[0];
    *tau_top = s->ph.ire * (s->cfg.u_top - ps[(M - 1) * kPlaneQ + PQ_SUM_U] / pl) / dc[M];
    if (!std::isfinite(*tau_bottom) || !std::isfinite(*tau_top)) return fail(NSPNP_ERR_NONFINITE, "non-finite wall stress");
    return NSPNP_OK;
}

int nspnp_ion_flux(nspnp_state *s, double *jp, double *jm, double *mass_p, double *mass_m) {
    if (!s || !jp || !jm || !mass_p || !mass_m) return fail(NSPNP_ERR_INVALID, "bad ion_flux arguments");
    std::vector<double> ps;
    int rc = plane_reduce(s, ps);
    if (rc) return rc;
    const int M = s->d.M;
    const double pl = (double)s->d.plane;
    const double *dn = host_dn(s);
    jp[0] = jm[0] = jp[M] = jm[M] = 0.0;
    for (int j = 1; j < M; ++j) {
        jp[j] = ps[j * kPlaneQ + PQ_FLUX_P] / pl;
        jm[j] = ps[j * kPlaneQ + PQ_FLUX_M] / pl;
    }
    double a = 0.0, b = 0.0;
    for (int j = 0; j < M; ++j) {
        a += ps[j * kPlaneQ + PQ_SUM_CP] * s->d.dx * dn[j] * s->d.dz;
        b += ps[j * kPlaneQ + PQ_SUM_CM] * s->d.dx * dn[j] * s->d.dz;
    }
    *mass_p = a;
    *mass_m = b;
    if (!std::isfinite(a) || !std::isfinite(b)) return fail(NSPNP_ERR_NONFINITE, "non-finite ion content");
    return NSPNP_OK;
}

int nspnp_get_field(nspnp_state *s, int32_t field, double *dev_out) {
    if (!s || !dev_out || field < 0 || field > 6) return fail(NSPNP_ERR_INVALID, "bad get_field arguments");
    HIP_TRY(launch_convert(s, field, nullptr, dev_out, false));
    return NSPNP_OK;
}

int nspnp_set_field(nspnp_state *s, int32_t field, const double *dev_in) {
    if (!s || !dev_in || field < 0 || field > 6) return fail(NSPNP_ERR_INVALID, "bad set_field arguments");
    HIP_TRY(launch_convert(s, field, dev_in, nullptr, true));
    return NSPNP_OK;
}

int nspnp_refresh_potential(nspnp_state *s) {
    if (!s) return fail(NSPNP_ERR_INVALID, "state is NULL");
    return solve_potential(s);
}

int nspnp_explicit_terms(nspnp_state *s, double *const dev_out[5]) {
    if (!s || !dev_out) return fail(NSPNP_ERR_INVALID, "bad explicit_terms arguments");
    for (int q = 0; q < 5; ++q)
        if (!dev_out[q]) return fail(NSPNP_ERR_INVALID, "explicit_terms output is NULL");
    HIP_TRY(launch_explicit_debug(s, dev_out));
    return NSPNP_OK;
}

int nspnp_diagnostics(nspnp_state *s, double out[6]) {
    if (!s || !out) return fail(NSPNP_ERR_INVALID, "bad diagnostics arguments");
    std::vector<double> ps;
    int rc = plane_reduce(s, ps);
    if (rc) return rc;
    double ke = 0.0, dv = 0.0, mp = 1e300, mm = 1e300, cs = 0.0, pe = 0.0;
    for (int j = 0; j < s->d.M; ++j) {
        const double *r = &ps[(size_t)j * kPlaneQ];
        ke += r[PQ_KE];
        dv = std::fmax(dv, r[PQ_MAX_DIV]);
        mp = std::fmin(mp, r[PQ_MIN_CP]);
        mm = std::fmin(mm, r[PQ_MIN_CM]);
        cs = std::fmax(cs, r[PQ_MAX_CSUM]);
        pe = std::fmax(pe, r[PQ_MAX_DPHI]);
    }
    out[0] = ke;
    out[1] = dv;
    out[2] = mp;
    out[3] = mm;
    out[4] = cs;
    out[5] = pe;
    for (int q = 0; q < 6; ++q)
        if (!std::isfinite(out[q])) return fail(NSPNP_ERR_NONFINITE, "non-finite diagnostics");
    return NSPNP_OK;
}

int nspnp_energy_budget(nspnp_state *s, double out[3]) {
    if (!s || !out) return fail(NSPNP_ERR_INVALID, "bad energy_budget arguments");
    const int M = s->d.M;
    HIP_TRY(launch_energy_sums(s, s->red));
    std::vector<double> h((size_t)4 * M);
    HIP_TRY(hipMemcpyAsync(h.data(), s->red, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    double dis = 0.0, fwk = 0.0;
    for (int j = 0; j < M; ++j) {
        dis += h[4 * (size_t)j];
        fwk += h[4 * (size_t)j + 1];
    }
    const double *dc = host_dc(s);
    const double area = s->d.dx * s->d.dz, ire = s->ph.ire;
    // power of the moving walls against the viscous wall stress
    out[0] = s->cfg.u_top * ire * h[4 * (size_t)(M - 1) + 2] / dc[M] * area -
             s->cfg.u_bot * ire * h[2] / dc[0] * area;
    out[1] = ire * dis;
    out[2] = fwk;
    for (int q = 0; q < 3; ++q)
        if (!std::isfinite(out[q])) return fail(NSPNP_ERR_NONFINITE, "non-finite energy budget");
    return NSPNP_OK;
}

int nspnp_get_clock(nspnp_state *s, double *t, double *dt, int32_t *stage, int64_t *substeps) {
    if (!s) return fail(NSPNP_ERR_INVALID, "state is NULL");
    double c[2];
    HIP_TRY(hipMemcpyAsync(c, s->clock, sizeof(c), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (t) *t = c[0];
    if (dt) *dt = c[1];
    if (stage) *stage = (int32_t)(s->substeps % 3);
    if (substeps) *substeps = s->substeps;
    return NSPNP_OK;
}

int nspnp_set_clock(nspnp_state *s, double t, double dt, int32_t stage, int64_t substeps) {
    if (!s || stage < 0 || stage > 2 || substeps < 0 || substeps % 3 != stage)
        return fail(NSPNP_ERR_INVALID, "bad set_clock arguments (stage must equal substeps mod 3)");
    const double c[kClockSlots] = {t, dt, 0.0, 0.0};  // also clears the health word
    HIP_TRY(hipMemcpyAsync(s->clock, c, sizeof(c), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->host_health) s->host_health[0] = s->host_health[1] = 0.0;
    s->substeps = substeps;
    s->cn_fresh = false;  // dt may have changed
    s->cn_coef_at = -1;
    return NSPNP_OK;
}

int nspnp_set_wall_potential(nspnp_state *s, const double *dev_bot, const double *dev_top) {
    if (!s) return fail(NSPNP_ERR_INVALID, "state is NULL");
    const size_t np = (size_t)s->d.plane;
    const double *src[2] = {dev_bot, dev_top};
    for (int w = 0; w < 2; ++w) {
        double *dst = s->phiw + w * np;
        if (src[w]) HIP_TRY(hipMemcpyAsync(dst, src[w], np * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
        else HIP_TRY(launch_fill(s, dst, (int64_t)np, 0.0));
    }
    s->phiw_on = dev_bot != nullptr || dev_top != nullptr;
    return NSPNP_OK;
}

int nspnp_stats_begin(nspnp_state *s, int32_t every) {
    if (!s || every < 0) return fail(NSPNP_ERR_INVALID, "bad stats_begin arguments");
    if (every > 0) HIP_TRY(launch_run_stats_begin(s));
    s->rstats_every = every;
    return NSPNP_OK;
}

int nspnp_stats_read(nspnp_state *s, double *time, int64_t *samples, double *out) {
    if (!s) return fail(NSPNP_ERR_INVALID, "state is NULL");
    const int M = s->d.M;
    std::vector<double> h((size_t)kRunStatsQ * M + kRunStatsTail);
    HIP_TRY(hipMemcpyAsync(h.data(), s->rstats, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const double T = h[(size_t)kRunStatsQ * M];
    if (time) *time = T;
    if (samples) *samples = (int64_t)h[(size_t)kRunStatsQ * M + 2];
    if (out)
        for (size_t e = 0; e < (size_t)kRunStatsQ * M; ++e) out[e] = T > 0.0 ? h[e] / T : 0.0;
    return NSPNP_OK;
}

int nspnp_stats_derived(nspnp_state *s, double out[6], double *rms, double *y_plus, double *u_plus) {
    if (!s || !out) return fail(NSPNP_ERR_INVALID, "bad stats_derived arguments");
    const int M = s->d.M;
    std::vector<double> h((size_t)kRunStatsQ * M + kRunStatsTail);
    HIP_TRY(hipMemcpyAsync(h.data(), s->rstats, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const double T = h[(size_t)kRunStatsQ * M];
    const double nan = std::nan("");
    auto mean = [&](int q, int j) { return h[(size_t)q * M + j] / T; };
    if (!(T > 0.0)) {  // nothing averaged yet
        for (int q = 0; q < 6; ++q) out[q] = nan;
        for (int e = 0; rms && e < kRunStatsFields * M; ++e) rms[e] = nan;
        for (int j = 0; j < M; ++j) {
            if (y_plus) y_plus[j] = nan;
            if (u_plus) u_plus[j] = nan;
        }
        return NSPNP_OK;
    }
    // wall shear stresses of the time-mean velocity: the viscous flux through
    // the wall faces over the half cell next to each wall (as nspnp_wall_shear_stress)
    const double *dc = host_dc(s), *yc = s->host_tables.data();
    const double tb = s->ph.ire * (mean(0, 0) - s->cfg.u_bot) / dc[0];
    const double tt = s->ph.ire * (s->cfg.u_top - mean(0, M - 1)) / dc[M];
    const double tau = 0.5 * (tb + tt);
    const double ut = std::sqrt(std::fabs(tb));
    out[0] = tb;
    out[1] = tt;
    out[2] = tau;
    out[3] = 2.0 * tau;                             // c_f = tau_w / (rho U^2 / 2)
    out[4] = s->cfg.re * std::sqrt(std::fabs(tau));  // Re_tau = u_tau h / nu
    out[5] = ut;
    if (rms)
        for (int q = 0; q < kRunStatsFields; ++q)
            for (int j = 0; j < M; ++j) {
                const double m = mean(q, j), v = mean(kRunStatsFields + q, j) - m * m;
                rms[(size_t)q * M + j] = std::sqrt(v > 0.0 ? v : 0.0);
            }
    for (int j = 0; j < M; ++j) {  // wall units of the lower wall
        if (y_plus) y_plus[j] = (1.0 + yc[j]) * s->cfg.re * ut;
        if (u_plus) u_plus[j] = ut > 0.0 ? (mean(0, j) - s->cfg.u_bot) / ut : nan;
    }
    return NSPNP_OK;
}

int nspnp_sync(nspnp_state *s) {
    if (!s) return fail(NSPNP_ERR_INVALID, "state is NULL");
    HIP_TRY(hipStreamSynchronize(s->stream));
    return check_health(s, -1);
}

// ---- checkpoints --------------------------------------------------------

namespace {
struct CkptHeader {
    char magic[8];     // "NSPNPCK1"
    uint32_t version;  // 3: followed by CkptStats, the arrays, then the run statistics
    uint32_t word;     // bytes per stored value: 8 (FP64) or 4 (mixed)
    nspnp_config cfg;
    double clock[kClockSlots];
    int64_t substeps;
    int64_t cells;
};
const char kCkptMagic[8] = {'N', 'S', 'P', 'N', 'P', 'C', 'K', '1'};

// Version 2: the run statistics travel with the state, so that a long
// averaging campaign can stop and resume.
struct CkptStats {
    int32_t every;  // sampling interval in substeps (0: not sampling)
    int32_t reserved;
    int64_t count;  // doubles of the statistics block stored after the arrays
};

// Every configuration value that the continuation depends on (seed and noise
// amplitudes only shape the initial state).
bool same_run(const nspnp_config &a, const nspnp_config &b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.precision == b.precision && a.lx == b.lx &&
           a.lz == b.lz && a.stretch == b.stretch && a.re == b.re && a.sc == b.sc && a.beta == b.beta &&
           a.debye == b.debye && a.vhat == b.vhat && a.u_top == b.u_top && a.u_bot == b.u_bot &&
           a.force_sign == b.force_sign && a.dt == b.dt && a.cfl == b.cfl && a.implicit_xz == b.implicit_xz &&
           a.migration_face == b.migration_face;
}

struct FileCloser {
    FILE *f;
    ~FileCloser() { if (f) std::fclose(f); }
};
}  // namespace

int nspnp_save(nspnp_state *s, const char *path) {
    if (!s || !path) return fail(NSPNP_ERR_INVALID, "bad save arguments");
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = 3;
    h.word = (uint32_t)s->wsize;
    h.cfg = s->cfg;
    h.substeps = s->substeps;
    h.cells = s->d.n;
    HIP_TRY(hipMemcpyAsync(h.clock, s->clock, sizeof(h.clock), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    FileCloser fc{std::fopen(path, "wb")};
    if (!fc.f) return fail(NSPNP_ERR_INVALID, std::string("save: cannot open ") + path);
    const CkptStats cs{s->rstats_every, 0, (int64_t)kRunStatsQ * s->d.M + kRunStatsTail};
    if (std::fwrite(&h, sizeof(h), 1, fc.f) != 1 || std::fwrite(&cs, sizeof(cs), 1, fc.f) != 1)
        return fail(NSPNP_ERR_INVALID, "save: write failed");
    const size_t bytes = (size_t)s->d.n * s->wsize;
    std::vector<char> buf(bytes);
    for (int a = 0; a < 12; ++a) {
        const void *src = a < 7 ? s->f[a] : s->h[a - 7];
        HIP_TRY(hipMemcpyAsync(buf.data(), src, bytes, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (std::fwrite(buf.data(), 1, bytes, fc.f) != bytes) return fail(NSPNP_ERR_INVALID, "save: write failed");
    }
    std::vector<double> st((size_t)cs.count);
    HIP_TRY(hipMemcpyAsync(st.data(), s->rstats, st.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (std::fwrite(st.data(), sizeof(double), st.size(), fc.f) != st.size())
        return fail(NSPNP_ERR_INVALID, "save: write failed");
    if (std::fflush(fc.f) != 0) return fail(NSPNP_ERR_INVALID, "save: flush failed");
    return NSPNP_OK;
}

int nspnp_load(nspnp_state *s, const char *path) {
    if (!s || !path) return fail(NSPNP_ERR_INVALID, "bad load arguments");
    FileCloser fc{std::fopen(path, "rb")};
    if (!fc.f) return fail(NSPNP_ERR_INVALID, std::string("load: cannot open ") + path);
    CkptHeader h{};
    // (earlier formats held a shorter configuration record and are not read)
    if (std::fread(&h, sizeof(h), 1, fc.f) != 1 || std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 3)
        return fail(NSPNP_ERR_INVALID, "load: not a checkpoint of this library version");
    CkptStats cs{0, 0, 0};
    if (std::fread(&cs, sizeof(cs), 1, fc.f) != 1 || cs.every < 0 ||
        cs.count != (int64_t)kRunStatsQ * s->d.M + kRunStatsTail)
        return fail(NSPNP_ERR_INVALID, "load: bad statistics record");
    if (h.word != s->wsize || h.cells != s->d.n || !same_run(h.cfg, s->cfg))
        return fail(NSPNP_ERR_INVALID, "load: the checkpoint was written for a different configuration");
    if (h.substeps < 0) return fail(NSPNP_ERR_INVALID, "load: bad substep count");
    const size_t bytes = (size_t)s->d.n * s->wsize;
    std::vector<char> buf(bytes);
    for (int a = 0; a < 12; ++a) {
        if (std::fread(buf.data(), 1, bytes, fc.f) != bytes) return fail(NSPNP_ERR_INVALID, "load: truncated file");
        void *dst = a < 7 ? s->f[a] : s->h[a - 7];
        HIP_TRY(hipMemcpyAsync(dst, buf.data(), bytes, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    {
        std::vector<double> st((size_t)cs.count);
        if (std::fread(st.data(), sizeof(double), st.size(), fc.f) != st.size())
            return fail(NSPNP_ERR_INVALID, "load: truncated file");
        HIP_TRY(hipMemcpyAsync(s->rstats, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    HIP_TRY(hipMemcpyAsync(s->clock, h.clock, sizeof(h.clock), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->substeps = h.substeps;
    s->cn_fresh = false;
    s->cn_coef_at = -1;
    s->rstats_every = cs.every;
    if (s->host_health) {
        s->host_health[0] = h.clock[2];
        s->host_health[1] = h.clock[3];
    }
    return NSPNP_OK;
}

void nspnp_destroy(nspnp_state *s) { delete s; }

}  // extern "C"
