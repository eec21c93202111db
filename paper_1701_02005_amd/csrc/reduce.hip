// reduce.hip -- seeded initial state, adaptive time step and the plane
// reductions behind the diagnostics (wall shear stress and friction of
// Sec. II, ion fluxes through the y-faces of Fig. 1, ion contents, kinetic
// energy, divergence).  Every reduction runs in a fixed order (fixed launch
// shape, fixed LDS tree) so results are bitwise reproducible.
#include <algorithm>

#include "internal.h"

namespace nspnp {
namespace {

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output n of the generator
// seeded with s is mix(s + n * 0x9E3779B97F4A7C15).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n) {
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// uniform on [-1, 1) from stream (field, index)
__device__ __forceinline__ double noise(uint64_t seed, int field, int64_t idx) {
    const uint64_t n = ((uint64_t)field << 40) + (uint64_t)idx + 1ull;
    const double u01 = (double)(splitmix64(seed, n) >> 11) * (1.0 / 9007199254740992.0);
    return 2.0 * u01 - 1.0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_init(Dims d, Tables tb, double u_top, double u_bot, uint64_t seed,
                                              double an, double cn, T *u, T *v, T *w, T *cp, T *cm, T *phi, T *p,
                                              T *h0, T *h1, T *h2, T *h3, T *h4) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    const int j = (int)(q / d.plane);
    const double ulin = 0.5 * (u_top + u_bot) + 0.5 * (u_top - u_bot) * tb.yc[j];
    u[q] = (T)(ulin + an * noise(seed, 0, q));
    v[q] = (T)((j > 0) ? an * noise(seed, 1, q) : 0.0);
    w[q] = (T)(an * noise(seed, 2, q));
    cp[q] = (T)(cn * noise(seed, 3, q));
    cm[q] = (T)(cn * noise(seed, 4, q));
    phi[q] = (T)0;
    p[q] = (T)0;
    h0[q] = h1[q] = h2[q] = h3[q] = h4[q] = (T)0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_shift_conc(Dims d, double mp, double mm, T *cp, T *cm) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    cp[q] = (T)(1.0 + ((double)cp[q] - mp));
    cm[q] = (T)(1.0 + ((double)cm[q] - mm));
}

constexpr int kRedThreads = 256;

// ---- adaptive time step: max of the advective rate and of c+ + c- ----
// Once per Runge-Kutta step: the quantities of the adaptive dt rule and the
// health check of every cell.  Each thread owns one (x, z) column and marches
// a slab of rows, carrying the next row's v and phi (the top-face values of
// the current row) so that every field is read about once.  Per block:
// [0] max CFL rate, [1] max(c+ + c-), [2] min(c+, c-), [3] 1 if any value is
// not finite, [4] max |dPhi| across the cell's x, z and upper y faces.  All
// five are maxima or minima, so the result does not depend on the order.
constexpr int kDtRows = 4;  // rows per load batch of k_dt_partial

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_dt_partial(Dims d, Tables tb, const Phys *phys, const T *u,
                                                            const T *v, const T *w, const T *cp, const T *cm,
                                                            const T *phi, double *part, int chunks,
                                                            int slab_rows, size_t ms) {
    __shared__ double s[kDtParts][kRedThreads];
    u = member_ptr(u, ms); v = member_ptr(v, ms); w = member_ptr(w, ms);
    cp = member_ptr(cp, ms); cm = member_ptr(cm, ms); phi = member_ptr(phi, ms); part = member_ptr(part, ms);
    const double e0 = member_ptr(phys, ms)->e0;
    double rate = 0.0, cmax = 0.0, cmin = 1e300, pe = 0.0;
    bool bad = false;
    // XCD-aware order: consecutive z-lines (chunks) run on one XCD, so the
    // z-neighbour line each reads comes from that XCD's L2
    const unsigned bt = xcd_tile(blockIdx.x, gridDim.x);
    const int chunk = (int)(bt % (unsigned)chunks), slab = (int)(bt / (unsigned)chunks);
    const int64_t pl = d.plane;
    const int64_t e = (int64_t)chunk * blockDim.x + threadIdx.x;
    const int j0 = slab * slab_rows;
    const int j1 = (j0 + slab_rows < d.M) ? j0 + slab_rows : d.M;
    if (e < pl && j0 < j1) {
        const int i = (int)(e % d.nx), k = (int)(e / d.nx);
        const int64_t exp_ = e - i + ((i + 1 == d.nx) ? 0 : i + 1);
        const int64_t ezp = e + (int64_t)(((k + 1 == d.nz) ? 0 : k + 1) - k) * d.nx;
        double v0 = (double)v[(int64_t)j0 * pl + e], f0 = (double)phi[(int64_t)j0 * pl + e];
        // Rows are reduced in batches of kDtRows: the batch's loads are all
        // issued before any is used (rows past the slab re-read its last row
        // and are ignored), one memory latency per batch.  Offsets within
        // one field fit in 32 bits.
        const unsigned upl = (unsigned)pl, ue = (unsigned)e, uxp = (unsigned)exp_, uzp = (unsigned)ezp;
        struct RowVals {
            T v1, f1, u0, w0, c1, c2, ux, wz, fx, fz;
        };
        auto load_row = [&](int j, RowVals &r) {
            const unsigned row = (unsigned)j * upl, q = row + ue;
            const unsigned qt = (j + 1 < d.M) ? q + upl : q;
            r.v1 = v[qt];
            r.f1 = phi[qt];
            r.u0 = u[q];
            r.w0 = w[q];
            r.c1 = ld_once(cp + q);
            r.c2 = ld_once(cm + q);
            r.ux = u[row + uxp];
            r.wz = w[row + uzp];
            r.fx = phi[row + uxp];
            r.fz = phi[row + uzp];
        };
        for (int jb = j0; jb < j1; jb += kDtRows) {
            RowVals rb[kDtRows];
#pragma unroll
            for (int t = 0; t < kDtRows; ++t) load_row(jb + t < j1 ? jb + t : j1 - 1, rb[t]);
#pragma unroll
            for (int t = 0; t < kDtRows; ++t) {
                const int j = jb + t;
                if (j >= j1) break;
                const RowVals &cur = rb[t];
                const bool top = j + 1 < d.M;
                const double v1 = top ? (double)cur.v1 : 0.0;
                const double f1 = top ? (double)cur.f1 : 0.0;
                const double u0 = (double)cur.u0, w0 = (double)cur.w0;
                const double c1 = (double)cur.c1, c2 = (double)cur.c2;
                const double uc = 0.5 * (u0 + (double)cur.ux);
                const double vc = 0.5 * (v0 + v1);
                const double wc = 0.5 * (w0 + (double)cur.wz);
                rate = fmax(rate, fabs(uc) / d.dx + fabs(vc) / uniform_load(tb.dn, j) + fabs(wc) / d.dz);
                cmax = fmax(cmax, c1 + c2);
                cmin = fmin(cmin, fmin(c1, c2));
                bad = bad || !__builtin_isfinite(u0) || !__builtin_isfinite(v0) || !__builtin_isfinite(w0) ||
                      !__builtin_isfinite(c1) || !__builtin_isfinite(c2) || !__builtin_isfinite(f0);
                double dphi = fmax(fabs((double)cur.fx - f0), fabs((double)cur.fz - f0));
                if (top) dphi = fmax(dphi, fabs(f1 - f0 + e0 * uniform_load(tb.dc, j + 1)));
                pe = fmax(pe, dphi);
                v0 = v1;
                f0 = f1;
            }
        }
    }
    s[0][threadIdx.x] = rate;
    s[1][threadIdx.x] = cmax;
    s[2][threadIdx.x] = cmin;
    s[3][threadIdx.x] = bad ? 1.0 : 0.0;
    s[4][threadIdx.x] = pe;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + o]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + o]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + o]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + o]);
            s[4][threadIdx.x] = fmax(s[4][threadIdx.x], s[4][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < kDtParts) part[kDtParts * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

// Combines the partials: the step dt (adaptive runs only, Sec. II time
// stepping with the limits of include/nspnp.h) and the sticky health word.
__global__ void __launch_bounds__(kRedThreads) k_dt_final(int nparts, const double *part, const Phys *phys,
                                                          Dims d, double *clock, size_t ms) {
    __shared__ double s[kDtParts][kRedThreads];
    part = member_ptr(part, ms);
    clock = member_ptr(clock, ms);
    const Phys ph = *member_ptr(phys, ms);
    double acc[kDtParts] = {0.0, 0.0, 1e300, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
        acc[0] = fmax(acc[0], part[kDtParts * b + 0]);
        acc[1] = fmax(acc[1], part[kDtParts * b + 1]);
        acc[2] = fmin(acc[2], part[kDtParts * b + 2]);
        acc[3] = fmax(acc[3], part[kDtParts * b + 3]);
        acc[4] = fmax(acc[4], part[kDtParts * b + 4]);
    }
#pragma unroll
    for (int q = 0; q < kDtParts; ++q) s[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + o]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + o]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + o]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + o]);
            s[4][threadIdx.x] = fmax(s[4][threadIdx.x], s[4][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double re = ph.re, rs = 1.0 / ph.kd;
        double dt = 1e30;
        if (s[0][0] > 0.0) dt = ph.cfl / s[0][0];
        if (s[1][0] > 0.0) dt = fmin(dt, 2.0 * ph.debye * ph.debye * rs / s[1][0]);
        const double nu_min = re < rs ? re : rs;
        if (ph.implicit_xz == 0.0)  // explicit x/z diffusion limit
            dt = fmin(dt, nu_min / (4.0 / (d.dx * d.dx) + 4.0 / (d.dz * d.dz)));
        int bits = (int)clock[2];
        if (s[3][0] != 0.0) bits |= kHealthNonFinite;
        if (s[2][0] < 0.0) bits |= kHealthNegative;
        if (ph.adaptive != 0.0) {
            if (!(dt > 0.0) || !__builtin_isfinite(dt)) bits |= kHealthNonFinite;
            else clock[1] = dt;
        }
        clock[2] = (double)bits;
        clock[3] = s[4][0];
    }
}

// ---- per-plane sums for diagnostics ----
// out[j * kPlaneQ + q], q as in PlaneQ: sums of u, c+, c-; total ion fluxes
// at node j; kinetic energy of row j; max |div u|; min c+, min c-,
// max (c+ + c-); max |dPhi| across the x, z and lower y faces of row j.

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_plane(Dims d, const Phys *phys, Tables tb, const T *u, const T *v,
                                                       const T *w, const T *cp, const T *cm, const T *phi,
                                                       double *out, size_t ms) {
    __shared__ double s[kPlaneQ][kRedThreads];
    u = member_ptr(u, ms); v = member_ptr(v, ms); w = member_ptr(w, ms);
    cp = member_ptr(cp, ms); cm = member_ptr(cm, ms); phi = member_ptr(phi, ms); out = member_ptr(out, ms);
    const Phys ph = *member_ptr(phys, ms);
    const int j = blockIdx.x;
    const int64_t pl = d.plane;
    const int64_t base = (int64_t)j * pl;
    double acc[kPlaneQ] = {0, 0, 0, 0, 0, 0, 0, 1e300, 1e300, 0, 0};
    static_assert(kPlaneQ == 11, "plane quantities");
    const double dn = tb.dn[j];
    const double dcj = tb.dc[j];
    for (int64_t e = threadIdx.x; e < pl; e += blockDim.x) {
        const int64_t q = base + e;
        const int i = (int)(e % d.nx), k = (int)(e / d.nx);
        const int64_t xp = q - i + ((i + 1 == d.nx) ? 0 : i + 1);
        const int64_t zp = q + (int64_t)(((k + 1 == d.nz) ? 0 : k + 1) - k) * d.nx;
        const double uu = (double)u[q], ww = (double)w[q], vv = (double)v[q];
        const double c1 = (double)cp[q], c2 = (double)cm[q];
        acc[0] += uu;
        acc[1] += c1;
        acc[2] += c2;
        if (j > 0) {
            const int64_t qd = q - pl;
            const double e_y = ph.e0 + ((double)phi[q] - (double)phi[qd]) / dcj;
            const double m1 = 0.5 * (c1 + (double)cp[qd]);
            const double m2 = 0.5 * (c2 + (double)cm[qd]);
            // advective face values: the mean, or the limited upwind value
            double f1 = m1, f2 = m2;
            if (ph.limited != 0.0) {
                const bool up = vv >= 0.0, have = up ? (j > 1) : (j + 1 < d.M);
                const int64_t quu = up ? q - 2 * pl : q + pl;
                f1 = adv_face((double)cp[qd], c1, have ? (double)cp[quu] : 0.0, up, have);
                f2 = adv_face((double)cm[qd], c2, have ? (double)cm[quu] : 0.0, up, have);
            }
            // migration face values (hybrid rule: upwind where |dPhi| >= 2)
            const bool hyb = ph.hybrid != 0.0;
            const double dpy = hyb ? y_dphi(ph.e0, dcj, (double)phi[q] - (double)phi[qd]) : 0.0;
            const double g1 = mig_face(hyb, m1, (double)cp[qd], c1, dpy, 1.0);
            const double g2 = mig_face(hyb, m2, (double)cm[qd], c2, dpy, -1.0);
            acc[3] += vv * f1 - ph.kd * ((c1 - (double)cp[qd]) / dcj + g1 * e_y);
            acc[4] += vv * f2 - ph.kd * ((c2 - (double)cm[qd]) / dcj - g2 * e_y);
            acc[5] += 0.5 * vv * vv * d.dx * dcj * d.dz;
            acc[10] = fmax(acc[10], fabs((double)phi[q] - (double)phi[qd] + ph.e0 * dcj));
        }
        const double f0 = (double)phi[q];
        acc[10] = fmax(acc[10], fmax(fabs((double)phi[xp] - f0), fabs((double)phi[zp] - f0)));
        acc[5] += 0.5 * (uu * uu + ww * ww) * d.dx * dn * d.dz;
        const double vt = (j + 1 < d.M) ? (double)v[q + pl] : 0.0;
        const double vb = (j > 0) ? vv : 0.0;
        const double div = ((double)u[xp] - uu) / d.dx + (vt - vb) / dn + ((double)w[zp] - ww) / d.dz;
        acc[6] = fmax(acc[6], fabs(div));
        acc[7] = fmin(acc[7], c1);
        acc[8] = fmin(acc[8], c2);
        acc[9] = fmax(acc[9], c1 + c2);
    }
#pragma unroll
    for (int qq = 0; qq < kPlaneQ; ++qq) s[qq][threadIdx.x] = acc[qq];
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            for (int qq = 0; qq < 6; ++qq) s[qq][threadIdx.x] += s[qq][threadIdx.x + o];
            s[6][threadIdx.x] = fmax(s[6][threadIdx.x], s[6][threadIdx.x + o]);
            s[7][threadIdx.x] = fmin(s[7][threadIdx.x], s[7][threadIdx.x + o]);
            s[8][threadIdx.x] = fmin(s[8][threadIdx.x], s[8][threadIdx.x + o]);
            s[9][threadIdx.x] = fmax(s[9][threadIdx.x], s[9][threadIdx.x + o]);
            s[10][threadIdx.x] = fmax(s[10][threadIdx.x], s[10][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < kPlaneQ) out[(int64_t)j * kPlaneQ + threadIdx.x] = s[threadIdx.x][0];
}

// Kinetic-energy budget terms of one cell row (one block per row), in the
// volume-weighted forms of the semi-discrete equations:
//   out[4 j + 0]  sum over the row's velocity unknowns of |grad u|^2 times the
//                 control volume of each difference (x, z differences of u, w
//                 and v; y differences of u, w across centre rows and of v
//                 across cell rows; the half cells next to the walls in rows
//                 0 and M-1), so that Re^-1 times its total is the dissipation
//   out[4 j + 1]  sum of u . f Omega, f the Coulomb force at the u, v, w points
//   out[4 j + 2]  row 0: sum of (u - u_bot); row M-1: sum of (u_top - u)
//   out[4 j + 3]  0
// The wall work follows on the host from out[2] of the two wall rows.
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_energy(Dims d, const Phys *phys, Tables tb, const T *u, const T *v,
                                                        const T *w, const T *cp, const T *cm, const T *phi,
                                                        double *out, size_t ms) {
    __shared__ double s[3][kRedThreads];
    u = member_ptr(u, ms); v = member_ptr(v, ms); w = member_ptr(w, ms);
    cp = member_ptr(cp, ms); cm = member_ptr(cm, ms); phi = member_ptr(phi, ms); out = member_ptr(out, ms);
    const Phys ph = *member_ptr(phys, ms);
    const int j = blockIdx.x, M = d.M;
    const int64_t pl = d.plane;
    const int64_t base = (int64_t)j * pl;
    const double dx = d.dx, dz = d.dz, dn = tb.dn[j];
    const double dcj = tb.dc[j], dcu = tb.dc[j + 1], dc0 = tb.dc[0], dcM = tb.dc[M];
    double dis = 0.0, fwk = 0.0, wall = 0.0;
    for (int64_t e = threadIdx.x; e < pl; e += blockDim.x) {
        const int64_t q = base + e;
        const int i = (int)(e % d.nx), k = (int)(e / d.nx);
        const int64_t xp = q - i + ((i + 1 == d.nx) ? 0 : i + 1);
        const int64_t xm = q - i + ((i == 0) ? d.nx - 1 : i - 1);
        const int64_t zp = q + (int64_t)(((k + 1 == d.nz) ? 0 : k + 1) - k) * d.nx;
        const int64_t zm = q + (int64_t)(((k == 0) ? d.nz - 1 : k - 1) - k) * d.nx;
        const double uu = (double)u[q], vv = (double)v[q], ww = (double)w[q];
        const double gux = ((double)u[xp] - uu) / dx, guz = ((double)u[zp] - uu) / dz;
        const double gwx = ((double)w[xp] - ww) / dx, gwz = ((double)w[zp] - ww) / dz;
        dis += (gux * gux + guz * guz + gwx * gwx + gwz * gwz) * dx * dn * dz;
        if (j + 1 < M) {
            const double guy = ((double)u[q + pl] - uu) / dcu, gwy = ((double)w[q + pl] - ww) / dcu;
            dis += (guy * guy + gwy * gwy) * dx * dcu * dz;
        }
        if (j > 0) {
            const double gvx = ((double)v[xp] - vv) / dx, gvz = ((double)v[zp] - vv) / dz;
            dis += (gvx * gvx + gvz * gvz) * dx * dcj * dz;
        }
        {
            const double vb = (j > 0) ? vv : 0.0, vt = (j + 1 < M) ? (double)v[q + pl] : 0.0;
            const double gvy = (vt - vb) / dn;
            dis += gvy * gvy * dx * dn * dz;
        }
        if (j == 0) {
            const double gub = (uu - ph.u_bot) / dc0, gwb = ww / dc0;
            dis += (gub * gub + gwb * gwb) * dx * dc0 * dz;
            wall += uu - ph.u_bot;
        }
        if (j == M - 1) {
            const double gut = (ph.u_top - uu) / dcM, gwt = -ww / dcM;
            dis += (gut * gut + gwt * gwt) * dx * dcM * dz;
            wall += ph.u_top - uu;
        }
        // Coulomb force sF K rho_face grad Phi at the u, w and v points
        const double f0 = (double)phi[q];
        const double r0 = (double)cp[q] - (double)cm[q];
        const double fu = ph.kf * 0.5 * (r0 + (double)cp[xm] - (double)cm[xm]) * (f0 - (double)phi[xm]) / dx;
        const double fw = ph.kf * 0.5 * (r0 + (double)cp[zm] - (double)cm[zm]) * (f0 - (double)phi[zm]) / dz;
        fwk += (uu * fu + ww * fw) * dx * dn * dz;
        if (j > 0) {
            const int64_t qd = q - pl;
            const double ey = ph.e0 + (f0 - (double)phi[qd]) / dcj;
            const double fv = ph.kf * 0.5 * (r0 + (double)cp[qd] - (double)cm[qd]) * ey;
            fwk += vv * fv * dx * dcj * dz;
        }
    }
    s[0][threadIdx.x] = dis;
    s[1][threadIdx.x] = fwk;
    s[2][threadIdx.x] = wall;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int qq = 0; qq < 3; ++qq) s[qq][threadIdx.x] += s[qq][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[(int64_t)j * 4 + threadIdx.x] = threadIdx.x < 3 ? s[threadIdx.x][0] : 0.0;
}

// time sums (weight alp dt) of the plane means of u, c+ - c- and phi per row
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_stats(Dims d, const T *u, const T *cp, const T *cm, const T *phi,
                                                       const double *clock, double *stats, double alp, size_t ms) {
    __shared__ double s[3][kRedThreads];
    u = member_ptr(u, ms); cp = member_ptr(cp, ms); cm = member_ptr(cm, ms); phi = member_ptr(phi, ms);
    clock = member_ptr(clock, ms);
    stats = member_ptr(stats, ms);
    const int j = blockIdx.x;
    const int64_t base = (int64_t)j * d.plane;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t e = threadIdx.x; e < d.plane; e += blockDim.x) {
        const int64_t q = base + e;
        a0 += (double)u[q];
        a1 += (double)cp[q] - (double)cm[q];
        a2 += (double)phi[q];
    }
    s[0][threadIdx.x] = a0;
    s[1][threadIdx.x] = a1;
    s[2][threadIdx.x] = a2;
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int qq = 0; qq < 3; ++qq) s[qq][threadIdx.x] += s[qq][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double wgt = alp * clock[1];
        const double inv = 1.0 / (double)d.plane;
        for (int qq = 0; qq < 3; ++qq) stats[3 * j + qq] += wgt * s[qq][0] * inv;
        if (j == 0) stats[3 * d.M] += wgt;
    }
}

__global__ void k_fill(double *p, int64_t n, double v, size_t ms) {
    p = member_ptr(p, ms);
    for (int64_t q = threadIdx.x; q < n; q += blockDim.x) p[q] = v;
}

inline dim3 grid1(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

hipError_t launch_init_fields(nspnp_state *s) {
    const nspnp_config &c = s->cfg;
    if (s->fp64) {
        double **f = (double **)s->f;
        double **h = (double **)s->h;
        k_init<double><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d, s->tb, c.u_top, c.u_bot, c.seed, c.u_noise,
                                                            c.c_noise, f[0], f[1], f[2], f[3], f[4], f[5], f[6],
                                                            h[0], h[1], h[2], h[3], h[4]);
    } else {
        float **f = (float **)s->f;
        float **h = (float **)s->h;
        k_init<float><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d, s->tb, c.u_top, c.u_bot, c.seed, c.u_noise,
                                                           c.c_noise, f[0], f[1], f[2], f[3], f[4], f[5], f[6],
                                                           h[0], h[1], h[2], h[3], h[4]);
    }
    return hipGetLastError();
}

hipError_t launch_shift_conc(nspnp_state *s, double mp, double mm) {
    if (s->fp64)
        k_shift_conc<double><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d, mp, mm, (double *)s->f[3], (double *)s->f[4]);
    else
        k_shift_conc<float><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d, mp, mm, (float *)s->f[3], (float *)s->f[4]);
    return hipGetLastError();
}

hipError_t launch_dt(nspnp_state *s) {
    ProfScope prof_(s, K_DT);
    // columns in chunks of one block; rows split into slabs so that the
    // partials fit kDtMaxBlocks per member
    static_assert(kDtThreads == kRedThreads, "dt block size");
    const int chunks = dt_chunks(s->d.plane);
    const int slabs = std::max(1, std::min(s->d.M, kDtMaxBlocks / chunks));
    const int slab_rows = (s->d.M + slabs - 1) / slabs;
    const unsigned nb = (unsigned)(chunks * ((s->d.M + slab_rows - 1) / slab_rows));
    if ((int64_t)nb * kDtParts > s->nred) return hipErrorInvalidValue;  // the layout sized red for this
    const dim3 g(nb, 1, (unsigned)s->nmem);
    if (s->fp64)
        k_dt_partial<double><<<g, kRedThreads, 0, s->stream>>>(
            s->d, s->tb, s->d_phys, (const double *)s->f[0], (const double *)s->f[1], (const double *)s->f[2],
            (const double *)s->f[3], (const double *)s->f[4], (const double *)s->f[5], s->red, chunks, slab_rows,
            s->mstride);
    else
        k_dt_partial<float><<<g, kRedThreads, 0, s->stream>>>(
            s->d, s->tb, s->d_phys, (const float *)s->f[0], (const float *)s->f[1], (const float *)s->f[2],
            (const float *)s->f[3], (const float *)s->f[4], (const float *)s->f[5], s->red, chunks, slab_rows,
            s->mstride);
    k_dt_final<<<dim3(1, 1, (unsigned)s->nmem), kRedThreads, 0, s->stream>>>((int)nb, s->red, s->d_phys, s->d,
                                                                             s->clock, s->mstride);
    return hipGetLastError();
}

// per-plane sums of every member (results in each member's dev_out copy)
hipError_t launch_plane_sums(nspnp_state *s, int /*what*/, double *dev_out) {
    const dim3 g((unsigned)s->d.M, 1, (unsigned)s->nmem);
    if (s->fp64)
        k_plane<double><<<g, kRedThreads, 0, s->stream>>>(
            s->d, s->d_phys, s->tb, (const double *)s->f[0], (const double *)s->f[1], (const double *)s->f[2],
            (const double *)s->f[3], (const double *)s->f[4], (const double *)s->f[5], dev_out, s->mstride);
    else
        k_plane<float><<<g, kRedThreads, 0, s->stream>>>(
            s->d, s->d_phys, s->tb, (const float *)s->f[0], (const float *)s->f[1], (const float *)s->f[2],
            (const float *)s->f[3], (const float *)s->f[4], (const float *)s->f[5], dev_out, s->mstride);
    return hipGetLastError();
}

// energy-budget partial sums, 4 per row (k_energy)
hipError_t launch_energy_sums(nspnp_state *s, double *dev_out) {
    const dim3 g((unsigned)s->d.M, 1, (unsigned)s->nmem);
    if (s->fp64)
        k_energy<double><<<g, kRedThreads, 0, s->stream>>>(
            s->d, s->d_phys, s->tb, (const double *)s->f[0], (const double *)s->f[1], (const double *)s->f[2],
            (const double *)s->f[3], (const double *)s->f[4], (const double *)s->f[5], dev_out, s->mstride);
    else
        k_energy<float><<<g, kRedThreads, 0, s->stream>>>(
            s->d, s->d_phys, s->tb, (const float *)s->f[0], (const float *)s->f[1], (const float *)s->f[2],
            (const float *)s->f[3], (const float *)s->f[4], (const float *)s->f[5], dev_out, s->mstride);
    return hipGetLastError();
}

// n doubles at p (on this handle's device) set to v, on the solver's stream
hipError_t launch_fill(nspnp_state *s, double *p, int64_t n, double v) {
    k_fill<<<dim3(1, 1, 1), 256, 0, s->stream>>>(p, n, v, 0);
    return hipGetLastError();
}

hipError_t launch_stats_reset(nspnp_state *s) {
    k_fill<<<dim3(1, 1, (unsigned)s->nmem), 256, 0, s->stream>>>(s->stats, 3 * (int64_t)s->d.M + 2, 0.0, s->mstride);
    return hipGetLastError();
}

namespace {

// Run statistics (the averages behind mean and RMS profiles, Sec. III).
// k_run_stats: block (chunk, row j) sums q and q^2 for q = u, v, w, c+, c-,
// phi, p over its part of the row, in batches of kStatBatch elements per
// thread whose loads are all issued first, and writes the kRunStatsQ sums to
// the scratch slot (j, chunk).  k_run_stats_close: thread (j, q) adds the chunks
// in order and accumulates w * (plane mean) with w = t - t_last, the time
// since the previous sample (t from the device clock, after this substep's
// advance); k_run_stats_tail then adds w to the accumulated time and sets
// t_last = t.  The
// sums never depend on timing (no atomics), so runs repeat bit for bit.
constexpr int kStatBatch = 4;

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_run_stats(Dims d, const T *f0, const T *f1, const T *f2, const T *f3,
                                                           const T *f4, const T *f5, const T *f6, double *part,
                                                           int chunks, size_t ms) {
    __shared__ double sm[kRunStatsQ][kRedThreads / 64];
    const T *f[kRunStatsFields] = {member_ptr(f0, ms), member_ptr(f1, ms), member_ptr(f2, ms), member_ptr(f3, ms),
                                   member_ptr(f4, ms), member_ptr(f5, ms), member_ptr(f6, ms)};
    part = member_ptr(part, ms);
    const int chunk = blockIdx.x, j = blockIdx.y;
    const int pl = (int)d.plane;
    const int per = (pl + chunks - 1) / chunks;
    const int e_lo = chunk * per, e_hi = (e_lo + per < pl) ? e_lo + per : pl;
    const unsigned base = (unsigned)j * (unsigned)pl;
    const int bd = (int)blockDim.x;
    double a[kRunStatsQ];
#pragma unroll
    for (int q = 0; q < kRunStatsQ; ++q) a[q] = 0.0;
    for (int e0 = e_lo + (int)threadIdx.x; e0 < e_hi; e0 += kStatBatch * bd) {
        T x[kStatBatch][kRunStatsFields];
#pragma unroll
        for (int u = 0; u < kStatBatch; ++u) {
            const int e = (e0 + u * bd < e_hi) ? e0 + u * bd : e0;  // in range; dropped below
#pragma unroll
            for (int q = 0; q < kRunStatsFields; ++q) x[u][q] = f[q][base + (unsigned)e];
        }
#pragma unroll
        for (int u = 0; u < kStatBatch; ++u) {
            if (e0 + u * bd < e_hi) {
#pragma unroll
                for (int q = 0; q < kRunStatsFields; ++q) {
                    const double v = (double)x[u][q];
                    a[q] += v;
                    a[kRunStatsFields + q] += v * v;
                }
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kRunStatsQ; ++q) {
        double v = a[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) sm[q][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < kRunStatsQ) {
        const int q = threadIdx.x;
        double v = 0.0;
        for (int w = 0; w < (bd >> 6); ++w) v += sm[q][w];
        part[((size_t)j * chunks + chunk) * kRunStatsQ + q] = v;
    }
}

__global__ void __launch_bounds__(kStatCloseThreads) k_run_stats_close(Dims d, const double *part, int chunks,
                                                                       const double *clock, double *rs, size_t ms) {
    part = member_ptr(part, ms);
    clock = member_ptr(clock, ms);
    rs = member_ptr(rs, ms);
    const int M = d.M;
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= M * kRunStatsQ) return;
    const int j = t / kRunStatsQ, q = t - j * kRunStatsQ;
    const double wgt = clock[0] - rs[kRunStatsQ * M + 1];
    const double *pj = part + (size_t)j * chunks * kRunStatsQ + q;
    double v = 0.0;
    for (int c0 = 0; c0 < chunks; c0 += 8) {  // chunks in order, 8 loads in flight
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = pj[(size_t)(c0 + u < chunks ? c0 + u : c0) * kRunStatsQ];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (c0 + u < chunks) v += x[u];
    }
    rs[q * M + j] += wgt * (v / (double)d.plane);
}

// after k_run_stats_close (which reads t_last): accumulated time, t_last, count
__global__ void k_run_stats_tail(int M, const double *clock, double *rs, size_t ms) {
    clock = member_ptr(clock, ms);
    rs = member_ptr(rs, ms);
    if (threadIdx.x == 0) {
        double *tail = rs + kRunStatsQ * M;
        tail[0] += clock[0] - tail[1];
        tail[1] = clock[0];
        tail[2] += 1.0;
    }
}

// Clear the run statistics and take the current time as the start.
__global__ void k_run_stats_begin(int M, const double *clock, double *rs, size_t ms) {
    clock = member_ptr(clock, ms);
    rs = member_ptr(rs, ms);
    const int n = kRunStatsQ * M + kRunStatsTail;
    for (int e = threadIdx.x; e < n; e += blockDim.x) rs[e] = (e == kRunStatsQ * M + 1) ? clock[0] : 0.0;
}

}  // namespace

hipError_t launch_run_stats_begin(nspnp_state *s) {
    k_run_stats_begin<<<dim3(1, 1, (unsigned)s->nmem), 256, 0, s->stream>>>(s->d.M, s->clock, s->rstats, s->mstride);
    return hipGetLastError();
}

hipError_t launch_run_stats(nspnp_state *s) {
    ProfScope prof_(s, K_STATS);
    const int chunks = run_stats_chunks(s->d.M);
    if ((int64_t)s->d.M * chunks * kRunStatsQ > s->nred) return hipErrorInvalidValue;  // the layout sized red for this
    const dim3 g((unsigned)chunks, (unsigned)s->d.M, (unsigned)s->nmem);
    if (s->fp64)
        k_run_stats<double><<<g, kRedThreads, 0, s->stream>>>(
            s->d, (const double *)s->f[0], (const double *)s->f[1], (const double *)s->f[2], (const double *)s->f[3],
            (const double *)s->f[4], (const double *)s->f[5], (const double *)s->f[6], s->red, chunks, s->mstride);
    else
        k_run_stats<float><<<g, kRedThreads, 0, s->stream>>>(
            s->d, (const float *)s->f[0], (const float *)s->f[1], (const float *)s->f[2], (const float *)s->f[3],
            (const float *)s->f[4], (const float *)s->f[5], (const float *)s->f[6], s->red, chunks, s->mstride);
    const unsigned nclose = (unsigned)((s->d.M * kRunStatsQ + kStatCloseThreads - 1) / kStatCloseThreads);
    k_run_stats_close<<<dim3(nclose, 1, (unsigned)s->nmem), kStatCloseThreads, 0, s->stream>>>(
        s->d, s->red, chunks, s->clock, s->rstats, s->mstride);
    k_run_stats_tail<<<dim3(1, 1, (unsigned)s->nmem), 64, 0, s->stream>>>(s->d.M, s->clock, s->rstats, s->mstride);
    return hipGetLastError();
}

hipError_t launch_stats_accum(nspnp_state *s, double alp) {
    const dim3 g((unsigned)s->d.M, 1, (unsigned)s->nmem);
    if (s->fp64)
        k_stats<double><<<g, kRedThreads, 0, s->stream>>>(s->d, (const double *)s->f[0], (const double *)s->f[3],
                                                          (const double *)s->f[4], (const double *)s->f[5], s->clock,
                                                          s->stats, alp, s->mstride);
    else
        k_stats<float><<<g, kRedThreads, 0, s->stream>>>(s->d, (const float *)s->f[0], (const float *)s->f[3],
                                                         (const float *)s->f[4], (const float *)s->f[5], s->clock,
                                                         s->stats, alp, s->mstride);
    return hipGetLastError();
}

}  // namespace nspnp
