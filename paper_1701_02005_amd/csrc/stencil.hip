// stencil.hip -- explicit right-hand sides, Crank-Nicolson wall-normal
// solves, divergence and projection correction of one Runge-Kutta substep of
// the NS-PNP scheme (Sec. II, Eqs. (1)-(3), Fig. 1), for gfx950.
//
// Layout: every field is [j][k][i] (i = x fastest, k = z, j = cell row).
// u lives on x-faces, w on z-faces, v on the bottom y-face of each row (row 0
// is the wall), c+-, phi and p at cell centres.  T is the storage and stencil
// type: double for the FP64 form, float for the mixed form.
#include "internal.h"

namespace nspnp {
namespace {

struct Idx {
    int i, j, k, ip, im, kp, km;
    int64_t c0, xp, xm, zp, zm;
};

__device__ __forceinline__ Idx make_idx(const Dims &d, int64_t q) {
    Idx t;
    t.i = (int)(q % d.nx);
    int64_t r = q / d.nx;
    t.k = (int)(r % d.nz);
    t.j = (int)(r / d.nz);
    t.ip = (t.i + 1 == d.nx) ? 0 : t.i + 1;
    t.im = (t.i == 0) ? d.nx - 1 : t.i - 1;
    t.kp = (t.k + 1 == d.nz) ? 0 : t.k + 1;
    t.km = (t.k == 0) ? d.nz - 1 : t.k - 1;
    t.c0 = q;
    t.xp = q - t.i + t.ip;
    t.xm = q - t.i + t.im;
    t.zp = q + (int64_t)(t.kp - t.k) * d.nx;
    t.zm = q + (int64_t)(t.km - t.k) * d.nx;
    return t;
}

struct ExplicitArgs {
    Dims d;
    Phys ph;
    Tables tb;
    Stage st;
    const void *u, *v, *w, *cp, *cm, *phi, *p;
    void *h[5];
    double *r[5];
    double *dbg[5];
    const double *clock;
    int mode;  // 0: substep (H update + CN right-hand sides); 1: H to dbg only
};

// Convection, horizontal diffusion, Coulomb force and ion transport at one
// cell, then the Crank-Nicolson right-hand side
//   r = dt [gam H^k + zet H^{k-1} - alp G p + alp nu L_y q].
template <typename T>
__global__ void __launch_bounds__(256) k_explicit(ExplicitArgs a) {
    const Dims &d = a.d;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    const T *__restrict__ u = (const T *)a.u;
    const T *__restrict__ v = (const T *)a.v;
    const T *__restrict__ w = (const T *)a.w;
    const T *__restrict__ cp = (const T *)a.cp;
    const T *__restrict__ cm = (const T *)a.cm;
    const T *__restrict__ phi = (const T *)a.phi;
    const T *__restrict__ p = (const T *)a.p;
    const Idx x = make_idx(d, q);
    const int j = x.j, M = d.M;
    const int64_t pl = d.plane;
    const bool has_up = (j + 1 < M), has_dn = (j > 0);
    const int64_t yp = q + pl, ym = q - pl;
    const T half = T(0.5);
    const T idx_ = T(1.0 / d.dx), idz_ = T(1.0 / d.dz);
    const T dnj = T(a.tb.dn[j]);
    const T idn = T(1) / dnj;
    const T ix2 = idx_ * idx_, iz2 = idz_ * idz_;

    const T uc = u[q], vc = v[q], wc = w[q];

    // ---------------- u on the x-face ----------------
    T hu;
    {
        const T uxp = u[x.xp], uxm = u[x.xm];
        const T a1 = half * (uxp + uc), a2 = half * (uc + uxm);
        const T cx = (a1 * a1 - a2 * a2) * idx_;
        T cy_t = T(0), cy_b = T(0);
        if (has_up) cy_t = half * (v[yp] + v[yp - x.i + x.im]) * half * (u[yp] + uc);
        if (has_dn) cy_b = half * (vc + v[x.xm]) * half * (uc + u[ym]);
        const T cy = (cy_t - cy_b) * idn;
        const T wf = half * (w[x.zp] + w[x.zp - x.i + x.im]);
        const T wb = half * (wc + w[x.xm]);
        const T cz = (wf * half * (u[x.zp] + uc) - wb * half * (uc + u[x.zm])) * idz_;
        const T lap = (uxp - T(2) * uc + uxm) * ix2 + (u[x.zp] - T(2) * uc + u[x.zm]) * iz2;
        const T rho0 = cp[q] - cm[q], rhox = cp[x.xm] - cm[x.xm];
        const T f = T(a.ph.kf) * half * (rho0 + rhox) * (phi[q] - phi[x.xm]) * idx_;
        hu = -(cx + cy + cz) + T(a.ph.ire) * lap + f;
    }
    // ---------------- w on the z-face ----------------
    T hw;
    {
        const T wzp = w[x.zp], wzm = w[x.zm];
        const T a1 = half * (wzp + wc), a2 = half * (wc + wzm);
        const T cz = (a1 * a1 - a2 * a2) * idz_;
        const T ur = half * (u[x.xp] + u[x.zm - x.i + x.ip]);
        const T ul = half * (uc + u[x.zm]);
        const T cx = (ur * half * (w[x.xp] + wc) - ul * half * (wc + w[x.xm])) * idx_;
        T cy_t = T(0), cy_b = T(0);
        if (has_up) cy_t = half * (v[yp] + v[yp + (x.km - x.k) * (int64_t)d.nx]) * half * (w[yp] + wc);
        if (has_dn) cy_b = half * (vc + v[x.zm]) * half * (wc + w[ym]);
        const T cy = (cy_t - cy_b) * idn;
        const T lap = (w[x.xp] - T(2) * wc + w[x.xm]) * ix2 + (wzp - T(2) * wc + wzm) * iz2;
        const T rho0 = cp[q] - cm[q], rhoz = cp[x.zm] - cm[x.zm];
        const T f = T(a.ph.kf) * half * (rho0 + rhoz) * (phi[q] - phi[x.zm]) * idz_;
        hw = -(cx + cy + cz) + T(a.ph.ire) * lap + f;
    }
    // ---------------- v on the bottom y-face of row j ----------------
    T hv = T(0);
    if (has_dn) {
        const T dcj = T(a.tb.dc[j]);
        const T idc = T(1) / dcj;
        const T vtop = has_up ? v[yp] : T(0);
        const T vbot = (j > 1) ? v[ym] : T(0);
        const T a1 = half * (vtop + vc), a2 = half * (vc + vbot);
        const T cy = (a1 * a1 - a2 * a2) * idc;
        const T wl = T(a.tb.dn[j - 1]), wu = dnj;
        const T i2dc = T(1) / (T(2) * dcj);
        const T ur = (u[ym - x.i + x.ip] * wl + u[x.xp] * wu) * i2dc;
        const T ul = (u[ym] * wl + uc * wu) * i2dc;
        const T cx = (ur * half * (v[x.xp] + vc) - ul * half * (vc + v[x.xm])) * idx_;
        const T wf = (w[ym + (x.kp - x.k) * (int64_t)d.nx] * wl + w[x.zp] * wu) * i2dc;
        const T wb = (w[ym] * wl + wc * wu) * i2dc;
        const T cz = (wf * half * (v[x.zp] + vc) - wb * half * (vc + v[x.zm])) * idz_;
        const T lap = (v[x.xp] - T(2) * vc + v[x.xm]) * ix2 + (v[x.zp] - T(2) * vc + v[x.zm]) * iz2;
        const T rho0 = cp[q] - cm[q], rhoy = cp[ym] - cm[ym];
        const T ey = T(a.ph.e0) + (phi[q] - phi[ym]) * idc;
        const T f = T(a.ph.kf) * half * (rho0 + rhoy) * ey;
        hv = -(cx + cy + cz) + T(a.ph.ire) * lap + f;
    }
    // ---------------- ions at the cell centre ----------------
    T hc[2];
    {
        const T kd = T(a.ph.kd), e0 = T(a.ph.e0);
        const T uxp = u[x.xp], wzp = w[x.zp];
        const T ph0 = phi[q];
        const T gx_r = (phi[x.xp] - ph0) * idx_, gx_l = (ph0 - phi[x.xm]) * idx_;
        const T gz_f = (phi[x.zp] - ph0) * idz_, gz_b = (ph0 - phi[x.zm]) * idz_;
        T ey_t = T(0), ey_b = T(0);
        if (has_up) ey_t = e0 + (phi[yp] - ph0) / T(a.tb.dc[j + 1]);
        if (has_dn) ey_b = e0 + (ph0 - phi[ym]) / T(a.tb.dc[j]);
        const T vt = has_up ? v[yp] : T(0);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            const T *__restrict__ c = sp == 0 ? cp : cm;
            const T zs = sp == 0 ? T(1) : T(-1);
            const T cc = c[q], cxp = c[x.xp], cxm = c[x.xm], czp = c[x.zp], czm = c[x.zm];
            const T fxr = half * (cxp + cc), fxl = half * (cc + cxm);
            const T fzf = half * (czp + cc), fzb = half * (cc + czm);
            const T ax = (uxp * fxr - uc * fxl) * idx_;
            const T az = (wzp * fzf - wc * fzb) * idz_;
            T at = T(0), ab = T(0), mt = T(0), mb = T(0);
            if (has_up) {
                const T fy = half * (c[yp] + cc);
                at = vt * fy;
                mt = fy * ey_t;
            }
            if (has_dn) {
                const T fy = half * (cc + c[ym]);
                ab = vc * fy;
                mb = fy * ey_b;
            }
            const T ay = (at - ab) * idn;
            const T mx = (fxr * gx_r - fxl * gx_l) * idx_;
            const T mz = (fzf * gz_f - fzb * gz_b) * idz_;
            const T my = (mt - mb) * idn;
            const T dxx = (cxp - T(2) * cc + cxm) * ix2 + (czp - T(2) * cc + czm) * iz2;
            hc[sp] = -(ax + ay + az) + kd * (dxx + zs * (mx + my + mz));
        }
    }

    if (a.mode == 1) {
        a.dbg[0][q] = (double)hu;
        a.dbg[1][q] = (double)hv;
        a.dbg[2][q] = (double)hw;
        a.dbg[3][q] = (double)hc[0];
        a.dbg[4][q] = (double)hc[1];
        return;
    }

    // ---------------- Crank-Nicolson right-hand sides ----------------
    const T dt = T(a.clock[1]);
    const T gam = T(a.st.gam), zet = T(a.st.zet), alp = T(a.st.alp);
    const bool use_old = (a.st.k > 0);
    const bool keep = (a.st.k < 2);
    const T H[5] = {hu, hv, hw, hc[0], hc[1]};
    // L_y of the current fields
    T ly[5], gp[5];
    {
        const T dcb = T(a.tb.dc[j]), dct = T(a.tb.dc[j + 1]);
        // u: wall values u_bot, u_top at the half-cell distance
        const T ub = has_dn ? u[ym] : T(a.ph.u_bot);
        const T ut = has_up ? u[yp] : T(a.ph.u_top);
        ly[0] = ((ut - uc) / dct - (uc - ub) / dcb) * idn;
        const T wb = has_dn ? w[ym] : T(0);
        const T wt = has_up ? w[yp] : T(0);
        ly[2] = ((wt - wc) / dct - (wc - wb) / dcb) * idn;
        for (int sp = 0; sp < 2; ++sp) {
            const T *__restrict__ c = sp == 0 ? cp : cm;
            const T cc = c[q];
            const T ft = has_up ? (c[yp] - cc) / dct : T(0);
            const T fb = has_dn ? (cc - c[ym]) / dcb : T(0);
            ly[3 + sp] = (ft - fb) * idn;
        }
        if (has_dn) {
            const T vt = has_up ? v[yp] : T(0);
            const T vb = (j > 1) ? v[ym] : T(0);
            ly[1] = ((vt - vc) / dnj - (vc - vb) / T(a.tb.dn[j - 1])) / dcb;
            gp[1] = (p[q] - p[ym]) / dcb;
        } else {
            ly[1] = T(0);
            gp[1] = T(0);
        }
        gp[0] = (p[q] - p[x.xm]) * idx_;
        gp[2] = (p[q] - p[x.zm]) * idz_;
        gp[3] = gp[4] = T(0);
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        T *__restrict__ hb = (T *)a.h[f];
        const T nu = f < 3 ? T(a.ph.ire) : T(a.ph.kd);
        const T hold = use_old ? hb[q] : T(0);
        T val = dt * (gam * H[f] + zet * hold - alp * gp[f] + alp * nu * ly[f]);
        if (f == 1 && !has_dn) val = T(0);
        a.r[f][q] = (double)val;
        if (keep) hb[q] = H[f];
    }
}

// ---------------------------------------------------------------------------
// Crank-Nicolson wall-normal solves (I - alp dt nu / 2 L_y) delta = r, one
// thread per (x, z) column, q += delta.  The tridiagonal matrix is the same
// for every column of a field, so its elimination factors c'_j are computed
// by the block (identically in every thread) and kept in LDS for the back
// substitution; only d'_j goes through memory (in place in r).
// ---------------------------------------------------------------------------

struct CnArgs {
    Dims d;
    Phys ph;
    Tables tb;
    Stage st;
    void *q[5];
    double *r[5];
    const double *clock;
};

template <typename T>
__global__ void __launch_bounds__(256) k_cn_solve(CnArgs a) {
    extern __shared__ double s_cp[];
    const int f = blockIdx.y;
    const Dims &d = a.d;
    const int M = d.M;
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = col < d.plane;
    const double dt = a.clock[1];
    const double nu = (f < 3) ? a.ph.ire : a.ph.kd;
    const double beta = 0.5 * a.st.alp * dt * nu;
    // system type: 0 Dirichlet centre (u, w), 1 node (v), 2 zero-flux centre (c+-)
    const int sys = (f == 1) ? 1 : (f >= 3 ? 2 : 0);
    const int j0 = (sys == 1) ? 1 : 0;
    double *__restrict__ r = a.r[f];
    T *__restrict__ qf = (T *)a.q[f];
    const int64_t pl = d.plane;

    double cprev = 0.0, dprev = 0.0;
    for (int j = j0; j < M; ++j) {
        double lo, up, di;
        if (sys == 1) {
            const double aa = a.tb.lyn_lo[j], cc = a.tb.lyn_up[j];
            lo = (j > 1) ? aa : 0.0;
            up = (j < M - 1) ? cc : 0.0;
            di = -(aa + cc);
        } else {
            const double aa = a.tb.lyc_lo[j], cc = a.tb.lyc_up[j];
            lo = (j > 0) ? aa : 0.0;
            up = (j < M - 1) ? cc : 0.0;
            di = -(lo + up);
            if (sys == 0) {
                if (j == 0) di -= aa;
                if (j == M - 1) di -= cc;
            }
        }
        const double A = -beta * lo, B = 1.0 - beta * di, C = -beta * up;
        const double den = B - A * cprev;
        const double cj = C / den;
        if (threadIdx.x == 0) s_cp[j] = cj;
        if (active) {
            const double dj = (r[j * pl + col] - A * dprev) / den;
            r[j * pl + col] = dj;
            dprev = dj;
        }
        cprev = cj;
    }
    __syncthreads();
    if (!active) return;
    double xn = 0.0;
    for (int j = M - 1; j >= j0; --j) {
        const double xj = r[j * pl + col] - s_cp[j] * xn;
        const int64_t o = j * pl + col;
        qf[o] = (T)((double)qf[o] + xj);
        xn = xj;
    }
}

// divergence of the velocity, times scale (1 / (alp dt) from the device
// clock when scale_by_alpha_dt > 0, else a fixed factor)
struct DivArgs {
    Dims d;
    Tables tb;
    const void *u, *v, *w;
    double *out;
    const double *clock;
    double alp;
    double fixed;
};

template <typename T>
__global__ void __launch_bounds__(256) k_divergence(DivArgs a) {
    const Dims &d = a.d;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    const T *u = (const T *)a.u, *v = (const T *)a.v, *w = (const T *)a.w;
    const Idx x = make_idx(d, q);
    const double vt = (x.j + 1 < d.M) ? (double)v[q + d.plane] : 0.0;
    const double vb = (x.j > 0) ? (double)v[q] : 0.0;
    const double div = ((double)u[x.xp] - (double)u[q]) / d.dx + (vt - vb) / a.tb.dn[x.j] +
                       ((double)w[x.zp] - (double)w[q]) / d.dz;
    const double s = (a.alp > 0.0) ? 1.0 / (a.alp * a.clock[1]) : a.fixed;
    a.out[q] = div * s;
}

// projection correction: u -= a G psi;  p += psi - (a / (2 Re)) L_y psi
struct CorrArgs {
    Dims d;
    Phys ph;
    Tables tb;
    void *u, *v, *w, *p;
    const double *psi;
    const double *clock;
    double alp;
    double fixed;
    int update_p;
};

template <typename T>
__global__ void __launch_bounds__(256) k_correct(CorrArgs a) {
    const Dims &d = a.d;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    T *u = (T *)a.u, *v = (T *)a.v, *w = (T *)a.w, *p = (T *)a.p;
    const double *psi = a.psi;
    const Idx x = make_idx(d, q);
    const int j = x.j;
    const double sc = (a.alp > 0.0) ? a.alp * a.clock[1] : a.fixed;
    const double s0 = psi[q];
    u[q] = (T)((double)u[q] - sc * (s0 - psi[x.xm]) / d.dx);
    w[q] = (T)((double)w[q] - sc * (s0 - psi[x.zm]) / d.dz);
    if (j > 0) v[q] = (T)((double)v[q] - sc * (s0 - psi[q - d.plane]) / a.tb.dc[j]);
    if (a.update_p) {
        const double ft = (j + 1 < d.M) ? (psi[q + d.plane] - s0) / a.tb.dc[j + 1] : 0.0;
        const double fb = (j > 0) ? (s0 - psi[q - d.plane]) / a.tb.dc[j] : 0.0;
        const double ly = (ft - fb) / a.tb.dn[j];
        p[q] = (T)((double)p[q] + s0 - 0.5 * sc * a.ph.ire * ly);
    }
}

// right-hand side of the potential equation: -(c+ - c-) / (2 lam^2)
template <typename T>
__global__ void __launch_bounds__(256) k_charge(Dims d, double ch, const T *cp, const T *cm, double *out) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    out[q] = ch * ((double)cp[q] - (double)cm[q]);
}

template <typename Src, typename Dst>
__global__ void __launch_bounds__(256) k_copy_convert(int64_t n, const Src *in, Dst *out) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    out[q] = (Dst)in[q];
}

template <typename T>
__global__ void k_advance_clock(double *clock, double alp) {
    if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] += alp * clock[1];
}

inline dim3 grid1(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

hipError_t launch_explicit(nspnp_state *s, const Stage &st, bool /*write_r*/) {
    ProfScope prof_(s, K_EXPLICIT);
    ExplicitArgs a{};
    a.d = s->d;
    a.ph = s->ph;
    a.tb = s->tb;
    a.st = st;
    a.u = s->f[0]; a.v = s->f[1]; a.w = s->f[2]; a.cp = s->f[3]; a.cm = s->f[4]; a.phi = s->f[5]; a.p = s->f[6];
    for (int q = 0; q < 5; ++q) { a.h[q] = s->h[q]; a.r[q] = s->r[q]; a.dbg[q] = nullptr; }
    a.clock = s->clock;
    a.mode = 0;
    if (s->fp64) k_explicit<double><<<grid1(s->d.n), 256, 0, s->stream>>>(a);
    else k_explicit<float><<<grid1(s->d.n), 256, 0, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_explicit_debug(nspnp_state *s, double *const out[5]) {
    ExplicitArgs a{};
    a.d = s->d;
    a.ph = s->ph;
    a.tb = s->tb;
    a.st = Stage{0, 0, 0, 0};
    a.u = s->f[0]; a.v = s->f[1]; a.w = s->f[2]; a.cp = s->f[3]; a.cm = s->f[4]; a.phi = s->f[5]; a.p = s->f[6];
    for (int q = 0; q < 5; ++q) { a.h[q] = s->h[q]; a.r[q] = s->r[q]; a.dbg[q] = out[q]; }
    a.clock = s->clock;
    a.mode = 1;
    if (s->fp64) k_explicit<double><<<grid1(s->d.n), 256, 0, s->stream>>>(a);
    else k_explicit<float><<<grid1(s->d.n), 256, 0, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_cn_solve(nspnp_state *s, const Stage &st) {
    ProfScope prof_(s, K_CN);
    CnArgs a{};
    a.d = s->d;
    a.ph = s->ph;
    a.tb = s->tb;
    a.st = st;
    for (int q = 0; q < 5; ++q) { a.q[q] = s->f[q]; a.r[q] = s->r[q]; }
    a.clock = s->clock;
    dim3 g((unsigned)((s->d.plane + 255) / 256), 5);
    size_t lds = (size_t)s->d.M * sizeof(double);
    if (s->fp64) k_cn_solve<double><<<g, 256, lds, s->stream>>>(a);
    else k_cn_solve<float><<<g, 256, lds, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_divergence(nspnp_state *s, double fixed, const Stage &st, double *out) {
    ProfScope prof_(s, K_DIV);
    DivArgs a{};
    a.d = s->d;
    a.tb = s->tb;
    a.u = s->f[0]; a.v = s->f[1]; a.w = s->f[2];
    a.out = out;
    a.clock = s->clock;
    a.alp = st.alp;
    a.fixed = fixed;
    if (s->fp64) k_divergence<double><<<grid1(s->d.n), 256, 0, s->stream>>>(a);
    else k_divergence<float><<<grid1(s->d.n), 256, 0, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_correct(nspnp_state *s, const Stage &st, bool update_p, double fixed) {
    ProfScope prof_(s, K_CORRECT);
    CorrArgs a{};
    a.d = s->d;
    a.ph = s->ph;
    a.tb = s->tb;
    a.u = s->f[0]; a.v = s->f[1]; a.w = s->f[2]; a.p = s->f[6];
    a.psi = s->psi;
    a.clock = s->clock;
    a.alp = st.alp;
    a.fixed = fixed;
    a.update_p = update_p ? 1 : 0;
    if (s->fp64) k_correct<double><<<grid1(s->d.n), 256, 0, s->stream>>>(a);
    else k_correct<float><<<grid1(s->d.n), 256, 0, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_charge(nspnp_state *s, double *out) {
    ProfScope prof_(s, K_CHARGE);
    if (s->fp64)
        k_charge<double><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d, s->ph.ch, (const double *)s->f[3],
                                                              (const double *)s->f[4], out);
    else
        k_charge<float><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d, s->ph.ch, (const float *)s->f[3],
                                                             (const float *)s->f[4], out);
    return hipGetLastError();
}

hipError_t launch_store_phi(nspnp_state *s, const double *src) {
    ProfScope prof_(s, K_STORE_PHI);
    if (s->fp64)
        k_copy_convert<double, double><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d.n, src, (double *)s->f[5]);
    else
        k_copy_convert<double, float><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d.n, src, (float *)s->f[5]);
    return hipGetLastError();
}

hipError_t launch_convert(nspnp_state *s, int field, const double *in, double *out, bool to_state) {
    if (to_state) {
        if (s->fp64)
            k_copy_convert<double, double><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d.n, in, (double *)s->f[field]);
        else
            k_copy_convert<double, float><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d.n, in, (float *)s->f[field]);
    } else {
        if (s->fp64)
            k_copy_convert<double, double><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d.n, (const double *)s->f[field], out);
        else
            k_copy_convert<float, double><<<grid1(s->d.n), 256, 0, s->stream>>>(s->d.n, (const float *)s->f[field], out);
    }
    return hipGetLastError();
}

hipError_t launch_advance_clock(nspnp_state *s, double alp) {
    ProfScope prof_(s, K_CLOCK);
    k_advance_clock<double><<<1, 64, 0, s->stream>>>(s->clock, alp);
    return hipGetLastError();
}

}  // namespace nspnp
