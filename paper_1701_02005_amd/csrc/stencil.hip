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
    const Phys *phys;
    size_t ms;
    Tables tb;
    Stage st;
    const void *u, *v, *w, *cp, *cm, *phi, *p;
    void *h[5];
    double *r[5];
    double *dbg[5];
    const double *clock;
    int mode;  // 0: substep (H update + CN right-hand sides); 1: H to dbg only
};

__device__ __forceinline__ void shift_explicit(ExplicitArgs &a) {
    const size_t ms = a.ms;
    a.phys = member_ptr(a.phys, ms);
    a.u = member_ptr(a.u, ms); a.v = member_ptr(a.v, ms); a.w = member_ptr(a.w, ms);
    a.cp = member_ptr(a.cp, ms); a.cm = member_ptr(a.cm, ms); a.phi = member_ptr(a.phi, ms); a.p = member_ptr(a.p, ms);
    for (int f = 0; f < 5; ++f) { a.h[f] = member_ptr(a.h[f], ms); a.r[f] = member_ptr(a.r[f], ms); }
    a.clock = member_ptr(a.clock, ms);
}

// Convection, horizontal diffusion, Coulomb force and ion transport at one
// cell, then the Crank-Nicolson right-hand side
//   r = dt [gam H^k + zet H^{k-1} - alp G p + alp nu L_y q].
// Grid: x = 256-cell chunks of one (x, z) plane, y = the cell row j, so the
// row tables are uniform per block.  Each field's H and r are computed and
// stored before the next field is started to keep register pressure low.
template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) k_explicit(ExplicitArgs a) {
    shift_explicit(a);
    const Phys ph = *a.phys;
    const Dims &d = a.d;
    const int nx = d.nx, nz = d.nz, M = d.M;
    const int pl = (int)d.plane;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= pl) return;
    const int j = blockIdx.y;
    const int k = e / nx;
    const int i = e - k * nx;
    const int ip = (i + 1 == nx) ? 0 : i + 1, im = (i == 0) ? nx - 1 : i - 1;
    const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
    const int q = j * pl + e;
    const int xp = q - i + ip, xm = q - i + im;
    const int zp = q + (kp - k) * nx, zm = q + (km - k) * nx;
    const bool has_up = (j + 1 < M), has_dn = (j > 0);
    const int yp = q + pl, ym = q - pl;

    const T *__restrict__ u = (const T *)a.u;
    const T *__restrict__ v = (const T *)a.v;
    const T *__restrict__ w = (const T *)a.w;
    const T *__restrict__ cp = (const T *)a.cp;
    const T *__restrict__ cm = (const T *)a.cm;
    const T *__restrict__ phi = (const T *)a.phi;
    const T *__restrict__ p = (const T *)a.p;

    const T half = T(0.5), two = T(2);
    const T idx_ = T(1.0 / d.dx), idz_ = T(1.0 / d.dz);
    const T ix2 = idx_ * idx_, iz2 = idz_ * idz_;
    const T idn = T(a.tb.idn[j]);
    const T idcb = T(a.tb.idc[j]), idct = T(a.tb.idc[j + 1]);
    const T kf = T(ph.kf), ire = T(ph.ire), kd = T(ph.kd), e0 = T(ph.e0);
    const int mode = a.mode;
    const T dt = T(a.clock[1]);
    const T gam = T(a.st.gam), zet = T(a.st.zet), alp = T(a.st.alp);
    const bool use_old = (a.st.k > 0) && mode == 0;
    const bool keep = (a.st.k < 2) && mode == 0;

    // store H (debug) or H and the Crank-Nicolson right-hand side (substep)
    auto emit = [&](int f, T hval, T gp, T nu_ly) {
        if (mode == 1) {
            a.dbg[f][q] = (double)hval;
            return;
        }
        T *__restrict__ hb = (T *)a.h[f];
        const T hold = use_old ? hb[q] : T(0);
        a.r[f][q] = (double)(dt * (gam * hval + zet * hold - alp * gp + alp * nu_ly));
        if (keep) hb[q] = hval;
    };

    const T uc = u[q], vc = v[q], wc = w[q];
    const T rho0 = cp[q] - cm[q];
    const T ph0 = phi[q];

    // ---------------- u on the x-face ----------------
    {
        const T uxp = u[xp], uxm = u[xm], uzp = u[zp], uzm = u[zm];
        const T a1 = half * (uxp + uc), a2 = half * (uc + uxm);
        const T cx = (a1 * a1 - a2 * a2) * idx_;
        T flux_t = T(0), flux_b = T(0), ut = T(ph.u_top), ub = T(ph.u_bot);
        if (has_up) {
            ut = u[yp];
            flux_t = half * (v[yp] + v[yp - i + im]) * half * (ut + uc);
        }
        if (has_dn) {
            ub = u[ym];
            flux_b = half * (vc + v[xm]) * half * (uc + ub);
        }
        const T cy = (flux_t - flux_b) * idn;
        const T wf = half * (w[zp] + w[zp - i + im]);
        const T wb = half * (wc + w[xm]);
        const T cz = (wf * half * (uzp + uc) - wb * half * (uc + uzm)) * idz_;
        const T lap = (uxp - two * uc + uxm) * ix2 + (uzp - two * uc + uzm) * iz2;
        const T rhox = cp[xm] - cm[xm];
        const T f = kf * half * (rho0 + rhox) * (ph0 - phi[xm]) * idx_;
        const T ly = ((ut - uc) * idct - (uc - ub) * idcb) * idn;
        emit(0, -(cx + cy + cz) + ire * lap + f, (p[q] - p[xm]) * idx_, ire * ly);
    }
    // ---------------- w on the z-face ----------------
    {
        const T wzp = w[zp], wzm = w[zm], wxp = w[xp], wxm = w[xm];
        const T a1 = half * (wzp + wc), a2 = half * (wc + wzm);
        const T cz = (a1 * a1 - a2 * a2) * idz_;
        const T ur = half * (u[xp] + u[zm - i + ip]);
        const T ul = half * (uc + u[zm]);
        const T cx = (ur * half * (wxp + wc) - ul * half * (wc + wxm)) * idx_;
        T flux_t = T(0), flux_b = T(0), wt = T(0), wb = T(0);
        if (has_up) {
            wt = w[yp];
            flux_t = half * (v[yp] + v[yp + (km - k) * nx]) * half * (wt + wc);
        }
        if (has_dn) {
            wb = w[ym];
            flux_b = half * (vc + v[zm]) * half * (wc + wb);
        }
        const T cy = (flux_t - flux_b) * idn;
        const T lap = (wxp - two * wc + wxm) * ix2 + (wzp - two * wc + wzm) * iz2;
        const T rhoz = cp[zm] - cm[zm];
        const T f = kf * half * (rho0 + rhoz) * (ph0 - phi[zm]) * idz_;
        const T ly = ((wt - wc) * idct - (wc - wb) * idcb) * idn;
        emit(2, -(cx + cy + cz) + ire * lap + f, (p[q] - p[zm]) * idz_, ire * ly);
    }
    // ---------------- v on the bottom y-face of row j ----------------
    if (has_dn) {
        const T vwl = T(a.tb.vwl[j]), vwu = T(a.tb.vwu[j]);
        const T idn_lo = T(a.tb.idn[j - 1]);
        const T vtop = has_up ? v[yp] : T(0);
        const T vbot = (j > 1) ? v[ym] : T(0);
        const T a1 = half * (vtop + vc), a2 = half * (vc + vbot);
        const T cy = (a1 * a1 - a2 * a2) * idcb;
        const T ur = u[ym - i + ip] * vwl + u[xp] * vwu;
        const T ul = u[ym] * vwl + uc * vwu;
        const T vxp = v[xp], vxm = v[xm], vzp = v[zp], vzm = v[zm];
        const T cx = (ur * half * (vxp + vc) - ul * half * (vc + vxm)) * idx_;
        const T wf = w[ym + (kp - k) * nx] * vwl + w[zp] * vwu;
        const T wbk = w[ym] * vwl + wc * vwu;
        const T cz = (wf * half * (vzp + vc) - wbk * half * (vc + vzm)) * idz_;
        const T lap = (vxp - two * vc + vxm) * ix2 + (vzp - two * vc + vzm) * iz2;
        const T rhoy = cp[ym] - cm[ym];
        const T ey = e0 + (ph0 - phi[ym]) * idcb;
        const T f = kf * half * (rho0 + rhoy) * ey;
        const T ly = ((vtop - vc) * idn - (vc - vbot) * idn_lo) * idcb;
        emit(1, -(cx + cy + cz) + ire * lap + f, (p[q] - p[ym]) * idcb, ire * ly);
    } else {
        emit(1, T(0), T(0), T(0));
        if (mode == 0) a.r[1][q] = 0.0;
    }
    // ---------------- ions at the cell centre ----------------
    {
        const T uxp = u[xp], wzp = w[zp];
        const T gx_r = (phi[xp] - ph0) * idx_, gx_l = (ph0 - phi[xm]) * idx_;
        const T gz_f = (phi[zp] - ph0) * idz_, gz_b = (ph0 - phi[zm]) * idz_;
        const T ey_t = has_up ? e0 + (phi[yp] - ph0) * idct : T(0);
        const T ey_b = has_dn ? e0 + (ph0 - phi[ym]) * idcb : T(0);
        const T vt = has_up ? v[yp] : T(0);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            const T *__restrict__ c = sp == 0 ? cp : cm;
            const T zs = sp == 0 ? T(1) : T(-1);
            const T cc = c[q], cxp = c[xp], cxm = c[xm], czp = c[zp], czm = c[zm];
            const T fxr = half * (cxp + cc), fxl = half * (cc + cxm);
            const T fzf = half * (czp + cc), fzb = half * (cc + czm);
            const T ax = (uxp * fxr - uc * fxl) * idx_;
            const T az = (wzp * fzf - wc * fzb) * idz_;
            T at = T(0), ab = T(0), mt = T(0), mb = T(0), dft = T(0), dfb = T(0);
            if (has_up) {
                const T cu = c[yp];
                const T fy = half * (cu + cc);
                at = vt * fy;
                mt = fy * ey_t;
                dft = (cu - cc) * idct;
            }
            if (has_dn) {
                const T cd = c[ym];
                const T fy = half * (cc + cd);
                ab = vc * fy;
                mb = fy * ey_b;
                dfb = (cc - cd) * idcb;
            }
            const T ay = (at - ab) * idn;
            const T mx = (fxr * gx_r - fxl * gx_l) * idx_;
            const T mz = (fzf * gz_f - fzb * gz_b) * idz_;
            const T my = (mt - mb) * idn;
            const T dxx = (cxp - two * cc + cxm) * ix2 + (czp - two * cc + czm) * iz2;
            emit(3 + sp, -(ax + ay + az) + kd * (dxx + zs * (mx + my + mz)), T(0), kd * (dft - dfb) * idn);
        }
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
    const Phys *phys;
    size_t ms;
    Tables tb;
    Stage st;
    void *q[5];
    double *r[5];
    const double *clock;
};

constexpr int kCnPf = 4;  // rows loaded ahead of the elimination

template <typename T>
__global__ void __launch_bounds__(256) k_cn_solve(CnArgs a) {
    extern __shared__ double s_cp[];
    const int f = blockIdx.y;
    const Dims &d = a.d;
    const int M = d.M;
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = col < d.plane;
    const Phys *ph = member_ptr(a.phys, a.ms);
    const double dt = member_ptr(a.clock, a.ms)[1];
    const double nu = (f < 3) ? ph->ire : ph->kd;
    const double beta = 0.5 * a.st.alp * dt * nu;
    // system type: 0 Dirichlet centre (u, w), 1 node (v), 2 zero-flux centre (c+-)
    const int sys = (f == 1) ? 1 : (f >= 3 ? 2 : 0);
    const int j0 = (sys == 1) ? 1 : 0;
    double *__restrict__ r = member_ptr(a.r[f], a.ms);
    T *__restrict__ qf = (T *)member_ptr(a.q[f], a.ms);
    const int64_t pl = d.plane;

    double cprev = 0.0, dprev = 0.0;
    double buf[kCnPf];
#pragma unroll
    for (int p = 0; p < kCnPf; ++p) buf[p] = (active && j0 + p < M) ? r[(j0 + p) * pl + col] : 0.0;
    for (int jb = j0; jb < M; jb += kCnPf) {
#pragma unroll
        for (int p = 0; p < kCnPf; ++p) {
            const int j = jb + p;
            if (j < M) {
                const double rj = buf[p];
                if (active && j + kCnPf < M) buf[p] = r[(j + kCnPf) * pl + col];
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
                    const double dj = (rj - A * dprev) / den;
                    r[j * pl + col] = dj;
                    dprev = dj;
                }
                cprev = cj;
            }
        }
    }
    __syncthreads();
    if (!active) return;
    double xn = 0.0;
    double bd[kCnPf];
    T bq[kCnPf];
#pragma unroll
    for (int p = 0; p < kCnPf; ++p) {
        const int j = M - 1 - p;
        bd[p] = (j >= j0) ? r[j * pl + col] : 0.0;
        bq[p] = (j >= j0) ? qf[j * pl + col] : T(0);
    }
    for (int jb = M - 1; jb >= j0; jb -= kCnPf) {
#pragma unroll
        for (int p = 0; p < kCnPf; ++p) {
            const int j = jb - p;
            if (j >= j0) {
                const double dj = bd[p];
                const T qj = bq[p];
                if (j - kCnPf >= j0) {
                    bd[p] = r[(j - kCnPf) * pl + col];
                    bq[p] = qf[(j - kCnPf) * pl + col];
                }
                const double xj = dj - s_cp[j] * xn;
                qf[j * pl + col] = (T)((double)qj + xj);
                xn = xj;
            }
        }
    }
}

// projection correction: u -= a G psi;  p += psi - (a / (2 Re)) L_y psi
struct CorrArgs {
    Dims d;
    const Phys *phys;
    size_t ms;
    Tables tb;
    void *u, *v, *w, *p;
    const double *psi;
    double *clock;
    double alp;
    double fixed;
    int update_p;
    int advance_clock;
};

template <typename T>
__global__ void __launch_bounds__(256) k_correct(CorrArgs a) {
    const Dims &d = a.d;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= d.n) return;
    const size_t ms = a.ms;
    double *clock = member_ptr(a.clock, ms);
    const Phys *ph = member_ptr(a.phys, ms);
    // substep time t += alp dt (dt is read, never written, by this kernel)
    if (a.advance_clock && q == 0) clock[0] += a.alp * clock[1];
    T *u = (T *)member_ptr(a.u, ms), *v = (T *)member_ptr(a.v, ms), *w = (T *)member_ptr(a.w, ms);
    T *p = (T *)member_ptr(a.p, ms);
    const double *psi = member_ptr(a.psi, ms);
    const Idx x = make_idx(d, q);
    const int j = x.j;
    const double sc = (a.alp > 0.0) ? a.alp * clock[1] : a.fixed;
    const double s0 = psi[q];
    u[q] = (T)((double)u[q] - sc * (s0 - psi[x.xm]) / d.dx);
    w[q] = (T)((double)w[q] - sc * (s0 - psi[x.zm]) / d.dz);
    if (j > 0) v[q] = (T)((double)v[q] - sc * (s0 - psi[q - d.plane]) / a.tb.dc[j]);
    if (a.update_p) {
        const double ft = (j + 1 < d.M) ? (psi[q + d.plane] - s0) / a.tb.dc[j + 1] : 0.0;
        const double fb = (j > 0) ? (s0 - psi[q - d.plane]) / a.tb.dc[j] : 0.0;
        const double ly = (ft - fb) / a.tb.dn[j];
        p[q] = (T)((double)p[q] + s0 - 0.5 * sc * ph->ire * ly);
    }
}

template <typename Src, typename Dst>
__global__ void __launch_bounds__(256) k_copy_convert(int64_t n, const Src *in, Dst *out) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    out[q] = (Dst)in[q];
}

inline dim3 grid1(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

hipError_t launch_explicit(nspnp_state *s, const Stage &st, bool /*write_r*/) {
    ProfScope prof_(s, K_EXPLICIT);
    ExplicitArgs a{};
    a.d = s->d;
    a.phys = s->d_phys;
    a.ms = s->mstride;
    a.tb = s->tb;
    a.st = st;
    a.u = s->f[0]; a.v = s->f[1]; a.w = s->f[2]; a.cp = s->f[3]; a.cm = s->f[4]; a.phi = s->f[5]; a.p = s->f[6];
    for (int q = 0; q < 5; ++q) { a.h[q] = s->h[q]; a.r[q] = s->r[q]; a.dbg[q] = nullptr; }
    a.clock = s->clock;
    a.mode = 0;
    const int tb = s->tiles.expl;
    const dim3 g((unsigned)((s->d.plane + tb - 1) / tb), (unsigned)s->d.M, (unsigned)s->nmem);
    if (s->fp64) k_explicit<double><<<g, tb, 0, s->stream>>>(a);
    else k_explicit<float><<<g, tb, 0, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_explicit_debug(nspnp_state *s, double *const out[5]) {
    ExplicitArgs a{};
    a.d = s->d;
    a.phys = s->d_phys;
    a.ms = 0;
    a.tb = s->tb;
    a.st = Stage{0, 0, 0, 0};
    a.u = s->f[0]; a.v = s->f[1]; a.w = s->f[2]; a.cp = s->f[3]; a.cm = s->f[4]; a.phi = s->f[5]; a.p = s->f[6];
    for (int q = 0; q < 5; ++q) { a.h[q] = s->h[q]; a.r[q] = s->r[q]; a.dbg[q] = out[q]; }
    a.clock = s->clock;
    a.mode = 1;
    const dim3 g((unsigned)((s->d.plane + 255) / 256), (unsigned)s->d.M);
    if (s->fp64) k_explicit<double><<<g, 256, 0, s->stream>>>(a);
    else k_explicit<float><<<g, 256, 0, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_cn_solve(nspnp_state *s, const Stage &st) {
    ProfScope prof_(s, K_CN);
    CnArgs a{};
    a.d = s->d;
    a.phys = s->d_phys;
    a.ms = s->mstride;
    a.tb = s->tb;
    a.st = st;
    for (int q = 0; q < 5; ++q) { a.q[q] = s->f[q]; a.r[q] = s->r[q]; }
    a.clock = s->clock;
    const int tb = s->tiles.cn;
    dim3 g((unsigned)((s->d.plane + tb - 1) / tb), 5, (unsigned)s->nmem);
    size_t lds = (size_t)s->d.M * sizeof(double);
    if (s->fp64) k_cn_solve<double><<<g, tb, lds, s->stream>>>(a);
    else k_cn_solve<float><<<g, tb, lds, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_correct(nspnp_state *s, const Stage &st, bool update_p, double fixed, bool advance_clock) {
    ProfScope prof_(s, K_CORRECT);
    CorrArgs a{};
    a.d = s->d;
    a.phys = s->d_phys;
    a.ms = s->mstride;
    a.tb = s->tb;
    a.u = s->f[0]; a.v = s->f[1]; a.w = s->f[2]; a.p = s->f[6];
    a.psi = s->psi;
    a.clock = s->clock;
    a.alp = st.alp;
    a.fixed = fixed;
    a.update_p = update_p ? 1 : 0;
    a.advance_clock = advance_clock ? 1 : 0;
    const int tb = s->tiles.corr;
    const dim3 g((unsigned)((s->d.n + tb - 1) / tb), 1, (unsigned)s->nmem);
    if (s->fp64) k_correct<double><<<g, tb, 0, s->stream>>>(a);
    else k_correct<float><<<g, tb, 0, s->stream>>>(a);
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

}  // namespace nspnp
