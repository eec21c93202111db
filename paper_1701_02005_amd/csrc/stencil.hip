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
    void *r[5];  // Crank-Nicolson right-hand sides, state type (computed in it)
    double *dbg[5];
    const double *clock;
    int mode;  // 0: substep (H update + CN right-hand sides); 1: H to dbg only
    int tx, tz;     // a block's (x, z) tile: tx columns of tz z-lines
    int ntx;        // tiles across x
    int chunks;     // tiles per (x, z) plane
    int slabs;      // row slabs per member
    int slab_rows;  // rows marched by one block
    int implicit_xz;  // 1: x/z diffusion goes to the implicit (alpha) part of r, not to H
    // Row-slab Crank-Nicolson with its first pass fused (NULL: not fused):
    // this stage's recurrence coefficients [3 systems][g, m, n][M] and the
    // method's scratch [2][5 fields][slabs][plane]; the block's slab is the
    // method's slab, and the kernel stores both exits of every column.
    const double *cn_coef;
    double *cn_scr;
};

__device__ __forceinline__ void shift_explicit(ExplicitArgs &a, unsigned mem) {
    const size_t ms = a.ms;
    a.phys = member_ptr_at(a.phys, ms, mem);
    a.u = member_ptr_at(a.u, ms, mem); a.v = member_ptr_at(a.v, ms, mem); a.w = member_ptr_at(a.w, ms, mem);
    a.cp = member_ptr_at(a.cp, ms, mem); a.cm = member_ptr_at(a.cm, ms, mem);
    a.phi = member_ptr_at(a.phi, ms, mem); a.p = member_ptr_at(a.p, ms, mem);
    for (int f = 0; f < 5; ++f) { a.h[f] = member_ptr_at(a.h[f], ms, mem); a.r[f] = member_ptr_at(a.r[f], ms, mem); }
    a.clock = member_ptr_at(a.clock, ms, mem);
    if (a.cn_coef) {
        a.cn_coef = member_ptr_at(a.cn_coef, ms, mem);
        a.cn_scr = member_ptr_at(a.cn_scr, ms, mem);
    }
}

// Convection, horizontal diffusion, Coulomb force and ion transport at one
// cell, then the Crank-Nicolson right-hand side
//   r = dt [gam H^k + zet H^{k-1} - alp G p + alp nu L_y q].
//
// Data movement.  A block owns a 2-D tile of (x, z) columns (tx along x, tz
// z-lines) and marches a slab of rows.  Rows j and j+1 of all seven fields,
// each over the tile plus a one-column halo (periodic in x and z), sit in a
// two-slot LDS ring.  The global loads of row j+2 (coalesced, two halo
// positions per thread) and of H^{k-1} at row j+1 are issued before row j is
// computed and land in LDS / registers after it, so the memory latency hides
// behind a whole row of arithmetic and every neighbour value is an LDS read.
// Own-column values of row j-1 and the two row-(j-1) neighbours the v-point
// needs are carried in registers from the previous row.
constexpr int kNF = 7;  // u v w c+ c- phi p

template <typename T, int kHalo>
struct HaloRegs {
    T v[kNF][kHalo];
};

// kMode (a compile-time copy of ExplicitArgs::mode): the export of H alone
// is its own instantiation, so the substep kernel carries none of its state.
// kTx > 0: the tile is kTx columns by kTz z-lines (a.tx, a.tz ignored), so
// every LDS neighbour offset is a compile-time constant.
template <typename T, int kHalo, int kWaves, int kMode, int kTx = 0, int kTz = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves))) k_explicit(ExplicitArgs a) {
    extern __shared__ unsigned char s_raw[];
    T *sm = (T *)s_raw;  // [slot 0..1][field 0..6][halo tile]
    const unsigned chunks = (unsigned)a.chunks, slabs = (unsigned)a.slabs;
    const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);  // x-tiles fastest: z-neighbour tiles share an L2
    const unsigned chunk = tile % chunks;
    const unsigned slab = (tile / chunks) % slabs;
    const unsigned mem = tile / (chunks * slabs);
    shift_explicit(a, mem);
    const Phys ph = *a.phys;
    const Dims &d = a.d;
    const int nx = d.nx, nz = d.nz, M = d.M;
    const int pl = (int)d.plane;
    const int tx = kTx ? kTx : a.tx, tz = kTx ? kTz : a.tz, hx = tx + 2, HS = hx * (tz + 2);
    const int i0 = (int)(chunk % (unsigned)a.ntx) * tx, k0 = (int)(chunk / (unsigned)a.ntx) * tz;
    const int lk = (int)threadIdx.x / tx, li = (int)threadIdx.x - lk * tx;
    const int i = i0 + li, k = k0 + lk;
    const bool active = lk < tz && i < nx && k < nz;
    const int c = (lk + 1) * hx + (li + 1);  // own position in the halo tile

    const T *__restrict__ F[kNF] = {(const T *)a.u, (const T *)a.v, (const T *)a.w, (const T *)a.cp,
                                    (const T *)a.cm, (const T *)a.phi, (const T *)a.p};
    // halo positions this thread loads: in-plane byte offsets, fixed for every
    // row.  Positions past the halo tile load the plane's first element
    // (which exists) and are never stored: the loads are unconditional, so a
    // row's loads go out together.  Every access is a field's base pointer plus
    // a 32-bit byte offset (row offset + in-plane offset; a field of every
    // supported grid is below 2^32 bytes), which the hardware adds itself.
    unsigned off[kHalo];
    int spos[kHalo];
    bool in_tile[kHalo];
#pragma unroll
    for (int q = 0; q < kHalo; ++q) {
        const int sp = (int)threadIdx.x + q * (int)blockDim.x;
        spos[q] = sp;
        in_tile[q] = sp < HS;
        const int hz = sp / hx, hxp = sp - hz * hx;
        int gi = (i0 - 1 + hxp) % nx, gk = (k0 - 1 + hz) % nz;
        if (gi < 0) gi += nx;
        if (gk < 0) gk += nz;
        off[q] = in_tile[q] ? (unsigned)(gk * nx + gi) * (unsigned)sizeof(T) : 0u;
    }
    const unsigned plb = (unsigned)pl * (unsigned)sizeof(T);  // bytes per row of a field
    auto load_rows = [&](int row, HaloRegs<T, kHalo> &r) {
        const unsigned base = (unsigned)row * plb;
#pragma unroll
        for (int f = 0; f < kNF; ++f)
#pragma unroll
            for (int q = 0; q < kHalo; ++q) r.v[f][q] = *byte_at(F[f], base + off[q]);
    };
    auto store_rows = [&](int slot, const HaloRegs<T, kHalo> &r) {
#pragma unroll
        for (int f = 0; f < kNF; ++f)
#pragma unroll
            for (int q = 0; q < kHalo; ++q)
                if (in_tile[q]) sm[(slot * kNF + f) * HS + spos[q]] = r.v[f][q];
    };
    auto X = [&](int slot, int f, int dx, int dz) -> T { return sm[(slot * kNF + f) * HS + c + dz * hx + dx]; };

    const T half = T(0.5), two = T(2);
    const T idx_ = T(1.0 / d.dx), idz_ = T(1.0 / d.dz);
    const T ix2 = idx_ * idx_, iz2 = idz_ * idz_;
    const T kf = T(ph.kf), ire = T(ph.ire), kd = T(ph.kd), e0 = T(ph.e0);
    constexpr int mode = kMode;
    const T dt = T(a.clock[1]);
    const T gam = T(a.st.gam), zet = T(a.st.zet), alp = T(a.st.alp);
    const bool use_old = (a.st.k > 0) && mode == 0;
    const bool keep = (a.st.k < 2) && mode == 0;
    const bool imp = a.implicit_xz != 0;  // x/z diffusion: implicit part of r instead of H
    // Fused first pass of the row-slab Crank-Nicolson solve: along the slab,
    // the local forward sweep l_j = g_j r_j + m_j l_{j-1} (l = 0 below the
    // slab) of each field's right-hand side, and its local backward sweep
    // taken at the slab's first row, k = sum_j (prod_{i<j} n_i) l_j (the
    // products are column-independent: a table per system, u, w / v / ions).
    const bool fuse = (mode == 0) && a.cn_coef != nullptr;
    double cl[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, ck[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int e = active ? k * nx + i : 0;
    const unsigned ueb = (unsigned)e * (unsigned)sizeof(T);  // own column, bytes
    const int ip = (i + 1 >= nx) ? 0 : i + 1;
    const int kp = (k + 1 >= nz) ? 0 : k + 1;
    const int e_xp = k * nx + ip, e_zp = kp * nx + i;

    const int j0 = (int)slab * a.slab_rows;
    const int j1 = (j0 + a.slab_rows < M) ? j0 + a.slab_rows : M;
    const int jl = (j1 < M - 1) ? j1 : M - 1;  // last row staged in LDS

    // row j0 - 1: own-column values and the two neighbours the v-point needs
    const T zero = T(0);
    T um = zero, vm = zero, wm = zero, am = zero, bm = zero, fm = zero, pm = zero, u_xp_m = zero, w_zp_m = zero;
    if (j0 > 0 && active) {
        const int q = (j0 - 1) * pl;
        um = F[0][q + e]; vm = F[1][q + e]; wm = F[2][q + e]; am = F[3][q + e]; bm = F[4][q + e];
        fm = F[5][q + e]; pm = F[6][q + e];
        u_xp_m = F[0][q + e_xp];
        w_zp_m = F[2][q + e_zp];
    }
    T hold_c[5], hold_n[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        hold_c[f] = (use_old && active) ? ld_once(byte_at((const T *)a.h[f], (unsigned)j0 * plb + ueb)) : zero;
        hold_n[f] = zero;
    }
    {
        HaloRegs<T, kHalo> r0;
        load_rows(j0, r0);
        store_rows(j0 & 1, r0);
        if (j0 + 1 < M) {
            load_rows(j0 + 1, r0);
            store_rows((j0 + 1) & 1, r0);
        }
    }
    __syncthreads();

    HaloRegs<T, kHalo> rn;
    for (int j = j0; j < j1; ++j) {
        const int sc = j & 1, sn = sc ^ 1;
        const bool pre = (j + 2 <= jl);
        // FP64: the wave issuing the next row's loads takes issue priority so
        // they leave before the other waves' arithmetic (measured: 0.418 ->
        // 0.415 ms at 256 x 193 x 256; the FP32 form is slower with it)
        if constexpr (sizeof(T) == 8) __builtin_amdgcn_s_setprio(2);
        if (pre) load_rows(j + 2, rn);  // lands in LDS after this row
        if (use_old && active && j + 1 < j1) {
#pragma unroll
            for (int f = 0; f < 5; ++f) hold_n[f] = ld_once(byte_at((const T *)a.h[f], (unsigned)(j + 1) * plb + ueb));
        }
        if constexpr (sizeof(T) == 8) __builtin_amdgcn_s_setprio(0);
        const bool has_up = (j + 1 < M), has_dn = (j > 0);
        const unsigned qb = (unsigned)j * plb + ueb;  // this cell, bytes
        if (active) {
            const T idn = T(uniform_load(a.tb.idn, j));
            const T idcb = T(uniform_load(a.tb.idc, j)), idct = T(uniform_load(a.tb.idc, j + 1));
            const T uc = X(sc, 0, 0, 0), vc = X(sc, 1, 0, 0), wc = X(sc, 2, 0, 0);
            const T ac = X(sc, 3, 0, 0), bc = X(sc, 4, 0, 0), ph0 = X(sc, 5, 0, 0), pc = X(sc, 6, 0, 0);
            const T up_ = has_up ? X(sn, 0, 0, 0) : zero, vp = has_up ? X(sn, 1, 0, 0) : zero;
            const T wp = has_up ? X(sn, 2, 0, 0) : zero, ap = has_up ? X(sn, 3, 0, 0) : zero;
            const T bp = has_up ? X(sn, 4, 0, 0) : zero, fp = has_up ? X(sn, 5, 0, 0) : zero;
            const T rho0 = ac - bc;
            const T uxp = X(sc, 0, 1, 0), wzp = X(sc, 2, 0, 1);

            auto emit = [&](int f, T hval, T gp, T nu_ly) {
                if constexpr (mode == 1) {
                    a.dbg[f][(size_t)j * (size_t)pl + (unsigned)e] = (double)hval;
                    return;
                }
                const T rv = dt * (gam * hval + zet * hold_c[f] - alp * gp + alp * nu_ly);
                st_once(byte_at((T *)a.r[f], qb), rv);
                if (keep) st_once(byte_at((T *)a.h[f], qb), hval);
                if (fuse) {
                    const int sys = (f == 1) ? 1 : (f >= 3 ? 2 : 0);
                    const double *cf = a.cn_coef + (size_t)sys * 3 * M;
                    const double *np = a.cn_coef + 9 * (size_t)M + 9 * kCnMaxSlabs + (size_t)sys * M;
                    cl[f] = uniform_load(cf, j) * (double)rv + uniform_load(cf + M, j) * cl[f];
                    ck[f] += uniform_load(np, j) * cl[f];
                }
            };

            // ---------------- u on the x-face ----------------
            {
                const T uxm = X(sc, 0, -1, 0), uzp = X(sc, 0, 0, 1), uzm = X(sc, 0, 0, -1);
                const T a1 = half * (uxp + uc), a2 = half * (uc + uxm);
                const T cx = (a1 * a1 - a2 * a2) * idx_;
                T flux_t = T(0), flux_b = T(0), ut = T(ph.u_top), ub = T(ph.u_bot);
                if (has_up) {
                    ut = up_;
                    flux_t = half * (vp + X(sn, 1, -1, 0)) * half * (ut + uc);
                }
                if (has_dn) {
                    ub = um;
                    flux_b = half * (vc + X(sc, 1, -1, 0)) * half * (uc + ub);
                }
                const T cy = (flux_t - flux_b) * idn;
                const T wf = half * (wzp + X(sc, 2, -1, 1));
                const T wb = half * (wc + X(sc, 2, -1, 0));
                const T cz = (wf * half * (uzp + uc) - wb * half * (uc + uzm)) * idz_;
                const T lap = (uxp - two * uc + uxm) * ix2 + (uzp - two * uc + uzm) * iz2;
                const T rhox = X(sc, 3, -1, 0) - X(sc, 4, -1, 0);
                const T f = kf * half * (rho0 + rhox) * (ph0 - X(sc, 5, -1, 0)) * idx_;
                const T ly = ((ut - uc) * idct - (uc - ub) * idcb) * idn;
                const T lapH = imp ? zero : lap, lapI = imp ? lap : zero;
                emit(0, -(cx + cy + cz) + ire * lapH + f, (pc - X(sc, 6, -1, 0)) * idx_, ire * (ly + lapI));
            }
            __builtin_amdgcn_sched_barrier(0);
            // ---------------- w on the z-face ----------------
            {
                const T wzm = X(sc, 2, 0, -1), wxp = X(sc, 2, 1, 0), wxm = X(sc, 2, -1, 0);
                const T a1 = half * (wzp + wc), a2 = half * (wc + wzm);
                const T cz = (a1 * a1 - a2 * a2) * idz_;
                const T ur = half * (uxp + X(sc, 0, 1, -1));
                const T ul = half * (uc + X(sc, 0, 0, -1));
                const T cx = (ur * half * (wxp + wc) - ul * half * (wc + wxm)) * idx_;
                T flux_t = T(0), flux_b = T(0), wt = T(0), wb = T(0);
                if (has_up) {
                    wt = wp;
                    flux_t = half * (vp + X(sn, 1, 0, -1)) * half * (wt + wc);
                }
                if (has_dn) {
                    wb = wm;
                    flux_b = half * (vc + X(sc, 1, 0, -1)) * half * (wc + wb);
                }
                const T cy = (flux_t - flux_b) * idn;
                const T lap = (wxp - two * wc + wxm) * ix2 + (wzp - two * wc + wzm) * iz2;
                const T rhoz = X(sc, 3, 0, -1) - X(sc, 4, 0, -1);
                const T f = kf * half * (rho0 + rhoz) * (ph0 - X(sc, 5, 0, -1)) * idz_;
                const T ly = ((wt - wc) * idct - (wc - wb) * idcb) * idn;
                const T lapH = imp ? zero : lap, lapI = imp ? lap : zero;
                emit(2, -(cx + cy + cz) + ire * lapH + f, (pc - X(sc, 6, 0, -1)) * idz_, ire * (ly + lapI));
            }
            __builtin_amdgcn_sched_barrier(0);
            // ---------------- v on the bottom y-face of row j ----------------
            if (has_dn) {
                const T vwl = T(uniform_load(a.tb.vwl, j)), vwu = T(uniform_load(a.tb.vwu, j));
                const T idn_lo = T(uniform_load(a.tb.idn, j - 1));
                const T vtop = has_up ? vp : T(0);
                const T vbot = (j > 1) ? vm : T(0);
                const T a1 = half * (vtop + vc), a2 = half * (vc + vbot);
                const T cy = (a1 * a1 - a2 * a2) * idcb;
                const T ur = u_xp_m * vwl + uxp * vwu;
                const T ul = um * vwl + uc * vwu;
                const T vxp = X(sc, 1, 1, 0), vxm = X(sc, 1, -1, 0), vzp = X(sc, 1, 0, 1), vzm = X(sc, 1, 0, -1);
                const T cx = (ur * half * (vxp + vc) - ul * half * (vc + vxm)) * idx_;
                const T wf = w_zp_m * vwl + wzp * vwu;
                const T wbk = wm * vwl + wc * vwu;
                const T cz = (wf * half * (vzp + vc) - wbk * half * (vc + vzm)) * idz_;
                const T lap = (vxp - two * vc + vxm) * ix2 + (vzp - two * vc + vzm) * iz2;
                const T rhoy = am - bm;
                const T ey = e0 + (ph0 - fm) * idcb;
                const T f = kf * half * (rho0 + rhoy) * ey;
                const T ly = ((vtop - vc) * idn - (vc - vbot) * idn_lo) * idcb;
                const T lapH = imp ? zero : lap, lapI = imp ? lap : zero;
                emit(1, -(cx + cy + cz) + ire * lapH + f, (pc - pm) * idcb, ire * (ly + lapI));
            } else {
                emit(1, T(0), T(0), T(0));
                if constexpr (mode == 0) st_once(byte_at((T *)a.r[1], qb), T(0));
            }
            __builtin_amdgcn_sched_barrier(0);
            // ---------------- ions at the cell centre ----------------
            {
                const T fxp = X(sc, 5, 1, 0), fxm = X(sc, 5, -1, 0), fzp = X(sc, 5, 0, 1), fzm = X(sc, 5, 0, -1);
                const T gx_r = (fxp - ph0) * idx_, gx_l = (ph0 - fxm) * idx_;
                const T gz_f = (fzp - ph0) * idz_, gz_b = (ph0 - fzm) * idz_;
                const T ey_t = has_up ? e0 + (fp - ph0) * idct : T(0);
                const T ey_b = has_dn ? e0 + (ph0 - fm) * idcb : T(0);
                const T vt = has_up ? vp : T(0);
                // potential differences across the six faces (the hybrid
                // migration rule's switch; block-uniform hyb)
                const bool hyb = ph.hybrid != 0.0;
                const T dpx_r = fxp - ph0, dpx_l = ph0 - fxm, dpz_f = fzp - ph0, dpz_b = ph0 - fzm;
                T dpy_t = T(0), dpy_b = T(0);
                if (hyb) {
                    if (has_up) dpy_t = y_dphi(e0, T(uniform_load(a.tb.dc, j + 1)), fp - ph0);
                    if (has_dn) dpy_b = y_dphi(e0, T(uniform_load(a.tb.dc, j)), ph0 - fm);
                }
#pragma unroll
                for (int sp = 0; sp < 2; ++sp) {
                    const int fi = 3 + sp;
                    const T zs = sp == 0 ? T(1) : T(-1);
                    const T cc = sp == 0 ? ac : bc;
                    const T cu = sp == 0 ? ap : bp;
                    const T cd = sp == 0 ? am : bm;
                    const T cxp = X(sc, fi, 1, 0), cxm = X(sc, fi, -1, 0), czp = X(sc, fi, 0, 1), czm = X(sc, fi, 0, -1);
                    const T fxr = half * (cxp + cc), fxl = half * (cc + cxm);
                    const T fzf = half * (czp + cc), fzb = half * (cc + czm);
                    const T ax = (uxp * fxr - uc * fxl) * idx_;
                    const T az = (wzp * fzf - wc * fzb) * idz_;
                    T at = T(0), ab = T(0), mt = T(0), mb = T(0), dft = T(0), dfb = T(0);
                    if (has_up) {
                        const T fy = half * (cu + cc);
                        at = vt * fy;
                        mt = mig_face(hyb, fy, cc, cu, dpy_t, zs) * ey_t;
                        dft = (cu - cc) * idct;
                    }
                    if (has_dn) {
                        const T fy = half * (cc + cd);
                        ab = vc * fy;
                        mb = mig_face(hyb, fy, cd, cc, dpy_b, zs) * ey_b;
                        dfb = (cc - cd) * idcb;
                    }
                    const T ay = (at - ab) * idn;
                    const T mx = (mig_face(hyb, fxr, cc, cxp, dpx_r, zs) * gx_r -
                                  mig_face(hyb, fxl, cxm, cc, dpx_l, zs) * gx_l) * idx_;
                    const T mz = (mig_face(hyb, fzf, cc, czp, dpz_f, zs) * gz_f -
                                  mig_face(hyb, fzb, czm, cc, dpz_b, zs) * gz_b) * idz_;
                    const T my = (mt - mb) * idn;
                    const T dxx = (cxp - two * cc + cxm) * ix2 + (czp - two * cc + czm) * iz2;
                    const T dxxH = imp ? zero : dxx;
                    const T diffI = imp ? kd * ((dft - dfb) * idn + dxx) : kd * (dft - dfb) * idn;
                    emit(fi, -(ax + ay + az) + kd * (dxxH + zs * (mx + my + mz)), T(0), diffI);
                }
            }
            // carry row j as row j - 1 of the next step
            um = uc; vm = vc; wm = wc; am = ac; bm = bc; fm = ph0; pm = pc;
            u_xp_m = uxp;
            w_zp_m = wzp;
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) hold_c[f] = hold_n[f];
        __syncthreads();  // every wave is done with slot sc (row j)
        if (pre) store_rows(sc, rn);
        __syncthreads();
    }
    if (fuse && active) {  // both exits of this column's slab (zero inputs)
        const unsigned S = slabs;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            a.cn_scr[((size_t)f * S + slab) * (size_t)pl + (unsigned)e] = cl[f];
            a.cn_scr[((size_t)(5 + f) * S + slab) * (size_t)pl + (unsigned)e] = ck[f];
        }
    }
}

struct CnArgs {
    Dims d;
    const Phys *phys;
    size_t ms;
    Tables tb;
    Stage st;
    void *q[5];
    const void *r[5];  // right-hand sides, state type
    const double *clock;
    double *coef;  // per stage: [3 systems][g, m, n][M], then [3 systems][P, Phi, Nu][kCnMaxSlabs]
    double *scr;   // row-slab method: per member [2][5 fields][slabs][plane] FP64 scratch
    int slab_rows; // row-slab method: rows per slab (0: lane-scan method)
    int slabs;
    int out_r;     // lane-scan method: write the solution back into r (a factor of the
                   // three-direction factorisation) instead of q += solution
};

// Row coefficients of the Crank-Nicolson matrix (I - beta L_y) of system
// sys: 0 = cell rows with wall values (u, w), 1 = interior nodes (v),
// 2 = cell rows with zero-flux walls (c+, c-).  lo/up are the L_y
// coefficient tables of the system's rows (node rows for sys 1).
__device__ __forceinline__ void cn_row(const double *lo_tab, const double *up_tab, int sys, int M, int j,
                                       double beta, double &A, double &B, double &C) {
    double lo, up, di;
    const double aa = lo_tab[j], cc = up_tab[j];
    if (sys == 1) {
        lo = (j > 1) ? aa : 0.0;
        up = (j < M - 1) ? cc : 0.0;
        di = -(aa + cc);
    } else {
        lo = (j > 0) ? aa : 0.0;
        up = (j < M - 1) ? cc : 0.0;
        di = -(lo + up);
        if (sys == 0) {
            if (j == 0) di -= aa;
            if (j == M - 1) di -= cc;
        }
    }
    A = -beta * lo;
    B = 1.0 - beta * di;
    C = -beta * up;
}


// The matrix is the same for every (x, z) column, so Thomas elimination
// reduces to two linear recurrences with column-independent coefficients:
//   d'_j = g_j r_j + m_j d'_{j-1},   x_j = d'_j + n_j x_{j+1}
// with g = 1/den, m = -A/den, n = -c' (den, c' of the Thomas forward pass).
// One block per member and Runge-Kutta stage (blockIdx.y): the L_y tables are
// staged in LDS, one thread per system runs the (serial) forward pass from
// LDS with one reciprocal per row, and the block stores the 9 M coefficients
// of its stage with coalesced writes.  Launched once per Runge-Kutta step
// (dt changes only at the first stage).
struct CnStages {
    double alp[3];
};

// Row-slab form of the same recurrences (used when the rows are split into
// slabs of L rows, one thread per column and slab): for slab [a, b) the
// column-independent quantities are P = prod m_j, Nu = prod n_j and Phi = the
// local backward sweep (zero input at b) of p_j = prod_{i=a..j} m_i, taken at
// row a.  A column's exact solution on the slab is then
//   x_j = kappa_j + phi_j D + nu_j X
// with D = d'_{a-1}, X = x_b and kappa the local backward sweep of the local
// forward sweep of r; D and X follow from scans across the slabs.

__global__ void __launch_bounds__(256) k_cn_coef(Dims d, Tables tb, const Phys *phys, const double *clock,
                                                 double *coef, CnStages stages, int slab_rows, size_t ms) {
    __shared__ double s_tab[4][kMaxRows];      // lyc_lo, lyc_up, lyn_lo, lyn_up
    __shared__ double s_out[9][kMaxRows];      // [sys][g, m, n][row]
    phys = member_ptr(phys, ms);
    clock = member_ptr(clock, ms);
    const int M = d.M;
    const int stage = blockIdx.y;
    coef = member_ptr(coef, ms) + (size_t)stage * cn_stage_stride(M);
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        s_tab[0][j] = tb.lyc_lo[j];
        s_tab[1][j] = tb.lyc_up[j];
        s_tab[2][j] = tb.lyn_lo[j];
        s_tab[3][j] = tb.lyn_up[j];
    }
    __syncthreads();
    const int sys = threadIdx.x;
    if (sys < 3) {
        const double nu = (sys == 2) ? phys->kd : phys->ire;
        const double beta = 0.5 * stages.alp[stage] * clock[1] * nu;
        const double *lo_tab = s_tab[sys == 1 ? 2 : 0], *up_tab = s_tab[sys == 1 ? 3 : 1];
        double *g = s_out[3 * sys], *m = s_out[3 * sys + 1], *n = s_out[3 * sys + 2];
        const int j0 = (sys == 1) ? 1 : 0;
        if (j0 == 1) g[0] = m[0] = n[0] = 0.0;  // node row 0 is the wall: no unknown
        double cprev = 0.0;
        for (int j = j0; j < M; ++j) {
            double A, B, C;
            cn_row(lo_tab, up_tab, sys, M, j, beta, A, B, C);
            const double rden = 1.0 / (B - A * cprev);
            const double cj = C * rden;
            g[j] = rden;
            m[j] = -A * rden;
            n[j] = -cj;
            cprev = cj;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 9 * M; e += blockDim.x) {
        const int sk = e / M, j = e - sk * M;
        coef[e] = s_out[sk][j];
    }
    if (slab_rows > 0) {
        const int nslab = (M + slab_rows - 1) / slab_rows;
        double *sl = coef + 9 * (size_t)M;
        for (int t = threadIdx.x; t < 3 * nslab; t += blockDim.x) {
            const int sy = t / nslab, sb = t - sy * nslab;
            const double *m = s_out[3 * sy + 1], *n = s_out[3 * sy + 2];
            const int a = sb * slab_rows, b = (a + slab_rows < M) ? a + slab_rows : M;
            double P = 1.0, Nu = 1.0;
            for (int j = a; j < b; ++j) { P *= m[j]; Nu *= n[j]; }
            // phi_j = p_j + n_j phi_{j+1}, phi_b = 0, with p_j = prod_{i=a..j} m_i
            double phi = 0.0;
            for (int j = b - 1; j >= a; --j) {
                double pj = 1.0;
                for (int i = a; i <= j; ++i) pj *= m[i];
                phi = pj + n[j] * phi;
            }
            sl[(3 * sy + 0) * kCnMaxSlabs + sb] = P;
            sl[(3 * sy + 1) * kCnMaxSlabs + sb] = phi;
            sl[(3 * sy + 2) * kCnMaxSlabs + sb] = Nu;
            // prod_{i=a}^{j-1} n_i for the rows of the slab (1 at its first row)
            double *np = sl + 9 * kCnMaxSlabs + (size_t)sy * M;
            double pr = 1.0;
            for (int j = a; j < b; ++j) {
                np[j] = pr;
                pr *= n[j];
            }
        }
    }
}

// Columns staged per block: 16 (one 128-byte line per row in FP64; two FP32
// tiles share a line) for blocks of up to 256 threads, 32 for 512-thread
// blocks (a whole line per row in FP32 at the same waves per CU).
inline int cn_tile_cols(int threads) { return threads > 256 ? 32 : 16; }

// Crank-Nicolson solve of one tile of kCnTx columns: the rows of r are staged
// in LDS with coalesced loads; each wave then solves one column at a time
// with its rows split into 64 contiguous lane segments.  Each recurrence is
// a local sweep per lane followed by a 6-step scan of affine maps across the
// wave (x -> T + Q x composed lane by lane) and a second local sweep from the
// correct incoming value.  Finally q += x with coalesced stores.
// Staging batches of the lane-scan solves: 48 bytes of loads per thread in
// flight per wait (6 FP64 or 12 FP32 values), measured best for both: more
// FP64 registers cost occupancy, fewer FP32 loads leave bandwidth unused.
constexpr int kCnBatchBytes = 48;
template <typename T>
constexpr int cn_batch() { return kCnBatchBytes / (int)sizeof(T); }

template <typename T, int kCnTx, int kCnMaxR>
__global__ void __launch_bounds__(512) k_cn_scan(CnArgs a) {
    extern __shared__ double s_r[];
    const uint3 blk = xcd_block3();  // adjacent column tiles share an L2
    const int f = (int)blk.y;
    const size_t ms = a.ms;
    const int sys = (f == 1) ? 1 : (f >= 3 ? 2 : 0);
    const int j0 = (sys == 1) ? 1 : 0;
    const int M = a.d.M;
    const int64_t pl = a.d.plane;
    const int64_t c0 = (int64_t)blk.x * kCnTx;
    const int ncol = (int)((pl - c0) < kCnTx ? (pl - c0) : kCnTx);
    const T *r = (const T *)member_ptr_at(a.r[f], ms, blk.z);  // may be rewritten in place (out_r)
    T *__restrict__ q = (T *)member_ptr_at(a.q[f], ms, blk.z);
    const double *__restrict__ coef =
        member_ptr_at(a.coef, ms, blk.z) + (size_t)a.st.k * cn_stage_stride(M) + (size_t)sys * 3 * M;
    const double *__restrict__ cg = coef, *__restrict__ cm = coef + M, *__restrict__ cn = coef + 2 * M;
    constexpr int LD = kCnTx + 1;
    const int nrow = M - j0;
    const int ntile = nrow * kCnTx, bd = (int)blockDim.x;
    // Staging in batches of cn_batch<T>() unconditional loads per thread (lanes
    // past the tile read its first element, which exists, and discard it), so
    // that a thread waits for memory once per batch, not once per element.
    // (offsets within one field: rows * plane < 2^32 for every supported grid)
    const unsigned upl = (unsigned)pl, uc0 = (unsigned)c0;
    const unsigned o_safe = (unsigned)j0 * upl + uc0;
    if constexpr (sizeof(T) == 4) {
        // FP32: two adjacent columns per 8-byte access (the plane, the tile
        // origin and ncol are even, so a pair is wholly inside or outside)
        constexpr int TXW = kCnTx / 2, B = cn_batch<T>() / 2;
        const int ntw = nrow * TXW;
        for (int e0 = threadIdx.x; e0 < ntw; e0 += B * bd) {
            nspnp_f2v v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int e = e0 + u * bd, jj = j0 + e / TXW, c = 2 * (e % TXW);
                v[u] = ld_once2((const float *)r + ((e < ntw && c < ncol) ? (unsigned)jj * upl + uc0 + (unsigned)c : o_safe));
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int e = e0 + u * bd, jj = j0 + e / TXW, c = 2 * (e % TXW);
                if (e < ntw) {
                    s_r[jj * LD + c] = (c < ncol) ? (double)v[u].x : 0.0;
                    s_r[jj * LD + c + 1] = (c < ncol) ? (double)v[u].y : 0.0;
                }
            }
        }
    } else {
        for (int e0 = threadIdx.x; e0 < ntile; e0 += cn_batch<T>() * bd) {
            T v[cn_batch<T>()];
#pragma unroll
            for (int u = 0; u < cn_batch<T>(); ++u) {
                const int e = e0 + u * bd, jj = j0 + e / kCnTx, c = e % kCnTx;
                v[u] = ld_once(r + ((e < ntile && c < ncol) ? (unsigned)jj * upl + uc0 + (unsigned)c : o_safe));
            }
#pragma unroll
            for (int u = 0; u < cn_batch<T>(); ++u) {
                const int e = e0 + u * bd, jj = j0 + e / kCnTx, c = e % kCnTx;
                if (e < ntile) s_r[jj * LD + c] = (c < ncol) ? (double)v[u] : 0.0;
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int R = kCnMaxR;  // rows per lane (the launcher picks ceil(rows / 64))
    const int js = j0 + lane * R;
    // this lane's recurrence coefficients (the same for every column)
    double g[kCnMaxR], mm[kCnMaxR], nn[kCnMaxR];
    double Qs = 1.0, Ss = 1.0;
#pragma unroll
    for (int t = 0; t < kCnMaxR; ++t) {
        const int j = js + t;
        const bool in = (t < R) && (j < M);
        g[t] = in ? cg[j] : 0.0;
        mm[t] = in ? cm[j] : 1.0;
        nn[t] = in ? cn[j] : 1.0;
        Qs *= mm[t];
        Ss *= nn[t];
    }
    // multipliers of the scans of the affine maps x -> T + Q x across lanes
    // (forward, from lane 0 up) and x -> U + S x (backward, from lane 63 down)
    double qm[6], sm[6];
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int sft = 1 << st;
        qm[st] = Qs;
        sm[st] = Ss;
        const double Qp = __shfl_up(Qs, sft, 64), Sp = __shfl_down(Ss, sft, 64);
        if (lane >= sft) Qs *= Qp;
        if (lane + sft < 64) Ss *= Sp;
    }
    for (int c = wave; c < ncol; c += nwave) {
        double *col = s_r + c;
        double x[kCnMaxR];
#pragma unroll
        for (int t = 0; t < kCnMaxR; ++t) {
            const int j = js + t;
            x[t] = (t < R && j < M) ? col[j * LD] : 0.0;
        }
        // forward d'_j = g_j r_j + m_j d'_{j-1}: local sweep, scan, sweep
        double Tf = 0.0;
#pragma unroll
        for (int t = 0; t < kCnMaxR; ++t) Tf = g[t] * x[t] + mm[t] * Tf;
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            const double Tp = __shfl_up(Tf, 1 << st, 64);
            if (lane >= (1 << st)) Tf += qm[st] * Tp;
        }
        double din = __shfl_up(Tf, 1, 64);
        if (lane == 0) din = 0.0;
#pragma unroll
        for (int t = 0; t < kCnMaxR; ++t) {
            din = g[t] * x[t] + mm[t] * din;
            x[t] = din;
        }
        // backward x_j = d'_j + n_j x_{j+1}
        double U = 0.0;
#pragma unroll
        for (int t = kCnMaxR - 1; t >= 0; --t) U = (g[t] != 0.0 ? x[t] : 0.0) + nn[t] * U;
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            const double Up = __shfl_down(U, 1 << st, 64);
            if (lane + (1 << st) < 64) U += sm[st] * Up;
        }
        double xin = __shfl_down(U, 1, 64);
        if (lane == 63) xin = 0.0;
#pragma unroll
        for (int t = kCnMaxR - 1; t >= 0; --t) {
            xin = (g[t] != 0.0 ? x[t] : 0.0) + nn[t] * xin;
            x[t] = xin;
        }
#pragma unroll
        for (int t = 0; t < kCnMaxR; ++t) {
            const int j = js + t;
            if (t < R && j < M) col[j * LD] = x[t];
        }
    }
    __syncthreads();
    if (a.out_r) {  // a factor of the three-direction factorisation: the solution replaces r
        T *rw = (T *)member_ptr_at(a.r[f], ms, blk.z);  // r was read before the barrier
        for (int e = threadIdx.x; e < ntile; e += bd) {
            const int jj = j0 + e / kCnTx, c = e % kCnTx;
            if (c < ncol) st_once(rw + ((unsigned)jj * upl + uc0 + (unsigned)c), (T)s_r[jj * LD + c]);
        }
        return;
    }
    if constexpr (sizeof(T) == 4) {
        constexpr int TXW = kCnTx / 2, B = cn_batch<T>() / 2;
        const int ntw = nrow * TXW;
        float *qf = (float *)q;
        for (int e0 = threadIdx.x; e0 < ntw; e0 += B * bd) {
            nspnp_f2v v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int e = e0 + u * bd, jj = j0 + e / TXW, c = 2 * (e % TXW);
                v[u] = ld_once2(qf + ((e < ntw && c < ncol) ? (unsigned)jj * upl + uc0 + (unsigned)c : o_safe));
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int e = e0 + u * bd, jj = j0 + e / TXW, c = 2 * (e % TXW);
                if (e < ntw && c < ncol) {
                    nspnp_f2v w;
                    w.x = (float)((double)v[u].x + s_r[jj * LD + c]);
                    w.y = (float)((double)v[u].y + s_r[jj * LD + c + 1]);
                    st_once2(qf + ((unsigned)jj * upl + uc0 + (unsigned)c), w);
                }
            }
        }
    } else {
        for (int e0 = threadIdx.x; e0 < ntile; e0 += cn_batch<T>() * bd) {
            T v[cn_batch<T>()];
#pragma unroll
            for (int u = 0; u < cn_batch<T>(); ++u) {
                const int e = e0 + u * bd, jj = j0 + e / kCnTx, c = e % kCnTx;
                v[u] = ld_once(q + ((e < ntile && c < ncol) ? (unsigned)jj * upl + uc0 + (unsigned)c : o_safe));
            }
#pragma unroll
            for (int u = 0; u < cn_batch<T>(); ++u) {
                const int e = e0 + u * bd, jj = j0 + e / kCnTx, c = e % kCnTx;
                if (e < ntile && c < ncol) st_once(q + ((unsigned)jj * upl + uc0 + (unsigned)c), (T)((double)v[u] + s_r[jj * LD + c]));
            }
        }
    }
}

// ---- implicit x/z diffusion (three-direction approximate factorisation) ----
// (I - b L) x = r along a periodic line of N points, L = (x_{+1} - 2 x + x_{-1}) / h^2,
// is a cyclic tridiagonal system with constant diagonal d = 1 + 2 b / h^2 and
// off-diagonal e = -b / h^2.  With gamma = -d, the corners move into a rank-one
// term (Sherman-Morrison): the tridiagonal B (first diagonal d - gamma, last
// d - e^2 / gamma) is solved for y = B^-1 r, and x = y - ((y_0 + (e/gamma) y_{N-1})
// / (1 + z_0 + (e/gamma) z_{N-1})) z with z = B^-1 (gamma, 0, .., 0, e).  B and z
// are the same for every line of a field, stage and direction: k_cyc_coef makes
// B's elimination recurrences (d'_i = g_i r_i + m_i d'_{i-1}, x_i = d'_i + n_i
// x_{i+1}) and z once per Runge-Kutta step.
struct CycArgs {
    Dims d;
    size_t ms;
    Stage st;
    void *q[5];
    void *r[5];
    const double *cyc;
    int dir;    // 0: x-lines (contiguous), 1: z-lines (stride nx)
    int out_r;  // 1: the solution replaces r; 0: q += solution
};

__global__ void __launch_bounds__(64) k_cyc_coef(Dims d, const Phys *phys, const double *clock, double *cyc,
                                                 CnStages stages, size_t ms) {
    phys = member_ptr(phys, ms);
    clock = member_ptr(clock, ms);
    cyc = member_ptr(cyc, ms);
    const int stage = blockIdx.y, sys = threadIdx.x;
    if (sys >= 4) return;
    const int ty = sys >> 1, dir = sys & 1;  // diffusivity (velocity, ions), direction
    const int N = dir == 0 ? d.nx : d.nz;
    const double h = dir == 0 ? d.dx : d.dz;
    const double nu = ty == 0 ? phys->ire : phys->kd;
    const double b = 0.5 * stages.alp[stage] * clock[1] * nu;
    const double dg = 1.0 + 2.0 * b / (h * h), e = -b / (h * h), gam = -dg;
    const int64_t nb = cyc_block_doubles(d.nx, d.nz), Nmax = (nb - 4) / 4;
    double *blk = cyc + ((int64_t)(stage * 2 + ty) * 2 + dir) * nb;
    double *g = blk, *m = blk + Nmax, *n = blk + 2 * Nmax, *z = blk + 3 * Nmax;
    double cprev = 0.0;
    for (int i = 0; i < N; ++i) {
        const double bi = (i == 0) ? dg - gam : (i == N - 1 ? dg - e * e / gam : dg);
        const double ai = (i == 0) ? 0.0 : e;
        const double rden = 1.0 / (bi - ai * cprev);
        const double ci = (i == N - 1) ? 0.0 : e * rden;
        g[i] = rden;
        m[i] = -ai * rden;
        n[i] = -ci;
        cprev = ci;
    }
    // z = B^-1 u, u = (gamma, 0, ..., 0, e)
    double dp = 0.0;
    for (int i = 0; i < N; ++i) {
        const double ui = (i == 0) ? gam : (i == N - 1 ? e : 0.0);
        dp = g[i] * ui + m[i] * dp;
        z[i] = dp;
    }
    for (int i = N - 2; i >= 0; --i) z[i] = z[i] + n[i] * z[i + 1];
    const double vf = e / gam;
    blk[4 * Nmax] = vf;
    blk[4 * Nmax + 1] = 1.0 / (1.0 + z[0] + vf * z[N - 1]);
}

// One tile of kCycTx periodic lines of one field per block, staged in LDS
// (x-lines: each line contiguous; z-lines: kCycTx neighbouring columns per
// element, 128-byte runs in FP64); each wave solves one line with its N points
// split into 64 contiguous lane segments, as in the Crank-Nicolson lane scans,
// then applies the periodic correction (the line's end values y_0, y_{N-1}
// broadcast from their lanes).
constexpr int kCycTx = 16;

constexpr int kCycBatch = 8;  // loads per thread per wait in the periodic line solves

template <typename T, int R>
__global__ void __launch_bounds__(256) k_cyc_scan(CycArgs a) {
    extern __shared__ double s_l[];
    const uint3 blk = xcd_block3();
    const int f = (int)blk.y, ty = f < 3 ? 0 : 1;
    const int dir = a.dir, nx = a.d.nx, nz = a.d.nz;
    const int N = dir == 0 ? nx : nz, L = dir == 0 ? nz : nx;  // points per line, lines per row
    const int ntl = (L + kCycTx - 1) / kCycTx;
    const int j = (int)blk.x / ntl, l0 = ((int)blk.x - j * ntl) * kCycTx;
    const int nl = (L - l0) < kCycTx ? (L - l0) : kCycTx;
    const unsigned upl = (unsigned)a.d.plane, row = (unsigned)j * upl;
    T *rr = (T *)member_ptr_at(a.r[f], a.ms, blk.z);
    T *qq = (T *)member_ptr_at(a.q[f], a.ms, blk.z);
    const int64_t nb = cyc_block_doubles(nx, nz), Nmax = (nb - 4) / 4;
    const double *cb = member_ptr_at(a.cyc, a.ms, blk.z) + ((int64_t)(a.st.k * 2 + ty) * 2 + dir) * nb;
    const double *cg = cb, *cm = cb + Nmax, *cn = cb + 2 * Nmax, *cz = cb + 3 * Nmax;
    const double vf = cb[4 * Nmax], sf = cb[4 * Nmax + 1];
    constexpr int LD = kCycTx + 1;
    const int ntile = N * kCycTx, bd = (int)blockDim.x;
    // element (point i, line c) of the tile: x-lines (l0 + c) nx + i, z-lines i nx + l0 + c
    auto addr = [&](int i, int c) -> unsigned {
        return row + (dir == 0 ? (unsigned)(l0 + c) * (unsigned)nx + (unsigned)i : (unsigned)i * (unsigned)nx + (unsigned)(l0 + c));
    };
    // staging order: along the contiguous direction of memory (point i, line c of element e)
    struct IC {
        int i, c;
    };
    auto split = [&](int e) -> IC {
        if (dir == 0) {
            const int c = e / N;
            return IC{e - c * N, c};
        }
        const int i = e / kCycTx;
        return IC{i, e - i * kCycTx};
    };
    for (int e0 = threadIdx.x; e0 < ntile; e0 += kCycBatch * bd) {
        T v[kCycBatch];
#pragma unroll
        for (int u = 0; u < kCycBatch; ++u) {
            const int e = e0 + u * bd;
            const IC p = split(e < ntile ? e : 0);
            v[u] = ld_once(rr + ((e < ntile && p.c < nl) ? addr(p.i, p.c) : row));
        }
#pragma unroll
        for (int u = 0; u < kCycBatch; ++u) {
            const int e = e0 + u * bd;
            if (e < ntile) {
                const IC p = split(e);
                s_l[p.i * LD + p.c] = (p.c < nl) ? (double)v[u] : 0.0;
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int js = lane * R;
    double g[R], mm[R], nn[R], zz[R];
    double Qs = 1.0, Ss = 1.0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int i = js + t;
        const bool in = i < N;
        g[t] = in ? cg[i] : 0.0;
        mm[t] = in ? cm[i] : 1.0;
        nn[t] = in ? cn[i] : 1.0;
        zz[t] = in ? cz[i] : 0.0;
        Qs *= mm[t];
        Ss *= nn[t];
    }
    double qm[6], sm[6];
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int sft = 1 << st;
        qm[st] = Qs;
        sm[st] = Ss;
        const double Qp = __shfl_up(Qs, sft, 64), Sp = __shfl_down(Ss, sft, 64);
        if (lane >= sft) Qs *= Qp;
        if (lane + sft < 64) Ss *= Sp;
    }
    const int last_lane = (N - 1) / R, last_t = (N - 1) - last_lane * R;
    for (int c = wave; c < nl; c += nwave) {
        double *col = s_l + c;
        double x[R];
#pragma unroll
        for (int t = 0; t < R; ++t) x[t] = (js + t < N) ? col[(js + t) * LD] : 0.0;
        double Tf = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) Tf = g[t] * x[t] + mm[t] * Tf;
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            const double Tp = __shfl_up(Tf, 1 << st, 64);
            if (lane >= (1 << st)) Tf += qm[st] * Tp;
        }
        double din = __shfl_up(Tf, 1, 64);
        if (lane == 0) din = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            din = g[t] * x[t] + mm[t] * din;
            x[t] = din;
        }
        double U = 0.0;
#pragma unroll
        for (int t = R - 1; t >= 0; --t) U = (g[t] != 0.0 ? x[t] : 0.0) + nn[t] * U;
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            const double Up = __shfl_down(U, 1 << st, 64);
            if (lane + (1 << st) < 64) U += sm[st] * Up;
        }
        double xin = __shfl_down(U, 1, 64);
        if (lane == 63) xin = 0.0;
#pragma unroll
        for (int t = R - 1; t >= 0; --t) {
            xin = (g[t] != 0.0 ? x[t] : 0.0) + nn[t] * xin;
            x[t] = xin;
        }
        // periodic correction from the line's end values
        double ylast = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t)
            if (t == last_t) ylast = x[t];
        const double y0 = __shfl(x[0], 0, 64);
        const double yl = __shfl(ylast, last_lane, 64);
        const double wcor = (y0 + vf * yl) * sf;
#pragma unroll
        for (int t = 0; t < R; ++t)
            if (js + t < N) col[(js + t) * LD] = x[t] - wcor * zz[t];
    }
    __syncthreads();
    for (int e0 = threadIdx.x; e0 < ntile; e0 += kCycBatch * bd) {
        T v[kCycBatch];
        if (!a.out_r) {
#pragma unroll
            for (int u = 0; u < kCycBatch; ++u) {
                const int e = e0 + u * bd;
                const IC p = split(e < ntile ? e : 0);
                v[u] = ld_once(qq + ((e < ntile && p.c < nl) ? addr(p.i, p.c) : row));
            }
        }
#pragma unroll
        for (int u = 0; u < kCycBatch; ++u) {
            const int e = e0 + u * bd;
            if (e < ntile) {
                const IC p = split(e);
                if (p.c < nl) {
                    const double xs = s_l[p.i * LD + p.c];
                    if (a.out_r) st_once(rr + addr(p.i, p.c), (T)xs);
                    else st_once(qq + addr(p.i, p.c), (T)((double)v[u] + xs));
                }
            }
        }
    }
}

// ---- Crank-Nicolson, row-slab method (large grids) ----
// One thread per (column, slab): every pass streams whole rows of a tile of
// 256 columns, so each DRAM page opened serves a long contiguous run.
__device__ __forceinline__ void cn_slab_site(const CnArgs &a, unsigned z, int &f, unsigned &mem, int &sys) {
    f = (int)(z % 5u);
    mem = z / 5u;
    sys = (f == 1) ? 1 : (f >= 3 ? 2 : 0);
}

// pass 1 (the exits of the local sweeps of each slab, zero inputs) runs in
// the explicit kernel as it produces r (ExplicitArgs::cn_coef).

// pass 2: scans across the slabs of each column; the slab inputs D (forward)
// and X (backward) replace the exits in place
__global__ void __launch_bounds__(256) k_cn_slab_scan(CnArgs a) {
    int f, sys;
    unsigned mem;
    cn_slab_site(a, blockIdx.z, f, mem, sys);
    const int64_t pl = a.d.plane;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= pl) return;
    const int M = a.d.M, S = a.slabs;
    const double *sl = member_ptr_at(a.coef, a.ms, mem) + (size_t)a.st.k * cn_stage_stride(M) + 9 * (size_t)M;
    const double *P = sl + (3 * sys + 0) * kCnMaxSlabs, *Phi = sl + (3 * sys + 1) * kCnMaxSlabs,
                 *Nu = sl + (3 * sys + 2) * kCnMaxSlabs;
    double *scr = member_ptr_at(a.scr, a.ms, mem);
    double *lam = scr + (int64_t)f * S * pl + e, *kap = scr + (int64_t)(5 + f) * S * pl + e;
    // batches of 8 slabs: loads first (slabs past the end re-read the last
    // one and are ignored), multipliers included, then the recurrence and
    // the stores
    constexpr int kB = 8;
    double D = 0.0;
    for (int s0 = 0; s0 < S; s0 += kB) {
        double ex[kB], pb[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int sb = s0 + u < S ? s0 + u : S - 1;
            ex[u] = lam[(int64_t)sb * pl];
            pb[u] = P[sb];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int sb = s0 + u;
            if (sb < S) {
                lam[(int64_t)sb * pl] = D;
                D = ex[u] + pb[u] * D;
            }
        }
    }
    double X = 0.0;
    for (int s1 = S - 1; s1 >= 0; s1 -= kB) {
        double ex[kB], din[kB], phb[kB], nub[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int sb = s1 - u >= 0 ? s1 - u : 0;
            ex[u] = kap[(int64_t)sb * pl];
            din[u] = lam[(int64_t)sb * pl];
            phb[u] = Phi[sb];
            nub[u] = Nu[sb];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int sb = s1 - u;
            if (sb >= 0) {
                kap[(int64_t)sb * pl] = X;
                X = ex[u] + phb[u] * din[u] + nub[u] * X;
            }
        }
    }
}

// pass 3: both sweeps of each slab from its exact inputs, then q += x
template <typename T, int L>
__global__ void __launch_bounds__(256) k_cn_slab_apply(CnArgs a) {
    int f, sys;
    unsigned mem;
    cn_slab_site(a, blockIdx.z, f, mem, sys);
    const int64_t pl = a.d.plane;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= pl) return;
    const int M = a.d.M, S = a.slabs, sb = blockIdx.y;
    const int j0 = sb * L, j1 = (j0 + L < M) ? j0 + L : M;
    const T *__restrict__ r = (const T *)member_ptr_at(a.r[f], a.ms, mem);
    T *__restrict__ q = (T *)member_ptr_at(a.q[f], a.ms, mem);
    const double *__restrict__ coef = member_ptr_at(a.coef, a.ms, mem) + (size_t)a.st.k * cn_stage_stride(M) +
                                      (size_t)sys * 3 * M;
    const double *g = coef, *m = coef + M, *n = coef + 2 * M;
    const double *scr = member_ptr_at(a.scr, a.ms, mem);
    double d = scr[((int64_t)(f * S + sb)) * pl + e];
    double x = scr[((int64_t)((5 + f) * S + sb)) * pl + e];
    // r and q of the slab's rows first, all in flight together (rows past the
    // slab re-read its last row and are ignored)
    const unsigned upl = (unsigned)pl, ue = (unsigned)e;
    T rv[L], qv[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const unsigned o = (unsigned)(j0 + t < j1 ? j0 + t : j1 - 1) * upl + ue;
        rv[t] = ld_once(r + o);
        qv[t] = ld_once(q + o);
    }
    double dv[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
        const int j = j0 + t;
        if (j < j1) d = g[j] * (double)rv[t] + m[j] * d;
        dv[t] = d;
    }
#pragma unroll
    for (int t = L - 1; t >= 0; --t) {
        const int j = j0 + t;
        if (j < j1) {
            x = dv[t] + n[j] * x;
            st_once(q + ((unsigned)j * upl + ue), (T)((double)qv[t] + x));
        }
    }
}

// projection correction: u -= a G psi;  p += psi - (a / (2 Re)) L_y psi.
// Each thread owns one (x, z) column of a 2-D tile and marches a slab of
// rows, carrying psi of rows j-1 and j, so psi is read about once; its x-
// and z-neighbours in row j come from the caches (mostly the block's own
// loads).
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
    int tx, tz, ntx, chunks, slabs, slab_rows;
};

constexpr int kCorrRows = 4;  // rows per load batch of k_correct

// kImp: the pressure update takes the full Laplacian of psi (x/z diffusion
// implicit too), p += psi - (a / (2 Re)) (L_x + L_y + L_z) psi.
template <typename T, bool kImp>
__global__ void __launch_bounds__(256) k_correct(CorrArgs a) {
    const Dims &d = a.d;
    const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
    const unsigned chunks = (unsigned)a.chunks, slabs = (unsigned)a.slabs;
    const unsigned chunk = tile % chunks;
    const unsigned slab = (tile / chunks) % slabs;
    const unsigned mem = tile / (chunks * slabs);
    const int nx = d.nx, nz = d.nz, M = d.M;
    const int lk = (int)threadIdx.x / a.tx;
    const int i = (int)(chunk % (unsigned)a.ntx) * a.tx + ((int)threadIdx.x - lk * a.tx);
    const int k = (int)(chunk / (unsigned)a.ntx) * a.tz + lk;
    if (lk >= a.tz || i >= nx || k >= nz) return;
    const int64_t pl = d.plane;
    const int e = k * nx + i;
    const int exm = e - i + ((i == 0) ? nx - 1 : i - 1);
    const int ezm = ((k == 0) ? nz - 1 : k - 1) * nx + i;
    const size_t ms = a.ms;
    double *clock = member_ptr_at(a.clock, ms, mem);
    const Phys *ph = member_ptr_at(a.phys, ms, mem);
    const int j0 = (int)slab * a.slab_rows;
    const int j1 = (j0 + a.slab_rows < M) ? j0 + a.slab_rows : M;
    // substep time t += alp dt (dt is read, never written, by this kernel)
    if (a.advance_clock && e == 0 && j0 == 0) clock[0] += a.alp * clock[1];
    T *u = (T *)member_ptr_at(a.u, ms, mem), *v = (T *)member_ptr_at(a.v, ms, mem);
    T *w = (T *)member_ptr_at(a.w, ms, mem), *p = (T *)member_ptr_at(a.p, ms, mem);
    const double *psi = member_ptr_at(a.psi, ms, mem);
    const double sc = (a.alp > 0.0) ? a.alp * clock[1] : a.fixed;
    const double ire = ph->ire;
    const double idx = 1.0 / d.dx, idz = 1.0 / d.dz;
    double s_dn = (j0 > 0) ? psi[(int64_t)(j0 - 1) * pl + e] : 0.0;  // psi of row j - 1
    double s0 = psi[(int64_t)j0 * pl + e];
    // Rows are corrected in batches of kCorrRows: the batch's loads are all
    // issued before any result is stored (rows past the slab re-read its last
    // row and are ignored), one memory latency per batch.  Offsets within one
    // field fit in 32 bits.
    const unsigned upl = (unsigned)pl;
    struct RowVals {
        double s_up, sxm, szm, sxp, szp;
        T u, v, w, p;
    };
    const int exp_ = e - i + ((i + 1 == nx) ? 0 : i + 1);
    const int ezp = ((k + 1 == nz) ? 0 : k + 1) * nx + i;
    auto load_row = [&](int j, RowVals &r) {
        const unsigned row = (unsigned)j * upl, q = row + (unsigned)e;
        r.s_up = psi[(j + 1 < M) ? q + upl : q];
        r.sxm = psi[row + (unsigned)exm];
        r.szm = psi[row + (unsigned)ezm];
        if (kImp) {
            r.sxp = psi[row + (unsigned)exp_];
            r.szp = psi[row + (unsigned)ezp];
        }
        r.u = ld_once(u + q);
        r.w = ld_once(w + q);
        r.v = ld_once(v + q);
        r.p = ld_once(p + q);  // unconditional (p is always allocated): no branch in the batch
    };
    for (int jb = j0; jb < j1; jb += kCorrRows) {
        RowVals rb[kCorrRows];
#pragma unroll
        for (int t = 0; t < kCorrRows; ++t) load_row(jb + t < j1 ? jb + t : j1 - 1, rb[t]);
#pragma unroll
        for (int t = 0; t < kCorrRows; ++t) {
            const int j = jb + t;
            if (j >= j1) break;
            const RowVals &cur = rb[t];
            const unsigned q = (unsigned)j * upl + (unsigned)e;
            const double s_up = (j + 1 < M) ? cur.s_up : 0.0;
            st_once(u + q, (T)((double)cur.u - sc * (s0 - cur.sxm) * idx));
            st_once(w + q, (T)((double)cur.w - sc * (s0 - cur.szm) * idz));
            const double idcb = uniform_load(a.tb.idc, j);
            if (j > 0) st_once(v + q, (T)((double)cur.v - sc * (s0 - s_dn) * idcb));
            if (a.update_p) {
                const double ft = (j + 1 < M) ? (s_up - s0) * uniform_load(a.tb.idc, j + 1) : 0.0;
                const double fb = (j > 0) ? (s0 - s_dn) * idcb : 0.0;
                double ly = (ft - fb) * uniform_load(a.tb.idn, j);
                if (kImp)
                    ly += (cur.sxp - 2.0 * s0 + cur.sxm) * (idx * idx) + (cur.szp - 2.0 * s0 + cur.szm) * (idz * idz);
                st_once(p + q, (T)((double)cur.p + s0 - 0.5 * sc * ire * ly));
            }
            s_dn = s0;
            s0 = s_up;
        }
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

// Column tiles of the explicit kernel: up to 64 columns along x in the mixed
// form, 32 in FP64 (whole x-lines when nx is smaller), times as many z-lines
// as the block has room for.  The FP64 32 x 8 tile loads 1.33 halo values
// per cell against 1.55 for 64 x 4 (256 bytes of a row per access run);
// the FP32 form keeps 64 columns, a whole 256-byte run of a row.
static void explicit_tiling(const Dims &d, bool fp64, int threads, int slab_rows, ExplicitArgs &a) {
    const int wx = fp64 ? 32 : 64;
    a.tx = d.nx < wx ? d.nx : wx;
    if (a.tx > threads) a.tx = threads;
    a.tz = threads / a.tx;
    a.ntx = (d.nx + a.tx - 1) / a.tx;
    a.chunks = a.ntx * ((d.nz + a.tz - 1) / a.tz);
    a.slab_rows = slab_rows;
    a.slabs = (d.M + slab_rows - 1) / slab_rows;
}

// Launch of the explicit kernel with its halo-tile LDS ring; kHalo halo
// positions per thread cover the tile plus halo ((tx+2)(tz+2) <= kHalo * threads).
static hipError_t explicit_launch(nspnp_state *s, const ExplicitArgs &a, int threads, unsigned blocks) {
    const int hs = (a.tx + 2) * (a.tz + 2);
    const size_t lds = 2 * (size_t)kNF * hs * s->wsize;
    const bool dbg = a.mode == 1;
    if (!dbg && threads == 256 && s->fp64 && a.tx == 32 && a.tz == 8) {  // the common tiles
        // three waves per SIMD (at most 168 VGPRs; 12 bytes per lane spill):
        // with the fused Crank-Nicolson first pass the compiler's own choice
        // (171 VGPRs, two waves) was measured 0.29 ms slower per launch at
        // 512 x 385 x 512 (3.73 against 3.44 ms)
        k_explicit<double, 2, 3, 0, 32, 8><<<blocks, threads, lds, s->stream>>>(a);
    } else if (!dbg && threads == 256 && !s->fp64 && a.tx == 64 && a.tz == 4) {
        k_explicit<float, 2, 3, 0, 64, 4><<<blocks, threads, lds, s->stream>>>(a);
    } else if (hs <= 2 * threads) {
        if (s->fp64) {
            if (dbg) k_explicit<double, 2, 2, 1><<<blocks, threads, lds, s->stream>>>(a);
            else k_explicit<double, 2, 2, 0><<<blocks, threads, lds, s->stream>>>(a);
        } else {
            if (dbg) k_explicit<float, 2, 3, 1><<<blocks, threads, lds, s->stream>>>(a);
            else k_explicit<float, 2, 3, 0><<<blocks, threads, lds, s->stream>>>(a);
        }
    } else if (hs <= 4 * threads) {
        if (s->fp64) {
            if (dbg) k_explicit<double, 4, 2, 1><<<blocks, threads, lds, s->stream>>>(a);
            else k_explicit<double, 4, 2, 0><<<blocks, threads, lds, s->stream>>>(a);
        } else {
            if (dbg) k_explicit<float, 4, 3, 1><<<blocks, threads, lds, s->stream>>>(a);
            else k_explicit<float, 4, 3, 0><<<blocks, threads, lds, s->stream>>>(a);
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Rows per slab of the row-slab CN method when it applies to this handle
// (0: lane-scan method).  Its scratch (two values per field, slab and column)
// lives in the spectrum buffers, unused between the explicit stage and the
// elliptic solves.
int cn_slab_rows(const nspnp_state *s) {
    const int L = s->tiles.cnslab;
    if (L != 16 && L != 32 || s->cfg.implicit_xz) return 0;  // the factorisation uses the lane-scan method
    const int S = (s->d.M + L - 1) / L;
    const int64_t need = 2 * 5 * (int64_t)S * s->d.plane;             // doubles
    const int64_t have = 4 * (int64_t)s->d.nxh * s->d.nz * s->d.M;      // two half spectra
    return (S <= kCnMaxSlabs && need <= have) ? L : 0;
}

// Crank-Nicolson recurrence coefficients of the three stages (and, for the
// row-slab method, its slab products): computed on the device once per
// Runge-Kutta step, after the step's dt, before the explicit kernel that may
// run the method's first pass; at most once per substep.
static hipError_t launch_cn_coef(nspnp_state *s, const Stage &st) {
    if (s->cn_coef_at == s->substeps) return hipSuccess;
    const int L = cn_slab_rows(s);
    if (st.k == 0 || !s->cn_fresh || s->cn_coef_slab != L) {
        CnStages cs;
        for (int q = 0; q < 3; ++q) cs.alp[q] = kRkAlp[q];
        k_cn_coef<<<dim3(1, 3, (unsigned)s->nmem), 256, 0, s->stream>>>(s->d, s->tb, s->d_phys, s->clock,
                                                                       s->cn_coef, cs, L, s->mstride);
        if (s->cfg.implicit_xz)
            k_cyc_coef<<<dim3(1, 3, (unsigned)s->nmem), 64, 0, s->stream>>>(s->d, s->d_phys, s->clock, s->cyc, cs,
                                                                            s->mstride);
        s->cn_fresh = true;
        s->cn_coef_slab = L;
    }
    s->cn_coef_at = s->substeps;
    return hipGetLastError();
}

namespace {

// Limited advective face values of the ions (migration_face 2).  The explicit
// kernel forms the central advective flux; this pass adds, cell by cell, the
// difference between the limited flux's divergence and the central one to
// the ions' H (when the stage keeps it) and to their Crank-Nicolson
// right-hand side (dt gam times the difference), or, in mode 1, to the
// exported H.  The face values reach two cells upwind (periodic in x and z;
// the upwind cell alone where it is a wall row).
//
// One thread per (x, z) column marches a slab of rows with rows j-2 .. j+2
// of c+- of its own column in registers (the next row loaded one step
// ahead); x and z neighbours come from the same row, which the neighbouring
// columns' threads read at the same time.  With the row-slab Crank-Nicolson
// method, whose first pass ran inside the explicit kernel on the r before
// this correction, the pass adds the slab exits of its own change of r to
// the method's scratch (the exits are linear in r), on the same slabs.
struct AdvArgs {
    Dims d;
    size_t ms;
    Tables tb;
    Stage st;
    const void *u, *v, *w, *c[2];
    void *h[2], *r[2];
    double *dbg[2];
    const double *clock;
    int mode;            // 0: substep (H, r of this stage); 1: dbg only
    int ntiles;          // 256-column tiles per plane
    int slabs, slab_rows;
    const double *cn_coef;  // this stage's row-slab CN coefficients (NULL: no exits to update)
    double *cn_scr;
};

template <typename T>
__global__ void __launch_bounds__(256) k_adv_limit(AdvArgs a) {
    const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);  // column tiles fastest: z-neighbours share an L2
    const unsigned ct = tile % (unsigned)a.ntiles;
    const unsigned slab = (tile / (unsigned)a.ntiles) % (unsigned)a.slabs;
    const unsigned mem = tile / ((unsigned)a.ntiles * (unsigned)a.slabs);
    const int pl = (int)a.d.plane;
    const int e = (int)(ct * blockDim.x + threadIdx.x);
    if (e >= pl) return;
    const int M = a.d.M, nx = a.d.nx, nz = a.d.nz;
    const size_t ms = a.ms;
    const int i = e % nx, k = e / nx;
    auto wrap = [](int q, int n) { return q < 0 ? q + n : (q >= n ? q - n : q); };  // n >= 4
    // a field's base plus a 32-bit byte offset (a field of every supported
    // grid is below 2^32 bytes); rows outside the grid are clamped to an
    // existing row and their values not used
    const unsigned W = (unsigned)sizeof(T), P = (unsigned)pl * W;
    const unsigned kx = (unsigned)(k * nx) * W;
    const unsigned ex = (unsigned)e * W;
    const unsigned dxp = kx + (unsigned)wrap(i + 1, nx) * W, dxm = kx + (unsigned)wrap(i - 1, nx) * W;
    const unsigned dxp2 = kx + (unsigned)wrap(i + 2, nx) * W, dxm2 = kx + (unsigned)wrap(i - 2, nx) * W;
    const unsigned dzp = (unsigned)(wrap(k + 1, nz) * nx + i) * W, dzm = (unsigned)(wrap(k - 1, nz) * nx + i) * W;
    const unsigned dzp2 = (unsigned)(wrap(k + 2, nz) * nx + i) * W, dzm2 = (unsigned)(wrap(k - 2, nz) * nx + i) * W;
    auto rowb = [&](int jj) { return (unsigned)(jj < 0 ? 0 : (jj >= M ? M - 1 : jj)) * P; };
    const T *u = member_ptr_at((const T *)a.u, ms, mem), *v = member_ptr_at((const T *)a.v, ms, mem);
    const T *w = member_ptr_at((const T *)a.w, ms, mem);
    const T *cf[2] = {member_ptr_at((const T *)a.c[0], ms, mem), member_ptr_at((const T *)a.c[1], ms, mem)};
    T *hf[2] = {member_ptr_at((T *)a.h[0], ms, mem), member_ptr_at((T *)a.h[1], ms, mem)};
    T *rf[2] = {member_ptr_at((T *)a.r[0], ms, mem), member_ptr_at((T *)a.r[1], ms, mem)};
    const T half = T(0.5);
    const T idx_ = T(1.0 / a.d.dx), idz_ = T(1.0 / a.d.dz);
    const T dtg = T(member_ptr_at(a.clock, ms, mem)[1]) * T(a.st.gam);
    const bool keep = a.st.k < 2;
    const bool fuse = a.mode == 0 && a.cn_coef != nullptr;
    const double *cnc = fuse ? member_ptr_at(a.cn_coef, ms, mem) : nullptr;
    double cl[2] = {0.0, 0.0}, ck[2] = {0.0, 0.0};
    const int j0 = (int)slab * a.slab_rows;
    const int j1 = (j0 + a.slab_rows < M) ? j0 + a.slab_rows : M;
    // own-column window rows j-2 .. j+2 of both species, and v at row j
    T win[2][5];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int q = 0; q < 5; ++q) win[sp][q] = *byte_at(cf[sp], rowb(j0 - 2 + q) + ex);
    T vj = *byte_at(v, rowb(j0) + ex);
    for (int j = j0; j < j1; ++j) {
        const unsigned rb = rowb(j);
        // this row's loads, then the next row's window entry (one step ahead)
        const T uL = *byte_at(u, rb + ex), uR = *byte_at(u, rb + dxp);
        const T wB = *byte_at(w, rb + ex), wF = *byte_at(w, rb + dzp);
        const T vn = *byte_at(v, rowb(j + 1) + ex);
        T nb[2][8];  // x +1 -1 +2 -2, z +1 -1 +2 -2
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            const unsigned off[8] = {dxp, dxm, dxp2, dxm2, dzp, dzm, dzp2, dzm2};
#pragma unroll
            for (int q = 0; q < 8; ++q) nb[sp][q] = *byte_at(cf[sp], rb + off[q]);
        }
        T hv[2], rv[2];
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            hv[sp] = *byte_at((const T *)hf[sp], rb + ex);  // (read in every mode and stage: unconditional)
            rv[sp] = *byte_at((const T *)rf[sp], rb + ex);
        }
        T nxt[2];
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) nxt[sp] = *byte_at(cf[sp], rowb(j + 3) + ex);
        const T vb = (j > 0) ? vj : T(0), vt = (j + 1 < M) ? vn : T(0);
        const T idn = T(uniform_load(a.tb.idn, j));
        const bool ur = uR >= T(0), ul = uL >= T(0), wf = wF >= T(0), wb = wB >= T(0);
        const bool upt = vt >= T(0), upb = vb >= T(0);
        const bool have_t = upt ? (j > 0) : (j + 2 < M), have_b = upb ? (j > 1) : (j + 1 < M);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            const T *q = nb[sp];
            const T cc = win[sp][2], cyp = win[sp][3], cym = win[sp][1];
            const T cxp = q[0], cxm = q[1], czp = q[4], czm = q[5];
            const T dR = adv_face(cc, cxp, ur ? cxm : q[2], ur, true) - half * (cxp + cc);
            const T dL = adv_face(cxm, cc, ul ? q[3] : cxp, ul, true) - half * (cc + cxm);
            const T dF = adv_face(cc, czp, wf ? czm : q[6], wf, true) - half * (czp + cc);
            const T dB = adv_face(czm, cc, wb ? q[7] : czp, wb, true) - half * (cc + czm);
            // top face (rows j, j + 1) and bottom face (rows j - 1, j)
            const T dT = (j + 1 < M) ? adv_face(cc, cyp, upt ? cym : win[sp][4], upt, have_t) - half * (cyp + cc)
                                     : T(0);
            const T dD = (j > 0) ? adv_face(cym, cc, upb ? win[sp][0] : cyp, upb, have_b) - half * (cc + cym) : T(0);
            const T delta = -((uR * dR - uL * dL) * idx_ + (wF * dF - wB * dB) * idz_ + (vt * dT - vb * dD) * idn);
            if (a.mode == 1) {
                a.dbg[sp][(size_t)j * (size_t)pl + (size_t)e] += (double)delta;
            } else {
                if (keep) *byte_at(hf[sp], rb + ex) = hv[sp] + delta;
                const T rn = rv[sp] + dtg * delta;
                *byte_at(rf[sp], rb + ex) = rn;
                if (fuse) {  // the ions' system (2): g, m at 2 * 3M; its n-products after the slab products
                    const double *cfc = cnc + 2 * 3 * (size_t)M;
                    const double *np = cnc + 9 * (size_t)M + 9 * kCnMaxSlabs + 2 * (size_t)M;
                    const double dr = (double)rn - (double)rv[sp];  // the change the CN solve will see
                    cl[sp] = uniform_load(cfc, j) * dr + uniform_load(cfc + M, j) * cl[sp];
                    ck[sp] += uniform_load(np, j) * cl[sp];
                }
            }
        }
        // advance the window
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
            for (int q = 0; q < 4; ++q) win[sp][q] = win[sp][q + 1];
            win[sp][4] = nxt[sp];
        }
        vj = vn;
    }
    if (fuse) {  // add this pass's slab exits to the explicit kernel's
        const unsigned S = (unsigned)a.slabs;
        double *scr = member_ptr_at(a.cn_scr, ms, mem);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            const int f = 3 + sp;
            scr[((size_t)f * S + slab) * (size_t)pl + (size_t)e] += cl[sp];
            scr[((size_t)(5 + f) * S + slab) * (size_t)pl + (size_t)e] += ck[sp];
        }
    }
}

}  // namespace

hipError_t launch_adv_limit(nspnp_state *s, const Stage &st, double *const out[5]) {
    AdvArgs a{};
    a.d = s->d;
    a.ms = out ? 0 : s->mstride;
    a.tb = s->tb;
    a.st = st;
    a.u = s->f[0]; a.v = s->f[1]; a.w = s->f[2];
    for (int q = 0; q < 2; ++q) {
        a.c[q] = s->f[3 + q];
        a.h[q] = s->h[3 + q];
        a.r[q] = s->r[3 + q];
        a.dbg[q] = out ? out[3 + q] : nullptr;
    }
    a.clock = s->clock;
    a.mode = out ? 1 : 0;
    a.ntiles = (int)((s->d.plane + 255) / 256);
    // the row-slab CN method's slabs (its exits get this pass's share), else
    // 32-row slabs
    const int L = out ? 0 : cn_slab_rows(s);
    a.slab_rows = L ? L : 32;
    a.slabs = (s->d.M + a.slab_rows - 1) / a.slab_rows;
    if (L) {
        a.cn_coef = s->cn_coef + (size_t)st.k * cn_stage_stride(s->d.M);
        a.cn_scr = (double *)s->spec;
    }
    const int nm = out ? 1 : s->nmem;
    const unsigned blocks = (unsigned)((int64_t)a.ntiles * a.slabs * nm);
    if (s->fp64) k_adv_limit<double><<<blocks, 256, 0, s->stream>>>(a);
    else k_adv_limit<float><<<blocks, 256, 0, s->stream>>>(a);
    return hipGetLastError();
}

hipError_t launch_explicit(nspnp_state *s, const Stage &st, bool /*write_r*/) {
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
    a.implicit_xz = s->cfg.implicit_xz;
    hipError_t e = launch_cn_coef(s, st);  // (not part of the explicit kernel's profiled time)
    if (e != hipSuccess) return e;
    ProfScope prof_(s, K_EXPLICIT);
    // row-slab Crank-Nicolson: this kernel marches the method's slabs and
    // runs its first pass
    const int L = cn_slab_rows(s);
    if (L) {
        a.cn_coef = s->cn_coef + (size_t)st.k * cn_stage_stride(s->d.M);
        a.cn_scr = (double *)s->spec;
    }
    const int tb = s->tiles.expl;
    explicit_tiling(s->d, s->fp64, tb, L ? L : s->tiles.slab, a);
    const hipError_t e2 = explicit_launch(s, a, tb, (unsigned)((int64_t)a.chunks * a.slabs * s->nmem));
    if (e2 != hipSuccess || s->cfg.migration_face != 2) return e2;
    return launch_adv_limit(s, st, nullptr);
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
    a.implicit_xz = s->cfg.implicit_xz;
    explicit_tiling(s->d, s->fp64, 256, s->tiles.slab, a);
    const hipError_t e = explicit_launch(s, a, 256, (unsigned)((int64_t)a.chunks * a.slabs));
    if (e != hipSuccess || s->cfg.migration_face != 2) return e;
    return launch_adv_limit(s, a.st, out);
}

static hipError_t launch_cn_lane(nspnp_state *s, const CnArgs &a);

// Periodic-line solves of the five fields along x (dir 0) or z (dir 1).
static hipError_t launch_cyc(nspnp_state *s, const Stage &st, int dir, int out_r) {
    CycArgs c{};
    c.d = s->d;
    c.ms = s->mstride;
    c.st = st;
    for (int q = 0; q < 5; ++q) { c.q[q] = s->f[q]; c.r[q] = s->r[q]; }
    c.cyc = s->cyc;
    c.dir = dir;
    c.out_r = out_r;
    const int N = dir == 0 ? s->d.nx : s->d.nz, L = dir == 0 ? s->d.nz : s->d.nx;
    const dim3 g((unsigned)(s->d.M * ((L + kCycTx - 1) / kCycTx)), 5, (unsigned)s->nmem);
    const size_t lds = (size_t)N * (kCycTx + 1) * sizeof(double);
    if (lds > (size_t)s->lds_max) return hipErrorInvalidValue;
    int rpl = (N + 63) / 64;  // points per lane, rounded up to an instantiated count
    const int have[] = {1, 2, 3, 4, 6, 8, 12, 16};
    int R = 0;
    for (int h : have)
        if (!R && h >= rpl) R = h;
    if (!R) return hipErrorInvalidValue;
    auto go = [&](const void *fn, auto kernel) -> hipError_t {
        const hipError_t e = lds_opt_in(fn, lds, s->lds_max);
        if (e != hipSuccess) return e;
        kernel<<<g, 256, lds, s->stream>>>(c);
        return hipGetLastError();
    };
#define NSPNP_CYC_CASE(RR)                                                                             \
    case RR:                                                                                           \
        return s->fp64 ? go((const void *)k_cyc_scan<double, RR>, k_cyc_scan<double, RR>)              \
                       : go((const void *)k_cyc_scan<float, RR>, k_cyc_scan<float, RR>);
    switch (R) {
        NSPNP_CYC_CASE(1)
        NSPNP_CYC_CASE(2)
        NSPNP_CYC_CASE(3)
        NSPNP_CYC_CASE(4)
        NSPNP_CYC_CASE(6)
        NSPNP_CYC_CASE(8)
        NSPNP_CYC_CASE(12)
        NSPNP_CYC_CASE(16)
        default:
            return hipErrorInvalidValue;
    }
#undef NSPNP_CYC_CASE
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
    a.coef = s->cn_coef;
    a.scr = (double *)s->spec;
    a.slab_rows = cn_slab_rows(s);
    a.slabs = a.slab_rows ? (s->d.M + a.slab_rows - 1) / a.slab_rows : 0;
    {
        const hipError_t e = launch_cn_coef(s, st);
        if (e != hipSuccess) return e;
    }
    if (a.slab_rows) {
        // the first pass (the exits of each slab's local sweeps) ran in the
        // explicit kernel of this substep; scans across the slabs, then both
        // sweeps from the exact slab inputs
        const dim3 g((unsigned)((s->d.plane + 255) / 256), (unsigned)a.slabs, 5u * (unsigned)s->nmem);
        const dim3 g1((unsigned)((s->d.plane + 255) / 256), 1, 5u * (unsigned)s->nmem);
        k_cn_slab_scan<<<g1, 256, 0, s->stream>>>(a);
        if (a.slab_rows == 16) {
            if (s->fp64) k_cn_slab_apply<double, 16><<<g, 256, 0, s->stream>>>(a);
            else k_cn_slab_apply<float, 16><<<g, 256, 0, s->stream>>>(a);
        } else {
            if (s->fp64) k_cn_slab_apply<double, 32><<<g, 256, 0, s->stream>>>(a);
            else k_cn_slab_apply<float, 32><<<g, 256, 0, s->stream>>>(a);
        }
        return hipGetLastError();
    }
    if (!s->cfg.implicit_xz) return launch_cn_lane(s, a);
    // three-direction factorisation: x-lines into r, y (this solve) into r, then z-lines with q += solution
    hipError_t e = launch_cyc(s, st, 0, 1);
    if (e != hipSuccess) return e;
    a.out_r = 1;
    if ((e = launch_cn_lane(s, a)) != hipSuccess) return e;
    return launch_cyc(s, st, 1, 0);
}

// Lane-scan Crank-Nicolson solve of the five fields (tiles of 16 or 32 columns).
static hipError_t launch_cn_lane(nspnp_state *s, const CnArgs &a) {
    const int tb = s->tiles.cn;
    const int tcols = cn_tile_cols(tb);
    const dim3 g((unsigned)((s->d.plane + tcols - 1) / tcols), 5, (unsigned)s->nmem);
    const size_t lds = (size_t)s->d.M * (tcols + 1) * sizeof(double);
    if (lds > (size_t)s->lds_max) return hipErrorInvalidValue;
    const int rpl = (s->d.M + 63) / 64;  // rows per lane (M <= 512: at most 8)
    // tiles above 64 KB of LDS (tall columns) use the device's larger limit
    auto launch = [&](const void *fn, auto kernel) -> hipError_t {
        const hipError_t e = lds_opt_in(fn, lds, s->lds_max);
        if (e != hipSuccess) return e;
        kernel<<<g, tb, lds, s->stream>>>(a);
        return hipGetLastError();
    };
#define NSPNP_CN_CASE(RR)                                                                              \
    case RR:                                                                                           \
        if (tcols == 32)                                                                               \
            return s->fp64 ? launch((const void *)k_cn_scan<double, 32, RR>, k_cn_scan<double, 32, RR>) \
                           : launch((const void *)k_cn_scan<float, 32, RR>, k_cn_scan<float, 32, RR>);  \
        return s->fp64 ? launch((const void *)k_cn_scan<double, 16, RR>, k_cn_scan<double, 16, RR>)    \
                       : launch((const void *)k_cn_scan<float, 16, RR>, k_cn_scan<float, 16, RR>);
    switch (rpl) {
        NSPNP_CN_CASE(1)
        NSPNP_CN_CASE(2)
        NSPNP_CN_CASE(3)
        NSPNP_CN_CASE(4)
        NSPNP_CN_CASE(5)
        NSPNP_CN_CASE(6)
        NSPNP_CN_CASE(7)
        NSPNP_CN_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef NSPNP_CN_CASE
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
    const int tb = s->tiles.corr < 256 ? s->tiles.corr : 256;
    a.tx = s->d.nx < 64 ? s->d.nx : 64;
    if (a.tx > tb) a.tx = tb;
    a.tz = tb / a.tx;
    a.ntx = (s->d.nx + a.tx - 1) / a.tx;
    a.chunks = a.ntx * ((s->d.nz + a.tz - 1) / a.tz);
    a.slab_rows = s->tiles.slab;
    a.slabs = (s->d.M + a.slab_rows - 1) / a.slab_rows;
    const dim3 g((unsigned)((int64_t)a.chunks * a.slabs * s->nmem));
    if (s->cfg.implicit_xz) {
        if (s->fp64) k_correct<double, true><<<g, tb, 0, s->stream>>>(a);
        else k_correct<float, true><<<g, tb, 0, s->stream>>>(a);
    } else {
        if (s->fp64) k_correct<double, false><<<g, tb, 0, s->stream>>>(a);
        else k_correct<float, false><<<g, tb, 0, s->stream>>>(a);
    }
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
