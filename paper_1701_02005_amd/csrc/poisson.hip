// poisson.hip -- elliptic solver of the pressure projection and of the
// potential (Sec. II): Fourier transform in the two periodic directions,
// then one tridiagonal (Thomas) system across the gap per Fourier mode,
// with zero-flux walls (pressure) or zero wall value (potential).
//
// Data flow for one solve, all FP64:
//   real [j][k][i]  --x R2C-->  half spectrum [j][kx][k] (kx < nx/2+1)
//   --z C2C--> [j][kx][kz]  --Thomas in j per (kx,kz)-->  --z C2C^-1-->
//   --x C2R--> real [j][k][i]
// The x transforms stage their output / input through LDS so that the
// spectrum is written and read in runs of consecutive z lines, and every z
// line is one contiguous run of nz values.
// The FFTs are self-sorting (Stockham) in LDS with radix 8, 4, 2 and 3 stages;
// two real x-lines share one complex transform.
#include <algorithm>
#include <mutex>
#include <set>
#include <utility>

#include "internal.h"

namespace nspnp {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ double2 rot(double2 a, bool inv) {
    return inv ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// In-place length-R DFT of v with kernel exp(-+ 2 pi i / R).
template <int R>
__device__ __forceinline__ void dft_small(double2 *v, bool inv);

template <>
__device__ __forceinline__ void dft_small<2>(double2 *v, bool) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft_small<4>(double2 *v, bool inv) {
    const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const double2 s13 = cadd(v[1], v[3]), d13 = rot(csub(v[1], v[3]), inv);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

// radix 8 as two radix-4 DFTs of the even and odd inputs joined by the
// eighth roots of unity: X_k = E_k + w^k O_k, X_{k+4} = E_k - w^k O_k
template <>
__device__ __forceinline__ void dft_small<8>(double2 *v, bool inv) {
    double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<4>(e, inv);
    dft_small<4>(o, inv);
    const double c = 0.70710678118654752440;  // cos(pi / 4)
    const double2 w1 = make_double2(c, inv ? c : -c), w3 = make_double2(-c, inv ? c : -c);
    const double2 t1 = cmul(o[1], w1), t2 = rot(o[2], inv), t3 = cmul(o[3], w3);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], t1);
    v[5] = csub(e[1], t1);
    v[2] = cadd(e[2], t2);
    v[6] = csub(e[2], t2);
    v[3] = cadd(e[3], t3);
    v[7] = csub(e[3], t3);
}

template <>
__device__ __forceinline__ void dft_small<3>(double2 *v, bool inv) {
    const double s3 = 0.86602540378443864676;  // sin(2 pi / 3)
    const double2 t1 = cadd(v[1], v[2]);
    const double2 t2 = csub(v[1], v[2]);
    const double2 m = make_double2(v[0].x - 0.5 * t1.x, v[0].y - 0.5 * t1.y);
    // -i s3 t2 (forward) / +i s3 t2 (inverse)
    const double2 r = rot(make_double2(s3 * t2.x, s3 * t2.y), inv);
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

// q = e / d and r = e % d for 0 <= e, d < 2^22 from a float reciprocal
// rd = 1/d: the product is within half a unit of the true quotient, so one
// correction step makes the result exact (integer division has no hardware
// instruction on the GPU).
__device__ __forceinline__ void divmod(int e, int d, float rd, int &q, int &r) {
    q = (int)((float)e * rd);
    r = e - q * d;
    if (r < 0) {
        --q;
        r += d;
    } else if (r >= d) {
        ++q;
        r -= d;
    }
}

// Quotient and remainder by a block-uniform divisor: shifts and a mask when
// it is a power of two, else the float-reciprocal divmod (same range).
struct Div {
    int d, sh;
    float rd;
    __device__ explicit Div(int dd) : d(dd), sh(((dd & (dd - 1)) == 0) ? __builtin_ctz((unsigned)dd) : -1),
                                      rd(1.0f / (float)dd) {}
    __device__ __forceinline__ void split(int e, int &q, int &r) const {
        if (sh >= 0) {
            q = e >> sh;
            r = e & (d - 1);
        } else {
            divmod(e, d, rd, q, r);
        }
    }
};

// One radix-R Stockham pass over nl lines of length N in LDS; tw holds this
// pass's twiddles exp(-2 pi i r k ts / N) as [r - 1][k] (k < Ns), staged in
// LDS, so the lanes of a wave (consecutive k) read consecutive entries.
template <int R>
__device__ __forceinline__ void stage_pass(const double2 *__restrict__ src, double2 *__restrict__ dst, int N,
                                           int nl, int Ns, const double2 *__restrict__ tw, bool inv, int tid,
                                           int nth) {
    const int NR = N / R;
    const float rNR = 1.0f / (float)NR, rNs = 1.0f / (float)Ns;
    // powers of two (every pass of a 2^a line): shifts and masks instead of
    // the float-reciprocal divmod (block-uniform choice)
    const bool p2 = ((NR & (NR - 1)) | (Ns & (Ns - 1))) == 0;
    const int lNR = __builtin_ctz((unsigned)NR), lNs = __builtin_ctz((unsigned)Ns);
    for (int e = tid; e < nl * NR; e += nth) {
        int line, jb, blk, k;
        if (p2) {
            line = e >> lNR;
            jb = e & (NR - 1);
            blk = jb >> lNs;
            k = jb & (Ns - 1);
        } else {
            divmod(e, NR, rNR, line, jb);
            divmod(jb, Ns, rNs, blk, k);
        }
        const double2 *in = src + line * N;
        double2 *out = dst + line * N;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[jb + r * NR];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            double2 w = tw[(r - 1) * Ns + k];
            if (inv) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
        dft_small<R>(v, inv);
        const int base = blk * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out[base + r * Ns] = v[r];
    }
}

// nl lines of length N in b0; returns the buffer (0 or 1) holding the result.
// kR8: the plan may hold radix-8 passes (instantiated only for such plans:
// the radix-8 pass's registers would otherwise bound every transform's
// occupancy).
template <bool kR8>
__device__ int lds_fft(double2 *b0, double2 *b1, int N, int nl, const FftPlan &pl, const double2 *tw, bool inv) {
    double2 *src = b0, *dst = b1;
    int which = 0;
    int Ns = 1, off = 0;  // off: this pass's twiddles in the staged table
    for (int s = 0; s < pl.nstages; ++s) {
        const int R = pl.radix[s];
        const double2 *twp = tw + off;
        if (kR8 && R == 8) stage_pass<kR8 ? 8 : 4>(src, dst, N, nl, Ns, twp, inv, threadIdx.x, blockDim.x);
        else if (R == 4) stage_pass<4>(src, dst, N, nl, Ns, twp, inv, threadIdx.x, blockDim.x);
        else if (R == 2) stage_pass<2>(src, dst, N, nl, Ns, twp, inv, threadIdx.x, blockDim.x);
        else stage_pass<3>(src, dst, N, nl, Ns, twp, inv, threadIdx.x, blockDim.x);
        off += Ns * (R - 1);
        __syncthreads();
        double2 *t = src;
        src = dst;
        dst = t;
        which ^= 1;
        Ns *= R;
    }
    return which;
}

// The twiddle table to LDS (before the caller's first barrier).  The table
// is laid out in pass order at init (pass after pass, [r - 1][k]).
__device__ __forceinline__ void stage_twiddles(double2 *s_tw, const double2 *tw, int N) {
    for (int e = threadIdx.x; e < N; e += blockDim.x) s_tw[e] = tw[e];
}

// ---- x direction: real lines <-> half spectra, two lines per transform ----
// The right-hand side of each line is produced while it is loaded: a plain
// FP64 array, the divergence of the staggered velocity (pressure), or the
// charge -(c+ - c-)/(2 lam^2) (potential).
// The line pairs of an x-transform block into LDS, as (line 2p, line 2p+1)
// complex values, for one source type S (block-uniform).  Each batch of kXB
// elements per thread issues all of its loads before any value is formed
// (elements past the block or lines past the grid read element 0 of line 0
// and are dropped), so a thread waits for memory once per batch.  Offsets
// within one field fit in 32 bits.
constexpr int kXB = 2;

template <typename T, int S>
__device__ __forceinline__ void r2c_stage(const PoissonSrc &src, const Dims &d, const Tables &tb, double ch,
                                          double sc, double idx, double idz, int64_t pair0, int ppb, double2 *buf) {
    const int nx = d.nx, nz = d.nz, M = d.M, n = ppb * nx, bd = (int)blockDim.x;
    const int64_t nlines = (int64_t)M * nz;
    const unsigned upl = (unsigned)d.plane;
    // (line = j nz + k < 512 * 1024 and e < ppb nx: the float-reciprocal
    // divmod is exact for both)
    const Div dnx(nx), dnz(nz);
    for (int e0 = threadIdx.x; e0 < n; e0 += kXB * bd) {
        unsigned q[kXB][2];
        bool ok[kXB][2];
        int jr[kXB][2], kr[kXB][2], ir[kXB];
#pragma unroll
        for (int u = 0; u < kXB; ++u) {
            const int e = e0 + u * bd;
            int p, i;
            dnx.split(e < n ? e : 0, p, i);
            ir[u] = i;
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const int64_t line = 2 * (pair0 + p) + l;
                ok[u][l] = e < n && line < nlines;
                const int li = ok[u][l] ? (int)line : 0;
                int j, k;
                dnz.split(li, j, k);
                q[u][l] = (unsigned)li * (unsigned)nx + (unsigned)i;
                jr[u][l] = j;
                kr[u][l] = k;
            }
        }
        double val[kXB][2];
        if constexpr (S == SRC_REAL) {
            const double *a = (const double *)src.a;
            double x[kXB][2];
#pragma unroll
            for (int u = 0; u < kXB; ++u)
#pragma unroll
                for (int l = 0; l < 2; ++l) x[u][l] = a[q[u][l]];
#pragma unroll
            for (int u = 0; u < kXB; ++u)
#pragma unroll
                for (int l = 0; l < 2; ++l) val[u][l] = x[u][l];
        } else if constexpr (S == SRC_CHARGE) {
            const T *cp = (const T *)src.a, *cm = (const T *)src.b;
            T xp[kXB][2], xm[kXB][2];
#pragma unroll
            for (int u = 0; u < kXB; ++u)
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    xp[u][l] = ld_once(cp + q[u][l]);
                    xm[u][l] = ld_once(cm + q[u][l]);
                }
#pragma unroll
            for (int u = 0; u < kXB; ++u)
#pragma unroll
                for (int l = 0; l < 2; ++l) val[u][l] = ch * ((double)xp[u][l] - (double)xm[u][l]);
            // wall values g of phi (inhomogeneous Dirichlet data): L_y at the
            // first / last row carries + g / (dn dc), moved to the right side
            if (src.wall) {
#pragma unroll
                for (int u = 0; u < kXB; ++u)
#pragma unroll
                    for (int l = 0; l < 2; ++l) {
                        const int j = jr[u][l];
                        if (j == 0 || j == M - 1) {
                            const unsigned in_plane = q[u][l] - (unsigned)j * upl;
                            const double g = src.wall[(j == 0 ? 0u : upl) + in_plane];
                            val[u][l] -= (j == 0 ? tb.lyc_lo[0] : tb.lyc_up[M - 1]) * g;
                        }
                    }
            }
        } else {
            // divergence: (u_{i+1} - u_i)/dx + (v_{j+1} - v_j)/dy_j + (w_{k+1} - w_k)/dz, times sc
            const T *uu = (const T *)src.a, *vv = (const T *)src.b, *ww = (const T *)src.c;
            T ux[kXB][2], u0[kXB][2], vt[kXB][2], vb[kXB][2], wz[kXB][2], w0[kXB][2];
            double idn[kXB][2];
#pragma unroll
            for (int u = 0; u < kXB; ++u)
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    const unsigned qq = q[u][l];
                    const int j = jr[u][l];
                    const unsigned i = (unsigned)ir[u], k = (unsigned)kr[u][l];
                    const unsigned xp = qq - i + ((i + 1 == (unsigned)nx) ? 0u : i + 1);
                    const unsigned zp = qq + ((k + 1 == (unsigned)nz) ? 0u : k + 1) * (unsigned)nx - k * (unsigned)nx;
                    ux[u][l] = uu[xp];
                    u0[u][l] = uu[qq];
                    vt[u][l] = vv[(j + 1 < M) ? qq + upl : qq];
                    vb[u][l] = vv[qq];
                    wz[u][l] = ww[zp];
                    w0[u][l] = ww[qq];
                    idn[u][l] = tb.idn[j];
                }
#pragma unroll
            for (int u = 0; u < kXB; ++u)
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    const int j = jr[u][l];
                    const double t = (j + 1 < M) ? (double)vt[u][l] : 0.0;
                    const double b = (j > 0) ? (double)vb[u][l] : 0.0;
                    const double div = ((double)ux[u][l] - (double)u0[u][l]) * idx + (t - b) * idn[u][l] +
                                       ((double)wz[u][l] - (double)w0[u][l]) * idz;
                    val[u][l] = div * sc;
                }
        }
#pragma unroll
        for (int u = 0; u < kXB; ++u) {
            const int e = e0 + u * bd;
            if (e < n) buf[e] = make_double2(ok[u][0] ? val[u][0] : 0.0, ok[u][1] ? val[u][1] : 0.0);
        }
    }
}

// Slots of each of the two FFT buffers of an x-transform block; the [kx][line]
// staging of the transposed spectrum stores / loads fits one of them.
__host__ __device__ inline int x_buffer_slots(int nx, int ppb) { return ppb * (nx + 2); }

template <typename T, bool kR8>
__global__ void __launch_bounds__(256) k_fft_x_r2c(Dims d, Tables tb, FftPlan pl, PoissonBatch b,
                                                   const double *clock, double2 *spec, int64_t nspec, int ppb) {
    extern __shared__ double2 sm[];
    const int prob = blockIdx.y;
    PoissonSrc src = b.src[prob];
    src.a = member_ptr(src.a, b.ms);
    src.b = member_ptr(src.b, b.ms);
    src.c = member_ptr(src.c, b.ms);
    if (src.wall) src.wall = member_ptr(src.wall, b.ms);
    clock = member_ptr(clock, b.ms);
    const double ch = member_ptr(b.phys, b.ms)->ch;
    double2 *out = member_ptr(spec, b.ms) + prob * nspec;
    const int nx = d.nx, nxh = d.nxh;
    const int64_t nlines = (int64_t)d.M * d.nz;
    const int bs = x_buffer_slots(nx, ppb);
    double2 *bf[2] = {sm, sm + bs};
    double2 *s_tw = sm + 2 * bs;
    stage_twiddles(s_tw, tb.twx, nx);
    const double sc = (src.type == SRC_DIV) ? ((src.alp > 0.0) ? 1.0 / (src.alp * clock[1]) : src.fixed) : 0.0;
    const double idx = 1.0 / d.dx, idz = 1.0 / d.dz;
    // XCD-aware block order: the pairs whose spectra share 128-byte lines of a
    // [j][kx][kz] row run on one XCD, so their partial-line stores merge in
    // that XCD's L2 before they reach memory
    const int64_t pair0 = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * ppb;
    if (src.type == SRC_DIV) r2c_stage<T, SRC_DIV>(src, d, tb, ch, sc, idx, idz, pair0, ppb, bf[0]);
    else if (src.type == SRC_CHARGE) r2c_stage<T, SRC_CHARGE>(src, d, tb, ch, sc, idx, idz, pair0, ppb, bf[0]);
    else r2c_stage<T, SRC_REAL>(src, d, tb, ch, sc, idx, idz, pair0, ppb, bf[0]);
    __syncthreads();
    const int w = lds_fft<kR8>(bf[0], bf[1], nx, ppb, pl, s_tw, false);
    // (offsets from the LDS base rather than bf[w]: a pointer picked from an
    // array at run time loses its address space and becomes a flat access,
    // which would also wait for every vector load in flight)
    const double2 *z = sm + w * bs;
    double2 *o = sm + (1 - w) * bs;  // [kk][line] staging for the transposed store
    const int nl2 = 2 * ppb;
    const Div dnxh(nxh), dnl2(nl2), dnz(d.nz);
    for (int e = threadIdx.x; e < ppb * nxh; e += blockDim.x) {
        int p, kk;
        dnxh.split(e, p, kk);
        const double2 zk = z[p * nx + kk];
        const double2 zc = z[p * nx + (kk == 0 ? 0 : nx - kk)];
        // A = (Z_k + conj(Z_{N-k}))/2, B = (Z_k - conj(Z_{N-k}))/(2i)
        o[kk * nl2 + 2 * p] = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y - zc.y));
        o[kk * nl2 + 2 * p + 1] = make_double2(0.5 * (zk.y + zc.y), -0.5 * (zk.x - zc.x));
    }
    __syncthreads();
    // spectrum layout [j][kx][kz]: consecutive lines (k) of one kx are contiguous
    for (int e = threadIdx.x; e < nl2 * nxh; e += blockDim.x) {
        int kk, l;
        dnl2.split(e, kk, l);
        const int64_t line = 2 * pair0 + l;
        if (line < nlines) {
            int j, k;
            dnz.split((int)line, j, k);
            out[((int64_t)j * nxh + kk) * d.nz + k] = o[e];
        }
    }
}

// Persistent blocks over tiles of ppb line pairs: the next tile's spectrum
// values (transposed load, whole runs of consecutive lines per kx) are loaded
// into registers while the current tile is transformed in LDS.
constexpr int kCPer = 12;  // prefetched values per thread: 2 ppb (nx/2+1) <= kCPer * 256

template <typename T, bool kR8>
__global__ void __launch_bounds__(256) k_fft_x_c2r(Dims d, Tables tb, FftPlan pl, PoissonBatch b,
                                                   const double2 *spec, int64_t nspec, int ppb) {
    extern __shared__ double2 sm[];
    const int prob = blockIdx.y;
    const double2 *in = member_ptr(spec, b.ms) + prob * nspec;
    const int nx = d.nx, nxh = d.nxh, nz = d.nz;
    const int64_t nlines = (int64_t)d.M * d.nz;
    const int ntiles = (int)(((nlines + 1) / 2 + ppb - 1) / ppb);
    const int bs = x_buffer_slots(nx, ppb);
    double2 *bf[2] = {sm, sm + bs};
    double2 *s_tw = sm + 2 * bs;
    stage_twiddles(s_tw, tb.twx, nx);
    const int nl2 = 2 * ppb, nst = nl2 * nxh;
    const Div dnl2(nl2), dnz(nz), dnx(nx);
    double2 *o = bf[1];  // [kk][line] staging of the transposed load
    const bool as_state = b.out_state[prob] != 0;
    double *o64 = (double *)member_ptr(b.out[prob], b.ms);
    T *ot = (T *)member_ptr(b.out[prob], b.ms);
    double2 nxt[kCPer];
    auto load = [&](int t) {
        const int64_t l0 = 2 * (int64_t)t * ppb;
#pragma unroll
        for (int q = 0; q < kCPer; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            double2 v = make_double2(0.0, 0.0);
            if (e < nst) {
                int kk, l, j, k;
                dnl2.split(e, kk, l);
                const int64_t line = l0 + l;
                if (line < nlines) {
                    dnz.split((int)line, j, k);
                    v = ld_once(in + ((int64_t)j * nxh + kk) * nz + k);
                }
            }
            nxt[q] = v;
        }
    };
    int t = blockIdx.x;
    if (t < ntiles) load(t);
    for (; t < ntiles; t += gridDim.x) {
        const int64_t pair0 = (int64_t)t * ppb;
#pragma unroll
        for (int q = 0; q < kCPer; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            if (e < nst) o[e] = nxt[q];
        }
        __syncthreads();
        if (t + (int)gridDim.x < ntiles) load(t + gridDim.x);  // lands during the passes
        for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
            int p, kk;
            dnx.split(e, p, kk);
            const bool lower = kk < nxh;
            const int src = lower ? kk : nx - kk;
            double2 A = o[src * nl2 + 2 * p];
            double2 B = o[src * nl2 + 2 * p + 1];
            if (!lower) {  // Hermitian continuation of a real line's spectrum
                A.y = -A.y;
                B.y = -B.y;
            }
            bf[0][e] = make_double2(A.x - B.y, A.y + B.x);  // Z = A + i B
        }
        __syncthreads();
        const double2 *z = sm + lds_fft<kR8>(bf[0], bf[1], nx, ppb, pl, s_tw, true) * bs;  // LDS base offset: no flat access
        for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
            int p, i;
            dnx.split(e, p, i);
            const int64_t la = 2 * (pair0 + p), lb = la + 1;
            const double2 v = z[e];
            if (as_state) {
                if (la < nlines) st_once(ot + la * nx + i, (T)v.x);
                if (lb < nlines) st_once(ot + lb * nx + i, (T)v.y);
            } else {
                if (la < nlines) st_once(o64 + la * nx + i, v.x);
                if (lb < nlines) st_once(o64 + lb * nx + i, v.y);
            }
        }
        __syncthreads();  // o and the result buffer are reused by the next tile
    }
}

// ---- z direction: contiguous complex lines, tiles of tk lines ----
// Persistent blocks: each block loops over tiles (j, kx0..kx0+tk-1) of its
// problem and member; the next tile's values are loaded into registers while
// the current tile is transformed in LDS, so the HBM latency overlaps the
// FFT passes.  kPer values per thread cover tk * nz <= kPer * 256 points.
constexpr int kZPer = 8;

template <bool kR8>
__global__ void __launch_bounds__(256) k_fft_z(Dims d, FftPlan pl, const double2 *tw, double2 *spec, int64_t nspec,
                                               int tk, int inverse, size_t ms) {
    extern __shared__ double2 sm[];
    double2 *data = member_ptr(spec, ms) + blockIdx.y * nspec;
    const int nz = d.nz, nxh = d.nxh;
    const int tiles_x = (nxh + tk - 1) / tk;
    const int ntiles = d.M * tiles_x;
    const int pts = tk * nz;
    double2 *bf[2] = {sm, sm + tk * nz};
    double2 *s_tw = sm + 2 * tk * nz;
    stage_twiddles(s_tw, tw, nz);
    double2 nxt[kZPer];
    auto tile_base = [&](int t, int &nt) -> double2 * {
        const int j = t / tiles_x;
        const int kx0 = (t - j * tiles_x) * tk;
        nt = (nxh - kx0 < tk) ? nxh - kx0 : tk;  // lines in this tile
        // lines (j, kx) are contiguous runs of nz values: the tile is one block of memory
        return data + ((int64_t)j * nxh + kx0) * nz;
    };
    auto load = [&](int t) {
        int nt;
        const double2 *base = tile_base(t, nt);
#pragma unroll
        for (int q = 0; q < kZPer; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            nxt[q] = (e < nt * nz) ? base[e] : make_double2(0.0, 0.0);
        }
    };
    int t = blockIdx.x;
    if (t < ntiles) load(t);
    for (; t < ntiles; t += gridDim.x) {
        int nt;
        double2 *base = tile_base(t, nt);
#pragma unroll
        for (int q = 0; q < kZPer; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            if (e < pts) bf[0][e] = nxt[q];
        }
        __syncthreads();
        if (t + (int)gridDim.x < ntiles) load(t + gridDim.x);  // lands during the passes
        const double2 *z = sm + lds_fft<kR8>(bf[0], bf[1], nz, tk, pl, s_tw, inverse != 0) * (tk * nz);  // no flat access
        for (int e = threadIdx.x; e < nt * nz; e += blockDim.x) base[e] = z[e];
        __syncthreads();  // bf[0] and the result buffer are reused by the next tile
    }
}

// ---- y direction: one tridiagonal solve per (kx, kz) mode ----
// (lo_j psi_{j-1} + (di_j - kx^2 - kz^2) psi_j + up_j psi_{j+1}) = rhs_j / (nx nz)
// kind 0: zero-flux walls, mode (0,0) pinned at row 0 then shifted to zero
// volume mean; kind 1: zero wall value at the half-cell distance.
//
// The matrices do not change in time, so the Thomas pivots of every mode are
// computed once (k_thomas_factors) and stored as fac[kind][mode][row] =
// (g, c') with g = 1/den.  Each solve is then two linear recurrences
//   d'_j = g_j r_j + m_j d'_{j-1}  (m_j = -lo_j g_j),   x_j = d'_j - c'_j x_{j+1}.

// One thread per (kind, mode): the forward pass of Thomas' algorithm on the
// matrix only.
// Also c' alone in row order, cpv[kind][row][mode], for the fused y-march
// (cpv_all may be NULL).
__global__ void __launch_bounds__(256) k_thomas_factors(Dims d, Tables tb, double2 *fac_all, double *cpv_all,
                                                        size_t ms) {
    const int kind = blockIdx.y;
    const int64_t nmodes = (int64_t)d.nxh * d.nz;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmodes) return;
    const int M = d.M;
    double2 *fac = member_ptr(fac_all, ms) + ((int64_t)kind * nmodes + m) * M;
    double *cpv = cpv_all ? member_ptr(cpv_all, ms) + (int64_t)kind * M * nmodes + m : nullptr;
    const int kx = (int)(m / d.nz), kz = (int)(m % d.nz);  // spectrum layout [j][kx][kz]
    const double k2 = tb.kx2[kx] + tb.kz2[kz];
    const bool pin = (kind == 0 && m == 0);
    double cprev = 0.0;
    for (int j = 0; j < M; ++j) {
        const double aa = tb.lyc_lo[j], cc = tb.lyc_up[j];
        const double lo = (j > 0) ? aa : 0.0;
        double up = (j < M - 1) ? cc : 0.0;
        double di = -(lo + up);
        if (kind == 1) {
            if (j == 0) di -= aa;
            if (j == M - 1) di -= cc;
        }
        double B = di - k2;
        if (pin && j == 0) {
            B = 1.0;
            up = 0.0;
        }
        const double den = B - lo * cprev;
        const double cj = up / den;
        fac[j] = make_double2(1.0 / den, cj);
        if (cpv) cpv[(int64_t)j * nmodes] = cj;
        cprev = cj;
    }
}

// Solve of one tile of tm consecutive modes of one problem: the tile's rows
// are staged in LDS with coalesced loads; each wave then solves one mode at
// a time with its rows split into 64 contiguous lane segments of R rows (the
// mode's pivots are one contiguous read per wave).  Each recurrence is a
// local sweep per lane, a 6-step scan of affine maps across the wave and a
// second sweep from the correct incoming value.  The tile is written back
// with coalesced stores.
constexpr int kThBatch = 12;  // a whole 16-mode tile of 192 rows in one batch

template <int R>
__global__ void __launch_bounds__(256) k_thomas_tile(Dims d, Tables tb, PoissonBatch b, double2 *spec_all,
                                                     const double2 *fac_all, int64_t nspec, int tm) {
    extern __shared__ double2 s_x[];
    const uint3 blk = xcd_block3();
    const int prob = (int)blk.y;
    const int kind = b.kind[prob];
    const int64_t nmodes = (int64_t)d.nxh * d.nz;
    const int M = d.M;
    double2 *spec = member_ptr_at(spec_all, b.ms, blk.z) + prob * nspec;
    const double2 *fac = member_ptr_at(fac_all, b.ms, blk.z) + (int64_t)kind * nmodes * M;
    const int64_t m0 = (int64_t)blk.x * tm;
    const int ncol = (int)((nmodes - m0) < tm ? (nmodes - m0) : tm);
    const int LD = tm + 1;
    // Staging in batches of kThBatch unconditional loads per thread (lanes
    // past the tile read its first mode and discard it): one wait per batch.
    // Offsets within one spectrum: rows * modes < 2^32 for every supported grid.
    const unsigned unm = (unsigned)nmodes, um0 = (unsigned)m0;
    const int ntile = M * tm, bd = (int)blockDim.x;
    const Div dtm(tm);  // (e < 2^22: the float-reciprocal divmod is exact)
    for (int e0 = threadIdx.x; e0 < ntile; e0 += kThBatch * bd) {
        double2 v[kThBatch];
#pragma unroll
        for (int u = 0; u < kThBatch; ++u) {
            const int e = e0 + u * bd;
            int j, c;
            dtm.split(e, j, c);
            v[u] = spec[(e < ntile && c < ncol) ? (unsigned)j * unm + um0 + (unsigned)c : um0];
        }
#pragma unroll
        for (int u = 0; u < kThBatch; ++u) {
            const int e = e0 + u * bd;
            int j, c;
            dtm.split(e, j, c);
            if (e < ntile) s_x[j * LD + c] = (c < ncol) ? v[u] : make_double2(0.0, 0.0);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int js = lane * R;
    const double scale = 1.0 / ((double)d.nx * (double)d.nz);
    double lo[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int j = js + t;
        lo[t] = (j > 0 && j < M) ? tb.lyc_lo[j] : 0.0;
    }
    // pivots (1/den, c') of a column: unconditional loads (padding rows read
    // the last row and ignore it); the next column's are fetched while the
    // current one is solved, unconditionally (the wave's last column re-reads
    // its own) so that the wait for the current pivots stays partial
    double2 fnext[R];
    auto load_pivots = [&](int c, double2 *f) {
        const double2 *fm = fac + (m0 + c) * M;
#pragma unroll
        for (int t = 0; t < R; ++t) f[t] = fm[(js + t < M) ? js + t : M - 1];
    };
    if (wave < ncol) load_pivots(wave, fnext);
    for (int c = wave; c < ncol; c += nwave) {
        const int64_t m = m0 + c;
        const bool pin = (kind == 0 && m == 0);
        double2 fcur[R];
#pragma unroll
        for (int t = 0; t < R; ++t) fcur[t] = fnext[t];
        load_pivots(c + nwave < ncol ? c + nwave : c, fnext);
        double g[R], mm[R], nn[R];
        double2 x[R];
        double Qs = 1.0, Ss = 1.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int j = js + t;
            if (j < M) {
                const double2 f = fcur[t];
                g[t] = f.x;
                mm[t] = -lo[t] * f.x;
                nn[t] = -f.y;
                const double2 r = s_x[j * LD + c];
                x[t] = (pin && j == 0) ? make_double2(0.0, 0.0) : make_double2(r.x * scale, r.y * scale);
            } else {  // padding rows pass values through
                g[t] = 0.0;
                mm[t] = 1.0;
                nn[t] = 1.0;
                x[t] = make_double2(0.0, 0.0);
            }
            Qs *= mm[t];
            Ss *= nn[t];
        }
        // multipliers of the scans of x -> T + Q x (forward, from lane 0 up)
        // and x -> U + S x (backward, from lane 63 down)
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
        // forward sweep
        double tx = 0.0, ty = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            tx = g[t] * x[t].x + mm[t] * tx;
            ty = g[t] * x[t].y + mm[t] * ty;
        }
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            const double px = __shfl_up(tx, 1 << st, 64), py = __shfl_up(ty, 1 << st, 64);
            if (lane >= (1 << st)) {
                tx += qm[st] * px;
                ty += qm[st] * py;
            }
        }
        double dx_ = __shfl_up(tx, 1, 64), dy_ = __shfl_up(ty, 1, 64);
        if (lane == 0) dx_ = dy_ = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            dx_ = g[t] * x[t].x + mm[t] * dx_;
            dy_ = g[t] * x[t].y + mm[t] * dy_;
            x[t] = make_double2(dx_, dy_);
        }
        // backward sweep
        double ux = 0.0, uy = 0.0;
#pragma unroll
        for (int t = R - 1; t >= 0; --t) {
            const bool in = g[t] != 0.0;
            ux = (in ? x[t].x : 0.0) + nn[t] * ux;
            uy = (in ? x[t].y : 0.0) + nn[t] * uy;
        }
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            const double px = __shfl_down(ux, 1 << st, 64), py = __shfl_down(uy, 1 << st, 64);
            if (lane + (1 << st) < 64) {
                ux += sm[st] * px;
                uy += sm[st] * py;
            }
        }
        double xx = __shfl_down(ux, 1, 64), xy = __shfl_down(uy, 1, 64);
        if (lane == 63) xx = xy = 0.0;
#pragma unroll
        for (int t = R - 1; t >= 0; --t) {
            const bool in = g[t] != 0.0;
            xx = (in ? x[t].x : 0.0) + nn[t] * xx;
            xy = (in ? x[t].y : 0.0) + nn[t] * xy;
            x[t] = make_double2(xx, xy);
        }
        if (pin) {  // zero volume mean of the pressure-type solution
            double sx = 0.0, sy = 0.0, vol = 0.0;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int j = js + t;
                if (j < M) {
                    const double h = tb.dn[j];
                    sx += x[t].x * h;
                    sy += x[t].y * h;
                    vol += h;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                sx += __shfl_xor(sx, o, 64);
                sy += __shfl_xor(sy, o, 64);
                vol += __shfl_xor(vol, o, 64);
            }
            const double mx = sx / vol, my = sy / vol;
#pragma unroll
            for (int t = 0; t < R; ++t) x[t] = make_double2(x[t].x - mx, x[t].y - my);
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int j = js + t;
            if (j < M) s_x[j * LD + c] = x[t];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ntile; e += bd) {
        int j, c;
        dtm.split(e, j, c);
        if (c < ncol) spec[(unsigned)j * unm + um0 + (unsigned)c] = s_x[j * LD + c];
    }
}

// ---- the elliptic chain fused along y (mode-solve method 0) ----
// One block per tile of tk x-modes (every kz) and problem.  The forward
// kernel marches the rows upward: the row's z transform in LDS, then one
// forward-elimination step of every (kx, kz) mode's tridiagonal system with
// the pivot formed on the way, den_j = B_j - lo_j c'_{j-1}, c'_j = up_j / den_j
// (the arithmetic of k_thomas_factors), and d'_j = (r_j - lo_j d'_{j-1}) /
// den_j stored in place.  The backward kernel marches down: x_j = d'_j -
// c'_j x_{j+1} with c' from the precomputed row-order table, then the row's
// inverse z transform.  Each solve thus reads and writes the spectrum twice
// (plus c'), against three times for separate z transforms and mode solves.
// The pressure problem's (0, 0) mode is pinned at row 0; its volume mean
// sum_j w_j x_j / sum_j w_j (w = cell height) is known after the forward
// march as sum_k a_k d'_k with a_k = w_k - c'_{k-1} a_{k-1} (a_0 = w_0),
// and the backward march removes it.
constexpr int kZtQ = 4;  // modes per thread (tk nz <= 1024)

// one row's (j) wall-normal operator terms of mode kind, as k_thomas_factors
__device__ __forceinline__ void ythomas_row(const Tables &tb, int kind, int M, int j, double &lo, double &up,
                                            double &di) {
    const double aa = uniform_load(tb.lyc_lo, j), cc = uniform_load(tb.lyc_up, j);
    lo = (j > 0) ? aa : 0.0;
    up = (j < M - 1) ? cc : 0.0;
    di = -(lo + up);
    if (kind == 1) {
        if (j == 0) di -= aa;
        if (j == M - 1) di -= cc;
    }
}

template <bool kR8>
__global__ void __launch_bounds__(256) k_zthomas_fwd(Dims d, Tables tb, FftPlan pl, PoissonBatch b,
                                                     double2 *spec_all, double2 *mu_all, int64_t nspec, int tk) {
    extern __shared__ double2 sm[];
    const int prob = blockIdx.y, kind = b.kind[prob];
    const int nz = d.nz, nxh = d.nxh, M = d.M;
    double2 *spec = member_ptr(spec_all, b.ms) + prob * nspec;
    const int kx0 = (int)blockIdx.x * tk;
    const int nt = (nxh - kx0 < tk) ? nxh - kx0 : tk;
    const int pts = nt * nz;
    const int bs = tk * nz;
    double2 *s_tw = sm + 2 * bs;
    stage_twiddles(s_tw, tb.twz, nz);
    const double scale = 1.0 / ((double)d.nx * (double)d.nz);
    double k2[kZtQ], cprev[kZtQ];
    double2 dprev[kZtQ];
    double nre[kZtQ], nim[kZtQ];  // the next row (two arrays of doubles stay in registers)
#pragma unroll
    for (int q = 0; q < kZtQ; ++q) {
        const int e = (int)threadIdx.x + q * (int)blockDim.x;
        const int ee = e < pts ? e : 0;
        k2[q] = tb.kx2[kx0 + ee / nz] + tb.kz2[ee % nz];
        cprev[q] = 0.0;
        dprev[q] = make_double2(0.0, 0.0);
    }
    const bool pin = (kind == 0 && kx0 == 0 && threadIdx.x == 0);  // mode (0, 0) of the pressure problem
    double a = 0.0, vol = 0.0, sx = 0.0, sy = 0.0;
    auto row_ptr = [&](int j) { return spec + ((int64_t)j * nxh + kx0) * nz; };
    {
        const double2 *r0 = row_ptr(0);
#pragma unroll
        for (int q = 0; q < kZtQ; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            const double2 v = r0[e < pts ? e : 0];
            nre[q] = v.x;
            nim[q] = v.y;
        }
    }
    for (int j = 0; j < M; ++j) {
#pragma unroll
        for (int q = 0; q < kZtQ; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            if (e < pts) sm[e] = make_double2(nre[q], nim[q]);
        }
        __syncthreads();
        if (j + 1 < M) {  // the next row's loads land during this row's passes
            const double2 *rn = row_ptr(j + 1);
#pragma unroll
            for (int q = 0; q < kZtQ; ++q) {
                const int e = (int)threadIdx.x + q * (int)blockDim.x;
                const double2 v = rn[e < pts ? e : 0];
                nre[q] = v.x;
                nim[q] = v.y;
            }
        }
        const int w = lds_fft<kR8>(sm, sm + bs, nz, nt, pl, s_tw, false);
        const double2 *z = sm + w * bs;  // (offset from the LDS base: no flat access)
        double lo, up0, di;
        ythomas_row(tb, kind, M, j, lo, up0, di);
        const double wj = tb.dn[j];
        double2 *out = row_ptr(j);
#pragma unroll
        for (int q = 0; q < kZtQ; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            if (e < pts) {
                double2 r = z[e];
                r.x *= scale;
                r.y *= scale;
                double B = di - k2[q], up = up0;
                if (pin && q == 0 && j == 0) {
                    B = 1.0;
                    up = 0.0;
                    r = make_double2(0.0, 0.0);
                }
                const double den = B - lo * cprev[q];
                const double g = 1.0 / den, mm = -lo * g;
                const double2 dn_ = make_double2(g * r.x + mm * dprev[q].x, g * r.y + mm * dprev[q].y);
                if (pin && q == 0) {  // volume-mean weights of the pinned mode
                    a = (j == 0) ? wj : wj - cprev[q] * a;
                    sx += a * dn_.x;
                    sy += a * dn_.y;
                    vol += wj;
                }
                cprev[q] = up / den;
                dprev[q] = dn_;
                out[e] = dn_;
            }
        }
        __syncthreads();  // the staging buffer is refilled next row
    }
    if (pin) member_ptr(mu_all, b.ms)[prob] = make_double2(sx / vol, sy / vol);
}

template <bool kR8>
__global__ void __launch_bounds__(256) k_zthomas_bwd(Dims d, Tables tb, FftPlan pl, PoissonBatch b,
                                                     double2 *spec_all, const double *cpv_all, const double2 *mu_all,
                                                     int64_t nspec, int tk) {
    extern __shared__ double2 sm[];
    const int prob = blockIdx.y, kind = b.kind[prob];
    const int nz = d.nz, nxh = d.nxh, M = d.M;
    const int64_t nmodes = (int64_t)nxh * nz;
    double2 *spec = member_ptr(spec_all, b.ms) + prob * nspec;
    const double *cpv = member_ptr(cpv_all, b.ms) + (int64_t)kind * M * nmodes;
    const int kx0 = (int)blockIdx.x * tk;
    const int nt = (nxh - kx0 < tk) ? nxh - kx0 : tk;
    const int pts = nt * nz;
    const int bs = tk * nz;
    double2 *s_tw = sm + 2 * bs;
    stage_twiddles(s_tw, tb.twz, nz);
    const bool pin = (kind == 0 && kx0 == 0 && threadIdx.x == 0);
    const double2 mu = pin ? member_ptr(mu_all, b.ms)[prob] : make_double2(0.0, 0.0);
    double2 xprev[kZtQ], nd[kZtQ];
    double nc[kZtQ];
    auto row_ptr = [&](int j) { return spec + ((int64_t)j * nxh + kx0) * nz; };
    auto cp_ptr = [&](int j) { return cpv + (int64_t)j * nmodes + (int64_t)kx0 * nz; };
    {
        const double2 *r0 = row_ptr(M - 1);
        const double *c0 = cp_ptr(M - 1);
#pragma unroll
        for (int q = 0; q < kZtQ; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            nd[q] = r0[e < pts ? e : 0];
            nc[q] = c0[e < pts ? e : 0];
            xprev[q] = make_double2(0.0, 0.0);
        }
    }
    for (int j = M - 1; j >= 0; --j) {
#pragma unroll
        for (int q = 0; q < kZtQ; ++q) {
            const int e = (int)threadIdx.x + q * (int)blockDim.x;
            if (e < pts) {
                const double2 x = make_double2(nd[q].x - nc[q] * xprev[q].x, nd[q].y - nc[q] * xprev[q].y);
                xprev[q] = x;
                sm[e] = (pin && q == 0) ? make_double2(x.x - mu.x, x.y - mu.y) : x;
            }
        }
        __syncthreads();
        if (j > 0) {  // the next row's d' and c' land during this row's passes
            const double2 *rn = row_ptr(j - 1);
            const double *cn = cp_ptr(j - 1);
#pragma unroll
            for (int q = 0; q < kZtQ; ++q) {
                const int e = (int)threadIdx.x + q * (int)blockDim.x;
                nd[q] = rn[e < pts ? e : 0];
                nc[q] = cn[e < pts ? e : 0];
            }
        }
        const int w = lds_fft<kR8>(sm, sm + bs, nz, nt, pl, s_tw, true);
        const double2 *z = sm + w * bs;
        double2 *out = row_ptr(j);
        for (int e = threadIdx.x; e < pts; e += blockDim.x) out[e] = z[e];
        __syncthreads();
    }
}

// modes per tile of the y solve: at most `want`, within 64 KB of LDS
inline int thomas_tile_modes(int M, int want) {
    int tm = 65536 / (M * (int)sizeof(double2)) - 1;
    if (tm > want) tm = want;
    return tm < 1 ? 1 : tm;
}

// line pairs per block of the x transforms: about `points` complex values,
// within 64 KB of LDS for the two staging buffers
inline int pairs_per_block(int nx, int points, int lds_bytes = 65536) {
    int p = nx >= points ? 1 : points / nx;
    // two buffers of x_buffer_slots(nx, p) plus the twiddle table
    const int lds_max = (lds_bytes - nx * (int)sizeof(double2)) / (2 * (nx + 2) * (int)sizeof(double2));
    if (p > lds_max) p = lds_max;
    return p < 1 ? 1 : p;
}
inline int modes_per_tile(int nz, int nxh, int points) {
    int t = nz >= points ? 1 : points / nz;
    if (t > 32) t = 32;
    if (t > nxh) t = nxh;
    // two staging buffers plus the twiddle table within 64 KB of LDS
    const int lds_max = (65536 - nz * (int)sizeof(double2)) / (2 * nz * (int)sizeof(double2));
    if (t > lds_max) t = lds_max;
    return t < 1 ? 1 : t;
}

}  // namespace

// Kernels that need more than 64 KB of dynamic LDS ask for the device's
// larger per-workgroup limit, once per (device, kernel); the record is
// shared by every handle and guarded for callers on several host threads.
hipError_t lds_opt_in(const void *fn, size_t bytes, int lds_max) {
    if (bytes <= 65536) return hipSuccess;
    if (bytes > (size_t)lds_max) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> opted;
    std::lock_guard<std::mutex> lock(mu);
    if (opted.count({dev, fn})) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (e == hipSuccess) opted.insert({dev, fn});
    return e;
}

// All members of the handle are solved when b.ms is the member stride;
// caller-owned arrays (b.ms = 0) are solved for member 0 only.
hipError_t launch_poisson_batch(nspnp_state *s, const PoissonBatch &b) {
    const Dims &d = s->d;
    const int nmem = b.ms ? s->nmem : 1;
    const int64_t nlines = (int64_t)d.M * d.nz;
    const int64_t nspec = (int64_t)d.nxh * d.nz * d.M;
    const int ppb = pairs_per_block(d.nx, s->tiles.fftx);
    const int64_t npairs = (nlines + 1) / 2;
    auto has_r8 = [](const FftPlan &p) {
        for (int q = 0; q < p.nstages; ++q)
            if (p.radix[q] == 8) return true;
        return false;
    };
    const bool r8x = has_r8(s->planx), r8z = has_r8(s->planz);
    {
        ProfScope prof_(s, K_FFTX_FWD);
        const dim3 gx((unsigned)((npairs + ppb - 1) / ppb), (unsigned)b.nprob, (unsigned)nmem);
        const size_t ldsx = (2 * (size_t)x_buffer_slots(d.nx, ppb) + d.nx) * sizeof(double2);
        const void *fn = s->fp64 ? (r8x ? (const void *)k_fft_x_r2c<double, true> : (const void *)k_fft_x_r2c<double, false>)
                                 : (r8x ? (const void *)k_fft_x_r2c<float, true> : (const void *)k_fft_x_r2c<float, false>);
        const hipError_t e = lds_opt_in(fn, ldsx, s->lds_max);
        if (e != hipSuccess) return e;
#define NSPNP_R2C(TT, RR) k_fft_x_r2c<TT, RR><<<gx, 256, ldsx, s->stream>>>(d, s->tb, s->planx, b, s->clock, s->spec, nspec, ppb)
        if (s->fp64) {
            if (r8x) NSPNP_R2C(double, true);
            else NSPNP_R2C(double, false);
        } else {
            if (r8x) NSPNP_R2C(float, true);
            else NSPNP_R2C(float, false);
        }
#undef NSPNP_R2C
    }
    if (s->tiles.thomas == 0 && s->cpv && s->mu) {
        // z transforms and mode solves fused into two row marches: tiles of
        // tk x-modes, about one mode of a row per thread (the marches are
        // serial in y, so the most tiles give the most parallelism)
        const int tk = std::max(1, std::min(d.nxh, 256 / d.nz));
        if (tk * d.nz > kZtQ * 256) return hipErrorInvalidValue;
        const dim3 gy((unsigned)((d.nxh + tk - 1) / tk), (unsigned)b.nprob, (unsigned)nmem);
        const size_t lds = (2 * (size_t)tk * d.nz + d.nz) * sizeof(double2);
        {
            ProfScope prof_(s, K_FFTZ_FWD);
            if (r8z) k_zthomas_fwd<true><<<gy, 256, lds, s->stream>>>(d, s->tb, s->planz, b, s->spec, s->mu, nspec, tk);
            else k_zthomas_fwd<false><<<gy, 256, lds, s->stream>>>(d, s->tb, s->planz, b, s->spec, s->mu, nspec, tk);
        }
        {
            ProfScope prof_(s, K_FFTZ_INV);
            if (r8z)
                k_zthomas_bwd<true><<<gy, 256, lds, s->stream>>>(d, s->tb, s->planz, b, s->spec, s->cpv, s->mu, nspec, tk);
            else
                k_zthomas_bwd<false><<<gy, 256, lds, s->stream>>>(d, s->tb, s->planz, b, s->spec, s->cpv, s->mu, nspec,
                                                                 tk);
        }
    } else {
        int tk = modes_per_tile(d.nz, d.nxh, s->tiles.fftz);
        if (tk * d.nz > kZPer * 256) tk = std::max(1, kZPer * 256 / d.nz);
        const int ztiles = d.M * ((d.nxh + tk - 1) / tk);
        // persistent blocks: about 8 per CU over all problems and members
        const int zblocks = std::max(1, std::min(ztiles, 2048 / std::max(1, b.nprob * nmem)));
        const dim3 gz((unsigned)zblocks, (unsigned)b.nprob, (unsigned)nmem);
        const size_t ldsz = (2 * (size_t)tk * d.nz + d.nz) * sizeof(double2);
        {
            ProfScope prof_(s, K_FFTZ_FWD);
            if (r8z) k_fft_z<true><<<gz, 256, ldsz, s->stream>>>(d, s->planz, s->tb.twz, s->spec, nspec, tk, 0, b.ms);
            else k_fft_z<false><<<gz, 256, ldsz, s->stream>>>(d, s->planz, s->tb.twz, s->spec, nspec, tk, 0, b.ms);
        }
        const int64_t nmodes = (int64_t)d.nxh * d.nz;
        {
            ProfScope prof_(s, K_THOMAS);
            const int tm = thomas_tile_modes(d.M, s->tiles.thomas);
            const dim3 gt((unsigned)((nmodes + tm - 1) / tm), (unsigned)b.nprob, (unsigned)nmem);
            const size_t ldst = (size_t)d.M * (tm + 1) * sizeof(double2);
            const int rpl = (d.M + 63) / 64;  // rows per lane (M <= 512: at most 8)
#define NSPNP_TH_CASE(RR)                                                                                \
        case RR:                                                                                             \
            k_thomas_tile<RR><<<gt, 256, ldst, s->stream>>>(d, s->tb, b, s->spec, s->fac, nspec, tm);        \
            break;
            switch (rpl) {
                NSPNP_TH_CASE(1)
                NSPNP_TH_CASE(2)
                NSPNP_TH_CASE(3)
                NSPNP_TH_CASE(4)
                NSPNP_TH_CASE(5)
                NSPNP_TH_CASE(6)
                NSPNP_TH_CASE(7)
                NSPNP_TH_CASE(8)
                default:
                    return hipErrorInvalidValue;
            }
#undef NSPNP_TH_CASE
        }
        {
            ProfScope prof_(s, K_FFTZ_INV);
            if (r8z) k_fft_z<true><<<gz, 256, ldsz, s->stream>>>(d, s->planz, s->tb.twz, s->spec, nspec, tk, 1, b.ms);
            else k_fft_z<false><<<gz, 256, ldsz, s->stream>>>(d, s->planz, s->tb.twz, s->spec, nspec, tk, 1, b.ms);
        }
    }
    {
        ProfScope prof_(s, K_FFTX_INV);
        // at least 8 lines per block, so that every kx of the transposed load
        // reads whole 128-byte lines of the [j][kx][kz] spectrum
        // (the device's whole LDS per workgroup may be used for that)
        int ppbc = std::max(ppb, pairs_per_block(d.nx, 4 * d.nx, s->lds_max));
        ppbc = std::max(1, std::min(ppbc, kCPer * 256 / (2 * d.nxh)));  // prefetch registers
        const int ctiles = (int)((npairs + ppbc - 1) / ppbc);
        const int cblocks = std::max(1, std::min(ctiles, 2048 / std::max(1, b.nprob * nmem)));
        const dim3 gc((unsigned)cblocks, (unsigned)b.nprob, (unsigned)nmem);
        const size_t ldsc = (2 * (size_t)x_buffer_slots(d.nx, ppbc) + d.nx) * sizeof(double2);
        const void *fn = s->fp64 ? (r8x ? (const void *)k_fft_x_c2r<double, true> : (const void *)k_fft_x_c2r<double, false>)
                                 : (r8x ? (const void *)k_fft_x_c2r<float, true> : (const void *)k_fft_x_c2r<float, false>);
        const hipError_t e = lds_opt_in(fn, ldsc, s->lds_max);
        if (e != hipSuccess) return e;
#define NSPNP_C2R(TT, RR) k_fft_x_c2r<TT, RR><<<gc, 256, ldsc, s->stream>>>(d, s->tb, s->planx, b, s->spec, nspec, ppbc)
        if (s->fp64) {
            if (r8x) NSPNP_C2R(double, true);
            else NSPNP_C2R(double, false);
        } else {
            if (r8x) NSPNP_C2R(float, true);
            else NSPNP_C2R(float, false);
        }
#undef NSPNP_C2R
    }
    return hipGetLastError();
}

// Raise the dynamic-LDS limit of the FP64 x transforms ahead of use (their
// blocks may take more than 64 KB), so that later launches find the record.
hipError_t prime_x_transform_lds(int lds_max) {
    const void *fns[4] = {(const void *)k_fft_x_r2c<double, false>, (const void *)k_fft_x_r2c<double, true>,
                          (const void *)k_fft_x_c2r<double, false>, (const void *)k_fft_x_c2r<double, true>};
    for (const void *fn : fns) {
        const hipError_t e = lds_opt_in(fn, (size_t)lds_max, lds_max);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Thomas pivots of both elliptic operators for every member of the handle
// (once, at init: they depend on the grid only).
hipError_t launch_thomas_factors(nspnp_state *s) {
    const int64_t nmodes = (int64_t)s->d.nxh * s->d.nz;
    const dim3 g((unsigned)((nmodes + 255) / 256), 2, (unsigned)s->nmem);
    k_thomas_factors<<<g, 256, 0, s->stream>>>(s->d, s->tb, s->fac, s->cpv, s->mstride);
    return hipGetLastError();
}

}  // namespace nspnp
