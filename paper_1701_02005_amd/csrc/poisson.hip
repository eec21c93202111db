// poisson.hip -- elliptic solver of the pressure projection and of the
// potential (Sec. II): Fourier transform in the two periodic directions,
// then one tridiagonal (Thomas) system across the gap per Fourier mode,
// with zero-flux walls (pressure) or zero wall value (potential).
//
// Data flow for one solve, all FP64:
//   real [j][k][i]  --x R2C-->  half spectrum [j][k][kx] (kx < nx/2+1)
//   --z C2C--> [j][kz][kx]  --Thomas in j per (kx,kz)-->  --z C2C^-1-->
//   --x C2R--> real [j][k][i]
// The FFTs are self-sorting (Stockham) in LDS with radix 4, 2 and 3 stages;
// two real x-lines share one complex transform.
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

template <int R>
__device__ __forceinline__ void stage_pass(const double2 *__restrict__ src, double2 *__restrict__ dst, int N,
                                           int nl, int Ns, const double2 *__restrict__ tw, bool inv, int tid,
                                           int nth) {
    const int NR = N / R;
    const int ts = N / (Ns * R);
    for (int e = tid; e < nl * NR; e += nth) {
        const int line = e / NR;
        const int jb = e - line * NR;
        const int k = jb % Ns;
        const double2 *in = src + line * N;
        double2 *out = dst + line * N;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[jb + r * NR];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            double2 w = tw[r * k * ts];
            if (inv) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
        dft_small<R>(v, inv);
        const int base = (jb / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out[base + r * Ns] = v[r];
    }
}

// nl lines of length N in buf[0]; returns the buffer (0 or 1) holding the result.
__device__ int lds_fft(double2 *b0, double2 *b1, int N, int nl, const FftPlan &pl, const double2 *tw, bool inv) {
    double2 *src = b0, *dst = b1;
    int which = 0;
    int Ns = 1;
    for (int s = 0; s < pl.nstages; ++s) {
        const int R = pl.radix[s];
        if (R == 4) stage_pass<4>(src, dst, N, nl, Ns, tw, inv, threadIdx.x, blockDim.x);
        else if (R == 2) stage_pass<2>(src, dst, N, nl, Ns, tw, inv, threadIdx.x, blockDim.x);
        else stage_pass<3>(src, dst, N, nl, Ns, tw, inv, threadIdx.x, blockDim.x);
        __syncthreads();
        double2 *t = src;
        src = dst;
        dst = t;
        which ^= 1;
        Ns *= R;
    }
    return which;
}

// ---- x direction: real lines <-> half spectra, two lines per transform ----
__global__ void __launch_bounds__(256) k_fft_x_r2c(Dims d, FftPlan pl, const double2 *tw, const double *in,
                                                   double2 *out, int ppb) {
    extern __shared__ double2 sm[];
    const int nx = d.nx, nxh = d.nxh;
    const int64_t nlines = (int64_t)d.M * d.nz;
    double2 *b[2] = {sm, sm + ppb * nx};
    const int64_t pair0 = (int64_t)blockIdx.x * ppb;
    for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
        const int p = e / nx, i = e - p * nx;
        const int64_t la = 2 * (pair0 + p), lb = la + 1;
        const double re = (la < nlines) ? in[la * nx + i] : 0.0;
        const double im = (lb < nlines) ? in[lb * nx + i] : 0.0;
        b[0][e] = make_double2(re, im);
    }
    __syncthreads();
    const double2 *z = b[lds_fft(b[0], b[1], nx, ppb, pl, tw, false)];
    for (int e = threadIdx.x; e < ppb * nxh; e += blockDim.x) {
        const int p = e / nxh, kk = e - p * nxh;
        const int64_t la = 2 * (pair0 + p), lb = la + 1;
        const double2 zk = z[p * nx + kk];
        const double2 zc = z[p * nx + (kk == 0 ? 0 : nx - kk)];
        // A = (Z_k + conj(Z_{N-k}))/2, B = (Z_k - conj(Z_{N-k}))/(2i)
        const double2 A = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y - zc.y));
        const double2 B = make_double2(0.5 * (zk.y + zc.y), -0.5 * (zk.x - zc.x));
        if (la < nlines) out[la * nxh + kk] = A;
        if (lb < nlines) out[lb * nxh + kk] = B;
    }
}

__global__ void __launch_bounds__(256) k_fft_x_c2r(Dims d, FftPlan pl, const double2 *tw, const double2 *in,
                                                   double *out, int ppb) {
    extern __shared__ double2 sm[];
    const int nx = d.nx, nxh = d.nxh;
    const int64_t nlines = (int64_t)d.M * d.nz;
    double2 *b[2] = {sm, sm + ppb * nx};
    const int64_t pair0 = (int64_t)blockIdx.x * ppb;
    for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
        const int p = e / nx, kk = e - p * nx;
        const int64_t la = 2 * (pair0 + p), lb = la + 1;
        const bool lower = kk < nxh;
        const int src = lower ? kk : nx - kk;
        double2 A = (la < nlines) ? in[la * nxh + src] : make_double2(0.0, 0.0);
        double2 B = (lb < nlines) ? in[lb * nxh + src] : make_double2(0.0, 0.0);
        if (!lower) {  // Hermitian continuation of a real line's spectrum
            A.y = -A.y;
            B.y = -B.y;
        }
        // Z = A + i B
        b[0][e] = make_double2(A.x - B.y, A.y + B.x);
    }
    __syncthreads();
    const double2 *z = b[lds_fft(b[0], b[1], nx, ppb, pl, tw, true)];
    for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
        const int p = e / nx, i = e - p * nx;
        const int64_t la = 2 * (pair0 + p), lb = la + 1;
        const double2 v = z[e];
        if (la < nlines) out[la * nx + i] = v.x;
        if (lb < nlines) out[lb * nx + i] = v.y;
    }
}

// ---- z direction: complex lines of stride nxh, a tile of tk modes per block ----
__global__ void __launch_bounds__(256) k_fft_z(Dims d, FftPlan pl, const double2 *tw, double2 *data, int tk,
                                               int inverse) {
    extern __shared__ double2 sm[];
    const int nz = d.nz, nxh = d.nxh;
    const int tiles = (nxh + tk - 1) / tk;
    const int j = blockIdx.x / tiles;
    const int kx0 = (blockIdx.x - j * tiles) * tk;
    double2 *b[2] = {sm, sm + tk * nz};
    double2 *base = data + (int64_t)j * nz * nxh;
    for (int e = threadIdx.x; e < tk * nz; e += blockDim.x) {
        const int t = e % tk, k = e / tk;
        const int kx = kx0 + t;
        b[0][t * nz + k] = (kx < nxh) ? base[(int64_t)k * nxh + kx] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const double2 *z = b[lds_fft(b[0], b[1], nz, tk, pl, tw, inverse != 0)];
    for (int e = threadIdx.x; e < tk * nz; e += blockDim.x) {
        const int t = e % tk, k = e / tk;
        const int kx = kx0 + t;
        if (kx < nxh) base[(int64_t)k * nxh + kx] = z[t * nz + k];
    }
}

// ---- y direction: one Thomas solve per (kx, kz) mode ----
// (lo_j psi_{j-1} + (di_j - kx^2 - kz^2) psi_j + up_j psi_{j+1}) = rhs_j / (nx nz)
// kind 0: zero-flux walls, mode (0,0) pinned at row 0 then shifted to zero
// volume mean; kind 1: zero wall value at the half-cell distance.
__global__ void __launch_bounds__(256) k_thomas_modes(Dims d, Tables tb, double2 *spec, double *cpr, int kind) {
    const int64_t nmodes = (int64_t)d.nxh * d.nz;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nmodes) return;
    const int kx = (int)(m % d.nxh), kz = (int)(m / d.nxh);
    const int M = d.M;
    const double k2 = tb.kx2[kx] + tb.kz2[kz];
    const double scale = 1.0 / ((double)d.nx * (double)d.nz);
    const bool pin = (kind == 0 && kx == 0 && kz == 0);
    double cprev = 0.0;
    double2 dprev = make_double2(0.0, 0.0);
    for (int j = 0; j < M; ++j) {
        const int64_t o = (int64_t)j * nmodes + m;
        const double aa = tb.lyc_lo[j], cc = tb.lyc_up[j];
        double lo = (j > 0) ? aa : 0.0;
        double up = (j < M - 1) ? cc : 0.0;
        double di = -(lo + up);
        if (kind == 1) {
            if (j == 0) di -= aa;
            if (j == M - 1) di -= cc;
        }
        double B = di - k2;
        double2 rhs = spec[o];
        rhs.x *= scale;
        rhs.y *= scale;
        if (pin && j == 0) {
            B = 1.0;
            up = 0.0;
            rhs = make_double2(0.0, 0.0);
        }
        const double den = B - lo * cprev;
        const double cj = up / den;
        const double2 dj = make_double2((rhs.x - lo * dprev.x) / den, (rhs.y - lo * dprev.y) / den);
        spec[o] = dj;
        cpr[o] = cj;
        cprev = cj;
        dprev = dj;
    }
    double2 xn = make_double2(0.0, 0.0);
    double sx = 0.0, sy = 0.0, vol = 0.0;
    for (int j = M - 1; j >= 0; --j) {
        const int64_t o = (int64_t)j * nmodes + m;
        const double cj = cpr[o];
        const double2 dj = spec[o];
        const double2 xj = make_double2(dj.x - cj * xn.x, dj.y - cj * xn.y);
        spec[o] = xj;
        xn = xj;
        if (pin) {
            sx += xj.x * tb.dn[j];
            sy += xj.y * tb.dn[j];
            vol += tb.dn[j];
        }
    }
    if (pin) {
        const double mx = sx / vol, my = sy / vol;
        for (int j = 0; j < M; ++j) {
            const int64_t o = (int64_t)j * nmodes + m;
            double2 x = spec[o];
            x.x -= mx;
            x.y -= my;
            spec[o] = x;
        }
    }
}

inline int pairs_per_block(int nx) { return nx >= 1024 ? 1 : 1024 / nx; }
inline int modes_per_tile(int nz, int nxh) {
    int t = nz >= 1024 ? 1 : 1024 / nz;
    if (t > 16) t = 16;
    if (t > nxh) t = nxh;
    return t;
}

}  // namespace

hipError_t launch_poisson(nspnp_state *s, int kind, const double *rhs, double *out) {
    const Dims &d = s->d;
    const int64_t nlines = (int64_t)d.M * d.nz;
    const int ppb = pairs_per_block(d.nx);
    const int64_t npairs = (nlines + 1) / 2;
    const unsigned gx = (unsigned)((npairs + ppb - 1) / ppb);
    const size_t ldsx = 2 * (size_t)ppb * d.nx * sizeof(double2);
    {
        ProfScope prof_(s, K_FFTX_FWD);
        k_fft_x_r2c<<<gx, 256, ldsx, s->stream>>>(d, s->planx, s->tb.twx, rhs, s->spec, ppb);
    }
    const int tk = modes_per_tile(d.nz, d.nxh);
    const unsigned gz = (unsigned)(d.M * ((d.nxh + tk - 1) / tk));
    const size_t ldsz = 2 * (size_t)tk * d.nz * sizeof(double2);
    {
        ProfScope prof_(s, K_FFTZ_FWD);
        k_fft_z<<<gz, 256, ldsz, s->stream>>>(d, s->planz, s->tb.twz, s->spec, tk, 0);
    }
    const int64_t nmodes = (int64_t)d.nxh * d.nz;
    {
        ProfScope prof_(s, K_THOMAS);
        k_thomas_modes<<<(unsigned)((nmodes + 255) / 256), 256, 0, s->stream>>>(d, s->tb, s->spec, s->cpr, kind);
    }
    {
        ProfScope prof_(s, K_FFTZ_INV);
        k_fft_z<<<gz, 256, ldsz, s->stream>>>(d, s->planz, s->tb.twz, s->spec, tk, 1);
    }
    {
        ProfScope prof_(s, K_FFTX_INV);
        k_fft_x_c2r<<<gx, 256, ldsx, s->stream>>>(d, s->planx, s->tb.twx, s->spec, out, ppb);
    }
    return hipGetLastError();
}

}  // namespace nspnp
