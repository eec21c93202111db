// internal.h -- device-side data structures shared by the HIP translation
// units of the gfx950 NS-PNP library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nspnp.h"

namespace nspnp {

constexpr int kMaxFftStages = 12;
// Most cell rows across the gap (ny - 1) of a supported grid: 8 rows per
// lane of the wall-normal scans.
constexpr int kMaxRows = 512;

// Radix decomposition of one FFT length (radices 4, 2, 3; product = n).
struct FftPlan {
    int n;
    int nstages;
    int radix[kMaxFftStages];
};

// Sizes and geometry constants passed by value to every kernel.
struct Dims {
    int nx, nz, M, nxh;   // nxh = nx/2 + 1 retained x modes
    int64_t n;            // nx * nz * M cells
    int64_t plane;        // nx * nz
    double dx, dz;
};

// Device tables built once from the grid (all FP64).
struct Tables {
    const double *yc;       // M
    const double *dn;       // M   cell heights
    const double *dc;       // M+1 centre-to-centre (half cells at the walls)
    const double *lyc_lo;   // M   1/(dn_j dc_j)
    const double *lyc_up;   // M   1/(dn_j dc_{j+1})
    const double *lyn_lo;   // M   1/(dc_j dn_{j-1}) (node rows, row 0 unused)
    const double *lyn_up;   // M   1/(dc_j dn_j)
    const double *idn;      // M   1/dn_j
    const double *idc;      // M+1 1/dc_j
    const double *vwl;      // M   dn_{j-1}/(2 dc_j): weight of row j-1 at node j
    const double *vwu;      // M   dn_j/(2 dc_j): weight of row j at node j
    const double *kx2;      // nxh modified wavenumbers (2 - 2 cos(2 pi m / nx)) / dx^2
    const double *kz2;      // nz
    const double2 *twx;     // nx  FFT twiddles of the x plan, in pass order (see build_tables)
    const double2 *twz;     // nz  the same for the z plan
};

// Physical constants of the nondimensional equations (one per member run;
// each member's copy lives in its own workspace).
struct Phys {
    double re, ire;     // Re, 1/Re
    double kd;          // 1 / (Re Sc)
    double kf;          // sF * beta / (2 Sc Re^2 lam^2)
    double e0;          // vhat / 2: dPhi_0/dy
    double ch;          // -1 / (2 lam^2): charge factor of the potential equation
    double u_top, u_bot;
    double debye, cfl;
    double adaptive;    // 1: dt from the CFL rule at stage 1; 0: fixed dt
    double implicit_xz; // 1: x/z diffusion implicit (no explicit diffusion limit on dt)
    double hybrid;      // 1: hybrid face value of c in the migration flux (mig_face)
    double limited;     // 1: limited face value of c in the advective flux (adv_face)
};

// Face value of c in the migration flux of a species of valence zs across a
// face with potential difference dphi = Phi_R - Phi_L (R the cell on the side
// of increasing index), given the mean of the two cells.  Sec. II's central
// differences take the mean; its stationary cell ratio
// (1 - zs dphi/2)/(1 + zs dphi/2) turns negative once |dphi| > 2.  The hybrid
// rule takes, on faces with |dphi| >= 2, the cell the species' drift
// -zs (Re Sc)^-1 grad Phi comes from: R when zs dphi > 0, else L.
template <typename T>
__device__ __forceinline__ T mig_face(bool hyb, T mean, T cl, T cr, T dphi, T zs) {
    if (hyb && fabs(dphi) >= T(2)) return (zs * dphi > T(0)) ? cr : cl;
    return mean;
}
// Face value of c in the advective flux, limited form (migration_face 2):
// the upwind cell U of the face velocity plus the van Leer slope a b/(a + b),
// a = c_U - c_UU, b = c_D - c_U (D the downwind cell, UU the cell beyond U),
// when a b > 0, else c_U alone; equal to the mean of the two cells on a linear
// profile of equal spacings, and no new extrema where it is not.  up: the face
// velocity is >= 0 (U = cl); have: UU exists.  U a wall row (no UU): the cell
// beyond the wall is an image of U (zero gradient, as the zero normal flux
// has it), so the face value is c_U.
template <typename T>
__device__ __forceinline__ T adv_face(T cl, T cr, T cuu, bool up, bool have) {
    const T cu = up ? cl : cr, cd = up ? cr : cl;
    if (!have) return cu;
    const T a = cu - cuu, b = cd - cu;
    const T ab = a * b;
    return (ab > T(0)) ? cu + ab / (a + b) : cu;
}
// Potential difference across a wall-normal face: the applied field e0 over
// the centre distance dc plus the perturbation difference, each operation
// rounded on its own (no fused multiply-add), so that the hybrid rule's
// threshold sees the same value wherever it is formed.
__device__ __forceinline__ double y_dphi(double e0, double dc, double dphi) {
    return __dadd_rn(__dmul_rn(e0, dc), dphi);
}
__device__ __forceinline__ float y_dphi(float e0, float dc, float dphi) {
    return __fadd_rn(__fmul_rn(e0, dc), dphi);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This bijection of the linear block id gives XCD x one contiguous range
// of tiles (the first nblocks % 8 XCDs one tile more), so tiles whose
// stencils overlap (neighbouring z rows) run in the same L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nblocks) {
    const unsigned x = b & 7u, l = b >> 3;
    const unsigned q = nblocks >> 3, r = nblocks & 7u;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// The same bijection over a whole (x, y, z) grid: the block's linear id (x
// fastest, the dispatch order) is remapped and split back into coordinates,
// so consecutive x tiles of one (y, z) slice share an XCD whatever gridDim.x.
__device__ __forceinline__ uint3 xcd_block3() {
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned t = xcd_tile(lin, gx * gy * gridDim.z);
    return make_uint3(t % gx, (t / gx) % gy, t / (gx * gy));
}

// Every member of a batch has the same workspace layout; device pointers in
// kernel arguments refer to member 0 and member blockIdx.z sits stride bytes
// further per member.
template <typename P>
__device__ __forceinline__ P *member_ptr(P *p, size_t stride) {
    return (P *)((char *)p + (size_t)blockIdx.z * stride);
}
template <typename P>
__device__ __forceinline__ P *member_ptr_at(P *p, size_t stride, unsigned member) {
    return (P *)((char *)p + (size_t)member * stride);
}

// A block-uniform element of a read-only table (grid metrics), read through
// the scalar cache: the load is counted apart from the vector memory loads,
// so using its value never waits for vector loads still in flight (vector
// loads retire in issue order).  i must be the same in every lane.
__device__ __forceinline__ double uniform_load(const double *p, int i) {
    typedef const __attribute__((address_space(4))) double cdouble;
    return ((cdouble *)p)[__builtin_amdgcn_readfirstlane(i)];
}

// Accesses to data that a kernel touches once (no neighbouring thread or
// block reads the same element) and that is not handed straight to the next
// kernel through the last-level cache: the non-temporal hint streams these
// lines, so they do not displace data that is reused.  The elliptic chain
// (forward transforms, mode solves, inverse z transform) keeps plain
// accesses: its two half spectra (about 200 MB at 256 x 193 x 256 in FP64)
// and the mode pivots stay in the 256 MB Infinity Cache between stages.
// Stencil halo loads stay plain too (neighbouring tiles re-read them).  Which
// accesses carry the hint was settled by measurement of the whole substep.
// NSPNP_NT=0 builds plain accesses everywhere.
#ifndef NSPNP_NT
#define NSPNP_NT 1
#endif
template <typename T>
__device__ __forceinline__ T ld_once(const T *p) {
#if NSPNP_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <typename T>
__device__ __forceinline__ void st_once(T *p, T v) {
#if NSPNP_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}
// Element at a 32-bit byte offset from a base pointer (the form the
// hardware's scalar-base + vector-offset addressing takes directly).
template <typename T>
__device__ __forceinline__ T *byte_at(T *base, unsigned bytes) {
    return (T *)((char *)base + bytes);
}
template <typename T>
__device__ __forceinline__ const T *byte_at(const T *base, unsigned bytes) {
    return (const T *)((const char *)base + bytes);
}
// Two adjacent FP32 values as one 8-byte access (non-temporal), for
// staging loops over rows of FP32 fields.
typedef float nspnp_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ nspnp_f2v ld_once2(const float *p) {
#if NSPNP_NT
    return __builtin_nontemporal_load((const nspnp_f2v *)p);
#else
    return *(const nspnp_f2v *)p;
#endif
}
__device__ __forceinline__ void st_once2(float *p, nspnp_f2v v) {
#if NSPNP_NT
    __builtin_nontemporal_store(v, (nspnp_f2v *)p);
#else
    *(nspnp_f2v *)p = v;
#endif
}
typedef double nspnp_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_once(const double2 *p) {
#if NSPNP_NT
    const nspnp_d2v v = __builtin_nontemporal_load((const nspnp_d2v *)p);
    return make_double2(v.x, v.y);
#else
    return *p;
#endif
}
__device__ __forceinline__ void st_once(double2 *p, double2 v) {
#if NSPNP_NT
    nspnp_d2v w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (nspnp_d2v *)p);
#else
    *p = v;
#endif
}

// Per-row quantities of the plane reduction (k_plane), kPlaneQ per row.
enum PlaneQ {
    PQ_SUM_U = 0, PQ_SUM_CP, PQ_SUM_CM,  // plane sums of u, c+, c-
    PQ_FLUX_P, PQ_FLUX_M,                // total wall-normal ion fluxes at node j (sums)
    PQ_KE,                               // kinetic energy of the row
    PQ_MAX_DIV, PQ_MIN_CP, PQ_MIN_CM, PQ_MAX_CSUM,
    PQ_MAX_DPHI,                         // max |Phi difference| across the row's faces
    kPlaneQ
};

// Health word of a run (device clock slot 2), sticky until the clock is set:
// bit 0 a non-finite field value or step, bit 1 a negative concentration.
// Slot 3 holds the largest potential difference across one cell face at the
// last check (the migration cell Peclet number).
constexpr int kHealthNonFinite = 1, kHealthNegative = 2;
constexpr int kClockSlots = 4;  // t, dt, health, max |dPhi|
// Partial results of the once-per-step check (dt rule and health): values
// per block, threads per block, and the block budget per member (more only
// when one block per kDtThreads columns already exceeds it).
constexpr int kDtParts = 5, kDtThreads = 256, kDtMaxBlocks = 1024;
inline int dt_chunks(int64_t plane) { return (int)((plane + kDtThreads - 1) / kDtThreads); }
inline int dt_max_blocks(int64_t plane) { return dt_chunks(plane) > kDtMaxBlocks ? dt_chunks(plane) : kDtMaxBlocks; }

// Low-storage third-order Runge-Kutta coefficients of the three stages:
// gamma, zeta and alpha = gamma + zeta.
constexpr double kRkGam[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
constexpr double kRkZet[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};
constexpr double kRkAlp[3] = {8.0 / 15.0 + 0.0, 5.0 / 12.0 - 17.0 / 60.0, 3.0 / 4.0 - 5.0 / 12.0};

// Runge-Kutta coefficients of one substep.
struct Stage {
    double gam, zet, alp;
    int k;              // 0, 1, 2
};

// Right-hand side of one elliptic solve, produced while the x-lines load.
enum PoissonSrcType { SRC_REAL = 0, SRC_DIV = 1, SRC_CHARGE = 2 };
struct PoissonSrc {
    int type;
    const void *a, *b, *c;  // REAL: a = FP64 array; DIV: u, v, w; CHARGE: c+, c-
    double fixed;           // DIV: scale when alp <= 0; CHARGE: -1/(2 lam^2)
    double alp;             // DIV: scale 1/(alp dt) with dt from the device clock
    const double *wall = nullptr;  // CHARGE: wall values of phi, [lower | upper] plane (NULL: zero)
};
// Up to two independent solves sharing one pipeline (pressure and potential).
struct PoissonBatch {
    int nprob;
    int kind[2];        // 0 pressure-type, 1 potential-type
    PoissonSrc src[2];
    void *out[2];       // result arrays
    int out_state[2];   // 1: store in the state type, 0: FP64
    size_t ms;          // member stride in bytes (0 for caller-owned arrays)
    const Phys *phys;   // member 0's constants (charge factor)
};

// Row-slab Crank-Nicolson method: the most slabs per column.
constexpr int kCnMaxSlabs = 32;
// Crank-Nicolson coefficients of one Runge-Kutta stage: [3 systems][g, m, n]
// [M] rows, the slab products [3 systems][P, Phi, Nu][kCnMaxSlabs], then for
// the row-slab method's fused first pass [3 systems][M] the products of n
// from the slab's first row up to the row below.
__host__ __device__ inline size_t cn_stage_stride(int M) {
    return 12 * (size_t)M + 9 * (size_t)kCnMaxSlabs;
}

// Launch shapes chosen by the autotuner.  None of them changes the
// arithmetic done per cell, column, line or mode, so results are bitwise
// independent of the choice.
struct Tiles {
    int expl;     // threads per block of the explicit kernel (64..256)
    int cn;       // threads per block (columns) of the Crank-Nicolson solve
    int fftx;     // complex points per block of the x transforms
    int fftz;     // complex points per block of the z transforms
    int thomas;   // modes per tile of the y solve of the elliptic problems (capped by LDS); 0: the z
                  // transforms and the y solve fused into two row marches
    int corr;     // threads per block of the projection correction
    int slab;     // rows marched by one block of the explicit kernel
    int cnslab;   // Crank-Nicolson: 0 lane-scan method, 16 or 32 row-slab method with that many rows
};

constexpr int kTileInts = 8;  // Tiles as exported through the ABI

// Run statistics: time sums of the plane means of u, v, w, c+, c-, phi, p
// and of their squares, per row (v per node row).
constexpr int kRunStatsFields = 7;
constexpr int kRunStatsQ = 2 * kRunStatsFields;
constexpr int kRunStatsTail = 4;  // accumulated time, time of the last sample, samples, unused
constexpr int kStatCloseThreads = 256;

// Implicit x/z diffusion: one block of doubles per (stage, velocity or ion
// diffusivity, direction): recurrence coefficients g, m, n and the
// periodic-correction vector z (Nmax each), then [e/gamma, 1/(1 + v.z), -, -].
constexpr int kCycBlocks = 3 * 2 * 2;
__host__ __device__ inline int64_t cyc_block_doubles(int nx, int nz) {
    return 4 * (int64_t)(nx > nz ? nx : nz) + 4;
}
// Blocks per row of the statistics pass: about 2048 blocks over the grid
// (at least one per row, at most 32); its partial sums, kRunStatsQ per block,
// live in the reduction scratch.
__host__ __device__ inline int run_stats_chunks(int M) {
    const int c = (2048 + M - 1) / M;
    return c < 1 ? 1 : (c > 32 ? 32 : c);
}

// Kernel classes timed by the optional event profiler.
enum KernelId {
    K_DT = 0, K_EXPLICIT, K_CN, K_FFTX_FWD, K_FFTZ_FWD, K_THOMAS, K_FFTZ_INV, K_FFTX_INV,
    K_CORRECT, K_STATS, K_NKERNEL
};

// hipEvent pairs around kernel launches on the solver's stream.
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ids;
    size_t used = 0;
    double total_ms[K_NKERNEL] = {};
    int64_t launches[K_NKERNEL] = {};
    hipEvent_t next() {
        if (used == ev.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev.push_back(e);
        }
        return ev[used++];
    }
};

}  // namespace nspnp

// Host handle (opaque to users).
struct nspnp_state {
    nspnp_config cfg;
    nspnp::Dims d;
    nspnp::Phys ph;       // host copy (member 0)
    nspnp::Phys *d_phys;  // device copy inside the workspace (member 0)
    int nmem;             // members batched in this handle (1 for a single run)
    size_t mstride;       // bytes between members' workspaces
    nspnp::Tables tb;
    nspnp::FftPlan planx, planz;
    nspnp::Tiles tiles;
    hipStream_t stream;
    int lds_max = 65536;  // LDS bytes one workgroup may use on this device
    bool fp64;
    size_t wsize;        // bytes of one state-type element
    void *f[7];          // u v w c+ c- phi p, state type
    void *h[5];          // H^{k-1} -> H^k, state type
    void *r[5];          // Crank-Nicolson right-hand sides, state type
    double *psi;         // pressure increment (n, FP64)
    double2 *spec;       // two half spectra, 2 * nxh * nz * M
    double2 *fac;        // Thomas pivots (1/den, c') of both elliptic operators, [kind][mode][row]
    double *cpv;         // c' alone, [kind][row][mode], for the fused y-march (NULL: not kept)
    double2 *mu;         // volume mean of the pinned pressure mode, per problem (fused y-march)
    double *cn_coef;     // Crank-Nicolson recurrence coefficients, 9 M per stage
    bool cn_fresh = false;  // cn_coef matches the device dt of the current step
    int cn_coef_slab = -1;  // slab rows the slab products in cn_coef were made for
    int64_t cn_coef_at = -1;  // substep count at which cn_coef was last brought up to date
    double *clock;       // device [t, dt, health, max |dPhi|]
    double *host_health = nullptr;  // pinned host mirror of each member's [health, max |dPhi|]
    bool owns_host_health = false;
    double *red;         // reduction scratch
    int64_t nred;
    double *stats;       // time sums of the plane means of u, c+ - c-, phi (3 per row) and the time
    bool stats_on;
    double *rstats;      // run statistics: kRunStatsQ time sums per row, then [time, t_last, samples, -]
    double *phiw;        // wall values of phi: lower-wall plane, then upper-wall plane (FP64)
    double *cyc;         // implicit x/z diffusion: periodic-line recurrences per stage, nu and direction
    bool phiw_on = false;  // phiw holds nonzero data (else the potential solve skips it)
    int rstats_every = 0;  // sample at the end of every rstats_every-th substep (0: off)
    char *tab_base;      // device tables (member 0)
    int64_t substeps;
    std::vector<double> host_tables;
    nspnp::Profiler prof;
    ~nspnp_state();
};

namespace nspnp {

// Records an event before and after the launches in its scope when the
// profiler is on.
class ProfScope {
  public:
    ProfScope(nspnp_state *s, int id) : s_(s), id_(id) {
        if (s_->prof.on) {
            hipEvent_t e = s_->prof.next();
            if (e) { (void)hipEventRecord(e, s_->stream); s_->prof.ids.push_back(id_); }
            else s_ = nullptr;
        } else {
            s_ = nullptr;
        }
    }
    ~ProfScope() {
        if (s_) {
            hipEvent_t e = s_->prof.next();
            if (e) (void)hipEventRecord(e, s_->stream);
        }
    }
  private:
    nspnp_state *s_;
    int id_;
};

// launchers (one translation unit each; all queue on s->stream)
hipError_t launch_explicit(nspnp_state *s, const Stage &st, bool write_r);
hipError_t launch_explicit_debug(nspnp_state *s, double *const out[5]);
hipError_t launch_adv_limit(nspnp_state *s, const Stage &st, double *const out[5]);
hipError_t launch_cn_solve(nspnp_state *s, const Stage &st);
hipError_t launch_correct(nspnp_state *s, const Stage &st, bool update_p, double fixed_scale, bool advance_clock);
hipError_t launch_poisson_batch(nspnp_state *s, const PoissonBatch &b);
// Raises a kernel's dynamic-LDS limit to the device maximum when bytes > 64 KB
// (once per device and kernel); hipErrorInvalidValue when bytes > lds_max.
hipError_t lds_opt_in(const void *fn, size_t bytes, int lds_max);
hipError_t launch_thomas_factors(nspnp_state *s);
hipError_t prime_x_transform_lds(int lds_max);
hipError_t launch_dt(nspnp_state *s);
hipError_t launch_init_fields(nspnp_state *s);
hipError_t launch_plane_sums(nspnp_state *s, int what, double *dev_out);
hipError_t launch_energy_sums(nspnp_state *s, double *dev_out);  // 4 doubles per row
hipError_t launch_shift_conc(nspnp_state *s, double mean_p, double mean_m);
hipError_t launch_convert(nspnp_state *s, int field, const double *in, double *out, bool to_state);
hipError_t launch_stats_accum(nspnp_state *s, double alp);
hipError_t launch_run_stats(nspnp_state *s);
hipError_t launch_run_stats_begin(nspnp_state *s);
hipError_t launch_stats_reset(nspnp_state *s);
hipError_t launch_fill(nspnp_state *s, double *p, int64_t n, double v);

// handle management shared by the single-run and ensemble entry points
int fail_code(int code, const std::string &msg);
void setup_common(nspnp_state *s, const nspnp_config *cfg, int nmem, hipStream_t stream);
void fill_tables(nspnp_state *s, double *dev_tab);  // host tables + device pointers at dev_tab
size_t tables_len(int M, int nx, int nz);           // doubles of the grid tables
int check(const nspnp_config *c);
size_t layout_bytes(const nspnp_config *c);
Phys make_phys(const nspnp_config *cfg);
void setup_handle(nspnp_state *s, const nspnp_config *cfg, char *base, int nmem, hipStream_t stream);
int upload_tables(nspnp_state *s);
nspnp_state *member_view(const nspnp_state *cls, int m, const nspnp_config *cfg);
int init_member(nspnp_state *s);
int step_handle(nspnp_state *s, int n);
int health_error(int bits, int member);
int alloc_host_health(nspnp_state *s);
int check_health(const nspnp_state *s, int first_id);
int queue_health_copy(nspnp_state *s);

}  // namespace nspnp
