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
    const double *kx2;      // nxh modified wavenumbers (2 - 2 cos(2 pi m / nx)) / dx^2
    const double *kz2;      // nz
    const double2 *twx;     // nx  exp(-2 pi i m / nx)
    const double2 *twz;     // nz
};

// Physical constants of the nondimensional equations.
struct Phys {
    double re, ire;     // Re, 1/Re
    double kd;          // 1 / (Re Sc)
    double kf;          // sF * beta / (2 Sc Re^2 lam^2)
    double e0;          // vhat / 2: dPhi_0/dy
    double ch;          // -1 / (2 lam^2): charge factor of the potential equation
    double u_top, u_bot;
    double debye, cfl;
};

// Runge-Kutta coefficients of one substep.
struct Stage {
    double gam, zet, alp;
    int k;              // 0, 1, 2
};

// Kernel classes timed by the optional event profiler.
enum KernelId {
    K_DT = 0, K_EXPLICIT, K_CN, K_DIV, K_FFTX_FWD, K_FFTZ_FWD, K_THOMAS, K_FFTZ_INV, K_FFTX_INV,
    K_CORRECT, K_CHARGE, K_STORE_PHI, K_CLOCK, K_NKERNEL
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
    nspnp::Phys ph;
    nspnp::Tables tb;
    nspnp::FftPlan planx, planz;
    hipStream_t stream;
    bool fp64;
    size_t wsize;        // bytes of one state-type element
    void *f[7];          // u v w c+ c- phi p, state type
    void *h[5];          // H^{k-1} -> H^k, state type
    double *r[5];        // Crank-Nicolson right-hand sides / Thomas scratch
    double *rhs;         // real Poisson scratch (n)
    double *psi;         // real Poisson solution (n)
    double2 *spec;       // half spectrum nxh * nz * M
    double *cpr;         // spectral Thomas elimination factors (nxh * nz * M)
    double *clock;       // device [t, dt]
    double *red;         // reduction scratch
    int64_t nred;
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
            if (e) { hipEventRecord(e, s_->stream); s_->prof.ids.push_back(id_); }
            else s_ = nullptr;
        } else {
            s_ = nullptr;
        }
    }
    ~ProfScope() {
        if (s_) {
            hipEvent_t e = s_->prof.next();
            if (e) hipEventRecord(e, s_->stream);
        }
    }
  private:
    nspnp_state *s_;
    int id_;
};

// launchers (one translation unit each; all queue on s->stream)
hipError_t launch_explicit(nspnp_state *s, const Stage &st, bool write_r);
hipError_t launch_explicit_debug(nspnp_state *s, double *const out[5]);
hipError_t launch_cn_solve(nspnp_state *s, const Stage &st);
hipError_t launch_divergence(nspnp_state *s, double scale_by_alpha_dt, const Stage &st, double *out);
hipError_t launch_correct(nspnp_state *s, const Stage &st, bool update_p, double fixed_scale);
hipError_t launch_charge(nspnp_state *s, double *out);
hipError_t launch_store_phi(nspnp_state *s, const double *src);
hipError_t launch_poisson(nspnp_state *s, int kind, const double *rhs, double *out);
hipError_t launch_dt(nspnp_state *s);
hipError_t launch_advance_clock(nspnp_state *s, double alp);
hipError_t launch_init_fields(nspnp_state *s);
hipError_t launch_plane_sums(nspnp_state *s, int what, double *dev_out);
hipError_t launch_shift_conc(nspnp_state *s, double mean_p, double mean_m);
hipError_t launch_convert(nspnp_state *s, int field, const double *in, double *out, bool to_state);

}  // namespace nspnp
