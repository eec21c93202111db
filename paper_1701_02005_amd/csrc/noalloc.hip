// noalloc.hip -- the elliptic solve of nspnp_poisson_solve without a handle
// and without any device allocation, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Its scratch (grid tables, the Thomas pivots of both
// elliptic operators, one half spectrum) lives in a file-scope device array
// that each GPU holds from the library's first use on it until the process
// ends; the kernels are those of the handle-based solve.
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace {

using namespace nspnp;

constexpr size_t kScratchBytes = (size_t)64 << 20;  // NSPNP_NOALLOC_SCRATCH_BYTES in include/nspnp.h
static_assert(kScratchBytes == NSPNP_NOALLOC_SCRATCH_BYTES, "scratch size and its public constant differ");

// The scratch array.  In host code its name stands for a host-side symbol,
// not a device address: host code uses the per-device pointer from
// hipGetSymbolAddress (Dev::ptr), never the name.
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

// Per-device record: the device address of the scratch array, the host
// copy of the grid tables (capacity reserved at set-up, so later grids reuse
// it) and the grid whose tables and pivots the scratch holds.
struct Dev {
    bool ready = false;
    char *ptr = nullptr;
    std::vector<double> host_tab;
    bool have_grid = false;
    nspnp_config grid{};
};

std::mutex g_mu;
Dev g_dev[kMaxDevices];

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct ScratchLayout {
    size_t tab, phys, fac, spec, total;
};

ScratchLayout scratch_layout(const nspnp_config *c) {
    const int64_t M = c->ny - 1, nxh = c->nx / 2 + 1;
    const int64_t nspec = nxh * c->nz * M;
    ScratchLayout L{};
    size_t o = 0;
    L.tab = o;
    o = align256(o + tables_len((int)M, c->nx, c->nz) * sizeof(double));
    L.phys = o;
    o = align256(o + sizeof(Phys));
    L.fac = o;  // [kind][mode][row], both operators
    o = align256(o + 2 * (size_t)nspec * sizeof(double2));
    L.spec = o;  // one half spectrum
    o = align256(o + (size_t)nspec * sizeof(double2));
    L.total = o;
    return L;
}

// Every value the tables and pivots depend on.
bool same_grid(const nspnp_config &a, const nspnp_config &b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.lx == b.lx && a.lz == b.lz && a.stretch == b.stretch;
}

}  // namespace

extern "C" int nspnp_poisson_solve_noalloc(const nspnp_config *cfg, int32_t kind, const double *dev_rhs,
                                           double *dev_out, void *hip_stream) {
    int rc = check(cfg);
    if (rc) return rc;
    if (!dev_rhs || !dev_out || (kind != 0 && kind != 1))
        return fail_code(NSPNP_ERR_INVALID, "bad poisson_solve_noalloc arguments");
    const ScratchLayout L = scratch_layout(cfg);
    if (L.total > kScratchBytes)
        return fail_code(NSPNP_ERR_SIZE, "poisson_solve_noalloc: this grid needs " + std::to_string(L.total) +
                                             " bytes of scratch, above the fixed " + std::to_string(kScratchBytes) +
                                             " (use nspnp_poisson_solve with a workspace)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_code(NSPNP_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail_code(NSPNP_ERR_INVALID, "device ordinal beyond 63");
    const hipStream_t stream = (hipStream_t)hip_stream;

    std::lock_guard<std::mutex> lock(g_mu);
    Dev &D = g_dev[dev];
    if (!D.ready) {
        // set-up, once per device with that device current: the device
        // address of this GPU's copy of the array, and host table capacity
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail_code(NSPNP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        D.ptr = (char *)p;
        D.host_tab.reserve(tables_len(kMaxRows, 1024, 1024));
        int lds = 65536;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds <= 0)
            lds = 65536;
        e = prime_x_transform_lds(lds);
        if (e != hipSuccess)
            return fail_code(NSPNP_ERR_HIP, std::string("poisson_solve_noalloc LDS limit: ") + hipGetErrorString(e));
        D.ready = true;
    }

    nspnp_state s;  // host-side view; every device pointer below is inside the scratch
    setup_common(&s, cfg, 1, stream);
    s.fp64 = true;  // caller arrays are FP64 (the state type is not involved)
    s.wsize = 8;
    s.d_phys = (Phys *)(D.ptr + L.phys);
    s.fac = (double2 *)(D.ptr + L.fac);
    s.spec = (double2 *)(D.ptr + L.spec);
    s.clock = nullptr;  // read only by divergence sources
    s.cpv = nullptr;    // (the default mode-solve method keeps no row-order c' table)
    s.mu = nullptr;
    s.host_tables.swap(D.host_tab);
    fill_tables(&s, (double *)(D.ptr + L.tab));  // also sets the device table pointers
    if (!D.have_grid || !same_grid(D.grid, *cfg)) {
        // a new grid: tables, constants and pivots into the scratch; the host
        // tables are the source of an asynchronous copy, so wait for it
        D.have_grid = false;
        e = hipMemcpyAsync(D.ptr + L.tab, s.host_tables.data(), s.host_tables.size() * sizeof(double),
                           hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_phys, &s.ph, sizeof(Phys), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = launch_thomas_factors(&s);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            s.host_tables.swap(D.host_tab);
            return fail_code(NSPNP_ERR_HIP, std::string("poisson_solve_noalloc set-up: ") + hipGetErrorString(e));
        }
        D.grid = *cfg;
        D.have_grid = true;
    }
    s.host_tables.swap(D.host_tab);

    PoissonBatch b{};
    b.ms = 0;
    b.phys = s.d_phys;
    b.nprob = 1;
    b.kind[0] = kind;
    b.src[0] = PoissonSrc{SRC_REAL, dev_rhs, nullptr, nullptr, 0.0, 0.0};
    b.out[0] = dev_out;
    b.out_state[0] = 0;
    e = launch_poisson_batch(&s, b);
    if (e != hipSuccess)
        return fail_code(NSPNP_ERR_HIP, std::string("poisson_solve_noalloc: ") + hipGetErrorString(e));
    return NSPNP_OK;
}
