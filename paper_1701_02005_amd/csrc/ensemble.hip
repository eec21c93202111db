// ensemble.hip -- many independent NS-PNP runs advanced together.
//
// Members with the same grid (nx, ny, nz, lx, lz, stretch, precision, dt
// mode) form a size class.  A class is one batched handle: member m's
// workspace has the single-run layout and starts m * stride bytes after
// member 0, and every kernel takes the member from blockIdx.z, so one launch
// covers all members of a class (per-member Re, Sc, beta, Debye length,
// voltage and dt are read from each member's own workspace).  A whole number
// of Runge-Kutta steps for all classes is captured once into a hipGraph and
// replayed.  Time-mean plane profiles of u, c+ - c- and phi are accumulated
// on the device when statistics are on.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <initializer_list>
#include <sstream>
#include <string>

#include "internal.h"

using namespace nspnp;

struct nspnp_ensemble {
    std::vector<nspnp_state *> classes;
    std::vector<int> cls_of, idx_in;     // member -> class, index inside the class
    std::vector<nspnp_config> cfgs;
    hipStream_t stream = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_sub = 0;                   // substeps per replay (multiple of 3)
    bool graph_stats = false;            // statistics flag at capture time
    int64_t substeps = 0;
    ~nspnp_ensemble() {
        if (graph) hipGraphExecDestroy(graph);
        for (nspnp_state *c : classes) delete c;
    }
};

namespace {

bool same_class(const nspnp_config &a, const nspnp_config &b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.lx == b.lx && a.lz == b.lz && a.stretch == b.stretch &&
           a.precision == b.precision && ((a.dt > 0.0) == (b.dt > 0.0)) && a.implicit_xz == b.implicit_xz;
}

// classes in order of first appearance; returns per-member class ids
std::vector<int> group(const nspnp_config *cfgs, int n, std::vector<int> &first) {
    std::vector<int> cls(n, -1);
    for (int m = 0; m < n; ++m) {
        for (size_t c = 0; c < first.size(); ++c)
            if (same_class(cfgs[first[c]], cfgs[m])) { cls[m] = (int)c; break; }
        if (cls[m] < 0) {
            cls[m] = (int)first.size();
            first.push_back(m);
        }
    }
    return cls;
}

#define E_TRY(expr)                                                                                       \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail_code(NSPNP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int drop_graph(nspnp_ensemble *e) {
    if (e->graph) {
        E_TRY(hipGraphExecDestroy(e->graph));
        e->graph = nullptr;
    }
    return NSPNP_OK;
}

int step_all(nspnp_ensemble *e, int n) {
    for (int it = 0; it < n; ++it)
        for (nspnp_state *c : e->classes) {
            int rc = step_handle(c, 1);
            if (rc) return rc;
        }
    e->substeps += n;
    return NSPNP_OK;
}

int capture(nspnp_ensemble *e, int nsub) {
    int rc = drop_graph(e);
    if (rc) return rc;
    for (nspnp_state *c : e->classes) c->prof.on = false;
    hipGraph_t g;
    E_TRY(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
    rc = step_all(e, nsub);
    hipError_t ec = hipStreamEndCapture(e->stream, &g);
    // the capture pass only recorded the work: undo the host counters
    e->substeps -= nsub;
    for (nspnp_state *c : e->classes) c->substeps -= nsub;
    if (rc) return rc;
    if (ec != hipSuccess) return fail_code(NSPNP_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ec));
    ec = hipGraphInstantiate(&e->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ec != hipSuccess) {
        e->graph = nullptr;
        return fail_code(NSPNP_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ec));
    }
    e->graph_sub = nsub;
    e->graph_stats = e->classes.empty() ? false : e->classes[0]->stats_on;
    return NSPNP_OK;
}

bool valid_member(const nspnp_ensemble *e, int m) { return e && m >= 0 && m < (int)e->cfgs.size(); }

// Health of every member from the last landed copy of the device checks.
int check_members(const nspnp_ensemble *e) {
    for (size_t m = 0; m < e->cfgs.size(); ++m) {
        const nspnp_state *c = e->classes[e->cls_of[m]];
        const int bits = c->host_health ? (int)c->host_health[2 * e->idx_in[m]] : 0;
        if (bits) return health_error(bits, (int)m);
    }
    return NSPNP_OK;
}

// ---- autotuner ----------------------------------------------------------
std::string tune_key(const nspnp_state *c) {
    std::ostringstream k;
    k << "gfx950v6:" << c->cfg.nx << "x" << c->cfg.ny << "x" << c->cfg.nz << ":" << (c->fp64 ? "fp64" : "mixed")
      << ":" << c->nmem << (c->cfg.implicit_xz ? ":ixz" : "");
    return k.str();
}

bool cache_lookup(const char *path, const std::string &key, Tiles &t) {
    if (!path || !*path) return false;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string k;
        Tiles v{};
        if (ls >> k >> v.expl >> v.cn >> v.fftx >> v.fftz >> v.thomas >> v.corr >> v.slab >> v.cnslab && k == key) {
            t = v;
            return true;
        }
    }
    return false;
}

void cache_store(const char *path, const std::string &key, const Tiles &t) {
    if (!path || !*path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << t.expl << " " << t.cn << " " << t.fftx << " " << t.fftz << " " << t.thomas << " " << t.corr
        << " " << t.slab << " " << t.cnslab << "\n";
}

// wall time (ms) of `trial` substeps of one class with its current tiles
int time_class(nspnp_state *c, int trial, float *ms) {
    hipEvent_t a, b;
    E_TRY(hipEventCreate(&a));
    E_TRY(hipEventCreate(&b));
    E_TRY(hipEventRecord(a, c->stream));
    int rc = step_handle(c, trial);
    E_TRY(hipEventRecord(b, c->stream));
    E_TRY(hipEventSynchronize(b));
    E_TRY(hipEventElapsedTime(ms, a, b));
    hipEventDestroy(a);
    hipEventDestroy(b);
    return rc;
}

void tiles_to_ints(const Tiles &t, int32_t *o) {
    o[0] = t.expl; o[1] = t.cn; o[2] = t.fftx; o[3] = t.fftz; o[4] = t.thomas; o[5] = t.corr; o[6] = t.slab;
    o[7] = t.cnslab;
}

// Launch shapes of one handle (a single run or a size class): from the cache
// when its key is there, else by coordinate descent over each shape, timing
// trial substeps per candidate (every trial advances the state; the shapes do
// not change any result).
int tune_handle(nspnp_state *c, const char *cache_path, int trial) {
    const std::string key = tune_key(c);
    Tiles best = c->tiles;
    if (!cache_lookup(cache_path, key, best)) {
        const int cand_expl[] = {64, 128, 256};
        const int cand_cn[] = {64, 128, 256, 512};
        const int cand_fft[] = {512, 1024, 2048};
        const int cand_th[] = {0, 4, 8, 16, 32};  // 0: z transforms and mode solves fused along y
        const int cand_corr[] = {128, 256};
        const int cand_slab[] = {4, 8, 16, 32};
        const int cand_cnslab[] = {0, 16, 32};
        float base_ms = 0.f;
        int rc;
        if ((rc = time_class(c, trial, &base_ms))) return rc;  // warm
        if ((rc = time_class(c, trial, &base_ms))) return rc;
        auto sweep = [&](int *field, const int *cand, int ncand) -> int {
            int keep = *field;
            float keep_ms = base_ms;
            for (int q = 0; q < ncand; ++q) {
                if (cand[q] == keep) continue;
                *field = cand[q];
                float ms = 0.f, ms2 = 0.f;
                int r = time_class(c, trial, &ms);
                if (!r) r = time_class(c, trial, &ms2);
                if (r) return r;
                ms = std::min(ms, ms2);
                if (ms < keep_ms) { keep_ms = ms; keep = cand[q]; }
            }
            *field = keep;
            base_ms = keep_ms;
            return NSPNP_OK;
        };
        if ((rc = sweep(&c->tiles.expl, cand_expl, 3))) return rc;
        if ((rc = sweep(&c->tiles.cn, cand_cn, 4))) return rc;
        if ((rc = sweep(&c->tiles.fftx, cand_fft, 3))) return rc;
        if ((rc = sweep(&c->tiles.fftz, cand_fft, 3))) return rc;
        if ((rc = sweep(&c->tiles.thomas, cand_th, 5))) return rc;
        if ((rc = sweep(&c->tiles.corr, cand_corr, 2))) return rc;
        if ((rc = sweep(&c->tiles.slab, cand_slab, 4))) return rc;
        if ((rc = sweep(&c->tiles.cnslab, cand_cnslab, 3))) return rc;
        best = c->tiles;
        cache_store(cache_path, key, best);
    }
    c->tiles = best;
    return NSPNP_OK;
}

int ensemble_advance(nspnp_ensemble *e, int32_t n_substeps);

}  // namespace

extern "C" {

size_t nspnp_ensemble_workspace_bytes(const nspnp_config *cfgs, int32_t n) {
    if (!cfgs || n <= 0) {
        fail_code(NSPNP_ERR_INVALID, "no members");
        return 0;
    }
    size_t total = 0;
    for (int m = 0; m < n; ++m) {
        if (check(&cfgs[m]) != NSPNP_OK) return 0;
        total += layout_bytes(&cfgs[m]);
    }
    return total;
}

int nspnp_ensemble_init(const nspnp_config *cfgs, int32_t n, void *dev_workspace, size_t bytes, void *hip_stream,
                        nspnp_ensemble **out) {
    if (!out) return fail_code(NSPNP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    const size_t need = nspnp_ensemble_workspace_bytes(cfgs, n);
    if (need == 0) return NSPNP_ERR_INVALID;
    if (!dev_workspace || bytes < need) return fail_code(NSPNP_ERR_WORKSPACE, "ensemble workspace too small");
    if (((uintptr_t)dev_workspace & 255) != 0) return fail_code(NSPNP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    nspnp_ensemble *e = new nspnp_ensemble();
    e->stream = (hipStream_t)hip_stream;
    e->cfgs.assign(cfgs, cfgs + n);
    std::vector<int> first;
    e->cls_of = group(cfgs, n, first);
    e->idx_in.assign(n, 0);
    std::vector<int> count(first.size(), 0);
    for (int m = 0; m < n; ++m) e->idx_in[m] = count[e->cls_of[m]]++;
    // class c occupies count[c] consecutive member workspaces
    char *base = (char *)dev_workspace;
    for (size_t c = 0; c < first.size(); ++c) {
        nspnp_state *h = new nspnp_state();
        setup_handle(h, &cfgs[first[c]], base, count[c], e->stream);
        e->classes.push_back(h);
        base += (size_t)count[c] * layout_bytes(&cfgs[first[c]]);
        int rc = alloc_host_health(h);
        if (!rc) rc = upload_tables(h);
        if (rc) { delete e; return rc; }
    }
    for (int m = 0; m < n; ++m) {
        nspnp_state *v = member_view(e->classes[e->cls_of[m]], e->idx_in[m], &cfgs[m]);
        int rc = init_member(v);
        delete v;
        if (rc) { delete e; return rc; }
    }
    hipError_t err = hipStreamSynchronize(e->stream);
    if (err != hipSuccess) {
        delete e;
        return fail_code(NSPNP_ERR_HIP, std::string("ensemble init: ") + hipGetErrorString(err));
    }
    *out = e;
    return NSPNP_OK;
}

int nspnp_ensemble_step(nspnp_ensemble *e, int32_t n_substeps) {
    if (!e || n_substeps < 0) return fail_code(NSPNP_ERR_INVALID, "bad ensemble step arguments");
    int rc0 = check_members(e);
    if (rc0) return rc0;
    rc0 = ensemble_advance(e, n_substeps);
    if (rc0 || n_substeps == 0) return rc0;
    for (nspnp_state *c : e->classes)
        if ((rc0 = queue_health_copy(c))) return rc0;
    return NSPNP_OK;
}

int nspnp_ensemble_sync(nspnp_ensemble *e) {
    if (!e) return fail_code(NSPNP_ERR_INVALID, "ensemble is NULL");
    E_TRY(hipStreamSynchronize(e->stream));
    return check_members(e);
}

}  // extern "C"

namespace {
int ensemble_advance(nspnp_ensemble *e, int32_t n_substeps) {
    int left = n_substeps;
    const bool stats = e->classes[0]->stats_on;
    if (e->graph && e->graph_stats != stats) {
        int rc = drop_graph(e);
        if (rc) return rc;
    }
    while (e->graph && left >= e->graph_sub && e->substeps % 3 == 0) {
        E_TRY(hipGraphLaunch(e->graph, e->stream));
        left -= e->graph_sub;
        e->substeps += e->graph_sub;
        for (nspnp_state *c : e->classes) c->substeps += e->graph_sub;
    }
    return step_all(e, left);
}
}  // namespace

extern "C" {

int nspnp_ensemble_capture(nspnp_ensemble *e, int32_t substeps_per_replay) {
    if (!e || substeps_per_replay <= 0 || substeps_per_replay % 3 != 0)
        return fail_code(NSPNP_ERR_INVALID, "graph length must be a positive multiple of 3 substeps");
    if (e->substeps % 3 != 0) return fail_code(NSPNP_ERR_INVALID, "capture at the start of a Runge-Kutta step");
    return capture(e, substeps_per_replay);
}

int nspnp_ensemble_stats(nspnp_ensemble *e, int32_t on) {
    if (!e) return fail_code(NSPNP_ERR_INVALID, "ensemble is NULL");
    for (nspnp_state *c : e->classes) {
        if (on) E_TRY(launch_stats_reset(c));
        c->stats_on = on != 0;
    }
    return NSPNP_OK;
}

int nspnp_ensemble_profiles(nspnp_ensemble *e, int32_t member, double *u, double *rho, double *phi,
                            double *time_weight) {
    if (!valid_member(e, member) || !u || !rho || !phi || !time_weight)
        return fail_code(NSPNP_ERR_INVALID, "bad profiles arguments");
    nspnp_state *c = e->classes[e->cls_of[member]];
    const int M = c->d.M;
    std::vector<double> h(3 * M + 2);
    const double *src = (const double *)((const char *)c->stats + (size_t)e->idx_in[member] * c->mstride);
    E_TRY(hipMemcpyAsync(h.data(), src, h.size() * sizeof(double), hipMemcpyDeviceToHost, e->stream));
    E_TRY(hipStreamSynchronize(e->stream));
    const double wt = h[3 * M];
    *time_weight = wt;
    for (int j = 0; j < M; ++j) {
        u[j] = wt > 0 ? h[3 * j] / wt : 0.0;
        rho[j] = wt > 0 ? h[3 * j + 1] / wt : 0.0;
        phi[j] = wt > 0 ? h[3 * j + 2] / wt : 0.0;
    }
    return NSPNP_OK;
}

// member view helpers: the single-run calls on one member
#define WITH_VIEW(e, member, call)                                                                   \
    do {                                                                                             \
        if (!valid_member(e, member)) return fail_code(NSPNP_ERR_INVALID, "member out of range");    \
        nspnp_state *v_ = member_view(e->classes[e->cls_of[member]], e->idx_in[member], &e->cfgs[member]); \
        v_->substeps = e->classes[e->cls_of[member]]->substeps;                                       \
        int rc_ = (call);                                                                            \
        delete v_;                                                                                   \
        return rc_;                                                                                  \
    } while (0)

int nspnp_ensemble_get_field(nspnp_ensemble *e, int32_t member, int32_t field, double *dev_out) {
    WITH_VIEW(e, member, nspnp_get_field(v_, field, dev_out));
}

int nspnp_ensemble_set_field(nspnp_ensemble *e, int32_t member, int32_t field, const double *dev_in) {
    WITH_VIEW(e, member, nspnp_set_field(v_, field, dev_in));
}

int nspnp_ensemble_diagnostics(nspnp_ensemble *e, int32_t member, double out[6]) {
    WITH_VIEW(e, member, nspnp_diagnostics(v_, out));
}

int nspnp_ensemble_refresh_potential(nspnp_ensemble *e, int32_t member) {
    WITH_VIEW(e, member, nspnp_refresh_potential(v_));
}

int nspnp_ensemble_wall_shear_stress(nspnp_ensemble *e, int32_t member, double *tau_bottom, double *tau_top) {
    WITH_VIEW(e, member, nspnp_wall_shear_stress(v_, tau_bottom, tau_top));
}

int nspnp_ensemble_ion_flux(nspnp_ensemble *e, int32_t member, double *jp, double *jm, double *mp, double *mm) {
    WITH_VIEW(e, member, nspnp_ion_flux(v_, jp, jm, mp, mm));
}

int nspnp_ensemble_clock(nspnp_ensemble *e, int32_t member, double *t, double *dt, int64_t *substeps) {
    WITH_VIEW(e, member, nspnp_get_clock(v_, t, dt, nullptr, substeps));
}

int nspnp_ensemble_autotune(nspnp_ensemble *e, const char *cache_path, int32_t trial_substeps, int32_t *tiles_out) {
    if (!e || trial_substeps <= 0 || trial_substeps % 3 != 0)
        return fail_code(NSPNP_ERR_INVALID, "trial length must be a positive multiple of 3 substeps");
    int rc = drop_graph(e);
    if (rc) return rc;
    for (size_t ci = 0; ci < e->classes.size(); ++ci) {
        if ((rc = tune_handle(e->classes[ci], cache_path, trial_substeps))) return rc;
        if (tiles_out) tiles_to_ints(e->classes[ci]->tiles, tiles_out + kTileInts * ci);
    }
    // classes may have advanced by different numbers of trial substeps
    int64_t mx = 0;
    for (nspnp_state *c : e->classes) mx = std::max<int64_t>(mx, c->substeps);
    for (nspnp_state *c : e->classes) {
        if (c->substeps < mx && (rc = step_handle(c, (int)(mx - c->substeps)))) return rc;
    }
    e->substeps = mx;
    E_TRY(hipStreamSynchronize(e->stream));
    return NSPNP_OK;
}

int nspnp_get_tiles(const nspnp_state *s, int32_t *tiles_out) {
    if (!s || !tiles_out) return fail_code(NSPNP_ERR_INVALID, "bad get_tiles arguments");
    tiles_to_ints(s->tiles, tiles_out);
    return NSPNP_OK;
}

int nspnp_set_tiles(nspnp_state *s, const int32_t *t) {
    if (!s || !t) return fail_code(NSPNP_ERR_INVALID, "bad set_tiles arguments");
    auto one_of = [](int v, std::initializer_list<int> ok) {
        for (int o : ok)
            if (v == o) return true;
        return false;
    };
    if (!one_of(t[0], {64, 128, 256}) || !one_of(t[1], {64, 128, 256, 512}) || t[2] < 64 || t[2] > 8192 ||
        t[3] < 64 || t[3] > 8192 || t[4] < 0 || t[4] > 64 || !one_of(t[5], {64, 128, 256}) ||
        t[6] < 1 || t[6] > kMaxRows || !one_of(t[7], {0, 16, 32}))
        return fail_code(NSPNP_ERR_INVALID, "launch shapes out of range");
    E_TRY(hipStreamSynchronize(s->stream));
    s->tiles = Tiles{t[0], t[1], t[2], t[3], t[4], t[5], t[6], t[7]};
    return NSPNP_OK;
}

int nspnp_autotune(nspnp_state *s, const char *cache_path, int32_t trial_substeps, int32_t *tiles_out) {
    if (!s || trial_substeps <= 0 || trial_substeps % 3 != 0)
        return fail_code(NSPNP_ERR_INVALID, "trial length must be a positive multiple of 3 substeps");
    int rc = check_health(s, -1);
    if (rc) return rc;
    if ((rc = tune_handle(s, cache_path, trial_substeps))) return rc;
    if (tiles_out) tiles_to_ints(s->tiles, tiles_out);
    E_TRY(hipStreamSynchronize(s->stream));
    return NSPNP_OK;
}

int32_t nspnp_ensemble_classes(const nspnp_ensemble *e) { return e ? (int32_t)e->classes.size() : 0; }

void nspnp_ensemble_destroy(nspnp_ensemble *e) {
    if (e && e->stream) hipStreamSynchronize(e->stream);
    delete e;
}

}  // extern "C"
