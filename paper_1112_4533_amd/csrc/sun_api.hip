// sun_api.hip -- the C ABI of libsun (declared in include/sun.h): argument
// checks, lattice handles, the phase schedule of a sweep, reductions and
// per-kernel event timing.  All device work is done by the kernels of
// sun_kernels.hpp; this file only validates and launches.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sun.h"
#include "sun_host.hpp"
#include "sun_kernels.hpp"
#include "sun_ops.hpp"

using namespace sun_host;

namespace {

constexpr int kKernels = 5;  // heatbath, overrelaxation, reunit, plaquette, polyakov

}  // namespace

struct sun_lattice_s {
    int nc = 0;
    int dtype = 0;
    sun::Geom g{};
    void* links = nullptr;
    double* scratch = nullptr;
    uint64_t step = 0;
    const sun::Ops* ops = nullptr;
    // event timing
    bool profiling = false;
    int profile_every = 1;           // record one launch in this many per kernel kind
    bool profile_runs = false;       // bracket runs of consecutive launches of one kind instead
    bool in_run = false;             // a run bracket is open: launches are not bracketed singly
    int64_t seen[kKernels] = {};     // launches issued since profiling started
    struct Pending {
        int kernel;
        hipEvent_t a, b;
        int count;                   // launches between the two events
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[kKernels] = {};
    int64_t launches[kKernels] = {};
    // launch shapes of the phase kernels (sun_set_launch); the overrelaxation
    // cap is set at creation from the link size
    sun::Shape shape[2] = {sun::Shape{256, 1, 16, 4}, sun::Shape{256, 1, 12, 4}};

    size_t link_bytes = 0;
    uint64_t phases_run = 0;  // alternates the walk direction of successive phases
    uint64_t tile_order = 0;  // sun_set_tile_order: random tile orders (race check), 0 = off
    // watchdog (sun_watchdog): threshold > 0 arms a check in every
    // re-unitarization; its state (3 doubles) sits in the last 256 bytes of
    // the scratch buffer
    double watch_threshold = 0.0;
    double* watch_state = nullptr;
    bool watch_reset = false;  // the state has been cleared by sun_watchdog
    sun::Ctx ctx(hipStream_t s) const {
        return sun::Ctx{links, g, s, {shape[0], shape[1]}, nc, link_bytes > sun::kPlainAccessMaxBytes ? 1 : 0, 0};
    }
};

namespace {

size_t link_bytes_of(int nc, const sun::Geom& g, int dtype) {
    const size_t rows = is_two_row(dtype) ? 2 : (size_t)nc;
    const size_t reals = (nc == 2) ? 4 : 2 * rows * nc;
    return reals * 4 * (size_t)g.V * (is_f64(dtype) ? 8 : 4);
}

// Bytes of the reduction partials: the largest partial array, per link
// block, per plaquette tile, or per Polyakov workgroup (at least 32 spatial
// sites each); the wide path reduces per link.
size_t partial_bytes_of(const sun::Geom& g, bool wide) {
    const int nblk = wide ? 4 * g.V
                          : std::max({sun::link_blocks(g), sun::plaquette_tiles(g), (g.V / g.L[3] + 31) / 32});
    const size_t b = 2 * sizeof(double) * (size_t)nblk;
    return (b + 255) & ~(size_t)255;
}

// The partials, then 256 bytes of watchdog state.
constexpr size_t kWatchBytes = 256;
size_t scratch_bytes_of(const sun::Geom& g, bool wide) { return partial_bytes_of(g, wide) + kWatchBytes; }

// kind: SUN_HEATBATH, SUN_OVERRELAX, or -1 for both.
int check_shape(int kind, int block, int waves, int tblock = 0) {
    if (kind < -1 || kind > 1) return fail(SUN_EINVAL, "kind %d is not -1, SUN_HEATBATH or SUN_OVERRELAX", kind);
    if (!sun::valid_phase_block(block)) return fail(SUN_EINVAL, "block %d is not 64, 128 or 256", block);
    if (!sun::valid_wave_cap(waves)) return fail(SUN_EINVAL, "wave cap %d is not 0, 8, 12 or 16", waves);
    if (!sun::valid_tblock(tblock)) return fail(SUN_EINVAL, "time block %d is not 0, 1, 2, 4 or 8", tblock);
    return SUN_OK;
}

// Records an event pair around one launch when profiling is on, or, with
// run_launches > 0, around a run of that many launches of kernel kind k (only
// in the run-timing mode; launches inside an open run are not bracketed).
struct Timed {
    sun_lattice_s* h;
    int kernel;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    int rc = SUN_OK;
    bool on = false;
    int count = 1;
    Timed(sun_lattice_s* h_, int k, hipStream_t s_, int run_launches = 0)
        : h(h_), kernel(k), s(s_), count(run_launches > 0 ? run_launches : 1) {
        if (!h->profiling) return;
        if (run_launches > 0) {
            if (!h->profile_runs) return;
        } else {
            if (h->in_run) return;
            if (!h->profile_runs && h->seen[k]++ % h->profile_every != 0) return;
        }
        on = true;
        for (hipEvent_t* e : {&a, &b}) {
            if (!h->pool.empty()) {
                *e = h->pool.back();
                h->pool.pop_back();
            } else if ((rc = hip_check(hipEventCreate(e), "hipEventCreate")) != SUN_OK) {
                return;
            }
        }
        rc = hip_check(hipEventRecord(a, s), "hipEventRecord");
    }
    int done() {
        if (!on || rc != SUN_OK) return rc;
        rc = hip_check(hipEventRecord(b, s), "hipEventRecord");
        if (rc == SUN_OK) h->pending.push_back({kernel, a, b, count});
        return rc;
    }
};

}  // namespace

extern "C" {

const char* sun_last_error(void) { return last_error.c_str(); }

int sun_lattice_bytes(int nc, const int L[4], int dtype, size_t* link_bytes, size_t* scratch_bytes) {
    if (int rc = check_lattice(nc, L, dtype)) return rc;
    const sun::Geom g = make_geom(L);
    if (link_bytes) *link_bytes = link_bytes_of(nc, g, dtype);
    if (scratch_bytes) *scratch_bytes = scratch_bytes_of(g, is_wide(nc, dtype));
    return SUN_OK;
}

int sun_lattice_create(int nc, const int L[4], int dtype, void* links, size_t link_bytes, void* scratch,
                       size_t scratch_bytes, sun_lattice_t* out) {
    if (!out) return fail(SUN_EINVAL, "out is null");
    *out = nullptr;
    if (int rc = check_lattice(nc, L, dtype)) return rc;
    const sun::Geom g = make_geom(L);
    if (!links || link_bytes < link_bytes_of(nc, g, dtype))
        return fail(SUN_ESIZE, "link buffer %p of %zu bytes, need %zu", links, link_bytes, link_bytes_of(nc, g, dtype));
    const size_t need_scratch = scratch_bytes_of(g, is_wide(nc, dtype));
    if (!scratch || scratch_bytes < need_scratch)
        return fail(SUN_ESIZE, "scratch buffer %p of %zu bytes, need %zu", scratch, scratch_bytes, need_scratch);
    if (((uintptr_t)links & 255) || ((uintptr_t)scratch & 255))
        return fail(SUN_EINVAL, "buffers must be 256-byte aligned");
    auto* h = new sun_lattice_s;
    h->nc = nc;
    h->dtype = dtype;
    h->g = g;
    h->links = links;
    h->link_bytes = link_bytes_of(nc, g, dtype);
    // Default wave caps, from launch-shape sweeps on SU(3) 32^4: the heatbath
    // runs best with 16 resident waves per CU whatever the storage; the
    // overrelaxation kernel with 12 for 48-byte links (FP32 two-row) and 8
    // for larger ones (18-real FP32: 70.0 -> 67.3 us, FP64: 161 -> 152 us).
    h->shape[SUN_OVERRELAX].waves = h->link_bytes / (4 * (size_t)g.V) > 48 ? 8 : 12;
    // On large lattices the heatbath takes two tiles per workgroup (SU(3)
    // 32^4 sweep: two-row 2.040 -> 2.004 ms, 18 reals 3.156 -> 3.151 ms, FP64
    // two-row 4.378 -> 4.356 ms); where that would leave fewer than 1024
    // workgroups (4 per CU) it takes one (SU(4) 12^4: 41 tiles; two per
    // workgroup cost 40% there).
    if (sun::half_blocks(g, 256) >= 2 * 1024) h->shape[SUN_HEATBATH].spt = 2;
    h->scratch = static_cast<double*>(scratch);
    h->watch_state = reinterpret_cast<double*>(static_cast<char*>(scratch) + partial_bytes_of(g, is_wide(nc, dtype)));
    h->ops = ops_for(nc, dtype);
    *out = h;
    return SUN_OK;
}

void sun_lattice_destroy(sun_lattice_t h) {
    if (!h) return;
    for (auto& p : h->pending) {
        (void)hipEventSynchronize(p.b);
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    delete h;
}

int sun_init(sun_lattice_t h, int hot, uint64_t seed, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    h->ops->init(h->ctx(as_stream(stream)), hot ? 1 : 0, (uint32_t)seed, (uint32_t)(seed >> 32));
    h->step = 0;
    return launch_check("init");
}

static int run_phase(sun_lattice_t h, int kind, int mu, int parity, double beta, uint64_t seed, uint64_t step,
                     hipStream_t s) {
    if (!((h->g.present >> mu) & 1)) return SUN_OK;  // absent direction: nothing to update
    Timed t(h, kind == SUN_HEATBATH ? 0 : 1, s);
    if (t.rc) return t.rc;
    sun::Ctx c = h->ctx(s);
    // a fresh random order per phase, from the handle's seed and the phase count
    if (h->tile_order) c.order = h->tile_order ^ (0xD1B54A32D192ED03ull * (h->phases_run + 1));
    c.rev = (int)(h->phases_run++ & 1);
    h->ops->update(c, kind, mu, parity, beta, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)step);
    if (int rc = launch_check(kind == SUN_HEATBATH ? "heatbath phase" : "overrelaxation phase")) return rc;
    return t.done();
}

int sun_phase(sun_lattice_t h, int kind, int mu, int parity, double beta, uint64_t seed, uint64_t step,
              sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (kind != SUN_HEATBATH && kind != SUN_OVERRELAX) return fail(SUN_EINVAL, "kind %d", kind);
    if (mu < 0 || mu > 3) return fail(SUN_EINVAL, "mu %d", mu);
    if (parity != 0 && parity != 1) return fail(SUN_EINVAL, "parity %d", parity);
    return run_phase(h, kind, mu, parity, beta, seed, step, as_stream(stream));
}

// Watchdog pass over the unitarity partials of h's scratch, if armed.
static void watch_partials(sun_lattice_t h, int nblk, hipStream_t s) {
    sun::k_watchdog<><<<1, sun::kBlock, 0, s>>>(h->scratch, nblk, h->watch_threshold, h->watch_state);
}

static int run_reunit(sun_lattice_t h, double* dev_out2, hipStream_t s) {
    Timed t(h, 2, s);
    if (t.rc) return t.rc;
    const bool watch = h->watch_threshold > 0.0;
    const int nblk = h->ops->reunit(h->ctx(s), (dev_out2 || watch) ? h->scratch : nullptr);
    if (dev_out2) sun::launch_finalize_max2(h->scratch, nblk, dev_out2, s);
    if (watch) watch_partials(h, nblk, s);
    if (int rc = launch_check("reunitarize")) return rc;
    return t.done();
}

int sun_sweep(sun_lattice_t h, double beta, int n_hb, int n_or, uint64_t seed, int reunit, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (n_hb < 0 || n_or < 0) return fail(SUN_EINVAL, "negative step count (n_hb %d, n_or %d)", n_hb, n_or);
    const hipStream_t s = as_stream(stream);
    int present = 0;
    for (int mu = 0; mu < 4; ++mu) present += (h->g.present >> mu) & 1;
    // the heatbath phases, then the overrelaxation phases, each a run of
    // consecutive launches of one kernel kind (bracketed as a whole in the
    // run-timing mode of sun_profile)
    for (int kind : {SUN_HEATBATH, SUN_OVERRELAX}) {
        const int steps = kind == SUN_HEATBATH ? n_hb : n_or;
        if (steps == 0) continue;
        Timed run(h, kind == SUN_HEATBATH ? 0 : 1, s, steps * 2 * present);
        if (run.rc) return run.rc;
        h->in_run = run.on;
        for (int k = 0; k < steps; ++k)
            for (int mu = 0; mu < 4; ++mu)
                for (int p = 0; p < 2; ++p)
                    if (int rc = run_phase(h, kind, mu, p, beta, seed,
                                           kind == SUN_HEATBATH ? h->step + (uint64_t)k : 0, s)) {
                        h->in_run = false;
                        return rc;
                    }
        h->in_run = false;
        if (int rc = run.done()) return rc;
    }
    if (reunit)
        if (int rc = run_reunit(h, nullptr, s)) return rc;
    h->step += (uint64_t)n_hb;
    return SUN_OK;
}

int sun_reunitarize(sun_lattice_t h, double* dev_out2, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    return run_reunit(h, dev_out2, as_stream(stream));
}

int sun_plaquette(sun_lattice_t h, double* dev_out3, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (!dev_out3) return fail(SUN_ESIZE, "dev_out3 is null");
    const hipStream_t s = as_stream(stream);
    Timed t(h, 3, s);
    if (t.rc) return t.rc;
    launch_plaquette(h->ops, h->ctx(s), h->scratch, dev_out3);
    if (int rc = launch_check("plaquette")) return rc;
    return t.done();
}

int sun_polyakov(sun_lattice_t h, double* dev_out2, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (!dev_out2) return fail(SUN_ESIZE, "dev_out2 is null");
    const hipStream_t s = as_stream(stream);
    Timed t(h, 4, s);
    if (t.rc) return t.rc;
    const double Vs = (double)(h->g.V / h->g.L[3]);
    const int nblk = h->ops->polyakov(h->ctx(s), h->scratch);
    sun::launch_finalize_sum2(h->scratch, nblk, dev_out2, 1.0 / (h->nc * Vs), s);
    if (int rc = launch_check("polyakov")) return rc;
    return t.done();
}

int sun_unitarity(sun_lattice_t h, double* dev_out2, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (!dev_out2) return fail(SUN_ESIZE, "dev_out2 is null");
    const hipStream_t s = as_stream(stream);
    const int nblk = h->ops->unitarity(h->ctx(s), h->scratch);
    sun::launch_finalize_max2(h->scratch, nblk, dev_out2, s);
    return launch_check("unitarity");
}

int sun_watchdog(sun_lattice_t h, double threshold, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (!(threshold >= 0.0) || threshold == __builtin_inf())
        return fail(SUN_EINVAL, "watchdog threshold %g is not finite and >= 0", threshold);
    h->watch_threshold = threshold;
    sun::k_fill<><<<1, 64, 0, as_stream(stream)>>>(h->watch_state, 3, 0.0);
    if (int rc = launch_check("watchdog reset")) return rc;
    h->watch_reset = true;
    return SUN_OK;
}

int sun_check(sun_lattice_t h, double* deviation, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (!h->watch_reset) return fail(SUN_EINVAL, "the watchdog was never set (call sun_watchdog first)");
    const hipStream_t s = as_stream(stream);
    double st[3] = {0.0, 0.0, 0.0};
    if (int rc = hip_check(hipMemcpyAsync(st, h->watch_state, sizeof st, hipMemcpyDeviceToHost, s), "watchdog read"))
        return rc;
    if (int rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize")) return rc;
    if (deviation) *deviation = st[1];
    if (st[0] > 0.0)
        return fail(SUN_ENUMERIC,
                    "watchdog: %.0f check(s) found a unitarity or determinant deviation above %g (largest %g; "
                    "a NaN or infinite entry counts as infinite)",
                    st[0], h->watch_threshold, st[1]);
    return SUN_OK;
}

int sun_export(sun_lattice_t h, double* dev_canonical, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (!dev_canonical) return fail(SUN_ESIZE, "dev_canonical is null");
    h->ops->export_field(h->ctx(as_stream(stream)), dev_canonical);
    return launch_check("export");
}

int sun_import(sun_lattice_t h, const double* dev_canonical, sun_stream_t stream) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (!dev_canonical) return fail(SUN_ESIZE, "dev_canonical is null");
    h->ops->import_field(h->ctx(as_stream(stream)), dev_canonical);
    return launch_check("import");
}

int sun_get_step(sun_lattice_t h, uint64_t* step) {
    if (!h || !step) return fail(SUN_EINVAL, "null argument");
    *step = h->step;
    return SUN_OK;
}

int sun_set_step(sun_lattice_t h, uint64_t step) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    h->step = step;
    return SUN_OK;
}

int sun_set_launch(sun_lattice_t h, int kind, int block, int xcd, int waves, int tblock) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (int rc = check_shape(kind, block, waves, tblock)) return rc;
    for (int k = 0; k < 2; ++k)
        if (kind < 0 || kind == k)
            h->shape[k] = sun::Shape{block, xcd ? 1 : 0, waves, tblock > 1 ? tblock : 0, h->shape[k].spt};
    return SUN_OK;
}

int sun_set_tile_order(sun_lattice_t h, uint64_t seed) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    h->tile_order = seed;
    return SUN_OK;
}

int sun_set_sites_per_item(sun_lattice_t h, int kind, int spt) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (kind < -1 || kind > 1) return fail(SUN_EINVAL, "kind %d is not -1, SUN_HEATBATH or SUN_OVERRELAX", kind);
    if (!sun::valid_spt(spt)) return fail(SUN_EINVAL, "sites per work-item %d is not 1, 2 or 4", spt);
    for (int k = 0; k < 2; ++k)
        if (kind < 0 || kind == k) h->shape[k].spt = spt;
    return SUN_OK;
}

int sun_get_sites_per_item(sun_lattice_t h, int kind, int* spt) {
    if (!h || !spt) return fail(SUN_EINVAL, "null argument");
    if (kind != SUN_HEATBATH && kind != SUN_OVERRELAX) return fail(SUN_EINVAL, "kind %d", kind);
    *spt = h->shape[kind].spt;
    return SUN_OK;
}

int sun_get_launch(sun_lattice_t h, int kind, int* block, int* xcd, int* waves, int* tblock) {
    if (!h || !block || !xcd || !waves || !tblock) return fail(SUN_EINVAL, "null argument");
    if (kind != SUN_HEATBATH && kind != SUN_OVERRELAX) return fail(SUN_EINVAL, "kind %d", kind);
    *block = h->shape[kind].block;
    *xcd = h->shape[kind].xcd;
    *waves = h->shape[kind].waves;
    *tblock = sun::walk_for(h->g, h->shape[kind]).tb;
    return SUN_OK;
}

int sun_profile(sun_lattice_t h, int every) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (every < -1) return fail(SUN_EINVAL, "profile sampling period %d", every);
    for (auto& p : h->pending) {
        if (int rc = hip_check(hipEventSynchronize(p.b), "hipEventSynchronize")) return rc;
        h->pool.push_back(p.a);
        h->pool.push_back(p.b);
    }
    h->pending.clear();
    for (int k = 0; k < kKernels; ++k) {
        h->total_ms[k] = 0.0;
        h->launches[k] = 0;
        h->seen[k] = 0;
    }
    h->profiling = every != 0;
    h->profile_runs = every == -1;
    h->profile_every = every > 0 ? every : 1;
    return SUN_OK;
}

int sun_profile_read(sun_lattice_t h, int kernel, double* total_ms, int64_t* launches) {
    if (!h) return fail(SUN_EINVAL, "null handle");
    if (kernel < 0 || kernel >= kKernels) return fail(SUN_EINVAL, "kernel id %d", kernel);
    for (auto& p : h->pending) {
        if (int rc = hip_check(hipEventSynchronize(p.b), "hipEventSynchronize")) return rc;
        float ms = 0.0f;
        if (int rc = hip_check(hipEventElapsedTime(&ms, p.a, p.b), "hipEventElapsedTime")) return rc;
        h->total_ms[p.kernel] += ms;
        h->launches[p.kernel] += p.count;
        h->pool.push_back(p.a);
        h->pool.push_back(p.b);
    }
    h->pending.clear();
    if (total_ms) *total_ms = h->total_ms[kernel];
    if (launches) *launches = h->launches[kernel];
    return SUN_OK;
}

int sun_sample_su2(int dtype, const double* dev_alpha, int n, uint64_t seed, uint32_t step, uint32_t mu_sg,
                   double* dev_x, int* dev_attempts, sun_stream_t stream) {
    if (dtype != SUN_F32 && dtype != SUN_F64 && dtype != SUN_F32_WIDE && dtype != SUN_F64_WIDE)
        return fail(SUN_EINVAL, "dtype %d", dtype);
    if (n < 0) return fail(SUN_EINVAL, "n = %d", n);
    if (n == 0) return SUN_OK;
    if (!dev_alpha || !dev_x || !dev_attempts) return fail(SUN_ESIZE, "null buffer");
    if (dtype == SUN_F32_WIDE || dtype == SUN_F64_WIDE)
        sun::launch_sample_su2_batched(is_f64(dtype), dev_alpha, n, (uint32_t)seed, (uint32_t)(seed >> 32), step,
                                       mu_sg, dev_x, dev_attempts, as_stream(stream));
    else
        sun::launch_sample_su2(dtype == SUN_F64, dev_alpha, n, (uint32_t)seed, (uint32_t)(seed >> 32), step, mu_sg,
                               dev_x, dev_attempts, as_stream(stream));
    return launch_check("sample_su2");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent chains.
// ---------------------------------------------------------------------------
struct sun_batch_s {
    struct Group {
        const sun::Ops* ops;
        int first, count;      // range of the device table
        int tiles[5];          // total tiles per grid kind (see TileKind)
        int nc;
        bool wide;             // workgroup-per-link path: tiles count links / sites, one workgroup each
    };
    std::vector<sun_lattice_t> chains;  // in the caller's order
    std::vector<Group> groups;
    std::vector<sun::ChainDesc> host;   // host copy of the table
    sun::ChainDesc* table = nullptr;    // device
    // per update kind; a batch's chains are small and mostly cache-resident,
    // so no wave cap (the launch-shape tuner's choice for the 64-chain batch:
    // 1.10e10 -> 1.13e10 link updates/s against a 12-wave overrelaxation cap)
    sun::Shape shape[2] = {sun::Shape{256, 1, 0}, sun::Shape{256, 1, 0}};
    uint64_t hb_steps_done = 0;         // heatbath steps run since creation (all chains alike)
    std::vector<uint64_t> step0;        // chain step counters at creation
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t hb_per_replay = 0;
};

// Couplings of a batch sweep from a device array in the caller's chain
// order: d[c].beta = beta[d[c].out_index].  Runs on the stream ahead of the
// sweep's phases, so a captured graph reads the array's contents at replay.
__global__ void k_set_betas(sun::ChainDesc* __restrict__ d, int n, const double* __restrict__ beta) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) d[c].beta = beta[d[c].out_index];
}

namespace {

int batch_sweep_launches(sun_batch_t b, int n_hb, int n_or, int reunit, const double* dev_beta, hipStream_t s) {
    if (dev_beta) {
        const int n = (int)b->chains.size();
        k_set_betas<<<(n + 63) / 64, 64, 0, s>>>(b->table, n, dev_beta);
    }
    for (const auto& gr : b->groups) {
        const sun::ChainDesc* d = b->table + gr.first;
        for (int k = 0; k < n_hb; ++k)
            for (int mu = 0; mu < 4; ++mu)
                for (int p = 0; p < 2; ++p)
                    gr.ops->update_batch(d, gr.count, gr.tiles[sun::TILE_HALF_HB], SUN_HEATBATH, mu, p, (uint32_t)k,
                                         b->shape[SUN_HEATBATH], gr.nc, s);
        for (int k = 0; k < n_or; ++k)
            for (int mu = 0; mu < 4; ++mu)
                for (int p = 0; p < 2; ++p)
                    gr.ops->update_batch(d, gr.count, gr.tiles[sun::TILE_HALF_OR], SUN_OVERRELAX, mu, p, 0,
                                         b->shape[SUN_OVERRELAX], gr.nc, s);
        if (reunit) gr.ops->reunit_batch(d, gr.count, gr.tiles[sun::TILE_LINK], gr.nc, s);
    }
    if (n_hb > 0) sun::launch_advance_steps(b->table, (int)b->chains.size(), n_hb, s);
    return launch_check("batch sweep");
}

// Assigns every chain its first tile in each grid kind (the phase grid in
// tiles of the batch's block size) and uploads the table.  Synchronous.
int upload_table(sun_batch_t b) {
    for (auto& gr : b->groups) {
        int t[5] = {0, 0, 0, 0, 0};
        for (int i = gr.first; i < gr.first + gr.count; ++i) {
            sun::ChainDesc& c = b->host[i];
            for (int k = 0; k < 5; ++k) c.tile0[k] = t[k];
            if (gr.wide) {  // one workgroup per updated link, per site, per link
                t[sun::TILE_HALF_HB] += c.g.Vh;
                t[sun::TILE_SITE] += c.g.V;
                t[sun::TILE_LINK] += 4 * c.g.V;
                t[sun::TILE_SPATIAL] += c.g.V / c.g.L[3];
                t[sun::TILE_HALF_OR] += c.g.Vh;
                continue;
            }
            t[sun::TILE_HALF_HB] += sun::half_blocks(c.g, b->shape[SUN_HEATBATH].block);
            t[sun::TILE_SITE] += sun::plaquette_tiles(c.g);
            t[sun::TILE_LINK] += sun::link_blocks(c.g);
            t[sun::TILE_SPATIAL] += sun::spatial_blocks(c.g);
            t[sun::TILE_HALF_OR] += sun::half_blocks(c.g, b->shape[SUN_OVERRELAX].block);
        }
        for (int k = 0; k < 5; ++k) gr.tiles[k] = t[k];
    }
    return hip_check(hipMemcpy(b->table, b->host.data(), sizeof(sun::ChainDesc) * b->host.size(),
                               hipMemcpyHostToDevice),
                     "batch table upload");
}

int batch_plaquette_launches(sun_batch_t b, double* out, hipStream_t s) {
    for (const auto& gr : b->groups)
        gr.ops->plaquette_batch(b->table + gr.first, gr.count, gr.tiles[sun::TILE_SITE], out, gr.nc, s);
    return launch_check("batch plaquette");
}

}  // namespace

// Rewrites a batch's launch shapes: waits for the device (the table holds
// the device step counters, so the host copy is brought up to date first),
// applies `apply` to the shape of each selected kind, drops any captured
// graph and uploads the table again.
template <typename F>
int batch_reshape(sun_batch_t b, int kind, F apply) {
    for (size_t i = 0; i < b->host.size(); ++i)
        b->host[i].step = b->step0[b->host[i].out_index] + b->hb_steps_done;
    if (int rc = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize")) return rc;
    for (int k = 0; k < 2; ++k)
        if (kind < 0 || kind == k) apply(b->shape[k]);
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    return upload_table(b);
}


extern "C" {

int sun_batch_bytes(int n, size_t* table_bytes) {
    if (n <= 0) return fail(SUN_EINVAL, "batch of %d chains", n);
    if (table_bytes) *table_bytes = ((sizeof(sun::ChainDesc) * (size_t)n) + 255) & ~(size_t)255;
    return SUN_OK;
}

int sun_batch_create(int n, const sun_lattice_t* chains, const double* betas, const uint64_t* seeds, void* table,
                     size_t table_bytes, sun_batch_t* out) {
    if (!out) return fail(SUN_EINVAL, "out is null");
    *out = nullptr;
    size_t need = 0;
    if (int rc = sun_batch_bytes(n, &need)) return rc;
    if (!chains || !betas || !seeds) return fail(SUN_EINVAL, "null chain, beta or seed array");
    if (!table || table_bytes < need) return fail(SUN_ESIZE, "table of %zu bytes, need %zu", table_bytes, need);
    if ((uintptr_t)table & 255) return fail(SUN_EINVAL, "table must be 256-byte aligned");
    for (int i = 0; i < n; ++i)
        if (!chains[i]) return fail(SUN_EINVAL, "chain %d is null", i);
    // Two descriptors over the same memory would update the same links (or
    // write the same partials) in one launch: refuse a lattice listed twice
    // and lattices whose link or scratch buffers overlap.
    {
        struct Range {
            uintptr_t lo, hi;
            int chain;
        };
        std::vector<Range> r;
        for (int i = 0; i < n; ++i) {
            const sun_lattice_t h = chains[i];
            const uintptr_t l = (uintptr_t)h->links, sc = (uintptr_t)h->scratch;
            r.push_back({l, l + h->link_bytes, i});
            r.push_back({sc, sc + scratch_bytes_of(h->g, is_wide(h->nc, h->dtype)), i});
        }
        std::sort(r.begin(), r.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
        for (size_t k = 1; k < r.size(); ++k)
            if (r[k].lo < r[k - 1].hi) {
                const int a = std::min(r[k].chain, r[k - 1].chain), b = std::max(r[k].chain, r[k - 1].chain);
                if (a == b) return fail(SUN_EINVAL, "chain %d: its link and scratch buffers overlap", a);
                return fail(SUN_EINVAL, "chains %d and %d share device memory (the same lattice listed twice, or "
                                        "overlapping buffers)", a, b);
            }
    }
    auto* b = new sun_batch_s;
    b->chains.assign(chains, chains + n);
    b->table = static_cast<sun::ChainDesc*>(table);
    // group by path, Nc and storage (register path: the dtype; workgroup-per-
    // link path: the precision), keeping the caller's order inside a group
    struct Key {
        int nc, dt;
        bool wide;
    };
    std::vector<Key> keys;
    for (int nc = 2; nc <= SUN_NC_MAX_REGISTER; ++nc)
        for (int dt = SUN_F32; dt <= SUN_F64_TWO_ROW; ++dt)
            if (!is_two_row(dt) || nc == 3) keys.push_back({nc, dt, false});
    for (int nc = 4; nc <= SUN_NC_MAX; ++nc)
        for (int f64 = 0; f64 <= 1; ++f64) keys.push_back({nc, f64 ? SUN_F64_WIDE : SUN_F32_WIDE, true});
    for (const Key& key : keys) {
        const int nc = key.nc, dt = key.dt;
        sun_batch_s::Group gr{ops_for(nc, dt), (int)b->host.size(), 0, {0, 0, 0, 0, 0}, nc, key.wide};
        for (int i = 0; i < n; ++i) {
            const sun_lattice_t h = chains[i];
            const bool w = is_wide(h->nc, h->dtype);
            if (h->nc != nc || w != key.wide) continue;
            if (w ? is_f64(h->dtype) != is_f64(dt) : h->dtype != dt) continue;
            sun::ChainDesc c{};
            c.links = h->links;
            c.scratch = h->scratch;
            c.g = h->g;
            c.beta = betas[i];
            c.k0 = (uint32_t)seeds[i];
            c.k1 = (uint32_t)(seeds[i] >> 32);
            c.step = h->step;
            c.out_index = i;
            b->host.push_back(c);
            ++gr.count;
        }
        if (gr.count) b->groups.push_back(gr);
    }
    for (int i = 0; i < n; ++i) b->step0.push_back(chains[i]->step);
    if (int rc = upload_table(b)) {
        delete b;
        return rc;
    }
    *out = b;
    return SUN_OK;
}

int sun_batch_sweep(sun_batch_t b, int n_hb, int n_or, int reunit, const double* dev_beta, sun_stream_t stream) {
    if (!b) return fail(SUN_EINVAL, "null batch");
    if (n_hb < 0 || n_or < 0) return fail(SUN_EINVAL, "negative step count (n_hb %d, n_or %d)", n_hb, n_or);
    if (int rc = batch_sweep_launches(b, n_hb, n_or, reunit, dev_beta, as_stream(stream))) return rc;
    b->hb_steps_done += (uint64_t)n_hb;
    return SUN_OK;
}

int sun_batch_plaquette(sun_batch_t b, double* dev_out, sun_stream_t stream) {
    if (!b) return fail(SUN_EINVAL, "null batch");
    if (!dev_out) return fail(SUN_ESIZE, "dev_out is null");
    return batch_plaquette_launches(b, dev_out, as_stream(stream));
}

int sun_batch_capture(sun_batch_t b, int n_sweeps, int n_hb, int n_or, int reunit, const double* dev_beta,
                      double* dev_plaq, sun_stream_t stream) {
    if (!b) return fail(SUN_EINVAL, "null batch");
    if (n_sweeps <= 0 || n_hb < 0 || n_or < 0) return fail(SUN_EINVAL, "n_sweeps %d, n_hb %d, n_or %d", n_sweeps, n_hb, n_or);
    const hipStream_t s = as_stream(stream);
    if (!s) return fail(SUN_EINVAL, "graph capture needs a non-null stream");
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (int rc = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture"))
        return rc;
    int rc = SUN_OK;
    for (int k = 0; k < n_sweeps && rc == SUN_OK; ++k) {
        rc = batch_sweep_launches(b, n_hb, n_or, reunit, dev_beta, s);
        if (rc == SUN_OK && dev_plaq) rc = batch_plaquette_launches(b, dev_plaq, s);
    }
    hipGraph_t g = nullptr;
    const int rc_end = hip_check(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
    if (rc != SUN_OK || rc_end != SUN_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc != SUN_OK ? rc : rc_end;
    }
    if (int rc2 = hip_check(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate")) {
        (void)hipGraphDestroy(g);
        return rc2;
    }
    b->graph = g;
    b->hb_per_replay = (uint64_t)n_sweeps * (uint64_t)n_hb;
    return SUN_OK;
}

int sun_batch_replay(sun_batch_t b, sun_stream_t stream) {
    if (!b) return fail(SUN_EINVAL, "null batch");
    if (!b->exec) return fail(SUN_EINVAL, "no captured graph (call sun_batch_capture first)");
    if (int rc = hip_check(hipGraphLaunch(b->exec, as_stream(stream)), "hipGraphLaunch")) return rc;
    b->hb_steps_done += b->hb_per_replay;
    return SUN_OK;
}

int sun_batch_set_launch(sun_batch_t b, int kind, int block, int xcd, int waves) {
    if (!b) return fail(SUN_EINVAL, "null batch");
    if (int rc = check_shape(kind, block, waves)) return rc;
    return batch_reshape(b, kind, [&](sun::Shape& sh) { sh = sun::Shape{block, xcd ? 1 : 0, waves, 0, sh.spt}; });
}

int sun_batch_set_sites_per_item(sun_batch_t b, int kind, int spt) {
    if (!b) return fail(SUN_EINVAL, "null batch");
    if (kind < -1 || kind > 1) return fail(SUN_EINVAL, "kind %d is not -1, SUN_HEATBATH or SUN_OVERRELAX", kind);
    if (!sun::valid_spt(spt)) return fail(SUN_EINVAL, "sites per work-item %d is not 1, 2 or 4", spt);
    return batch_reshape(b, kind, [&](sun::Shape& sh) { sh.spt = spt; });
}

int sun_batch_sync(sun_batch_t b) {
    if (!b) return fail(SUN_EINVAL, "null batch");
    for (size_t i = 0; i < b->chains.size(); ++i) b->chains[i]->step = b->step0[i] + b->hb_steps_done;
    return SUN_OK;
}

void sun_batch_destroy(sun_batch_t b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}

}  // extern "C"

namespace sun {

void launch_advance_steps(ChainDesc* d, int n, int n_hb, hipStream_t s) {
    k_advance_steps<><<<(n + 63) / 64, 64, 0, s>>>(d, n, n_hb);
}

void launch_finalize_max2(const double* partial, int nblk, double* out, hipStream_t s) {
    k_finalize<2, true><<<1, kBlock, 0, s>>>(partial, nblk, out, 1.0, 1.0, 1.0);
}

void launch_finalize_sum2(const double* partial, int nblk, double* out, double scale, hipStream_t s) {
    k_finalize<2, false><<<1, kBlock, 0, s>>>(partial, nblk, out, scale, scale, scale);
}

void launch_plaquette_final(const double* partial, int nblk, double* out, double norm_sp, double norm_tm,
                            double norm_all, hipStream_t s) {
    k_plaquette_final<2><<<1, kBlock, 0, s>>>(partial, nblk, out, norm_sp, norm_tm, norm_all);
}

void launch_sample_su2(int f64, const double* alpha, int n, uint32_t k0, uint32_t k1, uint32_t step,
                       uint32_t mu_sg, double* x, int* attempts, hipStream_t s) {
    if (f64)
        k_sample_su2<double><<<blocks_for(n), kBlock, 0, s>>>(alpha, n, k0, k1, step, mu_sg, x, attempts);
    else
        k_sample_su2<float><<<blocks_for(n), kBlock, 0, s>>>(alpha, n, k0, k1, step, mu_sg, x, attempts);
}

}  // namespace sun
