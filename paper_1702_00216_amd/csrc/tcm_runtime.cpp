// Host runtime of libtcm.so: the C-ABI of include/tcm.h over the HIP kernels
// in tcm_kernels.hip.  It validates the problem (eq.(4), media, thresholds),
// lays out device memory, issues each step's launches on the handle's stream
// (replayed as hipGraphs of several steps), and reports device-side errors
// at synchronisation points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <vector>

#include "tcm.h"
#include "tcm_internal.h"

using namespace tcmk;

namespace {

thread_local std::string g_create_error;
constexpr size_t SLOT_BYTES = sizeof(float) * SLOT;

std::string fmt(const char* f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

struct ShotHost {
    int nx, ny, nz;
    int media_kind;
    double cmax;
};

}  // namespace

struct tcm_handle {
    tcm_config cfg{};
    int engine = TCM_ENGINE_BLOCKS;
    int device = 0;
    int ncu = 256;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<void*> allocs;          // device memory owned by the handle
    std::string err;
    bool poisoned = false;

    std::vector<ShotHost> hshots;
    std::vector<Shot> shots;            // host copies holding device pointers
    Shot* d_shots = nullptr;
    Tables t{};
    long long nkeys = 0;
    size_t table_bytes = 0;

    int grid_step = 0, grid_plan = 0, grid_pool = 0, grid_emit = 0;
    long long hstep = 0;                // index of the next step to enqueue

    // sources / receivers (host mirrors)
    std::vector<Src> h_src;             // in the order added (the device copy is sorted by key)
    std::vector<float> h_srcw;
    Src* d_src = nullptr;
    size_t d_src_cap = 0;
    float* d_srcw = nullptr;
    size_t d_srcw_cap = 0;
    std::vector<Rec> h_rec;
    Rec* d_rec = nullptr;
    float* d_traces = nullptr;

    // graph replay
    hipGraphExec_t gexec = nullptr;
    int gsteps = 0;
    int tile_w = 4;                     // waves per stencil workgroup
    int tile_p = 1;                     // blocks per stencil wave (1 or 2)
    bool graph_failed = false;

    // timing (TCM_FLAG_TIMING)
    std::vector<hipEvent_t> events;
    double stencil_ms = 0.0;
    long long grad_cells = 0;           // gradient-term nodes of tcm_adjoint (timing flag)
    double af_ms = 0.0;                 // adjoint-field stencil of tcm_adjoint (timing flag)
    long long af_launches = 0, af_cells = 0, af_cells_u = 0, af_cells_l = 0;
    std::vector<hipEvent_t> gev;        // events around the timed gradient launches
    long long stencil_launches = 0, stencil_cells = 0, stencil_cells_u = 0, stencil_cells_l = 0;

    // dense engine
    float* d_phi[2] = {nullptr, nullptr};
    float* d_c2 = nullptr;
    long long dense_step = 0;

    // scratch for host reads
    float* d_scratch = nullptr;
    size_t scratch_bytes = 0;

    DevState* h_state = nullptr;        // pinned mirror of the device counters

    // receivers as given (positions of the adjoint sources)
    std::vector<int> rec_xyz, rec_shot;

    // forward checkpoints for tcm_adjoint at levels 0, K, 2K, ... (K =
    // checkpoint_every): sparse copies of the block-engine state (the active
    // list, its two phi planes and per-slot tables; see ck_save)
    struct Ckpt {
        long long step = -1;
        long long n = 0;                // active entries stored
        char* buf = nullptr;
        size_t cap = 0, bytes = 0;      // allocated, used
    };
    std::vector<Ckpt> ckpts;
    bool in_adjoint = false;
    tcm_handle* adj = nullptr;          // tables of the adjoint field (shares the media)
    long long media_gen = 0;            // tcm_set_media calls so far (snapshots record it)
    size_t adjoint_bytes = 0;           // device memory the last tcm_adjoint held
    // timed recomputed forward steps of tcm_adjoint (TCM_FLAG_TIMING)
    double rec_ms = 0.0;
    long long rec_launches = 0, rec_cells = 0, rec_cells_u = 0, rec_cells_l = 0;
    // source activation requests (keys, shots, keys in the shot, pins, source ranges)
    void* d_act_req = nullptr;
    size_t d_act_req_cap = 0;
};

namespace {

tcm_status set_err(tcm_handle* h, tcm_status s, const std::string& m) {
    if (h) h->err = m; else g_create_error = m;
    return s;
}

// stencil variant of these tables (mode: STEP_PLAIN / STEP_RECORD / STEP_GRAD)
int step_mode(const Tables& t, int mode = STEP_PLAIN) {
    return mode | (t.lat_c2 && !t.adaptive ? STEP_LAT : 0);
}

tcm_status dev_fail(tcm_handle* h, hipError_t e, const char* what) {
    std::string m = fmt("HIP error in %s: %s", what, hipGetErrorString(e));
    if (h) {
        h->poisoned = true;
        h->err = m;
    } else {
        g_create_error = m;
    }
    return TCM_E_DEVICE;
}

#define HIP_OR_FAIL(h, expr)                                  \
    do {                                                      \
        hipError_t e__ = (expr);                              \
        if (e__ != hipSuccess) return dev_fail((h), e__, #expr); \
    } while (0)

// Events that only time work on the handle's stream.  A default event makes a
// system-scope release and acquire at its record (cache write-back and
// invalidation between the launches it separates); these are only read for
// their timestamps once the stream has passed them, so they skip that fence.
hipError_t timing_event(hipEvent_t* e) {
    return hipEventCreateWithFlags(e, hipEventDisableSystemFence);
}

template <class T>
hipError_t dalloc(tcm_handle* h, T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        h->allocs.push_back(q);
        *p = (T*)q;
    }
    return e;
}

void dfree(tcm_handle* h, void* p) {
    if (!p) return;
    auto it = std::find(h->allocs.begin(), h->allocs.end(), p);
    if (it != h->allocs.end()) h->allocs.erase(it);
    (void)hipFree(p);
}

void drop_graph(tcm_handle* h) {
    if (h->gexec) {
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
}

tcm_status check_live(tcm_handle* h) {
    if (!h) return TCM_E_ARG;
    if (h->poisoned) return set_err(h, TCM_E_DEVICE, "handle is poisoned by an earlier device error");
    if (hipSetDevice(h->device) != hipSuccess) return dev_fail(h, hipGetLastError(), "hipSetDevice");
    return TCM_OK;
}

// ---- media validation (host) ---------------------------------------------
tcm_status validate_media(const tcm_media* m, int nx, int ny, int nz, double* cmax, std::string* why) {
    if (!m) { *why = "media is NULL"; return TCM_E_ARG; }
    double mx = 0.0;
    if (m->kind == TCM_MEDIA_DENSE) {
        if (!m->c) { *why = "dense media without an array"; return TCM_E_ARG; }
        const size_t N = (size_t)nx * ny * nz;
        for (size_t i = 0; i < N; i++) {
            const float v = m->c[i];
            if (!std::isfinite(v) || v < 0.f) { *why = fmt("wave speed %g at node %zu is negative or not finite", v, i); return TCM_E_ARG; }
            if (v > mx) mx = v;
        }
    } else if (m->kind == TCM_MEDIA_LAYERED) {
        if (m->nlayers < 1 || !m->z_top || !m->c_layer || m->z_top[0] != 0) { *why = "layered media needs nlayers >= 1 and z_top[0] == 0"; return TCM_E_ARG; }
        for (int k = 0; k < m->nlayers; k++) {
            if (k > 0 && m->z_top[k] <= m->z_top[k - 1]) { *why = "layer tops must ascend"; return TCM_E_ARG; }
            const float v = m->c_layer[k];
            if (!std::isfinite(v) || v < 0.f) { *why = "layer speed negative or not finite"; return TCM_E_ARG; }
            if (v > mx) mx = v;
        }
    } else if (m->kind == TCM_MEDIA_LATTICE) {
        if (!m->lattice || m->log2_spacing < 0 || m->log2_spacing > 20) { *why = "lattice media needs values and 0 <= log2_spacing <= 20"; return TCM_E_ARG; }
        const int s = m->log2_spacing;
        if (m->lx < ((nx - 1) >> s) + 2 || m->ly < ((ny - 1) >> s) + 2 || m->lz < ((nz - 1) >> s) + 2) {
            *why = "lattice too small for the grid"; return TCM_E_ARG;
        }
        const size_t L = (size_t)m->lx * m->ly * m->lz;
        for (size_t i = 0; i < L; i++) {
            const double v = m->lattice[i];
            if (!std::isfinite(v) || v < 0.0) { *why = "lattice speed negative or not finite"; return TCM_E_ARG; }
            if (v > mx) mx = v;
        }
        mx *= 1.0 + 1e-12;   // trilinear rounding can exceed the largest node by an ulp
    } else {
        *why = "unknown media kind";
        return TCM_E_ARG;
    }
    *cmax = mx;
    return TCM_OK;
}

tcm_status upload_media(tcm_handle* h, const tcm_media* m, Shot& S) {
    S.media_kind = m->kind;
    S.c = nullptr; S.z_top = nullptr; S.c_layer = nullptr; S.lattice = nullptr;
    S.nlayers = 0; S.lx = S.ly = S.lz = S.log2s = 0;
    if (m->kind == TCM_MEDIA_DENSE) {
        const size_t N = (size_t)S.nx * S.ny * S.nz;
        float* d = nullptr;
        HIP_OR_FAIL(h, dalloc(h, &d, N));
        HIP_OR_FAIL(h, hipMemcpy(d, m->c, N * sizeof(float), hipMemcpyHostToDevice));
        S.c = d;
        h->table_bytes += N * sizeof(float);
    } else if (m->kind == TCM_MEDIA_LAYERED) {
        int* zt = nullptr;
        float* cl = nullptr;
        HIP_OR_FAIL(h, dalloc(h, &zt, m->nlayers));
        HIP_OR_FAIL(h, dalloc(h, &cl, m->nlayers));
        HIP_OR_FAIL(h, hipMemcpy(zt, m->z_top, m->nlayers * sizeof(int), hipMemcpyHostToDevice));
        HIP_OR_FAIL(h, hipMemcpy(cl, m->c_layer, m->nlayers * sizeof(float), hipMemcpyHostToDevice));
        S.z_top = zt; S.c_layer = cl; S.nlayers = m->nlayers;
    } else {
        const size_t L = (size_t)m->lx * m->ly * m->lz;
        double* d = nullptr;
        HIP_OR_FAIL(h, dalloc(h, &d, L));
        HIP_OR_FAIL(h, hipMemcpy(d, m->lattice, L * sizeof(double), hipMemcpyHostToDevice));
        S.lattice = d; S.lx = m->lx; S.ly = m->ly; S.lz = m->lz; S.log2s = m->log2_spacing;
        h->table_bytes += L * sizeof(double);
    }
    return TCM_OK;
}

tcm_status sync_state(tcm_handle* h) {
    HIP_OR_FAIL(h, hipMemcpyAsync(h->h_state, h->t.st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    return TCM_OK;
}

void destroy_all(tcm_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->adj) destroy_all(h->adj);
    h->adj = nullptr;
    for (auto& c : h->ckpts)
        if (c.buf) (void)hipFree(c.buf);
    h->ckpts.clear();
    if (h->d_act_req) (void)hipFree(h->d_act_req);
    h->d_act_req = nullptr;
    drop_graph(h);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->events.clear();
    for (hipEvent_t e : h->gev) (void)hipEventDestroy(e);
    h->gev.clear();
    for (void* p : h->allocs) (void)hipFree(p);
    h->allocs.clear();
    if (h->h_state) (void)hipHostFree(h->h_state);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

// graphs hold whole activation-update intervals
int round_graph_steps(const tcm_handle* h, int gs) {
    const int k = h->t.interval > 1 ? h->t.interval : 1;
    return std::max(k, (gs + k - 1) / k * k);
}

// Device state of the engine (dense arrays or block tables) for the shots
// already in h->shots / h->d_shots.
tcm_status setup_engine(tcm_handle* h, long long word_base) {
    const tcm_config* cfg = &h->cfg;
    const int nshots = (int)h->shots.size();
    Tables& t = h->t;
    t.shots = h->d_shots;
    t.nshots = nshots;
    t.dt = cfg->dt;
    t.dx = cfg->dx;
    t.trigger = cfg->trigger;
    t.retire = cfg->retire;
    if (hipMalloc((void**)&t.st, sizeof(DevState)) != hipSuccess) return dev_fail(h, hipErrorOutOfMemory, "hipMalloc(state)");
    h->allocs.push_back(t.st);
    if (hipMemsetAsync(t.st, 0, sizeof(DevState), h->stream) != hipSuccess) return dev_fail(h, hipGetLastError(), "hipMemset(state)");

    if (h->engine == TCM_ENGINE_DENSE) {
        const Shot& S = h->shots[0];
        const size_t N = (size_t)S.nx * S.ny * S.nz;
        if (dalloc(h, &h->d_phi[0], N) != hipSuccess || dalloc(h, &h->d_phi[1], N) != hipSuccess ||
            dalloc(h, &h->d_c2, N) != hipSuccess)
            return set_err(h, TCM_E_NOMEM, "dense engine: device allocation failed");
        h->table_bytes += 3 * N * sizeof(float);
        if (hipMemsetAsync(h->d_phi[0], 0, N * sizeof(float), h->stream) != hipSuccess ||
            hipMemsetAsync(h->d_phi[1], 0, N * sizeof(float), h->stream) != hipSuccess)
            return dev_fail(h, hipGetLastError(), "hipMemset(dense)");
        if (launch_media_c2(S, h->d_shots, cfg->dt, cfg->dx, h->d_c2, h->stream) != hipSuccess)
            return dev_fail(h, hipGetLastError(), "media_c2");
        if (hipStreamSynchronize(h->stream) != hipSuccess) return dev_fail(h, hipGetLastError(), "sync");
        return TCM_OK;
    }

    // ---- block engine tables ----
    h->nkeys = word_base * 64;
    if (h->nkeys > 0x7fffffffLL)
        return set_err(h, TCM_E_ARG, "more than 2^31 block keys: grid too large for one handle");
    t.nwords = word_base;
    t.nchunks = (int)((word_base + CHUNK_WORDS - 1) / CHUNK_WORDS);
    // with several shots, the shot of every bitmap word (one load for the
    // management kernels instead of a search over the shots)
    t.word_shot = nullptr;
    if (nshots > 1) {
        std::vector<int> ws((size_t)word_base);
        for (int i = 0; i < nshots; i++)
            for (long long w = h->shots[i].word_base; w < h->shots[i].word_base + h->shots[i].nwords; w++)
                ws[(size_t)w] = i;
        int* d = nullptr;
        if (dalloc(h, &d, ws.size()) != hipSuccess) return set_err(h, TCM_E_NOMEM, "device allocation failed");
        if (hipMemcpy(d, ws.data(), ws.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            return dev_fail(h, hipGetLastError(), "hipMemcpy(word_shot)");
        t.word_shot = d;
    }
    // lattice records (the stencil's STEP_LAT variants): with constant levels,
    // for shots whose lattice spacing is at least the block edge
    bool lat_any = false;
    for (const Shot& S : h->shots) lat_any = lat_any || (S.media_kind == TCM_MEDIA_LATTICE && S.log2s >= 3);
    const bool adaptive = cfg->trigger_rel > 0.f || cfg->retire_rel > 0.f;
    // (TCM_FLAG_NO_UNIFORM_C2 asks for every C2 plane read, so it turns them off too)
    t.lat_c2 = (lat_any && !adaptive && !(cfg->flags & (TCM_FLAG_C2_PLANES | TCM_FLAG_NO_UNIFORM_C2))) ? 1 : 0;
    {
        int ex = 0;
        const double m = std::frexp(cfg->dx, &ex);
        t.dx_pow2 = m == 0.5 ? 1 : 0;
        t.rdx = 1.0 / cfg->dx;
    }
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    // per-slot bookkeeping bytes besides the 6 KiB slot
    const size_t per_slot_tab = 4 + 4 + 4 + 32 + 1 + 4 + 4 + 4 + 1 + 4 + 8 + 8 + 4 + 4 + 8 + (t.lat_c2 ? 80 : 0);
    const size_t fixed = (size_t)h->nkeys * 4 + (size_t)word_base * 8 + (size_t)t.nchunks * 4 + (1 << 20);
    long long cap;
    if (cfg->pool_bytes > 0) {
        cap = (long long)(cfg->pool_bytes / SLOT_BYTES);
        if (cap < 1) return set_err(h, TCM_E_ARG, "pool_bytes is below one slot (6 KiB)");
        if (!cfg->device_pool && (double)cap * (SLOT_BYTES + per_slot_tab) + fixed > 0.95 * (double)free_b)
            return set_err(h, TCM_E_NOMEM, fmt("pool of %lld slots does not fit in %.1f GB free", cap, free_b / 1e9));
    } else {
        // one slot per key (tiles padded at the domain edges included): new
        // blocks are then placed at slot = key, in the order of the list
        cap = h->nkeys;
        const double room = 0.9 * (double)free_b - (double)fixed;
        const long long fit = room > 0 ? (long long)(room / (double)(SLOT_BYTES + per_slot_tab)) : 0;
        if (cap > fit) cap = fit;
        if (cap < 1) return set_err(h, TCM_E_NOMEM, "no device memory for the pool");
    }
    if (cap > h->nkeys) cap = h->nkeys;
    if (cap > 0x7fffffffLL) cap = 0x7fffffffLL;
    t.cap = (int)cap;
    t.nkeys = h->nkeys;

    bool ok = true;
    if (cfg->device_pool) {
        t.pool = (float*)cfg->device_pool;
    } else {
        // Measured on the 4096^3 workload (64 GB pool): a pool taken by the
        // first allocation of its size in a process streamed 5.05 TB/s in the
        // stencil, one taken after an allocation of the same size had been
        // freed 5.44 TB/s, on every run; so the size is reserved and released
        // once before the pool is allocated (a few ms at creation).
        void* probe_alloc = nullptr;
        if (hipMalloc(&probe_alloc, (size_t)cap * SLOT * sizeof(float)) == hipSuccess) (void)hipFree(probe_alloc);
        (void)hipGetLastError();
        ok = ok && dalloc(h, &t.pool, (size_t)cap * SLOT) == hipSuccess;
    }
    ok = ok && dalloc(h, &t.cell2box, (size_t)h->nkeys) == hipSuccess;
    ok = ok && dalloc(h, &t.bitmap, (size_t)t.nchunks * CHUNK_WORDS) == hipSuccess;
    // the two-launch activation update (a block's slot is its key)
    t.nfchunks = (int)((word_base + FAST_WORDS - 1) / FAST_WORDS);
    t.fast = (!(cfg->flags & TCM_FLAG_THREE_PASS_UPDATE) && cfg->trigger_rel == 0.f && cfg->retire_rel == 0.f &&
              cfg->trigger_interval <= 1 && cfg->shutdown_steps == 0 && cap >= h->nkeys &&
              t.nfchunks <= FAST_MAX_CHUNKS) ? 1 : 0;
    if (t.fast) {
        ok = ok && dalloc(h, &t.bitmap2, (size_t)t.nchunks * CHUNK_WORDS) == hipSuccess;
        ok = ok && dalloc(h, &t.fc_cnt, (size_t)t.nfchunks) == hipSuccess;
        if (t.nfchunks <= FAST_DIRECT_CHUNKS) {
            t.nfblk = 0;
            ok = ok && dalloc(h, &t.fc_new, (size_t)t.nfchunks) == hipSuccess;
            ok = ok && dalloc(h, &t.fc_ret, (size_t)t.nfchunks) == hipSuccess;
            ok = ok && dalloc(h, &t.fc_cells, 3 * (size_t)t.nfchunks) == hipSuccess;
        } else {
            t.nfblk = (t.nfchunks + FAST_BLK - 1) / FAST_BLK;
            ok = ok && dalloc(h, &t.fc_blk, 6 * (size_t)t.nfblk) == hipSuccess;
        }
    }
    ok = ok && dalloc(h, &t.act_slot, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.act_shot, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.act_key, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.rows, (size_t)cap * 8) == hipSuccess;
    ok = ok && dalloc(h, &t.flags, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.pin_until, 2 * (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.slot_c2u, (size_t)cap) == hipSuccess;
    t.slot_lat = nullptr;
    t.slot_latm = nullptr;
    if (t.lat_c2) {
        ok = ok && dalloc(h, &t.slot_lat, 8 * (size_t)cap) == hipSuccess;
        ok = ok && dalloc(h, &t.slot_latm, (size_t)cap) == hipSuccess;
    }
    ok = ok && dalloc(h, &t.sdlog, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.dec_slot, (size_t)cap) == hipSuccess;
    t.shutdown_steps = cfg->shutdown_steps;
    t.shutdown_alpha = cfg->shutdown_alpha;
    t.adaptive = (cfg->trigger_rel > 0.f || cfg->retire_rel > 0.f) ? 1 : 0;
    t.trigger_rel = cfg->trigger_rel;
    t.retire_rel = cfg->retire_rel;
    ok = ok && dalloc(h, &t.bmax, t.adaptive ? (size_t)cap * 8 : 1) == hipSuccess;
    t.uniform_c2 = (cfg->flags & TCM_FLAG_NO_UNIFORM_C2) ? 0 : 1;
    ok = ok && dalloc(h, &t.slot_key, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.new_key, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.new_shot, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.ret_slot, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.ret_key, (size_t)cap) == hipSuccess;
    ok = ok && dalloc(h, &t.partial, (size_t)t.nchunks) == hipSuccess;
    ok = ok && dalloc(h, &t.wg_total, (size_t)POOL_COUNT_MAX_WG) == hipSuccess;
    ok = ok && dalloc(h, &t.ne_chunks, (size_t)t.nchunks) == hipSuccess;
    if (!ok) return set_err(h, TCM_E_NOMEM, "device allocation of the block tables failed");
    h->table_bytes += fixed + (size_t)cap * per_slot_tab;

    // a pool of one slot per key: every C2 plane is filled now, once
    t.c2_ready = cap >= h->nkeys ? 1 : 0;
    if (launch_init_tables(t, h->nkeys, h->stream) != hipSuccess) return dev_fail(h, hipGetLastError(), "init_tables");
    if (t.c2_ready && launch_prefill_c2(t, h->nkeys, h->stream) != hipSuccess)
        return dev_fail(h, hipGetLastError(), "prefill_c2");
    if (hipStreamSynchronize(h->stream) != hipSuccess) return dev_fail(h, hipGetLastError(), "sync");

    // persistent stencil grid of resident workgroups (a grid beyond residency
    // would leave a tail of workgroups that start after the first wave); by
    // default about 12 waves per CU, the best shape measured on full lists
    h->tile_p = cfg->blocks_per_wave > 1 ? cfg->blocks_per_wave : 1;
    h->tile_w = (cfg->blocks_per_wg > 0 ? cfg->blocks_per_wg : 4) / h->tile_p;
    const int occ = std::max(1, block_step_occupancy(t.adaptive != 0, h->tile_w, h->tile_p, step_mode(t)));
    const int wpc = cfg->wg_per_cu > 0 ? cfg->wg_per_cu : std::min(occ, std::max(1, 12 / h->tile_w));
    h->grid_step = std::max(8, (h->ncu * wpc) / 8 * 8);
    // one plan thread per entry up to 4 x 256 x CUs entries; the allocator
    // fills new blocks with 2 workgroups per CU, of which the first scan_wgs
    // also scan the bitmap
    h->grid_plan = std::max(1, h->ncu * 4);
    // up to 1024 chunks (64 Ki blocks) one workgroup scans the whole bitmap:
    // no completion chain between workgroups
    t.scan_wgs = t.nchunks <= 1024 ? 1
                                   : std::min(POOL_COUNT_MAX_WG, std::max(64, std::min((t.nchunks + 3) / 4, h->ncu)));
    t.chunks_per_wg = (t.nchunks + t.scan_wgs - 1) / t.scan_wgs;
    h->grid_pool = std::max(t.scan_wgs, h->ncu * 2);
    // compaction: 16-wave workgroups over the non-empty chunks
    h->grid_emit = std::max(1, std::min(t.nchunks, h->ncu * 2));
    t.interval = cfg->trigger_interval > 1 ? cfg->trigger_interval : 1;
    h->gsteps = round_graph_steps(h, cfg->graph_steps > 0 ? cfg->graph_steps : 16);
    return TCM_OK;
}

tcm_status create_common(const tcm_config* cfg, const tcm_shot* shots, int nshots, tcm_handle** out) {
    if (!out) return set_err(nullptr, TCM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg) return set_err(nullptr, TCM_E_ARG, "config is NULL");
    if (nshots < 1 || !shots) return set_err(nullptr, TCM_E_ARG, "need at least one shot");
    if (!(cfg->dx > 0.0) || !std::isfinite(cfg->dx) || !(cfg->dt >= 0.0) || !std::isfinite(cfg->dt))
        return set_err(nullptr, TCM_E_ARG, "dx must be > 0 and dt >= 0, both finite");
    if (!(cfg->trigger >= 0.f) || !(cfg->retire >= 0.f) || !std::isfinite(cfg->trigger) ||
        !std::isfinite(cfg->retire) || cfg->retire > cfg->trigger)
        return set_err(nullptr, TCM_E_ARG, "thresholds must satisfy 0 <= retire <= trigger (finite)");
    if (cfg->engine != TCM_ENGINE_BLOCKS && cfg->engine != TCM_ENGINE_DENSE)
        return set_err(nullptr, TCM_E_ARG, "unknown engine");
    if (cfg->shutdown_steps < 0 || cfg->shutdown_steps > 255 ||
        (cfg->shutdown_steps > 0 && !(std::isfinite(cfg->shutdown_alpha) && cfg->shutdown_alpha >= 0.f &&
                                      cfg->shutdown_alpha <= 1.f)))
        return set_err(nullptr, TCM_E_ARG, "shutdown needs 0 <= steps <= 255 and 0 <= alpha <= 1");
    if (!(cfg->trigger_rel >= 0.f) || !(cfg->retire_rel >= 0.f) || !std::isfinite(cfg->trigger_rel) ||
        !std::isfinite(cfg->retire_rel) || cfg->retire_rel > cfg->trigger_rel)
        return set_err(nullptr, TCM_E_ARG, "relative levels must satisfy 0 <= retire_rel <= trigger_rel");
    if (cfg->trigger_interval < 0 || cfg->trigger_interval > BE)
        return set_err(nullptr, TCM_E_ARG, "trigger_interval must be in [0, 8] (0 and 1: every step)");
    if (cfg->blocks_per_wg != 0 && cfg->blocks_per_wg != 2 && cfg->blocks_per_wg != 4 && cfg->blocks_per_wg != 8)
        return set_err(nullptr, TCM_E_ARG, "blocks_per_wg must be 0, 2, 4 or 8");
    if (cfg->blocks_per_wave < 0 || cfg->blocks_per_wave > 2 ||
        (cfg->blocks_per_wave == 2 && cfg->blocks_per_wg == 2))
        return set_err(nullptr, TCM_E_ARG, "blocks_per_wave must be 0, 1 or 2 (2 with a tile of 4 or 8 blocks)");
    if (cfg->device_pool && cfg->pool_bytes < SLOT_BYTES)
        return set_err(nullptr, TCM_E_ARG, "a caller device_pool needs its size in pool_bytes");
    if (cfg->engine == TCM_ENGINE_DENSE && nshots != 1)
        return set_err(nullptr, TCM_E_ARG, "the dense engine runs one shot");

    std::vector<ShotHost> hs(nshots);
    for (int s = 0; s < nshots; s++) {
        const tcm_shot& sh = shots[s];
        if (sh.nx <= 0 || sh.ny <= 0 || sh.nz <= 0 || sh.nx > (1 << 20) || sh.ny > (1 << 20) || sh.nz > (1 << 20))
            return set_err(nullptr, TCM_E_ARG, fmt("shot %d: grid edges must be in [1, 2^20]", s));
        std::string why;
        double cmax = 0.0;
        tcm_status st = validate_media(&sh.media, sh.nx, sh.ny, sh.nz, &cmax, &why);
        if (st != TCM_OK) return set_err(nullptr, st, fmt("shot %d: %s", s, why.c_str()));
        const double r = cmax * cfg->dt / cfg->dx;
        if (r * r * 3.0 > 1.0 + 4.0 * DBL_EPSILON)
            return set_err(nullptr, TCM_E_CFL, fmt("shot %d: eq.(4) violated: cmax dt / dx = %.9g > 1/sqrt(3)", s, r));
        hs[s] = ShotHost{sh.nx, sh.ny, sh.nz, sh.media.kind, cmax};
    }

    tcm_handle* h = new tcm_handle();
    h->cfg = *cfg;
    h->engine = cfg->engine;
    h->hshots = hs;
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return set_err(nullptr, TCM_E_DEVICE, "no HIP device"); }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) != hipSuccess) { delete h; return set_err(nullptr, TCM_E_DEVICE, "hipGetDeviceProperties failed"); }
    h->ncu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (cfg->stream) {
        h->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) { delete h; return set_err(nullptr, TCM_E_DEVICE, "hipStreamCreate failed"); }
        h->own_stream = true;
    }
    if (hipHostMalloc((void**)&h->h_state, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        destroy_all(h);
        return set_err(nullptr, TCM_E_NOMEM, "pinned host allocation failed");
    }

    auto fail = [&](tcm_status st) {
        std::string m = h->err.empty() ? g_create_error : h->err;
        destroy_all(h);
        return set_err(nullptr, st, m);
    };

    // ---- shots, key ranges ----
    long long word_base = 0;
    h->shots.resize(nshots);
    for (int s = 0; s < nshots; s++) {
        Shot S{};
        S.nx = hs[s].nx; S.ny = hs[s].ny; S.nz = hs[s].nz;
        S.bx = (S.nx + BE - 1) / BE; S.by = (S.ny + BE - 1) / BE; S.bz = (S.nz + BE - 1) / BE;
        S.tx = (S.bx + 3) / 4; S.ty = (S.by + 3) / 4; S.tz = (S.bz + 3) / 4;
        S.word_base = word_base;
        S.key_base = word_base * 64;
        S.nwords = (long long)S.tx * S.ty * S.tz;
        word_base += S.nwords;
        tcm_status st = upload_media(h, &shots[s].media, S);
        if (st != TCM_OK) return fail(st);
        h->shots[s] = S;
    }
    if (hipMalloc((void**)&h->d_shots, sizeof(Shot) * nshots) != hipSuccess) return fail(dev_fail(h, hipErrorOutOfMemory, "hipMalloc(shots)"));
    h->allocs.push_back(h->d_shots);
    if (hipMemcpy(h->d_shots, h->shots.data(), sizeof(Shot) * nshots, hipMemcpyHostToDevice) != hipSuccess)
        return fail(dev_fail(h, hipGetLastError(), "hipMemcpy(shots)"));

    tcm_status st = setup_engine(h, word_base);
    if (st != TCM_OK) return fail(st);
    *out = h;
    return TCM_OK;
}

// ---- per-step launch sequence ----------------------------------------------
// Step h->hstep: the stencil, then the activation update when the step ends
// an update interval ("Updating active cells", eq.(5)), else only the
// receivers and the step counter.
hipError_t enqueue_step(tcm_handle* h, hipEvent_t e0, hipEvent_t e1) {
    hipError_t e;
    const long long n = h->hstep++;
    const int k = h->t.interval > 1 ? h->t.interval : 1;
    // a step without an activation update: with no receivers to record and
    // constant levels the stencil advances the step itself (no k_advance)
    const bool update = (n + 1) % k == 0;
    const bool self = !update && h->t.nrec == 0 && !h->t.adaptive;
    h->t.self_advance = self ? 1 : 0;
    e = launch_block_step(h->t, h->grid_step, h->tile_w, h->tile_p, h->stream, e0, e1);
    h->t.self_advance = 0;
    if (e != hipSuccess) return e;
    if (!update) return self ? hipSuccess : launch_advance(h->t, h->stream);
    if (h->t.fast) return launch_fast_update(h->t, h->t.nfchunks, h->stream);
    if ((e = launch_plan(h->t, h->grid_plan, h->stream)) != hipSuccess) return e;
    if ((e = launch_pool_count(h->t, h->grid_pool, h->stream)) != hipSuccess) return e;
    return launch_emit(h->t, h->grid_emit, h->stream);
}

hipError_t enqueue_dense_step(tcm_handle* h, hipEvent_t e0, hipEvent_t e1) {
    const Shot& S = h->shots[0];
    const long long n = h->dense_step;
    DenseArgs a{S.nx, S.ny, S.nz, h->d_phi[n & 1], h->d_phi[1 - (n & 1)], h->d_c2};
    hipError_t e;
    if ((e = launch_dense_step(a, h->stream, e0, e1)) != hipSuccess) return e;
    const long long row = n - h->t.trace_step0;
    const int trow = (h->t.nrec > 0 && row >= 0 && row < h->t.trace_cap) ? (int)row : -1;
    if (h->t.nsrc > 0 || trow >= 0) {
        if ((e = launch_dense_inject(h->d_phi[1 - (n & 1)], (int)n, h->t.src, h->t.nsrc, h->t.srcw,
                                     h->t.rec, h->t.nrec, h->t.traces, trow, h->stream)) != hipSuccess)
            return e;
    }
    h->dense_step++;
    return hipSuccess;
}

long long current_step(tcm_handle* h) {
    if (h->engine == TCM_ENGINE_DENSE) return h->dense_step;
    return h->h_state->step;
}

tcm_status ensure_trace_capacity(tcm_handle* h, long long upto_row) {
    if (h->t.nrec <= 0 || upto_row <= h->t.trace_cap) return TCM_OK;
    long long cap = std::max<long long>(1024, h->t.trace_cap);
    while (cap < upto_row) cap *= 2;
    if (cap > 0x7fffffffLL) return set_err(h, TCM_E_ARG, "trace buffer too long");
    float* nt = nullptr;
    HIP_OR_FAIL(h, dalloc(h, &nt, (size_t)cap * h->t.nrec));
    HIP_OR_FAIL(h, hipMemsetAsync(nt, 0, (size_t)cap * h->t.nrec * sizeof(float), h->stream));
    if (h->d_traces && h->t.trace_cap > 0)
        HIP_OR_FAIL(h, hipMemcpyAsync(nt, h->d_traces, (size_t)h->t.trace_cap * h->t.nrec * sizeof(float),
                                      hipMemcpyDeviceToDevice, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    dfree(h, h->d_traces);
    h->d_traces = nt;
    h->t.traces = nt;
    h->t.trace_cap = (int)cap;
    drop_graph(h);
    return TCM_OK;
}

tcm_status scratch(tcm_handle* h, size_t bytes, float** p) {
    if (bytes > h->scratch_bytes) {
        dfree(h, h->d_scratch);
        h->d_scratch = nullptr;
        h->scratch_bytes = 0;
        HIP_OR_FAIL(h, dalloc(h, &h->d_scratch, (bytes + 3) / 4));
        h->scratch_bytes = bytes;
    }
    *p = h->d_scratch;
    return TCM_OK;
}


// ---- checkpoints ------------------------------------------------------------
// The state of the block engine between two steps is the device counters,
// the active list with its rows, and the slots of the active blocks (two phi
// planes and the per-slot tables); the block table holds exactly those
// blocks, the bitmap is clear and free slots carry no state.  A checkpoint
// stores that much (about 4 KiB per active block), so its size follows the
// active set; restoring re-initialises the tables, scatters the blocks back
// into the same slots and refills their C2 planes from the media.
using Ckpt = tcm_handle::Ckpt;

tcm_status ck_save(tcm_handle* h, Ckpt& c) {
    tcm_status st = sync_state(h);
    if (st) return st;
    const long long n = h->h_state->n_act;
    const size_t bytes = ck_sparse_bytes(n);
    if (c.cap < bytes) {
        if (c.buf) (void)hipFree(c.buf);
        c.buf = nullptr;
        c.cap = 0;
        void* q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return set_err(h, TCM_E_NOMEM, "no device memory for a state copy");
        }
        c.buf = (char*)q;
        c.cap = bytes;
    }
    HIP_OR_FAIL(h, hipMemcpyAsync(c.buf, h->t.st, sizeof(DevState), hipMemcpyDeviceToDevice, h->stream));
    HIP_OR_FAIL(h, launch_ck_gather(h->t, n, c.buf, h->stream));
    c.n = n;
    c.bytes = bytes;
    c.step = h->h_state->step;
    return TCM_OK;
}

tcm_status ck_restore(tcm_handle* h, const Ckpt& c) {
    HIP_OR_FAIL(h, launch_init_tables(h->t, h->nkeys, h->stream));
    HIP_OR_FAIL(h, launch_ck_scatter(h->t, c.n, c.buf, h->stream));
    HIP_OR_FAIL(h, hipMemcpyAsync(h->t.st, c.buf, sizeof(DevState), hipMemcpyDeviceToDevice, h->stream));
    return TCM_OK;
}

void ck_free(Ckpt& c) {
    if (c.buf) (void)hipFree(c.buf);
    c = Ckpt{};
}

void ck_clear(tcm_handle* h) {
    for (auto& c : h->ckpts) ck_free(c);
    h->ckpts.clear();
}

size_t ck_stored_bytes(const tcm_handle* h) {
    size_t b = 0;
    for (const auto& c : h->ckpts) b += c.bytes;
    return b;
}

// Issue n steps (graph replays where possible); no synchronisation.
tcm_status issue_steps(tcm_handle* h, int n) {
    int left = n;
    const int kint = h->t.interval > 1 ? h->t.interval : 1;
    // graphs hold whole update intervals: start them at an interval boundary
    while (kint > 1 && left > 0 && h->hstep % kint != 0) {
        HIP_OR_FAIL(h, enqueue_step(h, nullptr, nullptr));
        left--;
    }
    const bool use_graph = !(h->cfg.flags & TCM_FLAG_NO_GRAPH) && !h->graph_failed && h->own_stream;
    if (use_graph && left >= h->gsteps) {
        if (!h->gexec) {
            hipGraph_t g = nullptr;
            const long long keep_step = h->hstep;
            bool ok = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            hipError_t le = hipSuccess;
            for (int k = 0; ok && k < h->gsteps && le == hipSuccess; k++) le = enqueue_step(h, nullptr, nullptr);
            h->hstep = keep_step;          // capturing issues nothing
            if (ok) ok = hipStreamEndCapture(h->stream, &g) == hipSuccess && le == hipSuccess;
            if (ok) ok = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (!ok) {
                (void)hipGetLastError();
                h->gexec = nullptr;
                h->graph_failed = true;
            }
        }
        while (h->gexec && left >= h->gsteps) {
            HIP_OR_FAIL(h, hipGraphLaunch(h->gexec, h->stream));
            left -= h->gsteps;
            h->hstep += h->gsteps;
        }
    }
    for (; left > 0; left--) HIP_OR_FAIL(h, enqueue_step(h, nullptr, nullptr));
    return TCM_OK;
}

// Issue n steps directly, with HIP events around every stencil launch, and add
// their times to the statistics.  (Event records captured into a graph
// cannot be timed, so timed runs do not replay graphs.)
tcm_status issue_steps_timed(tcm_handle* h, int n) {
    while ((int)h->events.size() < 2 * n) {
        hipEvent_t e;
        HIP_OR_FAIL(h, timing_event(&e));
        h->events.push_back(e);
    }
    for (int k = 0; k < n; k++)
        HIP_OR_FAIL(h, enqueue_step(h, h->events[2 * k], h->events[2 * k + 1]));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < n; k++) {
        float ms = 0.f;
        HIP_OR_FAIL(h, hipEventElapsedTime(&ms, h->events[2 * k], h->events[2 * k + 1]));
        h->stencil_ms += ms;
    }
    h->stencil_launches += n;
    return TCM_OK;
}

// ---- sources ----------------------------------------------------------------
// The device source table holds the sources ordered by key (block key for the
// block engine, node for the dense engine), keeping the order in which
// sources of one key were added; a source block's slot records the range of
// its own sources in that table (packed as count << 24 | first), so the
// stencil visits only those, in the order they were added.
constexpr int SRC_RANGE_MAX = 127;          // sources of one block
constexpr int SRC_FIRST_MAX = 1 << 24;      // table entries

struct SrcKeyInfo {
    int first = 0, count = 0;
    int pin = 0;                            // largest t0 + ns of its sources
};

// Sorted device copy of h->h_src and the range of every key; uploads the
// table and the samples.  TCM_E_ARG if a block holds too many sources.
tcm_status upload_sources(tcm_handle* h, std::map<long long, SrcKeyInfo>* ranges) {
    const size_t ns = h->h_src.size();
    if (ns > (size_t)SRC_FIRST_MAX) return set_err(h, TCM_E_ARG, "too many sources");
    std::vector<int> ord(ns);
    for (size_t i = 0; i < ns; i++) ord[i] = (int)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return h->h_src[x].key < h->h_src[y].key; });
    std::vector<Src> sorted(ns);
    ranges->clear();
    for (size_t i = 0; i < ns; i++) {
        sorted[i] = h->h_src[ord[i]];
        SrcKeyInfo& r = (*ranges)[sorted[i].key];
        if (r.count == 0) r.first = (int)i;
        r.count++;
        r.pin = std::max(r.pin, sorted[i].t0 + sorted[i].ns);
        if (r.count > SRC_RANGE_MAX) return set_err(h, TCM_E_ARG, fmt("more than %d sources in one block", SRC_RANGE_MAX));
    }
    if (ns > h->d_src_cap) {
        size_t c = std::max<size_t>(16, h->d_src_cap * 2);
        while (c < ns) c *= 2;
        Src* d = nullptr;
        if (dalloc(h, &d, c) != hipSuccess) return set_err(h, TCM_E_NOMEM, "no device memory for the source table");
        dfree(h, h->d_src);
        h->d_src = d;
        h->d_src_cap = c;
    }
    if (h->h_srcw.size() > h->d_srcw_cap) {
        size_t c = std::max<size_t>(1024, h->d_srcw_cap * 2);
        while (c < h->h_srcw.size()) c *= 2;
        float* d = nullptr;
        if (dalloc(h, &d, c) != hipSuccess) return set_err(h, TCM_E_NOMEM, "no device memory for the source samples");
        dfree(h, h->d_srcw);
        h->d_srcw = d;
        h->d_srcw_cap = c;
    }
    if (ns) HIP_OR_FAIL(h, hipMemcpyAsync(h->d_src, sorted.data(), ns * sizeof(Src), hipMemcpyHostToDevice, h->stream));
    if (!h->h_srcw.empty())
        HIP_OR_FAIL(h, hipMemcpyAsync(h->d_srcw, h->h_srcw.data(), h->h_srcw.size() * sizeof(float),
                                      hipMemcpyHostToDevice, h->stream));
    // pageable copies return once the data are staged: the vectors may go
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    h->t.src = h->d_src;
    h->t.srcw = h->d_srcw;
    h->t.nsrc = (int)ns;
    drop_graph(h);
    return TCM_OK;
}

// One launch over a list of block requests (launch_activate_list).
tcm_status run_activation(tcm_handle* h, const std::vector<long long>& keys, const std::vector<int>& kshot,
                          const std::vector<unsigned>& kloc, const std::vector<int>& kpin,
                          const std::vector<int>& krange) {
    const size_t nk = keys.size();
    if (nk == 0) return TCM_OK;
    const size_t need = nk * (sizeof(long long) + 4 * sizeof(int));
    if (need > h->d_act_req_cap) {
        if (h->d_act_req) (void)hipFree(h->d_act_req);
        h->d_act_req = nullptr;
        h->d_act_req_cap = 0;
        if (hipMalloc(&h->d_act_req, need) != hipSuccess) {
            (void)hipGetLastError();
            return set_err(h, TCM_E_NOMEM, "no device memory for the source activation list");
        }
        h->d_act_req_cap = need;
    }
    std::vector<char> req(need);
    memcpy(req.data(), keys.data(), nk * sizeof(long long));
    memcpy(req.data() + nk * 8, kshot.data(), nk * 4);
    memcpy(req.data() + nk * 12, kloc.data(), nk * 4);
    memcpy(req.data() + nk * 16, kpin.data(), nk * 4);
    memcpy(req.data() + nk * 20, krange.data(), nk * 4);
    char* d = (char*)h->d_act_req;
    HIP_OR_FAIL(h, hipMemcpyAsync(d, req.data(), need, hipMemcpyHostToDevice, h->stream));
    HIP_OR_FAIL(h, launch_activate_list(h->t, (const long long*)d, (const int*)(d + nk * 8),
                                        (const unsigned*)(d + nk * 12), (const int*)(d + nk * 16),
                                        (const int*)(d + nk * 20), (int)nk, h->stream));
    HIP_OR_FAIL(h, launch_refresh_rows(h->t, h->stream));
    return sync_state(h);      // also keeps the request list alive until the launch has run
}

// Add n point sources at once ("Source insertion"): source k is at
// xyz[3k..3k+2] of shot shots[k] with samples w[k * ns .. k * ns + ns).  The
// table is uploaded once, and the blocks to box (each source block, and with
// an update interval above one the 26 blocks around it, since the source
// reaches them before the next update) are activated by one launch, each
// distinct block once with the largest pin among its sources; blocks of
// earlier sources only receive their new ranges.
tcm_status add_sources(tcm_handle* h, int n, const int* shots, const int* xyz, const float* w, int ns) {
    if (n < 0 || ns < 0 || (n > 0 && (!shots || !xyz)) || (n > 0 && ns > 0 && !w))
        return set_err(h, TCM_E_ARG, "bad source samples");
    for (int k = 0; k < n; k++) {
        if (shots[k] < 0 || shots[k] >= (int)h->shots.size()) return set_err(h, TCM_E_RANGE, "shot index out of range");
        const Shot& S = h->shots[shots[k]];
        const int ix = xyz[3 * k], iy = xyz[3 * k + 1], iz = xyz[3 * k + 2];
        if (ix < 0 || iy < 0 || iz < 0 || ix >= S.nx || iy >= S.ny || iz >= S.nz)
            return set_err(h, TCM_E_RANGE, fmt("source (%d,%d,%d) outside the %dx%dx%d grid", ix, iy, iz, S.nx, S.ny, S.nz));
    }
    for (size_t k = 0; k < (size_t)n * ns; k++)
        if (!std::isfinite(w[k])) return set_err(h, TCM_E_ARG, "source sample not finite");
    if (n == 0) return TCM_OK;
    tcm_status st;
    if (h->engine == TCM_ENGINE_BLOCKS) {
        st = sync_state(h);
        if (st) return st;
    }
    const long long step = current_step(h);
    const size_t keep_src = h->h_src.size(), keep_w = h->h_srcw.size();
    // block requests: global key -> (shot, key inside the shot, pin); pin -1:
    // an earlier source block, whose range is refreshed if it is active
    std::map<long long, size_t> at;
    std::vector<long long> keys;
    std::vector<int> kshot, kpin, krange;
    std::vector<unsigned> kloc;
    auto want = [&](int shot, int bx, int by, int bz, int pin) {
        const Shot& S = h->shots[shot];
        const unsigned tile = ((unsigned)(bz >> 2) * S.ty + (unsigned)(by >> 2)) * S.tx + (unsigned)(bx >> 2);
        const unsigned lk = tile * 64u + ((unsigned)(bz & 3) << 4) + ((unsigned)(by & 3) << 2) + (unsigned)(bx & 3);
        const long long G = S.key_base + lk;
        auto it = at.find(G);
        if (it != at.end()) {
            kpin[it->second] = std::max(kpin[it->second], pin);
            return;
        }
        at[G] = keys.size();
        keys.push_back(G);
        kshot.push_back(shot);
        kloc.push_back(lk);
        kpin.push_back(pin);
        krange.push_back(-1);
    };
    std::map<long long, std::pair<int, unsigned>> key_shot;    // source keys of this call: shot, local key
    for (int k = 0; k < n; k++) {
        const Shot& S = h->shots[shots[k]];
        const int ix = xyz[3 * k], iy = xyz[3 * k + 1], iz = xyz[3 * k + 2];
        Src e{};
        if (h->engine == TCM_ENGINE_DENSE) {
            e.key = (long long)ix + (long long)S.nx * ((long long)iy + (long long)S.ny * iz);
            e.local = 0;
        } else {
            const int bx = ix >> 3, by = iy >> 3, bz = iz >> 3;
            const unsigned tile = ((unsigned)(bz >> 2) * S.ty + (unsigned)(by >> 2)) * S.tx + (unsigned)(bx >> 2);
            e.key = S.key_base + tile * 64u + ((unsigned)(bz & 3) << 4) + ((unsigned)(by & 3) << 2) + (unsigned)(bx & 3);
            e.local = ((iz & 7) * 8 + (iy & 7)) * 8 + (ix & 7);
            want(shots[k], bx, by, bz, (int)(step + ns));
            if (h->t.interval > 1) {
                for (int d = 0; d < 27; d++) {
                    const int x2 = bx + d % 3 - 1, y2 = by + (d / 3) % 3 - 1, z2 = bz + d / 9 - 1;
                    if (d == 13 || x2 < 0 || y2 < 0 || z2 < 0 || x2 >= S.bx || y2 >= S.by || z2 >= S.bz) continue;
                    want(shots[k], x2, y2, z2, 0);
                }
            }
        }
        e.t0 = (int)step;
        e.ns = ns;
        e.pad = 0;
        e.w_off = (long long)h->h_srcw.size();
        h->h_srcw.insert(h->h_srcw.end(), w + (size_t)k * ns, w + (size_t)(k + 1) * ns);
        h->h_src.push_back(e);
    }
    std::map<long long, SrcKeyInfo> ranges;
    st = upload_sources(h, &ranges);
    if (st) {
        h->h_src.resize(keep_src);
        h->h_srcw.resize(keep_w);
        std::map<long long, SrcKeyInfo> r2;
        (void)upload_sources(h, &r2);
        return st;
    }
    if (h->engine != TCM_ENGINE_BLOCKS) return TCM_OK;
    // every source block receives its (possibly moved) range
    auto packed = [](const SrcKeyInfo& r) { return (r.count << 24) | r.first; };
    for (const auto& kv : ranges) {
        auto it = at.find(kv.first);
        if (it != at.end()) {
            krange[it->second] = packed(kv.second);
        } else {                                    // an earlier source's block: refresh only
            at[kv.first] = keys.size();
            keys.push_back(kv.first);
            kshot.push_back(0);
            kloc.push_back(0);
            kpin.push_back(-1);
            krange.push_back(packed(kv.second));
        }
    }
    st = run_activation(h, keys, kshot, kloc, kpin, krange);
    if (st) return st;
    if (h->h_state->add_error) {
        // no slot for some block: the sources are not added (blocks boxed so
        // far stay, as zero blocks, and are released when they stay quiet);
        // the table is cut back, earlier source blocks get their ranges back
        // and the blocks of only the dropped sources lose pin and range
        HIP_OR_FAIL(h, hipMemsetAsync(&h->t.st->add_error, 0, sizeof(int), h->stream));
        h->h_src.resize(keep_src);
        h->h_srcw.resize(keep_w);
        std::map<long long, SrcKeyInfo> back;
        st = upload_sources(h, &back);
        if (st) return st;
        std::vector<long long> k2;
        std::vector<int> s2, p2, r2;
        std::vector<unsigned> l2;
        for (const auto& kv : ranges) {
            auto it = back.find(kv.first);
            k2.push_back(kv.first);
            s2.push_back(0);
            l2.push_back(0);
            p2.push_back(it == back.end() ? -2 : -1);
            r2.push_back(it == back.end() ? -1 : packed(it->second));
        }
        st = run_activation(h, k2, s2, l2, p2, r2);
        if (st) return st;
        return set_err(h, TCM_E_POOL, "no free pool slot for a source block");
    }
    return TCM_OK;
}

// Tables for the adjoint field: same shots and media (shared), own pool.
// The adjoint field runs at threshold 0, whatever the forward's levels: its
// scale (C2_r times the residual) has nothing to do with theirs, and at
// threshold 0 the TCM of the adjoint field is exact, with the activation
// update every 8 steps (the 26-neighbour lookahead: exact at threshold 0,
// and a management pass on one step in eight).
tcm_status make_adjoint_handle(tcm_handle* h) {
    tcm_handle* a = new tcm_handle();
    a->cfg = h->cfg;
    a->cfg.checkpoint_every = 0;
    a->cfg.flags = TCM_FLAG_NO_GRAPH | (h->cfg.flags & (TCM_FLAG_NO_UNIFORM_C2 | TCM_FLAG_C2_PLANES));
    a->cfg.device_pool = nullptr;           // a capped forward pool caps the adjoint field's alike

    a->cfg.trigger = a->cfg.retire = 0.f;
    a->cfg.trigger_rel = a->cfg.retire_rel = 0.f;
    a->cfg.shutdown_steps = 0;
    a->cfg.trigger_interval = BE;
    a->cfg.stream = h->stream;
    a->engine = TCM_ENGINE_BLOCKS;
    a->device = h->device;
    a->ncu = h->ncu;
    a->stream = h->stream;
    a->own_stream = false;
    a->hshots = h->hshots;
    a->shots = h->shots;
    a->d_shots = h->d_shots;            // owned by h
    if (hipHostMalloc((void**)&a->h_state, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        delete a;
        return set_err(h, TCM_E_NOMEM, "pinned host allocation failed");
    }
    long long word_base = 0;
    for (const Shot& S : a->shots) word_base += S.nwords;
    tcm_status st = setup_engine(a, word_base);
    if (st != TCM_OK) {
        std::string m = a->err;
        destroy_all(a);
        return set_err(h, st, "adjoint tables: " + m);
    }
    h->adj = a;
    return TCM_OK;
}
}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

const char* tcm_version(void) { return "tcm-mi355x 0.1 (gfx950)"; }

tcm_status tcm_hbm_probe(const float* src, float* dst, uint64_t n, int32_t nread, int32_t wg_per_cu,
                         int32_t reps, void* stream, float* best_ms) {
    if (!src || !dst || !best_ms) return set_err(nullptr, TCM_E_ARG, "hbm probe: NULL pointer");
    const uint64_t chunk = (uint64_t)tcmk::hbm_probe_chunk();
    if (n == 0 || n % chunk) return set_err(nullptr, TCM_E_ARG, fmt("hbm probe: n must be a positive multiple of %llu", (unsigned long long)chunk));
    if (nread < 1 || nread > 3) return set_err(nullptr, TCM_E_ARG, "hbm probe: nread must be 1, 2 or 3");
    if (wg_per_cu < 0 || wg_per_cu > 32) return set_err(nullptr, TCM_E_ARG, "hbm probe: wg_per_cu must be 0..32");
    if (reps < 1 || reps > 1000) return set_err(nullptr, TCM_E_ARG, "hbm probe: reps must be 1..1000");
    if (((uintptr_t)src | (uintptr_t)dst) & 7u) return set_err(nullptr, TCM_E_ARG, "hbm probe: src and dst must be 8-byte aligned");
    const uintptr_t s0 = (uintptr_t)src, s1 = s0 + (uintptr_t)nread * n * sizeof(float);
    const uintptr_t d0 = (uintptr_t)dst, d1 = d0 + (uintptr_t)n * sizeof(float);
    if (d0 < s1 && s0 < d1) return set_err(nullptr, TCM_E_ARG, "hbm probe: dst overlaps src");
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return dev_fail(nullptr, e, "hbm probe: device query");
    const int grid = std::max(1, ncu * (wg_per_cu ? wg_per_cu : 8));
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = timing_event(&e0);
    if (e == hipSuccess) e = timing_event(&e1);
    float best = -1.0f;
    for (int r = 0; r < reps && e == hipSuccess; r++) {
        e = tcmk::launch_hbm_probe(src, dst, (long long)n, nread, grid, s, e0, e1);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && (best < 0.0f || ms < best)) best = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return dev_fail(nullptr, e, "hbm probe");
    *best_ms = best;
    return TCM_OK;
}

const char* tcm_last_error(const tcm_handle* h) {
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

tcm_status tcm_create(const tcm_config* cfg, const tcm_media* media, tcm_handle** out) {
    if (!cfg) return set_err(nullptr, TCM_E_ARG, "config is NULL");
    if (!media) return set_err(nullptr, TCM_E_ARG, "media is NULL");
    tcm_shot s{};
    s.nx = cfg->nx; s.ny = cfg->ny; s.nz = cfg->nz;
    s.media = *media;
    return create_common(cfg, &s, 1, out);
}

tcm_status tcm_create_batch(const tcm_config* cfg, const tcm_shot* shots, int32_t nshots, tcm_handle** out) {
    return create_common(cfg, shots, nshots, out);
}

void tcm_destroy(tcm_handle* h) { destroy_all(h); }

tcm_status tcm_add_source_shot(tcm_handle* h, int32_t shot, int32_t ix, int32_t iy, int32_t iz,
                               const float* w, int32_t nsamples) {
    tcm_status st = check_live(h);
    if (st) return st;
    const int xyz[3] = {ix, iy, iz};
    return add_sources(h, 1, &shot, xyz, w, nsamples);
}

tcm_status tcm_add_source(tcm_handle* h, int32_t ix, int32_t iy, int32_t iz, const float* w, int32_t nsamples) {
    return tcm_add_source_shot(h, 0, ix, iy, iz, w, nsamples);
}

tcm_status tcm_set_receivers(tcm_handle* h, const int32_t* xyz, const int32_t* rec_shot, int32_t nrec) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (nrec < 0 || (nrec > 0 && !xyz)) return set_err(h, TCM_E_ARG, "bad receiver array");
    std::vector<Rec> rec(nrec);
    for (int r = 0; r < nrec; r++) {
        const int s = rec_shot ? rec_shot[r] : 0;
        if (s < 0 || s >= (int)h->shots.size()) return set_err(h, TCM_E_RANGE, "receiver shot out of range");
        const Shot& S = h->shots[s];
        const int x = xyz[3 * r], y = xyz[3 * r + 1], z = xyz[3 * r + 2];
        if (x < 0 || y < 0 || z < 0 || x >= S.nx || y >= S.ny || z >= S.nz)
            return set_err(h, TCM_E_RANGE, fmt("receiver %d at (%d,%d,%d) outside the grid", r, x, y, z));
        if (h->engine == TCM_ENGINE_DENSE) {
            rec[r].key = (long long)x + (long long)S.nx * ((long long)y + (long long)S.ny * z);
            rec[r].local = 0;
        } else {
            const int bx = x >> 3, by = y >> 3, bz = z >> 3;
            const unsigned tile = ((unsigned)(bz >> 2) * S.ty + (unsigned)(by >> 2)) * S.tx + (unsigned)(bx >> 2);
            rec[r].key = S.key_base + tile * 64u + ((unsigned)(bz & 3) << 4) + ((unsigned)(by & 3) << 2) + (unsigned)(bx & 3);
            rec[r].local = ((z & 7) * 8 + (y & 7)) * 8 + (x & 7);
        }
    }
    if (h->engine == TCM_ENGINE_BLOCKS) {
        st = sync_state(h);
        if (st) return st;
    }
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    dfree(h, h->d_rec);
    dfree(h, h->d_traces);
    h->d_rec = nullptr;
    h->d_traces = nullptr;
    h->h_rec = rec;
    h->rec_xyz.assign(xyz, xyz + 3 * (size_t)nrec);
    h->rec_shot.assign((size_t)nrec, 0);
    if (rec_shot) h->rec_shot.assign(rec_shot, rec_shot + nrec);
    h->t.rec = nullptr;
    h->t.traces = nullptr;
    h->t.trace_cap = 0;
    h->t.nrec = nrec;
    h->t.trace_step0 = (int)current_step(h);
    if (nrec > 0) {
        HIP_OR_FAIL(h, dalloc(h, &h->d_rec, nrec));
        HIP_OR_FAIL(h, hipMemcpy(h->d_rec, rec.data(), nrec * sizeof(Rec), hipMemcpyHostToDevice));
        h->t.rec = h->d_rec;
        st = ensure_trace_capacity(h, 1024);
        if (st) return st;
    }
    drop_graph(h);
    return TCM_OK;
}

// The sticky device error of a state copy: a pool or table failure, else a
// non-finite value written by the stencil (0: none).
int dev_error(const DevState& d) { return d.error ? d.error : d.nf_step ? ERR_NONFINITE : 0; }

tcm_status report_device_error(tcm_handle* h) {
    const DevState& d = *h->h_state;
    const int code = dev_error(d);
    const long long at = d.error ? (long long)d.err_step + 1 : (long long)d.nf_step;
    if (code == ERR_NONFINITE)
        return set_err(h, TCM_E_NONFINITE, fmt("a field value that is not finite appeared at step %lld; the "
                                               "field is kept at that step and later steps do nothing", at));
    if (code == ERR_POOL)
        return set_err(h, TCM_E_POOL, fmt("pool of %d slots exhausted at step %lld; the field is kept at that step",
                                          h->t.cap, at));
    return set_err(h, (tcm_status)code, fmt("device error %d at step %lld", code, at));
}

tcm_status tcm_step(tcm_handle* h, int32_t nsteps) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (nsteps < 0) return set_err(h, TCM_E_ARG, "nsteps < 0");
    if (nsteps == 0) return TCM_OK;
    const bool timing = (h->cfg.flags & TCM_FLAG_TIMING) != 0;

    if (h->engine == TCM_ENGINE_DENSE) {
        st = ensure_trace_capacity(h, h->dense_step + nsteps - h->t.trace_step0);
        if (st) return st;
        if (timing) {
            while ((int)h->events.size() < 2 * nsteps) {
                hipEvent_t e;
                HIP_OR_FAIL(h, timing_event(&e));
                h->events.push_back(e);
            }
        }
        for (int k = 0; k < nsteps; k++)
            HIP_OR_FAIL(h, enqueue_dense_step(h, timing ? h->events[2 * k] : nullptr, timing ? h->events[2 * k + 1] : nullptr));
        HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
        if (timing) {
            const Shot& S = h->shots[0];
            for (int k = 0; k < nsteps; k++) {
                float ms = 0.f;
                HIP_OR_FAIL(h, hipEventElapsedTime(&ms, h->events[2 * k], h->events[2 * k + 1]));
                h->stencil_ms += ms;
            }
            h->stencil_launches += nsteps;
            h->stencil_cells += (long long)nsteps * S.nx * S.ny * S.nz;
        }
        return TCM_OK;
    }

    st = sync_state(h);
    if (st) return st;
    if (dev_error(*h->h_state)) return report_device_error(h);
    st = ensure_trace_capacity(h, h->h_state->step + (long long)nsteps - h->t.trace_step0);
    if (st) return st;
    // nodes stepped by this call: the lists C_0 .. C_{n-1} it runs (the list
    // left for the next call is not stepped here)
    const unsigned long long upd0 = h->h_state->updates;
    const unsigned long long updu0 = h->h_state->updates_u, updl0 = h->h_state->updates_l;
    h->hstep = h->h_state->step;

    // one run of n steps: graph replay, or direct launches with HIP events
    // around every stencil launch when timing
    auto run_chunk = [&](int n) -> tcm_status {
        return timing ? issue_steps_timed(h, n) : issue_steps(h, n);
    };
    if (h->cfg.checkpoint_every > 0 && !h->in_adjoint) {
        // stop at every checkpoint level and copy the state before stepping on
        const int K = h->cfg.checkpoint_every;
        long long cur = h->h_state->step;
        int left = nsteps;
        while (left > 0) {
            if (cur % K == 0) {
                const size_t idx = (size_t)(cur / K);
                if (h->ckpts.size() <= idx) h->ckpts.resize(idx + 1);
                if (h->ckpts[idx].step != cur) {
                    st = ck_save(h, h->ckpts[idx]);
                    if (st) return st;
                }
            }
            const int chunk = (int)std::min<long long>(left, K - cur % K);
            st = run_chunk(chunk);
            if (st) return st;
            st = sync_state(h);
            if (st) return st;
            if (dev_error(*h->h_state)) break;
            cur = h->h_state->step;
            h->hstep = cur;
            left -= chunk;
        }
    } else {
        st = run_chunk(nsteps);
        if (st) return st;
    }
    st = sync_state(h);
    if (st) return st;
    if (timing) {
        h->stencil_cells += (long long)(h->h_state->updates - upd0);
        h->stencil_cells_u += (long long)(h->h_state->updates_u - updu0);
        h->stencil_cells_l += (long long)(h->h_state->updates_l - updl0);
    }
    if (dev_error(*h->h_state)) return report_device_error(h);
    if (h->cfg.flags & TCM_FLAG_DEBUG_CHECKS) {
        int64_t bad = 0;
        st = tcm_check(h, &bad);
        if (st) return st;
        if (bad) return set_err(h, TCM_E_STATE, fmt("table invariants violated (%lld) after step %lld",
                                                    (long long)bad, (long long)h->h_state->step));
    }
    return TCM_OK;
}

tcm_status tcm_check(tcm_handle* h, int64_t* violations) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (!violations) return set_err(h, TCM_E_ARG, "violations is NULL");
    if (h->engine != TCM_ENGINE_BLOCKS) return set_err(h, TCM_E_STATE, "tcm_check applies to the block engine");
    st = sync_state(h);
    if (st) return st;
    int* mark = nullptr;
    unsigned long long* bad = nullptr;
    if (hipMalloc((void**)&mark, sizeof(int) * (size_t)h->t.cap) != hipSuccess ||
        hipMalloc((void**)&bad, 2 * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        if (mark) (void)hipFree(mark);
        return set_err(h, TCM_E_NOMEM, "no device memory for the check");
    }
    unsigned long long res[2] = {0, 0};
    hipError_t e = launch_fill_int(mark, h->t.cap, 0, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof res, h->stream);
    if (e == hipSuccess) e = launch_check(h->t, mark, bad, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(res, bad, sizeof res, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(mark);
    (void)hipFree(bad);
    if (e != hipSuccess) return dev_fail(h, e, "tcm_check");
    const int n_act = h->h_state->n_act;
    *violations = (int64_t)res[0] + (res[1] != (unsigned long long)n_act ? 1 : 0) +
                  (n_act < 0 || n_act > h->t.cap ? 1 : 0);
    return TCM_OK;
}

tcm_status tcm_read_shot(tcm_handle* h, int32_t shot, int32_t which, int32_t x0, int32_t y0, int32_t z0,
                         int32_t sx, int32_t sy, int32_t sz, float* out, int32_t out_is_device) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (shot < 0 || shot >= (int)h->shots.size()) return set_err(h, TCM_E_RANGE, "shot index out of range");
    if (which != 0 && which != 1) return set_err(h, TCM_E_ARG, "which must be 0 (phi^n) or 1 (phi^{n-1})");
    const Shot& S = h->shots[shot];
    if (sx < 0 || sy < 0 || sz < 0 || x0 < 0 || y0 < 0 || z0 < 0 || x0 + (long long)sx > S.nx ||
        y0 + (long long)sy > S.ny || z0 + (long long)sz > S.nz)
        return set_err(h, TCM_E_RANGE, "read box outside the grid");
    const size_t count = (size_t)sx * sy * sz;
    if (count == 0) return TCM_OK;
    if (!out) return set_err(h, TCM_E_ARG, "out is NULL");
    float* dst = out;
    if (!out_is_device) {
        st = scratch(h, count * sizeof(float), &dst);
        if (st) return st;
    }
    if (h->engine == TCM_ENGINE_DENSE) {
        const long long n = h->dense_step;
        const float* f = h->d_phi[which == 0 ? (n & 1) : 1 - (n & 1)];
        HIP_OR_FAIL(h, launch_read_dense(f, S.nx, S.ny, x0, y0, z0, sx, sy, sz, dst, h->stream));
    } else {
        HIP_OR_FAIL(h, launch_read(h->t, shot, which, x0, y0, z0, sx, sy, sz, dst, h->stream));
    }
    if (!out_is_device) {
        HIP_OR_FAIL(h, hipMemcpyAsync(out, dst, count * sizeof(float), hipMemcpyDeviceToHost, h->stream));
        HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    }
    return TCM_OK;
}

tcm_status tcm_read(tcm_handle* h, int32_t which, int32_t x0, int32_t y0, int32_t z0, int32_t sx, int32_t sy,
                    int32_t sz, float* out, int32_t out_is_device) {
    return tcm_read_shot(h, 0, which, x0, y0, z0, sx, sy, sz, out, out_is_device);
}

tcm_status tcm_read_noalloc(tcm_handle* h, int32_t shot, int32_t which, int32_t x0, int32_t y0, int32_t z0,
                            int32_t sx, int32_t sy, int32_t sz, float* out) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (shot < 0 || shot >= (int)h->shots.size()) return set_err(h, TCM_E_RANGE, "shot index out of range");
    if (which != 0 && which != 1) return set_err(h, TCM_E_ARG, "which must be 0 (phi^n) or 1 (phi^{n-1})");
    const Shot& S = h->shots[shot];
    if (sx < 0 || sy < 0 || sz < 0 || x0 < 0 || y0 < 0 || z0 < 0 || x0 + (long long)sx > S.nx ||
        y0 + (long long)sy > S.ny || z0 + (long long)sz > S.nz)
        return set_err(h, TCM_E_RANGE, "read box outside the grid");
    const long long count = (long long)sx * sy * sz;
    if (count == 0) return TCM_OK;
    if (count > NOALLOC_FLOATS)
        return set_err(h, TCM_E_ARG, fmt("box of %lld nodes exceeds the %lld-node staging array of "
                                         "tcm_read_noalloc", count, NOALLOC_FLOATS));
    if (!out) return set_err(h, TCM_E_ARG, "out is NULL");
    float* stage = nullptr;
    HIP_OR_FAIL(h, noalloc_staging(&stage));
    if (h->engine == TCM_ENGINE_DENSE) {
        const long long n = h->dense_step;
        const float* f = h->d_phi[which == 0 ? (n & 1) : 1 - (n & 1)];
        HIP_OR_FAIL(h, launch_read_dense(f, S.nx, S.ny, x0, y0, z0, sx, sy, sz, stage, h->stream));
    } else {
        HIP_OR_FAIL(h, launch_read(h->t, shot, which, x0, y0, z0, sx, sy, sz, stage, h->stream));
    }
    HIP_OR_FAIL(h, hipMemcpyAsync(out, stage, (size_t)count * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    return TCM_OK;
}

tcm_status tcm_read_traces(tcm_handle* h, float* out, int32_t out_is_device, int32_t* nsteps) {
    tcm_status st = check_live(h);
    if (st) return st;
    long long cur = 0;
    if (h->engine == TCM_ENGINE_BLOCKS) {
        st = sync_state(h);
        if (st) return st;
        cur = h->h_state->step;
    } else {
        HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
        cur = h->dense_step;
    }
    long long rows = cur - h->t.trace_step0;
    if (rows < 0 || h->t.nrec == 0) rows = 0;
    if (rows > h->t.trace_cap) rows = h->t.trace_cap;
    if (nsteps) *nsteps = (int32_t)rows;
    if (!out || rows == 0) return TCM_OK;
    const size_t bytes = (size_t)rows * h->t.nrec * sizeof(float);
    HIP_OR_FAIL(h, hipMemcpyAsync(out, h->d_traces, bytes, out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    return TCM_OK;
}

tcm_status tcm_stats(tcm_handle* h, tcm_stats_t* o) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (!o) return set_err(h, TCM_E_ARG, "out is NULL");
    memset(o, 0, sizeof *o);
    o->nshots = (int32_t)h->shots.size();
    o->stencil_ms = h->stencil_ms;
    o->stencil_launches = h->stencil_launches;
    o->stencil_cells = h->stencil_cells;
    o->stencil_cells_uniform = h->stencil_cells_u;
    o->stencil_cells_lattice = h->stencil_cells_l;
    o->grad_cells = h->grad_cells;
    o->adjoint_field_ms = h->af_ms;
    o->adjoint_field_launches = h->af_launches;
    o->adjoint_field_cells = h->af_cells;
    o->adjoint_field_cells_uniform = h->af_cells_u;
    o->adjoint_field_cells_lattice = h->af_cells_l;
    o->recompute_ms = h->rec_ms;
    o->recompute_launches = h->rec_launches;
    o->recompute_cells = h->rec_cells;
    o->recompute_cells_uniform = h->rec_cells_u;
    o->recompute_cells_lattice = h->rec_cells_l;
    o->checkpoint_bytes = (int64_t)ck_stored_bytes(h);
    o->checkpoints = (int64_t)h->ckpts.size();
    o->adjoint_bytes = (int64_t)h->adjoint_bytes;
    o->table_bytes = (int64_t)h->table_bytes;
    if (h->engine == TCM_ENGINE_DENSE) {
        HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
        const Shot& S = h->shots[0];
        const long long N = (long long)S.nx * S.ny * S.nz;
        o->step = h->dense_step;
        o->active_blocks = (long long)S.bx * S.by * S.bz;
        o->peak_active_blocks = o->active_blocks;
        o->cell_updates = N * h->dense_step;
        return TCM_OK;
    }
    st = sync_state(h);
    if (st) return st;
    const DevState& d = *h->h_state;
    o->step = d.step;
    o->active_blocks = d.n_act;
    o->peak_active_blocks = d.peak_act;
    o->pool_slots = h->t.cap;
    o->pool_bytes = (int64_t)h->t.cap * (int64_t)SLOT_BYTES;
    o->peak_pool_bytes = (int64_t)d.peak_act * (int64_t)SLOT_BYTES;
    o->activations = (int64_t)d.activations;
    o->retirements = (int64_t)d.retirements;
    o->cell_updates = (int64_t)d.updates;
    o->uniform_cell_updates = (int64_t)d.updates_u;
    o->lattice_cell_updates = (int64_t)d.updates_l;
    o->decay_block_steps = (int64_t)d.decays;
    o->trigger_level = d.trig_cur;
    o->retire_level = d.ret_cur;
    o->error = dev_error(d);
    return TCM_OK;
}

// A caller-owned copy of a handle's state (tcm_snapshot / tcm_restore).
struct SnapImpl {
    tcm_handle* owner = nullptr;
    char* buf = nullptr;                // dense engine: both field arrays
    Ckpt ck;                            // block engine: sparse state copy
    long long hstep = 0, dense_step = 0;
    size_t nsrc = 0;
    int nrec = 0;
    long long media_gen = 0;
};

tcm_status tcm_reset(tcm_handle* h) {
    tcm_status st = check_live(h);
    if (st) return st;
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    drop_graph(h);
    ck_clear(h);
    h->rec_xyz.clear();
    h->rec_shot.clear();
    h->h_src.clear();
    h->h_srcw.clear();
    h->t.nsrc = 0;
    h->h_rec.clear();
    h->t.nrec = 0;
    h->t.trace_cap = 0;
    h->t.trace_step0 = 0;
    dfree(h, h->d_rec);
    dfree(h, h->d_traces);
    h->d_rec = nullptr;
    h->d_traces = nullptr;
    h->t.rec = nullptr;
    h->t.traces = nullptr;
    h->stencil_ms = 0.0;
    h->stencil_launches = 0;
    h->stencil_cells = 0;
    h->stencil_cells_u = 0;
    h->stencil_cells_l = 0;
    h->grad_cells = 0;
    h->af_ms = 0.0;
    h->af_launches = 0;
    h->af_cells = 0;
    h->af_cells_u = 0;
    h->af_cells_l = 0;
    h->rec_ms = 0.0;
    h->rec_launches = 0;
    h->rec_cells = 0;
    h->rec_cells_u = 0;
    h->rec_cells_l = 0;
    if (h->engine == TCM_ENGINE_DENSE) {
        const Shot& S = h->shots[0];
        const size_t N = (size_t)S.nx * S.ny * S.nz;
        HIP_OR_FAIL(h, hipMemsetAsync(h->d_phi[0], 0, N * sizeof(float), h->stream));
        HIP_OR_FAIL(h, hipMemsetAsync(h->d_phi[1], 0, N * sizeof(float), h->stream));
        h->dense_step = 0;
    } else {
        HIP_OR_FAIL(h, launch_init_tables(h->t, h->nkeys, h->stream));
    }
    h->hstep = 0;
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    return TCM_OK;
}

tcm_status tcm_set_media(tcm_handle* h, int32_t shot, const tcm_media* media) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (!media) return set_err(h, TCM_E_ARG, "media is NULL");
    if (shot < 0 || shot >= (int)h->shots.size()) return set_err(h, TCM_E_RANGE, "shot index out of range");
    Shot& S = h->shots[shot];
    if (media->kind != S.media_kind) return set_err(h, TCM_E_ARG, "the media kind differs from the shot's");
    if (media->kind == TCM_MEDIA_LAYERED && media->nlayers != S.nlayers)
        return set_err(h, TCM_E_ARG, "the layer count differs from the shot's");
    if (media->kind == TCM_MEDIA_LATTICE &&
        (media->lx != S.lx || media->ly != S.ly || media->lz != S.lz || media->log2_spacing != S.log2s))
        return set_err(h, TCM_E_ARG, "the lattice size or spacing differs from the shot's");
    std::string why;
    double cmax = 0.0;
    st = validate_media(media, S.nx, S.ny, S.nz, &cmax, &why);
    if (st) return set_err(h, st, why);
    const double r = cmax * h->cfg.dt / h->cfg.dx;
    if (r * r * 3.0 > 1.0 + 4.0 * DBL_EPSILON)
        return set_err(h, TCM_E_CFL, fmt("eq.(4) violated: cmax dt / dx = %.9g > 1/sqrt(3)", r));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    // the shot's device media keep their buffers (same kind and sizes)
    if (media->kind == TCM_MEDIA_DENSE) {
        HIP_OR_FAIL(h, hipMemcpy((void*)S.c, media->c, (size_t)S.nx * S.ny * S.nz * sizeof(float),
                                 hipMemcpyHostToDevice));
    } else if (media->kind == TCM_MEDIA_LAYERED) {
        HIP_OR_FAIL(h, hipMemcpy((void*)S.z_top, media->z_top, S.nlayers * sizeof(int), hipMemcpyHostToDevice));
        HIP_OR_FAIL(h, hipMemcpy((void*)S.c_layer, media->c_layer, S.nlayers * sizeof(float), hipMemcpyHostToDevice));
    } else {
        HIP_OR_FAIL(h, hipMemcpy((void*)S.lattice, media->lattice, (size_t)S.lx * S.ly * S.lz * sizeof(double),
                                 hipMemcpyHostToDevice));
    }
    h->hshots[shot].cmax = cmax;
    h->media_gen++;
    // the adjoint field's pool holds C2 planes of the old media: made anew
    // by the next tcm_adjoint
    if (h->adj) {
        destroy_all(h->adj);
        h->adj = nullptr;
    }
    st = tcm_reset(h);
    if (st) return st;
    if (h->engine == TCM_ENGINE_DENSE) {
        HIP_OR_FAIL(h, launch_media_c2(S, h->d_shots, h->cfg.dt, h->cfg.dx, h->d_c2, h->stream));
    } else if (h->t.c2_ready) {
        HIP_OR_FAIL(h, launch_prefill_c2(h->t, h->nkeys, h->stream));
    }
    // (a capped pool fills a block's C2 plane when the block is activated)
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    return TCM_OK;
}

void tcm_snapshot_free(void* snap) {
    SnapImpl* s = (SnapImpl*)snap;
    if (!s) return;
    if (s->buf) (void)hipFree(s->buf);
    ck_free(s->ck);
    delete s;
}

tcm_status tcm_snapshot(tcm_handle* h, void** snap) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (!snap) return set_err(h, TCM_E_ARG, "snap is NULL");
    *snap = nullptr;
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    SnapImpl* s = new SnapImpl();
    s->owner = h;
    s->media_gen = h->media_gen;
    s->hstep = h->hstep;
    s->dense_step = h->dense_step;
    s->nsrc = h->h_src.size();
    s->nrec = h->t.nrec;
    auto fail = [&](tcm_status why) {
        tcm_snapshot_free(s);
        return why;
    };
    if (h->engine == TCM_ENGINE_DENSE) {
        const Shot& S = h->shots[0];
        const size_t N = (size_t)S.nx * S.ny * S.nz;
        if (hipMalloc((void**)&s->buf, 2 * N * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            s->buf = nullptr;
            return fail(set_err(h, TCM_E_NOMEM, "no device memory for the snapshot"));
        }
        hipError_t e = hipMemcpyAsync(s->buf, h->d_phi[0], N * sizeof(float), hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->buf + N * sizeof(float), h->d_phi[1], N * sizeof(float),
                               hipMemcpyDeviceToDevice, h->stream);
        if (e != hipSuccess) return fail(dev_fail(h, e, "snapshot copy"));
    } else {
        st = ck_save(h, s->ck);
        if (st) return fail(st);
    }
    const hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(dev_fail(h, e, "snapshot copy"));
    *snap = s;
    return TCM_OK;
}

tcm_status tcm_restore(tcm_handle* h, const void* snap) {
    tcm_status st = check_live(h);
    if (st) return st;
    const SnapImpl* s = (const SnapImpl*)snap;
    if (!s || s->owner != h) return set_err(h, TCM_E_ARG, "not a snapshot of this handle");
    if (s->media_gen != h->media_gen) return set_err(h, TCM_E_STATE, "the media changed after the snapshot");
    if (s->nsrc != h->h_src.size() || s->nrec != h->t.nrec)
        return set_err(h, TCM_E_STATE, "sources or receivers were added after the snapshot");
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    drop_graph(h);
    if (h->engine == TCM_ENGINE_DENSE) {
        const Shot& S = h->shots[0];
        const size_t N = (size_t)S.nx * S.ny * S.nz;
        HIP_OR_FAIL(h, hipMemcpyAsync(h->d_phi[0], s->buf, N * sizeof(float), hipMemcpyDeviceToDevice, h->stream));
        HIP_OR_FAIL(h, hipMemcpyAsync(h->d_phi[1], s->buf + N * sizeof(float), N * sizeof(float),
                                      hipMemcpyDeviceToDevice, h->stream));
        h->dense_step = s->dense_step;
    } else {
        st = ck_restore(h, s->ck);
        if (st) return st;
    }
    h->hstep = s->hstep;
    return sync_state(h);
}


tcm_status tcm_adjoint(tcm_handle* h, const float* resid, int32_t nt, int32_t resid_is_device,
                       float* grad_c, int32_t out_is_device) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (h->engine != TCM_ENGINE_BLOCKS || h->shots.size() != 1)
        return set_err(h, TCM_E_STATE, "tcm_adjoint runs on a single-shot block-engine handle");
    const int K = h->cfg.checkpoint_every;
    if (K <= 0) return set_err(h, TCM_E_STATE, "tcm_adjoint needs checkpoint_every > 0");
    const int nrec = h->t.nrec;
    if (nrec <= 0 || h->t.trace_step0 != 0)
        return set_err(h, TCM_E_STATE, "receivers must be set before the first step");
    if (!resid || !grad_c) return set_err(h, TCM_E_ARG, "resid and grad_c are required");
    st = sync_state(h);
    if (st) return st;
    if (dev_error(*h->h_state)) return set_err(h, TCM_E_STATE, "the forward run failed (pool or non-finite field)");
    const long long cur = h->h_state->step;
    if (nt <= 0 || nt > cur) return set_err(h, TCM_E_STATE, fmt("nt = %d outside the %lld recorded steps", nt, cur));
    const int nseg = (nt + K - 1) / K;
    if ((int)h->ckpts.size() < nseg) return set_err(h, TCM_E_STATE, "forward checkpoints missing (sources added after step 0?)");
    for (int j = 0; j < nseg; j++)
        if (h->ckpts[j].step != (long long)j * K) return set_err(h, TCM_E_STATE, "forward checkpoints missing");

    const Shot& S = h->shots[0];
    const size_t N = (size_t)S.nx * S.ny * S.nz;
    std::vector<float> r((size_t)nt * nrec);
    HIP_OR_FAIL(h, hipMemcpy(r.data(), resid, r.size() * sizeof(float),
                             resid_is_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    // C2 at the receivers (the adjoint sources are C2_r * resid)
    std::vector<float> c2r(nrec);
    {
        int* dx = nullptr;
        float* dc = nullptr;
        HIP_OR_FAIL(h, hipMalloc((void**)&dx, sizeof(int) * 3 * nrec));
        HIP_OR_FAIL(h, hipMalloc((void**)&dc, sizeof(float) * nrec));
        HIP_OR_FAIL(h, hipMemcpy(dx, h->rec_xyz.data(), sizeof(int) * 3 * nrec, hipMemcpyHostToDevice));
        HIP_OR_FAIL(h, launch_receiver_c2(h->d_shots, dx, nullptr, nrec, h->cfg.dt, h->cfg.dx, dc, h->stream));
        HIP_OR_FAIL(h, hipMemcpyAsync(c2r.data(), dc, sizeof(float) * nrec, hipMemcpyDeviceToHost, h->stream));
        HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
        (void)hipFree(dx);
        (void)hipFree(dc);
    }
    if (!h->adj) {
        st = make_adjoint_handle(h);
        if (st) return st;
    }
    tcm_handle* a = h->adj;
    st = tcm_reset(a);
    if (st) return set_err(h, st, std::string("adjoint tables: ") + a->err);
    a->hstep = 0;
    // the adjoint field runs at full occupancy (measured best for the sweep,
    // whose lists start at the receivers); the recomputation keeps the forward
    // handle's launch shape
    a->tile_w = 4;
    a->tile_p = 1;
    a->grid_step = std::min(GRAD_ACCUM_MAX_WG,
                            std::max(8, (a->ncu * std::max(1, block_step_occupancy(false, 4, 1, step_mode(a->t, STEP_GRAD)))) / 8 * 8));
    {
        // adjoint step k (k = 0..nt-1) produces mu^{nt-k}; its source sample at
        // receiver r is C2_r * resid[nt-1-k][r]; all receivers in one activation
        std::vector<float> w((size_t)nrec * nt);
        std::vector<int> zero_shot(nrec, 0);
        for (int q = 0; q < nrec; q++)
            for (int k = 0; k < nt; k++) w[(size_t)q * nt + k] = c2r[q] * r[(size_t)(nt - 1 - k) * nrec + q];
        st = add_sources(a, nrec, zero_shot.data(), h->rec_xyz.data(), w.data(), nt);
        if (st) return set_err(h, st, std::string("adjoint sources: ") + a->err);
    }
    // keep the caller's forward state
    Ckpt now;
    st = ck_save(h, now);
    if (st) return st;
    // L u^n of every forward step of a segment, one 512-float tile per list
    // entry (at most the run's largest list); per step a key -> entry map;
    // gradient blocks for at most the blocks ever activated in the forward
    const long long lapcap = std::max<long long>(1, h->h_state->peak_act);
    const long long nkeys = h->nkeys;
    const long long gcap = std::max<long long>(1, std::min<long long>(nkeys, (long long)h->h_state->activations));
    float* lap = nullptr;
    int* fidx = nullptr;
    float* gs = nullptr;
    double* gacc = nullptr;
    int* gslot = nullptr;
    unsigned long long* gterms = nullptr;
    int keep_grid_step = -1;
    auto cleanup = [&]() {
        if (keep_grid_step > 0) h->grid_step = keep_grid_step;
        for (void* q : {(void*)lap, (void*)fidx, (void*)gs, (void*)gacc, (void*)gslot, (void*)gterms})
            if (q) (void)hipFree(q);
        ck_free(now);
        h->in_adjoint = false;
        h->t.rec_lap = nullptr;
        h->t.rec_fidx = nullptr;
        a->t.g_lap = nullptr;
        a->t.g_fidx = nullptr;
        a->t.g_gs = nullptr;
        a->t.g_acc = nullptr;
        a->t.g_slot = nullptr;
        a->t.g_terms_wg = nullptr;
    };
    const size_t lap_b = sizeof(float) * (size_t)K * (size_t)lapcap * BV;
    const size_t fidx_b = sizeof(int) * (size_t)K * (size_t)nkeys;
    const size_t g_b = (sizeof(float) + sizeof(double)) * (size_t)gcap * BV + sizeof(int) * (size_t)nkeys;
    if (hipMalloc((void**)&lap, lap_b) != hipSuccess || hipMalloc((void**)&fidx, fidx_b) != hipSuccess ||
        hipMalloc((void**)&gs, sizeof(float) * (size_t)gcap * BV) != hipSuccess ||
        hipMalloc((void**)&gacc, sizeof(double) * (size_t)gcap * BV) != hipSuccess ||
        hipMalloc((void**)&gslot, sizeof(int) * (size_t)nkeys) != hipSuccess ||
        hipMalloc((void**)&gterms, sizeof(unsigned long long) * GRAD_ACCUM_MAX_WG) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return set_err(h, TCM_E_NOMEM, fmt("no device memory for the adjoint stores (%.2f GB)",
                                           (lap_b + fidx_b + g_b) / 1e9));
    }
    h->adjoint_bytes = lap_b + fidx_b + g_b + a->table_bytes + (size_t)a->t.cap * SLOT * sizeof(float);
    h->in_adjoint = true;
    const bool timing = (h->cfg.flags & TCM_FLAG_TIMING) != 0;
    while (timing && (int)h->gev.size() < 4 * K) {
        hipEvent_t ev;
        if (timing_event(&ev) != hipSuccess) {
            (void)hipGetLastError();
            cleanup();
            return set_err(h, TCM_E_DEVICE, "timing event creation failed");
        }
        h->gev.push_back(ev);
    }
    a->t.g_gs = gs;
    a->t.g_acc = gacc;
    a->t.g_slot = gslot;
    a->t.g_cap = (int)gcap;
    a->t.g_terms_wg = gterms;
    hipError_t e = launch_fill_int(gslot, nkeys, -1, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(gterms, 0, sizeof(unsigned long long) * GRAD_ACCUM_MAX_WG, h->stream);
    const unsigned long long a_upd0 = a->h_state->updates, a_updu0 = a->h_state->updates_u,
                             a_updl0 = a->h_state->updates_l;
    // the recomputing stencil keeps the forward's launch shape within its
    // own residency (a persistent grid beyond it would leave a tail)
    keep_grid_step = h->grid_step;
    h->grid_step = std::min(h->grid_step,
                            std::max(8, (h->ncu * std::max(1, block_step_occupancy(h->t.adaptive != 0, h->tile_w,
                                                                                   h->tile_p, step_mode(h->t, STEP_RECORD)))) / 8 * 8));
    for (int j = nseg - 1; j >= 0 && e == hipSuccess; j--) {
        const int s0 = j * K, end = std::min(s0 + K, nt);
        st = ck_restore(h, h->ckpts[j]);
        if (!st && timing) st = sync_state(h);
        if (st) { cleanup(); return st; }
        const unsigned long long rec_u0 = h->h_state->updates, rec_uu0 = h->h_state->updates_u,
                                 rec_ul0 = h->h_state->updates_l;
        h->hstep = s0;
        // recompute forward steps s0 .. end-1, storing L u^n (n = s0 .. end-1)
        e = launch_fill_int(fidx, (long long)(end - s0) * nkeys, -1, h->stream);
        for (int n = s0; n < end && e == hipSuccess; n++) {
            h->t.rec_lap = lap + (size_t)(n - s0) * (size_t)lapcap * BV;
            h->t.rec_fidx = fidx + (size_t)(n - s0) * (size_t)nkeys;
            h->t.rec_lapcap = (int)lapcap;
            const int q = n - s0;
            e = enqueue_step(h, timing ? h->gev[2 * K + 2 * q] : nullptr, timing ? h->gev[2 * K + 2 * q + 1] : nullptr);
        }
        h->t.rec_lap = nullptr;
        h->t.rec_fidx = nullptr;
        // adjoint levels mu^{end} .. mu^{s0+1}: the adjoint-field step that
        // forms mu^m also adds mu^m (L u^{m-1}) to the gradient
        for (int m = end; m > s0 && e == hipSuccess; m--) {
            const int q = end - m;
            a->t.g_lap = lap + (size_t)(m - 1 - s0) * (size_t)lapcap * BV;
            a->t.g_fidx = fidx + (size_t)(m - 1 - s0) * (size_t)nkeys;
            e = enqueue_step(a, timing ? h->gev[2 * q] : nullptr, timing ? h->gev[2 * q + 1] : nullptr);
            if (e == hipSuccess && (m - 1) % GRAD_GROUP == 0) e = launch_grad_flush(a->t, h->stream);
        }
        a->t.g_lap = nullptr;
        a->t.g_fidx = nullptr;
        if (timing && e == hipSuccess) {
            e = hipStreamSynchronize(h->stream);
            for (int q = 0; q < end - s0 && e == hipSuccess; q++) {
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, h->gev[2 * q], h->gev[2 * q + 1]);
                h->af_ms += ms;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, h->gev[2 * K + 2 * q], h->gev[2 * K + 2 * q + 1]);
                h->rec_ms += ms;
            }
            h->af_launches += end - s0;
            h->rec_launches += end - s0;
        }
        if (timing && e == hipSuccess) {
            // nodes the recomputation stepped in this segment
            st = sync_state(h);
            if (st) { cleanup(); return st; }
            h->rec_cells += (long long)(h->h_state->updates - rec_u0);
            h->rec_cells_u += (long long)(h->h_state->updates_u - rec_uu0);
            h->rec_cells_l += (long long)(h->h_state->updates_l - rec_ul0);
        }
    }
    if (e != hipSuccess) { cleanup(); return dev_fail(h, e, "adjoint sweep"); }
    float* dst = grad_c;
    if (!out_is_device) {
        st = scratch(h, N * sizeof(float), &dst);
        if (st) { cleanup(); return st; }
    }
    e = launch_grad_finish(a->t, S, h->d_shots, dst, h->stream);
    if (e == hipSuccess && !out_is_device)
        e = hipMemcpyAsync(grad_c, dst, N * sizeof(float), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) { cleanup(); return dev_fail(h, e, "adjoint gradient"); }
    st = sync_state(a);
    if (st) { cleanup(); return set_err(h, st, "adjoint tables failed"); }
    const int aerr = dev_error(*a->h_state), gerr = a->h_state->grad_error;
    if (timing) {
        h->af_cells += (long long)(a->h_state->updates - a_upd0);
        h->af_cells_u += (long long)(a->h_state->updates_u - a_updu0);
        h->af_cells_l += (long long)(a->h_state->updates_l - a_updl0);
        std::vector<unsigned long long> wg(GRAD_ACCUM_MAX_WG);
        if (hipMemcpy(wg.data(), gterms, sizeof(unsigned long long) * GRAD_ACCUM_MAX_WG, hipMemcpyDeviceToHost) !=
            hipSuccess) {
            cleanup();
            return dev_fail(h, hipGetLastError(), "gradient node counts");
        }
        for (unsigned long long v : wg) h->grad_cells += (long long)v;
    }
    st = ck_restore(h, now);
    if (st) { cleanup(); return st; }
    st = sync_state(h);
    cleanup();
    if (st) return st;
    if (aerr == ERR_NONFINITE) return set_err(h, TCM_E_NONFINITE, "the adjoint field became non-finite");
    if (aerr) return set_err(h, (tcm_status)aerr, "the adjoint field failed (pool)");
    if (gerr) return set_err(h, TCM_E_STATE, "adjoint stores overflowed (forward lists longer than the run's peak)");
    return TCM_OK;
}

tcm_status tcm_autotune(tcm_handle* h, int32_t probe_steps, tcm_tuning* out) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (h->engine != TCM_ENGINE_BLOCKS) return set_err(h, TCM_E_STATE, "autotune applies to the block engine");
    if (probe_steps < 1) return set_err(h, TCM_E_ARG, "probe_steps must be >= 1");
    st = sync_state(h);
    if (st) return st;
    if (dev_error(*h->h_state)) return set_err(h, TCM_E_STATE, "the run has failed (pool or non-finite field)");
    st = ensure_trace_capacity(h, h->h_state->step + (long long)probe_steps - h->t.trace_step0);
    if (st) return st;
    Ckpt snap;
    st = ck_save(h, snap);
    if (st) return st;
    const int keep_grid = h->grid_step, keep_gs = h->gsteps, keep_w = h->tile_w, keep_p = h->tile_p;
    const int keep_flags = h->cfg.flags;
    h->cfg.flags &= ~TCM_FLAG_TIMING;
    hipEvent_t e0, e1;
    HIP_OR_FAIL(h, timing_event(&e0));
    HIP_OR_FAIL(h, timing_event(&e1));
    tcm_tuning res{};
    res.ms_per_step = 1e300;
    int best_grid = keep_grid, best_gs = keep_gs, best_w = keep_w, best_p = keep_p;

    // time probe_steps steps of one shape (w waves of pb blocks) from the saved state
    auto probe = [&](int w, int pb, int wpc, int gs) -> tcm_status {
        h->tile_w = w;
        h->tile_p = pb;
        h->grid_step = std::max(8, (h->ncu * wpc) / 8 * 8);
        h->gsteps = round_graph_steps(h, gs);
        drop_graph(h);
        // one untimed graph launch so capture/instantiation is not timed
        const long long step0 = h->h_state->step;
        tcm_status s = ck_restore(h, snap);
        h->hstep = step0;
        if (!s) s = issue_steps(h, std::min(gs, probe_steps));
        if (!s) s = ck_restore(h, snap);
        h->hstep = step0;
        if (s) return s;
        HIP_OR_FAIL(h, hipEventRecord(e0, h->stream));
        s = issue_steps(h, probe_steps);
        if (s) return s;
        HIP_OR_FAIL(h, hipEventRecord(e1, h->stream));
        HIP_OR_FAIL(h, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_OR_FAIL(h, hipEventElapsedTime(&ms, e0, e1));
        const double per = ms / probe_steps;
        if (res.ncand < 32) {
            res.cand_blocks_per_wg[res.ncand] = w * pb;
            res.cand_blocks_per_wave[res.ncand] = pb;
            res.cand_wg_per_cu[res.ncand] = wpc;
            res.cand_graph_steps[res.ncand] = h->gsteps;
            res.cand_ms_per_step[res.ncand] = per;
            res.ncand++;
        }
        if (per < res.ms_per_step) {
            res.ms_per_step = per;
            res.blocks_per_wg = w * pb;
            res.blocks_per_wave = pb;
            res.wg_per_cu = wpc;
            res.graph_steps = h->gsteps;
            best_grid = h->grid_step;
            best_gs = h->gsteps;
            best_w = w;
            best_p = pb;
        }
        return TCM_OK;
    };
    // the workgroup tile (2, 4 or 8 x-adjacent blocks, one or two per wave)
    // x workgroups per CU, 4 to 24 waves per CU, at 16 steps per graph; then
    // the graph length
    const int shapes[5][2] = {{2, 1}, {4, 1}, {8, 1}, {2, 2}, {4, 2}};   // {waves, blocks per wave}
    for (const auto& sh : shapes) {
        const int w = sh[0], pb = sh[1];
        const int occ = std::max(1, block_step_occupancy(h->t.adaptive != 0, w, pb, step_mode(h->t)));
        for (int wpc : {1, 2, 3, 4, 6, 8, 12}) {
            if (st || wpc > occ || w * wpc < 4 || w * wpc > 24) continue;
            st = probe(w, pb, wpc, 16);
        }
    }
    const int bw = best_w, bp = best_p, bwpc = res.wg_per_cu;
    for (int gs : {8, 32}) {
        if (st || res.blocks_per_wg == 0) break;
        st = probe(bw, bp, bwpc, gs);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->cfg.flags = keep_flags;
    tcm_status rs = ck_restore(h, snap);
    if (!rs) rs = sync_state(h);
    ck_free(snap);
    drop_graph(h);
    if (st || rs) {
        h->grid_step = keep_grid;
        h->gsteps = keep_gs;
        h->tile_w = keep_w;
        h->tile_p = keep_p;
        return st ? st : rs;
    }
    h->grid_step = best_grid;
    h->gsteps = best_gs;
    h->tile_w = best_w;
    h->tile_p = best_p;
    st = sync_state(h);
    if (st) return st;
    if (out) *out = res;
    return TCM_OK;
}

// Whole-run launch-shape choice.  The shape that is fastest on one state
// need not be fastest over a run whose active set grows from a few blocks to
// the whole domain, so every candidate is probed at three states along the
// run (a quarter, half and three quarters of the way, reached with the
// current shape) and ranked by its summed probe time; the best candidate of
// each tile family (workgroup tile x blocks per wave) then runs the whole
// run from the current state twice, and the family with the fastest run
// wins.  The state is restored afterwards.
tcm_status tcm_autotune_run(tcm_handle* h, int32_t nsteps, int32_t probe_steps, tcm_tuning* out) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (h->engine != TCM_ENGINE_BLOCKS) return set_err(h, TCM_E_STATE, "autotune applies to the block engine");
    if (probe_steps < 1 || nsteps < 4) return set_err(h, TCM_E_ARG, "nsteps >= 4 and probe_steps >= 1 required");
    st = sync_state(h);
    if (st) return st;
    if (dev_error(*h->h_state)) return set_err(h, TCM_E_STATE, "the run has failed (pool or non-finite field)");
    const long long step0 = h->h_state->step;
    st = ensure_trace_capacity(h, step0 + (long long)nsteps + probe_steps - h->t.trace_step0);
    if (st) return st;
    const int keep_grid = h->grid_step, keep_gs = h->gsteps, keep_w = h->tile_w, keep_p = h->tile_p;
    const int keep_flags = h->cfg.flags;
    Ckpt s0;
    std::vector<Ckpt> states(3);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto finish = [&](tcm_status s) -> tcm_status {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        h->cfg.flags = keep_flags;
        tcm_status rs = TCM_OK;
        if (s0.buf) {
            rs = ck_restore(h, s0);
            h->hstep = step0;
            if (!rs) rs = sync_state(h);
        }
        ck_free(s0);
        for (auto& c : states) ck_free(c);
        drop_graph(h);
        if (s || rs) {
            h->grid_step = keep_grid;
            h->gsteps = keep_gs;
            h->tile_w = keep_w;
            h->tile_p = keep_p;
        }
        return s ? s : rs;
    };
    st = ck_save(h, s0);
    if (st) return finish(st);
    h->cfg.flags &= ~TCM_FLAG_TIMING;
    if (timing_event(&e0) != hipSuccess || timing_event(&e1) != hipSuccess)
        return finish(dev_fail(h, hipGetLastError(), "timing event creation"));
    // the probe states, reached with the current shape
    long long at = step0;
    for (int k = 0; k < 3; k++) {
        const long long target = step0 + (long long)nsteps * (k + 1) / 4;
        st = issue_steps(h, (int)(target - at));
        at = target;
        if (!st) st = sync_state(h);
        if (!st && dev_error(*h->h_state)) st = report_device_error(h);
        if (!st) st = ck_save(h, states[k]);
        if (st) return finish(st);
    }
    auto set_shape = [&](int w, int pb, int wpc, int gs) {
        h->tile_w = w;
        h->tile_p = pb;
        h->grid_step = std::max(8, (h->ncu * wpc) / 8 * 8);
        h->gsteps = round_graph_steps(h, gs);
        drop_graph(h);
    };
    // time n steps from a state (one untimed graph launch first, so capture
    // and instantiation are not timed)
    auto timed = [&](const Ckpt& c, int n, int gs, double* ms_out) -> tcm_status {
        const long long s = c.step;
        tcm_status r = ck_restore(h, c);
        h->hstep = s;
        if (!r) r = issue_steps(h, std::min(gs, n));
        if (!r) r = ck_restore(h, c);
        h->hstep = s;
        if (r) return r;
        HIP_OR_FAIL(h, hipEventRecord(e0, h->stream));
        r = issue_steps(h, n);
        if (r) return r;
        HIP_OR_FAIL(h, hipEventRecord(e1, h->stream));
        HIP_OR_FAIL(h, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_OR_FAIL(h, hipEventElapsedTime(&ms, e0, e1));
        *ms_out = ms;
        return TCM_OK;
    };
    // mean time per step over the three states
    auto probe = [&](int w, int pb, int wpc, int gs, double* per) -> tcm_status {
        set_shape(w, pb, wpc, gs);
        double sum = 0.0;
        for (const auto& c : states) {
            double ms = 0.0;
            tcm_status r = timed(c, probe_steps, gs, &ms);
            if (r) return r;
            sum += ms;
        }
        *per = sum / (3.0 * probe_steps);
        return TCM_OK;
    };
    tcm_tuning res{};
    res.ms_per_step = 1e300;
    struct Fam { int w, pb, wpc; double per; };
    std::vector<Fam> fams;
    const int shapes[5][2] = {{2, 1}, {4, 1}, {8, 1}, {2, 2}, {4, 2}};   // {waves, blocks per wave}
    for (const auto& sh : shapes) {
        const int w = sh[0], pb = sh[1];
        const int occ = std::max(1, block_step_occupancy(h->t.adaptive != 0, w, pb, step_mode(h->t)));
        Fam best{w, pb, 0, 1e300};
        for (int wpc : {1, 2, 3, 4, 6, 8, 12}) {
            if (wpc > occ || w * wpc < 4 || w * wpc > 24) continue;
            double per = 0.0;
            st = probe(w, pb, wpc, 16, &per);
            if (st) return finish(st);
            if (res.ncand < 32) {
                res.cand_blocks_per_wg[res.ncand] = w * pb;
                res.cand_blocks_per_wave[res.ncand] = pb;
                res.cand_wg_per_cu[res.ncand] = wpc;
                res.cand_graph_steps[res.ncand] = h->gsteps;
                res.cand_ms_per_step[res.ncand] = per;
                res.ncand++;
            }
            if (per < best.per) best = Fam{w, pb, wpc, per};
        }
        if (best.wpc > 0) fams.push_back(best);
    }
    if (fams.empty()) return finish(set_err(h, TCM_E_STATE, "no launch shape fits"));
    // steps per graph, on the family that probed fastest
    int gsteps = 16;
    {
        const Fam* f0 = &fams[0];
        for (const auto& f : fams)
            if (f.per < f0->per) f0 = &f;
        double best = f0->per;
        for (int gs : {8, 32}) {
            double per = 0.0;
            st = probe(f0->w, f0->pb, f0->wpc, gs, &per);
            if (st) return finish(st);
            if (per < best) {
                best = per;
                gsteps = gs;
            }
        }
    }
    // whole runs: each family's best probe shape, twice
    int win = -1;
    double win_ms = 1e300;
    for (size_t i = 0; i < fams.size(); i++) {
        const Fam& f = fams[i];
        set_shape(f.w, f.pb, f.wpc, gsteps);
        double run = 1e300;
        for (int r = 0; r < 2; r++) {
            double ms = 0.0;
            st = timed(s0, nsteps, h->gsteps, &ms);
            if (st) return finish(st);
            run = std::min(run, ms);
        }
        if (i < 8) {
            res.fam_blocks_per_wg[i] = f.w * f.pb;
            res.fam_blocks_per_wave[i] = f.pb;
            res.fam_wg_per_cu[i] = f.wpc;
            res.fam_run_ms[i] = run;
            res.nfam = (int)i + 1;
        }
        if (run < win_ms) {
            win_ms = run;
            win = (int)i;
        }
    }
    const Fam& f = fams[win];
    st = finish(TCM_OK);
    if (st) return st;
    set_shape(f.w, f.pb, f.wpc, gsteps);
    res.blocks_per_wg = f.w * f.pb;
    res.blocks_per_wave = f.pb;
    res.wg_per_cu = f.wpc;
    res.graph_steps = h->gsteps;
    res.ms_per_step = win_ms / nsteps;
    st = sync_state(h);
    if (st) return st;
    if (out) *out = res;
    return TCM_OK;
}

tcm_status tcm_set_launch(tcm_handle* h, int32_t wg_per_cu, int32_t graph_steps, int32_t blocks_per_wg,
                          int32_t blocks_per_wave) {
    tcm_status st = check_live(h);
    if (st) return st;
    if (h->engine != TCM_ENGINE_BLOCKS) return set_err(h, TCM_E_STATE, "launch shape applies to the block engine");
    const int b = blocks_per_wg > 0 ? blocks_per_wg : h->tile_w * h->tile_p;
    const int pb = blocks_per_wave > 0 ? blocks_per_wave : h->tile_p;
    if ((b != 2 && b != 4 && b != 8) || pb < 1 || pb > 2 || b % pb || !block_step_shape_ok(b / pb, pb))
        return set_err(h, TCM_E_ARG, "blocks_per_wg must be 0, 2, 4 or 8 and blocks_per_wave 0, 1 or 2 "
                                     "(2 with a tile of 4 or 8 blocks)");
    const int w = b / pb;
    const int occ = std::max(1, block_step_occupancy(h->t.adaptive != 0, w, pb, step_mode(h->t)));
    if (wg_per_cu < 1 || wg_per_cu > occ || graph_steps < 1)
        return set_err(h, TCM_E_ARG, fmt("launch shape needs 1 <= wg_per_cu <= %d and graph_steps >= 1", occ));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    h->tile_w = w;
    h->tile_p = pb;
    h->grid_step = std::max(8, (h->ncu * wg_per_cu) / 8 * 8);
    h->gsteps = round_graph_steps(h, graph_steps);
    drop_graph(h);
    return TCM_OK;
}

}  // extern "C"
