// C-ABI entry points (declared in include/sphcell.h).  Argument checking,
// error codes and the context; the work itself is in sph_build.hip and
// sph_interact.hip.
#include <cstring>
#include <mutex>

#include "sph_impl.h"

using sph::Err;

static sph_status fail(sph_ctx* ctx, const Err& e) {
    if (ctx && e.st != SPH_OK) ctx->last_error = e.msg;
    return e.st;
}

// why the last sph_ctx_create on this thread failed (read through
// sph_last_error(NULL))
static thread_local std::string g_create_error;

// ---------------------------------------------------------------------------
// The library's static scratch: the workspace of trees built through
// sph_build_cells_static, for callers that cannot allocate device memory.
// Each GPU the library runs on holds its own copy (STATIC_SCRATCH_BYTES)
// until the process ends.  In host code `scratch` is only a stand-in for the
// device array: its device address is taken once per device, when the first
// context on that device is created (g_scratch_ptr), and only that address is
// ever handed to kernels or copies.  One tree per device can use it at a
// time: attaching it to a tree (a new generation) retires the tree that held
// it before, whose later calls fail with SPH_E_STATE.
// ---------------------------------------------------------------------------
static constexpr size_t STATIC_SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
static constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES] = {};
static int g_scratch_gen[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// Calls on a tree that held the static scratch fail once another tree took it.
static sph_status check_tree(sph_ctx* ctx, sph_tree* t) {
    if (t->static_gen) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (ctx->device < 0 || ctx->device >= MAX_DEVICES || g_scratch_gen[ctx->device] != t->static_gen) {
            ctx->last_error = "this tree's static scratch was taken by a later sph_build_cells_static: build again";
            return SPH_E_STATE;
        }
    }
    t->stream = ctx->stream;
    return SPH_OK;
}

extern "C" {

const char* sph_version(void) { return "sphcell 0.1 (gfx950)"; }

const char* sph_status_str(sph_status st) {
    switch (st) {
        case SPH_OK: return "ok";
        case SPH_E_ARG: return "invalid argument";
        case SPH_E_HIP: return "HIP runtime error";
        case SPH_E_WORKSPACE: return "device allocation failed";
        case SPH_E_REBUILD: return "h outgrew the cell support: rebuild";
        case SPH_E_NOCONV: return "h solve did not converge";
        case SPH_E_CAPACITY: return "capacity exceeded";
        case SPH_E_STATE: return "call out of order";
        default: return "unknown status";
    }
}

void sph_params_default(sph_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->n_split = 400;
    p->split_frac = 0.875f;
    p->h_slack = 0.2f;
    p->max_depth = 12;
    p->top_grid = 0;
    p->n_target = 48.f;
    p->h_tol = 0.5f;
    p->max_iter = 30;
    p->gamma = 5.f / 3.f;
    p->alpha = 2.f;
    p->flags = 0;
}

sph_status sph_ctx_create(sph_ctx** out, int device, void* stream) {
    if (!out) return SPH_E_ARG;
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        g_create_error = std::string("hipGetDeviceCount: ") + (e != hipSuccess ? hipGetErrorString(e) : "no device");
        return SPH_E_HIP;
    }
    if (device < 0 || device >= ndev) {
        g_create_error = "device index out of range";
        return SPH_E_ARG;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return SPH_E_HIP;
    }
    if (device < MAX_DEVICES) {
        // the device address of this device's static scratch, once per device
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                g_create_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
                return SPH_E_HIP;
            }
            g_scratch_ptr[device] = p;
        }
    }
    sph_ctx* c = new sph_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->n_cu = prop.multiProcessorCount;
    sph::query_occupancy(c);
    if (hipMalloc(&c->d_counter, sph_ctx::CTR_WORDS * sizeof(int32_t)) != hipSuccess) {
        delete c;
        return SPH_E_WORKSPACE;
    }
    if (hipHostMalloc(&c->h_pin, sph_ctx::PIN_BYTES, hipHostMallocDefault) != hipSuccess) {
        c->h_pin = nullptr;
        (void)hipFree(c->d_counter);
        delete c;
        return SPH_E_WORKSPACE;
    }
    *out = c;
    return SPH_OK;
}

void sph_ctx_destroy(sph_ctx* ctx) {
    if (!ctx) return;
    for (auto& e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto& e : ctx->solve_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->d_counter) (void)hipFree(ctx->d_counter);
    if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
    delete ctx;
}

const char* sph_last_error(const sph_ctx* ctx) { return ctx ? ctx->last_error.c_str() : g_create_error.c_str(); }

sph_status sph_ctx_sync(sph_ctx* ctx) {
    if (!ctx) return SPH_E_ARG;
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        ctx->last_error = std::string("stream: ") + hipGetErrorString(e);
        return SPH_E_HIP;
    }
    return SPH_OK;
}

sph_status sph_workspace_size(int64_t n, int32_t nsets, const sph_params* p, size_t* bytes) {
    if (!bytes || n < 0 || nsets < 1) return SPH_E_ARG;
    (void)p;
    // Per particle: 124 B of cell-ordered state (keys and values twice,
    // permutations, position and remainder, velocity, h, u, bounds, pair-hash
    // terms), 48 B of the caller's data packed for the gather, 28 B density,
    // 13 B solve, 52 B force, 41 B saved Newton state, 16 B of radix and
    // scan scratch: ~323 B.  Sorted lists: 20 B per entry,
    // 13 entries per particle and tree level that holds pair tasks (29 per
    // particle on a clustered set with h over three decades: 580 B), plus
    // 24 B of radix keys and values per entry of the lists longer than
    // 16384 (about 10 per particle there: 240 B).  Cells, tasks and
    // interaction lists: ~120 B.  Heavy chunks: 4 KiB of partial sums per
    // piece, ~37 B per particle on the clustered mixture (a piece per ~110
    // particles), at most 64 B (one piece per 64 particles; 16 MiB on small
    // sets, inside the fixed reserve): 64 B.  Plus the set tables and a fixed reserve.  Measured
    // peaks: 548 B per particle on a 10^6 lattice, 1169 B on the 8*10^6
    // clustered mixture, before the packed records.
    const double per = 323.0 + 580.0 + 240.0 + 120.0 + 64.0;
    *bytes = (size_t)(per * (double)n) + (size_t)nsets * 4096 + ((size_t)24 << 20);
    return SPH_OK;
}

sph_status sph_footprint(int64_t n, const sph_params* p, size_t* bytes) { return sph_workspace_size(n, 1, p, bytes); }

sph_status sph_tree_create(sph_ctx* ctx, sph_tree** out) {
    if (!ctx || !out) return SPH_E_ARG;
    *out = new sph_tree();
    return SPH_OK;
}

void sph_tree_destroy(sph_ctx* ctx, sph_tree* t) {
    if (t && ctx) t->stream = ctx->stream;
    delete t;
}

sph_status sph_tree_bytes(const sph_tree* t, size_t* bytes) {
    if (!t || !bytes) return SPH_E_ARG;
    *bytes = t->bytes();
    return SPH_OK;
}

sph_status sph_tree_set_workspace(sph_ctx* ctx, sph_tree* t, void* ws, size_t ws_bytes) {
    if (!ctx || !t) return SPH_E_ARG;
    if (ws && ws_bytes < ((size_t)1 << 20)) return fail(ctx, Err{SPH_E_ARG, "a workspace needs at least 1 MiB"});
    t->stream = ctx->stream;   // (a tree leaving the static scratch needs no check)
    return fail(ctx, t->set_workspace(ws, ws_bytes, 0));
}

sph_status sph_tree_workspace_needed(const sph_tree* t, size_t* bytes) {
    if (!t || !bytes) return SPH_E_ARG;
    *bytes = std::max(t->ws_needed, t->ar.high);
    return SPH_OK;
}

sph_status sph_build_cells(sph_ctx* ctx, sph_tree* t, const sph_input* in, const sph_params* p) {
    if (!ctx || !t) return SPH_E_ARG;
    if (sph_status s = check_tree(ctx, t)) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPH_E_HIP;
    return fail(ctx, sph::build_tree(ctx, t, in, p));
}

sph_status sph_build_cells_static(sph_ctx* ctx, sph_tree* t, const sph_input* in, const sph_params* p) {
    if (!ctx || !t || !in || !p || !in->offsets || in->nsets < 1) return SPH_E_ARG;
    if (ctx->device < 0 || ctx->device >= MAX_DEVICES || !g_scratch_ptr[ctx->device])
        return fail(ctx, Err{SPH_E_STATE, "no static scratch on this device"});
    const int64_t n = in->offsets[in->nsets];
    size_t need = 0;
    if (sph_workspace_size(n, in->nsets, p, &need) != SPH_OK) return SPH_E_ARG;
    if (need > STATIC_SCRATCH_BYTES)
        return fail(ctx, Err{SPH_E_CAPACITY, std::to_string(n) + " particles need about " + std::to_string(need >> 20) +
                                                 " MiB; the static scratch holds " +
                                                 std::to_string(STATIC_SCRATCH_BYTES >> 20) + " MiB"});
    if (hipSetDevice(ctx->device) != hipSuccess) return SPH_E_HIP;
    t->stream = ctx->stream;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        const int dev = ctx->device;
        // a tree that holds the current generation keeps its blocks;
        // otherwise the scratch is taken over (a new generation)
        if (!(t->static_gen && t->static_gen == g_scratch_gen[dev])) {
            const int gen = ++g_scratch_gen[dev];
            Err e = t->set_workspace(g_scratch_ptr[dev], STATIC_SCRATCH_BYTES, gen);
            if (e.st) return fail(ctx, e);
        }
    }
    return fail(ctx, sph::build_tree(ctx, t, in, p));
}

sph_status sph_refresh_cells(sph_ctx* ctx, sph_tree* t, const sph_input* in) {
    if (!ctx || !t) return SPH_E_ARG;
    if (sph_status s = check_tree(ctx, t)) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return SPH_E_HIP;
    return fail(ctx, sph::refresh_tree(ctx, t, in));
}

sph_status sph_sort_pairs(sph_ctx* ctx, sph_tree* t) {
    if (!ctx || !t) return SPH_E_ARG;
    if (sph_status s = check_tree(ctx, t)) return s;
    return fail(ctx, sph::sort_pairs(ctx, t));
}

sph_status sph_density(sph_ctx* ctx, sph_tree* t, const sph_density_out* out) {
    if (!ctx || !t) return SPH_E_ARG;
    if (sph_status s = check_tree(ctx, t)) return s;
    return fail(ctx, sph::run_density(ctx, t, out));
}

sph_status sph_solve_h(sph_ctx* ctx, sph_tree* t, const sph_density_out* out, int32_t* n_unconverged,
                       int32_t* iterations) {
    if (!ctx || !t) return SPH_E_ARG;
    if (sph_status s = check_tree(ctx, t)) return s;
    return fail(ctx, sph::run_solve(ctx, t, out, n_unconverged, iterations));
}

sph_status sph_force(sph_ctx* ctx, sph_tree* t, const sph_force_out* out) {
    if (!ctx || !t) return SPH_E_ARG;
    if (sph_status s = check_tree(ctx, t)) return s;
    return fail(ctx, sph::run_force(ctx, t, out));
}

sph_status sph_set_halo(sph_ctx* ctx, sph_tree* t, const uint8_t* owned, const float* rho, const float* drho_dh) {
    if (!ctx || !t) return SPH_E_ARG;
    if (sph_status s = check_tree(ctx, t)) return s;
    return fail(ctx, sph::set_halo(ctx, t, owned, rho, drho_dh));
}

sph_status sph_run_graph(sph_ctx* ctx, sph_tree* t, int32_t k_iter, const sph_density_out* dout,
                         const sph_force_out* fout, int32_t* n_unconverged_dev) {
    if (!ctx || !t || k_iter < 1) return SPH_E_ARG;
    if (sph_status s = check_tree(ctx, t)) return s;
    return fail(ctx, sph::run_graph(ctx, t, k_iter, dout, fout, n_unconverged_dev));
}

int32_t sph_last_timings(sph_ctx* ctx, const char** names, double* ms, int32_t cap) {
    if (!ctx) return 0;
    if (ctx->nev > 0) {
        // intervals between consecutive stage events of one call
        (void)hipEventSynchronize(ctx->ev_pool[ctx->nev - 1]);
        ctx->last_ms.clear();
        for (size_t i = 1; i < ctx->nev; ++i) {
            if (std::strcmp(ctx->ev_name[i], "start") == 0) continue;
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ctx->ev_pool[i - 1], ctx->ev_pool[i]);
            ctx->last_ms.emplace_back(ctx->ev_name[i], (double)t);
        }
        ctx->nev = 0;
    }
    int32_t k = 0;
    for (const auto& e : ctx->last_ms) {
        if (k >= cap) break;
        if (names) names[k] = e.first;
        if (ms) ms[k] = e.second;
        ++k;
    }
    return k;
}

sph_status sph_last_work(sph_ctx* ctx, uint64_t* density_pairs, uint64_t* force_pairs) {
    if (!ctx) return SPH_E_ARG;
    // 2 x 8 counters of 64 bits, 128 bytes apart
    const void* d = ctx->d_counter + sph_ctx::CTR_WORK;
    if (hipMemcpyAsync(ctx->h_pin, d, 512 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return SPH_E_HIP;
    const uint64_t* v = (const uint64_t*)ctx->h_pin;
    uint64_t s[2] = {0, 0};
    for (int k = 0; k < 2; ++k)
        for (int g = 0; g < 8; ++g) s[k] += v[k * 128 + g * 16];
    if (density_pairs) *density_pairs = s[0];
    if (force_pairs) *force_pairs = s[1];
    return SPH_OK;
}

sph_status sph_last_reads(sph_ctx* ctx, uint64_t* density_records, uint64_t* force_records) {
    if (!ctx) return SPH_E_ARG;
    // the word after each pair-evaluation counter
    const void* d = ctx->d_counter + sph_ctx::CTR_WORK;
    if (hipMemcpyAsync(ctx->h_pin, d, 512 * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return SPH_E_HIP;
    const uint64_t* v = (const uint64_t*)ctx->h_pin;
    uint64_t s[2] = {0, 0};
    for (int k = 0; k < 2; ++k)
        for (int g = 0; g < 8; ++g) s[k] += v[k * 128 + g * 16 + 1];
    if (density_records) *density_records = s[0];
    if (force_records) *force_records = s[1];
    return SPH_OK;
}

void sph_enable_timing(sph_ctx* ctx, int32_t on) {
    if (ctx) ctx->timing = on != 0;
}

sph_status sph_tree_stats(const sph_tree* t, int64_t* stats, int32_t cap) {
    if (!t || !stats) return SPH_E_ARG;
    if (t->nsegent < 0 && t->d_counts) {
        // the sort kept its entry count on the device: read it on the
        // tree's stream (no device-wide synchronisation)
        uint32_t v = 0;
        if (hipMemcpyAsync(&v, t->d_counts, sizeof(v), hipMemcpyDeviceToHost, t->stream) != hipSuccess ||
            hipStreamSynchronize(t->stream) != hipSuccess)
            return SPH_E_HIP;
        const_cast<sph_tree*>(t)->nsegent = v;
    }
    int64_t v[13] = {t->n,
                     t->ncells,
                     t->nleaves,
                     t->ntasks,
                     t->npairs,
                     t->nsegent,
                     t->nchunks,
                     t->nlevels,
                     t->sets.empty() ? 0 : (int64_t)1 << t->sets[0].lgG,
                     t->max_leaf,
                     t->graph_captures,
                     t->nheavy,
                     t->npieces};
    for (int i = 0; i < cap && i < 13; ++i) stats[i] = v[i];
    return SPH_OK;
}

}  // extern "C"
