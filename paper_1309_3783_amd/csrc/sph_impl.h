// Host-side objects of the library: context, tree, allocation helpers and
// the orchestration entry points shared by the source files.
#pragma once

#include <algorithm>
#include <string>
#include <utility>
#include <vector>

#include "sph_internal.h"
#include "sph_prims.h"

struct sph_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 256;
    std::string last_error;
    bool timing = false;
    // stage events of the calls since the timings were last read: a pool
    // of events reused across calls (no create/destroy per stage, no
    // synchronisation until the timings are read)
    std::vector<hipEvent_t> ev_pool;
    std::vector<const char*> ev_name;
    size_t nev = 0;
    std::vector<std::pair<const char*, double>> last_ms;
    // device words (1024): [0, 256) density work counters, [256, 512) force
    // work counters, [512, 768) chunk-list counts, [CTR_CFL] Courant minimum
    int32_t* d_counter = nullptr;
    static constexpr int CTR_CFL = 768;
    // pinned host memory that device counts are read back into: one
    // asynchronous copy per read, then one stream synchronisation
    static constexpr size_t PIN_BYTES = 65536;
    void* h_pin = nullptr;
    hipStream_t cap_stream = nullptr; // private stream used only to capture graphs
};

struct sph_tree {
    // ---- configuration -------------------------------------------------
    sph_params prm{};
    int nsets = 0;
    int64_t n = 0;
    std::vector<int64_t> off;
    std::vector<sph::SetInfo> sets;
    int depth = 0, nlevels = 0, key_bits = 0;
    bool built = false, sorted = false, have_density = false, have_ghost = false, hash = false;

    // ---- device buffers ------------------------------------------------
    sph::DevBuf b_sets, b_small, b_key, b_key2, b_val, b_val2, b_perm, b_pos, b_plo, b_pv, b_ph, b_hdec, b_pu,
        b_bound, b_mix, b_rs, b_cell, b_taskA, b_taskB, b_final, b_chunk, b_csr, b_csr2, b_csroff,
        b_segoff, b_seglist, b_segproj, b_segidx, b_bigk, b_bigv, b_sc, b_dens, b_force, b_solve,
        b_red, b_misc, b_saved, b_split, b_counts, b_iperm;

    // ---- sizes (host) --------------------------------------------------
    int64_t ncells = 0, ntasks = 0, npairs = 0, nsegent = 0, nchunks = 0, max_leaf = 0;
    int64_t nleaves = 0;
    int64_t ncsr = 0;                   // interaction-list entries (a bound when ncsr_dev is set)
    const uint32_t* ncsr_dev = nullptr; // their exact count on the device
    std::vector<int64_t> lvl_start;
    int64_t sc_cap = 0;
    std::vector<int4> red_chunks;   // (set, first, count, 0) reduction chunks
    std::vector<int64_t> red_off;   // the set offsets red_chunks was made for
    int64_t nred = 0;

    // ---- device views --------------------------------------------------
    sph::SetInfo* d_sets = nullptr;
    uint64_t *key = nullptr, *key2 = nullptr, *mix = nullptr, *csr = nullptr, *csr2 = nullptr;
    uint32_t *val = nullptr, *val2 = nullptr, *perm = nullptr, *rs_tmp = nullptr;
    uint32_t* iperm = nullptr;   // caller order -> cell order
    float4 *pos = nullptr, *pv = nullptr;
    float4* plo = nullptr;   // FP32 remainders of the positions: pos.xyz + plo.xyz = offset to ~2^-48
    float *ph = nullptr, *hdec = nullptr, *pu = nullptr, *bound = nullptr;
    sph::Cell* cells = nullptr;
    int4 *taskA = nullptr, *taskB = nullptr, *finals = nullptr, *chunks = nullptr;
    uint32_t *csr_off = nullptr, *segoff = nullptr, *seglist = nullptr, *segidx = nullptr;
    float4* segpos = nullptr;   // sorted lists: the particle records (x, y, z, m) in list order
    uint32_t *sc_a = nullptr, *sc_b = nullptr, *sc_c = nullptr, *sc_d = nullptr, *sc_tmp = nullptr;
    uint32_t* split_idx = nullptr;   // split flags of one level, scanned in place
    uint32_t* d_counts = nullptr;    // [0] sorted-list entries when not read back (nsegent < 0)
    uint32_t* d_total = nullptr;
    int* d_maxleaf = nullptr;
    int* d_npairs = nullptr;
    // density state (cell order)
    float *rho = nullptr, *drho = nullptr, *nw = nullptr, *dnw = nullptr;
    int32_t* nngb = nullptr;
    uint64_t* hashd = nullptr;
    // solve state
    uint8_t* active = nullptr;
    uint32_t* alist = nullptr;   // chunks with active particles, per work range
    float *lo = nullptr, *hi = nullptr, *dstep = nullptr;
    int32_t* status = nullptr;   // [0] rebuild flag, [1] unconverged count
    // ghost + force state (cell order)
    float4* frec = nullptr;   // per particle after the ghost step: h, A, sound speed, 8/(pi h^5)
    float *fax = nullptr, *fay = nullptr, *faz = nullptr, *fdu = nullptr, *fvs = nullptr, *fS = nullptr;
    int32_t* fn = nullptr;
    uint64_t* hashf = nullptr;
    double* partial = nullptr;
    int32_t* part_cnt = nullptr;
    // Newton state saved when a solve stops for a rebuild (caller order)
    bool saved = false;
    int64_t saved_n = 0;
    sph::SolveState sv{};
    double* sums_int = nullptr;   // per-set sums of the last force pass
    int4* d_red = nullptr;

    // graph
    hipGraphExec_t gexec = nullptr;
    std::vector<const void*> gkey;

    ~sph_tree() { release(); }

    void invalidate_graph() {
        if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
        gkey.clear();
    }

    size_t bytes() const {
        size_t b = 0;
        for (const sph::DevBuf* d : bufs()) b += d->cap;
        return b;
    }

    std::vector<const sph::DevBuf*> bufs() const {
        return {&b_sets, &b_small, &b_key, &b_key2, &b_val, &b_val2, &b_perm, &b_pos, &b_plo, &b_pv, &b_ph, &b_hdec,
                &b_pu, &b_bound, &b_mix, &b_rs, &b_cell, &b_taskA, &b_taskB, &b_final, &b_chunk, &b_csr,
                &b_csr2, &b_csroff, &b_segoff, &b_seglist, &b_segproj, &b_segidx, &b_bigk, &b_bigv, &b_sc,
                &b_dens, &b_force, &b_solve, &b_red, &b_misc, &b_saved, &b_split, &b_counts, &b_iperm};
    }

    void release() {
        invalidate_graph();
        red_off.clear();
        for (const sph::DevBuf* d : bufs()) {
            sph::DevBuf* m = const_cast<sph::DevBuf*>(d);
            if (m->p) (void)hipFree(m->p);
            m->p = nullptr;
            m->cap = 0;
        }
    }

    // grow-only allocation (contents not kept)
    sph::Err alloc(sph::DevBuf& b, size_t bytes, void** out) {
        bytes = std::max<size_t>(bytes, 256);
        if (b.cap < bytes) {
            if (b.p) {
                (void)hipDeviceSynchronize();
                (void)hipFree(b.p);
                b.p = nullptr;
                b.cap = 0;
            }
            size_t want = bytes + bytes / 8;
            hipError_t e = hipMalloc(&b.p, want);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return sph::Err{SPH_E_WORKSPACE, "hipMalloc of " + std::to_string(want) + " bytes failed"};
            }
            b.cap = want;
        }
        *out = b.p;
        return sph::Err{};
    }

    // grow keeping the first `keep` bytes
    sph::Err grow(sph::DevBuf& b, size_t keep, size_t bytes, void** out) {
        if (b.cap >= bytes) { *out = b.p; return sph::Err{}; }
        void* np = nullptr;
        size_t want = bytes + bytes / 4;
        hipError_t e = hipMalloc(&np, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return sph::Err{SPH_E_WORKSPACE, "hipMalloc of " + std::to_string(want) + " bytes failed"};
        }
        (void)hipDeviceSynchronize();
        if (keep && b.p) {
            e = hipMemcpy(np, b.p, keep, hipMemcpyDeviceToDevice);
            if (e != hipSuccess) { (void)hipFree(np); return sph::Err{SPH_E_HIP, "grow copy failed"}; }
        }
        if (b.p) (void)hipFree(b.p);
        b.p = np;
        b.cap = want;
        *out = np;
        return sph::Err{};
    }

    sph::SolveState saved_state() const { return sv; }

    sph::Err ensure_saved() {
        const int64_t m = std::max<int64_t>(n, 1);
        void* p;
        sph::Err e = alloc(b_saved, (size_t)m * (1 + 7 * sizeof(float) + sizeof(int32_t) + sizeof(uint64_t)) + 256, &p);
        if (e.st) return e;
        sv.hash = (uint64_t*)p;
        sv.lo = (float*)(sv.hash + m);
        sv.hi = sv.lo + m;
        sv.dstep = sv.hi + m;
        sv.rho = sv.dstep + m;
        sv.drho = sv.rho + m;
        sv.nw = sv.drho + m;
        sv.dnw = sv.nw + m;
        sv.nngb = (int32_t*)(sv.dnw + m);
        sv.active = (uint8_t*)(sv.nngb + m);
        return sph::Err{};
    }

    // four uint32 scratch arrays of n entries plus scan scratch and counters
    sph::Err scratch(int64_t n) {
        n = std::max<int64_t>(n, 1);
        if (n <= sc_cap && sc_a) return sph::Err{};
        int64_t cap = std::max<int64_t>(n, sc_cap * 3 / 2);
        size_t words = 4 * (size_t)cap + sph::scan_tmp_words(cap) + 64;
        void* p;
        sph::Err e = alloc(b_sc, words * sizeof(uint32_t), &p);
        if (e.st) return e;
        uint32_t* w = (uint32_t*)p;
        sc_a = w;
        sc_b = w + cap;
        sc_c = w + 2 * cap;
        sc_d = w + 3 * cap;
        d_total = w + 4 * cap;
        d_maxleaf = (int*)(w + 4 * cap + 16);
        d_npairs = (int*)(w + 4 * cap + 32);
        sc_tmp = w + 4 * cap + 64;
        sc_cap = cap;
        return sph::Err{};
    }
};

namespace sph {
// Stage events: ev_mark records the end of a stage (a call's first mark,
// "start", opens it); nothing is synchronised here, the intervals are
// computed when the timings are read.
inline void ev_mark(sph_ctx* ctx, const char* name) {
    if (!ctx->timing) return;
    if (ctx->nev == ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        ctx->ev_pool.push_back(e);
        ctx->ev_name.push_back(name);
    }
    ctx->ev_name[ctx->nev] = name;
    (void)hipEventRecord(ctx->ev_pool[ctx->nev], ctx->stream);
    ++ctx->nev;
}

Err build_tree(sph_ctx* ctx, sph_tree* t, const sph_input* in, const sph_params* prm);
Err sort_pairs(sph_ctx* ctx, sph_tree* t);
Err run_density(sph_ctx* ctx, sph_tree* t, const sph_density_out* out);
Err run_solve(sph_ctx* ctx, sph_tree* t, const sph_density_out* out, int32_t* n_unconv, int32_t* iters);
Err run_force(sph_ctx* ctx, sph_tree* t, const sph_force_out* out);
Err run_graph(sph_ctx* ctx, sph_tree* t, int k_iter, const sph_density_out* dout, const sph_force_out* fout,
              int32_t* n_unconv_dev);
}  // namespace sph
