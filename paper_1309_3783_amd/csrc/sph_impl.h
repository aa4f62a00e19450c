// Host-side objects of the library: context, tree, allocation helpers and
// the orchestration entry points shared by the source files.
#pragma once

#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "sph_internal.h"
#include "sph_prims.h"

struct sph_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 256;
    // blocks of each persistent kernel that fit on a CU at once (occupancy,
    // asked once per kernel)
    std::map<const void*, int> resident;
    std::string last_error;
    bool timing = false;
    // stage events of the calls since the timings were last read: a pool
    // of events reused across calls (no create/destroy per stage, no
    // synchronisation until the timings are read)
    std::vector<hipEvent_t> ev_pool;
    std::vector<const char*> ev_name;
    size_t nev = 0;
    std::vector<std::pair<const char*, double>> last_ms;
    // device words (CTR_WORDS): [0, 256) density work counters, [256, 512)
    // force work counters, [512, 768) chunk-list counts, [CTR_CFL] Courant
    // minimum, [CTR_WORK, +512): 64-bit counts of pair evaluations, density
    // then force, each spread over 8 counters 128 bytes apart
    int32_t* d_counter = nullptr;
    static constexpr int CTR_CFL = 768;
    static constexpr int CTR_WORK = 1024;
    static constexpr int CTR_WORDS = 2048;
    // pinned host memory that device counts are read back into: one
    // asynchronous copy per read, then one stream synchronisation
    static constexpr size_t PIN_BYTES = 65536;
    void* h_pin = nullptr;
    // the Newton loop's status words, two slots at this offset of h_pin,
    // and the events that mark their copies done
    static constexpr size_t PIN_SOLVE = 32768;
    hipEvent_t solve_ev[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr; // private stream used only to capture graphs
};

namespace sph {
// Sub-allocator over one device region that the caller provides (a tree's
// workspace): first fit over a free list of 256-byte granules, neighbouring
// free blocks merged.  Blocks are given back and handed out again in stream
// order: every call on a tree enqueues its work on the one stream of its
// context, so a block freed by a call and reused by a later allocation is
// written only after every earlier use of it has run -- no synchronisation,
// no hipMalloc, no hipFree.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    size_t in_use = 0, high = 0;

    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }

    void reset(void* p, size_t bytes) {
        const size_t a = ((uintptr_t)p + 255) & ~(uintptr_t)255;   // aligned start
        const size_t skip = a - (uintptr_t)p;
        base = (char*)a;
        cap = bytes > skip ? (bytes - skip) & ~(size_t)255 : 0;
        free_.clear();
        if (cap) free_[0] = cap;
        in_use = high = 0;
    }

    bool take(size_t bytes, size_t* off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            in_use += bytes;
            high = std::max(high, in_use);
            return true;
        }
        return false;
    }

    void give(size_t off, size_t bytes) {
        bytes = round(bytes);
        in_use -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    size_t largest_free() const {
        size_t m = 0;
        for (const auto& f : free_) m = std::max(m, f.second);
        return m;
    }
};
}  // namespace sph

struct sph_tree {
    // ---- device memory ---------------------------------------------------
    // Either a workspace the caller attached (sph_tree_set_workspace: every
    // buffer is a block of it) or, with none attached, one hipMalloc per
    // buffer.  stream: the stream of the context of the current call.
    sph::Arena ar;
    bool ws = false;
    int static_gen = 0;          // > 0: the workspace is the library's static scratch (this generation)
    size_t ws_needed = 0;        // after SPH_E_WORKSPACE: bytes a larger workspace must offer at least
    hipStream_t stream = nullptr;
    int32_t* work_ctr = nullptr; // the context's pair-evaluation counters (set per call)

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
        b_red, b_misc, b_saved, b_split, b_counts, b_iperm, b_owned, b_blk, b_piece, b_plist, b_part, b_inrec;

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
    // one GPU's share of a decomposed set (sph_set_halo): 1 = owned, 0 = a
    // read-only halo particle; null when every particle is owned
    uint8_t* owned = nullptr;
    float4 *pos = nullptr, *pv = nullptr;
    float4* plo = nullptr;   // FP32 remainders of the positions: pos.xyz + plo.xyz = offset to ~2^-48
    float *ph = nullptr, *hdec = nullptr, *pu = nullptr, *bound = nullptr;
    sph::Cell* cells = nullptr;
    int4 *taskA = nullptr, *taskB = nullptr, *finals = nullptr;
    int4* chunks = nullptr;           // work chunks: (leaf, first particle, count, top cell of the leaf)
    uint32_t *csr_off = nullptr, *segoff = nullptr, *seglist = nullptr, *segidx = nullptr;
    float4* segpos = nullptr;   // sorted lists: the particle records (x, y, z, m) in list order
    // the particle array in blocks of 64 (aligned to particle indices): per
    // block a bit per particle that starts a top cell, and the bounding box
    // of the positions (2 float4: min, max; the whole space when the block
    // holds particles of two top cells); null for an empty tree
    uint64_t* blkbits = nullptr;
    float4* blkbox = nullptr;
    int64_t nblk = 0;
    // heavy chunks: per chunk the number of pieces it is handed out in (0:
    // with the others; 1: first, whole; 2..: first, split), the first slot of
    // its pieces; the list of pieces (chunk << 5 | piece) and per piece the
    // partial sums of its 64 particles (PART_WORDS doubles each)
    uint32_t* pcount = nullptr;
    uint32_t* poff = nullptr;
    uint32_t* plist = nullptr;
    double* part = nullptr;
    int64_t npieces = 0, nheavy = 0;
    int32_t max_sorted = INT32_MAX;   // partners with more particles have no sorted lists (read in cell order)
    // whether the interaction kernels need the code for heavy chunks and
    // cell-order reads: the tree has heavy chunks, or some partner cell may
    // hold SCAN_MIN particles (a one-level tree's partners are its leaves)
    bool ext() const { return npieces > 0 || !(nlevels == 1 && max_leaf < sph::SCAN_MIN); }
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
    int64_t graph_captures = 0;   // captures and instantiations so far (replays are not counted)

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
                &b_dens, &b_force, &b_solve, &b_red, &b_misc, &b_saved, &b_split, &b_counts, &b_iperm, &b_owned,
                &b_blk, &b_piece, &b_plist, &b_part, &b_inrec};
    }

    // Drop every buffer (the tree must be built again).  Library-owned
    // buffers are freed once the stream has finished with them.
    void release() {
        invalidate_graph();
        red_off.clear();
        if (!ws && stream) (void)hipStreamSynchronize(stream);
        for (const sph::DevBuf* d : bufs()) {
            sph::DevBuf* m = const_cast<sph::DevBuf*>(d);
            if (m->p && !ws) (void)hipFree(m->p);
            m->p = nullptr;
            m->cap = 0;
        }
        if (ws) ar.reset(ar.base, ar.cap);
        built = sorted = have_density = have_ghost = false;
        saved = false;
        nsegent = 0;
    }

    // A new block of at least `bytes` (want: the preferred, larger size).
    sph::Err take(size_t bytes, size_t want, void** p, size_t* got) {
        if (ws) {
            size_t off;
            if (ar.take(want, &off)) {
                *got = sph::Arena::round(want);
            } else if (ar.take(bytes, &off)) {
                *got = sph::Arena::round(bytes);
            } else {
                // what a workspace would need: the blocks in use plus this one
                ws_needed = std::max(ws_needed, ar.in_use + sph::Arena::round(bytes) + (ar.cap >> 3));
                return sph::Err{SPH_E_WORKSPACE, "workspace of " + std::to_string(ar.cap) + " bytes exhausted (" +
                                                     std::to_string(ar.in_use) + " in use, " +
                                                     std::to_string(bytes) + " more requested)"};
            }
            *p = ar.base + off;
            return sph::Err{};
        }
        hipError_t e = hipMalloc(p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return sph::Err{SPH_E_WORKSPACE, "hipMalloc of " + std::to_string(want) + " bytes failed"};
        }
        *got = want;
        return sph::Err{};
    }

    // Give a block back (stream-ordered reuse in a workspace; a library-owned
    // one is freed after the stream has finished with it).
    void give(void* p, size_t cap) {
        if (!p) return;
        if (ws) {
            ar.give((size_t)((char*)p - ar.base), cap);
        } else {
            if (stream) (void)hipStreamSynchronize(stream);
            (void)hipFree(p);
        }
    }

    // grow-only allocation (contents not kept)
    sph::Err alloc(sph::DevBuf& b, size_t bytes, void** out) {
        bytes = std::max<size_t>(bytes, 256);
        if (b.cap < bytes) {
            give(b.p, b.cap);
            b.p = nullptr;
            b.cap = 0;
            size_t got = 0;
            sph::Err e = take(bytes, bytes + bytes / 8, &b.p, &got);
            if (e.st) return e;
            b.cap = got;
        }
        *out = b.p;
        return sph::Err{};
    }

    // grow keeping the first `keep` bytes (copied on the stream)
    sph::Err grow(sph::DevBuf& b, size_t keep, size_t bytes, void** out) {
        if (b.cap >= bytes) { *out = b.p; return sph::Err{}; }
        void* np = nullptr;
        size_t got = 0;
        sph::Err er = take(bytes, bytes + bytes / 4, &np, &got);
        if (er.st) return er;
        if (keep && b.p) {
            hipError_t e = hipMemcpyAsync(np, b.p, keep, hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) {
                give(np, got);
                return sph::Err{SPH_E_HIP, "grow copy failed"};
            }
        }
        give(b.p, b.cap);
        b.p = np;
        b.cap = got;
        *out = np;
        return sph::Err{};
    }

    sph::SolveState saved_state() const { return sv; }

    static size_t saved_bytes(int64_t m) {
        return (size_t)m * (1 + 7 * sizeof(float) + sizeof(int32_t) + sizeof(uint64_t)) + 256;
    }

    sph::Err ensure_saved() {
        const int64_t m = std::max<int64_t>(n, 1);
        void* p;
        sph::Err e = alloc(b_saved, saved_bytes(m), &p);
        if (e.st) return e;
        layout_saved(p, m);
        return sph::Err{};
    }

    void layout_saved(void* p, int64_t m) {
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
    }

    // Attach a caller-provided workspace (null: go back to one hipMalloc per
    // buffer).  Every buffer is dropped -- the tree must be built again --
    // except the Newton state a solve saved for a rebuild, which is copied
    // into the new memory on the stream (the old memory must stay valid
    // until the stream has run the copy).
    sph::Err set_workspace(void* p, size_t bytes, int gen) {
        sph::DevBuf keep = b_saved;
        const bool had = saved;
        const int64_t sn = saved_n;
        const bool old_ws = ws;
        b_saved = sph::DevBuf{};
        release();
        ws = p != nullptr;
        if (ws) ar.reset(p, bytes);
        else ar = sph::Arena{};
        static_gen = gen;
        ws_needed = 0;
        sph::Err e{};
        if (had && keep.p) {
            const int64_t m = std::max<int64_t>(sn, 1);
            void* np = nullptr;
            e = alloc(b_saved, saved_bytes(m), &np);
            if (!e.st) {
                if (hipMemcpyAsync(np, keep.p, saved_bytes(m), hipMemcpyDeviceToDevice, stream) != hipSuccess)
                    e = sph::Err{SPH_E_HIP, "copy of the saved Newton state failed"};
                layout_saved(np, m);
                saved = e.st == SPH_OK;
                saved_n = sn;
            }
        }
        if (!old_ws && keep.p) {
            if (stream) (void)hipStreamSynchronize(stream);
            (void)hipFree(keep.p);
        }
        return e;
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

void query_occupancy(sph_ctx* ctx);
Err build_tree(sph_ctx* ctx, sph_tree* t, const sph_input* in, const sph_params* prm);
Err sort_pairs(sph_ctx* ctx, sph_tree* t);
Err refresh_tree(sph_ctx* ctx, sph_tree* t, const sph_input* in);
Err run_density(sph_ctx* ctx, sph_tree* t, const sph_density_out* out);
Err run_solve(sph_ctx* ctx, sph_tree* t, const sph_density_out* out, int32_t* n_unconv, int32_t* iters);
Err run_force(sph_ctx* ctx, sph_tree* t, const sph_force_out* out);
Err set_halo(sph_ctx* ctx, sph_tree* t, const uint8_t* owned, const float* rho, const float* drho);
Err run_graph(sph_ctx* ctx, sph_tree* t, int k_iter, const sph_density_out* dout, const sph_force_out* fout,
              int32_t* n_unconv_dev);
}  // namespace sph
