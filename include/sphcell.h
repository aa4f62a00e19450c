/*
 * sphcell.h -- C-ABI of the MI355X (gfx950) SPH density/force library.
 *
 * The library computes the two interaction stages of Section II
 * (Algorithms) of Gonnet, Schaller, Theuns and Chalk, "SWIFT: Fast
 * algorithms for multi-resolution SPH on multi-core architectures"
 * (arXiv:1309.3783):
 *   1. density: for every particle i, sums over all j within h_i;
 *   2. force:   for every particle i, sums over all j within max(h_i, h_j);
 * over a hierarchical cell decomposition (Section II-B) with sorted cell-pair
 * interactions (Section II-C), plus the per-particle solve of h_i to a target
 * neighbour number (N_ngb of Section III-B) and the per-cell "ghost" step
 * between the stages (Section II-D).
 *
 * Conventions
 *  - Every pointer marked [device] is a device pointer owned by the caller;
 *    pointers marked [host] are host memory.
 *  - Device memory of a tree: a caller-provided workspace (the intended use:
 *    sph_workspace_size, sph_tree_set_workspace), carved into the tree's
 *    buffers by the library with no allocation, free or device-wide
 *    synchronisation inside any call; SPH_E_WORKSPACE when it is too small
 *    (sph_tree_workspace_needed says how much to offer, then build again).
 *    Without a workspace the library allocates the tree's buffers itself
 *    (hipMalloc, grow-only; a growth frees the old buffer, which waits for
 *    the device) and frees them in sph_tree_destroy.  A context allocates a
 *    4 KiB device counter block and 64 KiB of pinned host memory once.
 *  - One context per HIP stream.  Every call enqueues work on the context's
 *    stream; outputs are valid once that stream has been synchronised, except
 *    where a host output is documented (those calls synchronise).
 *  - Particles are given as S >= 1 independent sets concatenated in one set
 *    of arrays; set s occupies [offsets[s], offsets[s+1]).  Each set lives in
 *    its own periodic cube [0, box[s])^3.  All per-particle outputs are in
 *    this caller order.
 *  - Errors: calls return SPH_OK (0) or a negative sph_status; host-side
 *    argument errors return before any work is enqueued.  sph_last_error()
 *    gives a text for the last failure on a context.
 *  - Not thread-safe for one context; distinct contexts are independent.
 */
#ifndef SPHCELL_H
#define SPHCELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sph_status;
enum {
    SPH_OK = 0,
    SPH_E_ARG = -1,        /* bad argument (null pointer, size, h too large for the box, ...) */
    SPH_E_HIP = -2,        /* a HIP runtime call failed */
    SPH_E_WORKSPACE = -3,  /* device allocation failed */
    SPH_E_REBUILD = -4,    /* some h_i left the range its cells support: rebuild the tree */
    SPH_E_NOCONV = -5,     /* the h solve did not converge within max_iter */
    SPH_E_CAPACITY = -6,   /* a size limit of the key layout or of a table was exceeded */
    SPH_E_STATE = -7       /* call out of order (e.g. force before density) */
};

typedef struct sph_ctx sph_ctx;
typedef struct sph_tree sph_tree;

/* Flags for sph_params.flags */
#define SPH_FLAG_PAIR_HASH 1u   /* also accumulate the pair-set hashes */
#define SPH_FLAG_RESUME 2u      /* sph_solve_h on a tree built with it continues the Newton state saved when
                                   the previous sph_solve_h on the same tree returned SPH_E_REBUILD
                                   (same particles); converged particles keep their density */
#define SPH_FLAG_NO_BLOCK_SKIP 4u /* read every particle of a partner read in cell order instead of
                                     passing over its blocks beyond a chunk's reach (bitwise the same
                                     results, more loads; for testing) */
#define SPH_FLAG_SORTED_ONLY 8u   /* sweep every partner through its sorted lists, also where the
                                     swept prefix is long and reading the partner in cell order
                                     would pass over most of it (same pairs, other summation order) */

/* Parameters.  Defaults (sph_params_default) follow Section III-B: N_ngb = 48,
 * gamma = 5/3, alpha = 2.0, split if more than 400 particles and more than
 * 87.5% of them have h below half the cell edge. */
typedef struct {
    int32_t n_split;     /* split a cell only if it holds more than this many particles (400) */
    float split_frac;    /* ... and more than this fraction has h < edge/2 (0.875) */
    float h_slack;       /* decisions use h*(1+h_slack) to leave room for h to grow (0.2) */
    int32_t max_depth;   /* levels below the top grid (12) */
    int32_t top_grid;    /* top cells per side (power of two), 0 = largest allowed */
    float n_target;      /* target N_w for the h solve (48) */
    float h_tol;         /* |N_w - n_target| <= h_tol is converged (0.5) */
    int32_t max_iter;    /* Newton iterations per sph_solve_h call (30) */
    float gamma;         /* adiabatic index (5/3) */
    float alpha;         /* viscosity coefficient (2.0) */
    uint32_t flags;      /* SPH_FLAG_* */
    int32_t blocks_per_cu; /* persistent interaction kernels: blocks of 4 wavefronts per CU, at most as
                              many as fit on a CU at once (0 = as many as fit) */
    int32_t max_replicas;  /* lanes per target particle for small chunks: 1, 2, 4, 8 or 16 (0 = 16) */
    int32_t top_coarsen;   /* with top_grid 0: this many levels coarser than the largest allowed top grid
                              (at least 2 cells per side remain) (0) */
    int32_t piece_records; /* heavy chunks: a chunk whose walk is estimated to read at least this many
                              partner records is handed out before the others, split into 8 pieces
                              (16 from twice as many records); 0 = 16384, -1 = off.  A tree on which
                              there would be more than one piece per 64 particles and more
                              than 4096 pieces gets none */
    int32_t reserved[1];
} sph_params;

/* Input particle sets (see Conventions).  h is the initial smoothing length
 * used for the cell decomposition; it is copied at build time. */
typedef struct {
    int32_t nsets;
    const int64_t* offsets;          /* [host]  nsets+1, offsets[0] = 0 */
    const double* box;               /* [host]  nsets periodic box sides */
    const double *x, *y, *z;         /* [device] positions (wrapped into [0,box) internally); the positions
                                        of one set must be distinct (a particle at distance zero from
                                        another one would be taken for itself) */
    const float* h;                  /* [device] smoothing lengths, 0 < h <= box/2 */
    const float *m, *u;              /* [device] masses, specific internal energies */
    const float *vx, *vy, *vz;       /* [device] velocities */
} sph_input;

/* Density-stage outputs (caller order); any pointer may be NULL. */
typedef struct {
    float* rho;          /* [device] rho_i = sum_j m_j W(r_ij, h_i), self included */
    float* drho_dh;      /* [device] d rho_i / d h_i */
    float* nw;           /* [device] N_w,i = (4 pi/3) h_i^3 sum_j W(r_ij, h_i) */
    float* dnw_dh;       /* [device] d N_w,i / d h_i */
    int32_t* nngb;       /* [device] #{j != i : r_ij < h_i} */
    uint64_t* hash;      /* [device] sum over those j of splitmix64(j - offsets[s]) mod 2^64;
                            needs SPH_FLAG_PAIR_HASH at build */
    float* h;            /* [device] the smoothing lengths used (after sph_solve_h: solved) */
} sph_density_out;

/* Force-stage outputs (caller order); any pointer may be NULL. */
typedef struct {
    float *ax, *ay, *az; /* [device] acceleration */
    float* dudt;         /* [device] du/dt */
    float* vsig;         /* [device] max signal velocity over the force neighbours */
    float* S;            /* [device] sum_j m_j |vector pair term| (error scale) */
    int32_t* nforce;     /* [device] #{j != i : r_ij < max(h_i, h_j)} */
    uint64_t* hash;      /* [device] pair-set hash over the same j (SPH_FLAG_PAIR_HASH) */
    double* sums;        /* [device] 8 doubles per set: Mx, My, Mz (sum m a), E (sum
                            m (v.a + du/dt)), sum m S, sum nngb, sum nforce (= 2 P, P the
                            number of unordered interacting pairs), 0 */
} sph_force_out;

/* Library version string and a text for a status code. */
const char* sph_version(void);
const char* sph_status_str(sph_status st);

/* Fill p with the defaults listed above. */
void sph_params_default(sph_params* p);

/* Create a context bound to device `device` and HIP stream `stream` (a
 * hipStream_t, NULL = the default stream).  *out receives the context.  On
 * failure sph_last_error(NULL) says why (per thread). */
sph_status sph_ctx_create(sph_ctx** out, int device, void* stream);
void sph_ctx_destroy(sph_ctx* ctx);
const char* sph_last_error(const sph_ctx* ctx);

/* Wait for everything enqueued on the context's stream (the calls are
 * asynchronous; outputs are valid after this, or after a stream
 * synchronisation or event of the caller's).  Returns SPH_E_HIP, with
 * sph_last_error saying which, when the stream reports an error of work
 * enqueued earlier.  Conditions the kernels detect on the device (h outgrew
 * its cells, no convergence) are not errors of the stream: sph_solve_h
 * returns them, and sph_run_graph leaves them in its status words. */
sph_status sph_ctx_sync(sph_ctx* ctx);

/* Workspace for a tree of n particles in nsets sets (contract of Section II:
 * the two stages' inputs and outputs plus the decomposition of Section II-B
 * and the sorted lists of Section II-C): an estimate for sets like uniform,
 * lattice and clumpy mixtures with up to ~3 decades of h (per particle:
 * ~323 B of particle state, ~580 B of sorted lists, ~240 B of radix scratch
 * for the longest lists, ~120 B of cells, tasks and interaction lists, up to
 * 64 B of partial sums of split heavy chunks; plus 4 KiB per set and
 * 24 MiB).  The need depends
 * on the data; a build that finds the workspace too small fails with
 * SPH_E_WORKSPACE and reports what it needs (sph_tree_workspace_needed).
 * sph_footprint(n, p) = sph_workspace_size(n, 1, p): the size admission
 * control charges per request.  Errors: SPH_E_ARG. */
sph_status sph_workspace_size(int64_t n, int32_t nsets, const sph_params* p, size_t* bytes);
sph_status sph_footprint(int64_t n, const sph_params* p, size_t* bytes);

/* Create an empty tree object (no device memory yet). */
sph_status sph_tree_create(sph_ctx* ctx, sph_tree** out);
void sph_tree_destroy(sph_ctx* ctx, sph_tree* t);
/* Device bytes currently held by the tree's buffers. */
sph_status sph_tree_bytes(const sph_tree* t, size_t* bytes);

/* Give the tree a workspace: ws [device] is a caller-owned region of ws_bytes
 * (at least 1 MiB) that every buffer of the tree is carved from from now on
 * (first fit, 256-byte granules; blocks are freed and reused in the order of
 * the context's stream, so no call allocates, frees or synchronises the
 * device).  ws = NULL returns the tree to library-owned buffers.  The tree's
 * previous buffers are dropped -- build again before the next density or
 * force call -- except the Newton state that a solve saved for a rebuild
 * (SPH_FLAG_RESUME), which is copied into the new memory on the stream: the
 * previous workspace must stay valid until the stream has run past this
 * call.  The workspace must outlive the tree's use of it and must not be
 * shared with another tree.  Errors: SPH_E_ARG, SPH_E_WORKSPACE (the saved
 * state does not fit), SPH_E_HIP. */
sph_status sph_tree_set_workspace(sph_ctx* ctx, sph_tree* t, void* ws, size_t ws_bytes);

/* Bytes a workspace must offer: after a call failed with SPH_E_WORKSPACE, at
 * least what it needed (the blocks in use plus the request, with an eighth of
 * the old size to spare; offer it and repeat the build); otherwise the peak
 * the tree's buffers have used in the current workspace. */
sph_status sph_tree_workspace_needed(const sph_tree* t, size_t* bytes);

/* Section II-B (spatial decomposition): for every set, a top grid of cells of
 * edge >= max h (a power of two per side, at least 2), Morton ordering of the
 * particles, recursive bisection of cells holding more than n_split particles
 * of which more than split_frac have h < edge/2, and the self/pair
 * interaction lists: a self task per non-empty cell, a pair task per
 * non-empty face/edge/corner neighbour (periodic), self tasks of split cells
 * replaced by their children's, pair tasks of split cells replaced by the
 * children pairs across the interface iff every particle in both has
 * h < edge/2.  Copies the inputs into cell-ordered FP32 arrays (positions
 * relative to the top cell origin).  Reuses the tree's device memory when it
 * is large enough.  Synchronises the stream (level sizes are read back).
 * Errors: SPH_E_ARG (bad sizes, h > box/2, non-positive values),
 * SPH_E_CAPACITY (key layout or table limits), SPH_E_WORKSPACE, SPH_E_HIP. */
sph_status sph_build_cells(sph_ctx* ctx, sph_tree* t, const sph_input* in, const sph_params* p);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): sph_build_cells
 * with the library's static scratch as the tree's workspace -- a file-scope
 * device array of 128 MiB per GPU, held until the process ends -- so that
 * neither this call nor the later calls on the tree (sort, density, solve,
 * force) allocate.  Sets needing more than the scratch holds
 * (sph_workspace_size above 128 MiB, roughly 82 000 particles) are refused
 * with SPH_E_CAPACITY; a build that still runs out fails with
 * SPH_E_WORKSPACE.  One tree per GPU can hold the scratch: the calls of a
 * tree that held it before another tree took it fail with SPH_E_STATE (build
 * it again), and calls on two such trees, or on one from two streams, that
 * overlap on the device race.  A repeated call on the tree that holds the
 * scratch keeps its blocks.  Errors as sph_build_cells, plus SPH_E_STATE when
 * the device has no static scratch (no context was created on it). */
sph_status sph_build_cells_static(sph_ctx* ctx, sph_tree* t, const sph_input* in, const sph_params* p);

/* Section II-C (sorted cell pair interactions): for every cell that is the
 * source side of a pair task, the particle indices sorted by their
 * projection on the task's cell-pair axis (one of 13 directions), stored per
 * (cell, axis) and reused by every density and force pass until the next
 * build.  In a tree with more than one level, or with a leaf of 256
 * particles or more, a cell of more than 4096 particles gets no lists
 * (unless SPH_FLAG_SORTED_ONLY): the passes read it in cell order, past its
 * 64-particle blocks out of reach.  Synchronises the stream once, to read
 * the list sizes back; the sorts themselves are enqueued after that and not
 * waited for. */
sph_status sph_sort_pairs(sph_ctx* ctx, sph_tree* t);

/* Section II-C, last paragraph (the sorted indices reused over several time
 * steps until the decomposition must be made again): new particle data for
 * the tree's particles -- the same sets, offsets and boxes, the same caller
 * order as the input of the last sph_build_cells, device pointers laid out as
 * for sph_build_cells (h is the starting h, as there) -- taken without
 * building or sorting again.  Every particle keeps its cell, its place in
 * cell order and its place in each sorted list; positions are stored
 * relative to the origin of the top cell they were built in (the periodic
 * image nearest the cell's centre).  Each set keeps a bound d on any particle's displacement
 * since the build (the largest displacement of every refresh, added up); the
 * density and force sweeps then reach 2 d further along the pair axis, so the
 * lists' build-time order still yields every pair, and the largest h the
 * cells support shrinks by 2 d.  A halo set by sph_set_halo stays set.
 * Synchronises the stream once (one count read back).
 * Errors: SPH_E_STATE (no build), SPH_E_ARG (null arrays, sets, offsets or
 * boxes unlike the build's), SPH_E_REBUILD (some particle's h is at or beyond
 * what its cells support after the displacement: the tree is left unbuilt,
 * call sph_build_cells), SPH_E_HIP. */
sph_status sph_refresh_cells(sph_ctx* ctx, sph_tree* t, const sph_input* in);

/* Density stage (Section II, item 1) for every particle at its current h.
 * Requires sph_sort_pairs. */
sph_status sph_density(sph_ctx* ctx, sph_tree* t, const sph_density_out* out);

/* Smoothing lengths: Section III-B fixes the target (48 neighbours, the
 * weighted count N_w here); the paper does not describe how h is found.
 * Safeguarded Newton iteration per particle on ln N_w against ln h, keeping
 * a bracket of the root, until |N_w,i - n_target| <= h_tol (convergence
 * tested in FP64), re-running the density stage on the particles not yet
 * converged.  Writes the density outputs at the solved h.  *n_unconverged
 * [host] receives the particles left; *iterations [host] the iterations run.
 * Returns SPH_E_REBUILD when some h_i must grow past what the tree supports
 * (out->h then holds the current h: rebuild with it and call again), and
 * SPH_E_NOCONV when max_iter is reached.  The host waits for each pass's
 * counts (the next pass is already enqueued meanwhile); the outputs are
 * written by work still on the stream when the call returns. */
sph_status sph_solve_h(sph_ctx* ctx, sph_tree* t, const sph_density_out* out,
                       int32_t* n_unconverged, int32_t* iterations);

/* Ghost step between the stages (Section II-D: all densities of a cell are
 * complete before its forces): pressure P = (gamma-1) rho u, sound speed,
 * grad-h factor f = 1/(1 + h/(3 rho) drho/dh), A = f P / rho^2; then the
 * force stage (Section II, item 2) and the per-set FP64 sums.  Requires a
 * density pass (sph_density or sph_solve_h) at the current h. */
sph_status sph_force(sph_ctx* ctx, sph_tree* t, const sph_force_out* out);

/* One GPU's share of a set decomposed over several GPUs (Section I: each
 * node works on its part of the data and exchanges what lies across its
 * surface; Section IV: that exchange modelled as tasks).  After a build of
 * the share's particles -- the ones it owns plus the halo, the layer of top
 * cells around them whose edge is at least the largest h, so that every
 * neighbour of an owned particle is present -- mark each particle owned (1)
 * or read-only halo (0) and give the halo particles' density and d rho/d h
 * as their owners computed them (what a halo exchange delivers); h of a
 * halo particle is the one given at build.  From then on until the next
 * build: halo particles are neighbours only -- never solved for h, never
 * targets of the density or force stages; the ghost step takes their given
 * density; the per-set sums cover the owned particles; the outputs of halo
 * particles are not written.  owned, rho, drho_dh: [device] caller order, n
 * entries (rho, drho_dh read for halo particles only).  owned = NULL: every
 * particle owned again.  Errors: SPH_E_STATE (no build), SPH_E_ARG,
 * SPH_E_WORKSPACE, SPH_E_HIP. */
sph_status sph_set_halo(sph_ctx* ctx, sph_tree* t, const uint8_t* owned, const float* rho, const float* drho_dh);

/* Enqueue the whole post-build pipeline -- density/Newton iterations with
 * device-side early exit (k_iter of them), ghost, force and sums -- as one
 * HIP graph on the context's stream: captured and instantiated on first use,
 * and replayed -- also after a new build -- as long as everything it
 * captured is unchanged (output pointers, k_iter, particle / set / chunk /
 * cell counts, parameters and the tree's device buffers, which keep their
 * place in a workspace that does not grow).  Does
 * not synchronise.  n_unconverged_dev [device int32[2 + 2*nsets]] receives
 * [0] the particles still unconverged after the graph, [1] 1 if some h_i
 * outgrew its cells, then per set s: [2+2s] unconverged, [3+2s] rebuild
 * flag.  The Newton passes of a set stop when that set's flag is raised;
 * the outputs of a set with a non-zero word are not valid (re-run that set:
 * rebuild with the returned h). */
sph_status sph_run_graph(sph_ctx* ctx, sph_tree* t, int32_t k_iter, const sph_density_out* dout,
                         const sph_force_out* fout, int32_t* n_unconverged_dev);

/* Time integration (Section III-A: the test runs advance all particles with
 * one fixed time step and recompute every force each step), as the pieces
 * of a kick-drift-kick leapfrog over caller-order arrays.  One step of size
 * dt: sph_kick(dt/2) with the forces a_n, sph_drift(dt), a second
 * sph_kick(dt/2) from the half-step velocities into separate arrays (the
 * velocities and energies predicted for the end of the step, which the
 * viscosity and pressure terms of the new forces use), build / solve_h /
 * force at the new positions, then sph_kick(dt/2) with a_{n+1}.
 *
 * sph_kick: v_out = v + dt a and u_out = u + dt du/dt, element-wise for n
 * particles ([device] arrays; the outputs may alias the inputs).
 * sph_drift: x += dt v (FP64 positions, FP32 velocities) for the particles
 * of every set, each wrapped into [0, box[s]) ([host] offsets, box as in
 * sph_input).
 * sph_cfl_dt: *dt [host] = c_cfl min_i h_i / vsig_i over the particles with
 * vsig_i > 0 (h from the density outputs, vsig from the force outputs;
 * +inf if there are none); synchronises the stream.
 * Errors: SPH_E_ARG (null pointers, bad sizes or a non-finite dt),
 * SPH_E_HIP. */
sph_status sph_kick(sph_ctx* ctx, int64_t n, float dt, const float* vx, const float* vy, const float* vz,
                    const float* u, const float* ax, const float* ay, const float* az, const float* dudt,
                    float* vx_out, float* vy_out, float* vz_out, float* u_out);
sph_status sph_drift(sph_ctx* ctx, int32_t nsets, const int64_t* offsets, const double* box, double dt, double* x,
                     double* y, double* z, const float* vx, const float* vy, const float* vz);
sph_status sph_cfl_dt(sph_ctx* ctx, int64_t n, const float* h, const float* vsig, float c_cfl, double* dt);

/* Per-stage timing (milliseconds, from HIP events recorded on the context's
 * stream while timing is enabled) of every call since the timings were last
 * read, in call order: names[i] = stage name, ms[i] = time.  Reading
 * synchronises with the last recorded event; recording does not.  Returns
 * the number of stages written (at most cap). */
int32_t sph_last_timings(sph_ctx* ctx, const char** names, double* ms, int32_t cap);
/* Pair evaluations counted on the device for the measurement of the
 * interaction kernels against their roofline: *density_pairs [host] = the
 * sum, over the particles each density pass evaluated, of their neighbour
 * counts (ordered pairs i <- j with r < h_i), over all passes of the last
 * sph_density / sph_solve_h call (or graph); *force_pairs [host] = the same
 * for the last force pass (ordered pairs with r < max(h_i, h_j), = 2 P).
 * Synchronises the context's stream.  Errors: SPH_E_ARG, SPH_E_HIP. */
sph_status sph_last_work(sph_ctx* ctx, uint64_t* density_pairs, uint64_t* force_pairs);

/* Records the interaction walks loaded in the same passes as sph_last_work
 * counts (self-task particles plus the swept or cell-order records of the
 * pair tasks, each time a chunk's frame reads them): *density_records and
 * *force_records [host].  Set beside the pair evaluations, they give the
 * share of loaded records that fall within reach (Section II-C: the sorted
 * sweeps bound the records read per pair task).  Synchronises the
 * context's stream.  Errors: SPH_E_ARG, SPH_E_HIP. */
sph_status sph_last_reads(sph_ctx* ctx, uint64_t* density_records, uint64_t* force_records);

/* Enable (1) or disable (0) per-stage event timing on the context. */
void sph_enable_timing(sph_ctx* ctx, int32_t on);

/* Tree statistics (host): [0] particles, [1] cells, [2] leaves, [3] tasks
 * (self + pair), [4] pair tasks, [5] sorted entries, [6] work chunks,
 * [7] levels, [8] top cells per side of set 0, [9] max leaf size, [10] HIP
 * graphs captured and instantiated by sph_run_graph on this tree so far,
 * [11] heavy chunks (handed out first, see sph_params.piece_records), [12]
 * their pieces.
 * May synchronise the tree's stream (a count the sort kept on the device). */
sph_status sph_tree_stats(const sph_tree* t, int64_t* stats, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* SPHCELL_H */
