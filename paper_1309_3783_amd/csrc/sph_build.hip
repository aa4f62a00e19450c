// Cell decomposition, interaction lists and per-(cell, axis) sorted lists.
//
//  * Spatial decomposition (Section II-B): per set a top grid of 2^k cells per
//    side with edge >= max h; particles ordered by Morton key; level-by-level
//    bisection of cells with more than n_split particles of which more than
//    split_frac have h < edge/2 (Section III-B gives 400 and 87.5%).
//  * Interaction lists (Section II-B): a self task per non-empty top cell and
//    a pair task per non-empty face/edge/corner neighbour (periodic images
//    included); a split cell's self task becomes its children's self tasks
//    plus the 28 child pairs; a pair of split cells becomes the child pairs
//    across the interface iff every particle of both has h < edge/2.
//  * Sorted lists (Section II-C): for every (cell, axis) that is the source
//    side of a pair task, the particles sorted by projection on the axis.
//
// Everything here is integer or compare work and bound by memory traffic;
// the level loop reads one count back per level to size the next one.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sph_impl.h"


namespace sph {

__device__ inline uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
    v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
    v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
    v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
    v = (v ^ (v >> 32)) & 0x1FFFFFull;
    return (uint32_t)v;
}

__device__ inline int set_of_particle(const SetInfo* sets, int nsets, int64_t i) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sets[mid].first <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline int set_of_top(const SetInfo* sets, int nsets, int c) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sets[mid].top_base <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline int64_t lower_bound_key(const uint64_t* key, int64_t lo, int64_t hi, uint64_t k) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (key[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline float wave_max_f(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}
__device__ inline int wave_sum_i(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ inline uint64_t splitmix64(uint64_t id) {
    uint64_t z = id + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Per-set max and min h and count of invalid h (not finite or <= 0).  Grid
// (chunks, sets); positive floats compare like their bit patterns, so the
// extremes are integer atomics.
__global__ __launch_bounds__(256) void k_set_hstats(const SetInfo* sets, const float* __restrict__ h,
                                                    int* __restrict__ hmax_bits, int* __restrict__ hmin_bits,
                                                    int* __restrict__ bad_out) {
    const SetInfo S = sets[blockIdx.y];
    float m = 0.f, mn = INFINITY;
    int bad = 0;
#pragma unroll 8
    for (int64_t i = S.first + (int64_t)blockIdx.x * 256 + threadIdx.x; i < S.first + S.count;
         i += (int64_t)gridDim.x * 256) {
        float v = h[i];
        if (!(v > 0.f) || !(v < INFINITY)) {
            bad++;
        } else {
            m = fmaxf(m, v);
            mn = fminf(mn, v);
        }
    }
    m = wave_max_f(m);
    mn = -wave_max_f(-mn);
    bad = wave_sum_i(bad);
    // one atomic per block: many blocks update the same word
    __shared__ float s_m[4], s_n[4];
    __shared__ int s_b[4];
    if ((threadIdx.x & 63) == 0) {
        s_m[threadIdx.x >> 6] = m;
        s_n[threadIdx.x >> 6] = mn;
        s_b[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]));
        mn = fminf(fminf(s_n[0], s_n[1]), fminf(s_n[2], s_n[3]));
        bad = s_b[0] + s_b[1] + s_b[2] + s_b[3];
        atomicMax(&hmax_bits[blockIdx.y], __float_as_int(m));
        atomicMin(&hmin_bits[blockIdx.y], __float_as_int(mn));
        if (bad) atomicAdd(&bad_out[blockIdx.y], bad);
    }
}

// Integer cell coordinate at 2^(lgG+depth) cells per side (same formula in
// k_keys and k_gather so both place a particle in the same cell).  The
// depth is per set (the levels its h range can need), so a set's keys -- and
// with them the order of its particles -- do not depend on the other sets of
// a batch.
__device__ inline int64_t fine_coord(double x, double box, int64_t R) {
    double w = x - box * floor(x / box);
    int64_t k = (int64_t)floor(w / box * (double)R);
    return k < 0 ? 0 : (k >= R ? R - 1 : k);
}

// The caller's particle data of one particle, packed in caller order (so
// that the gather into cell order reads one 48-byte record per particle
// instead of nine scattered words).
struct InRec {
    double x, y, z;
    float h, m, u, vx, vy, vz;
};
static_assert(sizeof(InRec) == 48, "packed input record");

__global__ void k_keys(const SetInfo* sets, int nsets, int64_t n, const double* __restrict__ x,
                       const double* __restrict__ y, const double* __restrict__ z, const float* __restrict__ h,
                       const float* __restrict__ m, const float* __restrict__ u, const float* __restrict__ vx,
                       const float* __restrict__ vy, const float* __restrict__ vz, int bmax,
                       uint64_t* __restrict__ key, uint32_t* __restrict__ val, InRec* __restrict__ rec) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s = set_of_particle(sets, nsets, i);
    const SetInfo S = sets[s];
    int64_t R = (int64_t)1 << (S.lgG + S.depth);
    const double xi = x[i], yi = y[i], zi = z[i];
    uint64_t ix = (uint64_t)fine_coord(xi, S.box, R);
    uint64_t iy = (uint64_t)fine_coord(yi, S.box, R);
    uint64_t iz = (uint64_t)fine_coord(zi, S.box, R);
    key[i] = ((uint64_t)s << (3 * bmax)) | (morton3(ix, iy, iz) << S.key_shift);
    val[i] = (uint32_t)i;
    InRec r;
    r.x = xi;
    r.y = yi;
    r.z = zi;
    r.h = h[i];
    r.m = m[i];
    r.u = u[i];
    r.vx = vx[i];
    r.vy = vy[i];
    r.vz = vz[i];
    rec[i] = r;
}

// The same packing alone (a refresh: the keys are the build's).
__global__ void k_pack_inputs(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                              const double* __restrict__ z, const float* __restrict__ h,
                              const float* __restrict__ m, const float* __restrict__ u,
                              const float* __restrict__ vx, const float* __restrict__ vy,
                              const float* __restrict__ vz, InRec* __restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    InRec r;
    r.x = x[i];
    r.y = y[i];
    r.z = z[i];
    r.h = h[i];
    r.m = m[i];
    r.u = u[i];
    r.vx = vx[i];
    r.vy = vy[i];
    r.vz = vz[i];
    rec[i] = r;
}

__global__ void k_gather(const SetInfo* sets, int nsets, int64_t n, int bmax,
                         const uint64_t* __restrict__ key, const uint32_t* __restrict__ val,
                         const InRec* __restrict__ rec, float slack, float4* __restrict__ pos,
                         float4* __restrict__ plo, float* __restrict__ ph, float* __restrict__ hdec, float* __restrict__ pu,
                         float4* __restrict__ pv, uint32_t* __restrict__ perm, uint32_t* __restrict__ iperm,
                         uint64_t* __restrict__ mix) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t i = val[p];
    int s = nsets > 1 ? (int)(key[p] >> (3 * bmax)) : 0;
    const SetInfo S = sets[s];
    int64_t R = (int64_t)1 << (S.lgG + S.depth);
    const InRec r = rec[i];
    double xs[3] = {r.x, r.y, r.z};
    float o[3], lo[3];
    for (int d = 0; d < 3; ++d) {
        double w = xs[d] - S.box * floor(xs[d] / S.box);
        int64_t top = fine_coord(xs[d], S.box, R) >> S.depth;
        // offset from the top cell origin: exact in FP64 (w and top L0 are
        // within a factor two of each other, or top = 0), then split into
        // its FP32 rounding and the FP32 rounding of the remainder
        const double off = w - (double)top * S.L0;
        o[d] = (float)off;
        lo[d] = (float)(off - (double)o[d]);
    }
    pos[p] = make_float4(o[0], o[1], o[2], r.m);
    plo[p] = make_float4(lo[0], lo[1], lo[2], 0.f);
    const float hh = r.h;
    ph[p] = hh;
    hdec[p] = hh * (1.0f + slack);
    pu[p] = r.u;
    pv[p] = make_float4(r.vx, r.vy, r.vz, 0.f);
    perm[p] = i;
    iperm[i] = (uint32_t)p;
    mix[p] = splitmix64((uint64_t)((int64_t)i - S.first));
}

__device__ inline void cell_key_range(const SetInfo& S, int bmax, int level, int ix, int iy, int iz, int set,
                                      uint64_t* lo, uint64_t* hi) {
    uint64_t code = morton3((uint64_t)ix, (uint64_t)iy, (uint64_t)iz);
    int sh = S.key_shift + 3 * (S.depth - level);
    uint64_t base = ((uint64_t)set << (3 * bmax));
    *lo = base | (code << sh);
    *hi = *lo + (1ull << sh);
}

__global__ void k_top_cells(const SetInfo* sets, int nsets, int ntop, int bmax,
                            const uint64_t* __restrict__ key, Cell* __restrict__ cells) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ntop) return;
    int s = set_of_top(sets, nsets, c);
    const SetInfo S = sets[s];
    uint64_t t = (uint64_t)(c - S.top_base);
    Cell C;
    C.ix = (int)compact3(t >> 2);
    C.iy = (int)compact3(t >> 1);
    C.iz = (int)compact3(t);
    C.level = 0;
    C.set = (int16_t)s;
    C.parent = -1;
    C.child = -1;
    uint64_t lo, hi;
    cell_key_range(S, bmax, 0, C.ix, C.iy, C.iz, s, &lo, &hi);
    int64_t a = lower_bound_key(key, S.first, S.first + S.count, lo);
    int64_t b = lower_bound_key(key, a, S.first + S.count, hi);
    C.first = (int32_t)a;
    C.count = (int32_t)(b - a);
    C.hmax = 0.f;
    C.hcur = 0.f;
    C.hcur_l = 0.f;
    C.bound = nextafterf((float)S.L0, INFINITY);
    C.split = 0;
    C.nsmall = 0;
    C.pad[0] = C.pad[1] = 0;
    cells[c] = C;
}

// One wave per cell of level `level`: particle range (children of a split
// parent look theirs up inside the parent's range), max decision h, the
// number with h < edge/2, and the split decision.
__global__ __launch_bounds__(256) void k_cell_stats(const SetInfo* sets, int bmax, int level,
                                                    int64_t c0, int64_t c1, const uint64_t* __restrict__ key,
                                                    const float* __restrict__ hdec, int n_split,
                                                    float split_frac, Cell* __restrict__ cells) {
    const int lane = threadIdx.x & 63;
    int64_t c = c0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= c1) return;
    Cell C = cells[c];
    const SetInfo S = sets[C.set];
    if (level > 0) {
        const Cell P = cells[C.parent];
        uint64_t lo, hi;
        cell_key_range(S, bmax, level, C.ix, C.iy, C.iz, C.set, &lo, &hi);
        int64_t a = lower_bound_key(key, P.first, (int64_t)P.first + P.count, lo);
        int64_t b = lower_bound_key(key, a, (int64_t)P.first + P.count, hi);
        C.first = (int32_t)a;
        C.count = (int32_t)(b - a);
    }
    const float half = (float)(0.5 * S.L0 / (double)(1 << level));
    float hm = 0.f;
    int nsmall = 0;
#pragma unroll 8
    for (int64_t p = C.first + lane; p < (int64_t)C.first + C.count; p += 64) {
        float hh = hdec[p];
        hm = fmaxf(hm, hh);
        nsmall += hh < half ? 1 : 0;
    }
    hm = wave_max_f(hm);
    nsmall = wave_sum_i(nsmall);
    if (lane == 0) {
        C.hmax = hm;
        C.split = (level < S.depth && C.count > n_split &&
                   (double)nsmall > (double)split_frac * (double)C.count) ? 1u : 0u;
        cells[c] = C;
    }
}

__global__ void k_split_flags(const Cell* __restrict__ cells, int64_t c0, int64_t c1, uint32_t* flags) {
    int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < c1) flags[c - c0] = cells[c].split;
}

__global__ void k_make_children(int64_t c0, int64_t c1, int64_t next0, const uint32_t* __restrict__ sidx,
                                Cell* __restrict__ cells) {
    int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    Cell P = cells[c];
    if (!P.split) return;
    int64_t base = next0 + 8 * (int64_t)sidx[c - c0];
    cells[c].child = (int32_t)base;
    for (int o = 0; o < 8; ++o) {
        Cell C;
        C.first = P.first;
        C.count = P.count;
        C.parent = (int32_t)c;
        C.child = -1;
        C.ix = 2 * P.ix + ((o >> 2) & 1);
        C.iy = 2 * P.iy + ((o >> 1) & 1);
        C.iz = 2 * P.iz + (o & 1);
        C.level = (int16_t)(P.level + 1);
        C.set = P.set;
        C.hmax = 0.f;
        C.hcur = 0.f;
        C.hcur_l = 0.f;
        C.bound = INFINITY;
        C.split = 0;
        C.nsmall = 0;
        C.pad[0] = C.pad[1] = 0;
        cells[base + o] = C;
    }
}

// ---------------------------------------------------------------------------
// Tasks: int4 (ci, cj, offset code, 0); self tasks have ci == cj, code 13.
// ---------------------------------------------------------------------------
__device__ inline int top_neighbour(const SetInfo& S, const Cell& A, int ox, int oy, int oz) {
    int G = 1 << S.lgG;
    int bx = (A.ix + ox + G) & (G - 1), by = (A.iy + oy + G) & (G - 1), bz = (A.iz + oz + G) & (G - 1);
    return S.top_base + (int)morton3((uint64_t)bx, (uint64_t)by, (uint64_t)bz);
}

__global__ void k_top_task_count(const SetInfo* sets, int ntop, const Cell* __restrict__ cells, uint32_t* cnt) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ntop) return;
    const Cell A = cells[c];
    if (A.count == 0) { cnt[c] = 0; return; }
    const SetInfo S = sets[A.set];
    uint32_t k = 1;
    for (int a = 0; a < 13; ++a) {
        int code = axis_code(a);
        int B = top_neighbour(S, A, ocx(code), ocy(code), ocz(code));
        if (cells[B].count > 0) ++k;
    }
    cnt[c] = k;
}

__global__ void k_top_task_emit(const SetInfo* sets, int ntop, const Cell* __restrict__ cells,
                                const uint32_t* __restrict__ off, int4* __restrict__ out) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ntop) return;
    const Cell A = cells[c];
    if (A.count == 0) return;
    const SetInfo S = sets[A.set];
    uint32_t k = off[c];
    out[k++] = make_int4(c, c, 13, 0);
    for (int a = 0; a < 13; ++a) {
        int code = axis_code(a);
        int B = top_neighbour(S, A, ocx(code), ocy(code), ocz(code));
        if (cells[B].count > 0) out[k++] = make_int4(c, B, code, 0);
    }
}

// Interaction-list keys: target << 37 | source << 5 | offset code.
constexpr int CSR_SRC_SHIFT = 5;
constexpr int CSR_TGT_SHIFT = 37;

// Interaction lists of a tree of one level, straight from the top grid: the
// entries of cell c are the pair tasks (c, B, o) it emits (one per non-empty
// neighbour in the 13 positive directions) and the tasks (A', c, o) of its
// non-empty neighbours A' in the 13 negative directions, in the order a
// stable sort of the task list by target gives: by emitting cell, then by
// axis (tasks are emitted per cell in cell order, each cell's in axis
// order).  COUNT: only the number of entries per cell.
template <bool COUNT>
__global__ void k_top_csr(const SetInfo* sets, int ntop, const Cell* __restrict__ cells,
                          const uint32_t* __restrict__ off, uint32_t* __restrict__ cnt,
                          uint64_t* __restrict__ csr) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ntop) return;
    const Cell A = cells[c];
    if (A.count == 0) {
        if (COUNT) cnt[c] = 0;
        return;
    }
    const SetInfo S = sets[A.set];
    int src[26];
    bool ok[26];
    int64_t key[26];
#pragma unroll
    for (int a = 0; a < 13; ++a) {
        const int code = axis_code(a);
        const int ox = ocx(code), oy = ocy(code), oz = ocz(code);
        const int B = top_neighbour(S, A, ox, oy, oz);
        const int Ap = top_neighbour(S, A, -ox, -oy, -oz);
        src[a] = B;
        ok[a] = cells[B].count > 0;
        key[a] = ((int64_t)c << 5) | a;
        src[13 + a] = Ap;
        ok[13 + a] = cells[Ap].count > 0;
        key[13 + a] = ((int64_t)Ap << 5) | a;
    }
    if (COUNT) {
        uint32_t k = 0;
#pragma unroll
        for (int i = 0; i < 26; ++i) k += ok[i] ? 1u : 0u;
        cnt[c] = k;
        return;
    }
    const uint32_t o = off[c];
#pragma unroll
    for (int i = 0; i < 26; ++i) {
        if (!ok[i]) continue;
        uint32_t pos = 0;
#pragma unroll
        for (int j = 0; j < 26; ++j) pos += (ok[j] && key[j] < key[i]) ? 1u : 0u;
        const int code = i < 13 ? axis_code(i) : 26 - axis_code(i - 13);
        csr[o + pos] = ((uint64_t)c << CSR_TGT_SHIFT) | ((uint64_t)src[i] << CSR_SRC_SHIFT) | (uint64_t)code;
    }
}

__device__ inline uint32_t nonempty_children(const Cell* cells, const Cell& A) {
    uint32_t m = 0;
    for (int o = 0; o < 8; ++o)
        if (cells[A.child + o].count > 0) m |= 1u << o;
    return m;
}

__device__ inline bool child_adjacent(int ox, int oy, int oz, int a, int b, int* cx, int* cy, int* cz) {
    *cx = 2 * ox + ((b >> 2) & 1) - ((a >> 2) & 1);
    *cy = 2 * oy + ((b >> 1) & 1) - ((a >> 1) & 1);
    *cz = 2 * oz + (b & 1) - (a & 1);
    return abs(*cx) <= 1 && abs(*cy) <= 1 && abs(*cz) <= 1;
}

// Decide each task of one level: final (kept) or replaced by child tasks.
// A pair of split cells is split iff max h (decision h) of both < edge/2;
// the cells then record edge/2 as the bound their particles' h must stay
// below.  All writes of one level store the same value, so races are benign.
__global__ void k_task_decide(const SetInfo* sets, const int4* __restrict__ tasks, int64_t nt,
                              Cell* __restrict__ cells, uint32_t* __restrict__ fin, uint32_t* __restrict__ nch) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int4 T = tasks[t];
    const Cell A = cells[T.x];
    if (T.x == T.y) {
        if (A.split) {
            uint32_t m = nonempty_children(cells, A);
            uint32_t k = __popc(m);
            fin[t] = 0;
            nch[t] = k + k * (k - 1) / 2;
        } else {
            fin[t] = 1;
            nch[t] = 0;
        }
        return;
    }
    const Cell B = cells[T.y];
    const SetInfo S = sets[A.set];
    const float half = (float)(0.5 * S.L0 / (double)(1 << A.level));
    if (A.split && B.split && fmaxf(A.hmax, B.hmax) < half) {
        uint32_t ma = nonempty_children(cells, A), mb = nonempty_children(cells, B);
        int ox = ocx(T.z), oy = ocy(T.z), oz = ocz(T.z);
        uint32_t k = 0;
        for (int a = 0; a < 8; ++a) {
            if (!((ma >> a) & 1)) continue;
            for (int b = 0; b < 8; ++b) {
                int cx, cy, cz;
                if (((mb >> b) & 1) && child_adjacent(ox, oy, oz, a, b, &cx, &cy, &cz)) ++k;
            }
        }
        fin[t] = 0;
        nch[t] = k;
        cells[T.x].bound = half;
        cells[T.y].bound = half;
    } else {
        fin[t] = 1;
        nch[t] = 0;
    }
}

__global__ void k_task_emit(const int4* __restrict__ tasks, int64_t nt, const Cell* __restrict__ cells,
                            const uint32_t* __restrict__ fin, const uint32_t* __restrict__ fpos,
                            const uint32_t* __restrict__ nch, const uint32_t* __restrict__ cpos,
                            int4* __restrict__ final_out, int4* __restrict__ next_out) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int4 T = tasks[t];
    if (fin[t]) {
        final_out[fpos[t]] = T;
        return;
    }
    if (nch[t] == 0) return;
    uint32_t k = cpos[t];
    const Cell A = cells[T.x];
    if (T.x == T.y) {
        uint32_t m = nonempty_children(cells, A);
        for (int a = 0; a < 8; ++a)
            if ((m >> a) & 1) next_out[k++] = make_int4(A.child + a, A.child + a, 13, 0);
        for (int a = 0; a < 8; ++a) {
            if (!((m >> a) & 1)) continue;
            for (int b = a + 1; b < 8; ++b) {
                if (!((m >> b) & 1)) continue;
                int code = ocode(((b >> 2) & 1) - ((a >> 2) & 1), ((b >> 1) & 1) - ((a >> 1) & 1),
                                 (b & 1) - (a & 1));
                next_out[k++] = make_int4(A.child + a, A.child + b, code, 0);
            }
        }
        return;
    }
    const Cell B = cells[T.y];
    uint32_t ma = nonempty_children(cells, A), mb = nonempty_children(cells, B);
    int ox = ocx(T.z), oy = ocy(T.z), oz = ocz(T.z);
    for (int a = 0; a < 8; ++a) {
        if (!((ma >> a) & 1)) continue;
        for (int b = 0; b < 8; ++b) {
            int cx, cy, cz;
            if (((mb >> b) & 1) && child_adjacent(ox, oy, oz, a, b, &cx, &cy, &cz))
                next_out[k++] = make_int4(A.child + a, B.child + b, ocode(cx, cy, cz), 0);
        }
    }
}

// ---------------------------------------------------------------------------
// Leaves -> work chunks of at most CHUNK particles; per-particle h bound.
// ---------------------------------------------------------------------------
// The number of non-empty leaves and the largest leaf (one atomic per block).
__global__ __launch_bounds__(256) void k_chunk_count(const Cell* __restrict__ cells, int64_t nc, int* stats) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool leaf = false;
    int count = 0;
    if (c < nc) {
        const Cell C = cells[c];
        leaf = !C.split && C.count > 0;
        count = leaf ? C.count : 0;
    }
    int nl = __popcll(__ballot(leaf));
    for (int d = 32; d >= 1; d >>= 1) count = max(count, __shfl_xor(count, d, 64));
    __shared__ int s_n[4], s_c[4];
    if ((threadIdx.x & 63) == 0) {
        s_n[threadIdx.x >> 6] = nl;
        s_c[threadIdx.x >> 6] = count;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        nl = s_n[0] + s_n[1] + s_n[2] + s_n[3];
        count = max(max(s_c[0], s_c[1]), max(s_c[2], s_c[3]));
        if (nl) {
            atomicAdd(&stats[0], nl);
            atomicMax(&stats[1], count);
        }
    }
}

// The chunks are numbered in particle (cell) order, so that the chunk list
// runs through space in Morton order: a leaf marks the first particle of each
// of its chunks, a scan of the marks gives the chunk numbers.
__global__ void k_chunk_mark(const Cell* __restrict__ cells, int64_t nc, uint32_t* __restrict__ mark) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const Cell C = cells[c];
    if (C.split || C.count == 0) return;
    for (int s = 0; s < C.count; s += CHUNK) mark[C.first + s] = 1u;
}

__global__ void k_chunk_emit(const Cell* __restrict__ cells, int64_t nc, const uint32_t* __restrict__ num,
                             int4* __restrict__ chunks) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const Cell C = cells[c];
    if (C.split || C.count == 0) return;
    int top = (int)c;   // the leaf's top cell
    while (cells[top].parent >= 0) top = cells[top].parent;
    for (int s = 0; s < C.count; s += CHUNK)
        chunks[num[C.first + s]] = make_int4((int)c, C.first + s, min(CHUNK, C.count - s), top);
}

// Heavy chunks.  A chunk whose walk reads far more partner records than
// most (a leaf of large h next to dense cells) would run alone at the end
// of a pass; such chunks are handed out before the others, split into
// pieces that each take every P-th group of the records the walk reads,
// and the pieces' partial sums are added in piece order after the pass.
// The records read are estimated as the sorted sweeps read them: per pair
// entry the partner's particle count times the fraction of the partner
// cell whose projection on the pair direction lies within the leaf's
// largest h of the leaf cell's farthest projection (particles spread
// evenly along the direction).  pcount: pieces per chunk (0 for the chunks handed out
// with the others); poff: the first list slot of its pieces, reserved with
// one atomic per heavy chunk (the slots' order changes no result: the
// pieces of a chunk are contiguous and added in piece order); total[0]
// counts the pieces, total[1] the heavy chunks.
// One wave per chunk, a lane per pair entry.
__global__ __launch_bounds__(256) void k_chunk_cost(const int4* __restrict__ chunks,
                                                    const uint32_t* __restrict__ nch_dev, int64_t cap,
                                                    const Cell* __restrict__ cells, const SetInfo* __restrict__ sets,
                                                    const uint32_t* __restrict__ csr_off,
                                                    const uint64_t* __restrict__ csr, float piece,
                                                    uint32_t* __restrict__ pcount, uint32_t* __restrict__ poff,
                                                    uint32_t* __restrict__ total) {
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= cap) return;
    if (c >= (int64_t)*nch_dev) {
        if (lane == 0) pcount[c] = 0;
        return;
    }
    const int4 ch = chunks[c];
    const Cell L = cells[ch.x];
    // lengths in top-cell edges; cell corners as integer coordinates times
    // the edge of their level (exact)
    const float hr = (float)((double)L.hmax / sets[L.set].L0);
    const float el = ldexpf(1.f, -L.level);
    const float lo[3] = {(float)L.ix * el, (float)L.iy * el, (float)L.iz * el};
    float est = 0.f;
    for (int A = ch.x; A >= 0;) {
        const Cell CA = cells[A];
        const float ea = ldexpf(1.f, -CA.level);
        const uint32_t e1 = csr_off[A + 1];
        for (uint32_t e = csr_off[A] + lane; e < e1; e += 64) {
            const uint64_t key = csr[e];
            const int B = (int)((key >> CSR_SRC_SHIFT) & 0xFFFFFFFFull), code = (int)(key & 31);
            const int o[3] = {ocx(code), ocy(code), ocz(code)};
            const int ci[3] = {CA.ix, CA.iy, CA.iz};
            // the leaf's farthest projection on o, the partner's range
            float tb = 0.f, p0 = 0.f, p1 = 0.f;
            for (int d = 0; d < 3; ++d) {
                const float b0 = (float)(ci[d] + o[d]) * ea;
                if (o[d] > 0) {
                    tb += lo[d] + el;
                    p0 += b0;
                    p1 += b0 + ea;
                } else if (o[d] < 0) {
                    tb -= lo[d];
                    p0 -= b0 + ea;
                    p1 -= b0;
                }
            }
            const int nz = abs(o[0]) + abs(o[1]) + abs(o[2]);
            const float dn = nz == 1 ? 1.f : (nz == 2 ? 1.41421356f : 1.73205081f);
            const float f = fminf(fmaxf((tb + hr * dn - p0) / (p1 - p0), 0.f), 1.f);
            est += (float)cells[B].count * f;
        }
        A = CA.parent;
    }
    for (int d = 32; d >= 1; d >>= 1) est += __shfl_xor(est, d, 64);
    if (lane != 0) return;
    // at the threshold 8 pieces, up to PIECE_MAX for twice as many records
    int pn = 0;
    if (piece > 0.f && est >= piece) pn = min((int)ceilf(8.f * est / piece), PIECE_MAX);
    pcount[c] = (uint32_t)pn;
    if (pn > 0) {
        poff[c] = atomicAdd(&total[0], (uint32_t)pn);
        atomicAdd(&total[1], 1u);
    }
}

__global__ void k_piece_emit(const uint32_t* __restrict__ nch_dev, const uint32_t* __restrict__ pcount,
                             const uint32_t* __restrict__ poff, uint32_t* __restrict__ list) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)*nch_dev) return;
    const uint32_t pn = pcount[c];
    for (uint32_t k = 0; k < pn; ++k) list[poff[c] + k] = ((uint32_t)c << 5) | k;
}

// One wave per chunk (the chunk count is read on the device).
// The bound of a particle is the smallest bound of its leaf and ancestors,
// less twice its set's accumulated displacement since the build (zero right
// after a build): two particles that moved by at most d each and interact
// now were within h + 2d at the build, and the cells only guarantee pairs
// closer than their bound.  With viol given, the particles whose current h
// is not below their bound are counted there.
__global__ __launch_bounds__(256) void k_particle_bound(const int4* __restrict__ chunks,
                                                        const uint32_t* __restrict__ nch_dev,
                                                        const Cell* __restrict__ cells, const SetInfo* sets,
                                                        const float* __restrict__ ph, float* __restrict__ bound,
                                                        uint32_t* __restrict__ viol) {
    const int64_t nch = *nch_dev;
    const int lane = threadIdx.x & 63;
    for (int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); q < nch; q += (int64_t)gridDim.x * 4) {
        const int4 ch = chunks[q];
        float b = INFINITY;
        for (int A = ch.x; A >= 0; A = cells[A].parent) b = fminf(b, cells[A].bound);
        const float d = sets[cells[ch.x].set].drift;
        if (d > 0.f) b -= 2.f * d;
        if (lane < ch.z) bound[ch.y + lane] = b;
        if (viol) {
            const bool bad = lane < ch.z && !(ph[ch.y + lane] < b);
            const uint64_t m = __ballot(bad);
            if (lane == 0 && m) atomicAdd(viol, (uint32_t)__popcll(m));
        }
    }
}

// ---------------------------------------------------------------------------
// Reuse of a built tree over time steps (Section II-C: the sorted indices
// are kept until the decomposition has to be made again).  The particles
// keep their cells, their place in cell order and their place in every
// sorted list; only their data are replaced.
// ---------------------------------------------------------------------------

// New data of every particle of a chunk (one wavefront per chunk, chunks
// strided over a bounded grid): the position as FP32 offset from the origin
// of the top cell it was built in (the periodic image nearest the cell's
// centre) plus FP32
// remainder, h, m, u, v.  The largest displacement against the stored
// position is folded into stepmax[set] (non-negative floats compare like
// their bit patterns): kept per wave while its chunks stay in one set,
// combined per block, one atomic per block and set (atomics on one word from
// every wave would serialise).
constexpr int REFRESH_BLOCKS = 2048;
__global__ __launch_bounds__(256) void k_refresh(const int4* __restrict__ chunks, const uint32_t* __restrict__ nch_dev,
                                                 const Cell* __restrict__ cells, const SetInfo* sets,
                                                 const uint32_t* __restrict__ perm, const InRec* __restrict__ rec,
                                                 float slack, float4* __restrict__ pos, float4* __restrict__ plo,
                                                 float* __restrict__ ph, float* __restrict__ hdec,
                                                 float* __restrict__ pu, float4* __restrict__ pv,
                                                 unsigned* __restrict__ stepmax) {
    const int64_t nch = *nch_dev;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int cur = -1;          // set of the running maximum
    float run = 0.f;
    for (int64_t q = (int64_t)blockIdx.x * 4 + w; q < nch; q += (int64_t)gridDim.x * 4) {
        const int4 ch = chunks[q];
        const Cell T = cells[ch.w];
        const SetInfo S = sets[T.set];
        double d2 = 0.0;
        if (lane < ch.z) {
            const int64_t p = ch.y + lane;
            const InRec r = rec[perm[p]];
            const double xs[3] = {r.x, r.y, r.z};
            const int tc[3] = {T.ix, T.iy, T.iz};
            const float4 o0 = pos[p], l0 = plo[p];
            const double old[3] = {(double)o0.x + (double)l0.x, (double)o0.y + (double)l0.y,
                                   (double)o0.z + (double)l0.z};
            float o[3], lo[3];
            for (int d = 0; d < 3; ++d) {
                // the periodic image nearest the top cell's centre (with two
                // top cells per side the nearest to its origin can be the
                // wrong one for a particle just past the far face)
                double off = xs[d] - S.box * floor(xs[d] / S.box) - (double)tc[d] * S.L0;
                off -= S.box * rint((off - 0.5 * S.L0) / S.box);
                o[d] = (float)off;
                lo[d] = (float)(off - (double)o[d]);
                const double dd = off - old[d];
                d2 += dd * dd;
            }
            pos[p] = make_float4(o[0], o[1], o[2], r.m);
            plo[p] = make_float4(lo[0], lo[1], lo[2], 0.f);
            const float hh = r.h;
            ph[p] = hh;
            hdec[p] = hh * (1.0f + slack);
            pu[p] = r.u;
            pv[p] = make_float4(r.vx, r.vy, r.vz, 0.f);
        }
        // rounded up so that the bound stays a bound
        float dm = (float)sqrt(d2);
        if ((double)dm < sqrt(d2)) dm = nextafterf(dm, INFINITY);
        dm = wave_max_f(dm);
        if (T.set != cur) {
            if (lane == 0 && cur >= 0 && run > 0.f) atomicMax(&stepmax[cur], __float_as_uint(run));
            cur = T.set;
            run = 0.f;
        }
        run = fmaxf(run, dm);
    }
    __shared__ int s_set[4];
    __shared__ float s_max[4];
    if (lane == 0) {
        s_set[w] = cur;
        s_max[w] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int a = 0; a < 4; ++a) {
            if (s_set[a] < 0) continue;
            float v = s_max[a];
            for (int b = a + 1; b < 4; ++b)
                if (s_set[b] == s_set[a]) {
                    v = fmaxf(v, s_max[b]);
                    s_set[b] = -1;
                }
            if (v > 0.f) atomicMax(&stepmax[s_set[a]], __float_as_uint(v));
        }
    }
}

__global__ void k_drift_add(SetInfo* sets, int nsets, const unsigned* __restrict__ stepmax) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsets) return;
    // rounded up: the sum stays a bound on the displacement since the build
    const float a = sets[s].drift, b = __uint_as_float(stepmax[s]);
    float t = a + b;
    if ((double)t < (double)a + (double)b) t = nextafterf(t, INFINITY);
    sets[s].drift = t;
}

// Block summaries of the particle array in cell order (blocks of BLK_PART
// particles at aligned indices): a bit per top cell's first particle, then
// per block the bounding box of its positions.  The cells nest in this
// order, so a block covers a small region, and a chunk reading a large cell
// in this order can pass over the blocks that lie beyond its reach without
// loading them.  A block that holds particles of two top cells (offsets from
// different origins) gets the whole space as its box and is never passed
// over.
constexpr int BLK_PART = 64;
__global__ void k_top_starts(const Cell* __restrict__ cells, int64_t nc, unsigned long long* __restrict__ bits) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const Cell C = cells[c];
    if (C.parent >= 0 || C.count == 0) return;
    atomicOr(&bits[C.first / BLK_PART], 1ull << (C.first % BLK_PART));
}

// One wavefront per block.
__global__ __launch_bounds__(256) void k_block_box(const float4* __restrict__ pos, int64_t n,
                                                   const unsigned long long* __restrict__ bits, int64_t nblk,
                                                   float4* __restrict__ box) {
    const int lane = threadIdx.x & 63;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nblk; b += (int64_t)gridDim.x * 4) {
        const int64_t e = b * BLK_PART + lane;
        const bool in = e < n;
        const float4 p = in ? pos[e] : make_float4(0.f, 0.f, 0.f, 0.f);
        float v[6] = {in ? -p.x : -INFINITY, in ? -p.y : -INFINITY, in ? -p.z : -INFINITY,
                      in ? p.x : -INFINITY, in ? p.y : -INFINITY, in ? p.z : -INFINITY};
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = wave_max_f(v[k]);
        if (lane == 0) {
            const bool mixed = (bits[b] & ~1ull) != 0ull;
            const float big = 3.0e38f;
            box[2 * b] = mixed ? make_float4(-big, -big, -big, 0.f) : make_float4(-v[0], -v[1], -v[2], 0.f);
            box[2 * b + 1] = mixed ? make_float4(big, big, big, 0.f) : make_float4(v[3], v[4], v[5], 0.f);
        }
    }
}

// Sorted lists: each entry's copy of its particle's record, in place (the
// order of the list is the one of the build).
__global__ void k_seg_refresh(const uint32_t* __restrict__ segidx, int64_t ne, const uint32_t* __restrict__ ne_dev,
                              const float4* __restrict__ pos, float4* __restrict__ segpos) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne || (ne_dev && e >= (int64_t)*ne_dev)) return;
    segpos[e] = pos[segidx[e]];
}

// ---------------------------------------------------------------------------
// Per-cell interaction lists: each pair task (A,B,o) gives A the source
// (B, o) and B the source (A, -o).  Keys sort by (target, source, code).
// ---------------------------------------------------------------------------

__global__ void k_csr_keys(const int4* __restrict__ tasks, int64_t nt, uint64_t* __restrict__ keys) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int4 T = tasks[t];
    if (T.x == T.y) {
        keys[2 * t] = ~0ull;
        keys[2 * t + 1] = ~0ull;
    } else {
        keys[2 * t] = ((uint64_t)T.x << CSR_TGT_SHIFT) | ((uint64_t)T.y << CSR_SRC_SHIFT) | (uint64_t)T.z;
        keys[2 * t + 1] = ((uint64_t)T.y << CSR_TGT_SHIFT) | ((uint64_t)T.x << CSR_SRC_SHIFT) |
                          (uint64_t)(26 - T.z);
    }
}

// CSR offsets from the sorted keys: off[c] = first entry with target >= c.
// The self entries (all ones, sorted last) count as target nc, so off[nc]
// is the number of pair entries.
__global__ void k_csr_offsets(const uint64_t* __restrict__ keys, int64_t ne, int64_t nc, uint32_t* __restrict__ off) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int64_t t = min((int64_t)(keys[e] >> CSR_TGT_SHIFT), nc);
    int64_t tp = e == 0 ? -1 : min((int64_t)(keys[e - 1] >> CSR_TGT_SHIFT), nc);
    for (int64_t c = tp + 1; c <= t; ++c) off[c] = (uint32_t)e;
    if (e == ne - 1)
        for (int64_t c = t + 1; c <= nc; ++c) off[c] = (uint32_t)ne;
}

// ---------------------------------------------------------------------------
// Sorted lists per (cell, axis).
// ---------------------------------------------------------------------------
// Partners of more than max_sorted particles are read in cell order by the
// interaction kernels and get no sorted list.
__global__ void k_seg_need(const uint64_t* __restrict__ ent, int64_t ne, const uint32_t* __restrict__ ne_dev,
                           const Cell* __restrict__ cells, int max_sorted, uint32_t* __restrict__ need) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne || (ne_dev && e >= (int64_t)*ne_dev)) return;
    uint64_t k = ent[e];
    if (k == ~0ull) return;   // self entry
    int src = (int)((k >> CSR_SRC_SHIFT) & 0xFFFFFFFFull);
    if (cells[src].count > max_sorted) return;
    int sg;
    int ax = axis_of((int)(k & 31), &sg);
    need[(int64_t)src * NAXES + ax] = 1u;
}

// Long lists up to this length are sorted in LDS by one block each; longer
// ones by the global radix sort.

// Per (cell, axis) list: its length where some pair entry needs it (0
// elsewhere), and its sort class: 65..SEG_LDS_MAX entries (a wave or a block
// sorts it in LDS) or longer (the long class: in LDS up to SEG_LARGE_MAX,
// else one global radix sort over all such lists).
// The total length is also summed in 64 bits (total64, zero on entry; one
// atomic per block): list positions are 32-bit, so the host refuses a tree
// whose lists hold 2^32 entries or more.
__global__ __launch_bounds__(256) void k_seg_lens(const uint32_t* __restrict__ need, int64_t nca,
                                                  const Cell* __restrict__ cells, uint32_t* __restrict__ lens,
                                                  uint32_t* __restrict__ mid, uint32_t* __restrict__ big,
                                                  unsigned long long* __restrict__ total64) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t n = 0;
    if (q < nca) {
        n = need[q] ? (uint32_t)cells[q / NAXES].count : 0u;
        lens[q] = n;
        if (mid) {   // null when no list can exceed 64 entries
            mid[q] = (n > 64u && n <= (uint32_t)SEG_LDS_MAX) ? 1u : 0u;
            big[q] = n > (uint32_t)SEG_LDS_MAX ? 1u : 0u;
        }
    }
    unsigned long long v = n;
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __shared__ unsigned long long s_v[4];
    if ((threadIdx.x & 63) == 0) s_v[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        v = s_v[0] + s_v[1] + s_v[2] + s_v[3];
        if (v) atomicAdd(total64, v);
    }
}

__global__ void k_copy_u32(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int n) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = src[threadIdx.x];
}

// After the scans: lists nobody needs get offset ~0; the mid-size and long
// lists are listed by (cell, axis) index.
__global__ void k_seg_post(const uint32_t* __restrict__ need, int64_t nca, const Cell* __restrict__ cells,
                           uint32_t* __restrict__ segoff, const uint32_t* __restrict__ mid_idx,
                           const uint32_t* __restrict__ big_idx, uint32_t* __restrict__ mids,
                           uint32_t* __restrict__ big, uint32_t* __restrict__ blen) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nca) return;
    if (!need[q]) {
        segoff[q] = 0xFFFFFFFFu;
        return;
    }
    if (!mids) return;   // no list exceeds 64 entries
    const uint32_t n = (uint32_t)cells[q / NAXES].count;
    if (n > 64u && n <= (uint32_t)SEG_LDS_MAX) {
        mids[mid_idx[q]] = (uint32_t)q;
    } else if (n > (uint32_t)SEG_LDS_MAX) {
        big[big_idx[q]] = (uint32_t)q;
        blen[big_idx[q]] = n > (uint32_t)SEG_LARGE_MAX ? n : 0u;   // entries of the radix sort
    }
}

__device__ inline float project(const float4& p, int ax) {
    int c = axis_code(ax);
    int dx = ocx(c), dy = ocy(c), dz = ocz(c);
    float r = (float)dx * p.x;
    r = r + (float)dy * p.y;
    r = r + (float)dz * p.z;
    return r;
}

__device__ inline float ord2f(uint32_t u) {
    uint32_t b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    return __uint_as_float(b);
}

// Sorted lists are split into a small-h part (h <= edge/8 at sort time)
// and a large-h part, each ordered by projection, so that a force sweep can
// bound its reach by the largest h of each part separately.
__device__ inline float small_h_limit(const SetInfo* sets, const Cell& C) {
    return (float)(sets[C.set].L0 / (double)(1 << C.level) / (double)SMALL_H_DIV);
}

__global__ __launch_bounds__(256) void k_cell_nsmall(const SetInfo* sets, Cell* __restrict__ cells, int64_t nc,
                                                     const float* __restrict__ ph) {
    int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nc) return;
    const int lane = threadIdx.x & 63;
    const Cell C = cells[c];
    const float lim = small_h_limit(sets, C);
    int k = 0;
#pragma unroll 8
    for (int p = C.first + lane; p < C.first + C.count; p += 64) k += ph[p] <= lim ? 1 : 0;
    k = wave_sum_i(k);
    if (lane == 0) cells[c].nsmall = k;
}

__device__ inline uint64_t seg_key(float proj, int cls, uint32_t e) {
    return ((uint64_t)cls << 63) | ((uint64_t)(f2ord(proj) >> 1) << 32) | e;
}

// Cells of at most 64 particles: one wavefront per cell sorts every list
// the cell needs (axes whose offset is set), loading the particles once.
// Lists of at most 32 entries go two at a time, one per half-wave.  Each
// lane holds one entry, key (class, ordered projection, local index) --
// unique within a list -- and counts the keys of its list below its own:
// that count is its place in the sorted list.
__global__ __launch_bounds__(256) void k_seg_sort_cell(int64_t nc, const SetInfo* sets,
                                                       const Cell* __restrict__ cells,
                                                       const uint32_t* __restrict__ segoff,
                                                       const float4* __restrict__ pos, const float* __restrict__ ph,
                                                       float4* __restrict__ sproj, uint32_t* __restrict__ sidx) {
    __shared__ __align__(16) uint64_t s_key[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t c = (int64_t)blockIdx.x * 4 + w; c < nc; c += (int64_t)gridDim.x * 4) {
        const Cell C = cells[c];
        const int n = __builtin_amdgcn_readfirstlane(C.count);
        if (n == 0 || n > 64) continue;
        const uint32_t so_l = lane < NAXES ? segoff[c * NAXES + lane] : 0xFFFFFFFFu;
        uint64_t need = __ballot(so_l != 0xFFFFFFFFu);
        if (need == 0) continue;
        const bool two = n <= 32;
        const bool upper = two && lane >= 32;
        const int e = two ? (lane & 31) : lane;
        const bool valid = e < n;
        const float4 rec = valid ? pos[C.first + e] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float lim = small_h_limit(sets, C);
        const int cls = (valid && ph[C.first + e] > lim) ? 1 : 0;
        while (need != 0) {
            const int a0 = __builtin_ctzll(need);
            need &= need - 1ull;
            int a1 = -1;
            if (two && need != 0) {
                a1 = __builtin_ctzll(need);
                need &= need - 1ull;
            }
            const int ax = upper ? a1 : a0;
            const bool act = valid && ax >= 0;
            const uint64_t k = act ? seg_key(project(rec, ax), cls, (uint32_t)e) : ~0ull;
            s_key[w][lane] = k;
            wave_lds_sync();
            // rank: keys of the list below this one (two keys per LDS read,
            // several reads in flight; the keys past n are ~0)
            const int first = upper ? 32 : 0;
            const ulonglong2* kp = (const ulonglong2*)&s_key[w][first];
            int rank = 0;
#pragma unroll 4
            for (int t = 0; t < (n + 1) >> 1; ++t) {
                const ulonglong2 kk = kp[t];
                rank += (kk.x < k ? 1 : 0) + (kk.y < k ? 1 : 0);
            }
            const uint32_t o0 = (uint32_t)__builtin_amdgcn_readlane((int)so_l, a0);
            const uint32_t o1 = a1 >= 0 ? (uint32_t)__builtin_amdgcn_readlane((int)so_l, a1) : 0u;
            if (act) {
                const uint32_t o = (upper ? o1 : o0) + (uint32_t)rank;
                sproj[o] = rec;
                sidx[o] = (uint32_t)(C.first + e);
            }
            wave_lds_sync();
        }
    }
}

// Segments of 65..SEG_LDS_MAX entries (their (cell, axis) indices listed in
// sel), sorted in LDS.  A block takes four lists at a time: each list of at
// most WAVE_SORT_MAX entries is sorted by one wavefront on its own
// (wave-level synchronisation only), the longer ones by the whole block.
// Lists of up to BITONIC_MAX entries take a bitonic network in LDS; longer
// ones a merge sort (runs of 16 sorted in registers, then merged pairwise
// through LDS), which moves each key through LDS once per doubling instead
// of once per bitonic stage.
constexpr int WAVE_SORT_MAX = 1024;
constexpr int BITONIC_MAX = 256;
constexpr int MS_RUN = 16;
static_assert(4 * WAVE_SORT_MAX <= SEG_LDS_MAX, "wave sorts share the block's array");
static_assert(SEG_LDS_MAX <= 256 * MS_RUN, "the block's threads hold the whole list in runs");

template <int NT>
__device__ __forceinline__ void group_sync() {
    if (NT == 64) wave_lds_sync();
    else __syncthreads();
}

template <int NT>
__device__ __forceinline__ void bitonic_lds(uint64_t* s, int P, int t) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = t; e < P / 2; e += NT) {
                const int i = 2 * e - (e & (stride - 1));
                const int j = i + stride;
                const bool up = ((i & size) == 0);
                const uint64_t a = s[i], b = s[j];
                if ((a > b) == up) {
                    s[i] = b;
                    s[j] = a;
                }
            }
            group_sync<NT>();
        }
    }
}

__device__ __forceinline__ void cmp_swap(uint64_t& x, uint64_t& y) {
    const uint64_t a = x, b = y;
    const bool sw = b < a;
    x = sw ? b : a;
    y = sw ? a : b;
}

// ascending sort of 16 keys held in registers (bitonic network, fixed indices)
__device__ __forceinline__ void sort_run(uint64_t (&r)[MS_RUN]) {
#pragma unroll
    for (int lg = 1; lg <= 4; ++lg) {
#pragma unroll
        for (int ls = lg - 1; ls >= 0; --ls) {
#pragma unroll
            for (int i = 0; i < MS_RUN; ++i) {
                const int j = i ^ (1 << ls);
                if (j > i) {
                    if ((i & (1 << lg)) == 0) cmp_swap(r[i], r[j]);
                    else cmp_swap(r[j], r[i]);
                }
            }
        }
    }
}

// Merge sort of the P keys in s (P a power of two, 2 * MS_RUN <= P <=
// NT * MS_RUN) by the NT threads of a wave (NT = 64) or block (NT = 256);
// thread t owns output positions [16 t, 16 t + 16).  Each round merges
// pairs of sorted runs of length L: a thread finds where its 16 outputs
// start on the merge path of its pair (binary search), merges them into
// registers, and all write back after a barrier.  Keys are compared as
// unsigned integers; equal keys (the padding) take the first run first.
template <int NT>
__device__ __forceinline__ void merge_sort_lds(uint64_t* s, int P, int t) {
    const bool on = t * MS_RUN < P;
    uint64_t r[MS_RUN];
    if (on) {
#pragma unroll
        for (int k = 0; k < MS_RUN; ++k) r[k] = s[t * MS_RUN + k];
        sort_run(r);
#pragma unroll
        for (int k = 0; k < MS_RUN; ++k) s[t * MS_RUN + k] = r[k];
    }
    group_sync<NT>();
    for (int L = MS_RUN; L < P; L <<= 1) {
        if (on) {
            const int d = (t * MS_RUN) & (2 * L - 1);   // position in the merged pair
            const uint64_t* A = s + (t * MS_RUN - d);
            const uint64_t* B = A + L;
            int lo = d > L ? d - L : 0, hi = d < L ? d : L;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (!(B[d - 1 - mid] < A[mid])) lo = mid + 1;
                else hi = mid;
            }
            int i = lo, j = d - lo;
            uint64_t a = i < L ? A[i] : 0ull, b = j < L ? B[j] : 0ull;
            // one LDS read per output: the successor of the key taken
#pragma unroll
            for (int k = 0; k < MS_RUN; ++k) {
                const bool ta = i < L && (j >= L || !(b < a));
                r[k] = ta ? a : b;
                i += ta ? 1 : 0;
                j += ta ? 0 : 1;
                const int q = ta ? i : j;
                const uint64_t v = q < L ? (ta ? A : B)[q] : 0ull;
                a = ta ? v : a;
                b = ta ? b : v;
            }
        }
        group_sync<NT>();
        if (on) {
#pragma unroll
            for (int k = 0; k < MS_RUN; ++k) s[t * MS_RUN + k] = r[k];
        }
        group_sync<NT>();
    }
}

__global__ __launch_bounds__(256) void k_seg_sort_lds(const uint32_t* __restrict__ sel, int64_t nsel,
                                                      const uint32_t* __restrict__ off, const SetInfo* sets,
                                                      const Cell* __restrict__ cells,
                                                      const float4* __restrict__ pos, const float* __restrict__ ph,
                                                      float4* __restrict__ sproj, uint32_t* __restrict__ sidx) {
    __shared__ uint64_t s[SEG_LDS_MAX];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t g0 = (int64_t)blockIdx.x * 4; g0 < nsel; g0 += (int64_t)gridDim.x * 4) {
        // short lists: one per wave
        if (g0 + w < nsel) {
            const uint32_t ca = sel[g0 + w];
            const Cell C = cells[ca / NAXES];
            const int ax = (int)(ca % NAXES);
            const int n = __builtin_amdgcn_readfirstlane(C.count);
            if (n > 64 && n <= WAVE_SORT_MAX) {
                uint64_t* sw = s + w * WAVE_SORT_MAX;
                int P = 1;
                while (P < n) P <<= 1;
                const float lim = small_h_limit(sets, C);
                for (int e = lane; e < P; e += 64) {
                    uint64_t k = ~0ull;
                    if (e < n) k = seg_key(project(pos[C.first + e], ax), ph[C.first + e] > lim ? 1 : 0, (uint32_t)e);
                    sw[e] = k;
                }
                wave_lds_sync();
                if (P <= BITONIC_MAX) bitonic_lds<64>(sw, P, lane);
                else merge_sort_lds<64>(sw, P, lane);
                const uint32_t o = off[ca];
                for (int e = lane; e < n; e += 64) {
                    const uint64_t k = sw[e];
                    const uint32_t j = (uint32_t)C.first + (uint32_t)(k & 0xFFFFFFFFu);
                    sproj[o + e] = pos[j];
                    sidx[o + e] = j;
                }
            }
        }
        __syncthreads();
        // longer lists: the whole block, one after the other
        for (int k4 = 0; k4 < 4 && g0 + k4 < nsel; ++k4) {
            const uint32_t ca = sel[g0 + k4];
            const Cell C = cells[ca / NAXES];
            const int ax = (int)(ca % NAXES);
            const int n = C.count;
            if (n <= WAVE_SORT_MAX || n > SEG_LDS_MAX) continue;
            int P = 1;
            while (P < n) P <<= 1;
            const float lim = small_h_limit(sets, C);
            for (int e = threadIdx.x; e < P; e += blockDim.x) {
                uint64_t k = ~0ull;
                if (e < n) k = seg_key(project(pos[C.first + e], ax), ph[C.first + e] > lim ? 1 : 0, (uint32_t)e);
                s[e] = k;
            }
            __syncthreads();
            merge_sort_lds<256>(s, P, threadIdx.x);
            const uint32_t o = off[ca];
            for (int e = threadIdx.x; e < n; e += blockDim.x) {
                const uint64_t k = s[e];
                const uint32_t j = (uint32_t)C.first + (uint32_t)(k & 0xFFFFFFFFu);
                sproj[o + e] = pos[j];
                sidx[o + e] = j;
            }
            __syncthreads();
        }
    }
}

// Lists of SEG_LDS_MAX+1 .. SEG_LARGE_MAX entries (the long class, listed in
// big): one block of LARGE_BS threads per list, the merge sort in 128 KB of
// LDS.  Longer lists are left to the global radix sort.
constexpr int LARGE_BS = 1024;
static_assert(SEG_LARGE_MAX <= LARGE_BS * MS_RUN, "the block's threads hold the whole list in runs");
__global__ __launch_bounds__(LARGE_BS) void k_seg_sort_large(const uint32_t* __restrict__ big,
                                                             const uint32_t* __restrict__ off, const SetInfo* sets,
                                                             const Cell* __restrict__ cells,
                                                             const float4* __restrict__ pos,
                                                             const float* __restrict__ ph,
                                                             float4* __restrict__ sproj, uint32_t* __restrict__ sidx) {
    __shared__ uint64_t s[SEG_LARGE_MAX];
    const uint32_t ca = big[blockIdx.x];
    const Cell C = cells[ca / NAXES];
    const int n = C.count;
    if (n <= SEG_LDS_MAX || n > SEG_LARGE_MAX) return;
    const int ax = (int)(ca % NAXES);
    int P = 1;
    while (P < n) P <<= 1;
    const float lim = small_h_limit(sets, C);
    for (int e = threadIdx.x; e < P; e += LARGE_BS) {
        uint64_t k = ~0ull;
        if (e < n) k = seg_key(project(pos[C.first + e], ax), ph[C.first + e] > lim ? 1 : 0, (uint32_t)e);
        s[e] = k;
    }
    __syncthreads();
    merge_sort_lds<LARGE_BS>(s, P, threadIdx.x);
    const uint32_t o = off[ca];
    for (int e = threadIdx.x; e < n; e += LARGE_BS) {
        const uint64_t k = s[e];
        const uint32_t j = (uint32_t)C.first + (uint32_t)(k & 0xFFFFFFFFu);
        sproj[o + e] = pos[j];
        sidx[o + e] = j;
    }
}

__global__ __launch_bounds__(256) void k_big_keys(const uint32_t* __restrict__ big,
                                                  const uint32_t* __restrict__ boff, const SetInfo* sets,
                                                  const Cell* __restrict__ cells, const float4* __restrict__ pos,
                                                  const float* __restrict__ ph,
                                                  uint64_t* __restrict__ key, uint32_t* __restrict__ val) {
    uint32_t r = blockIdx.x;
    uint32_t ca = big[r];
    const Cell C = cells[ca / NAXES];
    if (C.count <= SEG_LARGE_MAX) return;   // sorted in LDS (k_seg_sort_large)
    int ax = (int)(ca % NAXES);
    const float lim = small_h_limit(sets, C);
    uint32_t o = boff[r];
    for (int e = threadIdx.x; e < C.count; e += blockDim.x) {
        const uint64_t cls = ph[C.first + e] > lim ? 1ull : 0ull;
        key[o + e] = ((uint64_t)r << 33) | (cls << 32) | f2ord(project(pos[C.first + e], ax));
        val[o + e] = (uint32_t)C.first + (uint32_t)e;
    }
}

__global__ void k_big_write(const uint64_t* __restrict__ key, const uint32_t* __restrict__ val, int64_t ne,
                            const uint32_t* __restrict__ boff, const uint32_t* __restrict__ big,
                            const uint32_t* __restrict__ off, const float4* __restrict__ pos,
                            float4* __restrict__ sproj,
                            uint32_t* __restrict__ sidx) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ne) return;
    uint64_t k = key[p];
    uint32_t r = (uint32_t)(k >> 33);
    uint32_t local = (uint32_t)p - boff[r];
    uint32_t o = off[big[r]] + local;
    sproj[o] = pos[val[p]];
    sidx[o] = val[p];
}

// ===========================================================================
// Host orchestration
// ===========================================================================
static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

#define HIPTRY(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) return Err{SPH_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define ERRTRY(x)                          \
    do {                                   \
        Err e_ = (x);                      \
        if (e_.st != SPH_OK) return e_;    \
    } while (0)

// Device words read back through the context's pinned buffer: one
// asynchronous copy, one stream synchronisation.
static Err read_back(sph_ctx* ctx, const void* d, size_t bytes, const void** h) {
    if (bytes > sph_ctx::PIN_BYTES) return Err{SPH_E_STATE, "internal: read-back larger than the pinned buffer"};
    HIPTRY(hipMemcpyAsync(ctx->h_pin, d, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPTRY(hipStreamSynchronize(ctx->stream));
    *h = ctx->h_pin;
    return Err{};
}

// Block summaries of the particle array, for a tree whose interaction
// kernels may read partners in cell order (whether one is read so depends
// on that pair entry alone: a tree without them has no partner that would
// qualify).
static Err block_summaries(sph_ctx* ctx, sph_tree* t) {
    hipStream_t st = ctx->stream;
    t->blkbits = nullptr;
    t->blkbox = nullptr;
    t->nblk = 0;
    if (t->n <= 0 || !t->ext()) return Err{};
    const int64_t nb = (t->n + BLK_PART - 1) / BLK_PART;
    void* p;
    ERRTRY(t->alloc(t->b_blk, (sizeof(uint64_t) + 2 * sizeof(float4)) * nb, &p));
    t->blkbox = (float4*)p;
    t->blkbits = (uint64_t*)(t->blkbox + 2 * nb);
    t->nblk = nb;
    HIPTRY(fill_u32((uint32_t*)t->blkbits, 2 * nb, 0u, st));
    hipLaunchKernelGGL(k_top_starts, dim3(nblk(t->ncells, 256)), dim3(256), 0, st, t->cells, t->ncells,
                       (unsigned long long*)t->blkbits);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL(k_block_box, dim3((unsigned)std::min<int64_t>(nblk(nb, 4), 65535)), dim3(256), 0, st, t->pos,
                       t->n, (const unsigned long long*)t->blkbits, nb, t->blkbox);
    HIPTRY(hipGetLastError());
    return Err{};
}

Err build_tree(sph_ctx* ctx, sph_tree* t, const sph_input* in, const sph_params* prm) {
    hipStream_t st = ctx->stream;
    // ---- validate the host description ---------------------------------
    if (!in || !prm) return Err{SPH_E_ARG, "null input or params"};
    if (in->nsets < 1 || in->nsets > MAX_SETS) return Err{SPH_E_ARG, "nsets out of range"};
    if (!in->offsets || !in->box) return Err{SPH_E_ARG, "null offsets or box"};
    if (in->offsets[0] != 0) return Err{SPH_E_ARG, "offsets[0] must be 0"};
    for (int s = 0; s < in->nsets; ++s) {
        if (in->offsets[s + 1] < in->offsets[s]) return Err{SPH_E_ARG, "offsets must be non-decreasing"};
        if (!(in->box[s] > 0.0) || !std::isfinite(in->box[s])) return Err{SPH_E_ARG, "box must be positive"};
    }
    const int64_t n = in->offsets[in->nsets];
    if (n > ((int64_t)1 << 31) - 1) return Err{SPH_E_CAPACITY, "too many particles (limit 2^31-1)"};
    if (n > 0 && (!in->x || !in->y || !in->z || !in->h || !in->m || !in->u || !in->vx || !in->vy || !in->vz))
        return Err{SPH_E_ARG, "null particle array"};
    if (prm->n_split < 1 || !(prm->split_frac >= 0.f && prm->split_frac <= 1.f) || !(prm->h_slack >= 0.f) ||
        prm->max_depth < 0 || prm->max_depth > 16 || prm->top_coarsen < 0 || prm->top_coarsen > 8 ||
        prm->piece_records < -1)
        return Err{SPH_E_ARG, "bad decomposition parameters"};
    t->prm = *prm;
    t->nsets = in->nsets;
    t->n = n;
    t->off.assign(in->offsets, in->offsets + in->nsets + 1);
    t->built = t->sorted = t->have_density = false;
    t->owned = nullptr;   // a halo is set after every build
    t->hash = (prm->flags & SPH_FLAG_PAIR_HASH) != 0;
    ev_mark(ctx, "start");

    // ---- per-set h statistics -> top grids ------------------------------
    const int S = in->nsets;
    float* d_hmax;
    float* d_hmin;
    int* d_bad;
    SetInfo* d_sets;
    ERRTRY(t->alloc(t->b_sets, sizeof(SetInfo) * S, (void**)&d_sets));
    ERRTRY(t->alloc(t->b_counts, 64 * sizeof(uint32_t), (void**)&t->d_counts));
    ERRTRY(t->alloc(t->b_small, 2 * sizeof(float) * S + sizeof(int) * S + 64, (void**)&d_hmax));
    d_hmin = d_hmax + S;
    d_bad = (int*)(d_hmin + S);
    std::vector<SetInfo> sets(S);
    for (int s = 0; s < S; ++s) {
        sets[s].first = in->offsets[s];
        sets[s].count = in->offsets[s + 1] - in->offsets[s];
        sets[s].box = in->box[s];
        sets[s].drift = 0.f;
    }
    HIPTRY(hipMemcpyAsync(d_sets, sets.data(), sizeof(SetInfo) * S, hipMemcpyHostToDevice, st));
    std::vector<float> hmax(S, 0.f), hmin(S, INFINITY);
    std::vector<int> bad(S, 0);
    if (n > 0) {
        HIPTRY(fill_u32((uint32_t*)d_hmax, 3 * (int64_t)S, 0u, st));
        HIPTRY(fill_u32((uint32_t*)d_hmin, S, 0x7F800000u, st));   // +inf
        int64_t maxc = 0;
        for (int s = 0; s < S; ++s) maxc = std::max<int64_t>(maxc, sets[s].count);
        // a few hundred blocks per set at most: their atomics on one word serialise
        unsigned gx = (unsigned)std::min<int64_t>(std::max<int64_t>((maxc + 4095) / 4096, 1), 256);
        hipLaunchKernelGGL(k_set_hstats, dim3(gx, S), dim3(256), 0, st, d_sets, in->h, (int*)d_hmax, (int*)d_hmin,
                           d_bad);
        HIPTRY(hipGetLastError());
        const void* hs;
        ERRTRY(read_back(ctx, d_hmax, 3 * sizeof(float) * S, &hs));
        std::memcpy(hmax.data(), hs, sizeof(float) * S);
        std::memcpy(hmin.data(), (const float*)hs + S, sizeof(float) * S);
        std::memcpy(bad.data(), (const float*)hs + 2 * S, sizeof(int) * S);
    }
    int max_lg = 0;
    int64_t ntop = 0;
    for (int s = 0; s < S; ++s) {
        if (bad[s]) return Err{SPH_E_ARG, "set " + std::to_string(s) + ": h must be finite and > 0"};
        double box = sets[s].box;
        if (sets[s].count > 0 && !((double)hmax[s] < 0.5 * box))
            return Err{SPH_E_ARG, "set " + std::to_string(s) + ": h must be < box/2"};
        // decisions use h*(1+slack), but at most box/2 (two top cells per side)
        double hd = std::min((double)hmax[s] * (1.0 + (double)prm->h_slack), 0.5 * box);
        int lg = 1;
        if (prm->top_grid > 0) {
            int g = prm->top_grid;
            if ((g & (g - 1)) || g < 2) return Err{SPH_E_ARG, "top_grid must be a power of two >= 2"};
            lg = 0;
            while ((1 << lg) < g) ++lg;
            if (box / g < hd) return Err{SPH_E_ARG, "top_grid cells smaller than h"};
        } else if (sets[s].count == 0) {
            lg = 1;
        } else {
            while (lg < KEY_BITS_PER_DIM && box / (double)(1 << (lg + 1)) >= hd && (1 << (3 * (lg + 1))) <= (1 << 21))
                ++lg;
            lg = std::max(1, lg - prm->top_coarsen);
        }
        sets[s].lgG = lg;
        sets[s].L0 = box / (double)(1 << lg);
        // a cell splits only if some particle has a decision h below half
        // its edge: no level below the one whose edge first drops under
        // twice the smallest decision h (plus one) can hold a split cell, so
        // the keys need no finer resolution
        int d = 0;
        if (sets[s].count > 0) {
            const double hdmin = (double)hmin[s] * (1.0 + (double)prm->h_slack);
            d = 1;
            while (d < 30 && sets[s].L0 / (double)(1 << (d - 1)) > 2.0 * hdmin) ++d;
        }
        sets[s].depth = std::min(std::min(prm->max_depth, d), KEY_BITS_PER_DIM - lg);
        sets[s].top_base = (int32_t)ntop;
        ntop += (int64_t)1 << (3 * lg);
        max_lg = std::max(max_lg, lg);
    }
    if (ntop > (int64_t)1 << 26) return Err{SPH_E_CAPACITY, "too many top cells"};
    int depth = 0, bmax = 0;
    for (int s = 0; s < S; ++s) {
        if (sets[s].depth < 0) return Err{SPH_E_CAPACITY, "top grid too fine for the key layout"};
        depth = std::max(depth, sets[s].depth);
        bmax = std::max(bmax, sets[s].lgG + sets[s].depth);
    }
    int setbits = 0;
    while ((1 << setbits) < S) ++setbits;
    if (3 * bmax + setbits > 64) return Err{SPH_E_CAPACITY, "key layout exceeds 64 bits"};
    for (int s = 0; s < S; ++s) sets[s].key_shift = 3 * (bmax - sets[s].lgG - sets[s].depth);
    t->sets = sets;
    t->depth = depth;
    t->key_bits = 3 * bmax + setbits;
    HIPTRY(hipMemcpyAsync(d_sets, sets.data(), sizeof(SetInfo) * S, hipMemcpyHostToDevice, st));
    t->d_sets = d_sets;

    // ---- particles: keys, sort, gather ----------------------------------
    const int64_t nn = std::max<int64_t>(n, 1);
    ERRTRY(t->alloc(t->b_key, sizeof(uint64_t) * nn, (void**)&t->key));
    ERRTRY(t->alloc(t->b_key2, sizeof(uint64_t) * nn, (void**)&t->key2));
    ERRTRY(t->alloc(t->b_val, sizeof(uint32_t) * nn, (void**)&t->val));
    ERRTRY(t->alloc(t->b_val2, sizeof(uint32_t) * nn, (void**)&t->val2));
    ERRTRY(t->alloc(t->b_perm, sizeof(uint32_t) * nn, (void**)&t->perm));
    ERRTRY(t->alloc(t->b_iperm, sizeof(uint32_t) * nn, (void**)&t->iperm));
    ERRTRY(t->alloc(t->b_pos, sizeof(float4) * nn, (void**)&t->pos));
    ERRTRY(t->alloc(t->b_plo, sizeof(float4) * nn, (void**)&t->plo));
    ERRTRY(t->alloc(t->b_pv, sizeof(float4) * nn, (void**)&t->pv));
    ERRTRY(t->alloc(t->b_ph, sizeof(float) * nn, (void**)&t->ph));
    ERRTRY(t->alloc(t->b_hdec, sizeof(float) * nn, (void**)&t->hdec));
    ERRTRY(t->alloc(t->b_pu, sizeof(float) * nn, (void**)&t->pu));
    ERRTRY(t->alloc(t->b_bound, sizeof(float) * nn, (void**)&t->bound));
    ERRTRY(t->alloc(t->b_mix, sizeof(uint64_t) * nn, (void**)&t->mix));
    ERRTRY(t->alloc(t->b_rs, sizeof(uint32_t) * std::max(radix_tmp_words(nn), radix_tmp_words(1 << 20)),
                    (void**)&t->rs_tmp));
    InRec* rec;
    ERRTRY(t->alloc(t->b_inrec, sizeof(InRec) * nn, (void**)&rec));
    if (n > 0) {
        hipLaunchKernelGGL(k_keys, dim3(nblk(n, 256)), dim3(256), 0, st, d_sets, S, n, in->x, in->y, in->z, in->h,
                           in->m, in->u, in->vx, in->vy, in->vz, bmax, t->key2, t->val2, rec);
        HIPTRY(hipGetLastError());
        bool alt = false;
        HIPTRY(radix_sort(t->key2, t->val2, t->key, t->val, n, t->key_bits, t->rs_tmp, st, &alt));
        if (!alt) {   // result is in key2/val2: swap the roles
            std::swap(t->key, t->key2);
            std::swap(t->val, t->val2);
            std::swap(t->b_key, t->b_key2);
            std::swap(t->b_val, t->b_val2);
        }
        hipLaunchKernelGGL(k_gather, dim3(nblk(n, 256)), dim3(256), 0, st, d_sets, S, n, bmax, t->key,
                           t->val, rec, prm->h_slack, t->pos, t->plo, t->ph, t->hdec, t->pu, t->pv, t->perm,
                           t->iperm, t->mix);
        HIPTRY(hipGetLastError());
    }

    // ---- levels: cells and tasks ----------------------------------------
    // capacity estimate; grown on demand
    int64_t cap_cells = ntop + 8 * (n / (prm->n_split + 1) + 1) * (depth + 1) / 2 + 64;
    ERRTRY(t->alloc(t->b_cell, sizeof(Cell) * cap_cells, (void**)&t->cells));
    t->lvl_start.assign(1, 0);
    t->lvl_start.push_back(ntop);
    hipLaunchKernelGGL(k_top_cells, dim3(nblk(ntop, 256)), dim3(256), 0, st, d_sets, S, (int)ntop, bmax, t->key,
                       t->cells);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL(k_cell_stats, dim3(nblk(ntop, 4)), dim3(256), 0, st, d_sets, bmax, 0, (int64_t)0,
                       ntop, t->key, t->hdec, prm->n_split, prm->split_frac, t->cells);
    HIPTRY(hipGetLastError());

    // top-level tasks and the split flags of level 0: one read-back for both
    ERRTRY(t->scratch(ntop + 1));
    ERRTRY(t->alloc(t->b_split, sizeof(uint32_t) * (ntop + 1), (void**)&t->split_idx));
#define total (t->d_total)
    hipLaunchKernelGGL(k_top_task_count, dim3(nblk(ntop, 256)), dim3(256), 0, st, d_sets, (int)ntop, t->cells,
                       t->sc_a);
    HIPTRY(exclusive_scan(t->sc_a, t->sc_b, ntop, t->sc_tmp, total, st));
    hipLaunchKernelGGL(k_split_flags, dim3(nblk(ntop, 256)), dim3(256), 0, st, t->cells, (int64_t)0, ntop,
                       t->split_idx);
    HIPTRY(exclusive_scan(t->split_idx, t->split_idx, ntop, t->sc_tmp, total + 2, st));
    const void* rb;
    ERRTRY(read_back(ctx, total, 3 * sizeof(uint32_t), &rb));
    const uint32_t nt0 = ((const uint32_t*)rb)[0];
    uint32_t nsplit = ((const uint32_t*)rb)[2];   // split cells of the current level
    // no top cell splits: one level, whose interaction lists come straight
    // from the top grid (no task list is made)
    const bool flat = nsplit == 0;
    int64_t ncur = nt0;        // tasks of the current level (in taskA)
    int64_t nfinal = 0;        // final tasks (in finals)
    if (!flat) {
        ERRTRY(t->alloc(t->b_taskA, sizeof(int4) * std::max<int64_t>(nt0, 1), (void**)&t->taskA));
        hipLaunchKernelGGL(k_top_task_emit, dim3(nblk(ntop, 256)), dim3(256), 0, st, d_sets, (int)ntop, t->cells,
                           t->sc_b, t->taskA);
        HIPTRY(hipGetLastError());
        ERRTRY(t->alloc(t->b_final, sizeof(int4) * std::max<int64_t>(nt0, 1), (void**)&t->finals));
    }

    // One read-back per level: the task counts of this level and the split
    // count of the next, whose cells exist before this level's tasks are
    // decided (a task splits into tasks of the children).  A level without
    // split cells ends the loop: its tasks are all final.
    int level = 0;
    if (flat) {
        t->lvl_start.push_back(ntop);
        nfinal = nt0;
    }
    for (; !flat; ++level) {
        const int64_t c0 = t->lvl_start[level], c1 = t->lvl_start[level + 1];
        const int64_t nnext = 8 * (int64_t)nsplit;
        if (c1 + nnext > (int64_t)1 << 27) return Err{SPH_E_CAPACITY, "too many cells (limit 2^27)"};
        if (c1 + nnext > cap_cells) {
            int64_t nc = std::max<int64_t>(c1 + nnext, cap_cells * 3 / 2);
            ERRTRY(t->grow(t->b_cell, sizeof(Cell) * c1, sizeof(Cell) * nc, (void**)&t->cells));
            cap_cells = nc;
        }
        ERRTRY(t->scratch(std::max(nnext, ncur) + 1));
        if (nsplit > 0) {
            hipLaunchKernelGGL(k_make_children, dim3(nblk(c1 - c0, 256)), dim3(256), 0, st, c0, c1, c1,
                               t->split_idx, t->cells);
            HIPTRY(hipGetLastError());
            hipLaunchKernelGGL(k_cell_stats, dim3(nblk(nnext, 4)), dim3(256), 0, st, d_sets, bmax,
                               level + 1, c1, c1 + nnext, t->key, t->hdec, prm->n_split, prm->split_frac,
                               t->cells);
            HIPTRY(hipGetLastError());
            // the children's split flags (the buffer is free once the
            // children exist: a reallocation waits for the device)
            ERRTRY(t->alloc(t->b_split, sizeof(uint32_t) * (nnext + 1), (void**)&t->split_idx));
            hipLaunchKernelGGL(k_split_flags, dim3(nblk(nnext, 256)), dim3(256), 0, st, t->cells, c1, c1 + nnext,
                               t->split_idx);
            HIPTRY(exclusive_scan(t->split_idx, t->split_idx, nnext, t->sc_tmp, total + 2, st));
        }
        t->lvl_start.push_back(c1 + nnext);
        if (ncur == 0 && nsplit == 0) break;
        if (nsplit == 0) {
            // no cell of this level splits: every task of the level is final
            // (only tasks of split cells are replaced), in task order
            if (nfinal == 0) {
                std::swap(t->finals, t->taskA);
                std::swap(t->b_final, t->b_taskA);
            } else {
                ERRTRY(t->grow(t->b_final, sizeof(int4) * nfinal, sizeof(int4) * (nfinal + ncur),
                               (void**)&t->finals));
                HIPTRY(hipMemcpyAsync(t->finals + nfinal, t->taskA, sizeof(int4) * ncur, hipMemcpyDeviceToDevice,
                                      st));
            }
            if (nfinal + ncur > (int64_t)0x7FFFFFFF) return Err{SPH_E_CAPACITY, "too many tasks"};
            nfinal += ncur;
            ncur = 0;
            break;
        }
        if (ncur > 0) {
            hipLaunchKernelGGL(k_task_decide, dim3(nblk(ncur, 256)), dim3(256), 0, st, d_sets, t->taskA, ncur,
                               t->cells, t->sc_a, t->sc_c);
            HIPTRY(hipGetLastError());
            HIPTRY(exclusive_scan(t->sc_a, t->sc_b, ncur, t->sc_tmp, total, st));
            HIPTRY(exclusive_scan(t->sc_c, t->sc_d, ncur, t->sc_tmp, total + 1, st));
        }
        ERRTRY(read_back(ctx, total, 3 * sizeof(uint32_t), &rb));
        const uint32_t nf = ncur > 0 ? ((const uint32_t*)rb)[0] : 0u;
        const uint32_t nc = ncur > 0 ? ((const uint32_t*)rb)[1] : 0u;
        const uint32_t nsplit_next = ((const uint32_t*)rb)[2];
        if (ncur > 0) {
            if (nfinal + nf > (int64_t)0x7FFFFFFF) return Err{SPH_E_CAPACITY, "too many tasks"};
            ERRTRY(t->grow(t->b_final, sizeof(int4) * nfinal, sizeof(int4) * std::max<int64_t>(nfinal + nf, 1),
                           (void**)&t->finals));
            ERRTRY(t->alloc(t->b_taskB, sizeof(int4) * std::max<int64_t>(nc, 1), (void**)&t->taskB));
            hipLaunchKernelGGL(k_task_emit, dim3(nblk(ncur, 256)), dim3(256), 0, st, t->taskA, ncur, t->cells,
                               t->sc_a, t->sc_b, t->sc_c, t->sc_d, t->finals + nfinal, t->taskB);
            HIPTRY(hipGetLastError());
            nfinal += nf;
            std::swap(t->taskA, t->taskB);
            std::swap(t->b_taskA, t->b_taskB);
            ncur = nc;
        }
        nsplit = nsplit_next;
    }
    t->nlevels = level + 1;
    t->ncells = t->lvl_start.back();
    t->ntasks = nfinal;

    // ---- leaves -> chunks; particle h bounds ------------------------------
    // (the chunk and leaf counts are read back once, at the end)
    const int64_t nc = t->ncells;
    ERRTRY(t->scratch(std::max<int64_t>(nc, t->n) + 1));
    HIPTRY(fill_u32((uint32_t*)t->d_maxleaf, 2, 0, st));
    hipLaunchKernelGGL(k_chunk_count, dim3(nblk(nc, 256)), dim3(256), 0, st, t->cells, nc, t->d_maxleaf);
    HIPTRY(fill_u32(t->sc_c, t->n, 0u, st));
    hipLaunchKernelGGL(k_chunk_mark, dim3(nblk(nc, 256)), dim3(256), 0, st, t->cells, nc, t->sc_c);
    HIPTRY(exclusive_scan(t->sc_c, t->sc_d, t->n, t->sc_tmp, total, st));
    // a leaf of k particles gives ceil(k / CHUNK) <= k / CHUNK + 1 chunks
    const int64_t chunk_cap = nc + t->n / CHUNK + 1;
    ERRTRY(t->alloc(t->b_chunk, sizeof(int4) * chunk_cap, (void**)&t->chunks));
    hipLaunchKernelGGL(k_chunk_emit, dim3(nblk(nc, 256)), dim3(256), 0, st, t->cells, nc, t->sc_d, t->chunks);
    HIPTRY(hipGetLastError());
    if (t->n > 0) {
        hipLaunchKernelGGL(k_particle_bound, dim3((unsigned)std::min<int64_t>(nblk(chunk_cap, 4), 8192)), dim3(256),
                           0, st, t->chunks, total, t->cells, d_sets, t->ph, t->bound, nullptr);
        HIPTRY(hipGetLastError());
    }

    // ---- per-cell interaction lists (CSR) --------------------------------
    ERRTRY(t->alloc(t->b_csroff, sizeof(uint32_t) * (nc + 1), (void**)&t->csr_off));
    if (flat) {
        // at most 26 entries per top cell; the count stays on the device
        const int64_t ecap = 26 * ntop;
        ERRTRY(t->alloc(t->b_csr, sizeof(uint64_t) * std::max<int64_t>(ecap, 1), (void**)&t->csr));
        hipLaunchKernelGGL(k_top_csr<true>, dim3(nblk(ntop, 256)), dim3(256), 0, st, d_sets, (int)ntop, t->cells,
                           nullptr, t->sc_a, nullptr);
        HIPTRY(hipGetLastError());
        HIPTRY(exclusive_scan(t->sc_a, t->csr_off, ntop, t->sc_tmp, t->csr_off + ntop, st));
        hipLaunchKernelGGL(k_top_csr<false>, dim3(nblk(ntop, 256)), dim3(256), 0, st, d_sets, (int)ntop, t->cells,
                           t->csr_off, nullptr, t->csr);
        HIPTRY(hipGetLastError());
        t->ncsr = ecap;
        t->ncsr_dev = t->csr_off + ntop;
    } else {
        const int64_t ne = 2 * nfinal;
        ERRTRY(t->alloc(t->b_csr, sizeof(uint64_t) * std::max<int64_t>(ne, 1), (void**)&t->csr));
        ERRTRY(t->alloc(t->b_csr2, sizeof(uint64_t) * std::max<int64_t>(ne, 1), (void**)&t->csr2));
        if (ne > 0) {
            ERRTRY(t->alloc(t->b_rs, sizeof(uint32_t) * std::max(radix_tmp_words(ne), radix_tmp_words(nn)),
                            (void**)&t->rs_tmp));
            hipLaunchKernelGGL(k_csr_keys, dim3(nblk(nfinal, 256)), dim3(256), 0, st, t->finals, nfinal, t->csr);
            HIPTRY(hipGetLastError());
            bool alt = false;
            // stable sort on the target field only: a target's entries keep
            // the order of the task list, which the tree fixes; self tasks
            // (all ones) sort last
            int tbits = 1;
            while (((int64_t)1 << tbits) <= nc) ++tbits;
            HIPTRY(radix_sort(t->csr, nullptr, t->csr2, nullptr, ne, tbits, t->rs_tmp, st, &alt, CSR_TGT_SHIFT));
            if (alt) {
                std::swap(t->csr, t->csr2);
                std::swap(t->b_csr, t->b_csr2);
            }
            hipLaunchKernelGGL(k_csr_offsets, dim3(nblk(ne, 256)), dim3(256), 0, st, t->csr, ne, nc, t->csr_off);
            HIPTRY(hipGetLastError());
        } else {
            HIPTRY(fill_u32(t->csr_off, nc + 1, 0u, st));
        }
        t->ncsr = ne;
        t->ncsr_dev = nullptr;
    }
    // heavy chunks: pieces per chunk, the pieces and heavy chunks in total[18], total[19]
    // (a one-level tree is estimated only once its largest leaf is known
    // to allow a heavy chunk: its partners are leaves, at most 26 of them)
    const int piece_rec = prm->piece_records == 0 ? 16384 : prm->piece_records;
    const bool pieces = piece_rec > 0 && chunk_cap < ((int64_t)1 << 27);
    ERRTRY(t->alloc(t->b_piece, 2 * sizeof(uint32_t) * chunk_cap, (void**)&t->pcount));
    t->poff = t->pcount + chunk_cap;
    HIPTRY(fill_u32(total + 18, 2, 0u, st));
    auto chunk_cost = [&]() -> Err {
        hipLaunchKernelGGL(k_chunk_cost, dim3(nblk(chunk_cap, 4)), dim3(256), 0, st, t->chunks, total, chunk_cap,
                           t->cells, d_sets, t->csr_off, t->csr, (float)piece_rec, t->pcount, t->poff, total + 18);
        HIPTRY(hipGetLastError());
        return Err{};
    };
    const bool cost_now = pieces && t->nlevels > 1;
    if (cost_now) ERRTRY(chunk_cost());
    else HIPTRY(fill_u32(t->pcount, chunk_cap, 0u, st));
    // chunk count (total[0], untouched since its scan), leaves, largest
    // leaf, pieces, heavy chunks
    static_assert(sizeof(int) == sizeof(uint32_t), "layout of the count words");
    ERRTRY(read_back(ctx, total, 20 * sizeof(uint32_t), &rb));
    const uint32_t nchunks = ((const uint32_t*)rb)[0];
    t->nleaves = ((const int*)rb)[16];
    t->max_leaf = ((const int*)rb)[17];
    t->npieces = ((const uint32_t*)rb)[18];
    t->nheavy = ((const uint32_t*)rb)[19];
    t->nchunks = nchunks;
    if ((int64_t)nchunks > chunk_cap) return Err{SPH_E_STATE, "internal: chunk count above its bound"};
    if (pieces && !cost_now && 27 * t->max_leaf >= piece_rec) {
        ERRTRY(chunk_cost());
        ERRTRY(read_back(ctx, total + 18, 2 * sizeof(uint32_t), &rb));
        t->npieces = ((const uint32_t*)rb)[0];
        t->nheavy = ((const uint32_t*)rb)[1];
    }
    // the partial sums take 4 KiB per piece: a tree on which there would be
    // more than one piece per 64 particles (most chunks heavy: leaves far
    // above the split size, or a threshold far below it) is handed out
    // without them, which bounds them by 64 B per particle (16 MiB on sets
    // below 262144 particles)
    if (t->npieces > std::max<int64_t>(t->n / CHUNK, 4096)) {
        HIPTRY(fill_u32(t->pcount, chunk_cap, 0u, st));
        t->npieces = 0;
        t->nheavy = 0;
    }
    t->plist = nullptr;
    t->part = nullptr;
    if (t->npieces > 0) {
        ERRTRY(t->alloc(t->b_plist, sizeof(uint32_t) * t->npieces, (void**)&t->plist));
        ERRTRY(t->alloc(t->b_part, sizeof(double) * PART_WORDS * CHUNK * t->npieces, (void**)&t->part));
        hipLaunchKernelGGL(k_piece_emit, dim3(nblk(nchunks, 256)), dim3(256), 0, st, total, t->pcount, t->poff,
                           t->plist);
        HIPTRY(hipGetLastError());
    }
    // every non-empty leaf holds exactly one final self task
    t->npairs = nfinal - t->nleaves;
    ERRTRY(block_summaries(ctx, t));
    t->built = true;
    ev_mark(ctx, "build");
    return Err{};
}

Err refresh_tree(sph_ctx* ctx, sph_tree* t, const sph_input* in) {
    hipStream_t st = ctx->stream;
    if (!t->built) return Err{SPH_E_STATE, "refresh before build_cells"};
    if (!in) return Err{SPH_E_ARG, "null input"};
    if (in->nsets != t->nsets || !in->offsets || !in->box)
        return Err{SPH_E_ARG, "refresh: the sets differ from the build's"};
    for (int s = 0; s <= t->nsets; ++s)
        if (in->offsets[s] != t->off[s]) return Err{SPH_E_ARG, "refresh: set offsets differ from the build's"};
    for (int s = 0; s < t->nsets; ++s)
        if (in->box[s] != t->sets[s].box) return Err{SPH_E_ARG, "refresh: box differs from the build's"};
    const int64_t n = t->n;
    if (n > 0 && (!in->x || !in->y || !in->z || !in->h || !in->m || !in->u || !in->vx || !in->vy || !in->vz))
        return Err{SPH_E_ARG, "null particle array"};
    ev_mark(ctx, "start");
    t->have_density = t->have_ghost = false;
    if (n == 0) {
        ev_mark(ctx, "refresh");
        return Err{};
    }
    const int S = t->nsets;
    // the small per-set buffer of the build: S step maxima, the violation
    // count, the chunk count
    unsigned* stepmax = (unsigned*)t->b_small.p;
    uint32_t* viol = stepmax + S;
    uint32_t* nchw = viol + 1;
    HIPTRY(fill_u32(stepmax, S + 1, 0u, st));
    HIPTRY(fill_u32(nchw, 1, (uint32_t)t->nchunks, st));
    const unsigned gch = (unsigned)std::min<int64_t>(nblk(t->nchunks, 4), 8192);
    // the caller's data packed in caller order first (one record per
    // particle for the refresh's reads in cell order)
    InRec* rec = (InRec*)t->b_inrec.p;
    if (!rec || t->b_inrec.cap < sizeof(InRec) * (size_t)n) return Err{SPH_E_STATE, "refresh: no build to refresh"};
    hipLaunchKernelGGL(k_pack_inputs, dim3(nblk(n, 256)), dim3(256), 0, st, n, in->x, in->y, in->z, in->h, in->m,
                       in->u, in->vx, in->vy, in->vz, rec);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL(k_refresh, dim3((unsigned)std::min<int64_t>(gch, REFRESH_BLOCKS)), dim3(256), 0, st, t->chunks,
                       nchw, t->cells, t->d_sets, t->perm, rec, t->prm.h_slack, t->pos, t->plo, t->ph, t->hdec, t->pu,
                       t->pv, stepmax);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL(k_drift_add, dim3(nblk(S, 256)), dim3(256), 0, st, t->d_sets, S, stepmax);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL(k_particle_bound, dim3(gch), dim3(256), 0, st, t->chunks, nchw, t->cells, t->d_sets, t->ph,
                       t->bound, viol);
    HIPTRY(hipGetLastError());
    if (t->blkbox) {
        hipLaunchKernelGGL(k_block_box, dim3((unsigned)std::min<int64_t>(nblk(t->nblk, 4), 65535)), dim3(256), 0, st,
                           t->pos, n, (const unsigned long long*)t->blkbits, t->nblk, t->blkbox);
        HIPTRY(hipGetLastError());
    }
    if (t->sorted) {
        const int64_t ne = t->nsegent >= 0 ? t->nsegent : (int64_t)NAXES * n;
        if (ne > 0) {
            hipLaunchKernelGGL(k_seg_refresh, dim3(nblk(ne, 256)), dim3(256), 0, st, t->segidx, ne,
                               t->nsegent >= 0 ? nullptr : t->d_counts, t->pos, t->segpos);
            HIPTRY(hipGetLastError());
        }
    }
    const void* rb;
    ERRTRY(read_back(ctx, viol, sizeof(uint32_t), &rb));
    const uint32_t nv = ((const uint32_t*)rb)[0];
    if (nv > 0) {
        // the tree no longer covers every pair: nothing may run on it
        t->built = t->sorted = false;
        return Err{SPH_E_REBUILD, std::to_string(nv) + " particles have h at or beyond what the cells support after "
                                                        "the displacement since the build: build again"};
    }
    ev_mark(ctx, "refresh");
    return Err{};
}

Err sort_pairs(sph_ctx* ctx, sph_tree* t) {
    hipStream_t st = ctx->stream;
    if (!t->built) return Err{SPH_E_STATE, "sort_pairs before build_cells"};
    ev_mark(ctx, "start");
    const int64_t nc = t->ncells;
    const int64_t nca = nc * NAXES;
    ERRTRY(t->alloc(t->b_segoff, sizeof(uint32_t) * std::max<int64_t>(nca, 1), (void**)&t->segoff));
    ERRTRY(t->scratch(nca + 1));
    // which (cell, axis) lists a pair entry reads; their lengths and sort
    // classes; offsets and class ranks by scans over all (cell, axis)
    // slots.  A tree of one level whose leaves hold at most 64 particles
    // has no list longer than 64 and at most 13 n entries: its lists are
    // placed without reading anything back (the exact entry count is kept
    // on the device for the statistics).  Otherwise one read-back of the
    // entry count and of the two class counts.
    // (and whose 13 n entries cannot reach 2^32: past that the total is read
    // back to be checked)
    const bool flat = t->nlevels == 1 && t->max_leaf <= 64 && (int64_t)NAXES * t->n < ((int64_t)1 << 32);
    // partners longer than a block's LDS sort takes are read in cell order
    // where the kernels can (not with SPH_FLAG_SORTED_ONLY): on a clustered
    // set with h over three decades this halves the sort stage and leaves
    // the interaction passes as they were (from 1024 they slow down)
    t->max_sorted = t->ext() && !(t->prm.flags & SPH_FLAG_SORTED_ONLY) ? SEG_LDS_MAX : INT32_MAX;
    uint32_t* need = t->sc_a;
    uint32_t* mid_idx = t->sc_c;
    uint32_t* big_idx = t->sc_d;
    HIPTRY(fill_u32(need, nca, 0, st));
    unsigned long long* total64 = (unsigned long long*)(t->d_counts + 8);   // 8-byte aligned
    HIPTRY(fill_u32(t->d_counts + 8, 2, 0u, st));
    const int64_t ne = t->ncsr;
    if (ne > 0) {
        hipLaunchKernelGGL(k_seg_need, dim3(nblk(ne, 256)), dim3(256), 0, st, t->csr, ne, t->ncsr_dev, t->cells,
                           t->max_sorted, need);
        HIPTRY(hipGetLastError());
    }
    if (nca > 0) {
        hipLaunchKernelGGL(k_seg_lens, dim3(nblk(nca, 256)), dim3(256), 0, st, need, nca, t->cells, t->segoff,
                           flat ? nullptr : mid_idx, flat ? nullptr : big_idx, total64);
        HIPTRY(hipGetLastError());
    }
    HIPTRY(exclusive_scan(t->segoff, t->segoff, nca, t->sc_tmp, total, st));
    uint32_t nmid = 0, nbig = 0;
    int64_t nent = 0;
    if (flat) {
        hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(64), 0, st, total, t->d_counts, 1);
        HIPTRY(hipGetLastError());
        nent = NAXES * t->n;   // bound
        t->nsegent = -1;       // exact count on the device
    } else {
        HIPTRY(exclusive_scan(mid_idx, mid_idx, nca, t->sc_tmp, total + 1, st));
        HIPTRY(exclusive_scan(big_idx, big_idx, nca, t->sc_tmp, total + 2, st));
        HIPTRY(hipMemcpyAsync(total + 4, total64, sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        const void* rb;
        ERRTRY(read_back(ctx, total, 6 * sizeof(uint32_t), &rb));
        nmid = ((const uint32_t*)rb)[1];
        nbig = ((const uint32_t*)rb)[2];
        uint64_t n64;
        std::memcpy(&n64, (const uint32_t*)rb + 4, sizeof(n64));
        if (n64 >= ((uint64_t)1 << 32))
            return Err{SPH_E_CAPACITY, "sorted lists hold " + std::to_string(n64) +
                                           " entries (32-bit list positions: limit 2^32 - 1)"};
        nent = (int64_t)n64;
        t->nsegent = nent;
    }
    // mid-size list | long list | long lengths
    ERRTRY(t->alloc(t->b_seglist, sizeof(uint32_t) * ((int64_t)nmid + 2 * (int64_t)nbig + 1), (void**)&t->seglist));
    uint32_t* mids = t->seglist;
    uint32_t* big = t->seglist + nmid;
    uint32_t* blen = big + nbig;
    ERRTRY(t->alloc(t->b_segproj, sizeof(float4) * std::max<int64_t>(nent, 1), (void**)&t->segpos));
    ERRTRY(t->alloc(t->b_segidx, sizeof(uint32_t) * std::max<int64_t>(nent, 1), (void**)&t->segidx));
    if (nca > 0) {
        hipLaunchKernelGGL(k_seg_post, dim3(nblk(nca, 256)), dim3(256), 0, st, need, nca, t->cells, t->segoff,
                           mid_idx, big_idx, flat ? nullptr : mids, big, blen);
        HIPTRY(hipGetLastError());
    }
    if (nent > 0) {
        hipLaunchKernelGGL(k_cell_nsmall, dim3(nblk(nc, 4)), dim3(256), 0, st, t->d_sets, t->cells, nc, t->ph);
        hipLaunchKernelGGL(k_seg_sort_cell, dim3((unsigned)std::min<int64_t>((nc + 3) / 4, 16384)), dim3(256), 0,
                           st, nc, t->d_sets, t->cells, t->segoff, t->pos, t->ph, t->segpos, t->segidx);
        HIPTRY(hipGetLastError());
    }
    if (nmid > 0) {
        hipLaunchKernelGGL(k_seg_sort_lds, dim3((unsigned)std::min<uint32_t>((nmid + 3) / 4, 65535)), dim3(256), 0, st, mids,
                           (int64_t)nmid, t->segoff, t->d_sets, t->cells, t->pos, t->ph, t->segpos, t->segidx);
        HIPTRY(hipGetLastError());
    }
    if (nbig > 0) {
        // lists longer than SEG_LDS_MAX: up to SEG_LARGE_MAX entries one
        // block each in LDS, the longer ones one radix sort over all of them
        // (a second read-back, for their total length)
        hipLaunchKernelGGL(k_seg_sort_large, dim3(nbig), dim3(LARGE_BS), 0, st, big, t->segoff, t->d_sets, t->cells,
                           t->pos, t->ph, t->segpos, t->segidx);
        HIPTRY(hipGetLastError());
        const void* rb;
        ERRTRY(t->scratch(std::max<int64_t>(nca, nbig) + 1));
        uint32_t* boff = t->sc_b;
        HIPTRY(exclusive_scan(blen, boff, nbig, t->sc_tmp, total, st));
        ERRTRY(read_back(ctx, total, sizeof(uint32_t), &rb));
        const uint32_t nbe = ((const uint32_t*)rb)[0];
        if (nbe == 0) {
            t->sorted = true;
            ev_mark(ctx, "sort");
            return Err{};
        }
        uint64_t *bk, *bk2;
        uint32_t *bv, *bv2;
        ERRTRY(t->alloc(t->b_bigk, sizeof(uint64_t) * nbe * 2, (void**)&bk));
        ERRTRY(t->alloc(t->b_bigv, sizeof(uint32_t) * nbe * 2, (void**)&bv));
        bk2 = bk + nbe;
        bv2 = bv + nbe;
        ERRTRY(t->alloc(t->b_rs, sizeof(uint32_t) * std::max(radix_tmp_words(nbe), radix_tmp_words(t->n)),
                        (void**)&t->rs_tmp));
        hipLaunchKernelGGL(k_big_keys, dim3(nbig), dim3(256), 0, st, big, boff, t->d_sets, t->cells, t->pos, t->ph,
                           bk, bv);
        HIPTRY(hipGetLastError());
        int rb_bits = 0;
        while ((1u << rb_bits) < nbig) ++rb_bits;
        bool alt = false;
        HIPTRY(radix_sort(bk, bv, bk2, bv2, nbe, 33 + rb_bits, t->rs_tmp, st, &alt));
        if (alt) { bk = bk2; bv = bv2; }
        hipLaunchKernelGGL(k_big_write, dim3(nblk(nbe, 256)), dim3(256), 0, st, bk, bv, (int64_t)nbe, boff, big,
                           t->segoff, t->pos, t->segpos, t->segidx);
        HIPTRY(hipGetLastError());
    }
    HIPTRY(hipGetLastError());
    t->sorted = true;
    ev_mark(ctx, "sort");
    return Err{};
}
#undef total

}  // namespace sph
