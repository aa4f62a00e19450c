// Density and force stages, the h_i Newton iteration, the ghost step and the
// FP64 reductions.
//
// Work decomposition (owner computes, no floating-point atomics): one
// wavefront owns a chunk of at most 64 particles of one leaf cell, one lane
// per particle (2 to 16 lanes per particle for small chunks).  It walks, in
// a fixed order,
//   * the leaf's self task (all particle pairs in the leaf), then
//   * for the leaf and each of its ancestors, that cell's pair tasks
//     (Section II-B lists), sweeping the partner cell's particles in their
//     order along the cell-pair axis (Section II-C): the sweep stops as soon
//     as the next entry is farther along the axis than any lane's cutoff.
// The records met are staged in LDS tiles, tested, and the in-range ones
// evaluated (see the walk below).  Every particle therefore meets each
// in-range partner exactly once per stage, and sums in an order fixed by the
// tree alone.
//
// Precision.  A position is kept as two FP32 numbers, its offset from the
// origin of its top cell rounded to FP32 (pos) and the FP32 rounding of the
// remainder (plo).  A wave evaluates its chunk in one or more frames: a
// frame's origin o lies on a grid of pitch L0 / 2^20 (L0 the top cell edge)
// at the particle with the smallest h still to do, and takes the particles
// within FRAME_K of their own h of o (the smallest-h one always; usually all
// of the chunk).  Lane coordinates and staged partner records are formed as
// (offset + exact shift) + remainder, the shift -- the partner's top cell
// shift minus o -- being a multiple of the grid pitch and exact in FP32.  A
// coordinate therefore carries about one rounding of its own size, and a
// partner within the cutoff of a lane sits within (FRAME_K + 1) cutoffs of
// o: a distance carries ~(1.5 FRAME_K + 1) roundings of the cutoff whatever
// the input positions and however large the leaf (a leaf of a few hundred
// particles may hold a compact clump of particles with h hundreds of times
// below its edge).  The density sums and the
// acceleration are summed in FP32 within one staged tile (at most 64 terms
// per lane) and accumulated across tiles in FP64 (blocked compensated
// summation), so their rounding stays below ~65 units in the last place of
// the sum of magnitudes for any number of neighbours.  du/dt and the error
// scale S are plain FP32 sums (registers: carrying them in FP64 too would
// cost the force kernel a wave per SIMD); the recursive-sum bound keeps them
// within their bars up to ~1600 neighbours.
#include <cmath>
#include <cstring>

#include "sph_impl.h"

namespace sph {

constexpr float C8PI = 2.5464790894703255f;   // 8/pi: cubic-spline normalisation in 3-D
constexpr int BLK = 256;                      // 4 wavefronts per block, each independent

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Number of set bits of m in the lanes below this one (two mbcnt
// instructions; no 64-bit lane mask in registers).
__device__ __forceinline__ int bits_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// Hardware square root and reciprocal (1 ulp): the arguments here are
// normal numbers (r^2 >= 2^-48 for distinct particles), and 1-ulp results
// are far inside the stated tolerances.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Work distribution of the persistent interaction kernels.  The chunk list
// runs through space in Morton order; it is cut into NGRP contiguous ranges,
// one per XCD.  Block b starts on range b mod NGRP (workgroups are handed to
// the XCDs in turn), so the chunks one XCD works on at a time are neighbours
// and share partner data in that XCD's L2; a wave whose range is exhausted
// moves on to the following ranges.  ctr holds NGRP counters (CSTRIDE
// words apart), zero at launch.  In a Newton pass after the first, the
// ranges hold only the chunks that still have active particles: lcount[g *
// CSTRIDE] of them, listed from the start of range g in list (made by
// k_chunk_list), so that a pass in which few particles are left costs a
// few atomics rather than one per chunk.  A wave looking past its own range
// first reads the counter and skips a range already handed out, without an
// atomic.  Which wave takes which chunk changes no result.
constexpr int NGRP = 8;
// the counters sit 128 bytes apart: atomics on one cache line from all XCDs
// serialise
constexpr int CSTRIDE = 32;
__device__ __forceinline__ int next_chunk(int* __restrict__ ctr, int nchunks, const uint32_t* __restrict__ list,
                                          const int* __restrict__ lcount, int home, int& k) {
    const int lane = threadIdx.x & 63;
    while (k < NGRP) {
        const int g = (home + k) & (NGRP - 1);
        const int lo = (int)((int64_t)nchunks * g / NGRP);
        const int hi = (int)((int64_t)nchunks * (g + 1) / NGRP);
        const int cnt = list ? uni(lcount[g * CSTRIDE]) : hi - lo;
        const bool open =
            cnt > 0 && (k == 0 || __hip_atomic_load(&ctr[g * CSTRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < cnt);
        if (open) {
            int item = 0;
            if (lane == 0) item = atomicAdd(&ctr[g * CSTRIDE], 1);
            item = uni(__shfl(item, 0, 64));
            if (item < cnt) return list ? (int)list[lo + item] : lo + item;
        }
        ++k;
    }
    return -1;
}

// Heavy chunks go first: wave w of the grid's W takes pieces w, w + W, ...
// of the piece list before it turns to the chunk ranges (the grid is
// resident at once, so no counter is needed: one atomic on one word from
// every wave at the start would serialise).  Chunks with pieces are skipped
// in the ranges.

// The chunks that still hold particles in Newton state 1 (active), listed
// per work range for the next density pass: one thread per chunk, blocks
// within one range, one atomic per block.  lcount must be zero on entry; the
// order inside a range follows the blocks' atomics and changes no result.
// active is read as 8-byte words: its buffer is 8-byte aligned and padded
// past the last particle.
constexpr int LIST_BS = 256;
__global__ __launch_bounds__(LIST_BS) void k_chunk_list(const int4* __restrict__ chunks, int nchunks, int bpg,
                                                        const uint8_t* __restrict__ active, uint32_t* __restrict__ list,
                                                        int* __restrict__ lcount) {
    const int g = blockIdx.x / bpg, part = blockIdx.x - g * bpg;
    const int lo = (int)((int64_t)nchunks * g / NGRP);
    const int hi = (int)((int64_t)nchunks * (g + 1) / NGRP);
    const int c = lo + part * LIST_BS + (int)threadIdx.x;
    bool on = false;
    if (c < hi) {
        const int4 ch = chunks[c];
        const int64_t a = ch.y, b = (int64_t)ch.y + ch.z;   // particles [a, b)
        const uint64_t* w = reinterpret_cast<const uint64_t*>(active);
        uint64_t any = 0;
        for (int64_t q = a >> 3; q < (b + 7) >> 3; ++q) {
            uint64_t v = w[q];
            // bytes equal to 1 (states are 0, 1, 2)
            v = v & ~(v >> 1) & 0x0101010101010101ull;
            const int64_t first = q << 3;
            if (first < a) v &= ~0ull << (8 * (a - first));
            if (first + 8 > b) v &= ~0ull >> (8 * (first + 8 - b));
            any |= v;
        }
        on = any != 0;
    }
    __shared__ int s_n[LIST_BS / 64];
    __shared__ int s_base;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t bal = __ballot(on);
    if (lane == 0) s_n[wv] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int i = 0; i < LIST_BS / 64; ++i) {
            const int v = s_n[i];
            s_n[i] = tot;
            tot += v;
        }
        s_base = tot ? atomicAdd(&lcount[g * CSTRIDE], tot) : 0;
    }
    __syncthreads();
    if (on) list[lo + s_base + s_n[wv] + bits_below(bal)] = (uint32_t)c;
}

// Staged tiles hold TILE_PAD extra slots of far-away points, so that every
// lane's share of a tile has the same length and the test loops are
// uniform (scalar) loops.
#ifndef SPH_TCAP
#define SPH_TCAP 64
#endif
constexpr int TILE = SPH_TCAP + 16;
constexpr float FAR = 1.0e18f;
__device__ __forceinline__ float unif(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ float wmax(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}

// Largest value over the 64 lanes, returned on every lane: DPP row shifts
// and row broadcasts (no LDS round trips), on floats mapped to integers that
// order like them.
__device__ __forceinline__ int f2key(float v) {
    const int b = __float_as_int(v);
    return b ^ ((b >> 31) & 0x7FFFFFFF);
}
__device__ __forceinline__ float wave_max_dpp(float v) {
    constexpr int ID = (int)0x80000000;
    int x = f2key(v);
    x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x111, 0xF, 0xF, false));   // row_shr:1
    x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x112, 0xF, 0xF, false));   // row_shr:2
    x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x114, 0xF, 0xF, false));   // row_shr:4
    x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x118, 0xF, 0xF, false));   // row_shr:8
    x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x142, 0xA, 0xF, false));   // row_bcast:15
    x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x143, 0xC, 0xF, false));   // row_bcast:31
    const int m = __builtin_amdgcn_readlane(x, 63);
    return __int_as_float(m ^ ((m >> 31) & 0x7FFFFFFF));
}

// Geometry of one pair entry seen from target cell A: shift S added to the
// partner's stored positions, axis, sign, and the partner's projection offset.
struct PairGeo {
    float Sx, Sy, Sz;
    float ddx, ddy, ddz;   // canonical direction (components -1/0/1)
    float dn;              // its length
    float projoff;         // d . S
    int axis, sign;
};

// Canonical axis (0..12) of the offset codes 14..26, 4 bits each; code c and
// 26 - c share an axis, with opposite signs (codes below 13 have the sign -1).
constexpr uint64_t AXIS_OF_CODE = 0x93a506b4c7182ull;

__device__ __forceinline__ PairGeo pair_geo(const Cell& cA, int code, float L0) {
    PairGeo g;
    const int ox = ocx(code), oy = ocy(code), oz = ocz(code);
    const int l = cA.level;
    const int tx = ((cA.ix + ox) >> l) - (cA.ix >> l);
    const int ty = ((cA.iy + oy) >> l) - (cA.iy >> l);
    const int tz = ((cA.iz + oz) >> l) - (cA.iz >> l);
    g.Sx = (float)tx * L0;
    g.Sy = (float)ty * L0;
    g.Sz = (float)tz * L0;
    g.sign = code >= 13 ? 1 : -1;
    const int c2 = code >= 13 ? code : 26 - code;
    g.axis = (int)((AXIS_OF_CODE >> (4 * (c2 - 14))) & 15u);
    g.ddx = (float)(g.sign * ox);
    g.ddy = (float)(g.sign * oy);
    g.ddz = (float)(g.sign * oz);
    const int nz = abs(ox) + abs(oy) + abs(oz);
    g.dn = nz == 1 ? 1.f : (nz == 2 ? 1.41421356f : 1.73205081f);
    float po = g.ddx * g.Sx;
    po = po + g.ddy * g.Sy;
    po = po + g.ddz * g.Sz;
    g.projoff = po;
    return g;
}

// Frames of a chunk (see the header).  A frame takes the particles whose
// coordinates stay within FRAME_K of their own h of its origin; origins lie
// on a grid of pitch L0 / 2^FRAME_LG inside the top cell, so that a top-cell
// shift minus an origin is exact in FP32.
constexpr float FRAME_K = 4.f;
constexpr int FRAME_LG = 20;

// A frame origin: grid indices (wave-uniform integers, kept in scalar
// registers through the walk) and the grid pitch; the origin is k * pitch.
struct Frame {
    int kx, ky, kz;
    float g;
    // the positions' FP32 remainders are added only where the top cell edge
    // exceeds twice the frame's smallest h: elsewhere leaving them out moves
    // a distance by at most 2^-24 sqrt(3) L0 < 2.1e-7 of the cutoff
    bool lo;
    __device__ __forceinline__ float3 o() const { return make_float3((float)kx * g, (float)ky * g, (float)kz * g); }
};

// Coordinates of a particle in the frame with origin o (relative to the top
// cell): one rounding of their own size, then the remainder.
__device__ __forceinline__ float4 in_frame(const float4& x, const float4& lo, const float3& o) {
    return make_float4((x.x - o.x) + lo.x, (x.y - o.y) + lo.y, (x.z - o.z) + lo.z, x.w);
}

// The next frame of a chunk: pend holds the lanes (lane = particle of the
// chunk) still to do, x / lo / h this lane's particle.  Returns the lanes it
// takes (the smallest-h pending one always) and its origin in *f.
__device__ __forceinline__ uint64_t next_frame(uint64_t pend, const float4& x, const float4& lo, float h, float L0,
                                               Frame* f) {
    const int lane = threadIdx.x & 63;
    const bool pd = (pend >> lane) & 1ull;
    const float hm = -wave_max_dpp(pd ? -h : -INFINITY);
    const int lm = __builtin_ctzll(__ballot(pd && h == hm));
    f->g = L0 * (1.f / (float)(1 << FRAME_LG));   // exact: a power-of-two scale
    const float gi = (float)(1 << FRAME_LG) / L0;
    f->kx = __builtin_amdgcn_readlane((int)floorf(x.x * gi), lm);
    f->ky = __builtin_amdgcn_readlane((int)floorf(x.y * gi), lm);
    f->kz = __builtin_amdgcn_readlane((int)floorf(x.z * gi), lm);
    f->lo = L0 > 2.f * hm;
    const float4 c = in_frame(x, lo, f->o());
    const bool ok = pd && fmaxf(fabsf(c.x), fmaxf(fabsf(c.y), fabsf(c.z))) <= FRAME_K * h;
    return (__ballot(ok) | (1ull << lm)) & pend;
}

__device__ __forceinline__ float proj3(float dx, float dy, float dz, float x, float y, float z) {
    float r = dx * x;
    r = r + dy * y;
    r = r + dz * z;
    return r;
}

struct DensArgs {
    const Cell* cells;
    const SetInfo* sets;
    const int4* chunks;
    int nchunks;
    int* counter;
    const float4* pos;
    const float4* plo;
    const float* ph;
    const uint64_t* mix;
    const uint8_t* active;
    const uint8_t* owned;   // null, or 0 for read-only halo particles (never targets)
    const uint32_t* list;   // chunks with active particles (null: all chunks)
    const int* lcount;
    const uint64_t* csr;
    const uint32_t* csr_off;
    const uint32_t* segoff;
    const float4* segpos;
    const uint32_t* segidx;
    const float4* blkbox;   // block boxes of the particle array (null: no cell is read in cell order)
    int cellord;            // long sweeps may read the partner in cell order
    int max_sorted;         // partners of more particles have no sorted lists: always read in cell order
    int skip;               // ... passing over its blocks out of reach (0: test every record, same results)
    const uint32_t* pcount; // heavy chunks: pieces per chunk (0: handed out with the others)
    const uint32_t* plist;  // the pieces (chunk << 5 | piece), handed out first
    int npieces;
    double* part;           // partial sums of the pieces of split chunks
    const int32_t* status;
    float *rho, *drho, *nw, *dnw;
    int32_t* nngb;
    uint64_t* hash;
    unsigned long long* work;   // pair evaluations (sum of the counts written), for the measurement
    int rmax;
};

// Lanes per target particle: small chunks spread each particle over 2 to 16
// lanes, each taking a contiguous share of every staged tile; the shares are
// combined in a fixed order at the end.
// (log2 of the count; rmax is a power of two)
__device__ __forceinline__ int replicas_lg(int cnt, int rmax) {
    const int lg = cnt <= 4 ? 4 : (cnt <= 8 ? 3 : (cnt <= 16 ? 2 : (cnt <= 32 ? 1 : 0)));
    const int lgmax = 31 - __builtin_clz(rmax);
    return lg < lgmax ? lg : lgmax;
}

// Combine the partial sums of the replicas of one particle (lanes that
// differ in the bits above log2(T)); every replica ends with the same value.
// Butterfly over the replica bits (32, 16, ... down to T): a fixed pairing,
// so the result is the same on every replica and from run to run.
__device__ __forceinline__ float comb_f(float v, int R) {
    for (int d = 32, r = R; r > 1; d >>= 1, r >>= 1) v = v + __shfl_xor(v, d, 64);
    return v;
}
__device__ __forceinline__ double comb_d(double v, int R) {
    for (int d = 32, r = R; r > 1; d >>= 1, r >>= 1) v = v + __shfl_xor(v, d, 64);
    return v;
}
// Pair evaluations of a wave step: the counts its lanes write, summed over
// the wave (a wave-uniform value kept in a scalar register) ...
__device__ __forceinline__ int wave_count(int v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return __builtin_amdgcn_readfirstlane(v);
}
// ... and added up once per wave when it leaves the kernel, into one of 8
// counters 128 bytes apart (one same-address atomic per wave step from the
// whole GPU would serialise); the records loaded go to the word after each.
__device__ __forceinline__ void flush_work(unsigned long long* work, unsigned long long v) {
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(work + 16 * (blockIdx.x & 7), v);
}
__device__ __forceinline__ int comb_i(int v, int R) {
    for (int d = 32, r = R; r > 1; d >>= 1, r >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}
__device__ __forceinline__ uint64_t comb_u64(uint64_t v, int R) {
    for (int d = 32, r = R; r > 1; d >>= 1, r >>= 1)
        v += ((uint64_t)__shfl_xor((uint32_t)(v >> 32), d, 64) << 32) | __shfl_xor((uint32_t)v, d, 64);
    return v;
}
__device__ __forceinline__ float comb_max(float v, int R) {
    for (int d = 32, r = R; r > 1; d >>= 1, r >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
    return v;
}

// ---------------------------------------------------------------------------
// Wave-level walk shared by the density and force stages
// ---------------------------------------------------------------------------
// The partner records met along the walk are staged in LDS, TCAP records
// per tile; consecutive sources (the self task, then the pair tasks in turn)
// share a tile, so that a tile mixes records from several neighbouring
// cells.  A full tile is processed in two steps: every lane tests its share
// of the tile against its particle (one bit per record in range), then
// evaluates the set bits.  The wave runs the evaluation as often as its
// busiest lane has bits; mixing sources in one tile evens the lanes' counts
// out (a particle near one face of its cell has many partners in the cell
// beyond that face and few in the opposite one).
constexpr int TCAP = SPH_TCAP;
constexpr int NWORD = TCAP / 32;
static_assert(TCAP % 32 == 0 && TILE - TCAP >= 16, "tile layout");

// Test of a lane's share [j0, j0 + share) of the tile (share <= TCAP; the
// tile is padded past its end): bit k of word w set when record
// j0 + 32 w + k is in range.  SELF: the tile holds a block of the self task,
// and a record at distance zero (the lane's own particle; positions in a
// set are distinct) is not a neighbour.
template <class P, bool SELF>
__device__ __forceinline__ void tile_test(const float4* sp, int j0, int share, const float4& xi, float hi2,
                                          uint32_t (&m)[NWORD]) {
#pragma unroll
    for (int w = 0; w < NWORD; ++w) {
        uint32_t bits = 0;
        // records in descending order, each result shifted in at bit 0 by an
        // add with carry (bits + bits + [in range]: one instruction where a
        // select of a shifted constant takes three), so record k ends at
        // bit k.  In a block of the self task a zero distance (the particle
        // itself) is out: for non-negative floats 0 < r2 < lim is the
        // unsigned compare bits(r2) - 1 < bits(lim) - 1.
        const float4* base = sp + j0 + 32 * w;
        auto test = [&](const float4& q) {
            const float dx = xi.x - q.x, dy = xi.y - q.y, dz = xi.z - q.z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const float lim = P::lim2(hi2, q.w);
            if (SELF) {
                const uint32_t a = __float_as_uint(r2) - 1u, b = __float_as_uint(lim) - 1u;
                asm("v_cmp_lt_u32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc"
                    : "+v"(bits) : "v"(a), "v"(b) : "vcc");
            } else {
                asm("v_cmp_lt_f32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc"
                    : "+v"(bits) : "v"(r2), "v"(lim) : "vcc");
            }
        };
        // wave-uniform trip count, four records loaded ahead of their tests
        int k = uni(min(32, share - 32 * w)) - 1;
        for (; k >= 3; k -= 4) {
            const float4 q0 = base[k], q1 = base[k - 1], q2 = base[k - 2], q3 = base[k - 3];
            test(q0);
            test(q1);
            test(q2);
            test(q3);
        }
        for (; k >= 0; --k) test(base[k]);
        m[w] = bits;
    }
}

// Test and evaluation of the n (1 <= n <= TCAP) records staged in S; self:
// the tile holds a block of the self task (wave-uniform).
template <class P>
__device__ __forceinline__ void process_tile(typename P::Lds& S, int n, int R, int rep, const typename P::Lane& L,
                                             typename P::Acc& acc, bool self) {
    const int lane = threadIdx.x & 63;
    // far-away padding: every share has the same length (R * share - n < 16)
    if (lane < TILE - TCAP) {
        // the constant is made here, not kept live across the walk (the
        // compiler would otherwise hold it in four registers or spill it)
        float far = FAR;
        asm volatile("" : "+v"(far));
        S.p[n + lane] = make_float4(far, far, far, 0.f);
    }
    wave_lds_sync();
    const int share = (n + R - 1) >> (31 - __builtin_clz(R));
    const int j0 = rep * share;
    uint32_t m[NWORD];
    // (an idle lane sits at -FAR: no record is ever within its h)
    const float hi2 = L.h * L.h;
    if (self) tile_test<P, true>(S.p, j0, share, L.x, hi2, m);
    else tile_test<P, false>(S.p, j0, share, L.x, hi2, m);
    // set bits in increasing record order, 64 at a time
#pragma unroll
    for (int w = 0; w < NWORD; ++w) acc.nn += __popc(m[w]);
#pragma unroll
    for (int w = 0; w < NWORD; w += 2) {
        uint64_t mm = (uint64_t)m[w] | (w + 1 < NWORD ? (uint64_t)m[w + 1] << 32 : 0ull);
        while (mm) {
            const int k = __builtin_ctzll(mm);
            mm &= mm - 1ull;
            P::pair(acc, S, j0 + 32 * w + k, L);
        }
    }
    P::fold(acc);
    wave_lds_sync();   // the tile is overwritten next
}

// Sweep descriptors of the pair tasks being walked: for up to DBATCH
// interaction-list entries of one cell at a time, built with one entry per
// lane (all the loads and the geometry of the batch in one round instead of
// a chain of dependent loads and uniform float arithmetic per entry), two
// per entry (small-h and large-h part of the partner's list).  The sweep of
// a part covers the records whose o.(p + S) stays below the sweep limit --
// the largest o.y that a point y within the cutoff of a particle of the
// chunk can have, o the offset direction of the pair, S the shift into the
// target's frame.  The list is sorted along o, so these records form a
// prefix of the part in sweep order; its length is found by bisection, one
// part per lane.  Only parts with records keep a descriptor:
//   q: first list position, part length, sweep direction (+1/-1), 0;
//   f: the shift S and the square of the part's cutoff radius around the
//      chunk's bounding box (with a rounding margin);
//   o: number of records of the parts before (o[nd] = all of them),
// so that the records of all parts of the batch form one sequence that
// the walk loads 64 at a time.
constexpr int DBATCH = 32;
struct SweepTab {
    int4 q[2 * DBATCH];
    float4 f[2 * DBATCH];
    int o[2 * DBATCH + 1];
};

// A part is a sweep of a sorted list (z = +1 ascending, -1 descending, x
// its first list position, y its length) or a read of a partner's particles
// in cell order (z = 0, x its first particle, y its count).
// (a partner is read in cell order from SCAN_MIN swept records ...)
constexpr int SCAN_RATIO = 2;   // ... if it holds at most this many times as many particles

// Builds the descriptors of entries [e0, e0 + n) of cell cA (n <= DBATCH);
// returns their number, *total the number of records they cover,
// *cellorder whether some part is read in cell order.  bx:
// largest o_k x_k over the chunk's particles per axis and sign (bx[0..2] =
// max x, bx[3..5] = -min x); hmax: largest h of the chunk.
template <class P, bool EXT>
__device__ __forceinline__ int build_sweeps(const typename P::Args& a, const Cell& cA, float L0, const Frame& fr,
                                            uint32_t e0, int n, const float (&bx)[6], float hmax, SweepTab& T,
                                            int* total, bool* cellorder) {
    const int lane = threadIdx.x & 63;
    int4 q0 = make_int4(0, 0, 0, 0), q1 = q0;
    float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f), f1 = f0;
    float lim0 = 0.f, lim1 = 0.f;
    int code = 13;
    int bfirst = 0, bcount = 0;
    bool unsorted = false;   // a partner without sorted lists, within reach
    if (lane < n) {
        const uint64_t key = a.csr[e0 + lane];
        const int B = (int)((key >> 5) & 0xFFFFFFFFull);
        code = (int)(key & 31);
        const PairGeo g = pair_geo(cA, code, L0);
        const Cell cB = a.cells[B];
        bfirst = cB.first;
        bcount = cB.count;
        const uint32_t so = a.segoff[(int64_t)B * NAXES + g.axis];
        const int ox = ocx(code), oy = ocy(code), oz = ocz(code);
        // largest o . x over the box (x and the shifted records share the
        // target's frame), plus the cutoff along the axis
        const float tb = (ox > 0 ? bx[0] : (ox < 0 ? bx[3] : 0.f)) + (oy > 0 ? bx[1] : (oy < 0 ? bx[4] : 0.f)) +
                         (oz > 0 ? bx[2] : (oz < 0 ? bx[5] : 0.f));
        const float tiny = 1e-5f * L0;
        q0 = make_int4((int)so, cB.nsmall, g.sign, 0);
        q1 = make_int4((int)so + cB.nsmall, cB.count - cB.nsmall, g.sign, 0);
        const float r0 = fmaf(P::cut(hmax, cB.hcur), 1.000002f, tiny);
        const float r1 = fmaf(P::cut(hmax, cB.hcur_l), 1.000002f, tiny);
        // shift into the frame: top cell shift minus the frame origin (both
        // multiples of the frame grid pitch: exact)
        const float3 oA = fr.o();
        const float Dx = g.Sx - oA.x, Dy = g.Sy - oA.y, Dz = g.Sz - oA.z;
        f0 = make_float4(Dx, Dy, Dz, r0 * r0);
        f1 = make_float4(Dx, Dy, Dz, r1 * r1);
        // after a refresh the partner list is in the order of the build and
        // each entry's projection has moved by at most dn times the set's
        // displacement bound d: every entry within lim lies in the prefix
        // whose entries pass lim + 2 d dn, which the bisection still finds
        const float dr = 2.f * a.sets[cA.set].drift * g.dn;
        lim0 = tb + fmaf(P::cut(hmax, cB.hcur) * g.dn, 1.000002f, tiny) + dr;
        lim1 = tb + fmaf(P::cut(hmax, cB.hcur_l) * g.dn, 1.000002f, tiny) + dr;
        if (EXT && cB.count > a.max_sorted) {
            // a partner without sorted lists: read in cell order unless its
            // cell lies wholly beyond the reach along the pair direction (its
            // corner nearest the chunk, relative to its top cell, is exact)
            const int l = cB.level;
            const float e = ldexpf(L0, -l);
            const float cx = (float)(cB.ix - ((cB.ix >> l) << l)) * e;
            const float cy = (float)(cB.iy - ((cB.iy >> l) << l)) * e;
            const float cz = (float)(cB.iz - ((cB.iz >> l) << l)) * e;
            const float pmin = (ox > 0 ? cx + Dx : (ox < 0 ? -(cx + e + Dx) : 0.f)) +
                               (oy > 0 ? cy + Dy : (oy < 0 ? -(cy + e + Dy) : 0.f)) +
                               (oz > 0 ? cz + Dz : (oz < 0 ? -(cz + e + Dz) : 0.f));
            unsorted = pmin <= fmaxf(lim0, lim1) + tiny;
            q0.y = q1.y = 0;
        }
    }
    // the swept prefix of each part: the first record (in sweep order)
    // beyond the limit, by bisection
    const float fox = (float)ocx(code), foy = (float)ocy(code), foz = (float)ocz(code);
    auto prefix = [&](const int4& q, float lim) {
        int lo = 0, hi = q.y;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const float4 p = a.segpos[(uint32_t)q.x + (uint32_t)(q.z > 0 ? mid : q.y - 1 - mid)];
            const float t = fmaf(fox, p.x + f0.x, fmaf(foy, p.y + f0.y, foz * (p.z + f0.z)));
            if (t <= lim) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    int c0 = prefix(q0, lim0), c1 = prefix(q1, lim1);
    // a partner without sorted lists, or with a long swept prefix that is
    // not much longer than the partner itself, is read in cell order
    // instead, as one part with the larger radius: the blocks of it beyond
    // the chunk's reach are then passed over (skip_blocks)
    const bool scan = EXT && a.cellord && (unsorted || (c0 + c1 >= SCAN_MIN && bcount <= SCAN_RATIO * (c0 + c1)));
    if (scan) {
        q0 = make_int4(bfirst, bcount, 0, 0);
        f0.w = fmaxf(f0.w, f1.w);
        c0 = bcount;
        c1 = 0;
    }
    *cellorder = __ballot(scan) != 0ull;
    const bool ne0 = c0 > 0, ne1 = c1 > 0;
    const uint64_t b0 = __ballot(ne0), b1 = __ballot(ne1);
    const int pos = bits_below(b0) + bits_below(b1);
    // records of the parts before this lane's: inclusive scan of c0 + c1
    int cs = c0 + c1;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(cs, d, 64);
        if (lane >= d) cs += v;
    }
    const int before = cs - c0 - c1;
    if (ne0) {
        T.q[pos] = q0;
        T.f[pos] = f0;
        T.o[pos] = before;
    }
    if (ne1) {
        const int p1 = pos + (ne0 ? 1 : 0);
        T.q[p1] = q1;
        T.f[p1] = f1;
        T.o[p1] = before + c0;
    }
    const int nd = __popcll(b0) + __popcll(b1);
    const int all = __shfl(cs, 63, 64);
    if (lane == 0) T.o[nd] = all;
    wave_lds_sync();
    *total = all;
    return nd;
}

// Parts read in cell order: the records from sequence index g0 on are
// particles in blocks of 64 whose bounding boxes (and, for the force, the
// largest h) are known.  One block per lane is tested against the chunk's
// bounding box with the part's cutoff radius, bounded by the block's largest
// h where the records' own h bound their reach (the test the walk applies
// to each record of such a part, on the block's extremes: a block out of
// reach holds no record within reach, by the monotonicity of the rounded
// arithmetic).  Returns the new g0: past the leading blocks out
// of reach, rounded down to a multiple of 64 records from the old one, so
// that the records are loaded in the same groups of 64 as without the test
// and the staged sequence is bitwise the same.  *hold receives the sequence
// index before which no block needs to be tested again (the end of the run
// of blocks kept from the first kept one).
template <class P>
__device__ __forceinline__ int skip_blocks(const float4* __restrict__ blkbox, const SweepTab& T, int nd, int g0,
                                           float lox, float loy, float loz, const float (&bx)[6], float hmax,
                                           float tiny, int* hold) {
    constexpr int BLK = 64;   // particles per block
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = nd - 1;   // the part holding g0 (wave-uniform)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T.o[mid] <= g0) lo = mid;
        else hi = mid - 1;
    }
    const int pend = T.o[lo + 1];
    const int4 dq = T.q[lo];
    if (dq.z != 0 || pend - g0 < 2 * BLK) {
        *hold = pend;
        return g0;
    }
    const float4 df = T.f[lo];
    const int q0 = dq.x + (g0 - T.o[lo]);      // particle of record g0
    const int b0 = q0 / BLK, blast = (q0 + (pend - g0) - 1) / BLK;
    const int bl = b0 + lane;
    const bool valid = bl <= blast;
    bool keep = false;
    if (valid) {
        const float4 mn = blkbox[2 * bl], mx = blkbox[2 * bl + 1];
        const float gx = fmaxf(fmaxf(lox - (mx.x + df.x), (mn.x + df.x) - bx[0]), 0.f);
        const float gy = fmaxf(fmaxf(loy - (mx.y + df.y), (mn.y + df.y) - bx[1]), 0.f);
        const float gz = fmaxf(fmaxf(loz - (mx.z + df.z), (mn.z + df.z) - bx[2]), 0.f);
        keep = fmaf(gx, gx, fmaf(gy, gy, gz * gz)) <= P::blk_rad2(df.w, mn.w, hmax, tiny);
    }
    const uint64_t vm = __ballot(valid), km = __ballot(keep);
    // sequence index of the first record of block b0 + k (at most the part's end)
    auto first_of = [&](int k) { return min(pend, g0 + (b0 + k) * BLK - q0); };
    const int nv = __popcll(vm);   // the valid lanes are 0 .. nv-1
    int to;
    if (km == 0) {
        to = first_of(nv);
        *hold = to;
    } else {
        // from the first block kept to the first block out of reach after it
        const int f = __builtin_ctzll(km);
        const uint64_t after = vm & ~km & (~0ull << f);
        *hold = first_of(after ? __builtin_ctzll(after) : nv);
        to = f == 0 ? g0 : first_of(f);
    }
    return g0 + ((to - g0) & ~(BLK - 1));
}

// The walk of one chunk, in one frame (origin oA relative to the leaf's top
// cell; the lanes' coordinates are in that frame), or of piece k of P of a
// split chunk (pm = k | P << 5; 1 << 5 for a whole chunk: the piece takes
// the blocks of 64 self-task particles and the groups of 64 swept records
// whose index is k mod P): the leaf's self task, then the pair tasks of the
// leaf and of its ancestors; each pair task sweeps the partner's sorted
// list (small-h part, then large-h part) up to the largest reach of the
// chunk along the pair axis, bounded by the bounding box of its particles
// plus the largest cutoff, or (EXT) reads a dense partner in cell order.
// The swept records of a batch of pair tasks are staged in sequence, each
// step filling the current tile; written as one loop so that the tile
// processing is inlined once.  The records loaded are added to *nread (a
// word of the wave's in LDS, by its first lane).
template <class P, bool EXT>
__device__ __forceinline__ void walk(const typename P::Args& a, typename P::Lds& S, SweepTab& T,
                                    const typename P::Lane& L, typename P::Acc& acc, int leaf, const Frame& fr,
                                    int R, int rep, bool act, int pm, unsigned long long* nread) {
    const int lane = threadIdx.x & 63;
    const Cell C = a.cells[leaf];
    const int cend = C.first + C.count;
    const int pk = pm & 31, pn = pm >> 5;
    int sbase = C.first + 64 * pk;   // next record of the self task
    // bounding box and largest h of the lanes' particles
    float bx[6];
    bx[0] = wave_max_dpp(act ? L.x.x : -INFINITY);
    bx[1] = wave_max_dpp(act ? L.x.y : -INFINITY);
    bx[2] = wave_max_dpp(act ? L.x.z : -INFINITY);
    bx[3] = wave_max_dpp(act ? -L.x.x : -INFINITY);
    bx[4] = wave_max_dpp(act ? -L.x.y : -INFINITY);
    bx[5] = wave_max_dpp(act ? -L.x.z : -INFINITY);
    const float hmax = wave_max_dpp(act ? L.h : 0.f);
    // the cell whose pair tasks are walked and its entries still to load
    int A = leaf;
    Cell cA = C;
    float L0 = (float)a.sets[C.set].L0;
    uint32_t e = a.csr_off[A], e1 = a.csr_off[A + 1];
    int nd = 0, tot = 0, g0 = 0;     // descriptors of the batch, their records, records loaded
    int hold = 0;                    // records before this index need no block test
    int fill = 0;
    bool tself = false;   // the current tile holds records of the self task
    // a record is staged only if it lies within the cutoff of the chunk's
    // bounding box (the sweep bounds the distance along the pair axis only)
    const float lox = -bx[3], loy = -bx[4], loz = -bx[5];
    const float tiny = 1e-5f * L0;
    const float rw = 1.2f * fmaf(hmax, 1.000002f, tiny);
    const float rwide2 = rw * rw;
    const float rs = fmaf(P::cut(hmax, fmaxf(C.hcur, C.hcur_l)), 1.000002f, tiny);
    const float rself2 = rs * rs;
    for (;;) {
        bool done = false, self = false;
        int nuse = 0;
        uint32_t j = 0;                     // the lane's record: particle, position, shift, radius^2
        float4 pj = make_float4(0.f, 0.f, 0.f, 0.f);
        float Sx = 0.f, Sy = 0.f, Sz = 0.f, rad2 = 0.f;
        uint32_t q = 0;                     // where it was read: list position (or particle) and part
        int dl = -1;
        bool co = false;                    // a record of a part read in cell order
        typename P::Pre pre{};
        if (sbase < cend) {
            // a block of the self task
            nuse = min(64, cend - sbase);
            j = (uint32_t)(sbase + lane);
            q = j;
            if (lane < nuse) pj = a.pos[j];
            const float3 oA = fr.o();
            Sx = -oA.x;
            Sy = -oA.y;
            Sz = -oA.z;
            rad2 = rself2;
            self = true;
            sbase += 64 * pn;   // (a piece: the next block of its own)
            if (lane == 0) *nread += (unsigned long long)nuse;
        } else {
            // next batch of entries: of this cell, or of its ancestors
            // (a batch may sweep no records at all)
            for (;;) {
                while (g0 >= tot) {
                    while (e >= e1 && A >= 0) {
                        A = cA.parent;
                        if (A >= 0) {
                            cA = a.cells[A];
                            L0 = (float)a.sets[cA.set].L0;
                            e = a.csr_off[A];
                            e1 = a.csr_off[A + 1];
                        }
                    }
                    if (A < 0) {
                        done = true;
                        break;
                    }
                    const int n = (int)min(e1 - e, (uint32_t)DBATCH);
                    bool co_any;
                    nd = build_sweeps<P, EXT>(a, cA, L0, fr, e, n, bx, hmax, T, &tot, &co_any);
                    e += n;
                    g0 = 0;
                    hold = co_any ? 0 : tot;   // blocks are tested in parts read in cell order only
                }
                if (done) break;
                if (EXT && pn > 1) {
                    // a piece takes the groups of 64 records k, k + P, ...
                    const int r = ((g0 >> 6) - pk) % pn;
                    if (r != 0) g0 += 64 * (pn - (r < 0 ? r + pn : r));
                    if (g0 >= tot) continue;
                }
                if (!EXT || !a.skip || g0 < hold) break;
                // pass over the blocks of a part read in cell order that lie
                // beyond the chunk's reach
                g0 = skip_blocks<P>(a.blkbox, T, nd, g0, lox, loy, loz, bx, hmax, tiny, &hold);
            }
            // the next 64 records of the batch's sequence
            if (!done) nuse = min(64, tot - g0);
            if (lane == 0) *nread += (unsigned long long)nuse;
            if (lane < nuse) {
                const int g = g0 + lane;
                int lo = 0, hi = nd - 1;   // the last part starting at or before g
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (T.o[mid] <= g) lo = mid;
                    else hi = mid - 1;
                }
                const int4 dq = T.q[lo];
                const float4 df = T.f[lo];
                const int k = g - T.o[lo];
                q = (uint32_t)dq.x + (uint32_t)(dq.z >= 0 ? k : dq.y - 1 - k);
                dl = lo;
                if (EXT && dq.z == 0) {
                    pj = a.pos[q];
                    j = q;
                    co = true;
                } else {
                    pj = a.segpos[q];
                    j = a.segidx[q];
                }
                Sx = df.x;
                Sy = df.y;
                Sz = df.z;
                rad2 = df.w;
            }
            g0 += nuse;
        }
        // the records' own data bound their reach where some part reaches
        // more than 20% beyond the chunk's cutoff, and always in parts read
        // in cell order, whose blocks are passed over by the same bound
        // (wave-uniform)
        const bool early = P::kPre && __ballot(lane < nuse && (rad2 > rwide2 || co)) != 0ull;
        if (early) pre = P::pre(a, j, lane < nuse);
        // the records within reach, packed: the first ones complete the
        // current tile, the others start the next
        bool ok = false;
        if (lane < nuse) {
            if (early) rad2 = P::rad2(rad2, pre, hmax, tiny);
            const float px = pj.x + Sx, py = pj.y + Sy, pz = pj.z + Sz;
            const float ex = fmaxf(fmaxf(lox - px, px - bx[0]), 0.f);
            const float ey = fmaxf(fmaxf(loy - py, py - bx[1]), 0.f);
            const float ez = fmaxf(fmaxf(loz - pz, pz - bx[2]), 0.f);
            ok = fmaf(ex, ex, fmaf(ey, ey, ez * ez)) <= rad2;
        }
        const uint64_t okm = __ballot(ok);
        const int m = __popcll(okm);
        const int slot = bits_below(okm);
        const int room = TCAP - fill;
        if (ok && slot < room) P::stage(S, fill + slot, j, pj, Sx, Sy, Sz, a, pre, early, fr.lo);
        const int first = min(m, room);
        fill += first;
        tself = tself || (self && first > 0);
        if (done || fill == TCAP) {
            if (fill > 0) process_tile<P>(S, fill, R, rep, L, acc, tself);
            fill = 0;
            tself = false;
        }
        if (done) break;
        if (ok && slot >= room) {
            // read again rather than kept through the tile's evaluation
            if (dl < 0) {
                const float3 oA = fr.o();
                P::stage(S, slot - room, q, a.pos[q], -oA.x, -oA.y, -oA.z, a, pre, false, fr.lo);
            } else {
                const float4 df = T.f[dl];
                const bool cell_order = EXT && T.q[dl].z == 0;
                const uint32_t jj = cell_order ? q : a.segidx[q];
                const float4 pq = cell_order ? a.pos[q] : a.segpos[q];
                P::stage(S, slot - room, jj, pq, df.x, df.y, df.z, a, pre, false, fr.lo);
            }
        }
        fill += m - first;
        tself = tself || (self && m > first);
    }
}

// ---------------------------------------------------------------------------
// Density stage: rho, drho/dh, N_w, dN_w/dh, neighbour count, pair hash
// ---------------------------------------------------------------------------
template <bool HASH>
struct DensP {
    using Args = DensArgs;
    struct Lane {
        float4 x;   // position, mass
        float h, hinv;
    };
    struct Acc {
        float sf = 0, sg = 0, sw = 0, sq = 0;   // sums of m f, m (3f + q f'), f, q f' over one tile
        double tf = 0, tg = 0, tw = 0, tq = 0;  // the same over the tiles done
        int nn = 0;
        uint64_t hs = 0;
    };
    // a tile's partial sums (at most 64 terms per lane) into the FP64 totals
    static __device__ __forceinline__ void fold(Acc& A) {
        A.tf += (double)A.sf;
        A.tg += (double)A.sg;
        A.tw += (double)A.sw;
        A.tq += (double)A.sq;
        A.sf = A.sg = A.sw = A.sq = 0.f;
    }
    struct Lds {
        float4 p[TILE];     // x, y, z (shifted into the target's frame), m
        uint64_t m[TILE];   // pair-hash terms
    };
    static __device__ __forceinline__ float cut(float hmax, float) { return hmax; }
    // squared cutoff of a pair: the target's h (density gathers over h_i)
    static __device__ __forceinline__ float lim2(float hi2, float) { return hi2; }
    // data of a record read before it is filtered (none: the cutoff is the
    // target's h)
    struct Pre {};
    static constexpr bool kPre = false;
    static __device__ __forceinline__ Pre pre(const Args&, uint32_t, bool) { return Pre{}; }
    static __device__ __forceinline__ float rad2(float part2, const Pre&, float, float) { return part2; }
    static __device__ __forceinline__ float blk_rad2(float part2, float, float, float) { return part2; }
    static __device__ __forceinline__ void stage(Lds& S, int slot, uint32_t j, const float4& pj, float Sx, float Sy,
                                                 float Sz, const Args& a, const Pre&, bool, bool uselo) {
        const float4 lo = uselo ? a.plo[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        S.p[slot] = make_float4((pj.x + Sx) + lo.x, (pj.y + Sy) + lo.y, (pj.z + Sz) + lo.z, pj.w);
        if (HASH) S.m[slot] = a.mix[j];
    }
    static __device__ __forceinline__ void pair(Acc& A, const Lds& S, int j, const Lane& L) {
        const float4 q = S.p[j];
        const float dx = L.x.x - q.x, dy = L.x.y - q.y, dz = L.x.z - q.z;
        const float r = fsqrt(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        const float u = r * L.hinv;
        // the two pieces of the cubic spline without a branch:
        // f = 2 (1-u)^3 - 8 max(0, 1/2-u)^3,  f' = -6 (1-u)^2 + 24 max(0, 1/2-u)^2
        const float t1 = 1.f - u, s1 = fmaxf(0.5f - u, 0.f);
        const float t2 = t1 * t1, s2 = s1 * s1;
        const float f = fmaf(2.f * t2, t1, -8.f * s2 * s1);
        const float df = fmaf(24.f, s2, -6.f * t2);
        const float g = fmaf(u, df, 3.f * f);
        A.sf = fmaf(q.w, f, A.sf);
        A.sg = fmaf(q.w, g, A.sg);
        A.sw += f;
        A.sq = fmaf(u, df, A.sq);
        if (HASH) A.hs += S.m[j];
    }
};

// The outputs of a target from its sums over the partners (the self term
// m_i f(0) added here).
template <bool HASH>
__device__ __forceinline__ void dens_write(const DensArgs& a, int p, float hi, float mi, double sf, double sg,
                                           double sw, double sq, int nn, uint64_t hs) {
    const float hinv = 1.f / hi;
    const float h3 = hi * hi * hi;
    a.rho[p] = C8PI / h3 * (float)((double)mi + sf);
    a.drho[p] = -C8PI / (h3 * hi) * (float)(3.0 * (double)mi + sg);
    a.nw[p] = (32.f / 3.f) * (float)(1.0 + sw);
    a.dnw[p] = -(32.f / 3.f) * hinv * (float)sq;
    a.nngb[p] = nn;
    if (HASH) a.hash[p] = hs;
}

// EXT: the tree may have heavy chunks or partners read in cell order (the
// kernel without that code keeps more registers for the common case).
template <bool SOLVE, bool HASH, bool EXT>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(5))) void k_density(DensArgs a) {
    using P = DensP<HASH>;
    __shared__ typename P::Lds s_l[BLK / 64];
    __shared__ SweepTab s_t[BLK / 64];
    __shared__ int s_pick[BLK / 64][64];
    // the wave's pair evaluations and records loaded (kept in LDS, not in
    // registers through the walk)
    __shared__ unsigned long long s_cnt[BLK / 64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    typename P::Lds& S = s_l[w];
    const int home = blockIdx.x & (NGRP - 1);
    int grp = 0;
    // one step per frame of a chunk: the particles of the chunk that take
    // part -- all, or the still active ones of a Newton pass (state 1; 2 =
    // parked until a rebuild) -- are done frame by frame (pend: those left),
    // each frame's packed into the first slots
    int leaf = 0, p0 = 0, cnt = 0;
    uint64_t pend = 0;
    if (lane == 0) {
        s_cnt[w][0] = 0ull;
        s_cnt[w][1] = 0ull;
    }
    int pnext = uni(blockIdx.x * (BLK / 64) + w);   // this wave's next piece of a heavy chunk
    // the current piece: k | P << 5 (1 << 5: a whole chunk) and its slot (-1:
    // the sums go out directly)
    int pm = 1 << 5, pslot = -1;
    for (;;) {
        if (pend == 0) {
            int item;
            pm = 1 << 5;
            pslot = -1;
            if (EXT && pnext < a.npieces) {
                const uint32_t v = a.plist[pnext];
                item = uni((int)(v >> 5));
                const int pn = uni((int)a.pcount[item]);
                if (pn > 1) {
                    pm = uni((int)(v & 31)) | pn << 5;
                    pslot = pnext;
                }
                pnext += gridDim.x * (BLK / 64);
            } else {
                item = next_chunk(a.counter, a.nchunks, a.list, a.lcount, home, grp);
                if (item < 0) break;
                if (EXT && a.npieces > 0 && a.pcount[item] != 0) continue;   // handed out as pieces
            }
            const int4 ch = a.chunks[item];
            leaf = uni(ch.x);
            p0 = uni(ch.y);
            cnt = uni(ch.z);
            pend = cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
            if (SOLVE) pend = __ballot(lane < cnt && a.active[p0 + lane] == 1);   // (halo: never active)
            else if (a.owned) pend = __ballot(lane < cnt && a.owned[p0 + lane] != 0);
            if (pend == 0) continue;
        }
        const float L0 = (float)a.sets[a.cells[leaf].set].L0;
        Frame fr;
        uint64_t amask;
        {
            // the lane's particle, read again for every frame rather than
            // kept in registers through the walk
            int q = p0 + (lane < cnt ? lane : 0);
            asm volatile("" : "+v"(q));
            amask = next_frame(pend, a.pos[q], a.plo[q], a.ph[q], L0, &fr);
        }
        pend &= ~amask;
        const int nact = __popcll(amask);
        const int lgR = replicas_lg(nact, a.rmax), R = 1 << lgR, T = 64 >> lgR;
        const int slot = lane & (T - 1), rep = lane >> (6 - lgR);
        // slot -> particle: the slot-th set bit of amask
        if ((amask >> lane) & 1ull) s_pick[w][bits_below(amask)] = lane;
        wave_lds_sync();
        const int pick = slot < nact ? s_pick[w][slot] : 0;
        wave_lds_sync();
        const int p = p0 + pick;
        const bool act = slot < nact;
        typename P::Lane L;
        // an idle lane sits far away so no record is ever in its range
        L.x = act ? in_frame(a.pos[p], fr.lo ? a.plo[p] : make_float4(0.f, 0.f, 0.f, 0.f), fr.o())
                  : make_float4(-FAR, -FAR, -FAR, 0.f);
        L.h = act ? a.ph[p] : 1.f;
        L.hinv = 1.f / L.h;
        typename P::Acc acc;
        walk<P, EXT>(a, S, s_t[w], L, acc, leaf, fr, R, rep, act, pm, &s_cnt[w][1]);

        const double sf = comb_d(acc.tf, R), sg = comb_d(acc.tg, R);
        const double sw = comb_d(acc.tw, R), sq = comb_d(acc.tq, R);
        const int nn = comb_i(acc.nn, R);
        const uint64_t hs = HASH ? comb_u64(acc.hs, R) : 0ull;
        if (act && rep == 0) {
            if (EXT && pslot >= 0) {
                double* q = a.part + (size_t)pslot * PART_WORDS * CHUNK + pick;
                q[0 * CHUNK] = sf;
                q[1 * CHUNK] = sg;
                q[2 * CHUNK] = sw;
                q[3 * CHUNK] = sq;
                q[4 * CHUNK] = (double)nn;
                q[5 * CHUNK] = __longlong_as_double((long long)hs);
            } else {
                dens_write<HASH>(a, p, L.h, L.x.w, sf, sg, sw, sq, nn, hs);
            }
        }
        const int npair = wave_count(act && rep == 0 ? nn : 0);
        if (lane == 0) s_cnt[w][0] += (unsigned long long)npair;
    }
    if (lane == 0) {
        flush_work(a.work, s_cnt[w][0]);
        flush_work(a.work + 1, s_cnt[w][1]);
    }
}

// Split chunks: the partial sums of the pieces, added in piece order, give
// the outputs of the chunk's particles that took part (one wave per piece
// slot; the slot of piece 0 does the chunk).
template <bool SOLVE, bool HASH>
__global__ __launch_bounds__(256) void k_density_pieces(DensArgs a) {
    const int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= a.npieces) return;
    const uint32_t v = a.plist[i];
    const int c = (int)(v >> 5), pn = (int)a.pcount[c];
    if ((v & 31u) != 0u || pn < 2) return;
    const int4 ch = a.chunks[c];
    if (lane >= ch.z) return;
    const int p = ch.y + lane;
    if (SOLVE ? a.active[p] != 1 : (a.owned && a.owned[p] == 0)) return;
    double sf = 0.0, sg = 0.0, sw = 0.0, sq = 0.0;
    int nn = 0;
    uint64_t hs = 0;
    for (int k = 0; k < pn; ++k) {
        const double* q = a.part + (size_t)(i + k) * PART_WORDS * CHUNK + lane;
        sf += q[0 * CHUNK];
        sg += q[1 * CHUNK];
        sw += q[2 * CHUNK];
        sq += q[3 * CHUNK];
        nn += (int)q[4 * CHUNK];
        hs += (uint64_t)__double_as_longlong(q[5 * CHUNK]);
    }
    dens_write<HASH>(a, p, a.ph[p], a.pos[p].w, sf, sg, sw, sq, nn, hs);
}

// ---------------------------------------------------------------------------
// Force stage
// ---------------------------------------------------------------------------
struct ForceArgs {
    const Cell* cells;
    const SetInfo* sets;
    const int4* chunks;
    int nchunks;
    int* counter;
    const float4* pos;
    const float4* plo;
    const float4* pv;
    const float4* frec;   // h, A, sound speed, K = 8/(pi h^5); pv.w holds rho
    const uint8_t* owned;
    const uint64_t* mix;
    const uint64_t* csr;
    const uint32_t* csr_off;
    const uint32_t* segoff;
    const float4* segpos;
    const uint32_t* segidx;
    const float4* blkbox;   // block boxes of the particle array (null: no cell is read in cell order)
    int cellord;            // long sweeps may read the partner in cell order
    int max_sorted;         // partners of more particles have no sorted lists: always read in cell order
    int skip;               // ... passing over its blocks out of reach (0: test every record, same results)
    const uint32_t* pcount; // heavy chunks: pieces per chunk (0: handed out with the others)
    const uint32_t* plist;  // the pieces (chunk << 5 | piece), handed out first
    int npieces;
    double* part;           // partial sums of the pieces of split chunks
    float alpha;
    float *ax, *ay, *az, *du, *vsig, *S;
    int32_t* nf;
    uint64_t* hash;
    unsigned long long* work;
    int rmax;
};

__device__ __forceinline__ float gradF(float q, float h, float rinv) {
    // f'(q)/q of the cubic spline, zero outside the support
    float t = 1.f - q;
    float outer = q < 1.f ? -6.f * t * t * h * rinv : 0.f;
    return q < 0.5f ? fmaf(18.f, q, -12.f) : outer;
}

template <bool HASH>
struct ForceP {
    using Args = ForceArgs;
    struct Lane {
        float4 x;   // position, mass
        float4 v;   // velocity, rho
        float h, hinv, K, A, c, alpha;
    };
    struct Acc {
        float ax = 0, ay = 0, az = 0, du = 0, vs = 0, S = 0;   // a: over one tile; du, vs, S: over all
        double tx = 0, ty = 0, tz = 0;                         // a over the tiles done
        int nn = 0;
        uint64_t hs = 0;
    };
    static __device__ __forceinline__ void fold(Acc& A) {
        A.tx += (double)A.ax;
        A.ty += (double)A.ay;
        A.tz += (double)A.az;
        A.ax = A.ay = A.az = 0.f;
    }
    struct Lds {
        float4 p[TILE];    // x, y, z (shifted into the target's frame), h
        float4 h[TILE];    // m, 1/h, K = 8/(pi h^5), A
        float4 v[TILE];    // vx, vy, vz, rho
        float c[TILE];     // sound speed
        uint64_t m[TILE];  // pair-hash terms
    };
    static __device__ __forceinline__ float cut(float hmax, float hpart) { return fmaxf(hmax, hpart); }
    // squared cutoff of a pair: max(h_i, h_j)
    static __device__ __forceinline__ float lim2(float hi2, float hj) { return fmaxf(hi2, hj * hj); }
    // where a part's largest h reaches well beyond the chunk's own cutoff,
    // the partner's force record is read before the record is filtered: its
    // own h bounds its reach (the cutoff is max(h_i, h_j))
    struct Pre {
        float4 f;
    };
    static constexpr bool kPre = true;
    static __device__ __forceinline__ Pre pre(const Args& a, uint32_t j, bool valid) {
        Pre p;
        p.f = valid ? a.frec[j] : make_float4(1.f, 0.f, 0.f, 0.f);
        return p;
    }
    static __device__ __forceinline__ float rad2(float part2, const Pre& p, float hmax, float tiny) {
        const float r = fmaf(fmaxf(hmax, p.f.x), 1.000002f, tiny);
        return fminf(part2, r * r);
    }
    // the same for a block of records whose largest h is hb
    static __device__ __forceinline__ float blk_rad2(float part2, float hb, float hmax, float tiny) {
        const float r = fmaf(fmaxf(hmax, hb), 1.000002f, tiny);
        return fminf(part2, r * r);
    }
    static __device__ __forceinline__ void stage(Lds& S, int slot, uint32_t j, const float4& pj, float Sx, float Sy,
                                                 float Sz, const Args& a, const Pre& pr, bool loaded, bool uselo) {
        const float4 fj = loaded ? pr.f : a.frec[j];
        const float4 lo = uselo ? a.plo[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        S.p[slot] = make_float4((pj.x + Sx) + lo.x, (pj.y + Sy) + lo.y, (pj.z + Sz) + lo.z, fj.x);
        S.h[slot] = make_float4(pj.w, frcp(fj.x), fj.w, fj.y);
        S.v[slot] = a.pv[j];
        S.c[slot] = fj.z;
        if (HASH) S.m[slot] = a.mix[j];
    }
    static __device__ __forceinline__ void pair(Acc& A, const Lds& S, int j, const Lane& L) {
        const float4 q = S.p[j];
        const float4 sh = S.h[j];
        const float4 sv = S.v[j];
        const float cj = S.c[j];
        const float dx = L.x.x - q.x, dy = L.x.y - q.y, dz = L.x.z - q.z;
        // 1/r from one reciprocal square root, r = r^2 / r; two distinct
        // particles at one FP32 point (closer than a rounding of their
        // frame) give r = 0 and no vector term instead of a NaN
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float rinv = r2 > 0.f ? frsq(r2) : 0.f;
        const float r = r2 * rinv;
        const float ki = L.K * gradF(r * L.hinv, L.h, rinv);
        const float kj = sh.z * gradF(r * sh.y, q.w, rinv);
        const float vdx = L.v.x - sv.x, vdy = L.v.y - sv.y, vdz = L.v.z - sv.z;
        const float vdotx = fmaf(vdx, dx, fmaf(vdy, dy, vdz * dz));
        // approaching pairs only (w < 0): with w clamped at 0 the term
        // vanishes exactly, without a branch
        const float wn = fminf(vdotx * rinv, 0.f);
        const float vsig = fmaf(-3.f, wn, L.c + cj);
        const float visc = -L.alpha * vsig * wn * frcp(L.v.w + sv.w);
        const float kbar = 0.5f * (ki + kj);
        const float s = fmaf(L.A, ki, fmaf(sh.w, kj, visc * kbar));
        const float mj = sh.x;
        const float ms = mj * s;
        A.ax = fmaf(-ms, dx, A.ax);
        A.ay = fmaf(-ms, dy, A.ay);
        A.az = fmaf(-ms, dz, A.az);
        A.du = fmaf(mj * vdotx, fmaf(L.A, ki, 0.5f * visc * kbar), A.du);
        A.vs = fmaxf(A.vs, vsig);
        A.S = fmaf(fabsf(ms), r, A.S);
        if (HASH) A.hs += S.m[j];
    }
};

template <bool HASH, bool EXT>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(5))) void k_force(ForceArgs a) {
    using P = ForceP<HASH>;
    __shared__ typename P::Lds s_l[BLK / 64];
    __shared__ SweepTab s_t[BLK / 64];
    __shared__ int s_pick[BLK / 64][64];
    // the wave's pair evaluations and records loaded (kept in LDS, not in
    // registers through the walk)
    __shared__ unsigned long long s_cnt[BLK / 64][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    typename P::Lds& S = s_l[w];
    const int home = blockIdx.x & (NGRP - 1);
    int grp = 0;
    // one step per frame of a chunk (pend: the chunk's particles left, each
    // frame's packed into the first slots)
    int leaf = 0, p0 = 0, cnt = 0;
    uint64_t pend = 0;
    if (lane == 0) {
        s_cnt[w][0] = 0ull;
        s_cnt[w][1] = 0ull;
    }
    int pnext = uni(blockIdx.x * (BLK / 64) + w);   // this wave's next piece of a heavy chunk
    // the current piece: k | P << 5 (1 << 5: a whole chunk) and its slot (-1:
    // the sums go out directly)
    int pm = 1 << 5, pslot = -1;
    for (;;) {
        if (pend == 0) {
            int item;
            pm = 1 << 5;
            pslot = -1;
            if (EXT && pnext < a.npieces) {
                const uint32_t v = a.plist[pnext];
                item = uni((int)(v >> 5));
                const int pn = uni((int)a.pcount[item]);
                if (pn > 1) {
                    pm = uni((int)(v & 31)) | pn << 5;
                    pslot = pnext;
                }
                pnext += gridDim.x * (BLK / 64);
            } else {
                item = next_chunk(a.counter, a.nchunks, nullptr, nullptr, home, grp);
                if (item < 0) break;
                if (EXT && a.npieces > 0 && a.pcount[item] != 0) continue;   // handed out as pieces
            }
            const int4 ch = a.chunks[item];
            leaf = uni(ch.x);
            p0 = uni(ch.y);
            cnt = uni(ch.z);
            pend = cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
            if (a.owned) pend = __ballot(lane < cnt && a.owned[p0 + lane] != 0);
            if (pend == 0) continue;
        }
        const float L0 = (float)a.sets[a.cells[leaf].set].L0;
        Frame fr;
        uint64_t amask;
        {
            // the lane's particle, read again for every frame rather than
            // kept in registers through the walk
            int q = p0 + (lane < cnt ? lane : 0);
            asm volatile("" : "+v"(q));
            amask = next_frame(pend, a.pos[q], a.plo[q], a.frec[q].x, L0, &fr);
        }
        pend &= ~amask;
        const int nact = __popcll(amask);
        const int lgR = replicas_lg(nact, a.rmax), R = 1 << lgR, T = 64 >> lgR;
        const int slot = lane & (T - 1), rep = lane >> (6 - lgR);
        if ((amask >> lane) & 1ull) s_pick[w][bits_below(amask)] = lane;
        wave_lds_sync();
        const int pick = slot < nact ? s_pick[w][slot] : 0;
        wave_lds_sync();
        const int p = p0 + pick;
        const bool act = slot < nact;
        typename P::Lane L;
        // an idle lane sits far away so no record is ever in its range
        L.x = act ? in_frame(a.pos[p], fr.lo ? a.plo[p] : make_float4(0.f, 0.f, 0.f, 0.f), fr.o())
                  : make_float4(-FAR, -FAR, -FAR, 0.f);
        // the same records as the staged partners: the two sides of a pair
        // see identical values
        const float4 fi = act ? a.frec[p] : make_float4(1.f, 0.f, 0.f, 0.f);
        L.h = fi.x;
        L.hinv = frcp(L.h);
        L.K = fi.w;
        L.v = act ? a.pv[p] : make_float4(0.f, 0.f, 0.f, 1.f);
        L.A = fi.y;
        L.c = fi.z;
        L.alpha = a.alpha;
        typename P::Acc acc;
        walk<P, EXT>(a, S, s_t[w], L, acc, leaf, fr, R, rep, act, pm, &s_cnt[w][1]);

        const float du = comb_f(acc.du, R);
        const float vs = comb_max(acc.vs, R), Ss = comb_f(acc.S, R);
        const int nn = comb_i(acc.nn, R);
        const uint64_t hs = HASH ? comb_u64(acc.hs, R) : 0ull;
        if (EXT && pslot >= 0) {
            // a piece: its FP64 sums to its slot
            const double tx = comb_d(acc.tx, R), ty = comb_d(acc.ty, R), tz = comb_d(acc.tz, R);
            if (act && rep == 0) {
                double* q = a.part + (size_t)pslot * PART_WORDS * CHUNK + pick;
                q[0 * CHUNK] = tx;
                q[1 * CHUNK] = ty;
                q[2 * CHUNK] = tz;
                q[3 * CHUNK] = (double)du;
                q[4 * CHUNK] = (double)vs;
                q[5 * CHUNK] = (double)Ss;
                q[6 * CHUNK] = (double)nn;
                q[7 * CHUNK] = __longlong_as_double((long long)hs);
            }
        } else {
            const float ax = (float)comb_d(acc.tx, R), ay = (float)comb_d(acc.ty, R);
            const float az = (float)comb_d(acc.tz, R);
            if (act && rep == 0) {
                a.ax[p] = ax;
                a.ay[p] = ay;
                a.az[p] = az;
                a.du[p] = du;
                a.vsig[p] = vs;
                a.S[p] = Ss;
                a.nf[p] = nn;
                if (HASH) a.hash[p] = hs;
            }
        }
        const int npair = wave_count(act && rep == 0 ? nn : 0);
        if (lane == 0) s_cnt[w][0] += (unsigned long long)npair;
    }
    if (lane == 0) {
        flush_work(a.work, s_cnt[w][0]);
        flush_work(a.work + 1, s_cnt[w][1]);
    }
}

template <bool HASH>
__global__ __launch_bounds__(256) void k_force_pieces(ForceArgs a) {
    const int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= a.npieces) return;
    const uint32_t v = a.plist[i];
    const int c = (int)(v >> 5), pn = (int)a.pcount[c];
    if ((v & 31u) != 0u || pn < 2) return;
    const int4 ch = a.chunks[c];
    if (lane >= ch.z) return;
    const int p = ch.y + lane;
    if (a.owned && a.owned[p] == 0) return;
    double tx = 0.0, ty = 0.0, tz = 0.0;
    float du = 0.f, vs = 0.f, Ss = 0.f;
    int nn = 0;
    uint64_t hs = 0;
    for (int k = 0; k < pn; ++k) {
        const double* q = a.part + (size_t)(i + k) * PART_WORDS * CHUNK + lane;
        tx += q[0 * CHUNK];
        ty += q[1 * CHUNK];
        tz += q[2 * CHUNK];
        du += (float)q[3 * CHUNK];
        vs = fmaxf(vs, (float)q[4 * CHUNK]);
        Ss += (float)q[5 * CHUNK];
        nn += (int)q[6 * CHUNK];
        hs += (uint64_t)__double_as_longlong(q[7 * CHUNK]);
    }
    a.ax[p] = (float)tx;
    a.ay[p] = (float)ty;
    a.az[p] = (float)tz;
    a.du[p] = du;
    a.vsig[p] = vs;
    a.S[p] = Ss;
    a.nf[p] = nn;
    if (HASH) a.hash[p] = hs;
}

// ---------------------------------------------------------------------------
// Newton step on h (per particle), ghost, per-cell current h max, scatters,
// reductions, counters.
// ---------------------------------------------------------------------------
__global__ void k_zero_i32(int32_t* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_solve_init(int64_t n, const uint8_t* __restrict__ owned, uint8_t* active, float* lo, float* hi,
                             float* dstep) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    active[p] = (!owned || owned[p]) ? 1 : 0;   // a halo particle keeps the h it came with
    lo[p] = 0.f;
    hi[p] = INFINITY;
    dstep[p] = INFINITY;
}

// Status words of the h solve: [0] some set must be rebuilt, [1] particles
// still active (all sets), then per set s: [2+2s] rebuild flag, [3+2s]
// particles still active.
__device__ __forceinline__ int set_of(const SetInfo* sets, int nsets, int64_t p) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sets[mid].first <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One safeguarded Newton step on N_w(h) = target, taken on ln N_w against
// ln h (exact wherever N_w is a power of h), for every active particle
// (state 1).  Converged particles (|N_w - target| <= tol, tested in FP64)
// keep h and their density (state 0).  For the others the bracket [lo, hi]
// of the root is narrowed, and the Newton step is taken only if it stays in
// the bracket, changes h by at most a factor 2 and is shorter than half the
// previous step; otherwise the bracket is bisected (geometric mean; h is
// doubled or halved while a side is open).  The step-length rule keeps a
// particle whose N_w rises steeply over a short range of h (a dense clump
// entering its support) from alternating between the two sides.  A
// particle whose root lies beyond the largest h its cells support is parked
// (state 2, no more density passes) and raises the rebuild flag of its set;
// the other particles go on converging.
// Newton (or bracketing) step of particle p; returns whether it stays
// active.  hcap: half the box (the minimum-image convention needs h < box/2).
__device__ __forceinline__ bool newton_step(int64_t p, uint8_t* __restrict__ active, const float* __restrict__ nw,
                                            const float* __restrict__ dnw, float* __restrict__ ph,
                                            const float* __restrict__ bound, float* __restrict__ lo,
                                            float* __restrict__ hi, float* __restrict__ dstep, double target,
                                            double tol, double hcap, bool& rebuild_any) {
    if (active[p] != 1) return false;
    const double err = (double)nw[p] - target;
    if (fabs(err) <= tol) {
        active[p] = 0;
        return false;
    }
    const double h = ph[p];
    double l = lo[p], u = hi[p];
    if (err < 0) l = h; else u = h;
    const double d = dnw[p];
    const double Nw = (double)nw[p];
    const bool slope_ok = d > 0 && Nw > 0;
    const double dl = slope_ok ? -log(Nw / target) / (d * h / Nw) : 0.0;
    double hn = h * exp(dl);
    const bool newton = slope_ok && hn > l && hn < u && fabs(dl) <= M_LN2 && fabs(dl) < 0.5 * (double)dstep[p];
    if (!newton) hn = isinf(u) ? 2.0 * h : (l > 0 ? sqrt(l * u) : 0.5 * h);
    if (hn >= hcap) hn = 0.5 * (h + hcap);
    float hf = (float)hn;
    if (hf == (float)h) hf = err < 0 ? nextafterf((float)h, INFINITY) : nextafterf((float)h, 0.f);
    if (!((double)hf < hcap)) hf = nextafterf((float)hcap, 0.f);
    // a step past the largest h the cells support first probes just below
    // it; only if the root still lies beyond is a rebuild needed, and the
    // particle then keeps the step it would take, so that the rebuilt cells
    // are sized for it
    bool rebuild = false;
    const float hb = nextafterf(bound[p], 0.f);
    if (!(hf < bound[p])) {
        if ((float)h == hb && err < 0) rebuild = true;
        else hf = hb;
    }
    lo[p] = (float)l;
    hi[p] = (float)u;
    dstep[p] = (float)fabs(log((double)hf / h));
    ph[p] = hf;
    if (rebuild) {
        // parked: no density passes until the tree is rebuilt for it
        active[p] = 2;
        rebuild_any = true;
        return false;
    }
    return true;
}

// The step of every active particle (one thread each); the rare rebuild
// flags.  The particles still active are counted afterwards (k_count_active).
__global__ void k_newton(int64_t n, const SetInfo* __restrict__ sets, int nsets, uint8_t* __restrict__ active,
                         const float* __restrict__ nw, const float* __restrict__ dnw, float* __restrict__ ph,
                         const float* __restrict__ bound, float* __restrict__ lo, float* __restrict__ hi,
                         float* __restrict__ dstep, double target, double tol, int32_t* __restrict__ status) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || active[p] != 1) return;
    const int s = set_of(sets, nsets, p);
    bool rebuild = false;
    (void)newton_step(p, active, nw, dnw, ph, bound, lo, hi, dstep, target, tol, 0.5 * sets[s].box, rebuild);
    if (rebuild) {
        atomicExch(&status[0], 1);
        atomicExch(&status[2 + 2 * s], 1);
    }
}

// Particles still active, per reduction chunk (one block each) ...
__global__ __launch_bounds__(256) void k_count_active(const int4* __restrict__ red, const uint8_t* __restrict__ active,
                                                      int32_t* __restrict__ part) {
    __shared__ int s_w[4];
    const int4 R = red[blockIdx.x];
    int c = 0;
    for (int p = R.y + threadIdx.x; p < R.y + R.z; p += 256) c += active[p] == 1 ? 1 : 0;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// First reduction chunk of set s (the chunks of a set are consecutive).
__device__ __forceinline__ int first_red_chunk(const int4* __restrict__ red, int nred, int s) {
    int lo = 0, hi = nred;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (red[mid].x < s) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ... then per set (status[3 + 2s]) and in total (status[1]): one block;
// with few sets the whole block sums each set in turn, otherwise one
// wavefront per set, lanes striding over the set's chunks; integer sums,
// written (not accumulated).
constexpr int COUNT_BS = 1024;
__global__ __launch_bounds__(COUNT_BS) void k_count_final(const int4* __restrict__ red, int nred,
                                                          const int32_t* __restrict__ part, int nsets,
                                                          int32_t* __restrict__ status) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __shared__ int s_w[COUNT_BS / 64];
    if (nsets <= COUNT_BS / 64) {
        int tot = 0;   // (thread 0)
        for (int s = 0; s < nsets; ++s) {
            const int r0 = first_red_chunk(red, nred, s);
            int c = 0;
            for (int r = r0 + (int)threadIdx.x; r < nred && red[r].x == s; r += COUNT_BS) c += part[r];
            for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
            if (lane == 0) s_w[w] = c;
            __syncthreads();
            if (threadIdx.x == 0) {
                int t = 0;
                for (int k = 0; k < COUNT_BS / 64; ++k) t += s_w[k];
                status[3 + 2 * s] = t;
                tot += t;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) status[1] = tot;
        return;
    }
    int tot = 0;
    for (int s = w; s < nsets; s += COUNT_BS / 64) {
        int c = 0;
        const int r0 = first_red_chunk(red, nred, s);
#pragma unroll 8
        for (int r = r0 + lane; r < nred && red[r].x == s; r += 64) c += part[r];
        for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
        if (lane == 0) status[3 + 2 * s] = c;
        tot += c;
    }
    if (lane == 0) s_w[w] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < COUNT_BS / 64; ++k) t += s_w[k];
        status[1] = t;
    }
}

// Outputs in caller order are written in that order (coalesced), each read
// from its cell-order slot through the inverse permutation.
__global__ void k_save_state(int64_t n, const uint32_t* __restrict__ iperm, const uint8_t* active, const float* lo,
                             const float* hi, const float* dstep, const float* rho, const float* drho,
                             const float* nw, const float* dnw, const int32_t* nngb, const uint64_t* hash,
                             SolveState sv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = iperm[i];
    sv.active[i] = active[p];
    sv.lo[i] = lo[p];
    sv.hi[i] = hi[p];
    sv.dstep[i] = dstep[p];
    sv.rho[i] = rho[p];
    sv.drho[i] = drho[p];
    sv.nw[i] = nw[p];
    sv.dnw[i] = dnw[p];
    sv.nngb[i] = nngb[p];
    if (hash) sv.hash[i] = hash[p];
}

__global__ void k_load_state(int64_t n, const uint32_t* __restrict__ perm, uint8_t* active, float* lo, float* hi,
                             float* dstep, float* rho, float* drho, float* nw, float* dnw, int32_t* nngb,
                             uint64_t* hash, SolveState sv) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t i = perm[p];
    active[p] = sv.active[i] ? 1 : 0;   // parked particles resume
    lo[p] = sv.lo[i];
    hi[p] = sv.hi[i];
    dstep[p] = sv.dstep[i];
    rho[p] = sv.rho[i];
    drho[p] = sv.drho[i];
    nw[p] = sv.nw[i];
    dnw[p] = sv.dnw[i];
    nngb[p] = sv.nngb[i];
    if (hash) hash[p] = sv.hash[i];
}


__global__ void k_ghost(int64_t n, const float* __restrict__ ph, const float* __restrict__ rho,
                        const float* __restrict__ drho, const float* __restrict__ u, float gamma,
                        float4* __restrict__ frec, float4* __restrict__ pv) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float r = rho[p], h = ph[p];
    const float P = (gamma - 1.f) * r * u[p];
    const float f = 1.f / (1.f + h / (3.f * r) * drho[p]);
    const float hinv = 1.f / h;
    const float h2 = hinv * hinv;
    // h, A = f P / rho^2, sound speed, K = 8 / (pi h^5); rho beside the velocity
    frec[p] = make_float4(h, f * P / (r * r), sqrtf(gamma * (gamma - 1.f) * u[p]), C8PI * h2 * h2 * hinv);
    pv[p].w = r;
}

// Largest current h of the small-h and of the large-h entries of each
// cell's sorted lists (any axis holds the same entries); cells without a
// list get the largest h of all their particles in both.
__global__ __launch_bounds__(256) void k_cell_hcur(Cell* __restrict__ cells, int64_t nc, const float* __restrict__ ph,
                                                   const uint32_t* __restrict__ segoff,
                                                   const uint32_t* __restrict__ segidx) {
    int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nc) return;
    const int lane = threadIdx.x & 63;
    const int first = cells[c].first, count = cells[c].count, ns = cells[c].nsmall;
    uint32_t so = 0xFFFFFFFFu;
    for (int k = 0; k < NAXES && so == 0xFFFFFFFFu; ++k) so = segoff[c * NAXES + k];
    float ms = 0.f, ml = 0.f;
    if (so == 0xFFFFFFFFu) {
#pragma unroll 8
        for (int p = first + lane; p < first + count; p += 64) ms = fmaxf(ms, ph[p]);
        ms = wmax(ms);
        ml = ms;
    } else {
#pragma unroll 8
        for (int q = lane; q < count; q += 64) {
            float hv = ph[segidx[so + q]];
            if (q < ns) ms = fmaxf(ms, hv); else ml = fmaxf(ml, hv);
        }
        ms = wmax(ms);
        ml = wmax(ml);
    }
    if (lane == 0) {
        cells[c].hcur = ms;
        cells[c].hcur_l = ml;
    }
}

__global__ void k_scatter_density(int64_t n, const uint32_t* __restrict__ iperm, const float* rho,
                                  const float* drho, const float* nw, const float* dnw, const int32_t* nngb,
                                  const uint64_t* hash, const float* ph, const uint8_t* __restrict__ owned,
                                  sph_density_out o) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = iperm[i];
    if (owned && !owned[p]) return;   // halo particles: the caller's entries stay as they are
    if (o.rho) o.rho[i] = rho[p];
    if (o.drho_dh) o.drho_dh[i] = drho[p];
    if (o.nw) o.nw[i] = nw[p];
    if (o.dnw_dh) o.dnw_dh[i] = dnw[p];
    if (o.nngb) o.nngb[i] = nngb[p];
    if (o.hash && hash) o.hash[i] = hash[p];
    if (o.h) o.h[i] = ph[p];
}

__global__ void k_scatter_force(int64_t n, const uint32_t* __restrict__ iperm, const float* ax, const float* ay,
                                const float* az, const float* du, const float* vs, const float* S,
                                const int32_t* nf, const uint64_t* hash, const uint8_t* __restrict__ owned,
                                sph_force_out o) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = iperm[i];
    if (owned && !owned[p]) return;
    if (o.ax) o.ax[i] = ax[p];
    if (o.ay) o.ay[i] = ay[p];
    if (o.az) o.az[i] = az[p];
    if (o.dudt) o.dudt[i] = du[p];
    if (o.vsig) o.vsig[i] = vs[p];
    if (o.S) o.S[i] = S[p];
    if (o.nforce) o.nforce[i] = nf[p];
    if (o.hash && hash) o.hash[i] = hash[p];
}

constexpr int NRED = 8;
constexpr int RED_CHUNK = 2048;   // particles per reduction block

// One block per reduction chunk (a range of one set): FP64 partial sums in a
// fixed tree order.
__global__ __launch_bounds__(256) void k_reduce_partial(const int4* __restrict__ red, const float4* __restrict__ pos,
                                                        const float4* __restrict__ pv, const float* __restrict__ ax,
                                                        const float* __restrict__ ay, const float* __restrict__ az,
                                                        const float* __restrict__ du, const float* __restrict__ S,
                                                        const int32_t* __restrict__ nngb,
                                                        const int32_t* __restrict__ nf,
                                                        const uint8_t* __restrict__ owned, double* __restrict__ part) {
    __shared__ double s[NRED][256];
    const int4 R = red[blockIdx.x];
    double acc[NRED] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int p = R.y + threadIdx.x; p < R.y + R.z; p += 256) {
        if (owned && !owned[p]) continue;   // halo particles: no outputs of their own
        double m = pos[p].w;
        float4 v = pv[p];
        double a0 = ax[p], a1 = ay[p], a2 = az[p];
        acc[0] += m * a0;
        acc[1] += m * a1;
        acc[2] += m * a2;
        acc[3] += m * ((double)v.x * a0 + (double)v.y * a1 + (double)v.z * a2 + (double)du[p]);
        acc[4] += m * (double)S[p];
        acc[5] += (double)nngb[p];
        acc[6] += (double)nf[p];
    }
    for (int f = 0; f < NRED; ++f) s[f][threadIdx.x] = acc[f];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int f = 0; f < NRED; ++f) s[f][threadIdx.x] += s[f][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < NRED) part[(int64_t)blockIdx.x * NRED + threadIdx.x] = s[threadIdx.x][0];
}

// Per-set totals: one wavefront per set, lanes striding over the set's
// chunks, combined in a fixed butterfly (deterministic).
__global__ __launch_bounds__(256) void k_reduce_final(const int4* __restrict__ red, int nred,
                                                      const double* __restrict__ part, int nsets,
                                                      double* __restrict__ sums, double* __restrict__ sums2) {
    const int s = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (s >= nsets) return;
    double acc[NRED] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = first_red_chunk(red, nred, s) + lane; r < nred && red[r].x == s; r += 64)
        for (int f = 0; f < NRED; ++f) acc[f] += part[(int64_t)r * NRED + f];
    for (int f = 0; f < NRED; ++f)
        for (int d = 32; d >= 1; d >>= 1) acc[f] += __shfl_xor(acc[f], d, 64);
    if (lane < NRED) {
        double v = acc[0];
        for (int f = 1; f < NRED; ++f) v = lane == f ? acc[f] : v;
        if (sums) sums[(int64_t)s * NRED + lane] = v;
        if (sums2) sums2[(int64_t)s * NRED + lane] = v;
    }
}

// ===========================================================================
// Host orchestration
// ===========================================================================
static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

#define HIPTRY(x)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) return Err{SPH_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)
#define ERRTRY(x)                       \
    do {                                \
        Err e_ = (x);                   \
        if (e_.st != SPH_OK) return e_; \
    } while (0)

static Err ensure_state(sph_tree* t) {
    const int64_t n = std::max<int64_t>(t->n, 1);
    void* p;
    // density: rho, drho, nw, dnw (float), nngb (int), hash (u64)
    ERRTRY(t->alloc(t->b_dens, n * (4 * sizeof(float) + sizeof(int32_t) + sizeof(uint64_t)) + 64, &p));
    t->hashd = (uint64_t*)p;
    t->rho = (float*)(t->hashd + n);
    t->drho = t->rho + n;
    t->nw = t->drho + n;
    t->dnw = t->nw + n;
    t->nngb = (int32_t*)(t->dnw + n);
    // solve: lo, hi, dstep (float), status (2 + 2 per set), active (one byte
    // per particle; 256-byte aligned and padded, k_chunk_list reads it as
    // 8-byte words), the chunk list of the listed density passes
    const int64_t nst = 2 + 2 * (int64_t)t->nsets;
    const size_t act_off = (3 * n * sizeof(float) + sizeof(int32_t) * ((nst + 63) / 64) * 64 + 255) & ~(size_t)255;
    const size_t list_off = (act_off + n + 8 + 255) & ~(size_t)255;
    ERRTRY(t->alloc(t->b_solve, list_off + sizeof(uint32_t) * std::max<int64_t>(t->nchunks, 1), &p));
    t->lo = (float*)p;
    t->hi = t->lo + n;
    t->dstep = t->hi + n;
    t->status = (int32_t*)(t->dstep + n);
    t->active = (uint8_t*)p + act_off;
    t->alist = (uint32_t*)((uint8_t*)p + list_off);
    // force: frec (float4), ax, ay, az, du, vs, S (float), nf (int), hash (u64)
    ERRTRY(t->alloc(t->b_force, n * (sizeof(float4) + 6 * sizeof(float) + sizeof(int32_t) + sizeof(uint64_t)) + 64,
                    &p));
    t->frec = (float4*)p;
    t->hashf = (uint64_t*)(t->frec + n);
    t->fax = (float*)(t->hashf + n);
    t->fay = t->fax + n;
    t->faz = t->fay + n;
    t->fdu = t->faz + n;
    t->fvs = t->fdu + n;
    t->fS = t->fvs + n;
    t->fn = (int32_t*)(t->fS + n);
    // reduction chunks: RED_CHUNK particles of one set each
    if (t->red_off != t->off) {
        t->red_chunks.clear();
        for (int s = 0; s < t->nsets; ++s) {
            int64_t a = t->off[s], b = t->off[s + 1];
            if (a == b) t->red_chunks.push_back(make_int4(s, (int)a, 0, 0));
            for (int64_t q = a; q < b; q += RED_CHUNK)
                t->red_chunks.push_back(make_int4(s, (int)q, (int)std::min<int64_t>(RED_CHUNK, b - q), 0));
        }
        t->nred = (int64_t)t->red_chunks.size();
        ERRTRY(t->alloc(t->b_red, t->nred * (sizeof(int4) + NRED * sizeof(double) + sizeof(int32_t)) +
                                      (size_t)t->nsets * NRED * sizeof(double) + 64, &p));
        t->partial = (double*)p;
        t->sums_int = t->partial + t->nred * NRED;
        t->d_red = (int4*)(t->sums_int + (int64_t)t->nsets * NRED);
        t->part_cnt = (int32_t*)(t->d_red + t->nred);
        HIPTRY(hipMemcpyAsync(t->d_red, t->red_chunks.data(), sizeof(int4) * t->nred, hipMemcpyHostToDevice,
                              t->stream));
        t->red_off = t->off;
    }
    return Err{};
}


static int rmax_of(const sph_tree* t) {
    int r = t->prm.max_replicas;
    return (r == 1 || r == 2 || r == 4 || r == 8 || r == 16) ? r : 16;
}

// The resident blocks per CU of every persistent interaction kernel, asked
// when the context is made (not under a graph capture).
void query_occupancy(sph_ctx* ctx) {
    const void* ks[] = {(const void*)k_density<true, true, true>,   (const void*)k_density<true, false, true>,
                        (const void*)k_density<false, true, true>,  (const void*)k_density<false, false, true>,
                        (const void*)k_density<true, true, false>,  (const void*)k_density<true, false, false>,
                        (const void*)k_density<false, true, false>, (const void*)k_density<false, false, false>,
                        (const void*)k_force<true, true>,           (const void*)k_force<false, true>,
                        (const void*)k_force<true, false>,          (const void*)k_force<false, false>};
    for (const void* k : ks) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, BLK, 0) != hipSuccess || nb < 1) nb = 4;
        ctx->resident[k] = nb;
    }
}

// Grid of a persistent interaction kernel: at most as many blocks as fit on
// the GPU at once (blocks beyond that would only start when others leave,
// at the end of the pass, and the pieces of heavy chunks are dealt to every
// wave of the grid up front), fewer if blocks_per_cu asks for fewer.
static int persistent_blocks(sph_ctx* ctx, const sph_tree* t, int64_t items, const void* kernel) {
    const auto it = ctx->resident.find(kernel);
    int bpc = it != ctx->resident.end() ? it->second : 4;
    if (t->prm.blocks_per_cu > 0) bpc = std::min(bpc, t->prm.blocks_per_cu);
    const int64_t want = (items + 3) / 4;
    const int64_t cap = (int64_t)ctx->n_cu * bpc;
    return (int)std::max<int64_t>(1, std::min(want, cap));
}

static DensArgs dens_args(sph_tree* t, int* counter, const int* lcount) {
    DensArgs a;
    a.cells = t->cells;
    a.sets = t->d_sets;
    a.chunks = t->chunks;
    a.nchunks = (int)t->nchunks;
    a.counter = counter;
    a.pos = t->pos;
    a.plo = t->plo;
    a.ph = t->ph;
    a.mix = t->mix;
    a.active = t->active;
    a.owned = t->owned;
    a.list = lcount ? t->alist : nullptr;
    a.lcount = lcount;
    a.csr = t->csr;
    a.csr_off = t->csr_off;
    a.segoff = t->segoff;
    a.segpos = t->segpos;
    a.blkbox = t->blkbox;
    a.cellord = t->blkbox && !(t->prm.flags & SPH_FLAG_SORTED_ONLY);
    a.max_sorted = t->max_sorted;
    a.skip = a.cellord && !(t->prm.flags & SPH_FLAG_NO_BLOCK_SKIP);
    a.pcount = t->pcount;
    a.plist = t->plist;
    a.npieces = (int)t->npieces;
    a.part = t->part;
    a.segidx = t->segidx;
    a.status = t->status;
    a.rho = t->rho;
    a.drho = t->drho;
    a.nw = t->nw;
    a.dnw = t->dnw;
    a.nngb = t->nngb;
    a.hash = t->hashd;
    a.work = (unsigned long long*)(t->work_ctr);
    a.rmax = rmax_of(t);
    return a;
}

// listed: a Newton pass after the first, over the chunks that still hold
// active particles (k_chunk_list; its counts sit in the context's counter
// block after the force counters, zeroed here with the density counters)
static bool ext_kernels(const sph_tree* t) { return t->ext(); }

static void launch_density(sph_ctx* ctx, sph_tree* t, bool solve, bool listed, int* counter) {
    hipStream_t st = ctx->stream;
    int* lcount = nullptr;
    if (listed) {
        lcount = counter + 2 * NGRP * CSTRIDE;
        hipLaunchKernelGGL(k_zero_i32, dim3(3), dim3(256), 0, st, counter, 3 * NGRP * CSTRIDE);
        const int bpg = (int)((t->nchunks / NGRP + LIST_BS) / LIST_BS);
        hipLaunchKernelGGL(k_chunk_list, dim3(NGRP * bpg), dim3(LIST_BS), 0, st, t->chunks, (int)t->nchunks, bpg,
                           t->active, t->alist, lcount);
    } else {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, st, counter, NGRP * CSTRIDE);
    }
    DensArgs a = dens_args(t, counter, lcount);
    void (*kern)(DensArgs);
    if (ext_kernels(t)) {
        if (solve) kern = t->hash ? k_density<true, true, true> : k_density<true, false, true>;
        else kern = t->hash ? k_density<false, true, true> : k_density<false, false, true>;
    } else {
        if (solve) kern = t->hash ? k_density<true, true, false> : k_density<true, false, false>;
        else kern = t->hash ? k_density<false, true, false> : k_density<false, false, false>;
    }
    hipLaunchKernelGGL(kern, dim3(persistent_blocks(ctx, t, t->nchunks, (const void*)kern)), dim3(BLK), 0, st, a);
    if (t->npieces > 0) {
        const dim3 gp(nblk(t->npieces, 4));
        if (solve) {
            if (t->hash) hipLaunchKernelGGL((k_density_pieces<true, true>), gp, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((k_density_pieces<true, false>), gp, dim3(256), 0, st, a);
        } else {
            if (t->hash) hipLaunchKernelGGL((k_density_pieces<false, true>), gp, dim3(256), 0, st, a);
            else hipLaunchKernelGGL((k_density_pieces<false, false>), gp, dim3(256), 0, st, a);
        }
    }
}

// The largest h of each block of 64 particles (the force records' h, into
// the w of the block's lower corner), for the block test of the force pass.
__global__ __launch_bounds__(256) void k_block_h(const float4* __restrict__ frec, int64_t n, int64_t nb,
                                                 float4* __restrict__ box) {
    const int lane = threadIdx.x & 63;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nb; b += (int64_t)gridDim.x * 4) {
        const int64_t e = b * 64 + lane;
        float v = e < n ? frec[e].x : 0.f;
        for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
        if (lane == 0) box[2 * b].w = v;
    }
}

static void launch_force(sph_ctx* ctx, sph_tree* t, int* counter) {
    hipStream_t st = ctx->stream;
    const int64_t n = t->n;
    hipLaunchKernelGGL(k_ghost, dim3(nblk(n, 256)), dim3(256), 0, st, n, t->ph, t->rho, t->drho, t->pu,
                       t->prm.gamma, t->frec, t->pv);
    hipLaunchKernelGGL(k_cell_hcur, dim3(nblk(t->ncells, 4)), dim3(256), 0, st, t->cells, t->ncells, t->ph, t->segoff,
                       t->segidx);
    if (t->blkbox && t->ext())
        hipLaunchKernelGGL(k_block_h, dim3((unsigned)std::min<int64_t>(nblk(t->nblk, 4), 65535)), dim3(256), 0, st,
                           t->frec, n, t->nblk, t->blkbox);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, st, counter, NGRP * CSTRIDE);
    ev_mark(ctx, "ghost");
    ForceArgs a;
    a.cells = t->cells;
    a.sets = t->d_sets;
    a.chunks = t->chunks;
    a.nchunks = (int)t->nchunks;
    a.counter = counter;
    a.pos = t->pos;
    a.plo = t->plo;
    a.pv = t->pv;
    a.frec = t->frec;
    a.owned = t->owned;
    a.mix = t->mix;
    a.csr = t->csr;
    a.csr_off = t->csr_off;
    a.segoff = t->segoff;
    a.segpos = t->segpos;
    a.blkbox = t->blkbox;
    a.cellord = t->blkbox && !(t->prm.flags & SPH_FLAG_SORTED_ONLY);
    a.max_sorted = t->max_sorted;
    a.skip = a.cellord && !(t->prm.flags & SPH_FLAG_NO_BLOCK_SKIP);
    a.pcount = t->pcount;
    a.plist = t->plist;
    a.npieces = (int)t->npieces;
    a.part = t->part;
    a.segidx = t->segidx;
    a.alpha = t->prm.alpha;
    a.ax = t->fax;
    a.ay = t->fay;
    a.az = t->faz;
    a.du = t->fdu;
    a.vsig = t->fvs;
    a.S = t->fS;
    a.nf = t->fn;
    a.hash = t->hashf;
    a.work = (unsigned long long*)(t->work_ctr + 256);
    a.rmax = rmax_of(t);
    void (*kern)(ForceArgs);
    if (ext_kernels(t)) kern = t->hash ? k_force<true, true> : k_force<false, true>;
    else kern = t->hash ? k_force<true, false> : k_force<false, false>;
    hipLaunchKernelGGL(kern, dim3(persistent_blocks(ctx, t, t->nchunks, (const void*)kern)), dim3(BLK), 0, st, a);
    if (t->npieces > 0) {
        const dim3 gp(nblk(t->npieces, 4));
        if (t->hash) hipLaunchKernelGGL((k_force_pieces<true>), gp, dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_force_pieces<false>), gp, dim3(256), 0, st, a);
    }
}

// A Newton step of every active particle.
static void launch_newton(sph_ctx* ctx, sph_tree* t) {
    hipLaunchKernelGGL(k_newton, dim3(nblk(t->n, 256)), dim3(256), 0, ctx->stream, t->n, t->d_sets, t->nsets,
                       t->active, t->nw, t->dnw, t->ph, t->bound, t->lo, t->hi, t->dstep, (double)t->prm.n_target,
                       (double)t->prm.h_tol, t->status);
}

// status[1] and status[3+2s] = particles still active after the last Newton
// step (written, not accumulated: nothing to clear first)
static void launch_count(sph_ctx* ctx, sph_tree* t) {
    hipLaunchKernelGGL(k_count_active, dim3((unsigned)t->nred), dim3(256), 0, ctx->stream, t->d_red, t->active,
                       t->part_cnt);
    hipLaunchKernelGGL(k_count_final, dim3(1), dim3(COUNT_BS), 0, ctx->stream, t->d_red, (int)t->nred, t->part_cnt,
                       t->nsets, t->status);
}

static void launch_reduce(sph_ctx* ctx, sph_tree* t, double* sums_out) {
    hipStream_t st = ctx->stream;
    if (t->nred == 0) return;
    hipLaunchKernelGGL(k_reduce_partial, dim3((unsigned)t->nred), dim3(256), 0, st, t->d_red, t->pos, t->pv, t->fax,
                       t->fay, t->faz, t->fdu, t->fS, t->nngb, t->fn, t->owned, t->partial);
    hipLaunchKernelGGL(k_reduce_final, dim3(nblk(t->nsets, 4)), dim3(256), 0, st, t->d_red, (int)t->nred, t->partial,
                       t->nsets, sums_out, t->sums_int);
}

static void launch_scatter_density(sph_ctx* ctx, sph_tree* t, const sph_density_out* o) {
    if (!o || t->n == 0) return;
    hipLaunchKernelGGL(k_scatter_density, dim3(nblk(t->n, 256)), dim3(256), 0, ctx->stream, t->n, t->iperm, t->rho,
                       t->drho, t->nw, t->dnw, t->nngb, t->hash ? t->hashd : nullptr, t->ph, t->owned, *o);
}

static void launch_scatter_force(sph_ctx* ctx, sph_tree* t, const sph_force_out* o) {
    if (!o || t->n == 0) return;
    hipLaunchKernelGGL(k_scatter_force, dim3(nblk(t->n, 256)), dim3(256), 0, ctx->stream, t->n, t->iperm, t->fax,
                       t->fay, t->faz, t->fdu, t->fvs, t->fS, t->fn, t->hash ? t->hashf : nullptr, t->owned, *o);
}

// The pair-evaluation counters of a stage start at zero (density: words
// [0, 256), force: [256, 512) of the work block of the context's counters).
static void zero_work(sph_ctx* ctx, sph_tree* t, int first, int words) {
    t->work_ctr = ctx->d_counter + sph_ctx::CTR_WORK;
    hipLaunchKernelGGL(k_zero_i32, dim3(2), dim3(256), 0, ctx->stream, t->work_ctr + first, words);
}

Err run_density(sph_ctx* ctx, sph_tree* t, const sph_density_out* out) {
    if (!t->built || !t->sorted) return Err{SPH_E_STATE, "density before build_cells/sort_pairs"};
    if (out && out->hash && !t->hash) return Err{SPH_E_ARG, "pair hash requested without SPH_FLAG_PAIR_HASH"};
    ERRTRY(ensure_state(t));
    if (t->n == 0) return Err{};
    ev_mark(ctx, "start");
    zero_work(ctx, t, 0, 256);
    launch_density(ctx, t, false, false, ctx->d_counter);
    ev_mark(ctx, "density");
    launch_scatter_density(ctx, t, out);
    HIPTRY(hipGetLastError());
    ev_mark(ctx, "scatter");
    t->have_density = true;
    return Err{};
}

Err run_solve(sph_ctx* ctx, sph_tree* t, const sph_density_out* out, int32_t* n_unconv, int32_t* iters) {
    if (!t->built || !t->sorted) return Err{SPH_E_STATE, "solve_h before build_cells/sort_pairs"};
    if (out && out->hash && !t->hash) return Err{SPH_E_ARG, "pair hash requested without SPH_FLAG_PAIR_HASH"};
    if (t->prm.max_iter < 1 || !(t->prm.h_tol > 0.f) || !(t->prm.n_target > 0.f))
        return Err{SPH_E_ARG, "bad solve parameters"};
    ERRTRY(ensure_state(t));
    hipStream_t st = ctx->stream;
    const int64_t n = t->n;
    if (n_unconv) *n_unconv = 0;
    if (iters) *iters = 0;
    if (n == 0) return Err{};
    ev_mark(ctx, "start");
    const bool resume = (t->prm.flags & SPH_FLAG_RESUME) && t->saved && t->saved_n == n;
    if (resume) {
        hipLaunchKernelGGL(k_load_state, dim3(nblk(n, 256)), dim3(256), 0, st, n, t->perm, t->active, t->lo, t->hi,
                           t->dstep, t->rho, t->drho, t->nw, t->dnw, t->nngb, t->hash ? t->hashd : nullptr,
                           t->saved_state());
    } else {
        hipLaunchKernelGGL(k_solve_init, dim3(nblk(n, 256)), dim3(256), 0, st, n, t->owned, t->active, t->lo,
                           t->hi, t->dstep);
    }
    t->saved = false;
    const int nst = 2 + 2 * t->nsets;
    hipLaunchKernelGGL(k_zero_i32, dim3(nblk(nst, 256)), dim3(256), 0, st, t->status, nst);
    zero_work(ctx, t, 0, 256);
    // Each pass is enqueued before the host reads the status of the one
    // before, so the device runs pass k + 1 while the host waits for pass
    // k's counts (no idle gap per pass).  A pass enqueued after the last
    // one needed finds no active particle: an empty chunk list, no Newton
    // step, no change.  The status words of pass k go to pinned slot k mod 2.
    for (auto& e : ctx->solve_ev)
        if (!e) HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    int32_t* slots = (int32_t*)((char*)ctx->h_pin + sph_ctx::PIN_SOLVE);
    auto enqueue = [&](int k) -> hipError_t {
        ev_mark(ctx, "newton");
        launch_density(ctx, t, true, k > 0, ctx->d_counter);
        ev_mark(ctx, "density_pass");
        launch_newton(ctx, t);
        launch_count(ctx, t);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(slots + 2 * (k & 1), t->status, 2 * sizeof(int32_t),
                                                hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(ctx->solve_ev[k & 1], st);
        return e;
    };
    int32_t hstat[2] = {0, 0};
    int it = 0, enq = 1;
    bool rebuild = false;
    HIPTRY(enqueue(0));
    for (int k = 0; k < t->prm.max_iter; ++k) {
        if (k + 1 < t->prm.max_iter) {
            HIPTRY(enqueue(k + 1));
            enq = k + 2;
        }
        HIPTRY(hipEventSynchronize(ctx->solve_ev[k & 1]));
        hstat[0] = slots[2 * (k & 1)];
        hstat[1] = slots[2 * (k & 1) + 1];
        it = k + 1;
        if (hstat[1] == 0) break;
    }
    if (enq > it && ctx->timing) {
        // the pass enqueued after the last one needed did no work: its time
        // counts with the Newton bookkeeping, not as a density pass
        for (size_t e = ctx->nev; e-- > 0;)
            if (std::strcmp(ctx->ev_name[e], "density_pass") == 0) {
                ctx->ev_name[e] = "newton";
                break;
            }
    }
    rebuild = hstat[0] != 0;
    ev_mark(ctx, "newton");
    if (!rebuild && hstat[1] > 0) {
        // unconverged particles moved h after their last density: recompute
        // their density at the h they hold now
        launch_density(ctx, t, true, true, ctx->d_counter);
        ev_mark(ctx, "density_pass");
    }
    launch_scatter_density(ctx, t, out);
    if (rebuild) {
        ERRTRY(t->ensure_saved());
        hipLaunchKernelGGL(k_save_state, dim3(nblk(n, 256)), dim3(256), 0, st, n, t->iperm, t->active, t->lo, t->hi,
                           t->dstep, t->rho, t->drho, t->nw, t->dnw, t->nngb, t->hash ? t->hashd : nullptr,
                           t->saved_state());
        t->saved = true;
        t->saved_n = n;
    }
    HIPTRY(hipGetLastError());
    // the counts are known: the scatter (and a state save) run on without
    // the host waiting for them
    ev_mark(ctx, "scatter");
    if (iters) *iters = it;
    if (n_unconv) *n_unconv = hstat[1];
    t->have_density = !rebuild;
    if (rebuild) return Err{SPH_E_REBUILD, "h outgrew the cell support: rebuild with the returned h"};
    if (hstat[1] > 0) return Err{SPH_E_NOCONV, std::to_string(hstat[1]) + " particles unconverged"};
    return Err{};
}

Err run_force(sph_ctx* ctx, sph_tree* t, const sph_force_out* out) {
    if (!t->have_density) return Err{SPH_E_STATE, "force before a density pass at the current h"};
    if (out && out->hash && !t->hash) return Err{SPH_E_ARG, "pair hash requested without SPH_FLAG_PAIR_HASH"};
    ERRTRY(ensure_state(t));
    if (t->n == 0) return Err{};
    ev_mark(ctx, "start");
    zero_work(ctx, t, 256, 256);
    launch_force(ctx, t, ctx->d_counter + NGRP * CSTRIDE);
    ev_mark(ctx, "force");
    launch_reduce(ctx, t, out ? out->sums : nullptr);
    launch_scatter_force(ctx, t, out);
    HIPTRY(hipGetLastError());
    ev_mark(ctx, "reduce+scatter");
    return Err{};
}

// One GPU's share (Section I: a data decomposition gives each node its part
// of the data plus the data across the surface it exchanges; Section IV:
// that exchange becomes tasks): the ownership of every particle in cell
// order, and the density state of the read-only halo particles as their
// owners computed it.
__global__ void k_set_halo(int64_t n, const uint32_t* __restrict__ perm, const uint8_t* __restrict__ owned_in,
                           const float* __restrict__ rho_in, const float* __restrict__ drho_in,
                           uint8_t* __restrict__ owned, float* __restrict__ rho, float* __restrict__ drho) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t i = perm[p];
    const uint8_t o = owned_in[i] ? 1 : 0;
    owned[p] = o;
    if (!o) {
        rho[p] = rho_in[i];
        drho[p] = drho_in[i];
    }
}

Err set_halo(sph_ctx* ctx, sph_tree* t, const uint8_t* owned, const float* rho, const float* drho) {
    if (!t->built) return Err{SPH_E_STATE, "set_halo before build_cells"};
    if (!owned) {
        t->owned = nullptr;
        t->invalidate_graph();
        return Err{};
    }
    if (!rho || !drho) return Err{SPH_E_ARG, "halo densities missing"};
    ERRTRY(ensure_state(t));
    void* p;
    ERRTRY(t->alloc(t->b_owned, (size_t)std::max<int64_t>(t->n, 1), &p));
    t->owned = (uint8_t*)p;
    t->invalidate_graph();
    if (t->n > 0)
        hipLaunchKernelGGL(k_set_halo, dim3(nblk(t->n, 256)), dim3(256), 0, ctx->stream, t->n, t->perm, owned, rho, drho,
                           t->owned, t->rho, t->drho);
    HIPTRY(hipGetLastError());
    return Err{};
}

// caller layout: [0] unconverged total, [1] any rebuild, then per set
// [2+2s] unconverged, [3+2s] rebuild
__global__ void k_copy_status(const int32_t* __restrict__ status, int nsets, int32_t* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        out[0] = status[1];
        out[1] = status[0];
    }
    if (i < nsets) {
        out[2 + 2 * i] = status[3 + 2 * i];
        out[3 + 2 * i] = status[2 + 2 * i];
    }
}

// The post-build pipeline as one HIP graph: k_iter Newton iterations with
// device-side early exit (chunks without active particles return at once),
// one density pass for particles still active, ghost, force, sums and the
// scatters to caller order.  Captured on a private stream, launched on the
// context's stream; re-captured when the tree or the output pointers change.
Err run_graph(sph_ctx* ctx, sph_tree* t, int k_iter, const sph_density_out* dout, const sph_force_out* fout,
              int32_t* n_unconv_dev) {
    if (!t->built || !t->sorted) return Err{SPH_E_STATE, "graph before build_cells/sort_pairs"};
    if (!n_unconv_dev) return Err{SPH_E_ARG, "null n_unconverged_dev"};
    if (((dout && dout->hash) || (fout && fout->hash)) && !t->hash)
        return Err{SPH_E_ARG, "pair hash requested without SPH_FLAG_PAIR_HASH"};
    ERRTRY(ensure_state(t));
    if (t->n == 0) return Err{};
    std::vector<const void*> key;
    key.push_back((const void*)(intptr_t)k_iter);
    key.push_back(n_unconv_dev);
    const void* dk[7] = {dout ? dout->rho : nullptr, dout ? dout->drho_dh : nullptr, dout ? dout->nw : nullptr,
                         dout ? dout->dnw_dh : nullptr, dout ? dout->nngb : nullptr,
                         dout ? dout->hash : nullptr, dout ? dout->h : nullptr};
    const void* fk[9] = {fout ? fout->ax : nullptr, fout ? fout->ay : nullptr, fout ? fout->az : nullptr,
                         fout ? fout->dudt : nullptr, fout ? fout->vsig : nullptr, fout ? fout->S : nullptr,
                         fout ? fout->nforce : nullptr, fout ? fout->hash : nullptr, fout ? fout->sums : nullptr};
    key.insert(key.end(), dk, dk + 7);
    key.insert(key.end(), fk, fk + 9);
    // everything else the captured launches take: sizes, launch shapes,
    // parameters and the device buffers.  A build that leaves all of them
    // as they were (the same sets again, the buffers in place, as in a
    // batched step repeated on a workspace) replays the instantiated graph;
    // the kernels read the new data from the same buffers.
    auto val = [&](uint64_t v) { key.push_back((const void*)(uintptr_t)v); };
    auto fbits = [](float f) { uint32_t u; std::memcpy(&u, &f, 4); return (uint64_t)u; };
    val((uint64_t)t->n);
    val((uint64_t)t->nsets);
    val((uint64_t)t->nchunks);
    val((uint64_t)t->ncells);
    val((uint64_t)t->nred);
    val((uint64_t)t->npieces);
    // which kernels (with or without the heavy-chunk and cell-order code)
    // and which partners have sorted lists
    val((uint64_t)t->ext() | ((uint64_t)(uint32_t)t->max_sorted << 1));
    val(t->hash ? 1 : 0);
    val(fbits(t->prm.alpha) | (fbits(t->prm.gamma) << 32));
    val(t->prm.flags);
    val(fbits(t->prm.n_target) | (fbits(t->prm.h_tol) << 32));
    val((uint64_t)(uint32_t)t->prm.blocks_per_cu | ((uint64_t)(uint32_t)t->prm.max_replicas << 32));
    val((uint64_t)ctx->n_cu);
    const void* ptrs[] = {ctx->d_counter, t->d_sets, t->cells, t->chunks, t->csr, t->csr_off, t->segoff,
                          t->segpos, t->segidx, t->pos, t->plo, t->pv, t->ph, t->pu, t->bound, t->mix, t->iperm,
                          t->perm, t->owned, t->rho, t->hashd, t->lo, t->active, t->alist, t->status, t->frec,
                          t->hashf, t->partial, t->d_red, t->sums_int, t->part_cnt, t->blkbox, t->pcount,
                          t->plist, t->part};
    key.insert(key.end(), ptrs, ptrs + sizeof(ptrs) / sizeof(ptrs[0]));
    if (!t->gexec || key != t->gkey) {
        ++t->graph_captures;
        t->invalidate_graph();
        if (!ctx->cap_stream) HIPTRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipStream_t user = ctx->stream;
        bool timing = ctx->timing;
        ctx->stream = ctx->cap_stream;
        ctx->timing = false;
        hipStream_t st = ctx->stream;
        const int64_t n = t->n;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_solve_init, dim3(nblk(n, 256)), dim3(256), 0, st, n, t->owned, t->active, t->lo,
                               t->hi, t->dstep);
            zero_work(ctx, t, 0, 512);
            const int nst = 2 + 2 * t->nsets;
            hipLaunchKernelGGL(k_zero_i32, dim3(nblk(nst, 256)), dim3(256), 0, st, t->status, nst);
            for (int it = 0; it < k_iter; ++it) {
                launch_density(ctx, t, true, it > 0, ctx->d_counter);
                launch_newton(ctx, t);
            }
            // only the state after the last step is reported
            launch_count(ctx, t);
            launch_density(ctx, t, true, k_iter > 0, ctx->d_counter);
            launch_force(ctx, t, ctx->d_counter + NGRP * CSTRIDE);
            launch_reduce(ctx, t, fout ? fout->sums : nullptr);
            launch_scatter_density(ctx, t, dout);
            launch_scatter_force(ctx, t, fout);
            hipLaunchKernelGGL(k_copy_status, dim3(nblk(t->nsets, 256)), dim3(256), 0, st, t->status, t->nsets,
                               n_unconv_dev);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(st, &g);
            if (e == hipSuccess) {
                e = hipGraphInstantiate(&t->gexec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
            }
        }
        ctx->stream = user;
        ctx->timing = timing;
        if (e != hipSuccess) {
            t->gexec = nullptr;
            return Err{SPH_E_HIP, std::string("graph capture: ") + hipGetErrorString(e)};
        }
        t->gkey = key;
    }
    HIPTRY(hipGraphLaunch(t->gexec, ctx->stream));
    t->have_density = true;
    return Err{};
}

}  // namespace sph
