// Internal declarations of the gfx950 SPH library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sphcell.h"

namespace sph {

constexpr int WAVE = 64;
constexpr int NAXES = 13;
constexpr int MAX_SETS = 1 << 12;     // set id bits in the particle key
constexpr int KEY_BITS_PER_DIM = 17;  // log2(top grid) + max depth must fit
constexpr int SEG_LDS_MAX = 4096;     // largest (cell, axis) list sorted in LDS
constexpr int CHUNK = 64;             // target particles per work item (one wave)
constexpr int PIECE_MAX = 16;         // pieces a heavy chunk is split into at most
constexpr int PART_WORDS = 8;         // partial sums of a particle in one piece (doubles)
constexpr int SCAN_MIN = 256;         // swept records from which a partner may be read in cell order
constexpr int SEG_LARGE_MAX = 16384;  // longest list sorted in LDS (longer: radix sort)
constexpr int SMALL_H_DIV = 8;        // sorted lists split at h = cell edge / 8

// Orders a wavefront's LDS writes before its later LDS reads (the wave runs
// in lockstep; the fences keep the compiler from reordering across it).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------------
// Cell-pair axes (Section II-C: 13 possible axes).  Offsets o in {-1,0,1}^3
// are coded as (ox+1)*9 + (oy+1)*3 + (oz+1); code 13 is the zero offset.
// The 13 canonical directions have their first non-zero component +1.
// ------------------------------------------------------------------------
__host__ __device__ inline int ocode(int ox, int oy, int oz) { return (ox + 1) * 9 + (oy + 1) * 3 + (oz + 1); }
__host__ __device__ inline int ocx(int c) { return c / 9 - 1; }
__host__ __device__ inline int ocy(int c) { return (c / 3) % 3 - 1; }
__host__ __device__ inline int ocz(int c) { return c % 3 - 1; }

// canonical direction k -> offset code
__host__ __device__ inline int axis_code(int k) {
    // (1,0,0) (0,1,0) (0,0,1) (1,1,0) (1,-1,0) (1,0,1) (1,0,-1)
    // (0,1,1) (0,1,-1) (1,1,1) (1,1,-1) (1,-1,1) (1,-1,-1)
    const int t[13] = {22, 16, 14, 25, 19, 23, 21, 17, 15, 26, 24, 20, 18};
    return t[k];
}

// offset code -> (axis k, sign): sign = +1 when the offset is the canonical
// direction, -1 when it is its opposite.  Returns k (0..12), or -1 for 13.
__host__ __device__ inline int axis_of(int code, int* sign) {
    int ox = ocx(code), oy = ocy(code), oz = ocz(code);
    int s = 1;
    if (ox < 0 || (ox == 0 && (oy < 0 || (oy == 0 && oz < 0)))) {
        s = -1; ox = -ox; oy = -oy; oz = -oz;
    }
    *sign = s;
    int c = ocode(ox, oy, oz);
    for (int k = 0; k < 13; ++k)
        if (axis_code(k) == c) return k;
    return -1;
}

// ------------------------------------------------------------------------
// Morton keys: x bit highest within each triple.
// ------------------------------------------------------------------------
__host__ __device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFF;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
__host__ __device__ inline uint64_t morton3(uint64_t a, uint64_t b, uint64_t c) {
    return (spread3(a) << 2) | (spread3(b) << 1) | spread3(c);
}

// Order-preserving map of a float to uint32.
__host__ __device__ inline uint32_t f2ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ------------------------------------------------------------------------
// Per-set geometry (device table).
// ------------------------------------------------------------------------
struct SetInfo {
    int64_t first;     // particle range in cell order (== caller order range)
    int64_t count;
    double box;
    double L0;         // top cell edge = box / G
    int32_t lgG;       // log2 of top cells per side
    int32_t top_base;  // id of the first top cell of this set
    int32_t key_shift; // left shift that aligns this set's Morton code in the key
    int32_t depth;     // levels below the top grid the keys resolve for this set
    float drift;       // bound on any particle's displacement since the build (refreshes add up)
    float pad_;
};

// One cell of the hierarchy (all levels and sets in one table).  Cells of a
// level occupy a contiguous id range, in Morton order; the eight children of
// a split cell are consecutive (empty ones included).
struct Cell {
    int32_t first, count;    // particle range in cell order
    int32_t parent, child;   // parent id (-1 at the top), first child id (-1 if not split)
    int32_t ix, iy, iz;      // integer coordinates at this level
    int16_t level, set;
    float hmax;              // largest decision h (h * (1 + slack)) in the cell
    float hcur;              // largest current h among the small-h entries of its sorted lists
    float hcur_l;            // largest current h among the large-h entries
    float bound;             // h must stay below this for the tasks built at this level
    uint32_t split;          // 1 if bisected
    int32_t nsmall;          // sorted lists: entries [0, nsmall) have h <= edge/8 at sort time
    int32_t pad[2];
};
static_assert(sizeof(Cell) == 64, "Cell layout");

// Newton state of a solve interrupted by a rebuild, kept in caller order so
// that the solve on the rebuilt tree continues where it stopped.
struct SolveState {
    uint8_t* active;
    float *lo, *hi, *dstep, *rho, *drho, *nw, *dnw;
    int32_t* nngb;
    uint64_t* hash;
};

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

// Error carrier for the host orchestration.
struct Err {
    sph_status st = SPH_OK;
    std::string msg;
};

}  // namespace sph

