// Device-wide primitives for the cell build: exclusive scan of uint32 and a
// stable LSD radix sort of (uint64 key, uint32 value) pairs.  Both are
// written for 64-lane wavefronts: the scan uses wave shuffles, the radix
// scatter ranks equal digits inside a wave with eight ballots and across the
// four waves of a block through LDS, which keeps the sort stable.
#include "sph_prims.h"

namespace sph {

// ---------------------------------------------------------------------------
// Exclusive scan
// ---------------------------------------------------------------------------
constexpr int SCAN_BS = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IPT;

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Block exclusive scan of one value per thread; returns the block total.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* s_w, uint32_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        uint32_t x = s_w[k];
        if (k < w) base += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

__global__ __launch_bounds__(SCAN_BS) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                         uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s_w[SCAN_BS / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        int64_t i = base + (int64_t)k * SCAN_BS + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t tot;
    block_excl_scan(acc, s_w, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums, sequential over chunks.
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ bsum, int64_t nb,
                                                   uint32_t* __restrict__ total) {
    __shared__ uint32_t s_w[16];
    uint32_t carry = 0;
    for (int64_t s = 0; s < nb; s += 1024) {
        int64_t i = s + threadIdx.x;
        uint32_t v = i < nb ? bsum[i] : 0;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, s_w, tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(SCAN_BS) void k_scan_apply(const uint32_t* __restrict__ in,
                                                        uint32_t* __restrict__ out, int64_t n,
                                                        const uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s_w[SCAN_BS / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    uint32_t v[SCAN_IPT];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        acc += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(acc, s_w, tot) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
}

// Inputs up to SCAN_SMALL elements: one block stages them in LDS with
// coalesced loads, each thread scans a contiguous run of SCAN_SMALL / 1024,
// and the results go back coalesced (one launch instead of three).
constexpr int64_t SCAN_SMALL = 32768;
// (element i sits at i + i/32 in LDS: a thread's run of consecutive
// elements then spreads over all banks)
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }
__global__ __launch_bounds__(1024) void k_scan_small(const uint32_t* in, uint32_t* out, int64_t n,
                                                     uint32_t* __restrict__ total) {
    __shared__ uint32_t s_v[SCAN_SMALL + SCAN_SMALL / 32];
    __shared__ uint32_t s_w[16];
#pragma unroll 8
    for (int i = threadIdx.x; i < (int)n; i += 1024) s_v[scan_pad(i)] = in[i];
    __syncthreads();
    constexpr int PER = (int)(SCAN_SMALL / 1024);
    const int base = (int)threadIdx.x * PER;
    uint32_t v[PER];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = base + k < n ? s_v[scan_pad(base + k)] : 0u;
        acc += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(acc, s_w, tot);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (base + k < n) s_v[scan_pad(base + k)] = ex;
        ex += v[k];
    }
    __syncthreads();
#pragma unroll 8
    for (int i = threadIdx.x; i < (int)n; i += 1024) out[i] = s_v[scan_pad(i)];
    if (threadIdx.x == 0 && total) *total = tot;
}

// Up to SCAN_MID_BLOCKS tiles: the apply step sums the partial sums of the
// tiles before its own (two launches instead of three).
constexpr int64_t SCAN_MID_BLOCKS = 1024;
__global__ __launch_bounds__(SCAN_BS) void k_scan_apply_mid(const uint32_t* __restrict__ in,
                                                            uint32_t* __restrict__ out, int64_t n,
                                                            const uint32_t* __restrict__ bsum, int64_t nb,
                                                            uint32_t* __restrict__ total) {
    __shared__ uint32_t s_w[SCAN_BS / 64];
    // offset of this tile: sum of the partial sums of the tiles before it
    uint32_t pre = 0, all = 0;
    for (int64_t k = threadIdx.x; k < nb; k += SCAN_BS) {
        const uint32_t x = bsum[k];
        if (k < (int64_t)blockIdx.x) pre += x;
        all += x;
    }
    uint32_t tp, ta;
    block_excl_scan(pre, s_w, tp);
    block_excl_scan(all, s_w, ta);
    if (blockIdx.x == nb - 1 && threadIdx.x == 0 && total) *total = ta;
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    uint32_t v[SCAN_IPT];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        acc += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(acc, s_w, tot) + tp;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
}

size_t scan_tmp_words(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, uint32_t* total,
                          hipStream_t st) {
    if (n <= 0) return total ? fill_u32(total, 1, 0, st) : hipSuccess;
    if (n <= SCAN_SMALL) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, in, out, n, total);
        return hipGetLastError();
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb <= SCAN_MID_BLOCKS) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BS), 0, st, in, n, tmp);
        hipLaunchKernelGGL(k_scan_apply_mid, dim3((unsigned)nb), dim3(SCAN_BS), 0, st, in, out, n, tmp, nb, total);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BS), 0, st, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, tmp, nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_BS), 0, st, in, out, n, tmp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Radix sort (LSD, 8-bit digits)
// ---------------------------------------------------------------------------
constexpr int RS_BS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_BS * RS_ROUNDS;

__global__ __launch_bounds__(1024) void k_rs_hist(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                 uint32_t* __restrict__ hist, int64_t nb) {
    // the block's tile of RS_TILE elements, 1024 threads, all loads in flight
    __shared__ uint32_t h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    uint32_t d[RS_TILE / 1024];
#pragma unroll
    for (int r = 0; r < RS_TILE / 1024; ++r) {
        const int64_t i = base + (int64_t)r * 1024 + threadIdx.x;
        d[r] = i < n ? (uint32_t)(key[i] >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int r = 0; r < RS_TILE / 1024; ++r)
        if (d[r] < 256u) atomicAdd(&h[d[r]], 1u);
    __syncthreads();
    if (threadIdx.x < 256) hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// One pass: the tile of RS_TILE elements of this block is first placed in
// LDS in digit order (stable: within a digit, input order), then written
// out, so that runs of one digit go to consecutive addresses.  offs is the
// scanned histogram: offs[d * nb + b] = first output position of digit d of
// block b; the next entry bounds it, so the block's own digit counts (and
// their local starts) follow from offs alone.  RS_SBS threads take the tile
// in RS_TILE / RS_SBS rounds (the histogram kernel's tiling is the same).
constexpr int RS_SBS = 1024;
constexpr int RS_SROUNDS = RS_TILE / RS_SBS;
constexpr int RS_SW = RS_SBS / 64;
template <bool VALS>
__global__ __launch_bounds__(RS_SBS) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       uint64_t* __restrict__ kout,
                                                       uint32_t* __restrict__ vout, int64_t n, int shift,
                                                       const uint32_t* __restrict__ offs, int64_t nb) {
    __shared__ uint64_t s_k[RS_TILE];
    __shared__ uint32_t s_v[VALS ? RS_TILE : 1];
    __shared__ uint32_t g_off[256];
    __shared__ uint32_t l_off[256];
    __shared__ uint32_t d_base[256];
    __shared__ uint32_t w_cnt[RS_SW][256];
    __shared__ uint32_t w_sum[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t b = blockIdx.x;
    const int64_t base = b * RS_TILE;
    const int tile_n = (int)min((int64_t)RS_TILE, n - base);
    // the whole tile is loaded at once (all loads in flight together)
    uint64_t kr[RS_SROUNDS];
    uint32_t vr[RS_SROUNDS];
#pragma unroll
    for (int r = 0; r < RS_SROUNDS; ++r) {
        const int li = r * RS_SBS + tid;
        kr[r] = li < tile_n ? kin[base + li] : 0;
        vr[r] = (VALS && li < tile_n) ? vin[base + li] : 0;
    }
    // this block's digit counts and their local starts (exclusive scan);
    // threads 0..255 stand for the digits
    uint32_t cnt = 0, inc = 0;
    if (tid < 256) {
        const int64_t oi = (int64_t)tid * nb + b;
        const uint32_t go = offs[oi];
        const uint32_t gnext = oi + 1 < 256 * nb ? offs[oi + 1] : (uint32_t)n;
        cnt = gnext - go;
        inc = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t v = __shfl_up(inc, d, 64);
            if (lane >= d) inc += v;
        }
        if (lane == 63) w_sum[w] = inc;
        g_off[tid] = go;
        d_base[tid] = 0;
    }
    for (int i = tid; i < RS_SW * 256; i += RS_SBS) (&w_cnt[0][0])[i] = 0;
    __syncthreads();
    if (tid < 256) {
        uint32_t before = 0;
        for (int k = 0; k < w; ++k) before += w_sum[k];
        l_off[tid] = before + inc - cnt;
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < RS_SROUNDS; ++r) {
        const int li = r * RS_SBS + tid;
        const bool valid = li < tile_n;
        const uint64_t k = kr[r];
        const uint32_t v = vr[r];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bal = __ballot(valid && ((d >> bit) & 1u));
            match &= ((d >> bit) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = __popcll(match & lt);
        const bool leader = valid && ((match & lt) == 0);
        if (leader) w_cnt[w][d] = (uint32_t)__popcll(match);
        __syncthreads();
        if (tid < 256) {
            uint32_t run = d_base[tid];
            for (int q = 0; q < RS_SW; ++q) {
                const uint32_t c = w_cnt[q][tid];
                w_cnt[q][tid] = run;
                run += c;
            }
            d_base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = l_off[d] + w_cnt[w][d] + rank;
            s_k[pos] = k;
            if (VALS) s_v[pos] = v;
        }
        __syncthreads();
        for (int i = tid; i < RS_SW * 256; i += RS_SBS) (&w_cnt[0][0])[i] = 0;
        __syncthreads();
    }
    // write out in digit order: consecutive threads, consecutive addresses
    // within a digit's run
    for (int i = tid; i < tile_n; i += RS_SBS) {
        const uint64_t k = s_k[i];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t pos = g_off[d] + (uint32_t)i - l_off[d];
        kout[pos] = k;
        if (VALS) vout[pos] = s_v[i];
    }
}

size_t radix_tmp_words(int64_t n) {
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    return (size_t)(256 * nb) + scan_tmp_words(256 * nb) + 8;
}

hipError_t radix_sort(uint64_t* key, uint32_t* val, uint64_t* key_alt, uint32_t* val_alt, int64_t n,
                      int nbits, uint32_t* tmp, hipStream_t st, bool* result_in_alt, int lo_bit) {
    *result_in_alt = false;
    if (n <= 1 || nbits <= 0) return hipSuccess;
    if (lo_bit < 0 || lo_bit + nbits > 64) return hipErrorInvalidValue;
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    uint32_t* hist = tmp;
    uint32_t* stmp = tmp + 256 * nb;
    uint64_t *ka = key, *kb = key_alt;
    uint32_t *va = val, *vb = val_alt;
    for (int shift = lo_bit; shift < lo_bit + nbits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(1024), 0, st, ka, n, shift, hist, nb);
        hipError_t e = exclusive_scan(hist, hist, 256 * nb, stmp, nullptr, st);
        if (e != hipSuccess) return e;
        if (val)
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3((unsigned)nb), dim3(RS_SBS), 0, st, ka, va, kb, vb,
                               n, shift, hist, nb);
        else
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3((unsigned)nb), dim3(RS_SBS), 0, st, ka, va, kb,
                               vb, n, shift, hist, nb);
        std::swap(ka, kb);
        std::swap(va, vb);
        *result_in_alt = !*result_in_alt;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace sph
