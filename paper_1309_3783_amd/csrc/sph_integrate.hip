// Time integration over caller-order arrays: the pieces of a kick-drift-kick
// leapfrog with one step for all particles (the paper's test runs use a
// fixed time step and recompute every force each step, Section III-A), and
// the Courant step limit from the force stage's signal velocities.
// Per-particle streaming kernels: HBM-bound.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "sph_impl.h"

namespace sph {

constexpr int BS = 256;

// v_out = v_in + dt a, u_out = u_in + dt du/dt (in place allowed)
__global__ __launch_bounds__(BS) void k_kick(int64_t n, float dt, const float* vx, const float* vy, const float* vz,
                                             const float* u, const float* __restrict__ ax,
                                             const float* __restrict__ ay, const float* __restrict__ az,
                                             const float* __restrict__ dudt, float* ox, float* oy, float* oz,
                                             float* ou) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    const float a = ax[i], b = ay[i], c = az[i], d = dudt[i];
    ox[i] = fmaf(dt, a, vx[i]);
    oy[i] = fmaf(dt, b, vy[i]);
    oz[i] = fmaf(dt, c, vz[i]);
    ou[i] = fmaf(dt, d, u[i]);
}

__device__ __forceinline__ double wrap_box(double x, double box) {
    x -= box * floor(x / box);
    return x >= box ? x - box : x;   // a value just below zero rounds up to box
}

// x += dt v over particles [p0, p1) of one set, wrapped into [0, box)
__global__ __launch_bounds__(BS) void k_drift(int64_t p0, int64_t p1, double box, double dt, double* x, double* y,
                                              double* z, const float* __restrict__ vx, const float* __restrict__ vy,
                                              const float* __restrict__ vz) {
    const int64_t i = p0 + (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= p1) return;
    x[i] = wrap_box(fma(dt, (double)vx[i], x[i]), box);
    y[i] = wrap_box(fma(dt, (double)vy[i], y[i]), box);
    z[i] = wrap_box(fma(dt, (double)vz[i], z[i]), box);
}

__global__ void k_cfl_init(int32_t* p, int32_t v) { *p = v; }

// min over particles of c h_i / vsig_i into *slot (a positive float's bits
// order like the float, so the minimum is an integer atomicMin); a particle
// without force neighbours (vsig = 0) gives +inf
__global__ __launch_bounds__(BS) void k_cfl(int64_t n, const float* __restrict__ h, const float* __restrict__ vsig,
                                            float c, int32_t* slot) {
    float m = INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        const float v = vsig[i];
        if (v > 0.f) m = fminf(m, c * h[i] / v);
    }
    for (int d = 32; d >= 1; d >>= 1) m = fminf(m, __shfl_xor(m, d, 64));
    __shared__ float s[BS / 64];
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BS / 64; ++w) m = fminf(m, s[w]);
        atomicMin(slot, __float_as_int(m));
    }
}

}  // namespace sph

namespace {

using sph::BS;

unsigned nblk(int64_t n) { return (unsigned)((n + BS - 1) / BS); }

sph_status fail(sph_ctx* ctx, sph_status st, const std::string& msg) {
    if (ctx) ctx->last_error = msg;
    return st;
}

sph_status check_launch(sph_ctx* ctx, const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, SPH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return SPH_OK;
}

}  // namespace

extern "C" {

sph_status sph_kick(sph_ctx* ctx, int64_t n, float dt, const float* vx, const float* vy, const float* vz,
                    const float* u, const float* ax, const float* ay, const float* az, const float* dudt,
                    float* vx_out, float* vy_out, float* vz_out, float* u_out) {
    if (!ctx) return SPH_E_ARG;
    if (n < 0 || !std::isfinite(dt)) return fail(ctx, SPH_E_ARG, "sph_kick: bad n or dt");
    if (n == 0) return SPH_OK;
    if (!vx || !vy || !vz || !u || !ax || !ay || !az || !dudt || !vx_out || !vy_out || !vz_out || !u_out)
        return fail(ctx, SPH_E_ARG, "sph_kick: null pointer");
    hipLaunchKernelGGL(sph::k_kick, dim3(nblk(n)), dim3(BS), 0, ctx->stream, n, dt, vx, vy, vz, u, ax, ay, az, dudt,
                       vx_out, vy_out, vz_out, u_out);
    return check_launch(ctx, "sph_kick");
}

sph_status sph_drift(sph_ctx* ctx, int32_t nsets, const int64_t* offsets, const double* box, double dt, double* x,
                     double* y, double* z, const float* vx, const float* vy, const float* vz) {
    if (!ctx) return SPH_E_ARG;
    if (nsets < 1 || !offsets || !box || !std::isfinite(dt)) return fail(ctx, SPH_E_ARG, "sph_drift: bad arguments");
    if (offsets[0] != 0) return fail(ctx, SPH_E_ARG, "sph_drift: offsets[0] must be 0");
    for (int s = 0; s < nsets; ++s) {
        if (offsets[s + 1] < offsets[s]) return fail(ctx, SPH_E_ARG, "sph_drift: offsets not ascending");
        if (!(box[s] > 0.0) || !std::isfinite(box[s])) return fail(ctx, SPH_E_ARG, "sph_drift: bad box");
    }
    if (offsets[nsets] == 0) return SPH_OK;
    if (!x || !y || !z || !vx || !vy || !vz) return fail(ctx, SPH_E_ARG, "sph_drift: null pointer");
    for (int s = 0; s < nsets; ++s) {
        const int64_t a = offsets[s], b = offsets[s + 1];
        if (a == b) continue;
        hipLaunchKernelGGL(sph::k_drift, dim3(nblk(b - a)), dim3(BS), 0, ctx->stream, a, b, box[s], dt, x, y, z, vx, vy,
                           vz);
    }
    return check_launch(ctx, "sph_drift");
}

sph_status sph_cfl_dt(sph_ctx* ctx, int64_t n, const float* h, const float* vsig, float c_cfl, double* dt) {
    if (!ctx) return SPH_E_ARG;
    if (!dt || n < 0 || !(c_cfl > 0.f)) return fail(ctx, SPH_E_ARG, "sph_cfl_dt: bad arguments");
    *dt = INFINITY;
    if (n == 0) return SPH_OK;
    if (!h || !vsig) return fail(ctx, SPH_E_ARG, "sph_cfl_dt: null pointer");
    int32_t* slot = ctx->d_counter + sph_ctx::CTR_CFL;
    hipLaunchKernelGGL(sph::k_cfl_init, dim3(1), dim3(1), 0, ctx->stream, slot, (int32_t)0x7f800000);   // +inf
    // a few hundred blocks: one same-address atomic per block, and those
    // serialise (~25 ns each)
    const unsigned g = std::min<unsigned>(nblk(n), 256u);
    hipLaunchKernelGGL(sph::k_cfl, dim3(g), dim3(BS), 0, ctx->stream, n, h, vsig, c_cfl, slot);
    sph_status st = check_launch(ctx, "sph_cfl_dt");
    if (st != SPH_OK) return st;
    hipError_t e = hipMemcpyAsync(ctx->h_pin, slot, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, SPH_E_HIP, std::string("sph_cfl_dt: ") + hipGetErrorString(e));
    int32_t bits;
    std::memcpy(&bits, ctx->h_pin, sizeof(bits));
    float m;
    std::memcpy(&m, &bits, sizeof(m));
    *dt = (double)m;
    return SPH_OK;
}

}  // extern "C"
