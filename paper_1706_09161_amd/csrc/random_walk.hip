// random_walk.hip -- the paper's Levy-stable random walk on the GPU (Sec. 3.1,
// equations (RW_STABLE) and (distri); killed at the first exit from the box),
// the statistical counterpart of the LB solution: the density of the
// surviving particles solves the FADE with homogeneous Dirichlet walls.
//
// One thread per particle keeps its position in registers for the whole run
// and draws, per step and axis, two uniforms from Philox-4x32-10 (Salmon,
// Moraes, Dror, Shaw, SC 2011: ten rounds of two 32 x 32 -> 64-bit products
// by 0xD2511F53 and 0xCD9E8D57 mixed with the other counter words and the
// key, the key bumped by 0x9E3779B9 / 0xBB67AE85 between rounds) at the
// counter (particle low word, particle high word, step, purpose) under the
// 64-bit seed, so a path does not depend on the launch shape.  The stable
// variable S(alpha, beta) comes from Weron's formula (after Chambers, Mallows
// and Stuck), beta = 2 p - 1:
//   V = pi (u1 - 1/2), W = -log u2,
//   S = Sc sin(alpha (V + B)) / cos(V)^(1/alpha) (cos(V - alpha (V + B)) / W)^((1 - alpha)/alpha),
// with t = beta tan(pi alpha / 2), B = atan(t) / alpha, Sc = (1 + t^2)^(1/(2 alpha)),
// and the step is X_mu += u_mu dt + (D_mumu g_mu)^(1/alpha) (-cos(pi alpha/2) dt)^(1/alpha) S.
// A particle whose position is not strictly inside the box after a step is
// killed.  Everything is FP64 with contraction into FMA switched off: the
// exit and binning decisions are taken in FP64 with the same operation order
// as a plain CPU evaluation of these formulas.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/lbm_fade.h"
#include "lbm_internal.h"

namespace {

struct RwConsts {
    int dim;
    double lo[3], hi[3];
    double alpha[3], inv_alpha[3], expo[3];  // 1 / alpha, (1 - alpha) / alpha
    double B[3], Sc[3];                       // Weron's shift and scale of S(alpha, beta)
    double scale[3], udt[3];                  // step: udt + scale S
    uint32_t key0, key1;
};

constexpr uint32_t kPurposeStep = 0u;  // + axis
constexpr uint32_t kPurposeInit = 8u;  // + axis

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// uniform in (0, 1): (k + 1/2) 2^-53, k = top 27 bits of a, top 26 bits of b
__device__ __forceinline__ double u53(uint32_t a, uint32_t b)
{
    const uint64_t k = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)k + 0.5) * 0x1p-53;
}

__device__ __forceinline__ void draw2(const RwConsts& K, int64_t particle, uint32_t step, uint32_t purpose, double& u1,
                                      double& u2)
{
    uint32_t c0 = (uint32_t)(uint64_t)particle, c1 = (uint32_t)((uint64_t)particle >> 32), c2 = step, c3 = purpose;
    philox4x32_10(c0, c1, c2, c3, K.key0, K.key1);
    u1 = u53(c0, c1);
    u2 = u53(c2, c3);
}

__device__ __forceinline__ double stable(const RwConsts& K, int mu, double u1, double u2)
{
#pragma clang fp contract(off)
    const double a = K.alpha[mu];
    const double V = 3.14159265358979323846 * (u1 - 0.5);
    const double W = -log(u2);
    const double VB = V + K.B[mu];
    return K.Sc[mu] * sin(a * VB) / pow(cos(V), K.inv_alpha[mu]) * pow(cos(V - a * VB) / W, K.expo[mu]);
}

__device__ __forceinline__ bool inside(const RwConsts& K, const double (&x)[3])
{
    bool in = true;
    for (int mu = 0; mu < K.dim; ++mu) in = in && (x[mu] > K.lo[mu] && x[mu] < K.hi[mu]);
    return in;
}

__global__ __launch_bounds__(256) void rw_init_kernel(RwConsts K, double c0, double c1, double c2, double sigma0,
                                                      int64_t n, int64_t first, double* __restrict__ x,
                                                      uint8_t* __restrict__ alive)
{
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double c[3] = {c0, c1, c2};
    double p[3] = {0.0, 0.0, 0.0};
    for (int mu = 0; mu < K.dim; ++mu) {
        double u1, u2;
        draw2(K, first + k, 0u, kPurposeInit + (uint32_t)mu, u1, u2);
        p[mu] = c[mu] + sigma0 * sqrt(-2.0 * log(u2)) * cos(2.0 * 3.14159265358979323846 * u1);
        x[mu * n + k] = p[mu];
    }
    alive[k] = inside(K, p) ? 1 : 0;
}

template <int DIM>
__global__ __launch_bounds__(256) void rw_walk_kernel(RwConsts K, double* __restrict__ x,
                                                      uint8_t* __restrict__ alive, int64_t n, int64_t first,
                                                      uint32_t step0, uint32_t nsteps)
{
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (!alive[k]) return;
    double p[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int mu = 0; mu < DIM; ++mu) p[mu] = x[mu * n + k];
    bool live = true;
    for (uint32_t i = 0; i < nsteps; ++i) {
        const uint32_t s = step0 + 1 + i;
#pragma unroll
        for (int mu = 0; mu < DIM; ++mu) {
            double u1, u2;
            draw2(K, first + k, s, kPurposeStep + (uint32_t)mu, u1, u2);
            const double S = stable(K, mu, u1, u2);
            p[mu] += K.udt[mu] + K.scale[mu] * S;
        }
        bool in = true;
#pragma unroll
        for (int mu = 0; mu < DIM; ++mu) in = in && (p[mu] > K.lo[mu] && p[mu] < K.hi[mu]);
        if (!in) {
            live = false;
            break;
        }
    }
#pragma unroll
    for (int mu = 0; mu < DIM; ++mu) x[mu * n + k] = p[mu];
    if (!live) alive[k] = 0;
}

__global__ __launch_bounds__(256) void rw_fill_u32(uint32_t* __restrict__ p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

__global__ __launch_bounds__(256) void rw_hist_kernel(RwConsts K, const double* __restrict__ x,
                                                      const uint8_t* __restrict__ alive, int64_t n, int n0, int n1,
                                                      int n2, double dx, uint32_t* __restrict__ counts)
{
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !alive[k]) return;
    const int nn[3] = {n0, n1, n2};
    int64_t idx = 0, mul = 1;
    bool ok = true;
    for (int mu = 0; mu < K.dim; ++mu) {
        const double j = floor((x[mu * n + k] - K.lo[mu]) / dx + 0.5);
        ok = ok && j >= 0.0 && j < (double)nn[mu];
        idx += (ok ? (int64_t)j : 0) * mul;
        mul *= nn[mu];
    }
    if (ok) atomicAdd(&counts[idx], 1u);
}

int rw_fail(int code, const char* msg) { return lbm::set_error(code, msg); }

int make_consts(const lbm_rw_params* P, RwConsts& K)
{
    if (!P) return rw_fail(LBM_EINVAL, "null parameters");
    if (P->dim < 1 || P->dim > 3) return rw_fail(LBM_EINVAL, "dim must be 1, 2 or 3");
    if (!(P->dt > 0.0) || !isfinite(P->dt)) return rw_fail(LBM_EINVAL, "dt must be > 0");
    K = RwConsts{};
    K.dim = P->dim;
    for (int mu = 0; mu < P->dim; ++mu) {
        const double a = P->alpha[mu];
        if (!(a > 1.0 && a <= 2.0)) return rw_fail(LBM_EINVAL, "alpha must lie in (1, 2]");
        if (!(P->p[mu] >= 0.0 && P->p[mu] <= 1.0)) return rw_fail(LBM_EINVAL, "p must lie in [0, 1]");
        if (!(P->D[mu] >= 0.0) || !(P->g[mu] > 0.0) || !isfinite(P->D[mu]) || !isfinite(P->g[mu]))
            return rw_fail(LBM_EINVAL, "need D >= 0 and g > 0");
        if (!(P->lo[mu] < P->hi[mu])) return rw_fail(LBM_EINVAL, "need lo < hi");
        if (!isfinite(P->u[mu])) return rw_fail(LBM_EINVAL, "u must be finite");
        const double beta = 2.0 * P->p[mu] - 1.0;
        const double t = beta * tan(3.14159265358979323846 * a / 2.0);
        K.lo[mu] = P->lo[mu];
        K.hi[mu] = P->hi[mu];
        K.alpha[mu] = a;
        K.inv_alpha[mu] = 1.0 / a;
        K.expo[mu] = (1.0 - a) / a;
        K.B[mu] = atan(t) / a;
        K.Sc[mu] = pow(1.0 + t * t, 1.0 / (2.0 * a));
        K.scale[mu] = pow(P->D[mu] * P->g[mu], 1.0 / a) * pow(-cos(3.14159265358979323846 * a / 2.0) * P->dt, 1.0 / a);
        K.udt[mu] = P->u[mu] * P->dt;
    }
    K.key0 = (uint32_t)P->seed;
    K.key1 = (uint32_t)(P->seed >> 32);
    return LBM_OK;
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

int lbm_rw_init_gaussian(const lbm_rw_params* P, const double* center, double sigma0, int64_t n, int64_t first,
                         double* x, uint8_t* alive, void* stream)
{
    RwConsts K;
    int rc = make_consts(P, K);
    if (rc) return rc;
    if (!center || (n > 0 && (!x || !alive))) return rw_fail(LBM_EINVAL, "null argument");
    if (n < 0 || first < 0 || !(sigma0 >= 0.0)) return rw_fail(LBM_EINVAL, "need n >= 0, first >= 0, sigma0 >= 0");
    if (n > ((int64_t)1 << 40)) return rw_fail(LBM_EINVAL, "too many particles");
    if (n == 0) return LBM_OK;
    const double c[3] = {center[0], P->dim > 1 ? center[1] : 0.0, P->dim > 2 ? center[2] : 0.0};
    hipLaunchKernelGGL(rw_init_kernel, dim3(blocks_of(n)), dim3(256), 0, (hipStream_t)stream, K, c[0], c[1], c[2],
                       sigma0, n, first, x, alive);
    return hipGetLastError() == hipSuccess ? LBM_OK : rw_fail(LBM_EDEVICE, "launch of the initial-position kernel failed");
}

int lbm_rw_walk(const lbm_rw_params* P, double* x, uint8_t* alive, int64_t n, int64_t first, int64_t step0,
                int64_t nsteps, void* stream)
{
    RwConsts K;
    int rc = make_consts(P, K);
    if (rc) return rc;
    if (n > 0 && (!x || !alive)) return rw_fail(LBM_EINVAL, "null argument");
    if (n < 0 || first < 0 || step0 < 0 || nsteps < 0 || step0 + nsteps > 0xFFFFFFFFll)
        return rw_fail(LBM_EINVAL, "need n, first, step0, nsteps >= 0 and step0 + nsteps < 2^32");
    if (n > ((int64_t)1 << 40)) return rw_fail(LBM_EINVAL, "too many particles");
    if (n == 0 || nsteps == 0) return LBM_OK;
    hipStream_t s = (hipStream_t)stream;
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(blocks_of(n)), dim3(256), 0, s, K, x, alive, n, first, (uint32_t)step0,
                           (uint32_t)nsteps);
    };
    if (P->dim == 1) go(rw_walk_kernel<1>);
    else if (P->dim == 2) go(rw_walk_kernel<2>);
    else go(rw_walk_kernel<3>);
    return hipGetLastError() == hipSuccess ? LBM_OK : rw_fail(LBM_EDEVICE, "launch of the walk kernel failed");
}

int lbm_rw_histogram(const lbm_rw_params* P, const double* x, const uint8_t* alive, int64_t n, const int32_t* nodes,
                     double dx, uint32_t* counts, void* stream)
{
    RwConsts K;
    int rc = make_consts(P, K);
    if (rc) return rc;
    if (!nodes || !counts || (n > 0 && (!x || !alive))) return rw_fail(LBM_EINVAL, "null argument");
    if (n < 0 || !(dx > 0.0)) return rw_fail(LBM_EINVAL, "need n >= 0 and dx > 0");
    int64_t total = 1;
    int nn[3] = {1, 1, 1};
    for (int mu = 0; mu < P->dim; ++mu) {
        if (nodes[mu] < 1) return rw_fail(LBM_EINVAL, "need nodes >= 1 on every axis");
        nn[mu] = nodes[mu];
        total *= nodes[mu];
    }
    if (total > ((int64_t)1 << 34)) return rw_fail(LBM_EINVAL, "histogram too large");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(rw_fill_u32, dim3(blocks_of(total)), dim3(256), 0, s, counts, total);
    if (n > 0)
        hipLaunchKernelGGL(rw_hist_kernel, dim3(blocks_of(n)), dim3(256), 0, s, K, x, alive, n, nn[0], nn[1], nn[2],
                           dx, counts);
    return hipGetLastError() == hipSuccess ? LBM_OK : rw_fail(LBM_EDEVICE, "launch of the histogram kernel failed");
}

}  // extern "C"
