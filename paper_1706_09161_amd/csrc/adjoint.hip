// adjoint.hip -- vector-Jacobian product of n time steps (the paper has no
// adjoint; this is the reverse of the step of Algorithm 1 as implemented in
// collide_stream.hip and fractional_gemm.hip).
//
// For L = <gC, C_n> the reverse sweep carries fbar = dL/df^t:
//   Dirichlet rule + streaming, reversed: fbar*_i(y) = g_i(y + e_i) with
//       g_i(x) = fbar_i(x) - mean_{b unknown at x} fbar_b(x)  (0 if y + e_i is outside);
//   collision f* = f - R (f - f^eq) + w S dt, reversed:
//       fbar^eq = R^T fbar*,  fbar += fbar* - R^T fbar*,  dL/dS += dt <w, fbar*>,
//       dL/dR += fbar* (f^eq - f)^T;
//   equilibrium (Feq), (CoeffA) reversed: Cbar, Phibar_mu, dL/du_mu;
//   fractional term reversed: with K_mu = s (p W+ + (1 - p) W-) + boundary
//       columns (W+ the lower, W- the upper Toeplitz sums of the weights, unit
//       diagonal), the two triangular products U = s W+^T Phibar_mu and
//       L = s W-^T Phibar_mu (one GEMM's worth of MFMA work for the pair) give
//       Cbar += K_mu^T Phibar_mu = p U + (1 - p) L and
//       dL/dp_mu += <Phibar_mu, (dK_mu/dp_mu) C> = <U - L, C> + the boundary
//       columns' p-derivatives against C at the line's two walls;
//   moment reversed: fbar_i += Cbar.
// The transposed products omit the two boundary ROWS of K^T: they only add to
// Cbar at wall nodes, whose broadcast into fbar is cancelled exactly by the
// reversed Dirichlet rule (and by the reversed initial equilibrium, whose
// weights satisfy w0 = 2 w), so no gradient depends on them.
//
// Forward states are stored every ckpt_every steps; each segment is
// recomputed (populations, C and Phi of every step kept) and swept in
// reverse.  Field gradients accumulate in FP32; the scalar gradients are
// reduced in FP64 (per-workgroup partial sums, then a fixed-order sum), and
// the chain R -> Lambda -> lambda-bar -> D is applied on the host in FP64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "lbm_handle.h"

namespace lbm {

namespace {

constexpr int kBlock = 256;

struct AdjConsts {
    int dim, Q;
    int n[3];
    float w[kMaxQ];
    float adv[3];            // (dt/dx) u_mu w / e^2
    float uscale;            // (dt/dx) w / e^2
    float R[kMaxQ * kMaxQ];  // collision matrix, row-major
    float wdt[kMaxQ];        // w_i dt
};

// One 64-bit value moved between lanes by a DPP control (both halves alike);
// lanes of the rows outside ROWS get 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int lo = __double2loint(x), hi = __double2hiint(x);
    const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xF, false);
    const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xF, false);
    return __hiloint2double(h2, l2);
}

__device__ __forceinline__ double readlane_f64(double x, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// FP64 sum over the 64 lanes of a wavefront, taken from lane 63: rotations by
// 8, 4, 2 and 1 lanes inside each row of 16 (DPP row_ror; every source lane
// exists) leave each row's sum in its lanes; row_bcast:15 then adds row 0's sum
// into row 1 and row 2's into row 3, and row_bcast:31 adds that of rows 0-1
// (lane 31) into rows 2-3.  Fixed order, no LDS traffic.
__device__ __forceinline__ double wave_sum_f64(double x)
{
    x += dpp_f64<0x128>(x);       // row_ror:8
    x += dpp_f64<0x124>(x);       // row_ror:4
    x += dpp_f64<0x122>(x);       // row_ror:2
    x += dpp_f64<0x121>(x);       // row_ror:1
    x += dpp_f64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_f64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return readlane_f64(x, 63);
}

// Sum `v` over the workgroup in FP64 (fixed order) into out[0..NV): stored, or
// (ACC) added to what the slot holds (the workgroup's running sum over steps).
// Every thread of the workgroup must call it (the lane exchanges read all 64
// lanes).
template <int NV, bool ACC = false>
__device__ inline void block_sum_store(double (&v)[NV], double* __restrict__ out)
{
    __shared__ double sh[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double x = wave_sum_f64(v[k]);
        if (lane == 0) sh[wave][k] = x;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NV; k += kBlock) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += sh[w][k];
        out[k] = ACC ? out[k] + s : s;
    }
}

// fbar_i(x) = gC(x) for every population (L = <gC, sum_i f_i>)
__global__ void broadcast_kernel(const float* __restrict__ gC, float* __restrict__ fbar, int Q, int64_t nodes)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nodes) return;
    const float g = gC[x];
    for (int i = 0; i < Q; ++i) fbar[i * nodes + x] = g;
}

// The reversed fractional term of every axis at node x: returns
// sum_mu K_mu^T Phibar_mu = sum_mu (p U + (1 - p) L), and sets red[mu] to the
// node's part of <Phibar_mu, (dK_mu/dp) C>: (U - L)(x) C(x) plus
// Phibar_mu(x) (dc0_j C(x_0) + dcN_j C(x_N)), j = x's index along the line
// and x_0, x_N the line's wall nodes (the p-derivatives of the boundary
// columns).
struct RevConsts {
    int n[3];
    int64_t stride[3];
    float p[3];
    const float* dc0[3];
    const float* dcN[3];
};

// sum_mu K_mu^T Phibar_mu at node x from the two triangular products
template <int D>
__device__ inline float kt_at(const RevConsts& rc, const float* __restrict__ tu, const float* __restrict__ tl,
                              int64_t x, int64_t nodes)
{
    float kt = 0.f;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const float u = tu[mu * nodes + x], l = tl[mu * nodes + x];
        kt += fmaf(rc.p[mu], u - l, l);
    }
    return kt;
}

// red[mu] = the node's part of <Phibar_mu, (dK_mu/dp_mu) C> (x at grid coordinates c)
template <int D>
__device__ inline void p_terms(const RevConsts& rc, const float* __restrict__ tu, const float* __restrict__ tl,
                               const float* __restrict__ phibar, const float* __restrict__ C, int64_t x,
                               const int (&c)[3], int64_t nodes, double* red)
{
    const double Cx = (double)C[x];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const float u = tu[mu * nodes + x], l = tl[mu * nodes + x];
        const int j = c[mu], N = rc.n[mu] - 1;
        const double walls = (double)rc.dc0[mu][j] * (double)C[x - (int64_t)j * rc.stride[mu]] +
                             (double)rc.dcN[mu][j] * (double)C[x + (int64_t)(N - j) * rc.stride[mu]];
        red[mu] = ((double)u - (double)l) * Cx + (double)phibar[mu * nodes + x] * walls;
    }
}

template <int D>
__device__ inline float reversed_fractional(const RevConsts& rc, const float* __restrict__ tu,
                                            const float* __restrict__ tl, const float* __restrict__ phibar,
                                            const float* __restrict__ C, int64_t x, int64_t nodes, double (&red)[D])
{
    int c[3] = {0, 0, 0};
    c[0] = (int)(x % rc.n[0]);
    const int64_t r = x / rc.n[0];
    c[1] = (int)(r % rc.n[1]);
    c[2] = (int)(r / rc.n[1]);
    p_terms<D>(rc, tu, tl, phibar, C, x, c, nodes, red);
    return kt_at<D>(rc, tu, tl, x, nodes);
}

// Reverse of one step at every node (streaming + Dirichlet rule, collision,
// equilibrium).  Writes fdir (the part of fbar^t that does not go through C),
// Cbar (equilibrium part), Phibar, adds to dS, and per-workgroup FP64 partial
// sums of
//   the flux block of dL/dLambda: sum_x mbar_a(x) mdev_b(x), a, b < d, with
//     mbar = M^-T fbar* (flux rows: (fbar*_{2a+1} - fbar*_{2a+2}) / 2) and
//     mdev = M (f^eq - f) (flux rows: dev_{2b+1} - dev_{2b+2}),
//     which is all of dL/dR = fbar* (f^eq - f)^T that reaches D
//     (dL/dLambda = M^-T (dL/dR) M^T; only the flux block of Lambda depends on D);
//   dL/du_mu (d values);
//   tr dL/dR = sum_i fbar*_i (f^eq_i - f_i) (BGK: R = I / lambda).
// FUSED: fbar of the later step is not stored but formed where it is read,
// fbar_i(y) = fdir'_i(y) + Cbar'(y) + sum_mu K_mu^T Phibar'_mu(y) (the moment
// reversed; primes: that step's fields, the K^T products in tu / tl), and
// the later step's p-gradient terms <Phibar'_mu, (dK_mu/dp_mu) C'> at x are
// summed too (slots NV .. NV + d); otherwise fbar is read (the first step of
// the sweep) and those slots add zero.
// Grid: x across threads, y and z across workgroups (no integer division).
struct LaterStep {
    const float* fbar;    // !FUSED
    const float* fdir;    // FUSED: fields of the later step
    const float* cbar;
    const float* phibar;
    const float* tu;
    const float* tl;
    const float* C;
};

template <int Q, bool FUSED>
__global__ __launch_bounds__(kBlock) void adjoint_node(AdjConsts ac, RevConsts rc, LaterStep ls,
                                                       const float* __restrict__ f, const float* __restrict__ Phi,
                                                       float* __restrict__ fdir, float* __restrict__ cbar,
                                                       float* __restrict__ phibar, float* __restrict__ dS,
                                                       double* __restrict__ part, int64_t nodes)
{
    constexpr int d = (Q - 1) / 2;
    constexpr int NV = d * d + d + 1;
    const int c[3] = {(int)(blockIdx.x * kBlock + threadIdx.x), (int)blockIdx.y, (int)blockIdx.z};
    const int64_t x = ((int64_t)c[2] * ac.n[1] + c[1]) * ac.n[0] + c[0];
    double red[NV + d];
#pragma unroll
    for (int k = 0; k < NV + d; ++k) red[k] = 0.0;
    if (c[0] < ac.n[0]) {
        if (FUSED) p_terms<d>(rc, ls.tu, ls.tl, ls.phibar, ls.C, x, c, nodes, red + NV);
        // adjoint of f*(x): pulled from the node each population moved to
        float fsb[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int y[3] = {c[0], c[1], c[2]};
            if (i > 0) y[(i - 1) / 2] += ((i - 1) & 1) ? -1 : 1;
            bool inside = true;
#pragma unroll
            for (int mu = 0; mu < d; ++mu) inside = inside && y[mu] >= 0 && y[mu] < ac.n[mu];
            if (!inside) {
                fsb[i] = 0.f;
                continue;
            }
            const int64_t yi = ((int64_t)y[2] * ac.n[1] + y[1]) * ac.n[0] + y[0];
            const float cy = FUSED ? ls.cbar[yi] + kt_at<d>(rc, ls.tu, ls.tl, yi, nodes) : 0.f;
            auto fbar_at = [&](int b) {
                return FUSED ? ls.fdir[(int64_t)b * nodes + yi] + cy : ls.fbar[(int64_t)b * nodes + yi];
            };
            float g = fbar_at(i);
            // unknown populations at y (their sources lie outside) share its Dirichlet deficit
            int cnt = 0;
            float sum = 0.f;
#pragma unroll
            for (int b = 1; b < Q; ++b) {
                const int mu = (b - 1) / 2;
                const int src = y[mu] - (((b - 1) & 1) ? -1 : 1);
                if (src < 0 || src >= ac.n[mu]) {
                    ++cnt;
                    sum += fbar_at(b);
                }
            }
            if (cnt > 0) g -= sum / (float)cnt;
            fsb[i] = g;
        }
        // forward quantities at x
        float fx[Q], phi[d], C = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            fx[i] = f[(int64_t)i * nodes + x];
            C += fx[i];
        }
        float sphi = 0.f;
#pragma unroll
        for (int mu = 0; mu < d; ++mu) {
            phi[mu] = Phi[(int64_t)mu * nodes + x];
            sphi += phi[mu];
        }
        float feq[Q];
        feq[0] = C - ac.w[0] * sphi;
#pragma unroll
        for (int mu = 0; mu < d; ++mu) {
            const float a = ac.w[2 * mu + 1] * phi[mu];
            const float b = ac.adv[mu] * C;
            feq[2 * mu + 1] = a + b;
            feq[2 * mu + 2] = a - b;
        }
        // collision reversed
        float feqbar[Q];
        float sb = 0.f;
        double tr = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            float r = 0.f;
#pragma unroll
            for (int j = 0; j < Q; ++j) r = fmaf(ac.R[j * Q + i], fsb[j], r);
            feqbar[i] = r;
            fdir[(int64_t)i * nodes + x] = fsb[i] - r;
            sb = fmaf(ac.wdt[i], fsb[i], sb);
            tr += (double)fsb[i] * (double)(feq[i] - fx[i]);
        }
        dS[x] += sb;
#pragma unroll
        for (int a = 0; a < d; ++a) {
            const double mb = 0.5 * ((double)fsb[2 * a + 1] - (double)fsb[2 * a + 2]);
#pragma unroll
            for (int b = 0; b < d; ++b) {
                const double md = (double)(feq[2 * b + 1] - fx[2 * b + 1]) - (double)(feq[2 * b + 2] - fx[2 * b + 2]);
                red[a * d + b] = mb * md;
            }
        }
        // equilibrium reversed
        float cb = feqbar[0];
#pragma unroll
        for (int mu = 0; mu < d; ++mu) {
            const float dp = feqbar[2 * mu + 1], dm = feqbar[2 * mu + 2];
            cb = fmaf(ac.adv[mu], dp - dm, cb);
            phibar[(int64_t)mu * nodes + x] = -ac.w[0] * feqbar[0] + ac.w[2 * mu + 1] * (dp + dm);
            red[d * d + mu] = (double)ac.uscale * (double)C * (double)(dp - dm);
        }
        red[d * d + d] = tr;
        cbar[x] = cb;
    }
    const int64_t blk = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_sum_store<NV + d, true>(red, part + blk * (NV + d));  // running sum over the reverse sweep
}

// Reverse of the initial equilibrium f^0 = f^eq(C0', Phi(C0')): fbar^0 is the
// adjoint of f^eq.  Writes Cbar (equilibrium part), Phibar and partial sums of dL/du.
template <int Q>
__global__ __launch_bounds__(kBlock) void adjoint_init_node(AdjConsts ac, const float* __restrict__ fbar,
                                                            const float* __restrict__ C0, float* __restrict__ cbar,
                                                            float* __restrict__ phibar, double* __restrict__ part,
                                                            int64_t nodes)
{
    constexpr int d = (Q - 1) / 2;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double red[d];
#pragma unroll
    for (int k = 0; k < d; ++k) red[k] = 0.0;
    if (x < nodes) {
        float fb[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) fb[i] = fbar[(int64_t)i * nodes + x];
        const float C = C0[x];
        float cb = fb[0];
#pragma unroll
        for (int mu = 0; mu < d; ++mu) {
            const float dp = fb[2 * mu + 1], dm = fb[2 * mu + 2];
            cb = fmaf(ac.adv[mu], dp - dm, cb);
            phibar[(int64_t)mu * nodes + x] = -ac.w[0] * fb[0] + ac.w[2 * mu + 1] * (dp + dm);
            red[mu] = (double)ac.uscale * (double)C * (double)(dp - dm);
        }
        cbar[x] = cb;
    }
    block_sum_store<d>(red, part + (int64_t)blockIdx.x * d);
}

// acc[off + v] += sum over workgroups b of part[b * nv + v], fixed order
__global__ __launch_bounds__(kBlock) void reduce_partials(const double* __restrict__ part, int64_t nblocks, int nv,
                                                          double* __restrict__ acc, int off)
{
    __shared__ double sh[kBlock];
    const int v = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += kBlock) s += part[b * nv + v];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[off + v] += sh[0];
}

// fbar_i = fdir_i + Cbar + sum_mu K_mu^T Phibar_mu, and the per-workgroup FP64
// running sums of <Phibar_mu, (dK_mu/dp_mu) C>
template <int D>
__global__ __launch_bounds__(kBlock) void combine_dot(RevConsts rc, const float* __restrict__ fdir,
                                                      const float* __restrict__ cbar, const float* __restrict__ tu,
                                                      const float* __restrict__ tl, const float* __restrict__ phibar,
                                                      const float* __restrict__ C, float* __restrict__ fbar, int Q,
                                                      double* __restrict__ part, int64_t nodes)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double red[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) red[mu] = 0.0;
    if (x < nodes) {
        const float c = cbar[x] + reversed_fractional<D>(rc, tu, tl, phibar, C, x, nodes, red);
        for (int i = 0; i < Q; ++i) fbar[i * nodes + x] = fdir[i * nodes + x] + c;
    }
    block_sum_store<D, true>(red, part + (int64_t)blockIdx.x * D);  // running sum over the reverse sweep
}

// Reversed fractional term of the initial equilibrium: per-workgroup FP64
// sums of <Phibar_mu, (dK_mu/dp_mu) C0'>, and (when dC0 is given)
// dC0 = Cbar + sum_mu K_mu^T Phibar_mu, zero on the (overwritten) wall nodes
template <int D>
__global__ __launch_bounds__(kBlock) void combine_init(RevConsts rc, const float* __restrict__ cbar,
                                                       const float* __restrict__ tu, const float* __restrict__ tl,
                                                       const float* __restrict__ phibar, const float* __restrict__ C,
                                                       float* __restrict__ dC0, double* __restrict__ part,
                                                       int64_t nodes)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double red[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) red[mu] = 0.0;
    if (x < nodes) {
        const float v = cbar[x] + reversed_fractional<D>(rc, tu, tl, phibar, C, x, nodes, red);
        if (dC0) {
            bool wall = false;
            int64_t r = x;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
                const int c = (int)(r % rc.n[mu]);
                r /= rc.n[mu];
                wall = wall || c == 0 || c == rc.n[mu] - 1;
            }
            dC0[x] = wall ? 0.f : v;
        }
    }
    block_sum_store<D>(red, part + (int64_t)blockIdx.x * D);
}

unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

struct AdjointState {
    int64_t nodes = 0;
    int K = 0;           // checkpoint interval the buffers were sized for
    int64_t nseg = 0;    // checkpoints allocated
    float* ckpt = nullptr;
    // recomputed segments, double-buffered (nbuf = 2) when both fit, so that
    // the next segment's recompute runs on a side stream during this
    // segment's reverse sweep
    int nbuf = 0;
    float* seg_f[2] = {nullptr, nullptr};    // (K+1) slots of Q * nodes; slot 0 unused (the checkpoint is read directly)
    float* seg_phi[2] = {nullptr, nullptr};  // K slots of d * nodes
    float* seg_C[2] = {nullptr, nullptr};    // K slots of nodes
    hipStream_t side = nullptr;              // default priority, non-blocking
    hipEvent_t ev_fwd = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
    float* fbar = nullptr;
    // fdir, Cbar and Phibar of a step, two sets (by step parity): the kernel
    // of step t reads step t + 1's set at neighbouring nodes
    float* fdir = nullptr;
    float* cbar = nullptr;
    float* phibar = nullptr;
    float* fdir2 = nullptr;
    float* cbar2 = nullptr;
    float* phibar2 = nullptr;
    float* Ckeep = nullptr;  // C of the first step of the segment swept last
    float* tu = nullptr;  // s W+^T Phibar_mu (d fields)
    float* tl = nullptr;  // s W-^T Phibar_mu (d fields)
    float* dS = nullptr;
    double* part = nullptr;   // per-workgroup partial sums of adjoint_node
    double* part2 = nullptr;  // per-workgroup partial sums of the p-gradient
    double* acc = nullptr;
    void* opmem = nullptr;
    AxisOp opsU[3], opsL[3];
    RevConsts rc;
};

void adjoint_free(AdjointState* a)
{
    if (!a) return;
    void* ptrs[] = {a->ckpt, a->seg_f[0], a->seg_phi[0], a->seg_C[0], a->seg_f[1], a->seg_phi[1], a->seg_C[1],
                    a->fbar, a->fdir, a->cbar, a->phibar, a->fdir2, a->cbar2, a->phibar2, a->Ckeep,
                    a->tu, a->tl, a->dS, a->part, a->part2, a->acc, a->opmem};
    for (void* p : ptrs) (void)hipFree(p);
    hipEvent_t evs[] = {a->ev_fwd, a->ev_rec[0], a->ev_rec[1], a->ev_rev[0], a->ev_rev[1]};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    if (a->side) (void)hipStreamDestroy(a->side);
    delete a;
}

namespace {

// Build, per axis, the two triangular products of the reversed fractional
// term (generators of s W+^T and s W-^T, no boundary columns) and the
// p-derivatives of the forward operator's two boundary columns (FP64, then
// FP32).
bool build_ops(lbm_fade* h, AdjointState* A)
{
    const int d = h->dim;
    auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t bytes = 0;
    for (int mu = 0; mu < d; ++mu) {
        const size_t n = (size_t)h->grid.n[mu];
        bytes += 2 * r256(sizeof(float) * (2 * n - 1)) + 3 * r256(sizeof(float) * n);
    }
    std::vector<unsigned char> host(bytes, 0);
    if (hipMalloc(&A->opmem, bytes) != hipSuccess) return false;
    size_t off = 0;
    auto carve = [&](size_t nb) {
        size_t o = off;
        off += r256(nb);
        return o;
    };
    unsigned char* base = reinterpret_cast<unsigned char*>(A->opmem);
    RevConsts& rc = A->rc;
    memset(&rc, 0, sizeof(rc));
    for (int mu = 0; mu < 3; ++mu) rc.n[mu] = h->cc.n[mu];
    rc.stride[0] = 1;
    rc.stride[1] = h->cc.n[0];
    rc.stride[2] = (int64_t)h->cc.n[0] * h->cc.n[1];
    for (int mu = 0; mu < d; ++mu) {
        const int n = h->grid.n[mu], N = n - 1;
        const AxisCoeffs C = axis_coeffs(n, 2.0 - h->params.alpha[mu], h->params.g[mu], h->grid.dx);
        const double s = C.s;
        const size_t oU = carve(sizeof(float) * (2 * n - 1)), oL = carve(sizeof(float) * (2 * n - 1));
        const size_t oZ = carve(sizeof(float) * n);
        const size_t o0 = carve(sizeof(float) * n), oN = carve(sizeof(float) * n);
        float* gU = reinterpret_cast<float*>(host.data() + oU);
        float* gL = reinterpret_cast<float*>(host.data() + oL);
        float* pc0 = reinterpret_cast<float*>(host.data() + o0);
        float* pcN = reinterpret_cast<float*>(host.data() + oN);
        // generator index dd = j - k (output j, input k): W+ holds a_{j-k} for
        // j >= k, so s W+^T holds s a_{k-j} for j <= k (upper); W- holds
        // a_{k-j} for j <= k, so s W-^T holds s a_{j-k} for j >= k (lower)
        for (int dd = -N; dd <= N; ++dd) {
            gU[dd + N] = dd <= 0 ? (float)(s * C.a[-dd]) : 0.f;
            gL[dd + N] = dd >= 0 ? (float)(s * C.a[dd]) : 0.f;
        }
        // p-derivatives of the boundary corrections K[j][0] - T(j) and
        // K[j][N] - T(j - N) (the transposed Toeplitz parts U and L span every
        // column, the end columns included)
        {
            const double gm = 2.0 - h->params.alpha[mu];
            const double empty = pow(0.0, gm);  // c+_{00} = c-_{NN}
            std::vector<double> d0(n, 0.0), dN(n, 0.0);
            for (int j = 1; j <= N; ++j) d0[j] = s * (C.cp0[j] - C.a[j]);
            for (int j = 0; j <= N - 1; ++j) dN[j] = -s * (C.cmN[j] - C.a[N - j]);
            d0[0] = s * (empty - 1.0);
            dN[N] = -s * (empty - 1.0);
            if (h->params.flux_form == 1) {
                for (int j = 0; j <= N; ++j) {
                    d0[j] -= s * (1.0 + gm) * pow((double)j, gm);
                    dN[j] += s * (1.0 + gm) * pow((double)(N - j), gm);
                }
            }
            for (int j = 0; j <= N; ++j) {
                pc0[j] = (float)d0[j];
                pcN[j] = (float)dN[j];
            }
        }
        const float* zeros = reinterpret_cast<const float*>(base + oZ);
        AxisOp& U = A->opsU[mu];
        U.n = n;
        U.lower_only = 0;
        U.upper_only = 1;
        U.ends_excluded = 0;
        U.gen = reinterpret_cast<const float*>(base + oU);
        U.col0 = U.colN = zeros;
        U.gen_hi = U.gen_lo = nullptr;
        U.pw_hi = U.pw_lo = nullptr;
        AxisOp& L = A->opsL[mu];
        L = U;
        L.lower_only = 1;
        L.upper_only = 0;
        L.gen = reinterpret_cast<const float*>(base + oL);
        rc.p[mu] = (float)h->params.p[mu];
        rc.dc0[mu] = reinterpret_cast<const float*>(base + o0);
        rc.dcN[mu] = reinterpret_cast<const float*>(base + oN);
    }
    return hipMemcpy(A->opmem, host.data(), bytes, hipMemcpyHostToDevice) == hipSuccess;
}

// workgroups of the adjoint_node grid (x across threads, y and z across workgroups)
int64_t nb_node_max(const lbm_fade* h)
{
    const int64_t gx = (h->grid.n[0] + kBlock - 1) / kBlock;
    return gx * h->grid.n[1] * (h->dim == 3 ? h->grid.n[2] : 1);
}

bool alloc_state(lbm_fade* h, AdjointState* A, int64_t n, int K)
{
    const int64_t nodes = h->nodes;
    const int Q = h->Q, d = h->dim;
    const int64_t nseg = (n + K - 1) / K > 0 ? (n + K - 1) / K : 1;
    if (A->ckpt && A->K == K && A->nseg >= nseg) return true;
    void* old[] = {A->ckpt, A->seg_f[0], A->seg_phi[0], A->seg_C[0], A->seg_f[1], A->seg_phi[1], A->seg_C[1]};
    for (void* p : old) (void)hipFree(p);
    A->ckpt = nullptr;
    for (int b = 0; b < 2; ++b) A->seg_f[b] = A->seg_phi[b] = A->seg_C[b] = nullptr;
    A->nbuf = 0;
    A->K = K;
    A->nseg = nseg;
    const size_t fq = sizeof(float) * Q * nodes;
    if (hipMalloc(&A->ckpt, fq * nseg) != hipSuccess) return false;
    for (int b = 0; b < 2; ++b) {
        const bool ok = hipMalloc(&A->seg_f[b], fq * (K + 1)) == hipSuccess &&
                        hipMalloc(&A->seg_phi[b], sizeof(float) * d * nodes * K) == hipSuccess &&
                        hipMalloc(&A->seg_C[b], sizeof(float) * nodes * K) == hipSuccess;
        if (!ok) {
            // a second buffer is an optimisation: run single-buffered without it
            (void)hipGetLastError();
            (void)hipFree(A->seg_f[b]);
            (void)hipFree(A->seg_phi[b]);
            (void)hipFree(A->seg_C[b]);
            A->seg_f[b] = A->seg_phi[b] = A->seg_C[b] = nullptr;
            if (b == 0) return false;
            break;
        }
        A->nbuf = b + 1;
    }
    if (!A->side) {
        if (hipStreamCreateWithFlags(&A->side, hipStreamNonBlocking) != hipSuccess) return false;
        hipEvent_t* evs[] = {&A->ev_fwd, &A->ev_rec[0], &A->ev_rec[1], &A->ev_rev[0], &A->ev_rev[1]};
        for (hipEvent_t* e : evs)
            if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return false;
    }
    if (!A->fbar) {
        const int64_t nb = (nodes + kBlock - 1) / kBlock;
        if (hipMalloc(&A->fbar, fq) != hipSuccess || hipMalloc(&A->fdir, fq) != hipSuccess ||
            hipMalloc(&A->cbar, sizeof(float) * nodes) != hipSuccess ||
            hipMalloc(&A->phibar, sizeof(float) * d * nodes) != hipSuccess ||
            hipMalloc(&A->fdir2, fq) != hipSuccess || hipMalloc(&A->cbar2, sizeof(float) * nodes) != hipSuccess ||
            hipMalloc(&A->phibar2, sizeof(float) * d * nodes) != hipSuccess ||
            hipMalloc(&A->Ckeep, sizeof(float) * nodes) != hipSuccess ||
            hipMalloc(&A->tu, sizeof(float) * d * nodes) != hipSuccess ||
            hipMalloc(&A->tl, sizeof(float) * d * nodes) != hipSuccess ||
            hipMalloc(&A->dS, sizeof(float) * nodes) != hipSuccess ||
            hipMalloc(&A->part, sizeof(double) * nb_node_max(h) * (3 * 3 + 3 + 1 + 3)) != hipSuccess ||
            hipMalloc(&A->part2, sizeof(double) * nb * 3) != hipSuccess ||
            hipMalloc(&A->acc, sizeof(double) * 64) != hipSuccess)
            return false;
    }
    return true;
}

#define ADJ_TRY(expr)                                                           \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) {                                                 \
            msg = std::string(#expr) + ": " + hipGetErrorString(e_);            \
            return LBM_EDEVICE;                                                 \
        }                                                                       \
    } while (0)

}  // namespace

int adjoint_run(lbm_fade* h, int64_t n, int ckpt_every, const float* gC, int on_device, lbm_grads* out, float* dC0,
                float* dS, hipStream_t s, std::string& msg)
{
    if (dC0 && !h->at_initial_C) {
        msg = "dC0 needs the state set by set_C (no step or set_f since)";
        return LBM_ESTATE;
    }
    const int Q = h->Q, d = h->dim;
    const int64_t nodes = h->nodes;
    const int K = (int)(ckpt_every < n ? ckpt_every : (n > 0 ? n : 1));
    if (!h->adj) {
        h->adj = new AdjointState();
        h->adj->nodes = nodes;
        if (!build_ops(h, h->adj)) {
            adjoint_free(h->adj);
            h->adj = nullptr;
            msg = "allocation of the adjoint operators failed";
            return LBM_ENOMEM;
        }
    }
    AdjointState* A = h->adj;
    // a call that failed part-way may have left segment work on the side
    // stream; it must not overlap this call's use of the buffers
    if (A->side && hipStreamSynchronize(A->side) != hipSuccess) {
        msg = "side stream of an earlier adjoint failed";
        return LBM_EDEVICE;
    }
    if (!alloc_state(h, A, n, K)) {
        msg = "allocation of the adjoint checkpoints failed";
        return LBM_ENOMEM;
    }
    AdjConsts ac;
    memset(&ac, 0, sizeof(ac));
    ac.dim = d;
    ac.Q = Q;
    for (int mu = 0; mu < 3; ++mu) ac.n[mu] = h->cc.n[mu];
    for (int i = 0; i < Q; ++i) ac.w[i] = h->cc.w[i];
    for (int mu = 0; mu < d; ++mu) ac.adv[mu] = h->cc.adv[mu];
    ac.uscale = (float)(h->grid.dt / h->grid.dx * h->wi / h->e2);
    for (int i = 0; i < Q * Q; ++i) ac.R[i] = h->cc.R[i];
    for (int i = 0; i < Q; ++i) ac.wdt[i] = h->cc.wSdt[i];

    const int64_t nb = (nodes + kBlock - 1) / kBlock;
    const int NV = d * d + d + 1;  // flux block of dL/dLambda, dL/du, tr dL/dR
    const dim3 node_grid((unsigned)((ac.n[0] + kBlock - 1) / kBlock), (unsigned)ac.n[1], (unsigned)(d == 3 ? ac.n[2] : 1));
    const int64_t nb_node = (int64_t)node_grid.x * node_grid.y * node_grid.z;
    // the two triangular products of the reversed fractional term of every
    // axis, one launch: s W+^T Phibar (into tu) and s W-^T Phibar (into tl)
    AxisOp ops2[2 * 3];
    AxisLayout lays2[2 * 3];
    for (int mu = 0; mu < d; ++mu) {
        ops2[mu] = A->opsU[mu];
        ops2[d + mu] = A->opsL[mu];
        lays2[mu] = lays2[d + mu] = h->lays[mu];
    }
    auto reversed_phi = [&](const float* pb) -> hipError_t {
        const float* in[2 * 3];
        float* outp[2 * 3];
        for (int mu = 0; mu < d; ++mu) {
            in[mu] = in[d + mu] = pb + (int64_t)mu * nodes;
            outp[mu] = A->tu + (int64_t)mu * nodes;
            outp[d + mu] = A->tl + (int64_t)mu * nodes;
        }
        return launch_fractional_ops(ops2, lays2, in, outp, 2 * d, s);
    };
    const size_t fq = sizeof(float) * Q * nodes;
    const int64_t nseg = (n + K - 1) / K;
    float* gCdev = nullptr;
    if (!on_device) {
        ADJ_TRY(hipMalloc(&gCdev, sizeof(float) * nodes));
        ADJ_TRY(hipMemcpyAsync(gCdev, gC, sizeof(float) * nodes, hipMemcpyHostToDevice, s));
        gC = gCdev;
    }
    // Segment sg recomputed into buffer b from its checkpoint: populations, C
    // and Phi of each of its steps.
    auto seg_len = [&](int64_t sg) { return (int)((sg * K + K <= n ? sg * K + K : n) - sg * K); };
    auto f_of = [&](int64_t sg, int b, int j) -> const float* {
        return j == 0 ? A->ckpt + sg * Q * nodes : A->seg_f[b] + (int64_t)j * Q * nodes;
    };
    auto recompute = [&](int64_t sg, int b, hipStream_t st) -> int {
        const int len = seg_len(sg);
        ADJ_TRY(launch_moment(h->cc, f_of(sg, b, 0), A->seg_C[b], st));
        for (int j = 0; j < len; ++j) {
            float* phi_j = A->seg_phi[b] + (int64_t)j * d * nodes;
            int rc = fade_run_phi(h, A->seg_C[b] + (int64_t)j * nodes, phi_j, st);
            if (rc) {
                msg = "recompute fractional term failed";
                return rc;
            }
            if (j + 1 < len)
                ADJ_TRY(launch_collide_stream(h->cc, f_of(sg, b, j), A->seg_f[b] + (int64_t)(j + 1) * Q * nodes,
                                              phi_j, h->S, A->seg_C[b] + (int64_t)(j + 1) * nodes, st));
        }
        return LBM_OK;
    };
    // Double-buffered: the recompute of segment sg - 1 runs on the side stream
    // while segment sg is swept on s; events order each buffer's reuse.
    const char* ov = getenv("LBM_ADJOINT_OVERLAP");  // "0": one buffer, in order (measurement and tests)
    const bool overlap = A->nbuf == 2 && nseg > 1 && !(ov && ov[0] == '0');
    auto buf_of = [&](int64_t sg) { return overlap ? (int)(sg % 2) : 0; };

    // --- forward pass with checkpoints (the handle's state advances to step n).
    // The last segment runs as its own recompute, into the buffer the reverse
    // sweep reads first, and its last step from there: the same kernels on the
    // same inputs as the plain step (the moment kernel and the collide-stream
    // kernel sum C in the same order), so the state is the same.
    const int64_t t_last = (nseg - 1) * K;  // first step of the last segment
    for (int64_t t = 0; t < n; ++t) {
        if (t % K == 0) ADJ_TRY(hipMemcpyAsync(A->ckpt + (t / K) * Q * nodes, h->f[h->cur], fq,
                                               hipMemcpyDeviceToDevice, s));
        if (t == t_last) break;
        int rc = fade_forward_step(h, s);
        if (rc) {
            msg = "forward step failed";
            return rc;
        }
    }
    if (n == 0) ADJ_TRY(hipMemcpyAsync(A->ckpt, h->f[h->cur], fq, hipMemcpyDeviceToDevice, s));
    if (n > 0) {
        const int64_t sg = nseg - 1;
        const int b = buf_of(sg), len = seg_len(sg);
        int rc = recompute(sg, b, s);
        if (rc) return rc;
        ADJ_TRY(launch_collide_stream(h->cc, f_of(sg, b, len - 1), h->f[1 - h->cur],
                                      A->seg_phi[b] + (int64_t)(len - 1) * d * nodes, h->S, h->C, s));
        h->cur = 1 - h->cur;
        h->steps_done += len;
        h->at_initial_C = false;
    }
    // --- reverse sweep
    ADJ_TRY(hipMemsetAsync(A->acc, 0, sizeof(double) * 64, s));
    ADJ_TRY(hipMemsetAsync(A->dS, 0, sizeof(float) * nodes, s));
    // per-workgroup running sums of the scalar gradients over the sweep
    // (each workgroup adds its steps in order; one fixed-order reduction at the end)
    ADJ_TRY(hipMemsetAsync(A->part, 0, sizeof(double) * nb_node * (NV + d), s));
    ADJ_TRY(hipMemsetAsync(A->part2, 0, sizeof(double) * nb * d, s));
    hipLaunchKernelGGL(broadcast_kernel, dim3(nblk(nodes)), dim3(kBlock), 0, s, gC, A->fbar, Q, nodes);
    ADJ_TRY(hipGetLastError());
    const int offU = d * d, offTr = d * d + d, offP = NV;
    if (overlap) {
        // the side stream's first recompute (segment nseg - 2) reads checkpoints
        // written above
        ADJ_TRY(hipEventRecord(A->ev_fwd, s));
        ADJ_TRY(hipStreamWaitEvent(A->side, A->ev_fwd, 0));
    }
    bool swept[2] = {false, false};
    float* fdirB[2] = {A->fdir, A->fdir2};
    float* cbarB[2] = {A->cbar, A->cbar2};
    float* phibarB[2] = {A->phibar, A->phibar2};
    for (int64_t sg = nseg - 1; sg >= 0; --sg) {
        const int len = seg_len(sg);
        const int b = buf_of(sg);
        const bool ready = sg == nseg - 1;  // computed by the forward pass
        if (overlap) {
            if (!ready) ADJ_TRY(hipStreamWaitEvent(s, A->ev_rec[b], 0));
            if (sg >= 1) {
                const int nb2 = 1 - b;
                if (swept[nb2]) ADJ_TRY(hipStreamWaitEvent(A->side, A->ev_rev[nb2], 0));
                int rc = recompute(sg - 1, nb2, A->side);
                if (rc) return rc;
                ADJ_TRY(hipEventRecord(A->ev_rec[nb2], A->side));
            }
        } else if (!ready) {
            int rc = recompute(sg, 0, s);
            if (rc) return rc;
        }
        for (int j = len - 1; j >= 0; --j) {
            const int64_t t = sg * K + j;
            const float* phi_j = A->seg_phi[b] + (int64_t)j * d * nodes;
            float* fdir_t = fdirB[t & 1];
            float* cbar_t = cbarB[t & 1];
            float* phibar_t = phibarB[t & 1];
            // step t + 1's fields; its C is in this segment's buffer, or (for
            // the segment's last step) in the copy kept from the segment swept before
            LaterStep ls;
            ls.fbar = A->fbar;
            ls.fdir = fdirB[(t + 1) & 1];
            ls.cbar = cbarB[(t + 1) & 1];
            ls.phibar = phibarB[(t + 1) & 1];
            ls.tu = A->tu;
            ls.tl = A->tl;
            ls.C = j + 1 < len ? A->seg_C[b] + (int64_t)(j + 1) * nodes : A->Ckeep;
            const bool first = t == n - 1;  // fbar^n is the broadcast of gC
            auto node_kern = Q == 5 ? (first ? adjoint_node<5, false> : adjoint_node<5, true>)
                                    : (first ? adjoint_node<7, false> : adjoint_node<7, true>);
            hipLaunchKernelGGL(node_kern, node_grid, dim3(kBlock), 0, s, ac, A->rc, ls, f_of(sg, b, j), phi_j, fdir_t,
                               cbar_t, phibar_t, A->dS, A->part, nodes);
            ADJ_TRY(hipGetLastError());
            // fractional term reversed: the two triangular products of Phibar,
            // read by the next kernel (K^T Phibar and <Phibar, (dK/dp) C>)
            ADJ_TRY(reversed_phi(phibar_t));
        }
        // the next segment's sweep starts with a step whose later step is this
        // segment's first; its buffer is recomputed before that sweep ends
        if (sg > 0) ADJ_TRY(hipMemcpyAsync(A->Ckeep, A->seg_C[b], sizeof(float) * nodes, hipMemcpyDeviceToDevice, s));
        if (overlap) {
            ADJ_TRY(hipEventRecord(A->ev_rev[b], s));
            swept[b] = true;
        }
    }
    // fbar^0 = fdir^0 + Cbar^0 + sum_mu K_mu^T Phibar^0_mu and step 0's p-gradient terms
    // (C^0 is slot 0 of buffer 0, which segment 0 was recomputed into)
    if (n > 0) {
        if (d == 2)
            hipLaunchKernelGGL(combine_dot<2>, dim3(nblk(nodes)), dim3(kBlock), 0, s, A->rc, fdirB[0], cbarB[0], A->tu,
                               A->tl, phibarB[0], A->seg_C[0], A->fbar, Q, A->part2, nodes);
        else
            hipLaunchKernelGGL(combine_dot<3>, dim3(nblk(nodes)), dim3(kBlock), 0, s, A->rc, fdirB[0], cbarB[0], A->tu,
                               A->tl, phibarB[0], A->seg_C[0], A->fbar, Q, A->part2, nodes);
        ADJ_TRY(hipGetLastError());
    }
    // slots NV .. NV + d of the node partials are the p-gradient (offP == NV)
    hipLaunchKernelGGL(reduce_partials, dim3(NV + d), dim3(kBlock), 0, s, A->part, nb_node, NV + d, A->acc, 0);
    ADJ_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials, dim3(d), dim3(kBlock), 0, s, A->part2, nb, d, A->acc, offP);
    ADJ_TRY(hipGetLastError());
    // --- reverse of the initial equilibrium (C0' = C of the initial state)
    float* C0p = A->seg_C[0];  // segment 0 (buffer 0) left C^0 in slot 0 (or compute it when n == 0)
    if (n == 0) ADJ_TRY(launch_moment(h->cc, A->ckpt, C0p, s));
    if (Q == 5)
        hipLaunchKernelGGL(adjoint_init_node<5>, dim3(nblk(nodes)), dim3(kBlock), 0, s, ac, A->fbar, C0p, A->cbar,
                           A->phibar, A->part, nodes);
    else
        hipLaunchKernelGGL(adjoint_init_node<7>, dim3(nblk(nodes)), dim3(kBlock), 0, s, ac, A->fbar, C0p, A->cbar,
                           A->phibar, A->part, nodes);
    ADJ_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials, dim3(d), dim3(kBlock), 0, s, A->part, nb, d, A->acc, offU);
    ADJ_TRY(hipGetLastError());
    ADJ_TRY(reversed_phi(A->phibar));
    float* dC0dst = dC0 ? (on_device ? dC0 : A->fdir) : nullptr;  // fdir: scratch for a host destination
    if (d == 2)
        hipLaunchKernelGGL(combine_init<2>, dim3(nblk(nodes)), dim3(kBlock), 0, s, A->rc, A->cbar, A->tu, A->tl,
                           A->phibar, C0p, dC0dst, A->part, nodes);
    else
        hipLaunchKernelGGL(combine_init<3>, dim3(nblk(nodes)), dim3(kBlock), 0, s, A->rc, A->cbar, A->tu, A->tl,
                           A->phibar, C0p, dC0dst, A->part, nodes);
    ADJ_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials, dim3(d), dim3(kBlock), 0, s, A->part, nb, d, A->acc, offP);
    ADJ_TRY(hipGetLastError());
    if (dC0 && !on_device) ADJ_TRY(hipMemcpyAsync(dC0, dC0dst, sizeof(float) * nodes, hipMemcpyDeviceToHost, s));
    if (dS) ADJ_TRY(hipMemcpyAsync(dS, A->dS, sizeof(float) * nodes,
                                   on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    double acc[64];
    ADJ_TRY(hipMemcpyAsync(acc, A->acc, sizeof(double) * 64, hipMemcpyDeviceToHost, s));
    ADJ_TRY(hipStreamSynchronize(s));
    if (gCdev) ADJ_TRY(hipFree(gCdev));

    // --- host chain in FP64: dL/dR -> dL/dLambda -> dL/dlambda-bar -> dL/dD
    memset(out, 0, sizeof(*out));
    const double scale = h->grid.dt / (h->e2 * h->grid.dx * h->grid.dx);
    double G[9] = {0};
    if (h->params.collision == LBM_BGK) {
        // R = I / lambda: dL/dlambda = -tr(dL/dR) / lambda^2
        const double tr = acc[offTr];
        const double lam = h->lam_bar[0];
        const double dlam = -tr / (lam * lam);
        for (int a = 0; a < d; ++a) G[a * d + a] = dlam * scale / d;
    } else {
        // R = M^-1 Lambda M  =>  dL/dLambda = M^-T (dL/dR) M^T; its flux block
        // (summed on the device) is dL/dB for B = lambda-bar^-1, and
        // dL/dlambda-bar = -B^T (dL/dB) B^T
        double Bbar[9], BtBbar[9];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) Bbar[a * d + b] = acc[a * d + b];
        const double* B = h->lam_inv;
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                double sum = 0;
                for (int k = 0; k < d; ++k) sum += B[k * d + a] * Bbar[k * d + b];
                BtBbar[a * d + b] = sum;
            }
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                double sum = 0;
                for (int k = 0; k < d; ++k) sum += BtBbar[a * d + k] * B[b * d + k];
                G[a * d + b] = -sum * scale;
            }
    }
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) out->dD[a * d + b] = 0.5 * (G[a * d + b] + G[b * d + a]);
    for (int mu = 0; mu < d; ++mu) {
        out->du[mu] = acc[offU + mu];
        out->dp[mu] = acc[offP + mu];
    }
    return LBM_OK;
}

}  // namespace lbm
