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
//   fractional term reversed: Cbar += K_mu^T Phibar_mu (transposed Toeplitz GEMM),
//       dL/dp_mu += <Phibar_mu, (dK_mu/dp_mu) C> (one more Toeplitz GEMM);
//   moment reversed: fbar_i += Cbar.
// The transposed operator omits the two boundary ROWS of K^T: they only add to
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

__device__ inline void coords(const AdjConsts& a, int64_t x, int c[3])
{
    c[0] = (int)(x % a.n[0]);
    const int64_t r = x / a.n[0];
    c[1] = (int)(r % a.n[1]);
    c[2] = (int)(r / a.n[1]);
}

__device__ inline bool on_wall(const AdjConsts& a, const int c[3])
{
    bool w = false;
    for (int mu = 0; mu < a.dim; ++mu) w = w || c[mu] == 0 || c[mu] == a.n[mu] - 1;
    return w;
}

// Sum `v` over the workgroup in FP64 (fixed order) into out[0..NV): stored, or
// (ACC) added to what the slot holds (the workgroup's running sum over steps).
template <int NV, bool ACC = false>
__device__ inline void block_sum_store(double (&v)[NV], double* __restrict__ out)
{
    __shared__ double sh[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
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
// Grid: x across threads, y and z across workgroups (no integer division).
template <int Q>
__global__ __launch_bounds__(kBlock) void adjoint_node(AdjConsts ac, const float* __restrict__ fbar,
                                                       const float* __restrict__ f, const float* __restrict__ Phi,
                                                       float* __restrict__ fdir, float* __restrict__ cbar,
                                                       float* __restrict__ phibar, float* __restrict__ dS,
                                                       double* __restrict__ part, int64_t nodes)
{
    constexpr int d = (Q - 1) / 2;
    constexpr int NV = d * d + d + 1;
    const int c[3] = {(int)(blockIdx.x * kBlock + threadIdx.x), (int)blockIdx.y, (int)blockIdx.z};
    const int64_t x = ((int64_t)c[2] * ac.n[1] + c[1]) * ac.n[0] + c[0];
    double red[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k] = 0.0;
    if (c[0] < ac.n[0]) {
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
            float g = fbar[(int64_t)i * nodes + yi];
            // unknown populations at y (their sources lie outside) share its Dirichlet deficit
            int cnt = 0;
            float sum = 0.f;
#pragma unroll
            for (int b = 1; b < Q; ++b) {
                const int mu = (b - 1) / 2;
                const int src = y[mu] - (((b - 1) & 1) ? -1 : 1);
                if (src < 0 || src >= ac.n[mu]) {
                    ++cnt;
                    sum += fbar[(int64_t)b * nodes + yi];
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
    block_sum_store<NV, true>(red, part + blk * NV);  // running sum over the reverse sweep
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

// sum_x Phibar_mu(x) Psi_mu(x) per axis, FP64 partial sums per workgroup
template <int D>
__global__ __launch_bounds__(kBlock) void dot_axes(const float* __restrict__ a, const float* __restrict__ b,
                                                   double* __restrict__ part, int64_t nodes)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double red[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu)
        red[mu] = x < nodes ? (double)a[mu * nodes + x] * (double)b[mu * nodes + x] : 0.0;
    block_sum_store<D>(red, part + (int64_t)blockIdx.x * D);
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

// fbar_i = fdir_i + Cbar + sum_mu (K_mu^T Phibar_mu), and per-workgroup FP64
// partial sums of <Phibar_mu, (dK_mu/dp_mu) C> (psi = (dK/dp) C)
template <int D>
__global__ __launch_bounds__(kBlock) void combine_dot(const float* __restrict__ fdir, const float* __restrict__ cbar,
                                                      const float* __restrict__ kt, const float* __restrict__ phibar,
                                                      const float* __restrict__ psi, float* __restrict__ fbar, int Q,
                                                      double* __restrict__ part, int64_t nodes)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double red[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) red[mu] = 0.0;
    if (x < nodes) {
        float c = cbar[x];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
            c += kt[mu * nodes + x];
            red[mu] = (double)phibar[mu * nodes + x] * (double)psi[mu * nodes + x];
        }
        for (int i = 0; i < Q; ++i) fbar[i * nodes + x] = fdir[i * nodes + x] + c;
    }
    block_sum_store<D, true>(red, part + (int64_t)blockIdx.x * D);  // running sum over the reverse sweep
}

// fbar_i = fdir_i + Cbar + sum_mu (K_mu^T Phibar_mu)
__global__ void combine_kernel(const float* __restrict__ fdir, const float* __restrict__ cbar,
                               const float* __restrict__ kt, float* __restrict__ fbar, int Q, int d, int64_t nodes)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nodes) return;
    float c = cbar[x];
    for (int mu = 0; mu < d; ++mu) c += kt[mu * nodes + x];
    for (int i = 0; i < Q; ++i) fbar[i * nodes + x] = fdir[i * nodes + x] + c;
}

// dC0 = Cbar + sum_mu K_mu^T Phibar_mu, zero on the (overwritten) wall nodes
__global__ void final_dC0(AdjConsts ac, const float* __restrict__ cbar, const float* __restrict__ kt,
                          float* __restrict__ dC0, int64_t nodes)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nodes) return;
    int c[3];
    coords(ac, x, c);
    float v = cbar[x];
    for (int mu = 0; mu < ac.dim; ++mu) v += kt[mu * nodes + x];
    dC0[x] = on_wall(ac, c) ? 0.f : v;
}

unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

struct AdjointState {
    int64_t nodes = 0;
    int K = 0;           // checkpoint interval the buffers were sized for
    int64_t nseg = 0;    // checkpoints allocated
    float* ckpt = nullptr;
    float* seg_f = nullptr;    // (K+1) slots of Q * nodes; slot 0 unused (the checkpoint is read directly)
    float* seg_phi = nullptr;  // K slots of d * nodes
    float* seg_C = nullptr;    // K slots of nodes
    float* fbar = nullptr;
    float* fdir = nullptr;
    float* cbar = nullptr;
    float* phibar = nullptr;
    float* kt = nullptr;
    float* psi = nullptr;
    float* dS = nullptr;
    double* part = nullptr;   // per-workgroup partial sums of adjoint_node
    double* part2 = nullptr;  // per-workgroup partial sums of the p-gradient
    double* acc = nullptr;
    void* opmem = nullptr;
    AxisOp opsT[3], opsP[3];
};

void adjoint_free(AdjointState* a)
{
    if (!a) return;
    void* ptrs[] = {a->ckpt, a->seg_f, a->seg_phi, a->seg_C, a->fbar, a->fdir, a->cbar,
                    a->phibar, a->kt, a->psi, a->dS, a->part, a->part2, a->acc, a->opmem};
    for (void* p : ptrs) (void)hipFree(p);
    delete a;
}

namespace {

// Build the transposed operator (generator T(-d), no boundary columns) and the
// p-derivative operator dK/dp = s (W+ - W-) of every axis (FP32).
bool build_ops(lbm_fade* h, AdjointState* A)
{
    const int d = h->dim;
    auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t bytes = 0;
    for (int mu = 0; mu < d; ++mu) {
        const size_t n = (size_t)h->grid.n[mu];
        bytes += 2 * r256(sizeof(float) * (2 * n - 1)) + 4 * r256(sizeof(float) * n);
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
    for (int mu = 0; mu < d; ++mu) {
        const int n = h->grid.n[mu], N = n - 1;
        const double p = h->params.p[mu];
        const AxisCoeffs C = axis_coeffs(n, 2.0 - h->params.alpha[mu], h->params.g[mu], h->grid.dx);
        const double s = C.s;
        const size_t oT = carve(sizeof(float) * (2 * n - 1)), oP = carve(sizeof(float) * (2 * n - 1));
        const size_t oT0 = carve(sizeof(float) * n), oTN = carve(sizeof(float) * n);
        const size_t oP0 = carve(sizeof(float) * n), oPN = carve(sizeof(float) * n);
        float* gT = reinterpret_cast<float*>(host.data() + oT);
        float* gP = reinterpret_cast<float*>(host.data() + oP);
        float* pc0 = reinterpret_cast<float*>(host.data() + oP0);
        float* pcN = reinterpret_cast<float*>(host.data() + oPN);
        for (int dd = -N; dd <= N; ++dd) {
            // forward T(dd) and its transpose T^T(dd) = T(-dd)
            const int e = -dd;
            double tT;
            if (e > 0) tT = s * p * C.a[e];
            else if (e < 0) tT = s * (1.0 - p) * C.a[-e];
            else tT = s * (p * 1.0 + (1.0 - p) * 1.0);
            gT[dd + N] = (float)tT;
            double tP;
            if (dd > 0) tP = s * C.a[dd];
            else if (dd < 0) tP = -s * C.a[-dd];
            else tP = 0.0;
            gP[dd + N] = (float)tP;
        }
        // d(corr0)/dp and d(corrN)/dp of the forward operator (make_axis_weights), FP64
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
        AxisOp& T = A->opsT[mu];
        T.n = n;
        T.lower_only = h->ops[mu].upper_only;
        T.upper_only = h->ops[mu].lower_only;
        T.gen = reinterpret_cast<const float*>(base + oT);
        T.corr0 = reinterpret_cast<const float*>(base + oT0);  // zeros
        T.corrN = reinterpret_cast<const float*>(base + oTN);  // zeros
        T.gen_hi = T.gen_lo = nullptr;
        T.pw_hi = T.pw_lo = nullptr;
        AxisOp& P = A->opsP[mu];
        P.n = n;
        P.lower_only = P.upper_only = 0;
        P.gen = reinterpret_cast<const float*>(base + oP);
        P.corr0 = reinterpret_cast<const float*>(base + oP0);
        P.corrN = reinterpret_cast<const float*>(base + oPN);
        P.gen_hi = P.gen_lo = nullptr;
        P.pw_hi = P.pw_lo = nullptr;
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
    void* old[] = {A->ckpt, A->seg_f, A->seg_phi, A->seg_C};
    for (void* p : old) (void)hipFree(p);
    A->ckpt = A->seg_f = A->seg_phi = A->seg_C = nullptr;
    A->K = K;
    A->nseg = nseg;
    const size_t fq = sizeof(float) * Q * nodes;
    if (hipMalloc(&A->ckpt, fq * nseg) != hipSuccess) return false;
    if (hipMalloc(&A->seg_f, fq * (K + 1)) != hipSuccess) return false;
    if (hipMalloc(&A->seg_phi, sizeof(float) * d * nodes * K) != hipSuccess) return false;
    if (hipMalloc(&A->seg_C, sizeof(float) * nodes * K) != hipSuccess) return false;
    if (!A->fbar) {
        const int64_t nb = (nodes + kBlock - 1) / kBlock;
        if (hipMalloc(&A->fbar, fq) != hipSuccess || hipMalloc(&A->fdir, fq) != hipSuccess ||
            hipMalloc(&A->cbar, sizeof(float) * nodes) != hipSuccess ||
            hipMalloc(&A->phibar, sizeof(float) * d * nodes) != hipSuccess ||
            hipMalloc(&A->kt, sizeof(float) * d * nodes) != hipSuccess ||
            hipMalloc(&A->psi, sizeof(float) * d * nodes) != hipSuccess ||
            hipMalloc(&A->dS, sizeof(float) * nodes) != hipSuccess ||
            hipMalloc(&A->part, sizeof(double) * nb_node_max(h) * (3 * 3 + 3 + 1)) != hipSuccess ||
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
    // the two operators of the reversed fractional term of every axis, one launch:
    // K^T Phibar (into kt) and (dK/dp) C (into psi)
    AxisOp ops2[2 * 3];
    AxisLayout lays2[2 * 3];
    for (int mu = 0; mu < d; ++mu) {
        ops2[mu] = A->opsT[mu];
        ops2[d + mu] = A->opsP[mu];
        lays2[mu] = lays2[d + mu] = h->lays[mu];
    }
    auto reversed_phi = [&](const float* Cin) -> hipError_t {
        const float* in[2 * 3];
        float* outp[2 * 3];
        for (int mu = 0; mu < d; ++mu) {
            in[mu] = A->phibar + (int64_t)mu * nodes;
            outp[mu] = A->kt + (int64_t)mu * nodes;
            in[d + mu] = Cin;
            outp[d + mu] = A->psi + (int64_t)mu * nodes;
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
    // --- forward pass with checkpoints (the handle's state advances to step n)
    for (int64_t t = 0; t < n; ++t) {
        if (t % K == 0) ADJ_TRY(hipMemcpyAsync(A->ckpt + (t / K) * Q * nodes, h->f[h->cur], fq,
                                               hipMemcpyDeviceToDevice, s));
        int rc = fade_forward_step(h, s);
        if (rc) {
            msg = "forward step failed";
            return rc;
        }
    }
    if (n == 0) ADJ_TRY(hipMemcpyAsync(A->ckpt, h->f[h->cur], fq, hipMemcpyDeviceToDevice, s));
    // --- reverse sweep
    ADJ_TRY(hipMemsetAsync(A->acc, 0, sizeof(double) * 64, s));
    ADJ_TRY(hipMemsetAsync(A->dS, 0, sizeof(float) * nodes, s));
    // per-workgroup running sums of the scalar gradients over the sweep
    // (each workgroup adds its steps in order; one fixed-order reduction at the end)
    ADJ_TRY(hipMemsetAsync(A->part, 0, sizeof(double) * nb_node * NV, s));
    ADJ_TRY(hipMemsetAsync(A->part2, 0, sizeof(double) * nb * d, s));
    hipLaunchKernelGGL(broadcast_kernel, dim3(nblk(nodes)), dim3(kBlock), 0, s, gC, A->fbar, Q, nodes);
    ADJ_TRY(hipGetLastError());
    const int offU = d * d, offTr = d * d + d, offP = d * d + d + 1;
    for (int64_t sg = nseg - 1; sg >= 0; --sg) {
        const int64_t t0 = sg * K;
        const int len = (int)((t0 + K <= n ? t0 + K : n) - t0);
        const float* fck = A->ckpt + sg * Q * nodes;
        auto f_at = [&](int j) -> const float* { return j == 0 ? fck : A->seg_f + (int64_t)j * Q * nodes; };
        ADJ_TRY(launch_moment(h->cc, fck, A->seg_C, s));
        for (int j = 0; j < len; ++j) {
            float* phi_j = A->seg_phi + (int64_t)j * d * nodes;
            int rc = fade_run_phi(h, A->seg_C + (int64_t)j * nodes, phi_j, s);
            if (rc) {
                msg = "recompute fractional term failed";
                return rc;
            }
            if (j + 1 < len)
                ADJ_TRY(launch_collide_stream(h->cc, f_at(j), A->seg_f + (int64_t)(j + 1) * Q * nodes, phi_j, h->S,
                                              A->seg_C + (int64_t)(j + 1) * nodes, nullptr, s));
        }
        for (int j = len - 1; j >= 0; --j) {
            const float* phi_j = A->seg_phi + (int64_t)j * d * nodes;
            const float* C_j = A->seg_C + (int64_t)j * nodes;
            if (Q == 5)
                hipLaunchKernelGGL(adjoint_node<5>, node_grid, dim3(kBlock), 0, s, ac, A->fbar, f_at(j), phi_j, A->fdir,
                                   A->cbar, A->phibar, A->dS, A->part, nodes);
            else
                hipLaunchKernelGGL(adjoint_node<7>, node_grid, dim3(kBlock), 0, s, ac, A->fbar, f_at(j), phi_j, A->fdir,
                                   A->cbar, A->phibar, A->dS, A->part, nodes);
            ADJ_TRY(hipGetLastError());
            // fractional term reversed: K^T Phibar, and (dK/dp) C for <Phibar, dK/dp C>
            ADJ_TRY(reversed_phi(C_j));
            if (d == 2)
                hipLaunchKernelGGL(combine_dot<2>, dim3(nblk(nodes)), dim3(kBlock), 0, s, A->fdir, A->cbar, A->kt,
                                   A->phibar, A->psi, A->fbar, Q, A->part2, nodes);
            else
                hipLaunchKernelGGL(combine_dot<3>, dim3(nblk(nodes)), dim3(kBlock), 0, s, A->fdir, A->cbar, A->kt,
                                   A->phibar, A->psi, A->fbar, Q, A->part2, nodes);
            ADJ_TRY(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(reduce_partials, dim3(NV), dim3(kBlock), 0, s, A->part, nb_node, NV, A->acc, 0);
    ADJ_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials, dim3(d), dim3(kBlock), 0, s, A->part2, nb, d, A->acc, offP);
    ADJ_TRY(hipGetLastError());
    // --- reverse of the initial equilibrium (C0' = C of the initial state)
    float* C0p = A->seg_C;  // segment 0 left C^0 in slot 0 (or compute it when n == 0)
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
    ADJ_TRY(reversed_phi(C0p));
    if (d == 2) hipLaunchKernelGGL(dot_axes<2>, dim3(nblk(nodes)), dim3(kBlock), 0, s, A->phibar, A->psi, A->part, nodes);
    else hipLaunchKernelGGL(dot_axes<3>, dim3(nblk(nodes)), dim3(kBlock), 0, s, A->phibar, A->psi, A->part, nodes);
    ADJ_TRY(hipGetLastError());
    hipLaunchKernelGGL(reduce_partials, dim3(d), dim3(kBlock), 0, s, A->part, nb, d, A->acc, offP);
    ADJ_TRY(hipGetLastError());
    if (dC0) {
        float* dst = dC0;
        if (!on_device) dst = A->fdir;  // scratch
        hipLaunchKernelGGL(final_dC0, dim3(nblk(nodes)), dim3(kBlock), 0, s, ac, A->cbar, A->kt, dst, nodes);
        ADJ_TRY(hipGetLastError());
        if (!on_device) ADJ_TRY(hipMemcpyAsync(dC0, dst, sizeof(float) * nodes, hipMemcpyDeviceToHost, s));
    }
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
