// lbm_fade.hip -- host runtime and C ABI (include/lbm_fade.h).
//
// Create-time work happens here in FP64: the relaxation times from D
// (equations (Diffusion_Coefficient_3D), (D_ab)), the collision matrix
// M^-1 Lambda M (equations (MatrixD2), (MatrixS)), and the product-rule
// weights of the fractional integrals (equations (c+), (c-)) arranged as one
// Toeplitz generator plus two boundary columns per axis.  The step itself is
// a sequence of launches on the caller's stream (fractional_gemm.hip,
// collide_stream.hip).
#include "../../include/lbm_fade.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "lbm_handle.h"

namespace {

thread_local std::string g_error;

int fail(int code, const std::string& msg)
{
    g_error = msg;
    return code;
}

}  // namespace

namespace lbm {
// error reporting for the other translation units of the library
int set_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace lbm

namespace {

#define HIP_TRY(expr)                                                                                          \
    do {                                                                                                       \
        hipError_t e_ = (expr);                                                                                \
        if (e_ != hipSuccess) return fail(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

uint16_t bf16_bits_rne(float v)
{
    uint32_t u;
    memcpy(&u, &v, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

float bf16_to_float(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float v;
    memcpy(&v, &u, 4);
    return v;
}

// Round a double to the nearest BF16 (ties to even) through an exact
// double -> float -> bf16 route guarded against double rounding: the float
// rounding is done toward zero with a sticky bit.
uint16_t bf16_from_double(double x)
{
    float f = (float)x;  // round to nearest float
    // Double rounding can only matter when f lands exactly on a bf16 tie;
    // resolve it from the sign of the discarded part.
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0xffffu) == 0x8000u && (double)f != x) {
        if (((double)f < x) == (f > 0.f)) u += 1;  // true value beyond the tie: round away
        else u -= 1;
        memcpy(&f, &u, 4);
    }
    return bf16_bits_rne(f);
}

int64_t nodes_of(const lbm_grid& g)
{
    int64_t m = 1;
    for (int mu = 0; mu < g.dim; ++mu) m *= g.n[mu];
    return m;
}

// Inverse of a small SPD matrix (d <= 3) by the adjugate formula.
bool small_inverse(int d, const double* A, double* Ai)
{
    if (d == 2) {
        const double det = A[0] * A[3] - A[1] * A[2];
        if (!(fabs(det) > 0)) return false;
        Ai[0] = A[3] / det;
        Ai[1] = -A[1] / det;
        Ai[2] = -A[2] / det;
        Ai[3] = A[0] / det;
        return true;
    }
    const double a = A[0], b = A[1], c = A[2], d0 = A[3], e = A[4], f = A[5], g = A[6], h = A[7], i = A[8];
    const double co0 = e * i - f * h, co1 = -(d0 * i - f * g), co2 = d0 * h - e * g;
    const double det = a * co0 + b * co1 + c * co2;
    if (!(fabs(det) > 0)) return false;
    Ai[0] = co0 / det;
    Ai[1] = -(b * i - c * h) / det;
    Ai[2] = (b * f - c * e) / det;
    Ai[3] = co1 / det;
    Ai[4] = (a * i - c * g) / det;
    Ai[5] = -(a * f - c * d0) / det;
    Ai[6] = co2 / det;
    Ai[7] = -(a * h - b * g) / det;
    Ai[8] = (a * e - b * d0) / det;
    return true;
}

bool spd(int d, const double* D)
{
    // Cholesky
    double L[9] = {0};
    for (int i = 0; i < d; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = D[i * d + j];
            for (int k = 0; k < j; ++k) s -= L[i * d + k] * L[j * d + k];
            if (i == j) {
                if (!(s > 0)) return false;
                L[i * d + i] = sqrt(s);
            } else {
                L[i * d + j] = s / L[j * d + j];
            }
        }
    return true;
}

}  // namespace

namespace lbm {
// Product-rule coefficients of Sec. 2.4 for one axis with n nodes (N = n - 1):
//   a_0 = 1, a_k = (k+1)^{g+1} - 2 k^{g+1} + (k-1)^{g+1}       (interior of (c+) and (c-))
//   c+_{0j} = (1+g) j^g - j^{g+1} + (j-1)^{g+1}                 (first column, j >= 1)
//   c-_{Nj} = (1+g)(N-j)^g - (N-j)^{g+1} + (N-j-1)^{g+1}        (last column, j <= N-1)
// and the scale s = g_mu dx^gamma / Gamma(2 + gamma).
AxisCoeffs axis_coeffs(int n, double gamma, double g, double dx)
{
    const int N = n - 1;
    const double gp1 = gamma + 1.0;
    AxisCoeffs A;
    A.s = g * pow(dx, gamma) / tgamma(2.0 + gamma);
    A.a.assign(n, 0.0);
    A.cp0.assign(n, 0.0);
    A.cmN.assign(n, 0.0);
    A.a[0] = 1.0;
    for (int k = 1; k <= N; ++k)
        A.a[k] = pow((double)(k + 1), gp1) - 2.0 * pow((double)k, gp1) + pow((double)(k - 1), gp1);
    for (int j = 1; j <= N; ++j)
        A.cp0[j] = (1.0 + gamma) * pow((double)j, gamma) - pow((double)j, gp1) + pow((double)(j - 1), gp1);
    for (int j = 0; j <= N - 1; ++j) {
        const int m = N - j;
        A.cmN[j] = (1.0 + gamma) * pow((double)m, gamma) - pow((double)m, gp1) + pow((double)(m - 1), gp1);
    }
    return A;
}
}  // namespace lbm

namespace {

// ---------------------------------------------------------------------------
// Forward operator of one axis from the product-rule coefficients:
// K[j][k] = s (p c+_{kj} + (1-p) c-_{kj}), Toeplitz in its interior columns,
// K[j][k] = T(j - k) for 0 < k < N, and two boundary columns col0[j] = K[j][0],
// colN[j] = K[j][N]:
//   K[j][0] = s p c+_{0j} (j >= 1),  K[0][0] = s (p 0^gamma + (1 - p)),
//   K[j][N] = s (1-p) c-_{Nj} (j <= N-1),  K[N][N] = s (p + (1 - p) 0^gamma)
// (c-_{0j} and c+_{Nj} vanish off the diagonal; the diagonal entries that are
// not empty-interval integrals are 1).  The integrals over the empty
// intervals (c+_{00}, c-_{NN}) are 0^gamma: the value that keeps constants
// integrated exactly at j = 0 and j = N.
// flux_form 1 (the Caputo-type flux (Fg2) of Sec. 3.5): integration by parts
// (equations (PSRLdD-a), (PSRLdD-b), (CoeffA_FADE3DPS)) subtracts
// g C(x_0) (j dx)^gamma / Gamma(1 + gamma) (times p) and
// g C(x_N) ((N - j) dx)^gamma / Gamma(1 + gamma) (times 1 - p), a change of the
// two boundary columns only: s (1 + gamma) j^gamma in units of s.
struct AxisWeights {
    std::vector<double> T;     // T(d) at d + N, d in [-N, N]
    std::vector<double> col0;  // n: K[j][0]
    std::vector<double> colN;  // n: K[j][N]
};

AxisWeights make_axis_weights(int n, double gamma, double p, double g, double dx, int flux_form)
{
    const int N = n - 1;
    const lbm::AxisCoeffs A = lbm::axis_coeffs(n, gamma, g, dx);
    const double s = A.s;
    AxisWeights W;
    W.T.assign(2 * N + 1, 0.0);
    W.col0.assign(n, 0.0);
    W.colN.assign(n, 0.0);
    for (int d = -N; d <= N; ++d) {
        double v;
        if (d > 0) v = s * p * A.a[d];
        else if (d < 0) v = s * (1.0 - p) * A.a[-d];
        else v = s * (p * 1.0 + (1.0 - p) * 1.0);
        W.T[d + N] = v;
    }
    const double empty = pow(0.0, gamma);  // c+_{00} = c-_{NN}
    for (int j = 1; j <= N; ++j) W.col0[j] = s * p * A.cp0[j];
    for (int j = 0; j <= N - 1; ++j) W.colN[j] = s * (1.0 - p) * A.cmN[j];
    W.col0[0] = s * (p * empty + (1.0 - p));
    W.colN[N] = s * (p + (1.0 - p) * empty);
    if (flux_form == 1) {
        for (int j = 0; j <= N; ++j) {
            W.col0[j] -= s * p * (1.0 + gamma) * pow((double)j, gamma);
            W.colN[j] -= s * (1.0 - p) * (1.0 + gamma) * pow((double)(N - j), gamma);
        }
    }
    return W;
}

int validate(const lbm_grid* grid, int lattice, const lbm_params* P)
{
    if (!grid || !P) return fail(LBM_EINVAL, "null grid or params");
    if (grid->dim != 2 && grid->dim != 3) return fail(LBM_EINVAL, "dim must be 2 or 3");
    if (lattice != 2 * grid->dim + 1) return fail(LBM_EINVAL, "lattice must be LBM_D2Q5 in 2D, LBM_D3Q7 in 3D");
    if (!(grid->dx > 0) || !(grid->dt > 0)) return fail(LBM_EINVAL, "dx and dt must be > 0");
    const int d = grid->dim;
    int64_t nodes = 1;
    for (int mu = 0; mu < d; ++mu) {
        if (grid->n[mu] < 3) return fail(LBM_EINVAL, "every axis needs >= 3 nodes");
        if (grid->n[mu] > (1 << 20)) return fail(LBM_EINVAL, "axis too long");
        nodes *= grid->n[mu];
        if (!(P->alpha[mu] > 1.0 && P->alpha[mu] <= 2.0)) return fail(LBM_EINVAL, "alpha must lie in (1, 2]");
        if (!(P->p[mu] >= 0.0 && P->p[mu] <= 1.0)) return fail(LBM_EINVAL, "p must lie in [0, 1]");
        if (!(P->g[mu] > 0.0) || !isfinite(P->g[mu])) return fail(LBM_EINVAL, "g must be > 0");
        if (!isfinite(P->u[mu])) return fail(LBM_EINVAL, "u must be finite");
    }
    if (nodes > ((int64_t)1 << 34)) return fail(LBM_EINVAL, "grid too large");
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            const double x = P->D[a * d + b], y = P->D[b * d + a];
            if (!isfinite(x)) return fail(LBM_EINVAL, "D must be finite");
            if (fabs(x - y) > 1e-12 * (fabs(x) + fabs(y))) return fail(LBM_EINVAL, "D must be symmetric");
        }
    if (!spd(d, P->D)) return fail(LBM_EINVAL, "D must be positive definite");
    if (P->collision == LBM_BGK) {
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b)
                if ((a != b && P->D[a * d + b] != 0.0) || (a == b && P->D[a * d + b] != P->D[0]))
                    return fail(LBM_EINVAL, "BGK needs an isotropic D = D0 Id");
    } else if (P->collision == LBM_MRT) {
        if (!(P->tau0 > 0.0)) return fail(LBM_EINVAL, "tau0 must be > 0");
        for (int k = 0; k < 2 * d + 1 - d - 1; ++k)
            if (!(P->tau_free[k] > 0.5) || !isfinite(P->tau_free[k]))
                return fail(LBM_EINVAL, "tau_free must be > 1/2");
    } else {
        return fail(LBM_EINVAL, "unknown collision");
    }
    if (P->precision != LBM_FP32 && P->precision != LBM_BF16X3 && P->precision != LBM_FP32_SIMT)
        return fail(LBM_EINVAL, "unknown precision");
    if (P->precision == LBM_BF16X3 && !lbm::have_bf16x3())
        return fail(LBM_EINVAL, "the split-BF16 kernel is not part of this build");
    if (P->nonfinite_check_every < 0) return fail(LBM_EINVAL, "nonfinite_check_every must be >= 0");
    if (!isfinite(P->c_wall)) return fail(LBM_EINVAL, "c_wall must be finite");
    if (P->flux_form != 0 && P->flux_form != 1) return fail(LBM_EINVAL, "flux_form must be 0 or 1");
    return LBM_OK;
}

// Collision matrix R = M^-1 Lambda M in FP64 (MRT), or I/lambda (BGK).
void collision_matrix(lbm_fade* h, double* R)
{
    const int d = h->dim, Q = h->Q;
    const double scale = h->grid.dt / (h->e2 * h->grid.dx * h->grid.dx);
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) h->lam_bar[a * d + b] = h->params.D[a * d + b] * scale + (a == b ? 0.5 : 0.0);
    small_inverse(d, h->lam_bar, h->lam_inv);
    for (int i = 0; i < Q * Q; ++i) R[i] = 0.0;
    if (h->params.collision == LBM_BGK) {
        const double lam = h->lam_bar[0];
        for (int i = 0; i < Q; ++i) R[i * Q + i] = 1.0 / lam;
        return;
    }
    // M (rows: mass, fluxes, the paper's higher moments), equation (MatrixD2)
    double M[49] = {0};
    for (int i = 0; i < Q; ++i) M[i] = 1.0;
    for (int mu = 0; mu < d; ++mu) {
        M[(1 + mu) * Q + 2 * mu + 1] = 1.0;
        M[(1 + mu) * Q + 2 * mu + 2] = -1.0;
    }
    if (d == 2) {
        const double r3[5] = {4, -1, -1, -1, -1}, r4[5] = {0, 1, 1, -1, -1};
        for (int i = 0; i < 5; ++i) {
            M[3 * Q + i] = r3[i];
            M[4 * Q + i] = r4[i];
        }
    } else {
        const double r4[7] = {6, -1, -1, -1, -1, -1, -1}, r5[7] = {0, 2, 2, -1, -1, -1, -1},
                     r6[7] = {0, 0, 0, 1, 1, -1, -1};
        for (int i = 0; i < 7; ++i) {
            M[4 * Q + i] = r4[i];
            M[5 * Q + i] = r5[i];
            M[6 * Q + i] = r6[i];
        }
    }
    // Lambda: inverse of blockdiag(tau0, lambda-bar, tau_free) (equation (MatrixS))
    double Lam[49] = {0};
    Lam[0] = 1.0 / h->params.tau0;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) Lam[(1 + a) * Q + 1 + b] = h->lam_inv[a * d + b];
    for (int k = d + 1; k < Q; ++k) Lam[k * Q + k] = 1.0 / h->params.tau_free[k - d - 1];
    // M^-1 = M^T diag(1 / |row|^2): the rows of M are mutually orthogonal (Sec. 2.3)
    double rn[7];
    for (int r = 0; r < Q; ++r) {
        rn[r] = 0;
        for (int c = 0; c < Q; ++c) rn[r] += M[r * Q + c] * M[r * Q + c];
    }
    double LM[49];
    for (int r = 0; r < Q; ++r)
        for (int c = 0; c < Q; ++c) {
            double s = 0;
            for (int k = 0; k < Q; ++k) s += Lam[r * Q + k] * M[k * Q + c];
            LM[r * Q + c] = s;
        }
    for (int r = 0; r < Q; ++r)
        for (int c = 0; c < Q; ++c) {
            double s = 0;
            for (int k = 0; k < Q; ++k) s += M[k * Q + r] / rn[k] * LM[k * Q + c];
            R[r * Q + c] = s;
        }
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

hipMemcpyKind kind_to_dev(int on_device) { return on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind kind_from_dev(int on_device) { return on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

int check_device(lbm_fade* h)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) return fail(LBM_EINVAL, "call made with a different current device than create");
    return LBM_OK;
}

int run_phi(lbm_fade* h, const float* C, float* Phi, hipStream_t s)
{
    HIP_TRY(lbm::launch_fractional(h->ops, h->lays, h->dim, h->params.precision, C, 0, Phi, h->nodes, s));
    return LBM_OK;
}

int forward_step(lbm_fade* h, hipStream_t s)
{
    int rc = run_phi(h, h->C, h->Phi, s);
    if (rc) return rc;
    HIP_TRY(lbm::launch_collide_stream(h->cc, h->f[h->cur], h->f[1 - h->cur], h->Phi, h->S, h->C, s));
    h->cur = 1 - h->cur;
    h->steps_done += 1;
    h->at_initial_C = false;
    return LBM_OK;
}

// ---- step graph: kGraphSteps steps (an even number, so the population
// buffers end where they started) captured once per handle and replayed with
// one launch.  Kernels only (no memset or copy nodes).
constexpr int kGraphSteps = 10;

bool graphs_enabled()
{
    const char* v = getenv("LBM_STEP_GRAPH");
    return !(v && v[0] == '0');
}

void graph_key(int (&k)[4])
{
    k[0] = lbm::tile_choice("LBM_FP32_TILE");
    k[1] = lbm::tile_choice("LBM_BF16_TILE");
    const char* r = getenv("LBM_COLLIDE_ROWS");
    k[2] = r ? atoi(r) : 0;
    const char* t = getenv("LBM_COLLIDE_NT");
    k[3] = t ? 1 + (t[0] == '1') + 2 * (t[0] == '0') : 0;
}

void drop_graph(lbm_fade* h)
{
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
}

int build_step_graph(lbm_fade* h)
{
    drop_graph(h);
    if (!h->gstream) HIP_TRY(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    const int cur0 = h->cur;
    const int64_t done0 = h->steps_done;
    const bool init0 = h->at_initial_C;
    HIP_TRY(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeRelaxed));
    int rc = LBM_OK;
    for (int k = 0; k < kGraphSteps && rc == LBM_OK; ++k) rc = forward_step(h, h->gstream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->gstream, &g);
    h->cur = cur0;  // capturing ran nothing
    h->steps_done = done0;
    h->at_initial_C = init0;
    if (rc != LBM_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != LBM_OK ? rc : fail(LBM_EDEVICE, std::string("step graph capture: ") + hipGetErrorString(e));
    }
    const hipError_t e2 = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        (void)hipGraphDestroy(g);
        h->gexec = nullptr;
        return fail(LBM_EDEVICE, std::string("step graph instantiation: ") + hipGetErrorString(e2));
    }
    h->graph = g;
    h->gcur = cur0;
    h->gS = h->S;
    h->gdB = h->cc.dB;
    h->gCw = h->cc.Cw;
    graph_key(h->gkey);
    return LBM_OK;
}

// C := sum_i f_i of the current populations
int refresh_C(lbm_fade* h, hipStream_t s)
{
    HIP_TRY(lbm::launch_moment(h->cc, h->f[h->cur], h->C, s));
    return LBM_OK;
}

// The two fields of the space-dependent path, allocated together on first
// use with neutral contents (dB = 0, Cw = c_wall).
int ensure_var_fields(lbm_fade* h, hipStream_t s)
{
    if (h->dB) return LBM_OK;
    const int ncomp = h->dim * (h->dim + 1) / 2;
    float *dB = nullptr, *Cw = nullptr;
    if (hipMalloc(&dB, sizeof(float) * ncomp * h->nodes) != hipSuccess ||
        hipMalloc(&Cw, sizeof(float) * h->nodes) != hipSuccess) {
        (void)hipFree(dB);
        return fail(LBM_ENOMEM, "hipMalloc of the space-dependent fields failed");
    }
    h->dB = dB;
    h->Cw = Cw;
    HIP_TRY(lbm::launch_fill(dB, ncomp * h->nodes, 0.f, s));
    HIP_TRY(lbm::launch_fill(Cw, h->nodes, h->cc.c_wall, s));
    h->cc.dB = dB;
    h->cc.Cw = Cw;
    return LBM_OK;
}

// Frees the fields once neither is in use (the kernels go back to the
// constant path).
int release_var_fields(lbm_fade* h, hipStream_t s)
{
    if (h->var_D || h->var_wall || !h->dB) return LBM_OK;
    HIP_TRY(hipStreamSynchronize(s));
    drop_graph(h);  // a captured graph reads these fields
    (void)hipFree(h->dB);
    (void)hipFree(h->Cw);
    h->dB = h->Cw = nullptr;
    h->cc.dB = h->cc.Cw = nullptr;
    return LBM_OK;
}

// dB of every node from a field of d x d tensors, FP64 on the host:
// lambda-bar(x) = D(x) dt / (e^2 dx^2) + Id/2 (equation (D_ab) at each node),
// dB(x) = lambda-bar(x)^-1 - lambda-bar^-1.  D(x) must be finite, symmetric
// and positive semi-definite (every principal minor >= 0 up to FP32
// rounding); the node of the first violation is reported.
int diffusion_blocks(lbm_fade* h, const float* D, std::vector<float>& out)
{
    const int d = h->dim, ncomp = d * (d + 1) / 2;
    const int64_t nodes = h->nodes;
    const double scale = h->grid.dt / (h->e2 * h->grid.dx * h->grid.dx);
    out.assign((size_t)ncomp * nodes, 0.f);
    auto bad = [&](int64_t x, const char* why) {
        char msg[160];
        snprintf(msg, sizeof msg, "D(x) at node %lld is %s", (long long)x, why);
        return fail(LBM_EINVAL, msg);
    };
    for (int64_t x = 0; x < nodes; ++x) {
        double Dn[9], lam[9], inv[9];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                Dn[a * d + b] = (double)D[(int64_t)(a * d + b) * nodes + x];
                if (!isfinite(Dn[a * d + b])) return bad(x, "not finite");
            }
        for (int a = 0; a < d; ++a)
            for (int b = a + 1; b < d; ++b) {
                const double u = Dn[a * d + b], v = Dn[b * d + a];
                if (fabs(u - v) > 1e-6 * (fabs(u) + fabs(v))) return bad(x, "not symmetric");
                Dn[a * d + b] = Dn[b * d + a] = 0.5 * (u + v);
            }
        // principal minors
        const double tol = 1e-6;
        for (int a = 0; a < d; ++a)
            if (!(Dn[a * d + a] >= 0.0)) return bad(x, "not positive semi-definite");
        for (int a = 0; a < d; ++a)
            for (int b = a + 1; b < d; ++b) {
                const double p = Dn[a * d + a] * Dn[b * d + b];
                if (!(p - Dn[a * d + b] * Dn[a * d + b] >= -tol * p)) return bad(x, "not positive semi-definite");
            }
        if (d == 3) {
            const double det = Dn[0] * (Dn[4] * Dn[8] - Dn[5] * Dn[7]) - Dn[1] * (Dn[3] * Dn[8] - Dn[5] * Dn[6]) +
                               Dn[2] * (Dn[3] * Dn[7] - Dn[4] * Dn[6]);
            if (!(det >= -tol * Dn[0] * Dn[4] * Dn[8])) return bad(x, "not positive semi-definite");
        }
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) lam[a * d + b] = Dn[a * d + b] * scale + (a == b ? 0.5 : 0.0);
        if (!small_inverse(d, lam, inv)) return bad(x, "singular");
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b) {
                const int k = a * d - a * (a - 1) / 2 + (b - a);
                out[(size_t)k * nodes + x] = (float)(inv[a * d + b] - h->lam_inv[a * d + b]);
            }
    }
    return LBM_OK;
}

}  // namespace

namespace lbm {

int validate_config(const lbm_grid* grid, int32_t lattice, const lbm_params* params)
{
    return validate(grid, lattice, params);
}

// Every piece of the operator data sits at a 256-byte aligned offset.
static size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t operator_image_bytes(const lbm_grid& grid)
{
    size_t bytes = 0;
    for (int mu = 0; mu < grid.dim; ++mu) {
        const size_t n = (size_t)grid.n[mu];
        bytes += r256(sizeof(float) * (2 * n - 1)) + 2 * r256(sizeof(float) * n) +
                 2 * r256(sizeof(uint16_t) * (2 * n - 1)) + 2 * r256(sizeof(uint32_t) * pw_len_of((int)n));
    }
    return bytes;
}

void build_operator_image(const lbm_grid& grid, const lbm_params& P, unsigned char* host, const unsigned char* base,
                          AxisOp* ops)
{
    size_t off = 0;
    auto carve = [&](size_t nbytes) {
        const size_t o = off;
        off += r256(nbytes);
        return o;
    };
    for (int mu = 0; mu < grid.dim; ++mu) {
        const int n = grid.n[mu];
        const AxisWeights W = make_axis_weights(n, 2.0 - P.alpha[mu], P.p[mu], P.g[mu], grid.dx, P.flux_form);
        AxisOp& op = ops[mu];
        op.n = n;
        op.lower_only = P.p[mu] == 1.0;
        op.upper_only = P.p[mu] == 0.0;
        op.ends_excluded = 1;
        const size_t og = carve(sizeof(float) * (2 * n - 1));
        const size_t o0 = carve(sizeof(float) * n);
        const size_t oN = carve(sizeof(float) * n);
        const size_t oh = carve(sizeof(uint16_t) * (2 * n - 1));
        const size_t ol = carve(sizeof(uint16_t) * (2 * n - 1));
        const int64_t pwn = pw_len_of(n);
        const size_t oph = carve(sizeof(uint32_t) * pwn);
        const size_t opl = carve(sizeof(uint32_t) * pwn);
        float* g = reinterpret_cast<float*>(host + og);
        float* c0 = reinterpret_cast<float*>(host + o0);
        float* cN = reinterpret_cast<float*>(host + oN);
        uint16_t* gh = reinterpret_cast<uint16_t*>(host + oh);
        uint16_t* glo = reinterpret_cast<uint16_t*>(host + ol);
        for (int t = 0; t < 2 * n - 1; ++t) {
            const double v = W.T[t];
            g[t] = (float)v;
            gh[t] = bf16_from_double(v);
            glo[t] = bf16_from_double(v - (double)bf16_to_float(gh[t]));
        }
        // the whole boundary columns K[j][0] and K[j][N]: the kernels leave
        // k = 0 and k = N out of the Toeplitz sum, so no product of T with a
        // wall value is added and then cancelled
        for (int j = 0; j < n; ++j) {
            c0[j] = (float)W.col0[j];
            cN[j] = (float)W.colN[j];
        }
        // pair words of the BF16 split, d decreasing (operand order of the BF16 GEMM)
        uint32_t* pwh = reinterpret_cast<uint32_t*>(host + oph);
        uint32_t* pwl = reinterpret_cast<uint32_t*>(host + opl);
        const int top = pw_top_of(n);
        auto bits = [&](const uint16_t* b, int64_t dd) -> uint32_t {
            return (dd >= -(n - 1) && dd <= n - 1) ? (uint32_t)b[dd + n - 1] : 0u;
        };
        for (int64_t x = 0; x < pwn; ++x) {
            const int64_t dd = top - x;
            pwh[x] = bits(gh, dd) | (bits(gh, dd - 1) << 16);
            pwl[x] = bits(glo, dd) | (bits(glo, dd - 1) << 16);
        }
        op.gen = reinterpret_cast<const float*>(base + og);
        op.col0 = reinterpret_cast<const float*>(base + o0);
        op.colN = reinterpret_cast<const float*>(base + oN);
        op.gen_hi = reinterpret_cast<const uint16_t*>(base + oh);
        op.gen_lo = reinterpret_cast<const uint16_t*>(base + ol);
        op.pw_hi = reinterpret_cast<const uint32_t*>(base + oph);
        op.pw_lo = reinterpret_cast<const uint32_t*>(base + opl);
        op.pw_top = top;
    }
}

void make_layouts(const lbm_grid& grid, AxisLayout* lays)
{
    const int64_t nx = grid.n[0], ny = grid.n[1], nz = grid.dim == 3 ? grid.n[2] : 1;
    const int64_t nodes = nx * ny * nz;
    lays[0] = {1, nodes / nx, 1, 0, 1};
    if (grid.dim == 2) {
        lays[1] = {0, nx, nx, 0, 1};
    } else {
        lays[1] = {0, nx, nx, nx * ny, (int)nz};
        lays[2] = {0, nx * ny, nx * ny, 0, 1};
    }
}

}  // namespace lbm

namespace lbm {
// used by the adjoint driver
int fade_run_phi(lbm_fade* h, const float* C, float* Phi, hipStream_t s) { return run_phi(h, C, Phi, s); }
int fade_forward_step(lbm_fade* h, hipStream_t s) { return forward_step(h, s); }
}  // namespace lbm

extern "C" {

const char* lbm_fade_last_error(void) { return g_error.c_str(); }

const char* lbm_fade_version(void) { return "lbm_fade 0.1 (gfx950)"; }

int lbm_fade_create(const lbm_grid* grid, int32_t lattice, const lbm_params* params, lbm_fade_t* out)
{
    if (!out) return fail(LBM_EINVAL, "null output handle");
    *out = nullptr;
    int rc = validate(grid, lattice, params);
    if (rc) return rc;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LBM_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");

    lbm_fade* h = new lbm_fade();
    h->grid = *grid;
    h->params = *params;
    h->dim = grid->dim;
    h->Q = 2 * grid->dim + 1;
    h->nodes = nodes_of(*grid);
    h->device = dev;
    if (h->dim == 2) {
        h->w0 = 1.0 / 3.0;
        h->wi = 1.0 / 6.0;
        h->e2 = 1.0 / 3.0;
    } else {
        h->w0 = 1.0 / 4.0;
        h->wi = 1.0 / 8.0;
        h->e2 = 1.0 / 4.0;
    }
    const int d = h->dim, Q = h->Q;

    // collision constants
    double R[49];
    collision_matrix(h, R);
    if (params->collision == LBM_BGK && !(h->lam_bar[0] > 0.5)) {
        delete h;
        return fail(LBM_EINVAL, "BGK relaxation time must exceed 1/2");
    }
    lbm::CollideConsts& cc = h->cc;
    memset(&cc, 0, sizeof(cc));
    cc.dim = d;
    cc.Q = Q;
    for (int mu = 0; mu < 3; ++mu) cc.n[mu] = mu < d ? grid->n[mu] : 1;
    cc.w[0] = (float)h->w0;
    for (int i = 1; i < Q; ++i) cc.w[i] = (float)h->wi;
    for (int mu = 0; mu < d; ++mu) cc.adv[mu] = (float)(grid->dt / grid->dx * params->u[mu] * h->wi / h->e2);
    for (int i = 0; i < Q * Q; ++i) cc.R[i] = (float)R[i];
    cc.wSdt[0] = (float)(h->w0 * grid->dt);
    for (int i = 1; i < Q; ++i) cc.wSdt[i] = (float)(h->wi * grid->dt);
    cc.c_wall = (float)params->c_wall;

    // operator data
    const size_t bytes = lbm::operator_image_bytes(*grid);
    auto cleanup = [&]() { lbm_fade_destroy(h); };
    hipError_t e = hipMalloc(&h->opmem, bytes);
    if (e != hipSuccess) {
        cleanup();
        return fail(LBM_ENOMEM, "hipMalloc of operator data failed");
    }
    std::vector<unsigned char> host(bytes, 0);
    lbm::build_operator_image(*grid, *params, host.data(), reinterpret_cast<const unsigned char*>(h->opmem), h->ops);
    e = hipMemcpy(h->opmem, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        cleanup();
        return fail(LBM_EDEVICE, std::string("upload of operator data failed: ") + hipGetErrorString(e));
    }
    lbm::make_layouts(*grid, h->lays);
    // state
    const size_t fbytes = sizeof(float) * Q * h->nodes;
    if (hipMalloc(&h->f[0], fbytes) != hipSuccess || hipMalloc(&h->f[1], fbytes) != hipSuccess ||
        hipMalloc(&h->C, sizeof(float) * h->nodes) != hipSuccess ||
        hipMalloc(&h->Phi, sizeof(float) * d * h->nodes) != hipSuccess ||
        hipMalloc(&h->flag, sizeof(int) * 4) != hipSuccess) {
        cleanup();
        return fail(LBM_ENOMEM, "hipMalloc of the solver state failed");
    }
    *out = h;
    g_error.clear();
    return LBM_OK;
}

void lbm_fade_destroy(lbm_fade_t h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    drop_graph(h);
    if (h->gstream) (void)hipStreamDestroy(h->gstream);
    lbm::adjoint_free(h->adj);
    (void)hipFree(h->f[0]);
    (void)hipFree(h->f[1]);
    (void)hipFree(h->C);
    (void)hipFree(h->Phi);
    (void)hipFree(h->S);
    (void)hipFree(h->dB);
    (void)hipFree(h->Cw);
    (void)hipFree(h->opmem);
    (void)hipFree(h->flag);
    delete h;
}

int lbm_fade_set_C(lbm_fade_t h, const float* C0, int32_t on_device, void* stream)
{
    if (!h || !C0) return fail(LBM_EINVAL, "null argument");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(h->C, C0, sizeof(float) * h->nodes, kind_to_dev(on_device), s));
    HIP_TRY(lbm::launch_wall_overwrite(h->cc, h->C, s));
    rc = run_phi(h, h->C, h->Phi, s);
    if (rc) return rc;
    HIP_TRY(lbm::launch_equilibrium_init(h->cc, h->C, h->Phi, h->f[h->cur], s));
    rc = refresh_C(h, s);
    if (rc) return rc;
    if (!on_device) HIP_TRY(hipStreamSynchronize(s));  // the host buffer may be reused on return
    h->has_state = true;
    h->at_initial_C = true;
    h->steps_done = 0;
    return LBM_OK;
}

int lbm_fade_set_source(lbm_fade_t h, const float* S, int32_t on_device, void* stream)
{
    if (!h) return fail(LBM_EINVAL, "null handle");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    if (!S) {
        if (h->S) {
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipFree(h->S));
            h->S = nullptr;
        }
        return LBM_OK;
    }
    if (!h->S) {
        if (hipMalloc(&h->S, sizeof(float) * h->nodes) != hipSuccess) return fail(LBM_ENOMEM, "hipMalloc of S failed");
    }
    HIP_TRY(hipMemcpyAsync(h->S, S, sizeof(float) * h->nodes, kind_to_dev(on_device), s));
    if (!on_device) HIP_TRY(hipStreamSynchronize(s));
    return LBM_OK;
}

int lbm_fade_set_diffusion(lbm_fade_t h, const float* D, int32_t on_device, void* stream)
{
    if (!h) return fail(LBM_EINVAL, "null handle");
    if (h->params.collision != LBM_MRT)
        return fail(LBM_EINVAL, "a space-dependent D needs the MRT collision (BGK relaxes every moment alike)");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    const int d = h->dim, ncomp = d * (d + 1) / 2;
    if (!D) {
        if (h->var_D) {
            h->var_D = false;
            HIP_TRY(lbm::launch_fill(h->dB, ncomp * h->nodes, 0.f, s));
        }
        return release_var_fields(h, s);
    }
    std::vector<float> staged;
    const float* src = D;
    if (on_device) {
        staged.resize((size_t)d * d * h->nodes);
        HIP_TRY(hipMemcpyAsync(staged.data(), D, sizeof(float) * staged.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        src = staged.data();
    }
    std::vector<float> blocks;
    rc = diffusion_blocks(h, src, blocks);
    if (rc) return rc;
    rc = ensure_var_fields(h, s);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(h->dB, blocks.data(), sizeof(float) * blocks.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // blocks is freed on return
    h->var_D = true;
    return LBM_OK;
}

int lbm_fade_set_wall(lbm_fade_t h, const float* Cw, int32_t on_device, void* stream)
{
    if (!h) return fail(LBM_EINVAL, "null handle");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    if (!Cw) {
        if (h->var_wall) {
            h->var_wall = false;
            HIP_TRY(lbm::launch_fill(h->Cw, h->nodes, h->cc.c_wall, s));
        }
        return release_var_fields(h, s);
    }
    rc = ensure_var_fields(h, s);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(h->Cw, Cw, sizeof(float) * h->nodes, kind_to_dev(on_device), s));
    if (!on_device) HIP_TRY(hipStreamSynchronize(s));
    h->var_wall = true;
    return LBM_OK;
}

int lbm_fade_step(lbm_fade_t h, int64_t n, void* stream)
{
    if (!h) return fail(LBM_EINVAL, "null handle");
    if (n < 0) return fail(LBM_EINVAL, "negative step count");
    if (!h->has_state) return fail(LBM_ESTATE, "set_C or set_f must be called before step");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    const int every = h->params.nonfinite_check_every;
    if (every == 0 && n >= kGraphSteps && graphs_enabled()) {
        int key[4];
        graph_key(key);
        if (!h->gexec || h->gS != h->S || h->gdB != h->cc.dB || h->gCw != h->cc.Cw || key[0] != h->gkey[0] ||
            key[1] != h->gkey[1] ||
            key[2] != h->gkey[2] || key[3] != h->gkey[3]) {
            rc = build_step_graph(h);
            if (rc) return rc;
        }
        if (h->cur != h->gcur) {  // one direct step puts the populations where the graph starts
            rc = forward_step(h, s);
            if (rc) return rc;
            --n;
        }
        for (; n >= kGraphSteps; n -= kGraphSteps) {
            HIP_TRY(hipGraphLaunch(h->gexec, s));
            h->steps_done += kGraphSteps;
            h->at_initial_C = false;
        }
    }
    for (int64_t m = 0; m < n; ++m) {
        rc = forward_step(h, s);
        if (rc) return rc;
        if (every > 0 && h->steps_done % every == 0) {
            int flag = 0;
            HIP_TRY(hipMemsetAsync(h->flag, 0, sizeof(int), s));
            HIP_TRY(lbm::launch_nonfinite_check(h->C, h->nodes, h->flag, s));
            HIP_TRY(hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (flag) {
                char msg[128];
                snprintf(msg, sizeof msg, "non-finite concentration after step %lld", (long long)h->steps_done);
                return fail(LBM_ENONFINITE, msg);
            }
        }
    }
    return LBM_OK;
}

int lbm_fade_get_C(lbm_fade_t h, float* dst, int32_t on_device, void* stream)
{
    if (!h || !dst) return fail(LBM_EINVAL, "null argument");
    if (!h->has_state) return fail(LBM_ESTATE, "no state yet");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(dst, h->C, sizeof(float) * h->nodes, kind_from_dev(on_device), s));
    if (!on_device) HIP_TRY(hipStreamSynchronize(s));
    return LBM_OK;
}

int lbm_fade_get_f(lbm_fade_t h, float* dst, int32_t on_device, void* stream)
{
    if (!h || !dst) return fail(LBM_EINVAL, "null argument");
    if (!h->has_state) return fail(LBM_ESTATE, "no state yet");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(dst, h->f[h->cur], sizeof(float) * h->Q * h->nodes, kind_from_dev(on_device), s));
    if (!on_device) HIP_TRY(hipStreamSynchronize(s));
    return LBM_OK;
}

int lbm_fade_set_f(lbm_fade_t h, const float* src, int32_t on_device, void* stream)
{
    if (!h || !src) return fail(LBM_EINVAL, "null argument");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(h->f[h->cur], src, sizeof(float) * h->Q * h->nodes, kind_to_dev(on_device), s));
    rc = refresh_C(h, s);
    if (rc) return rc;
    if (!on_device) HIP_TRY(hipStreamSynchronize(s));
    h->has_state = true;
    h->at_initial_C = false;
    h->steps_done = 0;
    return LBM_OK;
}

int lbm_fade_apply_phi(lbm_fade_t h, const float* C, float* Phi, int32_t on_device, void* stream)
{
    if (!h || !Phi) return fail(LBM_EINVAL, "null argument");
    int rc = check_device(h);
    if (rc) return rc;
    hipStream_t s = as_stream(stream);
    if (!C) {
        // the solver's own concentration
        if (!h->has_state) return fail(LBM_ESTATE, "no state yet");
        if (!on_device) return fail(LBM_EINVAL, "C = NULL needs a device Phi");
        return run_phi(h, h->C, Phi, s);
    }
    if (on_device) return run_phi(h, C, Phi, s);
    float *dC = nullptr, *dP = nullptr;
    if (hipMalloc(&dC, sizeof(float) * h->nodes) != hipSuccess ||
        hipMalloc(&dP, sizeof(float) * h->dim * h->nodes) != hipSuccess) {
        (void)hipFree(dC);
        return fail(LBM_ENOMEM, "hipMalloc of temporaries failed");
    }
    hipError_t e = hipMemcpyAsync(dC, C, sizeof(float) * h->nodes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) rc = run_phi(h, dC, dP, s);
    if (e == hipSuccess && rc == LBM_OK)
        e = hipMemcpyAsync(Phi, dP, sizeof(float) * h->dim * h->nodes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dC);
    (void)hipFree(dP);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("apply_phi: ") + hipGetErrorString(e));
    return rc;
}

int lbm_fade_adjoint(lbm_fade_t h, int64_t n, int32_t ckpt_every, const float* gC, int32_t on_device,
                     lbm_grads* out, float* dC0, float* dS, void* stream)
{
    if (!h || !gC || !out) return fail(LBM_EINVAL, "null argument");
    if (n < 0 || ckpt_every <= 0) return fail(LBM_EINVAL, "need n >= 0 and ckpt_every > 0");
    if (!h->has_state) return fail(LBM_ESTATE, "set_C must be called before adjoint");
    if (h->cc.dB)
        return fail(LBM_EINVAL, "the adjoint takes constant D and wall values: reset set_diffusion / set_wall");
    int rc = check_device(h);
    if (rc) return rc;
    std::string msg;
    rc = lbm::adjoint_run(h, n, ckpt_every, gC, on_device, out, dC0, dS, as_stream(stream), msg);
    if (rc) return fail(rc, msg);
    return LBM_OK;
}

}  // extern "C"
