// lbm_handle.h -- the solver handle behind lbm_fade_t (internal).
#pragma once

#include <string>
#include <vector>

#include "../../include/lbm_fade.h"
#include "lbm_internal.h"

namespace lbm {
struct AdjointState;
}

struct lbm_fade {
    lbm_grid grid;
    lbm_params params;
    int dim = 0, Q = 0;
    int64_t nodes = 0;
    int device = 0;
    float* f[2] = {nullptr, nullptr};
    int cur = 0;  // f[cur] holds the current populations
    float* C = nullptr;
    float* Phi = nullptr;
    float* S = nullptr;
    // space-dependent coefficients (allocated together on first use; cc.dB / cc.Cw
    // point at them while either is in use)
    float* dB = nullptr;          // d(d+1)/2 fields: lambda-bar(x)^-1 - lambda-bar^-1 (upper triangle)
    float* Cw = nullptr;          // Dirichlet value of every node
    bool var_D = false;           // dB set by lbm_fade_set_diffusion (else zero)
    bool var_wall = false;        // Cw set by lbm_fade_set_wall (else c_wall)
    void* opmem = nullptr;  // generators, corrections and BF16 splits of all axes
    int* flag = nullptr;
    lbm::AxisOp ops[3];
    lbm::AxisLayout lays[3];
    lbm::CollideConsts cc;
    bool has_state = false;
    bool at_initial_C = false;  // state is f^eq(C0) from set_C, no step taken since
    int64_t steps_done = 0;
    // FP64 host copies used by the adjoint
    double lam_bar[9] = {0};  // flux-block relaxation times lambda-bar
    double lam_inv[9] = {0};  // lambda-bar^-1 (flux block of Lambda)
    double e2 = 0, w0 = 0, wi = 0;
    lbm::AdjointState* adj = nullptr;
    // step graph: a fixed number of steps captured once and replayed
    hipStream_t gstream = nullptr;  // capture stream (default priority)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gcur = 0;                   // f[gcur] holds the populations the graph starts from
    const float* gS = nullptr;      // source pointer the graph was captured with
    const float* gdB = nullptr;     // space-dependent field pointers the graph was captured with
    const float* gCw = nullptr;
    int gkey[4] = {0, 0, 0, 0};     // tuning variables at capture (FP32 tile, BF16 tile, collide rows, stores)
};

namespace lbm {
// Product-rule coefficients of one axis (Sec. 2.4), FP64.
struct AxisCoeffs {
    double s;                // g dx^gamma / Gamma(2 + gamma)
    std::vector<double> a;   // a_k, k = 0..N (a_0 = 1)
    std::vector<double> cp0; // c+_{0j}, j = 1..N (index j; entry 0 unused)
    std::vector<double> cmN; // c-_{Nj}, j = 0..N-1 (entry N unused)
};
AxisCoeffs axis_coeffs(int n, double gamma, double g, double dx);
// Fractional term of every axis of C into Phi (d consecutive node fields).
int fade_run_phi(lbm_fade* h, const float* C, float* Phi, hipStream_t s);
// One forward time step of the handle's state (fractional term, then the
// fused collide-stream kernel, which also refreshes C and its BF16 split).
int fade_forward_step(lbm_fade* h, hipStream_t s);
// Parameter checks of lbm_fade_create (error message set on failure).
int validate_config(const lbm_grid* grid, int32_t lattice, const lbm_params* params);
// Operator data of every axis (Toeplitz generator, boundary columns, BF16
// splits and pair words) as one host image of operator_image_bytes(grid)
// bytes, built in FP64; ops[mu] receives the device pointers the image has
// once copied to `base`.
size_t operator_image_bytes(const lbm_grid& grid);
void build_operator_image(const lbm_grid& grid, const lbm_params& params, unsigned char* host,
                          const unsigned char* base, AxisOp* ops);
// Strided views of a node field for the operator along each axis.
void make_layouts(const lbm_grid& grid, AxisLayout* lays);
// Adjoint driver (adjoint.hip).
int adjoint_run(lbm_fade* h, int64_t n, int ckpt_every, const float* gC, int on_device, lbm_grads* out,
                float* dC0, float* dS, hipStream_t s, std::string& msg);
void adjoint_free(AdjointState* a);
}  // namespace lbm
