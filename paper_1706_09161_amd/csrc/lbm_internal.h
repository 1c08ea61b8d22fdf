// lbm_internal.h -- structures shared by the host runtime (lbm_fade.hip) and
// the kernel launchers (fractional_gemm.hip, collide_stream.hip, adjoint.hip).
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kMaxQ = 7;

// Device-side description of the fractional operator along one axis
// (Sec. 2.4), with T and the boundary values pre-multiplied by
// g dx^gamma / Gamma(2 + gamma) and by p (lower part) / (1 - p) (upper part):
//   ends_excluded = 1 (the forward operators):
//     Phi[j] = sum_{0 < k < N} T(j - k) C[k] + col0[j] C[0] + colN[j] C[N],
//     col0 / colN the whole boundary columns K[j][0], K[j][N];
//   ends_excluded = 0 (the adjoint's transposed parts):
//     Phi[j] = sum_{0 <= k <= N} T(j - k) C[k] + col0[j] C[0] + colN[j] C[N].
struct AxisOp {
    int n;               // nodes on the axis, N = n - 1
    int lower_only;      // p == 1: T(d) = 0 for d < 0
    int upper_only;      // p == 0: T(d) = 0 for d > 0
    int ends_excluded;   // see above
    const float* gen;    // T(d) at gen[d + n - 1], d in [-(n-1), n-1]
    const float* col0;  // n values
    const float* colN;  // n values
    const uint16_t* gen_hi;  // BF16 bits of T split hi/lo (same indexing)
    const uint16_t* gen_lo;
    // Pair words of the split, W(d) = b(d) | b(d - 1) << 16 with b = hi or lo
    // bits (0 for |d| > n - 1), stored with d decreasing: pw[x] = W(pw_top - x)
    // for x in [0, pw_top + n + 32).  pw_top = 16 ceil((n + 512) / 16) - 1.
    const uint32_t* pw_hi;
    const uint32_t* pw_lo;
    int pw_top;
};

// Top index and length of the pair-word arrays of an axis of n nodes.
inline int pw_top_of(int n) { return 16 * ((n + 512 + 15) / 16) - 1; }
inline int64_t pw_len_of(int n) { return (int64_t)pw_top_of(n) + n + 32; }

// Workgroup barrier that orders LDS accesses only (release/acquire fences
// scoped to LDS): global loads in flight stay in flight, unlike
// __syncthreads(), which also waits for them.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Strided view of a node field for the operator along one axis.
//   contiguous axis (x): line l, node j  ->  l * n + j
//   other axes: batch b, node j, line l  ->  b * batch_stride + j * j_stride + l
struct AxisLayout {
    int contiguous;        // 1 for the x axis
    int64_t lines;         // lines per batch (contiguous axis: all lines)
    int64_t j_stride;      // stride of the axis index (strided case)
    int64_t batch_stride;  // strided case
    int batches;           // strided case
};

// One launch of the fractional term for all axes of a step, or for several
// operators at once (the adjoint applies two per axis): workgroup ids are split
// into per-operator ranges, in order.
constexpr int kMaxOps = 6;
struct FracLaunch {
    AxisOp op[kMaxOps];
    AxisLayout lay[kMaxOps];
    int tiles_m[kMaxOps], tiles_n[kMaxOps];
    int first[kMaxOps + 1];  // first workgroup id of every operator, first[naxes] = grid size
    const float* C[kMaxOps];  // input field of every operator
    float* Phi[kMaxOps];
    int naxes;  // operators in this launch
    int lgroup;  // one-sided operators: line tiles per group of the tile order (0 = all of an XCD's)
};

// Constants of the fused collide-stream kernel (Sec. 2.2-2.5).
struct CollideConsts {
    int dim, Q;
    int n[3];
    float w[kMaxQ];         // lattice weights
    float adv[3];           // (dt/dx) u_mu w / e^2: f^eq_{2mu+1} += adv C, f^eq_{2mu+2} -= adv C
    float R[kMaxQ * kMaxQ]; // M^-1 Lambda M (BGK: I / lambda), row-major
    float wSdt[kMaxQ];      // w_i dt (multiplies S)
    float c_wall;
    // Space-dependent coefficients (both null, or both set):
    //   dB: d(d+1)/2 node fields, the upper triangle (row by row) of
    //       lambda-bar(x)^-1 - lambda-bar^-1, added to the flux block of Lambda;
    //   Cw: one node field, the Dirichlet value of every wall node.
    const float* dB;
    const float* Cw;
};

// Kernel launchers (host functions).  All return a hipError_t.
// Fractional term of all axes: axis a reads C + a * in_stride (in_stride = 0:
// one field for every axis) and writes Phi + a * nodes.
hipError_t launch_fractional(const AxisOp* ops, const AxisLayout* lays, int naxes, int precision, const float* C,
                             int64_t in_stride, float* Phi, int64_t nodes, hipStream_t s);
// FP32 only: nops (<= kMaxOps) operators with their own layouts, inputs and
// outputs, in one launch.
hipError_t launch_fractional_ops(const AxisOp* ops, const AxisLayout* lays, const float* const* C, float* const* Phi,
                                 int nops, hipStream_t s);
// C_out receives the new moment.
hipError_t launch_collide_stream(const CollideConsts& cc, const float* f_in, float* f_out, const float* Phi,
                                 const float* S, float* C_out, hipStream_t s);
hipError_t launch_equilibrium_init(const CollideConsts& cc, const float* C, const float* Phi, float* f,
                                   hipStream_t s);
hipError_t launch_wall_overwrite(const CollideConsts& cc, float* C, hipStream_t s);
hipError_t launch_fill(float* p, int64_t count, float v, hipStream_t s);
hipError_t launch_moment(const CollideConsts& cc, const float* f, float* C, hipStream_t s);
hipError_t launch_nonfinite_check(const float* C, int64_t nodes, int* flag, hipStream_t s);
bool have_bf16x3();
// Records msg as the calling thread's last error (lbm_fade_last_error) and returns code.
int set_error(int code, const char* msg);
// Output tiles of 128 x 128 over all axes (sizes the GEMM launch).
int64_t big_tiles(const FracLaunch& L);
// Tile configuration forced through an environment variable (0 = automatic).
int tile_choice(const char* var);
hipError_t launch_fractional_bf16x3(FracLaunch& L, hipStream_t s);

}  // namespace lbm
