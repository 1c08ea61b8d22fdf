// fractional_gemm.hip -- the fractional term of Algorithm 1 (first stage of
// the time loop) on gfx950.
//
// Along axis mu every grid line is multiplied by the same matrix
//   K[j][k] = g dx^gamma / Gamma(2+gamma) * (p c+_{kj}(gamma) + (1-p) c-_{kj}(gamma, N))
// (Sec. 2.4, equations (1Dminus_discret), (c+), (c-), (XXminus_discret)),
// which is Toeplitz except in its first and last columns:
//   K[j][k] = T(j - k) + [k == 0] corr0[j] + [k == N] corrN[j].
// So Phi = K C for all lines at once is a dense contraction (n x n times
// n x lines).  It runs as a GEMM on the matrix cores; the Toeplitz operand is
// never stored as an n x n matrix: each workgroup keeps the 2n-1 generator
// values it needs in LDS and reads fragments from there, and the two boundary
// columns are a rank-2 epilogue.
//
// Layouts (see AxisLayout):
//   x axis  ("contiguous"): D[line][j]      = sum_k C[line][k] T(j - k)
//   y, z    ("strided")   : D[j][line]      = sum_k T(j - k) C[k][line]
// In both cases the MFMA's lane-varying output index is the memory-contiguous
// one, so stores are coalesced.
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

// ---------------------------------------------------------------------------
// Plain kernel: one thread per output, FP32 fused multiply-add, generator and
// corrections read from global memory.  A second, independent implementation
// of the operator used as a debugging and performance baseline.
__global__ __launch_bounds__(256) void fractional_simt(AxisOp op, AxisLayout lay, const float* __restrict__ C,
                                                       float* __restrict__ Phi)
{
    const int n = op.n, N = n - 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = lay.contiguous ? lay.lines * n : (int64_t)lay.batches * n * lay.lines;
    if (t >= total) return;
    const float* gen = op.gen + (n - 1);
    if (lay.contiguous) {
        const int64_t line = t / n;
        const int j = (int)(t % n);
        const float* c = C + line * n;
        float acc = 0.f;
        for (int k = 0; k < n; ++k) acc = fmaf(gen[j - k], c[k], acc);
        acc = fmaf(op.corr0[j], c[0], acc);
        acc = fmaf(op.corrN[j], c[N], acc);
        Phi[line * n + j] = acc;
    } else {
        const int64_t line = t % lay.lines;
        const int64_t rest = t / lay.lines;
        const int j = (int)(rest % n);
        const int64_t b = rest / n;
        const float* c = C + b * lay.batch_stride + line;
        float acc = 0.f;
        for (int k = 0; k < n; ++k) acc = fmaf(gen[j - k], c[(int64_t)k * lay.j_stride], acc);
        acc = fmaf(op.corr0[j], c[0], acc);
        acc = fmaf(op.corrN[j], c[(int64_t)N * lay.j_stride], acc);
        Phi[b * lay.batch_stride + (int64_t)j * lay.j_stride + line] = acc;
    }
}

// ---------------------------------------------------------------------------
// Tile bookkeeping shared by the MFMA kernels.
struct TileCoord {
    int m0, n0;  // first row / column of the output tile (GEMM coordinates)
    int batch;
};

// Map the linear workgroup id to a tile.  Consecutive workgroup ids go to
// different XCDs (round robin over 8); remap so that every XCD owns a
// contiguous range of tiles, and order tiles so that those sharing a panel of
// C (the large operand) are adjacent: they then hit the same L2.
__device__ inline TileCoord tile_of(int tiles_toep, int tiles_c, bool toep_is_m, int total)
{
    int bid = blockIdx.x;
    int lin = bid;
    if ((total & 7) == 0) lin = (bid & 7) * (total >> 3) + (bid >> 3);
    const int tt = lin % tiles_toep;
    const int rest = lin / tiles_toep;
    const int tc = rest % tiles_c;
    TileCoord r;
    r.batch = rest / tiles_c;
    if (toep_is_m) {
        r.m0 = tt;
        r.n0 = tc;
    } else {
        r.m0 = tc;
        r.n0 = tt;
    }
    return r;
}

// ---------------------------------------------------------------------------
// FP32 MFMA kernel, v_mfma_f32_32x32x2_f32.  Workgroup tile BM x BN, 4 waves
// in a 2 x 2 arrangement, each wave (BM/2) x (BN/2) in 32 x 32 blocks.
// Operand convention for 32x32x2: lane l supplies A(i = l%32, kk = l/32) and
// B(kk = l/32, j = l%32); accumulator register r of lane l holds
// D(8*(r/4) + 4*(l/32) + r%4, l%32).
template <bool CONTIG, int BM, int BN, int BK, int VEC>
__global__ __launch_bounds__(kThreads) void fractional_f32_mfma(AxisOp op, AxisLayout lay,
                                                                 const float* __restrict__ C,
                                                                 float* __restrict__ Phi, int tiles_m, int tiles_n,
                                                                 int total)
{
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int MB = WM / 32, NB = WN / 32;
    // C tile in LDS.  Strided: [BK][BN + PADS] (row k, column = line).
    // Contiguous: [BM][BK + PADC] (row = line, column k).
    constexpr int PADS = 4, PADC = 1;
    constexpr int TILE = CONTIG ? BM * (BK + PADC) : BK * (BN + PADS);
    extern __shared__ float smem[];
    float* tile0 = smem;
    float* tile1 = smem + TILE;
    float* gl = smem + 2 * TILE;  // generator window

    const int n = op.n, N = n - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // Toeplitz index runs over rows (strided) or columns (contiguous).
    const int tiles_toep = CONTIG ? tiles_n : tiles_m;
    const int tiles_c = CONTIG ? tiles_m : tiles_n;
    TileCoord tc = tile_of(tiles_toep, tiles_c, !CONTIG, total);
    const int m0 = tc.m0 * BM, n0 = tc.n0 * BN;
    const int R0 = CONTIG ? n0 : m0;
    constexpr int RB = CONTIG ? BN : BM;

    // k range (one-sided operators skip the zero triangle)
    int kb = 0, ke = n;
    if (op.lower_only) ke = min(n, R0 + RB);
    if (op.upper_only) kb = (R0 / BK) * BK;
    const int nk = (ke - kb + BK - 1) / BK;
    const int kend = kb + nk * BK;  // padded end

    // generator window: d in [R0 - (kend - 1), R0 + RB - 1 - kb]
    const int dmin = R0 - (kend - 1);
    const int glen = RB + (kend - kb) - 1;
    for (int t = threadIdx.x; t < glen; t += kThreads) {
        const int d = dmin + t;
        gl[t] = (d >= -N && d <= N) ? op.gen[d + N] : 0.f;
    }

    const int64_t lines = lay.lines;
    const float* Cb = C;
    float* Pb = Phi;
    if (!CONTIG) {
        Cb += (int64_t)tc.batch * lay.batch_stride;
        Pb += (int64_t)tc.batch * lay.batch_stride;
    }
    const int64_t js = lay.j_stride;

    // ---- global -> register staging of one C tile
    constexpr int ELEMS = CONTIG ? BM * BK : BK * BN;
    constexpr int PER_THREAD = ELEMS / (kThreads * VEC);
    static_assert(ELEMS % (kThreads * VEC) == 0, "tile not divisible");
    float stage[PER_THREAD][VEC];

    auto load_tile = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            const int e = (q * kThreads + threadIdx.x) * VEC;
            if constexpr (CONTIG) {
                const int r = e / BK, c = e % BK;  // row = line, col = k
                const int64_t line = (int64_t)m0 + r;
                const int k = k0 + c;
                if constexpr (VEC == 4) {
                    if (line < lines && k + 3 < n) {
                        const float4 v = *reinterpret_cast<const float4*>(Cb + line * n + k);
                        stage[q][0] = v.x;
                        stage[q][1] = v.y;
                        stage[q][2] = v.z;
                        stage[q][3] = v.w;
                        continue;
                    }
                }
#pragma unroll
                for (int v = 0; v < VEC; ++v) stage[q][v] = (line < lines && k + v < n) ? Cb[line * n + k + v] : 0.f;
            } else {
                const int r = e / BN, c = e % BN;  // row = k, col = line
                const int k = k0 + r;
                const int64_t line = (int64_t)n0 + c;
                if constexpr (VEC == 4) {
                    if (k < n && line + 3 < lines) {
                        const float4 v = *reinterpret_cast<const float4*>(Cb + (int64_t)k * js + line);
                        stage[q][0] = v.x;
                        stage[q][1] = v.y;
                        stage[q][2] = v.z;
                        stage[q][3] = v.w;
                        continue;
                    }
                }
#pragma unroll
                for (int v = 0; v < VEC; ++v)
                    stage[q][v] = (k < n && line + v < lines) ? Cb[(int64_t)k * js + line + v] : 0.f;
            }
        }
    };
    auto store_tile = [&](float* tile) {
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            const int e = (q * kThreads + threadIdx.x) * VEC;
            if constexpr (CONTIG) {
                const int r = e / BK, c = e % BK;
#pragma unroll
                for (int v = 0; v < VEC; ++v) tile[r * (BK + PADC) + c + v] = stage[q][v];
            } else {
                const int r = e / BN, c = e % BN;
                if constexpr (VEC == 4) {
                    *reinterpret_cast<float4*>(tile + r * (BN + PADS) + c) =
                        make_float4(stage[q][0], stage[q][1], stage[q][2], stage[q][3]);
                } else {
                    tile[r * (BN + PADS) + c] = stage[q][0];
                }
            }
        }
    };

    f32x16 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int li = lane & 31, lk = lane >> 5;
    if (nk > 0) {
        load_tile(kb);
        store_tile(tile0);
    }
    __syncthreads();

    for (int t = 0; t < nk; ++t) {
        const int k0 = kb + t * BK;
        float* cur = (t & 1) ? tile1 : tile0;
        float* nxt = (t & 1) ? tile0 : tile1;
        if (t + 1 < nk) load_tile(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 2) {
            float a[MB], b[NB];
            const int k = k0 + kk + lk;  // global k of this lane's operand element
            if constexpr (CONTIG) {
#pragma unroll
                for (int i = 0; i < MB; ++i) a[i] = cur[(wm * WM + i * 32 + li) * (BK + PADC) + kk + lk];
#pragma unroll
                for (int j = 0; j < NB; ++j) b[j] = gl[(n0 + wn * WN + j * 32 + li) - k - dmin];
            } else {
#pragma unroll
                for (int i = 0; i < MB; ++i) a[i] = gl[(m0 + wm * WM + i * 32 + li) - k - dmin];
#pragma unroll
                for (int j = 0; j < NB; ++j) b[j] = cur[(kk + lk) * (BN + PADS) + wn * WN + j * 32 + li];
            }
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (t + 1 < nk) store_tile(nxt);
        __syncthreads();
    }

    // ---- epilogue: boundary columns and store
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int mm = m0 + wm * WM + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                const int nn = n0 + wn * WN + j * 32 + li;
                if constexpr (CONTIG) {
                    const int64_t line = mm;
                    const int jj = nn;
                    if (line < lines && jj < n) {
                        const float* c = Cb + line * n;
                        float v = acc[i][j][r];
                        v = fmaf(op.corr0[jj], c[0], v);
                        v = fmaf(op.corrN[jj], c[N], v);
                        Pb[line * n + jj] = v;
                    }
                } else {
                    const int jj = mm;
                    const int64_t line = nn;
                    if (jj < n && line < lines) {
                        float v = acc[i][j][r];
                        v = fmaf(op.corr0[jj], Cb[line], v);
                        v = fmaf(op.corrN[jj], Cb[(int64_t)N * js + line], v);
                        Pb[(int64_t)jj * js + line] = v;
                    }
                }
            }
}

template <bool CONTIG, int BM, int BN, int BK, int VEC>
hipError_t run_f32(const AxisOp& op, const AxisLayout& lay, const float* C, float* Phi, hipStream_t s)
{
    const int n = op.n;
    int tiles_m, tiles_n, batches;
    if (CONTIG) {
        tiles_m = (int)((lay.lines + BM - 1) / BM);
        tiles_n = (n + BN - 1) / BN;
        batches = 1;
    } else {
        tiles_m = (n + BM - 1) / BM;
        tiles_n = (int)((lay.lines + BN - 1) / BN);
        batches = lay.batches;
    }
    const int64_t total64 = (int64_t)tiles_m * tiles_n * batches;
    if (total64 > 0x7fffffff) return hipErrorInvalidValue;
    const int total = (int)total64;
    constexpr int TILE = CONTIG ? BM * (BK + 1) : BK * (BN + 4);
    constexpr int RB = CONTIG ? BN : BM;
    const int kspan = ((n + BK - 1) / BK) * BK;
    const size_t lds = sizeof(float) * (2 * TILE + RB + kspan);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL((fractional_f32_mfma<CONTIG, BM, BN, BK, VEC>), dim3(total), dim3(kThreads), lds, s, op, lay,
                       C, Phi, tiles_m, tiles_n, total);
    return hipGetLastError();
}

}  // namespace

bool have_bf16x3() { return false; }

hipError_t launch_fractional(const AxisOp& op, const AxisLayout& lay, int precision, const float* C, float* Phi,
                             hipStream_t s)
{
    if (precision == 2) {
        const int64_t total = lay.contiguous ? lay.lines * op.n : (int64_t)lay.batches * op.n * lay.lines;
        const int64_t blocks = (total + 255) / 256;
        hipLaunchKernelGGL(fractional_simt, dim3((unsigned)blocks), dim3(256), 0, s, op, lay, C, Phi);
        return hipGetLastError();
    }
    // FP32 MFMA (the BF16 path dispatches here too until its kernel exists)
    if (lay.contiguous) {
        const bool vec = (op.n % 4) == 0;
        if (op.n <= 256 || lay.lines * op.n <= (1 << 22)) {
            return vec ? run_f32<true, 64, 64, 32, 4>(op, lay, C, Phi, s) : run_f32<true, 64, 64, 32, 1>(op, lay, C, Phi, s);
        }
        return vec ? run_f32<true, 128, 128, 32, 4>(op, lay, C, Phi, s) : run_f32<true, 128, 128, 32, 1>(op, lay, C, Phi, s);
    }
    const bool vec = (lay.lines % 4) == 0 && (lay.j_stride % 4) == 0 && (lay.batch_stride % 4) == 0;
    if (lay.lines * op.n * lay.batches <= (1 << 22)) {
        return vec ? run_f32<false, 64, 64, 32, 4>(op, lay, C, Phi, s) : run_f32<false, 64, 64, 32, 1>(op, lay, C, Phi, s);
    }
    return vec ? run_f32<false, 128, 128, 32, 4>(op, lay, C, Phi, s) : run_f32<false, 128, 128, 32, 1>(op, lay, C, Phi, s);
}

}  // namespace lbm
