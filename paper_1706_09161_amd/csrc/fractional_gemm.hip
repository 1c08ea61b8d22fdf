// fractional_gemm.hip -- the fractional term of Algorithm 1 (first stage of
// the time loop) on gfx950.
//
// Along axis mu every grid line is multiplied by the same matrix
//   K[j][k] = g dx^gamma / Gamma(2+gamma) * (p c+_{kj}(gamma) + (1-p) c-_{kj}(gamma, N))
// (Sec. 2.4, equations (1Dminus_discret), (c+), (c-), (XXminus_discret)),
// which is Toeplitz except in its first and last columns:
//   K[j][k] = T(j - k) for 0 < k < N,  K[j][0] = col0[j],  K[j][N] = colN[j].
// So Phi = K C for all lines at once is a dense contraction (n x n times
// n x lines).  It runs as a GEMM on the matrix cores over the interior columns
// (the end columns' C values are zeroed as they are loaded); the Toeplitz
// operand is never stored as an n x n matrix: each workgroup keeps the 2n-1
// generator values it needs in LDS and reads fragments from there, and the
// two boundary columns are a rank-2 epilogue.  (The adjoint's transposed
// parts, ends_excluded = 0, sum every column and add col0 / colN on top.)
//
// Layouts (see AxisLayout):
//   x axis  ("contiguous"): D[line][j]      = sum_k C[line][k] T(j - k)
//   y, z    ("strided")   : D[j][line]      = sum_k T(j - k) C[k][line]
// In both cases the MFMA's lane-varying output index is the memory-contiguous
// one, so stores are coalesced.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

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
    const int k_lo = op.ends_excluded ? 1 : 0, k_hi = op.ends_excluded ? N : n;  // Toeplitz columns summed
    if (lay.contiguous) {
        const int64_t line = t / n;
        const int j = (int)(t % n);
        const float* c = C + line * n;
        float acc = 0.f;
        for (int k = k_lo; k < k_hi; ++k) acc = fmaf(gen[j - k], c[k], acc);
        acc = fmaf(op.col0[j], c[0], acc);
        acc = fmaf(op.colN[j], c[N], acc);
        Phi[line * n + j] = acc;
    } else {
        const int64_t line = t % lay.lines;
        const int64_t rest = t / lay.lines;
        const int j = (int)(rest % n);
        const int64_t b = rest / n;
        const float* c = C + b * lay.batch_stride + line;
        float acc = 0.f;
        for (int k = k_lo; k < k_hi; ++k) acc = fmaf(gen[j - k], c[(int64_t)k * lay.j_stride], acc);
        acc = fmaf(op.col0[j], c[0], acc);
        acc = fmaf(op.colN[j], c[(int64_t)N * lay.j_stride], acc);
        Phi[b * lay.batch_stride + (int64_t)j * lay.j_stride + line] = acc;
    }
}

// ---------------------------------------------------------------------------
// FP32 MFMA kernel, v_mfma_f32_32x32x2_f32.
//
// Operand convention for 32x32x2: lane l supplies A(i = l%32, kk = l/32) and
// B(kk = l/32, j = l%32); accumulator register r of lane l holds
// D(8*(r/4) + 4*(l/32) + r%4, l%32).
//
// Workgroup tile BM x BN, 4 wavefronts arranged WAVES_M x WAVES_N x KSPLIT.
// Every wavefront owns a 64 x 64 output tile (2 x 2 blocks of 32 x 32, four
// independent accumulator chains); with KSPLIT > 1 the wavefronts of a
// workgroup split each k chunk between them and their partial tiles are
// summed through LDS at the end.  Small grids use 64 x 64 x (split-K 4) to
// keep enough workgroups for 256 CUs; large grids use 128 x 128.
//
// All axes of one time step go in one launch: workgroup ids are split into
// per-axis ranges, axis 0 (the contiguous x axis) first.


template <bool CONTIG, int BM, int BN, int BK, int WAVES_M, int WAVES_N, int KSPLIT, int VEC>
__device__ __forceinline__ void fractional_tile(const AxisOp& op, const AxisLayout& lay, const float* __restrict__ C,
                                                float* __restrict__ Phi, int tiles_m, int tiles_n, int bid, int total,
                                                float* smem)
{
    static_assert(WAVES_M * WAVES_N * KSPLIT == kWaves, "4 wavefronts per workgroup");
    static_assert(BM == WAVES_M * 64 && BN == WAVES_N * 64, "64 x 64 per wavefront");
    static_assert(BK % (2 * KSPLIT) == 0, "k chunk");
    constexpr int MB = 2, NB = 2;
    constexpr int KW = BK / KSPLIT;  // k values per wavefront and chunk
    constexpr int PADS = 4, PADC = 1;
    constexpr int TILE = CONTIG ? BM * (BK + PADC) : BK * (BN + PADS);
    float* tile0 = smem;
    float* tile1 = smem + TILE;
    float* gl = smem + 2 * TILE;  // generator window

    const int n = op.n, N = n - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wk = wave % KSPLIT;
    const int wmn = wave / KSPLIT;
    const int wm = wmn / WAVES_N, wn = wmn % WAVES_N;

    // tile of this workgroup; the Toeplitz index runs over rows (strided) or
    // columns (contiguous); consecutive ids on one XCD share a panel of C
    const int tiles_toep = CONTIG ? tiles_n : tiles_m;
    const int tiles_c = CONTIG ? tiles_m : tiles_n;
    int lin = bid;
    if ((total & 7) == 0) lin = (bid & 7) * (total >> 3) + (bid >> 3);
    const int tt = lin % tiles_toep;
    const int rest = lin / tiles_toep;
    const int tcid = rest % tiles_c;
    const int batch = rest / tiles_c;
    const int m0 = (CONTIG ? tcid : tt) * BM, n0 = (CONTIG ? tt : tcid) * BN;
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
        Cb += (int64_t)batch * lay.batch_stride;
        Pb += (int64_t)batch * lay.batch_stride;
    }
    const int64_t js = lay.j_stride;

    // ---- global -> register staging of one C tile
    constexpr int ELEMS = CONTIG ? BM * BK : BK * BN;
    constexpr int PER_THREAD = ELEMS / (kThreads * VEC);
    static_assert(ELEMS % (kThreads * VEC) == 0, "tile not divisible");
    float stage[PER_THREAD][VEC];

    // A chunk is "full" when all its lines and k are in range: then the loads
    // need no per-element checks (uniform branch per chunk).
    const bool lines_full = CONTIG ? ((int64_t)m0 + BM <= lines) : ((int64_t)n0 + BN <= lines);
    auto load_tile = [&](int k0) {
        if constexpr (VEC == 4) {
            if (lines_full && k0 + BK <= n) {
#pragma unroll
                for (int q = 0; q < PER_THREAD; ++q) {
                    const int e = (q * kThreads + threadIdx.x) * VEC;
                    float4 v;
                    if constexpr (CONTIG) {
                        const int r = e / BK, c = e % BK;
                        v = *reinterpret_cast<const float4*>(Cb + ((int64_t)m0 + r) * n + k0 + c);
                    } else {
                        const int r = e / BN, c = e % BN;
                        v = *reinterpret_cast<const float4*>(Cb + (int64_t)(k0 + r) * js + n0 + c);
                    }
                    stage[q][0] = v.x;
                    stage[q][1] = v.y;
                    stage[q][2] = v.z;
                    stage[q][3] = v.w;
                }
                return;
            }
        }
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
    // forward operators leave columns k = 0 and k = N out of the Toeplitz sum
    // (the epilogue adds the whole boundary columns): zero them in the staged
    // chunk that holds them
    auto mask_ends = [&](int k0) {
        if (!op.ends_excluded || (k0 > 0 && k0 + BK <= N)) return;
#pragma unroll
        for (int q = 0; q < PER_THREAD; ++q) {
            const int e = (q * kThreads + threadIdx.x) * VEC;
            if constexpr (CONTIG) {
                const int k = k0 + e % BK;
#pragma unroll
                for (int v = 0; v < VEC; ++v)
                    if (k + v == 0 || k + v == N) stage[q][v] = 0.f;
            } else {
                const int k = k0 + e / BN;
                if (k == 0 || k == N)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) stage[q][v] = 0.f;
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
    const int rowA = (CONTIG ? 0 : m0) + wm * 64;  // first Toeplitz row / C-tile row of this wavefront
    const int colB = (CONTIG ? n0 : 0) + wn * 64;
    load_tile(kb);
    mask_ends(kb);  // the first chunk is consumed right away
    store_tile(tile0);
    __syncthreads();

    for (int t = 0; t < nk; ++t) {
        const int k0 = kb + t * BK;
        const float* cur = (t & 1) ? tile1 : tile0;
        float* nxt = (t & 1) ? tile0 : tile1;
        if (t + 1 < nk) load_tile(k0 + BK);
        // operand fragments of k step kk (k = kk + lk within the chunk)
        auto frags = [&](int kk, float (&a)[MB], float (&b)[NB]) {
            const int k = k0 + kk + lk;  // global k of this lane's operand element
            if constexpr (CONTIG) {
#pragma unroll
                for (int i = 0; i < MB; ++i) a[i] = cur[(rowA + i * 32 + li) * (BK + PADC) + kk + lk];
#pragma unroll
                for (int j = 0; j < NB; ++j) b[j] = gl[(colB + j * 32 + li) - k - dmin];
            } else {
#pragma unroll
                for (int i = 0; i < MB; ++i) a[i] = gl[(rowA + i * 32 + li) - k - dmin];
#pragma unroll
                for (int j = 0; j < NB; ++j) b[j] = cur[(kk + lk) * (BN + PADS) + colB + j * 32 + li];
            }
        };
        // fragments are read two k steps ahead of the MFMAs that use them
        constexpr int NSTEP = KW / 2;
        float a[3][MB], b[3][NB];
        frags(wk * KW, a[0], b[0]);
        if (NSTEP > 1) frags(wk * KW + 2, a[1], b[1]);
#pragma unroll
        for (int st = 0; st < NSTEP; ++st) {
            if (st + 2 < NSTEP) frags(wk * KW + 2 * (st + 2), a[(st + 2) % 3], b[(st + 2) % 3]);
            // keep the reads of step st + 2 ahead of the MFMAs of step st (the
            // scheduler would otherwise sink them next to their use)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st % 3][i], b[st % 3][j], acc[i][j], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (t + 1 < nk) {
            mask_ends(k0 + BK);  // where the prefetched chunk is consumed
            store_tile(nxt);
        }
        __syncthreads();
    }

    // ---- split-K reduction: every wavefront parks its partial tile in LDS
    // (the C tiles are dead after the last barrier); the wavefronts of one
    // output tile then each finish one of its four 32 x 32 blocks.
    int blk_lo = 0, blk_hi = MB * NB;
    if constexpr (KSPLIT > 1) {
        float* red = smem;  // [KSPLIT * WAVES_M * WAVES_N][MB*NB][16][64]
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) red[((wave * MB * NB + i * NB + j) * 16 + r) * 64 + lane] = acc[i][j][r];
        __syncthreads();
        // wavefront wk of this output tile sums block(s) [wk * 4 / KSPLIT, (wk+1) * 4 / KSPLIT)
        blk_lo = wk * (MB * NB) / KSPLIT;
        blk_hi = (wk + 1) * (MB * NB) / KSPLIT;
#pragma unroll
        for (int bi = 0; bi < MB * NB; ++bi) {
            if (bi < blk_lo || bi >= blk_hi) continue;
            const int i = bi / NB, j = bi % NB;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float v = 0.f;
#pragma unroll
                for (int s = 0; s < KSPLIT; ++s)
                    v += red[(((wmn * KSPLIT + s) * MB * NB + bi) * 16 + r) * 64 + lane];
                acc[i][j][r] = v;
            }
        }
    }

    // ---- epilogue: boundary columns and store
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int bi = i * NB + j;
            if (bi < blk_lo || bi >= blk_hi) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int mm = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
                const int nn = n0 + wn * 64 + j * 32 + li;
                if constexpr (CONTIG) {
                    const int64_t line = mm;
                    const int jj = nn;
                    if (line < lines && jj < n) {
                        const float* c = Cb + line * n;
                        float v = acc[i][j][r];
                        v = fmaf(op.col0[jj], c[0], v);
                        v = fmaf(op.colN[jj], c[N], v);
                        Pb[line * n + jj] = v;
                    }
                } else {
                    const int jj = mm;
                    const int64_t line = nn;
                    if (jj < n && line < lines) {
                        float v = acc[i][j][r];
                        v = fmaf(op.col0[jj], Cb[line], v);
                        v = fmaf(op.colN[jj], Cb[(int64_t)N * js + line], v);
                        Pb[(int64_t)jj * js + line] = v;
                    }
                }
            }
        }
}

template <int BM, int BN, int BK, int WAVES_M, int WAVES_N, int KSPLIT, int VEC_X, int VEC_S>
__global__ __launch_bounds__(kThreads) void fractional_f32_mfma(FracLaunch L)
{
    extern __shared__ float smem[];
    const int bid = blockIdx.x;
    int axis = 0;
    while (axis + 1 < L.naxes && bid >= L.first[axis + 1]) ++axis;  // uniform per workgroup
    const int local = bid - L.first[axis];
    const int total = L.first[axis + 1] - L.first[axis];
    if (axis == 0)
        fractional_tile<true, BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, VEC_X>(L.op[0], L.lay[0], L.C[0], L.Phi[0],
                                                                          L.tiles_m[0], L.tiles_n[0], local, total,
                                                                          smem);
    else
        fractional_tile<false, BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, VEC_S>(L.op[axis], L.lay[axis], L.C[axis],
                                                                           L.Phi[axis], L.tiles_m[axis],
                                                                           L.tiles_n[axis], local, total, smem);
}

template <int BM, int BN, int BK, int WAVES_M, int WAVES_N, int KSPLIT>
hipError_t run_f32(FracLaunch& L, hipStream_t s)
{
    size_t lds = 0;
    int64_t grid = 0;
    for (int a = 0; a < L.naxes; ++a) {
        const AxisOp& op = L.op[a];
        const AxisLayout& lay = L.lay[a];
        const bool contig = lay.contiguous != 0;
        if (contig) {
            L.tiles_m[a] = (int)((lay.lines + BM - 1) / BM);
            L.tiles_n[a] = (op.n + BN - 1) / BN;
        } else {
            L.tiles_m[a] = (op.n + BM - 1) / BM;
            L.tiles_n[a] = (int)((lay.lines + BN - 1) / BN);
        }
        const int64_t tiles = (int64_t)L.tiles_m[a] * L.tiles_n[a] * (contig ? 1 : lay.batches);
        L.first[a] = (int)grid;
        grid += tiles;
        const int tile = contig ? BM * (BK + 1) : BK * (BN + 4);
        const int rb = contig ? BN : BM;
        const int kspan = ((op.n + BK - 1) / BK) * BK;
        size_t need = sizeof(float) * (2 * tile + rb + kspan);
        if (KSPLIT > 1) need = need > sizeof(float) * 4 * 4 * 16 * 64 ? need : sizeof(float) * 4 * 4 * 16 * 64;
        lds = need > lds ? need : lds;
    }
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    L.first[L.naxes] = (int)grid;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const bool vx = (L.op[0].n % 4) == 0;
    bool vs = true;
    for (int a = 1; a < L.naxes; ++a)
        vs = vs && (L.lay[a].lines % 4) == 0 && (L.lay[a].j_stride % 4) == 0 && (L.lay[a].batch_stride % 4) == 0;
    auto go = [&](auto kern) -> hipError_t {
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), lds, s, L);
        return hipGetLastError();
    };
    if (vx && vs) return go(fractional_f32_mfma<BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, 4, 4>);
    if (vx) return go(fractional_f32_mfma<BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, 4, 1>);
    if (vs) return go(fractional_f32_mfma<BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, 1, 4>);
    return go(fractional_f32_mfma<BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, 1, 1>);
}

// ---------------------------------------------------------------------------
// Register-direct kernel.  One wavefront computes 32 lines x (32 NBJ) outputs
// of one axis over its share of k with v_mfma_f32_32x32x2f32, in groups of 8 k
// (4 MFMA steps of 2 k).  The KSPLIT wavefronts of a line block take the
// groups of the k range round robin (wavefront wk: groups wk, wk + KSPLIT, ...;
// its first k is kw), and the k order inside a group is permuted so that each
// lane consumes 4 consecutive k: at step s of group g the lane half lh works
// on k = kw + 8 KSPLIT g + 4 lh + s (both operands use the same map, so the
// sum is unchanged).  Dealing the groups round robin puts every stretch of
// large products (a pulse in C) into all KSPLIT accumulators rather than one,
// and with 128-output tiles each wavefront alternates its groups between two
// accumulator sets: each FP32 running sum is then about 1/(2 KSPLIT) of the
// total, and so is its rounding error (at 4096^2 after 100 steps the C error
// against the FP64 oracle is 4.5e-6, 6.4e-6 with one set per wavefront,
// 1.5e-5 with contiguous k shares).  Hence
//  * C comes straight from global memory into registers, P groups ahead, one
//    16-byte load per lane and group along the contiguous axis (4 loads,
//    coalesced across consecutive lines, along a strided axis; the KSPLIT
//    wavefronts together read whole 32 KSPLIT-byte spans of a line); no LDS,
//    no barrier in the k loop;
//  * the Toeplitz values of a lane for one output block and group,
//    T(d0), T(d0 - 1), T(d0 - 2), T(d0 - 3), are 4 consecutive words of an LDS
//    window that stores T with d decreasing (two ds_read2 per block).
// A workgroup has 4 wavefronts: WL line blocks x KSPLIT k-shares, summed
// through LDS in a fixed order (deterministic).  Registers stay below 256 per
// lane, so two workgroups share a CU and one's set-up and epilogue overlap the
// other's MFMAs.
template <bool CONTIG, int NBJ, int WL, int KSPLIT, int P, bool KFULL>
__device__ __forceinline__ void f32_ring_tile(const AxisOp& op, const AxisLayout& lay, const float* __restrict__ C,
                                              float* __restrict__ Phi, int tiles_l, int tiles_j, int bid, int total,
                                              int lgroup, unsigned char* smem)
{
    static_assert(WL * KSPLIT == kWaves, "4 wavefronts per workgroup");
    constexpr int JT = 32 * NBJ;  // outputs per tile
    static_assert(JT <= kThreads, "one thread per output of the tile");
    constexpr int LT = 32 * WL;  // lines per tile
    const int n = op.n, N = n - 1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wl = wave / KSPLIT, wk = wave % KSPLIT;
    const int li = lane & 31, lh = lane >> 5;

    // tile of this workgroup: contiguous tile ranges per XCD; one-sided
    // operators start their longest tiles first (see the split-BF16 kernel),
    // within groups of `lgroup` line tiles: the C panels of one group fit the
    // XCD's L2 while all its output tiles run, so each panel is fetched once
    int lin = bid;
    if ((total & 7) == 0) {
        const int S = total >> 3, x = bid & 7, i = bid >> 3;
        lin = x * S + i;
        if ((op.lower_only || op.upper_only) && S % tiles_j == 0) {
            const int lpx = S / tiles_j;  // line tiles per XCD
            const int G = (lgroup > 0 && lpx % lgroup == 0) ? lgroup : lpx;
            const int per = G * tiles_j, g = i / per, r = i % per;
            lin = x * S + (g * G + r % G) * tiles_j + r / G;
        }
    }
    int jt = lin % tiles_j;
    if (op.lower_only) jt = tiles_j - 1 - jt;
    const int rest = lin / tiles_j;
    const int lt = rest % tiles_l;
    const int batch = rest / tiles_l;
    const int j0 = jt * JT;
    const int64_t lines = lay.lines;
    const int64_t line0 = (int64_t)lt * LT + 32 * wl;
    const int64_t js = lay.j_stride;
    const float* Cb = C;
    float* Pb = Phi;
    if (!CONTIG) {
        Cb += (int64_t)batch * lay.batch_stride;
        Pb += (int64_t)batch * lay.batch_stride;
    }

    // k range in groups of 8 (one-sided operators skip the zero triangle)
    int kb = 0, ke = n;
    if (op.lower_only) ke = min(n, j0 + JT);
    if (op.upper_only) kb = (min(j0, n - 1) / 8) * 8;
    const int groups = (ke - kb + 7) / 8;  // >= 1
    const int kend = kb + 8 * groups;
    // the wavefronts of a workgroup take the groups round robin: group g of
    // wavefront wk is group KSPLIT g + wk of the range
    constexpr int GS = 8 * KSPLIT;  // k distance between a wavefront's groups
    const int my_groups = groups > wk ? (groups - wk + KSPLIT - 1) / KSPLIT : 0;
    const int kw = kb + 8 * min(wk, groups - 1);
    const int last = max(my_groups, 1) - 1;

    // C of a group: lane = (line li, k half lh), 4 consecutive k
    const int64_t my_line = min(line0 + li, lines - 1);  // rows past the end are computed, never stored
    const float* q = CONTIG ? Cb + my_line * n + kw + 4 * lh : Cb + (int64_t)(kw + 4 * lh) * js + my_line;
    const bool ends = op.ends_excluded != 0;
    auto load_c = [&](int g, f32x4& v) {
        const int gc = min(g, last);
        if constexpr (KFULL) {
            if constexpr (CONTIG) {
                v = *reinterpret_cast<const f32x4*>(q + GS * gc);
            } else {
                const float* a = q + (int64_t)(GS * gc) * js;
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = a[(int64_t)e * js];
            }
        } else {
            const int k = kw + GS * gc + 4 * lh;
            const int64_t stride = CONTIG ? 1 : js;
            const float* a = q + (int64_t)(GS * gc) * stride;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = k + e < n;
                const float x = *(ok ? a + e * stride : Cb);
                v[e] = ok ? x : 0.f;
            }
        }
    };
    // Forward operators leave columns k = 0 and k = N out of the Toeplitz sum
    // (the epilogue adds the whole boundary columns).  k ranges start at
    // multiples of 8, so k = 0 is element 0 of lane half 0 in group 0 of the
    // wavefront that starts at 0 (zeroed once, before the loop), and k = N is
    // element N % 4 of lane half (N % 8) / 4 in the one group holding it;
    // with n % 8 == 0 that element is always the last.  It is zeroed with a
    // select where the group is consumed (no branch: the interleaved MFMA /
    // load block of a group stays one block).
    const bool lane_k0 = ends && kw == 0 && lh == 0;
    const bool lane_kN = ends && lh == (N % 8) / 4;
    const int g_kN = (ends && N >= kw && (N - kw) % GS < 8 && (N - kw) / GS < my_groups) ? (N - kw) / GS : -1;
    // C of group g as the MFMAs take it: zero past the end of the range (those
    // groups re-read the last one), and k = N left out.  One select per
    // element either way: with n % 8 == 0 the k = N condition only widens the
    // last element's mask.
    auto zero_dead_and_kN = [&](int g, f32x4& v) {
        const bool dead = g >= my_groups;
        const bool kn = lane_kN && g == g_kN;
        if constexpr (KFULL) {
#pragma unroll
            for (int e = 0; e < 3; ++e) v[e] = dead ? 0.f : v[e];
            v[3] = (dead || kn) ? 0.f : v[3];
        } else {
            const int e_kN = N % 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (dead || (kn && e == e_kN)) ? 0.f : v[e];
        }
    };

    // LDS: col0 | colN | C at the walls of each line (contiguous axis) |
    // Toeplitz window, d decreasing (later the k-share reduction)
    float* c0s = reinterpret_cast<float*>(smem);
    float* cNs = c0s + JT;
    float* w0s = cNs + JT;
    float* wNs = w0s + LT;
    float* win = wNs + LT;
    const int wlen = JT - 1 + (kend - kb);  // word m holds T(dmax - m)
    const int dmax = j0 + JT - 1 - kb;
    constexpr int FU = 8;
    auto fill_load = [&](int base, float (&v)[FU]) {
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int m = base + u * kThreads + threadIdx.x;
            const int d = dmax - m;
            v[u] = (m < wlen && d >= -N && d <= N) ? op.gen[d + N] : 0.f;
        }
    };
    auto fill_store = [&](int base, const float (&v)[FU]) {
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int m = base + u * kThreads + threadIdx.x;
            if (m < wlen) win[m] = v[u];
        }
    };
    // loads complete in issue order: set-up loads first, then the C prefetch
    float fv[FU];
    fill_load(0, fv);
    float cv0 = 0.f, cvN = 0.f, wv0 = 0.f, wvN = 0.f;
    {
        const int t = threadIdx.x;
        if (t < JT && j0 + t < n) {
            cv0 = op.col0[j0 + t];
            cvN = op.colN[j0 + t];
        }
        if (CONTIG && t < LT) {
            const int64_t line = min((int64_t)lt * LT + t, lines - 1);
            wv0 = Cb[line * n];
            wvN = Cb[line * n + N];
        }
    }
    float b0 = 0.f, bN = 0.f;
    if constexpr (!CONTIG) {
        b0 = Cb[my_line];
        bN = Cb[(int64_t)N * js + my_line];
    }
    f32x4 craw[P];
#pragma unroll
    for (int g = 0; g < P; ++g) load_c(g, craw[g]);
    fill_store(0, fv);
    {
        const int t = threadIdx.x;
        if (t < JT) {
            c0s[t] = cv0;
            cNs[t] = cvN;
        }
        if (CONTIG && t < LT) {
            w0s[t] = wv0;
            wNs[t] = wvN;
        }
    }
    for (int base = FU * kThreads; base < wlen; base += FU * kThreads) {  // long axes only
        fill_load(base, fv);
        fill_store(base, fv);
    }
    lds_barrier();  // the C prefetch stays in flight
    craw[0][0] = lane_k0 ? 0.f : craw[0][0];  // k = 0 is only ever in group 0

    // Two accumulator sets where registers allow (NBJ <= 4): groups alternate
    // between them, so each FP32 running sum takes half of the wavefront's
    // products (see the rounding note above the kernel).
    constexpr bool TWO = NBJ <= 4;
    constexpr int NA = TWO ? NBJ : 1;
    f32x16 acc[NBJ], acc2[NA];
#pragma unroll
    for (int c = 0; c < NBJ; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;
#pragma unroll
    for (int c = 0; c < NA; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc2[c][r] = 0.f;

    if (my_groups > 0) {
        // Toeplitz values of block c, group g: window words m0 .. m0 + 3
        const int mbase = dmax - j0 - li + kw + 4 * lh;
        auto load_t = [&](int g, f32x4 (&tv)[NBJ]) {
            const int gc = min(g, last);
#pragma unroll
            for (int c = 0; c < NBJ; ++c) {
                const int m0 = mbase - 32 * c + GS * gc;
#pragma unroll
                for (int e = 0; e < 4; ++e) tv[c][e] = win[m0 + e];
            }
        };
        f32x4 tf[2][NBJ];
        load_t(0, tf[0]);
        for (int g0 = 0; g0 < my_groups; g0 += 2 * P) {
#pragma unroll
            for (int u = 0; u < 2 * P; ++u) {
                const int g = g0 + u;
                // C of this group (zero past the end of the range), then reuse its slot for group g + P
                f32x4 cur = craw[u % P];
                zero_dead_and_kN(g, cur);
                load_c(g + P, craw[u % P]);
                load_t(g + 1, tf[(u + 1) & 1]);
#pragma unroll
                for (int st = 0; st < 4; ++st)
#pragma unroll
                    for (int c = 0; c < NBJ; ++c) {
                        f32x16& a = (TWO && (u & 1)) ? acc2[TWO ? c : 0] : acc[c];
                        if constexpr (CONTIG)
                            a = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[st], tf[u & 1][c][st], a, 0, 0, 0);
                        else
                            a = __builtin_amdgcn_mfma_f32_32x32x2f32(tf[u & 1][c][st], cur[st], a, 0, 0, 0);
                    }
#pragma unroll
                for (int i = 0; i < 4 * NBJ; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
                    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
                    __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);  // VALU
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    if constexpr (TWO) {
#pragma unroll
        for (int c = 0; c < NBJ; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[c][r] += acc2[TWO ? c : 0][r];
    }
    // The output of a wavefront is NBJ blocks x 4 groups of 4 rows ("units",
    // u = 4 c + r4).  With k split across waves, the partial tiles are summed
    // through LDS and the units are dealt out to the KSPLIT wavefronts.
    constexpr int U = 4 * NBJ;
    static_assert(U % KSPLIT == 0, "units divide among the k shares");
    int u_lo = 0, u_hi = U;
    if constexpr (KSPLIT > 1) {
        __syncthreads();  // every wavefront is done with the window
        float* red = win;
        u_lo = wk * (U / KSPLIT);
        u_hi = u_lo + U / KSPLIT;
        // the units other k shares sum go through LDS; a wavefront's own
        // units stay in registers (same fixed summation order, s = 0, 1, ...)
#pragma unroll
        for (int c = 0; c < NBJ; ++c)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int u = 4 * c + r4;
                if (u >= u_lo && u < u_hi) continue;
                float4 v = make_float4(acc[c][4 * r4], acc[c][4 * r4 + 1], acc[c][4 * r4 + 2], acc[c][4 * r4 + 3]);
                *reinterpret_cast<float4*>(red + (((wave * NBJ + c) * 4 + r4) * 64 + lane) * 4) = v;
            }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NBJ; ++c)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int u = 4 * c + r4;
                if (u < u_lo || u >= u_hi) continue;
                float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int s = 0; s < KSPLIT; ++s) {
                    const float4 v =
                        s == wk ? make_float4(acc[c][4 * r4], acc[c][4 * r4 + 1], acc[c][4 * r4 + 2], acc[c][4 * r4 + 3])
                                : *reinterpret_cast<const float4*>(
                                      red + ((((wl * KSPLIT + s) * NBJ + c) * 4 + r4) * 64 + lane) * 4);
                    sum.x += v.x;
                    sum.y += v.y;
                    sum.z += v.z;
                    sum.w += v.w;
                }
                acc[c][4 * r4] = sum.x;
                acc[c][4 * r4 + 1] = sum.y;
                acc[c][4 * r4 + 2] = sum.z;
                acc[c][4 * r4 + 3] = sum.w;
            }
    }

    // epilogue: boundary columns (rank-2 correction) and stores
    if constexpr (CONTIG) {
        // rows = lines (8 r4 + 4 lh + e), columns = outputs j0 + 32 c + li
#pragma unroll
        for (int c = 0; c < NBJ; ++c) {
            const int jl = 32 * c + li, j = j0 + jl;
            const float k0 = c0s[jl], kN = cNs[jl];
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int u = 4 * c + r4;
                if (u < u_lo || u >= u_hi) continue;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int tl = 32 * wl + 8 * r4 + 4 * lh + e;
                    const int64_t line = (int64_t)lt * LT + tl;
                    if (line < lines && j < n) {
                        float v = acc[c][4 * r4 + e];
                        v = fmaf(k0, w0s[tl], v);
                        v = fmaf(kN, wNs[tl], v);
                        Pb[line * n + j] = v;
                    }
                }
            }
        }
    } else {
        const int64_t line = line0 + li;
#pragma unroll
        for (int c = 0; c < NBJ; ++c)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                const int u = 4 * c + r4;
                if (u < u_lo || u >= u_hi) continue;
                const int jl0 = 32 * c + 8 * r4 + 4 * lh;  // 4 consecutive outputs
                const float4 k0 = *reinterpret_cast<const float4*>(c0s + jl0);
                const float4 kN = *reinterpret_cast<const float4*>(cNs + jl0);
                const float k0v[4] = {k0.x, k0.y, k0.z, k0.w}, kNv[4] = {kN.x, kN.y, kN.z, kN.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int j = j0 + jl0 + e;
                    if (line < lines && j < n) {
                        float v = acc[c][4 * r4 + e];
                        v = fmaf(k0v[e], b0, v);
                        v = fmaf(kNv[e], bN, v);
                        Pb[(int64_t)j * js + line] = v;
                    }
                }
            }
    }
}

template <int NBJ, int WL, int KSPLIT, int P, bool KFULL>
__global__ __launch_bounds__(kThreads, 2) void fractional_f32_ring(FracLaunch L)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_r[];
    const int bid = blockIdx.x;
    int axis = 0;
    while (axis + 1 < L.naxes && bid >= L.first[axis + 1]) ++axis;
    const int local = bid - L.first[axis];
    const int total = L.first[axis + 1] - L.first[axis];
    if (L.lay[axis].contiguous)
        f32_ring_tile<true, NBJ, WL, KSPLIT, P, KFULL>(L.op[axis], L.lay[axis], L.C[axis], L.Phi[axis],
                                                       L.tiles_m[axis], L.tiles_n[axis], local, total, L.lgroup,
                                                       smem_r);
    else
        f32_ring_tile<false, NBJ, WL, KSPLIT, P, KFULL>(L.op[axis], L.lay[axis], L.C[axis], L.Phi[axis],
                                                        L.tiles_m[axis], L.tiles_n[axis], local, total, L.lgroup,
                                                        smem_r);
}

// tiles_m = line tiles (32 WL lines), tiles_n = output tiles (32 NBJ outputs)
template <int NBJ, int WL, int KSPLIT>
void f32_ring_grid(FracLaunch& L, int64_t& grid, size_t& lds)
{
    grid = 0;
    lds = 0;
    for (int a = 0; a < L.naxes; ++a) {
        const AxisOp& op = L.op[a];
        const AxisLayout& lay = L.lay[a];
        L.tiles_m[a] = (int)((lay.lines + 32 * WL - 1) / (32 * WL));
        L.tiles_n[a] = (op.n + 32 * NBJ - 1) / (32 * NBJ);
        L.first[a] = (int)grid;
        grid += (int64_t)L.tiles_m[a] * L.tiles_n[a] * (lay.contiguous ? 1 : lay.batches);
        const size_t kspan = (size_t)((op.n + 7) / 8) * 8;
        size_t window = sizeof(float) * (32 * NBJ + kspan);
        const size_t red = KSPLIT > 1 ? sizeof(float) * kWaves * NBJ * 16 * 64 : 0;
        window = window > red ? window : red;
        const size_t need = sizeof(float) * (2 * 32 * NBJ + 2 * 32 * WL) + window;
        lds = need > lds ? need : lds;
    }
}

template <int NBJ, int WL, int KSPLIT, int P>
hipError_t run_f32_ring(FracLaunch& L, hipStream_t s)
{
    int64_t grid = 0;
    size_t lds = 0;
    f32_ring_grid<NBJ, WL, KSPLIT>(L, grid, lds);
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    L.first[L.naxes] = (int)grid;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    // One-sided operators: groups of line tiles whose C panels (32 WL lines x
    // n values each) fill at most the 4 MB L2 of an XCD.  At 4096^2 (8 tiles
    // of 32 lines per group) the GEMM's L2 misses fall from 5.3x to 1.3x the
    // C it needs, at the same speed (1107 / 1111 us; 4 tiles: 1.10x but
    // 1125 us, 2 tiles: 1.51x, 1182 us).  LBM_FP32_LGROUP overrides (tuning).
    {
        int64_t nmax = 1;
        for (int a = 0; a < L.naxes; ++a) nmax = L.op[a].n > nmax ? L.op[a].n : nmax;
        int g = 1;
        while (2 * g * (int64_t)(32 * WL) * nmax * 4 <= ((int64_t)4 << 20)) g *= 2;
        L.lgroup = g;
    }
    if (const char* e = getenv("LBM_FP32_LGROUP")) L.lgroup = atoi(e);
    auto go = [&](auto kern) -> hipError_t {
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), lds, s, L);
        return hipGetLastError();
    };
    bool kfull = true;  // every axis a multiple of 8: no group passes the end of an axis
    for (int a = 0; a < L.naxes; ++a) kfull = kfull && (L.op[a].n % 8) == 0;
    if (kfull) return go(fractional_f32_ring<NBJ, WL, KSPLIT, P, true>);
    return go(fractional_f32_ring<NBJ, WL, KSPLIT, P, false>);
}

}  // namespace

namespace {
hipError_t run_f32_auto(FracLaunch& L, hipStream_t s);
}

hipError_t launch_fractional(const AxisOp* ops, const AxisLayout* lays, int naxes, int precision, const float* C,
                             int64_t in_stride, float* Phi, int64_t nodes, hipStream_t s)
{
    if (precision == 2) {
        for (int a = 0; a < naxes; ++a) {
            const AxisOp& op = ops[a];
            const AxisLayout& lay = lays[a];
            const int64_t total = lay.contiguous ? lay.lines * op.n : (int64_t)lay.batches * op.n * lay.lines;
            const int64_t blocks = (total + 255) / 256;
            hipLaunchKernelGGL(fractional_simt, dim3((unsigned)blocks), dim3(256), 0, s, op, lay, C + a * in_stride,
                               Phi + a * nodes);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    FracLaunch L;
    memset(&L, 0, sizeof(L));
    L.naxes = naxes;
    for (int a = 0; a < naxes; ++a) {
        L.op[a] = ops[a];
        L.lay[a] = lays[a];
        L.C[a] = C + a * in_stride;
        L.Phi[a] = Phi + a * nodes;
    }
    if (precision == 1) return launch_fractional_bf16x3(L, s);
    return run_f32_auto(L, s);
}

hipError_t launch_fractional_ops(const AxisOp* ops, const AxisLayout* lays, const float* const* C, float* const* Phi,
                                 int nops, hipStream_t s)
{
    if (nops < 1 || nops > kMaxOps) return hipErrorInvalidValue;
    FracLaunch L;
    memset(&L, 0, sizeof(L));
    L.naxes = nops;
    for (int a = 0; a < nops; ++a) {
        L.op[a] = ops[a];
        L.lay[a] = lays[a];
        L.C[a] = C[a];
        L.Phi[a] = Phi[a];
    }
    return run_f32_auto(L, s);
}

namespace {

hipError_t run_f32_auto(FracLaunch& L, hipStream_t s)
{
    // Tile configuration: LBM_FP32_TILE (read once) selects one explicitly, for
    // tuning; by default the work is counted in 128 x 128 output tiles and
    // grids below ~2 such tiles per CU use the small split-K tiles.
    switch (tile_choice("LBM_FP32_TILE")) {
    case 1: return run_f32<64, 64, 64, 1, 1, 4>(L, s);
    case 2: return run_f32<64, 64, 128, 1, 1, 4>(L, s);
    case 3: return run_f32<128, 64, 64, 2, 1, 2>(L, s);
    case 4: return run_f32<64, 128, 64, 1, 2, 2>(L, s);
    case 5: return run_f32<128, 128, 32, 2, 2, 1>(L, s);
    case 6: return run_f32<128, 128, 64, 2, 2, 1>(L, s);
    case 7: return run_f32_ring<4, 1, 4, 2>(L, s);
    case 8: return run_f32_ring<4, 2, 2, 2>(L, s);
    case 9: return run_f32_ring<4, 4, 1, 2>(L, s);
    case 10: return run_f32_ring<8, 1, 4, 2>(L, s);
    case 11: return run_f32_ring<8, 2, 2, 2>(L, s);
    case 12: return run_f32_ring<8, 4, 1, 2>(L, s);
    case 13: return run_f32_ring<2, 1, 4, 2>(L, s);
    case 14: return run_f32_ring<2, 2, 2, 2>(L, s);
    case 15: return run_f32_ring<4, 1, 4, 1>(L, s);
    case 16: return run_f32_ring<4, 2, 2, 1>(L, s);
    default: break;
    }
    // Register-direct kernel: a large output tile that still fills the chip.
    // Tiles of 256 outputs when every axis has 129..256 nodes (C is then read
    // once per axis) and that gives >= 512 workgroups; else tiles of 128 with
    // the k loop split 2 ways (>= 512 workgroups, at most 128 groups of 8 k
    // per wavefront) or 4 ways (>= 256 workgroups); else tiles of 64.
    // Measured on MI355X (kernel trace, us): 64^3 21.8 -> 10.6, 96^3 43.7 ->
    // 20.6, 128^3 54.1 -> 26.9, 128^2 11.5 -> 5.9, 256^2 15.4 -> 7.0 against
    // 256-output tiles on grids below 512 workgroups; 384^3 1250 -> 1160
    // with the 2-way split in place of unsplit 128-line tiles.  The 128-output
    // tiles prefetch C one group ahead (P = 1: fewer registers, a 2-group
    // unroll): kernel trace, us, P = 2 -> 1: 4096^2 1130.8 -> 1110.2, 2048^2
    // 280.4 -> 273.9, 1024^2 39.8 -> 39.2 (4-way split); 96^3 17.8 -> 15.2,
    // 128^3 25.8 -> 25.5 (2-way split); the 256- and 64-output tiles keep
    // P = 2 (256^3 249.0 against 250.4 with P = 1; 512^2 9.5 against 10.6).
    int nmax = 0, nmin = 1 << 30;
    for (int a = 0; a < L.naxes; ++a) {
        nmax = L.op[a].n > nmax ? L.op[a].n : nmax;
        nmin = L.op[a].n < nmin ? L.op[a].n : nmin;
    }
    const int kgroups = (nmax + 7) / 8;
    FracLaunch T = L;
    int64_t grid = 0;
    size_t lds = 0;
    if (nmax <= 256 && nmin > 128) {
        f32_ring_grid<8, 4, 1>(T, grid, lds);
        if (grid >= 512) return run_f32_ring<8, 4, 1, 2>(L, s);
    }
    f32_ring_grid<4, 2, 2>(T, grid, lds);
    if (grid >= 512 && (kgroups + 1) / 2 <= 128) return run_f32_ring<4, 2, 2, 1>(L, s);
    f32_ring_grid<4, 1, 4>(T, grid, lds);
    if (grid >= 256) return run_f32_ring<4, 1, 4, 1>(L, s);
    // small grids: output tiles of 64 so that every CU gets a workgroup
    return run_f32_ring<2, 1, 4, 2>(L, s);
}

}  // namespace

int64_t big_tiles(const FracLaunch& L)
{
    int64_t t = 0;
    for (int a = 0; a < L.naxes; ++a) {
        const int64_t m = L.lay[a].contiguous ? L.lay[a].lines : L.op[a].n;
        const int64_t nn = L.lay[a].contiguous ? L.op[a].n : L.lay[a].lines * L.lay[a].batches;
        t += ((m + 127) / 128) * ((nn + 127) / 128);
    }
    return t;
}

int tile_choice(const char* var)
{
    // 0 = automatic; 1..16 = the explicit configurations listed at the call sites
    const char* v = getenv(var);
    if (!v || !*v) return 0;
    const int c = atoi(v);
    return (c >= 1 && c <= 16) ? c : 0;
}

}  // namespace lbm
