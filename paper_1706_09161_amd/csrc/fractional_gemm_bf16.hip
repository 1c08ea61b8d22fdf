// fractional_gemm_bf16.hip -- the fractional term (Sec. 2.4) as a 3-term
// split-BF16 GEMM on the BF16 matrix cores (v_mfma_f32_32x32x16_bf16) with
// FP32 accumulation.
//
// Both operands are split into a high and a low BF16 part, x = x_hi + x_lo
// with x_hi = bf16(x) and x_lo = bf16(x - x_hi) (round to nearest even):
//   K C  ~  K_hi C_hi + K_hi C_lo + K_lo C_hi     (the K_lo C_lo term is dropped).
// The Toeplitz weights are split on the host from their FP64 values; C is
// split once per step by its producer (the collide-stream kernel, or a pack
// kernel) into one packed word per node, which the staging only regroups.  Each dropped or rounded piece
// is of relative size 2^-16 or below, against 2^-24 for FP32 operands, for a
// 16 x (3 MFMA) rate advantage per product term over FP32 MFMA.
//
// Structure follows fractional_gemm.hip (same tiling, split-K, boundary-
// column epilogue and one launch for all axes).  Operand convention for
// 32x32x16 BF16: lane l supplies A(i = l%32, k = 8*(l/32) + e) and
// B(k = 8*(l/32) + e, j = l%32) for e = 0..7 (8 BF16 per lane); the
// accumulator layout is that of the 32x32x2 FP32 instruction.
//
// LDS holds C tiles as [line][k] BF16 rows (hi and lo planes) so a lane reads
// its 8 consecutive k with one 16-byte load, and the Toeplitz generator window
// as 32-bit words (hi | lo << 16): a lane reads the 8 generator values of its
// fragment with 8 aligned 4-byte loads (their start shifts with the lane's
// row, so no wider aligned load exists).
#include <hip/hip_runtime.h>
#include <string.h>

#include "lbm_internal.h"

namespace lbm {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

template <bool CONTIG, int BM, int BN, int BK, int WAVES_M, int WAVES_N, int KSPLIT, int VEC>
__device__ __forceinline__ void bf16x3_tile(const AxisOp& op, const AxisLayout& lay, const float* __restrict__ C,
                                            const uint32_t* __restrict__ Cp, float* __restrict__ Phi, int tiles_m,
                                            int tiles_n, int bid, int total, unsigned char* smem)
{
    static_assert(WAVES_M * WAVES_N * KSPLIT == kWaves, "4 wavefronts per workgroup");
    static_assert(BM == WAVES_M * 64 && BN == WAVES_N * 64, "64 x 64 per wavefront");
    constexpr int MB = 2, NB = 2;
    constexpr int KW = BK / KSPLIT;  // k values per wavefront and chunk
    static_assert(KW % 16 == 0, "whole MFMA k steps per wavefront");
    constexpr int CROWS = CONTIG ? BM : BN;  // lines in a C tile
    constexpr int RS = BK + 8;               // row stride in BF16 elements (16-byte pad)
    constexpr int CT = CROWS * RS;           // elements of one plane
    uint16_t* ctile = reinterpret_cast<uint16_t*>(smem);  // [2 buffers][hi, lo][CT]
    uint32_t* gw = reinterpret_cast<uint32_t*>(smem + sizeof(uint16_t) * 4 * CT);

    const int n = op.n, N = n - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wk = wave % KSPLIT;
    const int wmn = wave / KSPLIT;
    const int wm = wmn / WAVES_N, wn = wmn % WAVES_N;

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

    int kb = 0, ke = n;
    if (op.lower_only) ke = min(n, R0 + RB);
    if (op.upper_only) kb = (R0 / BK) * BK;
    const int nk = (ke - kb + BK - 1) / BK;
    const int kend = kb + nk * BK;

    const int dmin = R0 - (kend - 1);
    const int glen = RB + (kend - kb) - 1;
    for (int t = threadIdx.x; t < glen; t += kThreads) {
        const int d = dmin + t;
        gw[t] = (d >= -N && d <= N) ? ((uint32_t)op.gen_hi[d + N] | ((uint32_t)op.gen_lo[d + N] << 16)) : 0u;
    }

    const int64_t lines = lay.lines;
    const float* Cb = C;
    const uint32_t* Cpb = Cp;
    float* Pb = Phi;
    if (!CONTIG) {
        Cb += (int64_t)batch * lay.batch_stride;
        Cpb += (int64_t)batch * lay.batch_stride;
        Pb += (int64_t)batch * lay.batch_stride;
    }
    const int64_t js = lay.j_stride;

    // ---- staging: groups of 8 consecutive k of one line, read as packed
    // (hi | lo << 16) words and regrouped into a hi and a lo BF16 row
    constexpr int GROUPS = CROWS * (BK / 8);
    constexpr int GPT = GROUPS / kThreads;
    static_assert(GROUPS % kThreads == 0, "tile not divisible");
    uint32_t stage[GPT][8];

    auto load_tile = [&](int k0) {
#pragma unroll
        for (int q = 0; q < GPT; ++q) {
            const int id = q * kThreads + threadIdx.x;
            if constexpr (CONTIG) {
                const int g = id % (BK / 8), row = id / (BK / 8);
                const int64_t line = (int64_t)m0 + row;
                const int k = k0 + 8 * g;
                if constexpr (VEC == 4) {
                    if (line < lines && k + 7 < n) {
                        const u32x4 v0 = *reinterpret_cast<const u32x4*>(Cpb + line * n + k);
                        const u32x4 v1 = *reinterpret_cast<const u32x4*>(Cpb + line * n + k + 4);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            stage[q][e] = v0[e];
                            stage[q][4 + e] = v1[e];
                        }
                        continue;
                    }
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) stage[q][e] = (line < lines && k + e < n) ? Cpb[line * n + k + e] : 0u;
            } else {
                const int row = id % BN, g = id / BN;
                const int64_t line = (int64_t)n0 + row;
                const int k = k0 + 8 * g;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    stage[q][e] = (line < lines && k + e < n) ? Cpb[(int64_t)(k + e) * js + line] : 0u;
            }
        }
    };
    auto store_tile = [&](int buf) {
        uint16_t* hi = ctile + (2 * buf) * CT;
        uint16_t* lo = ctile + (2 * buf + 1) * CT;
#pragma unroll
        for (int q = 0; q < GPT; ++q) {
            const int id = q * kThreads + threadIdx.x;
            int g, row;
            if constexpr (CONTIG) {
                g = id % (BK / 8);
                row = id / (BK / 8);
            } else {
                row = id % BN;
                g = id / BN;
            }
            u32x4 hv, lv;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const uint32_t w0 = stage[q][2 * p], w1 = stage[q][2 * p + 1];
                hv[p] = (w0 & 0xffffu) | (w1 << 16);
                lv[p] = (w0 >> 16) | (w1 & 0xffff0000u);
            }
            *reinterpret_cast<u32x4*>(hi + row * RS + 8 * g) = hv;
            *reinterpret_cast<u32x4*>(lo + row * RS + 8 * g) = lv;
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
    // first row of the wavefront in the Toeplitz index (global) or in the C tile (local)
    const int toepBase = (CONTIG ? n0 + wn * 64 : m0 + wm * 64);
    const int ctBase = (CONTIG ? wm * 64 : wn * 64);
    load_tile(kb);
    store_tile(0);
    __syncthreads();

    for (int t = 0; t < nk; ++t) {
        const int k0 = kb + t * BK;
        const int buf = t & 1;
        const uint16_t* chi = ctile + (2 * buf) * CT;
        const uint16_t* clo = ctile + (2 * buf + 1) * CT;
        if (t + 1 < nk) load_tile(k0 + BK);
        struct Frags {
            bf16x8 c_hi[2], c_lo[2], t_hi[2], t_lo[2];
        };
        auto frags = [&](int ks, Frags& F) {
            // C-tile fragments (A in the contiguous case, B otherwise)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int row = ctBase + b * 32 + li;
                F.c_hi[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(chi + row * RS + ks + 8 * lk));
                F.c_lo[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(clo + row * RS + ks + 8 * lk));
            }
            // Toeplitz fragments: T(r - k) for k = k0 + ks + 8*lk + e, e = 0..7
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int r = toepBase + b * 32 + li;
                const int t0 = r - (k0 + ks + 8 * lk) - dmin;  // word of e = 0; e moves down
                uint32_t w[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) w[e] = gw[t0 - e];
                u32x4 hv, lv;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    hv[p] = (w[2 * p] & 0xffffu) | (w[2 * p + 1] << 16);
                    lv[p] = (w[2 * p] >> 16) | (w[2 * p + 1] & 0xffff0000u);
                }
                F.t_hi[b] = __builtin_bit_cast(bf16x8, hv);
                F.t_lo[b] = __builtin_bit_cast(bf16x8, lv);
            }
        };
        constexpr int NSTEP = KW / 16;
        Frags F[2];
        frags(wk * KW, F[0]);
#pragma unroll
        for (int st = 0; st < NSTEP; ++st) {
            if (st + 1 < NSTEP) frags(wk * KW + 16 * (st + 1), F[(st + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);  // reads of the next step stay ahead of these MFMAs
            const Frags& G = F[st & 1];
            // CONTIG: A = C tile (block i), B = Toeplitz (block j); else A = Toeplitz (i), B = C (j).
            // Small terms first; consecutive MFMAs go to different accumulators.
#pragma unroll
            for (int term = 0; term < 3; ++term)
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        const bf16x8 ah = CONTIG ? G.c_hi[i] : G.t_hi[i];
                        const bf16x8 al = CONTIG ? G.c_lo[i] : G.t_lo[i];
                        const bf16x8 bh = CONTIG ? G.t_hi[j] : G.c_hi[j];
                        const bf16x8 bl = CONTIG ? G.t_lo[j] : G.c_lo[j];
                        const bf16x8 a = term == 0 ? al : ah;
                        const bf16x8 b = term == 1 ? bl : bh;
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[i][j], 0, 0, 0);
                    }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (t + 1 < nk) store_tile(buf ^ 1);
        __syncthreads();
    }

    int blk_lo = 0, blk_hi = MB * NB;
    if constexpr (KSPLIT > 1) {
        float* red = reinterpret_cast<float*>(smem);
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) red[((wave * MB * NB + i * NB + j) * 16 + r) * 64 + lane] = acc[i][j][r];
        __syncthreads();
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
}

template <int BM, int BN, int BK, int WAVES_M, int WAVES_N, int KSPLIT, int VEC_X>
__global__ __launch_bounds__(kThreads) void fractional_bf16x3_mfma(FracLaunch L)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_b[];
    const int bid = blockIdx.x;
    int axis = 0;
    while (axis + 1 < L.naxes && bid >= L.first[axis + 1]) ++axis;
    const int local = bid - L.first[axis];
    const int total = L.first[axis + 1] - L.first[axis];
    if (axis == 0)
        bf16x3_tile<true, BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, VEC_X>(L.op[0], L.lay[0], L.C[0], L.Cp[0], L.Phi[0],
                                                                       L.tiles_m[0],
                                                                       L.tiles_n[0], local, total, smem_b);
    else
        bf16x3_tile<false, BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, 1>(L.op[axis], L.lay[axis], L.C[axis], L.Cp[axis],
                                                                    L.Phi[axis],
                                                                    L.tiles_m[axis], L.tiles_n[axis], local, total,
                                                                    smem_b);
}

template <int BM, int BN, int BK, int WAVES_M, int WAVES_N, int KSPLIT>
hipError_t run_bf16(FracLaunch& L, hipStream_t s)
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
        const int crows = contig ? BM : BN;
        const int rb = contig ? BN : BM;
        const int kspan = ((op.n + BK - 1) / BK) * BK;
        size_t need = sizeof(uint16_t) * 4 * crows * (BK + 8) + sizeof(uint32_t) * (rb + kspan);
        if (KSPLIT > 1) need = need > sizeof(float) * 4 * 4 * 16 * 64 ? need : sizeof(float) * 4 * 4 * 16 * 64;
        lds = need > lds ? need : lds;
    }
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    L.first[L.naxes] = (int)grid;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const bool vx = (L.op[0].n % 4) == 0;
    auto go = [&](auto kern) -> hipError_t {
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), lds, s, L);
        return hipGetLastError();
    };
    if (vx) return go(fractional_bf16x3_mfma<BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, 4>);
    return go(fractional_bf16x3_mfma<BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, 1>);
}

}  // namespace

bool have_bf16x3() { return true; }

hipError_t launch_fractional_bf16x3(FracLaunch& L, hipStream_t s)
{
    // LBM_BF16_TILE selects a configuration explicitly (tuning); see launch_fractional.
    switch (tile_choice("LBM_BF16_TILE")) {
    case 1: return run_bf16<64, 64, 64, 1, 1, 4>(L, s);
    case 2: return run_bf16<64, 64, 128, 1, 1, 4>(L, s);
    case 3: return run_bf16<128, 64, 64, 2, 1, 2>(L, s);
    case 4: return run_bf16<64, 128, 64, 1, 2, 2>(L, s);
    case 5: return run_bf16<128, 128, 32, 2, 2, 1>(L, s);
    case 6: return run_bf16<128, 128, 64, 2, 2, 1>(L, s);
    default: break;
    }
    if (big_tiles(L) < 512) return run_bf16<64, 64, 128, 1, 1, 4>(L, s);
    return run_bf16<128, 128, 32, 2, 2, 1>(L, s);
}

}  // namespace lbm
