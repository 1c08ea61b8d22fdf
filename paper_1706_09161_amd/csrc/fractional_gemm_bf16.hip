// fractional_gemm_bf16.hip -- the fractional term (Sec. 2.4) as a 3-term
// split-BF16 GEMM on the BF16 matrix cores (v_mfma_f32_32x32x16_bf16) with
// FP32 accumulation.
//
// Both operands are split into a high and a low BF16 part, x = x_hi + x_lo
// with x_hi = bf16(x) and x_lo = bf16(x - x_hi) (round to nearest even):
//   K C  ~  K_hi C_hi + K_hi C_lo + K_lo C_hi     (the K_lo C_lo term is dropped).
// The Toeplitz weights are split on the host from their FP64 values; the
// kernels read C in FP32 and split it as they load it (v_cvt_pk_bf16_f32, two
// values per instruction), so no split copy of C is stored.  Each dropped or
// rounded piece is of relative size 2^-16 or below, against 2^-24 for FP32
// operands, for a 16 x (3 MFMA) rate advantage per product term over FP32
// MFMA.
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
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

// BF16 split of two FP32 values of C: hi = bf16(c), lo = bf16(c - hi), both
// rounded to nearest even by v_cvt_pk_bf16_f32 (c - hi is exact in FP32);
// returned as the packed pairs hi0 | hi1 << 16 and lo0 | lo1 << 16.
__device__ __forceinline__ void split_pair(float a, float b, uint32_t& hp, uint32_t& lp)
{
    hp = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
    const float ra = a - __uint_as_float(hp << 16), rb = b - __uint_as_float(hp & 0xffff0000u);
    lp = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{ra, rb}, bf16x2));
}

template <bool CONTIG, int BM, int BN, int BK, int WAVES_M, int WAVES_N, int KSPLIT, int VEC>
__device__ __forceinline__ void bf16x3_tile(const AxisOp& op, const AxisLayout& lay, const float* __restrict__ C,
                                            float* __restrict__ Phi, int tiles_m, int tiles_n, int bid, int total,
                                            unsigned char* smem)
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
    float* Pb = Phi;
    if (!CONTIG) {
        Cb += (int64_t)batch * lay.batch_stride;
        Pb += (int64_t)batch * lay.batch_stride;
    }
    const uint32_t* Cbits = reinterpret_cast<const uint32_t*>(Cb);  // the FP32 values' bits
    const int64_t js = lay.j_stride;

    // ---- staging: groups of 8 consecutive k of one line, read as FP32 and
    // split into a hi and a lo BF16 row
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
                        const u32x4 v0 = *reinterpret_cast<const u32x4*>(Cbits + line * n + k);
                        const u32x4 v1 = *reinterpret_cast<const u32x4*>(Cbits + line * n + k + 4);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            stage[q][e] = v0[e];
                            stage[q][4 + e] = v1[e];
                        }
                        continue;
                    }
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) stage[q][e] = (line < lines && k + e < n) ? Cbits[line * n + k + e] : 0u;
            } else {
                const int row = id % BN, g = id / BN;
                const int64_t line = (int64_t)n0 + row;
                const int k = k0 + 8 * g;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    stage[q][e] = (line < lines && k + e < n) ? Cbits[(int64_t)(k + e) * js + line] : 0u;
            }
        }
    };
    // forward operators leave columns k = 0 and k = N out of the Toeplitz sum
    // (the epilogue adds the whole boundary columns): zero them in the staged
    // chunk that holds them
    auto mask_ends = [&](int k0) {
        if (!op.ends_excluded || (k0 > 0 && k0 + BK <= N)) return;
#pragma unroll
        for (int q = 0; q < GPT; ++q) {
            const int id = q * kThreads + threadIdx.x;
            const int g = CONTIG ? id % (BK / 8) : id / BN;
            const int k = k0 + 8 * g;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (k + e == 0 || k + e == N) stage[q][e] = 0u;
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
                uint32_t hp, lp;
                split_pair(__uint_as_float(stage[q][2 * p]), __uint_as_float(stage[q][2 * p + 1]), hp, lp);
                hv[p] = hp;
                lv[p] = lp;
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
    mask_ends(kb);  // the first chunk is consumed right away
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
        if (t + 1 < nk) {
            mask_ends(k0 + BK);  // where the prefetched chunk is consumed
            store_tile(buf ^ 1);
        }
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
        bf16x3_tile<true, BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, VEC_X>(L.op[0], L.lay[0], L.C[0], L.Phi[0],
                                                                       L.tiles_m[0],
                                                                       L.tiles_n[0], local, total, smem_b);
    else
        bf16x3_tile<false, BM, BN, BK, WAVES_M, WAVES_N, KSPLIT, 1>(L.op[axis], L.lay[axis], L.C[axis],
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


// ---------------------------------------------------------------------------
// Register-ring kernel.  One wavefront computes 32 lines x (32 NBJ) outputs
// of one axis over its share of k, in steps of 16 k:
//  * the C fragment of a step (32 lines x 16 k) is loaded straight from the
//    FP32 field into registers, P steps ahead (no LDS, no barrier in the
//    k loop), and split into its hi and lo BF16 planes there: along the
//    contiguous axis a lane reads 8 consecutive values (two 16-byte loads),
//    along a strided axis 8 values of one line at successive k, each load
//    coalesced across the lanes (consecutive lines);
//  * the Toeplitz fragment of output block c at step t equals that of block
//    0 at step t - 2c (T(j + 32c - k) = T(j - (k - 32c))), so only the
//    block-0 fragment of each new step is read; the last 2 NBJ of them stay
//    in a register ring indexed by the step modulo 2 NBJ (the k loop is
//    unrolled by that period so every ring index is static);
//  * Toeplitz fragments are read from an LDS window of pair words
//    W(d) = T(d) | T(d - 1) << 16 (hi and lo planes) stored with d
//    decreasing: the 8 values of a lane, T(d0), T(d0 - 1), ..., T(d0 - 7),
//    are the four words W(d0), W(d0 - 2), W(d0 - 4), W(d0 - 6) at increasing
//    addresses (two ds_read2), already in MFMA operand order.
// A workgroup has 4 wavefronts: WL line blocks x KSPLIT k-shares; k-shares
// are summed through LDS in a fixed order (deterministic).
template <bool CONTIG, int NBJ, int WL, int KSPLIT, int P, bool VEC, bool KFULL>
__device__ __forceinline__ void bf16x3_ring_tile(const AxisOp& op, const AxisLayout& lay, const float* __restrict__ C,
                                                 float* __restrict__ Phi,
                                                 int tiles_l, int tiles_j, int bid, int total, unsigned char* smem)
{
    static_assert(WL * KSPLIT == kWaves, "4 wavefronts per workgroup");
    static_assert(NBJ % KSPLIT == 0, "output blocks divide among the k shares");
    constexpr int R = 2 * NBJ;  // Toeplitz ring period (steps)
    static_assert(R % P == 0, "prefetch depth divides the ring period");
    constexpr int JT = 32 * NBJ;  // outputs per tile
    static_assert(JT <= kThreads && JT <= 512, "one thread per output of the tile; pair-word arrays sized for 512");
    constexpr int LT = 32 * WL;  // lines per tile
    const int n = op.n, N = n - 1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: keeps the k loop scalar
    const int wl = wave / KSPLIT, wk = wave % KSPLIT;
    const int li = lane & 31, lh = lane >> 5;

    // Tile of this workgroup.  Workgroups are dealt to the 8 XCDs round robin;
    // each XCD gets a contiguous range of tiles (the output tiles of a few line
    // blocks, which share C in its L2).  One-sided operators make the k range
    // grow (p = 1) or shrink (p = 0) with the output tile: there each XCD
    // starts its longest tiles first.
    int lin = bid;
    if ((total & 7) == 0) {
        const int S = total >> 3, x = bid & 7, i = bid >> 3;
        lin = x * S + i;
        if ((op.lower_only || op.upper_only) && S % tiles_j == 0) {
            const int lpx = S / tiles_j;  // line blocks per XCD
            lin = x * S + (i % lpx) * tiles_j + i / lpx;
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

    // k range of the tile (one-sided operators skip the zero triangle)
    int kb = 0, ke = n;
    if (op.lower_only) ke = min(n, j0 + JT);
    if (op.upper_only) kb = (min(j0, n - 1) / 16) * 16;
    const int steps = (ke - kb + 15) / 16;  // >= 1
    const int kend = kb + 16 * steps;
    const int spw = (steps + KSPLIT - 1) / KSPLIT;
    const int t_first = wk * spw;
    const int my_steps = max(0, min(steps, t_first + spw) - t_first);
    const int kw = kb + 16 * min(t_first, steps - 1);  // first k of this wavefront (clamped when it has none)
    const int last = max(my_steps, 1) - 1;             // last step whose C is read

    // ---- C fragments: lane = (line li, k group lh).  Steps past the end of
    // the range re-read the last step, so every step issues the same loads.
    const int64_t my_line = min(line0 + li, lines - 1);  // rows past the end are computed, never stored
    // the FP32 field's bits, split into BF16 planes in registers
    const uint32_t* Cw = reinterpret_cast<const uint32_t*>(Cb);
    const uint32_t* q = CONTIG ? Cw + my_line * n + kw + 8 * lh : Cw + (int64_t)(kw + 8 * lh) * js + my_line;
    const bool ends = op.ends_excluded != 0;
    auto load_raw = [&](int t, uint32_t (&w)[8]) {
        const int tc = min(t, last);
        if constexpr (KFULL) {
            // every k of every step is < n: no guards, no branches
            if constexpr (CONTIG) {
                const u32x4 v0 = *reinterpret_cast<const u32x4*>(q + 16 * tc);
                const u32x4 v1 = *reinterpret_cast<const u32x4*>(q + 16 * tc + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    w[e] = v0[e];
                    w[4 + e] = v1[e];
                }
            } else {
                const uint32_t* a = q + (int64_t)(16 * tc) * js;
#pragma unroll
                for (int e = 0; e < 8; ++e) w[e] = a[(int64_t)e * js];
            }
        } else {
            // the last step may pass the end of the axis: values there are 0
            const int k = kw + 16 * tc + 8 * lh;  // first k of this lane
            if constexpr (CONTIG && VEC) {
                const bool ok = k < n;  // n % 8 == 0: all 8 values in range, or none
                const uint32_t* a = ok ? q + 16 * tc : Cw;
                const u32x4 v0 = *reinterpret_cast<const u32x4*>(a);
                const u32x4 v1 = *reinterpret_cast<const u32x4*>(a + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    w[e] = ok ? v0[e] : 0u;
                    w[4 + e] = ok ? v1[e] : 0u;
                }
            } else {
                const int64_t stride = CONTIG ? 1 : js;
                const uint32_t* a = q + (int64_t)(16 * tc) * stride;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const bool ok = k + e < n;
                    const uint32_t v = *(ok ? a + e * stride : Cw);
                    w[e] = ok ? v : 0u;
                }
            }
        }
    };
    // Forward operators leave columns k = 0 and k = N out of the Toeplitz sum
    // (the epilogue adds the whole boundary columns).  k ranges start at
    // multiples of 16, so k = 0 is element 0 of lane half 0 in step 0 of the
    // wavefront that starts at 0, and k = N is element N % 8 of lane half
    // (N % 16) / 8 in the one step holding it; with n % 8 == 0 that element
    // is always the last.  Their C values are zeroed with selects before the
    // step is split (no branch: the interleaved MFMA / load block of the loop
    // body stays one block).
    const bool lane_k0 = ends && kw == 0 && lh == 0;
    const bool lane_kN = ends && lh == (N % 16) / 8;
    const int t_kN = (ends && N >= kw && N < kw + 16 * my_steps) ? (N - kw) / 16 : -1;
    auto kill_kN = [&](int t, uint32_t (&w)[8]) {
        const bool kn = lane_kN && t == t_kN;
        if constexpr (KFULL || VEC) {
            w[7] = kn ? 0u : w[7];
        } else {
            const int e_kN = N % 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) w[e] = (kn && e == e_kN) ? 0u : w[e];
        }
    };
    // BF16 hi and lo planes of a C fragment; zero for steps past the end of
    // this wavefront's range (their products then add nothing, so every step
    // runs the same straight-line code)
    auto cvt = [&](const uint32_t (&w)[8], bool live, bf16x8& hi, bf16x8& lo) {
        u32x4 h, l;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            uint32_t hp, lp;
            split_pair(__uint_as_float(w[2 * p]), __uint_as_float(w[2 * p + 1]), hp, lp);
            h[p] = live ? hp : 0u;
            l[p] = live ? lp : 0u;
        }
        hi = __builtin_bit_cast(bf16x8, h);
        lo = __builtin_bit_cast(bf16x8, l);
    };
    // ---- LDS: col0 | colN | C at the two walls of each line (contiguous
    // axis) | pair-word window hi | lo (later the k-share reduction)
    float* c0s = reinterpret_cast<float*>(smem);
    float* cNs = c0s + JT;
    float* w0s = cNs + JT;
    float* wNs = w0s + LT;
    uint32_t* pwh = reinterpret_cast<uint32_t*>(wNs + LT);
    const int wlen = JT - 1 + (kend - kb);  // d in [dmax - wlen + 1, dmax], word m holds d = dmax - m
    const int wpad = (wlen + 3) & ~3;
    const int dmax = j0 + JT - 1 - kb;      // = 15 (mod 16), so the copy below starts 64-byte aligned
    uint32_t* pwl = pwh + wpad;
    const int nq = wpad / 4;                // 16-byte words per plane
    const int x0 = op.pw_top - dmax;
    constexpr int FU = 8;                   // 16-byte words per thread and round of the copy
    auto fill_load = [&](int base, u32x4 (&v)[FU]) {
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int idx = base + u * kThreads + threadIdx.x;
            if (idx < 2 * nq) {
                const bool lo = idx >= nq;
                const int qq = lo ? idx - nq : idx;
                v[u] = *reinterpret_cast<const u32x4*>((lo ? op.pw_lo : op.pw_hi) + x0 + 4 * qq);
            }
        }
    };
    auto fill_store = [&](int base, const u32x4 (&v)[FU]) {
#pragma unroll
        for (int u = 0; u < FU; ++u) {
            const int idx = base + u * kThreads + threadIdx.x;
            if (idx < 2 * nq) {
                const bool lo = idx >= nq;
                const int qq = lo ? idx - nq : idx;
                *reinterpret_cast<u32x4*>((lo ? pwl : pwh) + 4 * qq) = v[u];
            }
        }
    };
    // Loads complete in issue order, so the set-up loads go first, then the
    // first P steps of C (their latency overlaps the set-up), then the stores.
    u32x4 fv[FU];
    fill_load(0, fv);
    float cv0 = 0.f, cvN = 0.f, wv0 = 0.f, wvN = 0.f;
    {
        const int t = threadIdx.x;  // JT <= kThreads
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
    // strided axes: the wall values of this lane's line
    float b0 = 0.f, bN = 0.f;
    if constexpr (!CONTIG) {
        b0 = Cb[my_line];
        bN = Cb[(int64_t)N * js + my_line];
    }
    uint32_t raw[P][8];
#pragma unroll
    for (int t = 0; t < P; ++t) load_raw(t, raw[t]);
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
    for (int base = FU * kThreads; base < 2 * nq; base += FU * kThreads) {  // long axes only
        fill_load(base, fv);
        fill_store(base, fv);
    }
    lds_barrier();  // the C prefetch stays in flight

    f32x16 acc[NBJ];
#pragma unroll
    for (int c = 0; c < NBJ; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0.f;

    if (my_steps > 0) {
        // block-0 Toeplitz fragment of step t: lane = (output j0 + li, k group lh)
        const int mbase = dmax - (j0 + li - 8 * lh - kw);  // window word of d0 at t = 0
        auto load_t = [&](int t, bf16x8& hi, bf16x8& lo) {
            const int m0 = min(mbase + 16 * t, wlen - 7);  // steps past the end read a clamped (unused) fragment
            u32x4 h, l;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                h[p] = pwh[m0 + 2 * p];
                l[p] = pwl[m0 + 2 * p];
            }
            hi = __builtin_bit_cast(bf16x8, h);
            lo = __builtin_bit_cast(bf16x8, l);
        };

        bf16x8 th[R], tl[R];
        bf16x8 ch[2], cl[2];
        // ring slots of steps -R+2 .. 0 (blocks c >= 1 of the first steps)
#pragma unroll
        for (int t = -(R - 2); t <= 0; ++t) load_t(t, th[(t + R) % R], tl[(t + R) % R]);
        raw[0][0] = lane_k0 ? 0u : raw[0][0];  // k = 0 is only ever in step 0
        kill_kN(0, raw[0]);
        cvt(raw[0], true, ch[0], cl[0]);

        for (int t0 = 0; t0 < my_steps; t0 += R) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int t = t0 + u;
                // prefetch the Toeplitz fragment of step t + 1 and the C of step
                // t + P (into the slot of step t, converted already), then split
                // the C of step t + 1 (its column N zeroed first)
                load_t(t + 1, th[(u + 1) % R], tl[(u + 1) % R]);
                load_raw(t + P, raw[u % P]);
                kill_kN(t + 1, raw[(u + 1) % P]);
                cvt(raw[(u + 1) % P], t + 1 < my_steps, ch[(u + 1) & 1], cl[(u + 1) & 1]);
                const bf16x8 chh = ch[u & 1], cll = cl[u & 1];
#pragma unroll
                for (int term = 0; term < 3; ++term)
#pragma unroll
                    for (int c = 0; c < NBJ; ++c) {
                        const int slot = ((u - 2 * c) % R + R) % R;
                        const bf16x8 tt = term == 1 ? tl[slot] : th[slot];
                        const bf16x8 cc = term == 0 ? cll : chh;
                        if constexpr (CONTIG)
                            acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cc, tt, acc[c], 0, 0, 0);
                        else
                            acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(tt, cc, acc[c], 0, 0, 0);
                    }
                // interleave the prefetch and conversion of the next steps with
                // this step's MFMAs (one MFMA, then a few other instructions)
#pragma unroll
                for (int i = 0; i < 3 * NBJ; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
                    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);  // VMEM read
                    __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // VALU
                    __builtin_amdgcn_sched_group_barrier(0x004, 2, 0);  // SALU
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    int c_lo = 0, c_hi = NBJ;
    if constexpr (KSPLIT > 1) {
        __syncthreads();  // every wavefront is done with the pair-word window
        float* red = reinterpret_cast<float*>(pwh);
        c_lo = wk * (NBJ / KSPLIT);
        c_hi = c_lo + NBJ / KSPLIT;
        // blocks other k shares sum go through LDS; a wavefront's own blocks
        // stay in registers (same fixed summation order, s = 0, 1, ...)
#pragma unroll
        for (int c = 0; c < NBJ; ++c) {
            if (c >= c_lo && c < c_hi) continue;
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
                float4 v = make_float4(acc[c][4 * r4], acc[c][4 * r4 + 1], acc[c][4 * r4 + 2], acc[c][4 * r4 + 3]);
                *reinterpret_cast<float4*>(red + (((wave * NBJ + c) * 4 + r4) * 64 + lane) * 4) = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NBJ; ++c) {
            if (c < c_lo || c >= c_hi) continue;
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
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
    }

    // epilogue: boundary columns (rank-2 correction) and stores
    if constexpr (CONTIG) {
        // rows = lines (8 (r / 4) + 4 lh + r % 4), columns = outputs j0 + 32 c + li
        float cb0[16], cbN[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int tl = 32 * wl + 8 * (r >> 2) + 4 * lh + (r & 3);
            cb0[r] = w0s[tl];
            cbN[r] = wNs[tl];
        }
#pragma unroll
        for (int c = 0; c < NBJ; ++c) {
            if (c < c_lo || c >= c_hi) continue;
            const int jl = 32 * c + li, j = j0 + jl;
            const float k0 = c0s[jl], kN = cNs[jl];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t line = line0 + 8 * (r >> 2) + 4 * lh + (r & 3);
                if (line < lines && j < n) {
                    float v = acc[c][r];
                    v = fmaf(k0, cb0[r], v);
                    v = fmaf(kN, cbN[r], v);
                    Pb[line * n + j] = v;
                }
            }
        }
    } else {
        // rows = outputs j0 + 32 c + 8 (r / 4) + 4 lh + r % 4, columns = lines line0 + li
        const int64_t line = line0 + li;
#pragma unroll
        for (int c = 0; c < NBJ; ++c) {
            if (c < c_lo || c >= c_hi) continue;
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
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
}

template <int NBJ, int WL, int KSPLIT, int P, bool VEC_X, bool KFULL>
__global__ __launch_bounds__(kThreads, NBJ <= 4 ? 2 : 1) void fractional_bf16x3_ring(FracLaunch L)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_r[];
    const int bid = blockIdx.x;
    int axis = 0;
    while (axis + 1 < L.naxes && bid >= L.first[axis + 1]) ++axis;
    const int local = bid - L.first[axis];
    const int total = L.first[axis + 1] - L.first[axis];
    if (axis == 0)
        bf16x3_ring_tile<true, NBJ, WL, KSPLIT, P, VEC_X, KFULL>(L.op[0], L.lay[0], L.C[0], L.Phi[0], L.tiles_m[0],
                                                          L.tiles_n[0], local, total, smem_r);
    else
        bf16x3_ring_tile<false, NBJ, WL, KSPLIT, P, false, KFULL>(L.op[axis], L.lay[axis], L.C[axis],
                                                           L.Phi[axis], L.tiles_m[axis], L.tiles_n[axis], local, total,
                                                           smem_r);
}

// tiles_m = line tiles (32 WL lines), tiles_n = output tiles (32 NBJ outputs)
template <int NBJ, int WL, int KSPLIT>
void ring_grid(FracLaunch& L, int64_t& grid, size_t& lds)
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
        const size_t kspan = (size_t)((op.n + 15) / 16) * 16;
        size_t window = sizeof(uint32_t) * 2 * (32 * NBJ + kspan);  // two planes of wpad words
        const size_t red = KSPLIT > 1 ? sizeof(float) * kWaves * NBJ * 16 * 64 : 0;
        window = window > red ? window : red;
        const size_t need = sizeof(float) * (2 * 32 * NBJ + 2 * 32 * WL) + window;
        lds = need > lds ? need : lds;
    }
}

template <int NBJ, int WL, int KSPLIT, int P>
hipError_t run_ring(FracLaunch& L, hipStream_t s)
{
    int64_t grid = 0;
    size_t lds = 0;
    ring_grid<NBJ, WL, KSPLIT>(L, grid, lds);
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    L.first[L.naxes] = (int)grid;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    auto go = [&](auto kern) -> hipError_t {
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), lds, s, L);
        return hipGetLastError();
    };
    bool kfull = true;  // every axis a multiple of 16: no step passes the end of an axis
    for (int a = 0; a < L.naxes; ++a) kfull = kfull && (L.op[a].n % 16) == 0;
    if (kfull) return go(fractional_bf16x3_ring<NBJ, WL, KSPLIT, P, true, true>);
    if (L.op[0].n % 8 == 0) return go(fractional_bf16x3_ring<NBJ, WL, KSPLIT, P, true, false>);
    return go(fractional_bf16x3_ring<NBJ, WL, KSPLIT, P, false, false>);
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
    case 7: return run_ring<8, 1, 4, 4>(L, s);
    case 8: return run_ring<8, 2, 2, 4>(L, s);
    case 9: return run_ring<8, 4, 1, 4>(L, s);
    case 10: return run_ring<8, 1, 4, 8>(L, s);
    case 11: return run_ring<8, 2, 2, 8>(L, s);
    case 12: return run_ring<8, 4, 1, 8>(L, s);
    case 13: return run_ring<4, 1, 4, 4>(L, s);
    case 14: return run_ring<4, 2, 2, 4>(L, s);
    default: break;
    }
    // Register-ring kernel: wavefront tiles of 32 x 256 outputs, 4 line blocks
    // per workgroup, when that gives >= 512 workgroups (in 3D only when 256
    // divides every axis: no part-empty tiles); otherwise in 3D tiles of
    // 32 x 128 with 2 line blocks and k split 2 ways, in 2D tiles of 32 x 128
    // with k split 4 ways.  Measured on MI355X (kernel trace, us, against the
    // other choice): 64^3 8.9 (11.1), 96^3 14.5 (19.9), 128^3 21.2 (30.6),
    // 320^3 406 (491), 384^3 579 (664); 256^3 128 (142); 2D 512^2 9.0 (11.3),
    // 1536^2 51.0 (53.3).  At 1024^2 (timed per launch) 15.7-16.8 us against
    // 16.7-36.3 for the other ring tiles of the table.
    {
        bool batched = false, whole = true;
        for (int a = 0; a < L.naxes; ++a) {
            batched = batched || (!L.lay[a].contiguous && L.lay[a].batches > 1);
            whole = whole && L.op[a].n % 256 == 0;
        }
        FracLaunch T = L;
        int64_t grid = 0;
        size_t lds = 0;
        ring_grid<8, 4, 1>(T, grid, lds);
        if (grid >= 512 && (!batched || whole)) return run_ring<8, 4, 1, 4>(L, s);
        if (batched) return run_ring<4, 2, 2, 4>(L, s);
        return run_ring<4, 1, 4, 4>(L, s);
    }
}

}  // namespace lbm
