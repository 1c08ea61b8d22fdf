// collide_stream.hip -- equilibrium, collision, streaming, Dirichlet rule and
// moment of one LB time step, fused into one pass over the populations
// (Algorithm 1, time-loop stages 2-5; Sec. 2.2, 2.3, 2.5).
//
// State between steps: populations f after streaming and the Dirichlet rule,
// and their moment C = <1|f> (written by this kernel for the next step's
// fractional term).  For every node x the kernel
//   1. recomputes C(x) = sum_i f_i(x),
//   2. builds f^eq(C, Phi, u) (equations (Feq), (CoeffA_FADE3D)),
//   3. collides: f* = f - R (f - f^eq) + w S dt with R = M^-1 Lambda M
//      (equation (MRT-Coll); BGK: R = I / lambda, equation (LBE_FADE)),
//   4. and the new populations are pulled: f_i(x) <- f*_i(x - e_i)
//      (equation (Def_Translation)); a population whose source lies outside
//      the box is unknown and the Dirichlet rule (Dirichlet_BC) sets it:
//      f_b = (C_wall - sum of the known) / |unknown| (equal share at edges and
//      corners);
//   5. and writes the new f and C = sum_i f_i.
//
// 2D (D2Q5): each wavefront owns a strip of 64 columns starting on a
// multiple of 64 (its loads and stores are whole 128-byte lines) and marches
// up the y axis: the collision of row y+1 is computed once, its f*_4 is used
// for row y and its f*_3 for row y+2.  The rows read ahead stop at the first
// row past the chunk (the last block of a march refills only what it needs).
// f*_1 / f*_2 cross columns by lane shuffles; at the strip's two edges lanes
// 0 and 63 also read the node just outside the strip and compute the one
// population that crosses (one row of the collision operator).  Every node is
// collided once (plus 2 halo rows per march), every population is read once
// and written once: (2Q + d + 1) * 4 bytes per node from HBM (52 B for D2Q5).
//
// 3D (D3Q7): a workgroup of NY wavefronts covers 64 x (NY - 2) nodes of one z
// plane (one wave per y row, rows 0 and NY-1 halo, the x edges as in 2D) and
// marches along z; f*_3/f*_4 cross rows through LDS, f*_5/f*_6 cross planes in
// registers.
//
// Both kernels deal their tiles to the XCDs in contiguous ranges (halo lines
// shared in one L2), store their outputs non-temporally once a step's traffic
// exceeds the Infinity Cache, and round every node alike whatever the launch
// shape (explicit fmaf only), so results do not depend on the march length.
//
// Offsets are 32-bit byte offsets from uniform base pointers (one VALU add per
// address) while every array fits in 4 GiB, 64-bit otherwise.
#include <hip/hip_runtime.h>
#include <stdlib.h>

#include <type_traits>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kStrip = 64;  // output columns per wavefront

// Tile index of workgroup b of nb.  Workgroups are dealt to the 8 XCDs round
// robin (b mod 8); this gives each XCD one contiguous range of tiles instead,
// so the halo lines that neighbouring tiles both read (the node columns beside
// a strip, the rows or planes beside a march) are fetched once into that XCD's
// L2 rather than once per XCD.  A bijection of [0, nb): the first nb mod 8
// XCDs take one tile more.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// 1 / (number of unknown populations) of the Dirichlet rule (at most 3)
__device__ __forceinline__ float inv_count(int nu) { return nu == 1 ? 1.f : (nu == 2 ? 0.5f : 1.f / 3.f); }

template <typename OFF>
__device__ __forceinline__ float ldf(const float* base, OFF boff)
{
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + boff);
}
// Output store; NT: non-temporal (the line is not kept in L2 for reuse), for
// grids whose state does not fit the Infinity Cache, so that the L2 keeps the
// input lines that neighbouring tiles read again.
template <bool NT, typename OFF, typename T>
__device__ __forceinline__ void stv(T* base, OFF boff, T v)
{
    T* p = reinterpret_cast<T*>(reinterpret_cast<char*>(base) + boff);
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Index of entry (a, b), a <= b, of a symmetric d x d block stored as its
// upper triangle row by row: (00, 01, 11) in 2D, (00, 01, 02, 11, 12, 22) in 3D.
__host__ __device__ constexpr int sym_index(int d, int a, int b) { return a * d - a * (a - 1) / 2 + (b - a); }

// Space-dependent diffusion tensor (Sec. 2.3: lambda-bar and Lambda may vary
// with x): the node's flux block of Lambda is the constant block plus dB (the
// symmetric difference lambda-bar(x)^-1 - lambda-bar^-1).  The flux moments
// are m_{1+b} = dev_{2b+1} - dev_{2b+2}, and column 1+a of M^-1 holds +1/2 at
// population 2a+1 and -1/2 at 2a+2, so the extra relaxation
// M^-1 (0, dB m_flux, 0) moves -delta_a/2 into f*_{2a+1} and +delta_a/2 into
// f*_{2a+2}, delta_a = sum_b dB_ab m_{1+b}.
template <int Q>
__device__ __forceinline__ float flux_delta(const float (&dev)[Q], const float* db, int a)
{
    constexpr int d = (Q - 1) / 2;
    float s = 0.f;
#pragma unroll
    for (int b = 0; b < d; ++b) {
        const float m = dev[2 * b + 1] - dev[2 * b + 2];
        s = fmaf(db[a <= b ? sym_index(d, a, b) : sym_index(d, b, a)], m, s);
    }
    return s;
}

// The equilibrium carries the node's mass: sum_i f^eq_i = C = sum_i f_i
// (equation (Feq)), so the deviations f - f^eq have zero sum and the collision
// conserves mass.  In FP32 the rounded f^eq_i leave a sum of a few ulp of C,
// which the mass row of the collision operator turns into a mass change of
// the same size at every node and step; it does not decay (mass is
// conserved) and over thousands of steps it is the largest error of the FP32
// scheme.  Taking the rounded sum off the rest population restores the zero
// sum up to an ulp of the deviations (exact arithmetic subtracts 0).
template <int Q>
__device__ __forceinline__ void remove_mass_defect(float (&dev)[Q])
{
#pragma clang fp contract(off)
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) m += dev[i];
    dev[0] -= m;
}

template <int Q, bool VAR>
__device__ inline void collide_node(const CollideConsts& cc, const float (&f)[Q], const float (&phi)[(Q - 1) / 2],
                                    float S, const float* db, float (&fs)[Q])
{
    // Products are fused only where fmaf says so (and fmaf is used wherever a
    // product meets a sum): every inlined copy of this function (the rows
    // before a march, the march, its last block) then rounds alike, and a
    // node's result does not depend on where in a march it falls or on the
    // march length.
#pragma clang fp contract(off)
    constexpr int d = (Q - 1) / 2;
    float C = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) C += f[i];
    float feq[Q];
    float sphi = 0.f;
#pragma unroll
    for (int mu = 0; mu < d; ++mu) sphi += phi[mu];
    feq[0] = fmaf(-cc.w[0], sphi, C);
#pragma unroll
    for (int mu = 0; mu < d; ++mu) {
        const float a = cc.w[2 * mu + 1] * phi[mu];
        feq[2 * mu + 1] = fmaf(cc.adv[mu], C, a);
        feq[2 * mu + 2] = fmaf(-cc.adv[mu], C, a);
    }
    float dev[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) dev[i] = f[i] - feq[i];
    remove_mass_defect<Q>(dev);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        float r = 0.f;
#pragma unroll
        for (int j = 0; j < Q; ++j) r = fmaf(cc.R[i * Q + j], dev[j], r);
        fs[i] = f[i] - r;
        fs[i] = fmaf(cc.wSdt[i], S, fs[i]);
    }
    if (VAR) {
#pragma unroll
        for (int a = 0; a < d; ++a) {
            const float delta = flux_delta<Q>(dev, db, a);
            fs[2 * a + 1] = fmaf(-0.5f, delta, fs[2 * a + 1]);
            fs[2 * a + 2] = fmaf(0.5f, delta, fs[2 * a + 2]);
        }
    }
}

// Post-collision populations 1 and 2 (the two that cross x) of one node (a
// halo node at a strip edge).  With VAR, db holds row 0 of the node's dB.
template <int Q, bool VAR>
__device__ inline void collide_x_pair(const CollideConsts& cc, const float (&f)[Q], const float (&phi)[(Q - 1) / 2],
                                      float S, const float* db, float& f1, float& f2)
{
    // the same operations as collide_node's populations 1 and 2, fused alike
#pragma clang fp contract(off)
    constexpr int d = (Q - 1) / 2;
    float C = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) C += f[i];
    float feq[Q];
    float sphi = 0.f;
#pragma unroll
    for (int mu = 0; mu < d; ++mu) sphi += phi[mu];
    feq[0] = fmaf(-cc.w[0], sphi, C);
#pragma unroll
    for (int mu = 0; mu < d; ++mu) {
        const float x = cc.w[2 * mu + 1] * phi[mu];
        feq[2 * mu + 1] = fmaf(cc.adv[mu], C, x);
        feq[2 * mu + 2] = fmaf(-cc.adv[mu], C, x);
    }
    float dev[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) dev[j] = f[j] - feq[j];
    remove_mass_defect<Q>(dev);
    float ra = 0.f, rb = 0.f;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        ra = fmaf(cc.R[1 * Q + j], dev[j], ra);
        rb = fmaf(cc.R[2 * Q + j], dev[j], rb);
    }
    f1 = fmaf(cc.wSdt[1], S, f[1] - ra);
    f2 = fmaf(cc.wSdt[2], S, f[2] - rb);
    if (VAR) {
        // row 0 of dB: db[b] = dB_0b
        float s = 0.f;
#pragma unroll
        for (int b = 0; b < d; ++b) s = fmaf(db[b], dev[2 * b + 1] - dev[2 * b + 2], s);
        f1 = fmaf(-0.5f, s, f1);
        f2 = fmaf(0.5f, s, f2);
    }
}

// ---------------------------------------------------------------------------
// 2D D2Q5 fused kernel.  Rows move through a ring of D slots: while row y + 1
// is collided, the loads of rows y + 2 .. y + D are in flight.
template <bool HAS_S, bool VAR, bool NT, typename OFF>
__global__ __launch_bounds__(256) void collide_stream_2d(CollideConsts cc, const float* __restrict__ fin,
                                                         float* __restrict__ fout, const float* __restrict__ Phi,
                                                         const float* __restrict__ S, float* __restrict__ Cout,
                                                         int rows_per_wave, int strips, int total_waves)
{
    constexpr int D = 4;
    const int nx = cc.n[0], ny = cc.n[1];
    const int64_t nodes = (int64_t)nx * ny;
    const int lane = threadIdx.x & 63;
    const int gw = xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (gw >= total_waves) return;  // whole wavefront exits together
    const int strip = gw % strips, chunk = gw / strips;
    const int x0 = strip * kStrip;
    const int x = x0 + lane;
    const bool out_lane = x < nx;
    const int y0 = chunk * rows_per_wave;
    const int y1 = min(ny, y0 + rows_per_wave);

    // uniform base pointers of every array
    const float* fi[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) fi[i] = fin + i * nodes;
    const float* ph1 = Phi + nodes;
    const float* dbk[3];  // VAR: the three fields of dB (00, 01, 11)
#pragma unroll
    for (int k = 0; k < 3; ++k) dbk[k] = VAR ? cc.dB + k * nodes : nullptr;

    struct Row {
        float f[5], phi[2], s;  // this lane's node
        float h[5], hphi[2], hs;  // the node just outside the strip (left half: x0 - 1, right half: x0 + 64)
        float db[3], hdb[2];      // VAR: dB of the node, row 0 of dB of the halo node
    };
    // Nodes outside the box read the nearest node inside it: every population
    // they send into the box arrives through a wall and is replaced by the
    // Dirichlet rule, and they are never stored, so their values do not matter
    // (and the loads need no guard, no branch, no early wait).
    const int xc = min(x, nx - 1);
    const int hx = lane < 32 ? max(x0 - 1, 0) : min(x0 + kStrip, nx - 1);
    auto load_row = [&](int y, Row& r) {
        const int64_t rowoff = (int64_t)min(max(y, 0), ny - 1) * nx;
        const OFF b = (OFF)((rowoff + xc) * 4), bh = (OFF)((rowoff + hx) * 4);
#pragma unroll
        for (int i = 0; i < 5; ++i) r.f[i] = ldf(fi[i], b);
        r.phi[0] = ldf(Phi, b);
        r.phi[1] = ldf(ph1, b);
        r.s = HAS_S ? ldf(S, b) : 0.f;
#pragma unroll
        for (int i = 0; i < 5; ++i) r.h[i] = ldf(fi[i], bh);
        r.hphi[0] = ldf(Phi, bh);
        r.hphi[1] = ldf(ph1, bh);
        r.hs = HAS_S ? ldf(S, bh) : 0.f;
        if (VAR) {
#pragma unroll
            for (int k = 0; k < 3; ++k) r.db[k] = ldf(dbk[k], b);
#pragma unroll
            for (int k = 0; k < 2; ++k) r.hdb[k] = ldf(dbk[k], bh);
        }
    };
    // collision of a row: this lane's node, and the population its halo node
    // sends into the strip (f*_1 from the left neighbour, f*_2 from the right)
    auto collide_row = [&](const Row& r, float (&fs)[5], float& hv) {
        collide_node<5, VAR>(cc, r.f, r.phi, r.s, r.db, fs);
        float h1, h2;
        collide_x_pair<5, VAR>(cc, r.h, r.hphi, r.hs, r.hdb, h1, h2);
        hv = lane < 32 ? h1 : h2;
    };

    Row ring[D];
    load_row(y0 - 1, ring[D - 1]);  // halo row below the chunk (its f*_3 enters row y0)
#pragma unroll
    for (int k = 0; k < D - 1; ++k) load_row(y0 + k, ring[k]);
    float prev3, cur[5], hcur;
    {
        float t[5], th;
        collide_row(ring[D - 1], t, th);
        prev3 = t[3];
    }
    load_row(y0 + D - 1, ring[D - 1]);
    collide_row(ring[0], cur, hcur);
    // One output row y from ring slot u: refill the slot with row y + D (when
    // the chunk still needs that row), collide row y + 1, stream, store.
    auto row_step = [&](const int u, const int y, const bool refill) __attribute__((always_inline)) {
            if (refill) load_row(y + D, ring[u]);
            float nxt[5], hnxt;
            collide_row(ring[(u + 1) % D], nxt, hnxt);  // row y + 1
            // pull: f_1 from x-1, f_2 from x+1, f_3 from y-1, f_4 from y+1
            const float sl = __shfl_up(cur[1], 1, 64);
            const float sr = __shfl_down(cur[2], 1, 64);
            const float from_left = lane == 0 ? hcur : sl;
            const float from_right = lane == 63 ? hcur : sr;
            float f[5] = {cur[0], from_left, from_right, prev3, nxt[4]};
            const bool unk[5] = {false, x == 0, x == nx - 1, y == 0, y == ny - 1};
            int nu = 0;
            float known = 0.f;
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                if (unk[i]) ++nu;
                else known += f[i];
            }
            if (nu > 0) {
                // Dirichlet value of this wall node (clamped address: lanes past
                // the grid and rows past the chunk are never stored)
                const float cw =
                    VAR ? ldf(cc.Cw, (OFF)(((int64_t)min(y, ny - 1) * nx + xc) * 4)) : cc.c_wall;
                const float share = (cw - known) * inv_count(nu);
#pragma unroll
                for (int i = 0; i < 5; ++i)
                    if (unk[i]) f[i] = share;
            }
            if (out_lane && y < y1) {
                const OFF b = (OFF)(((int64_t)y * nx + x) * 4);
                float c = 0.f;
#pragma unroll
                for (int i = 0; i < 5; ++i) {
                    stv<NT>(fout + i * nodes, b, f[i]);
                    c += f[i];
                }
                stv<NT>(Cout, b, c);
            }
            prev3 = cur[3];
#pragma unroll
            for (int i = 0; i < 5; ++i) cur[i] = nxt[i];
            hcur = hnxt;
    };
    // The chunk needs rows y0 - 1 .. y1: blocks whose refills all stay within
    // y1 run without a condition; the last block refills only what is needed.
    int yb = y0;
    for (; yb + 2 * D - 1 <= y1; yb += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) row_step(u, yb + u, true);
    }
    for (; yb < y1; yb += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) row_step(u, yb + u, yb + u + D <= y1);
    }
}

// ---------------------------------------------------------------------------
// 3D D3Q7 fused kernel: workgroup = NY wavefronts (one per y row), rows 0 and
// NY-1 of the workgroup are halo rows; marches along z with a ring of D
// planes (the loads of planes z + 2 .. z + D are in flight while plane z + 1
// is collided).  f*_3 / f*_4 cross rows through LDS, double-buffered by plane
// parity so one barrier per plane suffices.
template <int NY, bool HAS_S, bool VAR, bool NT, typename OFF>
__global__ __launch_bounds__(64 * NY) void collide_stream_3d(CollideConsts cc, const float* __restrict__ fin,
                                                             float* __restrict__ fout, const float* __restrict__ Phi,
                                                             const float* __restrict__ S, float* __restrict__ Cout,
                                                             int planes_per_block, int strips_x, int strips_y)
{
    // Two ring slots: the loads of plane z + 2 are in flight while plane z + 1
    // is collided.  Fewer registers than a deeper ring (86 against 110 VGPRs)
    // and faster on MI355X (256^3: 307 us against 313 with three slots, 339
    // with four).
    constexpr int D = 2;
    const int nx = cc.n[0], ny = cc.n[1], nz = cc.n[2];
    const int64_t plane = (int64_t)nx * ny;
    const int64_t nodes = plane * nz;
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
    int b = xcd_tile(blockIdx.x, gridDim.x);
    const int sx = b % strips_x;
    b /= strips_x;
    const int sy = b % strips_y;
    const int chunk = b / strips_y;
    const int x0 = sx * kStrip;
    const int x = x0 + lane;
    const int y = sy * (NY - 2) - 1 + row;
    const bool out = x < nx && y >= 0 && y < ny && row >= 1 && row <= NY - 2;
    const int z0 = chunk * planes_per_block;
    const int z1 = min(nz, z0 + planes_per_block);

    // f*_3 (moving +y) and f*_4 (moving -y) of the current plane, by plane parity
    __shared__ float sh3[2][NY][64];
    __shared__ float sh4[2][NY][64];

    // one base per array and field offsets added per load (keeps the scalar
    // registers for the collision operator)
    const OFF fb = (OFF)(nodes * 4);  // bytes per field

    struct Plane {
        float f[7], phi[3], s;
        float h[7], hphi[3], hs;  // the node just outside the strip (left half: x0 - 1, right half: x0 + 64)
        float db[6], hdb[3];      // VAR: dB of the node, row 0 of dB of the halo node
    };
    // nodes outside the box read the nearest node inside it (see the 2D kernel)
    const int64_t yoff = (int64_t)min(max(y, 0), ny - 1) * nx;
    const int64_t xyc = yoff + min(x, nx - 1);
    const int64_t xyh = yoff + (lane < 32 ? max(x0 - 1, 0) : min(x0 + kStrip, nx - 1));
    auto load_at = [&](int z, Plane& p) {
        const int64_t zoff = (int64_t)min(max(z, 0), nz - 1) * plane;
        const OFF bm = (OFF)((zoff + xyc) * 4), bh = (OFF)((zoff + xyh) * 4);
#pragma unroll
        for (int i = 0; i < 7; ++i) p.f[i] = ldf(fin, bm + i * fb);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) p.phi[mu] = ldf(Phi, bm + mu * fb);
        p.s = HAS_S ? ldf(S, bm) : 0.f;
#pragma unroll
        for (int i = 0; i < 7; ++i) p.h[i] = ldf(fin, bh + i * fb);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) p.hphi[mu] = ldf(Phi, bh + mu * fb);
        p.hs = HAS_S ? ldf(S, bh) : 0.f;
        if (VAR) {
#pragma unroll
            for (int k = 0; k < 6; ++k) p.db[k] = ldf(cc.dB, bm + k * fb);
#pragma unroll
            for (int k = 0; k < 3; ++k) p.hdb[k] = ldf(cc.dB, bh + k * fb);
        }
    };
    auto collide_at = [&](const Plane& p, float (&fs)[7], float& hv) {
        collide_node<7, VAR>(cc, p.f, p.phi, p.s, p.db, fs);
        float h1, h2;
        collide_x_pair<7, VAR>(cc, p.h, p.hphi, p.hs, p.hdb, h1, h2);
        hv = lane < 32 ? h1 : h2;
    };

    Plane ring[D];
    load_at(z0 - 1, ring[D - 1]);  // halo plane below the chunk
#pragma unroll
    for (int k = 0; k < D - 1; ++k) load_at(z0 + k, ring[k]);
    float prev5, cur[7], hcur;
    {
        float t[7], th;
        collide_at(ring[D - 1], t, th);
        prev5 = t[5];
    }
    load_at(z0 + D - 1, ring[D - 1]);
    collide_at(ring[0], cur, hcur);
    // One output plane z from ring slot u (the refill condition is the same
    // for the whole workgroup, so every wave reaches the same barriers).
    auto plane_step = [&](const int u, const int z, const bool refill) __attribute__((always_inline)) {
            const int par = (z - z0) & 1;
            sh3[par][row][lane] = cur[3];
            sh4[par][row][lane] = cur[4];
            if (refill) load_at(z + D, ring[u]);
            float nxt[7], hnxt;
            collide_at(ring[(u + 1) % D], nxt, hnxt);  // plane z + 1
            lds_barrier();
            const float sl = __shfl_up(cur[1], 1, 64);
            const float sr = __shfl_down(cur[2], 1, 64);
            const float from_left = lane == 0 ? hcur : sl;
            const float from_right = lane == 63 ? hcur : sr;
            const float from_below = row >= 1 ? sh3[par][row - 1][lane] : 0.f;       // f*_3 of y-1
            const float from_above = row + 1 < NY ? sh4[par][row + 1][lane] : 0.f;  // f*_4 of y+1
            float f[7] = {cur[0], from_left, from_right, from_below, from_above, prev5, nxt[6]};
            const bool unk[7] = {false, x == 0, x == nx - 1, y == 0, y == ny - 1, z == 0, z == nz - 1};
            int nu = 0;
            float known = 0.f;
#pragma unroll
            for (int i = 0; i < 7; ++i) {
                if (unk[i]) ++nu;
                else known += f[i];
            }
            if (nu > 0) {
                const float cw =
                    VAR ? ldf(cc.Cw, (OFF)(((int64_t)min(z, nz - 1) * plane + xyc) * 4)) : cc.c_wall;
                const float share = (cw - known) * inv_count(nu);
#pragma unroll
                for (int i = 0; i < 7; ++i)
                    if (unk[i]) f[i] = share;
            }
            if (out && z < z1) {
                const OFF bo = (OFF)(((int64_t)z * plane + (int64_t)y * nx + x) * 4);
                float c = 0.f;
#pragma unroll
                for (int i = 0; i < 7; ++i) {
                    stv<NT>(fout, bo + i * fb, f[i]);
                    c += f[i];
                }
                stv<NT>(Cout, bo, c);
            }
            prev5 = cur[5];
#pragma unroll
            for (int i = 0; i < 7; ++i) cur[i] = nxt[i];
            hcur = hnxt;
    };
    // planes z0 - 1 .. z1 are needed; only the last block has refills to skip
    int zb = z0;
    for (; zb + 2 * D - 1 <= z1; zb += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) plane_step(u, zb + u, true);
    }
    for (; zb < z1; zb += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) plane_step(u, zb + u, zb + u + D <= z1);
    }
}

// ---------------------------------------------------------------------------
// f := f^eq(C, Phi) at every node (initial state).
template <int Q>
__global__ void equilibrium_init(CollideConsts cc, const float* __restrict__ C, const float* __restrict__ Phi,
                                 float* __restrict__ f, int64_t nodes)
{
    constexpr int d = (Q - 1) / 2;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nodes) return;
    const float c = C[x];
    float sphi = 0.f;
    float phi[d];
#pragma unroll
    for (int mu = 0; mu < d; ++mu) {
        phi[mu] = Phi[mu * nodes + x];
        sphi += phi[mu];
    }
    f[x] = c - cc.w[0] * sphi;
#pragma unroll
    for (int mu = 0; mu < d; ++mu) {
        const float a = cc.w[2 * mu + 1] * phi[mu];
        const float b = cc.adv[mu] * c;
        f[(2 * mu + 1) * nodes + x] = a + b;
        f[(2 * mu + 2) * nodes + x] = a - b;
    }
}

__global__ void wall_overwrite(CollideConsts cc, float* __restrict__ C, int64_t nodes)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nodes) return;
    int64_t r = i;
    bool wall = false;
    for (int mu = 0; mu < cc.dim; ++mu) {
        const int c = (int)(r % cc.n[mu]);
        r /= cc.n[mu];
        wall = wall || c == 0 || c == cc.n[mu] - 1;
    }
    if (wall) C[i] = cc.Cw ? cc.Cw[i] : cc.c_wall;
}

__global__ void fill_kernel(float* __restrict__ p, int64_t count, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

template <int Q>
__global__ void moment_kernel(const float* __restrict__ f, float* __restrict__ C, int64_t nodes)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nodes) return;
    float c = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) c += f[i * nodes + x];
    C[x] = c;
}


__global__ void nonfinite_kernel(const float* __restrict__ C, int64_t nodes, int* flag)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nodes) return;
    const float v = C[x];
    if (!(v == v) || fabsf(v) == __builtin_inff()) atomicOr(flag, 1);
}

int64_t nodes_of(const CollideConsts& cc)
{
    int64_t m = 1;
    for (int mu = 0; mu < cc.dim; ++mu) m *= cc.n[mu];
    return m;
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Calls f(integral_constant<bool, a>, ..., ...) for the run-time flags a, b, c:
// picks one of the eight instantiations of a kernel template.
template <typename F>
void with_bool(bool v, F&& f)
{
    if (v)
        f(std::true_type{});
    else
        f(std::false_type{});
}

// f(integral_constant<bool, a>, integral_constant<bool, b>, integral_constant<bool, c>)
template <typename F>
void with_flags(bool a, bool b, bool c, F&& f)
{
    with_bool(a, [&](auto A) { with_bool(b, [&](auto B) { with_bool(c, [&](auto C) { f(A, B, C); }); }); });
}

// March length forced by LBM_COLLIDE_ROWS (tuning; 0 = automatic): rows per
// wavefront of the 2D kernel, planes per workgroup of the 3D kernel.
int collide_rows_override()
{
    const char* e = getenv("LBM_COLLIDE_ROWS");
    const int r = e ? atoi(e) : 0;
    return (r >= 1 && r <= 1024) ? r : 0;
}

}  // namespace

hipError_t launch_collide_stream(const CollideConsts& cc, const float* f_in, float* f_out, const float* Phi,
                                 const float* S, float* C_out, hipStream_t s)
{
    // 32-bit byte offsets while every array (at most 7 fields of the node count) fits in 4 GiB
    const bool small = nodes_of(cc) * 7 * 4 < ((int64_t)1 << 32);
    // space-dependent diffusion tensor and wall values (both fields present)
    const bool var = cc.dB != nullptr;
    if (var && !cc.Cw) return hipErrorInvalidValue;
    // Non-temporal output stores once a step's traffic exceeds the 256 MB
    // Infinity Cache (below it, the next step reads the outputs from there).
    // Measured: 4096^2 177 -> 172 us, 256^3 303 -> 293 us; 1024^2 11.7 ->
    // 15.6 us if used there.  LBM_COLLIDE_NT = 0 / 1 forces it (tuning).
    bool nt = nodes_of(cc) * (2 * cc.Q + cc.dim + 1) * 4 > ((int64_t)256 << 20);
    if (const char* e = getenv("LBM_COLLIDE_NT")) {
        if (e[0] == '0') nt = false;
        if (e[0] == '1') nt = true;
    }
    if (cc.dim == 2) {
        const int nx = cc.n[0], ny = cc.n[1];
        const int strips = (nx + kStrip - 1) / kStrip;
        // Rows per wavefront: short marches leave more wavefronts to share the
        // chip, long ones amortise the two halo rows (which the neighbouring
        // march on the same XCD mostly has in L2 already).  Measured on
        // MI355X (4 / 8 / 16 / 32 rows): 512^2 5.0 / 6.8 / 9.8 / 15.6 us,
        // 1024^2 11.7 / 11.5 / 11.8 / 17.0, 2048^2 33.6 / 36.3 / 35.5 / 34.9,
        // 4096^2 182 / 180 / 175 / 175.  Shorter marches (2 or 3 rows) time
        // faster per kernel at 512^2 (5.8 us) but the 500-step 512^2 run is
        // slower with them (7.32 ms against 7.11 with 4 rows).
        int rows = collide_rows_override();
        if (rows <= 0) rows = (int64_t)nx * ny >= ((int64_t)1 << 23) ? 16 : 4;
        const int chunks = (ny + rows - 1) / rows;
        const int waves = strips * chunks;
        const unsigned blocks = (unsigned)((waves + 3) / 4);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, cc, f_in, f_out, Phi, S, C_out, rows, strips,
                               waves);
        };
        with_flags(S != nullptr, var, nt, [&](auto hs, auto vr, auto ntc) {
            constexpr bool HS = decltype(hs)::value, VR = decltype(vr)::value, NT = decltype(ntc)::value;
            if (small)
                go(collide_stream_2d<HS, VR, NT, uint32_t>);
            else
                go(collide_stream_2d<HS, VR, NT, uint64_t>);
        });
        return hipGetLastError();
    }
    // Rows per workgroup (one wave per row, the first and last are halo):
    // NY = 10 (8 output rows, so 8 | ny tiles the usual sizes exactly) for the
    // constant tensor: two workgroups fill a CU's 20 wave slots at 86 VGPRs,
    // and the y-halo rows come from L2 lines the neighbouring workgroup on the
    // same XCD fetched.  Measured at 256^3 (kernel trace; L2 fetches against
    // the algorithmic reads): NY = 8 with 16-plane marches 308.2 us, 1.43x;
    // NY = 10 with 16 planes 304.6 us, 1.16x; with 32 planes 290.7 us, 1.11x;
    // NY = 12 or 16 were slower (one workgroup per CU).  The space-dependent
    // variant (9 more values per ring plane, up to 256 VGPRs) keeps NY = 8.
    auto launch3d = [&](auto ny_c, auto hs, auto vr, auto ntc) {
        constexpr int NY = decltype(ny_c)::value;
        const int nx = cc.n[0], ny = cc.n[1], nz = cc.n[2];
        const int sx = (nx + kStrip - 1) / kStrip;
        const int sy = (ny + (NY - 2) - 1) / (NY - 2);
        // Long z marches amortise the two halo planes; a queue of several
        // workgroups per CU lets a new one start its ring while the others
        // march.  Measured on MI355X with NY = 8 (8 / 16 / 32 / 64 planes):
        // 128^3 33 / 38 / 39 / 69 us, 256^3 319 / 309 / 312 / 318, 384^3 1019 /
        // 975 / 946 / 939: the longest march that still gives 2048 workgroups;
        // with NY = 10 (256^3: 16 planes 304.6 us, 32 planes 290.7 us) the
        // longest that gives 1024.
        int planes = collide_rows_override();
        if (planes <= 0) {
            const int64_t want = NY == 8 ? 2048 : 1024;
            planes = 64;
            while (planes > 8 && (int64_t)sx * sy * ((nz + planes - 1) / planes) < want) planes /= 2;
        }
        const int chunks = (nz + planes - 1) / planes;
        const int64_t blocks = (int64_t)sx * sy * chunks;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        constexpr bool HS = decltype(hs)::value, VR = decltype(vr)::value, NT = decltype(ntc)::value;
        auto kern = small ? collide_stream_3d<NY, HS, VR, NT, uint32_t> : collide_stream_3d<NY, HS, VR, NT, uint64_t>;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * NY), 0, s, cc, f_in, f_out, Phi, S, C_out, planes,
                           sx, sy);
        return hipSuccess;
    };
    hipError_t e = hipSuccess;
    with_flags(S != nullptr, var, nt, [&](auto hs, auto vr, auto ntc) {
        if constexpr (decltype(vr)::value)
            e = launch3d(std::integral_constant<int, 8>{}, hs, vr, ntc);
        else
            e = launch3d(std::integral_constant<int, 10>{}, hs, vr, ntc);
    });
    if (e != hipSuccess) return e;
    return hipGetLastError();
}


hipError_t launch_equilibrium_init(const CollideConsts& cc, const float* C, const float* Phi, float* f, hipStream_t s)
{
    const int64_t nodes = nodes_of(cc);
    if (cc.Q == 5)
        hipLaunchKernelGGL(equilibrium_init<5>, dim3(blocks_for(nodes, 256)), dim3(256), 0, s, cc, C, Phi, f, nodes);
    else
        hipLaunchKernelGGL(equilibrium_init<7>, dim3(blocks_for(nodes, 256)), dim3(256), 0, s, cc, C, Phi, f, nodes);
    return hipGetLastError();
}

hipError_t launch_wall_overwrite(const CollideConsts& cc, float* C, hipStream_t s)
{
    const int64_t nodes = nodes_of(cc);
    hipLaunchKernelGGL(wall_overwrite, dim3(blocks_for(nodes, 256)), dim3(256), 0, s, cc, C, nodes);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t count, float v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, count, v);
    return hipGetLastError();
}

hipError_t launch_moment(const CollideConsts& cc, const float* f, float* C, hipStream_t s)
{
    const int64_t nodes = nodes_of(cc);
    if (cc.Q == 5)
        hipLaunchKernelGGL(moment_kernel<5>, dim3(blocks_for(nodes, 256)), dim3(256), 0, s, f, C, nodes);
    else
        hipLaunchKernelGGL(moment_kernel<7>, dim3(blocks_for(nodes, 256)), dim3(256), 0, s, f, C, nodes);
    return hipGetLastError();
}

hipError_t launch_nonfinite_check(const float* C, int64_t nodes, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(nonfinite_kernel, dim3(blocks_for(nodes, 256)), dim3(256), 0, s, C, nodes, flag);
    return hipGetLastError();
}

}  // namespace lbm
