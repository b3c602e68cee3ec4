// Dense-cell spreading and interpolation on the matrix cores (FP32 path).
//
// For the points of one densely populated base cell every tap of the
// (2m)^3 window block is shared, so both operations are dense matrix products
// over that block:
//   interp:  Y[point, r] = sum_tap  Wt[point, tap] * H[tap, r]
//   spread:  G[tap, r]  += sum_point Wt[tap, point] * V[point, r]
// with Wt[point, tap] = wx(ox) wy(oy) wz(oz) the separable window weights.
// Both run as v_mfma_f32_16x16x4_f32 products with 16 right-hand sides as
// the N dimension.  Lane l of a wave supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[4 (l / 16) + i][l % 16], i = 0..3.
//
// interp: M = 16 points, K = 4 taps along x.  The grid block is streamed
//   through LDS one z-slab (2m x 2m cells x 16 RHS) at a time, double
//   buffered; each wave covers 64 points (four M tiles).
// spread: M = 16 taps of one z-slab, K = 4 points.  Each wave owns a set of
//   z-slabs (all their taps in accumulators); points are staged in LDS in
//   rounds of 16 with their products wx*wy over the slab's taps.
#include <hip/hip_runtime.h>

#include "addk_internal.h"

namespace addk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// Matrix-core types per precision: one 16 x 16 x 4 product per instruction,
// v_mfma_f32_16x16x4f32 (FP32) or v_mfma_f64_16x16x4f64 (FP64).  Both take
// A[l % 16][l / 16] and B[l / 16][l % 16] from lane l; the FP32 product
// returns D[4 (l / 16) + i][l % 16] in register i, the FP64 one
// D[4 i + l / 16][l % 16] (out_row).
template <typename real>
struct MfmaT;
template <>
struct MfmaT<float> {
    typedef f4 v4;
    typedef float2 v2;
};
template <>
struct MfmaT<double> {
    typedef d4 v4;
    typedef double2 v2;
};
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ d4 mfma4(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename real>
__device__ __forceinline__ constexpr int out_row(int q, int i)
{
    return sizeof(real) == 4 ? 4 * q + i : 4 * i + q;
}

// psi(z) = m sinh(b s) / (sinh(b m) s), s = sqrt(m^2 - z^2), evaluated as
//   m e^{-b z^2 / (s + m)} (1 - e^{-2 b s}) / ((1 - e^{-2 b m}) s),
// using b (s - m) = -b z^2 / (s + m): the exponent is then small, and accurate
// to a few ulp, where psi is large.  Hardware sqrt / exp2 / rcp (about 1 ulp).
__device__ __forceinline__ float kb_psi_f(float z, float m, float b, float inv_e2bm)
{
    const float z2 = z * z;
    float s2 = m * m - z2;
    s2 = s2 > 1e-12f ? s2 : 1e-12f;
    const float s = __builtin_amdgcn_sqrtf(s2);
    const float bl = b * 1.4426950408889634f;
    const float e1 = __builtin_amdgcn_exp2f(-bl * z2 * __builtin_amdgcn_rcpf(s + m));
    const float e2 = __builtin_amdgcn_exp2f(-2.f * bl * s);
    return m * e1 * (1.f - e2) * inv_e2bm * __builtin_amdgcn_rcpf(s);
}

// FP64: the same stable form with IEEE sqrt and exp.
__device__ __forceinline__ double kb_psi_m(double z, double m, double b, double inv_e2bm)
{
    const double z2 = z * z;
    double s2 = m * m - z2;
    s2 = s2 > 1e-24 ? s2 : 1e-24;
    const double s = sqrt(s2);
    return m * exp(-b * z2 / (s + m)) * (1.0 - exp(-2.0 * b * s)) * inv_e2bm / s;
}
__device__ __forceinline__ float kb_psi_m(float z, float m, float b, float inv_e2bm) { return kb_psi_f(z, m, b, inv_e2bm); }

// Dense item anchor: base cell (bx, by, bz) and the number of cells in z
// (1, or 2 for two z-adjacent dense cells sharing one item).
__device__ __forceinline__ void unpack_cell_m(int packed, int &bx, int &by, int &bz, int &nzc)
{
    bx = packed & 1023;
    by = (packed >> 10) & 1023;
    bz = (packed >> 20) & 1023;
    nzc = ((packed >> 30) & 1) + 1;
}

__device__ __forceinline__ ProbDev get_prob_m(const IoArgs &io, int p) { return io.table ? io.table[p] : io.single; }

// Products of one z-slab for NG point groups and NO outputs (kernel and
// derivative-kernel grids).  One A fragment (the weights of 16 points at 4
// taps) feeds NO MFMAs and one B fragment (16 RHS at 4 taps) feeds NG MFMAs;
// the NG * NO accumulator chains are independent.  With one output, NA = 2
// accumulators per group take the even and odd y rows, so that there are
// still 2 NG independent chains to cover the matrix op's latency (they are
// summed at the end).
template <int NO>
constexpr int acc_rows() { return NO == 1 ? 2 : NO; }

template <typename real, int SW, int NT, int SX, int NG, int NO>
__device__ __forceinline__ void slab_products(typename MfmaT<real>::v4 (&acc)[acc_rows<NO>()][NG],
                                              const real (&wxq)[NG][NT], const real *wyl, const real (&wz)[NG],
                                              const bool (&live)[NG], const real (*sl)[16], int ny, int q, int mrow)
{
    constexpr int C = SW * SX;  // cells of one output's slab
    // rows in pairs, so that the accumulator row of a one-output product
    // (oy & 1) is known at compile time even where the row loop stays rolled
#pragma unroll
    for (int oy0 = 0; oy0 < SW; oy0 += 2)
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        const int oy = oy0 + par;
        if (oy >= SW || oy >= ny)
            break;
        real wyz[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g)
            wyz[g] = wyl[(g * SW + oy) * 16 + mrow] * wz[g];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            real b[NO];
#pragma unroll
            for (int o = 0; o < NO; ++o)
                b[o] = sl[o * C + oy * SX + 4 * t + q][mrow];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (!live[g])  // wave-uniform: no point of the group reaches this slab
                    continue;
                const real a = wyz[g] * wxq[g][t];
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    const int ai = NO == 1 ? par : o;
                    acc[ai][g] = mfma4(a, b[o], acc[ai][g]);
                }
            }
        }
    }
}

// Stream the z-slabs of an (SX x SW x nz) box of NO output grids, starting at
// grid cell (x0, y0, z0), through LDS (NB = 2: double buffered; NB = 1: one
// buffer and a second barrier per slab, for more blocks per CU; the next
// slab is prefetched into registers either way) and accumulate the products
// of the wave's NG point groups.  Cells outside the window's grid box read as
// zero.  Every thread of the block calls this with the same nz, so the
// barriers inside match.
template <typename real, int SW, int SX, int NT, int NG, int NO, int NB = 2>
__device__ __forceinline__ void stream_slabs(const WinDev &w, real (*slab)[NO][SW * SX][16], int r0, int nr, int x0,
                                             int y0, int z0, int sx, int sy, int nz,
                                             typename MfmaT<real>::v4 (&acc)[acc_rows<NO>()][NG],
                                             const real (&wxq)[NG][NT], const real *wyl,
                                             const real (&uzr)[NG], const int (&lbz)[NG], bool zmask)
{
    typedef typename MfmaT<real>::v2 v2;
    constexpr int C = SW * SX;
    constexpr int SL = (8 * C + kBlock - 1) / kBlock;  // complex values per thread per slab and output
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, mrow = lane & 15;
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    const gptr<const real> H = gbl((const real *)w.H);
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2];
    const int p0 = r0 >> 1;
    const int np = (nr + 1) >> 1;
    // Thread element idx covers RHS pair idx % 8 of cell idx / 8: the LDS
    // stores are then consecutive 8-byte words (no bank conflicts), and the
    // global loads read 64-byte runs of 8 cells in each pair's grid.
    v2 pre[NO][SL];
    auto load = [&](int oz) {
        const int gz = z0 + oz;
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int idx = threadIdx.x + k * kBlock;
                const int pi = idx & 7, c = idx >> 3;
                const int ox = c % SX, oy = c / SX;
                const int gx = x0 + ox, gy = y0 + oy;
                v2 v = {real(0), real(0)};
                if (idx < 8 * C && pi < np && ox < sx && oy < sy && gx < ex && gy < ey && gz < ez) {
                    const int64_t off =
                        ((int64_t)(o * w.npair_cap + p0 + pi) * w.szH + ((int64_t)gz * ey + gy) * ex + gx) * 2;
                    typedef real n2 __attribute__((ext_vector_type(2)));
                    const n2 t2 = *(gptr<const n2>)(H + off);
                    v = v2{t2.x, t2.y};
                }
                pre[o][k] = v;
            }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int k = 0; k < SL; ++k) {
                const int idx = threadIdx.x + k * kBlock;
                if (idx < 8 * C) {
                    const int pi = idx & 7, c = idx >> 3;
                    *(v2 *)&slab[buf][o][c][2 * pi] = v2{pre[o][k].x, (2 * pi + 1 < nr) ? pre[o][k].y : real(0)};
                }
            }
    };
    load(0);
    store(0);
    __syncthreads();
    for (int oz = 0; oz < nz; ++oz) {
        if (oz + 1 < nz)
            load(oz + 1);  // in flight during this slab's products
        real wz[NG];
        bool live[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            // lbz: the point's first z slab in the box (far away for inactive lanes)
            const bool in = (unsigned)(oz - lbz[g]) < (unsigned)w.W;
            live[g] = __builtin_amdgcn_readfirstlane(__any(in)) != 0;
            wz[g] = (!zmask || in) ? kb_psi_m(uzr[g] - (real)(z0 + oz), mm, kb, ie) : real(0);
        }
        slab_products<real, SW, NT, SX, NG, NO>(acc, wxq, wyl, wz, live, &slab[NB == 2 ? oz & 1 : 0][0][0], sy, q,
                                                mrow);
        if (oz + 1 < nz) {
            if (NB == 1)
                __syncthreads();  // every wave is done with the buffer
            store(NB == 2 ? (oz + 1) & 1 : 0);
        }
        __syncthreads();
    }
}

// One dense item: every wave takes NG of the item's 16-point groups (group
// wave + 4 g); groups past the item's end carry zero weights.
template <typename real, int W, int NO, int NG>
__device__ __forceinline__ void interp_dense_item(const WinDev &w, const Chunk &it, int r0, int nr,
                                                  real (*slab)[NO][W * W][16], real *wy_lds)
{
    typedef typename MfmaT<real>::v4 v4;
    constexpr int NT = W / 4;  // K steps per x row
    int bx, by, bz, nzc;
    unpack_cell_m(it.tile, bx, by, bz, nzc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, mrow = lane & 15;
    const gptr<const real> coords = gbl((const real *)w.coords);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    // x weights stay in registers (lane q holds taps 4t + q); the y weights of
    // the wave's points go to its LDS area [g][oy][16 points], each lane
    // computing the taps 4t + q of its point
    real *wyl = wy_lds + wave * (4 * W * 16);
    real wxq[NG][NT], uz[NG];
    int lbz[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int p = (wave + 4 * g) * 16 + mrow;
        const bool act = p < it.count;
        const int j = it.start + (act ? p : 0);
        const real ux = coords[j], uy = coords[w.N + j];
        uz[g] = coords[2 * w.N + j];
        lbz[g] = act ? (int)floorf(uz[g]) - w.m + 1 - bz : (1 << 20);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            wxq[g][t] = act ? kb_psi_m(ux - (real)(bx + 4 * t + q), mm, kb, ie) : real(0);
            wyl[(g * W + 4 * t + q) * 16 + mrow] = kb_psi_m(uy - (real)(by + 4 * t + q), mm, kb, ie);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    constexpr int NA = acc_rows<NO>();
    v4 acc[NA][NG];
#pragma unroll
    for (int o = 0; o < NA; ++o)
#pragma unroll
        for (int g = 0; g < NG; ++g)
            acc[o][g] = v4{real(0), real(0), real(0), real(0)};
    // With two z cells, one of the 2m + 1 slabs lies just outside each point's
    // window, where the window formula does not vanish (~2.5e-7 at m = 4,
    // 3e-11 at m = 6), so the z weights are masked to the point's own 2m
    // slabs; a group whose points all lie in one of the cells skips its
    // outside slab altogether.
    stream_slabs<real, W, W, NT, NG, NO, 1>(w, slab, r0, nr, bx, by, bz, W, W, W + nzc - 1, acc, wxq, wyl, uz, lbz,
                                            true);
    if (NO == 1)
#pragma unroll
        for (int g = 0; g < NG; ++g)
            acc[0][g] += acc[NA - 1][g];
    if (mrow >= nr)
        return;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const gptr<real> dst = gbl((real *)w.Yw) + (int64_t)o * w.N * w.Rcap + r0 + mrow;
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = (wave + 4 * g) * 16 + out_row<real>(q, i);
                if (p < it.count)
                    dst[(int64_t)gbl(w.perm)[it.start + p] * w.Rcap] = acc[o][g][i];
            }
    }
}

// ---------------------------------------------------------------------------
// Dense interp with one RHS: the item's 2m + 1 z-slabs take the 16 columns.
// T[point][slab] = sum over the slab's taps A[point][tap] H[tap][slab] is one
// matrix product over the (2m)^2 x-y taps (K steps of four taps, lane q taking
// tap 4 t + q as in the slab kernel), then Y[point] = sum_slab wz T, a sum over
// the 16 lanes of a row.  The item's block of RHS 0 is staged in LDS once,
// [o][slab][tap] with the row padded by one word; slabs past the item's are
// zero.
template <int W, int NO, int NG>
__device__ __forceinline__ void interp_dense_item_z1(const WinDev &w, const Chunk &it, const float *hl, float *wy_lds)
{
    constexpr int WW = W * W, NT = W / 4, HS = WW + 1;
    int bx, by, bz, nzc;
    unpack_cell_m(it.tile, bx, by, bz, nzc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, mrow = lane & 15;
    const gptr<const float> coords = gbl((const float *)w.coords);
    const float mm = (float)w.m, kb = (float)w.b, ie = (float)w.inv_e2bm;
    float *wyl = wy_lds + wave * (4 * W * 16);
    float wxq[NG][NT];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int p = (wave + 4 * g) * 16 + mrow;
        const bool act = p < it.count;
        const int j = it.start + (act ? p : 0);
        const float ux = coords[j], uy = coords[w.N + j];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            wxq[g][t] = act ? kb_psi_f(ux - (float)(bx + 4 * t + q), mm, kb, ie) : 0.f;
            wyl[(g * W + 4 * t + q) * 16 + mrow] = kb_psi_f(uy - (float)(by + 4 * t + q), mm, kb, ie);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    f4 acc[NO][NG];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int g = 0; g < NG; ++g)
            acc[o][g] = f4{0.f, 0.f, 0.f, 0.f};
    // K step (oy, t): taps oy W + 4 t + q; B[tap][slab mrow] = hl[o][mrow][tap]
#pragma unroll
    for (int oy = 0; oy < W; ++oy) {
        float wy[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g)
            wy[g] = wyl[(g * W + oy) * 16 + mrow];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            float b[NO];
#pragma unroll
            for (int o = 0; o < NO; ++o)
                b[o] = hl[(o * 16 + mrow) * HS + oy * W + 4 * t + q];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const float a = wy[g] * wxq[g][t];
#pragma unroll
                for (int o = 0; o < NO; ++o)
                    acc[o][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[o], acc[o][g], 0, 0, 0);
            }
        }
    }
    // lane (q, mrow) holds T[point 4 q + i][slab mrow]: weight by the point's z
    // window at that slab, then sum the slabs over the 16 lanes of the row
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = (wave + 4 * g) * 16 + 4 * q + i;
            const bool act = p < it.count;
            const float uz = coords[2 * w.N + it.start + (act ? p : 0)];
            const int dz = (int)floorf(uz) - w.m + 1 - bz;  // the point's first slab in the item
            const bool in = act && (unsigned)(mrow - dz) < (unsigned)W;
            const float wz = in ? kb_psi_f(uz - (float)(bz + mrow), mm, kb, ie) : 0.f;
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                float v = wz * acc[o][g][i];
#pragma unroll
                for (int s = 8; s > 0; s >>= 1)
                    v += __shfl_xor(v, s, 16);
                if (act && mrow == 0)
                    gbl((float *)w.Yw)[((int64_t)o * w.N + gbl(w.perm)[it.start + p]) * w.Rcap] = v;
            }
        }
    }
}

template <int W, int NO>
__global__ __launch_bounds__(kBlock) void k_interp_mfma_z1(const WinDev *__restrict__ wins,
                                                           const Chunk *__restrict__ items)
{
    constexpr int WW = W * W, HS = WW + 1;
    __shared__ __align__(16) float hl[NO * 16 * HS];
    __shared__ __align__(16) float wy_lds[4 * 4 * W * 16];
    const Chunk it = items[blockIdx.x];
    const WinDev &w = wins[it.win];
    int bx, by, bz, nzc;
    unpack_cell_m(it.tile, bx, by, bz, nzc);
    const int NS = W + nzc - 1;
    // stage RHS 0 (the real part of pair 0) of the item's block, zero outside
    // the grid box and past the item's slabs
    const gptr<const float> H = gbl((const float *)w.H);
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2];
    for (int e = threadIdx.x; e < NO * 16 * WW; e += kBlock) {
        const int o = e / (16 * WW), rem = e - o * (16 * WW), oz = rem / WW, tap = rem - oz * WW;
        const int gx = bx + tap % W, gy = by + tap / W, gz = bz + oz;
        float v = 0.f;
        if (oz < NS && gx < ex && gy < ey && gz < ez)
            v = H[((int64_t)o * w.npair_cap * w.szH + ((int64_t)gz * ey + gy) * ex + gx) * 2];
        hl[(o * 16 + oz) * HS + tap] = v;
    }
    __syncthreads();
    const int ng = (((it.count + 15) >> 4) + 3) >> 2;
    switch (ng) {
    case 1: interp_dense_item_z1<W, NO, 1>(w, it, hl, wy_lds); break;
    case 2: interp_dense_item_z1<W, NO, 2>(w, it, hl, wy_lds); break;
    case 3: interp_dense_item_z1<W, NO, 3>(w, it, hl, wy_lds); break;
    default: interp_dense_item_z1<W, NO, 4>(w, it, hl, wy_lds); break;
    }
}

// ---------------------------------------------------------------------------
// Dense interp: one block per dense item (<= 256 points) and 16 RHS, NO
// outputs at once.  The number of groups per wave is uniform in the block, so
// the dispatch below is a uniform branch and every wave runs the same slab
// loop (and barriers).
template <typename real, int W, int NO>
__global__ __launch_bounds__(kBlock, sizeof(real) == 4 ? 5 : 2) void k_interp_mfma(const WinDev *__restrict__ wins,
                                                                                  const Chunk *__restrict__ items,
                                                                                  int R)
{
    // one slab buffer (31 KB of LDS with the y weights at 2m = 12, two outputs)
    // and at most 96 registers (a few spills at the slab barriers): five blocks
    // per CU in FP32; in FP64 the 61 KB of LDS allow two
    __shared__ __align__(16) real slab[1][NO][W * W][16];
    __shared__ __align__(16) real wy_lds[4 * 4 * W * 16];
    const Chunk it = items[blockIdx.x];
    const WinDev &w = wins[it.win];
    const int r0 = blockIdx.y * 16;
    if (r0 >= R)
        return;
    const int nr = min(16, R - r0);
    const int ng = (((it.count + 15) >> 4) + 3) >> 2;
    switch (ng) {
    case 1: interp_dense_item<real, W, NO, 1>(w, it, r0, nr, slab, wy_lds); break;
    case 2: interp_dense_item<real, W, NO, 2>(w, it, r0, nr, slab, wy_lds); break;
    case 3: interp_dense_item<real, W, NO, 3>(w, it, r0, nr, slab, wy_lds); break;
    default: interp_dense_item<real, W, NO, 4>(w, it, r0, nr, slab, wy_lds); break;
    }
}

// ---------------------------------------------------------------------------
// Dense spread: one block per spread item (one or two dense cells) and 16 RHS;
// the item's (2m)^2 x (2m + 1) block is written to its scratch slot and summed
// into the grid by k_gather_blocks.
// The x-y taps of a z-slab are tiled as 4 x 4 squares: M tile (tx, ty) holds
// the taps x = 4 tx + (row & 3), y = 4 ty + (row >> 2), so the A operand of
// lane (q, mrow), wx(x) wy(y), is the product of one of 2m / 4 x weights and
// one of 2m / 4 y weights of point 4 ks + q; both come straight from the
// round's window table in LDS (no product table, one barrier per round).
// Z1 (one RHS, FP32): the 2m + 1 z-slabs take the N dimension instead of the
// RHS, D[16 taps][16 slabs] += A[taps][4 points] B[4 points][slabs] with
// B = v wz(slab); wave w owns the M tiles w + 4 j of the whole block (linear
// tap order), and the flush writes the block with one value per tap (the
// gather's one-RHS layout).
// MS: the M tiles are split over MS blocks (blockIdx.z), each owning MTB
// consecutive tiles (whole rows of squares) of every slab; FP64 uses MS = 2
// or 3 so that the accumulators (twice the registers of FP32) stay in the
// register file, at the price of evaluating each point's window values MS
// times.
template <typename real, int W, bool Z1, int MS, bool TWO>
__global__ __launch_bounds__(kBlock) void k_spread_mfma(const WinDev *__restrict__ wins, const Chunk *__restrict__ items,
                                                        int item0, IoArgs io, int R, real *__restrict__ scratch)
{
    typedef typename MfmaT<real>::v4 v4;
    constexpr int WW = W * W;
    constexpr int NX = W / 4;          // squares per row of taps
    constexpr int MT = WW / 16;        // M tiles (16 taps) per z-slab
    constexpr int MTB = (MT + MS - 1) / MS;  // M tiles of this block
    static_assert(Z1 || MTB * MS == MT && MTB % NX == 0, "blocks own whole rows of squares");
    constexpr int NYB = Z1 ? 1 : MTB / NX;  // rows of squares of this block
    constexpr int SPW = W / 4;         // z-slabs per wave: slabs wave + 4 s, s < SPW (the first 2m)
    constexpr int XT = (MTB + 3) / 4;  // M tiles per wave of slab 2m (two-cell items only)
    constexpr int PB = 32;             // points per round (PB / 4 K steps; FP64 measured 8.55 ms at 16, 8.15 at 32)
    constexpr int KV = PB * 16 / kBlock;             // RHS values staged per thread and round
    constexpr int NYV = Z1 ? W : 4 * NYB;  // y window values per point: the y taps of this block's squares
    constexpr int ZO = W + NYV;            // offset of the z values
    constexpr int PS = ZO + W + 1;         // window values per point: x [W], y [NYV], z [W + 1] (item slabs)
    constexpr int NWE = PB * PS;                     // window values per round
    constexpr int KW = (NWE + kBlock - 1) / kBlock;  // window values per thread and round
    struct Round {
        real pw[KW * kBlock];  // [PB][PS] and the last thread slice's unused entries
        real pv[PB][16];
    };
    __shared__ __align__(16) Round rd[2];

    const int ii = item0 + (int)blockIdx.x;  // the item (and its scratch slot)
    const Chunk it = items[ii];
    const WinDev &w = wins[it.win];
    const int r0 = blockIdx.y * 16;
    if (r0 >= R)
        return;
    const int mt0 = MS > 1 ? (int)blockIdx.z * MTB : 0;  // first M tile of this block
    const int ty0 = mt0 / NX;                              // its first row of squares
    int bx, by, bz, nzc;
    unpack_cell_m(it.tile, bx, by, bz, nzc);
    const int NS = W + nzc - 1;  // z-slabs of the item's block
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: slab branches are scalar
    const int q = lane >> 4, mrow = lane & 15;
    const int xi = mrow & 3, yi = mrow >> 2;  // the lane's tap within a square
    const gptr<const real> coords = gbl((const real *)w.coords);
    const ProbDev pio = get_prob_m(io, w.prob);
    const gptr<const real> vp = gbl((const real *)pio.Vp);
    const gptr<const int32_t> perm = gbl(w.perm);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    const int t = threadIdx.x;

    // prefetch registers: the coordinates behind this thread's window values
    // (entry e = p * PS + o of the round's table, o < W: x, o < 2W: y, else z;
    // e = t + k * kBlock) and KV RHS values; all threads then share the
    // window evaluations.  The RHS values are gathered through the point
    // permutation, whose entries are loaded one round earlier still (pix), so
    // that no load waits for another one issued just before it.
    real pcs[KW];
    real pvv[KV];
    int pix[KV];
#pragma unroll
    for (int k = 0; k < KV; ++k)
        pvv[k] = real(0);
    auto load_pix = [&](int p0) {
        const int np = min(PB, it.count - p0);
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            const int p = (t + k * kBlock) >> 4;
            pix[k] = p < np ? perm[it.start + p0 + p] : -1;
        }
    };
    auto load = [&](int p0) {  // round p0's coordinates, and its RHS values through pix
        const int np = min(PB, it.count - p0);
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int e = t + k * kBlock;
            const int p = e / PS, o = e - p * PS;
            const int dd = o < W ? 0 : (o < ZO ? 1 : 2);
            pcs[k] = (e < NWE && p < np) ? coords[dd * w.N + it.start + p0 + p] : real(0);
        }
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            const int r = r0 + ((t + k * kBlock) & 15);
            pvv[k] = (pix[k] >= 0 && r < R) ? vp[(int64_t)pix[k] * pio.ldvp + r] : real(0);
        }
    };
    // Straight-line code (selects, no branches) so that the compiler can
    // interleave it with the matrix ops of the current round.
    auto store_raw = [&](Round &d, int p0) {
        const int np = min(PB, it.count - p0);
        real *pw = d.pw;
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int e = t + k * kBlock;
            const int p = e / PS, o = e - p * PS;
            // x and y: tap o of the item's block; z: slab oz of the item, inside the
            // point's own window only
            const int oz = o - ZO;
            const int dz = (int)floor(pcs[k]) - w.m + 1 - bz;
            const real c = o < W ? (real)(bx + o) : (o < ZO ? (real)(by + 4 * ty0 + o - W) : (real)(bz + oz));
            const bool live = p < np && (o < ZO || (unsigned)(oz - dz) < (unsigned)W);
            const real v = kb_psi_m(pcs[k] - c, mm, kb, ie);
            if (KW * kBlock == NWE || e < NWE)
                pw[e] = live ? v : real(0);
        }
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            const int e = t + k * kBlock;
            d.pv[e >> 4][e & 15] = pvv[k];
        }
    };
    // The same work in slices, one per K step of round p0 (FP32): slice k < KW
    // writes window value slice k of round p0 + PB to nx and loads its
    // coordinate for round p0 + 2 PB; slice KW + j writes RHS slice j, loads
    // it for round p0 + 2 PB (through pix) and pix for round p0 + 3 PB.  Every
    // lane loads from a valid address and keeps the value as loaded (no select
    // that the compiler would turn into a branch around the load and a wait
    // for it): lanes past the item take its first point, whose window values
    // there are zero, and RHS columns past R read the zero padding of the
    // point-major copy.  The slices are then straight-line code that the
    // scheduler can place among the matrix ops.
    auto slice = [&](Round &nx, int p0, int k) {
        if (k < KW) {
            const int np = min(PB, it.count - (p0 + PB));
            const int e = t + k * kBlock;
            const int p = e / PS, o = e - p * PS;
            const int oz = o - ZO;
            const int dz = (int)floor(pcs[k]) - w.m + 1 - bz;
            const real c = o < W ? (real)(bx + o) : (o < ZO ? (real)(by + 4 * ty0 + o - W) : (real)(bz + oz));
            const bool live = p < np && (o < ZO || (unsigned)(oz - dz) < (unsigned)W);
            const real v = kb_psi_m(pcs[k] - c, mm, kb, ie);
            nx.pw[e] = live ? v : real(0);
            const int np2 = min(PB, it.count - (p0 + 2 * PB));
            const int dd = o < W ? 0 : (o < ZO ? 1 : 2);
            pcs[k] = coords[dd * w.N + it.start + (e < NWE && p < np2 ? p0 + 2 * PB + p : 0)];
        } else if (k < KW + KV) {
            const int j = k - KW;
            const int e = t + j * kBlock;
            nx.pv[e >> 4][e & 15] = pvv[j];
            const int r = r0 + (e & 15);  // r < ldvp (RHS padded to 16 with zeros)
            pvv[j] = vp[(int64_t)max(pix[j], 0) * pio.ldvp + r];
            const int np3 = min(PB, it.count - (p0 + 3 * PB));
            const int p = e >> 4;
            pix[j] = perm[it.start + (p < np3 ? p0 + 3 * PB + p : 0)];
        }
    };

    // wave `wave` owns slabs wave + 4 s of the first 2m and, for two-cell
    // items, the M tiles mt0 + wave + 4 j of slab 2m (Z1: the M tiles wave + 4 j
    // of every slab, accz)
    constexpr int JT = (MT + 3) / 4;
    v4 acc[Z1 ? 1 : SPW][Z1 ? 1 : MTB], accx[XT], accz[Z1 ? JT : 1];
    const v4 zero4 = v4{real(0), real(0), real(0), real(0)};
#pragma unroll
    for (int s = 0; s < (Z1 ? 1 : SPW); ++s)
#pragma unroll
        for (int mt = 0; mt < (Z1 ? 1 : MTB); ++mt)
            acc[s][mt] = zero4;
#pragma unroll
    for (int j = 0; j < XT; ++j)
        accx[j] = zero4;
#pragma unroll
    for (int j = 0; j < (Z1 ? JT : 1); ++j)
        accz[j] = zero4;

    // Z1: lane mrow's tap of M tile wave + 4 j is (x, y) = (zx[j], zy[j] - W)
    // (linear tap order).  Otherwise: the x and y window-table entries of the
    // lane's A operand in the slab-2m tiles mt0 + wave + 4 j (squares).
    int zx[Z1 ? JT : XT], zy[Z1 ? JT : XT];
#pragma unroll
    for (int j = 0; j < (Z1 ? JT : XT); ++j) {
        if constexpr (Z1) {
            const int c = min((wave + 4 * j) * 16 + mrow, WW - 1);
            zx[j] = c % W;
            zy[j] = W + c / W;
        } else {
            const int mt = min(mt0 + wave + 4 * j, MT - 1);
            zx[j] = 4 * (mt % NX) + xi;
            zy[j] = W + 4 * (mt / NX - ty0) + yi;
        }
    }
    // Operands of one K step (four points): the lane's x weights (one per
    // column of squares) and y weights (one per row of squares of this
    // block), the slab-2m A values, and the B factors (RHS value, z weights of
    // the wave's slabs).  In full rounds the next step's operands are read
    // from LDS before this step's matrix ops issue, so the reads overlap them.
    struct Ops {
        real wx[NX], wy[NYB], ax[XT], v, wz[SPW + 1];
    };
    auto fetch = [&](const Round &cr, int ks, Ops &o) {
        const int pk = 4 * ks + q;
        const real *pw = cr.pw + pk * PS;
#pragma unroll
        for (int i = 0; i < NX; ++i)
            o.wx[i] = pw[4 * i + xi];
#pragma unroll
        for (int i = 0; i < NYB; ++i)
            o.wy[i] = pw[W + 4 * i + yi];
#pragma unroll
        for (int j = 0; j < XT; ++j)
            o.ax[j] = pw[zx[j]] * pw[zy[j]];
        o.v = cr.pv[pk][mrow];
#pragma unroll
        for (int s = 0; s < SPW; ++s)
            o.wz[s] = pw[ZO + wave + 4 * s];
        o.wz[SPW] = pw[ZO + W];  // slab 2m: zero for single-cell items
    };
    auto step = [&](const Ops &o, auto xtag) {
        real a[MTB];
#pragma unroll
        for (int mt = 0; mt < MTB; ++mt)
            a[mt] = o.wx[mt % NX] * o.wy[mt / NX];
        // the point's z weight of the slab scales the B operand (its RHS
        // values), so the A operand is the plain x-y weight product
#pragma unroll
        for (int s = 0; s < SPW; ++s) {
            const real b = o.v * o.wz[s];
#pragma unroll
            for (int mt = 0; mt < MTB; ++mt)
                acc[s][mt] = mfma4(a[mt], b, acc[s][mt]);
        }
        if constexpr (decltype(xtag)::value) {  // slab 2m: two-cell items only
            const real bx2 = o.v * o.wz[SPW];
#pragma unroll
            for (int j = 0; j < XT; ++j)
                accx[j] = mfma4(o.ax[j], bx2, accx[j]);
        }
    };
    const std::integral_constant<bool, TWO> with_x;

    // FP32 (not Z1): the full rounds in the main loop, and a partial last
    // round after it with only the K steps it fills; otherwise every round in
    // the main loop (in FP64 the separate last-round loop costs registers:
    // 228 -> 308)
    constexpr bool TAIL = !Z1 && sizeof(real) == 4;
    // FP32 (not Z1): the next round's window values and loads in slices inside
    // the K loop
    constexpr bool PIPE = TAIL;
    static_assert(!PIPE || KW + KV <= PB / 4, "one slice per K step");
    // FP32 two-cell items: the points before the first one with a weight in
    // slab 2m (the item's points are ordered by cell, the lower one first)
    // skip slab 2m's matrix ops in the rounds they fill
    constexpr bool SKIPX = PIPE && TWO;
    __shared__ int first_x[SKIPX ? 4 : 1];
    if constexpr (SKIPX) {
        int f = it.count;
        for (int j = t; j < it.count; j += kBlock) {
            const real uz = coords[2 * w.N + it.start + j];
            if ((int)floor(uz) - w.m + 1 - bz > 0)
                f = min(f, j);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            f = min(f, __shfl_xor(f, o));
        if (lane == 0)
            first_x[wave] = f;  // read after the barrier below
    }
    load_pix(0);
    load(0);
    if (PB < it.count)
        load_pix(PB);
    store_raw(rd[0], 0);
    if (PB < it.count) {
        load(PB);  // the registers run one round ahead of the window values
        if (2 * PB < it.count)
            load_pix(2 * PB);
    }
    __syncthreads();
    int buf = 0;
    const int pend = TAIL ? it.count / PB * PB : it.count;
    auto round = [&](int p0, auto xtag) {
        const bool more = p0 + PB < it.count;
        // the next round's window values go to the other buffer, which no wave
        // reads any more (every wave passed the last round's closing barrier);
        // then the registers take the round after it (and pix the one after that)
        if (!PIPE && more) {
            store_raw(rd[buf ^ 1], p0 + PB);
            if (p0 + 2 * PB < it.count) {
                load(p0 + 2 * PB);
                if (p0 + 3 * PB < it.count)
                    load_pix(p0 + 3 * PB);
            }
        }
        Round &cr = rd[buf];
        if constexpr (Z1) {
#pragma unroll
            for (int ks = 0; ks < PB / 4; ++ks) {
                const int pk = 4 * ks + q;
                // B[point][slab mrow] = v wz(slab); zero past the item's 2m + 1 slabs
                const real *pw = cr.pw + pk * PS;
                const real b = mrow <= W ? cr.pv[pk][0] * pw[ZO + min(mrow, W)] : real(0);
#pragma unroll
                for (int j = 0; j < JT; ++j) {
                    const int mt = wave + 4 * j;
                    if (mt < MT)
                        accz[j] = mfma4(pw[zx[j]] * pw[zy[j]], b, accz[j]);
                }
            }
        } else {
            Ops ops[2];
            fetch(cr, 0, ops[0]);
#pragma unroll
            for (int ks = 0; ks < PB / 4; ++ks) {
                const Ops &o = ops[ks & 1];
                if (ks + 1 < PB / 4)
                    fetch(cr, ks + 1, ops[(ks + 1) & 1]);
                if constexpr (PIPE)
                    slice(rd[buf ^ 1], p0, ks);  // past the last round: unused values, no reads past the item
                step(o, xtag);
                // schedule the step as: the next step's LDS reads, this step's
                // operand products, its matrix ops (left to itself, the compiler
                // interleaves the reads with the matrix ops and waits for each)
                __builtin_amdgcn_sched_group_barrier(0x100, 64, 0);  // LDS reads
                __builtin_amdgcn_sched_group_barrier(0x002, 64, 0);  // vector ALU
                __builtin_amdgcn_sched_group_barrier(0x008, 64, 0);  // matrix ops
                if constexpr (PIPE) {
                    // the slice's LDS write and loads stay in their step, a
                    // round ahead of the slice that uses the loaded values
                    __builtin_amdgcn_sched_group_barrier(0x200, 8, 0);  // LDS writes
                    __builtin_amdgcn_sched_group_barrier(0x020, 8, 0);  // memory reads
                }
            }
        }
        __syncthreads();
        buf ^= 1;
    };
    int p0 = 0;
    if constexpr (SKIPX) {
        const int fx = min(min(first_x[0], first_x[1]), min(first_x[2], first_x[3]));
        for (; p0 + PB <= min(fx, pend); p0 += PB)
            round(p0, std::false_type());
    }
    for (; p0 < pend; p0 += PB)
        round(p0, with_x);
    if constexpr (TAIL) {
        // the last round's points (its window values are in rd[buf])
        const int nks = (it.count - pend + 3) >> 2;
#pragma unroll 1
        for (int ks = 0; ks < nks; ++ks) {
            Ops o;
            fetch(rd[buf], ks, o);
            step(o, with_x);
        }
    }

    // write the item's block [oz][oy][ox][16 RHS] to its scratch slot (plain
    // stores; the blocks of all items are summed by k_gather_blocks).  A lane
    // holds 4 taps of one RHS per M tile; for one register the 16 lanes of a
    // quarter-wave write the 16 RHS of one tap (64 contiguous bytes).
    if constexpr (Z1) {
        // lane (q, mrow) holds taps mt 16 + 4 q + i of slab mrow; one RHS per tap
        real *dz = scratch + (int64_t)ii * ((W + 1) * WW);
#pragma unroll
        for (int j = 0; j < JT; ++j) {
            const int mt = wave + 4 * j;
            if (mt < MT && mrow < NS)
                *(v4 *)(dz + mrow * WW + mt * 16 + 4 * q) = accz[j];
        }
        return;
    }
    real *dst = scratch + ((int64_t)ii * gridDim.y + blockIdx.y) * ((W + 1) * WW * 16);
    // D row `row` of square (tx, ty) is tap (4 ty + (row >> 2)) W + 4 tx + (row & 3);
    // the block's taps are the contiguous range from mt0 16 (whole rows of squares)
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        real *ds = dst + ((int64_t)(wave + 4 * s) * WW + mt0 * 16) * 16;
#pragma unroll
        for (int mt = 0; mt < MTB; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = out_row<real>(q, i);
                const int tap = (4 * (mt / NX) + (row >> 2)) * W + 4 * (mt % NX) + (row & 3);
                ds[tap * 16 + mrow] = acc[s][mt][i];
            }
    }
    if (NS > W) {
#pragma unroll
        for (int j = 0; j < XT; ++j) {
            const int mt = mt0 + wave + 4 * j;
            if (wave + 4 * j >= MTB || mt >= MT)
                break;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = out_row<real>(q, i);
                const int tap = (4 * (mt / NX) + (row >> 2)) * W + 4 * (mt % NX) + (row & 3);
                dst[((int64_t)W * WW + tap) * 16 + mrow] = accx[j][i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Sparse spread (d = 3, points of sparsely populated cells), by output tiles:
// one block per 4 x 4 x 4 tile of grid cells and 16 RHS computes
//   G[cell][r] = sum over the sparse points p whose window reaches the tile
//                of wx(p, x) wy(p, y) wz(p, z) V[p][r]
// as a matrix product D[16 cells of a z layer][16 RHS] += A[cells][4 points]
// B[4 points][RHS] per wave (wave = z layer), with window values of zero for
// cells outside a point's 2m taps.  The points come from the NT^3 point tiles
// (4^3 base cells each) that can reach the tile, in rounds of 64.  Every grid
// value is written once, by one lane: no atomics, and the sum order is fixed.
// The grid holds the sum when the dense-cell blocks are added (the gather
// reads it).
template <typename real, int W>
__global__ __launch_bounds__(kBlock) void k_spread_sparse_mfma(const WinDev *__restrict__ wins,
                                                               const LineGroup *__restrict__ tiles, IoArgs io, int R)
{
    typedef typename MfmaT<real>::v4 v4;
    typedef typename MfmaT<real>::v2 v2;
    constexpr int NT = (W + 2) / 4 + 1;  // point tiles per dimension that reach an output tile
    constexpr int NT3 = NT * NT * NT;
    constexpr int PB = 64;               // points per round (16 K steps)
    __shared__ int pre[NT3 + 1];
    __shared__ int2 rng[NT3];
    __shared__ __align__(16) real pw[PB][3][4];  // window values at the tile's 4 cells per dimension
    __shared__ __align__(16) real pv[PB][16];
    const LineGroup g = tiles[blockIdx.x];
    const WinDev &w = wins[g.win];
    const int r0 = blockIdx.y * 16;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int q = lane >> 4, mrow = lane & 15;
    const int otx = (w.ext[0] + 3) >> 2, oty = (w.ext[1] + 3) >> 2;
    const int to[3] = {g.grp % otx, (g.grp / otx) % oty, g.grp / (otx * oty)};
    if (t < NT3) {
        const int tx = to[0] - (NT - 1) + t % NT, ty = to[1] - (NT - 1) + (t / NT) % NT,
                  tz = to[2] - (NT - 1) + t / (NT * NT);
        int2 r = make_int2(0, 0);
        if (tx >= 0 && ty >= 0 && tz >= 0 && tx < w.ntile[0] && ty < w.ntile[1] && tz < w.ntile[2])
            r = ld_int2(gbl(w.sp_rng) + ((int64_t)tz * w.ntile[1] + ty) * w.ntile[0] + tx);
        rng[t] = r;
    }
    __syncthreads();
    if (t == 0) {
        pre[0] = 0;
        for (int i = 0; i < NT3; ++i)
            pre[i + 1] = pre[i] + rng[i].y;
    }
    __syncthreads();
    const int total = pre[NT3];
    const gptr<const real> coords = gbl((const real *)w.coords);
    const ProbDev pio = get_prob_m(io, w.prob);
    const gptr<const real> Vp = gbl((const real *)pio.Vp);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    // staging: thread (pi = t / 4, k = t % 4) loads RHS 4k .. 4k + 3 of point pi
    // and, for k < 3, the point's window values along dimension k at the
    // tile's four cells
    const int pi = t >> 2, kq = t & 3;
    v4 acc[2];
    acc[0] = acc[1] = v4{real(0), real(0), real(0), real(0)};
    for (int p0 = 0; p0 < total; p0 += PB) {
        const int f = p0 + pi;
        real v[4] = {real(0), real(0), real(0), real(0)};
        real wk[4] = {real(0), real(0), real(0), real(0)};
        if (f < total) {
            int lo = 0, hi = NT3 - 1;  // last tile k with pre[k] <= f
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= f)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const int j = rng[lo].x + (f - pre[lo]);
            const int64_t orig = gbl(w.perm)[j];
            const gptr<const real> vr = Vp + orig * pio.ldvp + r0 + 4 * kq;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                v[i] = vr[i];
            if (kq < 3) {
                const real u = coords[(int64_t)kq * w.N + j];
                const int b = (int)floor(u) - w.m + 1;  // the point's first cell
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = 4 * to[kq] + i;
                    wk[i] = (unsigned)(c - b) < (unsigned)W ? kb_psi_m(u - (real)c, mm, kb, ie) : real(0);
                }
            }
        }
        // one 4-vector store per array: the lanes' stores are consecutive
        // (four scalar stores at a stride of four words conflict in the banks)
        *(v4 *)&pv[pi][4 * kq] = v4{r0 + 4 * kq < R ? v[0] : real(0), r0 + 4 * kq + 1 < R ? v[1] : real(0),
                                    r0 + 4 * kq + 2 < R ? v[2] : real(0), r0 + 4 * kq + 3 < R ? v[3] : real(0)};
        if (kq < 3)
            *(v4 *)&pw[pi][kq][0] = v4{wk[0], wk[1], wk[2], wk[3]};
        __syncthreads();
        const int np = min(PB, total - p0);
#pragma unroll
        for (int ks = 0; ks < PB / 4; ++ks) {
            if (4 * ks >= np)
                break;
            const int pk = 4 * ks + q;
            // A[cell mrow of layer `wave`][point pk], B[point pk][RHS mrow]
            const real a = pw[pk][0][mrow & 3] * pw[pk][1][mrow >> 2] * pw[pk][2][wave];
            acc[ks & 1] = mfma4(a, pv[pk][mrow], acc[ks & 1]);
        }
        __syncthreads();
    }
    const v4 sum = acc[0] + acc[1];
    const int r = r0 + mrow;
    if (r >= R)
        return;
    const gptr<real> G = gbl((real *)w.G);
    const int z = 4 * to[2] + wave;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int cell = out_row<real>(q, i);
        const int x = 4 * to[0] + (cell & 3), y = 4 * to[1] + (cell >> 2);
        if (x < w.ext[0] && y < w.ext[1] && z < w.ext[2])
            G[((int64_t)(r >> 1) * w.szG + ((int64_t)z * w.ext[1] + y) * w.ext[0] + x) * 2 + (r & 1)] = sum[i];
    }
}

void launch_spread_sparse_mfma(Engine &E, int R, IoArgs io, hipStream_t st)
{
    for (int wi = 0; wi < 2; ++wi) {
        if (!E.nsptiles[wi])
            continue;
        const dim3 grid(E.nsptiles[wi], (R + 15) / 16);
        if (E.precision == ADDK_FP32) {
            if (wi == 0)
                hipLaunchKernelGGL((k_spread_sparse_mfma<float, 8>), grid, dim3(kBlock), 0, st, E.d_wins,
                                   E.d_sptiles[wi], io, R);
            else
                hipLaunchKernelGGL((k_spread_sparse_mfma<float, 12>), grid, dim3(kBlock), 0, st, E.d_wins,
                                   E.d_sptiles[wi], io, R);
        } else {
            if (wi == 0)
                hipLaunchKernelGGL((k_spread_sparse_mfma<double, 8>), grid, dim3(kBlock), 0, st, E.d_wins,
                                   E.d_sptiles[wi], io, R);
            else
                hipLaunchKernelGGL((k_spread_sparse_mfma<double, 12>), grid, dim3(kBlock), 0, st, E.d_wins,
                                   E.d_sptiles[wi], io, R);
        }
    }
}

// ---------------------------------------------------------------------------
// Sum the per-item blocks into the spread grid.  A block owns a 4 x 4 x 4 tile
// of grid cells and 16 RHS; it visits, in a fixed order, every base cell whose
// (2m)^3 window block overlaps the tile and adds the overlapping part of each
// of its items' blocks.  Every grid value is written by exactly one thread, so
// no atomics are needed and the sum order is fixed.
template <typename real>
struct GatherTypes;
template <>
struct GatherTypes<float> {
    typedef f4 v4;
    typedef float2 v2;
    static constexpr int CB = 4;  // cells whose loads are in flight together
};
template <>
struct GatherTypes<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    typedef double2 v2;
    static constexpr int CB = 2;
};

template <int W, typename real>
__global__ __launch_bounds__(kBlock) void k_gather_blocks(const WinDev *__restrict__ wins,
                                                          const LineGroup *__restrict__ tiles,
                                                          const real *__restrict__ scratch, int R)
{
    typedef typename GatherTypes<real>::v4 f4;  // four RHS values
    typedef typename GatherTypes<real>::v2 r2;
    constexpr int CB = GatherTypes<real>::CB;
    constexpr int WW = W * W;
    __shared__ f4 red[3][64][4];
    __shared__ int2 cand[(W + 3) * (W + 3) * (W + 4)];  // base-cell map of the candidate region
    const LineGroup tg = tiles[blockIdx.x];
    const WinDev &w = wins[tg.win];
    const int rb = blockIdx.y;
    const int r0 = rb * 16;
    if (r0 >= R)
        return;
    const int nrb = gridDim.y;
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2];
    const int nt0 = (ex + 3) / 4, nt1 = (ey + 3) / 4;
    const int tx = tg.grp % nt0, ty = (tg.grp / nt0) % nt1, tz = tg.grp / (nt0 * nt1);
    // lane = grid cell of the tile (all 16 RHS); the four waves split the base cells
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gx = tx * 4 + (lane & 3), gy = ty * 4 + ((lane >> 2) & 3), gz = tz * 4 + (lane >> 4);
    const int nb0 = w.nbase[0], nb1 = w.nbase[1], nb2 = w.nbase[2];
    const gptr<const int2> map = gbl(w.dmap);
    f4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        acc[i] = f4{real(0), real(0), real(0), real(0)};
    // anchors: an item anchored at bz covers z cells bz .. bz + 2m - 2 + (nzc - 1)
    const int z0 = max(0, tz * 4 - W), z1 = min(nb2 - 1, tz * 4 + 3);
    const int y0 = max(0, ty * 4 - (W - 1)), y1 = min(nb1 - 1, ty * 4 + 3);
    const int x0 = max(0, tx * 4 - (W - 1)), x1 = min(nb0 - 1, tx * 4 + 3);
    const bool any = x1 >= x0 && y1 >= y0 && z1 >= z0;
    const int nx = any ? x1 - x0 + 1 : 0, ny = any ? y1 - y0 + 1 : 0, nz = any ? z1 - z0 + 1 : 0;
    // stage the base-cell map of the candidate region in LDS (coalesced rows)
    for (int idx = threadIdx.x; idx < nx * ny * nz; idx += kBlock) {
        const int dx = idx % nx, dy = (idx / nx) % ny, dz = idx / (nx * ny);
        cand[idx] = ld_int2(map + ((int64_t)(z0 + dz) * nb1 + y0 + dy) * nb0 + x0 + dx);
    }
    __syncthreads();
    // Per row of candidate cells, the cells holding items (a ballot over the
    // row) are taken CB at a time: the loads of all of them are issued before
    // any is added, so that a wave keeps CB cells' reads in flight.  The sum
    // order is the row order, as in a plain loop over the cells.
    const f4 zero4 = f4{real(0), real(0), real(0), real(0)};
    for (int dz = wave; dz < nz; dz += 4) {
        const int bz = z0 + dz, oz = gz - bz;
        for (int dy = 0; dy < ny; ++dy) {
            const int by = y0 + dy, oy = gy - by;
            const int2 *crow = cand + (dz * ny + dy) * nx;
            uint64_t live = __ballot(lane < nx && crow[lane < nx ? lane : 0].y != 0);
            while (live) {
                int2 its[CB];
                bool in[CB];
                gptr<const f4> src[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    const int dx = live ? __builtin_ctzll(live) : 0;
                    const bool valid = live != 0;
                    live &= live - 1;
                    its[k] = valid ? crow[dx] : int2{0, 0};
                    const int nzc = (its[k].y >> 16) + 1;
                    const int ox = gx - x0 - dx;
                    in[k] = valid && (unsigned)ox < (unsigned)W && (unsigned)oy < (unsigned)W &&
                            (unsigned)oz < (unsigned)(W + nzc - 1);
                    const int tap = in[k] ? (oz * W + oy) * W + ox : 0;
                    src[k] = (gptr<const f4>)(gbl(scratch) + (((int64_t)its[k].x * nrb + rb) * ((W + 1) * WW) + tap) * 16);
                }
                f4 v[CB][4];
#pragma unroll
                for (int k = 0; k < CB; ++k)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        v[k][j] = in[k] ? src[k][j] : zero4;
#pragma unroll
                for (int k = 0; k < CB; ++k) {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[j] += v[k][j];
                    // further items of a cell with more than one (rare)
                    const int cnt = its[k].y & 0xffff;
                    for (int i = 1; i < cnt; ++i) {
                        if (!in[k])
                            break;
                        const gptr<const f4> s2 = src[k] + (int64_t)i * nrb * ((W + 1) * WW) * 4;
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[j] += s2[j];
                    }
                }
            }
        }
    }
    // fixed-order reduction over the four waves
    if (wave > 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            red[wave - 1][lane][i] = acc[i];
    }
    __syncthreads();
    if (wave > 0)
        return;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            acc[i] += red[k][lane][i];
    if (gx >= ex || gy >= ey || gz >= ez)
        return;
    const gptr<real> G = gbl((real *)w.G);
    const int64_t c = ((int64_t)gz * ey + gy) * ex + gx;
    // all loads of the cell's 8 complex grid values first, then the stores
    r2 g[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        typedef real n2 __attribute__((ext_vector_type(2)));
        const n2 t2 = r0 + 2 * p < R ? *(gptr<const n2>)(G + ((int64_t)((r0 >> 1) + p) * w.szG + c) * 2) : n2{real(0), real(0)};
        g[p] = r2{t2.x, t2.y};
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int r = r0 + 2 * p;
        if (r < R)
            G[((int64_t)(r >> 1) * w.szG + c) * 2] = g[p].x + acc[(2 * p) >> 2][(2 * p) & 3];
        if (r + 1 < R)
            G[((int64_t)(r >> 1) * w.szG + c) * 2 + 1] = g[p].y + acc[(2 * p + 1) >> 2][(2 * p + 1) & 3];
    }
}

// One RHS: the same sum over blocks with one value per tap (the one-RHS
// scratch layout), into the real part of pair 0.
template <int W, typename real>
__global__ __launch_bounds__(kBlock) void k_gather_blocks_1(const WinDev *__restrict__ wins,
                                                            const LineGroup *__restrict__ tiles,
                                                            const real *__restrict__ scratch)
{
    constexpr int WW = W * W, CB = 8;
    __shared__ real red[3][64];
    __shared__ int2 cand[(W + 3) * (W + 3) * (W + 4)];
    const LineGroup tg = tiles[blockIdx.x];
    const WinDev &w = wins[tg.win];
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2];
    const int nt0 = (ex + 3) / 4, nt1 = (ey + 3) / 4;
    const int tx = tg.grp % nt0, ty = (tg.grp / nt0) % nt1, tz = tg.grp / (nt0 * nt1);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gx = tx * 4 + (lane & 3), gy = ty * 4 + ((lane >> 2) & 3), gz = tz * 4 + (lane >> 4);
    const int nb0 = w.nbase[0], nb1 = w.nbase[1], nb2 = w.nbase[2];
    const gptr<const int2> map = gbl(w.dmap);
    real acc = real(0);
    const int z0 = max(0, tz * 4 - W), z1 = min(nb2 - 1, tz * 4 + 3);
    const int y0 = max(0, ty * 4 - (W - 1)), y1 = min(nb1 - 1, ty * 4 + 3);
    const int x0 = max(0, tx * 4 - (W - 1)), x1 = min(nb0 - 1, tx * 4 + 3);
    const bool any = x1 >= x0 && y1 >= y0 && z1 >= z0;
    const int nx = any ? x1 - x0 + 1 : 0, ny = any ? y1 - y0 + 1 : 0, nz = any ? z1 - z0 + 1 : 0;
    for (int idx = threadIdx.x; idx < nx * ny * nz; idx += kBlock) {
        const int dx = idx % nx, dy = (idx / nx) % ny, dz = idx / (nx * ny);
        cand[idx] = ld_int2(map + ((int64_t)(z0 + dz) * nb1 + y0 + dy) * nb0 + x0 + dx);
    }
    __syncthreads();
    for (int dz = wave; dz < nz; dz += 4) {
        const int bz = z0 + dz, oz = gz - bz;
        for (int dy = 0; dy < ny; ++dy) {
            const int by = y0 + dy, oy = gy - by;
            const int2 *crow = cand + (dz * ny + dy) * nx;
            uint64_t live = __ballot(lane < nx && crow[lane < nx ? lane : 0].y != 0);
            while (live) {
                int2 its[CB];
                bool in[CB];
                gptr<const real> src[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    const int dx = live ? __builtin_ctzll(live) : 0;
                    const bool valid = live != 0;
                    live &= live - 1;
                    its[k] = valid ? crow[dx] : int2{0, 0};
                    const int nzc = (its[k].y >> 16) + 1;
                    const int ox = gx - x0 - dx;
                    in[k] = valid && (unsigned)ox < (unsigned)W && (unsigned)oy < (unsigned)W &&
                            (unsigned)oz < (unsigned)(W + nzc - 1);
                    const int tap = in[k] ? (oz * W + oy) * W + ox : 0;
                    src[k] = gbl(scratch) + (int64_t)its[k].x * ((W + 1) * WW) + tap;
                }
                real v[CB];
#pragma unroll
                for (int k = 0; k < CB; ++k)
                    v[k] = in[k] ? *src[k] : real(0);
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    acc += v[k];
                    const int cnt = its[k].y & 0xffff;  // further items of the cell (rare)
                    for (int i = 1; i < cnt; ++i) {
                        if (!in[k])
                            break;
                        acc += src[k][(int64_t)i * ((W + 1) * WW)];
                    }
                }
            }
        }
    }
    if (wave > 0)
        red[wave - 1][lane] = acc;
    __syncthreads();
    if (wave > 0)
        return;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        acc += red[k][lane];
    if (gx >= ex || gy >= ey || gz >= ez)
        return;
    const gptr<real> G = gbl((real *)w.G);
    const int64_t c = ((int64_t)gz * ey + gy) * ex + gx;
    G[c * 2] += acc;
}

// ---------------------------------------------------------------------------
// interp for the sparsely populated cells of one tile on the matrix cores: the
// tile's sub-grid (tile + window halo, x padded to 16) plays the role of the
// dense cell's window block; weights outside a point's support are zero.
// One pass (<= 64 GMAX points) of a sparse tile chunk on the tile's sub-grid.
template <typename real>
constexpr int tile_gmax() { return sizeof(real) == 4 ? 4 : 2; }  // point groups per wave and pass

template <typename real, int W, int NO, int NG>
__device__ __forceinline__ void interp_tile_pass(const WinDev &w, const Chunk &ch, int pass, int r0, int nr, int x0,
                                                 int y0, int z0, real (*slab)[NO][(3 + W) * 16][16], real *wy_lds)
{
    constexpr int SX = 16, SY = 3 + W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, mrow = lane & 15;
    typedef typename MfmaT<real>::v4 v4;
    const gptr<const real> coords = gbl((const real *)w.coords);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    real *wyl = wy_lds + wave * (tile_gmax<real>() * SY * 16);  // [g][oy][16 points]
    real wxq[NG][4], uz[NG];
    int lbz[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int p = pass + (wave + 4 * g) * 16 + mrow;
        const bool act = p < ch.count;
        const int j = ch.start + (act ? p : 0);
        const real ux = coords[j], uy = coords[w.N + j];
        uz[g] = coords[2 * w.N + j];
        const int lx = (int)floor(ux) - w.m + 1 - x0, ly = (int)floor(uy) - w.m + 1 - y0;
        lbz[g] = act ? (int)floor(uz[g]) - w.m + 1 - z0 : (1 << 20);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ox = 4 * t + q;
            wxq[g][t] =
                (act && (unsigned)(ox - lx) < (unsigned)W) ? kb_psi_m(ux - (real)(x0 + ox), mm, kb, ie) : real(0);
        }
#pragma unroll
        for (int t = 0; t < (SY + 3) / 4; ++t) {
            const int oy = 4 * t + q;
            if (oy < SY)
                wyl[(g * SY + oy) * 16 + mrow] =
                    ((unsigned)(oy - ly) < (unsigned)W) ? kb_psi_m(uy - (real)(y0 + oy), mm, kb, ie) : real(0);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    constexpr int NA = acc_rows<NO>();
    v4 acc[NA][NG];
#pragma unroll
    for (int o = 0; o < NA; ++o)
#pragma unroll
        for (int g = 0; g < NG; ++g)
            acc[o][g] = v4{real(0), real(0), real(0), real(0)};
    stream_slabs<real, SY, SX, 4, NG, NO, 1>(w, slab, r0, nr, x0, y0, z0, w.S[0], w.S[1], w.S[2], acc, wxq, wyl, uz,
                                              lbz, true);
    if (NO == 1)
#pragma unroll
        for (int g = 0; g < NG; ++g)
            acc[0][g] += acc[NA - 1][g];
    if (mrow >= nr)
        return;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const gptr<real> dst = gbl((real *)w.Yw) + (int64_t)o * w.N * w.Rcap + r0 + mrow;
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = pass + (wave + 4 * g) * 16 + out_row<real>(q, i);
                if (p < ch.count)
                    dst[(int64_t)gbl(w.perm)[ch.start + p] * w.Rcap] = acc[o][g][i];
            }
    }
}

// Sparse-tile interp on the matrix cores: the points of a tile chunk (any base
// cells of the tile) against the tile's (4 + 2m - 1)^3 sub-grid, taken as one
// super-cell with x padded to 16; weights outside a point's support are zero.
template <typename real, int W, int NO>
__global__ __launch_bounds__(kBlock, sizeof(real) == 4 ? 3 : 2) void k_interp_tile_mfma(const WinDev *__restrict__ wins,
                                                                                        const Chunk *__restrict__ chunks,
                                                                                        int R)
{
    // one slab buffer (46 KB of LDS with the y weights at 2m = 12, two outputs,
    // FP32) and at most 168 registers: three blocks per CU; FP64 takes passes
    // of 128 points (76 KB): two
    constexpr int GMAX = tile_gmax<real>();
    __shared__ __align__(16) real slab[1][NO][(3 + W) * 16][16];
    __shared__ __align__(16) real wy_lds[4 * GMAX * (3 + W) * 16];
    const Chunk ch = chunks[blockIdx.x];
    const WinDev &w = wins[ch.win];
    const int r0 = blockIdx.y * 16;
    if (r0 >= R)
        return;
    const int nr = min(16, R - r0);
    int tl = ch.tile;
    const int tx = tl % w.ntile[0];
    tl /= w.ntile[0];
    const int ty = tl % w.ntile[1];
    const int tz = tl / w.ntile[1];
    const int x0 = tx * w.tb[0], y0 = ty * w.tb[1], z0 = tz * w.tb[2];
    for (int pass = 0; pass < ch.count; pass += 64 * GMAX) {
        const int npass = min(64 * GMAX, ch.count - pass);
        const int ng = (((npass + 15) >> 4) + 3) >> 2;
        switch (ng) {
        case 1: interp_tile_pass<real, W, NO, 1>(w, ch, pass, r0, nr, x0, y0, z0, slab, wy_lds); break;
        case 2: interp_tile_pass<real, W, NO, 2>(w, ch, pass, r0, nr, x0, y0, z0, slab, wy_lds); break;
        case 3: interp_tile_pass<real, W, NO, GMAX < 3 ? GMAX : 3>(w, ch, pass, r0, nr, x0, y0, z0, slab, wy_lds); break;
        default: interp_tile_pass<real, W, NO, GMAX>(w, ch, pass, r0, nr, x0, y0, z0, slab, wy_lds); break;
        }
        __syncthreads();  // the next pass overwrites the slab buffers
    }
}

// ---------------------------------------------------------------------------
// launchers (FP32, d = 3, 2m in {8, 12}); return false when not applicable

bool launch_interp_mfma(Engine &E, int wi, int R, int nout, hipStream_t st)
{
    if (!E.ndense[3][wi])
        return false;
    dim3 grid(E.ndense[3][wi], (R + 15) / 16);
    const Chunk *items = E.d_dense[3][wi];
    if (E.precision == ADDK_FP64) {  // 16 RHS columns only (no one-RHS form)
        if (R == 1)
            return false;
        if (wi == 0 && nout == 1)
            hipLaunchKernelGGL((k_interp_mfma<double, 8, 1>), grid, dim3(kBlock), 0, st, E.d_wins, items, R);
        else if (wi == 0)
            hipLaunchKernelGGL((k_interp_mfma<double, 8, 2>), grid, dim3(kBlock), 0, st, E.d_wins, items, R);
        else if (nout == 1)
            hipLaunchKernelGGL((k_interp_mfma<double, 12, 1>), grid, dim3(kBlock), 0, st, E.d_wins, items, R);
        else
            hipLaunchKernelGGL((k_interp_mfma<double, 12, 2>), grid, dim3(kBlock), 0, st, E.d_wins, items, R);
        return true;
    }
    if (R == 1) {  // the z-slabs as columns
        if (wi == 0 && nout == 1)
            hipLaunchKernelGGL((k_interp_mfma_z1<8, 1>), grid, dim3(kBlock), 0, st, E.d_wins, items);
        else if (wi == 0)
            hipLaunchKernelGGL((k_interp_mfma_z1<8, 2>), grid, dim3(kBlock), 0, st, E.d_wins, items);
        else if (nout == 1)
            hipLaunchKernelGGL((k_interp_mfma_z1<12, 1>), grid, dim3(kBlock), 0, st, E.d_wins, items);
        else
            hipLaunchKernelGGL((k_interp_mfma_z1<12, 2>), grid, dim3(kBlock), 0, st, E.d_wins, items);
        return true;
    }
    if (wi == 0 && nout == 1)
        hipLaunchKernelGGL((k_interp_mfma<float, 8, 1>), grid, dim3(kBlock), 0, st, E.d_wins, items, R);
    else if (wi == 0)
        hipLaunchKernelGGL((k_interp_mfma<float, 8, 2>), grid, dim3(kBlock), 0, st, E.d_wins, items, R);
    else if (nout == 1)
        hipLaunchKernelGGL((k_interp_mfma<float, 12, 1>), grid, dim3(kBlock), 0, st, E.d_wins, items, R);
    else
        hipLaunchKernelGGL((k_interp_mfma<float, 12, 2>), grid, dim3(kBlock), 0, st, E.d_wins, items, R);
    return true;
}

bool launch_spread_mfma(Engine &E, int wi, int R, IoArgs io, hipStream_t st)
{
    if (!E.ndense_sp[3][wi] || !E.scratch[wi])
        return false;
    if (E.precision == ADDK_FP64 && R == 1)  // FP64 takes 16 RHS columns
        return false;
    const Chunk *items = E.d_dense_sp[3][wi];
    const int n2 = E.ndense_sp2[wi], n = E.ndense_sp[3][wi];
    const int ry = (R + 15) / 16;
    // the two-cell items (2m + 1 slabs) lead the list, then the single-cell ones
    auto run = [&](auto kern2, auto kern1, int ms, auto *scratch) {
        if (n2)
            hipLaunchKernelGGL(kern2, dim3(n2, ry, ms), dim3(kBlock), 0, st, E.d_wins, items, 0, io, R, scratch);
        if (n > n2)
            hipLaunchKernelGGL(kern1, dim3(n - n2, ry, ms), dim3(kBlock), 0, st, E.d_wins, items, n2, io, R, scratch);
    };
    if (E.precision == ADDK_FP64) {
        // the M tiles split over blocks: 2m = 8: 4 over two; 2m = 12: 9 over three
        // (measured on the large workload: 14.4 ms with two blocks, 11.0 with
        // three, 15.7 with five)
        double *sd = (double *)E.scratch[wi];
        if (wi == 0)
            run(k_spread_mfma<double, 8, false, 2, true>, k_spread_mfma<double, 8, false, 2, false>, 2, sd);
        else
            run(k_spread_mfma<double, 12, false, 3, true>, k_spread_mfma<double, 12, false, 3, false>, 3, sd);
        return true;
    }
    float *sf = (float *)E.scratch[wi];
    const bool split = (E.knobs & ADDK_KNOB_SPREAD_SPLIT) != 0;
    if (wi == 0 && R == 1)
        run(k_spread_mfma<float, 8, true, 1, false>, k_spread_mfma<float, 8, true, 1, false>, 1, sf);
    else if (wi == 0 && split)
        run(k_spread_mfma<float, 8, false, 2, true>, k_spread_mfma<float, 8, false, 2, false>, 2, sf);
    else if (wi == 0)
        run(k_spread_mfma<float, 8, false, 1, true>, k_spread_mfma<float, 8, false, 1, false>, 1, sf);
    else if (R == 1)
        run(k_spread_mfma<float, 12, true, 1, false>, k_spread_mfma<float, 12, true, 1, false>, 1, sf);
    else if (split)
        run(k_spread_mfma<float, 12, false, 3, true>, k_spread_mfma<float, 12, false, 3, false>, 3, sf);
    else
        run(k_spread_mfma<float, 12, false, 1, true>, k_spread_mfma<float, 12, false, 1, false>, 1, sf);
    return true;
}

void launch_gather_blocks(Engine &E, int wi, int R, hipStream_t st)
{
    if (!E.ngtiles[wi])
        return;
    dim3 grid(E.ngtiles[wi], (R + 15) / 16);
    const float *sf = (const float *)E.scratch[wi];
    const double *sd = (const double *)E.scratch[wi];
    const bool fp64 = E.precision == ADDK_FP64;
    if (R == 1) {  // one value per tap
        if (wi == 0 && !fp64)
            hipLaunchKernelGGL((k_gather_blocks_1<8, float>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_gtiles[wi], sf);
        else if (wi == 0)
            hipLaunchKernelGGL((k_gather_blocks_1<8, double>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_gtiles[wi], sd);
        else if (!fp64)
            hipLaunchKernelGGL((k_gather_blocks_1<12, float>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_gtiles[wi], sf);
        else
            hipLaunchKernelGGL((k_gather_blocks_1<12, double>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_gtiles[wi],
                               sd);
        return;
    }
    if (wi == 0 && !fp64)
        hipLaunchKernelGGL((k_gather_blocks<8, float>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_gtiles[wi], sf, R);
    else if (wi == 0)
        hipLaunchKernelGGL((k_gather_blocks<8, double>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_gtiles[wi], sd, R);
    else if (!fp64)
        hipLaunchKernelGGL((k_gather_blocks<12, float>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_gtiles[wi], sf, R);
    else
        hipLaunchKernelGGL((k_gather_blocks<12, double>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_gtiles[wi], sd, R);
}

}  // namespace addk

namespace addk {

bool launch_interp_tile_mfma(Engine &E, int R, int nout, hipStream_t st)
{
    const int W = E.tile_w[3];
    if (!E.nchunks_i[3] || (W != 8 && W != 12))
        return false;
    dim3 grid(E.nchunks_i[3], (R + 15) / 16);
    const Chunk *ch = E.d_chunks_i[3];
    auto go = [&](auto k81, auto k82, auto k121, auto k122) {
        auto k = W == 8 ? (nout == 1 ? k81 : k82) : (nout == 1 ? k121 : k122);
        hipLaunchKernelGGL(k, grid, dim3(kBlock), 0, st, E.d_wins, ch, R);
    };
    if (E.precision == ADDK_FP32)
        go(k_interp_tile_mfma<float, 8, 1>, k_interp_tile_mfma<float, 8, 2>, k_interp_tile_mfma<float, 12, 1>,
           k_interp_tile_mfma<float, 12, 2>);
    else
        go(k_interp_tile_mfma<double, 8, 1>, k_interp_tile_mfma<double, 8, 2>, k_interp_tile_mfma<double, 12, 1>,
           k_interp_tile_mfma<double, 12, 2>);
    return true;
}

}  // namespace addk
