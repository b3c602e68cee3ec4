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

__device__ __forceinline__ float kb_psi_f(float z, float m, float b, float inv_e2bm)
{
    float s2 = m * m - z * z;
    s2 = s2 > 0.f ? s2 : 0.f;
    float s = __builtin_sqrtf(s2);
    s = s > 1e-6f ? s : 1e-6f;
    const float l2e = 1.4426950408889634f;
    return m * (__builtin_amdgcn_exp2f(b * (s - m) * l2e) - __builtin_amdgcn_exp2f(-b * (s + m) * l2e)) * inv_e2bm *
           __builtin_amdgcn_rcpf(s);
}

__device__ __forceinline__ void unpack_cell_m(int packed, int &bx, int &by, int &bz)
{
    bx = packed & 1023;
    by = (packed >> 10) & 1023;
    bz = packed >> 20;
}

__device__ __forceinline__ ProbDev get_prob_m(const IoArgs &io, int p) { return io.table ? io.table[p] : io.single; }

// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void k_interp_mfma(const WinDev *__restrict__ wins, const Chunk *__restrict__ items,
                                                        int R)
{
    constexpr int WW = W * W;
    constexpr int NT = W / 4;  // K steps per x row
    __shared__ __align__(16) float slab[2][WW][16];

    const Chunk it = items[blockIdx.x];
    const WinDev &w = wins[it.win];
    const int r0 = blockIdx.y * 16;
    if (r0 >= R)
        return;
    const int o = blockIdx.z;
    const int nr = min(16, R - r0);
    int bx, by, bz;
    unpack_cell_m(it.tile, bx, by, bz);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, mrow = lane & 15;
    const float *coords = (const float *)w.coords;
    const float mm = (float)w.m, kb = (float)w.b, ie = (float)w.inv_e2bm;

    // window values of the lane's point (A row) in each of the wave's four groups
    float wxq[4][NT], wy[4][W], uz[4];
    bool gact[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int gbase = wave * 64 + g * 16;
        gact[g] = gbase < it.count;
        const int p = gbase + mrow;
        const bool act = p < it.count;
        const int j = it.start + (act ? p : 0);
        const float ux = coords[j], uy = coords[w.N + j];
        uz[g] = coords[2 * w.N + j];
#pragma unroll
        for (int t = 0; t < NT; ++t)
            wxq[g][t] = act ? kb_psi_f(ux - (float)(bx + 4 * t + q), mm, kb, ie) : 0.f;
#pragma unroll
        for (int k = 0; k < W; ++k)
            wy[g][k] = kb_psi_f(uy - (float)(by + k), mm, kb, ie);
    }

    const float *H = (const float *)w.H;
    const int ex = w.ext[0], ey = w.ext[1];
    const int p0 = r0 >> 1;
    const int np = (nr + 1) >> 1;
    constexpr int SL = (8 * WW + kBlock - 1) / kBlock;  // complex values per thread per slab
    float2 pre[SL];
    // load slab oz (8 complex grids x 2m x 2m cells) into registers
    auto load = [&](int oz) {
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int idx = threadIdx.x + k * kBlock;
            const int pi = idx / WW, c = idx - pi * WW;
            float2 v = {0.f, 0.f};
            if (idx < 8 * WW && pi < np) {
                const int ox = c % W, oy = c / W;
                const int64_t off =
                    ((int64_t)(o * w.npair_cap + p0 + pi) * w.szH + ((int64_t)(bz + oz) * ey + by + oy) * ex + bx + ox) *
                    2;
                v = *(const float2 *)(H + off);
            }
            pre[k] = v;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int idx = threadIdx.x + k * kBlock;
            if (idx < 8 * WW) {
                const int pi = idx / WW, c = idx - pi * WW;
                slab[buf][c][2 * pi] = pre[k].x;
                slab[buf][c][2 * pi + 1] = (2 * pi + 1 < nr) ? pre[k].y : 0.f;
            }
        }
    };

    f4 acc[4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
        acc[g] = f4{0.f, 0.f, 0.f, 0.f};

    load(0);
    store(0);
    __syncthreads();
    for (int oz = 0; oz < W; ++oz) {
        if (oz + 1 < W)
            load(oz + 1);  // in flight during this slab's products
        const int cur = oz & 1;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (!gact[g])
                continue;
            const float wz = kb_psi_f(uz[g] - (float)(bz + oz), mm, kb, ie);
#pragma unroll
            for (int oy = 0; oy < W; ++oy) {
                const float wyz = wy[g][oy] * wz;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const float a = wyz * wxq[g][t];
                    const float b = slab[cur][oy * W + 4 * t + q][mrow];
                    acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[g], 0, 0, 0);
                }
            }
        }
        if (oz + 1 < W)
            store((oz + 1) & 1);
        __syncthreads();
    }

    if (mrow >= nr)
        return;
    double *dst = w.Yw + ((int64_t)o * w.Rcap + r0 + mrow) * w.N;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = wave * 64 + g * 16 + 4 * q + i;
            if (p < it.count)
                dst[w.perm[it.start + p]] = (double)acc[g][i];
        }
    }
}

// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kBlock) void k_spread_mfma(const WinDev *__restrict__ wins, const Chunk *__restrict__ items,
                                                        IoArgs io, int R)
{
    constexpr int WW = W * W;
    constexpr int MT = WW / 16;  // M tiles per z-slab
    constexpr int SPW = W / 4;   // z-slabs per wave (4 waves)
    constexpr int PB = 32;       // points per round (8 K steps)
    constexpr int FL = WW * 17;  // per-wave flush tile [tap][16 RHS + 1 pad]
    struct Round {
        float pxy[PB][WW];
        float pw[PB][3][W];
        float pv[PB][16];
    };
    constexpr int RB_BYTES = 2 * (int)sizeof(Round);
    constexpr int FL_BYTES = 4 * FL * (int)sizeof(float);
    __shared__ __align__(16) unsigned char lds[RB_BYTES > FL_BYTES ? RB_BYTES : FL_BYTES];
    Round *rd = (Round *)lds;

    const Chunk it = items[blockIdx.x];
    const WinDev &w = wins[it.win];
    const int r0 = blockIdx.y * 16;
    if (r0 >= R)
        return;
    int bx, by, bz;
    unpack_cell_m(it.tile, bx, by, bz);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, mrow = lane & 15;
    const float *coords = (const float *)w.coords;
    const ProbDev pio = get_prob_m(io, w.prob);
    const float mm = (float)w.m, kb = (float)w.b, ie = (float)w.inv_e2bm;
    const int t = threadIdx.x;

    // prefetch registers: thread t < 3*PB holds one coordinate, every thread two RHS values
    float pc = 0.f;
    float pvv[2] = {0.f, 0.f};
    auto load = [&](int p0) {
        const int np = min(PB, it.count - p0);
        if (t < 3 * PB) {
            const int p = t / 3, dd = t - 3 * (t / 3);
            pc = p < np ? coords[dd * w.N + it.start + p0 + p] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int e = t + k * kBlock;  // e < PB * 16
            const int p = e >> 4, i = e & 15;
            const int r = r0 + i;
            pvv[k] = (p < np && r < R) ? (float)pio.V[w.perm[it.start + p0 + p] + (int64_t)r * pio.ldv] : 0.f;
        }
    };
    auto store_raw = [&](Round &d, int p0) {
        const int np = min(PB, it.count - p0);
        if (t < 3 * PB) {
            const int p = t / 3, dd = t - 3 * (t / 3);
            const int b0 = dd == 0 ? bx : (dd == 1 ? by : bz);
#pragma unroll
            for (int o = 0; o < W; ++o)
                d.pw[p][dd][o] = p < np ? kb_psi_f(pc - (float)(b0 + o), mm, kb, ie) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int e = t + k * kBlock;
            d.pv[e >> 4][e & 15] = pvv[k];
        }
    };
    auto products = [&](Round &d) {
        for (int e = t; e < PB * WW; e += kBlock) {
            const int p = e / WW, c = e - p * WW;
            d.pxy[p][c] = d.pw[p][0][c % W] * d.pw[p][1][c / W];
        }
    };

    f4 acc[SPW][MT];
#pragma unroll
    for (int s = 0; s < SPW; ++s)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            acc[s][mt] = f4{0.f, 0.f, 0.f, 0.f};

    load(0);
    store_raw(rd[0], 0);
    __syncthreads();
    products(rd[0]);
    __syncthreads();
    int buf = 0;
    for (int p0 = 0; p0 < it.count; p0 += PB) {
        const bool more = p0 + PB < it.count;
        if (more)
            load(p0 + PB);  // in flight during this round's products
        Round &cr = rd[buf];
#pragma unroll
        for (int ks = 0; ks < PB / 4; ++ks) {
            const int pk = 4 * ks + q;
            const float b = cr.pv[pk][mrow];
#pragma unroll
            for (int s = 0; s < SPW; ++s) {
                const float wz = cr.pw[pk][2][wave + 4 * s];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const float a = cr.pxy[pk][mt * 16 + mrow] * wz;
                    acc[s][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[s][mt], 0, 0, 0);
                }
            }
        }
        if (more) {
            store_raw(rd[buf ^ 1], p0 + PB);
            __syncthreads();
            products(rd[buf ^ 1]);
        }
        __syncthreads();
        buf ^= 1;
    }

    // flush: transpose each slab through LDS so that consecutive lanes add to
    // consecutive grid cells of one complex grid
    float *fl = (float *)lds + wave * FL;
    float *G = (float *)w.G;
    const int ex = w.ext[0], ey = w.ext[1];
    const int nr = min(16, R - r0);
    const int np2 = (nr + 1) >> 1;
    const int pbase = r0 >> 1;
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
        const int oz = wave + 4 * s;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                fl[(mt * 16 + 4 * q + i) * 17 + mrow] = acc[s][mt][i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int idx = lane; idx < np2 * WW; idx += 64) {
            const int pi = idx / WW, tap = idx - pi * WW;
            const int ox = tap % W, oy = tap / W;
            const int64_t cell = ((int64_t)(bz + oz) * ey + by + oy) * ex + bx + ox;
            float *gp = G + ((int64_t)(pbase + pi) * w.szG + cell) * 2;
            unsafeAtomicAdd(gp, fl[tap * 17 + 2 * pi]);
            if (2 * pi + 1 < nr)
                unsafeAtomicAdd(gp + 1, fl[tap * 17 + 2 * pi + 1]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---------------------------------------------------------------------------
// launchers (FP32, d = 3, 2m in {8, 12}); return false when not applicable

bool launch_interp_mfma(Engine &E, int wi, int R, int nout, hipStream_t st)
{
    if (E.precision != ADDK_FP32 || !E.ndense[3][wi])
        return false;
    dim3 grid(E.ndense[3][wi], (R + 15) / 16, nout);
    if (wi == 0)
        hipLaunchKernelGGL(k_interp_mfma<8>, grid, dim3(kBlock), 0, st, E.d_wins, E.d_dense[3][wi], R);
    else
        hipLaunchKernelGGL(k_interp_mfma<12>, grid, dim3(kBlock), 0, st, E.d_wins, E.d_dense[3][wi], R);
    return true;
}

bool launch_spread_mfma(Engine &E, int wi, int R, IoArgs io, hipStream_t st)
{
    if (E.precision != ADDK_FP32 || !E.ndense[3][wi])
        return false;
    dim3 grid(E.ndense[3][wi], (R + 15) / 16);
    if (wi == 0)
        hipLaunchKernelGGL(k_spread_mfma<8>, grid, dim3(kBlock), 0, st, E.d_wins, E.d_dense[3][wi], io, R);
    else
        hipLaunchKernelGGL(k_spread_mfma<12>, grid, dim3(kBlock), 0, st, E.d_wins, E.d_dense[3][wi], io, R);
    return true;
}

}  // namespace addk
