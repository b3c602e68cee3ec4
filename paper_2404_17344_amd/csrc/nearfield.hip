// Near-field part of the corrected Matern-1/2 products (ADDK_NEAR_FIELD).
//
// The Fourier part of such a plan uses the multipliers of the regularised
// kernel, which differs from the true kernel only for pairs closer than eps:
// there, the kernel's cusp at r = 0 is replaced by an even polynomial p.  This
// file adds the difference back by summing K_NE(r) = kappa(r) - p(r) over the
// pairs with r < eps, for kappa = e^{-r/l} and for the derivative kernel
// (r/l) e^{-r/l} with its own polynomial (eq. (4) restricted to close pairs).
//
// Layout.  The plan sorted every window's points by tile (a box of base cells
// of the spreading grid); the points of tile t are the range
// [tile_off[t], tile_off[t+1]) of the sorted order, coordinates in grid units.
// A block is one wave: it takes up to 64 consecutive sorted points (targets,
// one per lane, all in one tile), bounds them by a box, and walks the rows of
// tiles (along x, contiguous in the sorted order) that come within eps of the
// box, each row cut to the ball's chord.  The sources of a row are staged in
// LDS 64 at a time (coordinates and the point-major right-hand sides) and read
// by all lanes as broadcasts.  Each target is owned by one lane, which adds its
// sums to the window's product buffer after the interpolation has written it,
// in a fixed order.
//
// With one right-hand side and targets = sources (the plain K v and dK/dl v
// products), k_near_sym evaluates each close pair once instead of twice: the
// kernels are symmetric, so K_ij serves both i's sum and j's.  Its sums are
// added atomically, so their rounding order varies from call to call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "addk_internal.h"

namespace addk {

namespace {

__device__ __forceinline__ ProbDev nf_prob(const IoArgs &io, int p) { return io.table ? io.table[p] : io.single; }

__device__ __forceinline__ float nf_exp(float x) { return __expf(x); }
__device__ __forceinline__ double nf_exp(double x) { return exp(x); }
// FP32: the hardware square root (about 1 ulp), without the rounding fix-up
__device__ __forceinline__ float nf_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double nf_sqrt(double x) { return sqrt(x); }

template <typename real>
__device__ __forceinline__ real horner(const real *a, real t2)
{
    real p = a[kNearQ];
#pragma unroll
    for (int k = kNearQ - 1; k >= 0; --k)
        p = p * t2 + a[k];
    return p;
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// DOT = false: Yw[o][i][r0 + r] += sum_j K_NE,o(ij) Vp[j][r0 + r], o < NO
//               (o = 0 kernel, o = 1 derivative kernel).
// DOT = true:  partial[(blockIdx.x * gridDim.y + blockIdx.y) * 2 + o] =
//               sum over the block's targets i of sum_j K_NE,o(ij) <Vt_i, Vp_j>
//               (RHS r0 .. r0 + RT - 1), Vt_i read from the caller's V.
constexpr int kNearBlock = 64;  // one wave per block

template <typename real, int D, int RT, int NO, bool DOT>
__global__ __launch_bounds__(kNearBlock) void k_near(const WinDev *__restrict__ wins, const Chunk *__restrict__ chunks,
                                                 IoArgs io, int R, const double *__restrict__ Vt, int64_t ldvt,
                                                 double *__restrict__ partial)
{
    __shared__ real sc[kNearBlock][4];                // source coordinates (grid units); [3] = value if RT = 1
    __shared__ real sv[RT > 1 ? kNearBlock : 1][RT];  // source right-hand sides (RT > 1)
    const Chunk ch = chunks[blockIdx.x];
    const WinDev &w = wins[ch.win];
    const int r0 = blockIdx.y * RT;
    const int t = threadIdx.x;
    const ProbDev pio = nf_prob(io, w.prob);
    const gptr<const real> coords = gbl((const real *)w.coords);
    const bool own = t < ch.count;
    const int64_t i = ch.start + (own ? t : 0);
    real u[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
        u[a] = coords[(int64_t)a * w.N + i];
    // box of the wave's targets
    float bmin[3] = {0.f, 0.f, 0.f}, bmax[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        bmin[a] = wave_min(own ? (float)u[a] : 3.0e38f);
        bmax[a] = wave_max(own ? (float)u[a] : -3.0e38f);
    }
    const real eps2 = (real)w.nf_eps2, ie2 = (real)w.nf_inv_eps2, hl = (real)w.nf_hl;
    const bool m32 = w.nf == 2;  // Matern-3/2: (1 + a r) e^{-a r} and (a r)^2 e^{-a r}, with rl = a r
    const float eg = sqrtf((float)w.nf_eps2) + 1e-3f;  // slightly generous for the box tests
    real pa[kNearQ + 1], pd[kNearQ + 1];
#pragma unroll
    for (int k = 0; k <= kNearQ; ++k) {
        pa[k] = (real)w.nf_a[k];
        pd[k] = (real)w.nf_ad[k];
    }
    // tile range per axis: the coordinates are relative to the grid box, and the
    // base cell of a point u is floor(u) - m + 1
    int t0[3] = {0, 0, 0}, t1[3] = {0, 0, 0};
    bool none = false;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int nb = w.ext[a] - w.W + 1;
        const int b0 = max(0, (int)floorf(bmin[a] - eg) - w.m + 1);
        const int b1 = min(nb - 1, (int)floorf(bmax[a] + eg) - w.m + 1);
        none = none || b1 < b0;
        t0[a] = b0 / w.tb[a];
        t1[a] = min(w.ntile[a] - 1, b1 / w.tb[a]);
    }
    // targets' values (DOT) and accumulators
    real vt[RT];
    real acc[NO][RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        vt[r] = real(0);
#pragma unroll
        for (int o = 0; o < NO; ++o)
            acc[o][r] = real(0);
    }
    real sk = real(0), sd = real(0);
    if (DOT && own) {
        const int orig = gbl(w.perm)[i];
#pragma unroll
        for (int r = 0; r < RT; ++r)
            vt[r] = r0 + r < R ? (real)Vt[orig + (int64_t)(r0 + r) * ldvt] : real(0);
    }
    const gptr<const real> vp = gbl((const real *)pio.Vp);
    const gptr<const int32_t> toff = gbl(w.tile_off);
    if (!none) {
        for (int tz = t0[2]; tz <= t1[2]; ++tz) {
            for (int ty = t0[1]; ty <= t1[1]; ++ty) {
                // distance of the target box to the row's box in y and z
                float g2 = 0.f;
                if (D > 1) {
                    const float rlo = (float)(ty * w.tb[1] + w.m - 1);
                    const float rhi = rlo + (float)w.tb[1];
                    const float g = fmaxf(0.f, fmaxf(rlo - bmax[1], bmin[1] - rhi));
                    g2 += g * g;
                }
                if (D > 2) {
                    const float rlo = (float)(tz * w.tb[2] + w.m - 1);
                    const float rhi = rlo + (float)w.tb[2];
                    const float g = fmaxf(0.f, fmaxf(rlo - bmax[2], bmin[2] - rhi));
                    g2 += g * g;
                }
                if (g2 >= eg * eg)
                    continue;
                // x tiles within the ball's chord at this row's y/z distance
                const float rx = sqrtf(eg * eg - g2);
                const int nbx = w.ext[0] - w.W + 1;
                const int bx0 = max(0, (int)floorf(bmin[0] - rx) - w.m + 1);
                const int bx1 = min(nbx - 1, (int)floorf(bmax[0] + rx) - w.m + 1);
                if (bx1 < bx0)
                    continue;
                const int tx0 = bx0 / w.tb[0], tx1 = min(w.ntile[0] - 1, bx1 / w.tb[0]);
                const int64_t trow = ((int64_t)tz * w.ntile[1] + ty) * w.ntile[0];
                const int s = toff[trow + tx0], e = toff[trow + tx1 + 1];
                for (int b = s; b < e; b += kNearBlock) {
                    __syncthreads();
                    const int j = b + t;
                    if (j < e) {
#pragma unroll
                        for (int a = 0; a < D; ++a)
                            sc[t][a] = coords[(int64_t)a * w.N + j];
                        const int64_t orig = gbl(w.perm)[j];
                        if (RT == 1)
                            sc[t][3] = vp[orig * pio.ldvp + r0];
                        else
#pragma unroll
                            for (int r = 0; r < RT; ++r)
                                sv[RT > 1 ? t : 0][r] = vp[orig * pio.ldvp + r0 + r];
                    } else {  // padding up to a multiple of 4: far away, never within eps
#pragma unroll
                        for (int a = 0; a < 4; ++a)
                            sc[t][a] = real(a < D ? 1.0e6 : 0.0);
                    }
                    __syncthreads();
                    const int nsrc4 = __builtin_amdgcn_readfirstlane((min(kNearBlock, e - b) + 3) & ~3);
                    for (int j4 = 0; j4 < nsrc4; j4 += 4) {
                        // four sources per step: their loads issue together
                        real s4[4][4];
#pragma unroll
                        for (int k = 0; k < 4; ++k)
#pragma unroll
                            for (int a = 0; a < 4; ++a)
                                s4[k][a] = sc[j4 + k][a];
                        real d2v[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            real d2 = real(0);
#pragma unroll
                            for (int a = 0; a < D; ++a) {
                                const real dx = u[a] - s4[k][a];
                                d2 += dx * dx;
                            }
                            d2v[k] = d2;
                        }
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int jj = j4 + k;
                            const real d2 = d2v[k];
                            const real *s4k = s4[k];
                            if (d2 < eps2) {
                                const real rl = nf_sqrt(d2) * hl;
                                const real ex = nf_exp(-rl);
                                const real t2 = d2 * ie2;
                                const real kn = (m32 ? real(1) + rl : real(1)) * ex - horner(pa, t2);
                                const real kd =
                                    (NO > 1 || DOT) ? rl * (m32 ? rl : real(1)) * ex - horner(pd, t2) : real(0);
                                if (DOT) {
                                    real dot = real(0);
#pragma unroll
                                    for (int r = 0; r < RT; ++r)
                                        dot += vt[r] * (RT == 1 ? s4k[3] : sv[RT > 1 ? jj : 0][r]);
                                    sk += kn * dot;
                                    sd += kd * dot;
                                } else {
#pragma unroll
                                    for (int r = 0; r < RT; ++r) {
                                        const real v = RT == 1 ? s4k[3] : sv[RT > 1 ? jj : 0][r];
                                        acc[0][r] += kn * v;
                                        if (NO > 1)
                                            acc[NO > 1 ? 1 : 0][r] += kd * v;
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    if (DOT) {
        double a0 = own ? (double)sk : 0.0, a1 = own ? (double)sd : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o, 64);
            a1 += __shfl_xor(a1, o, 64);
        }
        if (t == 0) {
            double *pp = partial + ((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * 2;
            pp[0] = a0;
            pp[1] = a1;
        }
        return;
    }
    if (!own)
        return;
    const int64_t orig = gbl(w.perm)[i];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const gptr<real> dst = gbl((real *)w.Yw) + ((int64_t)o * w.N + orig) * w.Rcap + r0;
#pragma unroll
        for (int r = 0; r < RT; ++r)
            if (r0 + r < R)
                dst[r] += acc[o][r];
    }
}

// One right-hand side, targets = sources: each close pair once.  A block's
// targets are the sorted points [cs, ce).  Sources inside that range are taken
// as ordered pairs (the lane of target i adds K_ij v_j), sources at positions
// >= ce symmetrically (the lane also adds K_ij v_i to source j's sum), and
// sources before cs are left to the blocks that own them, which meet this
// block's points as their symmetric partners: every ordered pair is counted
// once.  A staged batch of n sources is walked diagonally, lane t pairing with
// source (t + k) mod n at step k, so that the lanes of one step add to distinct
// source sums in LDS (FP64 LDS adds; lanes t and t + n share a sum when n < 64).  Both sides' sums go by atomic adds to the window's
// buffer of sums by sorted position, where one wave's adds fall on consecutive
// words (their rounding order is not fixed); k_near_scatter then adds that
// buffer to the product buffer (after the interpolation) and clears it.
__device__ __forceinline__ float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// KT: 1 every window Matern-1/2, 2 every window Matern-3/2 (the kernel's form is
// then fixed at compile time: the close-pair loop is bound by instruction issue),
// 0 mixed (chosen per window).
template <typename real, int D, int NO, int KT>
__global__ __launch_bounds__(kNearBlock) void k_near_sym(const WinDev *__restrict__ wins,
                                                         const Chunk *__restrict__ chunks, IoArgs io)
{
    __shared__ __align__(16) real sc[kNearBlock][4];  // x, y, z (grid units), value
    __shared__ double sa[kNearBlock][NO];             // the staged sources' symmetric sums
    const Chunk ch = chunks[blockIdx.x];
    const WinDev &w = wins[ch.win];
    const int t = threadIdx.x;
    const ProbDev pio = nf_prob(io, w.prob);
    const gptr<const real> coords = gbl((const real *)w.coords);
    const gptr<const real> vp = gbl((const real *)pio.Vp);
    const bool own = t < ch.count;
    const int64_t i = ch.start + (own ? t : 0);
    const int cs = ch.start, ce = ch.start + ch.count;
    real u[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
        u[a] = coords[(int64_t)a * w.N + i];
    const int64_t oi = gbl(w.perm)[i];
    const real vi = own ? vp[oi * pio.ldvp] : real(0);
    float bmin[3] = {0.f, 0.f, 0.f}, bmax[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        bmin[a] = uniform(wave_min(own ? (float)u[a] : 3.0e38f));
        bmax[a] = uniform(wave_max(own ? (float)u[a] : -3.0e38f));
    }
    const real eps2 = (real)w.nf_eps2, ie2 = (real)w.nf_inv_eps2, hl = (real)w.nf_hl;
    // Matern-3/2: (1 + a r) e^{-a r} and (a r)^2 e^{-a r}, with rl = a r
    const bool m32 = KT == 0 ? w.nf == 2 : KT == 2;
    const float eg = sqrtf((float)w.nf_eps2) + 1e-3f;
    real pa[kNearQ + 1], pd[kNearQ + 1];
#pragma unroll
    for (int k = 0; k <= kNearQ; ++k) {
        pa[k] = (real)w.nf_a[k];
        pd[k] = (real)w.nf_ad[k];
    }
    int t0[3] = {0, 0, 0}, t1[3] = {0, 0, 0};
    bool none = false;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int nb = w.ext[a] - w.W + 1;
        const int b0 = max(0, (int)floorf(bmin[a] - eg) - w.m + 1);
        const int b1 = min(nb - 1, (int)floorf(bmax[a] + eg) - w.m + 1);
        none = none || b1 < b0;
        t0[a] = b0 / w.tb[a];
        t1[a] = min(w.ntile[a] - 1, b1 / w.tb[a]);
    }
    real acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o)
        acc[o] = real(0);
    const gptr<double> ys = gbl(w.nf_ys);
    // the sources [b, e), at most 64 of them
    auto batch = [&](int b, int e, bool sym) {
        const int n = __builtin_amdgcn_readfirstlane(e - b);
        __syncthreads();
        if (t < n) {
            const int64_t j = b + t;
#pragma unroll
            for (int a = 0; a < D; ++a)
                sc[t][a] = coords[(int64_t)a * w.N + j];
            sc[t][3] = vp[(int64_t)gbl(w.perm)[j] * pio.ldvp];
#pragma unroll
            for (int o = 0; o < NO; ++o)
                sa[t][o] = 0.0;
        }
        __syncthreads();
        int idx = t % n;
        for (int k = 0; k < n; k += 4) {
            real s4[4][4];
            int id4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                id4[q] = idx;
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    s4[q][a] = sc[idx][a];
                idx = idx + 1 == n ? 0 : idx + 1;
            }
            real d2v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                real d2 = real(0);
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    const real dx = u[a] - s4[q][a];
                    d2 += dx * dx;
                }
                d2v[q] = d2;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool hit = own && k + q < n && d2v[q] < eps2;
                real kn = real(0), kd = real(0);
                if (hit) {
                    const real rl = nf_sqrt(d2v[q]) * hl;
                    const real ex = nf_exp(-rl);
                    const real t2 = d2v[q] * ie2;
                    kn = (m32 ? real(1) + rl : real(1)) * ex - horner(pa, t2);
                    acc[0] += kn * s4[q][3];
                    if (NO > 1) {
                        kd = rl * (m32 ? rl : real(1)) * ex - horner(pd, t2);
                        acc[NO > 1 ? 1 : 0] += kd * s4[q][3];
                    }
                }
                if (sym && hit) {
                    atomicAdd(&sa[id4[q]][0], (double)(kn * vi));
                    if (NO > 1)
                        atomicAdd(&sa[id4[q]][NO > 1 ? 1 : 0], (double)(kd * vi));
                }
            }
        }
        if (sym) {
            __syncthreads();
            if (t < n) {
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    const double c = sa[t][o];
                    if (c != 0.0)
                        __hip_atomic_fetch_add(ys + o * w.N + b + t, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    };
    const gptr<const int32_t> toff = gbl(w.tile_off);
    if (!none) {
        for (int tz = t0[2]; tz <= t1[2]; ++tz) {
            for (int ty = t0[1]; ty <= t1[1]; ++ty) {
                float g2 = 0.f;
                if (D > 1) {
                    const float rlo = (float)(ty * w.tb[1] + w.m - 1);
                    const float g = fmaxf(0.f, fmaxf(rlo - bmax[1], bmin[1] - (rlo + (float)w.tb[1])));
                    g2 += g * g;
                }
                if (D > 2) {
                    const float rlo = (float)(tz * w.tb[2] + w.m - 1);
                    const float g = fmaxf(0.f, fmaxf(rlo - bmax[2], bmin[2] - (rlo + (float)w.tb[2])));
                    g2 += g * g;
                }
                if (g2 >= eg * eg)
                    continue;
                const float rx = sqrtf(eg * eg - g2);
                const int nbx = w.ext[0] - w.W + 1;
                const int bx0 = max(0, (int)floorf(bmin[0] - rx) - w.m + 1);
                const int bx1 = min(nbx - 1, (int)floorf(bmax[0] + rx) - w.m + 1);
                if (bx1 < bx0)
                    continue;
                const int tx0 = bx0 / w.tb[0], tx1 = min(w.ntile[0] - 1, bx1 / w.tb[0]);
                const int64_t trow = ((int64_t)tz * w.ntile[1] + ty) * w.ntile[0];
                const int s = toff[trow + tx0], e = toff[trow + tx1 + 1];
                if (e <= cs)  // all before the block's points
                    continue;
                for (int b = max(s, cs); b < min(e, ce); b += kNearBlock)  // the block's own points
                    batch(b, min(b + kNearBlock, min(e, ce)), false);
                for (int b = max(s, ce); b < e; b += kNearBlock)  // the points after them
                    batch(b, min(b + kNearBlock, e), true);
            }
        }
    }
    if (own) {
#pragma unroll
        for (int o = 0; o < NO; ++o)
            __hip_atomic_fetch_add(ys + o * w.N + i, (double)acc[o], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Yw[o][perm[j]][0] += ys[o][j], then ys[o][j] = 0, for the near-field windows
// (blockIdx.y = window).
template <typename real>
__global__ void k_near_scatter(const WinDev *__restrict__ wins, int nout)
{
    const WinDev &w = wins[blockIdx.y];
    if (!w.nf)
        return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= w.N)
        return;
    const int64_t oj = gbl(w.perm)[j];
    for (int o = 0; o < nout; ++o) {
        const gptr<double> src = gbl(w.nf_ys) + o * w.N + j;
        gbl((real *)w.Yw)[(o * w.N + oj) * w.Rcap] += (real)*src;
        *src = 0.0;
    }
}

// Per window: grad_ell += der_scale * sum of the derivative partials,
// grad_sig += dsig * sum of the kernel partials (fixed order).
__global__ void k_near_dot_finish(const WinDev *__restrict__ wins, int win, const double *partial, int nblk,
                                  double *grad_ell, double *grad_sig)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    double sk = 0.0, sd = 0.0;
    for (int b = 0; b < nblk; ++b) {
        sk += partial[2 * b];
        sd += partial[2 * b + 1];
    }
    const WinDev &w = wins[win];
    if (grad_ell)
        grad_ell[0] += w.der_scale * sd;
    if (grad_sig)
        grad_sig[0] += w.dsig * sk;
}

int near_rt(int R) { return R == 1 ? 1 : (R <= 4 ? 4 : 16); }

template <typename real, int D, int RT, bool DOT>
void launch_near_rt(Engine &E, int R, int nout, IoArgs io, const double *Vt, int64_t ldvt, double *partial,
                    hipStream_t st)
{
    dim3 grid(E.nnear[D], (R + RT - 1) / RT);
    if (DOT)
        hipLaunchKernelGGL((k_near<real, D, RT, 2, true>), grid, dim3(kNearBlock), 0, st, E.d_wins, E.d_near[D], io,
                           R, Vt, ldvt, partial);
    else if (nout > 1)
        hipLaunchKernelGGL((k_near<real, D, RT, 2, false>), grid, dim3(kNearBlock), 0, st, E.d_wins, E.d_near[D], io,
                           R, Vt, ldvt, partial);
    else
        hipLaunchKernelGGL((k_near<real, D, RT, 1, false>), grid, dim3(kNearBlock), 0, st, E.d_wins, E.d_near[D], io,
                           R, Vt, ldvt, partial);
}

template <typename real, int D, bool DOT>
void launch_near_d(Engine &E, int R, int nout, IoArgs io, const double *Vt, int64_t ldvt, double *partial,
                   hipStream_t st)
{
    switch (near_rt(R)) {
    case 1: launch_near_rt<real, D, 1, DOT>(E, R, nout, io, Vt, ldvt, partial, st); break;
    case 4: launch_near_rt<real, D, 4, DOT>(E, R, nout, io, Vt, ldvt, partial, st); break;
    default: launch_near_rt<real, D, 16, DOT>(E, R, nout, io, Vt, ldvt, partial, st); break;
    }
}

template <bool DOT>
void launch_near_all(Engine &E, int R, int nout, IoArgs io, const double *Vt, int64_t ldvt, double *const *part,
                     hipStream_t st)
{
    for (int d = 1; d <= 3; ++d) {
        if (!E.nnear[d])
            continue;
        double *p = part ? part[d] : nullptr;
        if (E.precision == ADDK_FP32) {
            if (d == 1) launch_near_d<float, 1, DOT>(E, R, nout, io, Vt, ldvt, p, st);
            if (d == 2) launch_near_d<float, 2, DOT>(E, R, nout, io, Vt, ldvt, p, st);
            if (d == 3) launch_near_d<float, 3, DOT>(E, R, nout, io, Vt, ldvt, p, st);
        } else {
            if (d == 1) launch_near_d<double, 1, DOT>(E, R, nout, io, Vt, ldvt, p, st);
            if (d == 2) launch_near_d<double, 2, DOT>(E, R, nout, io, Vt, ldvt, p, st);
            if (d == 3) launch_near_d<double, 3, DOT>(E, R, nout, io, Vt, ldvt, p, st);
        }
    }
}

template <typename real, int D, int KT>
void launch_near_sym_k(Engine &E, int nout, IoArgs io, hipStream_t st)
{
    const dim3 grid(E.nnear[D]);
    if (nout > 1)
        hipLaunchKernelGGL((k_near_sym<real, D, 2, KT>), grid, dim3(kNearBlock), 0, st, E.d_wins, E.d_near[D], io);
    else
        hipLaunchKernelGGL((k_near_sym<real, D, 1, KT>), grid, dim3(kNearBlock), 0, st, E.d_wins, E.d_near[D], io);
}

template <typename real, int D>
void launch_near_sym_d(Engine &E, int nout, IoArgs io, hipStream_t st)
{
    // the near-field windows' kernel form: all Matern-1/2 (1), all Matern-3/2 (2), or both (0)
    bool m12 = false, m32 = false;
    for (const WinDev &w : E.wdev) {
        m12 = m12 || w.nf == 1;
        m32 = m32 || w.nf == 2;
    }
    if (m12 && !m32)
        launch_near_sym_k<real, D, 1>(E, nout, io, st);
    else if (m32 && !m12)
        launch_near_sym_k<real, D, 2>(E, nout, io, st);
    else
        launch_near_sym_k<real, D, 0>(E, nout, io, st);
}

template <typename real>
void launch_near_sym(Engine &E, int nout, IoArgs io, hipStream_t st)
{
    int64_t nmax = 0;
    for (const WinDev &w : E.wdev)
        nmax = std::max<int64_t>(nmax, w.nf ? w.N : 0);
    if (E.nnear[1])
        launch_near_sym_d<real, 1>(E, nout, io, st);
    if (E.nnear[2])
        launch_near_sym_d<real, 2>(E, nout, io, st);
    if (E.nnear[3])
        launch_near_sym_d<real, 3>(E, nout, io, st);
    if (nmax > 0)
        hipLaunchKernelGGL(k_near_scatter<real>, dim3((unsigned)((nmax + 255) / 256), (unsigned)E.wdev.size()),
                           dim3(256), 0, st, E.d_wins, nout);
}

}  // namespace

void launch_near(Engine &E, int R, int nout, IoArgs io, hipStream_t st)
{
    if (nout < 1)
        return;
    bool square = true;  // every near-field window's targets are its sources
    for (const Plan *pl : E.plans)
        square = square && !pl->rect;
    if (R == 1 && square) {
        if (E.precision == ADDK_FP32)
            launch_near_sym<float>(E, std::min(nout, 2), io, st);
        else
            launch_near_sym<double>(E, std::min(nout, 2), io, st);
        return;
    }
    launch_near_all<false>(E, R, std::min(nout, 2), io, nullptr, 0, nullptr, st);
}

addk_status engine_near_dot(Engine &E, int R, IoArgs io, const double *V, int64_t ldv, double *grad_ell,
                            double *grad_sig, hipStream_t st)
{
    const int ny = (R + near_rt(R) - 1) / near_rt(R);
    int64_t need = 0;
    for (int d = 1; d <= 3; ++d)
        need += (int64_t)E.nnear[d] * ny * 2;
    if (need == 0)
        return ADDK_OK;
    if (E.near_part_cap < need) {
        if (E.d_near_part)
            (void)hipFree(E.d_near_part);
        E.d_near_part = nullptr;
        E.near_part_cap = 0;
        hipError_t e = hipMalloc(&E.d_near_part, need * sizeof(double));
        if (e != hipSuccess)
            return hip_fail(e, "near-field partials");
        E.near_part_cap = need;
    }
    double *part[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t off = 0;
    for (int d = 1; d <= 3; ++d) {
        part[d] = E.d_near_part + off;
        off += (int64_t)E.nnear[d] * ny * 2;
    }
    if (!io.table) {
        io.single.Vp = E.vpack;
        io.single.ldvp = E.vpack_ld;
    }
    launch_near_all<true>(E, R, 2, io, V, ldv, part, st);
    for (int wi = 0; wi < (int)E.wdev.size(); ++wi) {
        const WinDev &w = E.wdev[wi];
        const int2 rg = E.near_rng[wi];
        if (!w.nf || rg.y <= rg.x)
            continue;
        const double *p = part[w.d] + (int64_t)rg.x * ny * 2;
        hipLaunchKernelGGL(k_near_dot_finish, dim3(1), dim3(64), 0, st, E.d_wins, wi, p, (rg.y - rg.x) * ny,
                           grad_ell ? grad_ell + E.wlocal[wi] : nullptr, grad_sig ? grad_sig + E.wlocal[wi] : nullptr);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "near-field launch");
    return ADDK_OK;
}

}  // namespace addk
