// Stage kernels of the NFFT-based fast summation (eqs. (4)-(6)) for gfx950 and
// the engine that launches them over work lists spanning many windows.
//
//   spread  : g_l = sum_j v_j prod_i psi(u_ji - l_i)           (adjoint NFFT gridding)
//   FFT     : forward line FFTs, keeping the modes k in [-n/2, n/2]
//   multiply: h_k = B_k g_k  (B = periodised kernel coefficients / window transform^2)
//   IFFT    : inverse line FFTs back to the grid box
//   interp  : y_j = sum_l h_l prod_i psi(u_ji - l_i)            (NFFT gathering)
//   combine : FP64 window sum y = sum_w sigma_w^2 y_w and derivative scalings
//
// Spreading and interpolation work on tiles of base cells: a block owns one
// chunk of <= kChunk points of one tile and keeps the tile's sub-grid
// (tile + window halo) for a block of RHS in LDS.  Sixteen lanes cooperate on
// one point: lane g handles the taps g, g+16, ... so that the 16 LDS addresses
// of one instruction are distinct.  Spreading accumulates with LDS atomics and
// flushes the sub-grid to the global grid with float atomics; interpolation
// stages the sub-grid with plain loads and reduces the 16 partial sums with
// cross-lane shuffles.  The FFT keeps a group of lines in LDS and runs a
// radix-2 Stockham transform; a fused pass does forward transform, the
// multiplication for one or two multipliers and the inverse transform
// without leaving LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "addk_internal.h"

namespace addk {

template <typename real>
struct cpx {
    real x, y;
};

// a complex value in device memory (one 2-vector access)
template <typename real>
__device__ __forceinline__ cpx<real> ldc(gptr<const cpx<real>> p)
{
    typedef real n2 __attribute__((ext_vector_type(2)));
    const n2 v = *(gptr<const n2>)p;
    return {v.x, v.y};
}
template <typename real>
__device__ __forceinline__ void stc(gptr<cpx<real>> p, cpx<real> v)
{
    typedef real n2 __attribute__((ext_vector_type(2)));
    *(gptr<n2>)p = n2{v.x, v.y};
}

template <typename real>
__device__ __forceinline__ cpx<real> cadd(cpx<real> a, cpx<real> b) { return {a.x + b.x, a.y + b.y}; }
template <typename real>
__device__ __forceinline__ cpx<real> csub(cpx<real> a, cpx<real> b) { return {a.x - b.x, a.y - b.y}; }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void lds_add(float *p, float v) { __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ void lds_add(double *p, double v) { __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ void gbl_add(gptr<float> p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gbl_add(gptr<double> p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Normalised Kaiser-Bessel window in grid units (psi(0) = 1):
//   psi(z) = (m / sinh(b m)) sinh(b s) / s,  s = sqrt(m^2 - z^2),  |z| <= m,
// written as m e^{-b z^2/(s+m)} (1 - e^{-2bs}) / ((1 - e^{-2bm}) s): finite in
// FP32, with a small (hence accurate) exponent where psi is large.
template <typename real>
__device__ __forceinline__ real kb_psi(real z, real m, real b, real inv_e2bm)
{
    const real z2 = z * z;
    real s2 = m * m - z2;
    s2 = s2 > real(1e-12) ? s2 : real(1e-12);
    const real s = sqrt(s2);
    return m * exp(-b * z2 / (s + m)) * (real(1) - exp(real(-2) * b * s)) * inv_e2bm / s;
}

// First tap of a point at grid coordinate u: taps are base .. base + 2m - 1.
template <typename real>
__device__ __forceinline__ int base_cell(real u, int m)
{
    return (int)floor(u) - m + 1;
}

__device__ __forceinline__ ProbDev get_prob(const IoArgs &io, int p) { return io.table ? io.table[p] : io.single; }

// V (FP64, column-major, caller order) -> Vp (engine precision, point-major,
// RHS padded with zeros to ldvp), through an LDS tile of 64 points x 16 RHS so
// that both sides are accessed contiguously.  The spread kernels then read one
// contiguous run per point.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_pack_v(IoArgs io, int R)
{
    __shared__ double tile[16][65];
    const ProbDev p = get_prob(io, blockIdx.y);
    const gptr<real> vp = gbl((real *)p.Vp);
    const int t = threadIdx.x, il = t & 63, rq = t >> 6;
    for (int64_t i0 = blockIdx.x * (int64_t)64; i0 < p.N; i0 += (int64_t)gridDim.x * 64) {
        for (int r0 = 0; r0 < p.ldvp; r0 += 16) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int r = r0 + rq + 4 * k;
                const int64_t i = i0 + il;
                tile[rq + 4 * k][il] = (i < p.nsrc && r < R) ? gbl(p.V)[i + (int64_t)r * p.ldv] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = t + kBlock * k, pl = e >> 4, rr = e & 15;
                const int64_t i = i0 + pl;
                if (i < p.N)
                    vp[i * p.ldvp + r0 + rr] = (real)tile[rr][pl];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// zero the spread grids of every window (npair grids each)

template <typename real>
__global__ __launch_bounds__(kBlock) void k_zero_grids(const WinDev *__restrict__ wins, int npair)
{
    const WinDev &w = wins[blockIdx.y];
    const gptr<real> G = gbl((real *)w.G);
    const int64_t n = 2 * w.szG * (int64_t)npair;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        G[i] = real(0);
}

// ---------------------------------------------------------------------------
// spreading

template <typename real, int D, int RB>
__global__ __launch_bounds__(kBlock) void k_spread(const WinDev *__restrict__ wins, const Chunk *__restrict__ chunks,
                                                   IoArgs io, int R)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Chunk ch = chunks[blockIdx.x];
    const WinDev &w = wins[ch.win];
    const int r0 = blockIdx.y * RB;
    if (r0 >= R)
        return;
    const int nr = min(RB, R - r0);
    const int S0 = w.S[0], S1 = D > 1 ? w.S[1] : 1, S2 = D > 2 ? w.S[2] : 1;
    const int vol = S0 * S1 * S2;
    real *sub = (real *)smem_raw;
    real *wv = sub + RB * vol;  // [16 groups][D][kMaxW]

    int t = ch.tile;
    const int tx = t % w.ntile[0];
    t /= w.ntile[0];
    const int ty = t % w.ntile[1];
    const int tz = t / w.ntile[1];
    const int ox0 = tx * w.tb[0], oy0 = ty * w.tb[1], oz0 = tz * w.tb[2];

    for (int i = threadIdx.x; i < RB * vol; i += kBlock)
        sub[i] = real(0);
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, g = lane & 15;
    real *mywv = wv + (wave * 4 + grp) * (D * kMaxW);
    const gptr<const real> coords = gbl((const real *)w.coords);
    const ProbDev pio = get_prob(io, w.prob);
    const int W = w.W, m = w.m;
    const real mm = (real)m, bb = (real)w.b, ie = (real)w.inv_e2bm;

    for (int base = wave * 4; base < ch.count; base += 16) {
        const int p = base + grp;
        const bool act = p < ch.count;
        const int j = ch.start + (act ? p : 0);
        real u[3];
        int bc[3];
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            u[dd] = coords[dd * w.N + j];
            bc[dd] = base_cell(u[dd], m);
        }
        for (int q = g; q < D * W; q += kGroup) {
            const int dd = q / W, o = q - dd * W;
            const real uu = dd == 0 ? u[0] : (dd == 1 ? u[D > 1 ? 1 : 0] : u[D > 2 ? 2 : 0]);
            const int b0 = dd == 0 ? bc[0] : (dd == 1 ? bc[D > 1 ? 1 : 0] : bc[D > 2 ? 2 : 0]);
            mywv[dd * kMaxW + o] = kb_psi(uu - (real)(b0 + o), mm, bb, ie);
        }
        real v[RB];
        const int orig = gbl(w.perm)[j];
#pragma unroll
        for (int i = 0; i < RB; ++i)
            v[i] = (act && i < nr) ? gbl((const real *)pio.Vp)[orig * pio.ldvp + r0 + i] : real(0);
        wave_sync();
        if (act) {
            const int lx = bc[0] - ox0;
            const int ly = D > 1 ? bc[D > 1 ? 1 : 0] - oy0 : 0;
            const int lz = D > 2 ? bc[D > 2 ? 2 : 0] - oz0 : 0;
            if (D == 3) {
                for (int pq = g; pq < W * W; pq += kGroup) {
                    const int ox = pq % W, oy = pq / W;
                    const real wxy = mywv[ox] * mywv[kMaxW + oy];
                    int cell = (lz * S1 + ly + oy) * S0 + lx + ox;
                    for (int oz = 0; oz < W; ++oz, cell += S0 * S1) {
                        const real wt = wxy * mywv[2 * kMaxW + oz];
#pragma unroll
                        for (int i = 0; i < RB; ++i)
                            lds_add(&sub[i * vol + cell], wt * v[i]);
                    }
                }
            } else if (D == 2) {
                for (int pq = g; pq < W * W; pq += kGroup) {
                    const int ox = pq % W, oy = pq / W;
                    const real wt = mywv[ox] * mywv[kMaxW + oy];
                    const int cell = (ly + oy) * S0 + lx + ox;
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        lds_add(&sub[i * vol + cell], wt * v[i]);
                }
            } else {
                for (int ox = g; ox < W; ox += kGroup) {
                    const real wt = mywv[ox];
                    const int cell = lx + ox;
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        lds_add(&sub[i * vol + cell], wt * v[i]);
                }
            }
        }
        wave_sync();
    }
    __syncthreads();

    // flush the sub-grid: RHS r goes to component r % 2 of complex grid r / 2
    const gptr<real> G = gbl((real *)w.G);
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2];
    for (int idx = threadIdx.x; idx < nr * vol; idx += kBlock) {
        const int i = idx / vol, c = idx - i * vol;
        const real val = sub[i * vol + c];
        if (val == real(0))
            continue;
        const int cx = c % S0, cy = (c / S0) % S1, cz = c / (S0 * S1);
        const int gx = ox0 + cx, gy = oy0 + cy, gz = oz0 + cz;
        if (gx >= ex || gy >= ey || gz >= ez)
            continue;
        const int r = r0 + i;
        const int64_t off = ((int64_t)(r >> 1) * w.szG + ((int64_t)gz * ey + gy) * ex + gx) * 2 + (r & 1);
        gbl_add(&G[off], val);
    }
}

// ---------------------------------------------------------------------------
// interpolation

template <typename real, int D, int RB>
__global__ __launch_bounds__(kBlock) void k_interp(const WinDev *__restrict__ wins, const Chunk *__restrict__ chunks,
                                                   int R)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Chunk ch = chunks[blockIdx.x];
    const WinDev &w = wins[ch.win];
    const int r0 = blockIdx.y * RB;
    if (r0 >= R)
        return;
    const int o = blockIdx.z;
    const int nr = min(RB, R - r0);
    const int S0 = w.S[0], S1 = D > 1 ? w.S[1] : 1, S2 = D > 2 ? w.S[2] : 1;
    const int vol = S0 * S1 * S2;
    real *sub = (real *)smem_raw;
    real *wv = sub + RB * vol;

    int t = ch.tile;
    const int tx = t % w.ntile[0];
    t /= w.ntile[0];
    const int ty = t % w.ntile[1];
    const int tz = t / w.ntile[1];
    const int ox0 = tx * w.tb[0], oy0 = ty * w.tb[1], oz0 = tz * w.tb[2];

    // stage the sub-grid (both components of each complex grid at once)
    const gptr<const real> H = gbl((const real *)w.H);
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2];
    const int np = (nr + 1) >> 1;
    const int p0 = r0 >> 1;
    for (int idx = threadIdx.x; idx < np * vol; idx += kBlock) {
        const int pi = idx / vol, c = idx - pi * vol;
        const int cx = c % S0, cy = (c / S0) % S1, cz = c / (S0 * S1);
        const int gx = ox0 + cx, gy = oy0 + cy, gz = oz0 + cz;
        real re = 0, im = 0;
        if (gx < ex && gy < ey && gz < ez) {
            const int64_t off =
                ((int64_t)(o * w.npair_cap + p0 + pi) * w.szH + ((int64_t)gz * ey + gy) * ex + gx) * 2;
            re = H[off];
            im = H[off + 1];
        }
        sub[(2 * pi) * vol + c] = re;
        if (2 * pi + 1 < RB)
            sub[(2 * pi + 1) * vol + c] = im;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane >> 4, g = lane & 15;
    real *mywv = wv + (wave * 4 + grp) * (D * kMaxW);
    const gptr<const real> coords = gbl((const real *)w.coords);
    const int W = w.W, m = w.m;
    const real mm = (real)m, bb = (real)w.b, ie = (real)w.inv_e2bm;
    const gptr<real> dst = gbl((real *)w.Yw) + (int64_t)o * w.N * w.Rcap + r0;

    for (int base = wave * 4; base < ch.count; base += 16) {
        const int p = base + grp;
        const bool act = p < ch.count;
        const int j = ch.start + (act ? p : 0);
        real u[3];
        int bc[3];
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            u[dd] = coords[dd * w.N + j];
            bc[dd] = base_cell(u[dd], m);
        }
        for (int q = g; q < D * W; q += kGroup) {
            const int dd = q / W, oo = q - dd * W;
            const real uu = dd == 0 ? u[0] : (dd == 1 ? u[D > 1 ? 1 : 0] : u[D > 2 ? 2 : 0]);
            const int b0 = dd == 0 ? bc[0] : (dd == 1 ? bc[D > 1 ? 1 : 0] : bc[D > 2 ? 2 : 0]);
            mywv[dd * kMaxW + oo] = kb_psi(uu - (real)(b0 + oo), mm, bb, ie);
        }
        wave_sync();
        real acc[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i)
            acc[i] = real(0);
        if (act) {
            const int lx = bc[0] - ox0;
            const int ly = D > 1 ? bc[D > 1 ? 1 : 0] - oy0 : 0;
            const int lz = D > 2 ? bc[D > 2 ? 2 : 0] - oz0 : 0;
            if (D == 3) {
                for (int pq = g; pq < W * W; pq += kGroup) {
                    const int ox = pq % W, oy = pq / W;
                    const real wxy = mywv[ox] * mywv[kMaxW + oy];
                    int cell = (lz * S1 + ly + oy) * S0 + lx + ox;
                    for (int oz = 0; oz < W; ++oz, cell += S0 * S1) {
                        const real wt = wxy * mywv[2 * kMaxW + oz];
#pragma unroll
                        for (int i = 0; i < RB; ++i)
                            acc[i] += wt * sub[i * vol + cell];
                    }
                }
            } else if (D == 2) {
                for (int pq = g; pq < W * W; pq += kGroup) {
                    const int ox = pq % W, oy = pq / W;
                    const real wt = mywv[ox] * mywv[kMaxW + oy];
                    const int cell = (ly + oy) * S0 + lx + ox;
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i] += wt * sub[i * vol + cell];
                }
            } else {
                for (int ox = g; ox < W; ox += kGroup) {
                    const real wt = mywv[ox];
                    const int cell = lx + ox;
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i] += wt * sub[i * vol + cell];
                }
            }
        }
        // reduce the 16 partial sums of the group
#pragma unroll
        for (int i = 0; i < RB; ++i) {
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1)
                acc[i] += __shfl_xor(acc[i], off, kGroup);
        }
        if (act) {
            const int orig = gbl(w.perm)[j];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if (i == g && i < nr)
                    dst[(int64_t)orig * w.Rcap + i] = acc[i];
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// line FFTs in LDS (radix-2 Stockham), pruned to the box and to the kept modes

// Each wave transforms its own L / 4 lines, so the passes only need the
// wave to be in step (no block barrier between passes).  Stockham passes of
// radix 4 (a 4-point DFT in registers per butterfly), then one radix-2 pass
// when log2(nos) is odd.  tw holds e^{2 pi i q / nos} for q < nos / 2; the
// other half of the circle is its negative.
template <typename real>
__device__ cpx<real> *fft_lines(cpx<real> *a, cpx<real> *b, const cpx<real> *tw, int nos, int L, real sign)
{
    const int h = nos >> 1, qn = nos >> 2;
    const int lane = threadIdx.x & 63, lpw = L / (kBlock / 64), l0 = (threadIdx.x >> 6) * lpw;
    auto twid = [&](int q) -> cpx<real> {  // e^{sign 2 pi i q / nos}, 0 <= q < nos
        const cpx<real> c = q < h ? tw[q] : cpx<real>{-tw[q - h].x, -tw[q - h].y};
        return {c.x, sign * c.y};
    };
    auto cmul = [](cpx<real> x, cpx<real> c) -> cpx<real> { return {x.x * c.x - x.y * c.y, x.x * c.y + x.y * c.x}; };
    int Ns = 1;
    for (; Ns * 4 <= nos; Ns <<= 2) {
        for (int t = lane; t < lpw * qn; t += 64) {
            const int l = l0 + t / qn, j = t - (t / qn) * qn;
            const int k = j & (Ns - 1);
            const int step = k * (qn / Ns);  // twiddle index unit of this butterfly
            cpx<real> x0 = a[l * nos + j], x1 = a[l * nos + j + qn], x2 = a[l * nos + j + 2 * qn],
                      x3 = a[l * nos + j + 3 * qn];
            if (Ns > 1) {
                x1 = cmul(x1, twid(step));
                x2 = cmul(x2, twid(2 * step));
                x3 = cmul(x3, twid(3 * step));
            }
            const cpx<real> a0 = cadd(x0, x2), a1 = csub(x0, x2), a2 = cadd(x1, x3), a3 = csub(x1, x3);
            const cpx<real> ja3 = {-sign * a3.y, sign * a3.x};  // (sign i) a3
            const int idx = ((j - k) << 2) + k;
            b[l * nos + idx] = cadd(a0, a2);
            b[l * nos + idx + Ns] = cadd(a1, ja3);
            b[l * nos + idx + 2 * Ns] = csub(a0, a2);
            b[l * nos + idx + 3 * Ns] = csub(a1, ja3);
        }
        wave_sync();
        cpx<real> *s = a;
        a = b;
        b = s;
    }
    for (; Ns < nos; Ns <<= 1) {  // at most one radix-2 pass
        for (int t = lane; t < lpw * h; t += 64) {
            const int l = l0 + t / h, j = t - (t / h) * h;
            const cpx<real> x0 = a[l * nos + j], x1 = a[l * nos + j + h];
            const int k = j & (Ns - 1);
            const cpx<real> c = tw[k * (h / Ns)];
            const real sy = sign * c.y;
            const cpx<real> y1 = {x1.x * c.x - x1.y * sy, x1.x * sy + x1.y * c.x};
            const int idx = ((j - k) << 1) + k;
            b[l * nos + idx] = cadd(x0, y1);
            b[l * nos + idx + Ns] = csub(x0, y1);
        }
        wave_sync();
        cpx<real> *s = a;
        a = b;
        b = s;
    }
    return a;
}

struct FftCall {
    int nos_lds;    // line length the LDS buffers are laid out for (the engine's largest grid)
    int npair;
    int nout;       // fused: number of multipliers / inverse outputs (0, 1, 2)
    int modes_sel;  // fused: 0 none, 1 store forward modes into Vm, 2 into Gm
};

// Array dims (x, y, z) of the stage's input and output and their pointers.
template <typename real>
struct StageArrays {
    gptr<const cpx<real>> in;
    gptr<cpx<real>> out;
    int din[3], dout[3];
};

template <typename real, int AXIS, int MODE>
__device__ __forceinline__ void select_arrays(const WinDev &w, int pair, int o, StageArrays<real> &sa)
{
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2], n1 = w.n1;
    const int64_t po = (int64_t)o * w.npair_cap + pair;
    auto set = [](int *dd, int a, int b, int c) { dd[0] = a; dd[1] = b; dd[2] = c; };
    if (MODE == 0 && AXIS == 0) {  // G -> A1
        sa.in = gbl((const cpx<real> *)w.G) + pair * w.szG;
        sa.out = gbl((cpx<real> *)w.A1) + pair * w.szA1;
        set(sa.din, ex, ey, ez);
        set(sa.dout, n1, ey, ez);
    } else if (MODE == 0 && AXIS == 1) {  // A1 -> A2
        sa.in = gbl((const cpx<real> *)w.A1) + pair * w.szA1;
        sa.out = gbl((cpx<real> *)w.A2) + pair * w.szA2;
        set(sa.din, n1, ey, ez);
        set(sa.dout, n1, n1, ez);
    } else if (MODE == 2 && AXIS == 2) {  // A2 -> A3[o]
        sa.in = gbl((const cpx<real> *)w.A2) + pair * w.szA2;
        sa.out = gbl((cpx<real> *)w.A3) + po * w.szA3;
        set(sa.din, n1, n1, ez);
        set(sa.dout, n1, n1, ez);
    } else if (MODE == 2 && AXIS == 1) {  // d = 2: A1 -> A3[o]
        sa.in = gbl((const cpx<real> *)w.A1) + pair * w.szA1;
        sa.out = gbl((cpx<real> *)w.A3) + po * w.szA3;
        set(sa.din, n1, ey, 1);
        set(sa.dout, n1, ey, 1);
    } else if (MODE == 2 && AXIS == 0) {  // d = 1: G -> H[o]
        sa.in = gbl((const cpx<real> *)w.G) + pair * w.szG;
        sa.out = gbl((cpx<real> *)w.H) + po * w.szH;
        set(sa.din, ex, 1, 1);
        set(sa.dout, ex, 1, 1);
    } else if (MODE == 1 && AXIS == 1) {  // A3[o] -> A4[o]
        sa.in = gbl((const cpx<real> *)w.A3) + po * w.szA3;
        sa.out = gbl((cpx<real> *)w.A4) + po * w.szA4;
        set(sa.din, n1, n1, ez);
        set(sa.dout, n1, ey, ez);
    } else {  // MODE 1, AXIS 0: d = 3 A4[o] -> H[o], d = 2 A3[o] -> H[o]
        sa.in = w.d == 3 ? gbl((const cpx<real> *)w.A4) + po * w.szA4 : gbl((const cpx<real> *)w.A3) + po * w.szA3;
        sa.out = gbl((cpx<real> *)w.H) + po * w.szH;
        set(sa.din, n1, ey, ez);
        set(sa.dout, ex, ey, ez);
    }
}

__device__ __forceinline__ int64_t line_addr(const int *dims, int axis, int i0, int i1, int i2)
{
    return ((int64_t)i2 * dims[1] + i1) * dims[0] + i0;
}

template <typename real, int AXIS, int MODE, int L>
__global__ __launch_bounds__(kBlock) void k_fft(const WinDev *__restrict__ wins, const LineGroup *__restrict__ groups,
                                                FftCall call)
{
    using C = cpx<real>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const LineGroup lg = groups[blockIdx.x];
    const WinDev &w = wins[lg.win];
    const int nos = w.nos, n1 = w.n1, half = w.n >> 1;
    int pair, o;
    if (MODE == 1) {
        pair = blockIdx.y % call.npair;
        o = blockIdx.y / call.npair;
    } else {
        pair = blockIdx.y;
        o = 0;
    }
    StageArrays<real> sa;
    select_arrays<real, AXIS, MODE>(w, pair, o, sa);

    C *tw = (C *)smem_raw;
    C *buf0 = tw + call.nos_lds / 2;
    C *buf1 = buf0 + L * call.nos_lds;
    C *buf2 = buf1 + L * call.nos_lds;  // allocated for MODE 2 only
    for (int q = threadIdx.x; q < nos / 2; q += kBlock)
        tw[q] = ldc<real>(gbl((const C *)w.tw) + q);

    // lines of this group: coordinates (a, b) of the two non-transform axes
    const int *dims = sa.din;
    int la0 = 0, lb = 0, nvalid = 0;  // first line's inner index and outer index
    if (AXIS == 0) {
        const int rows = dims[1] * dims[2];
        la0 = lg.grp * L;  // row index
        nvalid = min(L, rows - la0);
    } else {
        const int e0 = dims[0];
        const int ng0 = (e0 + L - 1) / L;
        lb = lg.grp / ng0;
        la0 = (lg.grp % ng0) * L;
        nvalid = min(L, e0 - la0);
    }
    const int Lin = dims[AXIS];
    const int Lout = sa.dout[AXIS];

    auto addr = [&](const int *dd, int l, int q) -> int64_t {
        if (AXIS == 0) {
            const int row = la0 + l;
            return (int64_t)row * dd[0] + q;
        } else if (AXIS == 1) {
            return line_addr(dd, 1, la0 + l, q, lb);
        } else {
            return line_addr(dd, 2, la0 + l, lb, q);
        }
    };

    for (int i = threadIdx.x; i < L * nos; i += kBlock)
        buf0[i] = {real(0), real(0)};
    __syncthreads();
    for (int t = threadIdx.x; t < L * Lin; t += kBlock) {
        int l, q;
        if (AXIS == 0) {
            l = t / Lin;
            q = t - l * Lin;
        } else {
            l = t % L;
            q = t / L;
        }
        if (l < nvalid) {
            const int p = MODE == 1 ? (q - half + nos) % nos : w.lo[AXIS] + q;
            buf0[l * nos + p] = ldc<real>(sa.in + addr(sa.din, l, q));
        }
    }
    __syncthreads();
    const real sgn = MODE == 1 ? real(1) : real(-1);
    C *res = fft_lines<real>(buf0, buf1, tw, nos, L, sgn);
    __syncthreads();  // results are read across waves below

    if (MODE == 0 || MODE == 1) {
        for (int t = threadIdx.x; t < L * Lout; t += kBlock) {
            int l, q;
            if (AXIS == 0) {
                l = t / Lout;
                q = t - l * Lout;
            } else {
                l = t % L;
                q = t / L;
            }
            if (l < nvalid) {
                const int p = MODE == 0 ? (q - half + nos) % nos : w.lo[AXIS] + q;
                stc<real>(sa.out + addr(sa.dout, l, q), res[l * nos + p]);
            }
        }
        return;
    }

    // fused: forward result in res; multiply and transform back for each output
    C *fw = res;
    C *x0 = res == buf0 ? buf1 : buf0;
    C *x1 = buf2;
    // mode-space offset of each line inside the multiplier array
    auto lineoff = [&](int l) -> int64_t {
        if (AXIS == 2)
            return (int64_t)lb * n1 + la0 + l;
        if (AXIS == 1)
            return la0 + l;
        return 0;
    };
    int64_t stride_c = 1;
    for (int a = 0; a < AXIS; ++a)
        stride_c *= n1;
    if (call.modes_sel) {
        const gptr<C> M = gbl((C *)(call.modes_sel == 1 ? w.Vm : w.Gm)) + (int64_t)pair * w.szM;
        for (int t = threadIdx.x; t < L * n1; t += kBlock) {
            const int l = t % L, c = t / L;
            if (l < nvalid)
                stc<real>(M + c * stride_c + lineoff(l), fw[l * nos + (c - half + nos) % nos]);
        }
    }
    for (int oo = 0; oo < call.nout; ++oo) {
        const gptr<const real> B = gbl((const real *)(oo == 0 ? w.Bk : w.Bd));
        for (int i = threadIdx.x; i < L * nos; i += kBlock)
            x0[i] = {real(0), real(0)};
        __syncthreads();
        for (int t = threadIdx.x; t < L * n1; t += kBlock) {
            const int l = t % L, c = t / L;
            if (l < nvalid) {
                const int p = (c - half + nos) % nos;
                const real bm = B[c * stride_c + lineoff(l)];
                const C v = fw[l * nos + p];
                x0[l * nos + p] = {v.x * bm, v.y * bm};
            }
        }
        __syncthreads();
        C *r2 = fft_lines<real>(x0, x1, tw, nos, L, real(1));
        __syncthreads();
        const gptr<C> out = sa.out + (int64_t)oo * w.npair_cap * w.szH * (AXIS == 0) +
                 (int64_t)oo * w.npair_cap * w.szA3 * (AXIS != 0);
        for (int t = threadIdx.x; t < L * Lout; t += kBlock) {
            int l, q;
            if (AXIS == 0) {
                l = t / Lout;
                q = t - l * Lout;
            } else {
                l = t % L;
                q = t / L;
            }
            if (l < nvalid)
                stc<real>(out + addr(sa.dout, l, q), r2[l * nos + w.lo[AXIS] + q]);
        }
        __syncthreads();
        if (r2 != x0) {  // keep x0/x1 roles for the next output
            C *s = x0;
            x0 = x1;
            x1 = s;
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 window sum, derivative scalings, caller order

// Few RHS (R <= kCombineRowsMaxR): one thread per output row and all its RHS.
// A wave's reads of the point-major window products cover one contiguous run
// and its writes of each caller column are contiguous, so no LDS transpose is
// needed; the 16-RHS tiles of k_combine would leave most lanes idle here.
constexpr int kCombineRowsMaxR = 4;

template <typename real>
__global__ __launch_bounds__(kBlock) void k_combine_rows(const WinDev *__restrict__ wins, IoArgs io, int R, int mode)
{
    const ProbDev p = get_prob(io, blockIdx.y);
    const int nwin = p.wend - p.wbeg;
    const bool want_y = (mode & 1) && p.Y, want_ds = (mode & 2) && p.dYs, want_dl = (mode & 4) && p.dYl;
    for (int64_t i = p.yoff + blockIdx.x * (int64_t)kBlock + threadIdx.x; i < p.N; i += (int64_t)gridDim.x * kBlock) {
        const int64_t iy = i - p.yoff;  // output row
        double y[kCombineRowsMaxR] = {};
        for (int k = 0; k < nwin; ++k) {
            const WinDev &w = wins[p.wbeg + k];
            const gptr<const real> src = gbl((const real *)w.Yw) + i * w.Rcap;
            const gptr<const real> dsrc = gbl((const real *)w.Yw) + ((int64_t)w.N + i) * w.Rcap;
            const int64_t blk = (int64_t)k * p.ldy * R;  // window k's block of dY/dl, dY/dsigma
#pragma unroll
            for (int r = 0; r < kCombineRowsMaxR; ++r) {
                if (r >= R)
                    break;
                const double v = (double)src[r];
                const int64_t at = blk + iy + (int64_t)r * p.ldy;
                y[r] += w.sig2 * v;
                if (want_ds)
                    gbl(p.dYs)[at] = w.dsig * v;
                if (want_dl)
                    gbl(p.dYl)[at] = w.der_scale * (double)dsrc[r];
            }
        }
        if (want_y)
#pragma unroll
            for (int r = 0; r < kCombineRowsMaxR; ++r)
                if (r < R)
                    gbl(p.Y)[iy + (int64_t)r * p.ldy] = y[r];
    }
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_combine(const WinDev *__restrict__ wins, IoArgs io, int R, int mode)
{
    typedef real v4r __attribute__((ext_vector_type(4)));
    // Tiles of 64 points x 16 RHS: the window products (point-major) are read
    // row by row into LDS and written out column by column, so that both the
    // reads and the writes of the caller's column-major matrices are coalesced.
    // The (window, output) blocks of a tile are software pipelined: the loads
    // of the next kCombineDepth blocks are in flight while the current one goes
    // through LDS.
    __shared__ double tile[64][17];
    const ProbDev p = get_prob(io, blockIdx.y);
    const int t = threadIdx.x, il = t & 63, rq = t >> 6;
    const int nout = (mode & 4) && p.dYl ? 2 : 1;
    const int nblk = (p.wend - p.wbeg) * nout;
    for (int64_t i0 = p.yoff + blockIdx.x * (int64_t)64; i0 < p.N; i0 += (int64_t)gridDim.x * 64) {
        const int64_t i = i0 + il;
        const bool own = i < p.N;
        const int64_t iy = i - p.yoff;  // output row
        for (int r0 = 0; r0 < R; r0 += 16) {
            const int nr = min(16, R - r0);
            // thread t loads RHS 4 (t % 4) .. + 3 of point t / 4 of the tile (rows
            // padded to a multiple of 4: one 4-vector)
            const int pl = t >> 2, r4 = (t & 3) * 4;
            auto load = [&](int k, v4r &v) {
                const WinDev &w = wins[p.wbeg + k / nout];
                const int o = k % nout;
                const int64_t ip = i0 + pl;
                v = ip < p.N && r4 < nr ? *(gptr<const v4r>)(gbl((const real *)w.Yw) + ((int64_t)o * w.N + ip) * w.Rcap + r0 + r4)
                                        : v4r{real(0), real(0), real(0), real(0)};
            };
            constexpr int DEP = kCombineDepth;
            double y[4] = {0.0, 0.0, 0.0, 0.0};
            v4r ring[DEP + 1];
#pragma unroll
            for (int k = 0; k < DEP; ++k)
                if (k < nblk)
                    load(k, ring[k]);
            // ring[0] holds block k; ring[1 ..] the next ones (shifted down each step)
            for (int k = 0; k < nblk; ++k) {
                if (k + DEP < nblk)
                    load(k + DEP, ring[DEP]);
                const int wi = p.wbeg + k / nout, o = k % nout;
                const WinDev &w = wins[wi];
                const int64_t blk = (int64_t)(wi - p.wbeg) * p.ldy * R;
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 4; ++q)  // columns past nr are zero (masked rows of the 4-vector)
                    tile[pl][r4 + q] = r4 + q < nr ? (double)ring[0][q] : 0.0;
#pragma unroll
                for (int j = 0; j < DEP; ++j)
                    ring[j] = ring[j + 1];
                __syncthreads();
                if (own) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int rr = rq + 4 * q;
                        if (rr >= nr)
                            continue;
                        const double v = tile[il][rr];
                        const int64_t at = iy + (int64_t)(r0 + rr) * p.ldy;
                        if (o == 0) {
                            y[q] += w.sig2 * v;
                            if ((mode & 2) && p.dYs)
                                gbl(p.dYs)[blk + at] = w.dsig * v;
                        } else {
                            gbl(p.dYl)[blk + at] = w.der_scale * v;
                        }
                    }
                }
            }
            if ((mode & 1) && p.Y && own)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (rq + 4 * q < nr)
                        gbl(p.Y)[iy + (int64_t)(r0 + rq + 4 * q) * p.ldy] = y[q];
        }
    }
}

// ---------------------------------------------------------------------------
// Fourier-domain inner products for the vjp: sum over pairs and modes of
// Re(conj(G^_k) B_k V^_k) for the kernel and derivative multipliers.

template <typename real>
__global__ __launch_bounds__(kBlock) void k_mode_dot(const WinDev *__restrict__ wins, int win, int npair,
                                                     double *partial)
{
    const WinDev &w = wins[win];
    const int64_t total = (int64_t)npair * w.szM;
    const gptr<const cpx<real>> Gm = gbl((const cpx<real> *)w.Gm);
    const gptr<const cpx<real>> Vm = gbl((const cpx<real> *)w.Vm);
    const gptr<const real> Bk = gbl((const real *)w.Bk);
    const gptr<const real> Bd = gbl((const real *)w.Bd);
    double sk = 0.0, sd = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
        const int64_t idx = e % w.szM;
        const cpx<real> g = ldc<real>(Gm + e), v = ldc<real>(Vm + e);
        const double re = (double)g.x * (double)v.x + (double)g.y * (double)v.y;
        sk += (double)Bk[idx] * re;
        sd += (double)Bd[idx] * re;
    }
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = sk;
    red[1][threadIdx.x] = sd;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = red[0][0];
        partial[2 * blockIdx.x + 1] = red[1][0];
    }
}

__global__ void k_mode_dot_finish(const WinDev *__restrict__ wins, int win, int nblk, const double *partial,
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
        grad_ell[0] = w.der_scale * sd;
    if (grad_sig)
        grad_sig[0] = w.dsig * sk;
}

// ---------------------------------------------------------------------------
// Global sensitivity indices (Algorithm 1): the trigonometric polynomial of a
// window has coefficients w_k b_k a_k, a_k = sum_j v_j e^{-2 pi i k x_j}; the
// variance of its ANOVA term on the features u is the sum of |w_k b_k a_k|^2
// over the modes whose support is u.  With B_k = w_k b_k / prod Psi(k_i)^2
// and the spread-and-transformed modes g^_k = a_k prod Psi(k_i), that is
// |B_k prod Psi(k_i) g^_k|^2.  Bins: bit i of the mask set iff k_i != 0.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_gsi_theta(const cpx<real> *__restrict__ Vm, const double *__restrict__ B,
                                                      const double *__restrict__ psi, int d, int n, int64_t szM,
                                                      double *partial)
{
    const int n1 = n + 1, half = n / 2;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x; idx < szM; idx += (int64_t)gridDim.x * kBlock) {
        int64_t r = idx;
        int mask = 0;
        double ps = 1.0;
        for (int i = 0; i < d; ++i) {
            const int c = (int)(r % n1);
            r /= n1;
            mask |= (c != half) << i;
            ps *= psi[c];
        }
        const cpx<real> g = Vm[idx];
        const double cf = B[idx] * ps;
        const double val = cf * cf * ((double)g.x * (double)g.x + (double)g.y * (double)g.y);
#pragma unroll
        for (int b = 0; b < 8; ++b)
            acc[b] += b == mask ? val : 0.0;
    }
    __shared__ double red[8][kBlock];
#pragma unroll
    for (int b = 0; b < 8; ++b)
        red[b][threadIdx.x] = acc[b];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int b = 0; b < 8; ++b)
                red[b][threadIdx.x] += red[b][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 8)
        partial[(int64_t)blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_gsi_finish(int nblk, const double *partial, double *theta)
{
    const int b = threadIdx.x;
    if (blockIdx.x != 0 || b >= 8)
        return;
    double s = 0.0;
    for (int k = 0; k < nblk; ++k)
        s += partial[(int64_t)k * 8 + b];
    theta[b] = s;
}

static void free_dev(void *p);

// theta: device array of 8 doubles per window (window order of the engine)
addk_status engine_gsi(Engine &E, const std::vector<const double *> &B64, const double *psi, int n, double *theta,
                       hipStream_t st)
{
    const int nblk = 128;
    const int64_t need = (int64_t)8 * nblk;
    if (E.partial_cap < need) {
        free_dev(E.d_partial);
        E.d_partial = nullptr;
        hipError_t e = hipMalloc(&E.d_partial, need * sizeof(double));
        if (e != hipSuccess)
            return hip_fail(e, "hipMalloc(partials)");
        E.partial_cap = need;
    }
    for (size_t wi = 0; wi < E.wdev.size(); ++wi) {
        const WinDev &w = E.wdev[wi];
        if (E.precision == ADDK_FP32)
            hipLaunchKernelGGL(k_gsi_theta<float>, dim3(nblk), dim3(kBlock), 0, st, (const cpx<float> *)w.Vm, B64[wi],
                               psi, w.d, n, w.szM, E.d_partial);
        else
            hipLaunchKernelGGL(k_gsi_theta<double>, dim3(nblk), dim3(kBlock), 0, st, (const cpx<double> *)w.Vm,
                               B64[wi], psi, w.d, n, w.szM, E.d_partial);
        hipLaunchKernelGGL(k_gsi_finish, dim3(1), dim3(64), 0, st, nblk, E.d_partial, theta + 8 * wi);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "gsi launch");
    return ADDK_OK;
}

// ---------------------------------------------------------------------------
// host side

// Lines per FFT block: 8 in FP32 (more blocks per CU than 16, and 64-byte
// runs per access in the y and z passes; 4 was slower), 8 in FP64 for lines of
// up to 128 points and 4 for 256-point grids, so that the three line buffers
// stay within 64 KiB of LDS.
static int lines_per_group(int precision, int nos_max)
{
    if (precision == ADDK_FP32)
        return 8;
    return nos_max > 128 ? 4 : 8;
}

static size_t real_size(int precision) { return precision == ADDK_FP32 ? sizeof(float) : sizeof(double); }

static int pick_rb(int vol, int precision, int D)
{
    const size_t rs = real_size(precision);
    const size_t wv = (size_t)16 * D * kMaxW * rs;
    int rb = 16;
    while (rb > 1 && (size_t)rb * vol * rs + wv > (size_t)kLdsBudget)
        rb >>= 1;
    return rb;
}

static int ngroups_stage(const WinDev &w, int st, int L)
{
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2], n1 = w.n1;
    auto cdiv = [](int a, int b) { return (a + b - 1) / b; };
    switch (st) {
    case ST_FWD0:
        return w.d >= 2 ? cdiv(ey * ez, L) : 0;
    case ST_FWD1:
        return w.d == 3 ? ez * cdiv(n1, L) : 0;
    case ST_FUSED2:
        return w.d == 3 ? n1 * cdiv(n1, L) : 0;
    case ST_FUSED1:
        return w.d == 2 ? cdiv(n1, L) : 0;
    case ST_FUSED0:
        return w.d == 1 ? 1 : 0;
    case ST_INV1:
        return w.d == 3 ? ez * cdiv(n1, L) : 0;
    case ST_INV0:
        return w.d >= 2 ? cdiv(ey * ez, L) : 0;
    }
    return 0;
}

static void free_dev(void *p)
{
    if (p)
        (void)hipFree(p);
}

static hipEvent_t take_event(Engine &E)
{
    if (!E.evpool.empty()) {
        hipEvent_t e = E.evpool.back();
        E.evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

StageTimer::StageTimer(Engine &e, int s, hipStream_t t) : E(e), stage(s), st(t)
{
    if (E.prof) {
        a = take_event(E);
        if (a)
            (void)hipEventRecord(a, st);
    }
}

StageTimer::~StageTimer()
{
    if (E.prof && a) {
        hipEvent_t b = take_event(E);
        if (b) {
            (void)hipEventRecord(b, st);
            E.recs.push_back({stage, a, b});
        } else {
            E.evpool.push_back(a);
        }
    }
}

addk_status engine_profile_read(Engine &E, double *ms, int32_t *count)
{
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceSynchronize");
    for (int s = 0; s < PS_COUNT; ++s) {
        if (ms)
            ms[s] = 0.0;
        if (count)
            count[s] = 0;
    }
    for (const ProfRec &r : E.recs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            if (ms)
                ms[r.stage] += t;
            if (count)
                count[r.stage] += 1;
        }
        E.evpool.push_back(r.a);
        E.evpool.push_back(r.b);
    }
    E.recs.clear();
    return ADDK_OK;
}

void engine_free(Engine &E)
{
    free_dev(E.d_wins);
    for (int d = 0; d < 4; ++d) {
        free_dev(E.d_chunks[d]);
        free_dev(E.d_chunks_i[d]);
        free_dev(E.d_dense[d][0]);
        free_dev(E.d_dense[d][1]);
        free_dev(E.d_dense_sp[d][0]);
        free_dev(E.d_dense_sp[d][1]);
    }
    for (int s = 0; s < ST_COUNT; ++s)
        free_dev(E.d_groups[s]);
    free_dev(E.ws);
    free_dev(E.yw);
    free_dev(E.d_probs);
    free_dev(E.d_partial);
    for (int wi = 0; wi < 2; ++wi) {
        free_dev(E.d_dmap[wi]);
        free_dev(E.d_gtiles[wi]);
        free_dev(E.d_sptiles[wi]);
        free_dev(E.scratch[wi]);
    }
    free_dev(E.vpack);
    free_dev(E.d_tw);
    for (int d = 1; d <= 3; ++d) {
        free_dev(E.d_near[d]);
        E.d_near[d] = nullptr;
        E.nnear[d] = 0;
    }
    free_dev(E.d_near_part);
    E.d_near_part = nullptr;
    free_dev(E.d_near_ys);
    E.d_near_ys = nullptr;
    free_dev(E.d_sprng);
    E.d_sprng = nullptr;
    E.near_part_cap = 0;
    for (const ProfRec &r : E.recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t ev : E.evpool)
        (void)hipEventDestroy(ev);
    E = Engine();
}

// Device work lists for the engine's windows (descriptors are uploaded by
// engine_ensure_workspace, which knows the workspace pointers).
// Twiddle tables e^{2 pi i q / nos}, q < nos / 2, for nos = 16 .. 128, computed
// in FP64 on the host and rounded once; offset of the table of nos, in entries.
static int tw_offset(int nos)
{
    int off = 0;
    for (int s = 16; s < nos; s <<= 1)
        off += s / 2;
    return off;
}

static addk_status build_twiddles(Engine &E)
{
    free_dev(E.d_tw);
    E.d_tw = nullptr;
    const int total = tw_offset(2 * kMaxNos);
    std::vector<double> re(total), im(total);
    for (int nos = 16; nos <= kMaxNos; nos <<= 1)
        for (int q = 0; q < nos / 2; ++q) {
            re[tw_offset(nos) + q] = std::cos(2.0 * M_PI * q / nos);
            im[tw_offset(nos) + q] = std::sin(2.0 * M_PI * q / nos);
        }
    const size_t rs = real_size(E.precision);
    std::vector<unsigned char> host(total * 2 * rs);
    for (int i = 0; i < total; ++i) {
        if (E.precision == ADDK_FP32) {
            const float v[2] = {(float)re[i], (float)im[i]};
            std::memcpy(&host[i * 2 * rs], v, sizeof(v));
        } else {
            const double v[2] = {re[i], im[i]};
            std::memcpy(&host[i * 2 * rs], v, sizeof(v));
        }
    }
    hipError_t e = hipMalloc(&E.d_tw, host.size());
    if (e == hipSuccess)
        e = hipMemcpy(E.d_tw, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return hip_fail(e, "twiddle tables");
    for (WinDev &w : E.wdev)
        w.tw = (const char *)E.d_tw + (size_t)tw_offset(w.nos) * 2 * rs;
    return ADDK_OK;
}

addk_status engine_build_device(Engine &E, int precision)
{
    E.precision = precision;
    {
        addk_status s = build_twiddles(E);
        if (s != ADDK_OK)
            return s;
    }
    E.nos_max = 16;
    for (const WinDev &w : E.wdev)
        E.nos_max = std::max(E.nos_max, w.nos);
    const int L = lines_per_group(precision, E.nos_max);
    E.fft_L = L;
    std::vector<Chunk> ch[4], chi[4];
    std::vector<Chunk> dn[4][2], dsp[4][2];
    std::vector<LineGroup> gr[ST_COUNT];
    for (int d = 0; d < 4; ++d) {
        E.maxvol[d] = 0;
        E.rb[d] = 0;
        E.tile_w[d] = 0;
    }
    for (size_t wi = 0; wi < E.wdev.size(); ++wi) {
        const WinDev &w = E.wdev[wi];
        const WinHost &h = E.plans[E.wplan[wi]]->wins[E.wlocal[wi]];
        for (const Chunk &c : h.chunks) {
            Chunk cc = c;
            cc.win = (int)wi;
            ch[w.d].push_back(cc);
        }
        for (const Chunk &c : h.split ? h.chunks_i : h.chunks) {
            Chunk cc = c;
            cc.win = (int)wi;
            chi[w.d].push_back(cc);
        }
        for (const Chunk &c : h.dense) {
            Chunk cc = c;
            cc.win = (int)wi;
            dn[w.d][w.W == 8 ? 0 : 1].push_back(cc);
        }
        for (const Chunk &c : h.dense_sp) {
            Chunk cc = c;
            cc.win = (int)wi;
            dsp[w.d][w.W == 8 ? 0 : 1].push_back(cc);
        }
        E.maxvol[w.d] = std::max(E.maxvol[w.d], w.S[0] * w.S[1] * w.S[2]);
        if (!h.chunks.empty() || !h.chunks_i.empty()) {
            if (E.tile_w[w.d] == 0)
                E.tile_w[w.d] = w.W;
            else if (E.tile_w[w.d] != w.W)
                E.tile_w[w.d] = -1;
        }
        for (int s = 0; s < ST_COUNT; ++s) {
            const int ng = ngroups_stage(w, s, L);
            for (int g = 0; g < ng; ++g)
                gr[s].push_back({(int)wi, g});
        }
    }
    for (int d = 1; d <= 3; ++d) {
        if (E.maxvol[d])
            E.rb[d] = pick_rb(E.maxvol[d], precision, d);
        // sparse-tile chunks heaviest first (as the dense items; the tile spreads
        // add to the grids with atomics, in any order)
        std::stable_sort(ch[d].begin(), ch[d].end(), [](const Chunk &x, const Chunk &y) { return x.count > y.count; });
        std::stable_sort(chi[d].begin(), chi[d].end(), [](const Chunk &x, const Chunk &y) { return x.count > y.count; });
        for (int side = 0; side < 2; ++side) {  // spreading, interpolation
            const std::vector<Chunk> &v = side == 0 ? ch[d] : chi[d];
            Chunk *&dp = side == 0 ? E.d_chunks[d] : E.d_chunks_i[d];
            (side == 0 ? E.nchunks[d] : E.nchunks_i[d]) = (int)v.size();
            free_dev(dp);
            dp = nullptr;
            if (!v.empty()) {
                hipError_t e = hipMalloc(&dp, v.size() * sizeof(Chunk));
                if (e != hipSuccess)
                    return hip_fail(e, "hipMalloc(chunks)");
                e = hipMemcpy(dp, v.data(), v.size() * sizeof(Chunk), hipMemcpyHostToDevice);
                if (e != hipSuccess)
                    return hip_fail(e, "hipMemcpy(chunks)");
            }
        }
    }
    auto upload_items = [](const std::vector<Chunk> &v, Chunk *&dptr, int &n) -> addk_status {
        n = (int)v.size();
        free_dev(dptr);
        dptr = nullptr;
        if (v.empty())
            return ADDK_OK;
        hipError_t e = hipMalloc(&dptr, v.size() * sizeof(Chunk));
        if (e == hipSuccess)
            e = hipMemcpy(dptr, v.data(), v.size() * sizeof(Chunk), hipMemcpyHostToDevice);
        return e == hipSuccess ? ADDK_OK : hip_fail(e, "dense item lists");
    };
    // near-field target blocks: runs of <= kNearChunk sorted points of one tile
    {
        std::vector<Chunk> nl[4];
        E.near_rng.assign(E.wdev.size(), make_int2(0, 0));
        for (size_t wi = 0; wi < E.wdev.size(); ++wi) {
            const WinHost &h = E.plans[E.wplan[wi]]->wins[E.wlocal[wi]];
            const std::vector<int32_t> &to = h.split ? h.tile_off_t : h.tile_off;  // the targets' tiles
            if (!h.nf || to.empty())
                continue;
            std::vector<Chunk> &l = nl[h.d];
            E.near_rng[wi].x = (int)l.size();
            for (int64_t t = 0; t < h.ntiles; ++t)
                for (int32_t s = to[t]; s < to[t + 1]; s += kNearChunk)
                    l.push_back({(int32_t)wi, (int32_t)t, s, std::min<int32_t>(kNearChunk, to[t + 1] - s)});
            E.near_rng[wi].y = (int)l.size();
        }
        for (int d = 1; d <= 3; ++d) {
            addk_status s = upload_items(nl[d], E.d_near[d], E.nnear[d]);
            if (s != ADDK_OK)
                return s;
        }
    }
    // d = 3 spread items: two-cell items first (stable, so that the items of one
    // anchor cell stay consecutive), each part spread by its own kernel variant.
    // Inside each part the anchors run heaviest first (by their first item, the
    // largest), so that the long blocks do not start last; an anchor's items
    // stay consecutive and in order (the gather's block map and its sum order
    // depend only on that).
    for (int wi = 0; wi < 2; ++wi) {
        std::vector<Chunk> &v = dsp[3][wi];
        auto two = [](const Chunk &c) { return ((c.tile >> 30) & 1) != 0; };
        std::stable_partition(v.begin(), v.end(), two);
        E.ndense_sp2[wi] = (int)std::count_if(v.begin(), v.end(), two);
        auto heaviest_first = [&v](size_t b, size_t e) {
            std::vector<std::pair<size_t, size_t>> runs;  // [first, end) of each anchor's items
            for (size_t i = b; i < e;) {
                size_t j = i + 1;
                while (j < e && v[j].win == v[i].win && v[j].tile == v[i].tile)
                    ++j;
                runs.push_back({i, j});
                i = j;
            }
            std::stable_sort(runs.begin(), runs.end(), [&v](const std::pair<size_t, size_t> &x,
                                                            const std::pair<size_t, size_t> &y) {
                return v[x.first].count > v[y.first].count;
            });
            std::vector<Chunk> out;
            out.reserve(e - b);
            for (const auto &r : runs)
                out.insert(out.end(), v.begin() + r.first, v.begin() + r.second);
            std::copy(out.begin(), out.end(), v.begin() + b);
        };
        heaviest_first(0, E.ndense_sp2[wi]);
        heaviest_first(E.ndense_sp2[wi], v.size());
    }
    // d <= 2 spread items (added to the grids with atomics, in any order): heaviest first
    for (int d = 1; d <= 2; ++d)
        for (int wi = 0; wi < 2; ++wi)
            std::stable_sort(dsp[d][wi].begin(), dsp[d][wi].end(),
                             [](const Chunk &x, const Chunk &y) { return x.count > y.count; });
    // interpolation items (each point's products written once, in any order):
    // the classes of 16-point groups per wave heaviest first, so that the long
    // blocks do not start last, and cell order inside a class, so that blocks
    // running together share window blocks in L2 (sorting by the exact count
    // was 1% faster but read 8.3 GB per call instead of 2.4)
    auto by_groups = [](const Chunk &x, const Chunk &y) { return (x.count + 63) / 64 > (y.count + 63) / 64; };
    for (int d = 1; d <= 3; ++d)
        for (int wi = 0; wi < 2; ++wi) {
            std::stable_sort(dn[d][wi].begin(), dn[d][wi].end(), by_groups);
            addk_status s = upload_items(dn[d][wi], E.d_dense[d][wi], E.ndense[d][wi]);
            if (s == ADDK_OK)
                s = upload_items(dsp[d][wi], E.d_dense_sp[d][wi], E.ndense_sp[d][wi]);
            if (s != ADDK_OK)
                return s;
        }
    // base-cell maps and gather tiles for the matrix-core dense spread (d = 3)
    for (WinDev &d : E.wdev)
        d.dmap = nullptr;
    for (int wi = 0; wi < 2; ++wi) {
        free_dev(E.d_dmap[wi]);
        free_dev(E.d_gtiles[wi]);
        E.d_dmap[wi] = nullptr;
        E.d_gtiles[wi] = nullptr;
        E.ngtiles[wi] = 0;
        const std::vector<Chunk> &items = dsp[3][wi];  // the spread items own the blocks
        if (items.empty())
            continue;
        std::vector<int64_t> moff(E.wdev.size(), -1);
        int64_t mtot = 0;
        for (size_t w = 0; w < E.wdev.size(); ++w) {
            WinDev &d = E.wdev[w];
            if (d.d != 3 || d.W != (wi == 0 ? 8 : 12))
                continue;
            for (int a = 0; a < 3; ++a)
                d.nbase[a] = d.ext[a] - d.W + 1;
            moff[w] = mtot;
            mtot += (int64_t)d.nbase[0] * d.nbase[1] * d.nbase[2];
        }
        std::vector<int2> map(mtot, make_int2(0, 0));
        std::vector<std::vector<int32_t>> mark(E.wdev.size());  // per gather tile: the item blocks reaching it
        for (size_t i = 0; i < items.size(); ++i) {
            const Chunk &c = items[i];
            const WinDev &d = E.wdev[c.win];
            const int bx = c.tile & 1023, by = (c.tile >> 10) & 1023, bz = (c.tile >> 20) & 1023;
            const int nzc = ((c.tile >> 30) & 1) + 1;
            int2 &e = map[moff[c.win] + ((int64_t)bz * d.nbase[1] + by) * d.nbase[0] + bx];
            if (e.y == 0)
                e.x = (int)i;
            e.y = ((e.y & 0xffff) + 1) | ((nzc - 1) << 16);  // item count, z cells of the anchor's items
            const int nt0 = (d.ext[0] + 3) / 4, nt1 = (d.ext[1] + 3) / 4, nt2 = (d.ext[2] + 3) / 4;
            if (mark[c.win].empty())
                mark[c.win].assign((size_t)nt0 * nt1 * nt2, 0);
            for (int tz = bz / 4; tz <= (bz + d.W + nzc - 2) / 4 && tz < nt2; ++tz)
                for (int ty = by / 4; ty <= (by + d.W - 1) / 4 && ty < nt1; ++ty)
                    for (int tx = bx / 4; tx <= (bx + d.W - 1) / 4 && tx < nt0; ++tx)
                        mark[c.win][((size_t)tz * nt1 + ty) * nt0 + tx] += 1;
        }
        // gather tiles heaviest first (each tile's sums do not depend on the order)
        std::vector<LineGroup> tiles;
        for (size_t w = 0; w < E.wdev.size(); ++w)
            for (size_t t = 0; t < mark[w].size(); ++t)
                if (mark[w][t])
                    tiles.push_back({(int)w, (int)t});
        std::stable_sort(tiles.begin(), tiles.end(), [&mark](const LineGroup &x, const LineGroup &y) {
            return mark[x.win][x.grp] > mark[y.win][y.grp];
        });
        hipError_t e = hipMalloc(&E.d_dmap[wi], std::max<int64_t>(1, mtot) * sizeof(int2));
        if (e == hipSuccess)
            e = hipMemcpy(E.d_dmap[wi], map.data(), mtot * sizeof(int2), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMalloc(&E.d_gtiles[wi], std::max<size_t>(1, tiles.size()) * sizeof(LineGroup));
        if (e == hipSuccess && !tiles.empty())
            e = hipMemcpy(E.d_gtiles[wi], tiles.data(), tiles.size() * sizeof(LineGroup), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return hip_fail(e, "dense block maps");
        E.ngtiles[wi] = (int)tiles.size();
        for (size_t w = 0; w < E.wdev.size(); ++w)
            if (moff[w] >= 0)
                E.wdev[w].dmap = E.d_dmap[wi] + moff[w];
    }
    // Sparse spread of d = 3 windows by output tiles (4^3 grid cells each):
    // per window, the range of every point tile's sparse points and the list
    // of output tiles that such points reach.  Used when every d = 3 window
    // with sparse points has 4^3-cell point tiles and 2m in {8, 12}.
    {
        free_dev(E.d_sprng);
        E.d_sprng = nullptr;
        for (int wi = 0; wi < 2; ++wi) {
            free_dev(E.d_sptiles[wi]);
            E.d_sptiles[wi] = nullptr;
            E.nsptiles[wi] = 0;
        }
        for (WinDev &d : E.wdev)
            d.sp_rng = nullptr;
        bool ok = true;
        int64_t ntot = 0;
        std::vector<int64_t> roff(E.wdev.size(), -1);
        for (size_t wi = 0; wi < E.wdev.size(); ++wi) {
            const WinDev &d = E.wdev[wi];
            const WinHost &h = E.plans[E.wplan[wi]]->wins[E.wlocal[wi]];
            if (d.d != 3 || h.chunks.empty())
                continue;
            if (d.tb[0] != 4 || d.tb[1] != 4 || d.tb[2] != 4 || (d.W != 8 && d.W != 12))
                ok = false;
            roff[wi] = ntot;
            ntot += (int64_t)d.ntile[0] * d.ntile[1] * d.ntile[2];
        }
        E.sparse_gather = ok && ntot > 0;
        if (E.sparse_gather) {
            std::vector<int2> rng(ntot, make_int2(0, 0));
            std::vector<LineGroup> lists[2];
            std::vector<std::pair<int64_t, LineGroup>> work[2];
            for (size_t wi = 0; wi < E.wdev.size(); ++wi) {
                if (roff[wi] < 0)
                    continue;
                const WinDev &d = E.wdev[wi];
                const WinHost &h = E.plans[E.wplan[wi]]->wins[E.wlocal[wi]];
                int2 *r = rng.data() + roff[wi];
                for (const Chunk &c : h.chunks) {  // the sources' sparse chunks, consecutive per tile
                    if (r[c.tile].y == 0)
                        r[c.tile].x = c.start;
                    r[c.tile].y += c.count;
                }
                const int ot[3] = {(d.ext[0] + 3) / 4, (d.ext[1] + 3) / 4, (d.ext[2] + 3) / 4};
                const int reach = (d.W + 2) / 4;  // a point tile reaches output tiles tp .. tp + reach
                std::vector<int64_t> load((size_t)ot[0] * ot[1] * ot[2], -1);  // points reaching a tile
                for (int tz = 0; tz < d.ntile[2]; ++tz)
                    for (int ty = 0; ty < d.ntile[1]; ++ty)
                        for (int tx = 0; tx < d.ntile[0]; ++tx) {
                            const int cnt = r[((int64_t)tz * d.ntile[1] + ty) * d.ntile[0] + tx].y;
                            if (cnt == 0)
                                continue;
                            for (int oz = tz; oz <= std::min(ot[2] - 1, tz + reach); ++oz)
                                for (int oy = ty; oy <= std::min(ot[1] - 1, ty + reach); ++oy)
                                    for (int ox = tx; ox <= std::min(ot[0] - 1, tx + reach); ++ox) {
                                        int64_t &l = load[((size_t)oz * ot[1] + oy) * ot[0] + ox];
                                        l = (l < 0 ? 0 : l) + cnt;
                                    }
                        }
                for (size_t t = 0; t < load.size(); ++t)
                    if (load[t] >= 0)
                        work[d.W == 8 ? 0 : 1].push_back({load[t], LineGroup{(int)wi, (int)t}});
            }
            // heaviest tiles first (the points per tile vary by two orders of
            // magnitude near the dense core): the last blocks to start are short
            for (int k = 0; k < 2; ++k) {
                std::stable_sort(work[k].begin(), work[k].end(),
                                 [](const std::pair<int64_t, LineGroup> &a, const std::pair<int64_t, LineGroup> &b) {
                                     return a.first > b.first;
                                 });
                for (const auto &pw : work[k])
                    lists[k].push_back(pw.second);
            }
            hipError_t e = hipMalloc(&E.d_sprng, ntot * sizeof(int2));
            if (e == hipSuccess)
                e = hipMemcpy(E.d_sprng, rng.data(), ntot * sizeof(int2), hipMemcpyHostToDevice);
            for (int wi = 0; wi < 2 && e == hipSuccess; ++wi) {
                E.nsptiles[wi] = (int)lists[wi].size();
                if (lists[wi].empty())
                    continue;
                e = hipMalloc(&E.d_sptiles[wi], lists[wi].size() * sizeof(LineGroup));
                if (e == hipSuccess)
                    e = hipMemcpy(E.d_sptiles[wi], lists[wi].data(), lists[wi].size() * sizeof(LineGroup),
                                  hipMemcpyHostToDevice);
            }
            if (e != hipSuccess)
                return hip_fail(e, "sparse spread lists");
            for (size_t wi = 0; wi < E.wdev.size(); ++wi)
                if (roff[wi] >= 0)
                    E.wdev[wi].sp_rng = E.d_sprng + roff[wi];
        }
    }
    for (int s = 0; s < ST_COUNT; ++s) {
        E.ngroups[s] = (int)gr[s].size();
        free_dev(E.d_groups[s]);
        E.d_groups[s] = nullptr;
        if (!gr[s].empty()) {
            hipError_t e = hipMalloc(&E.d_groups[s], gr[s].size() * sizeof(LineGroup));
            if (e != hipSuccess)
                return hip_fail(e, "hipMalloc(groups)");
            e = hipMemcpy(E.d_groups[s], gr[s].data(), gr[s].size() * sizeof(LineGroup), hipMemcpyHostToDevice);
            if (e != hipSuccess)
                return hip_fail(e, "hipMemcpy(groups)");
        }
    }
    // the descriptor table (uploaded with the workspace pointers)
    if (!E.d_wins) {
        hipError_t e = hipMalloc(&E.d_wins, std::max<size_t>(1, E.wdev.size()) * sizeof(WinDev));
        if (e != hipSuccess)
            return hip_fail(e, "hipMalloc(descriptors)");
    }
    // one square plan whose windows are all d = 1 (no near field, one window
    // width): interpolation fused with the window sum, in the caller's order
    E.fused_d1 = !E.wdev.empty() && E.plans.size() == 1 && !E.plans[0]->rect;
    for (const WinDev &w : E.wdev)
        if (w.d != 1 || !w.ucoords || w.nf || w.W != E.wdev[0].W)
            E.fused_d1 = false;
    if (E.fused_d1 && interp_combine_d1_lds(E, 2) > 64 * 1024)
        E.fused_d1 = false;
    E.fused_no = 0;
    return ADDK_OK;
}

// Sizes of the per-call workspace for cap complex grids per window and rcap
// right-hand sides (also fills the per-window grid sizes of the descriptors).
WsLayout engine_ws_layout(Engine &E, int cap, int64_t rcap)
{
    WsLayout L;
    L.cap = cap;
    // more than four RHS: rows of the per-window products padded to a multiple
    // of four, so that the window sum reads them as 4-vectors
    L.rcap = rcap > kCombineRowsMaxR ? (rcap + 3) / 4 * 4 : rcap;
    const size_t cs = 2 * real_size(E.precision);
    int64_t total = 0, ytotal = 0, ys = 0;
    for (WinDev &w : E.wdev) {
        const int64_t ex = w.ext[0], ey = w.ext[1], ez = w.ext[2], n1 = w.n1;
        w.szG = ex * ey * ez;
        w.szH = w.szG;
        w.szA1 = w.d >= 2 ? n1 * ey * ez : 0;
        w.szA2 = w.d == 3 ? n1 * n1 * ez : 0;
        w.szA3 = w.d == 3 ? n1 * n1 * ez : (w.d == 2 ? n1 * ey : 0);
        w.szA4 = w.d == 3 ? n1 * ey * ez : 0;
        w.szM = w.d == 3 ? n1 * n1 * n1 : (w.d == 2 ? n1 * n1 : n1);
        total += (int64_t)cap * (w.szG + w.szA1 + w.szA2 + 2 * (w.szA3 + w.szA4 + w.szH) + 2 * w.szM);
        ytotal += 2 * L.rcap * w.N;  // rows of the (padded) row length
        ys += w.nf ? 2 * w.N : 0;
    }
    L.grid_bytes = std::max<int64_t>(total * (int64_t)cs, 256);
    L.y_bytes = std::max<int64_t>(ytotal * (int64_t)real_size(E.precision), 256);
    L.nys_bytes = ys * (int64_t)sizeof(double);
    int64_t packN = 0;
    for (const Plan *pl : E.plans)
        packN += pl->N;
    L.vpack_ld = (L.rcap + 15) / 16 * 16;
    L.vpack_bytes = std::max<int64_t>(packN * L.vpack_ld * (int64_t)real_size(E.precision), 256);
    for (int wi = 0; wi < 2; ++wi) {
        const int W = wi == 0 ? 8 : 12;
        L.scratch_elems[wi] = (int64_t)E.ndense_sp[3][wi] * ((L.rcap + 15) / 16) * (W + 1) * W * W * 16;
    }
    return L;
}

// Point the engine's descriptors and problem records at workspace buffers of
// layout L (grids, per-window products, close-pair sums, RHS staging, dense
// spread blocks).  Host-side only: the descriptors still need an upload.
void engine_bind_ws(Engine &E, const WsLayout &L, void *ws, void *yw, double *nys, void *vpack, void *scr0,
                    void *scr1)
{
    const size_t cs = 2 * real_size(E.precision);
    E.ws = ws;
    E.ws_bytes = L.grid_bytes + L.nys_bytes + L.vpack_bytes +
                 (L.scratch_elems[0] + L.scratch_elems[1]) * (int64_t)real_size(E.precision);
    E.yw = yw;
    E.yw_bytes = L.y_bytes;
    E.d_near_ys = nys;
    E.vpack = vpack;
    E.vpack_bytes = L.vpack_bytes;
    E.vpack_ld = L.vpack_ld;
    E.scratch[0] = L.scratch_elems[0] > 0 ? scr0 : nullptr;
    E.scratch[1] = L.scratch_elems[1] > 0 ? scr1 : nullptr;
    E.scratch_cap[0] = E.scratch[0] ? L.scratch_elems[0] : 0;
    E.scratch_cap[1] = E.scratch[1] ? L.scratch_elems[1] : 0;
    int64_t off = 0;
    for (size_t p = 0; p < E.probs.size(); ++p) {
        E.probs[p].Vp = (const char *)vpack + off * real_size(E.precision);
        E.probs[p].ldvp = L.vpack_ld;
        off += E.probs[p].N * L.vpack_ld;
    }
    char *p = (char *)ws, *yp = (char *)yw;
    double *q = nys;
    for (WinDev &w : E.wdev) {
        auto take = [&](int64_t n) {
            void *r = p;
            p += n * cs;
            return r;
        };
        w.G = take(L.cap * w.szG);
        w.A1 = take(L.cap * w.szA1);
        w.A2 = take(L.cap * w.szA2);
        w.A3 = take(2 * L.cap * w.szA3);
        w.A4 = take(2 * L.cap * w.szA4);
        w.H = take(2 * L.cap * w.szH);
        w.Vm = take(L.cap * w.szM);
        w.Gm = take(L.cap * w.szM);
        w.npair_cap = L.cap;
        w.Rcap = L.rcap;
        w.Yw = yp;
        yp += 2 * L.rcap * w.N * (int64_t)real_size(E.precision);
        w.nf_ys = w.nf ? q : nullptr;
        q += w.nf ? 2 * w.N : 0;
    }
    E.npair_cap = L.cap;
    E.rcap = L.rcap;
    E.dirty = true;
}

// Allocate grids for at least ceil(R/2) complex grids per window and the FP64
// per-window products for R right-hand sides; upload the descriptors.
addk_status engine_ensure_workspace(Engine &E, int R)
{
    const int npair = (R + 1) / 2;
    const bool grow = npair > E.npair_cap || R > E.rcap || !E.ws;
    if (!grow)
        return E.dirty ? engine_upload(E) : ADDK_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceSynchronize");
    const WsLayout L = engine_ws_layout(E, std::max(npair, E.npair_cap), std::max<int64_t>(R, E.rcap));
    free_dev(E.ws);
    free_dev(E.yw);
    free_dev(E.d_near_ys);
    free_dev(E.vpack);
    free_dev(E.scratch[0]);
    free_dev(E.scratch[1]);
    E.ws = E.yw = nullptr;
    E.d_near_ys = nullptr;
    E.vpack = E.scratch[0] = E.scratch[1] = nullptr;
    void *ws = nullptr, *vp = nullptr, *scr[2] = {nullptr, nullptr};
    void *yw = nullptr;
    double *nys = nullptr;
    auto release = [&]() {
        free_dev(ws);
        free_dev(yw);
        free_dev(nys);
        free_dev(vp);
        free_dev(scr[0]);
        free_dev(scr[1]);
    };
    if (hipMalloc(&ws, L.grid_bytes) != hipSuccess) {
        release();
        set_error("workspace allocation of " + std::to_string(L.grid_bytes) + " bytes failed");
        return ADDK_ERR_OOM;
    }
    if (hipMalloc(&yw, L.y_bytes) != hipSuccess) {
        release();
        set_error("per-window product buffer allocation failed");
        return ADDK_ERR_OOM;
    }
    // close-pair sums of the near-field windows by sorted position, cleared here
    // once and by every pass that reads them
    if (L.nys_bytes > 0) {
        e = hipMalloc(&nys, L.nys_bytes);
        if (e == hipSuccess)
            e = hipMemset(nys, 0, L.nys_bytes);
        if (e != hipSuccess) {
            release();
            return hip_fail(e, "near-field sum buffer");
        }
    }
    // point-major copy of the right-hand sides of every problem
    if (hipMalloc(&vp, L.vpack_bytes) != hipSuccess) {
        release();
        set_error("right-hand side staging allocation failed");
        return ADDK_ERR_OOM;
    }
    // per-item blocks of the d = 3 dense spread (either kernel), in the engine's
    // precision: items x RHS blocks x (2m + 1) (2m)^2 x 16
    for (int wi = 0; wi < 2; ++wi)
        if (L.scratch_elems[wi] > 0 && hipMalloc(&scr[wi], L.scratch_elems[wi] * (int64_t)real_size(E.precision)) !=
                                           hipSuccess) {
            release();
            set_error("dense spread scratch allocation failed");
            return ADDK_ERR_OOM;
        }
    engine_bind_ws(E, L, ws, yw, nys, vp, scr[0], scr[1]);
    return engine_upload(E);
}

// Upload the window descriptors (after workspace or parameter changes).  Synchronous.
addk_status engine_upload(Engine &E)
{
    hipError_t e;
    if (!E.d_wins) {
        e = hipMalloc(&E.d_wins, std::max<size_t>(1, E.wdev.size()) * sizeof(WinDev));
        if (e != hipSuccess)
            return hip_fail(e, "hipMalloc(descriptors)");
    }
    if (!E.wdev.empty()) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess)
            return hip_fail(e, "hipDeviceSynchronize");
        e = hipMemcpy(E.d_wins, E.wdev.data(), E.wdev.size() * sizeof(WinDev), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return hip_fail(e, "hipMemcpy(descriptors)");
    }
    E.dirty = false;
    return ADDK_OK;
}

template <typename real, int D, int RB>
static void launch_spread_rb(Engine &E, int R, IoArgs io, hipStream_t st)
{
    const size_t sh = ((size_t)RB * E.maxvol[D] + 16 * D * kMaxW) * sizeof(real);
    dim3 grid(E.nchunks[D], (R + RB - 1) / RB);
    hipLaunchKernelGGL((k_spread<real, D, RB>), grid, dim3(kBlock), sh, st, E.d_wins, E.d_chunks[D], io, R);
}

template <typename real, int D, int RB>
static void launch_interp_rb(Engine &E, int R, int nout, hipStream_t st)
{
    const size_t sh = ((size_t)RB * E.maxvol[D] + 16 * D * kMaxW) * sizeof(real);
    dim3 grid(E.nchunks_i[D], (R + RB - 1) / RB, nout);
    hipLaunchKernelGGL((k_interp<real, D, RB>), grid, dim3(kBlock), sh, st, E.d_wins, E.d_chunks_i[D], R);
}

static int rb_for(const Engine &E, int D, int R)
{
    int rb = 1;
    while (rb < R && rb < E.rb[D])
        rb <<= 1;
    return rb;
}

template <typename real, int D>
static void launch_spread(Engine &E, int R, IoArgs io, hipStream_t st)
{
    switch (rb_for(E, D, R)) {
    case 1: launch_spread_rb<real, D, 1>(E, R, io, st); break;
    case 2: launch_spread_rb<real, D, 2>(E, R, io, st); break;
    case 4: launch_spread_rb<real, D, 4>(E, R, io, st); break;
    case 8: launch_spread_rb<real, D, 8>(E, R, io, st); break;
    default: launch_spread_rb<real, D, 16>(E, R, io, st); break;
    }
}

template <typename real, int D>
static void launch_interp(Engine &E, int R, int nout, hipStream_t st)
{
    switch (rb_for(E, D, R)) {
    case 1: launch_interp_rb<real, D, 1>(E, R, nout, st); break;
    case 2: launch_interp_rb<real, D, 2>(E, R, nout, st); break;
    case 4: launch_interp_rb<real, D, 4>(E, R, nout, st); break;
    case 8: launch_interp_rb<real, D, 8>(E, R, nout, st); break;
    default: launch_interp_rb<real, D, 16>(E, R, nout, st); break;
    }
}

template <typename real, int AXIS, int MODE>
static void launch_fft(Engine &E, int st_id, int ny, FftCall call, hipStream_t st)
{
    if (!E.ngroups[st_id] || ny <= 0)
        return;
    constexpr int LF = sizeof(real) == 4 ? 16 : 8;  // lines per block for grids up to 128 points
    call.nos_lds = E.nos_max;
    // twiddles and the line buffers: two for a plain pass, a third for the
    // inverse transforms of the fused pass (more blocks per CU without it)
    const size_t nbuf = MODE == 2 ? 3 : 2;
    const size_t sh = ((size_t)E.nos_max / 2 + nbuf * (size_t)E.fft_L * E.nos_max) * sizeof(cpx<real>);
    if (E.fft_L == LF)
        hipLaunchKernelGGL((k_fft<real, AXIS, MODE, LF>), dim3(E.ngroups[st_id], ny), dim3(kBlock), sh, st, E.d_wins,
                           E.d_groups[st_id], call);
    else
        hipLaunchKernelGGL((k_fft<real, AXIS, MODE, LF / 2>), dim3(E.ngroups[st_id], ny), dim3(kBlock), sh, st,
                           E.d_wins, E.d_groups[st_id], call);
}

template <typename real>
static addk_status run_t(Engine &E, int R, int nout, int modes_sel, bool interp, IoArgs io, hipStream_t st)
{
    E.fused_no = 0;
    const int npair = (R + 1) / 2;
    const int nw = (int)E.wdev.size();
    if (nw == 0)
        return ADDK_OK;
    {
        StageTimer t(E, PS_ZERO, st);
        hipLaunchKernelGGL(k_zero_grids<real>, dim3(64, nw), dim3(kBlock), 0, st, E.d_wins, npair);
        int64_t maxN = io.table ? 0 : io.single.N;
        for (const ProbDev &p : E.probs)
            maxN = std::max(maxN, p.N);
        const int bx = (int)std::max<int64_t>(1, std::min<int64_t>((maxN + 63) / 64, 16384));
        hipLaunchKernelGGL(k_pack_v<real>, dim3(bx, io.table ? E.nprob : 1), dim3(kBlock), 0, st, io, R);
    }
    for (int d = 1; d <= 3; ++d) {
        if (!E.nchunks[d])
            continue;
        StageTimer t(E, PS_SPREAD, st);
        if (d == 3 && E.sparse_gather && !E.no_mfma && !(E.knobs & ADDK_KNOB_SPARSE_ATOMIC)) {
            launch_spread_sparse_mfma(E, R, io, st);
            continue;
        }
        if (launch_spread_tile(E, d, R, io, st))
            continue;
        if (d == 1) launch_spread<real, 1>(E, R, io, st);
        if (d == 2) launch_spread<real, 2>(E, R, io, st);
        if (d == 3) launch_spread<real, 3>(E, R, io, st);
    }
    for (int d = 1; d <= 3; ++d)
        for (int wi = 0; wi < 2; ++wi) {
            if (!E.ndense_sp[d][wi])
                continue;
            if (d == 3 && E.scratch[wi]) {  // per-item blocks, then the gather
                {
                    StageTimer t(E, PS_SPREAD_DENSE, st);
                    if (!(use_mfma(E, ADDK_KNOB_SPREAD_MFMA, R) && launch_spread_mfma(E, wi, R, io, st)))
                        launch_spread_dense(E, d, wi, R, io, st);
                }
                StageTimer t(E, PS_GATHER, st);
                launch_gather_blocks(E, wi, R, st);
                continue;
            }
            StageTimer t(E, PS_SPREAD_DENSE, st);
            launch_spread_dense(E, d, wi, R, io, st);
        }
    FftCall fc{E.nos_max, npair, nout, modes_sel};
    if (E.ngroups[ST_FWD0]) {
        StageTimer t(E, PS_FFT_X_FWD, st);
        launch_fft<real, 0, 0>(E, ST_FWD0, npair, fc, st);
    }
    if (E.ngroups[ST_FWD1]) {
        StageTimer t(E, PS_FFT_Y_FWD, st);
        launch_fft<real, 1, 0>(E, ST_FWD1, npair, fc, st);
    }
    if (E.ngroups[ST_FUSED2]) {
        StageTimer t(E, PS_FFT_FUSED, st);
        launch_fft<real, 2, 2>(E, ST_FUSED2, npair, fc, st);
    }
    if (E.ngroups[ST_FUSED1]) {
        StageTimer t(E, PS_FFT_FUSED, st);
        launch_fft<real, 1, 2>(E, ST_FUSED1, npair, fc, st);
    }
    if (E.ngroups[ST_FUSED0]) {
        StageTimer t(E, PS_FFT_FUSED, st);
        launch_fft<real, 0, 2>(E, ST_FUSED0, npair, fc, st);
    }
    if (nout > 0) {
        if (E.ngroups[ST_INV1]) {
            StageTimer t(E, PS_FFT_Y_INV, st);
            launch_fft<real, 1, 1>(E, ST_INV1, npair * nout, fc, st);
        }
        if (E.ngroups[ST_INV0]) {
            StageTimer t(E, PS_FFT_X_INV, st);
            launch_fft<real, 0, 1>(E, ST_INV0, npair * nout, fc, st);
        }
        if (interp) {
            // all-d = 1 plans: the interpolation runs in the window sum (engine_combine)
            const bool fuse = E.fused_d1 && !io.table;
            if (fuse)
                E.fused_no = nout;
            for (int d = 1; d <= 3; ++d) {
                if (!E.nchunks_i[d] || (fuse && d == 1))
                    continue;
                StageTimer t(E, PS_INTERP, st);
                if (d == 3 && use_mfma(E, ADDK_KNOB_INTERP_TILE_MFMA, R) && launch_interp_tile_mfma(E, R, nout, st))
                    continue;
                if (d == 1) launch_interp<real, 1>(E, R, nout, st);
                if (d == 2) launch_interp<real, 2>(E, R, nout, st);
                if (d == 3) launch_interp<real, 3>(E, R, nout, st);
            }
            for (int d = 1; d <= 3; ++d)
                for (int wi = 0; wi < 2; ++wi) {
                    if (!E.ndense[d][wi] || (fuse && d == 1))
                        continue;
                    StageTimer t(E, PS_INTERP_DENSE, st);
                    if (d == 3 && use_mfma(E, ADDK_KNOB_INTERP_DENSE_MFMA, R) && launch_interp_mfma(E, wi, R, nout, st))
                        continue;
                    launch_interp_dense(E, d, wi, R, nout, st);
                }
            if (E.nnear[1] || E.nnear[2] || E.nnear[3]) {
                StageTimer t(E, PS_NEAR, st);
                launch_near(E, R, nout, io, st);
            }
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "stage kernel launch");
    return ADDK_OK;
}

// Matrix-core variant of a stage: off with ADDK_VECTOR_ALU_ONLY; FP64 engines
// have them with R >= 2 only; otherwise the knob decides, and untuned engines
// also require the stage's fewest RHS (kMfmaMinR*).
bool use_mfma(const Engine &E, uint32_t knob, int R)
{
    if (E.no_mfma || !(E.knobs & knob))
        return false;
    if (E.precision != ADDK_FP32 && R == 1)
        return false;
    const int rmin = knob == ADDK_KNOB_SPREAD_MFMA       ? kMfmaMinRSpread
                     : knob == ADDK_KNOB_INTERP_TILE_MFMA ? kMfmaMinRInterpTile
                                                          : kMfmaMinRInterpDense;
    // one RHS: the dense variants with the z-slabs as columns
    return E.tuned || R >= rmin || (knob != ADDK_KNOB_INTERP_TILE_MFMA && R == 1);
}

addk_status engine_run(Engine &E, int R, int nout, bool vmodes_only, bool store_gmodes, IoArgs io, hipStream_t st)
{
    addk_status s = engine_ensure_workspace(E, R);
    if (s != ADDK_OK)
        return s;
    return engine_run_bound(E, R, nout, vmodes_only, store_gmodes, io, st);
}

// Tuning cache (see addk_internal.h).
namespace {
struct TuneKey {
    int dev, dmask, nos, m, R, nbucket, precision, nout;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(dev, dmask, nos, m, R, nbucket, precision, nout) <
               std::tie(o.dev, o.dmask, o.nos, o.m, o.R, o.nbucket, o.precision, o.nout);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, uint32_t> g_tune;

TuneKey tune_key(const Engine &E, int R, int nout)
{
    TuneKey k{};
    (void)hipGetDevice(&k.dev);
    int64_t n = 0;
    for (const WinDev &w : E.wdev) {
        k.dmask |= 1 << w.d;
        k.nos = std::max(k.nos, w.nos);
        k.m = std::max(k.m, w.m);
        n = std::max(n, w.N);
    }
    while ((int64_t(1) << (k.nbucket + 1)) <= n)  // the power of two at or below N
        ++k.nbucket;
    k.R = R;
    k.precision = E.precision;
    k.nout = nout;
    return k;
}
}  // namespace

bool tune_cache_get(const Engine &E, int R, int nout, uint32_t *knobs)
{
    const TuneKey k = tune_key(E, R, nout);
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(k);
    if (it == g_tune.end())
        return false;
    *knobs = it->second;
    return true;
}

void tune_cache_put(const Engine &E, int R, int nout, uint32_t knobs)
{
    const TuneKey k = tune_key(E, R, nout);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[k] = knobs;
}

void tune_cache_clear()
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.clear();
}

// engine_run on the workspace already bound and uploaded (room for R RHS).  A
// plan's engine that was not tuned itself runs with the knobs the tuning cache
// holds for its shape, if any.
addk_status engine_run_bound(Engine &E, int R, int nout, bool vmodes_only, bool store_gmodes, IoArgs io,
                             hipStream_t st)
{
    const int modes_sel = vmodes_only ? 1 : (store_gmodes ? 2 : 0);
    const int no = vmodes_only ? 0 : nout;
    if (!io.table) {
        io.single.Vp = E.vpack;
        io.single.ldvp = E.vpack_ld;
    }
    const uint32_t knobs0 = E.knobs;
    const bool tuned0 = E.tuned;
    uint32_t kc = 0;
    if (!E.tuned && !io.table && tune_cache_get(E, R, nout, &kc)) {
        E.knobs = kc;
        E.tuned = true;
    }
    const addk_status s = E.precision == ADDK_FP32 ? run_t<float>(E, R, no, modes_sel, !vmodes_only, io, st)
                                                   : run_t<double>(E, R, no, modes_sel, !vmodes_only, io, st);
    E.knobs = knobs0;
    E.tuned = tuned0;
    return s;
}

addk_status engine_combine(Engine &E, int R, int mode, IoArgs io, hipStream_t st)
{
    if (E.wdev.empty())
        return ADDK_OK;
    int64_t maxN = 0;
    for (const ProbDev &p : E.probs)
        maxN = std::max(maxN, p.N - p.yoff);
    if (!io.table)
        maxN = io.single.N - io.single.yoff;
    if (maxN <= 0 || R == 0)
        return ADDK_OK;
    const int ny = io.table ? E.nprob : 1;
    StageTimer t(E, PS_COMBINE, st);
    if (E.fused_no > 0 && !io.table) {  // the d = 1 interpolation the last run left to the sum
        const int no = E.fused_no;
        E.fused_no = 0;
        launch_interp_combine_d1(E, R, no, mode, io, st);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? ADDK_OK : hip_fail(e, "fused interp and window sum launch");
    }
    if (R <= kCombineRowsMaxR) {
        const int bx1 = (int)std::min<int64_t>((maxN + kBlock - 1) / kBlock, 16384);
        if (E.precision == ADDK_FP32)
            hipLaunchKernelGGL(k_combine_rows<float>, dim3(bx1, ny), dim3(kBlock), 0, st, E.d_wins, io, R, mode);
        else
            hipLaunchKernelGGL(k_combine_rows<double>, dim3(bx1, ny), dim3(kBlock), 0, st, E.d_wins, io, R, mode);
    } else {
        const int bx = (int)std::min<int64_t>((maxN + 63) / 64, 16384);
        if (E.precision == ADDK_FP32)
            hipLaunchKernelGGL(k_combine<float>, dim3(bx, ny), dim3(kBlock), 0, st, E.d_wins, io, R, mode);
        else
            hipLaunchKernelGGL(k_combine<double>, dim3(bx, ny), dim3(kBlock), 0, st, E.d_wins, io, R, mode);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "combine launch");
    return ADDK_OK;
}

// grad outputs: d_out_ell[w], d_out_sig[w] for every window (device pointers, may be null)
addk_status engine_mode_dot(Engine &E, int npair, double *grad_ell, double *grad_sig, hipStream_t st)
{
    const int nblk = 256;
    const int64_t need = (int64_t)2 * nblk * std::max<int64_t>(1, (int64_t)E.wdev.size());
    if (E.partial_cap < need) {
        free_dev(E.d_partial);
        E.d_partial = nullptr;
        hipError_t e = hipMalloc(&E.d_partial, need * sizeof(double));
        if (e != hipSuccess)
            return hip_fail(e, "hipMalloc(partials)");
        E.partial_cap = need;
    }
    StageTimer t(E, PS_MODE_DOT, st);
    for (int wi = 0; wi < (int)E.wdev.size(); ++wi) {
        double *part = E.d_partial + (int64_t)2 * nblk * wi;
        if (E.precision == ADDK_FP32)
            hipLaunchKernelGGL(k_mode_dot<float>, dim3(nblk), dim3(kBlock), 0, st, E.d_wins, wi, npair, part);
        else
            hipLaunchKernelGGL(k_mode_dot<double>, dim3(nblk), dim3(kBlock), 0, st, E.d_wins, wi, npair, part);
        hipLaunchKernelGGL(k_mode_dot_finish, dim3(1), dim3(64), 0, st, E.d_wins, wi, nblk, part,
                           grad_ell ? grad_ell + E.wlocal[wi] : nullptr, grad_sig ? grad_sig + E.wlocal[wi] : nullptr);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_fail(e, "mode-dot launch");
    return ADDK_OK;
}

}  // namespace addk
