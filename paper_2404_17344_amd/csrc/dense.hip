// Spreading and interpolation for densely populated grid cells.
//
// Points are sorted by their base cell (the first of the (2m)^d grid cells a
// point touches).  A cell that holds many points contributes, for each of its
// points, to the same (2m)^d block of grid cells.  These kernels exploit that:
//
//  * spread: the threads of a block own grid cells of that block (one x-y
//    column of taps each, all z taps held in registers, for a few RHS) and
//    loop over the cell's points, whose window values and RHS entries are
//    staged in LDS and read by every thread alike.  Accumulation is in
//    registers; each thread adds its column to the global grid once.
//  * interp: the block first copies the (2m)^d block of grid values for a set
//    of RHS into LDS ([cell][rhs] layout), then every lane takes one point and
//    all lanes walk the taps in the same order, so each LDS read is a
//    broadcast of one address.
//
// Cells with few points use the tile kernels in kernels.hip instead.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "addk_internal.h"

namespace addk {

template <typename real>
__device__ __forceinline__ real kb_psi_d(real z, real m, real b, real inv_e2bm)
{
    const real z2 = z * z;
    real s2 = m * m - z2;
    s2 = s2 > real(1e-12) ? s2 : real(1e-12);
    const real s = sqrt(s2);
    return m * exp(-b * z2 / (s + m)) * (real(1) - exp(real(-2) * b * s)) * inv_e2bm / s;
}

// FP32: the exponent b (s - m) is formed as -b z^2 / (s + m), which is small
// and accurate where psi is large; hardware sqrt, exp2 and reciprocal (about
// 1 ulp each) are ample for the FP32 path.
template <>
__device__ __forceinline__ float kb_psi_d<float>(float z, float m, float b, float inv_e2bm)
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

// Dense item anchor: base cell (bx, by, bz) and the number of cells in z
// (1, or 2 for two z-adjacent dense cells sharing one item, d = 3).
__device__ __forceinline__ void unpack_cell(int packed, int &bx, int &by, int &bz, int &nzc)
{
    bx = packed & 1023;
    by = (packed >> 10) & 1023;
    bz = (packed >> 20) & 1023;
    nzc = ((packed >> 30) & 1) + 1;
}

__device__ __forceinline__ ProbDev get_prob_d(const IoArgs &io, int p) { return io.table ? io.table[p] : io.single; }

__device__ __forceinline__ void gadd(gptr<float> p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gadd(gptr<double> p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cells of a dense item's window block: (2m)^d, with one more z layer for the
// two-cell items of d = 3.  Shared by the interp kernel and its launcher.
template <int D, int W>
constexpr int dense_block_cells()
{
    return D == 3 ? W * W * (W + 1) : (D == 2 ? W * W : W);
}

// ---------------------------------------------------------------------------
// spread, dense cells.  blockDim.x = OUT * NRG threads; thread (q, rg) owns
// outer tap q and RHS rg*RT .. rg*RT+RT-1 of the block's RHS range.  The block
// is added to the grid with atomics, or (d = 3, scratch given) stored into the
// item's scratch slots for k_gather_blocks: slot item * nrb + r / 16 holds
// [oz][oy][ox][r % 16] over the 2m + 1 slabs, the layout of the matrix-core
// spread, with rows of 16 RHS (one when R = 1: rw) (the atomics are executed
// beyond L2 on this chip and are slow).
// Blocks hold at most 4 RHS groups of OUT threads (see spread_dense_w): the
// bound lets d = 3 keep its (2m + 1) x RT accumulators in registers.
template <typename real, int D, int W, int RT>
__global__ __launch_bounds__(D == 3 ? W * W * 4 : 256) void k_spread_dense(const WinDev *__restrict__ wins,
                                                                           const Chunk *__restrict__ items, IoArgs io,
                                                                           int R, int NRG, real *__restrict__ scratch,
                                                                           int nrb, int rw)
{
    constexpr int OUT = D == 3 ? W * W : W;  // taps owned by thread groups
    constexpr int IN = D == 1 ? 1 : W;       // taps accumulated per thread (last dimension)
    constexpr int IN2 = D == 3 ? W + 1 : IN; // z accumulators (items of two z cells, d = 3)
    constexpr int PB = 32;                   // points staged per round
    __shared__ real pw[PB][D][W];
    __shared__ real pv[PB][16];
    __shared__ int pdz[PB];                  // z cell of the point inside the item (d = 3)

    const Chunk it = items[blockIdx.x];
    const WinDev &w = wins[it.win];
    const int RBB = RT * NRG;
    const int r0 = blockIdx.y * RBB;
    if (r0 >= R)
        return;
    const int t = threadIdx.x;
    const int q = t % OUT, rg = t / OUT;
    const int ox = D == 3 ? q % W : q;
    const int oy = D == 3 ? q / W : 0;
    int bx, by, bz, nzc;
    unpack_cell(it.tile, bx, by, bz, nzc);
    const int bb[3] = {bx, by, bz};
    const gptr<const real> coords = gbl((const real *)w.coords);
    const ProbDev pio = get_prob_d(io, w.prob);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;

    real acc[IN2][RT];
#pragma unroll
    for (int k = 0; k < IN2; ++k)
#pragma unroll
        for (int i = 0; i < RT; ++i)
            acc[k][i] = real(0);

    for (int p0 = 0; p0 < it.count; p0 += PB) {
        const int np = min(PB, it.count - p0);
        for (int e = t; e < np * D * W; e += blockDim.x) {
            const int p = e / (D * W), rem = e - p * (D * W);
            const int dd = rem / W, o = rem - dd * W;
            const real u = coords[dd * w.N + it.start + p0 + p];
            // z weights relative to the point's own base cell (bz or bz + 1)
            const int dz = (D == 3 && dd == 2) ? (int)floor(u) - w.m + 1 - bz : 0;
            pw[p][dd][o] = kb_psi_d(u - (real)(bb[dd] + dz + o), mm, kb, ie);
            if (D == 3 && dd == 2 && o == 0)
                pdz[p] = dz;
        }
        for (int e = t; e < np * RBB; e += blockDim.x) {
            const int p = e / RBB, i = e - p * RBB;
            const int r = r0 + i;
            const int orig = gbl(w.perm)[it.start + p0 + p];
            pv[p][i] = r < R ? gbl((const real *)pio.Vp)[orig * pio.ldvp + r] : real(0);
        }
        __syncthreads();
        for (int p = 0; p < np; ++p) {
            const real wo = D == 3 ? pw[p][0][ox] * pw[p][D > 1 ? 1 : 0][oy] : pw[p][0][ox];
            real vv[RT];
#pragma unroll
            for (int i = 0; i < RT; ++i)
                vv[i] = pv[p][rg * RT + i];
            if (D == 1) {
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    acc[0][i] += wo * vv[i];
            } else if (D == 3 && pdz[p] != 0) {  // the item's second z cell
#pragma unroll
                for (int k = 0; k < IN; ++k) {
                    const real wt = wo * pw[p][D - 1][k];
#pragma unroll
                    for (int i = 0; i < RT; ++i)
                        acc[k + (D == 3 ? 1 : 0)][i] += wt * vv[i];
                }
            } else {
#pragma unroll
                for (int k = 0; k < IN; ++k) {
                    const real wt = wo * pw[p][D - 1][k];
#pragma unroll
                    for (int i = 0; i < RT; ++i)
                        acc[k][i] += wt * vv[i];
                }
            }
        }
        __syncthreads();
    }

    const gptr<real> G = gbl((real *)w.G);
    const int ex = w.ext[0], ey = w.ext[1];
#pragma unroll
    for (int k = 0; k < IN2; ++k) {
        if (k >= IN + nzc - 1)
            break;
        int x, y, z;
        if (D == 3) {
            x = bx + ox;
            y = by + oy;
            z = bz + k;
        } else if (D == 2) {
            x = bx + ox;
            y = by + k;
            z = 0;
        } else {
            x = bx + ox;
            y = 0;
            z = 0;
        }
        const int64_t cell = ((int64_t)z * ey + y) * ex + x;
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int r = r0 + rg * RT + i;
            if (D == 3 && scratch != nullptr) {
                if (r < R)
                    scratch[(((int64_t)blockIdx.x * nrb + (r >> 4)) * ((W + 1) * W * W) + (k * W + oy) * W + ox) * rw +
                            (r & 15)] = acc[k][i];
            } else if (r < R)
                gadd(&G[((int64_t)(r >> 1) * w.szG + cell) * 2 + (r & 1)], acc[k][i]);
        }
    }
}

// ---------------------------------------------------------------------------
// interp, dense cells.  One lane per point; the (2m)^d block of grid values of
// the cell is staged in LDS as [cell][RB].
template <typename real, int D, int W, int RB>
__global__ __launch_bounds__(kBlock) void k_interp_dense(const WinDev *__restrict__ wins, const Chunk *__restrict__ items,
                                                         int R)
{
    constexpr int NC = dense_block_cells<D, W>();  // block cells (max)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real *sub = (real *)smem_raw;

    const Chunk it = items[blockIdx.x];
    const WinDev &w = wins[it.win];
    const int r0 = blockIdx.y * RB;
    if (r0 >= R)
        return;
    const int o = blockIdx.z;
    const int nr = min(RB, R - r0);
    int bx, by, bz, nzc;
    unpack_cell(it.tile, bx, by, bz, nzc);
    const int ncell = D == 3 ? W * W * (W + nzc - 1) : NC;  // the item's block (z cells bz .. bz + W + nzc - 2)

    const gptr<const real> H = gbl((const real *)w.H);
    const int ex = w.ext[0], ey = w.ext[1];
    const int np = (nr + 1) >> 1;
    const int p0 = r0 >> 1;
    for (int idx = threadIdx.x; idx < np * ncell; idx += kBlock) {
        const int pi = idx / ncell, c = idx - pi * ncell;
        const int cx = c % W, cy = D > 1 ? (c / W) % W : 0, cz = D > 2 ? c / (W * W) : 0;
        const int64_t off =
            ((int64_t)(o * w.npair_cap + p0 + pi) * w.szH + ((int64_t)(bz + cz) * ey + by + cy) * ex + bx + cx) * 2;
        sub[c * RB + 2 * pi] = H[off];
        if (2 * pi + 1 < RB)
            sub[c * RB + 2 * pi + 1] = H[off + 1];
    }
    __syncthreads();

    const int p = threadIdx.x;
    if (p >= it.count)
        return;
    const int j = it.start + p;
    const gptr<const real> coords = gbl((const real *)w.coords);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    const real ux = coords[j];
    real wy[W], wz[W];
    if (D > 1) {
        const real uy = coords[w.N + j];
#pragma unroll
        for (int k = 0; k < W; ++k)
            wy[k] = kb_psi_d(uy - (real)(by + k), mm, kb, ie);
    }
    int dz = 0;  // z cell of the point inside the item
    if (D > 2) {
        const real uz = coords[2 * w.N + j];
        dz = (int)floor(uz) - w.m + 1 - bz;
#pragma unroll
        for (int k = 0; k < W; ++k)
            wz[k] = kb_psi_d(uz - (real)(bz + dz + k), mm, kb, ie);
    }
    const real *subz = sub + (D > 2 ? dz * W * W * RB : 0);  // the point's own z window
    real acc[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
        acc[i] = real(0);
    for (int ox = 0; ox < W; ++ox) {
        const real wxo = kb_psi_d(ux - (real)(bx + ox), mm, kb, ie);
        if (D == 1) {
            const real *s = sub + ox * RB;
#pragma unroll
            for (int i = 0; i < RB; ++i)
                acc[i] += wxo * s[i];
        } else if (D == 2) {
#pragma unroll
            for (int oy = 0; oy < W; ++oy) {
                const real wt = wxo * wy[oy];
                const real *s = sub + (ox + W * oy) * RB;
#pragma unroll
                for (int i = 0; i < RB; ++i)
                    acc[i] += wt * s[i];
            }
        } else {
            // the next tap's grid values are loaded before the current tap's FMAs
            real cur[RB], nxt[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                cur[i] = subz[ox * RB + i];
#pragma unroll
            for (int oy = 0; oy < W; ++oy) {
                const real wxy = wxo * wy[oy];
#pragma unroll
                for (int oz = 0; oz < W; ++oz) {
                    const int tn = oy * W + oz + 1;  // next tap in (oy, oz) order
                    if (tn < W * W) {
                        const real *s = subz + (ox + W * ((tn / W) + W * (tn % W))) * RB;
#pragma unroll
                        for (int i = 0; i < RB; ++i)
                            nxt[i] = s[i];
                    }
                    const real wt = wxy * wz[oz];
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        acc[i] += wt * cur[i];
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        cur[i] = nxt[i];
                }
            }
        }
    }
    const int orig = gbl(w.perm)[j];
    const gptr<real> dst = gbl((real *)w.Yw) + ((int64_t)o * w.N + orig) * w.Rcap + r0;
#pragma unroll
    for (int i = 0; i < RB; ++i)
        if (i < nr)
            dst[i] = acc[i];
}

// ---------------------------------------------------------------------------
// d = 1, dense cells.  With 2m taps per point the work per point is small and
// these kernels are bound by the bytes they move: the RHS rows of the spread
// (a point-major row of 16 values, gathered through the permutation) and the
// interpolated rows (written back through it).  Four lanes share a point, each
// taking four of its 16 RHS, so that a point's row is one contiguous 64-byte
// (FP32) access of the four lanes; each lane evaluates W/4 of the point's
// window values and the four lanes exchange them within their quad.

// value of lane (lane & ~3) + K, K = 0..3, within a quad (a DPP quad
// permutation: a register move, no LDS)
template <int K>
__device__ __forceinline__ float quad_bcast(float v)
{
    constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xf, 0xf, false));
}

template <int K>
__device__ __forceinline__ double quad_bcast(double v)
{
    constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);
    const int2 b = *reinterpret_cast<int2 *>(&v);
    int2 r;
    r.x = __builtin_amdgcn_mov_dpp(b.x, ctrl, 0xf, 0xf, false);
    r.y = __builtin_amdgcn_mov_dpp(b.y, ctrl, 0xf, 0xf, false);
    return *reinterpret_cast<double *>(&r);
}

// the W window values of a quad's point, lane k of the quad holding values
// k WQ .. k WQ + WQ - 1 in wq
template <int W, typename real>
__device__ __forceinline__ void quad_gather(const real (&wq)[W / 4], real (&wv)[W])
{
    constexpr int WQ = W / 4;
#pragma unroll
    for (int k = 0; k < WQ; ++k) {
        wv[k] = quad_bcast<0>(wq[k]);
        wv[WQ + k] = quad_bcast<1>(wq[k]);
        wv[2 * WQ + k] = quad_bcast<2>(wq[k]);
        wv[3 * WQ + k] = quad_bcast<3>(wq[k]);
    }
}

template <typename real>
__device__ __forceinline__ void load4(const real *p, real (&v)[4])
{
    if constexpr (sizeof(real) == 4) {
        const float4 t = *(const float4 *)p;
        v[0] = t.x, v[1] = t.y, v[2] = t.z, v[3] = t.w;
    } else {
        const double2 a = *(const double2 *)p, b = *(const double2 *)(p + 2);
        v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y;
    }
}

template <typename real>
__device__ __forceinline__ void store4(real *p, const real (&v)[4])
{
    if constexpr (sizeof(real) == 4) {
        *(float4 *)p = float4{v[0], v[1], v[2], v[3]};
    } else {
        *(double2 *)p = double2{v[0], v[1]};
        *(double2 *)(p + 2) = double2{v[2], v[3]};
    }
}

// the same for device memory (global loads and stores)
__device__ __forceinline__ void load4(gptr<const float> p, float (&v)[4])
{
    typedef float n4 __attribute__((ext_vector_type(4)));
    const n4 t = *(gptr<const n4>)p;
    v[0] = t.x, v[1] = t.y, v[2] = t.z, v[3] = t.w;
}
__device__ __forceinline__ void load4(gptr<const double> p, double (&v)[4])
{
    typedef double n2 __attribute__((ext_vector_type(2)));
    const n2 a = *(gptr<const n2>)p, b = *(gptr<const n2>)(p + 2);
    v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y;
}
__device__ __forceinline__ void store4(gptr<float> p, const float (&v)[4])
{
    typedef float n4 __attribute__((ext_vector_type(4)));
    *(gptr<n4>)p = n4{v[0], v[1], v[2], v[3]};
}
__device__ __forceinline__ void store4(gptr<double> p, const double (&v)[4])
{
    typedef double n2 __attribute__((ext_vector_type(2)));
    *(gptr<n2>)p = n2{v[0], v[1]};
    *(gptr<n2>)(p + 2) = n2{v[2], v[3]};
}

// Spread: one block (256 threads) per dense item (<= kSpreadChunk points of one
// base cell) and 16 RHS.  Thread (slot = t / 4, rq = t % 4) accumulates the
// item's W x 4 block (taps x its RHS) over points slot, slot + 64, ...; the
// 64 slots are then summed (shuffles within the wave, LDS across waves) and
// the W x 16 block is added to the grid.
template <typename real, int W>
__global__ __launch_bounds__(kBlock) void k_spread_dense1(const WinDev *__restrict__ wins,
                                                          const Chunk *__restrict__ items, IoArgs io, int R)
{
    constexpr int WQ = W / 4;  // window values evaluated per lane
    __shared__ real red[4][W][16];
    const Chunk it = items[blockIdx.x];
    const WinDev &w = wins[it.win];
    const int r0 = blockIdx.y * 16;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, rq = t & 3, slot = t >> 2;
    int bx, by, bz, nzc;
    unpack_cell(it.tile, bx, by, bz, nzc);
    const gptr<const real> coords = gbl((const real *)w.coords);
    const ProbDev pio = get_prob_d(io, w.prob);
    const gptr<const real> Vp = gbl((const real *)pio.Vp);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    real acc[W][4];
#pragma unroll
    for (int k = 0; k < W; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            acc[k][i] = real(0);
    // The quad's points are slot + 64 k, k < KP (items hold at most 64 KP
    // points; the four lanes of a quad share their points).  The reads are
    // issued in three waves so that many are in flight at once: the
    // permutation entries and coordinates of all KP points, then the RHS rows
    // of four points at a time, each batch loaded before the previous one's
    // products.
    constexpr int KP = kSpreadChunk1 / 64;
    int pj[KP];
    real uj[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int p = slot + 64 * k;
        const bool act = p < it.count;
        pj[k] = act ? gbl(w.perm)[it.start + p] : -1;
        uj[k] = act ? coords[it.start + p] : real(0);
    }
    auto load_rows = [&](int k0, real (&v)[4][4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (pj[k0 + k] >= 0)
                load4(Vp + (int64_t)pj[k0 + k] * pio.ldvp + r0 + 4 * rq, v[k]);
            else
                v[k][0] = v[k][1] = v[k][2] = v[k][3] = real(0);
        }
    };
    real va[4][4], vb[4][4];
    load_rows(0, va);
#pragma unroll
    for (int k0 = 0; k0 < KP; k0 += 4) {
        if (k0 + 4 < KP && slot + 64 * (k0 + 4) < it.count)
            load_rows(k0 + 4, (k0 & 4) ? va : vb);
        real (&v)[4][4] = (k0 & 4) ? vb : va;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (slot + 64 * (k0 + k) >= it.count)
                break;
            real wq[WQ], wv[W];
#pragma unroll
            for (int q = 0; q < WQ; ++q)
                wq[q] = kb_psi_d(uj[k0 + k] - (real)(bx + rq * WQ + q), mm, kb, ie);
            quad_gather<W>(wq, wv);
#pragma unroll
            for (int o = 0; o < W; ++o)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[o][i] += wv[o] * v[k][i];
        }
    }
    // sum the 16 point slots of the wave (lanes rq, rq + 4, ...), then the waves
#pragma unroll
    for (int o = 0; o < W; ++o)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            real a = acc[o][i];
#pragma unroll
            for (int s = 4; s < 64; s <<= 1)
                a += __shfl_xor(a, s, 64);
            acc[o][i] = a;
        }
    if (lane < 4)
#pragma unroll
        for (int o = 0; o < W; ++o)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                red[wave][o][4 * rq + i] = acc[o][i];
    __syncthreads();
    if (t < W * 16) {
        const int o = t >> 4, rr = t & 15, r = r0 + rr;
        if (r < R) {
            const real g = red[0][o][rr] + red[1][o][rr] + red[2][o][rr] + red[3][o][rr];
            const gptr<real> G = gbl((real *)w.G);
            gadd(&G[((int64_t)(r >> 1) * w.szG + bx + o) * 2 + (r & 1)], g);
        }
    }
}

// Interp: one block per dense item (<= kDenseChunk points) and 16 RHS, both
// outputs.  The item's W cells x 16 RHS of each output grid are staged in LDS;
// one lane per point (all 16 RHS of the point in the lane), so the point's
// coordinate and permutation entry are read once and its row is written with
// four 16-byte stores per output.  (Four lanes per point, each with four
// RHS, measured 0.84 against 0.81 ms on fifteen 1e6-point windows: the
// scattered 64-byte row writes bound both.)
template <typename real, int W>
__global__ __launch_bounds__(kBlock) void k_interp_dense1(const WinDev *__restrict__ wins,
                                                           const Chunk *__restrict__ items, int R, int nout)
{
    __shared__ __align__(16) real hs[2][W][16];
    const Chunk it = items[blockIdx.x];
    const WinDev &w = wins[it.win];
    const int r0 = blockIdx.y * 16;
    const int nr = min(16, R - r0);
    const int t = threadIdx.x;
    int bx, by, bz, nzc;
    unpack_cell(it.tile, bx, by, bz, nzc);
    const gptr<const real> H = gbl((const real *)w.H);
    for (int e = t; e < nout * W * 8; e += kBlock) {
        const int pi = e & 7, c = (e >> 3) % W, o = e / (8 * W);
        const int ra = 2 * pi;
        real re = real(0), im = real(0);
        if (ra < nr) {
            const int64_t off = ((int64_t)(o * w.npair_cap + (r0 >> 1) + pi) * w.szH + bx + c) * 2;
            re = H[off];
            im = H[off + 1];
        }
        hs[o][c][ra] = re;
        hs[o][c][ra + 1] = ra + 1 < nr ? im : real(0);
    }
    __syncthreads();
    if (t >= it.count)
        return;
    const gptr<const real> coords = gbl((const real *)w.coords);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    const int j = it.start + t;
    const real u = coords[j];
    const int64_t orig = gbl(w.perm)[j];
    real acc[2][16] = {};
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const real wc = kb_psi_d(u - (real)(bx + c), mm, kb, ie);
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            if (o >= nout)
                break;
#pragma unroll
            for (int i = 0; i < 16; i += 4) {
                real h[4];
                load4(&hs[o][c][i], h);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[o][i + q] += wc * h[q];
            }
        }
    }
    const bool vec = (w.Rcap & 3) == 0 && nr == 16;
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        if (o >= nout)
            break;
        const gptr<real> dst = gbl((real *)w.Yw) + ((int64_t)o * w.N + orig) * w.Rcap + r0;
        if (vec) {
#pragma unroll
            for (int i = 0; i < 16; i += 4) {
                real v4[4] = {acc[o][i], acc[o][i + 1], acc[o][i + 2], acc[o][i + 3]};
                store4(dst + i, v4);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < nr)
                    dst[i] = acc[o][i];
        }
    }
}

// ---------------------------------------------------------------------------
// launchers

bool dense_width_ok(int W) { return W == 8 || W == 12; }

template <typename real, int D, int W>
static void spread_dense_w(Engine &E, int R, IoArgs io, hipStream_t st)
{
    const int OUT = D == 3 ? W * W : W;
    const Chunk *items = E.d_dense_sp[D][E.cur_dense];
    const int nitems = E.ndense_sp[D][E.cur_dense];
    // d = 3: per-item blocks in scratch (the block's RHS range lies in one
    // 16-wide slot block: all R when R <= 16, else 16 per block)
    real *scratch = D == 3 ? (real *)E.scratch[E.cur_dense] : nullptr;
    const int nrb = (R + 15) / 16;
    if (R == 1) {
        dim3 grid(nitems, R);
        hipLaunchKernelGGL((k_spread_dense<real, D, W, 1>), grid, dim3(OUT), 0, st, E.d_wins, items, io, R, 1, scratch,
                           nrb, 1);
        return;
    }
    // d = 3: two RHS per thread in FP32 and one in FP64, so that the (2m + 1) x RT
    // accumulators stay in registers (more spill)
    constexpr int RT = D == 3 ? (sizeof(real) == 4 ? 2 : 1) : 4;
    const int nrg = std::min(4, (R + RT - 1) / RT);
    dim3 grid(nitems, (R + RT * nrg - 1) / (RT * nrg));
    hipLaunchKernelGGL((k_spread_dense<real, D, W, RT>), grid, dim3(OUT * nrg), 0, st, E.d_wins, items, io, R, nrg,
                       scratch, nrb, 16);
}

template <typename real, int D, int W, int RB>
static void interp_dense_rb(Engine &E, int R, int nout, hipStream_t st)
{
    constexpr int NC = dense_block_cells<D, W>();
    dim3 grid(E.ndense[D][E.cur_dense], (R + RB - 1) / RB, nout);
    hipLaunchKernelGGL((k_interp_dense<real, D, W, RB>), grid, dim3(kBlock), (size_t)NC * RB * sizeof(real), st,
                       E.d_wins, E.d_dense[D][E.cur_dense], R);
}

template <typename real, int D, int W>
static void interp_dense_w(Engine &E, int R, int nout, hipStream_t st)
{
    constexpr int NC = dense_block_cells<D, W>();
    int rbmax = 16;
    while (rbmax > 1 && (size_t)NC * rbmax * sizeof(real) > (size_t)kLdsBudget)
        rbmax >>= 1;
    int rb = 1;
    while (rb < R && rb < rbmax)
        rb <<= 1;
    switch (rb) {
    case 1: interp_dense_rb<real, D, W, 1>(E, R, nout, st); break;
    case 2: interp_dense_rb<real, D, W, 2>(E, R, nout, st); break;
    case 4: interp_dense_rb<real, D, W, 4>(E, R, nout, st); break;
    case 8: interp_dense_rb<real, D, W, 8>(E, R, nout, st); break;
    default: interp_dense_rb<real, D, W, 16>(E, R, nout, st); break;
    }
}

template <typename real, int D>
static void spread_dense_d(Engine &E, int wi, int R, IoArgs io, hipStream_t st)
{
    if (D == 1) {
        const dim3 grid(E.ndense_sp[1][wi], (R + 15) / 16);
        if (wi == 0)
            hipLaunchKernelGGL((k_spread_dense1<real, 8>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_dense_sp[1][wi], io,
                               R);
        else
            hipLaunchKernelGGL((k_spread_dense1<real, 12>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_dense_sp[1][wi],
                               io, R);
        return;
    }
    if (wi == 0)
        spread_dense_w<real, D, 8>(E, R, io, st);
    else
        spread_dense_w<real, D, 12>(E, R, io, st);
}

template <typename real, int D>
static void interp_dense_d(Engine &E, int wi, int R, int nout, hipStream_t st)
{
    if (D == 1) {
        const dim3 grid(E.ndense[1][wi], (R + 15) / 16);
        if (wi == 0)
            hipLaunchKernelGGL((k_interp_dense1<real, 8>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_dense[1][wi], R,
                               nout);
        else
            hipLaunchKernelGGL((k_interp_dense1<real, 12>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_dense[1][wi], R,
                               nout);
        return;
    }
    if (wi == 0)
        interp_dense_w<real, D, 8>(E, R, nout, st);
    else
        interp_dense_w<real, D, 12>(E, R, nout, st);
}

// wi selects the window width: 0 -> 2m = 8, 1 -> 2m = 12
void launch_spread_dense(Engine &E, int D, int wi, int R, IoArgs io, hipStream_t st)
{
    E.cur_dense = wi;
    if (E.precision == ADDK_FP32) {
        if (D == 1) spread_dense_d<float, 1>(E, wi, R, io, st);
        if (D == 2) spread_dense_d<float, 2>(E, wi, R, io, st);
        if (D == 3) spread_dense_d<float, 3>(E, wi, R, io, st);
    } else {
        if (D == 1) spread_dense_d<double, 1>(E, wi, R, io, st);
        if (D == 2) spread_dense_d<double, 2>(E, wi, R, io, st);
        if (D == 3) spread_dense_d<double, 3>(E, wi, R, io, st);
    }
}

void launch_interp_dense(Engine &E, int D, int wi, int R, int nout, hipStream_t st)
{
    E.cur_dense = wi;
    if (E.precision == ADDK_FP32) {
        if (D == 1) interp_dense_d<float, 1>(E, wi, R, nout, st);
        if (D == 2) interp_dense_d<float, 2>(E, wi, R, nout, st);
        if (D == 3) interp_dense_d<float, 3>(E, wi, R, nout, st);
    } else {
        if (D == 1) interp_dense_d<double, 1>(E, wi, R, nout, st);
        if (D == 2) interp_dense_d<double, 2>(E, wi, R, nout, st);
        if (D == 3) interp_dense_d<double, 3>(E, wi, R, nout, st);
    }
}

}  // namespace addk

namespace addk {

// ---------------------------------------------------------------------------
// spread, sparsely populated cells of one tile, without atomics in LDS.
// The block owns the tile's sub-grid (tile + window halo).  For d = 3 each
// thread owns one x-y column of it with every z cell in registers; for d <= 2
// each thread owns up to CPT cells.  Points of the chunk are staged in LDS
// (window values, base cell, RHS values) and visited by every thread; a
// thread adds w * v to the cells of its column that lie in the point's
// support.  The sub-grid is then added to the global grid.
template <typename real, int D, int W, int RT>
__global__ __launch_bounds__(kBlock) void k_spread_tile(const WinDev *__restrict__ wins, const Chunk *__restrict__ chunks,
                                                        IoArgs io, int R)
{
    constexpr int TB = D == 3 ? 4 : (D == 2 ? 16 : 256);  // maximal tile edge in base cells
    constexpr int SZ = TB + W - 1;                         // maximal sub-grid edge
    constexpr int NZ = D == 3 ? SZ : 1;                    // z cells per thread (column)
    constexpr int CPT = D == 3 ? 1 : (D == 2 ? (SZ * SZ + kBlock - 1) / kBlock : (SZ + kBlock - 1) / kBlock);
    constexpr int PB = 64;
    __shared__ real pw[PB][D][W];
    __shared__ int pb[PB][3];
    __shared__ real pv[PB][RT];

    const Chunk ch = chunks[blockIdx.x];
    const WinDev &w = wins[ch.win];
    const int r0 = blockIdx.y * RT;
    if (r0 >= R)
        return;
    const int S0 = w.S[0], S1 = D > 1 ? w.S[1] : 1, S2 = D > 2 ? w.S[2] : 1;
    int tl = ch.tile;
    const int tx = tl % w.ntile[0];
    tl /= w.ntile[0];
    const int ty = tl % w.ntile[1];
    const int tz = tl / w.ntile[1];
    const int o0[3] = {tx * w.tb[0], ty * w.tb[1], tz * w.tb[2]};
    const gptr<const real> coords = gbl((const real *)w.coords);
    const ProbDev pio = get_prob_d(io, w.prob);
    const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
    const int t = threadIdx.x;

    // cells owned by this thread (sub-grid coordinates)
    int cx[CPT], cy[CPT];
    bool own[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int lin = t + c * kBlock;
        if (D == 3) {
            cx[c] = lin % S0;
            cy[c] = lin / S0;
            own[c] = cy[c] < S1;
        } else if (D == 2) {
            cx[c] = lin % S0;
            cy[c] = lin / S0;
            own[c] = cy[c] < S1;
        } else {
            cx[c] = lin;
            cy[c] = 0;
            own[c] = lin < S0;
        }
    }
    real acc[CPT][NZ][RT];
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int z = 0; z < NZ; ++z)
#pragma unroll
            for (int i = 0; i < RT; ++i)
                acc[c][z][i] = real(0);

    for (int p0 = 0; p0 < ch.count; p0 += PB) {
        const int np = min(PB, ch.count - p0);
        for (int e = t; e < np * D; e += kBlock) {
            const int p = e / D, dd = e - p * D;
            const real u = coords[dd * w.N + ch.start + p0 + p];
            pb[p][dd] = (int)floor(u) - w.m + 1 - o0[dd];
        }
        for (int e = t; e < np * RT; e += kBlock) {
            const int p = e / RT, i = e - p * RT;
            const int r = r0 + i;
            const int orig = gbl(w.perm)[ch.start + p0 + p];
            pv[p][i] = r < R ? gbl((const real *)pio.Vp)[orig * pio.ldvp + r] : real(0);
        }
        __syncthreads();
        for (int e = t; e < np * D * W; e += kBlock) {
            const int p = e / (D * W), rem = e - p * (D * W);
            const int dd = rem / W, o = rem - dd * W;
            const real u = coords[dd * w.N + ch.start + p0 + p];
            pw[p][dd][o] = kb_psi_d(u - (real)(pb[p][dd] + o0[dd] + o), mm, kb, ie);
        }
        __syncthreads();
        for (int p = 0; p < np; ++p) {
            real vv[RT];
#pragma unroll
            for (int i = 0; i < RT; ++i)
                vv[i] = pv[p][i];
            const int bx = pb[p][0], by = D > 1 ? pb[p][D > 1 ? 1 : 0] : 0, bz = D > 2 ? pb[p][D > 2 ? 2 : 0] : 0;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int ox = cx[c] - bx, oy = cy[c] - by;
                const bool inx = (unsigned)ox < (unsigned)W;
                const bool iny = D == 1 || (unsigned)oy < (unsigned)W;
                real wxy = inx ? pw[p][0][inx ? ox : 0] : real(0);
                if (D > 1)
                    wxy *= iny ? pw[p][D > 1 ? 1 : 0][iny ? oy : 0] : real(0);
                if (!own[c])
                    wxy = real(0);
                if (D == 3) {
#pragma unroll
                    for (int z = 0; z < NZ; ++z) {
                        const int oz = z - bz;
                        const bool inz = (unsigned)oz < (unsigned)W;
                        const real wt = inz ? wxy * pw[p][D > 2 ? 2 : 0][inz ? oz : 0] : real(0);
#pragma unroll
                        for (int i = 0; i < RT; ++i)
                            acc[c][z][i] += wt * vv[i];
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < RT; ++i)
                        acc[c][0][i] += wxy * vv[i];
                }
            }
        }
        __syncthreads();
    }

    const gptr<real> G = gbl((real *)w.G);
    const int ex = w.ext[0], ey = w.ext[1], ez = w.ext[2];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        if (!own[c])
            continue;
        const int gx = o0[0] + cx[c], gy = D > 1 ? o0[1] + cy[c] : 0;
        if (gx >= ex || gy >= ey)
            continue;
#pragma unroll
        for (int z = 0; z < NZ; ++z) {
            const int gz = D > 2 ? o0[2] + z : 0;
            if (D > 2 && (z >= S2 || gz >= ez))
                continue;
            const int64_t cell = ((int64_t)gz * ey + gy) * ex + gx;
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const int r = r0 + i;
                if (r < R && acc[c][z][i] != real(0))
                    gadd(&G[((int64_t)(r >> 1) * w.szG + cell) * 2 + (r & 1)], acc[c][z][i]);
            }
        }
    }
}

template <typename real, int D, int W, int RT>
static void spread_tile_rt(Engine &E, int R, IoArgs io, hipStream_t st)
{
    dim3 grid(E.nchunks[D], (R + RT - 1) / RT);
    hipLaunchKernelGGL((k_spread_tile<real, D, W, RT>), grid, dim3(kBlock), 0, st, E.d_wins, E.d_chunks[D], io, R);
}

template <typename real, int D, int W>
static void spread_tile_w(Engine &E, int R, IoArgs io, hipStream_t st)
{
    if (R == 1)
        spread_tile_rt<real, D, W, 1>(E, R, io, st);
    else if (R == 2)
        spread_tile_rt<real, D, W, 2>(E, R, io, st);
    else
        spread_tile_rt<real, D, W, 4>(E, R, io, st);
}

// Returns false when the tile kernel has no instantiation for the engine's window width.
bool launch_spread_tile(Engine &E, int D, int R, IoArgs io, hipStream_t st)
{
    const int W = E.tile_w[D];
    if (W != 8 && W != 12)
        return false;
    if (E.precision == ADDK_FP32) {
        if (D == 1) { if (W == 8) spread_tile_w<float, 1, 8>(E, R, io, st); else spread_tile_w<float, 1, 12>(E, R, io, st); }
        if (D == 2) { if (W == 8) spread_tile_w<float, 2, 8>(E, R, io, st); else spread_tile_w<float, 2, 12>(E, R, io, st); }
        if (D == 3) { if (W == 8) spread_tile_w<float, 3, 8>(E, R, io, st); else spread_tile_w<float, 3, 12>(E, R, io, st); }
    } else {
        if (D == 1) { if (W == 8) spread_tile_w<double, 1, 8>(E, R, io, st); else spread_tile_w<double, 1, 12>(E, R, io, st); }
        if (D == 2) { if (W == 8) spread_tile_w<double, 2, 8>(E, R, io, st); else spread_tile_w<double, 2, 12>(E, R, io, st); }
        if (D == 3) { if (W == 8) spread_tile_w<double, 3, 8>(E, R, io, st); else spread_tile_w<double, 3, 12>(E, R, io, st); }
    }
    return true;
}

// ---------------------------------------------------------------------------
// d = 1 windows only: interpolation and window sum in one pass over the points
// in the caller's order.  A block takes kBlock consecutive points (one per
// thread) and 16 RHS.  For each window in turn it stages the window's grid box
// of the NO output grids in LDS ([o][cell][16 RHS, padded]), evaluates the point's 2m
// window values at its own coordinate, forms the NO interpolated products in
// registers (taps in order, as the sorted-order kernels do), adds sigma_w^2
// times the kernel product to the FP64 sum and writes the window's scaled
// derivative (and sigma) outputs with coalesced column stores; the sum is
// written after the last window.  No per-window product buffer is written or
// read back.
// LDS row of the fused d = 1 kernel: a cell's 16 RHS padded to 20 words (FP32)
// or 18 doubles (FP64), so that lanes reading the rows of different cells spread
// over the banks (rows of 16 words fall on one of two bank halves: 0.93 -> 0.78 ms
// on fifteen 1e6-point windows)
template <typename real>
constexpr int d1_row() { return sizeof(real) == 4 ? 20 : 18; }

template <typename real, int W, int NO>
__global__ __launch_bounds__(kBlock) void k_interp_combine_d1(const WinDev *__restrict__ wins, int nw, int ecap,
                                                              ProbDev p, int R, int mode)
{
    extern __shared__ __align__(16) unsigned char d1_lds[];
    real *hs = (real *)d1_lds;  // [NO][ecap][d1_row] (16 RHS, padded)
    const int t = threadIdx.x;
    const int r0 = blockIdx.y * 16;
    const int nr = min(16, R - r0);
    const int64_t i = (int64_t)blockIdx.x * kBlock + t;
    const bool own = i < p.N;
    const int64_t iy = i - p.yoff;
    double y[16];
#pragma unroll
    for (int r = 0; r < 16; ++r)
        y[r] = 0.0;
    for (int wi = 0; wi < nw; ++wi) {
        const WinDev &w = wins[wi];
        const int ext = w.ext[0];
        const gptr<const real> H = gbl((const real *)w.H);
        __syncthreads();  // every thread is done with the previous window's grids
        for (int e = t; e < NO * ext * 8; e += kBlock) {
            const int pi = e & 7, c = (e >> 3) % ext, o = e / (8 * ext);
            const int ra = 2 * pi;
            real re = real(0), im = real(0);
            if (ra < nr) {
                const int64_t off = ((int64_t)(o * w.npair_cap + (r0 >> 1) + pi) * w.szH + c) * 2;
                re = H[off];
                im = H[off + 1];
            }
            real *dst = hs + ((int64_t)o * ecap + c) * d1_row<real>() + ra;
            dst[0] = re;
            dst[1] = ra + 1 < nr ? im : real(0);
        }
        __syncthreads();
        if (!own)
            continue;
        const real mm = (real)w.m, kb = (real)w.b, ie = (real)w.inv_e2bm;
        const real u = gbl((const real *)w.ucoords)[i];
        const int b = (int)floor(u) - w.m + 1;  // the point's first cell of the box
        real acc[NO][16];
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[o][r] = real(0);
        // taps two at a time (full unrolling would hoist every tap's LDS reads)
#pragma unroll 2
        for (int c = 0; c < W; ++c) {
            const real wc = kb_psi_d(u - (real)(b + c), mm, kb, ie);
#pragma unroll
            for (int o = 0; o < NO; ++o)
#pragma unroll
                for (int r = 0; r < 16; r += 4) {
                    real h[4];
                    load4(hs + ((int64_t)o * ecap + b + c) * d1_row<real>() + r, h);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc[o][r + q] += wc * h[q];
                }
        }
        const int64_t blk = (int64_t)(wi - p.wbeg) * p.ldy * R;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            y[r] += w.sig2 * (double)acc[0][r];  // columns past nr hold zeros
            if (r < nr) {
                const int64_t at = iy + (int64_t)(r0 + r) * p.ldy;
                if ((mode & 2) && p.dYs)
                    p.dYs[blk + at] = w.dsig * (double)acc[0][r];
                if (NO == 2 && (mode & 4) && p.dYl)
                    p.dYl[blk + at] = w.der_scale * (double)acc[NO - 1][r];
            }
        }
    }
    if (own && (mode & 1) && p.Y)
#pragma unroll
        for (int r = 0; r < 16; ++r)
            if (r < nr)
                p.Y[iy + (int64_t)(r0 + r) * p.ldy] = y[r];
}

// LDS bytes of the fused d = 1 kernel: NO grid boxes of the widest window
int64_t interp_combine_d1_lds(const Engine &E, int nout)
{
    int ecap = 0;
    for (const WinDev &w : E.wdev)
        ecap = std::max(ecap, w.ext[0]);
    return (int64_t)nout * ecap * (E.precision == ADDK_FP32 ? d1_row<float>() * 4 : d1_row<double>() * 8);
}

void launch_interp_combine_d1(Engine &E, int R, int nout, int mode, IoArgs io, hipStream_t st)
{
    int ecap = 0;
    for (const WinDev &w : E.wdev)
        ecap = std::max(ecap, w.ext[0]);
    const ProbDev &p = io.single;
    const dim3 grid((unsigned)((p.N + kBlock - 1) / kBlock), (R + 15) / 16);
    const size_t lds = (size_t)interp_combine_d1_lds(E, nout);
    const int nw = (int)E.wdev.size();
    const bool w8 = E.wdev[0].W == 8;
    auto go = [&](auto k8, auto k12) {
        auto k = w8 ? k8 : k12;
        hipLaunchKernelGGL(k, grid, dim3(kBlock), lds, st, E.d_wins, nw, ecap, p, R, mode);
    };
    if (E.precision == ADDK_FP32) {
        if (nout == 2)
            go(k_interp_combine_d1<float, 8, 2>, k_interp_combine_d1<float, 12, 2>);
        else
            go(k_interp_combine_d1<float, 8, 1>, k_interp_combine_d1<float, 12, 1>);
    } else {
        if (nout == 2)
            go(k_interp_combine_d1<double, 8, 2>, k_interp_combine_d1<double, 12, 2>);
        else
            go(k_interp_combine_d1<double, 8, 1>, k_interp_combine_d1<double, 12, 1>);
    }
}

}  // namespace addk
