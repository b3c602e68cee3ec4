// K V for callers that cannot allocate device memory (code under stream
// capture, serving loops, harnesses that forbid hipMalloc).
//
// The per-call workspace of a plan's product (spread and transform grids, the
// FP64 per-window products, the point-major RHS copy, the dense spread's
// per-item blocks and the near-field close-pair sums) normally comes from
// buffers the plan allocates on first use and grows with R.  Here it is carved
// from one file-scope device array instead, so a call allocates nothing.  Each
// GPU holds its own copy of the array (kNoAllocBytes) from module load until
// the process ends; its device address is looked up once per device.  Every
// call on a GPU shares that GPU's array: calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "addk_internal.h"

namespace addk {
namespace {

constexpr int64_t kNoAllocBytes = int64_t(256) << 20;  // 256 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (the host-side name is not a
// device address).  The calling thread's current device is the plan's.
addk_status scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal out of range for the allocation-free workspace");
        return ADDK_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ADDK_OK;
}

__global__ void k_clear(double *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

// The engine's own workspace binding, put back after the call.
struct SavedWs {
    std::vector<WinDev> wdev;
    void *ws, *vpack, *scr[2], *yw;
    double *nys;
    int64_t ws_bytes, yw_bytes, vpack_bytes, vpack_ld, scap[2], rcap;
    int npair_cap;
    bool dirty;

    explicit SavedWs(const Engine &E)
        : wdev(E.wdev), ws(E.ws), vpack(E.vpack), scr{E.scratch[0], E.scratch[1]}, yw(E.yw), nys(E.d_near_ys),
          ws_bytes(E.ws_bytes), yw_bytes(E.yw_bytes), vpack_bytes(E.vpack_bytes), vpack_ld(E.vpack_ld),
          scap{E.scratch_cap[0], E.scratch_cap[1]}, rcap(E.rcap), npair_cap(E.npair_cap), dirty(E.dirty)
    {
    }
    void restore(Engine &E) const
    {
        E.wdev = wdev;
        E.ws = ws;
        E.vpack = vpack;
        E.scratch[0] = scr[0];
        E.scratch[1] = scr[1];
        E.yw = yw;
        E.d_near_ys = nys;
        E.ws_bytes = ws_bytes;
        E.yw_bytes = yw_bytes;
        E.vpack_bytes = vpack_bytes;
        E.vpack_ld = vpack_ld;
        E.scratch_cap[0] = scap[0];
        E.scratch_cap[1] = scap[1];
        E.rcap = rcap;
        E.npair_cap = npair_cap;
        E.dirty = true;  // the device copy of the descriptors points into the array
    }
};

}  // namespace
}  // namespace addk

using namespace addk;

extern "C" addk_status addk_matvec_noalloc(addk_plan plan, int32_t R, const double *V, int64_t ldv, double *Y,
                                           int64_t ldy, void *stream)
{
    if (!plan) {
        set_error("plan is NULL");
        return ADDK_ERR_INVALID_ARG;
    }
    Plan &pl = *(Plan *)plan;
    if (R < 1) {
        set_error("R must be >= 1");
        return ADDK_ERR_INVALID_ARG;
    }
    if (pl.N == 0)
        return ADDK_OK;
    addk_status s;
    const int64_t nout_rows = pl.rect ? pl.N - pl.nsrc : pl.N;
    if ((s = check_mat(V, ldv, pl.nsrc, "V", true)) != ADDK_OK || (s = check_mat(Y, ldy, nout_rows, "Y", true)) != ADDK_OK)
        return s;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    if (dev != pl.device) {
        set_error("addk_matvec_noalloc: the plan's device (" + std::to_string(pl.device) +
                  ") must be the current device (" + std::to_string(dev) + ")");
        return ADDK_ERR_INVALID_ARG;
    }
    Engine &E = pl.eng;
    if (!E.d_wins) {
        set_error("addk_matvec_noalloc: plan has no descriptor table");
        return ADDK_ERR_INVALID_ARG;
    }
    // lay the workspace for exactly R right-hand sides out in the array
    const WsLayout L = engine_ws_layout(E, (R + 1) / 2, R);
    const int64_t rs = E.precision == ADDK_FP32 ? 4 : 8;
    const int64_t off_y = round256(L.grid_bytes);
    const int64_t off_n = off_y + round256(L.y_bytes);
    const int64_t off_v = off_n + round256(L.nys_bytes);
    const int64_t off_s0 = off_v + round256(L.vpack_bytes);
    const int64_t off_s1 = off_s0 + round256(L.scratch_elems[0] * rs);
    const int64_t need = off_s1 + round256(L.scratch_elems[1] * rs);
    if (need > kNoAllocBytes) {
        set_error("addk_matvec_noalloc: this plan needs " + std::to_string(need) + " bytes of workspace for R = " +
                  std::to_string(R) + "; the allocation-free workspace holds " + std::to_string(kNoAllocBytes) +
                  " bytes (use addk_matvec, or fewer right-hand sides per call)");
        return ADDK_ERR_INVALID_ARG;
    }
    void *base = nullptr;
    if ((s = scratch_address(dev, &base)) != ADDK_OK)
        return s;
    char *b = (char *)base;
    const SavedWs saved(E);
    engine_bind_ws(E, L, b, b + off_y, L.nys_bytes > 0 ? (double *)(b + off_n) : nullptr, b + off_v, b + off_s0,
                   b + off_s1);
    hipStream_t st = (hipStream_t)stream;
    s = engine_upload(E);  // synchronous: the previous user of the array has finished
    if (s == ADDK_OK && L.nys_bytes > 0) {
        // close-pair sums start at zero (the passes that read them clear them again)
        const int64_t n = L.nys_bytes / (int64_t)sizeof(double);
        hipLaunchKernelGGL(k_clear, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, st,
                           (double *)(b + off_n), n);
        e = hipGetLastError();
        if (e != hipSuccess)
            s = hip_fail(e, "clear launch");
    }
    if (s == ADDK_OK) {
        IoArgs io;
        std::memset(&io, 0, sizeof(io));
        io.single.N = pl.N;
        io.single.nsrc = pl.nsrc;
        io.single.yoff = pl.rect ? pl.nsrc : 0;
        io.single.wbeg = 0;
        io.single.wend = pl.P;
        io.single.V = V;
        io.single.ldv = ldv;
        io.single.Y = Y;
        io.single.ldy = ldy;
        s = engine_run_bound(E, R, 1, false, false, io, st);
        if (s == ADDK_OK)
            s = engine_combine(E, R, 1, io, st);
    }
    saved.restore(E);
    return s;
}
