// Internal declarations of the additive-kernel fast summation library.
//
// Device data layout (per window w of a plan):
//   coords   real [d][N]   point coordinates in oversampled-grid units, relative
//                          to the window's grid box, sorted by spreading tile
//   perm     int32 [N]     sorted position -> caller's point index
//   Bk, Bd   real [(n+1)^d] Fourier multipliers of the kernel / derivative kernel
//                          over the modes k in {-n/2..n/2}^d (deconvolution folded in)
// Workspace (per engine; npair_cap complex grids per window, 2 real RHS per grid):
//   G   [pair][ez][ey][ex]            spread grid (box only)
//   A1  [pair][ez][ey][n1]            after the forward x pass (n1 = n + 1 modes)
//   A2  [pair][ez][n1][n1]            after the forward y pass
//   A3  [o][pair][ez][n1][n1]         after the fused z pass (o = kernel, derivative)
//   A4  [o][pair][ez][ey][n1]         after the inverse y pass
//   H   [o][pair][ez][ey][ex]         after the inverse x pass, read by interpolation
//   Vp  [N][ceil16(Rcap)] (real)      the RHS, point-major, converted once per call
//   Yw  [o][N][Rcap] (real)           per-window interpolated products in the engine's
//                                     precision, caller point order, point-major (one
//                                     point's RHS contiguous); summed over windows in FP64
// Lower-dimensional windows use the same arrays with unit extents.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "addk.h"

namespace addk {

constexpr int kBlock = 256;      // threads per block of every stage kernel
constexpr int kGroup = 16;       // lanes cooperating on one point in spread/interp
constexpr int kChunk = 1024;     // maximal points per spread/interp work item
constexpr int kMaxW = 16;        // maximal taps per dimension (m <= 8)
constexpr int kMaxNos = 256;     // maximal oversampled grid per dimension
constexpr int kLdsBudget = 64 * 1024;
constexpr int kCombineDepth = 1;  // window-sum blocks whose loads are in flight ahead of the current one (1 to 6 measured alike)
constexpr int kDenseMin = 16;    // points per base cell for the dense kernels
constexpr int kDenseChunk = 256; // maximal points per dense interp item
constexpr int kSpreadChunk = 1024; // maximal points per d = 3 dense spread item (one window block each;
                                   // bounds the FP32 accumulation length)
constexpr int kSpreadChunk1 = 2048; // maximal points per d = 1 dense spread item (32 per quad of lanes)
// Fewest RHS for which untuned engines use a matrix-core variant (it always
// computes 16 columns): where the autotuner's choice switches on the large
// workload (1e6 points, five d = 3 windows, K and dK/dl outputs).
constexpr int kMfmaMinRSpread = 3;       // dense spread (and R = 1, slabs as columns)
constexpr int kMfmaMinRInterpTile = 3;   // sparse-tile interp
constexpr int kMfmaMinRInterpDense = 6;  // dense interp (and R = 1, slabs as columns)
constexpr uint32_t kFlagNoDense = ADDK_TILE_KERNELS_ONLY;

// Per-window descriptor read by every stage kernel (device copy per engine).
constexpr int kNearQ = 8;        // matched derivatives of the near-field polynomial
constexpr int kNearChunk = 64;   // targets per near-field block (one wave)

struct WinDev {
    int d, n, n1, nos, m, W, prob, flags;
    int64_t N;
    int lo[3];      // box origin in absolute torus grid cells (x, y, z)
    int ext[3];     // box extent; unit for unused dimensions
    int tb[3];      // tile edge in base cells
    int ntile[3];   // tiles per dimension
    int S[3];       // sub-grid edge of a tile: tb + W - 1 (unit for unused dims)
    double b;       // Kaiser-Bessel shape parameter pi (2 - 1/sigma)
    double inv_e2bm;  // 1 / (1 - exp(-2 b m))
    double sig2, der_scale, dsig;  // sigma^2, sigma^2 * (2/l or 1/l), 2 sigma
    const void *coords;
    const int32_t *perm;
    const void *ucoords;  // d = 1: the grid coordinates in the caller's point order (else nullptr)
    const void *Bk;
    const void *Bd;
    void *G, *A1, *A2, *A3, *A4, *H, *Gm, *Vm;  // workspace (complex interleaved)
    int64_t szG, szA1, szA2, szA3, szA4, szH, szM;  // complex elements per pair
    void *Yw;       // [2][N][Rcap], engine precision
    int64_t Rcap;
    int npair_cap;
    int nbase[3];        // base cells per dimension: ext - 2m + 1 (unit for unused dims)
    const int2 *dmap;    // base cell -> {first, count} of its dense items in the engine's
                         // matrix-core item list (d = 3 only), or nullptr
    const void *tw;      // twiddles e^{2 pi i q / nos}, q < nos / 2 (complex real)
    // near-field correction (Matern-1/2 with ADDK_NEAR_FIELD; nf = 0 otherwise)
    int nf;
    double nf_eps2;      // radius^2 in grid units^2
    double nf_inv_eps2;
    double nf_hl;        // (data units per grid unit) / l: r / l = sqrt(d2) * nf_hl
    double nf_a[kNearQ + 1], nf_ad[kNearQ + 1];  // even polynomials in (r / eps) of kernel and derivative kernel
    const int32_t *tile_off;  // tile t's points are [tile_off[t], tile_off[t + 1]) of the sorted order
    const int2 *sp_rng;       // d = 3: {first, count} of tile t's sparsely populated cells' points (sources)
    double *nf_ys;            // [2][N] close-pair sums by sorted position (zero between calls)
};

// Problem-level input/output pointers (one per plan inside a batch).
struct ProbDev {
    int64_t N;
    int32_t wbeg, wend;       // windows [wbeg, wend) of the engine belong to it
    int64_t nsrc;             // points [0, nsrc) carry V (the rest are targets only)
    int64_t yoff;             // outputs are points [yoff, N), row i - yoff of Y
    const double *V;
    int64_t ldv;
    const void *Vp;           // point-major copy of V in the engine's precision,
    int64_t ldvp;             // Vp[i * ldvp + r], r < ldvp (RHS padded to 16 with zeros)
    double *Y;
    int64_t ldy;
    double *dYl;
    double *dYs;
};

struct IoArgs {
    const ProbDev *table;  // device table (batches) or nullptr
    ProbDev single;        // used when table == nullptr
};

struct Chunk {
    int32_t win, tile, start, count;
};

struct LineGroup {
    int32_t win, grp;
};

// Device memory reached through a pointer held in a descriptor, as a pointer in
// the global address space: its loads and stores then compile to global, not
// flat, instructions.  A flat access counts on the LDS counter as well as on
// the vector-memory counter, so a wave that waits for its LDS reads would also
// wait for every HBM load it still has in flight.
template <typename T> using gptr = T __attribute__((address_space(1))) *;
template <typename T> __device__ __forceinline__ gptr<T> gbl(T *p) { return (gptr<T>)p; }
__device__ __forceinline__ int2 ld_int2(gptr<const int2> p)
{
    typedef int n2i __attribute__((ext_vector_type(2)));
    const n2i t = *(gptr<const n2i>)p;
    return make_int2(t.x, t.y);
}

// Stage identifiers for the FFT passes (axis, mode).
enum FftStage { ST_FWD0 = 0, ST_FWD1, ST_FUSED2, ST_FUSED1, ST_FUSED0, ST_INV1, ST_INV0, ST_COUNT };

// Host-side record of one window of a plan.
struct WinHost {
    int d;
    int feat[3];
    double ell, sigma, T, L, eta, center[3];
    int lo[3], ext[3], tb[3], ntile[3], S[3];
    int64_t ntiles;
    void *coords = nullptr;
    int32_t *perm = nullptr;
    void *ucoords = nullptr;  // d = 1 windows of square plans: coordinates in the caller's order
    void *Bk = nullptr, *Bd = nullptr;
    double *Bk64 = nullptr, *Bd64 = nullptr;
    std::vector<Chunk> chunks;  // sparse tile chunks; win field is filled by the engine
    std::vector<Chunk> dense;   // dense cell runs for interp (<= kDenseChunk points); tile field holds
                                // the packed base cell
    std::vector<Chunk> dense_sp;  // the same runs for spreading, <= kSpreadChunk points each
    int64_t ndense_pts = 0;
    // near-field correction
    bool nf = false;
    double nf_eps = 0.0;                          // radius in data units
    double nf_Lf = 0.0;                           // half-width of the unfolded region (L, or l if L = 0)
    double nf_a[kNearQ + 1], nf_ad[kNearQ + 1];
    std::vector<int32_t> tile_off;                // host copy (ntiles + 1)
    int32_t *d_tile_off = nullptr;
    // plans with separate target points sort the sources and the targets as two
    // segments of the same arrays: the lists above (chunks, dense_sp, tile_off)
    // then cover the sources, dense covers the targets, and these the targets
    bool split = false;
    std::vector<Chunk> chunks_i;                  // sparse tile chunks of the targets (interp)
    std::vector<int32_t> tile_off_t;              // targets' tile ranges (near-field blocks)
};

struct Plan;

enum ProfStage { PS_ZERO = 0, PS_SPREAD, PS_FFT_X_FWD, PS_FFT_Y_FWD, PS_FFT_FUSED, PS_FFT_Y_INV, PS_FFT_X_INV,
                 PS_INTERP, PS_COMBINE, PS_MODE_DOT, PS_SPREAD_DENSE, PS_INTERP_DENSE, PS_GATHER, PS_NEAR,
                 PS_COUNT };

struct ProfRec {
    int stage;
    hipEvent_t a, b;
};

// An engine runs the stage kernels over a set of windows (one plan or a batch).
struct Engine {
    int precision = ADDK_FP64;
    int nprob = 0;
    std::vector<const Plan *> plans;
    std::vector<WinDev> wdev;      // host mirror of the device descriptors
    std::vector<int> wplan;        // plan index of each window
    std::vector<int> wlocal;       // window index inside its plan
    WinDev *d_wins = nullptr;
    Chunk *d_chunks[4] = {nullptr, nullptr, nullptr, nullptr};  // sparse tile chunks for spreading, per d (1..3)
    int nchunks[4] = {0, 0, 0, 0};
    Chunk *d_chunks_i[4] = {nullptr, nullptr, nullptr, nullptr};  // ... for interpolation (the same list for
    int nchunks_i[4] = {0, 0, 0, 0};                                // square plans, the targets' otherwise)
    Chunk *d_dense[4][2] = {};     // dense cell runs (interp items) per d and window width (2m = 8, 12)
    int ndense[4][2] = {};
    Chunk *d_dense_sp[4][2] = {};  // dense cell runs for spreading (larger items, one block each)
    int ndense_sp[4][2] = {};
    int ndense_sp2[2] = {};        // d = 3: the two-cell items, which lead each spread item list
    bool fused_d1 = false;         // every window d = 1 (single problem): interp and window sum fused
    int fused_no = 0;              // outputs of the fused interp the next engine_combine owes (0: none)
    int fft_L = 16;                // lines per FFT block (halved when some window's grid exceeds 128)
    int nos_max = 16;              // largest oversampled grid edge of the engine's windows
    Chunk *d_near[4] = {};         // near-field target blocks per d (tile field = tile index)
    int nnear[4] = {};
    std::vector<int2> near_rng;    // per window: [first, end) of its blocks in the list of its d
    double *d_near_part = nullptr; // near-field inner-product partials
    double *d_near_ys = nullptr;   // near-field sums by sorted position (WinDev::nf_ys)
    int64_t near_part_cap = 0;
    int cur_dense = 0;
    int tile_w[4] = {0, 0, 0, 0};  // common window width of the tile work lists per d (0: mixed)
    bool no_mfma = false;          // use the vector-ALU dense kernels only
    uint32_t knobs = ADDK_KNOB_ALL_MFMA;  // matrix-core variant per stage (ADDK_KNOB_*)
    bool tuned = false;            // knobs chosen by measurement: no R threshold
    int2 *d_dmap[2] = {nullptr, nullptr};        // base-cell maps of all windows (per 2m = 8, 12)
    int2 *d_sprng = nullptr;                     // sparse point ranges per tile, all d = 3 windows (WinDev::sp_rng)
    LineGroup *d_sptiles[2] = {nullptr, nullptr};  // output tiles of the sparse spread (per 2m = 8, 12)
    int nsptiles[2] = {0, 0};
    bool sparse_gather = false;  // d = 3 sparse spread by output tiles (k_spread_sparse_mfma)
    LineGroup *d_gtiles[2] = {nullptr, nullptr};  // output tiles of the dense block gather
    int ngtiles[2] = {0, 0};
    void *scratch[2] = {nullptr, nullptr};        // per-item dense spread blocks (engine precision, d = 3)
    int64_t scratch_cap[2] = {0, 0};              // elements
    LineGroup *d_groups[ST_COUNT] = {};
    int ngroups[ST_COUNT] = {};
    int maxvol[4] = {0, 0, 0, 0};  // largest tile sub-grid volume per d
    int rb[4] = {0, 0, 0, 0};      // RHS per spread/interp pass per d (capacity)
    void *ws = nullptr;            // grid workspace
    int64_t ws_bytes = 0;
    void *yw = nullptr;            // per-window products (engine precision)
    int64_t yw_bytes = 0;
    void *d_tw = nullptr;          // twiddle tables for n_os = 16, 32, 64, 128 (engine precision)
    void *vpack = nullptr;         // point-major copies of the problems' V (see ProbDev::Vp)
    int64_t vpack_bytes = 0;
    int64_t vpack_ld = 0;
    int npair_cap = 0;
    int64_t rcap = 0;
    ProbDev *d_probs = nullptr;
    std::vector<ProbDev> probs;
    double *d_partial = nullptr;   // reduction scratch for the vjp
    int64_t partial_cap = 0;
    bool dirty = true;             // descriptors need an upload
    bool prof = false;             // record stage events
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> evpool;
};

// Records a HIP event pair around one stage launch when profiling is on.
struct StageTimer {
    Engine &E;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr;
    StageTimer(Engine &e, int s, hipStream_t t);
    ~StageTimer();
};

struct Plan {
    int64_t N = 0;
    int64_t nsrc = 0;  // sources are points [0, nsrc); targets [nsrc, N) if nsrc < N (rectangular plan)
    bool rect = false;
    int32_t D = 0, P = 0;
    int32_t kernel = ADDK_GAUSSIAN, n = 0, m = 0, nos = 0, precision = ADDK_FP64;
    uint32_t flags = 0;
    double sigma_os = 2.0;
    std::vector<WinHost> wins;
    std::vector<double> psi_tab;   // Psi(k), k = -n/2..n/2
    double *d_psi = nullptr;
    Engine eng;
    int device = 0;
    uint64_t param_gen = 0;  // counts addk_plan_update_params calls (batches refresh their copies)
};

// Per-call workspace of an engine for cap complex grids per window and rcap
// right-hand sides (bytes; dense spread blocks in elements of the engine's
// precision).
struct WsLayout {
    int cap = 0;
    int64_t rcap = 0;
    int64_t grid_bytes = 0, y_bytes = 0, nys_bytes = 0, vpack_bytes = 0, vpack_ld = 0;
    int64_t scratch_elems[2] = {0, 0};
};

// ---- helpers implemented in the .hip files --------------------------------
void set_error(const std::string &msg);
addk_status hip_fail(hipError_t e, const char *what);

// kernels.hip
addk_status engine_build_device(Engine &E, int device_precision);
addk_status engine_ensure_workspace(Engine &E, int R);
WsLayout engine_ws_layout(Engine &E, int cap, int64_t rcap);
void engine_bind_ws(Engine &E, const WsLayout &L, void *ws, void *yw, double *nys, void *vpack, void *scr0,
                    void *scr1);
addk_status engine_run(Engine &E, int R, int nout, bool store_vmodes_only, bool store_gmodes,
                       IoArgs io, hipStream_t st);
addk_status engine_run_bound(Engine &E, int R, int nout, bool store_vmodes_only, bool store_gmodes,
                             IoArgs io, hipStream_t st);
addk_status engine_combine(Engine &E, int R, int mode, IoArgs io, hipStream_t st);
addk_status engine_mode_dot(Engine &E, int npair, double *grad_ell, double *grad_sig, hipStream_t st);
addk_status engine_gsi(Engine &E, const std::vector<const double *> &B64, const double *psi, int n, double *theta,
                       hipStream_t st);
addk_status engine_upload(Engine &E);
void engine_free(Engine &E);
bool use_mfma(const Engine &E, uint32_t knob, int R);
addk_status engine_profile_read(Engine &E, double *ms, int32_t *count);

// dense.hip
void launch_spread_dense(Engine &E, int D, int wi, int R, IoArgs io, hipStream_t st);
void launch_interp_dense(Engine &E, int D, int wi, int R, int nout, hipStream_t st);
bool dense_width_ok(int W);
bool launch_spread_tile(Engine &E, int D, int R, IoArgs io, hipStream_t st);

// mfma.hip (FP32 matrix-core variants of the dense-cell kernels, d = 3)
bool launch_interp_mfma(Engine &E, int wi, int R, int nout, hipStream_t st);
bool launch_spread_mfma(Engine &E, int wi, int R, IoArgs io, hipStream_t st);
void launch_interp_combine_d1(Engine &E, int R, int nout, int mode, IoArgs io, hipStream_t st);
int64_t interp_combine_d1_lds(const Engine &E, int nout);
// Knobs chosen by measurement, by problem shape (device, window dimensions,
// largest oversampled grid, m, R, point-count bucket, precision, outputs),
// shared by the plans of the process.
bool tune_cache_get(const Engine &E, int R, int nout, uint32_t *knobs);
void tune_cache_put(const Engine &E, int R, int nout, uint32_t knobs);
void tune_cache_clear();
void launch_gather_blocks(Engine &E, int wi, int R, hipStream_t st);
bool launch_interp_tile_mfma(Engine &E, int R, int nout, hipStream_t st);
void launch_spread_sparse_mfma(Engine &E, int R, IoArgs io, hipStream_t st);

// nearfield.hip (ADDK_NEAR_FIELD)
void launch_near(Engine &E, int R, int nout, IoArgs io, hipStream_t st);
addk_status engine_near_dot(Engine &E, int R, IoArgs io, const double *V, int64_t ldv, double *grad_ell,
                            double *grad_sig, hipStream_t st);

// plan.hip
addk_status plan_compute_multipliers(Plan &pl, hipStream_t st);

// api.hip: a device FP64 matrix argument (ld >= N, device memory; NULL allowed unless required)
addk_status check_mat(const void *p, int64_t ld, int64_t N, const char *name, bool required);

}  // namespace addk
