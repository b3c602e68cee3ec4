// Products exposed through the C ABI: K V, the derivative products, the
// vector-Jacobian product and batched products captured into a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "addk_internal.h"

namespace addk {

static addk_status fail2(addk_status s, const std::string &msg)
{
    set_error(msg);
    return s;
}

static bool on_device(const void *p)
{
    if (!p)
        return false;
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

addk_status check_mat(const void *p, int64_t ld, int64_t N, const char *name, bool required)
{
    if (!p) {
        if (required)
            return fail2(ADDK_ERR_INVALID_ARG, std::string(name) + " is NULL");
        return ADDK_OK;
    }
    if (ld < N || ld < 1)
        return fail2(ADDK_ERR_INVALID_ARG, std::string("leading dimension of ") + name + " is smaller than N");
    if (!on_device(p))
        return fail2(ADDK_ERR_INVALID_ARG, std::string(name) + " must be a device pointer");
    return ADDK_OK;
}

static ProbDev single_prob(const Plan &pl)
{
    ProbDev p;
    std::memset(&p, 0, sizeof(p));
    p.N = pl.N;
    p.nsrc = pl.nsrc;
    p.yoff = pl.rect ? pl.nsrc : 0;
    p.wbeg = 0;
    p.wend = pl.P;
    return p;
}

struct Batch {
    Engine eng;
    std::vector<Plan *> plans;
    std::vector<uint64_t> gens;  // each plan's parameter generation the descriptors hold
    int R = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
};

// The batch holds copies of its plans' window descriptors.  After
// addk_plan_update_params on a plan, copy its new parameters (amplitude
// factors, near-field polynomials, multiplier pointers) into the batch's
// descriptors and upload them; the graph reads them from device memory, so
// it needs no new capture.
static addk_status batch_refresh_params(Batch &b)
{
    bool stale = false;
    for (size_t p = 0; p < b.plans.size(); ++p) {
        const Plan &pl = *b.plans[p];
        if (b.gens[p] == pl.param_gen)
            continue;
        stale = true;
        const int wbeg = b.eng.probs[p].wbeg;
        for (int w = 0; w < pl.P; ++w) {
            const WinDev &src = pl.eng.wdev[w];
            WinDev &dst = b.eng.wdev[wbeg + w];
            dst.sig2 = src.sig2;
            dst.der_scale = src.der_scale;
            dst.dsig = src.dsig;
            dst.Bk = src.Bk;
            dst.Bd = src.Bd;
            dst.nf_eps2 = src.nf_eps2;
            dst.nf_inv_eps2 = src.nf_inv_eps2;
            dst.nf_hl = src.nf_hl;
            for (int j = 0; j <= kNearQ; ++j) {
                dst.nf_a[j] = src.nf_a[j];
                dst.nf_ad[j] = src.nf_ad[j];
            }
        }
        b.gens[p] = pl.param_gen;
    }
    if (!stale)
        return ADDK_OK;
    b.eng.dirty = true;
    return engine_upload(b.eng);
}

static addk_status batch_enqueue(Batch &b, hipStream_t st)
{
    IoArgs io;
    std::memset(&io, 0, sizeof(io));
    io.table = b.eng.d_probs;
    addk_status s = engine_run(b.eng, b.R, 1, false, false, io, st);
    if (s == ADDK_OK)
        s = engine_combine(b.eng, b.R, 1, io, st);
    return s;
}

// (Re)capture the batch's stage sequence into a graph on its private stream.
static addk_status batch_capture(Batch &b)
{
    hipError_t e;
    if (b.exec) {
        (void)hipGraphExecDestroy(b.exec);
        b.exec = nullptr;
    }
    if (b.graph) {
        (void)hipGraphDestroy(b.graph);
        b.graph = nullptr;
    }
    e = hipStreamBeginCapture(b.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    addk_status s2 = batch_enqueue(b, b.cap_stream);
    e = hipStreamEndCapture(b.cap_stream, &b.graph);
    if (s2 != ADDK_OK)
        return s2;
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
    if (e != hipSuccess)
        return hip_fail(e, "hipGraphInstantiate");
    return ADDK_OK;
}

// Time `reps` runs of fn (after one warm-up) on the stream; average ms.
template <typename Fn>
static addk_status time_runs(Fn fn, int reps, hipStream_t st, double *ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    if (e != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    addk_status s = fn();
    if (s == ADDK_OK && (e = hipEventRecord(a, st)) != hipSuccess)
        s = hip_fail(e, "hipEventRecord");
    for (int r = 0; r < reps && s == ADDK_OK; ++r)
        s = fn();
    if (s == ADDK_OK && (e = hipEventRecord(b, st)) != hipSuccess)
        s = hip_fail(e, "hipEventRecord");
    if (s == ADDK_OK && (e = hipEventSynchronize(b)) != hipSuccess)
        s = hip_fail(e, "hipEventSynchronize");
    float t = 0.f;
    if (s == ADDK_OK && (e = hipEventElapsedTime(&t, a, b)) != hipSuccess)
        s = hip_fail(e, "hipEventElapsedTime");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t / std::max(reps, 1);
    return s;
}

// Candidate knob sets of an engine: every subset of the matrix-core stages
// that the engine has work for (others are left on, they have no effect).
static std::vector<uint32_t> knob_candidates(const Engine &E, int R)
{
    if (E.no_mfma)
        return {0u};
    bool dense = false, dense_sp = false, tile = false;
    for (int wi = 0; wi < 2; ++wi) {
        dense = dense || E.ndense[3][wi] > 0;
        dense_sp = dense_sp || E.ndense_sp[3][wi] > 0;
    }
    tile = E.nchunks_i[3] > 0 && (E.tile_w[3] == 8 || E.tile_w[3] == 12);
    // the split spread shape: FP32 matrix-core spread with 16 RHS columns
    const bool split = E.precision == ADDK_FP32 && dense_sp && R >= 2;
    std::vector<uint32_t> out;
    for (uint32_t k = 0; k <= ADDK_KNOB_ALL; ++k) {
        if (!dense && (k & (ADDK_KNOB_SPREAD_MFMA | ADDK_KNOB_INTERP_DENSE_MFMA)) !=
                          (ADDK_KNOB_SPREAD_MFMA | ADDK_KNOB_INTERP_DENSE_MFMA))
            continue;
        if (!tile && !(k & ADDK_KNOB_INTERP_TILE_MFMA))
            continue;
        if ((k & ADDK_KNOB_SPREAD_SPLIT) && !(split && (k & ADDK_KNOB_SPREAD_MFMA)))
            continue;
        out.push_back(k);
    }
    return out;
}

}  // namespace addk

using namespace addk;

extern "C" {

addk_status addk_matvec(addk_plan plan, int32_t R, const double *V, int64_t ldv, double *Y, int64_t ldy, void *stream)
{
    if (!plan)
        return fail2(ADDK_ERR_INVALID_ARG, "plan is NULL");
    Plan &pl = *(Plan *)plan;
    if (R < 1)
        return fail2(ADDK_ERR_INVALID_ARG, "R must be >= 1");
    if (pl.N == 0)
        return ADDK_OK;
    addk_status s;
    const int64_t nout_rows = pl.rect ? pl.N - pl.nsrc : pl.N;
    if ((s = check_mat(V, ldv, pl.nsrc, "V", true)) != ADDK_OK || (s = check_mat(Y, ldy, nout_rows, "Y", true)) != ADDK_OK)
        return s;
    IoArgs io;
    std::memset(&io, 0, sizeof(io));
    io.single = single_prob(pl);
    io.single.V = V;
    io.single.ldv = ldv;
    io.single.Y = Y;
    io.single.ldy = ldy;
    hipStream_t st = (hipStream_t)stream;
    s = engine_run(pl.eng, R, 1, false, false, io, st);
    if (s != ADDK_OK)
        return s;
    return engine_combine(pl.eng, R, 1, io, st);
}

addk_status addk_dmatvec(addk_plan plan, int32_t R, const double *V, int64_t ldv, double *dY_dell, double *dY_dsigma,
                         double *Y, int64_t ldy, void *stream)
{
    if (!plan)
        return fail2(ADDK_ERR_INVALID_ARG, "plan is NULL");
    Plan &pl = *(Plan *)plan;
    if (R < 1)
        return fail2(ADDK_ERR_INVALID_ARG, "R must be >= 1");
    if (!dY_dell && !dY_dsigma && !Y)
        return fail2(ADDK_ERR_INVALID_ARG, "no output requested");
    if (pl.N == 0)
        return ADDK_OK;
    addk_status s;
    const int64_t nout_rows = pl.rect ? pl.N - pl.nsrc : pl.N;
    if ((s = check_mat(V, ldv, pl.nsrc, "V", true)) != ADDK_OK || (s = check_mat(Y, ldy, nout_rows, "Y", false)) != ADDK_OK ||
        (s = check_mat(dY_dell, ldy, nout_rows, "dY_dell", false)) != ADDK_OK ||
        (s = check_mat(dY_dsigma, ldy, nout_rows, "dY_dsigma", false)) != ADDK_OK)
        return s;
    IoArgs io;
    std::memset(&io, 0, sizeof(io));
    io.single = single_prob(pl);
    io.single.V = V;
    io.single.ldv = ldv;
    io.single.Y = Y;
    io.single.ldy = ldy;
    io.single.dYl = dY_dell;
    io.single.dYs = dY_dsigma;
    hipStream_t st = (hipStream_t)stream;
    const int nout = dY_dell ? 2 : 1;
    s = engine_run(pl.eng, R, nout, false, false, io, st);
    if (s != ADDK_OK)
        return s;
    const int mode = (Y ? 1 : 0) | (dY_dsigma ? 2 : 0) | (dY_dell ? 4 : 0);
    return engine_combine(pl.eng, R, mode, io, st);
}

addk_status addk_vjp(addk_plan plan, int32_t R, const double *V, int64_t ldv, const double *G, int64_t ldg,
                     double *grad_V, int64_t ldgv, double *grad_ell, double *grad_sigma, void *stream)
{
    if (!plan)
        return fail2(ADDK_ERR_INVALID_ARG, "plan is NULL");
    Plan &pl = *(Plan *)plan;
    if (R < 1)
        return fail2(ADDK_ERR_INVALID_ARG, "R must be >= 1");
    if (pl.rect)
        return fail2(ADDK_ERR_UNSUPPORTED, "addk_vjp needs a square plan (targets = sources)");
    addk_status s;
    const bool scalars = grad_ell || grad_sigma;
    if ((grad_ell && !on_device(grad_ell)) || (grad_sigma && !on_device(grad_sigma)))
        return fail2(ADDK_ERR_INVALID_ARG, "grad_ell and grad_sigma must be device pointers");
    if (pl.N == 0) {
        if (scalars) {
            std::vector<double> z(pl.P, 0.0);
            hipError_t e = hipSuccess;
            if (grad_ell)
                e = hipMemcpy(grad_ell, z.data(), pl.P * sizeof(double), hipMemcpyHostToDevice);
            if (e == hipSuccess && grad_sigma)
                e = hipMemcpy(grad_sigma, z.data(), pl.P * sizeof(double), hipMemcpyHostToDevice);
            if (e != hipSuccess)
                return hip_fail(e, "hipMemcpy");
        }
        return ADDK_OK;
    }
    if ((s = check_mat(G, ldg, pl.N, "G", true)) != ADDK_OK || (s = check_mat(V, ldv, pl.N, "V", scalars)) != ADDK_OK ||
        (s = check_mat(grad_V, ldgv, pl.N, "grad_V", false)) != ADDK_OK)
        return s;
    hipStream_t st = (hipStream_t)stream;
    IoArgs io;
    std::memset(&io, 0, sizeof(io));
    io.single = single_prob(pl);
    if (scalars) {
        io.single.V = V;
        io.single.ldv = ldv;
        s = engine_run(pl.eng, R, 0, true, false, io, st);  // V^ modes only
        if (s != ADDK_OK)
            return s;
    }
    io.single.V = G;
    io.single.ldv = ldg;
    io.single.Y = grad_V;
    io.single.ldy = ldgv;
    s = engine_run(pl.eng, R, grad_V ? 1 : 0, false, scalars, io, st);
    if (s != ADDK_OK)
        return s;
    if (grad_V && (s = engine_combine(pl.eng, R, 1, io, st)) != ADDK_OK)
        return s;
    if (scalars) {
        s = engine_mode_dot(pl.eng, (R + 1) / 2, grad_ell, grad_sigma, st);
        if (s == ADDK_OK)
            s = engine_near_dot(pl.eng, R, io, V, ldv, grad_ell, grad_sigma, st);  // close pairs of V and G
        return s;
    }
    return ADDK_OK;
}

addk_status addk_gsi(addk_plan plan, const double *v, double *theta, void *stream)
{
    if (!plan)
        return fail2(ADDK_ERR_INVALID_ARG, "plan is NULL");
    if (!theta)
        return fail2(ADDK_ERR_INVALID_ARG, "theta is NULL");
    Plan &pl = *(Plan *)plan;
    std::memset(theta, 0, sizeof(double) * 8 * pl.P);
    if (pl.flags & ADDK_NEAR_FIELD)
        return fail2(ADDK_ERR_UNSUPPORTED, "addk_gsi: the variances are those of the plain Fourier series; create "
                                           "the plan without ADDK_NEAR_FIELD");
    if (pl.N == 0)
        return ADDK_OK;
    addk_status s;
    if ((s = check_mat(v, pl.nsrc, pl.nsrc, "v", true)) != ADDK_OK)
        return s;
    hipStream_t st = (hipStream_t)stream;
    IoArgs io;
    std::memset(&io, 0, sizeof(io));
    io.single = single_prob(pl);
    io.single.V = v;
    io.single.ldv = pl.nsrc;
    s = engine_run(pl.eng, 1, 0, true, false, io, st);  // spread and forward transform: modes into Vm
    if (s != ADDK_OK)
        return s;
    double *dth = nullptr;
    hipError_t e = hipMalloc(&dth, sizeof(double) * 8 * pl.P);
    if (e != hipSuccess)
        return fail2(ADDK_ERR_OOM, "gsi output allocation failed");
    std::vector<const double *> B64(pl.P);
    for (int w = 0; w < pl.P; ++w)
        B64[w] = pl.wins[w].Bk64;
    s = engine_gsi(pl.eng, B64, pl.d_psi, pl.n, dth, st);
    if (s == ADDK_OK) {
        e = hipMemcpyAsync(theta, dth, sizeof(double) * 8 * pl.P, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            s = hip_fail(e, "gsi result copy");
    }
    (void)hipFree(dth);
    return s;
}

addk_status addk_gsi_indices(addk_plan plan, const double *v, int32_t cap, int32_t *subsets, double *rho,
                             int32_t *count, void *stream)
{
    if (!plan)
        return fail2(ADDK_ERR_INVALID_ARG, "plan is NULL");
    if (!count || cap < 0 || (cap > 0 && (!subsets || !rho)))
        return fail2(ADDK_ERR_INVALID_ARG, "addk_gsi_indices: count, and subsets and rho for cap > 0, are required");
    Plan &pl = *(Plan *)plan;
    std::vector<double> theta(8 * (size_t)pl.P, 0.0);
    addk_status s = addk_gsi(plan, v, theta.data(), stream);
    if (s != ADDK_OK)
        return s;
    // Algorithm 1, last steps: the variance of every feature subset u is the sum
    // of theta over the windows and support masks whose features are u; the
    // indices divide by the total over all nonempty subsets.
    std::vector<std::vector<int32_t>> keys;
    std::vector<double> var;
    for (int w = 0; w < pl.P; ++w) {
        const WinHost &wh = pl.wins[w];
        for (int mask = 1; mask < (1 << wh.d); ++mask) {
            std::vector<int32_t> k;
            for (int i = 0; i < wh.d; ++i)
                if (mask >> i & 1)
                    k.push_back(wh.feat[i]);
            std::sort(k.begin(), k.end());
            size_t j = 0;
            while (j < keys.size() && keys[j] != k)
                ++j;
            if (j == keys.size()) {
                keys.push_back(k);
                var.push_back(0.0);
            }
            var[j] += theta[8 * (size_t)w + mask];
        }
    }
    double total = 0.0;
    for (double x : var)
        total += x;
    *count = (int32_t)keys.size();
    if ((int32_t)keys.size() > cap)
        return fail2(ADDK_ERR_INVALID_ARG, "addk_gsi_indices: " + std::to_string(keys.size()) +
                                               " feature subsets, more than cap = " + std::to_string(cap));
    for (size_t j = 0; j < keys.size(); ++j) {
        for (int i = 0; i < 3; ++i)
            subsets[3 * j + i] = i < (int)keys[j].size() ? keys[j][i] : -1;
        rho[j] = total > 0.0 ? var[j] / total : 0.0;
    }
    return ADDK_OK;
}

addk_status addk_plan_profile(addk_plan plan, int32_t enable)
{
    if (!plan)
        return fail2(ADDK_ERR_INVALID_ARG, "plan is NULL");
    ((Plan *)plan)->eng.prof = enable != 0;
    return ADDK_OK;
}

addk_status addk_plan_profile_read(addk_plan plan, double *total_ms, int32_t *launches)
{
    if (!plan)
        return fail2(ADDK_ERR_INVALID_ARG, "plan is NULL");
    return engine_profile_read(((Plan *)plan)->eng, total_ms, launches);
}

const char *addk_stage_name(int32_t stage)
{
    static const char *names[PS_COUNT] = {"zero",      "spread",    "fft_x_fwd", "fft_y_fwd",    "fft_fused",
                                          "fft_y_inv", "fft_x_inv", "interp",    "combine",      "mode_dot",
                                          "spread_dense", "interp_dense", "gather",       "near"};
    if (stage < 0 || stage >= PS_COUNT)
        return nullptr;
    return names[stage];
}

addk_status addk_batch_create(addk_batch *out, int32_t nprob, const addk_plan *plans, int32_t R,
                              const double *const *V, const int64_t *ldv, double *const *Y, const int64_t *ldy,
                              void *stream)
{
    if (!out || nprob < 1 || !plans || R < 1 || !V || !ldv || !Y || !ldy)
        return fail2(ADDK_ERR_INVALID_ARG, "bad batch arguments");
    *out = nullptr;
    const int prec = ((Plan *)plans[0])->precision;
    for (int p = 0; p < nprob; ++p) {
        if (!plans[p])
            return fail2(ADDK_ERR_INVALID_ARG, "NULL plan in batch");
        const Plan &pl = *(Plan *)plans[p];
        if (pl.precision != prec)
            return fail2(ADDK_ERR_INVALID_ARG, "all plans of a batch must share one precision");
        if (pl.rect)
            return fail2(ADDK_ERR_UNSUPPORTED, "plans with separate targets cannot be batched");
        if (pl.N > 0) {
            addk_status s;
            if ((s = check_mat(V[p], ldv[p], pl.N, "V[p]", true)) != ADDK_OK ||
                (s = check_mat(Y[p], ldy[p], pl.N, "Y[p]", true)) != ADDK_OK)
                return s;
        }
    }
    Batch *b = new (std::nothrow) Batch();
    if (!b)
        return fail2(ADDK_ERR_OOM, "host allocation failed");
    b->R = R;
    Engine &E = b->eng;
    E.nprob = nprob;
    E.probs.resize(nprob);
    for (int p = 0; p < nprob; ++p) {
        Plan *pl = (Plan *)plans[p];
        b->plans.push_back(pl);
        b->gens.push_back(pl->param_gen);
        E.plans.push_back(pl);
        ProbDev &pd = E.probs[p];
        std::memset(&pd, 0, sizeof(pd));
        pd.N = pl->N;
        pd.nsrc = pl->N;
        pd.yoff = 0;
        pd.wbeg = (int)E.wdev.size();
        for (int w = 0; w < pl->P; ++w) {
            WinDev d = pl->eng.wdev[w];
            d.prob = p;
            E.wdev.push_back(d);
            E.wplan.push_back(p);
            E.wlocal.push_back(w);
        }
        pd.wend = (int)E.wdev.size();
        pd.V = V[p];
        pd.ldv = ldv[p];
        pd.Y = Y[p];
        pd.ldy = ldy[p];
    }
    for (int p = 0; p < nprob; ++p)
        E.no_mfma = E.no_mfma || (((Plan *)plans[p])->flags & ADDK_VECTOR_ALU_ONLY);
    addk_status s = engine_build_device(E, prec);
    if (s == ADDK_OK)
        s = engine_ensure_workspace(E, R);
    hipError_t e = hipSuccess;
    if (s == ADDK_OK) {
        e = hipMalloc(&E.d_probs, nprob * sizeof(ProbDev));
        if (e == hipSuccess)
            e = hipMemcpy(E.d_probs, E.probs.data(), nprob * sizeof(ProbDev), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            s = hip_fail(e, "batch problem table");
    }
    if (s == ADDK_OK) {
        e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            s = hip_fail(e, "hipStreamCreate");
    }
    if (s == ADDK_OK)
        s = batch_capture(*b);
    if (s != ADDK_OK) {
        addk_batch_destroy((addk_batch)b);
        return s;
    }
    (void)stream;
    *out = (addk_batch)b;
    return ADDK_OK;
}

addk_status addk_plan_autotune(addk_plan plan, int32_t R, int32_t nout, int32_t reps, uint32_t *knobs, void *stream)
{
    if (!plan)
        return fail2(ADDK_ERR_INVALID_ARG, "plan is NULL");
    if (R < 1 || (nout != 1 && nout != 2) || reps < 1)
        return fail2(ADDK_ERR_INVALID_ARG, "autotune: R >= 1, nout in {1, 2} and reps >= 1 required");
    Plan &pl = *(Plan *)plan;
    Engine &E = pl.eng;
    hipStream_t st = (hipStream_t)stream;
    const std::vector<uint32_t> cand = knob_candidates(E, R);
    if (cand.size() <= 1 || pl.N == 0) {
        E.knobs = cand.empty() ? 0u : cand[0];
        E.tuned = true;
        if (knobs)
            *knobs = E.knobs;
        return ADDK_OK;
    }
    double *V = nullptr, *Y = nullptr, *dl = nullptr;
    const int64_t n = pl.N * (int64_t)R;
    hipError_t e = hipMalloc(&V, n * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc(&Y, n * sizeof(double));
    if (e == hipSuccess && nout == 2)
        e = hipMalloc(&dl, n * pl.P * sizeof(double));
    if (e == hipSuccess)
        e = hipMemsetAsync(V, 0, n * sizeof(double), st);  // timing does not depend on the values
    addk_status s = e == hipSuccess ? ADDK_OK : fail2(ADDK_ERR_OOM, "autotune buffers");
    const uint32_t saved = E.knobs;
    const bool saved_tuned = E.tuned;
    double best = INFINITY;
    uint32_t best_k = saved;
    for (size_t c = 0; c < cand.size() && s == ADDK_OK; ++c) {
        E.knobs = cand[c];
        E.tuned = true;
        double ms = 0.0;
        s = time_runs(
            [&]() {
                return nout == 1 ? addk_matvec(plan, R, V, pl.N, Y, pl.N, stream)
                                 : addk_dmatvec(plan, R, V, pl.N, dl, nullptr, Y, pl.N, stream);
            },
            reps, st, &ms);
        if (s == ADDK_OK && ms < best) {
            best = ms;
            best_k = cand[c];
        }
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(V);
    (void)hipFree(Y);
    (void)hipFree(dl);
    if (s != ADDK_OK) {
        E.knobs = saved;
        E.tuned = saved_tuned;
        return s;
    }
    E.knobs = best_k;
    E.tuned = true;
    tune_cache_put(E, R, nout, best_k);
    if (knobs)
        *knobs = best_k;
    return ADDK_OK;
}

addk_status addk_plan_set_knobs(addk_plan plan, uint32_t knobs)
{
    if (!plan || knobs > (ADDK_KNOB_ALL | ADDK_KNOB_SPARSE_ATOMIC))
        return fail2(ADDK_ERR_INVALID_ARG, "set knobs: plan and knobs <= ADDK_KNOB_ALL | ADDK_KNOB_SPARSE_ATOMIC required");
    Engine &E = ((Plan *)plan)->eng;
    E.knobs = knobs;
    E.tuned = true;
    return ADDK_OK;
}

addk_status addk_tune_cache_lookup(addk_plan plan, int32_t R, int32_t nout, uint32_t *knobs, int32_t *found)
{
    if (!plan || !found || R < 1 || nout < 1 || nout > 2)
        return fail2(ADDK_ERR_INVALID_ARG, "tune cache lookup: plan, found, R >= 1 and nout in {1, 2} required");
    uint32_t k = 0;
    *found = tune_cache_get(((Plan *)plan)->eng, R, nout, &k) ? 1 : 0;
    if (knobs)
        *knobs = k;
    return ADDK_OK;
}

addk_status addk_tune_cache_clear(void)
{
    tune_cache_clear();
    return ADDK_OK;
}

addk_status addk_batch_autotune(addk_batch batch, int32_t reps, uint32_t *knobs, void *stream)
{
    if (!batch)
        return fail2(ADDK_ERR_INVALID_ARG, "batch is NULL");
    if (reps < 1)
        return fail2(ADDK_ERR_INVALID_ARG, "autotune: reps >= 1 required");
    Batch &b = *(Batch *)batch;
    Engine &E = b.eng;
    hipStream_t st = (hipStream_t)stream;
    {
        addk_status s0 = batch_refresh_params(b);
        if (s0 != ADDK_OK)
            return s0;
    }
    const std::vector<uint32_t> cand = knob_candidates(E, b.R);
    const uint32_t saved = E.knobs;
    const bool saved_tuned = E.tuned;
    double best = INFINITY;
    uint32_t best_k = saved;
    addk_status s = ADDK_OK;
    for (size_t c = 0; c < cand.size() && s == ADDK_OK && cand.size() > 1; ++c) {
        E.knobs = cand[c];
        E.tuned = true;
        s = batch_capture(b);
        double ms = 0.0;
        if (s == ADDK_OK)
            s = time_runs(
                [&]() {
                    hipError_t e = hipGraphLaunch(b.exec, st);
                    return e == hipSuccess ? ADDK_OK : hip_fail(e, "hipGraphLaunch");
                },
                reps, st, &ms);
        if (s == ADDK_OK && ms < best) {
            best = ms;
            best_k = cand[c];
        }
    }
    E.knobs = s == ADDK_OK ? (cand.size() > 1 ? best_k : (cand.empty() ? 0u : cand[0])) : saved;
    E.tuned = s == ADDK_OK ? true : saved_tuned;
    addk_status s2 = batch_capture(b);  // the graph of the chosen knobs
    if (s == ADDK_OK)
        s = s2;
    if (s == ADDK_OK && knobs)
        *knobs = E.knobs;
    return s;
}

addk_status addk_batch_launch(addk_batch batch, void *stream)
{
    if (!batch)
        return fail2(ADDK_ERR_INVALID_ARG, "batch is NULL");
    Batch &b = *(Batch *)batch;
    addk_status s = batch_refresh_params(b);
    if (s != ADDK_OK)
        return s;
    hipError_t e = hipGraphLaunch(b.exec, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "hipGraphLaunch");
    return ADDK_OK;
}

addk_status addk_batch_run_eager(addk_batch batch, void *stream)
{
    if (!batch)
        return fail2(ADDK_ERR_INVALID_ARG, "batch is NULL");
    Batch &b = *(Batch *)batch;
    addk_status s = batch_refresh_params(b);
    if (s != ADDK_OK)
        return s;
    return batch_enqueue(b, (hipStream_t)stream);
}

addk_status addk_batch_destroy(addk_batch batch)
{
    if (!batch)
        return fail2(ADDK_ERR_INVALID_ARG, "batch is NULL");
    Batch *b = (Batch *)batch;
    (void)hipDeviceSynchronize();
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->cap_stream)
        (void)hipStreamDestroy(b->cap_stream);
    engine_free(b->eng);
    delete b;
    return ADDK_OK;
}

}  // extern "C"
