/*
 * addk.h -- C ABI of the MI355X (gfx950) additive-kernel fast summation library.
 *
 * The library computes, for points x_1..x_N in R^D, feature windows W_1..W_P
 * (|W_w| = d_w <= 3) and right-hand sides V (N x R):
 *
 *   Y        = sum_w sigma_w^2 K_w V                          (K V)
 *   dY_dl_w  = sigma_w^2 (dK_w/dl_w) V                        (dK/dl_w V)
 *   dY_ds_w  = 2 sigma_w K_w V                                (dK/dsigma_w V)
 *
 * with (K_w)_ij = kappa(||x_i^{W_w} - x_j^{W_w}||; l_w).  The kernel is the
 * windowed additive kernel of eqs. (3), (7)-(8) of Wagner, Nestler & Stoll, "Fast
 * evaluation of additive kernels" (Gaussian, "Implementing the NFFT approach";
 * Matern-1/2 and Matern-3/2, "Extension to other kernels"); its derivatives are those of the
 * same sections.  Each window's product is evaluated by the NFFT-based fast
 * summation of eqs. (4)-(6): window-function spreading onto an oversampled
 * torus grid, FFT, multiplication by the kernel's periodised Fourier
 * coefficients, inverse FFT and interpolation back to the points; the
 * windows are then summed in FP64.  The trigonometric sum of eq. (6) runs
 * over the modes k in {-n/2, ..., n/2-1}^d and its real part is returned.
 *
 * Conventions
 *  - Every entry point returns an addk_status; no exception crosses the ABI.
 *    A descriptive message for the last failure on the calling thread is
 *    available from addk_last_error().
 *  - Arguments are validated before any device work is queued.
 *  - V, Y, G and all gradient/derivative outputs are DEVICE pointers to FP64
 *    column-major N x R matrices with a leading dimension (element (i, r) at
 *    ptr[i + r * ld]).  Outputs are in the caller's point order.
 *  - "stream" is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work is queued on it asynchronously; the call returns before the
 *    results are ready.  A plan must not be used on two streams at once.
 *  - The plan owns its device copies of the sorted points, permutation,
 *    Fourier multipliers and workspace; the caller keeps ownership of every
 *    pointer it passes.  Plan creation is synchronous.
 */
#ifndef ADDK_H
#define ADDK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ADDK_OK = 0,
    ADDK_ERR_INVALID_ARG = 1, /* bad sizes, pointers, parameters                      */
    ADDK_ERR_UNSUPPORTED = 2, /* d_w > 3, grid > 128 per dimension, torus too small   */
    ADDK_ERR_ACCURACY = 3,    /* requested parameters cannot be resolved (eta < 1)    */
    ADDK_ERR_OOM = 4,         /* device or host allocation failed                     */
    ADDK_ERR_HIP = 5          /* a HIP runtime call or kernel launch failed           */
} addk_status;

typedef enum {
    ADDK_GAUSSIAN = 1, /* kappa(r) = exp(-r^2/(2 l^2)); derivative kernel r^2/(2l^2) kappa */
    ADDK_MATERN12 = 3, /* kappa(r) = exp(-r/l);        derivative kernel (r/l) kappa       */
    ADDK_MATERN32 = 5  /* kappa(r) = (1 + a r) exp(-a r), a = sqrt(3)/l ("Extension to other
                          kernels" names it as a further kernel); derivative kernel
                          l dkappa/dl = (a r)^2 exp(-a r)                                   */
} addk_kernel;

typedef enum {
    ADDK_FP64 = 0, /* spreading, FFT and interpolation in FP64                       */
    ADDK_FP32 = 1  /* spreading, FFT and interpolation in FP32 with FP32 accumulation;
                      multipliers are computed in FP64, window sums are FP64          */
} addk_precision;

/* flags for addk_plan_create (bitwise OR) */
#define ADDK_COEF_ANALYTIC 0u   /* coefficients of the periodisation by summation (default)  */
#define ADDK_COEF_SAMPLED 1u    /* DFT of n^d kernel samples of the simple periodic
                                   continuation (Lemma 1 of the paper)                        */
#define ADDK_TORUS_AUTO 0u      /* per-window torus period balancing image/truncation errors  */
#define ADDK_TORUS_PAPER 2u     /* prescaling rule: period 2 * Lmax * sqrt(d_max)              */
#define ADDK_NO_ACCURACY_CHECK 4u /* do not refuse windows with eta < 1                       */
#define ADDK_TILE_KERNELS_ONLY 8u /* route every point through the tile kernels (no dense-cell
                                     kernels); same results up to rounding, for comparison     */
#define ADDK_VECTOR_ALU_ONLY 16u  /* run the dense-cell kernels on the vector ALUs instead of
                                     the matrix cores; for comparison                         */
#define ADDK_NEAR_FIELD 32u       /* Matern kernels only: near-field corrected products (below) */

/*
 * ADDK_NEAR_FIELD.  The Matern-1/2 kernel has a cusp at r = 0, so its
 * truncated Fourier series alone stays near 1e-2 (relative) at n = 64; the
 * Matern-3/2 kernel is smooth at r = 0 only to second order (an r^3 term), so
 * its series stays near 1e-3.  With
 * this flag (regularisation for non-smooth kernels in NFFT-based fast
 * summation, which the kernel extension of section 5 builds on):
 *  - each window's torus period is T_w = 5 L_w / 2 and the periodic kernel has
 *    no images: per coordinate, x^2 is replaced by a smooth even T-periodic
 *    fold that equals x^2 on [-L_w, L_w];
 *  - inside r < eps_w = 5 T_w / n the kernel (and the derivative kernel) is
 *    replaced by the even polynomial of degree 16 that matches its value and
 *    first 8 derivatives at eps_w; the Fourier multipliers are those of this
 *    regularised kernel (DFT of (2n)^d samples);
 *  - pairs closer than eps_w are summed directly with kernel minus polynomial.
 *    With one right-hand side and no separate targets, each such pair is
 *    evaluated once for both of its points (the kernels are symmetric) and the
 *    sums are added atomically: repeated calls then agree to rounding, not to
 *    the bit.
 * Every product (matvec, dmatvec, vjp, batches, targets, CG) then agrees with
 * the direct sum to about 1e-5 relative or better.  The direct part costs
 * O(N x neighbours within eps_w).  Errors: UNSUPPORTED with ADDK_GAUSSIAN,
 * with ADDK_COEF_SAMPLED or ADDK_TORUS_PAPER, for n < 16, and in addk_gsi
 * (whose variances are defined by the plain Fourier series).
 */

typedef struct addk_plan_s *addk_plan;
typedef struct addk_batch_s *addk_batch;

/*
 * Create a plan: points, windows, kernel, parameters and grid sizes.
 *
 *  N, D, X, ldx     N points with D features, row-major (X[j*ldx + f]),
 *                   host or device memory; copied, may be freed on return.
 *                   N >= 0 (N = 0 gives a plan whose products are empty).
 *  P, win_offsets, win_features
 *                   window w uses features win_features[win_offsets[w] ..
 *                   win_offsets[w+1]-1]; 1 <= d_w <= 3; host memory.
 *  kernel           ADDK_GAUSSIAN, ADDK_MATERN12 or ADDK_MATERN32.
 *  ell, sigma       P length scales (> 0) and P amplitudes sigma_w (>= 0), host.
 *                   ell is in the units of X.
 *  n                Fourier bandwidth per dimension (even, >= 4): modes
 *                   k in {-n/2, ..., n/2-1}^d (the paper's m).
 *  m                window half-width in oversampled grid cells (2..8);
 *                   every point touches (2m)^d grid cells.
 *  oversampling     sigma = n_os / n; n_os = round(sigma * n) must be a power
 *                   of two in [16, 256] and exceed n.
 *  precision        ADDK_FP64 or ADDK_FP32.
 *  flags            ADDK_COEF_* | ADDK_TORUS_* | ADDK_NO_ACCURACY_CHECK |
 *                   ADDK_TILE_KERNELS_ONLY | ADDK_VECTOR_ALU_ONLY | ADDK_NEAR_FIELD.
 *  stream           stream used for the set-up kernels.
 * Errors: INVALID_ARG (bad sizes/values/pointers), UNSUPPORTED (d_w > 3,
 * n_os outside [16,256] or not a power of two, data extent plus window wider
 * than the torus), ACCURACY (eta_w = pi n l_w / (sqrt2 T_w) < 1), OOM, HIP.
 */
addk_status addk_plan_create(addk_plan *out, int64_t N, int32_t D, const double *X, int64_t ldx,
                             int32_t P, const int32_t *win_offsets, const int32_t *win_features,
                             int32_t kernel, const double *ell, const double *sigma,
                             int32_t n, int32_t m, double oversampling,
                             int32_t precision, uint32_t flags, void *stream);

/*
 * A plan whose products are evaluated at separate target points x'_1..x'_Nt
 * (eq. (4) with x' != x, e.g. prediction points):
 *   Y_i = sum_w sigma_w^2 sum_j kappa(||x'_i^{W_w} - x_j^{W_w}||; l_w) V_j.
 * Xs (Ns x D) are the sources, Xt (Nt x D) the targets, row-major with their
 * own leading dimensions, host or device, copied.  Torus periods and grid
 * boxes cover sources and targets together.  The plan then serves
 * addk_matvec / addk_dmatvec with V of Ns rows and Y (and the derivative
 * outputs) of Nt rows, addk_gsi with v of Ns rows; addk_vjp and batches need
 * square plans (ADDK_ERR_UNSUPPORTED).  Other arguments and errors as in
 * addk_plan_create.  Sources and targets are sorted separately: the sources
 * are spread and the targets interpolated (and, with ADDK_NEAR_FIELD, each
 * target meets only the sources within the near-field radius).
 */
addk_status addk_plan_create_targets(addk_plan *out, int64_t Ns, int64_t Nt, int32_t D, const double *Xs,
                                     int64_t ldxs, const double *Xt, int64_t ldxt, int32_t P,
                                     const int32_t *win_offsets, const int32_t *win_features, int32_t kernel,
                                     const double *ell, const double *sigma, int32_t n, int32_t m,
                                     double oversampling, int32_t precision, uint32_t flags, void *stream);

/*
 * Y = sum_w sigma_w^2 K_w V (eqs. (4)-(6) per window, then the window sum of
 * eq. (7)).  V: N x R (ldv >= N), Y: N x R (ldy >= N); device pointers.
 * R >= 1.  V and Y must not overlap.
 */
addk_status addk_matvec(addk_plan plan, int32_t R, const double *V, int64_t ldv,
                        double *Y, int64_t ldy, void *stream);

/*
 * addk_matvec for callers that cannot allocate device memory: code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, products and errors as addk_matvec, and the same stage
 * kernels; the per-call workspace (grids, per-window FP64 products, the
 * point-major RHS copy, the dense spread's per-item blocks, near-field
 * close-pair sums) is taken from one fixed array of 256 MiB per GPU that the
 * library holds from load until the process ends, instead of from buffers the
 * plan allocates.  The call allocates nothing; it uploads the plan's window
 * descriptors with a synchronous copy (so it synchronises the device first)
 * and then queues the kernels on `stream`.  The plan's device must be the
 * current device.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams or two threads) race; results of calls
 * queued on one stream are independent.  Errors: as addk_matvec, and
 * INVALID_ARG when the workspace for this plan and R exceeds 256 MiB (the
 * message gives the size needed; call addk_matvec or split the RHS).
 */
addk_status addk_matvec_noalloc(addk_plan plan, int32_t R, const double *V, int64_t ldv,
                                double *Y, int64_t ldy, void *stream);

/*
 * Derivative products ("Implementing the NFFT approach", "Extension to other
 * kernels"): one spreading and forward FFT per window feed both the kernel's
 * and the derivative kernel's multipliers.
 *   dY_dell  : P blocks of N x R, block w at dY_dell + w * ldy * R:
 *              sigma_w^2 (dK_w/dl_w) V = sigma_w^2 (2/l_w) K_der,w V (Gaussian)
 *                                      = sigma_w^2 (1/l_w) K_derM,w V (Matern-1/2, -3/2)
 *   dY_dsigma: P blocks, 2 sigma_w K_w V
 *   Y        : sum_w sigma_w^2 K_w V
 * Any of the three may be NULL (not all three).  All use leading dimension ldy.
 */
addk_status addk_dmatvec(addk_plan plan, int32_t R, const double *V, int64_t ldv,
                         double *dY_dell, double *dY_dsigma, double *Y, int64_t ldy,
                         void *stream);

/*
 * Vector-Jacobian product of Y = K(l, sigma) V for a cotangent G (N x R):
 *   grad_V         = K G        (K is symmetric)               N x R, ld ldgv
 *   grad_ell[w]    = <G, sigma_w^2 dK_w/dl_w V>                 P doubles, device
 *   grad_sigma[w]  = <G, 2 sigma_w K_w V>                       P doubles, device
 * The scalar gradients are computed as Fourier-domain inner products of the
 * spread-and-transformed G and V with the multipliers, so they are the exact
 * derivatives of the approximate operator with the torus frozen.  Any output
 * may be NULL.  ldv, ldg, ldgv >= N.
 */
addk_status addk_vjp(addk_plan plan, int32_t R, const double *V, int64_t ldv,
                     const double *G, int64_t ldg, double *grad_V, int64_t ldgv,
                     double *grad_ell, double *grad_sigma, void *stream);

/*
 * Conjugate gradients for the kernel ridge regression system of eq. (9),
 * (K + beta I) X = Y, with K the plan's product (square plans only).  The R
 * columns are solved together, each with its own step sizes, until
 * ||Y - (K + beta I) X||_2 <= tol ||Y||_2 per column (residual recurrence) or
 * maxit iterations.  X holds the initial guess on entry and the solution on
 * return; Y and X are device FP64, column-major, ld >= N.  iters (host, may
 * be NULL) receives the iterations run, relres (host, R doubles, may be NULL)
 * the final relative residuals.  Synchronous (the host checks convergence
 * each iteration).  Errors: INVALID_ARG, UNSUPPORTED (plan with separate
 * targets), OOM, HIP.
 */
addk_status addk_cg(addk_plan plan, double beta, int32_t R, const double *Y, int64_t ldy, double *X, int64_t ldx,
                    double tol, int32_t maxit, int32_t *iters, double *relres, void *stream);

/*
 * Global sensitivity analysis of the fitted function h(x) = sum_j v_j K(x, x_j)
 * (section "Computing the GSI in the kernel setting", Algorithm 1).  For each
 * window w, its trigonometric approximation sum_k w_k b_k a_k e^{2 pi i k x}
 * (the same coefficients as the products; a_k = sum_j v_j e^{-2 pi i k x_j}
 * on the window's torus) is split by the support of k: theta[8 w + mask] is
 * the sum of |w_k b_k a_k|^2 over the modes k with k_i != 0 exactly for the
 * bits i set in mask (bit i = i-th feature of the window; mask 0 is the
 * constant term, not part of the variance).  The amplitudes sigma_w do not
 * enter.  Summing theta over windows per feature subset and dividing by the
 * total over nonzero masks gives the indices rho_u.
 *   v      N doubles, device (one right-hand side)
 *   theta  8 P doubles, host; written on return (synchronous)
 * Errors: INVALID_ARG, OOM, HIP.
 */
addk_status addk_gsi(addk_plan plan, const double *v, double *theta, void *stream);

/*
 * The global sensitivity indices of Algorithm 1 (section "Computing the GSI
 * in the kernel setting") over all windows: addk_gsi's theta summed, per
 * feature subset u (of the plan's feature indices), over every window and
 * support mask whose features are u, divided by the total over all nonempty
 * subsets, so the indices sum to 1 (all 0 if the total is 0).
 *   v        N doubles, device (one right-hand side)
 *   cap      room in subsets / rho (at most 7 P subsets occur)
 *   subsets  host int32 [cap][3]: the subset's features ascending, -1 padded
 *   rho      host double [cap]: the index of each subset
 *   count    host: the number of subsets (set also when it exceeds cap)
 * Subsets are listed in order of first appearance (windows in order, masks
 * ascending).  Synchronous.  Errors: as addk_gsi; INVALID_ARG when count > cap.
 */
addk_status addk_gsi_indices(addk_plan plan, const double *v, int32_t cap, int32_t *subsets, double *rho,
                             int32_t *count, void *stream);

/* Replace l_w and sigma_w (host arrays of P) and recompute the multipliers; the
 * torus periods, grids and point sort are kept, so products stay differentiable
 * in l.  Errors: INVALID_ARG, ACCURACY (as in addk_plan_create). */
addk_status addk_plan_update_params(addk_plan plan, const double *ell, const double *sigma,
                                    void *stream);

/*
 * Kernel-variant knobs: which stages run on the matrix cores
 * (v_mfma_f32_16x16x4f32; FP64 plans: v_mfma_f64_16x16x4f64, with R >= 2)
 * instead of the vector ALUs.  Both variants compute the same products; they
 * differ in speed and in summation order.
 */
#define ADDK_KNOB_SPREAD_MFMA 1u       /* dense-cell spreading (d = 3)      */
#define ADDK_KNOB_INTERP_DENSE_MFMA 2u /* dense-cell interpolation (d = 3)  */
#define ADDK_KNOB_INTERP_TILE_MFMA 4u  /* sparse-tile interpolation (d = 3) */
#define ADDK_KNOB_ALL_MFMA 7u
/* Work shape of the matrix-core dense spread (FP32, R >= 2): its taps' M tiles
 * split over 3 (2m = 12) or 2 (2m = 8) blocks per item, each evaluating the
 * window values again, for fewer accumulators and more blocks per CU.  FP64
 * always splits.  Same products, other block shape. */
#define ADDK_KNOB_SPREAD_SPLIT 8u
#define ADDK_KNOB_ALL 15u
/* Sparse d = 3 points spread per point tile into a register sub-grid that is
 * added to the grid with atomic adds, instead of by output tiles that write
 * every grid value once.  Faster where sparsely populated cells hold many of
 * the points (each point is then read once, not by every output tile it
 * reaches), but the sums' order depends on timing: the products are no longer
 * bitwise reproducible.  Never chosen by the autotuner; set it with
 * addk_plan_set_knobs. */
#define ADDK_KNOB_SPARSE_ATOMIC 16u

/* Plan facts.  Arrays are host memory with room for P entries (any may be NULL). */
typedef struct {
    int64_t N;
    int32_t P;
    int32_t n, m, n_os, precision, kernel;
    int64_t workspace_bytes;    /* device bytes currently held by the plan           */
    double err_estimate;        /* a-priori relative error estimate (max over windows) */
    int64_t dense_points;       /* source point-window pairs spread by the dense-cell kernels */
    int64_t tile_points;        /* source point-window pairs spread by the tile kernels       */
    uint32_t knobs;             /* ADDK_KNOB_* in effect                                 */
    int32_t tuned;              /* 1 once addk_plan_autotune chose the knobs             */
    int64_t n_sources;          /* rows of V (= N unless the plan has separate targets) */
    int64_t n_targets;          /* rows of Y                                             */
} addk_plan_info;
addk_status addk_plan_query(addk_plan plan, addk_plan_info *info, double *torus_period,
                            double *eta, int32_t *window_dim);

addk_status addk_plan_destroy(addk_plan plan);

/*
 * Batched products of many independent plans (uneven N, mixed d) with one
 * fixed set of device buffers: the whole sequence of stage kernels of all
 * plans is captured once into a hipGraph; every addk_batch_launch replays it.
 * Each stage kernel covers the windows of all plans in a single launch.
 *  plans[p]  plans of identical precision (they must outlive the batch)
 *  R         RHS per problem (same for all)
 *  V[p], ldv[p], Y[p], ldy[p]   device buffers bound to the graph (host arrays
 *            of nprob device pointers / leading dimensions).
 * addk_plan_update_params on a plan of the batch takes effect at the batch's
 * next launch (launch, eager run or autotune), which then uploads the new
 * parameters synchronously before queueing the work; the graph is kept.
 * Errors: INVALID_ARG, OOM, HIP.
 */
addk_status addk_batch_create(addk_batch *out, int32_t nprob, const addk_plan *plans, int32_t R,
                              const double *const *V, const int64_t *ldv,
                              double *const *Y, const int64_t *ldy, void *stream);
/*
 * Autotuner.  Times every applicable combination of ADDK_KNOB_* on this plan
 * (products of R right-hand sides; nout = 1: addk_matvec, 2: addk_dmatvec
 * with K V and dK/dl V) or on this batch (graph replays), `reps` timed runs
 * each after one warm-up, keeps the fastest combination and returns it in
 * *knobs (may be NULL).  Temporary inputs are allocated and freed inside.
 * Synchronous.
 * Errors: INVALID_ARG, OOM, HIP.
 */
addk_status addk_plan_autotune(addk_plan plan, int32_t R, int32_t nout, int32_t reps, uint32_t *knobs,
                               void *stream);
/* Set the plan's knobs directly (ADDK_KNOB_* mask, <= ADDK_KNOB_ALL | ADDK_KNOB_SPARSE_ATOMIC), as if
 * chosen by addk_plan_autotune (no RHS thresholds, the tuning cache is not
 * consulted); e.g. to reuse a choice measured before.  Knobs a stage cannot
 * use are ignored.  Errors: INVALID_ARG. */
addk_status addk_plan_set_knobs(addk_plan plan, uint32_t knobs);
/*
 * Tuning cache.  addk_plan_autotune also records its choice under the plan's
 * shape: (device, the set of window dimensions, the largest oversampled grid
 * edge, m, R, the power of two at or below the largest window's point count,
 * precision, nout).  A plan that was not tuned itself runs its products with
 * the recorded knobs of its shape (R and nout of the call), if there are any;
 * otherwise with its own.  Process-wide, thread-safe, never evicted.
 *  addk_tune_cache_lookup: *found = 1 and *knobs (may be NULL) the recorded
 *  knobs of the plan's shape at (R, nout in {1, 2}), else *found = 0.
 *  addk_tune_cache_clear: forget every entry.
 * Errors: INVALID_ARG.
 */
addk_status addk_tune_cache_lookup(addk_plan plan, int32_t R, int32_t nout, uint32_t *knobs, int32_t *found);
addk_status addk_tune_cache_clear(void);
addk_status addk_batch_autotune(addk_batch batch, int32_t reps, uint32_t *knobs, void *stream);

/* Y[p] = K_p V[p] for all p: replays the captured graph on the stream. */
addk_status addk_batch_launch(addk_batch batch, void *stream);
/* The same products, launched eagerly (no graph); for comparison and debugging. */
addk_status addk_batch_run_eager(addk_batch batch, void *stream);
addk_status addk_batch_destroy(addk_batch batch);

/*
 * Stage timing for measurement.  When enabled, a pair of HIP events is recorded
 * on the call's stream around every stage kernel launch of the plan's products
 * (asynchronous; no synchronisation is added to the products themselves).
 * addk_plan_profile_read synchronises the device, returns the summed kernel
 * time in milliseconds and the number of launches per stage since the last
 * read, and clears them.  Stage ids: see addk_stage_name (0 .. ADDK_NSTAGES-1).
 * Errors: INVALID_ARG (NULL plan), HIP.
 */
#define ADDK_NSTAGES 14
addk_status addk_plan_profile(addk_plan plan, int32_t enable);
addk_status addk_plan_profile_read(addk_plan plan, double *total_ms, int32_t *launches);
/* "zero", "spread", "fft_x_fwd", "fft_y_fwd", "fft_fused", "fft_y_inv",
 * "fft_x_inv", "interp", "combine", "mode_dot", "spread_dense", "interp_dense",
 * "gather", "near"; NULL for other ids.  Spreading and interpolation run in two kernels: tile
 * kernels for sparsely populated cells and dense-cell kernels. */
const char *addk_stage_name(int32_t stage);

/* ---- host-only helpers (no GPU needed) ---------------------------------- */

/* Torus period of a window: rule ADDK_TORUS_AUTO or ADDK_TORUS_PAPER.
 * L = maximal per-coordinate extent of the window's points, dmax = largest
 * window dimension of the plan (PAPER rule only). */
addk_status addk_torus_period(int32_t kernel, double L, double ell, int32_t n, uint32_t rule,
                              int32_t dmax, double *T);

/* Smallest bandwidth n for one window of extent L (largest per-coordinate
 * range of its points, data units) and length scale l whose a-priori error
 * estimate (image, truncation and window terms, automatic torus period) is at
 * most tol, among the n the library supports for this m and oversampling
 * (round(oversampling n) a power of two in [16, 256], eta >= 1, data box
 * inside the torus).  For a plan, take the largest n over its windows.
 * err_estimate (optional) receives the estimate at the chosen n.
 * Errors: INVALID_ARG; ACCURACY when no supported n reaches tol. */
addk_status addk_choose_n(int32_t kernel, double L, double ell, int32_t m, double oversampling, double tol,
                          int32_t *n, double *err_estimate);

/* The bandwidth for a whole plan: addk_choose_n for every window, with L the
 * largest per-feature range of the window's points, and the largest of those
 * n.  X is N x D row-major (X[j*ldx + f]), host or device memory (device: the
 * ranges are reduced on the GPU, on `stream`); windows as in addk_plan_create.
 * err_estimate (optional) receives the largest per-window estimate at the
 * chosen n.  Synchronous.  Errors: INVALID_ARG; ACCURACY when some window
 * reaches tol with no supported n; OOM, HIP. */
addk_status addk_choose_n_windows(int32_t kernel, int64_t N, int32_t D, const double *X, int64_t ldx, int32_t P,
                                  const int32_t *win_offsets, const int32_t *win_features, const double *ell,
                                  int32_t m, double oversampling, double tol, int32_t *n, double *err_estimate,
                                  void *stream);

/* Fourier transform of the normalised Kaiser-Bessel window used for spreading,
 * Psi(k) = int psi(z) e^{-2 pi i z k / n_os} dz, evaluated by Gauss-Legendre
 * quadrature; psi(0) = 1. */
addk_status addk_window_ft(int32_t m, int32_t n_os, double oversampling_b, double k, double *value);

const char *addk_status_string(addk_status s);
const char *addk_last_error(void);
const char *addk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ADDK_H */
