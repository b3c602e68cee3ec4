// Plan construction (torus map, grid box, tile sort) and the Fourier
// multipliers of the NFFT-based fast summation.
//
// Torus map ("Scaling the data" section, generalised per window): a window's
// points are centred on their bounding box and divided by a torus period T_w,
// x~ = (x - c_w) / T_w, so that all differences lie well inside one period.
// T_w follows either the automatic rule (the image error of the periodised
// kernel balanced against the error of truncating its Fourier series to
// |k| <= n/2) or the paper's prescaling rule.
//
// Multipliers: the trigonometric sum of eq. (6) uses coefficients c_k of the
// T-periodic kernel, either the continuous Fourier transform sampled at k/T
// (periodisation by summation) or the DFT of n^d kernel samples (Lemma 1).
// The real part of the sum over the non-symmetric index set I_n equals the sum
// over k in {-n/2..n/2}^d with weight 1/2 on modes that lie in exactly one of
// I_n and -I_n; that symmetric form keeps real inputs real, which lets two
// real right-hand sides share one complex grid.  The window deconvolution
// 1 / prod_i Psi(k_i)^2 (Psi: Fourier transform of the spreading window) is
// folded into the same array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "addk_internal.h"

namespace addk {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

addk_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return ADDK_ERR_HIP;
}

static addk_status fail(addk_status s, const std::string &msg)
{
    set_error(msg);
    return s;
}

// ADDK_LOG=1 prints plan facts and set-up timings to stderr.
static bool log_on()
{
    static const bool on = [] {
        const char *v = std::getenv("ADDK_LOG");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}

static double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// host math

static double kb_psi_host(double z, int m, double b)
{
    const double mm = m;
    double s2 = mm * mm - z * z;
    if (s2 < 0.0)
        s2 = 0.0;
    double s = std::sqrt(s2);
    const double ie = 1.0 / (1.0 - std::exp(-2.0 * b * mm));
    if (s < 1e-12)
        return mm * 2.0 * b * std::exp(-b * mm) * ie;
    return mm * (std::exp(b * (s - mm)) - std::exp(-b * (s + mm))) * ie / s;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), z1, dp;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            dp = n * (z * p1 - p2) / (z * z - 1.0);
            z1 = z;
            z = z1 - p1 / dp;
            if (std::fabs(z - z1) < 1e-16)
                break;
        }
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
            const double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        dp = n * (z * p1 - p2) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Psi(k) = int_{-m}^{m} psi(z) cos(2 pi z k / nos) dz (psi is even and smooth on
// [-m, m], so Gauss-Legendre converges quickly).
static double window_ft(int m, int nos, double b, double k)
{
    static std::mutex mu;
    static std::vector<double> gx, gw;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (gx.empty())
            gauss_legendre(160, gx, gw);
    }
    double s = 0.0;
    for (size_t q = 0; q < gx.size(); ++q) {
        const double z = m * gx[q];
        s += gw[q] * kb_psi_host(z, m, b) * std::cos(2.0 * M_PI * z * k / nos);
    }
    return m * s;
}

static double torus_period(int kernel, double L, double ell, int n, uint32_t rule, int dmax)
{
    if ((rule & ADDK_TORUS_PAPER) && L > 0.0)
        return 2.0 * L * std::sqrt((double)dmax);
    if (kernel == ADDK_GAUSSIAN)
        return 0.5 * (L + std::sqrt(L * L + 4.0 * M_PI * ell * ell * n));
    if (kernel == ADDK_MATERN32)  // image factor e^{-sqrt3 (T - L) / l} at the n^-3 truncation level
        return L + std::sqrt(3.0) * ell * std::log((double)n);
    return L + ell * std::log((double)n);
}

// ---------------------------------------------------------------------------
// Near-field correction of the Matern-1/2 kernel (ADDK_NEAR_FIELD).  The cusp
// of exp(-r/l) at r = 0 is moved into a compactly supported near-field kernel
// summed directly over close pairs; the rest is smooth and periodic and goes
// through the Fourier method:
//   period      T = 5 L / 2 (L by l if all points coincide), with each coordinate's square x^2 replaced by a
//               fold s(x) = x^2 (1 - h) + (T - x)^2 h on [0, T) (h: degree-7
//               smoothstep from x = L to x = T - L), so that the periodic
//               kernel equals the true one for every difference of two points;
//   radius      eps = 5 T / n;
//   polynomial  p(r) = sum_j a_j (r / eps)^(2j), j <= 8, with the value and the
//               first 8 derivatives of the kernel at eps;
//   near field  K_NE(r) = kappa(r) - p(r) for r < eps, 0 beyond;
//   multipliers DFT of (2n)^d samples of kappa(sqrt(sum_i s(x_i))) - K_NE(|x|).
// The derivative kernel (r/l) e^{-r/l} gets its own polynomial.
constexpr double kNearFold = 2.5;
constexpr double kNearRadius = 5.0;  // in units of T / n

// Half-width of the unfolded region: L, or l when all points coincide (L = 0),
// so that the radius 5 T / n = 12.5 L_f / n stays inside it for n >= 16.
static double near_fold_width(double L, double ell) { return L > 0.0 ? L : ell; }

// Solve sum_j a_j C(2j, s) = eps^s kappa^(s)(eps) / s!, s = 0..q (the Taylor
// conditions at t = r / eps = 1, rows divided by s!), by Gaussian elimination
// with partial pivoting.  Matern-1/2: kappa^(s)(r) = (-1/l)^s e^{-r/l} for
// exp(-r/l) and (-1/l)^s e^{-r/l} (r - s l) / l for (r/l) e^{-r/l}.
// Matern-3/2, a = sqrt3 / l: (-a)^s e^{-a r} (1 + a r - s) for (1 + a r) e^{-a r}
// and (-a)^s e^{-a r} ((a r)^2 - 2 s a r + s (s - 1)) for (a r)^2 e^{-a r}
// (Leibniz on r^k e^{-a r}).
static void near_poly(int kernel, double ell, double eps, bool der, double *a)
{
    constexpr int Q = kNearQ + 1;
    double A[Q][Q + 1];
    double fact = 1.0;
    for (int s = 0; s < Q; ++s) {
        if (s > 0)
            fact *= s;
        for (int j = 0; j < Q; ++j) {
            double c = 0.0;  // binomial C(2j, s)
            if (s <= 2 * j) {
                c = 1.0;
                for (int i = 0; i < s; ++i)
                    c = c * (2 * j - i) / (i + 1);
            }
            A[s][j] = c;
        }
        if (kernel == ADDK_MATERN32) {
            const double ae = std::sqrt(3.0) * eps / ell;
            const double e = std::exp(-ae) * std::pow(-ae, (double)s);
            A[s][Q] = (der ? e * (ae * ae - 2.0 * s * ae + s * (s - 1.0)) : e * (1.0 + ae - s)) / fact;
        } else {
            const double e = std::exp(-eps / ell) * std::pow(-eps / ell, (double)s);
            A[s][Q] = (der ? e * (eps - s * ell) / ell : e) / fact;
        }
    }
    for (int c = 0; c < Q; ++c) {
        int piv = c;
        for (int r = c + 1; r < Q; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c]))
                piv = r;
        for (int k = 0; k <= Q; ++k)
            std::swap(A[c][k], A[piv][k]);
        for (int r = c + 1; r < Q; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int k = c; k <= Q; ++k)
                A[r][k] -= f * A[c][k];
        }
    }
    for (int c = Q - 1; c >= 0; --c) {
        double v = A[c][Q];
        for (int k = c + 1; k < Q; ++k)
            v -= A[c][k] * a[k];
        a[c] = v / A[c][c];
    }
}

static void near_setup(WinHost &w, int kernel, int n)
{
    w.nf_eps = kNearRadius * w.T / n;
    near_poly(kernel, w.ell, w.nf_eps, false, w.nf_a);
    near_poly(kernel, w.ell, w.nf_eps, true, w.nf_ad);
}

// A-priori relative error estimate of one window: image + truncation + window terms.
static double error_estimate(int kernel, double L, double T, double ell, int n, int m, double sig)
{
    double img, trunc;
    if (kernel == ADDK_GAUSSIAN) {
        img = std::exp(-(T - L) * (T - L) / (2.0 * ell * ell));
        trunc = std::exp(-2.0 * M_PI * M_PI * ell * ell * (n / 2.0) * (n / 2.0) / (T * T));
    } else if (kernel == ADDK_MATERN32) {
        // kernel value at the nearest image; tail of the transform beyond n / (2T)
        // (coefficients decaying like |k|^-(d+3)), in one dimension
        const double ai = std::sqrt(3.0) * (T - L) / ell;
        img = (1.0 + ai) * std::exp(-ai);
        const double q = T / (ell * n);
        trunc = 12.0 / (std::sqrt(3.0) * M_PI * M_PI * M_PI * M_PI) * q * q * q;
    } else {
        img = std::exp(-(T - L) / ell);
        trunc = T / (M_PI * M_PI * ell * n);
    }
    const double win = 4.0 * std::exp(-2.0 * M_PI * m * std::sqrt(1.0 - 1.0 / sig));
    return img + trunc + win;
}

// ---------------------------------------------------------------------------
// plan kernels

__global__ void k_minmax(const double *__restrict__ X, int64_t ldx, int64_t N, int d, int f0, int f1, int f2,
                         double *partial)
{
    __shared__ double red[6][256];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int f[3] = {f0, f1, f2};
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x)
        for (int dd = 0; dd < d; ++dd) {
            const double x = X[j * ldx + f[dd]];
            mn[dd] = fmin(mn[dd], x);
            mx[dd] = fmax(mx[dd], x);
        }
    for (int dd = 0; dd < 3; ++dd) {
        red[dd][threadIdx.x] = mn[dd];
        red[3 + dd][threadIdx.x] = mx[dd];
    }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int dd = 0; dd < 3; ++dd) {
                red[dd][threadIdx.x] = fmin(red[dd][threadIdx.x], red[dd][threadIdx.x + s]);
                red[3 + dd][threadIdx.x] = fmax(red[3 + dd][threadIdx.x], red[3 + dd][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6)
        partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

struct KeyArgs {
    int d, nos, m, W, cpt;
    int64_t nsrc;   // points at or after nsrc form the second (target) segment, if split
    int32_t nkeys;  // keys per segment
    int split;
    int f[3];
    double c[3];
    double invT;
    int lo[3], ext[3], tb[3], ntile[3];
};

template <typename real>
__device__ __forceinline__ int base_cell_p(real u, int m)
{
    return (int)floor(u) - m + 1;
}

// grid coordinate relative to the box, rounded to the plan's precision; tile key
template <typename real>
__global__ void k_keys(const double *__restrict__ X, int64_t ldx, int64_t N, KeyArgs a, real *ucoord,
                       int32_t *key, int32_t *hist, int32_t *bad, int nhist_lds)
{
    // Few keys (d = 1 windows: a few hundred cells for 1e6 points): the counts
    // gather in a block-private LDS histogram first, so that the global atomics
    // are one per block and non-empty key, not one per point.
    extern __shared__ int32_t lh[];
    for (int k = threadIdx.x; k < nhist_lds; k += blockDim.x)
        lh[k] = 0;
    if (nhist_lds)
        __syncthreads();
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        int t[3] = {0, 0, 0}, b3[3] = {0, 0, 0};
        bool ok = true;
        for (int dd = 0; dd < a.d; ++dd) {
            const double x = X[j * ldx + a.f[dd]];
            const double u = ((x - a.c[dd]) * a.invT + 0.5) * a.nos - a.lo[dd];
            const real ur = (real)u;
            ucoord[dd * N + j] = ur;
            const int b = base_cell_p(ur, a.m);
            b3[dd] = b;
            if (b < 0 || b + a.W > a.ext[dd])
                ok = false;
            t[dd] = b / a.tb[dd];
            if (t[dd] >= a.ntile[dd])
                ok = false;
        }
        if (!ok) {
            atomicOr(bad, 1);
            key[j] = 0;
            continue;
        }
        // cell key: tile-major, then the base cell inside the tile
        const int tl = t[0] + a.ntile[0] * (t[1] + a.ntile[1] * t[2]);
        const int c = (b3[0] - t[0] * a.tb[0]) + a.tb[0] * ((b3[1] - t[1] * a.tb[1]) + a.tb[1] * (b3[2] - t[2] * a.tb[2]));
        const int k = tl * a.cpt + c + (a.split && j >= a.nsrc ? a.nkeys : 0);
        key[j] = k;
        if (nhist_lds)
            atomicAdd(&lh[k], 1);
        else
            atomicAdd(&hist[k], 1);
    }
    if (nhist_lds) {
        __syncthreads();
        for (int k = threadIdx.x; k < nhist_lds; k += blockDim.x)
            if (lh[k])
                atomicAdd(&hist[k], lh[k]);
    }
}

// Place the points in their sorted positions.  (ks, js) are the (key, index)
// pairs sorted by key with a stable radix sort, so the points of one key come
// in increasing index order; the point at sorted rank idx goes to off[k] plus
// its rank among its key's points, idx - kstart[k] (kstart: exclusive prefix
// sum of the key counts in key order; off: the key's first position in the
// plan's order).  The result does not depend on scheduling.
template <typename real>
__global__ void k_place(int64_t N, int d, const real *__restrict__ ucoord, const uint32_t *__restrict__ ks,
                        const int32_t *__restrict__ js, const int32_t *__restrict__ off,
                        const int32_t *__restrict__ kstart, real *sorted, int32_t *perm)
{
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < N; idx += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = ks[idx];
        const int32_t j = js[idx];
        const int64_t pos = off[k] + (idx - kstart[k]);
        for (int dd = 0; dd < d; ++dd)
            sorted[dd * N + pos] = ucoord[dd * N + j];
        perm[pos] = j;
    }
}

__global__ void k_iota(int32_t *a, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (int32_t)i;
}

// Continuous Fourier transform of the kernel (der = 0) or of its derivative
// kernel (der = 1) at squared frequency xi2, in d dimensions.
__device__ double kernel_ft_dev(int kernel, double xi2, double ell, int d, int der)
{
    const double pi = 3.14159265358979323846;
    if (kernel == ADDK_GAUSSIAN) {
        const double base = pow(ell * sqrt(2.0 * pi), (double)d) * exp(-2.0 * pi * pi * ell * ell * xi2);
        return der ? (0.5 * d - 2.0 * pi * pi * ell * ell * xi2) * base : base;
    }
    const double u = 4.0 * pi * pi * ell * ell * xi2;
    if (kernel == ADDK_MATERN32) {
        // the Matern spectral density at smoothness 3/2: c_d l^d (1 + u/3)^{-(d+3)/2},
        // c_d = int_{R^d} (1 + a|x|) e^{-a|x|} dx / l^d with a = sqrt3 / l
        const double cd = d == 1 ? 4.0 / sqrt(3.0) : (d == 2 ? 2.0 * pi : 32.0 * pi / (3.0 * sqrt(3.0)));
        const double u3 = u / 3.0;
        const double base = cd * pow(ell, (double)d) / pow(1.0 + u3, 0.5 * (d + 3));
        return der ? (d - (d + 3) * u3 / (1.0 + u3)) * base : base;  // l d/dl of the transform
    }
    const double cd = d == 1 ? 2.0 : (d == 2 ? 2.0 * pi : 8.0 * pi);
    const double base = cd * pow(ell, (double)d) / pow(1.0 + u, 0.5 * (d + 1));
    return der ? (d - (d + 1) * u / (1.0 + u)) * base : base;
}

__device__ __forceinline__ double herm_weight(const int *k, int d, int half)
{
    int kp = 0, km = 0;
    for (int i = 0; i < d; ++i) {
        kp += k[i] == half;
        km += k[i] == -half;
    }
    return 0.5 * ((kp == 0 ? 1.0 : 0.0) + (km == 0 ? 1.0 : 0.0));
}

__global__ void k_coef_analytic(double *Bk, double *Bd, int d, int n, double T, double ell, int kernel,
                                const double *__restrict__ psi)
{
    const int n1 = n + 1, half = n / 2;
    int64_t tot = n1;
    for (int i = 1; i < d; ++i)
        tot *= n1;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
        int k[3] = {0, 0, 0}, c[3] = {0, 0, 0};
        int64_t r = idx;
        double xi2 = 0.0, dec = 1.0;
        for (int i = 0; i < d; ++i) {
            c[i] = (int)(r % n1);
            r /= n1;
            k[i] = c[i] - half;
            xi2 += (double)k[i] * k[i];
            dec /= psi[c[i]] * psi[c[i]];
        }
        xi2 /= T * T;
        const double om = herm_weight(k, d, half) * dec / pow(T, (double)d);
        Bk[idx] = om * kernel_ft_dev(kernel, xi2, ell, d, 0);
        Bd[idx] = om * kernel_ft_dev(kernel, xi2, ell, d, 1);
    }
}

// kernel samples kappa(T j / n), j in I_n^d (array index j + n/2 per axis); complex output
__global__ void k_samples(double2 *s, int d, int n, double T, double ell, int kernel, int der)
{
    int64_t tot = n;
    for (int i = 1; i < d; ++i)
        tot *= n;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = idx;
        double r2 = 0.0;
        for (int i = 0; i < d; ++i) {
            const int j = (int)(r % n) - n / 2;
            r /= n;
            const double x = T * j / n;
            r2 += x * x;
        }
        double v;
        if (kernel == ADDK_GAUSSIAN) {
            const double e = exp(-r2 / (2.0 * ell * ell));
            v = der ? r2 / (2.0 * ell * ell) * e : e;
        } else if (kernel == ADDK_MATERN32) {
            const double ar = sqrt(3.0 * r2) / ell;
            const double e = exp(-ar);
            v = der ? ar * ar * e : (1.0 + ar) * e;
        } else {
            const double rr = sqrt(r2);
            const double e = exp(-rr / ell);
            v = der ? rr / ell * e : e;
        }
        s[idx] = make_double2(v, 0.0);
    }
}

// exp(-2 pi i q / M), q < M, on the device (caller frees)
static hipError_t dft_twiddles(int M, double2 **out)
{
    std::vector<double2> t(M);
    for (int q = 0; q < M; ++q)
        t[q] = make_double2(std::cos(2.0 * M_PI * q / M), -std::sin(2.0 * M_PI * q / M));
    hipError_t e = hipMalloc(out, M * sizeof(double2));
    if (e == hipSuccess)
        e = hipMemcpy(*out, t.data(), M * sizeof(double2), hipMemcpyHostToDevice);
    return e;
}

struct NearPoly {
    double a[kNearQ + 1];
};

// Samples of the regularised near-field kernel at T j / M, j in I_M^d (array
// index j + M/2, axis 0 fastest): kappa(sqrt(sum_i s(x_i))) - K_NE(|x|) with
// the folded squares s and K_NE(r) = kappa(r) - p(r) for r < eps.
__device__ __forceinline__ double matern_value(int kernel, double r, double ell, int der)
{
    if (kernel == ADDK_MATERN32) {
        const double ar = sqrt(3.0) * r / ell;
        const double e = exp(-ar);
        return der ? ar * ar * e : (1.0 + ar) * e;
    }
    const double e = exp(-r / ell);
    return der ? r / ell * e : e;
}

__global__ void k_samples_near(double2 *s, int d, int M, double T, double L, double ell, double eps, NearPoly p,
                               int der, int kernel)
{
    int64_t tot = M;
    for (int i = 1; i < d; ++i)
        tot *= M;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = idx;
        double sf = 0.0, r2 = 0.0;
        for (int i = 0; i < d; ++i) {
            const int j = (int)(r % M) - M / 2;
            r /= M;
            const double ax = fabs(T * j / M);
            r2 += ax * ax;
            if (ax <= L) {
                sf += ax * ax;
            } else {
                const double t = (ax - L) / (T - 2.0 * L);
                const double h = t * t * t * t * (35.0 - 84.0 * t + 70.0 * t * t - 20.0 * t * t * t);
                sf += ax * ax * (1.0 - h) + (T - ax) * (T - ax) * h;
            }
        }
        const double rf = sqrt(sf);
        double v = matern_value(kernel, rf, ell, der);
        const double r0 = sqrt(r2);
        if (r0 < eps) {
            const double t2 = r2 / (eps * eps);
            double q = p.a[kNearQ];
            for (int k = kNearQ - 1; k >= 0; --k)
                q = q * t2 + p.a[k];
            v -= matern_value(kernel, r0, ell, der) - q;
        }
        s[idx] = make_double2(v, 0.0);
    }
}

// out_k = sum_j in_j exp(-2 pi i j k / n) along one axis; j, k in I_n (index + n/2);
// tw[q] = exp(-2 pi i q / n), q < n
__global__ void k_dft_axis(const double2 *__restrict__ in, double2 *out, int d, int n, int axis,
                           const double2 *__restrict__ tw)
{
    int64_t tot = n, stride = 1;
    for (int i = 1; i < d; ++i)
        tot *= n;
    for (int i = 0; i < axis; ++i)
        stride *= n;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
        const int kc = (int)((idx / stride) % n);
        const int64_t basei = idx - (int64_t)kc * stride;
        const int k = kc - n / 2;
        double re = 0.0, im = 0.0;
        for (int jc = 0; jc < n; ++jc) {
            const int j = jc - n / 2;
            const int jk = (int)((((int64_t)j * k) % n + n) % n);
            const double cs = tw[jk].x, sn = tw[jk].y;
            const double2 v = in[basei + (int64_t)jc * stride];
            re += v.x * cs - v.y * sn;
            im += v.x * sn + v.y * cs;
        }
        out[idx] = make_double2(re, im);
    }
}

// B_k for k in {-n/2..n/2}^d from the DFT c^ of M^d samples (M >= n; k is
// read at index k + M/2 of each axis, c^ being M-periodic in k)
__global__ void k_coef_from_hat(const double2 *__restrict__ chat, double *B, int d, int n, int M,
                                const double *__restrict__ psi)
{
    const int n1 = n + 1, half = n / 2;
    int64_t tot = n1;
    for (int i = 1; i < d; ++i)
        tot *= n1;
    double scale = 1.0;
    for (int i = 0; i < d; ++i)
        scale /= M;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
        int k[3] = {0, 0, 0};
        int64_t r = idx, hidx = 0, hs = 1;
        double dec = 1.0;
        for (int i = 0; i < d; ++i) {
            const int c = (int)(r % n1);
            r /= n1;
            k[i] = c - half;
            const int kk = k[i] == M / 2 ? -M / 2 : k[i];  // c^ is M-periodic in k
            hidx += (int64_t)(kk + M / 2) * hs;
            hs *= M;
            dec /= psi[c] * psi[c];
        }
        B[idx] = herm_weight(k, d, half) * dec * scale * chat[hidx].x;
    }
}

__global__ void k_to_float(const double *__restrict__ in, float *out, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------

static int64_t ipow(int64_t a, int d)
{
    int64_t r = 1;
    for (int i = 0; i < d; ++i)
        r *= a;
    return r;
}

static hipError_t free_win_arrays(WinHost &w)
{
    auto f = [](void *p) {
        if (p)
            (void)hipFree(p);
    };
    f(w.coords);
    f(w.perm);
    f(w.ucoords);
    w.ucoords = nullptr;
    if (w.Bk != (void *)w.Bk64)
        f(w.Bk);
    if (w.Bd != (void *)w.Bd64)
        f(w.Bd);
    f(w.Bk64);
    f(w.Bd64);
    f(w.d_tile_off);
    w.d_tile_off = nullptr;
    w.coords = nullptr;
    w.perm = nullptr;
    w.Bk = w.Bd = nullptr;
    w.Bk64 = w.Bd64 = nullptr;
    return hipSuccess;
}

addk_status plan_compute_multipliers(Plan &pl, hipStream_t st)
{
    const int n1 = pl.n + 1;
    const double b = M_PI * (2.0 - 1.0 / pl.sigma_os);
    if (pl.psi_tab.empty()) {
        pl.psi_tab.resize(n1);
        for (int c = 0; c < n1; ++c)
            pl.psi_tab[c] = window_ft(pl.m, pl.nos, b, (double)(c - pl.n / 2));
        hipError_t e = hipMalloc(&pl.d_psi, n1 * sizeof(double));
        if (e != hipSuccess)
            return hip_fail(e, "hipMalloc(psi)");
        e = hipMemcpy(pl.d_psi, pl.psi_tab.data(), n1 * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return hip_fail(e, "hipMemcpy(psi)");
    }
    for (WinHost &w : pl.wins) {
        const int64_t tot = ipow(n1, w.d);
        hipError_t e;
        if (!w.Bk64) {
            if ((e = hipMalloc(&w.Bk64, tot * sizeof(double))) != hipSuccess ||
                (e = hipMalloc(&w.Bd64, tot * sizeof(double))) != hipSuccess)
                return fail(ADDK_ERR_OOM, "multiplier allocation failed");
            if (pl.precision == ADDK_FP32) {
                if ((e = hipMalloc(&w.Bk, tot * sizeof(float))) != hipSuccess ||
                    (e = hipMalloc(&w.Bd, tot * sizeof(float))) != hipSuccess)
                    return fail(ADDK_ERR_OOM, "multiplier allocation failed");
            } else {
                w.Bk = w.Bk64;
                w.Bd = w.Bd64;
            }
        }
        const int nb = (int)std::min<int64_t>((tot + 255) / 256, 1024);
        if (w.nf) {
            const int M = 2 * pl.n;
            const int64_t ns = ipow(M, w.d);
            double2 *s0 = nullptr, *s1 = nullptr, *dtw = nullptr;
            if ((e = hipMalloc(&s0, ns * sizeof(double2))) != hipSuccess ||
                (e = hipMalloc(&s1, ns * sizeof(double2))) != hipSuccess || (e = dft_twiddles(M, &dtw)) != hipSuccess) {
                (void)hipFree(s0);
                (void)hipFree(s1);
                return fail(ADDK_ERR_OOM, "sample buffer allocation failed");
            }
            const int nbs = (int)std::min<int64_t>((ns + 255) / 256, 4096);
            for (int der = 0; der < 2; ++der) {
                NearPoly p;
                for (int j = 0; j <= kNearQ; ++j)
                    p.a[j] = der ? w.nf_ad[j] : w.nf_a[j];
                hipLaunchKernelGGL(k_samples_near, dim3(nbs), dim3(256), 0, st, s0, w.d, M, w.T, w.nf_Lf, w.ell,
                                   w.nf_eps, p, der, pl.kernel);
                double2 *a = s0, *bb = s1;
                for (int ax = 0; ax < w.d; ++ax) {
                    hipLaunchKernelGGL(k_dft_axis, dim3(nbs), dim3(256), 0, st, a, bb, w.d, M, ax, dtw);
                    std::swap(a, bb);
                }
                hipLaunchKernelGGL(k_coef_from_hat, dim3(nb), dim3(256), 0, st, a, der ? w.Bd64 : w.Bk64, w.d,
                                   pl.n, M, pl.d_psi);
            }
            e = hipStreamSynchronize(st);
            (void)hipFree(s0);
            (void)hipFree(s1);
            (void)hipFree(dtw);
            if (e != hipSuccess)
                return hip_fail(e, "near-field multipliers");
        } else if (pl.flags & ADDK_COEF_SAMPLED) {
            const int64_t ns = ipow(pl.n, w.d);
            double2 *s0 = nullptr, *s1 = nullptr, *dtw = nullptr;
            if ((e = hipMalloc(&s0, ns * sizeof(double2))) != hipSuccess ||
                (e = hipMalloc(&s1, ns * sizeof(double2))) != hipSuccess ||
                (e = dft_twiddles(pl.n, &dtw)) != hipSuccess) {
                (void)hipFree(s0);
                (void)hipFree(s1);
                return fail(ADDK_ERR_OOM, "sample buffer allocation failed");
            }
            const int nbs = (int)std::min<int64_t>((ns + 255) / 256, 1024);
            for (int der = 0; der < 2; ++der) {
                hipLaunchKernelGGL(k_samples, dim3(nbs), dim3(256), 0, st, s0, w.d, pl.n, w.T, w.ell, pl.kernel, der);
                double2 *a = s0, *bb = s1;
                for (int ax = 0; ax < w.d; ++ax) {
                    hipLaunchKernelGGL(k_dft_axis, dim3(nbs), dim3(256), 0, st, a, bb, w.d, pl.n, ax, dtw);
                    std::swap(a, bb);
                }
                hipLaunchKernelGGL(k_coef_from_hat, dim3(nb), dim3(256), 0, st, a, der ? w.Bd64 : w.Bk64, w.d,
                                   pl.n, pl.n, pl.d_psi);
            }
            e = hipStreamSynchronize(st);
            (void)hipFree(s0);
            (void)hipFree(s1);
            (void)hipFree(dtw);
            if (e != hipSuccess)
                return hip_fail(e, "sampled coefficients");
        } else {
            hipLaunchKernelGGL(k_coef_analytic, dim3(nb), dim3(256), 0, st, w.Bk64, w.Bd64, w.d, pl.n, w.T, w.ell,
                               pl.kernel, pl.d_psi);
        }
        if (pl.precision == ADDK_FP32) {
            hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(256), 0, st, w.Bk64, (float *)w.Bk, tot);
            hipLaunchKernelGGL(k_to_float, dim3(nb), dim3(256), 0, st, w.Bd64, (float *)w.Bd, tot);
        }
        e = hipGetLastError();
        if (e != hipSuccess)
            return hip_fail(e, "multiplier kernels");
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return hip_fail(e, "multiplier kernels");
    return ADDK_OK;
}

static bool is_device_ptr(const void *p)
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

static void fill_near(const Plan &pl, const WinHost &w, WinDev &d)
{
    d.nf = !w.nf ? 0 : (pl.kernel == ADDK_MATERN32 ? 2 : 1);
    d.tile_off = w.d_tile_off;
    if (!w.nf)
        return;
    const double eg = w.nf_eps * pl.nos / w.T;  // radius in grid units
    d.nf_eps2 = eg * eg;
    d.nf_inv_eps2 = 1.0 / (eg * eg);
    // r / l (Matern-1/2) or sqrt3 r / l (Matern-3/2) per grid unit of distance
    d.nf_hl = w.T / pl.nos / w.ell * (pl.kernel == ADDK_MATERN32 ? std::sqrt(3.0) : 1.0);
    for (int j = 0; j <= kNearQ; ++j) {
        d.nf_a[j] = w.nf_a[j];
        d.nf_ad[j] = w.nf_ad[j];
    }
}

static void fill_windesc(const Plan &pl, const WinHost &w, int prob, WinDev &d)
{
    std::memset(&d, 0, sizeof(d));
    d.d = w.d;
    d.n = pl.n;
    d.n1 = pl.n + 1;
    d.nos = pl.nos;
    d.m = pl.m;
    d.W = 2 * pl.m;
    d.prob = prob;
    d.N = pl.N;
    for (int i = 0; i < 3; ++i) {
        d.lo[i] = w.lo[i];
        d.ext[i] = w.ext[i];
        d.tb[i] = w.tb[i];
        d.ntile[i] = w.ntile[i];
        d.S[i] = w.S[i];
    }
    d.b = M_PI * (2.0 - 1.0 / pl.sigma_os);
    d.inv_e2bm = 1.0 / (1.0 - std::exp(-2.0 * d.b * pl.m));
    d.sig2 = w.sigma * w.sigma;
    d.der_scale = d.sig2 * (pl.kernel == ADDK_GAUSSIAN ? 2.0 / w.ell : 1.0 / w.ell);
    d.dsig = 2.0 * w.sigma;
    d.coords = w.coords;
    d.perm = w.perm;
    d.ucoords = w.ucoords;
    d.Bk = w.Bk;
    d.Bd = w.Bd;
    fill_near(pl, w, d);
}

static addk_status build_plan_engine(Plan &pl)
{
    Engine &E = pl.eng;
    E.plans.assign(1, &pl);
    E.nprob = 1;
    E.wdev.resize(pl.P);
    E.wplan.assign(pl.P, 0);
    E.wlocal.resize(pl.P);
    for (int w = 0; w < pl.P; ++w) {
        fill_windesc(pl, pl.wins[w], 0, E.wdev[w]);
        E.wlocal[w] = w;
    }
    E.dirty = true;
    E.no_mfma = (pl.flags & ADDK_VECTOR_ALU_ONLY) != 0;
    return engine_build_device(E, pl.precision);
}

// Lay out one window: box, tiles, sorted coordinates, permutation, chunks.
static addk_status plan_window(Plan &pl, WinHost &w, const double *dX, int64_t ldx, int dmax, hipStream_t st)
{
    const int64_t N = pl.N;
    const int m = pl.m, W = 2 * m, nos = pl.nos;
    double mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    hipError_t e;
    if (N > 0) {
        const int nb = (int)std::min<int64_t>((N + 255) / 256, 512);
        double *part = nullptr;
        if ((e = hipMalloc(&part, nb * 6 * sizeof(double))) != hipSuccess)
            return fail(ADDK_ERR_OOM, "allocation failed");
        hipLaunchKernelGGL(k_minmax, dim3(nb), dim3(256), 0, st, dX, ldx, N, w.d, w.feat[0], w.feat[1], w.feat[2],
                           part);
        std::vector<double> hp(nb * 6);
        e = hipMemcpyAsync(hp.data(), part, nb * 6 * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        (void)hipFree(part);
        if (e != hipSuccess)
            return hip_fail(e, "bounding box");
        for (int dd = 0; dd < w.d; ++dd) {
            mn[dd] = INFINITY;
            mx[dd] = -INFINITY;
            for (int b = 0; b < nb; ++b) {
                mn[dd] = std::min(mn[dd], hp[b * 6 + dd]);
                mx[dd] = std::max(mx[dd], hp[b * 6 + 3 + dd]);
            }
            if (!std::isfinite(mn[dd]) || !std::isfinite(mx[dd]))
                return fail(ADDK_ERR_INVALID_ARG, "point coordinates must be finite");
        }
    }
    double L = 0.0;
    for (int dd = 0; dd < w.d; ++dd) {
        w.center[dd] = 0.5 * (mn[dd] + mx[dd]);
        L = std::max(L, mx[dd] - mn[dd]);
    }
    w.L = L;
    w.nf = (pl.flags & ADDK_NEAR_FIELD) != 0;
    if (w.nf)
        w.nf_Lf = near_fold_width(L, w.ell);
    w.T = w.nf ? kNearFold * w.nf_Lf : torus_period(pl.kernel, L, w.ell, pl.n, pl.flags & ADDK_TORUS_PAPER, dmax);
    if (w.nf)
        near_setup(w, pl.kernel, pl.n);
    w.eta = M_PI * pl.n * w.ell / (std::sqrt(2.0) * w.T);
    if (w.eta < 1.0 && !(pl.flags & ADDK_NO_ACCURACY_CHECK))
        return fail(ADDK_ERR_ACCURACY, "window length scale too small for the grid: eta = pi n l / (sqrt2 T) = " +
                                           std::to_string(w.eta) + " < 1 (increase n or l)");
    // box in grid cells (one cell of margin on both sides covers rounding of u)
    for (int dd = 0; dd < 3; ++dd) {
        if (dd < w.d) {
            const double umin = ((mn[dd] - w.center[dd]) / w.T + 0.5) * nos;
            const double umax = ((mx[dd] - w.center[dd]) / w.T + 0.5) * nos;
            const int lo = (int)std::floor(umin) - m;
            const int hi = (int)std::floor(umax) + m + 1;
            if (lo < 0 || hi > nos - 1)
                return fail(ADDK_ERR_UNSUPPORTED,
                            "data extent plus window support does not fit the torus (increase n or oversampling, "
                            "or use the automatic torus rule)");
            w.lo[dd] = lo;
            w.ext[dd] = hi - lo + 1;
            const int nbase = w.ext[dd] - W + 1;
            const int tb = w.d == 3 ? 4 : (w.d == 2 ? 16 : 256);
            w.tb[dd] = std::min(tb, nbase);
            w.ntile[dd] = (nbase + w.tb[dd] - 1) / w.tb[dd];
            w.S[dd] = w.tb[dd] + W - 1;
        } else {
            w.lo[dd] = 0;
            w.ext[dd] = 1;
            w.tb[dd] = 1;
            w.ntile[dd] = 1;
            w.S[dd] = 1;
        }
    }
    w.ntiles = (int64_t)w.ntile[0] * w.ntile[1] * w.ntile[2];
    const size_t rs = pl.precision == ADDK_FP32 ? sizeof(float) : sizeof(double);
    if ((e = hipMalloc(&w.coords, std::max<int64_t>(1, N * w.d) * rs)) != hipSuccess ||
        (e = hipMalloc(&w.perm, std::max<int64_t>(1, N) * sizeof(int32_t))) != hipSuccess)
        return fail(ADDK_ERR_OOM, "point arrays allocation failed");
    w.chunks.clear();
    w.chunks_i.clear();
    w.tile_off.clear();
    w.tile_off_t.clear();
    w.split = pl.rect;
    w.dense.clear();
    w.dense_sp.clear();
    if (N == 0)
        return ADDK_OK;
    void *ucoord = nullptr;
    int32_t *key = nullptr, *hist = nullptr, *bad = nullptr;
    if ((e = hipMalloc(&ucoord, N * w.d * rs)) != hipSuccess || (e = hipMalloc(&key, N * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&hist, (w.ntiles * w.tb[0] * w.tb[1] * w.tb[2] * (w.split ? 2 : 1) + 1) * sizeof(int32_t))) !=
            hipSuccess ||
        (e = hipMalloc(&bad, sizeof(int32_t))) != hipSuccess)
        return fail(ADDK_ERR_OOM, "sort buffers allocation failed");
    KeyArgs ka;
    std::memset(&ka, 0, sizeof(ka));
    ka.d = w.d;
    ka.nos = nos;
    ka.m = m;
    ka.W = W;
    ka.invT = 1.0 / w.T;
    ka.cpt = w.tb[0] * w.tb[1] * w.tb[2];
    for (int dd = 0; dd < 3; ++dd) {
        ka.f[dd] = dd < w.d ? w.feat[dd] : 0;
        ka.c[dd] = dd < w.d ? w.center[dd] : 0.0;
        ka.lo[dd] = w.lo[dd];
        ka.ext[dd] = w.ext[dd];
        ka.tb[dd] = w.tb[dd];
        ka.ntile[dd] = w.ntile[dd];
    }
    const int64_t cpt = (int64_t)w.tb[0] * w.tb[1] * w.tb[2];
    const int64_t nkeys = w.ntiles * cpt;
    const int nseg = w.split ? 2 : 1;
    ka.nsrc = pl.nsrc;
    ka.nkeys = (int32_t)nkeys;
    ka.split = w.split ? 1 : 0;
    {
        std::vector<int32_t> zeros(1, 0);
        e = hipMemcpy(bad, zeros.data(), sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemsetAsync(hist, 0, nseg * nkeys * sizeof(int32_t), st);  // plan set-up is never captured
        if (e != hipSuccess)
            return hip_fail(e, "clear histogram");
    }
    const int nb = (int)std::min<int64_t>((N + 255) / 256, 4096);
    const int nhl = nseg * nkeys <= 8192 ? (int)(nseg * nkeys) : 0;  // LDS histogram (32 KB at most)
    if (pl.precision == ADDK_FP32)
        hipLaunchKernelGGL(k_keys<float>, dim3(nb), dim3(256), nhl * sizeof(int32_t), st, dX, ldx, N, ka,
                           (float *)ucoord, key, hist, bad, nhl);
    else
        hipLaunchKernelGGL(k_keys<double>, dim3(nb), dim3(256), nhl * sizeof(int32_t), st, dX, ldx, N, ka,
                           (double *)ucoord, key, hist, bad, nhl);
    std::vector<int32_t> hall(nseg * nkeys);
    int32_t hbad = 0;
    e = hipMemcpyAsync(hall.data(), hist, nseg * nkeys * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return hip_fail(e, "tile histogram");
    if (hbad)
        return fail(ADDK_ERR_INVALID_ARG, "internal: a point fell outside its grid box");
    // Order inside a tile: points of sparsely populated cells first (one
    // contiguous range, processed by the tile kernels), then each densely
    // populated cell (processed by the dense-cell kernels).
    // With separate targets the sources' segment comes first: its tile chunks
    // and dense runs feed the spreading, the targets' the interpolation.
    const bool dense_ok = dense_width_ok(W) && !(pl.flags & kFlagNoDense);
    std::vector<int32_t> offall(nseg * nkeys, 0);
    int64_t pos = 0;
    w.ndense_pts = 0;
    for (int seg = 0; seg < nseg; ++seg) {
    const int32_t *h = hall.data() + seg * nkeys;
    int32_t *off = offall.data() + seg * nkeys;
    const bool spread_side = seg == 0, interp_side = seg == nseg - 1;
    std::vector<Chunk> &tchunks = seg == 0 ? w.chunks : w.chunks_i;
    std::vector<int32_t> &toff = seg == 0 ? w.tile_off : w.tile_off_t;
    if (w.nf)
        toff.assign(w.ntiles + 1, 0);
    for (int64_t t = 0; t < w.ntiles; ++t) {
        const int64_t k0 = t * cpt;
        const int64_t s0 = pos;
        if (w.nf)
            toff[t] = (int32_t)s0;
        for (int64_t c = 0; c < cpt; ++c)
            if (!(dense_ok && h[k0 + c] >= kDenseMin)) {
                off[k0 + c] = (int32_t)pos;
                pos += h[k0 + c];
            }
        for (int64_t s = s0; s < pos; s += kChunk)
            tchunks.push_back({0, (int32_t)t, (int32_t)s, (int32_t)std::min<int64_t>(kChunk, pos - s)});
        const int tx = (int)(t % w.ntile[0]), ty = (int)((t / w.ntile[0]) % w.ntile[1]),
                  tz = (int)(t / ((int64_t)w.ntile[0] * w.ntile[1]));
        // dense cells of the tile, z fastest; for d = 3 two dense cells adjacent
        // in z form one item (their points consecutive), whose window block is
        // (2m) x (2m) x (2m + 1): half the blocks of single cells
        const bool isdense_any = dense_ok;
        auto is_dense = [&](int64_t c) { return isdense_any && h[k0 + c] >= kDenseMin; };
        for (int64_t cxy = 0; cxy < (int64_t)w.tb[0] * w.tb[1]; ++cxy) {
            for (int cz = 0; cz < w.tb[2]; ++cz) {
                const int64_t c = cxy + (int64_t)cz * w.tb[0] * w.tb[1];
                if (!is_dense(c))
                    continue;
                const int64_t c2 = c + (int64_t)w.tb[0] * w.tb[1];
                const int nzc = (w.d == 3 && cz + 1 < w.tb[2] && is_dense(c2)) ? 2 : 1;
                const int cx = (int)(cxy % w.tb[0]), cy = (int)(cxy / w.tb[0]);
                const int bx = tx * w.tb[0] + cx, by = ty * w.tb[1] + cy, bz = tz * w.tb[2] + cz;
                const int packed = bx | (by << 10) | (bz << 20) | ((nzc - 1) << 30);
                int cnt = 0;
                for (int k = 0; k < nzc; ++k) {
                    const int64_t ck = c + (int64_t)k * w.tb[0] * w.tb[1];
                    off[k0 + ck] = (int32_t)(pos + cnt);
                    cnt += h[k0 + ck];
                }
                if (interp_side)
                    for (int s = 0; s < cnt; s += kDenseChunk)
                        w.dense.push_back({0, packed, (int32_t)(pos + s), std::min(kDenseChunk, cnt - s)});
                // spread items: up to kSpreadChunk points for d = 3 (one window block
                // each), kSpreadChunk1 for d = 1 (fewer, longer blocks amortise the
                // quad-per-point kernel's reduction and atomic flush: 0.92 ms on
                // fifteen 1e6-point windows with 256 points, 0.34 with 1024, 0.29
                // with 2048), the interp item size for d = 2
                const int spc = w.d == 3 ? kSpreadChunk : (w.d == 1 ? kSpreadChunk1 : kDenseChunk);
                if (spread_side)
                    for (int s = 0; s < cnt; s += spc)
                        w.dense_sp.push_back({0, packed, (int32_t)(pos + s), std::min(spc, cnt - s)});
                pos += cnt;
                if (spread_side)
                    w.ndense_pts += cnt;
                cz += nzc - 1;
            }
        }
    }
    if (w.nf)
        toff[w.ntiles] = (int32_t)pos;
    }
    if (w.nf) {
        e = hipMalloc(&w.d_tile_off, (w.ntiles + 1) * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(w.d_tile_off, w.tile_off.data(), (w.ntiles + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return hip_fail(e, "near-field tile ranges");
    }
    // stable sort of (key, index) pairs, then placement (deterministic)
    std::vector<int32_t> kstart(nseg * nkeys, 0);
    for (int64_t k = 1; k < nseg * nkeys; ++k)
        kstart[k] = kstart[k - 1] + hall[k - 1];
    int32_t *dkstart = nullptr, *js_in = nullptr, *js_out = nullptr;
    uint32_t *ks_out = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    int end_bit = 1;
    while (end_bit < 32 && ((int64_t)1 << end_bit) < nseg * nkeys)
        ++end_bit;
    auto release = [&]() {
        (void)hipFree(ucoord);
        (void)hipFree(key);
        (void)hipFree(hist);
        (void)hipFree(bad);
        (void)hipFree(dkstart);
        (void)hipFree(js_in);
        (void)hipFree(js_out);
        (void)hipFree(ks_out);
        (void)hipFree(tmp);
    };
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, (const uint32_t *)key, ks_out, js_in, js_out, (int)N, 0,
                                           end_bit, st);
    if (e == hipSuccess && ((e = hipMalloc(&dkstart, nseg * nkeys * sizeof(int32_t))) != hipSuccess ||
                            (e = hipMalloc(&js_in, N * sizeof(int32_t))) != hipSuccess ||
                            (e = hipMalloc(&js_out, N * sizeof(int32_t))) != hipSuccess ||
                            (e = hipMalloc(&ks_out, N * sizeof(uint32_t))) != hipSuccess ||
                            (e = hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16))) != hipSuccess)) {
        release();
        return fail(ADDK_ERR_OOM, "sort buffers allocation failed");
    }
    if (e == hipSuccess)
        e = hipMemcpy(hist, offall.data(), nseg * nkeys * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(dkstart, kstart.data(), nseg * nkeys * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_iota, dim3(nb), dim3(256), 0, st, js_in, N);
        e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, (const uint32_t *)key, ks_out, js_in, js_out, (int)N, 0,
                                               end_bit, st);
    }
    if (e == hipSuccess) {
        if (pl.precision == ADDK_FP32)
            hipLaunchKernelGGL(k_place<float>, dim3(nb), dim3(256), 0, st, N, w.d, (const float *)ucoord, ks_out,
                               js_out, hist, dkstart, (float *)w.coords, w.perm);
        else
            hipLaunchKernelGGL(k_place<double>, dim3(nb), dim3(256), 0, st, N, w.d, (const double *)ucoord, ks_out,
                               js_out, hist, dkstart, (double *)w.coords, w.perm);
        e = hipStreamSynchronize(st);
    }
    if (e == hipSuccess && w.d == 1 && !pl.rect) {
        // d = 1: the interpolation runs in the caller's point order, fused with
        // the window sum; it keeps these coordinates
        if (w.ucoords)
            (void)hipFree(w.ucoords);
        w.ucoords = ucoord;
        ucoord = nullptr;
    }
    release();
    if (e != hipSuccess)
        return hip_fail(e, "tile sort");
    return ADDK_OK;
}

static void plan_release(Plan *pl)
{
    if (!pl)
        return;
    for (WinHost &w : pl->wins)
        free_win_arrays(w);
    if (pl->d_psi)
        (void)hipFree(pl->d_psi);
    engine_free(pl->eng);
    delete pl;
}

}  // namespace addk

using namespace addk;

extern "C" {

const char *addk_status_string(addk_status s)
{
    switch (s) {
    case ADDK_OK: return "ok";
    case ADDK_ERR_INVALID_ARG: return "invalid argument";
    case ADDK_ERR_UNSUPPORTED: return "unsupported configuration";
    case ADDK_ERR_ACCURACY: return "accuracy requirement cannot be met";
    case ADDK_ERR_OOM: return "out of memory";
    case ADDK_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *addk_last_error(void) { return g_last_error.c_str(); }

const char *addk_version(void) { return "addk 0.1 (gfx950)"; }

addk_status addk_torus_period(int32_t kernel, double L, double ell, int32_t n, uint32_t rule, int32_t dmax, double *T)
{
    if (!T || !(L >= 0.0) || !(ell > 0.0) || n < 2 || dmax < 1 ||
        (kernel != ADDK_GAUSSIAN && kernel != ADDK_MATERN12 && kernel != ADDK_MATERN32))
        return fail(ADDK_ERR_INVALID_ARG, "addk_torus_period: bad argument");
    *T = torus_period(kernel, L, ell, n, rule, dmax);
    return ADDK_OK;
}

addk_status addk_choose_n(int32_t kernel, double L, double ell, int32_t m, double oversampling, double tol,
                          int32_t *n, double *err_estimate)
{
    if (!n || !(L >= 0.0) || !std::isfinite(L) || !(ell > 0.0) || !std::isfinite(ell) || m < 2 || m > kMaxW / 2 ||
        !(oversampling > 1.0) || !std::isfinite(oversampling) || !(tol > 0.0) ||
        (kernel != ADDK_GAUSSIAN && kernel != ADDK_MATERN12 && kernel != ADDK_MATERN32))
        return fail(ADDK_ERR_INVALID_ARG, "addk_choose_n: bad argument");
    // Candidates: even n whose oversampled grid round(sigma n) is a power of two
    // in [16, 256] with room for the window; the first (smallest, cheapest) one
    // whose a-priori estimate meets tol and whose data box fits the torus wins.
    double best_err = INFINITY;
    for (int c = 4; c < kMaxNos; c += 2) {
        const long nos = std::lround(oversampling * c);
        if (nos < 16 || nos > kMaxNos || (nos & (nos - 1)) || nos <= c || 4 * m > nos)
            continue;
        const double T = torus_period(kernel, L, ell, c, 0, 1);
        const double eta = M_PI * c * ell / (std::sqrt(2.0) * T);
        if (eta < 1.0)
            continue;
        if (L / T * (double)nos + 2.0 * m + 4.0 > (double)nos)
            continue;
        const double est = error_estimate(kernel, L, T, ell, c, m, (double)nos / c);
        best_err = std::min(best_err, est);
        if (est <= tol) {
            *n = c;
            if (err_estimate)
                *err_estimate = est;
            return ADDK_OK;
        }
    }
    return fail(ADDK_ERR_ACCURACY, "addk_choose_n: no supported n reaches the tolerance (best estimate " +
                                       std::to_string(best_err) + "; increase m or l)");
}

addk_status addk_choose_n_windows(int32_t kernel, int64_t N, int32_t D, const double *X, int64_t ldx, int32_t P,
                                  const int32_t *win_offsets, const int32_t *win_features, const double *ell,
                                  int32_t m, double oversampling, double tol, int32_t *n, double *err_estimate,
                                  void *stream)
{
    if (!n || N < 0 || D <= 0 || (N > 0 && (!X || ldx < D)) || P <= 0 || !win_offsets || !win_features || !ell ||
        win_offsets[0] != 0)
        return fail(ADDK_ERR_INVALID_ARG, "addk_choose_n_windows: bad sizes or NULL pointers");
    for (int w = 0; w < P; ++w) {
        const int dw = win_offsets[w + 1] - win_offsets[w];
        if (dw <= 0 || dw > 3)
            return fail(ADDK_ERR_INVALID_ARG, "addk_choose_n_windows: window dimensions must be 1..3");
        for (int q = win_offsets[w]; q < win_offsets[w + 1]; ++q)
            if (win_features[q] < 0 || win_features[q] >= D)
                return fail(ADDK_ERR_INVALID_ARG, "addk_choose_n_windows: feature index out of range");
    }
    // per-feature ranges of the points (host loop, or one reduction kernel per
    // window for device memory)
    std::vector<double> L(P, 0.0);
    if (N > 0) {
        hipStream_t st = (hipStream_t)stream;
        const bool dev = is_device_ptr(X);
        for (int w = 0; w < P; ++w) {
            const int dw = win_offsets[w + 1] - win_offsets[w];
            int f[3] = {0, 0, 0};
            for (int i = 0; i < dw; ++i)
                f[i] = win_features[win_offsets[w] + i];
            double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
            if (dev) {
                const int nb = (int)std::min<int64_t>((N + 255) / 256, 512);
                double *part = nullptr;
                hipError_t e = hipMalloc(&part, nb * 6 * sizeof(double));
                if (e != hipSuccess)
                    return fail(ADDK_ERR_OOM, "allocation failed");
                hipLaunchKernelGGL(k_minmax, dim3(nb), dim3(256), 0, st, X, ldx, N, dw, f[0], f[1], f[2], part);
                std::vector<double> hp(nb * 6);
                e = hipMemcpyAsync(hp.data(), part, nb * 6 * sizeof(double), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess)
                    e = hipStreamSynchronize(st);
                (void)hipFree(part);
                if (e != hipSuccess)
                    return hip_fail(e, "feature ranges");
                for (int i = 0; i < dw; ++i)
                    for (int b = 0; b < nb; ++b) {
                        mn[i] = std::min(mn[i], hp[b * 6 + i]);
                        mx[i] = std::max(mx[i], hp[b * 6 + 3 + i]);
                    }
            } else {
                for (int64_t j = 0; j < N; ++j)
                    for (int i = 0; i < dw; ++i) {
                        const double x = X[j * ldx + f[i]];
                        mn[i] = std::min(mn[i], x);
                        mx[i] = std::max(mx[i], x);
                    }
            }
            for (int i = 0; i < dw; ++i) {
                if (!std::isfinite(mn[i]) || !std::isfinite(mx[i]))
                    return fail(ADDK_ERR_INVALID_ARG, "point coordinates must be finite");
                L[w] = std::max(L[w], mx[i] - mn[i]);
            }
        }
    }
    // the plan's bandwidth is the largest per-window choice; its estimate is the
    // largest per-window estimate at that bandwidth
    int32_t best = 0;
    for (int w = 0; w < P; ++w) {
        int32_t nw = 0;
        addk_status s = addk_choose_n(kernel, L[w], ell[w], m, oversampling, tol, &nw, nullptr);
        if (s != ADDK_OK)
            return s;
        best = std::max(best, nw);
    }
    const long nos = std::lround(oversampling * best);
    double est = 0.0;
    for (int w = 0; w < P; ++w) {
        const double T = torus_period(kernel, L[w], ell[w], best, 0, 1);
        est = std::max(est, error_estimate(kernel, L[w], T, ell[w], best, m, (double)nos / best));
    }
    *n = best;
    if (err_estimate)
        *err_estimate = est;
    return ADDK_OK;
}

addk_status addk_window_ft(int32_t m, int32_t n_os, double oversampling, double k, double *value)
{
    if (!value || m < 1 || n_os < 2 || !(oversampling > 1.0))
        return fail(ADDK_ERR_INVALID_ARG, "addk_window_ft: bad argument");
    *value = window_ft(m, n_os, M_PI * (2.0 - 1.0 / oversampling), k);
    return ADDK_OK;
}

// Plan over N points; with rect, points [nsrc, N) are separate targets.
static addk_status plan_create_impl(addk_plan *out, int64_t N, int64_t nsrc, bool rect, int32_t D, const double *X,
                                    int64_t ldx, int32_t P, const int32_t *win_offsets, const int32_t *win_features,
                                    int32_t kernel, const double *ell, const double *sigma, int32_t n, int32_t m,
                                    double oversampling, int32_t precision, uint32_t flags, void *stream)
{
    if (!out)
        return fail(ADDK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (N < 0 || N > INT32_MAX || D <= 0 || (N > 0 && (!X || ldx < D)) || P <= 0 || !win_offsets || !win_features ||
        !ell || !sigma)
        return fail(ADDK_ERR_INVALID_ARG, "bad sizes or NULL pointers");
    if (kernel != ADDK_GAUSSIAN && kernel != ADDK_MATERN12 && kernel != ADDK_MATERN32)
        return fail(ADDK_ERR_INVALID_ARG, "kernel must be ADDK_GAUSSIAN, ADDK_MATERN12 or ADDK_MATERN32");
    if (precision != ADDK_FP64 && precision != ADDK_FP32)
        return fail(ADDK_ERR_INVALID_ARG, "precision must be ADDK_FP64 or ADDK_FP32");
    if (flags & ~(ADDK_COEF_SAMPLED | ADDK_TORUS_PAPER | ADDK_NO_ACCURACY_CHECK | ADDK_TILE_KERNELS_ONLY |
                  ADDK_VECTOR_ALU_ONLY | ADDK_NEAR_FIELD))
        return fail(ADDK_ERR_INVALID_ARG, "unknown flags");
    if (flags & ADDK_NEAR_FIELD) {
        if (kernel != ADDK_MATERN12 && kernel != ADDK_MATERN32)
            return fail(ADDK_ERR_UNSUPPORTED, "ADDK_NEAR_FIELD applies to the Matern kernels only");
        if (flags & (ADDK_COEF_SAMPLED | ADDK_TORUS_PAPER))
            return fail(ADDK_ERR_UNSUPPORTED, "ADDK_NEAR_FIELD sets its own period and multipliers (no "
                                              "ADDK_COEF_SAMPLED / ADDK_TORUS_PAPER)");
        if (n < 16)
            return fail(ADDK_ERR_UNSUPPORTED, "ADDK_NEAR_FIELD needs n >= 16");
    }
    if (n < 4 || (n & 1))
        return fail(ADDK_ERR_INVALID_ARG, "n must be even and >= 4");
    if (m < 2 || m > kMaxW / 2)
        return fail(ADDK_ERR_UNSUPPORTED, "m must be in [2, 8]");
    if (!(oversampling > 1.0) || !std::isfinite(oversampling))
        return fail(ADDK_ERR_INVALID_ARG, "oversampling must be > 1");
    const long nos = std::lround(oversampling * n);
    if (nos < 16 || nos > kMaxNos || (nos & (nos - 1)) || nos <= n)
        return fail(ADDK_ERR_UNSUPPORTED, "oversampled grid n_os = round(sigma n) must be a power of two in [16, 256] "
                                          "and exceed n");
    if (4 * m > nos)
        return fail(ADDK_ERR_UNSUPPORTED, "window support 2m must not exceed half the oversampled grid");
    if (win_offsets[0] != 0)
        return fail(ADDK_ERR_INVALID_ARG, "win_offsets[0] must be 0");
    int dmax = 1;
    for (int w = 0; w < P; ++w) {
        const int dw = win_offsets[w + 1] - win_offsets[w];
        if (dw <= 0)
            return fail(ADDK_ERR_INVALID_ARG, "empty or decreasing window offsets");
        if (dw > 3)
            return fail(ADDK_ERR_UNSUPPORTED, "window dimension d_w must be <= 3");
        for (int q = win_offsets[w]; q < win_offsets[w + 1]; ++q)
            if (win_features[q] < 0 || win_features[q] >= D)
                return fail(ADDK_ERR_INVALID_ARG, "window feature index out of range");
        if (!(ell[w] > 0.0) || !std::isfinite(ell[w]))
            return fail(ADDK_ERR_INVALID_ARG, "length scales must be positive and finite");
        if (!(sigma[w] >= 0.0) || !std::isfinite(sigma[w]))
            return fail(ADDK_ERR_INVALID_ARG, "amplitudes sigma_w must be >= 0 and finite");
        dmax = std::max(dmax, dw);
    }
    hipStream_t st = (hipStream_t)stream;
    Plan *pl = new (std::nothrow) Plan();
    if (!pl)
        return fail(ADDK_ERR_OOM, "host allocation failed");
    (void)hipGetDevice(&pl->device);
    pl->N = N;
    pl->nsrc = nsrc;
    pl->rect = rect;
    pl->D = D;
    pl->P = P;
    pl->kernel = kernel;
    pl->n = n;
    pl->m = m;
    pl->nos = (int)nos;
    pl->precision = precision;
    pl->flags = flags;
    pl->sigma_os = (double)nos / n;
    pl->wins.resize(P);
    for (int w = 0; w < P; ++w) {
        WinHost &wh = pl->wins[w];
        wh.d = win_offsets[w + 1] - win_offsets[w];
        for (int q = 0; q < 3; ++q)
            wh.feat[q] = q < wh.d ? win_features[win_offsets[w] + q] : 0;
        wh.ell = ell[w];
        wh.sigma = sigma[w];
    }
    // device copy of X (contiguous rows)
    double *dX = nullptr;
    addk_status s = ADDK_OK;
    hipError_t e = hipSuccess;
    if (N > 0) {
        e = hipMalloc(&dX, N * D * sizeof(double));
        if (e != hipSuccess) {
            plan_release(pl);
            return fail(ADDK_ERR_OOM, "allocation of the point copy failed");
        }
        const bool dev = is_device_ptr(X);
        if (ldx == D) {
            e = hipMemcpy(dX, X, N * D * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
        } else if (dev) {
            e = hipMemcpy2D(dX, D * sizeof(double), X, ldx * sizeof(double), D * sizeof(double), N,
                            hipMemcpyDeviceToDevice);
        } else {
            std::vector<double> packed((size_t)N * D);
            for (int64_t j = 0; j < N; ++j)
                std::memcpy(&packed[(size_t)j * D], X + j * ldx, D * sizeof(double));
            e = hipMemcpy(dX, packed.data(), N * D * sizeof(double), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            (void)hipFree(dX);
            plan_release(pl);
            return hip_fail(e, "copy of the points");
        }
    }
    double t0 = now_ms();
    for (int w = 0; w < P && s == ADDK_OK; ++w)
        s = plan_window(*pl, pl->wins[w], dX, D, dmax, st);
    if (dX)
        (void)hipFree(dX);
    double t1 = now_ms();
    if (s == ADDK_OK)
        s = plan_compute_multipliers(*pl, st);
    double t2 = now_ms();
    if (s == ADDK_OK)
        s = build_plan_engine(*pl);
    double t3 = now_ms();
    if (log_on() && s == ADDK_OK) {
        std::fprintf(stderr, "[addk] plan N=%lld P=%d n=%d m=%d n_os=%d prec=%s: sort %.1f ms, multipliers %.1f ms, "
                             "work lists %.1f ms\n",
                     (long long)N, P, n, m, (int)nos, precision == ADDK_FP32 ? "fp32" : "fp64", t1 - t0, t2 - t1,
                     t3 - t2);
        for (int w = 0; w < P; ++w) {
            const WinHost &wh = pl->wins[w];
            std::fprintf(stderr, "[addk]   window %d: d=%d l=%g T=%.6g L=%.6g eta=%.3g box=%dx%dx%d tiles=%lld "
                                 "sparse chunks=%zu dense items=%zu dense points=%lld\n",
                         w, wh.d, wh.ell, wh.T, wh.L, wh.eta, wh.ext[0], wh.ext[1], wh.ext[2], (long long)wh.ntiles,
                         wh.chunks.size(), wh.dense.size(), (long long)wh.ndense_pts);
        }
    }
    if (s != ADDK_OK) {
        plan_release(pl);
        return s;
    }
    *out = (addk_plan)pl;
    return ADDK_OK;
}

addk_status addk_plan_create(addk_plan *out, int64_t N, int32_t D, const double *X, int64_t ldx, int32_t P,
                             const int32_t *win_offsets, const int32_t *win_features, int32_t kernel,
                             const double *ell, const double *sigma, int32_t n, int32_t m, double oversampling,
                             int32_t precision, uint32_t flags, void *stream)
{
    return plan_create_impl(out, N, N, false, D, X, ldx, P, win_offsets, win_features, kernel, ell, sigma, n, m,
                            oversampling, precision, flags, stream);
}

addk_status addk_plan_create_targets(addk_plan *out, int64_t Ns, int64_t Nt, int32_t D, const double *Xs,
                                     int64_t ldxs, const double *Xt, int64_t ldxt, int32_t P,
                                     const int32_t *win_offsets, const int32_t *win_features, int32_t kernel,
                                     const double *ell, const double *sigma, int32_t n, int32_t m,
                                     double oversampling, int32_t precision, uint32_t flags, void *stream)
{
    if (!out)
        return fail(ADDK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (Ns < 0 || Nt < 0 || D <= 0 || Ns + Nt > INT32_MAX || (Ns > 0 && (!Xs || ldxs < D)) ||
        (Nt > 0 && (!Xt || ldxt < D)))
        return fail(ADDK_ERR_INVALID_ARG, "bad sizes or NULL pointers");
    // one point set [sources; targets], sorted as two segments: the torus and
    // grid box cover both, the sources are spread and the targets interpolated
    const int64_t N = Ns + Nt;
    double *dX = nullptr;
    hipError_t e = hipSuccess;
    if (N > 0 && (e = hipMalloc(&dX, N * D * sizeof(double))) != hipSuccess)
        return fail(ADDK_ERR_OOM, "allocation of the point copy failed");
    if (Ns > 0)
        e = hipMemcpy2D(dX, D * sizeof(double), Xs, ldxs * sizeof(double), D * sizeof(double), Ns, hipMemcpyDefault);
    if (e == hipSuccess && Nt > 0)
        e = hipMemcpy2D(dX + Ns * D, D * sizeof(double), Xt, ldxt * sizeof(double), D * sizeof(double), Nt,
                        hipMemcpyDefault);
    if (e != hipSuccess) {
        (void)hipFree(dX);
        return hip_fail(e, "copy of the points");
    }
    addk_status s = plan_create_impl(out, N, Ns, true, D, dX, D, P, win_offsets, win_features, kernel, ell, sigma,
                                     n, m, oversampling, precision, flags, stream);
    (void)hipFree(dX);
    return s;
}

addk_status addk_plan_destroy(addk_plan plan)
{
    if (!plan)
        return fail(ADDK_ERR_INVALID_ARG, "plan is NULL");
    hipError_t e = hipDeviceSynchronize();
    plan_release((Plan *)plan);
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceSynchronize");
    return ADDK_OK;
}

addk_status addk_plan_update_params(addk_plan plan, const double *ell, const double *sigma, void *stream)
{
    if (!plan || !ell || !sigma)
        return fail(ADDK_ERR_INVALID_ARG, "NULL argument");
    Plan &pl = *(Plan *)plan;
    for (int w = 0; w < pl.P; ++w) {
        if (!(ell[w] > 0.0) || !std::isfinite(ell[w]) || !(sigma[w] >= 0.0) || !std::isfinite(sigma[w]))
            return fail(ADDK_ERR_INVALID_ARG, "length scales must be > 0 and amplitudes >= 0");
        const double eta = M_PI * pl.n * ell[w] / (std::sqrt(2.0) * pl.wins[w].T);
        if (eta < 1.0 && !(pl.flags & ADDK_NO_ACCURACY_CHECK))
            return fail(ADDK_ERR_ACCURACY, "eta < 1 for the new length scale");
    }
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return hip_fail(e, "hipDeviceSynchronize");
    for (int w = 0; w < pl.P; ++w) {
        pl.wins[w].ell = ell[w];
        pl.wins[w].sigma = sigma[w];
        pl.wins[w].eta = M_PI * pl.n * ell[w] / (std::sqrt(2.0) * pl.wins[w].T);
        if (pl.wins[w].nf)
            near_setup(pl.wins[w], pl.kernel, pl.n);  // T and the radius stay, the polynomials follow l
    }
    addk_status s = plan_compute_multipliers(pl, (hipStream_t)stream);
    if (s != ADDK_OK)
        return s;
    for (int w = 0; w < pl.P; ++w) {
        WinDev &d = pl.eng.wdev[w];
        d.sig2 = sigma[w] * sigma[w];
        d.der_scale = d.sig2 * (pl.kernel == ADDK_GAUSSIAN ? 2.0 / ell[w] : 1.0 / ell[w]);
        d.dsig = 2.0 * sigma[w];
        fill_near(pl, pl.wins[w], d);
    }
    ++pl.param_gen;
    pl.eng.dirty = true;
    return engine_upload(pl.eng);
}

addk_status addk_plan_query(addk_plan plan, addk_plan_info *info, double *torus_period, double *eta,
                            int32_t *window_dim)
{
    if (!plan)
        return fail(ADDK_ERR_INVALID_ARG, "plan is NULL");
    const Plan &pl = *(const Plan *)plan;
    if (info) {
        info->N = pl.N;
        info->P = pl.P;
        info->n = pl.n;
        info->m = pl.m;
        info->n_os = pl.nos;
        info->precision = pl.precision;
        info->kernel = pl.kernel;
        info->workspace_bytes = pl.eng.ws_bytes + pl.eng.yw_bytes;
        double est = 0.0;
        for (const WinHost &w : pl.wins)
            est = std::max(est, error_estimate(pl.kernel, w.L, w.T, w.ell, pl.n, pl.m, pl.sigma_os));
        info->err_estimate = est;
        info->dense_points = 0;
        for (const WinHost &w : pl.wins)
            info->dense_points += w.ndense_pts;
        info->tile_points = pl.nsrc * pl.P - info->dense_points;
        info->knobs = pl.eng.no_mfma ? 0u : pl.eng.knobs;
        info->tuned = pl.eng.tuned ? 1 : 0;
        info->n_sources = pl.nsrc;
        info->n_targets = pl.rect ? pl.N - pl.nsrc : pl.N;
    }
    for (int w = 0; w < pl.P; ++w) {
        if (torus_period)
            torus_period[w] = pl.wins[w].T;
        if (eta)
            eta[w] = pl.wins[w].eta;
        if (window_dim)
            window_dim[w] = pl.wins[w].d;
    }
    return ADDK_OK;
}

}  // extern "C"
