// Conjugate gradients for the regularised kernel system (K + beta I) X = Y of
// eq. (9) (kernel ridge regression), with the plan's fast products for K.
// The R right-hand sides run in lockstep, each with its own step sizes; a
// column stops updating once its relative residual is below the tolerance.
// Vectors are FP64; the per-iteration dot products are reduced on the device
// and read back by the host, which decides the step sizes and convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "addk_internal.h"

namespace addk {

constexpr int kDotBlocks = 128;

// partial[(b * R + r) * 2 + s]: block b's share of <a_r, b_r> (s = 0) and
// <c_r, c_r> (s = 1) for column r (blockIdx.y); a, b, c are N x R, ld = N.
__global__ __launch_bounds__(kBlock) void k_cg_dots(int64_t N, int R, const double *__restrict__ a,
                                                    const double *__restrict__ b, const double *__restrict__ c,
                                                    double *partial)
{
    const int r = blockIdx.y;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock) {
        const int64_t e = i + (int64_t)r * N;
        s0 += a[e] * b[e];
        if (c)
            s1 += c[e] * c[e];
    }
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[((int64_t)blockIdx.x * R + r) * 2] = red[0][0];
        partial[((int64_t)blockIdx.x * R + r) * 2 + 1] = red[1][0];
    }
}

// Fixed-order sum of the partials: out[2 r + s].
__global__ void k_cg_dots_finish(int R, int nblk, const double *partial, double *out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 2 * R)
        return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b)
        s += partial[(int64_t)b * 2 * R + k];
    out[k] = s;
}

// q += beta p  (the beta I part of the operator), all columns
__global__ __launch_bounds__(kBlock) void k_cg_shift(int64_t n, double beta, const double *__restrict__ p, double *q)
{
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock)
        q[e] += beta * p[e];
}

// r = y - q (initial residual); p = r.  y has leading dimension ldy.
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t N, int R, const double *__restrict__ y, int64_t ldy,
                                                    const double *__restrict__ q, double *r, double *p)
{
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < N * R; e += (int64_t)gridDim.x * kBlock) {
        const int64_t c = e / N, i = e - c * N;
        const double v = y[i + c * ldy] - q[e];
        r[e] = v;
        p[e] = v;
    }
}

// x += alpha_c p; r -= alpha_c q  (x has leading dimension ldx)
__global__ __launch_bounds__(kBlock) void k_cg_step(int64_t N, int R, const double *__restrict__ alpha,
                                                    const double *__restrict__ p, const double *__restrict__ q,
                                                    double *x, int64_t ldx, double *r)
{
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < N * R; e += (int64_t)gridDim.x * kBlock) {
        const int64_t c = e / N, i = e - c * N;
        const double a = alpha[c];
        x[i + c * ldx] += a * p[e];
        r[e] -= a * q[e];
    }
}

// p = r + gamma_c p
__global__ __launch_bounds__(kBlock) void k_cg_dir(int64_t N, int R, const double *__restrict__ gamma,
                                                   const double *__restrict__ r, double *p)
{
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < N * R; e += (int64_t)gridDim.x * kBlock) {
        const int64_t c = e / N;
        p[e] = r[e] + gamma[c] * p[e];
    }
}

}  // namespace addk

using namespace addk;

extern "C" {

addk_status addk_cg(addk_plan plan, double beta, int32_t R, const double *Y, int64_t ldy, double *X, int64_t ldx,
                    double tol, int32_t maxit, int32_t *iters, double *relres, void *stream)
{
    if (!plan)
        return ADDK_ERR_INVALID_ARG;
    Plan &pl = *(Plan *)plan;
    if (pl.rect) {
        set_error("addk_cg needs a square plan (targets = sources)");
        return ADDK_ERR_UNSUPPORTED;
    }
    if (R < 1 || !Y || !X || ldy < pl.N || ldx < pl.N || !(tol > 0.0) || maxit < 0 || !(beta >= 0.0) ||
        !std::isfinite(beta)) {
        set_error("addk_cg: bad arguments (R >= 1, ld >= N, tol > 0, maxit >= 0, beta >= 0 required)");
        return ADDK_ERR_INVALID_ARG;
    }
    const int64_t N = pl.N;
    if (iters)
        *iters = 0;
    if (N == 0)
        return ADDK_OK;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = N * R;
    double *buf = nullptr;
    const int64_t nbuf = 3 * n + (int64_t)kDotBlocks * 2 * R + 4 * R;
    hipError_t e = hipMalloc(&buf, nbuf * sizeof(double));
    if (e != hipSuccess) {
        set_error(std::string("addk_cg workspace allocation of ") + std::to_string(nbuf * sizeof(double)) +
                  " bytes failed: " + hipGetErrorName(e));
        return ADDK_ERR_OOM;
    }
    double *r = buf, *p = r + n, *q = p + n, *partial = q + n, *dots = partial + (int64_t)kDotBlocks * 2 * R,
           *coef = dots + 2 * R;
    const int gb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    addk_status s = ADDK_OK;
    auto apply = [&](const double *in, double *out) {  // out = (K + beta I) in
        addk_status s2 = addk_matvec(plan, R, in, N, out, N, stream);
        if (s2 == ADDK_OK && beta != 0.0)
            hipLaunchKernelGGL(k_cg_shift, dim3(gb), dim3(kBlock), 0, st, n, beta, in, out);
        return s2;
    };
    std::vector<double> h(2 * R), alpha(R), gamma(R), rr(R), ynorm(R);
    auto dot = [&](const double *a, const double *b2, const double *c) -> addk_status {
        hipLaunchKernelGGL(k_cg_dots, dim3(kDotBlocks, R), dim3(kBlock), 0, st, N, R, a, b2, c, partial);
        hipLaunchKernelGGL(k_cg_dots_finish, dim3((2 * R + 63) / 64), dim3(64), 0, st, R, kDotBlocks, partial, dots);
        hipError_t e2 = hipMemcpyAsync(h.data(), dots, 2 * R * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e2 == hipSuccess)
            e2 = hipStreamSynchronize(st);
        return e2 == hipSuccess ? ADDK_OK : hip_fail(e2, "cg reduction");
    };
    // initial residual r = y - A x0 (x0 = X on entry), p = r; then ||y||, ||r||
    if (ldx == N) {
        s = apply(X, q);
    } else {
        e = hipMemcpy2DAsync(r, N * sizeof(double), X, ldx * sizeof(double), N * sizeof(double), R,
                             hipMemcpyDeviceToDevice, st);
        s = e == hipSuccess ? apply(r, q) : hip_fail(e, "cg copy");
    }
    if (s == ADDK_OK) {
        hipLaunchKernelGGL(k_cg_init, dim3(gb), dim3(kBlock), 0, st, N, R, Y, ldy, q, r, p);
        e = hipMemcpy2DAsync(q, N * sizeof(double), Y, ldy * sizeof(double), N * sizeof(double), R,
                             hipMemcpyDeviceToDevice, st);  // packed copy of y for its norm
        s = e == hipSuccess ? dot(q, q, r) : hip_fail(e, "cg copy");
    }
    std::vector<char> active(R, 1);
    int it = 0;
    if (s == ADDK_OK) {
        for (int c = 0; c < R; ++c) {
            ynorm[c] = std::sqrt(h[2 * c]);
            rr[c] = h[2 * c + 1];
            active[c] = ynorm[c] > 0.0 && std::sqrt(rr[c]) > tol * ynorm[c];
            if (relres)
                relres[c] = ynorm[c] > 0.0 ? std::sqrt(rr[c]) / ynorm[c] : 0.0;
        }
    }
    while (s == ADDK_OK && it < maxit && std::any_of(active.begin(), active.end(), [](char a) { return a != 0; })) {
        s = apply(p, q);
        if (s != ADDK_OK)
            break;
        if ((s = dot(p, q, nullptr)) != ADDK_OK)
            break;
        for (int c = 0; c < R; ++c)
            alpha[c] = (active[c] && h[2 * c] > 0.0) ? rr[c] / h[2 * c] : 0.0;
        e = hipMemcpyAsync(coef, alpha.data(), R * sizeof(double), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            s = hip_fail(e, "cg coefficients");
            break;
        }
        hipLaunchKernelGGL(k_cg_step, dim3(gb), dim3(kBlock), 0, st, N, R, coef, p, q, X, ldx, r);
        if ((s = dot(r, r, nullptr)) != ADDK_OK)
            break;
        ++it;
        for (int c = 0; c < R; ++c) {
            const double rn = h[2 * c];
            gamma[c] = (active[c] && rr[c] > 0.0) ? rn / rr[c] : 0.0;
            if (active[c]) {
                rr[c] = rn;
                if (relres)
                    relres[c] = std::sqrt(rn) / ynorm[c];
                if (std::sqrt(rn) <= tol * ynorm[c])
                    active[c] = 0;
            }
        }
        e = hipMemcpyAsync(coef + R, gamma.data(), R * sizeof(double), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            s = hip_fail(e, "cg coefficients");
            break;
        }
        hipLaunchKernelGGL(k_cg_dir, dim3(gb), dim3(kBlock), 0, st, N, R, coef + R, r, p);
    }
    if (s == ADDK_OK && (e = hipGetLastError()) != hipSuccess)
        s = hip_fail(e, "cg kernels");
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (iters)
        *iters = it;
    return s;
}

}  // extern "C"
