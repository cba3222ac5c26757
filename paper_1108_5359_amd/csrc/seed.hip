// Seed matrix recovery (Sec. 3.1, eq. SPCP) in FP64 on the device.
//
// Solves  min ||L||_* + lam ||S||_1  s.t.  Ms = L + S  on the p x q seed block
// by the inexact augmented Lagrange multiplier method, each step being a
// proximal map: singular value thresholding for L (Sec. 2, eqs. Proxy, SVT)
// and soft thresholding for S.  Order and constants:
//     Y_0 = Ms / max(||Ms||_2, ||Ms||_inf / lam),  S_0 = 0,
//     mu_0 = mu0_scale / ||Ms||_2,  mu_bar = mu_max_scale * mu_0,
//     L_{k+1} = SVT_{1/mu_k}(Ms - S_k + Y_k/mu_k)
//     S_{k+1} = S_{lam/mu_k}(Ms - L_{k+1} + Y_k/mu_k)
//     Y_{k+1} = Y_k + mu_k (Ms - L_{k+1} - S_{k+1}),  mu_{k+1} = min(rho mu_k, mu_bar)
// until ||Ms - L - S||_F / ||Ms||_F < tol.  The SVD is rocSOLVER's dgesvd;
// everything else is a handful of small FP64 kernels.  The skinny SVD of the
// final L (the factors U, Sigma = sigma - 1/mu, V used by l1 filtering,
// Sec. 3.2) comes from the last thresholding step.
#include "rpca_internal.h"

#include <rocsolver/rocsolver.h>

#include <chrono>
#include <cmath>
#include <vector>

namespace {

constexpr int kThreads = 256;

__global__ void gather_seed(const float *__restrict__ M, int64_t ldm, const int64_t *__restrict__ rows,
                            int64_t p, const int64_t *__restrict__ cols, int64_t q,
                            double *__restrict__ Ms)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * q) return;
    const int64_t a = t % p, b = t / p;
    Ms[t] = (double)M[rows[a] + cols[b] * ldm];
}

// partial[block] = (sum x^2, max |x|, count of non-finite)
__global__ void norms_kernel(const double *__restrict__ X, int64_t len, double *__restrict__ partial)
{
    __shared__ double ss[kThreads], sm[kThreads], sb[kThreads];
    double s = 0.0, mx = 0.0, bad = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double v = X[t];
        if (!isfinite(v)) bad += 1.0;
        else {
            s += v * v;
            mx = fmax(mx, fabs(v));
        }
    }
    ss[threadIdx.x] = s;
    sm[threadIdx.x] = mx;
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ss[threadIdx.x] += ss[threadIdx.x + w];
            sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x + 0] = ss[0];
        partial[3 * blockIdx.x + 1] = sm[0];
        partial[3 * blockIdx.x + 2] = sb[0];
    }
}

__global__ void scale_copy(const double *__restrict__ X, int64_t len, double s, double *__restrict__ Y)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) Y[t] = X[t] * s;
}

// W = Ms - S + Y / mu
__global__ void svt_input(const double *__restrict__ Ms, const double *__restrict__ S,
                          const double *__restrict__ Y, int64_t len, double inv_mu,
                          double *__restrict__ W)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len) W[t] = Ms[t] - S[t] + Y[t] * inv_mu;
}

// L = Uw[:, :k] diag(s[:k] - tau) Vt[:k, :]    (Uw: p x kk ld p, Vt: kk x q ld kk)
__global__ void svt_product(const double *__restrict__ Uw, const double *__restrict__ s,
                            const double *__restrict__ Vt, int64_t p, int64_t q, int kk, int k,
                            double tau, double *__restrict__ L)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * q) return;
    const int64_t a = t % p, b = t / p;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += Uw[a + (int64_t)c * p] * (s[c] - tau) * Vt[c + b * (int64_t)kk];
    L[t] = acc;
}

// S = shrink(Ms - L + Y/mu, lam/mu); Z = Ms - L - S; Y += mu Z; partial ||Z||^2
__global__ void sparse_dual_step(const double *__restrict__ Ms, const double *__restrict__ L,
                                 double *__restrict__ S, double *__restrict__ Y, int64_t len,
                                 double mu, double thr, double *__restrict__ partial)
{
    __shared__ double ss[kThreads];
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double T = Ms[t] - L[t] + Y[t] / mu;
        const double sv = T > thr ? T - thr : (T < -thr ? T + thr : 0.0);
        const double z = Ms[t] - L[t] - sv;
        S[t] = sv;
        Y[t] += mu * z;
        acc += z * z;
    }
    ss[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) ss[threadIdx.x] += ss[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = ss[0];
}

// Copy the kept factors into the caller's r-column buffers (zero the rest).
__global__ void write_factors(const double *__restrict__ Uw, const double *__restrict__ s,
                              const double *__restrict__ Vt, int64_t p, int64_t q, int kk,
                              int keep, int r, double tau, double *__restrict__ U,
                              double *__restrict__ sigma, double *__restrict__ V)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nu = p * r, nv = q * r;
    if (t < nu) {
        const int64_t a = t % p, c = t / p;
        U[t] = c < keep ? Uw[a + c * p] : 0.0;
    } else if (t < nu + nv) {
        const int64_t tt = t - nu;
        const int64_t b = tt % q, c = tt / q;
        V[tt] = c < keep ? Vt[c + b * (int64_t)kk] : 0.0;
    } else if (t < nu + nv + r) {
        const int c = (int)(t - nu - nv);
        sigma[c] = c < keep ? s[c] - tau : 0.0;
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

} // namespace

int run_seed(rpca_ctx *ctx, const float *M, int64_t ldm, const int64_t *seed_rows, int64_t p,
             const int64_t *seed_cols, int64_t q, int32_t r, const rpca_opts &o, double *U,
             double *sigma, double *V, SeedOut *out, hipStream_t stream)
{
    const int64_t len = p * q;
    const int kk = (int)(p < q ? p : q);
    const int kRedBlocks = 64;
    // workspace: Ms, S, Y, W, L, Uw (p x kk), Vt (kk x q), s, e, partials, info
    const size_t doubles = 5 * (size_t)len + (size_t)p * kk + (size_t)kk * q + 2 * (size_t)kk +
                           3 * kRedBlocks + 8;
    int st = ensure_buf(ctx, ctx->seed_ws, doubles * sizeof(double));
    if (st != RPCA_OK) return st;
    double *Ms = static_cast<double *>(ctx->seed_ws.ptr);
    double *Sm = Ms + len, *Y = Sm + len, *W = Y + len, *Lm = W + len;
    double *Uw = Lm + len, *Vt = Uw + (size_t)p * kk, *sv = Vt + (size_t)kk * q, *ev = sv + kk;
    double *partial = ev + kk;
    rocblas_int *info = reinterpret_cast<rocblas_int *>(partial + 3 * kRedBlocks);

    rocblas_status bs = rocblas_set_stream(ctx->blas, stream);
    if (bs != rocblas_status_success) return set_status(ctx, RPCA_ERR_DEVICE, "seed: rocblas_set_stream failed");

    hipLaunchKernelGGL(gather_seed, dim3(blocks_for(len)), dim3(kThreads), 0, stream, M, ldm,
                       seed_rows, p, seed_cols, q, Ms);
    hipLaunchKernelGGL(norms_kernel, dim3(kRedBlocks), dim3(kThreads), 0, stream, Ms, len, partial);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    std::vector<double> hp(3 * kRedBlocks);
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(hp.data(), partial, hp.size() * sizeof(double),
                                     hipMemcpyDeviceToHost, stream));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(stream));
    double ss = 0.0, mx = 0.0, bad = 0.0;
    for (int b = 0; b < kRedBlocks; ++b) {
        ss += hp[3 * b];
        mx = std::fmax(mx, hp[3 * b + 1]);
        bad += hp[3 * b + 2];
    }
    if (bad > 0) return set_status(ctx, RPCA_ERR_NUMERIC, "seed: non-finite entry in the seed block");
    const double normF = std::sqrt(ss);
    if (normF == 0.0) return set_status(ctx, RPCA_ERR_SEED, "seed: the seed block is zero");

    std::vector<double> hs(kk);
    auto svd = [&](double *A) -> int {
        // A (p x q, ld p) is destroyed.
        rocblas_status s = rocsolver_dgesvd(ctx->blas, rocblas_svect_singular, rocblas_svect_singular,
                                            (rocblas_int)p, (rocblas_int)q, A, (rocblas_int)p, sv, Uw,
                                            (rocblas_int)p, Vt, (rocblas_int)kk, ev,
                                            rocblas_outofplace, info);
        if (s != rocblas_status_success)
            return set_status(ctx, RPCA_ERR_DEVICE, "seed: rocsolver_dgesvd failed");
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(hs.data(), sv, kk * sizeof(double), hipMemcpyDeviceToHost, stream));
        rocblas_int hinfo = 0;
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, stream));
        RPCA_HIP_TRY(ctx, hipStreamSynchronize(stream));
        if (hinfo != 0) return set_status(ctx, RPCA_ERR_DEVICE, "seed: SVD did not converge");
        return RPCA_OK;
    };

    // ||Ms||_2 from an SVD of a copy
    hipLaunchKernelGGL(scale_copy, dim3(blocks_for(len)), dim3(kThreads), 0, stream, Ms, len, 1.0, W);
    if ((st = svd(W)) != RPCA_OK) return st;
    const double norm2 = hs[0];
    const double lam = o.seed_lambda > 0 ? o.seed_lambda : 1.0 / std::sqrt((double)(p > q ? p : q));
    hipLaunchKernelGGL(scale_copy, dim3(blocks_for(len)), dim3(kThreads), 0, stream, Ms, len,
                       1.0 / std::fmax(norm2, mx / lam), Y);
    RPCA_HIP_TRY(ctx, hipMemsetAsync(Sm, 0, len * sizeof(double), stream));
    double mu = o.seed_mu0_scale / norm2;
    const double mu_bar = o.seed_mu_max_scale * mu;

    int k = 0, svp = 0;
    double mu_used = mu;
    bool converged = false;
    for (k = 1; k <= o.seed_max_iter; ++k) {
        hipLaunchKernelGGL(svt_input, dim3(blocks_for(len)), dim3(kThreads), 0, stream, Ms, Sm, Y,
                           len, 1.0 / mu, W);
        if ((st = svd(W)) != RPCA_OK) return st;
        const double tau = 1.0 / mu;
        svp = 0;
        while (svp < kk && hs[svp] > tau) ++svp;
        hipLaunchKernelGGL(svt_product, dim3(blocks_for(len)), dim3(kThreads), 0, stream, Uw, sv, Vt,
                           p, q, kk, svp, tau, Lm);
        hipLaunchKernelGGL(sparse_dual_step, dim3(kRedBlocks), dim3(kThreads), 0, stream, Ms, Lm, Sm,
                           Y, len, mu, lam / mu, partial);
        RPCA_HIP_TRY(ctx, hipGetLastError());
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(hp.data(), partial, kRedBlocks * sizeof(double),
                                         hipMemcpyDeviceToHost, stream));
        RPCA_HIP_TRY(ctx, hipStreamSynchronize(stream));
        double zz = 0.0;
        for (int b = 0; b < kRedBlocks; ++b) zz += hp[b];
        mu_used = mu;
        mu = std::fmin(o.seed_rho * mu, mu_bar);
        if (std::sqrt(zz) / normF < o.seed_tol) {
            converged = true;
            break;
        }
    }
    if (k > o.seed_max_iter) k = o.seed_max_iter;

    // rank of the recovered seed: thresholded values above the floor
    const double tau = 1.0 / mu_used;
    int rank = 0;
    if (svp > 0) {
        const double top = hs[0] - tau;
        while (rank < svp && (hs[rank] - tau) > o.seed_rank_floor * top) ++rank;
    }
    const int keep = rank < r ? rank : r;
    const int64_t nw = (p + q) * (int64_t)r + r;
    hipLaunchKernelGGL(write_factors, dim3(blocks_for(nw)), dim3(kThreads), 0, stream, Uw, sv, Vt, p,
                       q, kk, keep, r, tau, U, sigma, V);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(stream));
    out->iters = k;
    out->converged = converged ? 1 : 0;
    out->rank_found = rank;
    out->r_used = keep;
    if (rank == 0) return set_status(ctx, RPCA_ERR_SEED, "seed: the recovered seed has rank 0");
    if (rank != r)
        return set_status(ctx, RPCA_WARN_RANK,
                          "seed: rank of L^s is " + std::to_string(rank) + ", target " + std::to_string(r));
    if (!converged) return set_status(ctx, RPCA_WARN_NOT_CONVERGED, "seed: tolerance not met");
    return RPCA_OK;
}
