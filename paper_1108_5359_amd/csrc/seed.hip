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
// until ||Ms - L - S||_F / ||Ms||_F < tol.  The skinny SVD of the final L (the
// factors U, Sigma = sigma - 1/mu, V used by l1 filtering, Sec. 3.2) comes
// from the last thresholding step.
//
// SVD route: the thresholding only needs the singular triplets above 1/mu.
// They come from the symmetric eigen-decomposition of the Gram matrix on the
// smaller side (G = W^T W, rocSOLVER dsyevd; about 25x faster than dgesvd at
// 200 x 200 and 60x at 500 x 500 on MI355X): sigma_i = sqrt(lambda_i), V from
// the eigenvectors and U = W V Sigma^{-1} (rocBLAS dgemm), or the mirror
// image when p < q.  Squaring the spectrum costs relative accuracy only on
// singular values far below the kept ones.
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

// L = Uk diag(s[:k] - tau) Vk^T    (Uk: p x k ld p, Vk: q x k ld q)
__global__ void svt_product(const double *__restrict__ Uk, const double *__restrict__ s,
                            const double *__restrict__ Vk, int64_t p, int64_t q, int k, double tau,
                            double *__restrict__ L)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * q) return;
    const int64_t a = t % p, b = t / p;
    double acc = 0.0;
    for (int c = 0; c < k; ++c) acc += Uk[a + (int64_t)c * p] * (s[c] - tau) * Vk[b + (int64_t)c * q];
    L[t] = acc;
}

// Eigenvectors of the Gram matrix (ascending eigenvalues, columns of E, ld
// nn) -> the k leading ones in descending order: out[:, c] = E[:, nn-1-c].
__global__ void take_leading(const double *__restrict__ E, int64_t nn, int k, double *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * k) return;
    const int64_t a = t % nn, c = t / nn;
    out[t] = E[a + (nn - 1 - c) * nn];
}

// X[:, c] *= 1 / s[c]   (X: rows x k, ld rows)
__global__ void scale_cols_inv(double *__restrict__ X, int64_t rows, int k, const double *__restrict__ s)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * k) return;
    X[t] /= s[t / rows];
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
__global__ void write_factors(const double *__restrict__ Uk, const double *__restrict__ s,
                              const double *__restrict__ Vk, int64_t p, int64_t q, int keep,
                              int r, double tau, double *__restrict__ U,
                              double *__restrict__ sigma, double *__restrict__ V)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nu = p * r, nv = q * r;
    if (t < nu) {
        const int64_t c = t / p;
        U[t] = c < keep ? Uk[t] : 0.0;
    } else if (t < nu + nv) {
        const int64_t tt = t - nu;
        const int64_t c = tt / q;
        V[tt] = c < keep ? Vk[tt] : 0.0;
    } else if (t < nu + nv + r) {
        const int c = (int)(t - nu - nv);
        sigma[c] = c < keep ? s[c] - tau : 0.0;
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

} // namespace

int seed_status_message(rpca_ctx *ctx, int status, const SeedOut &so, int32_t r)
{
    switch (status) {
    case RPCA_ERR_NUMERIC: return set_status(ctx, status, "seed: non-finite entry in the seed block");
    case RPCA_ERR_SEED: return set_status(ctx, status, "seed: the recovered seed has rank 0");
    case RPCA_WARN_RANK:
        return set_status(ctx, status, "seed: rank of L^s is " + std::to_string(so.rank_found) +
                                           ", target " + std::to_string(r));
    case RPCA_WARN_NOT_CONVERGED: return set_status(ctx, status, "seed: tolerance not met");
    default: return status;
    }
}

int run_seed(rpca_ctx *ctx, const float *M, int64_t ldm, const int64_t *seed_rows, int64_t p,
             const int64_t *seed_cols, int64_t q, int32_t r, const rpca_opts &o, double *U,
             double *sigma, double *V, SeedOut *out, hipStream_t stream)
{
    // The device-resident solvers where the block fits them: the whole ALM
    // in one workgroup (Jacobi SVD in LDS up to 6400 entries, seed_small.hip;
    // subspace iteration up to 512 x 512, seed_large.hip, only when asked
    // for: for one block alone the eigen-decomposition route below is the
    // faster, the subspace route pays off when a batch runs many blocks in
    // one launch); else, or when the subspace iteration needs more
    // directions than it holds, the eigen-decomposition route.
    bool fell_back = false;
    if (o.seed_route != 1) {
        const bool small = p * q <= 6400 && seed_small_fits(ctx, p, q);
        const bool large = !small && o.seed_route == 2 && seed_large_fits(ctx, p, q);
        if (small || large) {
            SmallSeedArgs a{M, ldm, seed_rows, seed_cols, p, q, r, U, sigma, V};
            int st = ensure_buf(ctx, ctx->seed_ws, small ? seed_small_workspace(&a, 1)
                                                         : seed_large_workspace(&a, 1));
            if (st != RPCA_OK) return st;
            SeedOut so;
            int sst = RPCA_OK;
            st = small ? run_seed_small(ctx, &a, 1, o, ctx->seed_ws.ptr, &so, &sst, stream)
                       : run_seed_large(ctx, &a, 1, o, ctx->seed_ws.ptr, &so, &sst, stream);
            if (st != RPCA_OK) return st;
            if (!(large && so.fallback)) {
                *out = so;
                return seed_status_message(ctx, sst, so, r);
            }
            fell_back = true;
        }
    }
    const int64_t len = p * q;
    const int kk = (int)(p < q ? p : q);          // Gram side
    const bool gram_right = q <= p;               // G = W^T W (q x q), else W W^T (p x p)
    const int kRedBlocks = 64;
    // workspace: Ms, S, Y, W, L, G (kk x kk), Uk (p x kk), Vk (q x kk), eig, sig, partials, info
    const size_t doubles = 5 * (size_t)len + (size_t)kk * kk + (size_t)p * kk + (size_t)q * kk +
                           2 * (size_t)kk + 3 * kRedBlocks + 8;
    int st = ensure_buf(ctx, ctx->seed_ws, doubles * sizeof(double));
    if (st != RPCA_OK) return st;
    double *Ms = static_cast<double *>(ctx->seed_ws.ptr);
    double *Sm = Ms + len, *Y = Sm + len, *W = Y + len, *Lm = W + len;
    double *Gm = Lm + len, *Uk = Gm + (size_t)kk * kk, *Vk = Uk + (size_t)p * kk;
    double *eig = Vk + (size_t)q * kk, *sv = eig + kk;
    double *partial = sv + kk;
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

    // Singular values of A (p x q, ld p) in descending order into hs (host) and
    // sv (device); with want_vectors, the k leading singular vectors above tau
    // into Uk (p x k) and Vk (q x k).  Returns the count k through *kout.
    std::vector<double> hs(kk), heig(kk);
    const double one = 1.0, zero = 0.0;
    auto svd_above = [&](const double *A, double tau, bool want_vectors, int *kout) -> int {
        rocblas_status s1 = gram_right
            ? rocblas_dgemm(ctx->blas, rocblas_operation_transpose, rocblas_operation_none, kk, kk,
                            (rocblas_int)p, &one, A, (rocblas_int)p, A, (rocblas_int)p, &zero, Gm, kk)
            : rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_transpose, kk, kk,
                            (rocblas_int)q, &one, A, (rocblas_int)p, A, (rocblas_int)p, &zero, Gm, kk);
        if (s1 != rocblas_status_success) return set_status(ctx, RPCA_ERR_DEVICE, "seed: rocblas_dgemm failed");
        rocblas_status s2 = rocsolver_dsyevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, kk, Gm,
                                             kk, eig, sv, info);   // sv used as the off-diagonal scratch
        if (s2 != rocblas_status_success) return set_status(ctx, RPCA_ERR_DEVICE, "seed: rocsolver_dsyevd failed");
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(heig.data(), eig, kk * sizeof(double), hipMemcpyDeviceToHost, stream));
        rocblas_int hinfo = 0;
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(&hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, stream));
        RPCA_HIP_TRY(ctx, hipStreamSynchronize(stream));
        if (hinfo != 0) return set_status(ctx, RPCA_ERR_DEVICE, "seed: eigen-decomposition did not converge");
        for (int i = 0; i < kk; ++i) hs[i] = std::sqrt(std::fmax(heig[kk - 1 - i], 0.0));
        int k = 0;
        while (k < kk && hs[k] > tau) ++k;
        *kout = k;
        if (!want_vectors || k == 0) return RPCA_OK;
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(sv, hs.data(), k * sizeof(double), hipMemcpyHostToDevice, stream));
        double *side = gram_right ? Vk : Uk;          // eigenvectors: the Gram side
        double *other = gram_right ? Uk : Vk;
        const int64_t nside = gram_right ? q : p, nother = gram_right ? p : q;
        hipLaunchKernelGGL(take_leading, dim3(blocks_for(nside * k)), dim3(kThreads), 0, stream, Gm,
                           nside, k, side);
        // other = A side Sigma^{-1}   (U = W V / sigma, or V = W^T U / sigma)
        rocblas_status s3 = gram_right
            ? rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)p, k,
                            (rocblas_int)q, &one, A, (rocblas_int)p, side, (rocblas_int)q, &zero, other,
                            (rocblas_int)p)
            : rocblas_dgemm(ctx->blas, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)q, k,
                            (rocblas_int)p, &one, A, (rocblas_int)p, side, (rocblas_int)p, &zero, other,
                            (rocblas_int)q);
        if (s3 != rocblas_status_success) return set_status(ctx, RPCA_ERR_DEVICE, "seed: rocblas_dgemm failed");
        hipLaunchKernelGGL(scale_cols_inv, dim3(blocks_for(nother * k)), dim3(kThreads), 0, stream, other,
                           nother, k, sv);
        RPCA_HIP_TRY(ctx, hipGetLastError());
        return RPCA_OK;
    };

    // ||Ms||_2 from the largest eigenvalue of its Gram matrix
    int kdummy = 0;
    if ((st = svd_above(Ms, 0.0, false, &kdummy)) != RPCA_OK) return st;
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
        const double tau = 1.0 / mu;
        if ((st = svd_above(W, tau, true, &svp)) != RPCA_OK) return st;
        hipLaunchKernelGGL(svt_product, dim3(blocks_for(len)), dim3(kThreads), 0, stream, Uk, sv, Vk,
                           p, q, svp, tau, Lm);
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
    hipLaunchKernelGGL(write_factors, dim3(blocks_for(nw)), dim3(kThreads), 0, stream, Uk, sv, Vk, p,
                       q, keep, r, tau, U, sigma, V);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(stream));
    out->iters = k;
    out->converged = converged ? 1 : 0;
    out->rank_found = rank;
    out->r_used = keep;
    out->route = fell_back ? RPCA_SEED_ROUTE_FELL_BACK : RPCA_SEED_ROUTE_EIGEN;
    if (rank == 0) return set_status(ctx, RPCA_ERR_SEED, "seed: the recovered seed has rank 0");
    if (rank != r)
        return set_status(ctx, RPCA_WARN_RANK,
                          "seed: rank of L^s is " + std::to_string(rank) + ", target " + std::to_string(r));
    if (!converged) return set_status(ctx, RPCA_WARN_NOT_CONVERGED, "seed: tolerance not met");
    return RPCA_OK;
}
