// Seed matrix recovery (Sec. 3.1, eq. SPCP) for many small seed blocks at
// once: one workgroup per problem runs the whole inexact ALM of the seed
// solver (same order and constants as seed.hip, see there) without returning
// to the host between iterations.
//
// Singular value thresholding (Sec. 2, eq. SVT) uses a one-sided Jacobi SVD
// (Hestenes' method) in FP64 on the work matrix X held in LDS: X is the SVT
// input W (p x q) when p >= q, else its transpose, so its n2 = min(p, q)
// columns of length n1 = max(p, q) are orthogonalised by plane rotations
// accumulated into V (n2 x n2, also in LDS).  At convergence the column norms
// are the singular values, X = U Sigma, and the thresholded product is
//   L = sum_{sigma_i > tau} x_i (1 - tau / sigma_i) v_i^T.
// Rotations of disjoint column pairs are independent, so the pairs of a
// round-robin tournament round run in parallel, 8 lanes per pair; a sweep is
// n2 - 1 (or n2) rounds and sweeps repeat until no pair is rotated.  The
// factors U, Sigma = sigma - tau, V of the final step are written in
// descending order of sigma, and the rank rule is that of seed.hip.
//
// The matrices Ms, S, Y of the iteration live in a global workspace (3 p q
// doubles per problem, L2 resident); LDS holds X, V and the singular values,
// which, with speed, bounds the problems this path accepts (seed_small_fits).
#include "rpca_internal.h"
#include "seed_jacobi.h"

#include <cfloat>
#include <cmath>
#include <algorithm>
#include <vector>

namespace seedk {

using namespace seedj;

constexpr int64_t kMaxElems = 80 * 80;      // largest seed block (p q) of this route
// Jacobi of the SVT: 4 lanes per column pair (the 40 pairs of an 80-column
// round in one pass; shorter lane sums than with 8, two elements per 16-byte
// LDS access) and the absolute orthogonality test (8.4 -> 7.2 sweeps per ALM
// step on the median).  On 256 seed blocks of 10 x 10 to 80 x 80: 639 ->
// 378 ms, with the same ALM step counts and L^s.
constexpr int kPairLanes = 4;

struct SmallSeedJob {
    const float *M;
    int64_t ldm;
    const int64_t *rows, *cols;
    int32_t p, q, r, pad;
    double *U, *sigma, *V;      // outputs: p x r (ld p), r, q x r (ld q)
    double *ws;                 // 3 p q doubles: Ms, S, Y (column-major, ld p)
    int32_t *result;            // status, r_used, iters, converged, rank_found
};

struct SmallSeedConsts {
    double lam, tol, rho, mu0_scale, mu_max_scale, rank_floor;
    int32_t max_iter;
};

// X <- the SVT input W = Ms - S + Y inv_mu (transposed when p < q).
__device__ void load_x(double *X, const double *Ms, const double *S, const double *Y, int p, int q,
                       bool tall, double inv_mu)
{
    const int pq = p * q;
    for (int t = threadIdx.x; t < pq; t += kThreads) {
        const int a = t % p, b = t / p;
        const double w = Ms[t] - S[t] + Y[t] * inv_mu;
        if (tall) X[t] = w;                       // X = W, n1 = p
        else X[b + (int64_t)a * q] = w;           // X = W^T, n1 = q
    }
    __syncthreads();
}

constexpr int kRowChunk = 8;                    // rows of W staged per step of the product

// X <- W^(T) V for the V of the previous step (warm start), kRowChunk rows of
// the work matrix at a time through the staging area stg (kRowChunk x n2).
__device__ void load_x_rotated(double *X, const double *V, double *stg, const double *Ms,
                               const double *S, const double *Y, int p, int q, bool tall,
                               double inv_mu)
{
    const int n1 = tall ? p : q, n2 = tall ? q : p;
    for (int a0 = 0; a0 < n1; a0 += kRowChunk) {
        const int rows = n1 - a0 < kRowChunk ? n1 - a0 : kRowChunk;
        // stage rows a0 .. a0 + rows of the work matrix: row a of X's source
        for (int t = threadIdx.x; t < rows * n2; t += kThreads) {
            const int ra = t % rows, b = t / rows, a = a0 + ra;
            const int w = tall ? a + b * p : b + a * p;          // W[a][b] or W[b][a]
            stg[ra + b * kRowChunk] = Ms[w] - S[w] + Y[w] * inv_mu;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < rows * n2; t += kThreads) {
            const int ra = t % rows, c = t / rows;
            double acc = 0.0;
            for (int b = 0; b < n2; ++b) acc = fma(stg[ra + b * kRowChunk], V[b + (int64_t)c * n2], acc);
            X[(a0 + ra) + (int64_t)c * n1] = acc;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kThreads)
seed_small_kernel(const SmallSeedJob *__restrict__ jobs, SmallSeedConsts C)
{
    extern __shared__ __align__(16) double lds[];
    __shared__ double red[4];
    __shared__ int flag;
    const SmallSeedJob &J = jobs[blockIdx.x];
    const int p = J.p, q = J.q, tid = threadIdx.x;
    const int pq = p * q;
    const bool tall = p >= q;
    const int n1 = tall ? p : q, n2 = tall ? q : p;
    double *X = lds;
    double *V = X + (int64_t)n1 * n2;
    double *sig = V + (int64_t)n2 * n2;
    double *wt = sig + n2;
    double *stg = wt + n2;                                  // kRowChunk x n2
    int *ord = reinterpret_cast<int *>(stg + (int64_t)kRowChunk * n2);
    double *Ms = J.ws, *S = Ms + pq, *Y = S + pq;

    // ---- gather M^s (FP64), its norms, non-finite entries
    double ss = 0.0, mx = 0.0, bad = 0.0;
    for (int t = tid; t < pq; t += kThreads) {
        const int a = t % p, b = t / p;
        const double v = (double)J.M[J.rows[a] + J.cols[b] * J.ldm];
        Ms[t] = v;
        if (!isfinite(v)) bad += 1.0;
        else {
            ss = fma(v, v, ss);
            mx = fmax(mx, fabs(v));
        }
    }
    const double normF = sqrt(block_sum(ss, red));
    mx = block_max(mx, red);
    bad = block_sum(bad, red);
    if (bad > 0.0 || normF == 0.0) {
        if (tid == 0) {
            J.result[0] = bad > 0.0 ? RPCA_ERR_NUMERIC : RPCA_ERR_SEED;
            J.result[1] = J.result[2] = J.result[3] = J.result[4] = 0;
        }
        return;
    }

    // ---- ||M^s||_2: the largest singular value of M^s
    for (int t = tid; t < pq; t += kThreads) {
        const int a = t % p, b = t / p;
        if (tall) X[t] = Ms[t];
        else X[b + (int64_t)a * q] = Ms[t];
    }
    __syncthreads();
    jacobi_svd(X, V, n1, n2, &flag, true, kPairLanes, true);
    column_norms(X, n1, n2, sig);
    double norm2 = 0.0;
    for (int c = 0; c < n2; ++c) norm2 = fmax(norm2, sig[c]);

    const double lam = C.lam > 0.0 ? C.lam : 1.0 / sqrt((double)(p > q ? p : q));
    const double y0 = 1.0 / fmax(norm2, mx / lam);
    for (int t = tid; t < pq; t += kThreads) {
        Y[t] = Ms[t] * y0;
        S[t] = 0.0;
    }
    double mu = C.mu0_scale / norm2;
    const double mu_bar = C.mu_max_scale * mu;
    double mu_used = mu;
    bool converged = false;
    int k;
    __syncthreads();
    for (k = 1; k <= C.max_iter; ++k) {
        // L = SVT_{1/mu}(Ms - S + Y / mu); the right rotations of the previous
        // step start the Jacobi sweeps (restarted from the identity every
        // kColdEvery steps so that rounding in V cannot accumulate)
        const bool cold = (k - 1) % kColdEvery == 0;
        if (cold) load_x(X, Ms, S, Y, p, q, tall, 1.0 / mu);
        else load_x_rotated(X, V, stg, Ms, S, Y, p, q, tall, 1.0 / mu);
        jacobi_svd(X, V, n1, n2, &flag, cold, kPairLanes, true);
        column_norms(X, n1, n2, sig);
        const double tau = 1.0 / mu;
        for (int c = tid; c < n2; c += kThreads) wt[c] = sig[c] > tau ? 1.0 - tau / sig[c] : 0.0;
        __syncthreads();
        // S = shrink(Ms - L + Y / mu, lam / mu), Z = Ms - L - S, Y += mu Z
        const double thr = lam / mu;
        double zz = 0.0;
        for (int t = tid; t < pq; t += kThreads) {
            const int a = t % p, b = t / p;
            const int ax = tall ? a : b, bx = tall ? b : a;     // (row of X, row of V)
            double l = 0.0;
            for (int c = 0; c < n2; ++c)
                l = fma(X[(int64_t)c * n1 + ax] * wt[c], V[(int64_t)c * n2 + bx], l);
            const double T = Ms[t] - l + Y[t] / mu;
            const double sv = T > thr ? T - thr : (T < -thr ? T + thr : 0.0);
            const double z = Ms[t] - l - sv;
            S[t] = sv;
            Y[t] += mu * z;
            zz = fma(z, z, zz);
        }
        zz = block_sum(zz, red);
        mu_used = mu;
        mu = fmin(C.rho * mu, mu_bar);
        if (sqrt(zz) / normF < C.tol) {
            converged = true;
            break;
        }
    }
    if (k > C.max_iter) k = C.max_iter;

    // ---- order of the singular values (descending; ties by index), rank
    for (int c = tid; c < n2; c += kThreads) {
        int pos = 0;
        for (int d = 0; d < n2; ++d)
            pos += (sig[d] > sig[c]) || (sig[d] == sig[c] && d < c);
        ord[pos] = c;
    }
    __syncthreads();
    const double tau = 1.0 / mu_used;
    int svp = 0;
    while (svp < n2 && sig[ord[svp]] > tau) ++svp;
    int rank = 0;
    if (svp > 0) {
        const double top = sig[ord[0]] - tau;
        while (rank < svp && (sig[ord[rank]] - tau) > C.rank_floor * top) ++rank;
    }
    const int r = J.r;
    const int keep = rank < r ? rank : r;
    // U (p x r), sigma (r), V (q x r); columns beyond keep are zero
    for (int t = tid; t < p * r; t += kThreads) {
        const int a = t % p, c = t / p;
        double v = 0.0;
        if (c < keep) {
            const int i = ord[c];
            v = tall ? X[(int64_t)i * n1 + a] / sig[i] : V[(int64_t)i * n2 + a];
        }
        J.U[t] = v;
    }
    for (int t = tid; t < q * r; t += kThreads) {
        const int b = t % q, c = t / q;
        double v = 0.0;
        if (c < keep) {
            const int i = ord[c];
            v = tall ? V[(int64_t)i * n2 + b] : X[(int64_t)i * n1 + b] / sig[i];
        }
        J.V[t] = v;
    }
    for (int c = tid; c < r; c += kThreads) J.sigma[c] = c < keep ? sig[ord[c]] - tau : 0.0;
    if (tid == 0) {
        J.result[0] = rank == 0 ? RPCA_ERR_SEED
                                : (rank != r ? RPCA_WARN_RANK : (converged ? RPCA_OK : RPCA_WARN_NOT_CONVERGED));
        J.result[1] = keep;
        J.result[2] = k;
        J.result[3] = converged ? 1 : 0;
        J.result[4] = rank;
    }
}

size_t lds_bytes(int p, int q)
{
    const int n1 = p > q ? p : q, n2 = p > q ? q : p;
    return ((size_t)n1 * n2 + (size_t)n2 * n2 + (2 + kRowChunk) * (size_t)n2) * sizeof(double) +
           (size_t)n2 * sizeof(int);
}

} // namespace seedk

bool seed_small_fits(rpca_ctx *ctx, int64_t p, int64_t q)
{
    // above ~80 x 80 one workgroup's Jacobi sweeps are slower than the
    // device-wide eigen-solver route (measured: 100 x 100, 6 ms vs 1.8 ms per step)
    if (p < 1 || q < 1 || p * q > seedk::kMaxElems) return false;
    const size_t limit = ctx->max_lds ? ctx->max_lds : 65536;
    return seedk::lds_bytes((int)p, (int)q) + 1024 <= limit;
}

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace layout: the Ms, S, Y matrices of every problem, the job table,
// the per-problem results.
void layout(const SmallSeedArgs *args, int n, size_t *mats, size_t *table, size_t *results,
            size_t *total)
{
    size_t d = 0;
    for (int k = 0; k < n; ++k) d += 3 * (size_t)args[k].p * args[k].q;
    *mats = 0;
    *table = align256(d * sizeof(double));
    *results = align256(*table + (size_t)n * sizeof(seedk::SmallSeedJob));
    *total = align256(*results + (size_t)n * 8 * sizeof(int32_t));
}

} // namespace

size_t seed_small_workspace(const SmallSeedArgs *args, int n)
{
    size_t a, b, c, t;
    layout(args, n, &a, &b, &c, &t);
    return t;
}

int run_seed_small(rpca_ctx *ctx, const SmallSeedArgs *args, int n, const rpca_opts &o, void *ws,
                   SeedOut *outs, int *statuses, hipStream_t stream)
{
    if (n <= 0) return RPCA_OK;
    using namespace seedk;
    size_t o_mats, o_table, o_res, total;
    layout(args, n, &o_mats, &o_table, &o_res, &total);
    char *base = static_cast<char *>(ws);
    double *mats = reinterpret_cast<double *>(base + o_mats);
    SmallSeedJob *dj = reinterpret_cast<SmallSeedJob *>(base + o_table);
    int32_t *results = reinterpret_cast<int32_t *>(base + o_res);
    std::vector<SmallSeedJob> hj((size_t)n);
    size_t off = 0, lds = 0;
    for (int k = 0; k < n; ++k) {
        const SmallSeedArgs &a = args[k];
        if (!seed_small_fits(ctx, a.p, a.q))
            return set_status(ctx, RPCA_ERR_UNSUPPORTED, "seed: block too large for the batched seed solver");
        hj[k] = SmallSeedJob{a.M, a.ldm, a.rows, a.cols, (int32_t)a.p, (int32_t)a.q, a.r, 0,
                             a.U, a.sigma, a.V, mats + off, results + 8 * k};
        off += 3 * (size_t)a.p * a.q;
        lds = std::max(lds, seedk::lds_bytes((int)a.p, (int)a.q));
    }
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(dj, hj.data(), hj.size() * sizeof(SmallSeedJob),
                                     hipMemcpyHostToDevice, stream));
    SmallSeedConsts c{o.seed_lambda, o.seed_tol, o.seed_rho, o.seed_mu0_scale, o.seed_mu_max_scale,
                      o.seed_rank_floor, o.seed_max_iter};
    RPCA_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(seed_small_kernel),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(seed_small_kernel, dim3((unsigned)n), dim3(kThreads), lds, stream, dj, c);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    std::vector<int32_t> hr((size_t)8 * n);
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(hr.data(), results, hr.size() * sizeof(int32_t),
                                     hipMemcpyDeviceToHost, stream));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(stream));
    for (int k = 0; k < n; ++k) {
        statuses[k] = hr[8 * k];
        outs[k].r_used = hr[8 * k + 1];
        outs[k].iters = hr[8 * k + 2];
        outs[k].converged = hr[8 * k + 3];
        outs[k].rank_found = hr[8 * k + 4];
        outs[k].route = RPCA_SEED_ROUTE_LDS_JACOBI;
    }
    return RPCA_OK;
}
