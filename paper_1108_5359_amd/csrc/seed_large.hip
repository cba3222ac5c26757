// Seed matrix recovery (Sec. 3.1, eq. SPCP) on blocks above the LDS-resident
// solver of seed_small.hip: one workgroup per problem runs the whole inexact
// ALM of the seed solver (order and constants of seed.hip) on the device,
// with the matrices of the iteration in an L2-resident workspace, so no step
// returns to the host.
//
// Singular value thresholding (Sec. 2, eq. SVT) needs only the singular
// triplets above tau = 1/mu, and their number (the rank of the iterate L) is
// far below min(p, q).  They come from a subspace iteration on
// W = Ms - S + Y/mu with a Rayleigh-Ritz step: with V (q x k) orthonormal,
//   B = W V,  B = Q R  (Cholesky QR, twice, of B with its columns scaled to
//                       unit norm),
//   R = Ut diag(sigma) Vt^T  (one-sided Jacobi in LDS, seed_jacobi.h),
//   U = Q Ut,  V <- V Vt,
// which is the exact SVD of W restricted to span(V); then one power step
// V <- orth(W^T U), and again, until the thresholded product
//   L = sum_{sigma_i > tau} (sigma_i - tau) u_i v_i^T
// moves by at most tol_in ||L||_F between two Ritz steps.  tol_in =
// min(1e-6, max(1e-13, 1e-3 r)) follows the ALM's relative residual r of the
// previous step, so the SVT is as exact as the iterate needs and exact to
// rounding at the end.  Each ALM step starts from the previous step's Ritz
// basis; the basis widens by kGuard directions whenever fewer than kGuard/2
// of its Ritz values fall at or below tau, so that the directions just below
// the threshold are resolved as well, and narrows back to the kept
// directions plus the guard band at the start of the next step.  (A basis
// that would have to exceed
// kKMax columns reports kFallback; the caller then takes the eigen-solver
// route of seed.hip.)  ||Ms||_2, which sets mu_0 and Y_0, comes from the same
// iteration on Ms, run until the largest Ritz value is stable to 1e-15.
#include "rpca_internal.h"
#include "seed_jacobi.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

namespace seedl {

using namespace seedj;

constexpr int kKMax = 72;          // widest subspace (LDS: three kKMax^2 buffers)
constexpr int kGuard = 16;         // directions added at a time
constexpr int kInnerCap = 64;      // Ritz steps per ALM step at most
constexpr int kNormCap = 100;      // Ritz steps of the norm estimate at most
constexpr int kFallback = 1;       // result[6]: the subspace would exceed kKMax

struct LargeSeedJob {
    const float *M;
    int64_t ldm;
    const int64_t *rows, *cols;
    int32_t p, q, r, kmax;
    double *U, *sigma, *V;      // outputs: p x r (ld p), r, q x r (ld q)
    double *ws;                 // workspace, ws_doubles(p, q) doubles
    int32_t *result;            // status, r_used, iters, converged, rank_found, ritz steps, fallback
};

struct LargeSeedConsts {
    double lam, tol, rho, mu0_scale, mu_max_scale, rank_floor;
    int32_t max_iter;
};

__host__ __device__ inline int64_t ws_doubles(int p, int q)
{
    return 6 * (int64_t)p * q + (2 * (int64_t)p + 2 * (int64_t)q) * kKMax;
}

// Uniform value in [-1, 1) keyed by (salt, index): SplitMix64 (Steele, Lea,
// Flood, OOPSLA 2014) of the index, for the deterministic start vectors.
__device__ inline double hash_unit(uint64_t salt, uint64_t idx)
{
    uint64_t z = idx * 0x9E3779B97F4A7C15ull + salt + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Workgroup GEMM on FP64 MFMA (v_mfma_f64_16x16x4f64):
//   C (m x n, ldc) = op(A) diag(dk) op(B),
// column-major, op(A) m x kk (A, or A^T of a kk x m A) and op(B) kk x n (B,
// or B^T of an n x kk B); dk (length kk, in LDS) only with DK.  A lives in
// global memory, B in global memory or LDS (BP), C anywhere; C must not
// overlap A or B.  Each wave owns 16 x (16 NT) output units (NT <= 4
// MFMA tiles side by side sharing the A operand) and streams its operands
// from L2 straight into registers, 16 rows of the inner dimension per block,
// the next block's loads in flight while the current block's MFMAs run.
// Called by all threads of the workgroup; no LDS staging and no barrier but
// the one at the end.
typedef double gemm_d4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) double *gptr;   // global
typedef const __attribute__((address_space(3))) double *lptr;   // LDS
constexpr int kWaves = kThreads / 64;

template <bool TA, bool TB, bool DK, int NT, class BP>
__device__ inline void gemm_unit(int m, int n, int kk, gptr A, int64_t lda, BP Bm, int64_t ldb, lptr dk,
                                 double *C, int64_t ldc, int r0, int c0)
{
    const int lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
    // operand layout: lane (li, lk) holds A(r0 + li, l) and B(l, c0 + 16 t + li)
    // for inner index l = l0 + 4 s + lk; indexes past the edges are clamped
    // (always in bounds) and their products masked to zero
    const int64_t ai = min(r0 + li, m - 1);
    int64_t bj[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) bj[t] = min(c0 + 16 * t + li, n - 1);
    gemm_d4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = gemm_d4{0.0, 0.0, 0.0, 0.0};
    // two register sets in turn, so no register copy separates a block's
    // loads from its MFMAs
    double a0[4], d0[4], b0[4][NT], a1[4], d1[4], b1[4][NT];
    auto load = [&](int l0, double (&an)[4], double (&dn)[4], double (&bn)[4][NT]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t l = min(l0 + 4 * s + lk, kk - 1);
            an[s] = TA ? A[l + ai * lda] : A[ai + l * lda];
            dn[s] = DK ? dk[l] : 1.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) bn[s][t] = TB ? Bm[bj[t] + l * ldb] : Bm[l + bj[t] * ldb];
        }
    };
    auto compute = [&](int l0, const double (&an)[4], const double (&dn)[4], const double (&bn)[4][NT]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool lin = l0 + 4 * s + lk < kk;
            const double av = lin ? (DK ? an[s] * dn[s] : an[s]) : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bn[s][t], acc[t], 0, 0, 0);
        }
    };
    // blocks in pairs; the prefetch is unconditional so that every path has
    // the same loads in flight (the waits then stay partial)
    load(0, a0, d0, b0);
    int l0 = 0;
    for (; l0 + 16 < kk; l0 += 32) {
        load(l0 + 16, a1, d1, b1);
        compute(l0, a0, d0, b0);
        load(l0 + 32, a0, d0, b0);
        compute(l0 + 16, a1, d1, b1);
    }
    if (l0 < kk) compute(l0, a0, d0, b0);
    // result: register r of lane (li, lk) holds row lk + 4 r, column li of the tile
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int j = c0 + 16 * t + li;
        if (j < n) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = r0 + lk + 4 * r;
                if (i < m) C[i + (int64_t)j * ldc] = acc[t][r];
            }
        }
    }
}

template <bool TA, bool TB, bool DK, class BP>
__device__ void wg_gemm(int m, int n, int kk, const double *A, int64_t lda, const double *Bm, int64_t ldb,
                        const double *dk, double *C, int64_t ldc)
{
    const gptr Ag = (gptr)A;
    const BP Bp = (BP)Bm;
    const lptr dl = (lptr)dk;
    const int wave = threadIdx.x / 64;
    const int mt = (m + 15) / 16, ng = (n + 63) / 64;
    for (int u = wave; u < mt * ng; u += kWaves) {
        const int r0 = (u % mt) * 16, c0 = (u / mt) * 64;
        switch (min(4, (n - c0 + 15) / 16)) {
        case 1: gemm_unit<TA, TB, DK, 1, BP>(m, n, kk, Ag, lda, Bp, ldb, dl, C, ldc, r0, c0); break;
        case 2: gemm_unit<TA, TB, DK, 2, BP>(m, n, kk, Ag, lda, Bp, ldb, dl, C, ldc, r0, c0); break;
        case 3: gemm_unit<TA, TB, DK, 3, BP>(m, n, kk, Ag, lda, Bp, ldb, dl, C, ldc, r0, c0); break;
        default: gemm_unit<TA, TB, DK, 4, BP>(m, n, kk, Ag, lda, Bp, ldb, dl, C, ldc, r0, c0); break;
        }
    }
    __syncthreads();
}

// Upper Cholesky factor of the k x k symmetric G (ld k, LDS) in place,
// G = R^T R, strict lower part zeroed; piv (LDS, k doubles) is scratch.
// Right-looking elimination on unscaled rows: step j subtracts
// g_ja g_jb / g_jj from g_ab (j < a <= b), which reads only row j (final
// after step j - 1), so one barrier per step; row j is scaled by
// 1 / sqrt(g_jj) at the end.  False (in every thread) on a pivot that is not a
// positive finite number.
__device__ bool wg_cholesky(double *G, int k, double *piv)
{
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    for (int j = 0; j < k; ++j) {
        const double d = G[j + j * k];
        if (!(d > 0.0) || !(d <= DBL_MAX)) {
            __syncthreads();
            return false;
        }
        const double inv = 1.0 / d;
        const int t = k - j - 1;
        for (int b0 = 0; b0 < t; b0 += 16) {
            const int b = j + 1 + b0 + ty;
            if (b < k) {
                const double gb = G[j + b * k] * inv;
                for (int a0 = 0; a0 <= b0; a0 += 16) {
                    const int a = j + 1 + a0 + tx;
                    if (a <= b) G[a + b * k] = fma(-G[j + a * k], gb, G[a + b * k]);
                }
            }
        }
        __syncthreads();
    }
    for (int a = threadIdx.x; a < k; a += kThreads) piv[a] = sqrt(G[a + a * k]);
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += kThreads) {
        const int a = e % k, b = e / k;
        G[e] = a > b ? 0.0 : (a == b ? piv[a] : G[e] / piv[a]);
    }
    __syncthreads();
    return true;
}

// X (n x k, ld n, global) <- X R^{-1} for the upper triangular k x k R (ld k,
// LDS): each thread solves y R = x for rows of X by forward substitution,
// eight columns at a time in registers.
__device__ void wg_trsm_right(double *X, int n, int k, const double *R)
{
    for (int i = threadIdx.x; i < n; i += kThreads) {
        double *x = X + i;                 // x[j n] = X(i, j)
        for (int j0 = 0; j0 < k; j0 += 8) {
            double acc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] = j0 + u < k ? x[(int64_t)(j0 + u) * n] : 0.0;
#pragma unroll 8
            for (int l = 0; l < j0; ++l) {          // j0 is a multiple of 8
                const double y = x[(int64_t)l * n];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (j0 + u < k) acc[u] = fma(-y, R[l + (j0 + u) * k], acc[u]);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (j0 + u < k) {
                    const double y = acc[u] / R[(j0 + u) * (k + 1)];
#pragma unroll
                    for (int v = u + 1; v < 8; ++v)
                        if (j0 + v < k) acc[v] = fma(-y, R[(j0 + u) + (j0 + v) * k], acc[v]);
                    x[(int64_t)(j0 + u) * n] = y;
                }
            }
        }
    }
    __syncthreads();
}

// Column norms of X (n x k, ld n, global memory) into d[0..k).
__device__ void col_norms_global(const double *X, int n, int k, double *d)
{
    const int grp = threadIdx.x / kG, gl = threadIdx.x % kG;
    for (int c0 = 0; c0 < k; c0 += kGroups) {
        const int c = c0 + grp;
        double s = 0.0;
        if (c < k)
            for (int e = gl; e < n; e += kG) s = fma(X[(int64_t)c * n + e], X[(int64_t)c * n + e], s);
        s = group_sum(s);
        if (c < k && gl == 0) d[c] = sqrt(s);
    }
    __syncthreads();
}

struct Lds {
    double *B1, *B2, *B3;      // kKMax^2 each
    double *sig, *w, *dn, *piv;   // kKMax each
    double *red;               // 4
    int *flag;
};

// Orthonormalise the k columns of X (n x k, ld n) in place: columns scaled
// to unit norm (a zero or non-finite column is replaced by a start vector),
// then Cholesky QR twice (X <- X R^{-1} by forward substitution).  With
// want_r, B2 receives R (k x k, ld k, upper) with X_in = Q R.  Uses B1, B2,
// B3.
__device__ void wg_orth(double *X, int n, int k, bool want_r, const Lds &s,
                        uint64_t salt)
{
    col_norms_global(X, n, k, s.dn);
    // replace degenerate columns (rare: W without that many directions)
    for (int c = 0; c < k; ++c) {
        const double d = s.dn[c];
        if (!(d > 1e-300) || !(d <= DBL_MAX)) {
            for (int e = threadIdx.x; e < n; e += kThreads) X[(int64_t)c * n + e] = hash_unit(salt + c, e);
            __syncthreads();
            double a = 0.0;
            for (int e = threadIdx.x; e < n; e += kThreads) a = fma(X[(int64_t)c * n + e], X[(int64_t)c * n + e], a);
            a = block_sum(a, s.red);
            if (threadIdx.x == 0) s.dn[c] = 0.0;       // contributes nothing to R
            for (int e = threadIdx.x; e < n; e += kThreads) X[(int64_t)c * n + e] /= sqrt(a);
            __syncthreads();
        } else {
            for (int e = threadIdx.x; e < n; e += kThreads) X[(int64_t)c * n + e] /= d;
        }
    }
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        wg_gemm<true, false, false, gptr>(k, k, n, X, n, X, n, nullptr, s.B1, k);
        if (!wg_cholesky(s.B1, k, s.piv)) {
            // Gram matrix singular to rounding: shift its diagonal (shifted
            // Cholesky QR) and factor again; the second pass cleans up
            wg_gemm<true, false, false, gptr>(k, k, n, X, n, X, n, nullptr, s.B1, k);
            for (int c = threadIdx.x; c < k; c += kThreads) s.B1[c + c * k] += 1e-13 * (double)n;
            __syncthreads();
            if (!wg_cholesky(s.B1, k, s.piv)) {
                for (int e = threadIdx.x; e < k * k; e += kThreads) s.B1[e] = (e % k == e / k) ? 1.0 : 0.0;
                __syncthreads();
            }
        }
        wg_trsm_right(X, n, k, s.B1);
        if (want_r && pass == 0)           // B3 = R1 D
            for (int e = threadIdx.x; e < k * k; e += kThreads) s.B3[e] = s.B1[e] * s.dn[e / k];
        __syncthreads();
    }
    if (want_r) {                          // B2 = R2 (B1) x R1 D (B3), both upper
        for (int e = threadIdx.x; e < k * k; e += kThreads) {
            const int i = e % k, j = e / k;
            double a = 0.0;
            for (int l = i; l <= j; ++l) a = fma(s.B1[i + l * k], s.B3[l + j * k], a);
            s.B2[e] = i <= j ? a : 0.0;
        }
    }
    __syncthreads();
}

// One Rayleigh-Ritz step on the subspace V (q x k): B = W V -> Q (in Qb), R;
// SVD of R -> sigma (s.sig), U = Q Ut (Ub), V <- V Vt (Vb, swapped with Vt).
__device__ void ritz_step(const double *W, int p, int q, int k, double *&Vb, double *&Vt, double *Qb,
                          double *Ub, const Lds &s, uint64_t salt)
{
    wg_gemm<false, false, false, gptr>(p, k, q, W, p, Vb, q, nullptr, Qb, p);
    wg_orth(Qb, p, k, true, s, salt);
    // SVD of R (B2): one-sided Jacobi on its columns, right rotations in B1
    jacobi_svd(s.B2, s.B1, k, k, s.flag, true);
    column_norms(s.B2, k, k, s.sig);
    for (int e = threadIdx.x; e < k * k; e += kThreads) {
        const double sg = s.sig[e / k];
        s.B2[e] = sg > 0.0 ? s.B2[e] / sg : 0.0;            // Ut
    }
    __syncthreads();
    wg_gemm<false, false, false, lptr>(p, k, k, Qb, p, s.B2, k, nullptr, Ub, p);
    wg_gemm<false, false, false, lptr>(q, k, k, Vb, q, s.B1, k, nullptr, Vt, q);
    double *tmp = Vb;
    Vb = Vt;
    Vt = tmp;
}

// One power step: V <- orth(W^T U) with U the left Ritz vectors of the last
// Ritz step.  U = Q Ut spans the same subspace as Q, so the iteration is the
// same; but once the Ritz vectors settle, W^T U is V Sigma up to a small
// remainder, the next step's R is nearly diagonal and its Jacobi SVD takes
// two or three sweeps instead of starting from a full rotation.
__device__ void power_step(const double *W, int p, int q, int k, double *&Vb, double *&Vt,
                           const double *Ub, const Lds &s, uint64_t salt)
{
    wg_gemm<true, false, false, gptr>(q, k, p, W, p, Ub, p, nullptr, Vt, q);
    double *tmp = Vb;
    Vb = Vt;
    Vt = tmp;
    wg_orth(Vb, q, k, false, s, salt);
}

__global__ void __launch_bounds__(kThreads)
seed_large_kernel(const LargeSeedJob *__restrict__ jobs, LargeSeedConsts C)
{
    extern __shared__ double lds[];
    __shared__ double red[4];
    __shared__ int flag;
    const LargeSeedJob &J = jobs[blockIdx.x];
    const int p = J.p, q = J.q, tid = threadIdx.x;
    const int64_t pq = (int64_t)p * q;
    const int kmax = J.kmax;
    Lds s;
    s.B1 = lds;
    s.B2 = s.B1 + kKMax * kKMax;
    s.B3 = s.B2 + kKMax * kKMax;
    s.sig = s.B3 + kKMax * kKMax;
    s.w = s.sig + kKMax;
    s.dn = s.w + kKMax;
    s.piv = s.dn + kKMax;
    s.red = red;
    s.flag = &flag;
    double *Ms = J.ws, *S = Ms + pq, *Y = S + pq, *W = Y + pq, *L = W + pq, *Lp = L + pq;
    double *Vb = Lp + pq, *Vt = Vb + (int64_t)q * kKMax, *Qb = Vt + (int64_t)q * kKMax;
    double *Ub = Qb + (int64_t)p * kKMax;
    // start vectors keyed by the block's shape only, never by its place in
    // the launch: a block gives the same result alone or in any batch
    const uint64_t salt = 0x5EEDull + ((uint64_t)p << 32) + (uint64_t)q;

    // ---- gather M^s (FP64), its norms, non-finite entries
    double ss = 0.0, mx = 0.0, bad = 0.0;
    for (int64_t t = tid; t < pq; t += kThreads) {
        const int64_t a = t % p, b = t / p;
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
            for (int i = 1; i < 8; ++i) J.result[i] = 0;
        }
        return;
    }

    // ---- ||M^s||_2 by the same iteration on Ms
    int k = kGuard < kmax ? kGuard : kmax;
    for (int64_t e = tid; e < (int64_t)q * k; e += kThreads) Vb[e] = hash_unit(salt, (uint64_t)e);
    __syncthreads();
    wg_orth(Vb, q, k, false, s, salt + 17);
    double norm2 = 0.0;
    int ritz = 0;
    for (int it = 0; it < kNormCap; ++it) {
        ritz_step(Ms, p, q, k, Vb, Vt, Qb, Ub, s, salt + 31 * it);
        double smax = 0.0;
        for (int c = 0; c < k; ++c) smax = fmax(smax, s.sig[c]);
        const bool done = it > 0 && fabs(smax - norm2) <= 1e-15 * smax;
        norm2 = smax;
        ++ritz;
        if (done || k == (p < q ? p : q)) break;
        power_step(Ms, p, q, k, Vb, Vt, Ub, s, salt + 37 * it);
    }

    const double lam = C.lam > 0.0 ? C.lam : 1.0 / sqrt((double)(p > q ? p : q));
    const double y0 = 1.0 / fmax(norm2, mx / lam);
    for (int64_t t = tid; t < pq; t += kThreads) {
        Y[t] = Ms[t] * y0;
        S[t] = 0.0;
    }
    double mu = C.mu0_scale / norm2;
    const double mu_bar = C.mu_max_scale * mu;
    double mu_used = mu, res = 1.0;
    bool converged = false, fallback = false;
    int kiter;
    int kept = 0;
    bool ritz_basis = false;   // Vb holds the Ritz vectors of s.sig (the last inner step was a Ritz step)
    __syncthreads();
    for (kiter = 1; kiter <= C.max_iter; ++kiter) {
        if (ritz_basis) {
            // narrow the basis to the previous step's kept directions plus a
            // guard band (the iterate's rank rises and falls: a basis widened
            // for a transient would otherwise keep every later step wide)
            const int knext = std::min(k, std::max(std::min(kGuard, kmax), std::min(kmax, kept + kGuard)));
            if (knext < k) {
                int *ord = reinterpret_cast<int *>(s.dn);
                for (int c = tid; c < k; c += kThreads) {
                    int pos = 0;
                    for (int d = 0; d < k; ++d)
                        pos += (s.sig[d] > s.sig[c]) || (s.sig[d] == s.sig[c] && d < c);
                    ord[pos] = c;
                }
                __syncthreads();
                for (int64_t e = tid; e < (int64_t)q * knext; e += kThreads)
                    Vt[e] = Vb[(int64_t)ord[e / q] * q + e % q];
                __syncthreads();
                double *tmp = Vb;
                Vb = Vt;
                Vt = tmp;
                k = knext;
            }
        }
        const double inv_mu = 1.0 / mu, tau = inv_mu;
        for (int64_t t = tid; t < pq; t += kThreads) W[t] = Ms[t] - S[t] + Y[t] * inv_mu;
        __syncthreads();
        const double tol_in = fmin(1e-6, fmax(1e-13, 1e-3 * res));
        bool have_prev = false;
        for (int it = 0; it < kInnerCap; ++it) {
            ritz_step(W, p, q, k, Vb, Vt, Qb, Ub, s, salt + 131 * it);
            ++ritz;
            kept = 0;
            for (int c = 0; c < k; ++c) kept += s.sig[c] > tau;
            if (kept > k - kGuard / 2 && k < (p < q ? p : q)) {
                if (k >= kmax) {               // the subspace cannot widen: give up
                    fallback = true;
                    break;
                }
                const int k2 = k + kGuard < kmax ? k + kGuard : kmax;
                for (int64_t e = (int64_t)q * k + tid; e < (int64_t)q * k2; e += kThreads)
                    Vb[e] = hash_unit(salt + 7 * kiter, (uint64_t)e);
                __syncthreads();
                k = k2;
                wg_orth(Vb, q, k, false, s, salt + 11 * kiter);
                have_prev = false;
                ritz_basis = false;
                --it;                          // a widening (at most kKMax / kGuard of them) is not a step
                continue;
            }
            // L = U diag(w) V^T with w = sigma - tau above tau, else 0
            for (int c = tid; c < k; c += kThreads) s.w[c] = s.sig[c] > tau ? s.sig[c] - tau : 0.0;
            __syncthreads();
            double *Lnew = have_prev ? Lp : L;          // the buffer not holding the last L
            const double *Lold = have_prev ? L : Lp;
            wg_gemm<false, true, true, gptr>(p, q, k, Ub, p, Vb, q, s.w, Lnew, p);
            double dd = 0.0, nn = 0.0;
            for (int64_t t = tid; t < pq; t += kThreads) {
                const double a = Lnew[t];
                nn = fma(a, a, nn);
                if (have_prev) dd = fma(a - Lold[t], a - Lold[t], dd);
            }
            dd = block_sum(dd, red);
            nn = block_sum(nn, red);
            if (have_prev) {                   // keep the newest product in L
                double *tmp = L;
                L = Lp;
                Lp = tmp;
            }
            const bool stable = have_prev && sqrt(dd) <= tol_in * sqrt(nn);
            have_prev = true;
            ritz_basis = true;
            if (stable || it + 1 >= kInnerCap || k == (p < q ? p : q)) break;
            ritz_basis = false;
            power_step(W, p, q, k, Vb, Vt, Ub, s, salt + 137 * it);
        }
        if (fallback) break;
        // S = shrink(Ms - L + Y / mu, lam / mu), Z = Ms - L - S, Y += mu Z
        const double thr = lam / mu;
        double zz = 0.0;
        for (int64_t t = tid; t < pq; t += kThreads) {
            const double l = L[t];
            const double T = Ms[t] - l + Y[t] * inv_mu;
            const double sv = T > thr ? T - thr : (T < -thr ? T + thr : 0.0);
            const double z = Ms[t] - l - sv;
            S[t] = sv;
            Y[t] += mu * z;
            zz = fma(z, z, zz);
        }
        zz = block_sum(zz, red);
        mu_used = mu;
        mu = fmin(C.rho * mu, mu_bar);
        res = sqrt(zz) / normF;
        if (res < C.tol) {
            converged = true;
            break;
        }
    }
    if (kiter > C.max_iter) kiter = C.max_iter;
    if (fallback) {
        if (tid == 0) {
            J.result[0] = RPCA_ERR_UNSUPPORTED;
            for (int i = 1; i < 6; ++i) J.result[i] = 0;
            J.result[5] = ritz;
            J.result[6] = kFallback;
        }
        return;
    }

    // ---- order of the last step's singular values (descending; ties by index), rank
    int *ord = reinterpret_cast<int *>(s.dn);            // k ints fit in kKMax doubles
    for (int c = tid; c < k; c += kThreads) {
        int pos = 0;
        for (int d = 0; d < k; ++d) pos += (s.sig[d] > s.sig[c]) || (s.sig[d] == s.sig[c] && d < c);
        ord[pos] = c;
    }
    __syncthreads();
    const double tau = 1.0 / mu_used;
    int svp = 0;
    while (svp < k && s.sig[ord[svp]] > tau) ++svp;
    int rank = 0;
    if (svp > 0) {
        const double top = s.sig[ord[0]] - tau;
        while (rank < svp && (s.sig[ord[rank]] - tau) > C.rank_floor * top) ++rank;
    }
    const int r = J.r;
    const int keep = rank < r ? rank : r;
    for (int64_t t = tid; t < (int64_t)p * r; t += kThreads) {
        const int64_t a = t % p, c = t / p;
        J.U[t] = c < keep ? Ub[(int64_t)ord[c] * p + a] : 0.0;
    }
    for (int64_t t = tid; t < (int64_t)q * r; t += kThreads) {
        const int64_t b = t % q, c = t / q;
        J.V[t] = c < keep ? Vb[(int64_t)ord[c] * q + b] : 0.0;
    }
    for (int c = tid; c < r; c += kThreads) J.sigma[c] = c < keep ? s.sig[ord[c]] - tau : 0.0;
    if (tid == 0) {
        J.result[0] = rank == 0 ? RPCA_ERR_SEED
                                : (rank != r ? RPCA_WARN_RANK : (converged ? RPCA_OK : RPCA_WARN_NOT_CONVERGED));
        J.result[1] = keep;
        J.result[2] = kiter;
        J.result[3] = converged ? 1 : 0;
        J.result[4] = rank;
        J.result[5] = ritz;
        J.result[6] = 0;
    }
}

size_t lds_bytes()
{
    return (3 * (size_t)kKMax * kKMax + 4 * (size_t)kKMax) * sizeof(double);
}

} // namespace seedl

bool seed_large_fits(rpca_ctx *ctx, int64_t p, int64_t q)
{
    // above 512 rows or columns the single workgroup's products take longer
    // than the device-wide eigen-solver route
    if (p < 1 || q < 1 || p > 512 || q > 512) return false;
    const size_t limit = ctx->max_lds ? ctx->max_lds : 65536;
    return seedl::lds_bytes() + 1024 <= limit;
}

size_t seed_large_workspace(const SmallSeedArgs *args, int n)
{
    size_t d = 0;
    for (int k = 0; k < n; ++k) d += (size_t)seedl::ws_doubles((int)args[k].p, (int)args[k].q);
    const size_t table = (d * sizeof(double) + 255) / 256 * 256;
    const size_t results = (table + (size_t)n * sizeof(seedl::LargeSeedJob) + 255) / 256 * 256;
    return (results + (size_t)n * 8 * sizeof(int32_t) + 255) / 256 * 256;
}

int run_seed_large(rpca_ctx *ctx, const SmallSeedArgs *args, int n, const rpca_opts &o, void *ws,
                   SeedOut *outs, int *statuses, hipStream_t stream)
{
    if (n <= 0) return RPCA_OK;
    using namespace seedl;
    size_t d = 0;
    for (int k = 0; k < n; ++k) d += (size_t)ws_doubles((int)args[k].p, (int)args[k].q);
    const size_t o_table = (d * sizeof(double) + 255) / 256 * 256;
    const size_t o_res = (o_table + (size_t)n * sizeof(LargeSeedJob) + 255) / 256 * 256;
    char *base = static_cast<char *>(ws);
    double *mats = reinterpret_cast<double *>(base);
    LargeSeedJob *dj = reinterpret_cast<LargeSeedJob *>(base + o_table);
    int32_t *results = reinterpret_cast<int32_t *>(base + o_res);
    std::vector<LargeSeedJob> hj((size_t)n);
    size_t off = 0;
    for (int k = 0; k < n; ++k) {
        const SmallSeedArgs &a = args[k];
        if (!seed_large_fits(ctx, a.p, a.q))
            return set_status(ctx, RPCA_ERR_UNSUPPORTED, "seed: block outside the device-resident seed solver");
        const int kmax = (int)std::min<int64_t>(kKMax, std::min(a.p, a.q));
        hj[k] = LargeSeedJob{a.M, a.ldm, a.rows, a.cols, (int32_t)a.p, (int32_t)a.q, a.r, kmax,
                             a.U, a.sigma, a.V, mats + off, results + 8 * k};
        off += (size_t)ws_doubles((int)a.p, (int)a.q);
    }
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(dj, hj.data(), hj.size() * sizeof(LargeSeedJob),
                                     hipMemcpyHostToDevice, stream));
    LargeSeedConsts c{o.seed_lambda, o.seed_tol, o.seed_rho, o.seed_mu0_scale, o.seed_mu_max_scale,
                      o.seed_rank_floor, o.seed_max_iter};
    const size_t lds = lds_bytes();
    RPCA_HIP_TRY(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(seed_large_kernel),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(seed_large_kernel, dim3((unsigned)n), dim3(kThreads), lds, stream, dj, c);
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
        outs[k].ritz_steps = hr[8 * k + 5];
        outs[k].fallback = hr[8 * k + 6];
        outs[k].route = outs[k].fallback ? RPCA_SEED_ROUTE_FELL_BACK : RPCA_SEED_ROUTE_SUBSPACE;
    }
    return RPCA_OK;
}
