// One-sided Jacobi SVD (Hestenes' method) of a matrix held in LDS, and the
// workgroup reductions around it, shared by the FP64 seed solvers
// (seed_small.hip: the whole SVT; seed_large.hip: the SVD of the small
// triangular factor of its Rayleigh-Ritz step).  Every function is called by
// all kThreads threads of a workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace seedj {

constexpr int kThreads = 256;
constexpr int kG = 8;                       // lanes per column (column norms)
constexpr int kGroups = kThreads / kG;      // columns in flight (column norms)
constexpr int kMaxSweeps = 40;
constexpr double kJacobiEps = 1e-15;        // orthogonality threshold of a column pair
constexpr int kColdEvery = 64;              // ALM steps between Jacobi starts from the identity

// Sum over aligned groups of g = 4 or 8 lanes (g uniform over the workgroup).
__device__ __forceinline__ double group_sum_n(double v, int g)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    if (g == 8) v += __shfl_xor(v, 4);
    return v;
}

// Sum over the kG lanes of a column group.
__device__ __forceinline__ double group_sum(double v) { return group_sum_n(v, kG); }

// Sum / max over the workgroup (every thread gets the result).
__device__ inline double block_sum(double v, double *red)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__device__ inline double block_max(double v, double *red)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Pair pr of round k of a round-robin tournament on m2 (even) players.
__device__ __forceinline__ void tournament_pair(int k, int pr, int m2, int &i, int &j)
{
    const int n = m2 - 1;
    int a, b;
    if (pr == 0) {
        a = n;
        b = k % n;
    } else {
        a = (k + pr) % n;
        b = (k - pr + n) % n;
    }
    i = a < b ? a : b;
    j = a < b ? b : a;
}

// One-sided Jacobi on the columns of X (n1 x n2, column-major in LDS) with
// the rotations accumulated into V (n2 x n2): set to the identity first when
// `cold`, else X already holds W V for the V of a previous step (warm start:
// its columns are nearly orthogonal, so few sweeps are needed).
//
// G lanes per pair (4 or 8).  With `absolute`, a pair counts as orthogonal
// once its inner product is below eps ||X||_F times its larger norm: rotating
// it could then move a singular value by no more than about eps ||X||_F, the
// absolute accuracy of a backward-stable SVD, which is all an SVT needs.
// Otherwise the test is against the pair's own norms (eps ||x_i|| ||x_j||:
// high relative accuracy for the small singular values too, at the price of
// more sweeps where the matrix has many small columns).
__device__ inline void jacobi_svd(double *X, double *V, int n1, int n2, int *flag, bool cold,
                                  int G = 8, bool absolute = false)
{
    const int tid = threadIdx.x;
    if (cold)
        for (int t = tid; t < n2 * n2; t += kThreads) V[t] = (t % n2 == t / n2) ? 1.0 : 0.0;
    const int m2 = n2 + (n2 & 1);
    const int npairs = m2 / 2;
    const int groups = kThreads / G;
    // 16-byte accesses where every column starts 16-byte aligned (X and V
    // aligned, even n1 and n2); with 4 lanes per pair only, which keeps the
    // 8-lane callers' code and results as they were
    const bool pairs2 = G == 4 && (n1 & 1) == 0 && (n2 & 1) == 0 &&
                        ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(V)) & 15) == 0;
    const int grp = tid / G, gl = tid % G;
    // ||X||_F, which the rotations keep (absolute test only)
    double fro2 = 0.0;
    if (absolute) {
        __shared__ double fro_red[4];
        double f2 = 0.0;
        for (int t = tid; t < n1 * n2; t += kThreads) f2 = fma(X[t], X[t], f2);
        fro2 = block_sum(f2, fro_red);
    }
    __syncthreads();
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        if (tid == 0) *flag = 0;
        __syncthreads();
        for (int round = 0; round < m2 - 1; ++round) {
            for (int base = 0; base < npairs; base += groups) {
                const int pr = base + grp;
                int i = 0, j = 0;
                if (pr < npairs) tournament_pair(round, pr, m2, i, j);
                const bool live = pr < npairs && j < n2;     // same for the G lanes of a group
                if (live) {
                    double al = 0.0, be = 0.0, ga = 0.0;
                    const double *xi = X + (int64_t)i * n1, *xj = X + (int64_t)j * n1;
                    if (pairs2) {
                        // two adjacent elements per lane and load (16-byte LDS accesses)
#pragma unroll 2
                        for (int e = 2 * gl; e < n1; e += 2 * G) {
                            const double2 a = *reinterpret_cast<const double2 *>(xi + e);
                            const double2 b = *reinterpret_cast<const double2 *>(xj + e);
                            al = fma(a.x, a.x, al);
                            be = fma(b.x, b.x, be);
                            ga = fma(a.x, b.x, ga);
                            al = fma(a.y, a.y, al);
                            be = fma(b.y, b.y, be);
                            ga = fma(a.y, b.y, ga);
                        }
                    } else {
#pragma unroll 4
                        for (int e = gl; e < n1; e += G) {
                            const double a = xi[e], b = xj[e];
                            al = fma(a, a, al);
                            be = fma(b, b, be);
                            ga = fma(a, b, ga);
                        }
                    }
                    al = group_sum_n(al, G);
                    be = group_sum_n(be, G);
                    ga = group_sum_n(ga, G);
                    if (ga * ga > (kJacobiEps * kJacobiEps) * (absolute ? fro2 * fmax(al, be) : al * be)) {
                        // t = tan of the rotation: the root of smaller modulus of
                        // t^2 + 2 zeta t - 1 = 0, zeta = (be - al) / (2 ga), written
                        // with one division: sign(zeta) |2 ga| / (|d| + sqrt(d^2 + 4 ga^2))
                        const double d = be - al, g2 = 2.0 * ga;
                        const double sg = (d == 0.0 || ((d > 0.0) == (ga > 0.0))) ? 1.0 : -1.0;
                        const double t = sg * fabs(g2) / (fabs(d) + sqrt(fma(d, d, g2 * g2)));
                        const double c = 1.0 / sqrt(fma(t, t, 1.0)), s = c * t;
                        double *wi = X + (int64_t)i * n1, *wj = X + (int64_t)j * n1;
                        double *vi = V + (int64_t)i * n2, *vj = V + (int64_t)j * n2;
                        if (pairs2) {
#pragma unroll 2
                            for (int e = 2 * gl; e < n1; e += 2 * G) {
                                const double2 a = *reinterpret_cast<const double2 *>(wi + e);
                                const double2 b = *reinterpret_cast<const double2 *>(wj + e);
                                *reinterpret_cast<double2 *>(wi + e) = double2{c * a.x - s * b.x, c * a.y - s * b.y};
                                *reinterpret_cast<double2 *>(wj + e) = double2{s * a.x + c * b.x, s * a.y + c * b.y};
                            }
#pragma unroll 2
                            for (int e = 2 * gl; e < n2; e += 2 * G) {
                                const double2 a = *reinterpret_cast<const double2 *>(vi + e);
                                const double2 b = *reinterpret_cast<const double2 *>(vj + e);
                                *reinterpret_cast<double2 *>(vi + e) = double2{c * a.x - s * b.x, c * a.y - s * b.y};
                                *reinterpret_cast<double2 *>(vj + e) = double2{s * a.x + c * b.x, s * a.y + c * b.y};
                            }
                        } else {
#pragma unroll 4
                            for (int e = gl; e < n1; e += G) {
                                const double a = wi[e], b = wj[e];
                                wi[e] = c * a - s * b;
                                wj[e] = s * a + c * b;
                            }
#pragma unroll 4
                            for (int e = gl; e < n2; e += G) {
                                const double a = vi[e], b = vj[e];
                                vi[e] = c * a - s * b;
                                vj[e] = s * a + c * b;
                            }
                        }
                        if (gl == 0) *flag = 1;
                    }
                }
            }
            __syncthreads();      // the next round pairs columns of this one
        }
        if (*flag == 0) break;
        __syncthreads();
    }
    __syncthreads();
}

// Column norms of X into sig[0..n2).
__device__ inline void column_norms(const double *X, int n1, int n2, double *sig)
{
    const int grp = threadIdx.x / kG, gl = threadIdx.x % kG;
    for (int c0 = 0; c0 < n2; c0 += kGroups) {
        const int c = c0 + grp;
        double s = 0.0;
        if (c < n2)
            for (int e = gl; e < n1; e += kG) s = fma(X[(int64_t)c * n1 + e], X[(int64_t)c * n1 + e], s);
        s = group_sum(s);
        if (c < n2 && gl == 0) sig[c] = sqrt(s);
    }
    __syncthreads();
}

} // namespace seedj
