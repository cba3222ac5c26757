// Device code of the completion (Algorithm 2, step 5 and output), shared by
// the single-problem launch (reconstruct.hip) and the batched launch
// (batch.hip).
//
// The four blocks of L (eqs. partition, row-column-recovery, l1s, l1s')
//   L[I_s,J_s] = U Sigma V^T,  L[I_s,J_c] = U Q~,
//   L[I_c,J_s] = P~^T V^T,     L[I_c,J_c] = P~^T Sigma^{-1} Q~
// are one rank-r product L = F G^T over the whole matrix once the row factor
// F (m x r) and column factor G (n x r) are assembled as
//   F[I_s] = U Sigma,  F[I_c] = P~^T,   G[J_s] = V,  G[J_c] = Q~^T Sigma^{-1}.
// (The pseudo-inverse of L^s = U Sigma V^T is V Sigma^{-1} U^T, so the
// Nystrom block needs only r FP64 reciprocals.)  The product is HBM bound
// (12 bytes per element: read M, write L and S, for 2r flops), so one pass
// streams M with non-temporal loads, keeps the row factor of 4 rows per lane
// in VGPRs and the column factor in scalar registers (uniform across the
// wave), and writes L and S with non-temporal stores.
#pragma once

#include "rpca_internal.h"

namespace reconk {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Index of the first element >= key in the sorted array a[0..n).
__device__ __forceinline__ int64_t lower_bound_i64(const int64_t *a, int64_t n, int64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

constexpr int kAssembleThreads = 256;
constexpr int kIdxLds = 4096;

// One workgroup of the factor assembly.  F: m x R4 row-major, G: n x R4
// row-major, zero-padded to R4 >= r.  Threads [0, m) of the problem build
// rows of F, threads [m, m + n) rows of G; `first` is the problem's thread
// index of this workgroup's thread 0; threads at or beyond `end` only take
// part in the barrier.  The sorted seed indices are staged in LDS (when they
// fit) for the binary searches.  Contains a workgroup barrier: every thread
// of the workgroup must call it.
__device__ __forceinline__ void assemble_block(int64_t first, int64_t end, int64_t *sidx,
                                               const int64_t *__restrict__ seed_rows, int64_t p,
                                               const int64_t *__restrict__ seed_cols, int64_t q,
                                               const double *__restrict__ U,
                                               const double *__restrict__ sigma,
                                               const double *__restrict__ V, int r,
                                               const float *__restrict__ Qt,
                                               const float *__restrict__ Pt, int64_t m, int64_t n,
                                               int R4, float *__restrict__ F, float *__restrict__ G)
{
    // a block lies entirely in the F part, entirely in the G part, or straddles
    const bool need_rows = first < m;
    const bool need_cols = first + blockDim.x > m;
    const bool rows_in_lds = need_rows && !need_cols && p <= kIdxLds;
    const bool cols_in_lds = need_cols && !need_rows && q <= kIdxLds;
    if (rows_in_lds)
        for (int64_t a = threadIdx.x; a < p; a += blockDim.x) sidx[a] = seed_rows[a];
    if (cols_in_lds)
        for (int64_t a = threadIdx.x; a < q; a += blockDim.x) sidx[a] = seed_cols[a];
    __syncthreads();

    const int64_t t = first + threadIdx.x;
    if (t >= end) return;                 // after the barrier: nothing below waits
    if (t < m) {
        const int64_t i = t;
        const int64_t *idx = rows_in_lds ? sidx : seed_rows;
        const int64_t a = lower_bound_i64(idx, p, i);
        float *f = F + i * R4;
        if (a < p && idx[a] == i) {
            for (int k = 0; k < R4; ++k) f[k] = k < r ? (float)(U[a + (int64_t)k * p] * sigma[k]) : 0.0f;
        } else {
            const int64_t b = i - a;   // position of i in the sorted complement
            const bool ok = b >= 0 && b < m - p;
            for (int k = 0; k < R4; ++k) f[k] = (ok && k < r) ? Pt[k + b * r] : 0.0f;
        }
    } else if (t < m + n) {
        const int64_t jj = t - m;
        const int64_t *idx = cols_in_lds ? sidx : seed_cols;
        const int64_t a = lower_bound_i64(idx, q, jj);
        float *gp = G + jj * R4;
        if (a < q && idx[a] == jj) {
            for (int k = 0; k < R4; ++k) gp[k] = k < r ? (float)V[a + (int64_t)k * q] : 0.0f;
        } else {
            const int64_t b = jj - a;
            const bool ok = b >= 0 && b < n - q;
            for (int k = 0; k < R4; ++k)
                gp[k] = (ok && k < r) ? (float)((double)Qt[k + b * r] / sigma[k]) : 0.0f;
        }
    }
}

constexpr int kRowsPerLane = 4;
constexpr int kRowsPerWave = 64 * kRowsPerLane;
constexpr int kColBatch = 4;    // columns whose loads are in flight together

// One wave of the completion: rows [256 bx, 256 bx + 256) and the column
// range [n by / gy, n (by + 1) / gy), so the gy waves sharing a row block
// stream the same number of bytes.  VEC (16-byte aligned columns): lane l
// owns rows 4l .. 4l+3 of the block and moves float4s; otherwise lane l owns
// rows l, l+64, l+128, l+192, so each load and store instruction of the wave
// is one contiguous 256-byte run whatever the alignment of the column.
template <int R4, bool VEC>
__device__ __forceinline__ void recon_wave(const float *__restrict__ M, int64_t ldm,
                                           const float *__restrict__ F,
                                           const float *__restrict__ G, int64_t m, int64_t n,
                                           float *__restrict__ Lo, int64_t ldl,
                                           float *__restrict__ So, int64_t lds, uint32_t bx,
                                           uint32_t by, uint32_t gy, int lane)
{
    const int64_t blk = (int64_t)bx * kRowsPerWave;
    const int64_t j0 = n * (int64_t)by / gy;
    const int64_t jend = n * ((int64_t)by + 1) / gy;
    // row of register rr of this lane
    auto row = [&](int rr) -> int64_t {
        return VEC ? blk + lane * kRowsPerLane + rr : blk + lane + 64 * rr;
    };

    float f[kRowsPerLane][R4];
#pragma unroll
    for (int rr = 0; rr < kRowsPerLane; ++rr) {
        const int64_t i = row(rr);
#pragma unroll
        for (int k = 0; k < R4; k += 4) {
            floatx4 v = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            if (i < m) v = *reinterpret_cast<const floatx4 *>(F + i * R4 + k);
            f[rr][k] = v[0];
            f[rr][k + 1] = v[1];
            f[rr][k + 2] = v[2];
            f[rr][k + 3] = v[3];
        }
    }
    const bool full_rows = blk + kRowsPerWave <= m;
    int64_t j = j0;
    if (full_rows) {
        // batches of kColBatch columns, loads issued first
#pragma unroll 1
        for (; j + kColBatch <= jend; j += kColBatch) {
            floatx4 mv[kColBatch];
#pragma unroll
            for (int cb = 0; cb < kColBatch; ++cb) {
                if constexpr (VEC) {
                    mv[cb] = __builtin_nontemporal_load(
                        reinterpret_cast<const floatx4 *>(M + (j + cb) * ldm + row(0)));
                } else {
#pragma unroll
                    for (int rr = 0; rr < kRowsPerLane; ++rr)
                        mv[cb][rr] = __builtin_nontemporal_load(M + (j + cb) * ldm + row(rr));
                }
            }
#pragma unroll
            for (int cb = 0; cb < kColBatch; ++cb) {
                const float *gj = G + (j + cb) * R4;     // uniform across the wave
                floatx4 lv = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int k = 0; k < R4; ++k) {
                    const float gk = gj[k];
#pragma unroll
                    for (int rr = 0; rr < kRowsPerLane; ++rr) lv[rr] = fmaf(f[rr][k], gk, lv[rr]);
                }
                const floatx4 sv = mv[cb] - lv;
                if constexpr (VEC) {
                    __builtin_nontemporal_store(lv, reinterpret_cast<floatx4 *>(Lo + (j + cb) * ldl + row(0)));
                    __builtin_nontemporal_store(sv, reinterpret_cast<floatx4 *>(So + (j + cb) * lds + row(0)));
                } else {
#pragma unroll
                    for (int rr = 0; rr < kRowsPerLane; ++rr) {
                        __builtin_nontemporal_store(lv[rr], Lo + (j + cb) * ldl + row(rr));
                        __builtin_nontemporal_store(sv[rr], So + (j + cb) * lds + row(rr));
                    }
                }
            }
        }
    }
    for (; j < jend; ++j) {
        const float *gj = G + j * R4;     // uniform across the wave
        float acc[kRowsPerLane] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < R4; ++k) {
            const float gk = gj[k];
#pragma unroll
            for (int rr = 0; rr < kRowsPerLane; ++rr) acc[rr] = fmaf(f[rr][k], gk, acc[rr]);
        }
        if (VEC && full_rows) {
            const floatx4 mv = __builtin_nontemporal_load(
                reinterpret_cast<const floatx4 *>(M + j * ldm + row(0)));
            const floatx4 lv = floatx4{acc[0], acc[1], acc[2], acc[3]};
            __builtin_nontemporal_store(lv, reinterpret_cast<floatx4 *>(Lo + j * ldl + row(0)));
            __builtin_nontemporal_store(mv - lv, reinterpret_cast<floatx4 *>(So + j * lds + row(0)));
        } else {
#pragma unroll
            for (int rr = 0; rr < kRowsPerLane; ++rr) {
                const int64_t i = row(rr);
                if (i < m) {
                    const float mv = M[j * ldm + i];
                    Lo[j * ldl + i] = acc[rr];
                    So[j * lds + i] = mv - acc[rr];
                }
            }
        }
    }
}

} // namespace reconk
