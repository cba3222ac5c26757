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
// streams M, keeps the row factor of 4 rows per lane in VGPRs and the column
// factor in scalar registers (uniform across the wave), and writes L and S
// with non-temporal stores (ordinary stores measured 8-12% slower on MI355X).
// M is read with non-temporal loads, or with ordinary ones up to rank 8
// (the batched form's ranks: completion 16.2 -> 15.6 ms over its 256
// problems; at rank 50 ordinary loads cost 25%, 6.1 -> 7.6 ms, and at rank
// 20 they made no difference in the whole step).
#pragma once

#include "rpca_internal.h"

#include <algorithm>
#include <type_traits>

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
// row-major, zero-padded to R4 >= r (R4 a multiple of 4).  The work is cut
// into units of one row and 4 ranks (Q = R4 / 4 units per row): units
// [0, m Q) of the problem build F, units [m Q, (m + n) Q) build G, each with
// one float4 store, so a thread's loads are few and independent.  `first` is
// the problem's unit index of this workgroup's thread 0; threads at or beyond
// `end` only take part in the barrier.  The sorted seed indices are staged in
// LDS (when they fit) for the binary searches.  Contains a workgroup barrier:
// every thread of the workgroup must call it.
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
    const int Q = R4 / 4;
    const int64_t mq = m * Q;
    // a block lies entirely in the F part, entirely in the G part, or straddles
    const bool need_rows = first < mq;
    const bool need_cols = first + blockDim.x > mq;
    const bool rows_in_lds = need_rows && !need_cols && p <= kIdxLds;
    const bool cols_in_lds = need_cols && !need_rows && q <= kIdxLds;
    if (rows_in_lds)
        for (int64_t a = threadIdx.x; a < p; a += blockDim.x) sidx[a] = seed_rows[a];
    if (cols_in_lds)
        for (int64_t a = threadIdx.x; a < q; a += blockDim.x) sidx[a] = seed_cols[a];
    __syncthreads();

    const int64_t t = first + threadIdx.x;
    if (t >= end) return;                 // after the barrier: nothing below waits
    const int64_t rowq = t / Q;
    const int k0 = 4 * (int)(t - rowq * Q);
    floatx4 v = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    if (rowq < m) {
        const int64_t i = rowq;
        const int64_t *idx = rows_in_lds ? sidx : seed_rows;
        const int64_t a = lower_bound_i64(idx, p, i);
        if (a < p && idx[a] == i) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + e;
                if (k < r) v[e] = (float)(U[a + (int64_t)k * p] * sigma[k]);
            }
        } else {
            const int64_t b = i - a;   // position of i in the sorted complement
            if (b >= 0 && b < m - p) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = k0 + e;
                    if (k < r) v[e] = Pt[k + b * r];
                }
            }
        }
        *reinterpret_cast<floatx4 *>(F + i * R4 + k0) = v;
    } else if (rowq < m + n) {
        const int64_t jj = rowq - m;
        const int64_t *idx = cols_in_lds ? sidx : seed_cols;
        const int64_t a = lower_bound_i64(idx, q, jj);
        if (a < q && idx[a] == jj) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + e;
                if (k < r) v[e] = (float)V[a + (int64_t)k * q];
            }
        } else {
            const int64_t b = jj - a;
            if (b >= 0 && b < n - q) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = k0 + e;
                    if (k < r) v[e] = (float)((double)Qt[k + b * r] / sigma[k]);
                }
            }
        }
        *reinterpret_cast<floatx4 *>(G + jj * R4 + k0) = v;
    }
}

// Rows of F a lane keeps in VGPRs: 4 (16-byte loads and stores of M, L, S
// per lane, and each scalar G value feeds 4 FMAs), or 2 above rank 52, where
// 4 rows of F no longer fit 256 VGPRs.  At rank 52 the 4-row form holds 256
// VGPRs (two waves per SIMD) and still beats the 2-row form at three: measured
// on MI355X at m = n = 50000, 5.0 TB/s against 4.6.
constexpr int rows_per_lane(int R4) { return R4 > 52 ? 2 : 4; }
constexpr int rows_per_wave(int R4) { return 64 * rows_per_lane(R4); }
constexpr int kColBatch = 4;    // columns whose loads are in flight together

template <int N> struct VecOf;
template <> struct VecOf<2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<4> { typedef float type __attribute__((ext_vector_type(4))); };

// One wave of the completion: RPL = rows_per_lane(R4) rows per lane, the
// row block [RPW bx, RPW (bx + 1)) with RPW = 64 RPL, and a share of the
// nb = ceil(n / 4) batches of 4 columns, one of gy shares per row block:
//   * R4 <= 32 (most waves resident at once): batches by, by + gy, by + 2 gy,
//     ... -- the waves of a row block take turns along the columns, so the
//     whole grid sweeps the matrix together and the addresses in flight stay
//     in one narrow band of columns whatever the leading dimensions
//     (measured on MI355X at m = n = 10000: 13% more bandwidth than
//     contiguous ranges when the columns are not 512-byte aligned, the same
//     when they are);
//   * R4 > 32 (the grid runs in many rounds): the contiguous batches
//     [nb by / gy, nb (by + 1) / gy).
// Only the matrix's last batch can be partial.  VEC (16-byte aligned
// columns): lane l owns rows RPL l .. RPL l + RPL - 1 of the block and moves
// RPL-float vectors; otherwise lane l owns rows l, l + 64, ..., so each load
// and store instruction of the wave is one contiguous 256-byte run whatever
// the alignment of the column.  The loads of a batch's 4 columns are issued
// together, with no condition on any of them.
//
// The ragged last row block (m not a multiple of RPW) runs as a full block
// shifted to end at row m, in the element-wise layout: its rows that the
// previous block also covers are computed again by the same arithmetic and
// written again with the same bits.  Only a matrix of fewer than RPW rows
// takes a guarded, column-by-column path.
template <int R4, bool VEC>
__device__ __forceinline__ void recon_wave(const float *__restrict__ M, int64_t ldm,
                                           const float *__restrict__ F,
                                           const float *__restrict__ G, int64_t m, int64_t n,
                                           float *__restrict__ Lo, int64_t ldl,
                                           float *__restrict__ So, int64_t lds, uint32_t bx,
                                           uint32_t by, uint32_t gy, int lane)
{
    constexpr int RPL = rows_per_lane(R4);
    constexpr int RPW = rows_per_wave(R4);
    typedef typename VecOf<RPL>::type vec;

    constexpr bool kSweep = R4 <= 32;
    const int64_t nb = (n + kColBatch - 1) / kColBatch;
    const int64_t step = kSweep ? (int64_t)gy * kColBatch : kColBatch;
    const int64_t jbeg = kSweep ? (int64_t)by * kColBatch : kColBatch * (nb * (int64_t)by / gy);
    // end of the wave's columns (the sweep runs to n)
    const int64_t jend = kSweep ? n : std::min<int64_t>(n, kColBatch * (nb * ((int64_t)by + 1) / gy));

    float f[RPL][R4];
    // L of column j for this lane's rows, from the factor row G[j]
    auto product = [&](int64_t j) -> vec {
        const float *gj = G + j * R4;     // uniform across the wave
        vec lv;
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) lv[rr] = 0.0f;
#pragma unroll
        for (int k = 0; k < R4; ++k) {
            const float gk = gj[k];
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) lv[rr] = fmaf(f[rr][k], gk, lv[rr]);
        }
        return lv;
    };
    // the factor rows of this lane (rows past m read row m - 1 and are zeroed;
    // no branch, so all R4 / 4 loads per row go out together)
    auto load_f = [&](auto row) {
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int64_t i = row(rr);
            const bool in = i < m;
            const float *fi = F + (in ? i : m - 1) * R4;
#pragma unroll
            for (int k = 0; k < R4; k += 4) {
                const floatx4 v = *reinterpret_cast<const floatx4 *>(fi + k);
#pragma unroll
                for (int e = 0; e < 4; ++e) f[rr][k + e] = in ? v[e] : 0.0f;
            }
        }
    };
    // a full block starting at row blk0, vector (V) or element-wise layout
    auto full_block = [&](auto vec_tag, int64_t blk0) {
        constexpr bool V = decltype(vec_tag)::value;
        auto row = [&](int rr) -> int64_t { return V ? blk0 + lane * RPL + rr : blk0 + lane + 64 * rr; };
        load_f(row);
        auto load = [&](int64_t jj) -> vec {
            if constexpr (V) {
                const vec *src = reinterpret_cast<const vec *>(M + jj * ldm + row(0));
                if constexpr (R4 <= 8) return *src;
                else return __builtin_nontemporal_load(src);
            } else {
                vec mv;
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr)
                    mv[rr] = R4 <= 8 ? M[jj * ldm + row(rr)] : __builtin_nontemporal_load(M + jj * ldm + row(rr));
                return mv;
            }
        };
        auto store = [&](int64_t jj, const vec &mv) {
            const vec lv = product(jj);
            const vec sv = mv - lv;
            if constexpr (V) {
                __builtin_nontemporal_store(lv, reinterpret_cast<vec *>(Lo + jj * ldl + row(0)));
                __builtin_nontemporal_store(sv, reinterpret_cast<vec *>(So + jj * lds + row(0)));
            } else {
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr) {
                    __builtin_nontemporal_store(lv[rr], Lo + jj * ldl + row(rr));
                    __builtin_nontemporal_store(sv[rr], So + jj * lds + row(rr));
                }
            }
        };
        int64_t j = jbeg;
#pragma unroll 1
        for (; j + kColBatch <= jend; j += step) {
            vec mv[kColBatch];
#pragma unroll
            for (int cb = 0; cb < kColBatch; ++cb) mv[cb] = load(j + cb);
#pragma unroll
            for (int cb = 0; cb < kColBatch; ++cb) store(j + cb, mv[cb]);
        }
        // the matrix's last, partial batch (j < jend only for the wave that owns it)
        for (; j < jend; ++j) store(j, load(j));
    };

    const int64_t blk = (int64_t)bx * RPW;
    if (blk + RPW <= m) {
        full_block(std::integral_constant<bool, VEC>{}, blk);
    } else if (m >= RPW) {
        full_block(std::integral_constant<bool, false>{}, m - RPW);
    } else {
        // fewer than RPW rows in the matrix: guarded, one column at a time
        auto row = [&](int rr) -> int64_t { return lane + 64 * rr; };
        load_f(row);
#pragma unroll 1
        for (int64_t j = jbeg; j < jend; j += (kSweep ? step : 1)) {
#pragma unroll 1
            for (int cb = 0; cb < (kSweep ? kColBatch : 1); ++cb) {
                const int64_t jj = j + cb;
                if (jj >= jend) break;
                const vec lv = product(jj);
#pragma unroll
                for (int rr = 0; rr < RPL; ++rr)
                    if (row(rr) < m) {
                        const float mv = M[jj * ldm + row(rr)];
                        Lo[jj * ldl + row(rr)] = lv[rr];
                        So[jj * lds + row(rr)] = mv - lv[rr];
                    }
            }
        }
    }
}

} // namespace reconk
