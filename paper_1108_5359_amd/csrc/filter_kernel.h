// l1 filtering kernel: many independent regressions min ||x - A z||_1 with
// A^T A = I (eq. l1g), each solved by the ADM of Algorithm 1.
//
// Arithmetic: the iteration is carried in the equivalent "clip" form that
// follows from S_tau(t) = t - clip(t, -tau, tau) and A^T A = I:
//     g     = clip(beta u + y, -1, 1)            with u = x - A z
//     w     = A^T g,   z += w / beta,   v = A w
//     y_new = g - v,   u -= v / beta
//     ||x - A z_new - e_new||_inf = ||y_new - y||_inf / beta   (stopping test)
//     beta  = min(rho beta, beta_bar)
// It is algebraically identical to steps 1-3 of Algorithm 1 (E is never
// formed), only the well-scaled g in [-1, 1] and w enter the contractions,
// and u is recomputed from x every `refresh` steps to cancel FP32 drift.
//
// Layout on the chip (one wavefront = a tile of 16 regressions):
//   * both contractions run on MFMA v_mfma_f32_16x16x4_f32.  The state u, y
//     (p x 16) sits in VGPRs in the MFMA accumulator layout: lane l = 16 g + c
//     holds rows 16 t + 4 g + v (v = 0..3) of regression column c for every
//     16-row tile t.  That layout is directly the B operand of both
//     contractions once the contraction index is permuted consistently in the
//     A operand, so no data moves between lanes except two xor-shuffles for
//     ||.||_inf per step.
//   * A (FP64 in HBM) is converted once per workgroup into two FP32 copies in
//     LDS, stored in "fragment order" so that each MFMA's A operand comes from
//     one conflict-free ds_read_b128 per lane.
//   * rank permutation: row c of output tile mt of w = A^T g holds rank
//     16 mt + 4 (c % 4) + c / 4, so lane (g, c) register v holds rank
//     16 mt + 4 v + g and the K-step ks = 4 mt + v of v = A w covers ranks
//     4 ks .. 4 ks + 3: only KS = ceil(r / 4) K-steps are issued.
//   * beta, ||x||_inf, the stopping flag and the iteration count are per
//     regression (per lane column); a converged regression is frozen through a
//     zero step size, never by branching around MFMA.
//   * PT (16-row tiles of p) and KS are compile-time: the loop body is
//     straight-line code.
#pragma once

#include "rpca_internal.h"

#include <climits>
#include <type_traits>

namespace filterk {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWavesPerBlock = 4;

struct FilterLaunch {
    FilterSide side[2];
    const float *frag32[2];   // precision form: FP32 refresh fragments in HBM (or null = in LDS)
    int32_t nblocks0;         // blocks of side 0; the rest belong to side 1
    int32_t qtiles;           // precision form, p > 256: tiles per workgroup (1 or 2)
    FilterConsts c;
};

// Built classes: PT = tiles of 16 elements, KS = K-steps of 4 ranks.
constexpr int kPT[] = {1, 2, 3, 4, 5, 7, 8, 10, 13, 16, 19};
constexpr int kNumPT = sizeof(kPT) / sizeof(kPT[0]);
constexpr int kKS[] = {1, 2, 3, 4, 5, 6, 8, 10, 13, 16};
constexpr int kNumKS = sizeof(kKS) / sizeof(kKS[0]);

// Precision form: more tile classes (p up to 512).
constexpr int kPTh[] = {1, 2, 3, 4, 5, 7, 8, 10, 13, 16, 19, 26, 32};
constexpr int kNumPTh = sizeof(kPTh) / sizeof(kPTh[0]);

inline size_t lds_bytes(int PT, int KS)
{
    const int RT = (KS + 3) / 4;
    return (size_t)2 * PT * RT * 256 * sizeof(float) + (size_t)PT * 16 * sizeof(int64_t);
}

// Precision form: FP16 fragments (w = A^T g over tile pairs, v = A w over
// rank-tile pairs) plus, when ref_in_lds, the FP32 fragments of the refresh.
inline size_t lds_bytes_f16(int PT, int KS, bool ref_in_lds)
{
    const int RT = (KS + 3) / 4, PP = (PT + 1) / 2, RP = (RT + 1) / 2;
    size_t b = (size_t)PP * RT * 512 * sizeof(_Float16) + (size_t)PT * RP * 512 * sizeof(_Float16) +
               (size_t)PT * 16 * sizeof(int64_t);
    if (ref_in_lds) b += (size_t)PT * RT * 256 * sizeof(float);
    return b;
}

typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 acc)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// v_mfma_f32_4x4x1_16b_f32: 16 independent 4x4x1 blocks.  Lane 4 b + i
// gives row i of block b's A operand, lane 4 b + j column j of its B
// operand, and accumulator register i of lane 4 b + j is D_b[i][j].
__device__ __forceinline__ floatx4 mfma4x4(float a, float b, floatx4 acc)
{
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc, 0, 0, 0);
}

__device__ __forceinline__ floatx4 mfma16h(halfx8 a, halfx8 b, floatx4 acc)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
}

__device__ __forceinline__ halfx8 pack8(const float *lo, const float *hi)
{
    halfx8 h;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h[i] = (_Float16)lo[i];
        h[i + 4] = (_Float16)hi[i];
    }
    return h;
}

// Max / sum over the four lanes that share a regression column (c, c+16, c+32,
// c+48).  v_permlane16_swap / v_permlane32_swap exchange rows of 16 (32)
// lanes between two registers inside the VALU, with no LDS round trip as a
// ds_bpermute shuffle takes; called with both registers holding v, they leave
// v of lane l in one and v of lane l ^ 16 (l ^ 32) in the other, which are
// then combined: the same two operands as the xor shuffle form, so the same
// result bit for bit.
__device__ __forceinline__ float colmax(float v)
{
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return fmaxf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}

__device__ __forceinline__ float colsum(float v)
{
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Column sums of four values, scattered by row: lane (g, c) receives the sum
// of t_g over lanes c, c+16, c+32, c+48.  The first swap pairs rows 0/1 and
// 2/3 of t0 with t1 (and of t2 with t3) so that one add forms the row-pair
// sums of both values; the second pairs rows 0/1 with 2/3 across the two
// results.  Three swaps and three adds instead of four column sums and a
// selection, with the same operands in the same order (the same result).
__device__ __forceinline__ float colsum4_scatter(float t0, float t1, float t2, float t3)
{
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(t0), __float_as_uint(t1), false, false);
    const float s01 = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    auto b = __builtin_amdgcn_permlane16_swap(__float_as_uint(t2), __float_as_uint(t3), false, false);
    const float s23 = __uint_as_float(b[0]) + __uint_as_float(b[1]);
    auto c = __builtin_amdgcn_permlane32_swap(__float_as_uint(s01), __float_as_uint(s23), false, false);
    return __uint_as_float(c[0]) + __uint_as_float(c[1]);
}

template <int PT, int KS>
__global__ void __launch_bounds__(kWavesPerBlock * 64)
__attribute__((amdgpu_waves_per_eu(PT <= 13 ? 2 : 1)))
l1_filter_kernel(FilterLaunch L)
{
    constexpr int RT = (KS + 3) / 4;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float *fragA1 = reinterpret_cast<float *>(lds_raw);          // for w = A^T g
    float *fragA2 = fragA1 + PT * RT * 256;                        // for v = A w, A z
    int64_t *eoff = reinterpret_cast<int64_t *>(fragA2 + PT * RT * 256);

    // Pick this block's side field by field (scalar selects on kernel
    // arguments; no copy of the argument struct).
    const bool second = (int)blockIdx.x >= L.nblocks0;
#define SIDE(f) (second ? L.side[1].f : L.side[0].f)
    const int block_in_side = second ? (int)blockIdx.x - L.nblocks0 : (int)blockIdx.x;
    const int p = SIDE(p), r = SIDE(r);
    const double *__restrict__ A = SIDE(A);
    const int lda = SIDE(lda);
    const int64_t *__restrict__ elem_idx = SIDE(elem_idx);
    const int64_t *__restrict__ reg_idx = SIDE(reg_idx);
    const int64_t elem_stride = SIDE(elem_stride), reg_stride = SIDE(reg_stride);
    const int64_t elem_bound = SIDE(elem_bound), reg_bound = SIDE(reg_bound);
    const int64_t nreg = SIDE(nreg);
    const float *__restrict__ M = SIDE(M);
    float *__restrict__ Zout = SIDE(Z);
    const int64_t ldz = SIDE(ldz);
    int32_t *__restrict__ iters = SIDE(iters);
    floatx4 *__restrict__ xbuf = reinterpret_cast<floatx4 *>(SIDE(xbuf));
    const int64_t *range = SIDE(range);
#undef SIDE
    // positions served: [jbeg, jend) (a device range when the launch serves
    // one chunk of a side whose size is known only on the device)
    int64_t jbeg = 0, jend = nreg;
    if (range) {
        jbeg = range[0];
        jend = range[1];
    }

    // ---- stage the basis in LDS, in the two fragment orders -------------
    for (int idx = threadIdx.x; idx < PT * RT * 256; idx += kWavesPerBlock * 64) {
        const int v = idx & 3;
        const int ln = (idx >> 2) & 63;
        const int tm = idx >> 8;
        const int t = tm / RT, mt = tm - t * RT;
        const int g = ln >> 4, c = ln & 15;
        const int e1 = 16 * t + 4 * g + v, k1 = 16 * mt + 4 * (c & 3) + (c >> 2);
        fragA1[idx] = (e1 < p && k1 < r) ? (float)A[e1 + (int64_t)k1 * lda] : 0.0f;
        const int e2 = 16 * t + c, k2 = 16 * mt + 4 * v + g;
        fragA2[idx] = (e2 < p && k2 < r) ? (float)A[e2 + (int64_t)k2 * lda] : 0.0f;
    }
    for (int e = threadIdx.x; e < PT * 16; e += kWavesPerBlock * 64) {
        int64_t off = -1;
        if (e < p) {
            const int64_t ei = elem_idx[e];
            if (ei >= 0 && ei < elem_bound) off = ei * elem_stride;
        }
        eoff[e] = off;
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const int64_t tile = (int64_t)block_in_side * kWavesPerBlock + wave;
    const int64_t j = jbeg + tile * 16 + c;
    if (jbeg + tile * 16 >= jend) return;     // whole wave idle (no barrier follows)

    bool valid = j < jend;
    int64_t roff = 0;
    if (valid) {
        const int64_t ri = reg_idx[j];
        if (ri >= 0 && ri < reg_bound) roff = ri * reg_stride;
        else valid = false;
    }

    // ---- load x, its norms, and the starting state -----------------------
    float u[PT][4], y[PT][4];
    float xinf = 0.0f, xx = 0.0f;
    // x is gathered once from M (random seed rows / columns) and kept in
    // fragment order in HBM, so the refresh reads it back coalesced.
    floatx4 *xtile = xbuf + tile * PT * 64 + lane;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
        floatx4 xv;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t off = eoff[16 * t + 4 * g + v];
            const float x = (valid && off >= 0) ? M[roff + off] : 0.0f;
            xv[v] = x;
            u[t][v] = x;
            y[t][v] = 0.0f;
            xinf = fmaxf(xinf, fabsf(x));
            xx = fmaf(x, x, xx);
        }
        xtile[t * 64] = xv;
    }
    xinf = colmax(xinf);
    xx = colsum(xx);

    float beta = xx > 0.0f ? L.c.beta0_scale / sqrtf(xx) : 1.0f;
    const float beta_bar = L.c.beta_max_scale * beta;
    const float tol = L.c.eps * xinf;
    const bool bad = valid && nonfinite_norm(xx);     // x holds Inf / NaN
    bool done = !(valid && xinf > 0.0f) || bad;
    int K = 0;

    floatx4 z[RT];
#pragma unroll
    for (int mt = 0; mt < RT; ++mt) z[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    const floatx4 *F1 = reinterpret_cast<const floatx4 *>(fragA1) + lane;
    const floatx4 *F2 = reinterpret_cast<const floatx4 *>(fragA2) + lane;

    for (int k = 0; k < L.c.max_iter; ++k) {
        if (!__any(!done)) break;                                   // wave-uniform
        // The basis fragments are re-read from LDS every step instead of
        // being kept in VGPRs: that leaves room for two waves per SIMD.
        asm volatile("" ::: "memory");

        // w = A^T g, two accumulator chains (even / odd tiles) for ILP
        floatx4 Wa[RT], Wb[RT];
#pragma unroll
        for (int mt = 0; mt < RT; ++mt) {
            Wa[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            Wb[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            float gv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v)
                gv[v] = __builtin_amdgcn_fmed3f(fmaf(beta, u[t][v], y[t][v]), -1.0f, 1.0f);
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) {
                const floatx4 a = F1[(t * RT + mt) * 64];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (t & 1) Wb[mt] = mfma4(a[v], gv[v], Wb[mt]);
                    else Wa[mt] = mfma4(a[v], gv[v], Wa[mt]);
                }
            }
        }
        floatx4 W[RT];
#pragma unroll
        for (int mt = 0; mt < RT; ++mt) W[mt] = Wa[mt] + Wb[mt];

        // A converged regression keeps z and u frozen through a zero step
        // size; its y keeps moving but feeds nothing that is kept.
        const float inv_beta = 1.0f / beta;
        const float ib = done ? 0.0f : inv_beta;
#pragma unroll
        for (int mt = 0; mt < RT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) z[mt][v] = fmaf(W[mt][v], ib, z[mt][v]);

        // v = A w for two tiles at a time, then the dual / residual update
        float res = 0.0f;
#pragma unroll
        for (int t = 0; t < PT; t += 2) {
            floatx4 Va = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            floatx4 Vb = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) {
                const floatx4 a0 = F2[(t * RT + mt) * 64];
                floatx4 a1 = a0;
                if (t + 1 < PT) a1 = F2[((t + 1) * RT + mt) * 64];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (4 * mt + v < KS) {
                        Va = mfma4(a0[v], W[mt][v], Va);
                        if (t + 1 < PT) Vb = mfma4(a1[v], W[mt][v], Vb);
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int tt = t + h;
                if (tt < PT) {
                    const floatx4 Vt = h ? Vb : Va;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        // g again from the unchanged u, y (cheaper than keeping it)
                        const float gg =
                            __builtin_amdgcn_fmed3f(fmaf(beta, u[tt][v], y[tt][v]), -1.0f, 1.0f);
                        const float yn = gg - Vt[v];
                        res = fmaxf(res, fabsf(yn - y[tt][v]));
                        u[tt][v] = fmaf(-Vt[v], ib, u[tt][v]);
                        y[tt][v] = yn;
                    }
                }
            }
        }
        res = colmax(res);
        if (!done) {
            ++K;
            if (!(res * inv_beta >= tol)) done = true;   // ||x-Az-e||_inf < eps ||x||_inf
        }
        beta = fminf(L.c.rho * beta, beta_bar);

        // periodic u = x - A z from the input, against FP32 drift
        if (L.c.refresh > 0 && ((k + 1) % L.c.refresh) == 0) {
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                floatx4 Az = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int mt = 0; mt < RT; ++mt) {
                    const floatx4 a = F2[(t * RT + mt) * 64];
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (4 * mt + v < KS) Az = mfma4(a[v], z[mt][v], Az);
                }
                const floatx4 xv = xtile[t * 64];
#pragma unroll
                for (int v = 0; v < 4; ++v) u[t][v] = xv[v] - Az[v];
            }
        }
    }

    if (j < jend) {
        if (valid) {
#pragma unroll
            for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int kk = 16 * mt + 4 * v + g;
                    if (kk < r) Zout[kk + j * ldz] = bad ? __builtin_nanf("") : z[mt][v];
                }
        }
        if (iters && g == 0)
            iters[j] = !valid ? RPCA_ITERS_BAD_INDEX
                               : (bad ? RPCA_ITERS_NONFINITE : (done ? K : -L.c.max_iter));
    }
}

// ---------------------------------------------------------------------------
// Split form (FP32): one 16-regression tile per workgroup.  The PT 16-element
// tiles of the tile are dealt to the four waves (wave part w takes tiles
// [w PT / 4, (w + 1) PT / 4), the part rotated with the tile so that the
// heavier parts spread over the SIMDs); each wave keeps its slice of both
// basis fragments, of x and of the state u, y in VGPRs, contracts its slice
// and publishes its partial w = A^T g in LDS.  After one barrier every wave
// sums the four partials in part order, so all waves hold the identical w and
// z, and a regression's result does not depend on the tile it sits in.  The residual of step k is published with the partials of step
// k + 1, so the stopping test of a step is taken one step later (the state
// it reads is not changed by that delay: a stopped regression only stops
// moving z and u).  Used where a launch has too few tiles to give every SIMD
// the same number of tile waves: there each SIMD gets about a quarter of the
// contraction work of each tile in flight instead of all of it.
// ---------------------------------------------------------------------------
// Classes with a split kernel: PT >= 4 (below, a quarter of a tile is too
// little work per step for the exchange), and the state kept per lane (both
// fragments, x, u, y for PTW tiles; z and the two w partials) within 176 VGPRs
// so that two waves fit per SIMD.
constexpr bool split_built(int PT, int KS)
{
    const int RT = (KS + 3) / 4, PTW = (PT + kWavesPerBlock - 1) / kWavesPerBlock;
    return PT >= 4 && 2 * PTW * RT * 4 + 3 * PTW * 4 + 4 * RT * 4 <= 176;
}

template <int PT, int KS>
struct SplitShape {
    static constexpr int RT = (KS + 3) / 4;
    static constexpr int PTW = (PT + kWavesPerBlock - 1) / kWavesPerBlock;   // tiles of the heaviest part
    // The last rank tile holds NQ = KS - 4 (RT - 1) quads of ranks.  When it
    // holds one or two (NQ <= 2), its part of w = A^T g runs on
    // v_mfma_f32_4x4x1_16b_f32 (a quarter of the cycles of a 16x16x4 per quad)
    // instead of a padded 16x16x4 tile; with three the saving is small and the
    // accumulators do not fit.  NCH accumulator chains per quad: one (measured
    // at r = 20: filter 0.306 ms with four chains, 0.301 with two, 0.298 with
    // one -- the adds that join the chains cost more than the 4x4x1 latency
    // they hide).
    static constexpr int LT = RT - 1;
    static constexpr int NQ = KS - 4 * LT;
    static constexpr bool kQuad = NQ <= 2;
    static constexpr int NCH = 1;
    static constexpr int FT = kQuad ? LT : RT;   // rank tiles of w on 16x16x4
    // floats a lane publishes per step: w partials (of the quad part only the
    // lane's own rank, summed over the four g lanes before the exchange),
    // residual
    static constexpr int NV = 4 * FT + (kQuad ? NQ : 0) + 1;
    // three waves per SIMD (168 VGPRs) where the loop fits them without
    // spilling (checked at build time for every class), else two
    static constexpr int kWavesPerEU = (KS <= 5 && PTW <= 4) ? 3 : 2;
};

template <int PT, int KS>
__global__ void __launch_bounds__(kWavesPerBlock * 64)
__attribute__((amdgpu_waves_per_eu(SplitShape<PT, KS>::kWavesPerEU)))
l1_filter_split_kernel(FilterLaunch L)
{
    using Sh = SplitShape<PT, KS>;
    constexpr int RT = Sh::RT, PTW = Sh::PTW, NV = Sh::NV;
    constexpr int LT = Sh::LT, NQ = Sh::NQ, FT = Sh::FT;
    constexpr bool kQuad = Sh::kQuad;
    constexpr int NQA = kQuad ? NQ : 1;          // array extent of the quad parts
    constexpr int NCH = Sh::NCH;
    __shared__ float xch[2][kWavesPerBlock][NV][64];
    // x of each wave's slice, read back by the refresh (LDS instead of VGPRs)
    __shared__ floatx4 xs[kWavesPerBlock][PTW][64];

    const bool second = (int)blockIdx.x >= L.nblocks0;
#define SIDE(f) (second ? L.side[1].f : L.side[0].f)
    const int64_t tile = second ? (int)blockIdx.x - L.nblocks0 : (int)blockIdx.x;
    const int p = SIDE(p), r = SIDE(r);
    const double *__restrict__ A = SIDE(A);
    const int lda = SIDE(lda);
    const int64_t *__restrict__ elem_idx = SIDE(elem_idx);
    const int64_t *__restrict__ reg_idx = SIDE(reg_idx);
    const int64_t elem_stride = SIDE(elem_stride), reg_stride = SIDE(reg_stride);
    const int64_t elem_bound = SIDE(elem_bound), reg_bound = SIDE(reg_bound);
    const int64_t nreg = SIDE(nreg);
    const float *__restrict__ M = SIDE(M);
    float *__restrict__ Zout = SIDE(Z);
    const int64_t ldz = SIDE(ldz);
    int32_t *__restrict__ iters = SIDE(iters);
    const int64_t *range = SIDE(range);
#undef SIDE
    int64_t jbeg = 0, jend = nreg;
    if (range) {
        jbeg = range[0];
        jend = range[1];
    }
    if (jbeg + tile * 16 >= jend) return;           // the whole block is idle (before any barrier)

    // the wave index through readfirstlane: the compiler then knows every
    // quantity derived from it (part, slice, slot count) is wave-uniform and
    // branches on it with scalar branches instead of exec masks
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const int rot = (int)(tile & 3);
    const int part = (wave + rot) & 3;                       // wave of part pp: (pp - rot) & 3
    const int t0 = part * PT / kWavesPerBlock;
    const int cnt = (part + 1) * PT / kWavesPerBlock - t0;   // wave-uniform, 1 <= cnt <= PTW
    const int64_t j = jbeg + tile * 16 + c;
    bool valid = j < jend;
    int64_t roff = 0;
    if (valid) {
        const int64_t ri = reg_idx[j];
        if (ri >= 0 && ri < reg_bound) roff = ri * reg_stride;
        else valid = false;
    }

    // ---- this wave's slice of the basis (FP64 -> FP32), x and the state ----
    // a1: A operand of w = A^T g on 16x16x4 (rank tiles 0 .. FT-1);
    // a1q: A operand on 4x4x1 for quad q of the last rank tile: lane (g, c) is
    //      row c % 4 of block 4 g + c / 4, whose K-step is element 16 t + 4 g + v;
    // a2: A operand of v = A w and of the refresh.
    floatx4 a1[PTW][FT > 0 ? FT : 1], a1q[PTW][NQA], a2[PTW][RT];
    float u[PTW][4], y[PTW][4];
    float xinf = 0.0f, xx = 0.0f;
#pragma unroll
    for (int s = 0; s < PTW; ++s) {
        const int t = t0 + s;
        const bool on = s < cnt;
#pragma unroll
        for (int mt = 0; mt < RT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e1 = 16 * t + 4 * g + v;
                if (mt < FT) {
                    const int k1 = 16 * mt + 4 * (c & 3) + (c >> 2);
                    a1[s][mt][v] = (on && e1 < p && k1 < r) ? (float)A[e1 + (int64_t)k1 * lda] : 0.0f;
                }
                const int e2 = 16 * t + c, k2 = 16 * mt + 4 * v + g;
                a2[s][mt][v] = (on && e2 < p && k2 < r) ? (float)A[e2 + (int64_t)k2 * lda] : 0.0f;
            }
        if constexpr (kQuad) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int e1 = 16 * t + 4 * g + v, k1 = 16 * LT + 4 * q + (c & 3);
                    a1q[s][q][v] = (on && e1 < p && k1 < r) ? (float)A[e1 + (int64_t)k1 * lda] : 0.0f;
                }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = 16 * t + 4 * g + v;
            float xv = 0.0f;
            if (valid && on && e < p) {
                const int64_t ei = elem_idx[e];
                if (ei >= 0 && ei < elem_bound) xv = M[roff + ei * elem_stride];
            }
            xs[wave][s][lane][v] = xv;
            u[s][v] = xv;
            y[s][v] = 0.0f;
            xinf = fmaxf(xinf, fabsf(xv));
            xx = fmaf(xv, xv, xx);
        }
    }
    // norms of x over the four parts, summed in part order: the same value in
    // every wave, and the same for a regression wherever it sits
    xch[0][wave][0][lane] = xinf;
    xch[0][wave][1][lane] = xx;
    __syncthreads();
    xinf = 0.0f;
    xx = 0.0f;
#pragma unroll
    for (int pp = 0; pp < kWavesPerBlock; ++pp) {
        const int w = (pp - rot) & 3;
        xinf = fmaxf(xinf, xch[0][w][0][lane]);
        xx += xch[0][w][1][lane];
    }
    xinf = colmax(xinf);
    xx = colsum(xx);

    float beta = xx > 0.0f ? L.c.beta0_scale / sqrtf(xx) : 1.0f;
    const float beta_bar = L.c.beta_max_scale * beta;
    const float tol = L.c.eps * xinf;
    const bool bad = valid && nonfinite_norm(xx);     // x holds Inf / NaN
    bool done = !(valid && xinf > 0.0f) || bad;
    int K = 0;
    float inv_beta_prev = 0.0f, res_part = 0.0f;
    floatx4 z[RT];
#pragma unroll
    for (int mt = 0; mt < RT; ++mt) z[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    // The step loop, for a compile-time number NC of element tiles: no branch
    // per tile, so the MFMA chains of all the wave's tiles run back to back
    // (a branch per tile would end a basic block after each and wait out the
    // MFMA latency to move the accumulators).  Buffer 0 was read above; the
    // first step writes buffer 1.
    auto sweep = [&](auto nc_tag) {
        constexpr int NC = decltype(nc_tag)::value;
        for (int k = 0;; ++k) {
            // after max_iter steps only the pending stopping test is left (the
            // partial w of that pass is computed but not used)
            const bool last = k >= L.c.max_iter;
            floatx4 Wa[FT > 0 ? FT : 1], Wb[FT > 0 ? FT : 1];
            floatx4 Wq[NQA][NCH];                // quad part: NCH chains (by v)
#pragma unroll
            for (int mt = 0; mt < FT; ++mt) {
                Wa[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                Wb[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            }
#pragma unroll
            for (int q = 0; q < NQA; ++q)
#pragma unroll
                for (int h = 0; h < NCH; ++h) Wq[q][h] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                float gv[4];
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    gv[v] = __builtin_amdgcn_fmed3f(fmaf(beta, u[s][v], y[s][v]), -1.0f, 1.0f);
#pragma unroll
                for (int mt = 0; mt < FT; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (s & 1) Wb[mt] = mfma4(a1[s][mt][v], gv[v], Wb[mt]);
                        else Wa[mt] = mfma4(a1[s][mt][v], gv[v], Wa[mt]);
                    }
                if constexpr (kQuad) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            Wq[q][v % NCH] = mfma4x4(a1q[s][q][v], gv[v], Wq[q][v % NCH]);
                }
            }
            const int buf = (k + 1) & 1;
#pragma unroll
            for (int mt = 0; mt < FT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) xch[buf][wave][4 * mt + v][lane] = Wa[mt][v] + Wb[mt][v];
            if constexpr (kQuad) {
                // lane (g, c) register i: ranks 16 LT + 4 q + i of regression c,
                // summed over this lane's elements (rows 4 g .. 4 g + 3 of each
                // tile); summed over the four g lanes of the regression here,
                // lane (g, c) publishes rank 16 LT + 4 q + g, the layout of the
                // 16x16 tiles
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    floatx4 wq = Wq[q][0];
#pragma unroll
                    for (int h = 1; h < NCH; ++h) wq += Wq[q][h];
                    xch[buf][wave][4 * FT + q][lane] = colsum4_scatter(wq[0], wq[1], wq[2], wq[3]);
                }
            }
            // the residual partial, its maximum over the four g lanes taken
            // here (before the barrier, off the step's critical path)
            xch[buf][wave][NV - 1][lane] = colmax(res_part);
            __syncthreads();
            // w = sum of the partials in part order
            floatx4 W[RT];
            float res = 0.0f;
            {
                float ws[NV - 1];
                const int w0 = (0 - rot) & 3;
#pragma unroll
                for (int e = 0; e < NV - 1; ++e) ws[e] = xch[buf][w0][e][lane];
#pragma unroll
                for (int pp = 1; pp < kWavesPerBlock; ++pp) {
                    const int w = (pp - rot) & 3;
#pragma unroll
                    for (int e = 0; e < NV - 1; ++e) ws[e] += xch[buf][w][e][lane];
                }
#pragma unroll
                for (int mt = 0; mt < FT; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) W[mt][v] = ws[4 * mt + v];
                if constexpr (kQuad) {
                    W[LT] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int q = 0; q < NQ; ++q) W[LT][q] = ws[4 * FT + q];
                }
            }
#pragma unroll
            for (int w = 0; w < kWavesPerBlock; ++w) res = fmaxf(res, xch[buf][w][NV - 1][lane]);
            // the stopping test of step k - 1
            if (k > 0 && !done) {
                ++K;
                if (!(res * inv_beta_prev >= tol)) done = true;
            }
            if (last || !__any(!done)) break;                 // the same in every wave of the block

            const float inv_beta = __builtin_amdgcn_rcpf(beta);
            const float ib = done ? 0.0f : inv_beta;
#pragma unroll
            for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) z[mt][v] = fmaf(W[mt][v], ib, z[mt][v]);

            // v = A w for two tiles at a time (K-step outer: two interleaved
            // chains), then their dual / residual update
            res_part = 0.0f;
#pragma unroll
            for (int s0 = 0; s0 < NC; s0 += 2) {
                constexpr int kPair = 2;
                floatx4 V[kPair];
#pragma unroll
                for (int h = 0; h < kPair; ++h) V[h] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (4 * mt + v < KS)
#pragma unroll
                            for (int h = 0; h < kPair; ++h)
                                if (s0 + h < NC) V[h] = mfma4(a2[s0 + h][mt][v], W[mt][v], V[h]);
#pragma unroll
                for (int h = 0; h < kPair; ++h) {
                    const int s = s0 + h;
                    if (s < NC) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            // g again from the unchanged u, y (cheaper than keeping it)
                            const float gg =
                                __builtin_amdgcn_fmed3f(fmaf(beta, u[s][v], y[s][v]), -1.0f, 1.0f);
                            const float yn = gg - V[h][v];
                            res_part = fmaxf(res_part, fabsf(yn - y[s][v]));
                            u[s][v] = fmaf(-V[h][v], ib, u[s][v]);
                            y[s][v] = yn;
                        }
                    }
                }
            }
            inv_beta_prev = inv_beta;
            beta = fminf(L.c.rho * beta, beta_bar);

            if (L.c.refresh > 0 && ((k + 1) % L.c.refresh) == 0) {
#pragma unroll
                for (int s0 = 0; s0 < NC; s0 += 2) {
                    floatx4 Az[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) Az[h] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (4 * mt + v < KS)
#pragma unroll
                                for (int h = 0; h < 2; ++h)
                                    if (s0 + h < NC) Az[h] = mfma4(a2[s0 + h][mt][v], z[mt][v], Az[h]);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (s0 + h < NC) {
                            const floatx4 xv = xs[wave][s0 + h][lane];
#pragma unroll
                            for (int v = 0; v < 4; ++v) u[s0 + h][v] = xv[v] - Az[h][v];
                        }
                    }
                }
            }
        }
    };
    if constexpr (PT % kWavesPerBlock == 0) {
        sweep(std::integral_constant<int, PTW>{});
    } else {
        // parts hold floor(PT / 4) or ceil(PT / 4) tiles
        if (cnt == PTW) sweep(std::integral_constant<int, PTW>{});
        else sweep(std::integral_constant<int, PTW - 1>{});
    }

    // every wave holds the same z: wave 0 writes it
    if (wave == 0 && j < jend) {
        if (valid) {
#pragma unroll
            for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int kk = 16 * mt + 4 * v + g;
                    if (kk < r) Zout[kk + j * ldz] = bad ? __builtin_nanf("") : z[mt][v];
                }
        }
        if (iters && g == 0)
            iters[j] = !valid ? RPCA_ITERS_BAD_INDEX
                               : (bad ? RPCA_ITERS_NONFINITE : (done ? K : -L.c.max_iter));
    }
}


// ---------------------------------------------------------------------------
// Precision form: the two contractions on v_mfma_f32_16x16x32_f16 (FP16
// operands, FP32 accumulation); the residual u = x - A z is recomputed from x
// in FP32 (v_mfma_f32_16x16x4_f32) every `refresh` steps, which cancels the
// drift of the FP16 products (FP32 residual refinement).  g in [-1, 1] and
// the orthonormal basis fit FP16's range; z, u, y, beta stay FP32.
//
// Operand layouts (K = 32 per MFMA; any K order shared by A and B is exact):
//   w = A^T g : lane (g, c) slot i <-> element 16 (2 pp + i / 4) + 4 g + i % 4
//               (tiles 2 pp and 2 pp + 1 of the FP32 state, no data movement);
//               A operand row c <-> rank 16 mt + 4 (c % 4) + c / 4 as before.
//   v = A w   : lane (g, c) slot i <-> rank 16 (2 rp + i / 4) + 4 (i % 4) + g,
//               i.e. registers v = i % 4 of W tiles 2 rp and 2 rp + 1.
// ---------------------------------------------------------------------------
template <int PT, int KS>
__global__ void __launch_bounds__(kWavesPerBlock * 64)
__attribute__((amdgpu_waves_per_eu(PT <= 13 ? 2 : 1)))
l1_filter_kernel_f16(FilterLaunch L)
{
    constexpr int RT = (KS + 3) / 4;
    constexpr int PP = (PT + 1) / 2;
    constexpr int RP = (RT + 1) / 2;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    _Float16 *h1 = reinterpret_cast<_Float16 *>(lds_raw);              // [PP][RT][64][8]
    _Float16 *h2 = h1 + PP * RT * 512;                                   // [PT][RP][64][8]
    int64_t *eoff = reinterpret_cast<int64_t *>(h2 + PT * RP * 512);    // [PT*16]
    float *f2lds = reinterpret_cast<float *>(eoff + PT * 16);            // [PT][RT][64][4]

    const bool second = (int)blockIdx.x >= L.nblocks0;
#define SIDE(f) (second ? L.side[1].f : L.side[0].f)
    const int block_in_side = second ? (int)blockIdx.x - L.nblocks0 : (int)blockIdx.x;
    const int p = SIDE(p), r = SIDE(r);
    const double *__restrict__ A = SIDE(A);
    const int lda = SIDE(lda);
    const int64_t *__restrict__ elem_idx = SIDE(elem_idx);
    const int64_t *__restrict__ reg_idx = SIDE(reg_idx);
    const int64_t elem_stride = SIDE(elem_stride), reg_stride = SIDE(reg_stride);
    const int64_t elem_bound = SIDE(elem_bound), reg_bound = SIDE(reg_bound);
    const int64_t nreg = SIDE(nreg);
    const float *__restrict__ M = SIDE(M);
    float *__restrict__ Zout = SIDE(Z);
    const int64_t ldz = SIDE(ldz);
    int32_t *__restrict__ iters = SIDE(iters);
    floatx4 *__restrict__ xbuf = reinterpret_cast<floatx4 *>(SIDE(xbuf));
    const int64_t *range = SIDE(range);
#undef SIDE
    // positions served: [jbeg, jend) (a device range when the launch serves
    // one chunk of a side whose size is known only on the device)
    int64_t jbeg = 0, jend = nreg;
    if (range) {
        jbeg = range[0];
        jend = range[1];
    }
    const float *f2glob = second ? L.frag32[1] : L.frag32[0];

    // ---- stage the basis -------------------------------------------------
    for (int idx = threadIdx.x; idx < PP * RT * 512; idx += kWavesPerBlock * 64) {
        const int i = idx & 7, ln = (idx >> 3) & 63, pm = idx >> 9;
        const int pp = pm / RT, mt = pm - pp * RT;
        const int g = ln >> 4, c = ln & 15;
        const int e = 16 * (2 * pp + (i >> 2)) + 4 * g + (i & 3);
        const int k = 16 * mt + 4 * (c & 3) + (c >> 2);
        h1[idx] = (_Float16)((e < p && k < r) ? A[e + (int64_t)k * lda] : 0.0);
    }
    for (int idx = threadIdx.x; idx < PT * RP * 512; idx += kWavesPerBlock * 64) {
        const int i = idx & 7, ln = (idx >> 3) & 63, tr = idx >> 9;
        const int t = tr / RP, rp = tr - t * RP;
        const int g = ln >> 4, c = ln & 15;
        const int e = 16 * t + c;
        const int k = 16 * (2 * rp + (i >> 2)) + 4 * (i & 3) + g;
        h2[idx] = (_Float16)((e < p && k < r) ? A[e + (int64_t)k * lda] : 0.0);
    }
    if (!f2glob) {
        for (int idx = threadIdx.x; idx < PT * RT * 256; idx += kWavesPerBlock * 64) {
            const int v = idx & 3, ln = (idx >> 2) & 63, tm = idx >> 8;
            const int t = tm / RT, mt = tm - t * RT;
            const int g = ln >> 4, c = ln & 15;
            const int e2 = 16 * t + c, k2 = 16 * mt + 4 * v + g;
            f2lds[idx] = (e2 < p && k2 < r) ? (float)A[e2 + (int64_t)k2 * lda] : 0.0f;
        }
    }
    for (int e = threadIdx.x; e < PT * 16; e += kWavesPerBlock * 64) {
        int64_t off = -1;
        if (e < p) {
            const int64_t ei = elem_idx[e];
            if (ei >= 0 && ei < elem_bound) off = ei * elem_stride;
        }
        eoff[e] = off;
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const int64_t tile = (int64_t)block_in_side * kWavesPerBlock + wave;
    const int64_t j = jbeg + tile * 16 + c;
    if (jbeg + tile * 16 >= jend) return;     // whole wave idle (no barrier follows)

    bool valid = j < jend;
    int64_t roff = 0;
    if (valid) {
        const int64_t ri = reg_idx[j];
        if (ri >= 0 && ri < reg_bound) roff = ri * reg_stride;
        else valid = false;
    }

    // Large p: the dual y is held as packed FP16 (y is in [-1, 1]; measured
    // effect on the result: 1.2e-7 -> 1.5e-7 relative), halving its registers.
    constexpr bool Y16 = PT >= 19;
    typedef _Float16 half2v __attribute__((ext_vector_type(2)));
    float u[PT][4];
    float y[Y16 ? 1 : PT][4];
    half2v yh[Y16 ? PT : 1][2];
    auto yget = [&](int t, int v) -> float {
        if constexpr (Y16) return (float)yh[t][v >> 1][v & 1];
        else return y[t][v];
    };
    auto yset = [&](int t, int v, float val) {
        if constexpr (Y16) yh[t][v >> 1][v & 1] = (_Float16)val;
        else y[t][v] = val;
    };
    float xinf = 0.0f, xx = 0.0f;
    // x is gathered once from M (random seed rows / columns) and kept in
    // fragment order in HBM, so the refresh reads it back coalesced.
    floatx4 *xtile = xbuf + tile * PT * 64 + lane;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
        floatx4 xv;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t off = eoff[16 * t + 4 * g + v];
            const float x = (valid && off >= 0) ? M[roff + off] : 0.0f;
            xv[v] = x;
            u[t][v] = x;
            yset(t, v, 0.0f);
            xinf = fmaxf(xinf, fabsf(x));
            xx = fmaf(x, x, xx);
        }
        xtile[t * 64] = xv;
    }
    xinf = colmax(xinf);
    xx = colsum(xx);

    float beta = xx > 0.0f ? L.c.beta0_scale / sqrtf(xx) : 1.0f;
    const float beta_bar = L.c.beta_max_scale * beta;
    const float tol = L.c.eps * xinf;
    const bool bad = valid && nonfinite_norm(xx);     // x holds Inf / NaN
    bool done = !(valid && xinf > 0.0f) || bad;
    int K = 0;

    floatx4 z[RT];
#pragma unroll
    for (int mt = 0; mt < RT; ++mt) z[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    const halfx8 *H1 = reinterpret_cast<const halfx8 *>(h1) + lane;
    const halfx8 *H2 = reinterpret_cast<const halfx8 *>(h2) + lane;
    const floatx4 *F2 = f2glob ? reinterpret_cast<const floatx4 *>(f2glob) + lane
                               : reinterpret_cast<const floatx4 *>(f2lds) + lane;

    for (int k = 0; k < L.c.max_iter; ++k) {
        if (!__any(!done)) break;                                   // wave-uniform
        asm volatile("" ::: "memory");

        // w = A^T g over tile pairs (K = 32 elements per MFMA)
        floatx4 Wa[RT], Wb[RT];
#pragma unroll
        for (int mt = 0; mt < RT; ++mt) {
            Wa[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            Wb[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int pp = 0; pp < PP; ++pp) {
            // large p: bound how far the scheduler hoists fragment loads
            if constexpr (PT >= 19) __builtin_amdgcn_sched_barrier(0);
            float glo[4], ghi[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                glo[v] = __builtin_amdgcn_fmed3f(fmaf(beta, u[2 * pp][v], yget(2 * pp, v)), -1.0f, 1.0f);
                constexpr int dummy = 0;
                (void)dummy;
                const int t1 = 2 * pp + 1 < PT ? 2 * pp + 1 : 0;
                ghi[v] = (2 * pp + 1 < PT)
                    ? __builtin_amdgcn_fmed3f(fmaf(beta, u[t1][v], yget(t1, v)), -1.0f, 1.0f)
                    : 0.0f;
            }
            const halfx8 gb = pack8(glo, ghi);
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) {
                const halfx8 a = H1[(pp * RT + mt) * 64];
                // one rank tile: alternate two chains for ILP; several: one chain each
                if (RT == 1 && (pp & 1)) Wb[mt] = mfma16h(a, gb, Wb[mt]);
                else Wa[mt] = mfma16h(a, gb, Wa[mt]);
            }
        }
        floatx4 W[RT];
#pragma unroll
        for (int mt = 0; mt < RT; ++mt) W[mt] = (RT == 1) ? Wa[mt] + Wb[mt] : Wa[mt];

        const float inv_beta = 1.0f / beta;
        const float ib = done ? 0.0f : inv_beta;
#pragma unroll
        for (int mt = 0; mt < RT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) z[mt][v] = fmaf(W[mt][v], ib, z[mt][v]);

        // w as the FP16 B operand of v = A w, rank-tile pairs
        halfx8 wb[RP];
#pragma unroll
        for (int rp = 0; rp < RP; ++rp) {
            float lo[4], hi[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                lo[v] = W[2 * rp][v];
                hi[v] = (2 * rp + 1 < RT) ? W[2 * rp + 1 < RT ? 2 * rp + 1 : 0][v] : 0.0f;
            }
            wb[rp] = pack8(lo, hi);
        }

        float res = 0.0f;
#pragma unroll
        for (int t = 0; t < PT; t += 2) {
            if constexpr (PT >= 19) __builtin_amdgcn_sched_barrier(0);
            floatx4 Va = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            floatx4 Vb = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int rp = 0; rp < RP; ++rp) {
                Va = mfma16h(H2[(t * RP + rp) * 64], wb[rp], Va);
                if (t + 1 < PT) Vb = mfma16h(H2[((t + 1) * RP + rp) * 64], wb[rp], Vb);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int tt = t + h;
                if (tt < PT) {
                    const floatx4 Vt = h ? Vb : Va;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float yo = yget(tt, v);
                        const float gg = __builtin_amdgcn_fmed3f(fmaf(beta, u[tt][v], yo), -1.0f, 1.0f);
                        const float yn = gg - Vt[v];
                        res = fmaxf(res, fabsf(yn - yo));
                        u[tt][v] = fmaf(-Vt[v], ib, u[tt][v]);
                        yset(tt, v, yn);
                    }
                }
            }
        }
        res = colmax(res);
        if (!done) {
            ++K;
            if (!(res * inv_beta >= tol)) done = true;   // ||x-Az-e||_inf < eps ||x||_inf
        }
        beta = fminf(L.c.rho * beta, beta_bar);

        // FP32 residual refinement: u = x - A z from the input
        if (L.c.refresh > 0 && ((k + 1) % L.c.refresh) == 0) {
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                // keep the refresh tile by tile (it runs rarely; hoisting all
                // of its fragment loads would cost registers the loop needs)
                __builtin_amdgcn_sched_barrier(0);
                floatx4 Az = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int mt = 0; mt < RT; ++mt) {
                    const floatx4 a = F2[(t * RT + mt) * 64];
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (4 * mt + v < KS) Az = mfma4(a[v], z[mt][v], Az);
                }
                const floatx4 xv = xtile[t * 64];
#pragma unroll
                for (int v = 0; v < 4; ++v) u[t][v] = xv[v] - Az[v];
            }
        }
    }

    if (j < jend) {
        if (valid) {
#pragma unroll
            for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int kk = 16 * mt + 4 * v + g;
                    if (kk < r) Zout[kk + j * ldz] = bad ? __builtin_nanf("") : z[mt][v];
                }
        }
        if (iters && g == 0)
            iters[j] = !valid ? RPCA_ITERS_BAD_INDEX
                               : (bad ? RPCA_ITERS_NONFINITE : (done ? K : -L.c.max_iter));
    }
}

// ---------------------------------------------------------------------------
// Quarter-tile persistent form for large p (PT >= 19).  One
// wave holding all PT element tiles of its 16 regressions needs 8 PT floats of
// u, y per lane (256 at p = 512: the whole register file, so the tile kernel
// spills, and the basis fragments of a contraction cannot be kept in flight).
// Here four waves serve one 16-regression tile together, each holding a
// quarter of the element-tile pairs; a workgroup serves one or two tile
// slots (TPB, below) that step together.  The workgroup stages the FP16
// basis fragments in LDS once; each slot then serves the regressions of its
// tiles (its index, plus the side's workgroup count, ...) as one sequence,
// one regression per column at a time, a stopped regression's column taking
// the next one at the next refill point (one refresh period apart).  Per step
// each wave contracts its quarter (w = A^T g) and publishes the partial w and
// the previous step's residual partial in LDS; after a barrier every wave
// adds the four partials in quarter order (identical w and z in all four
// waves, and the same bits for a regression wherever it sits), and a second
// barrier frees the buffer.  The stopping test of a step is taken one step
// later; a stopped regression only stops moving z and u until its column is
// refilled.  The refresh reads its FP32 fragments from HBM.  The same shape
// serves the FP32 form beyond the FP32 tile classes (p > 304): the basis is
// staged in LDS as FP32 for w = A^T g, and v = A w reads the refresh
// fragments, one element tile ahead of its 16x16x4 FP32 MFMAs.
// ---------------------------------------------------------------------------
// Fourth word of a raw buffer resource on gfx950 (32-bit data, no swizzle).
constexpr int kBufWord3 = 0x00020000;

// 16 bytes per lane through a buffer resource: byte offset voff (per lane)
// plus soff (wave-uniform, an SGPR); both must stay inside the resource.
__device__ __forceinline__ floatx4 buf_load4(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

template <int PT, int KS>
struct QuarterShape {
    static constexpr int RT = (KS + 3) / 4;
    static constexpr int RP = (RT + 1) / 2;
    static constexpr int PP = (PT + 1) / 2;          // element-tile pairs
    static constexpr int NPP = (PP + 3) / 4;         // pairs per quarter (the last may pad)
    static constexpr int PPA = 4 * NPP;              // pairs staged (padded)
    static constexpr int TA = 2 * PPA;               // element tiles staged (padded)
    // floats a lane publishes per step: its values of w for the real ranks
    // (register v of rank tile mt holds rank 16 mt + 4 v + g: real while
    // 4 mt + v < KS), then the residual
    static constexpr int NV = KS + 1;
};

constexpr bool half_form(int PT) { return PT >= 19; }

// TPB tiles per workgroup (4 TPB waves).  With two, each SIMD holds two
// waves (of different tiles) that hide each other's latencies; the element
// indices are then staged as 32-bit values so that the fragments, indices
// and both tiles' exchange buffers fit in 160 KB.
inline size_t lds_bytes_f16q(int PT, int KS, int TPB)
{
    const int RT = (KS + 3) / 4, RP = (RT + 1) / 2, PP = (PT + 1) / 2, NPP = (PP + 3) / 4;
    const int PPA = 4 * NPP, TA = 2 * PPA, NV = KS + 1;
    return (size_t)PPA * RT * 512 * sizeof(_Float16) + (size_t)TA * RP * 512 * sizeof(_Float16) +
           (size_t)TA * 16 * (TPB == 2 ? sizeof(int32_t) : sizeof(int64_t)) +
           (size_t)TPB * kWavesPerBlock * NV * 64 * sizeof(float);
}

// The same workgroup shape with FP32 contractions (the plain form beyond the
// FP32 tile classes): the basis in the w = A^T g order is staged in LDS as
// FP32 (the tile kernel's first fragment order), and v = A w streams the
// refresh fragments from HBM (L2), as the refresh does with z.
inline size_t lds_bytes_q32(int PT, int KS, int TPB)
{
    const int RT = (KS + 3) / 4, PP = (PT + 1) / 2, NPP = (PP + 3) / 4, TA = 8 * NPP, NV = KS + 1;
    return (size_t)PT * RT * 256 * sizeof(float) +
           (size_t)TA * 16 * (TPB == 2 ? sizeof(int32_t) : sizeof(int64_t)) +
           (size_t)TPB * kWavesPerBlock * NV * 64 * sizeof(float);
}

// H = true: FP16 contractions (h1, h2 in LDS; the precision form from
// PT = 19).  H = false: FP32 contractions (a1 in LDS, v = A w from the refresh
// fragments; the FP32 form beyond PT = 19).
template <int PT, int KS, int TPB, bool H>
__global__ void __launch_bounds__(TPB * kWavesPerBlock * 64)
l1_filter_kernel_quarter(FilterLaunch L)
{
    using Sh = QuarterShape<PT, KS>;
    constexpr int RT = Sh::RT, RP = Sh::RP, NPP = Sh::NPP, PPA = Sh::PPA, TA = Sh::TA;
    constexpr int NV = Sh::NV;
    constexpr int NT = TPB * kWavesPerBlock * 64;    // threads of the workgroup
    // FP32 mode: when the last rank tile holds a single quad of ranks (KS =
    // 4 RT - 3), its part of w = A^T g runs on v_mfma_f32_4x4x1_16b_f32 (a
    // quarter of the cycles of the padded 16x16x4 tile)
    constexpr int LT = RT - 1;
    constexpr bool kQ1 = !H && KS == 4 * LT + 1;
    // element index of the gathered x: offset (TPB = 1) or 32-bit row/column
    // index, scaled by the stride when read (TPB = 2)
    using EIdx = typename std::conditional<TPB == 2, int32_t, int64_t>::type;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    _Float16 *h1 = reinterpret_cast<_Float16 *>(lds_raw);              // [PPA][RT][64][8]
    _Float16 *h2 = h1 + PPA * RT * 512;                                  // [TA][RP][64][8]
    float *a1 = reinterpret_cast<float *>(lds_raw);                      // FP32: [PT][RT][64][4]
    EIdx *eoff = H ? reinterpret_cast<EIdx *>(h2 + TA * RP * 512)       // [TA*16]
                   : reinterpret_cast<EIdx *>(a1 + PT * RT * 256);
    float *xch = reinterpret_cast<float *>(eoff + TA * 16);              // [TPB][4 waves][NV][64]

    const bool second = (int)blockIdx.x >= L.nblocks0;
#define SIDE(f) (second ? L.side[1].f : L.side[0].f)
    const int block_in_side = second ? (int)blockIdx.x - L.nblocks0 : (int)blockIdx.x;
    const int side_blocks = second ? (int)gridDim.x - L.nblocks0 : L.nblocks0;
    const int p = SIDE(p), r = SIDE(r);
    const double *__restrict__ A = SIDE(A);
    const int lda = SIDE(lda);
    const int64_t *__restrict__ elem_idx = SIDE(elem_idx);
    const int64_t *__restrict__ reg_idx = SIDE(reg_idx);
    const int64_t elem_stride = SIDE(elem_stride), reg_stride = SIDE(reg_stride);
    const int64_t elem_bound = SIDE(elem_bound), reg_bound = SIDE(reg_bound);
    const int64_t nreg = SIDE(nreg);
    const float *__restrict__ M = SIDE(M);
    float *__restrict__ Zout = SIDE(Z);
    const int64_t ldz = SIDE(ldz);
    int32_t *__restrict__ iters = SIDE(iters);
    floatx4 *__restrict__ xbuf = reinterpret_cast<floatx4 *>(SIDE(xbuf));
    const int64_t *range = SIDE(range);
#undef SIDE
    int64_t jbeg = 0, jend = nreg;
    if (range) {
        jbeg = range[0];
        jend = range[1];
    }
    const float *f2glob = second ? L.frag32[1] : L.frag32[0];
    if (jbeg + (int64_t)block_in_side * TPB * 16 >= jend) return;   // no tile for this block (before any barrier)

    // ---- stage the basis once (padded pairs and tiles are zero) -----------
    if constexpr (H) {
        for (int idx = threadIdx.x; idx < PPA * RT * 512; idx += NT) {
            const int i = idx & 7, ln = (idx >> 3) & 63, pm = idx >> 9;
            const int pp = pm / RT, mt = pm - pp * RT;
            const int g = ln >> 4, c = ln & 15;
            const int e = 16 * (2 * pp + (i >> 2)) + 4 * g + (i & 3);
            const int k = 16 * mt + 4 * (c & 3) + (c >> 2);
            h1[idx] = (_Float16)((e < p && k < r) ? A[e + (int64_t)k * lda] : 0.0);
        }
        for (int idx = threadIdx.x; idx < TA * RP * 512; idx += NT) {
            const int i = idx & 7, ln = (idx >> 3) & 63, tr = idx >> 9;
            const int t = tr / RP, rp = tr - t * RP;
            const int g = ln >> 4, c = ln & 15;
            const int e = 16 * t + c;
            const int k = 16 * (2 * rp + (i >> 2)) + 4 * (i & 3) + g;
            h2[idx] = (_Float16)((e < p && k < r) ? A[e + (int64_t)k * lda] : 0.0);
        }
    } else {
        // register v of lane (g, c) in (t, mt): A[16 t + 4 g + v][16 mt + 4 (c & 3) + (c >> 2)],
        // so that the MFMA's output register v is rank 16 mt + 4 v + g, as z
        for (int idx = threadIdx.x; idx < PT * RT * 256; idx += NT) {
            const int v = idx & 3, ln = (idx >> 2) & 63, tm = idx >> 8;
            const int t = tm / RT, mt = tm - t * RT;
            const int g = ln >> 4, c = ln & 15;
            // (4x4x1 quad: lane (g, c) is row c % 4 of block 4 g + c / 4, whose
            // K-step is element 16 t + 4 g + v)
            const int e = 16 * t + 4 * g + v;
            const int k = (kQ1 && mt == LT) ? 16 * LT + (c & 3) : 16 * mt + 4 * (c & 3) + (c >> 2);
            a1[idx] = (e < p && k < r) ? (float)A[e + (int64_t)k * lda] : 0.0f;
        }
    }
    for (int e = threadIdx.x; e < TA * 16; e += NT) {
        int64_t off = -1;
        if (e < p) {
            const int64_t ei = elem_idx[e];
            // (TPB = 2: the launcher checked that the bound fits 32 bits)
            if (ei >= 0 && ei < elem_bound) off = TPB == 2 ? ei : ei * elem_stride;
        }
        eoff[e] = (EIdx)off;
    }
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, c = lane & 15;
    const int tl = wave / kWavesPerBlock;             // this wave's tile slot of the block
    const int part = wave % kWavesPerBlock;           // its quarter
    const int pp0 = part * NPP;                       // this quarter's first pair
    const halfx8 *H1 = reinterpret_cast<const halfx8 *>(h1) + lane;
    const halfx8 *H2 = reinterpret_cast<const halfx8 *>(h2) + lane;
    const floatx4 *A1 = reinterpret_cast<const floatx4 *>(a1) + lane;
    const floatx4 *F2 = reinterpret_cast<const floatx4 *>(f2glob) + lane;
    float *mine = xch + wave * NV * 64 + lane;
    const float *all = xch + tl * kWavesPerBlock * NV * 64 + lane;   // this slot's quarters

    // ---- the slot's regressions ------------------------------------------
    // A slot serves the regressions of its tiles (tb TPB + slot, tb =
    // block_in_side, + side_blocks, ...) as one sequence, one regression per
    // column at a time: a column whose regression has stopped takes the next
    // one of the sequence at the next refill point.  Refill points are one
    // refresh period apart, so every regression starts its steps at the same
    // phase of the refresh schedule; with the per-column arithmetic of the
    // contractions (an MFMA output column depends on its own input column
    // only) and the per-column sums, a regression's result does not depend
    // on its column-mates.  A refilled column loads its x (refill step), sums
    // its norms over the quarters (next step, in place of its w partials) and
    // takes its step 0 one step later.
    const int RA = L.c.refresh > 0 ? L.c.refresh : 1;
    auto seq_pos = [&](int64_t i) -> int64_t {        // position of sequence entry i
        return jbeg + ((block_in_side + (i >> 4) * side_blocks) * TPB + tl) * 16 + (i & 15);
    };
    constexpr int64_t kNone = INT64_MAX;              // a column holding no regression
    // x of the slot's columns in fragment order (read back by the refresh)
    floatx4 *xslot_base = xbuf + ((int64_t)block_in_side * TPB + tl) * PT * 64;
    floatx4 *xslot = xslot_base + lane;
    int64_t cursor = 0;                               // next sequence entry (uniform)
    uint64_t fresh_m = 0;                             // lanes of columns set up in this step
    int64_t j = kNone, roff = 0;
    bool valid = false, bad = false, done = true;
    int K = 0;
    float u[2 * NPP][4], y[2 * NPP][4];
    floatx4 z[RT];
#pragma unroll
    for (int s = 0; s < 2 * NPP; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            u[s][v] = 0.0f;
            y[s][v] = 0.0f;
        }
#pragma unroll
    for (int mt = 0; mt < RT; ++mt) z[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float beta = 1.0f, beta_bar = 1.0f, tol = 0.0f, inv_beta_prev = 0.0f, res_part = 0.0f;

    // the result of the column's regression (quarter 0 writes it)
    auto store = [&]() __attribute__((always_inline)) {
        if (part == 0 && j < jend) {
            if (valid) {
#pragma unroll
                for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int kk = 16 * mt + 4 * v + g;
                        if (kk < r) Zout[kk + j * ldz] = bad ? __builtin_nanf("") : z[mt][v];
                    }
            }
            if (iters && g == 0)
                iters[j] = !valid ? RPCA_ITERS_BAD_INDEX : (bad ? RPCA_ITERS_NONFINITE : K);
        }
    };

    // Block steps from -2: the first refill (step -2) and norm sums (step -1)
    // of every column, then step 0 of the first regressions.
#pragma unroll 1
    for (int k = -2;; ++k) {
        const bool fl = (fresh_m >> lane) & 1;        // this column is set up in this step
        floatx4 Wp[RT];
        // g of this step, kept for the dual update (u, y do not change in between)
        float gk[2 * NPP][4];
        if constexpr (H) {
            // partial w = A^T g over this quarter's pairs (K = 32 elements per
            // MFMA); the quarter's fragments are read from LDS all at once, so
            // their latency is paid once per contraction, not once per MFMA
            halfx8 f1[NPP][RT];
#pragma unroll
            for (int q = 0; q < NPP; ++q)
#pragma unroll
                for (int mt = 0; mt < RT; ++mt) f1[q][mt] = H1[((pp0 + q) * RT + mt) * 64];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) Wp[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int q = 0; q < NPP; ++q) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        gk[2 * q + h][v] =
                            __builtin_amdgcn_fmed3f(fmaf(beta, u[2 * q + h][v], y[2 * q + h][v]), -1.0f, 1.0f);
                const halfx8 gb = pack8(gk[2 * q], gk[2 * q + 1]);
#pragma unroll
                for (int mt = 0; mt < RT; ++mt) Wp[mt] = mfma16h(f1[q][mt], gb, Wp[mt]);
            }
        } else {
            // partial w = A^T g on 16x16x4 FP32 MFMAs (K = 4 elements:
            // 16 t + 4 g + v over g), two element tiles per batch of LDS
            // reads.  A tile past PT (the last quarter's padding) reads the
            // last real tile's fragments against g = 0 (its x is 0), adding 0.
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) Wp[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s0 = 0; s0 < 2 * NPP; s0 += 2) {
                floatx4 fa[2][RT];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int t = min(2 * pp0 + s0 + h, PT - 1);
#pragma unroll
                    for (int mt = 0; mt < RT; ++mt) fa[h][mt] = A1[(t * RT + mt) * 64];
                }
                // (g is formed again for the dual update: registers, not VALU, bind here)
                float gl[2][4];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        gl[h][v] = __builtin_amdgcn_fmed3f(fmaf(beta, u[s0 + h][v], y[s0 + h][v]), -1.0f, 1.0f);
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
#pragma unroll
                        for (int mt = 0; mt < RT; ++mt)
                            Wp[mt] = (kQ1 && mt == LT) ? mfma4x4(fa[h][mt][v], gl[h][v], Wp[mt])
                                                       : mfma4(fa[h][mt][v], gl[h][v], Wp[mt]);
            }
        }
        // partial w (a column being set up publishes its x norms in slots 0
        // and NV - 1 instead, written in the refill step); the residual
        // partial, or -1 for a stopped regression (0 in one lane while the
        // slot still has regressions to take: the block goes on)
        const bool pend = seq_pos(cursor) < jend;
        if constexpr (kQ1) {
            // quad part: lane (g, c) register i holds rank 16 LT + i of regression
            // c over this lane's elements; summed over the four g lanes and
            // scattered, lane (g, c) holds rank 16 LT + g: the 16x16 layout
            Wp[LT][0] = colsum4_scatter(Wp[LT][0], Wp[LT][1], Wp[LT][2], Wp[LT][3]);
        }
#pragma unroll
        for (int mt = 0; mt < RT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (4 * mt + v < KS && (4 * mt + v > 0 || !fl)) mine[(4 * mt + v) * 64] = Wp[mt][v];
        if (!fl) mine[(NV - 1) * 64] = done ? ((pend && lane == 0) ? 0.0f : -1.0f) : res_part;
        __syncthreads();
        floatx4 W[RT];
        float res = all[(NV - 1) * 64];
#pragma unroll
        for (int mt = 0; mt < RT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) W[mt][v] = (4 * mt + v < KS) ? all[(4 * mt + v) * 64] : 0.0f;
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) {
#pragma unroll
            for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (4 * mt + v < KS) W[mt][v] += all[(w * NV + 4 * mt + v) * 64];
            res = fmaxf(res, all[(w * NV + NV - 1) * 64]);
        }
        // whether any column of the block was still moving (or being set up,
        // or could take a regression) at this step's publication: the same in
        // every wave
        bool live_prev;
        {
            const float f0 = xch[(NV - 1) * 64 + lane];
            if constexpr (TPB == 2) {
                const float f1 = xch[(kWavesPerBlock * NV + NV - 1) * 64 + lane];
                live_prev = __any(f0 >= 0.0f || f1 >= 0.0f);
            } else {
                live_prev = __any(f0 >= 0.0f);
            }
        }
        res = colmax(res);
        // the stopping test of the previous step (a column past its step 0);
        // after max_iter steps a regression stops unconverged
        if (inv_beta_prev > 0.0f && !done) {
            ++K;
            if (!(res * inv_beta_prev >= tol)) done = true;
            else if (K >= L.c.max_iter) {
                done = true;
                K = -L.c.max_iter;
            }
        }
        // columns being set up: their norms over the four quarters (slot 0
        // holds each quarter's max, slot NV - 1 its sum of squares)
        if (fresh_m != 0) {
            float xinf = all[0], xx = all[(NV - 1) * 64];
#pragma unroll
            for (int w = 1; w < kWavesPerBlock; ++w) {
                xinf = fmaxf(xinf, all[w * NV * 64]);
                xx += all[(w * NV + NV - 1) * 64];
            }
            if (fl) {
                beta = xx > 0.0f ? L.c.beta0_scale / sqrtf(xx) : 1.0f;
                beta_bar = L.c.beta_max_scale * beta;
                tol = L.c.eps * xinf;
                bad = valid && nonfinite_norm(xx);     // x holds Inf / NaN
                done = !(valid && xinf > 0.0f) || bad;
                K = 0;
                res_part = 0.0f;
            }
        }
        __syncthreads();                              // every wave has read the partials
        if (!live_prev) break;                        // the same in every wave of the block

        const float inv_beta = __builtin_amdgcn_rcpf(beta);
        // (a column set up in this step is frozen until its step 0)
        const float ib = (done || fl) ? 0.0f : inv_beta;
#pragma unroll
        for (int mt = 0; mt < RT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (4 * mt + v < KS) z[mt][v] = fmaf(W[mt][v], ib, z[mt][v]);

        if constexpr (H) {
            // w as the FP16 B operand of v = A w, rank-tile pairs
            halfx8 wb[RP];
#pragma unroll
            for (int rp = 0; rp < RP; ++rp) {
                float lo[4], hi[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    lo[v] = W[2 * rp][v];
                    hi[v] = (2 * rp + 1 < RT) ? W[2 * rp + 1 < RT ? 2 * rp + 1 : 0][v] : 0.0f;
                }
                wb[rp] = pack8(lo, hi);
            }
            res_part = 0.0f;
            // fragments of v = A w, read from LDS in batches of KB tile pairs
            constexpr int KB = NPP >= 4 ? NPP / 2 : NPP;
            halfx8 f2[2 * KB][RP];
#pragma unroll
            for (int s = 0; s < 2 * NPP; s += 2) {
                if ((s / 2) % KB == 0) {
#pragma unroll
                    for (int b = 0; b < 2 * KB; ++b)
#pragma unroll
                        for (int rp = 0; rp < RP; ++rp)
                            f2[b][rp] = (s + b < 2 * NPP) ? H2[((2 * pp0 + s + b) * RP + rp) * 64] : f2[b][rp];
                    __builtin_amdgcn_sched_barrier(0);
                }
                const int sb = s % (2 * KB);
                floatx4 Va = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                floatx4 Vb = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int rp = 0; rp < RP; ++rp) {
                    Va = mfma16h(f2[sb][rp], wb[rp], Va);
                    Vb = mfma16h(f2[sb + 1][rp], wb[rp], Vb);
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const floatx4 Vt = h ? Vb : Va;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float yo = y[s + h][v];
                        const float yn = gk[s + h][v] - Vt[v];
                        res_part = fmaxf(res_part, fabsf(yn - yo));
                        u[s + h][v] = fmaf(-Vt[v], ib, u[s + h][v]);
                        y[s + h][v] = yn;
                    }
                }
            }
        } else {
            // v = A w on 16x16x4 FP32 MFMAs from the refresh fragments in
            // HBM (L2), one element tile at a time with the next tile's
            // loads in flight under this tile's MFMAs; a tile past PT reads
            // the last real tile and contributes 0
            res_part = 0.0f;
            const __amdgpu_buffer_rsrc_t f2r =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(f2glob), 0, PT * RT * 1024, kBufWord3);
            floatx4 fb[2][RT];
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) fb[0][mt] = buf_load4(f2r, 16 * lane, (min(2 * pp0, PT - 1) * RT + mt) * 1024);
#pragma unroll
            for (int s = 0; s < 2 * NPP; ++s) {
                const int cur = s & 1;
                if (s + 1 < 2 * NPP) {
                    const int t = min(2 * pp0 + s + 1, PT - 1);
#pragma unroll
                    for (int mt = 0; mt < RT; ++mt) fb[cur ^ 1][mt] = buf_load4(f2r, 16 * lane, (t * RT + mt) * 1024);
                }
                floatx4 Vq = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (4 * mt + v < KS) Vq = mfma4(fb[cur][mt][v], W[mt][v], Vq);
                const bool real = 2 * pp0 + s < PT;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float Vt = real ? Vq[v] : 0.0f;
                    const float yo = y[s][v];
                    const float gs = __builtin_amdgcn_fmed3f(fmaf(beta, u[s][v], yo), -1.0f, 1.0f);
                    const float yn = gs - Vt;
                    res_part = fmaxf(res_part, fabsf(yn - yo));
                    u[s][v] = fmaf(-Vt, ib, u[s][v]);
                    y[s][v] = yn;
                }
            }
        }
        inv_beta_prev = fl ? 0.0f : inv_beta;
        beta = fl ? beta : fminf(L.c.rho * beta, beta_bar);

        // FP32 residual refinement: u = x - A z from the input, two element
        // tiles at a time: their fragments and x are loaded from HBM (L2) in
        // one batch before any of their MFMAs, so the load latency is paid
        // once per batch (the compiler's own order waited once per rank tile)
        if (L.c.refresh > 0 && ((k + 1) % L.c.refresh) == 0) {
            if constexpr (H) {
                constexpr int QB = 2;
#pragma unroll
                for (int s0 = 0; s0 < 2 * NPP; s0 += QB) {
                    const int t0 = 2 * pp0 + s0;
                    if (t0 < PT) {                    // wave-uniform
                        floatx4 fa[QB][RT], xq[QB];
                        const floatx4 zero4 = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                        for (int h = 0; h < QB; ++h) {
                            const bool on = s0 + h < 2 * NPP && t0 + h < PT;
#pragma unroll
                            for (int mt = 0; mt < RT; ++mt) fa[h][mt] = on ? F2[((t0 + h) * RT + mt) * 64] : zero4;
                            xq[h] = on ? xslot[(t0 + h) * 64] : zero4;
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        floatx4 Az[QB];
#pragma unroll
                        for (int h = 0; h < QB; ++h) Az[h] = zero4;
#pragma unroll
                        for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                if (4 * mt + v < KS)
#pragma unroll
                                    for (int h = 0; h < QB; ++h) Az[h] = mfma4(fa[h][mt][v], z[mt][v], Az[h]);
#pragma unroll
                        for (int h = 0; h < QB; ++h) {
                            if (s0 + h < 2 * NPP && t0 + h < PT) {
#pragma unroll
                                for (int v = 0; v < 4; ++v) u[s0 + h][v] = xq[h][v] - Az[h][v];
                            }
                        }
                    }
                }
            } else {
                // one element tile at a time, the next tile's fragments and x
                // in flight under this tile's MFMAs (x of an idle tile: the
                // first tile's slot, never used)
                const __amdgpu_buffer_rsrc_t f2r =
                    __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(f2glob), 0, PT * RT * 1024, kBufWord3);
                const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
                    xslot_base, 0, PT * 1024, kBufWord3);
                floatx4 fr[2][RT], xv[2];
                {
                    const int t = min(2 * pp0, PT - 1);
#pragma unroll
                    for (int mt = 0; mt < RT; ++mt) fr[0][mt] = buf_load4(f2r, 16 * lane, (t * RT + mt) * 1024);
                    xv[0] = buf_load4(xr, 16 * lane, t * 1024);
                }
#pragma unroll
                for (int s = 0; s < 2 * NPP; ++s) {
                    const int cur = s & 1;
                    if (s + 1 < 2 * NPP) {
                        const int t = min(2 * pp0 + s + 1, PT - 1);
#pragma unroll
                        for (int mt = 0; mt < RT; ++mt) fr[cur ^ 1][mt] = buf_load4(f2r, 16 * lane, (t * RT + mt) * 1024);
                        xv[cur ^ 1] = buf_load4(xr, 16 * lane, t * 1024);
                    }
                    floatx4 Az = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (4 * mt + v < KS) Az = mfma4(fr[cur][mt][v], z[mt][v], Az);
                    const bool real = 2 * pp0 + s < PT;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        u[s][v] = real ? xv[cur][v] - Az[v] : u[s][v];
                }
            }
        }
        if (fresh_m != 0) {
            // the dual state of a column set up in this step starts at 0
#pragma unroll
            for (int s = 0; s < 2 * NPP; ++s)
#pragma unroll
                for (int v = 0; v < 4; ++v) y[s][v] = fl ? 0.0f : y[s][v];
            res_part = fl ? 0.0f : res_part;
            fresh_m = 0;
        }

        // refill point: stopped columns store their result and take the next
        // regressions of the sequence, in column order
        if ((k + 2) % RA == 0 && pend) {
            const uint32_t cm = (uint32_t)(__ballot(done) & 0xFFFFull);   // lanes 0..15: one per column
            if (cm != 0) {                            // wave-uniform
                const bool fr = (cm >> c) & 1;
                if (fr) store();
                const int64_t pos = seq_pos(cursor + __popc(cm & ((1u << c) - 1u)));
                float xinf = 0.0f, xx = 0.0f;
                if (fr) {
                    j = pos < jend ? pos : kNone;
                    valid = j < jend;
                    roff = 0;
                    if (valid) {
                        const int64_t ri = reg_idx[j];
                        if (ri >= 0 && ri < reg_bound) roff = ri * reg_stride;
                        else valid = false;
                    }
#pragma unroll
                    for (int mt = 0; mt < RT; ++mt) z[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
                    // every load issued before the first use (an element outside
                    // the block reads M[0] and is replaced by 0): one memory
                    // latency per refill
#pragma unroll
                    for (int s = 0; s < 2 * NPP; ++s)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int64_t e = eoff[16 * (2 * pp0 + s) + 4 * g + v];
                            const bool ok = valid && e >= 0;
                            const int64_t off = ok ? roff + (TPB == 2 ? e * elem_stride : e) : 0;
                            const float x = M[off];
                            u[s][v] = ok ? x : 0.0f;
                        }
#pragma unroll
                    for (int s = 0; s < 2 * NPP; ++s) {
                        const int t = 2 * pp0 + s;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            y[s][v] = 0.0f;
                            xinf = fmaxf(xinf, fabsf(u[s][v]));
                            xx = fmaf(u[s][v], u[s][v], xx);
                        }
                        if (t < PT) xslot[t * 64] = floatx4{u[s][0], u[s][1], u[s][2], u[s][3]};
                    }
                }
                // the column's norms over this quarter, published for the next step
                xinf = colmax(xinf);
                xx = colsum(xx);
                if (fr) {
                    mine[0] = xinf;
                    mine[(NV - 1) * 64] = xx;
                }
                fresh_m = __ballot(fr);
                cursor += __popc(cm);
            }
        }
    }
    store();                                          // the regressions still held
}



// FP32 refresh fragments of the precision form (and of the FP32 quarter-tile
// form's v = A w), for classes whose LDS cannot hold them:
// out[(t RT + mt) 256 + lane 4 + v] = A[16 t + c][16 mt + 4 v + g].
static __global__ void prep_frag32(const double *__restrict__ A, int lda, int p, int r, int PT, int RT,
                            float *__restrict__ out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= PT * RT * 256) return;
    const int v = idx & 3, ln = (idx >> 2) & 63, tm = idx >> 8;
    const int t = tm / RT, mt = tm - t * RT;
    const int g = ln >> 4, c = ln & 15;
    const int e = 16 * t + c, k = 16 * mt + 4 * v + g;
    out[idx] = (e < p && k < r) ? (float)A[e + (int64_t)k * lda] : 0.0f;
}

template <int PT, int KS>
int launch_pt_ks(rpca_ctx *ctx, const FilterLaunch &L, int nblocks, bool split, hipStream_t stream)
{
    if constexpr (split_built(PT, KS)) {
        if (split && L.c.precision == 0) {
            hipLaunchKernelGGL((l1_filter_split_kernel<PT, KS>), dim3(nblocks), dim3(kWavesPerBlock * 64),
                               0, stream, L);
            RPCA_HIP_TRY(ctx, hipGetLastError());
            return RPCA_OK;
        }
    }
    if (split) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: split form not built for this class");
    if constexpr (half_form(PT)) {
        if (L.c.precision == 1) {
            // quarter-tile persistent variant: refresh fragments in HBM; one
            // or two tiles per workgroup (chosen by the launcher)
            auto go = [&](auto tpb_tag) -> int {
                constexpr int TPB = decltype(tpb_tag)::value;
                const size_t lds = lds_bytes_f16q(PT, KS, TPB);
                // once per process (thread-safe static initialisation), before
                // any launch can be captured in a graph
                static const hipError_t attr =
                    hipFuncSetAttribute((const void *)l1_filter_kernel_quarter<PT, KS, TPB, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                RPCA_HIP_TRY(ctx, attr);
                hipLaunchKernelGGL((l1_filter_kernel_quarter<PT, KS, TPB, true>), dim3(nblocks),
                                   dim3(TPB * kWavesPerBlock * 64), lds, stream, L);
                RPCA_HIP_TRY(ctx, hipGetLastError());
                return RPCA_OK;
            };
            return L.qtiles == 2 ? go(std::integral_constant<int, 2>{}) : go(std::integral_constant<int, 1>{});
        }
    } else if (L.c.precision == 1) {
        // the FP32 refresh fragments live in HBM when the launcher prepared them
        const size_t lds = lds_bytes_f16(PT, KS, L.frag32[0] == nullptr);
        static const hipError_t attr = hipFuncSetAttribute(
            (const void *)l1_filter_kernel_f16<PT, KS>, hipFuncAttributeMaxDynamicSharedMemorySize,
            (int)lds_bytes_f16(PT, KS, true) > (int)ctx->max_lds ? (int)lds_bytes_f16(PT, KS, false)
                                                                 : (int)lds_bytes_f16(PT, KS, true));
        RPCA_HIP_TRY(ctx, attr);
        hipLaunchKernelGGL((l1_filter_kernel_f16<PT, KS>), dim3(nblocks), dim3(kWavesPerBlock * 64),
                           lds, stream, L);
        RPCA_HIP_TRY(ctx, hipGetLastError());
        return RPCA_OK;
    }
    if constexpr (half_form(PT) && PT > 19) {
        // FP32 beyond the tile classes: the quarter-tile shape with FP32
        // contractions (v = A w from the fragments the launcher prepared)
        if (!L.frag32[0] || !L.frag32[1])
            return set_status(ctx, RPCA_ERR_ARG, "filter: FP32 quarter-tile form without its fragments");
        auto go = [&](auto tpb_tag) -> int {
            constexpr int TPB = decltype(tpb_tag)::value;
            const size_t lds = lds_bytes_q32(PT, KS, TPB);
            static const hipError_t attr =
                hipFuncSetAttribute((const void *)l1_filter_kernel_quarter<PT, KS, TPB, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            RPCA_HIP_TRY(ctx, attr);
            hipLaunchKernelGGL((l1_filter_kernel_quarter<PT, KS, TPB, false>), dim3(nblocks),
                               dim3(TPB * kWavesPerBlock * 64), lds, stream, L);
            RPCA_HIP_TRY(ctx, hipGetLastError());
            return RPCA_OK;
        };
        return L.qtiles == 2 ? go(std::integral_constant<int, 2>{}) : go(std::integral_constant<int, 1>{});
    } else if constexpr (PT <= 19) {
        const size_t lds = lds_bytes(PT, KS);
        static const hipError_t attr = hipFuncSetAttribute(
            (const void *)l1_filter_kernel<PT, KS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        RPCA_HIP_TRY(ctx, attr);
        hipLaunchKernelGGL((l1_filter_kernel<PT, KS>), dim3(nblocks), dim3(kWavesPerBlock * 64),
                           lds, stream, L);
        RPCA_HIP_TRY(ctx, hipGetLastError());
        return RPCA_OK;
    } else {
        return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: FP32 form not built for this p class");
    }
}

// Launch the class (PT, KS); defined in filter_inst.hip, one object per PT.
template <int PT>
int launch_filter_pt(rpca_ctx *ctx, int KS, const FilterLaunch &L, int nblocks, bool split,
                     hipStream_t stream)
{
    switch (KS) {
    case 1: return launch_pt_ks<PT, 1>(ctx, L, nblocks, split, stream);
    case 2: return launch_pt_ks<PT, 2>(ctx, L, nblocks, split, stream);
    case 3: return launch_pt_ks<PT, 3>(ctx, L, nblocks, split, stream);
    case 4: return launch_pt_ks<PT, 4>(ctx, L, nblocks, split, stream);
    case 5: return launch_pt_ks<PT, 5>(ctx, L, nblocks, split, stream);
    case 6: return launch_pt_ks<PT, 6>(ctx, L, nblocks, split, stream);
    case 8: return launch_pt_ks<PT, 8>(ctx, L, nblocks, split, stream);
    case 10: return launch_pt_ks<PT, 10>(ctx, L, nblocks, split, stream);
    case 13: return launch_pt_ks<PT, 13>(ctx, L, nblocks, split, stream);
    case 16: return launch_pt_ks<PT, 16>(ctx, L, nblocks, split, stream);
    default: return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: rank class not built");
    }
}

} // namespace filterk
