// Batched form of steps 3-5 of Algorithm 2 over many independent problems.
//
// Filter, lane form.  For small seeds (p <= 80, r <= 8: e.g. the 10r x 10r
// seeds of low-rank video backgrounds) a 16-regression tile wastes most of a
// 16x16 MFMA on the rank axis.  Here every lane owns one regression and both
// contractions of the clip form of Algorithm 1 (see filter_kernel.h)
//     w = A^T g   and   v = A w
// run on v_mfma_f32_4x4x1_16b_f32: 16 blocks of 4x4x1 per instruction, block
// b serving lanes 4b..4b+3.  Measured lane layout: the A operand of row i of
// block b comes from lane 4b+i, the B operand of column j from lane 4b+j, and
// accumulator register i of lane 4b+j holds D_b[i][j].  So with the basis in
// the A operand (identical in every block) and the lane's own vector in the
// B operand, each lane receives its own product:
//   * w:  K-step = element e, A = A[e][4 rb + i], B = g_lane[e]
//         -> register i of lane l holds w_l[4 rb + i];
//   * v:  K-step = rank k, A = A[4 t + i][k], B = w_l[k]
//         -> register i of lane l holds v_l[4 t + i].
// Nothing moves between lanes: u, y, g (p values each) and z (r values) are
// per-lane registers, the stopping test needs no reduction, and a regression
// of p elements costs ceil(r/4) p + ceil(p/4) r instructions of 8 cycles per
// 64 regressions.
//
// Scheduling.  One persistent kernel serves a work queue of items (64
// consecutive regressions of one side of one problem): each wave takes the
// next item with an atomic add on the queue head, re-stages the basis in its
// own LDS slice when the side changes, and leaves when the queue is empty,
// so every wave reaches the exit.  The host orders the items (costliest sides
// first by default) and resets the head with a kernel (graph-safe).
//
// Completion.  The factor assembly and the completion of every problem run as
// one launch each, with a table giving each workgroup its problem.
#include "recon_kernel.h"

#include <climits>

namespace batchk {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4x4(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

constexpr int kMaxP4 = kLaneMaxP / 4;   // 20 element quads
constexpr int kMaxRB = kLaneMaxR / 4;   // 2 rank blocks
constexpr int kWaves = 4;               // waves per workgroup
constexpr int kVC = 4;                  // element quads per chunk of v = A w

// Per-wave LDS slice: the basis in the two operand orders, the element
// offsets, and the lanes' x (XQ element quads per lane) for the refresh, which
// then reads x back from LDS instead of gathering it from M again.
// a1[(4 rb + i) S1 + e] = A[e][4 rb + i] with an odd number S1/4 of float4 per
// row (conflict-free ds_read_b128 of 4 rows); a2[e RR + k] = A[e][k] with
// RR = 4 RB.
template <int XQ>
struct WaveLds {
    static constexpr int kXQ = XQ;
    float a1[kMaxRB * 4 * 4 * (kMaxP4 | 1)];
    float a2[kMaxP4 * 4 * 4 * kMaxRB];
    int64_t eoff[kMaxP4 * 4];            // element offsets in M (floats), -1 = padding
    floatx4 xc[XQ][64];                  // x of lane l's quad t at xc[t][l]
};

// Built classes (P4L element quads per lane, LPR lanes per regression); the
// rank blocks RB = ceil(r / 4) in {1, 2} double the list.  A regression of p
// elements runs in the smallest class of its LPR with 4 LPR P4L >= p.
struct LaneClassDesc {
    int p4l, lpr;
};
// At most 8 quads per lane: with every class in one kernel (whose register
// budget is that of its largest branch) 10 quads spill at two waves per SIMD.
constexpr LaneClassDesc kLaneCls[] = {
    {1, 1}, {2, 1}, {3, 1}, {4, 1}, {5, 1}, {6, 1}, {8, 1},               // p <= 32
    {2, 2}, {3, 2}, {4, 2}, {5, 2}, {6, 2}, {7, 2}, {8, 2},               // p <= 64
    {1, 4}, {2, 4}, {3, 4}, {4, 4}, {5, 4},                               // p <= 80
};
constexpr int kNumLaneCls = sizeof(kLaneCls) / sizeof(kLaneCls[0]);

__device__ __forceinline__ void wave_lds_sync()
{
    // LDS operations of one wave complete in order; this keeps the compiler
    // from moving LDS accesses across the re-staging of the slice.
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Sum / max over the LPR lanes that share a regression (lanes reg, reg + 64/LPR, ...):
// v_permlane16_swap / v_permlane32_swap exchange rows of 16 (32) lanes inside
// the VALU, giving each lane v of lane l ^ 16 (l ^ 32) next to its own, the
// same two operands as an xor shuffle (same result), without its LDS round trip.
__device__ __forceinline__ float xor16_sum(float v)
{
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}
__device__ __forceinline__ float xor32_sum(float v)
{
    auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}
__device__ __forceinline__ float xor16_max(float v)
{
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
}
__device__ __forceinline__ float xor32_max(float v)
{
    auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
}
template <int LPR>
__device__ __forceinline__ float part_sum(float v)
{
    if constexpr (LPR >= 4) v = xor16_sum(v);
    if constexpr (LPR >= 2) v = xor32_sum(v);
    return v;
}
template <int LPR>
__device__ __forceinline__ float part_max(float v)
{
    if constexpr (LPR >= 4) v = xor16_max(v);
    if constexpr (LPR >= 2) v = xor32_max(v);
    return v;
}

// Element x_e of a lane's regression, 0 for padding elements, bad element
// indices and invalid lanes.  The element's offset is wave-uniform: it is
// read from LDS and moved to scalar registers, and the lane's regression
// offset voff is a 32-bit byte offset, so the load is the scalar-base +
// vector-offset form and every element shares one VGPR of address.  Masked
// lanes read an in-bounds element and select 0 (no branch per element).
// With LPR > 1 the lanes of different parts read different elements: e is
// then lane-dependent and the offset stays in VGPRs.
template <bool UNIFORM>
__device__ __forceinline__ float load_x(const float *M, const int64_t *eoff, int e, uint32_t voff,
                                        bool valid)
{
    int64_t off = eoff[e];
    if constexpr (UNIFORM) {
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)off);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)off >> 32));
        off = (int64_t)(((uint64_t)hi << 32) | lo);
    }
    const bool ok = off >= 0;
    const char *base = reinterpret_cast<const char *>(M + (ok ? off : 0));
    const float x = *reinterpret_cast<const float *>(base + voff);
    return (ok && valid) ? x : 0.0f;
}

// One item: regressions first .. first + 64/LPR - 1 of side s.  Lane l serves
// regression l mod (64/LPR) on its part l div (64/LPR) of the elements: 4 P4L
// consecutive elements, whose u, y, g sit in VGPRs (x is re-read from M by the
// refresh).  The lanes of one 4x4 MFMA block always belong to one part, so
// the K-step element is common to the block; partial w and the residual are
// summed / maxed over the parts with xor shuffles.
template <int P4L, int RB, int LPR, class WL>
__device__ __forceinline__ void lane_item(const LaneSide &s, int64_t first, int lane, WL &w,
                                          bool restage, const FilterConsts &C)
{
    static_assert(P4L <= WL::kXQ, "the wave's x cache holds every quad of the class");
    constexpr int NR = 64 / LPR;        // regressions per item
    constexpr int PL = 4 * P4L;         // elements per lane
    constexpr int PP = LPR * PL;        // padded p
    constexpr int S1 = 4 * ((PP / 4) | 1);   // a1 row stride
    constexpr int RR = 4 * RB;          // padded r
    constexpr int NCH = 1;              // accumulator chains per rank block of w (one: the adds
                                        // joining more cost more than the latency they hide)
    const int p = s.p, r = s.r;
    const int q4 = lane & 3;
    const int reg = lane % NR, part = lane / NR;
    const int ebase = part * PL;

    if (restage) {
        wave_lds_sync();
        for (int idx = lane; idx < RB * 4 * S1; idx += 64) {
            const int k = idx / S1, e = idx - k * S1;
            w.a1[idx] = (e < p && k < r) ? (float)s.A[e + (int64_t)k * s.lda] : 0.0f;
        }
        for (int idx = lane; idx < PP * RR; idx += 64) {
            const int e = idx / RR, k = idx - e * RR;
            w.a2[idx] = (e < p && k < r) ? (float)s.A[e + (int64_t)k * s.lda] : 0.0f;
        }
        for (int e = lane; e < PP; e += 64) {
            int64_t off = -1;
            if (e < p) {
                const int64_t ei = s.elem_idx[e];
                if (ei >= 0 && ei < s.elem_bound) off = ei * s.elem_stride;
            }
            w.eoff[e] = off;
        }
        wave_lds_sync();
    }

    // the host admits a side to the lane form only if every regression's
    // offset reg_idx * reg_stride * 4 fits in 32 bits
    const int64_t j = first + reg;
    bool valid = j < s.nreg;
    uint32_t voff = 0;
    if (valid) {
        const int64_t ri = s.reg_idx[j];
        if (ri >= 0 && ri < s.reg_bound) voff = (uint32_t)(ri * s.reg_stride * 4);
        else valid = false;
    }
    const float *M = s.M;
    const int64_t *eoff = w.eoff + ebase;

    // ---- x, its norms, the starting state (u = x, y = 0, z = 0)
    float u[P4L][4], y[P4L][4], gk[P4L][4];
    float xinf = 0.0f, xx = 0.0f;
#pragma unroll
    for (int t = 0; t < P4L; ++t) {
        floatx4 xq;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float x = load_x<LPR == 1>(M, eoff, 4 * t + i, voff, valid);
            xq[i] = x;
            u[t][i] = x;
            y[t][i] = 0.0f;
            xinf = fmaxf(xinf, fabsf(x));
            xx = fmaf(x, x, xx);
        }
        w.xc[t][lane] = xq;
        __builtin_amdgcn_sched_barrier(0);
    }
    xinf = part_max<LPR>(xinf);
    xx = part_sum<LPR>(xx);
    float beta = xx > 0.0f ? C.beta0_scale / sqrtf(xx) : 1.0f;
    const float beta_bar = C.beta_max_scale * beta;
    const float tol = C.eps * xinf;
    const bool bad = valid && nonfinite_norm(xx);     // x holds Inf / NaN
    bool done = !(valid && xinf > 0.0f) || bad;
    int K = 0;
    floatx4 z[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) z[rb] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    const floatx4 *A1 = reinterpret_cast<const floatx4 *>(w.a1);
    const floatx4 *A2 = reinterpret_cast<const floatx4 *>(w.a2);

    for (int k = 0; k < C.max_iter; ++k) {
        if (!__any(!done)) break;                                   // wave-uniform
        asm volatile("" ::: "memory");   // the basis is re-read from LDS each step
        // The lane's offsets into the two fragment arrays, opaque to the
        // optimizer: every fragment address is then formed inside the step
        // (an immediate offset from these) instead of being hoisted out of
        // the loop into one live VGPR per address.
        uint32_t q1 = (uint32_t)(q4 * S1 + ebase) / 4, q2 = (uint32_t)((ebase + q4) * RR) / 4;
        asm volatile("" : "+v"(q1), "+v"(q2));
        const floatx4 *F1 = A1 + q1;
        const floatx4 *F2 = A2 + q2;

        // ---- g = clip(beta u + y, -1, 1) and the lane's part of w = A^T g
        floatx4 acc[RB][NCH];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int c = 0; c < NCH; ++c) acc[rb][c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        // basis fragments one quad ahead; the scheduling barrier per quad keeps
        // the compiler from hoisting every quad's loads (register pressure)
        floatx4 an[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) an[rb] = F1[(4 * rb * S1) / 4];
#pragma unroll
        for (int t = 0; t < P4L; ++t) {
            floatx4 a[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                a[rb] = an[rb];
                if (t + 1 < P4L) an[rb] = F1[(4 * rb * S1 + 4 * (t + 1)) / 4];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
                gk[t][i] = __builtin_amdgcn_fmed3f(fmaf(beta, u[t][i], y[t][i]), -1.0f, 1.0f);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[rb][i % NCH] = mfma4x4(a[rb][i], gk[t][i], acc[rb][i % NCH]);
            __builtin_amdgcn_sched_barrier(0);
        }
        floatx4 W[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            W[rb] = acc[rb][0];
#pragma unroll
            for (int c = 1; c < NCH; ++c) W[rb] += acc[rb][c];
#pragma unroll
            for (int i = 0; i < 4; ++i) W[rb][i] = part_sum<LPR>(W[rb][i]);
        }

        // A converged regression keeps z and u frozen through a zero step size.
        const float inv_beta = 1.0f / beta;
        const float ib = done ? 0.0f : inv_beta;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) z[rb][i] = fmaf(W[rb][i], ib, z[rb][i]);

        // ---- v = A w on the lane's elements in chunks of kVC quads, then the
        // dual and residual update
        float res = 0.0f;
#pragma unroll
        for (int t0 = 0; t0 < P4L; t0 += kVC) {
            floatx4 D[kVC];
#pragma unroll
            for (int c = 0; c < kVC; ++c) D[c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < RB; ++kb) {
                floatx4 a[kVC];
#pragma unroll
                for (int c = 0; c < kVC; ++c)
                    if (t0 + c < P4L) a[c] = F2[(4 * (t0 + c) * RR + 4 * kb) / 4];
                // ranks >= r have zero basis columns and zero w: the padded
                // K-steps add exact zeros, and straight-line code keeps the
                // register allocation in one block
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                    for (int c = 0; c < kVC; ++c)
                        if (t0 + c < P4L) D[c] = mfma4x4(a[c][kk], W[kb][kk], D[c]);
            }
#pragma unroll
            for (int c = 0; c < kVC; ++c) {
                const int t = t0 + c;
                if (t < P4L) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float yn = gk[t][i] - D[c][i];
                        res = fmaxf(res, fabsf(yn - y[t][i]));
                        u[t][i] = fmaf(-D[c][i], ib, u[t][i]);
                        y[t][i] = yn;
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        res = part_max<LPR>(res);
        if (!done) {
            ++K;
            if (!(res * inv_beta >= tol)) done = true;   // ||x-Az-e||_inf < eps ||x||_inf
        }
        beta = fminf(C.rho * beta, beta_bar);

        // ---- periodic u = x - A z from the input, against FP32 drift
        if (C.refresh > 0 && ((k + 1) % C.refresh) == 0) {
            asm volatile("" ::: "memory");
#pragma unroll
            for (int t0 = 0; t0 < P4L; t0 += kVC) {
                floatx4 D[kVC];
#pragma unroll
                for (int c = 0; c < kVC; ++c) D[c] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kb = 0; kb < RB; ++kb) {
                    floatx4 a[kVC];
#pragma unroll
                    for (int c = 0; c < kVC; ++c)
                        if (t0 + c < P4L) a[c] = F2[(4 * (t0 + c) * RR + 4 * kb) / 4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int c = 0; c < kVC; ++c)
                            if (t0 + c < P4L) D[c] = mfma4x4(a[c][kk], z[kb][kk], D[c]);
                }
#pragma unroll
                for (int c = 0; c < kVC; ++c) {
                    const int t = t0 + c;
                    if (t < P4L) {
                        const floatx4 xq = w.xc[t][lane];
#pragma unroll
                        for (int i = 0; i < 4; ++i) u[t][i] = xq[i] - D[c][i];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    if (part == 0) {
        if (valid) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int kk = 4 * rb + i;
                    if (kk < r) s.Z[kk + j * s.ldz] = bad ? __builtin_nanf("") : z[rb][i];
                }
        }
        if (j < s.nreg && s.iters) s.iters[j] = !valid ? RPCA_ITERS_BAD_INDEX
                                                : (bad ? RPCA_ITERS_NONFINITE : (done ? K : -C.max_iter));
    }
}

// Register group of each class case (index 2 ci + rb - 1).  A kernel's
// register budget is that of its largest branch: one kernel holding every
// class needs all 256 VGPRs (two waves per SIMD) and spills a few.  Group 0
// is a set of four-lane classes that compiled together fit 168 VGPRs without
// spilling (three waves per SIMD): among them p4l 5 with two rank blocks, the
// class of the longest regressions (p 65-80, r 5-8) and most of the batched
// workload's work.  Each group has its own kernel and work queue.  (Larger
// sets were tried: every one that fits 168 registers alone per class spilled
// 17-75 registers once compiled together.)
constexpr int8_t kLaneGroup[2 * kNumLaneCls] = {
    1, 1,  1, 1,  1, 1,  1, 1,  1, 1,  1, 1,  1, 1,     // lpr 1: p4l 1 2 3 4 5 6 8
    1, 1,  1, 1,  1, 1,  1, 1,  1, 1,  1, 1,  1, 1,     // lpr 2: p4l 2 3 4 5 6 7 8
    1, 1,  1, 0,  1, 0,  0, 0,  1, 0,                   // lpr 4: p4l 1 2 3 4 5
};

#define LANE_CASE(ci, rb)                                                                  \
    case 2 * (ci) + (rb) - 1:                                                              \
        if constexpr (kLaneGroup[2 * (ci) + (rb) - 1] == G)                                \
            lane_item<kLaneCls[ci].p4l, rb, kLaneCls[ci].lpr>(s, first, lane, w, restage, C); \
        break;
#define LANE_CASES(ci) LANE_CASE(ci, 1) LANE_CASE(ci, 2)

template <int G>
__global__ void __launch_bounds__(kWaves * 64) __attribute__((amdgpu_waves_per_eu(G == 0 ? 3 : 2)))
lane_filter_kernel(const LaneSide *__restrict__ sides, const int32_t *__restrict__ items,
                   int32_t nitems, uint32_t *counter, FilterConsts C)
{
    // x cache: the largest class of the group (5 quads per lane in group 0, 8 in 1)
    typedef WaveLds<G == 0 ? 5 : 8> Lds;
    __shared__ Lds lds[kWaves];
    const int lane = threadIdx.x & 63;
    Lds &w = lds[threadIdx.x >> 6];
    int cached = -1;
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(counter, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= (uint32_t)nitems) break;               // every wave leaves here
        const int sidx = items[2 * it];
        const int64_t first = items[2 * it + 1];
        const LaneSide &s = sides[sidx];
        const bool restage = sidx != cached;
        cached = sidx;
        switch (s.cls) {
            LANE_CASES(0) LANE_CASES(1) LANE_CASES(2) LANE_CASES(3) LANE_CASES(4) LANE_CASES(5)
            LANE_CASES(6) LANE_CASES(7) LANE_CASES(8) LANE_CASES(9) LANE_CASES(10) LANE_CASES(11)
            LANE_CASES(12) LANE_CASES(13) LANE_CASES(14) LANE_CASES(15) LANE_CASES(16)
            LANE_CASES(17) LANE_CASES(18)
        default: break;                                  // rejected on the host
        }                                                // (other group: never queued here)
    }
}
#undef LANE_CASES
#undef LANE_CASE
static_assert(kNumLaneCls == 19, "LANE_CASES list covers every class");

__global__ void reset_counters(uint32_t *counter)
{
    if (threadIdx.x < 2) counter[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------- completion
__global__ void __launch_bounds__(reconk::kAssembleThreads)
batch_assemble(const ReconJob *__restrict__ jobs, const int32_t *__restrict__ block_job,
               const int64_t *__restrict__ block_first)
{
    __shared__ int64_t sidx[reconk::kIdxLds];
    const ReconJob &J = jobs[block_job[blockIdx.x]];
    reconk::assemble_block(block_first[blockIdx.x], (J.m + J.n) * (J.R4 / 4), sidx, J.seed_rows, J.p,
                           J.seed_cols, J.q, J.U,
                           J.sigma, J.V, J.r, J.Qt, J.Pt, J.m, J.n, J.R4,
                           const_cast<float *>(J.F), const_cast<float *>(J.G));
}

__global__ void __launch_bounds__(64)
batch_reconstruct(const ReconJob *__restrict__ jobs, const int32_t *__restrict__ block_job,
                  const uint32_t *__restrict__ block_local)
{
    const ReconJob &J = jobs[block_job[blockIdx.x]];
    const uint32_t local = block_local[blockIdx.x];
    const uint32_t bx = local % J.row_blocks, by = local / J.row_blocks;
    const int lane = threadIdx.x;
    if (J.R4 == 4) {
        if (J.vec) reconk::recon_wave<4, true>(J.M, J.ldm, J.F, J.G, J.m, J.n, J.L, J.ldl, J.S, J.lds, bx, by, J.col_parts, lane);
        else reconk::recon_wave<4, false>(J.M, J.ldm, J.F, J.G, J.m, J.n, J.L, J.ldl, J.S, J.lds, bx, by, J.col_parts, lane);
    } else {
        if (J.vec) reconk::recon_wave<8, true>(J.M, J.ldm, J.F, J.G, J.m, J.n, J.L, J.ldl, J.S, J.lds, bx, by, J.col_parts, lane);
        else reconk::recon_wave<8, false>(J.M, J.ldm, J.F, J.G, J.m, J.n, J.L, J.ldl, J.S, J.lds, bx, by, J.col_parts, lane);
    }
}

} // namespace batchk

using namespace batchk;

int lane_class(int p, int r, int lpr)
{
    if (p < 1 || r < 1 || p > kLaneMaxP || r > kLaneMaxR) return -1;
    for (int i = 0; i < kNumLaneCls; ++i)
        if (kLaneCls[i].lpr == lpr && 4 * kLaneCls[i].lpr * kLaneCls[i].p4l >= p)
            return 2 * i + (r + 3) / 4 - 1;
    return -1;
}

int lane_regs_per_item(int cls) { return 64 / kLaneCls[cls / 2].lpr; }

int lane_group(int cls) { return kLaneGroup[cls]; }

int launch_lane_filter(rpca_ctx *ctx, const BatchTables &t, const FilterConsts &c,
                       hipStream_t stream)
{
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, stream, t.counter);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    // With both groups present, the second runs on the second stream, so its
    // waves take the CUs that the first group's waves leave as its queue
    // drains.  The queues have counters of their own and no wave waits on
    // another, so the two grids finish in any order of residency.
    const bool both = t.nitems0 > 0 && t.nitems > t.nitems0;
    hipStream_t s1 = stream;
    if (both) {
        int st = ensure_aux(ctx);
        if (st != RPCA_OK) return st;
        RPCA_HIP_TRY(ctx, hipEventRecord(ctx->pev[0], stream));
        RPCA_HIP_TRY(ctx, hipStreamWaitEvent(ctx->aux, ctx->pev[0], 0));
        s1 = ctx->aux;
    }
    if (t.nitems0 > 0) {
        const int blocks = (t.grid_waves[0] + kWaves - 1) / kWaves;
        hipLaunchKernelGGL(lane_filter_kernel<0>, dim3((unsigned)blocks), dim3(kWaves * 64), 0, stream,
                           t.sides, t.items, t.nitems0, t.counter, c);
        RPCA_HIP_TRY(ctx, hipGetLastError());
    }
    if (t.nitems > t.nitems0) {
        const int blocks = (t.grid_waves[1] + kWaves - 1) / kWaves;
        hipLaunchKernelGGL(lane_filter_kernel<1>, dim3((unsigned)blocks), dim3(kWaves * 64), 0, s1,
                           t.sides, t.items + 2 * (int64_t)t.nitems0, t.nitems - t.nitems0, t.counter + 1, c);
        RPCA_HIP_TRY(ctx, hipGetLastError());
    }
    if (both) {
        RPCA_HIP_TRY(ctx, hipEventRecord(ctx->pev[1], ctx->aux));
        RPCA_HIP_TRY(ctx, hipStreamWaitEvent(stream, ctx->pev[1], 0));
    }
    return RPCA_OK;
}

int launch_batch_reconstruct(rpca_ctx *ctx, const BatchTables &t, hipStream_t stream)
{
    if (t.asm_blocks > 0) {
        hipLaunchKernelGGL(batch_assemble, dim3((unsigned)t.asm_blocks),
                           dim3(reconk::kAssembleThreads), 0, stream, t.jobs, t.asm_block_job,
                           t.asm_block_first);
        RPCA_HIP_TRY(ctx, hipGetLastError());
    }
    if (t.rec_blocks > 0) {
        if (t.rec_lds_bytes > 0) {
            // the reservation only limits residency; the kernel does not touch it
            // once per process (thread-safe static initialisation), before any
            // launch can be captured in a graph
            static const hipError_t attr =
                hipFuncSetAttribute((const void *)batch_reconstruct, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(ctx->max_lds ? ctx->max_lds : 65536));
            RPCA_HIP_TRY(ctx, attr);
        }
        hipLaunchKernelGGL(batch_reconstruct, dim3((unsigned)t.rec_blocks), dim3(64),
                           (size_t)t.rec_lds_bytes, stream, t.jobs, t.rec_block_job, t.rec_block_local);
        RPCA_HIP_TRY(ctx, hipGetLastError());
    }
    return RPCA_OK;
}
