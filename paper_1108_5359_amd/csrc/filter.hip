// l1 filtering kernels: many independent regressions min ||x - A z||_1 with
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
//   * the two contractions w = A^T g and v = A w run on MFMA
//     v_mfma_f32_16x16x4_f32.  The per-regression state u, y (p x 16) sits in
//     VGPRs in the MFMA accumulator layout: lane l = 16 g + c holds rows
//     16 t + 4 g + v (v = 0..3) of regression column c for every 16-row tile t.
//     That layout is directly the B operand of both contractions once the
//     contraction index is permuted consistently in the A operand, so no
//     data moves between lanes except two xor-shuffles for ||.||_inf.
//   * A (FP64 in HBM) is converted once per workgroup into two FP32 copies in
//     LDS, stored in "fragment order" so that each MFMA's A operand is one
//     conflict-free ds_read_b128 per lane.
//   * beta, ||x||_inf, the stopping flag and the iteration count are per
//     regression (per lane column); converged columns are frozen by select,
//     never by branching around MFMA.
#include "rpca_internal.h"

#include <algorithm>
#include <cmath>
#include <climits>

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWavesPerBlock = 4;

struct FilterLaunch {
    FilterSide side[2];
    int32_t nblocks0;   // blocks of side 0; the rest belong to side 1
    FilterConsts c;
};

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 acc)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

__device__ __forceinline__ float clamp1(float t)
{
    return fminf(fmaxf(t, -1.0f), 1.0f);
}

// Max over the four lanes that share a regression column (c, c+16, c+32, c+48).
__device__ __forceinline__ float colmax(float v)
{
    v = fmaxf(v, __shfl_xor(v, 16));
    v = fmaxf(v, __shfl_xor(v, 32));
    return v;
}

__device__ __forceinline__ float colsum(float v)
{
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

template <int PT, int RT>
__global__ void __launch_bounds__(kWavesPerBlock * 64)
l1_filter_kernel(FilterLaunch L)
{
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
#undef SIDE

    // ---- stage the basis in LDS, in the two fragment orders -------------
    for (int idx = threadIdx.x; idx < PT * RT * 256; idx += kWavesPerBlock * 64) {
        const int v = idx & 3;
        const int ln = (idx >> 2) & 63;
        const int tm = idx >> 8;
        const int t = tm / RT, mt = tm - t * RT;
        const int g = ln >> 4, c = ln & 15;
        const int e1 = 16 * t + 4 * g + v, k1 = 16 * mt + c;          // A1: A[e1][k1]
        fragA1[idx] = (e1 < p && k1 < r) ? (float)A[e1 + (int64_t)k1 * lda] : 0.0f;
        const int e2 = 16 * t + c, k2 = 16 * mt + 4 * g + v;          // A2: A[e2][k2]
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
    const int64_t j = tile * 16 + c;
    if (tile * 16 >= nreg) return;     // whole wave idle (no barrier follows)

    bool valid = j < nreg;
    int64_t roff = 0;
    if (valid) {
        const int64_t ri = reg_idx[j];
        if (ri >= 0 && ri < reg_bound) roff = ri * reg_stride;
        else valid = false;
    }

    // ---- load x, its norms, and the starting state -----------------------
    float u[PT][4], y[PT][4];
    float xinf = 0.0f, xx = 0.0f;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t off = eoff[16 * t + 4 * g + v];
            const float x = (valid && off >= 0) ? M[roff + off] : 0.0f;
            u[t][v] = x;
            y[t][v] = 0.0f;
            xinf = fmaxf(xinf, fabsf(x));
            xx = fmaf(x, x, xx);
        }
    }
    xinf = colmax(xinf);
    xx = colsum(xx);

    float beta = xx > 0.0f ? L.c.beta0_scale / sqrtf(xx) : 1.0f;
    const float beta_bar = L.c.beta_max_scale * beta;
    const float tol = L.c.eps * xinf;
    bool done = !(valid && xinf > 0.0f);
    int K = 0;

    floatx4 z[RT];
#pragma unroll
    for (int mt = 0; mt < RT; ++mt) z[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    const floatx4 *F1 = reinterpret_cast<const floatx4 *>(fragA1) + lane;
    const floatx4 *F2 = reinterpret_cast<const floatx4 *>(fragA2) + lane;

    for (int k = 0; k < L.c.max_iter; ++k) {
        if (!__any(!done)) break;                                   // wave-uniform

        // w = A^T g   (g built tile by tile from u, y)
        floatx4 W[RT];
#pragma unroll
        for (int mt = 0; mt < RT; ++mt) W[mt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            float gv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) gv[v] = clamp1(fmaf(beta, u[t][v], y[t][v]));
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) {
                const floatx4 a = F1[(t * RT + mt) * 64];
#pragma unroll
                for (int v = 0; v < 4; ++v) W[mt] = mfma4(a[v], gv[v], W[mt]);
            }
        }

        const float ib = 1.0f / beta;
#pragma unroll
        for (int mt = 0; mt < RT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) z[mt][v] = done ? z[mt][v] : fmaf(W[mt][v], ib, z[mt][v]);

        // v = A w, then the dual / residual update, tile by tile
        float res = 0.0f;
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            floatx4 Vt = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int mt = 0; mt < RT; ++mt) {
                const floatx4 a = F2[(t * RT + mt) * 64];
#pragma unroll
                for (int v = 0; v < 4; ++v) Vt = mfma4(a[v], W[mt][v], Vt);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float gg = clamp1(fmaf(beta, u[t][v], y[t][v]));
                const float yn = gg - Vt[v];
                res = fmaxf(res, fabsf(yn - y[t][v]));
                u[t][v] = done ? u[t][v] : fmaf(-Vt[v], ib, u[t][v]);
                y[t][v] = done ? y[t][v] : yn;
            }
        }
        res = colmax(res);
        if (!done) {
            ++K;
            if (!(res * ib >= tol)) done = true;    // ||x-Az-e||_inf < eps ||x||_inf
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
                    for (int v = 0; v < 4; ++v) Az = mfma4(a[v], z[mt][v], Az);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t off = eoff[16 * t + 4 * g + v];
                    const float x = (valid && off >= 0) ? M[roff + off] : 0.0f;
                    u[t][v] = done ? u[t][v] : x - Az[v];
                }
            }
        }
    }

    if (j < nreg) {
        if (valid) {
#pragma unroll
            for (int mt = 0; mt < RT; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int kk = 16 * mt + 4 * g + v;
                    if (kk < r) Zout[kk + j * ldz] = z[mt][v];
                }
        }
        if (iters && g == 0)
            iters[j] = !valid ? INT_MIN : (done ? K : -L.c.max_iter);
    }
}

// Smallest built tile count >= need.
constexpr int kPT[] = {1, 2, 3, 4, 5, 7, 8, 10, 13, 16, 19};
constexpr int kNumPT = sizeof(kPT) / sizeof(kPT[0]);

size_t lds_bytes(int PT, int RT)
{
    return (size_t)2 * PT * RT * 256 * sizeof(float) + (size_t)PT * 16 * sizeof(int64_t);
}

int pick_pt(int p)
{
    const int need = (p + 15) / 16;
    for (int i = 0; i < kNumPT; ++i)
        if (kPT[i] >= need) return kPT[i];
    return -1;
}

template <int PT, int RT>
int launch_pt_rt(rpca_ctx *ctx, const FilterLaunch &L, int nblocks, hipStream_t stream)
{
    const size_t lds = lds_bytes(PT, RT);
    static bool attr_set[64] = {};
    const int dev = ctx->device & 63;
    if (!attr_set[dev]) {
        RPCA_HIP_TRY(ctx, hipFuncSetAttribute((const void *)l1_filter_kernel<PT, RT>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)lds));
        attr_set[dev] = true;
    }
    hipLaunchKernelGGL((l1_filter_kernel<PT, RT>), dim3(nblocks), dim3(kWavesPerBlock * 64), lds,
                       stream, L);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    return RPCA_OK;
}

template <int PT>
int launch_pt(rpca_ctx *ctx, int RT, const FilterLaunch &L, int nblocks, hipStream_t stream)
{
    switch (RT) {
    case 1: return launch_pt_rt<PT, 1>(ctx, L, nblocks, stream);
    case 2: return launch_pt_rt<PT, 2>(ctx, L, nblocks, stream);
    case 3: return launch_pt_rt<PT, 3>(ctx, L, nblocks, stream);
    case 4: return launch_pt_rt<PT, 4>(ctx, L, nblocks, stream);
    default: return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: rank above 64");
    }
}

} // namespace

bool filter_supported(rpca_ctx *ctx, int p, int r)
{
    if (p < 1 || r < 1 || r > 64) return false;
    const int PT = pick_pt(p);
    if (PT < 0) return false;
    const int RT = (r + 15) / 16;
    return lds_bytes(PT, RT) <= (ctx->max_lds ? ctx->max_lds : 65536);
}

bool filter_same_class(int p0, int r0, int p1, int r1)
{
    return pick_pt(p0) == pick_pt(p1) && (r0 + 15) / 16 == (r1 + 15) / 16;
}

int launch_filter(rpca_ctx *ctx, const FilterSide *sides, int nsides, const FilterConsts &c,
                  hipStream_t stream)
{
    if (nsides < 1 || nsides > 2) return set_status(ctx, RPCA_ERR_ARG, "filter: bad side count");
    const int PT = pick_pt(sides[0].p);
    const int RT = (sides[0].r + 15) / 16;
    for (int s = 0; s < nsides; ++s) {
        if (!filter_supported(ctx, sides[s].p, sides[s].r))
            return set_status(ctx, RPCA_ERR_UNSUPPORTED,
                              "filter: p = " + std::to_string(sides[s].p) + ", r = " +
                                  std::to_string(sides[s].r) + " outside the built kernel classes");
        if (pick_pt(sides[s].p) != PT || (sides[s].r + 15) / 16 != RT)
            return set_status(ctx, RPCA_ERR_ARG, "filter: fused sides must share a class");
    }
    FilterLaunch L{};
    L.c = c;
    int nblocks = 0;
    for (int s = 0; s < nsides; ++s) {
        L.side[s] = sides[s];
        const int64_t tiles = (sides[s].nreg + 15) / 16;
        const int64_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
        if (blocks > INT_MAX / 2) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: too many regressions");
        if (s == 0) L.nblocks0 = (int)blocks;
        nblocks += (int)blocks;
    }
    if (nsides == 1) L.side[1] = sides[0];
    if (nblocks == 0) return RPCA_OK;
    switch (PT) {
    case 1: return launch_pt<1>(ctx, RT, L, nblocks, stream);
    case 2: return launch_pt<2>(ctx, RT, L, nblocks, stream);
    case 3: return launch_pt<3>(ctx, RT, L, nblocks, stream);
    case 4: return launch_pt<4>(ctx, RT, L, nblocks, stream);
    case 5: return launch_pt<5>(ctx, RT, L, nblocks, stream);
    case 7: return launch_pt<7>(ctx, RT, L, nblocks, stream);
    case 8: return launch_pt<8>(ctx, RT, L, nblocks, stream);
    case 10: return launch_pt<10>(ctx, RT, L, nblocks, stream);
    case 13: return launch_pt<13>(ctx, RT, L, nblocks, stream);
    case 16: return launch_pt<16>(ctx, RT, L, nblocks, stream);
    case 19: return launch_pt<19>(ctx, RT, L, nblocks, stream);
    default: return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: p class not built");
    }
}
