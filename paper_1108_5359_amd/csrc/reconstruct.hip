// Completion of L and S = M - L for one problem (Algorithm 2, step 5 and
// output); the arithmetic is in recon_kernel.h.
#include "recon_kernel.h"

#include <algorithm>
#include <climits>
#include <mutex>

using namespace reconk;

namespace {

__global__ void __launch_bounds__(kAssembleThreads)
assemble_factors(int64_t first, int64_t end, const int64_t *__restrict__ seed_rows, int64_t p,
                 const int64_t *__restrict__ seed_cols, int64_t q,
                 const double *__restrict__ U, const double *__restrict__ sigma,
                 const double *__restrict__ V, int r,
                 const float *__restrict__ Qt, const float *__restrict__ Pt,
                 int64_t m, int64_t n, int R4, float *__restrict__ F, float *__restrict__ G)
{
    __shared__ int64_t sidx[kIdxLds];
    assemble_block(first + (int64_t)blockIdx.x * blockDim.x, end, sidx, seed_rows, p, seed_cols, q,
                   U, sigma, V, r, Qt, Pt, m, n, R4, F, G);
}

// Ranks 33..52 hold 4 rows of F per lane (up to 256 VGPRs): ask for two
// waves per SIMD, or the compiler may take a few acc VGPRs beyond 256 and
// leave one.  (No __restrict__ on these arguments: with it the compiler keeps
// two more values live at rank 52 and spills them.)
template <int R4, bool VEC>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(R4 > 32 && rows_per_lane(R4) == 4 ? 2 : 1)))
reconstruct_kernel(const float *M, int64_t ldm, const float *F, const float *G, int64_t m, int64_t n,
                   float *Lo, int64_t ldl, float *So, int64_t lds)
{
    recon_wave<R4, VEC>(M, ldm, F, G, m, n, Lo, ldl, So, lds, blockIdx.x, blockIdx.y, gridDim.y,
                        threadIdx.x);
}

__global__ void iota_kernel(int64_t *__restrict__ dst, int64_t count)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = t;
}

template <int R4>
int launch_r4(rpca_ctx *ctx, const ReconArgs &a, const float *F, const float *G, bool vec,
              hipStream_t stream)
{
    // ~recon_waves_per_cu waves per CU across the chip (32 measured best) for
    // the column sweep (rank <= 32); eight times as many above, where each
    // wave takes a contiguous column range and two waves per SIMD are
    // resident: shorter ranges balance the many rounds of the grid better
    // (measured at rank 50, m = n = 50000: 6.40, 6.24, 6.12, 6.05, 6.01, 5.95,
    // 6.06 ms at 48, 64, 96, 128, 192, 256, 384 waves per CU); at least one
    // batch of 4 columns each
    const int64_t row_blocks = (a.m + rows_per_wave(R4) - 1) / rows_per_wave(R4);
    const int64_t target_waves = (int64_t)(ctx->num_cu > 0 ? ctx->num_cu : 256) *
                                 ctx->recon_waves_per_cu * (R4 > 32 ? 8 : 1);
    int64_t per_block = (target_waves + row_blocks - 1) / row_blocks;
    per_block = std::max<int64_t>(1, std::min<int64_t>(per_block, (a.n + 3) / 4));
    per_block = std::min<int64_t>(per_block, 65535);
    const dim3 grid((unsigned)row_blocks, (unsigned)per_block);
    if (vec)
        hipLaunchKernelGGL((reconstruct_kernel<R4, true>), grid, dim3(64), 0, stream, a.M, a.ldm, F,
                           G, a.m, a.n, a.L, a.ldl, a.S, a.lds);
    else
        hipLaunchKernelGGL((reconstruct_kernel<R4, false>), grid, dim3(64), 0, stream, a.M, a.ldm,
                           F, G, a.m, a.n, a.L, a.ldl, a.S, a.lds);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    return RPCA_OK;
}

} // namespace

int launch_reconstruct(rpca_ctx *ctx, const ReconArgs &a, hipStream_t stream)
{
    const int R4 = (a.r + 3) / 4 * 4;
    if (R4 > 64) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "reconstruct: rank above 64");
    const size_t fbytes = (size_t)(a.m + a.n) * R4 * sizeof(float);
    int st = ensure_buf(ctx, ctx->factors, fbytes);
    if (st != RPCA_OK) return st;
    return launch_reconstruct_with(ctx, a, static_cast<float *>(ctx->factors.ptr), stream);
}

int launch_iota(rpca_ctx *ctx, int64_t *dst, int64_t count, hipStream_t stream)
{
    if (count <= 0) return RPCA_OK;
    hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, dst,
                       count);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    return RPCA_OK;
}

int launch_reconstruct_with(rpca_ctx *ctx, const ReconArgs &a, float *factors, hipStream_t stream)
{
    const int R4 = (a.r + 3) / 4 * 4;
    if (R4 > 64) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "reconstruct: rank above 64");
    float *F = factors;
    float *G = F + (size_t)a.m * R4;
    int st = launch_assemble_range(ctx, a, R4, F, G, 0, a.m + a.n, stream);
    if (st != RPCA_OK) return st;
    return launch_complete_slab(ctx, a, R4, F, G, 0, a.n, stream);
}

// ---------------------------------------------------------------- no-allocation form
// The factors F and G of rpca_reconstruct_noalloc live in this file-scope
// device array instead of the context's workspace.  Each device that loads
// the library holds its own copy (kNoAllocScratchBytes, until the process
// ends); in host code `scratch` names a host-side stand-in, so kernels get
// the device address taken once per device by noalloc_scratch_setup.
namespace {
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
} // namespace

int noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return RPCA_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return RPCA_OK;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return RPCA_ERR_DEVICE;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return RPCA_ERR_DEVICE;
    }
    g_scratch_ptr[device] = ptr;
    return RPCA_OK;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

int launch_assemble_range(rpca_ctx *ctx, const ReconArgs &a, int R4, float *F, float *G,
                          int64_t first_row, int64_t end_row, hipStream_t stream)
{
    if (end_row <= first_row) return RPCA_OK;
    // units of one row and 4 ranks
    const int64_t first = first_row * (R4 / 4), end = end_row * (R4 / 4);
    hipLaunchKernelGGL(assemble_factors,
                       dim3((unsigned)((end - first + kAssembleThreads - 1) / kAssembleThreads)),
                       dim3(kAssembleThreads), 0, stream, first, end, a.seed_rows, a.p, a.seed_cols,
                       a.q, a.U, a.sigma, a.V, a.r, a.Qt, a.Pt, a.m, a.n, R4, F, G);
    RPCA_HIP_TRY(ctx, hipGetLastError());
    return RPCA_OK;
}

int launch_complete_slab(rpca_ctx *ctx, const ReconArgs &full, int R4, const float *F,
                         const float *G, int64_t j0, int64_t j1, hipStream_t stream)
{
    if (j1 <= j0) return RPCA_OK;
    // the slab is the matrix of columns j0 .. j1 - 1 (contiguous in memory)
    ReconArgs a = full;
    a.M = full.M + j0 * full.ldm;
    a.L = full.L + j0 * full.ldl;
    a.S = full.S + j0 * full.lds;
    a.n = j1 - j0;
    G = G + j0 * R4;
    const bool vec = (a.ldm % 4 == 0) && (a.ldl % 4 == 0) && (a.lds % 4 == 0) &&
                     ((uintptr_t)a.M % 16 == 0) && ((uintptr_t)a.L % 16 == 0) &&
                     ((uintptr_t)a.S % 16 == 0);
    switch (R4) {
    case 4: return launch_r4<4>(ctx, a, F, G, vec, stream);
    case 8: return launch_r4<8>(ctx, a, F, G, vec, stream);
    case 12: return launch_r4<12>(ctx, a, F, G, vec, stream);
    case 16: return launch_r4<16>(ctx, a, F, G, vec, stream);
    case 20: return launch_r4<20>(ctx, a, F, G, vec, stream);
    case 24: return launch_r4<24>(ctx, a, F, G, vec, stream);
    case 28: return launch_r4<28>(ctx, a, F, G, vec, stream);
    case 32: return launch_r4<32>(ctx, a, F, G, vec, stream);
    case 36: return launch_r4<36>(ctx, a, F, G, vec, stream);
    case 40: return launch_r4<40>(ctx, a, F, G, vec, stream);
    case 44: return launch_r4<44>(ctx, a, F, G, vec, stream);
    case 48: return launch_r4<48>(ctx, a, F, G, vec, stream);
    case 52: return launch_r4<52>(ctx, a, F, G, vec, stream);
    case 56: return launch_r4<56>(ctx, a, F, G, vec, stream);
    case 60: return launch_r4<60>(ctx, a, F, G, vec, stream);
    case 64: return launch_r4<64>(ctx, a, F, G, vec, stream);
    default: return set_status(ctx, RPCA_ERR_UNSUPPORTED, "reconstruct: rank class not built");
    }
}
