// Steps 3-5 of one problem with the completion overlapped with the filter.
//
// The filter is bound by the ALUs and the completion by HBM, so they can
// share the chip.  The completion of a column slab of L and S needs every
// row regression (the whole row factor F) and the column regressions of that
// slab (its rows of G).  So the row regressions run first; then the column
// regressions run in `chunks` slabs of columns on the caller's stream, and
// the completion of slab k runs on a second stream as soon as slab k's
// regressions are done, while slab k + 1's regressions run.  How many
// regressions a slab holds depends on the seed columns, which live on the
// device: a one-thread kernel writes each slab's range of positions in the
// sorted complement, and the filter launches read their range from there
// (their grids are sized for the slab's column count, an upper bound).
#include "rpca_internal.h"

#include <algorithm>

namespace {

constexpr int kMaxChunks = 16;

// ranges[k] = number of complement columns below floor(k n / chunks), k = 0..chunks
__global__ void slab_ranges(const int64_t *__restrict__ seed_cols, int64_t q, int64_t n,
                            int chunks, int64_t *__restrict__ ranges)
{
    const int k = threadIdx.x;
    if (k > chunks) return;
    const int64_t jk = n * k / chunks;
    int64_t lo = 0, hi = q;            // seed columns below jk
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (seed_cols[mid] < jk) lo = mid + 1;
        else hi = mid;
    }
    ranges[k] = jk - lo;
}

} // namespace

int ensure_aux(rpca_ctx *ctx)
{
    if (ctx->aux) return RPCA_OK;
    RPCA_HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    for (auto &e : ctx->pev)
        RPCA_HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return RPCA_OK;
}

int launch_filter_complete(rpca_ctx *ctx, const PipelineArgs &pa, const FilterConsts &c,
                           int chunks, hipStream_t stream)
{
    const ReconArgs &a = pa.rec;
    const int64_t nc = a.n - a.q, mr = a.m - a.p;
    const int R4 = (a.r + 3) / 4 * 4;
    if (R4 > 64) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "reconstruct: rank above 64");
    int st = ensure_aux(ctx);
    if (st != RPCA_OK) return st;
    const int K = std::max(1, std::min(chunks, kMaxChunks));
    st = ensure_buf(ctx, ctx->factors, (size_t)(a.m + a.n) * R4 * sizeof(float));
    if (st != RPCA_OK) return st;
    st = ensure_buf(ctx, ctx->scratch, (kMaxChunks + 1) * sizeof(int64_t));
    if (st != RPCA_OK) return st;
    float *F = static_cast<float *>(ctx->factors.ptr);
    float *G = F + (size_t)a.m * R4;
    int64_t *ranges = static_cast<int64_t *>(ctx->scratch.ptr);
    hipEvent_t ev_start = ctx->pev[0], ev_rows = ctx->pev[1], ev_end = ctx->pev[2];
    hipEvent_t *ev_slab = ctx->pev + 3;

    // the second stream starts after everything already on the caller's stream
    RPCA_HIP_TRY(ctx, hipEventRecord(ev_start, stream));
    RPCA_HIP_TRY(ctx, hipStreamWaitEvent(ctx->aux, ev_start, 0));

    FilterSide rows{a.M, a.seed_cols, pa.rows, a.ldm, 1, a.n, a.m, a.V, (int32_t)a.q, (int32_t)a.q,
                    a.r, mr, const_cast<float *>(a.Pt), a.r, pa.row_iters, nullptr, nullptr};
    FilterSide cols{a.M, a.seed_rows, pa.cols, 1, a.ldm, a.m, a.n, a.U, (int32_t)a.p, (int32_t)a.p,
                    a.r, nc, const_cast<float *>(a.Qt), a.r, pa.col_iters, nullptr, nullptr};
    // step 4 (all rows), then the rows of F
    if (mr > 0 && (st = launch_filter(ctx, &rows, 1, c, stream)) != RPCA_OK) return st;
    if (nc > 0) {
        hipLaunchKernelGGL(slab_ranges, dim3(1), dim3(64), 0, stream, a.seed_cols, a.q, a.n, K, ranges);
        RPCA_HIP_TRY(ctx, hipGetLastError());
    }
    RPCA_HIP_TRY(ctx, hipEventRecord(ev_rows, stream));
    RPCA_HIP_TRY(ctx, hipStreamWaitEvent(ctx->aux, ev_rows, 0));
    if ((st = launch_assemble_range(ctx, a, R4, F, G, 0, a.m, ctx->aux)) != RPCA_OK) return st;
    // step 3 slab by slab, each slab's completion on the second stream
    for (int k = 0; k < K; ++k) {
        const int64_t j0 = a.n * k / K, j1 = a.n * (k + 1) / K;
        if (nc > 0) {
            FilterSide cs = cols;
            cs.range = ranges + k;
            cs.nreg = j1 - j0;                     // bound: a slab holds at most its columns
            if ((st = launch_filter(ctx, &cs, 1, c, stream)) != RPCA_OK) return st;
        }
        RPCA_HIP_TRY(ctx, hipEventRecord(ev_slab[k], stream));
        RPCA_HIP_TRY(ctx, hipStreamWaitEvent(ctx->aux, ev_slab[k], 0));
        if ((st = launch_assemble_range(ctx, a, R4, F, G, a.m + j0, a.m + j1, ctx->aux)) != RPCA_OK)
            return st;
        if ((st = launch_complete_slab(ctx, a, R4, F, G, j0, j1, ctx->aux)) != RPCA_OK) return st;
    }
    // the caller's stream continues after the last slab
    RPCA_HIP_TRY(ctx, hipEventRecord(ev_end, ctx->aux));
    RPCA_HIP_TRY(ctx, hipStreamWaitEvent(stream, ev_end, 0));
    return RPCA_OK;
}
