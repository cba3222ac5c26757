// Internal declarations shared by the host runtime (api.cpp) and the HIP
// kernels (filter.hip, reconstruct.hip, seed.hip) of librpca.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <string>

#include "../../include/rpca.h"

// Grow-only device buffer owned by a context.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct rpca_ctx {
    int device = 0;
    int32_t last_seed_route = 0;    // route of the last rpca_seed call (RPCA_SEED_ROUTE_*)
    hipStream_t aux = nullptr;      // second stream of the overlapped form (created on first use)
    hipEvent_t pev[40] = {};        // its events
    int num_cu = 0;
    size_t max_lds = 0;
    std::string last_error;
    int recon_waves_per_cu = 32;  // launch shape of the completion (tunable)
    rocblas_handle blas = nullptr;
    hipEvent_t ev[6] = {};
    DevBuf seed_ws;     // FP64 matrices of the seed solver
    DevBuf factors;     // F (m x R4) and G (n x R4), FP32, for the completion
    DevBuf solve_ws;    // indices and filter outputs inside rpca_solve
    DevBuf scratch;     // small reductions / flags
    DevBuf frag_ws;     // FP32 refresh fragments of the precision form (large p)
    DevBuf xbuf_ws;     // the regressions' x in fragment order (read by the refresh)
    DevBuf iota_ws;     // column indices 0..n-1 of the online column filter
    DevBuf rank_ws;     // indices and factors of the rank-estimation seeds
};

// Set ctx->last_error and return status.
int set_status(rpca_ctx *ctx, int status, const std::string &msg);

// Create ctx->aux (default priority) and its events on first use.
int ensure_aux(rpca_ctx *ctx);

// Make sure buf holds at least `bytes`; returns RPCA_OK or RPCA_ERR_NOMEM.
int ensure_buf(rpca_ctx *ctx, DevBuf &buf, size_t bytes);

// Summary of per-regression iteration codes (see RPCA_ITERS_*): total of
// |count|, regressions that missed the stopping test, largest count, and
// regressions with a bad index or a non-finite input.
struct IterSummary {
    int64_t total = 0, not_converged = 0, bad_index = 0, nonfinite = 0;
    int32_t max = 0;
};
IterSummary summarize_iters(const int32_t *its, size_t n);

struct FilterConsts;
// Range checks of the options (RPCA_ERR_ARG with a message on failure).
int check_opts(rpca_ctx *ctx, const rpca_opts &o);
// The filter's constants in the precision the kernels use.
FilterConsts consts_of(const rpca_opts &o);

#define RPCA_HIP_TRY(ctx, expr)                                                        \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess)                                                          \
            return set_status((ctx), RPCA_ERR_DEVICE,                                  \
                              std::string(#expr ": ") + hipGetErrorString(_e));        \
    } while (0)

// ---------------------------------------------------------------- filter
// One family of independent regressions: element e of regression k is
// M[elem_idx[e] * elem_stride + reg_idx[k] * reg_stride], regressed on the
// p x r FP64 basis A (ld lda); the coefficients go to Z[:, k] (ld ldz).
struct FilterSide {
    const float *M;
    const int64_t *elem_idx;
    const int64_t *reg_idx;
    int64_t elem_stride;
    int64_t reg_stride;
    int64_t elem_bound;   // valid element indices are [0, elem_bound)
    int64_t reg_bound;    // valid regression indices are [0, reg_bound)
    const double *A;
    int32_t lda;
    int32_t p;
    int32_t r;
    int64_t nreg;
    float *Z;
    int64_t ldz;
    int32_t *iters;
    float *xbuf;          // workspace: x in fragment order, for the periodic refresh
    const int64_t *range; // optional device [begin, end): regression positions served
                          // (nreg then only bounds end - begin); null = [0, nreg)
};

struct FilterConsts {
    float eps, rho, beta0_scale, beta_max_scale;
    int32_t max_iter, refresh;
    int32_t precision;    // 0 = FP32 contractions, 1 = FP16 contractions + FP32 refinement
    int32_t form;         // FP32 kernels: 0 = automatic, 1 = tile form, 2 = split form
    int64_t plan_regs;    // regressions of the whole call the launch belongs to (0 = the
                          // launch's own): the automatic form choice is made on this count,
                          // so a call cut into several launches picks the form the single
                          // launch would
};

// Enqueue the regressions of up to two sides (same p class and r class) in
// one launch.  Returns an RPCA status.
int launch_filter(rpca_ctx *ctx, const FilterSide *sides, int nsides, const FilterConsts &c,
                  hipStream_t stream);

// Whether launch_filter supports (p, r) in the given precision mode.
bool filter_supported(rpca_ctx *ctx, int p, int r, int precision);

// The kernel form launch_filter takes for `regs` regressions of size (p, r):
// 0 = FP16 contractions (precision form), 1 = FP32 tile form, 2 = FP32 split form.
int filter_form_of(rpca_ctx *ctx, int p, int r, int precision, int form, int64_t regs);

// Whether two (p, r) pairs use the same kernel and can share one launch.
bool filter_same_class(int p0, int r0, int p1, int r1);

// ---------------------------------------------------------------- completion
struct ReconArgs {
    const float *M;
    int64_t m, n, ldm;
    const int64_t *seed_rows;
    int64_t p;
    const int64_t *seed_cols;
    int64_t q;
    const double *U, *sigma, *V;
    int32_t r;
    const float *Qt, *Pt;
    float *L;
    int64_t ldl;
    float *S;
    int64_t lds;
};

int launch_reconstruct(rpca_ctx *ctx, const ReconArgs &a, hipStream_t stream);
// dst[k] = k for k < count (device int64).
int launch_iota(rpca_ctx *ctx, int64_t *dst, int64_t count, hipStream_t stream);
// The same into caller-provided factor storage ((m + n) * R4 floats, R4 = r
// rounded up to 4); allocates nothing.
int launch_reconstruct_with(rpca_ctx *ctx, const ReconArgs &a, float *factors, hipStream_t stream);

// Scratch of the no-allocation completion: a file-scope device array of this
// size per device.  noalloc_scratch_setup takes its device address once per
// device (that device current); noalloc_scratch returns it (null before).
constexpr size_t kNoAllocScratchBytes = RPCA_NOALLOC_SCRATCH_BYTES;
int noalloc_scratch_setup(int device);
void *noalloc_scratch(int device);

// Pieces of the completion for the overlapped form: assemble rows
// [first_row, end_row) of the stacked factors (F rows are [0, m), G row j is
// m + j) and complete the column slab [j0, j1) of L and S.
int launch_assemble_range(rpca_ctx *ctx, const ReconArgs &a, int R4, float *F, float *G,
                          int64_t first_row, int64_t end_row, hipStream_t stream);
int launch_complete_slab(rpca_ctx *ctx, const ReconArgs &a, int R4, const float *F,
                         const float *G, int64_t j0, int64_t j1, hipStream_t stream);

// Steps 3-5 of one problem with the completion of column slab k overlapped
// with the filtering of the column regressions of slab k + 1 (second stream).
struct PipelineArgs {
    ReconArgs rec;               // M, sizes, seed indices and factors, Qt, Pt, L, S
    const int64_t *cols;         // sorted complement of the seed columns (n - q)
    const int64_t *rows;         // sorted complement of the seed rows (m - p)
    int32_t *col_iters, *row_iters;
};
int launch_filter_complete(rpca_ctx *ctx, const PipelineArgs &a, const FilterConsts &c,
                           int chunks, hipStream_t stream);

// ---------------------------------------------------------------- seed
struct SeedOut {
    int32_t r_used = 0;
    int32_t iters = 0;
    int32_t converged = 0;
    int32_t rank_found = 0;
    int32_t ritz_steps = 0;      // device-resident route: Rayleigh-Ritz steps in all
    int32_t fallback = 0;        // device-resident route: 1 = the subspace would exceed its cap
    int32_t route = 0;           // RPCA_SEED_ROUTE_*
};

int run_seed(rpca_ctx *ctx, const float *M, int64_t ldm, const int64_t *seed_rows, int64_t p,
             const int64_t *seed_cols, int64_t q, int32_t r, const rpca_opts &o, double *U,
             double *sigma, double *V, SeedOut *out, hipStream_t stream);
// Status of a seed solve as returned to callers, with its message set.
int seed_status_message(rpca_ctx *ctx, int status, const SeedOut &so, int32_t r);

// Many small seed blocks in one launch (one workgroup each, Jacobi SVD in LDS).
struct SmallSeedArgs {
    const float *M;
    int64_t ldm;
    const int64_t *rows, *cols;
    int64_t p, q;
    int32_t r;
    double *U, *sigma, *V;
};
// Whether a p x q seed block fits the batched solver's LDS budget.
bool seed_small_fits(rpca_ctx *ctx, int64_t p, int64_t q);
// Device workspace (bytes) run_seed_small needs for these problems.
size_t seed_small_workspace(const SmallSeedArgs *args, int n);
// Solve them; per problem, the status of run_seed and its SeedOut.  Synchronous.
int run_seed_large(rpca_ctx *ctx, const SmallSeedArgs *args, int n, const rpca_opts &o, void *ws,
                   SeedOut *outs, int *statuses, hipStream_t stream);
// The device-resident route (seed_large.hip): whether a p x q block fits it,
// and the workspace (bytes) n problems need.  A problem whose SVT would need
// more directions than the route holds comes back with RPCA_ERR_UNSUPPORTED
// and SeedOut::fallback = 1.
bool seed_large_fits(rpca_ctx *ctx, int64_t p, int64_t q);
size_t seed_large_workspace(const SmallSeedArgs *args, int n);
int run_seed_small(rpca_ctx *ctx, const SmallSeedArgs *args, int n, const rpca_opts &o, void *ws,
                   SeedOut *outs, int *statuses, hipStream_t stream);

// ---------------------------------------------------------------- batched form
// One side (columns or rows) of one problem, filtered in the lane form: one
// regression per lane, p <= kLaneMaxP, r <= kLaneMaxR.  Fields mean what
// they mean in FilterSide; cls is the compiled (P4, RB) class index.
constexpr int kLaneMaxP = 80;
constexpr int kLaneMaxR = 8;

// A regression whose input holds an Inf or NaN: its sum of squares ||x||_2^2
// is NaN or +Inf (so is one that overflows FP32).  Costs nothing per element:
// every filter kernel forms that sum for beta_0 anyway.
__device__ __forceinline__ bool nonfinite_norm(float xx) { return !(xx <= 3.40282347e38f); }

struct LaneSide {
    const float *M;
    const int64_t *elem_idx;
    const int64_t *reg_idx;
    int64_t elem_stride, reg_stride;
    int64_t elem_bound, reg_bound;
    const double *A;
    int64_t nreg;
    float *Z;
    int64_t ldz;
    int32_t *iters;
    int32_t lda, p, r, cls;
};

// Class index of (p, r) in the lane form with lpr lanes per regression (1, 2
// or 4), or -1 outside it; and the regressions one work item of a class covers.
int lane_class(int p, int r, int lpr);
int lane_regs_per_item(int cls);

// Completion of one problem inside the batched launch (R4 in {4, 8}).
struct ReconJob {
    const float *M;
    float *L, *S;
    const float *F, *G;          // assembled factors, m x R4 and n x R4 row-major
    int64_t m, n, ldm, ldl, lds;
    const int64_t *seed_rows, *seed_cols;
    int64_t p, q;
    const double *U, *sigma, *V;
    const float *Qt, *Pt;
    int32_t r, R4, vec;
    uint32_t row_blocks, col_parts;   // completion waves of this problem: row_blocks x col_parts
};

// The device tables of a batched run.
struct BatchTables {
    const LaneSide *sides;
    const int32_t *items;        // 2 per item: side index, first regression; the
                                 // items of register group 0 first, then group 1
    int32_t nitems;
    int32_t nitems0;             // items of group 0
    uint32_t *counter;           // work-queue heads of the two groups (reset by the launch)
    int32_t grid_waves[2];       // persistent waves of each group's lane filter
    const ReconJob *jobs;
    const int32_t *asm_block_job;    // job of each workgroup of the factor assembly
    const int64_t *asm_block_first;  // the job's thread index of that workgroup's thread 0
    int32_t asm_blocks;
    const int32_t *rec_block_job;    // job of each completion wave
    const uint32_t *rec_block_local; // its index among the job's waves
    int32_t rec_blocks;
    int32_t rec_lds_bytes;           // LDS reserved per completion wave (caps residency), 0 = none
};

// Register group of a lane class (lane_class() value): 0 = three waves per
// SIMD, 1 = two.
int lane_group(int cls);

// Enqueue the lane-form filter over every item (queue reset included).
int launch_lane_filter(rpca_ctx *ctx, const BatchTables &t, const FilterConsts &c,
                       hipStream_t stream);

// Enqueue factor assembly + completion of every job of the table.
int launch_batch_reconstruct(rpca_ctx *ctx, const BatchTables &t, hipStream_t stream);

// The batch plan, reusable (the request loop re-plans one object per batch so
// that its device buffers only grow).
struct rpca_batch;
int batch_check_tuning(rpca_ctx *ctx, const rpca_batch_tuning &tun);
rpca_batch *batch_new(rpca_ctx *ctx, const rpca_opts &o, const rpca_batch_tuning &tun, int *status);
// Lay out and check a new set of jobs; the index arrays are read after the
// work enqueued on `stream`.
int batch_plan(rpca_batch *b, const rpca_job *jobs, int64_t njobs, hipStream_t stream);
hipStream_t batch_stream(rpca_batch *b);
