/*
 * rpca.h -- l1 filtering for Principal Component Pursuit on AMD MI355X (gfx950).
 *
 * The method (Liu, Lin, Wei, Su, "Solving Principal Component Pursuit in
 * Linear Time via l1 Filtering") recovers M = L + S, L low rank and S sparse,
 * in the five steps of Algorithm 2:
 *   1. sample p = os_r*r seed rows I_s and q = os_c*r seed columns J_s (Sec. 3.1);
 *   2. solve the small PCP (eq. SPCP) on M^s = M[I_s, J_s]            -> rpca_seed
 *   3. column l1 filtering (eq. l1c'), one l1 regression per column     -> rpca_filter_cols
 *   4. row l1 filtering (eq. l1r'), one l1 regression per row           -> rpca_filter_rows
 *   5. complete L (eqs. l1s, l1s') and S = M - L                        -> rpca_reconstruct
 * rpca_solve runs all five.  Each regression of steps 3-4 is
 *   min_z ||x - A z||_1,  A^T A = I   (eq. l1g),
 * solved by the alternating direction method of Algorithm 1.
 *
 * Conventions
 *   Layout     every matrix is column-major with an explicit leading dimension
 *              (element (i, j) of M is M[i + j*ldm]); a row-major (n, ld)
 *              tensor holds the same bytes.  Index arrays are int64.
 *   Memory     M, L, S, the index arrays, U/sigma/V, Qt/Pt and iters are
 *              DEVICE pointers on the context's device.  rpca_opts,
 *              rpca_info and scalar outputs (r_used, seed_iters) are host
 *              pointers.  rpca_sample_indices works on host arrays.
 *   Ownership  the caller allocates and frees every argument; the library
 *              never frees or retains caller memory after a call returns (or,
 *              for asynchronous calls, after the stream reaches the call).
 *              The context owns only its own workspace.
 *   Errors     arguments are checked on the host before anything is
 *              enqueued.  Negative status = error, outputs untouched (or, for
 *              errors detected on the device, unspecified).  Positive status =
 *              warning, outputs valid.  rpca_last_error() describes the last
 *              status of a context in words.
 *   Streams    filter and reconstruct calls are asynchronous on `stream`
 *              (NULL = the default stream); seed and solve synchronize.
 *   Threads    a context is used by one host thread at a time.
 */
#ifndef RPCA_H
#define RPCA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpca_ctx *rpca_ctx_t;

/* Status codes. */
enum {
    RPCA_OK = 0,
    RPCA_WARN_NOT_CONVERGED = 1, /* some regression or the seed missed its stopping test */
    RPCA_WARN_RANK = 2,          /* rank of the recovered seed differs from the target r */
    RPCA_ERR_ARG = -1,           /* invalid argument (null, size, layout, indices)        */
    RPCA_ERR_NOMEM = -2,         /* device workspace could not be allocated              */
    RPCA_ERR_DEVICE = -3,        /* HIP / rocSOLVER runtime error                         */
    RPCA_ERR_SEED = -4,          /* the seed PCP returned rank 0                          */
    RPCA_ERR_NUMERIC = -5,       /* non-finite value in the input                         */
    RPCA_ERR_UNSUPPORTED = -6    /* shape outside what the kernels were built for        */
};

/* Codes a filter call writes to iters[k] in place of an iteration count:
 *   RPCA_ITERS_BAD_INDEX  the regression index cols[k] / rows[k] is outside M;
 *                         Qt[:, k] / Pt[:, k] is not written.
 *   RPCA_ITERS_NONFINITE  the regression's input x holds an Inf or NaN (or
 *                         ||x||_2^2 overflows FP32): no iteration runs and the
 *                         output column is NaN.  The synchronous calls
 *                         (rpca_solve, rpca_solve_factored, rpca_batch_job_info,
 *                         served requests) then return RPCA_ERR_NUMERIC. */
#define RPCA_ITERS_BAD_INDEX (-2147483647 - 1)
#define RPCA_ITERS_NONFINITE (-2147483647)

/*
 * Constants of the method.  The paper fixes s_r = s_c = 10 (Sec. 3.1) and
 * lambda~ = 1/sqrt(max(p, q)) (eq. SPCP); it leaves eps, rho, beta_0 and
 * beta_bar of Algorithm 1 ("eps > 0, rho > 1, beta_bar >> beta_0 > 0") and
 * the seed solver's constants open.  rpca_opts_default() gives the values
 * this library uses; they match the FP64 reference used by the tests.
 */
typedef struct {
    int32_t os_r, os_c;          /* oversampling s_r, s_c: p = os_r*r, q = os_c*r (10, 10) */
    double seed_lambda;          /* <= 0: 1/sqrt(max(p, q))                                */
    double seed_tol;             /* stop when ||M^s-L-S||_F/||M^s||_F < seed_tol (1e-9)    */
    double seed_rho;             /* mu_{k+1} = min(seed_rho*mu_k, mu_bar) (1.5)             */
    double seed_mu0_scale;       /* mu_0 = seed_mu0_scale / ||M^s||_2 (1.25)                */
    double seed_mu_max_scale;    /* mu_bar = seed_mu_max_scale * mu_0 (1e7)                 */
    int32_t seed_max_iter;       /* (500)                                                   */
    double seed_rank_floor;      /* drop thresholded sigma_i <= floor*sigma_1 (1e-6)        */
    double filt_eps;             /* Alg. 1 eps, on ||x-Az-e||_inf/||x||_inf (1e-9)          */
    double filt_rho;             /* Alg. 1 rho (1.5)                                        */
    double filt_beta0_scale;     /* beta_0 = filt_beta0_scale/||x||_2 per regression (1.25) */
    double filt_beta_max_scale;  /* beta_bar = filt_beta_max_scale*beta_0 (1e10)            */
    int32_t filt_max_iter;       /* (500)                                                   */
    int32_t filt_refresh;        /* recompute x - A z from x every this many steps (8)      */
    uint64_t rng_seed;           /* seed of rpca_sample_indices inside rpca_solve           */
    int32_t precision;           /* 0 = FP32 filter; 1 = FP16 MFMA contractions + FP32      */
                                 /* refinement for regressions with p >= 48 (0)             */
    int32_t overlap_chunks;      /* rpca_filter_complete / rpca_solve: column slabs whose   */
                                 /* completion overlaps the filtering of the next slab;     */
                                 /* 0 = filter, then complete (0: a filter launch whose     */
                                 /* grid does not fill the chip lasts one wave's latency,   */
                                 /* so slicing it costs more than the overlap saves)        */
    int32_t filter_form;         /* FP32 filter kernels: 0 = chosen from the regression     */
                                 /* count (automatic), 1 = tile form (one wave per 16      */
                                 /* regressions), 2 = split form (one workgroup of four    */
                                 /* waves per 16 regressions, each wave a quarter of the   */
                                 /* elements) where built for the class, else the tile     */
                                 /* form.  Results agree within rounding, not bit for bit. */
                                 /* Beyond p = 304 the FP32 filter is the quarter-tile    */
                                 /* form (four waves per 16 regressions, a workgroup per   */
                                 /* CU), whatever this says. (0)                           */
    int32_t seed_route;          /* FP64 SVD inside the seed solver: 0 = automatic (blocks  */
                                 /* of up to 6400 entries: Jacobi SVD in LDS; blocks up to */
                                 /* 512 x 512 of a batch: one launch of the device-resident*/
                                 /* subspace iteration, a workgroup each, whatever the     */
                                 /* batch holds; one block alone (rpca_seed, rpca_solve):  */
                                 /* the eigen-decomposition of the Gram matrix, the faster */
                                 /* of the two there);                                     */
                                 /* 1 = always the Gram eigen-decomposition (rocSOLVER,    */
                                 /* one host synchronisation per ALM step); 2 = the        */
                                 /* device-resident routes wherever they apply (0)         */
} rpca_opts;

/* What rpca_solve reports. */
typedef struct {
    int32_t r_used;              /* rank of the recovered seed that was used                */
    int32_t seed_iters;          /* ALM iterations of the seed PCP                          */
    int32_t seed_converged;      /* 1 if the seed met seed_tol                              */
    int32_t filt_iters_max;      /* largest iteration count over all regressions            */
    int64_t filt_iters_total;    /* sum of iteration counts (|count| for unconverged ones)  */
    int64_t filt_not_converged;  /* number of regressions that missed filt_eps              */
    double t_seed_ms;            /* wall time of step 2 (seed)                              */
    double t_filter_ms;          /* device time of steps 3 + 4 (with overlap_chunks > 0:    */
                                 /* of steps 3-5, which then share the chip)                */
    double t_reconstruct_ms;     /* device time of step 5 (0 with overlap_chunks > 0)       */
    int32_t seed_route;          /* how the seed's SVT ran: RPCA_SEED_ROUTE_*               */
} rpca_info;

/* Routes of the seed solver (rpca_info.seed_route, rpca_last_seed_route). */
#define RPCA_SEED_ROUTE_EIGEN 1        /* Gram matrix + rocSOLVER eigen-decomposition     */
#define RPCA_SEED_ROUTE_SUBSPACE 2     /* device-resident subspace iteration, completed   */
#define RPCA_SEED_ROUTE_LDS_JACOBI 3   /* device-resident Jacobi SVD in LDS               */
#define RPCA_SEED_ROUTE_FELL_BACK 4    /* the subspace iteration needed more directions   */
                                       /* than it holds; the eigen route finished         */

/* Which filter kernel a call with these options takes for `nreg`
 * regressions of p elements and rank r (nreg: all regressions of the call,
 * both families): *form = 0 FP16 contractions (precision form), 1 FP32 tile
 * form, 2 FP32 split form (see filter_form), 3 FP32 quarter-tile form (p > 304).
 * Host only; launches nothing.
 * Errors: RPCA_ERR_ARG (null pointer, bad options, p < 1, r < 1, nreg < 0). */
int rpca_filter_form(rpca_ctx_t ctx, int64_t p, int32_t r, int64_t nreg, const rpca_opts *opts,
                     int32_t *form);

/* Fill *opts with the defaults listed above. */
void rpca_opts_default(rpca_opts *opts);

/* Create a context on HIP device `device`.  *ctx receives the handle.
 * Errors: RPCA_ERR_ARG (null ctx, bad device), RPCA_ERR_DEVICE. */
int rpca_ctx_create(int device, rpca_ctx_t *ctx);

/* Destroy a context and free its workspace (not caller memory). */
int rpca_ctx_destroy(rpca_ctx_t ctx);

/* Text of the last status set on ctx ("" after success); valid until the
 * next call on ctx.  With ctx == NULL, the last error of a failed create. */
const char *rpca_last_error(rpca_ctx_t ctx);

/* Name of a status code. */
const char *rpca_status_string(int status);

/*
 * Step 1 (Sec. 3.1; Algorithm 2, step 1): draw p distinct rows of m and q
 * distinct columns of n, uniformly without replacement, into HOST arrays
 * rows[p], cols[q], each sorted ascending.  The draw is a partial
 * Fisher-Yates shuffle driven by SplitMix64 (Steele, Lea, Flood, OOPSLA 2014)
 * seeded with `seed`; the same seed gives the same indices on every machine.
 * Errors: RPCA_ERR_ARG unless 1 <= p <= m, 1 <= q <= n and arrays non-null.
 */
int rpca_sample_indices(int64_t m, int64_t n, int64_t p, int64_t q, uint64_t seed,
                        int64_t *rows, int64_t *cols);

/*
 * Step 2 (Sec. 3.1, eq. SPCP; Sec. 3.2 for the factors): solve
 *   min ||L^s||_* + lambda~ ||S^s||_1  s.t.  M^s = L^s + S^s
 * on M^s = M[seed_rows, seed_cols] (p x q) by the inexact augmented Lagrange
 * multiplier method with singular value thresholding (Sec. 2, eqs. Proxy,
 * SVT), in FP64 on the device (SVD by rocSOLVER).  From the final
 * thresholding step, U (p x r_used, ld p), sigma (r_used) and V (q x r_used,
 * ld q) are the skinny SVD of L^s (singular values already shrunk).
 *   M          device FP32, m x n, leading dimension ldm >= m.
 *   seed_rows  device int64[p], sorted, distinct, in [0, m).
 *   seed_cols  device int64[q], sorted, distinct, in [0, n).
 *   r          target rank; U, sigma, V are caller buffers for r columns.
 *   U, sigma, V  device FP64 outputs; columns beyond r_used are zeroed.
 *   r_used, seed_iters  host outputs (may be NULL).
 * Synchronous.  Returns RPCA_WARN_RANK when rank(L^s) != r (when larger, the
 * r leading components are kept), RPCA_WARN_NOT_CONVERGED when seed_tol was
 * not met, RPCA_ERR_SEED when rank(L^s) = 0, RPCA_ERR_NUMERIC on a
 * non-finite entry of M^s.
 */
int rpca_seed(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
              const int64_t *seed_rows, int64_t p, const int64_t *seed_cols, int64_t q,
              int32_t r, const rpca_opts *opts, double *U, double *sigma, double *V,
              int32_t *r_used, int32_t *seed_iters);

/* Route the last rpca_seed call on ctx took (RPCA_SEED_ROUTE_*; 0 before the
 * first).  Host only.  Errors: RPCA_ERR_ARG (null ctx or route). */
int rpca_last_seed_route(rpca_ctx_t ctx, int32_t *route);

/*
 * Step 3 (Sec. 3.2, eq. l1c'; Algorithm 1): for each k < nc, with j = cols[k],
 * solve min ||M[seed_rows, j] - U q||_1 and write q to Qt[:, k].
 *   seed_rows  device int64[p], distinct, in [0, m) (the rows U is indexed by).
 *   cols       device int64[nc], in [0, n) (normally the sorted complement of
 *              the seed columns; any columns may be filtered).
 *   U          device FP64, p x r, ld p, orthonormal columns.
 *   Qt         device FP32 output, r x nc, ld r.
 *   iters      device int32[nc] output or NULL: iterations used; -filt_max_iter
 *              when the stopping test was not met (then Qt holds the last
 *              iterate); 0 for an all-zero column; RPCA_ITERS_NONFINITE for a
 *              column holding Inf or NaN, RPCA_ITERS_BAD_INDEX for an index
 *              outside M.
 * Asynchronous on `stream`.  Returns RPCA_ERR_UNSUPPORTED for p or r beyond
 * the built kernel classes (p <= 512, r <= 64).
 */
int rpca_filter_cols(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                     const int64_t *seed_rows, int64_t p, const int64_t *cols, int64_t nc,
                     const double *U, int32_t r, const rpca_opts *opts, float *Qt,
                     int32_t *iters, hipStream_t stream);

/*
 * Step 4 (Sec. 3.2, eq. l1r'): M^r = P~^T V^T + S^r transposes to
 * (M^r)^T = V P~ + (S^r)^T, so for each k < nr, with i = rows[k], solve
 * min ||M[i, seed_cols]^T - V p||_1 and write p to Pt[:, k].
 *   seed_cols  device int64[q], distinct, in [0, n).
 *   rows       device int64[nr], in [0, m) (normally the complement of the
 *              seed rows).
 *   V          device FP64, q x r, ld q, orthonormal columns.
 *   Pt         device FP32 output, r x nr, ld r.   iters as for columns.
 */
int rpca_filter_rows(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                     const int64_t *seed_cols, int64_t q, const int64_t *rows, int64_t nr,
                     const double *V, int32_t r, const rpca_opts *opts, float *Pt,
                     int32_t *iters, hipStream_t stream);

/*
 * Steps 3 and 4 together (Sec. 3.3: the two steps of Algorithm 2 are
 * independent and may run in parallel): the column regressions of `cols`
 * against U and the row regressions of `rows` against V, enqueued as one
 * launch so that both families share the device.  Arguments mean what they
 * mean in rpca_filter_cols (seed_rows, p, cols, nc, U, Qt, col_iters) and
 * rpca_filter_rows (seed_cols, q, rows, nr, V, Pt, row_iters); either family
 * may be empty (nc = 0 or nr = 0).  Asynchronous on `stream`.
 */
int rpca_filter(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                const int64_t *seed_rows, int64_t p, const int64_t *seed_cols, int64_t q,
                const int64_t *cols, int64_t nc, const int64_t *rows, int64_t nr,
                const double *U, const double *V, int32_t r, const rpca_opts *opts, float *Qt,
                int32_t *col_iters, float *Pt, int32_t *row_iters, hipStream_t stream);

/*
 * Step 5 (Sec. 3.2, eqs. row-column-recovery, l1s, l1s'; Algorithm 2,
 * output): write the whole low-rank part
 *   L[I_s, J_s] = U Sigma V^T,   L[I_s, J_c] = U Q~,
 *   L[I_c, J_s] = P~^T V^T,      L[I_c, J_c] = P~^T Sigma^{-1} Q~,
 * and S = M - L, where I_c, J_c are the sorted complements of the seed
 * indices.  Qt (r x (n-q), ld r) holds the column filtering of the sorted
 * J_c, Pt (r x (m-p), ld r) the row filtering of the sorted I_c.
 *   seed_rows, seed_cols  device int64, sorted ascending, distinct.
 *   U, sigma, V           device FP64 seed factors (sigma > 0).
 *   L, S                  device FP32 outputs, m x n, ld ldl / lds >= m.
 *                         L and S must not overlap M or each other.
 * Asynchronous on `stream`.
 */
int rpca_reconstruct(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                     const int64_t *seed_rows, int64_t p, const int64_t *seed_cols,
                     int64_t q, const double *U, const double *sigma, const double *V,
                     int32_t r, const float *Qt, const float *Pt, float *L, int64_t ldl,
                     float *S, int64_t lds, hipStream_t stream);

/*
 * rpca_reconstruct for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, same kernels and the same results, bit for
 * bit, as rpca_reconstruct; the assembled factors (the only scratch of the
 * completion) go to a fixed device array of RPCA_NOALLOC_SCRATCH_BYTES per
 * device, which the library holds from its first context on that device until
 * the process ends, instead of the context's workspace.  The call allocates
 * nothing (no hipMalloc, no library allocator).
 * Limit: (m + n) * 4 * ceil4(r) bytes <= RPCA_NOALLOC_SCRATCH_BYTES, i.e.
 * (m + n) * ceil4(r) <= 8388608 (m = n = 50000 at r = 50 fits); larger
 * problems get RPCA_ERR_ARG, and ranks above 64 RPCA_ERR_UNSUPPORTED.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (two streams, two host threads) race and give wrong results, so
 * order them on one stream.  Nothing in the array needs clearing: every call
 * writes all the factor rows it reads.  Asynchronous on `stream`.
 */
#define RPCA_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int rpca_reconstruct_noalloc(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                             const int64_t *seed_rows, int64_t p, const int64_t *seed_cols,
                             int64_t q, const double *U, const double *sigma, const double *V,
                             int32_t r, const float *Qt, const float *Pt, float *L, int64_t ldl,
                             float *S, int64_t lds, hipStream_t stream);

/*
 * Steps 3, 4 and 5 together (Sec. 3.2-3.3; eqs. l1c', l1r', l1s'): what
 * rpca_filter followed by rpca_reconstruct computes, with the completion of
 * L and S overlapped with the filtering when opts->overlap_chunks > 0: the
 * row regressions run first, then the column regressions in overlap_chunks
 * slabs of columns, and the completion of each slab (on a second stream of
 * the context) runs while the next slab's regressions are filtered.  The
 * results are identical to the two calls made one after the other.
 *   cols, rows   device int64: the sorted complements of seed_cols (n - q)
 *                and seed_rows (m - p) (every other argument as in
 *                rpca_filter and rpca_reconstruct; Qt / Pt and the iteration
 *                arrays are outputs as there, iteration arrays may be NULL).
 * Asynchronous on `stream`; later work on `stream` follows the whole call.
 * Calls on one context must be ordered on one stream.
 */
int rpca_filter_complete(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                         const int64_t *seed_rows, int64_t p, const int64_t *seed_cols, int64_t q,
                         const int64_t *cols, const int64_t *rows, const double *U,
                         const double *sigma, const double *V, int32_t r, const rpca_opts *opts,
                         float *Qt, int32_t *col_iters, float *Pt, int32_t *row_iters, float *L,
                         int64_t ldl, float *S, int64_t lds, hipStream_t stream);

/*
 * Algorithm 2 end to end on M (m x n): steps 1-5 with target rank r.
 * seed_rows / seed_cols: device int64 arrays of os_r*r and os_c*r sorted
 * indices, or both NULL to draw them with rpca_sample_indices(opts->rng_seed).
 * L, S: device FP32 outputs.  info (host, may be NULL) receives the summary.
 * Synchronous.  Returns the most severe status of the steps; RPCA_ERR_NUMERIC
 * when M^s or the input of some regression holds an Inf or NaN.  (An Inf or
 * NaN in M[I_c, J_c], which no regression reads, only passes into S there.)
 */
int rpca_solve(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm, int32_t r,
               const rpca_opts *opts, const int64_t *seed_rows, const int64_t *seed_cols,
               float *L, int64_t ldl, float *S, int64_t lds, rpca_info *info,
               hipStream_t stream);

/*
 * Algorithm 2, steps 2-4, stopping at the factored form of the low-rank part
 * (Sec. 3.4: apart from M, l1 filtering needs only O(r(m + n)) storage):
 *   L = [ U Sigma V^T   U Q~               ]   rows I_s
 *       [ P~^T V^T      P~^T Sigma^-1 Q~   ]   rows I_c     (eqs. partition, l1s')
 * with columns J_s on the left and J_c on the right.  No m x n output is
 * written; rpca_reconstruct turns the factors into L and S when wanted, and
 * rpca_filter_new_cols completes columns that arrive later.
 *   seed_rows  device int64[p], seed_cols device int64[q]: sorted, distinct,
 *              in range (any p, q with r <= min(p, q); normally os_r*r, os_c*r).
 *   r          target rank: U (p x r, ld p), sigma (r), V (q x r, ld q) are
 *              device FP64 outputs (columns beyond the rank used are zero).
 *   Qt, Pt     device FP32 buffers of r * (n-q) and r * (m-p) floats: the
 *              filtering of the sorted complements J_c and I_c, written as
 *              r_used x (n-q) and r_used x (m-p) with ld r_used, where r_used
 *              (info->r_used, <= r) is the rank of the seed that was used;
 *              pass r_used as the rank to rpca_reconstruct and
 *              rpca_filter_new_cols.
 *   col_iters  device int32[n-q] or NULL, row_iters device int32[m-p] or NULL
 *              (codes as for rpca_filter_cols).
 *   info       host, may be NULL (t_reconstruct_ms = 0).
 * Synchronous.  Status as rpca_solve's.
 */
int rpca_solve_factored(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                        int32_t r, const rpca_opts *opts, const int64_t *seed_rows, int64_t p,
                        const int64_t *seed_cols, int64_t q, double *U, double *sigma, double *V,
                        float *Qt, int32_t *col_iters, float *Pt, int32_t *row_iters,
                        rpca_info *info, hipStream_t stream);

/*
 * Online column filtering (Sec. 3.2, eq. l1c', applied to columns that arrive
 * after the fit, e.g. the frames of a video in background modelling, Sec. 4.3):
 * with the row factors of an earlier fit of the same m rows fixed, each new
 * column j < nnew of Mnew is filtered against U (Algorithm 1 on
 * x = Mnew[seed_rows, j]) into Qt_new[:, j], and only these columns are
 * completed:
 *   L[I_s, j] = U q~_j,   L[I_c, j] = P~^T Sigma^-1 q~_j   (eq. l1s'),
 *   S[:, j] = Mnew[:, j] - L[:, j].
 * The cost is O(r m) per column; the fitted matrix is not touched again.
 *   Mnew        device FP32, m x nnew, ld ldm >= m (the new columns).
 *   seed_rows   device int64[p]: the fit's sorted seed rows I_s.
 *   U, sigma    device FP64 seed factors of the fit (p x r ld p, r), sigma > 0;
 *               r is the rank the fit used.
 *   Pt          device FP32 r x (m-p), ld r: the fit's row filtering over the
 *               sorted I_c (as rpca_solve_factored writes it).
 *   Qt_new      device FP32 output r x nnew, ld r; iters device int32[nnew] or
 *               NULL (codes as for rpca_filter_cols).
 *   L, S        device FP32 outputs m x nnew (ld ldl, lds >= m), distinct from
 *               Mnew and from each other.
 * Asynchronous on `stream`.  Errors: RPCA_ERR_ARG, RPCA_ERR_UNSUPPORTED (p, r
 * outside the kernel classes), RPCA_ERR_NOMEM.  A column whose seed rows hold
 * an Inf or NaN gets iters = RPCA_ITERS_NONFINITE and NaN in L and S.
 */
int rpca_filter_new_cols(rpca_ctx_t ctx, const float *Mnew, int64_t m, int64_t nnew, int64_t ldm,
                         const int64_t *seed_rows, int64_t p, const double *U, const double *sigma,
                         int32_t r, const float *Pt, const rpca_opts *opts, float *Qt_new,
                         int32_t *iters, float *L, int64_t ldl, float *S, int64_t lds,
                         hipStream_t stream);

/*
 * Target-rank estimation (Sec. 3.6, eqs. rank_test and rank_test1) for when
 * r is not known.  Starting from the guess r0, the seed PCP (eq. SPCP) is
 * solved on an m' x n' = (os_r r_k) x (os_c r_k) block and the rank r' of L^s
 * is read off (as rpca_seed counts it, before any truncation).  If
 * m'/r' >= os_r and n'/r' >= os_c (eq. rank_test) the seed is accepted and
 * r' is the estimate; otherwise the block grows to (os_r r') x (os_c r') and
 * the test repeats, unless the grown block would exceed half of M in either
 * direction (eq. rank_test1): then the data are not low rank enough for
 * l1 filtering and the loop stops (accepted = 0).  The blocks grow as
 * prefixes of two caller-given orders, so each block contains the previous
 * one: the seed rows of a block of p rows are row_order[0..p) sorted.  With
 * cross_validate, one more block of the accepted size, disjoint from it
 * (row_order[p..2p), col_order[q..2q)), is solved and its rank reported
 * (Sec. 3.6, last paragraph); it runs only when 2p <= m and 2q <= n.
 *   row_order   HOST int64[m], a permutation of 0..m-1 (checked).
 *   col_order   HOST int64[n], a permutation of 0..n-1 (checked).
 *   r0          initial guess, >= 1, with os_r r0 <= m/2 and os_c r0 <= n/2.
 *   info        host output.
 * The accepted seed's factors are those rpca_seed (or rpca_solve_factored)
 * returns for the block's sorted indices and r = r_est (same arithmetic).
 * Synchronous.  Returns RPCA_OK when eq. rank_test held (and the
 * cross-validation block, if run, has the same rank); RPCA_WARN_RANK when
 * the loop stopped at eq. rank_test1 or the cross-validation rank differs;
 * RPCA_ERR_SEED when a seed has rank 0; RPCA_ERR_ARG, RPCA_ERR_NUMERIC as
 * rpca_seed.
 */
#define RPCA_RANK_MAX_ROUNDS 16
typedef struct {
    int32_t r_est;                         /* rank of the last seed solved             */
    int32_t accepted;                      /* 1: eq. rank_test held; 0: stopped        */
    int32_t rounds;                        /* seed PCPs of the growing loop            */
    int32_t cv_rank;                       /* rank of the cross-validation block, or -1 */
    int64_t p, q;                          /* size of the last seed block solved        */
    int32_t ranks[RPCA_RANK_MAX_ROUNDS];   /* r' found in each round                    */
    int64_t ps[RPCA_RANK_MAX_ROUNDS];      /* block size of each round                  */
    int64_t qs[RPCA_RANK_MAX_ROUNDS];
} rpca_rank_info;
int rpca_estimate_rank(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                       int32_t r0, const rpca_opts *opts, const int64_t *row_order,
                       const int64_t *col_order, int32_t cross_validate, rpca_rank_info *info);

/* ------------------------------------------------------------------------
 * Batched form: steps 2-5 of Algorithm 2 for many independent problems
 * ("jobs") of uneven sizes.  The regressions of every job are independent
 * (Sec. 3.3), so the column and row regressions of all jobs are served from
 * one work queue by one persistent kernel, and the completions of all jobs
 * by one launch; the launches of a run can be replayed from a HIP graph.
 *
 * Life cycle: rpca_batch_create (checks, workspace) -> rpca_batch_seed
 * (step 2 for every job) -> rpca_batch_run (steps 3-5 for every job; may be
 * called repeatedly, e.g. after the caller rewrites the M buffers in place)
 * -> rpca_batch_destroy.  The batch keeps the job descriptors (pointers
 * included): the caller's buffers must stay valid until destroy.
 * ------------------------------------------------------------------------ */

/* One problem of a batch.  All pointers are DEVICE pointers on the context's
 * device; layouts as everywhere (column-major, explicit leading dims). */
typedef struct {
    const float *M;              /* m x n input, ld ldm >= m                                */
    int64_t m, n, ldm;
    int32_t r;                   /* target rank, 1 <= r <= min(p, q)                        */
    const int64_t *seed_rows;    /* p sorted distinct row indices in [0, m)                 */
    int64_t p;
    const int64_t *seed_cols;    /* q sorted distinct column indices in [0, n)              */
    int64_t q;
    float *L;                    /* m x n output, ld ldl >= m                               */
    int64_t ldl;
    float *S;                    /* m x n output, ld lds >= m                               */
    int64_t lds;
} rpca_job;

/* Launch-shape choices of a batch (what the autotuner searches over). */
typedef struct {
    int32_t lane_max_p;          /* regressions with p <= lane_max_p (<= 80) and r <= 8 use */
    int32_t lane_max_r;          /* the lane form (one regression per 1, 2 or 4 lanes, 4x4  */
                                 /* MFMA); others the 16-regression tile form (80, 8)       */
    int32_t lane_split2_p;       /* lane form: p > this runs on 2 lanes per regression      */
                                 /* (32; at most 32)                                        */
    int32_t lane_split4_p;       /* ... and p > this on 4 lanes (64; split2 .. 64)          */
    int32_t filter_waves_per_cu; /* persistent grid of the lane form (8)                    */
    int32_t recon_cols_per_wave; /* columns streamed by one wave of the completion (32)     */
    int32_t order;               /* work-queue order: 0 = costliest job sides first,        */
                                 /* 1 = job order (0)                                       */
    int32_t graph;               /* 1 = replay runs after the first from HIP graphs (1)     */
    int32_t seed_batched;        /* 1 = seed blocks that fit in LDS are solved together, one */
                                 /* workgroup each (Jacobi SVD); 0 = one by one (1)         */
    int32_t recon_waves_per_cu;  /* completion waves resident per CU at most, enforced by   */
                                 /* each wave's LDS reservation; 0 = no cap (4: fewer       */
                                 /* concurrent column streams keep HBM pages open longer)   */
} rpca_batch_tuning;

typedef struct rpca_batch *rpca_batch_t;

/* Fill *t with the defaults listed above. */
void rpca_batch_tuning_default(rpca_batch_tuning *t);

/*
 * Check njobs jobs (host array `jobs`, copied) and allocate the batch's
 * device workspace (complement indices, seed factors, filter outputs,
 * completion factors, work queue).  opts as for rpca_solve (os_r, os_c and
 * rng_seed unused: every job brings its seed indices); tuning may be NULL
 * (defaults).  The seed index arrays are read after the work enqueued on the
 * default (NULL) stream.  Synchronous.  Errors: RPCA_ERR_ARG (bad job: the
 * message names it), RPCA_ERR_NOMEM, RPCA_ERR_UNSUPPORTED (a job outside
 * every kernel class).
 */
int rpca_batch_create(rpca_ctx_t ctx, const rpca_job *jobs, int64_t njobs, const rpca_opts *opts,
                      const rpca_batch_tuning *tuning, rpca_batch_t *batch);

/*
 * Step 2 (Sec. 3.1, eq. SPCP) for every job, as rpca_seed does for one, into
 * the batch's workspace; then builds the work queue of steps 3-4 from the
 * ranks found.  Seed blocks that fit in LDS are solved together by one launch
 * (one workgroup each, Jacobi SVD), the others one at a time (rocSOLVER).
 * The M buffers are read after the work enqueued on `stream`.  Synchronous.
 * Returns the most severe job status (the message names the first job with
 * it); RPCA_ERR_SEED if a seed has rank 0.
 */
int rpca_batch_seed(rpca_batch_t batch, hipStream_t stream);

/*
 * Steps 3-5 (Sec. 3.2-3.3, Algorithm 1 per regression; eqs. l1s, l1s') for
 * every job: writes L and S of each job.  Requires a successful
 * rpca_batch_seed.  Asynchronous on `stream`; with tuning.graph, the first
 * run records the launches into two HIP graphs (filter, completion) that later
 * runs replay.  The work queue lives in the batch: runs of one batch must not
 * overlap (serialize them on one stream).
 */
int rpca_batch_run(rpca_batch_t batch, hipStream_t stream);

/*
 * Per-job summary of the last seed and run (host *info): rank used, seed
 * iterations, filter iteration statistics; t_seed_ms is the job's seed wall
 * time, t_filter_ms / t_reconstruct_ms the device time of the whole batch's
 * filter / completion phase of the last run.  Synchronizes with the last run.
 * Returns the job's seed warning, RPCA_WARN_NOT_CONVERGED, or
 * RPCA_ERR_NUMERIC when one of its regressions read an Inf or NaN of M (its
 * L and S then hold NaN in that row or column).
 */
int rpca_batch_job_info(rpca_batch_t batch, int64_t job, rpca_info *info);

/*
 * The seed factors of `job` after rpca_batch_seed (Sec. 3.2: L^s = U Sigma
 * V^T), copied into caller DEVICE buffers: U (p x r, ld p), sigma (r), V
 * (q x r, ld q), FP64, columns beyond the rank used zero.  Synchronous.
 * Errors: RPCA_ERR_ARG (bad job, NULL buffer, batch not seeded).
 */
int rpca_batch_job_factors(rpca_batch_t batch, int64_t job, double *U, double *sigma, double *V);

/* Free the batch's workspace and graphs (never caller memory). */
int rpca_batch_destroy(rpca_batch_t batch);

/* ------------------------------------------------------------------------
 * Served form: a request loop over the batched form.  Requests (one rpca_job
 * each) queue in arrival order; `workers` host threads each take requests
 * from the head of the queue while the device memory of all admitted,
 * unfinished requests stays within hbm_budget_bytes (a request larger than
 * the budget is admitted alone), up to max_batch at a time, and run steps 2-5
 * for them as one batch on their own stream, so batches of different workers
 * overlap on the device and requests that arrive meanwhile join the next
 * batch.  A batch that fails as a whole is retried request by request.
 * ------------------------------------------------------------------------ */
typedef struct {
    double hbm_budget_bytes;     /* admission budget: M, L, S and workspace of the admitted */
                                 /* unfinished requests (200e9)                             */
    int32_t workers;             /* concurrent batches, 1..16 (3)                           */
    int32_t max_batch;           /* requests per batch (64)                                 */
} rpca_server_opts;

/* What a finished request reports (times: host clock, ms since creation). */
typedef struct {
    int32_t status;              /* the request's status (as rpca_solve's)                  */
    int32_t batch_size;          /* requests in the batch it ran in                         */
    rpca_info info;              /* rank, iterations; phase times of its batch              */
    double t_submit_ms, t_admit_ms, t_done_ms;
} rpca_request_info;

typedef struct {
    int64_t submitted, completed, failed, batches, queued;
    double peak_inflight_bytes;  /* largest admitted footprint seen                         */
    double inflight_bytes;       /* admitted footprint now                                  */
} rpca_server_stats;

typedef struct rpca_server *rpca_server_t;

/* Fill *o with the defaults listed above. */
void rpca_server_opts_default(rpca_server_opts *o);

/*
 * Start a request loop on HIP device `device` with the method's options
 * (opts, as for rpca_solve), the launch shapes of its batches (tuning, may be
 * NULL; graph replay is off: every batch runs once) and the server options
 * (sopts, may be NULL).  Errors: RPCA_ERR_ARG, RPCA_ERR_DEVICE; the message
 * is rpca_server_error(NULL).
 */
int rpca_server_create(int device, const rpca_opts *opts, const rpca_batch_tuning *tuning,
                       const rpca_server_opts *sopts, rpca_server_t *server);

/*
 * Queue one request (host *job, copied; its device buffers belong to the
 * caller and must stay valid and untouched until the request is done; M is
 * read after the work enqueued on the default stream when its batch starts).
 * *ticket receives its handle.  Errors: RPCA_ERR_ARG (NULL, sizes, rank).
 */
int rpca_server_submit(rpca_server_t server, const rpca_job *job, int64_t *ticket);

/* Block until the request is done, fill *info (may be NULL) and forget the
 * ticket.  Returns the request's status when negative, else RPCA_OK. */
int rpca_server_wait(rpca_server_t server, int64_t ticket, rpca_request_info *info);

/* *done = 1 if the request is done (the ticket stays valid until waited). */
int rpca_server_poll(rpca_server_t server, int64_t ticket, int32_t *done);

/* Counters of the loop. */
int rpca_server_get_stats(rpca_server_t server, rpca_server_stats *stats);

/* Text of the last error of the server (NULL: of the last failed create). */
const char *rpca_server_error(rpca_server_t server);

/* Finish every queued request, stop the workers, free everything the server
 * owns. */
int rpca_server_destroy(rpca_server_t server);

#ifdef __cplusplus
}
#endif

#endif /* RPCA_H */
