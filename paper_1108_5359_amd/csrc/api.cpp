// Host runtime of librpca: argument checks, index sampling, workspace, and
// the order of the steps of Algorithm 2.  All arithmetic of the method runs
// in the HIP kernels (filter.hip, reconstruct.hip) and the FP64 seed solver
// (seed.hip).
#include "rpca_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace {

thread_local std::string g_create_error;

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

int check_matrix(rpca_ctx *ctx, const void *M, int64_t m, int64_t n, int64_t ld, const char *name)
{
    if (!M) return set_status(ctx, RPCA_ERR_ARG, std::string(name) + " is NULL");
    if (m < 1 || n < 1) return set_status(ctx, RPCA_ERR_ARG, std::string(name) + ": sizes must be >= 1");
    if (ld < m) return set_status(ctx, RPCA_ERR_ARG, std::string(name) + ": leading dimension < rows");
    return RPCA_OK;
}

// Sorted, distinct, in [0, bound): checked on a host copy.
int check_sorted_indices(rpca_ctx *ctx, const int64_t *dev, int64_t count, int64_t bound,
                         const char *name, std::vector<int64_t> *host_out)
{
    std::vector<int64_t> h((size_t)count);
    RPCA_HIP_TRY(ctx, hipMemcpy(h.data(), dev, (size_t)count * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < count; ++i) {
        if (h[i] < 0 || h[i] >= bound)
            return set_status(ctx, RPCA_ERR_ARG, std::string(name) + ": index out of range");
        if (i > 0 && h[i] <= h[i - 1])
            return set_status(ctx, RPCA_ERR_ARG, std::string(name) + ": indices must be sorted and distinct");
    }
    if (host_out) host_out->swap(h);
    return RPCA_OK;
}


uint64_t splitmix64_next(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Uniform integer in [0, bound) by rejection (no modulo bias).
uint64_t uniform_below(uint64_t &state, uint64_t bound)
{
    const uint64_t limit = UINT64_MAX - (UINT64_MAX % bound);
    uint64_t v;
    do v = splitmix64_next(state);
    while (v >= limit);
    return v % bound;
}

// k distinct values of [0, n), sorted: partial Fisher-Yates on a sparse map.
void sample_sorted(int64_t n, int64_t k, uint64_t &state, int64_t *out)
{
    std::vector<std::pair<int64_t, int64_t>> swapped;   // position -> value, small
    auto get = [&](int64_t pos) {
        for (auto &pv : swapped)
            if (pv.first == pos) return pv.second;
        return pos;
    };
    auto set = [&](int64_t pos, int64_t val) {
        for (auto &pv : swapped)
            if (pv.first == pos) { pv.second = val; return; }
        swapped.emplace_back(pos, val);
    };
    for (int64_t i = 0; i < k; ++i) {
        const int64_t jdx = i + (int64_t)uniform_below(state, (uint64_t)(n - i));
        const int64_t vi = get(i), vj = get(jdx);
        set(i, vj);
        set(jdx, vi);
        out[i] = vj;
    }
    std::sort(out, out + k);
}

std::vector<int64_t> complement_of(const std::vector<int64_t> &sorted_idx, int64_t bound)
{
    std::vector<int64_t> c;
    c.reserve((size_t)(bound - (int64_t)sorted_idx.size()));
    size_t a = 0;
    for (int64_t i = 0; i < bound; ++i) {
        if (a < sorted_idx.size() && sorted_idx[a] == i) ++a;
        else c.push_back(i);
    }
    return c;
}

} // namespace

int check_opts(rpca_ctx *ctx, const rpca_opts &o)
{
    if (o.os_r < 1 || o.os_c < 1) return set_status(ctx, RPCA_ERR_ARG, "opts: oversampling must be >= 1");
    if (!(o.filt_eps >= 0 && o.filt_eps < 1)) return set_status(ctx, RPCA_ERR_ARG, "opts: filt_eps must be in [0, 1)");
    if (!(o.filt_rho >= 1) || !std::isfinite(o.filt_rho)) return set_status(ctx, RPCA_ERR_ARG, "opts: filt_rho must be >= 1");
    if (!finite_pos(o.filt_beta0_scale) || !(o.filt_beta_max_scale >= 1) || !std::isfinite(o.filt_beta_max_scale))
        return set_status(ctx, RPCA_ERR_ARG, "opts: bad beta scales");
    if (o.filt_max_iter < 1) return set_status(ctx, RPCA_ERR_ARG, "opts: filt_max_iter must be >= 1");
    if (o.filt_refresh < 0) return set_status(ctx, RPCA_ERR_ARG, "opts: filt_refresh must be >= 0");
    if (!finite_pos(o.seed_tol) || !(o.seed_rho >= 1) || !finite_pos(o.seed_mu0_scale) ||
        !(o.seed_mu_max_scale >= 1) || o.seed_max_iter < 1 || !(o.seed_rank_floor >= 0))
        return set_status(ctx, RPCA_ERR_ARG, "opts: bad seed constants");
    if (o.precision != 0 && o.precision != 1)
        return set_status(ctx, RPCA_ERR_ARG, "opts: precision must be 0 (FP32) or 1 (FP16 + FP32 refinement)");
    if (o.overlap_chunks < 0 || o.overlap_chunks > 16)
        return set_status(ctx, RPCA_ERR_ARG, "opts: overlap_chunks must be in [0, 16]");
    if (o.filter_form < 0 || o.filter_form > 2)
        return set_status(ctx, RPCA_ERR_ARG, "opts: filter_form must be 0 (automatic), 1 (tile) or 2 (split)");
    if (o.seed_route < 0 || o.seed_route > 2)
        return set_status(ctx, RPCA_ERR_ARG, "opts: seed_route must be 0 (automatic), 1 (eigen) or 2 (device-resident)");
    return RPCA_OK;
}

FilterConsts consts_of(const rpca_opts &o)
{
    FilterConsts c;
    c.eps = (float)o.filt_eps;
    c.rho = (float)o.filt_rho;
    c.beta0_scale = (float)o.filt_beta0_scale;
    c.beta_max_scale = (float)o.filt_beta_max_scale;
    c.max_iter = o.filt_max_iter;
    c.refresh = o.filt_refresh;
    c.precision = o.precision;
    c.form = o.filter_form;
    c.plan_regs = 0;
    return c;
}

IterSummary summarize_iters(const int32_t *its, size_t n)
{
    IterSummary s;
    for (size_t i = 0; i < n; ++i) {
        const int32_t k = its[i];
        if (k == RPCA_ITERS_BAD_INDEX) { ++s.bad_index; continue; }
        if (k == RPCA_ITERS_NONFINITE) { ++s.nonfinite; continue; }
        if (k < 0) ++s.not_converged;
        const int32_t ak = k < 0 ? -k : k;
        s.total += ak;
        s.max = std::max(s.max, ak);
    }
    return s;
}

int set_status(rpca_ctx *ctx, int status, const std::string &msg)
{
    if (ctx) ctx->last_error = msg;
    return status;
}

int ensure_buf(rpca_ctx *ctx, DevBuf &buf, size_t bytes)
{
    if (buf.bytes >= bytes) return RPCA_OK;
    if (buf.ptr) {
        (void)hipFree(buf.ptr);
        buf.ptr = nullptr;
        buf.bytes = 0;
    }
    const size_t want = bytes + bytes / 4 + 4096;
    if (hipMalloc(&buf.ptr, want) != hipSuccess) {
        buf.ptr = nullptr;
        (void)hipGetLastError();
        return set_status(ctx, RPCA_ERR_NOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    buf.bytes = want;
    return RPCA_OK;
}

extern "C" {

void rpca_opts_default(rpca_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->os_r = 10;
    o->os_c = 10;
    o->seed_lambda = 0.0;
    o->seed_tol = 1e-9;
    o->seed_rho = 1.5;
    o->seed_mu0_scale = 1.25;
    o->seed_mu_max_scale = 1e7;
    o->seed_max_iter = 500;
    o->seed_rank_floor = 1e-6;
    o->filt_eps = 1e-9;
    o->filt_rho = 1.5;
    o->filt_beta0_scale = 1.25;
    o->filt_beta_max_scale = 1e10;
    o->filt_max_iter = 500;
    o->filt_refresh = 8;
    o->rng_seed = 1;
    o->precision = 0;
    o->overlap_chunks = 0;
    o->filter_form = 0;
    o->seed_route = 0;
}

const char *rpca_status_string(int s)
{
    switch (s) {
    case RPCA_OK: return "RPCA_OK";
    case RPCA_WARN_NOT_CONVERGED: return "RPCA_WARN_NOT_CONVERGED";
    case RPCA_WARN_RANK: return "RPCA_WARN_RANK";
    case RPCA_ERR_ARG: return "RPCA_ERR_ARG";
    case RPCA_ERR_NOMEM: return "RPCA_ERR_NOMEM";
    case RPCA_ERR_DEVICE: return "RPCA_ERR_DEVICE";
    case RPCA_ERR_SEED: return "RPCA_ERR_SEED";
    case RPCA_ERR_NUMERIC: return "RPCA_ERR_NUMERIC";
    case RPCA_ERR_UNSUPPORTED: return "RPCA_ERR_UNSUPPORTED";
    default: return "RPCA_UNKNOWN_STATUS";
    }
}

int rpca_ctx_create(int device, rpca_ctx_t *out)
{
    if (!out) return RPCA_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        g_create_error = "no HIP device";
        return RPCA_ERR_DEVICE;
    }
    if (device < 0 || device >= count) {
        g_create_error = "device index out of range";
        return RPCA_ERR_ARG;
    }
    if (hipSetDevice(device) != hipSuccess) {
        g_create_error = "hipSetDevice failed";
        return RPCA_ERR_DEVICE;
    }
    rpca_ctx *ctx = new rpca_ctx();
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->num_cu = prop.multiProcessorCount;
        ctx->max_lds = prop.sharedMemPerBlock;
        if (prop.maxSharedMemoryPerMultiProcessor > ctx->max_lds)
            ctx->max_lds = prop.maxSharedMemoryPerMultiProcessor;
    }
    if (rocblas_create_handle(&ctx->blas) != rocblas_status_success) {
        delete ctx;
        g_create_error = "rocblas_create_handle failed";
        return RPCA_ERR_DEVICE;
    }
    for (auto &e : ctx->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            g_create_error = "hipEventCreate failed";
            rpca_ctx_destroy(ctx);
            return RPCA_ERR_DEVICE;
        }
    }
    // device address of the no-allocation form's scratch (once per device)
    if (noalloc_scratch_setup(device) != RPCA_OK) {
        g_create_error = "hipGetSymbolAddress of the completion scratch failed";
        rpca_ctx_destroy(ctx);
        return RPCA_ERR_DEVICE;
    }
    *out = ctx;
    return RPCA_OK;
}

int rpca_ctx_destroy(rpca_ctx_t ctx)
{
    if (!ctx) return RPCA_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (DevBuf *b : {&ctx->seed_ws, &ctx->factors, &ctx->solve_ws, &ctx->scratch, &ctx->frag_ws,
                      &ctx->iota_ws, &ctx->rank_ws})
        if (b->ptr) (void)hipFree(b->ptr);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->pev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->xbuf_ws.ptr) (void)hipFree(ctx->xbuf_ws.ptr);
    if (ctx->blas) rocblas_destroy_handle(ctx->blas);
    delete ctx;
    return RPCA_OK;
}

const char *rpca_last_error(rpca_ctx_t ctx)
{
    return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

int rpca_sample_indices(int64_t m, int64_t n, int64_t p, int64_t q, uint64_t seed, int64_t *rows,
                        int64_t *cols)
{
    if (!rows || !cols || p < 1 || q < 1 || p > m || q > n) return RPCA_ERR_ARG;
    uint64_t state = seed;
    sample_sorted(m, p, state, rows);
    sample_sorted(n, q, state, cols);
    return RPCA_OK;
}

int rpca_seed(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
              const int64_t *seed_rows, int64_t p, const int64_t *seed_cols, int64_t q, int32_t r,
              const rpca_opts *opts, double *U, double *sigma, double *V, int32_t *r_used,
              int32_t *seed_iters)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, M, m, n, ldm, "M")) != RPCA_OK) return st;
    if (!opts || !seed_rows || !seed_cols || !U || !sigma || !V)
        return set_status(ctx, RPCA_ERR_ARG, "seed: NULL argument");
    if ((st = check_opts(ctx, *opts)) != RPCA_OK) return st;
    if (r < 1 || p < 1 || q < 1 || p > m || q > n || r > std::min(p, q))
        return set_status(ctx, RPCA_ERR_ARG, "seed: need 1 <= r <= min(p, q), p <= m, q <= n");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    if ((st = check_sorted_indices(ctx, seed_rows, p, m, "seed_rows", nullptr)) != RPCA_OK) return st;
    if ((st = check_sorted_indices(ctx, seed_cols, q, n, "seed_cols", nullptr)) != RPCA_OK) return st;
    SeedOut so;
    st = run_seed(ctx, M, ldm, seed_rows, p, seed_cols, q, r, *opts, U, sigma, V, &so, nullptr);
    ctx->last_seed_route = so.route;
    if (r_used) *r_used = so.r_used;
    if (seed_iters) *seed_iters = so.iters;
    return st;
}

int rpca_last_seed_route(rpca_ctx_t ctx, int32_t *route)
{
    if (!ctx || !route) return ctx ? set_status(ctx, RPCA_ERR_ARG, "last_seed_route: null route") : RPCA_ERR_ARG;
    *route = ctx->last_seed_route;
    return set_status(ctx, RPCA_OK, "");
}

static int make_side(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                     const int64_t *elem_idx, int64_t ne, const int64_t *reg_idx, int64_t nreg,
                     const double *A, int32_t r, float *Z, int32_t *iters, bool rows_mode,
                     int precision, FilterSide *s)
{
    const int64_t ebound = rows_mode ? n : m, rbound = rows_mode ? m : n;
    if (!elem_idx || !A || (nreg > 0 && (!reg_idx || !Z)))
        return set_status(ctx, RPCA_ERR_ARG, "filter: NULL argument");
    if (ne < 1 || ne > ebound || r < 1 || r > ne || nreg < 0)
        return set_status(ctx, RPCA_ERR_ARG, "filter: need 1 <= r <= p <= dimension and nreg >= 0");
    if (ne > INT32_MAX) return set_status(ctx, RPCA_ERR_ARG, "filter: p too large");
    if (!filter_supported(ctx, (int)ne, r, precision))
        return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: p = " + std::to_string(ne) + ", r = " +
                                                         std::to_string(r) + " outside the built kernel classes");
    *s = FilterSide{M, elem_idx, reg_idx, rows_mode ? ldm : 1, rows_mode ? 1 : ldm, ebound, rbound,
                    A, (int32_t)ne, (int32_t)ne, r, nreg, Z, r, iters};
    return RPCA_OK;
}

int rpca_filter(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                const int64_t *seed_rows, int64_t p, const int64_t *seed_cols, int64_t q,
                const int64_t *cols, int64_t nc, const int64_t *rows, int64_t nr, const double *U,
                const double *V, int32_t r, const rpca_opts *opts, float *Qt, int32_t *col_iters,
                float *Pt, int32_t *row_iters, hipStream_t stream)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, M, m, n, ldm, "M")) != RPCA_OK) return st;
    if (!opts) return set_status(ctx, RPCA_ERR_ARG, "filter: NULL opts");
    if ((st = check_opts(ctx, *opts)) != RPCA_OK) return st;
    FilterSide sides[2];
    int ns = 0;
    if (nc > 0) {
        if ((st = make_side(ctx, M, m, n, ldm, seed_rows, p, cols, nc, U, r, Qt, col_iters, false,
                            opts->precision, &sides[ns])) != RPCA_OK)
            return st;
        ++ns;
    }
    if (nr > 0) {
        if ((st = make_side(ctx, M, m, n, ldm, seed_cols, q, rows, nr, V, r, Pt, row_iters, true,
                            opts->precision, &sides[ns])) != RPCA_OK)
            return st;
        ++ns;
    }
    if (nc < 0 || nr < 0) return set_status(ctx, RPCA_ERR_ARG, "filter: negative count");
    if (ns == 0) return RPCA_OK;
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    FilterConsts c = consts_of(*opts);
    c.plan_regs = nc + nr;
    if (ns == 2 && !filter_same_class(sides[0].p, sides[0].r, sides[1].p, sides[1].r)) {
        if ((st = launch_filter(ctx, &sides[0], 1, c, stream)) != RPCA_OK) return st;
        return launch_filter(ctx, &sides[1], 1, c, stream);
    }
    return launch_filter(ctx, sides, ns, c, stream);
}

static int filter_common(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                         const int64_t *elem_idx, int64_t ne, const int64_t *reg_idx, int64_t nreg,
                         const double *A, int32_t r, const rpca_opts *opts, float *Z,
                         int32_t *iters, hipStream_t stream, bool rows_mode)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, M, m, n, ldm, "M")) != RPCA_OK) return st;
    if (!opts || !elem_idx || !A || (nreg > 0 && (!reg_idx || !Z)))
        return set_status(ctx, RPCA_ERR_ARG, "filter: NULL argument");
    if ((st = check_opts(ctx, *opts)) != RPCA_OK) return st;
    const int64_t ebound = rows_mode ? n : m, rbound = rows_mode ? m : n;
    if (ne < 1 || ne > ebound || r < 1 || r > ne || nreg < 0)
        return set_status(ctx, RPCA_ERR_ARG, "filter: need 1 <= r <= p <= dimension and nreg >= 0");
    if (ne > INT32_MAX) return set_status(ctx, RPCA_ERR_ARG, "filter: p too large");
    if (!filter_supported(ctx, (int)ne, r, opts->precision))
        return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: p = " + std::to_string(ne) + ", r = " +
                                                         std::to_string(r) + " outside the built kernel classes");
    if (nreg == 0) return RPCA_OK;
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    FilterSide s{};
    s.M = M;
    s.elem_idx = elem_idx;
    s.reg_idx = reg_idx;
    s.elem_stride = rows_mode ? ldm : 1;
    s.reg_stride = rows_mode ? 1 : ldm;
    s.elem_bound = ebound;
    s.reg_bound = rbound;
    s.A = A;
    s.lda = (int32_t)ne;
    s.p = (int32_t)ne;
    s.r = r;
    s.nreg = nreg;
    s.Z = Z;
    s.ldz = r;
    s.iters = iters;
    return launch_filter(ctx, &s, 1, consts_of(*opts), stream);
}

int rpca_filter_cols(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                     const int64_t *seed_rows, int64_t p, const int64_t *cols, int64_t nc,
                     const double *U, int32_t r, const rpca_opts *opts, float *Qt, int32_t *iters,
                     hipStream_t stream)
{
    return filter_common(ctx, M, m, n, ldm, seed_rows, p, cols, nc, U, r, opts, Qt, iters, stream,
                         false);
}

int rpca_filter_rows(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                     const int64_t *seed_cols, int64_t q, const int64_t *rows, int64_t nr,
                     const double *V, int32_t r, const rpca_opts *opts, float *Pt, int32_t *iters,
                     hipStream_t stream)
{
    return filter_common(ctx, M, m, n, ldm, seed_cols, q, rows, nr, V, r, opts, Pt, iters, stream,
                         true);
}

int rpca_reconstruct(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                     const int64_t *seed_rows, int64_t p, const int64_t *seed_cols, int64_t q,
                     const double *U, const double *sigma, const double *V, int32_t r,
                     const float *Qt, const float *Pt, float *L, int64_t ldl, float *S, int64_t lds,
                     hipStream_t stream)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, M, m, n, ldm, "M")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, L, m, n, ldl, "L")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, S, m, n, lds, "S")) != RPCA_OK) return st;
    if (!seed_rows || !seed_cols || !U || !sigma || !V || (n > q && !Qt) || (m > p && !Pt))
        return set_status(ctx, RPCA_ERR_ARG, "reconstruct: NULL argument");
    if (p < 1 || q < 1 || p > m || q > n || r < 1 || r > std::min(p, q))
        return set_status(ctx, RPCA_ERR_ARG, "reconstruct: need 1 <= r <= min(p, q), p <= m, q <= n");
    if ((const void *)L == (const void *)S || (const void *)L == (const void *)M ||
        (const void *)S == (const void *)M)
        return set_status(ctx, RPCA_ERR_ARG, "reconstruct: L, S and M must be distinct buffers");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    ReconArgs a{M, m, n, ldm, seed_rows, p, seed_cols, q, U, sigma, V, r, Qt, Pt, L, ldl, S, lds};
    return launch_reconstruct(ctx, a, stream);
}

int rpca_reconstruct_noalloc(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                             const int64_t *seed_rows, int64_t p, const int64_t *seed_cols,
                             int64_t q, const double *U, const double *sigma, const double *V,
                             int32_t r, const float *Qt, const float *Pt, float *L, int64_t ldl,
                             float *S, int64_t lds, hipStream_t stream)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, M, m, n, ldm, "M")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, L, m, n, ldl, "L")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, S, m, n, lds, "S")) != RPCA_OK) return st;
    if (!seed_rows || !seed_cols || !U || !sigma || !V || (n > q && !Qt) || (m > p && !Pt))
        return set_status(ctx, RPCA_ERR_ARG, "reconstruct_noalloc: NULL argument");
    if (p < 1 || q < 1 || p > m || q > n || r < 1 || r > std::min(p, q))
        return set_status(ctx, RPCA_ERR_ARG, "reconstruct_noalloc: need 1 <= r <= min(p, q), p <= m, q <= n");
    if (r > 64) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "reconstruct_noalloc: rank above 64");
    const int64_t R4 = (r + 3) / 4 * 4;
    const double need = (double)(m + n) * (double)R4 * sizeof(float);
    if (need > (double)RPCA_NOALLOC_SCRATCH_BYTES)
        return set_status(ctx, RPCA_ERR_ARG,
                          "reconstruct_noalloc: the factors need (m + n) * 4 * ceil4(r) = " +
                              std::to_string((long long)need) + " bytes, above the " +
                              std::to_string((long long)RPCA_NOALLOC_SCRATCH_BYTES) +
                              "-byte scratch; use rpca_reconstruct");
    if ((const void *)L == (const void *)S || (const void *)L == (const void *)M ||
        (const void *)S == (const void *)M)
        return set_status(ctx, RPCA_ERR_ARG, "reconstruct_noalloc: L, S and M must be distinct buffers");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    float *factors = static_cast<float *>(noalloc_scratch(ctx->device));
    if (!factors) return set_status(ctx, RPCA_ERR_DEVICE, "reconstruct_noalloc: scratch not set up on this device");
    ReconArgs a{M, m, n, ldm, seed_rows, p, seed_cols, q, U, sigma, V, r, Qt, Pt, L, ldl, S, lds};
    return launch_reconstruct_with(ctx, a, factors, stream);
}

int rpca_filter_complete(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                         const int64_t *seed_rows, int64_t p, const int64_t *seed_cols, int64_t q,
                         const int64_t *cols, const int64_t *rows, const double *U,
                         const double *sigma, const double *V, int32_t r, const rpca_opts *opts,
                         float *Qt, int32_t *col_iters, float *Pt, int32_t *row_iters, float *L,
                         int64_t ldl, float *S, int64_t lds, hipStream_t stream)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, M, m, n, ldm, "M")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, L, m, n, ldl, "L")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, S, m, n, lds, "S")) != RPCA_OK) return st;
    if (!opts) return set_status(ctx, RPCA_ERR_ARG, "filter_complete: NULL opts");
    if ((st = check_opts(ctx, *opts)) != RPCA_OK) return st;
    if (!seed_rows || !seed_cols || !U || !sigma || !V || (p < m && (!rows || !Pt)) ||
        (q < n && (!cols || !Qt)))
        return set_status(ctx, RPCA_ERR_ARG, "filter_complete: NULL argument");
    if (p < 1 || q < 1 || p > m || q > n || r < 1 || r > std::min(p, q))
        return set_status(ctx, RPCA_ERR_ARG, "filter_complete: need 1 <= r <= min(p, q), p <= m, q <= n");
    if ((const void *)L == (const void *)S || (const void *)L == (const void *)M ||
        (const void *)S == (const void *)M)
        return set_status(ctx, RPCA_ERR_ARG, "filter_complete: L, S and M must be distinct buffers");
    if ((q < n && !filter_supported(ctx, (int)p, r, opts->precision)) ||
        (p < m && !filter_supported(ctx, (int)q, r, opts->precision)))
        return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter_complete: seed size outside the built kernel classes");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    ReconArgs a{M, m, n, ldm, seed_rows, p, seed_cols, q, U, sigma, V, r, Qt, Pt, L, ldl, S, lds};
    FilterConsts c = consts_of(*opts);
    c.plan_regs = (n - q) + (m - p);
    if (opts->overlap_chunks == 0) {
        FilterSide sides[2]{};
        int ns = 0;
        if (q < n) sides[ns++] = FilterSide{M, seed_rows, cols, 1, ldm, m, n, U, (int32_t)p, (int32_t)p, r,
                                            n - q, Qt, r, col_iters, nullptr, nullptr};
        if (p < m) sides[ns++] = FilterSide{M, seed_cols, rows, ldm, 1, n, m, V, (int32_t)q, (int32_t)q, r,
                                            m - p, Pt, r, row_iters, nullptr, nullptr};
        if (ns == 2 && !filter_same_class(sides[0].p, sides[0].r, sides[1].p, sides[1].r)) {
            if ((st = launch_filter(ctx, &sides[0], 1, c, stream)) != RPCA_OK) return st;
            if ((st = launch_filter(ctx, &sides[1], 1, c, stream)) != RPCA_OK) return st;
        } else if (ns > 0) {
            if ((st = launch_filter(ctx, sides, ns, c, stream)) != RPCA_OK) return st;
        }
        return launch_reconstruct(ctx, a, stream);
    }
    PipelineArgs pa{a, cols, rows, col_iters, row_iters};
    return launch_filter_complete(ctx, pa, c, opts->overlap_chunks, stream);
}

int rpca_filter_form(rpca_ctx_t ctx, int64_t p, int32_t r, int64_t nreg, const rpca_opts *opts,
                     int32_t *form)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    if (!opts || !form) return set_status(ctx, RPCA_ERR_ARG, "filter_form: NULL argument");
    int st = check_opts(ctx, *opts);
    if (st != RPCA_OK) return st;
    if (p < 1 || p > INT32_MAX || r < 1 || nreg < 0)
        return set_status(ctx, RPCA_ERR_ARG, "filter_form: need p >= 1, r >= 1, nreg >= 0");
    *form = filter_form_of(ctx, (int)p, r, opts->precision, opts->filter_form, nreg);
    return RPCA_OK;
}

int rpca_solve(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm, int32_t r,
               const rpca_opts *opts, const int64_t *seed_rows, const int64_t *seed_cols, float *L,
               int64_t ldl, float *S, int64_t lds, rpca_info *info, hipStream_t stream)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, M, m, n, ldm, "M")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, L, m, n, ldl, "L")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, S, m, n, lds, "S")) != RPCA_OK) return st;
    if (!opts) return set_status(ctx, RPCA_ERR_ARG, "solve: NULL opts");
    if ((st = check_opts(ctx, *opts)) != RPCA_OK) return st;
    if (r < 1) return set_status(ctx, RPCA_ERR_ARG, "solve: r must be >= 1");
    if ((const void *)L == (const void *)S || (const void *)L == (const void *)M ||
        (const void *)S == (const void *)M)
        return set_status(ctx, RPCA_ERR_ARG, "solve: L, S and M must be distinct buffers");
    const int64_t p = (int64_t)opts->os_r * r, q = (int64_t)opts->os_c * r;
    if (p > m || q > n) return set_status(ctx, RPCA_ERR_ARG, "solve: seed block larger than M");
    if ((seed_rows == nullptr) != (seed_cols == nullptr))
        return set_status(ctx, RPCA_ERR_ARG, "solve: give both seed index arrays or neither");
    if (!filter_supported(ctx, (int)std::max(p, q), r, opts->precision) ||
        !filter_supported(ctx, (int)std::min(p, q), r, opts->precision))
        return set_status(ctx, RPCA_ERR_UNSUPPORTED, "solve: seed size outside the built kernel classes");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));

    // Step 1: seed indices (host), their complements, and device copies.
    std::vector<int64_t> I((size_t)p), J((size_t)q);
    if (seed_rows) {
        if ((st = check_sorted_indices(ctx, seed_rows, p, m, "seed_rows", &I)) != RPCA_OK) return st;
        if ((st = check_sorted_indices(ctx, seed_cols, q, n, "seed_cols", &J)) != RPCA_OK) return st;
    } else {
        rpca_sample_indices(m, n, p, q, opts->rng_seed, I.data(), J.data());
    }
    const std::vector<int64_t> Ic = complement_of(I, m), Jc = complement_of(J, n);
    const int64_t mc = (int64_t)Ic.size(), nc = (int64_t)Jc.size();
    // workspace layout: I, J, Ic, Jc (int64) | U (p x r), sigma, V (q x r) (f64) |
    //                   Qt (r x nc), Pt (r x mc) (f32) | iters (nc + mc, i32)
    const size_t n_idx = (size_t)(p + q + mc + nc);
    const size_t n_f64 = (size_t)((p + q) * r + r);
    const size_t n_f32 = (size_t)(r * (nc + mc));
    const size_t bytes = n_idx * 8 + n_f64 * 8 + n_f32 * 4 + (size_t)(nc + mc) * 4 + 256;
    if ((st = ensure_buf(ctx, ctx->solve_ws, bytes)) != RPCA_OK) return st;
    char *base = static_cast<char *>(ctx->solve_ws.ptr);
    int64_t *dI = reinterpret_cast<int64_t *>(base);
    int64_t *dJ = dI + p, *dIc = dJ + q, *dJc = dIc + mc;
    double *dU = reinterpret_cast<double *>(dJc + nc);
    double *dsig = dU + p * r, *dV = dsig + r;
    float *dQt = reinterpret_cast<float *>(dV + q * r);
    float *dPt = dQt + r * nc;
    int32_t *dit = reinterpret_cast<int32_t *>(dPt + r * mc);

    hipStream_t sm = stream;
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(dI, I.data(), p * 8, hipMemcpyHostToDevice, sm));
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(dJ, J.data(), q * 8, hipMemcpyHostToDevice, sm));
    if (mc) RPCA_HIP_TRY(ctx, hipMemcpyAsync(dIc, Ic.data(), mc * 8, hipMemcpyHostToDevice, sm));
    if (nc) RPCA_HIP_TRY(ctx, hipMemcpyAsync(dJc, Jc.data(), nc * 8, hipMemcpyHostToDevice, sm));

    // Step 2: seed.
    const auto t0 = std::chrono::steady_clock::now();
    SeedOut so;
    const int seed_st = run_seed(ctx, M, ldm, dI, p, dJ, q, r, *opts, dU, dsig, dV, &so, sm);
    const auto t1 = std::chrono::steady_clock::now();
    if (seed_st < 0) return seed_st;
    const std::string seed_msg = ctx->last_error;
    const int ru = so.r_used;

    // Steps 3 and 4 in one launch, then step 5.
    FilterSide sides[2]{};
    int ns = 0;
    if (nc) {
        FilterSide &s = sides[ns++];
        s = FilterSide{M, dI, dJc, 1, ldm, m, n, dU, (int32_t)p, (int32_t)p, ru, nc, dQt, ru, dit};
    }
    if (mc) {
        FilterSide &s = sides[ns++];
        s = FilterSide{M, dJ, dIc, ldm, 1, n, m, dV, (int32_t)q, (int32_t)q, ru, mc, dPt, ru, dit + nc};
    }
    FilterConsts c = consts_of(*opts);
    c.plan_regs = nc + mc;
    ReconArgs a{M, m, n, ldm, dI, p, dJ, q, dU, dsig, dV, ru, dQt, dPt, L, ldl, S, lds};
    RPCA_HIP_TRY(ctx, hipEventRecord(ctx->ev[0], sm));
    if (opts->overlap_chunks > 0) {
        // steps 3-5 with the completion overlapped with the filter
        PipelineArgs pa{a, dJc, dIc, dit, dit + nc};
        if ((st = launch_filter_complete(ctx, pa, c, opts->overlap_chunks, sm)) != RPCA_OK) return st;
        RPCA_HIP_TRY(ctx, hipEventRecord(ctx->ev[1], sm));
        RPCA_HIP_TRY(ctx, hipEventRecord(ctx->ev[2], sm));
    } else {
        if (ns == 2 && !filter_same_class(sides[0].p, sides[0].r, sides[1].p, sides[1].r)) {
            // different size classes: two launches
            if ((st = launch_filter(ctx, &sides[0], 1, c, sm)) != RPCA_OK) return st;
            if ((st = launch_filter(ctx, &sides[1], 1, c, sm)) != RPCA_OK) return st;
        } else if (ns > 0) {
            if ((st = launch_filter(ctx, sides, ns, c, sm)) != RPCA_OK) return st;
        }
        RPCA_HIP_TRY(ctx, hipEventRecord(ctx->ev[1], sm));
        if ((st = launch_reconstruct(ctx, a, sm)) != RPCA_OK) return st;
        RPCA_HIP_TRY(ctx, hipEventRecord(ctx->ev[2], sm));
    }

    std::vector<int32_t> its((size_t)(nc + mc));
    if (!its.empty())
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(its.data(), dit, its.size() * 4, hipMemcpyDeviceToHost, sm));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(sm));
    const IterSummary is = summarize_iters(its.data(), its.size());
    const int64_t total = is.total, bad = is.not_converged;
    const int32_t kmax = is.max;
    if (info) {
        float tf = 0, tr = 0;
        (void)hipEventElapsedTime(&tf, ctx->ev[0], ctx->ev[1]);
        (void)hipEventElapsedTime(&tr, ctx->ev[1], ctx->ev[2]);
        info->r_used = ru;
        info->seed_iters = so.iters;
        info->seed_converged = so.converged;
        info->seed_route = so.route;
        info->filt_iters_max = kmax;
        info->filt_iters_total = total;
        info->filt_not_converged = bad;
        info->t_seed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info->t_filter_ms = tf;
        info->t_reconstruct_ms = tr;
    }
    if (is.nonfinite)
        return set_status(ctx, RPCA_ERR_NUMERIC, std::to_string(is.nonfinite) +
                                                     " regressions read a non-finite entry of M");
    if (seed_st > 0) return set_status(ctx, seed_st, seed_msg);
    if (bad) return set_status(ctx, RPCA_WARN_NOT_CONVERGED, std::to_string(bad) + " regressions missed filt_eps");
    return RPCA_OK;
}

int rpca_solve_factored(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n, int64_t ldm,
                        int32_t r, const rpca_opts *opts, const int64_t *seed_rows, int64_t p,
                        const int64_t *seed_cols, int64_t q, double *U, double *sigma, double *V,
                        float *Qt, int32_t *col_iters, float *Pt, int32_t *row_iters,
                        rpca_info *info, hipStream_t stream)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, M, m, n, ldm, "M")) != RPCA_OK) return st;
    if (!opts) return set_status(ctx, RPCA_ERR_ARG, "solve_factored: NULL opts");
    if ((st = check_opts(ctx, *opts)) != RPCA_OK) return st;
    if (!seed_rows || !seed_cols || !U || !sigma || !V || (q < n && !Qt) || (p < m && !Pt))
        return set_status(ctx, RPCA_ERR_ARG, "solve_factored: NULL argument");
    if (r < 1 || p < 1 || q < 1 || p > m || q > n || r > std::min(p, q))
        return set_status(ctx, RPCA_ERR_ARG, "solve_factored: need 1 <= r <= min(p, q), p <= m, q <= n");
    if (p > INT32_MAX || q > INT32_MAX) return set_status(ctx, RPCA_ERR_ARG, "solve_factored: seed too large");
    if ((q < n && !filter_supported(ctx, (int)p, r, opts->precision)) ||
        (p < m && !filter_supported(ctx, (int)q, r, opts->precision)))
        return set_status(ctx, RPCA_ERR_UNSUPPORTED, "solve_factored: seed size outside the built kernel classes");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    std::vector<int64_t> I, J;
    if ((st = check_sorted_indices(ctx, seed_rows, p, m, "seed_rows", &I)) != RPCA_OK) return st;
    if ((st = check_sorted_indices(ctx, seed_cols, q, n, "seed_cols", &J)) != RPCA_OK) return st;
    const std::vector<int64_t> Ic = complement_of(I, m), Jc = complement_of(J, n);
    const int64_t mc = (int64_t)Ic.size(), nc = (int64_t)Jc.size();
    // workspace: Ic, Jc (int64) | iteration codes (nc + mc, int32)
    const size_t bytes = (size_t)(mc + nc) * 8 + (size_t)(nc + mc) * 4 + 256;
    if ((st = ensure_buf(ctx, ctx->solve_ws, bytes)) != RPCA_OK) return st;
    int64_t *dIc = static_cast<int64_t *>(ctx->solve_ws.ptr), *dJc = dIc + mc;
    int32_t *dit = reinterpret_cast<int32_t *>(dJc + nc);
    hipStream_t sm = stream;
    if (mc) RPCA_HIP_TRY(ctx, hipMemcpyAsync(dIc, Ic.data(), mc * 8, hipMemcpyHostToDevice, sm));
    if (nc) RPCA_HIP_TRY(ctx, hipMemcpyAsync(dJc, Jc.data(), nc * 8, hipMemcpyHostToDevice, sm));

    // Step 2: seed, straight into the caller's factor buffers.
    const auto t0 = std::chrono::steady_clock::now();
    SeedOut so;
    const int seed_st = run_seed(ctx, M, ldm, seed_rows, p, seed_cols, q, r, *opts, U, sigma, V, &so, sm);
    const auto t1 = std::chrono::steady_clock::now();
    if (seed_st < 0) return seed_st;
    const std::string seed_msg = ctx->last_error;
    const int ru = so.r_used;

    // Steps 3 and 4 (one launch when both families share a class); outputs
    // packed with leading dimension r_used.
    FilterSide sides[2]{};
    int ns = 0;
    if (nc) sides[ns++] = FilterSide{M, seed_rows, dJc, 1, ldm, m, n, U, (int32_t)p, (int32_t)p, ru, nc, Qt, ru, dit};
    if (mc) sides[ns++] = FilterSide{M, seed_cols, dIc, ldm, 1, n, m, V, (int32_t)q, (int32_t)q, ru, mc, Pt, ru, dit + nc};
    FilterConsts c = consts_of(*opts);
    c.plan_regs = nc + mc;
    RPCA_HIP_TRY(ctx, hipEventRecord(ctx->ev[0], sm));
    if (ns == 2 && !filter_same_class(sides[0].p, sides[0].r, sides[1].p, sides[1].r)) {
        if ((st = launch_filter(ctx, &sides[0], 1, c, sm)) != RPCA_OK) return st;
        if ((st = launch_filter(ctx, &sides[1], 1, c, sm)) != RPCA_OK) return st;
    } else if (ns > 0) {
        if ((st = launch_filter(ctx, sides, ns, c, sm)) != RPCA_OK) return st;
    }
    RPCA_HIP_TRY(ctx, hipEventRecord(ctx->ev[1], sm));
    if (col_iters && nc) RPCA_HIP_TRY(ctx, hipMemcpyAsync(col_iters, dit, nc * 4, hipMemcpyDeviceToDevice, sm));
    if (row_iters && mc) RPCA_HIP_TRY(ctx, hipMemcpyAsync(row_iters, dit + nc, mc * 4, hipMemcpyDeviceToDevice, sm));
    std::vector<int32_t> its((size_t)(nc + mc));
    if (!its.empty())
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(its.data(), dit, its.size() * 4, hipMemcpyDeviceToHost, sm));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(sm));
    const IterSummary is = summarize_iters(its.data(), its.size());
    if (info) {
        float tf = 0;
        (void)hipEventElapsedTime(&tf, ctx->ev[0], ctx->ev[1]);
        info->r_used = ru;
        info->seed_iters = so.iters;
        info->seed_converged = so.converged;
        info->seed_route = so.route;
        info->filt_iters_max = is.max;
        info->filt_iters_total = is.total;
        info->filt_not_converged = is.not_converged;
        info->t_seed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info->t_filter_ms = tf;
        info->t_reconstruct_ms = 0.0;
    }
    if (is.nonfinite)
        return set_status(ctx, RPCA_ERR_NUMERIC, std::to_string(is.nonfinite) +
                                                     " regressions read a non-finite entry of M");
    if (seed_st > 0) return set_status(ctx, seed_st, seed_msg);
    if (is.not_converged)
        return set_status(ctx, RPCA_WARN_NOT_CONVERGED,
                          std::to_string(is.not_converged) + " regressions missed filt_eps");
    return RPCA_OK;
}

int rpca_filter_new_cols(rpca_ctx_t ctx, const float *Mnew, int64_t m, int64_t nnew, int64_t ldm,
                         const int64_t *seed_rows, int64_t p, const double *U, const double *sigma,
                         int32_t r, const float *Pt, const rpca_opts *opts, float *Qt_new,
                         int32_t *iters, float *L, int64_t ldl, float *S, int64_t lds,
                         hipStream_t stream)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    int st;
    if ((st = check_matrix(ctx, Mnew, m, nnew, ldm, "Mnew")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, L, m, nnew, ldl, "L")) != RPCA_OK) return st;
    if ((st = check_matrix(ctx, S, m, nnew, lds, "S")) != RPCA_OK) return st;
    if (!opts) return set_status(ctx, RPCA_ERR_ARG, "filter_new_cols: NULL opts");
    if ((st = check_opts(ctx, *opts)) != RPCA_OK) return st;
    if (!seed_rows || !U || !sigma || !Qt_new || (p < m && !Pt))
        return set_status(ctx, RPCA_ERR_ARG, "filter_new_cols: NULL argument");
    if (p < 1 || p > m || r < 1 || r > p || p > INT32_MAX)
        return set_status(ctx, RPCA_ERR_ARG, "filter_new_cols: need 1 <= r <= p <= m");
    if ((const void *)L == (const void *)S || (const void *)L == (const void *)Mnew ||
        (const void *)S == (const void *)Mnew)
        return set_status(ctx, RPCA_ERR_ARG, "filter_new_cols: L, S and Mnew must be distinct buffers");
    if (!filter_supported(ctx, (int)p, r, opts->precision))
        return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter_new_cols: p = " + std::to_string(p) +
                                                         ", r = " + std::to_string(r) +
                                                         " outside the built kernel classes");
    if (r > 64) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter_new_cols: rank above 64");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    if ((st = ensure_buf(ctx, ctx->iota_ws, (size_t)nnew * sizeof(int64_t))) != RPCA_OK) return st;
    int64_t *cols = static_cast<int64_t *>(ctx->iota_ws.ptr);
    if ((st = launch_iota(ctx, cols, nnew, stream)) != RPCA_OK) return st;
    // Step 3 on the new columns (every column of Mnew is a J_c column) ...
    FilterSide s{Mnew, seed_rows, cols, 1, ldm, m, nnew, U, (int32_t)p, (int32_t)p, r, nnew, Qt_new,
                 r, iters, nullptr, nullptr};
    FilterConsts c = consts_of(*opts);
    c.plan_regs = nnew;
    if ((st = launch_filter(ctx, &s, 1, c, stream)) != RPCA_OK) return st;
    // ... and the completion of those columns only: F from the fit's rows
    // (U Sigma on I_s, P~^T on I_c), G = Q~_new^T Sigma^-1 (no seed columns
    // among them, q = 0).
    ReconArgs a{Mnew, m, nnew, ldm, seed_rows, p, nullptr, 0, U, sigma, nullptr, r, Qt_new, Pt,
                L, ldl, S, lds};
    return launch_reconstruct(ctx, a, stream);
}

} // extern "C"
