// Host runtime of the batched form: checks, workspace layout, the work queue
// of the lane-form filter, the completion tables, and HIP graph replay.
#include "rpca_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

namespace {

// Index checks and complements on host copies (as rpca_solve does).
int fetch_sorted(rpca_ctx *ctx, const int64_t *dev, int64_t count, int64_t bound,
                 const std::string &name, std::vector<int64_t> &out, hipStream_t stream)
{
    out.resize((size_t)count);
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(out.data(), dev, (size_t)count * sizeof(int64_t),
                                     hipMemcpyDeviceToHost, stream));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(stream));
    for (int64_t i = 0; i < count; ++i) {
        if (out[i] < 0 || out[i] >= bound) return set_status(ctx, RPCA_ERR_ARG, name + ": index out of range");
        if (i > 0 && out[i] <= out[i - 1])
            return set_status(ctx, RPCA_ERR_ARG, name + ": indices must be sorted and distinct");
    }
    return RPCA_OK;
}

std::vector<int64_t> complement_sorted(const std::vector<int64_t> &idx, int64_t bound)
{
    std::vector<int64_t> c;
    c.reserve((size_t)(bound - (int64_t)idx.size()));
    size_t a = 0;
    for (int64_t i = 0; i < bound; ++i) {
        if (a < idx.size() && idx[a] == i) ++a;
        else c.push_back(i);
    }
    return c;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Relative per-iteration cost of one lane-form regression, in SIMD cycles:
// 6 VALU ops per element (4 cycles each per 64 lanes), ceil(r/4) 4x4x1 MFMAs
// per element for w and 4 ceil(r/4) per element quad for v (8 cycles each
// per 64 lanes).  Used to order the work queue (costliest sides first).
double lane_reg_cost(int p, int r)
{
    const int P4 = (p + 3) / 4, RB = (r + 3) / 4;
    return P4 * (96.0 + 64.0 * RB) / 64.0;
}

// Lanes per regression of a lane-form side with p elements.
int lane_lpr(const rpca_batch_tuning &t, int64_t p)
{
    return p > t.lane_split4_p ? 4 : (p > t.lane_split2_p ? 2 : 1);
}

} // namespace

struct BatchJobState {
    int64_t mc = 0, nc = 0;        // complement sizes
    int R4 = 4;                    // completion padding (from r)
    bool lane_cols = false, lane_rows = false;
    // byte offsets into the batch workspace
    size_t o_Ic = 0, o_Jc = 0, o_U = 0, o_sig = 0, o_V = 0, o_Qt = 0, o_Pt = 0, o_it = 0, o_F = 0;
    SeedOut so;
    int seed_status = 0;
    double t_seed_ms = 0;
};

// eigen-route seed blocks of one batch that run side by side (helper contexts)
constexpr int kSeedHelpers = 4;

struct rpca_batch {
    rpca_ctx *ctx = nullptr;       // owner context (seed solver, BLAS handle)
    rpca_ctx *wctx = nullptr;      // the batch's own workspace for tile-form / large-rank launches
    std::vector<rpca_job> jobs;
    std::vector<BatchJobState> js;
    rpca_opts opts{};
    rpca_batch_tuning tun{};
    DevBuf ws;                     // per-job arrays
    DevBuf tables;                 // queue, side and completion tables
    DevBuf seed_ws;                // batched seed solver
    BatchTables bt{};
    bool seeded = false;
    int64_t runs = 0;
    hipStream_t bs = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t ev[5] = {};
    std::vector<rpca_ctx *> helpers;      // contexts of the eigen-route seeds run side by side
    std::vector<hipStream_t> hstreams;    // and their streams
    std::vector<FilterSide> tile_sides;   // sides in the tile form (one launch each)
    std::vector<ReconArgs> single_recon;  // completions with R4 > 8 (one launch each)

    char *at(size_t off) const { return static_cast<char *>(ws.ptr) + off; }
};

namespace {

void drop_graphs(rpca_batch *b)
{
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
        b->exec[i] = nullptr;
        b->graph[i] = nullptr;
    }
}

int fail(rpca_batch *b, int st)
{
    // errors of the batch's own workspace context are reported on the owner
    if (b->wctx && !b->wctx->last_error.empty()) {
        b->ctx->last_error = b->wctx->last_error;
        b->wctx->last_error.clear();
    }
    return st;
}

int enqueue_filter(rpca_batch *b, hipStream_t s)
{
    const FilterConsts c = consts_of(b->opts);
    int st = launch_lane_filter(b->wctx, b->bt, c, s);
    if (st != RPCA_OK) return fail(b, st);
    for (const FilterSide &fs : b->tile_sides)
        if ((st = launch_filter(b->wctx, &fs, 1, c, s)) != RPCA_OK) return fail(b, st);
    return RPCA_OK;
}

int enqueue_recon(rpca_batch *b, hipStream_t s)
{
    int st = launch_batch_reconstruct(b->wctx, b->bt, s);
    if (st != RPCA_OK) return fail(b, st);
    for (const ReconArgs &a : b->single_recon)
        if ((st = launch_reconstruct(b->wctx, a, s)) != RPCA_OK) return fail(b, st);
    return RPCA_OK;
}

// Build the device tables of the filter queue and of the batched completion
// from the seed ranks.
int build_tables(rpca_batch *b)
{
    rpca_ctx *ctx = b->ctx;
    const int64_t nj = (int64_t)b->jobs.size();
    std::vector<LaneSide> sides;
    std::vector<double> side_cost;
    b->tile_sides.clear();
    b->single_recon.clear();
    std::vector<ReconJob> rjobs;

    for (int64_t j = 0; j < nj; ++j) {
        const rpca_job &J = b->jobs[j];
        BatchJobState &S = b->js[j];
        const int ru = S.so.r_used;
        const int64_t *dIc = reinterpret_cast<const int64_t *>(b->at(S.o_Ic));
        const int64_t *dJc = reinterpret_cast<const int64_t *>(b->at(S.o_Jc));
        const double *dU = reinterpret_cast<const double *>(b->at(S.o_U));
        const double *dsig = reinterpret_cast<const double *>(b->at(S.o_sig));
        const double *dV = reinterpret_cast<const double *>(b->at(S.o_V));
        float *dQt = reinterpret_cast<float *>(b->at(S.o_Qt));
        float *dPt = reinterpret_cast<float *>(b->at(S.o_Pt));
        int32_t *dit = reinterpret_cast<int32_t *>(b->at(S.o_it));
        // column side: elements = seed rows (p), regressions = J_c, basis U
        if (S.nc > 0) {
            if (S.lane_cols) {
                LaneSide ls{J.M, J.seed_rows, dJc, 1, J.ldm, J.m, J.n, dU, S.nc, dQt, ru, dit,
                            (int32_t)J.p, (int32_t)J.p, ru,
                            lane_class((int)J.p, ru, lane_lpr(b->tun, J.p))};
                sides.push_back(ls);
                side_cost.push_back(lane_reg_cost((int)J.p, ru));
            } else {
                b->tile_sides.push_back(FilterSide{J.M, J.seed_rows, dJc, 1, J.ldm, J.m, J.n, dU,
                                                   (int32_t)J.p, (int32_t)J.p, ru, S.nc, dQt, ru,
                                                   dit, nullptr});
            }
        }
        // row side: elements = seed columns (q), regressions = I_c, basis V
        if (S.mc > 0) {
            if (S.lane_rows) {
                LaneSide ls{J.M, J.seed_cols, dIc, J.ldm, 1, J.n, J.m, dV, S.mc, dPt, ru,
                            dit + S.nc, (int32_t)J.q, (int32_t)J.q, ru,
                            lane_class((int)J.q, ru, lane_lpr(b->tun, J.q))};
                sides.push_back(ls);
                side_cost.push_back(lane_reg_cost((int)J.q, ru));
            } else {
                b->tile_sides.push_back(FilterSide{J.M, J.seed_cols, dIc, J.ldm, 1, J.n, J.m, dV,
                                                   (int32_t)J.q, (int32_t)J.q, ru, S.mc, dPt, ru,
                                                   dit + S.nc, nullptr});
            }
        }
        ReconArgs a{J.M, J.m, J.n, J.ldm, J.seed_rows, J.p, J.seed_cols, J.q, dU, dsig, dV, ru,
                    dQt, dPt, J.L, J.ldl, J.S, J.lds};
        const int R4 = (ru + 3) / 4 * 4;   // <= S.R4, the class the workspace was laid out for
        if (S.R4 <= 8) {
            ReconJob rj{};
            rj.M = J.M;
            rj.L = J.L;
            rj.S = J.S;
            rj.F = reinterpret_cast<const float *>(b->at(S.o_F));
            rj.G = rj.F + (size_t)J.m * R4;
            rj.m = J.m;
            rj.n = J.n;
            rj.ldm = J.ldm;
            rj.ldl = J.ldl;
            rj.lds = J.lds;
            rj.seed_rows = J.seed_rows;
            rj.seed_cols = J.seed_cols;
            rj.p = J.p;
            rj.q = J.q;
            rj.U = dU;
            rj.sigma = dsig;
            rj.V = dV;
            rj.Qt = dQt;
            rj.Pt = dPt;
            rj.r = ru;
            rj.R4 = R4;
            rj.vec = (J.ldm % 4 == 0) && (J.ldl % 4 == 0) && (J.lds % 4 == 0) &&
                     ((uintptr_t)J.M % 16 == 0) && ((uintptr_t)J.L % 16 == 0) &&
                     ((uintptr_t)J.S % 16 == 0);
            const int64_t cpw = std::max<int32_t>(1, b->tun.recon_cols_per_wave);
            rj.row_blocks = (uint32_t)((J.m + 255) / 256);
            // waves per row block: one per recon_cols_per_wave columns, at most one
            // per batch of 4 columns (the unit a completion wave takes)
            rj.col_parts = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((J.n + 3) / 4, (J.n + cpw - 1) / cpw));
            rjobs.push_back(rj);
        } else {
            b->single_recon.push_back(a);
        }
    }

    // work queue: items of 64 / LPR regressions, costliest sides first (or job order)
    std::vector<int32_t> order(sides.size());
    std::iota(order.begin(), order.end(), 0);
    if (b->tun.order == 0)
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t x, int32_t y) { return side_cost[x] > side_cost[y]; });
    // (one queue per register group: the classes whose kernel fits three waves
    // per SIMD, then the rest)
    std::vector<int32_t> items, items1;
    for (int32_t sidx : order) {
        const int64_t nreg = sides[sidx].nreg;
        const int64_t per = lane_regs_per_item(sides[sidx].cls);
        std::vector<int32_t> &q = lane_group(sides[sidx].cls) == 0 ? items : items1;
        for (int64_t f = 0; f < nreg; f += per) {
            if (f > INT32_MAX) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "batch: too many regressions in one side");
            q.push_back(sidx);
            q.push_back((int32_t)f);
        }
    }
    const int64_t nitems0 = (int64_t)items.size() / 2;
    items.insert(items.end(), items1.begin(), items1.end());
    const int64_t nitems = (int64_t)items.size() / 2;
    if (nitems > INT32_MAX) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "batch: too many work items");

    // completion tables
    std::vector<int32_t> asm_job, rec_job;
    std::vector<int64_t> asm_first;
    std::vector<uint32_t> rec_local;
    for (size_t k = 0; k < rjobs.size(); ++k) {
        const ReconJob &rj = rjobs[k];
        const int64_t units = (rj.m + rj.n) * (rj.R4 / 4);   // one row, 4 ranks each
        for (int64_t f = 0; f < units; f += 256) {
            asm_job.push_back((int32_t)k);
            asm_first.push_back(f);
        }
        const uint64_t waves = (uint64_t)rj.row_blocks * rj.col_parts;
        if (waves > UINT32_MAX) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "batch: completion grid too large");
        for (uint64_t w = 0; w < waves; ++w) {
            rec_job.push_back((int32_t)k);
            rec_local.push_back((uint32_t)w);
        }
    }
    if (asm_job.size() > (size_t)INT32_MAX || rec_job.size() > (size_t)INT32_MAX)
        return set_status(ctx, RPCA_ERR_UNSUPPORTED, "batch: completion grid too large");

    // one device buffer: sides | items | counter | jobs | asm tables | rec tables
    size_t off = 0;
    const size_t o_sides = off; off = align_up(off + sides.size() * sizeof(LaneSide), 256);
    const size_t o_items = off; off = align_up(off + items.size() * sizeof(int32_t), 256);
    const size_t o_ctr = off;   off = align_up(off + 256, 256);
    const size_t o_jobs = off;  off = align_up(off + rjobs.size() * sizeof(ReconJob), 256);
    const size_t o_aj = off;    off = align_up(off + asm_job.size() * sizeof(int32_t), 256);
    const size_t o_af = off;    off = align_up(off + asm_first.size() * sizeof(int64_t), 256);
    const size_t o_rj = off;    off = align_up(off + rec_job.size() * sizeof(int32_t), 256);
    const size_t o_rl = off;    off = align_up(off + rec_local.size() * sizeof(uint32_t), 256);
    int st = ensure_buf(ctx, b->tables, off);
    if (st != RPCA_OK) return st;
    char *base = static_cast<char *>(b->tables.ptr);
    auto put = [&](size_t o, const void *src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(base + o, src, bytes, hipMemcpyHostToDevice, b->bs) : hipSuccess;
    };
    RPCA_HIP_TRY(ctx, put(o_sides, sides.data(), sides.size() * sizeof(LaneSide)));
    RPCA_HIP_TRY(ctx, put(o_items, items.data(), items.size() * sizeof(int32_t)));
    RPCA_HIP_TRY(ctx, put(o_jobs, rjobs.data(), rjobs.size() * sizeof(ReconJob)));
    RPCA_HIP_TRY(ctx, put(o_aj, asm_job.data(), asm_job.size() * sizeof(int32_t)));
    RPCA_HIP_TRY(ctx, put(o_af, asm_first.data(), asm_first.size() * sizeof(int64_t)));
    RPCA_HIP_TRY(ctx, put(o_rj, rec_job.data(), rec_job.size() * sizeof(int32_t)));
    RPCA_HIP_TRY(ctx, put(o_rl, rec_local.data(), rec_local.size() * sizeof(uint32_t)));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));     // the host vectors die here

    BatchTables &t = b->bt;
    t.sides = reinterpret_cast<const LaneSide *>(base + o_sides);
    t.items = reinterpret_cast<const int32_t *>(base + o_items);
    t.nitems = (int32_t)nitems;
    t.nitems0 = (int32_t)nitems0;
    t.counter = reinterpret_cast<uint32_t *>(base + o_ctr);
    // filter_waves_per_cu: persistent waves per CU at two waves per SIMD; the
    // three-wave group gets half as many again
    const int64_t wpc = b->tun.filter_waves_per_cu > 0 ? b->tun.filter_waves_per_cu : 8;
    const int64_t ncu = std::max(1, ctx->num_cu);
    t.grid_waves[0] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nitems0, (3 * wpc + 1) / 2 * ncu));
    t.grid_waves[1] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(nitems - nitems0, wpc * ncu));
    t.jobs = reinterpret_cast<const ReconJob *>(base + o_jobs);
    t.asm_block_job = reinterpret_cast<const int32_t *>(base + o_aj);
    t.asm_block_first = reinterpret_cast<const int64_t *>(base + o_af);
    t.asm_blocks = (int32_t)asm_job.size();
    t.rec_block_job = reinterpret_cast<const int32_t *>(base + o_rj);
    t.rec_block_local = reinterpret_cast<const uint32_t *>(base + o_rl);
    t.rec_blocks = (int32_t)rec_job.size();
    // at most recon_waves_per_cu completion waves per CU: each reserves its share of the LDS
    const size_t lds_cu = ctx->max_lds ? ctx->max_lds : 65536;
    t.rec_lds_bytes = b->tun.recon_waves_per_cu > 0
                          ? (int32_t)((lds_cu / (size_t)b->tun.recon_waves_per_cu) & ~(size_t)255)
                          : 0;
    return RPCA_OK;
}

} // namespace

int batch_check_tuning(rpca_ctx *ctx, const rpca_batch_tuning &tun)
{
    if (tun.lane_max_p < 0 || tun.lane_max_p > kLaneMaxP || tun.lane_max_r < 0 ||
        tun.lane_max_r > kLaneMaxR || tun.lane_split2_p < 0 || tun.lane_split2_p > 32 ||
        tun.lane_split4_p < tun.lane_split2_p || tun.lane_split4_p > 64 ||
        tun.filter_waves_per_cu < 0 || tun.filter_waves_per_cu > 64 ||
        tun.recon_cols_per_wave < 1 || tun.recon_waves_per_cu < 0 || tun.recon_waves_per_cu > 64 ||
        (tun.order != 0 && tun.order != 1) ||
        (tun.graph != 0 && tun.graph != 1) || (tun.seed_batched != 0 && tun.seed_batched != 1))
        return set_status(ctx, RPCA_ERR_ARG, "batch: bad tuning");
    return RPCA_OK;
}

rpca_batch *batch_new(rpca_ctx *ctx, const rpca_opts &o, const rpca_batch_tuning &tun, int *status)
{
    *status = check_opts(ctx, o);
    if (*status != RPCA_OK) return nullptr;
    if ((*status = batch_check_tuning(ctx, tun)) != RPCA_OK) return nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) {
        *status = set_status(ctx, RPCA_ERR_DEVICE, "batch: hipSetDevice failed");
        return nullptr;
    }
    rpca_batch *b = new rpca_batch();
    b->ctx = ctx;
    b->opts = o;
    b->tun = tun;
    // the batch's own launch workspace, stream and events
    b->wctx = new rpca_ctx();
    b->wctx->device = ctx->device;
    b->wctx->num_cu = ctx->num_cu;
    b->wctx->max_lds = ctx->max_lds;
    b->wctx->recon_waves_per_cu = ctx->recon_waves_per_cu;
    bool ok = hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking) == hipSuccess;
    for (auto &e : b->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    // the second stream of the lane filter, made here and not on first use,
    // so that no run, captured or not, creates a stream
    ok = ok && ensure_aux(b->wctx) == RPCA_OK;
    if (!ok) {
        *status = set_status(ctx, RPCA_ERR_DEVICE, "batch: stream or event creation failed");
        rpca_batch_destroy(b);
        return nullptr;
    }
    *status = RPCA_OK;
    return b;
}

hipStream_t batch_stream(rpca_batch *b) { return b->bs; }

// Order the batch stream after the work already enqueued on `stream`.
int order_after(rpca_batch *b, hipStream_t stream)
{
    RPCA_HIP_TRY(b->ctx, hipEventRecord(b->ev[4], stream));
    RPCA_HIP_TRY(b->ctx, hipStreamWaitEvent(b->bs, b->ev[4], 0));
    return RPCA_OK;
}

int batch_plan(rpca_batch *b, const rpca_job *jobs, int64_t njobs, hipStream_t stream)
{
    rpca_ctx *ctx = b->ctx;
    const rpca_batch_tuning &tun = b->tun;
    const rpca_opts &o = b->opts;
    if (!jobs || njobs < 1) return set_status(ctx, RPCA_ERR_ARG, "batch: need at least one job");
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));
    int ost = order_after(b, stream);      // the index arrays may still be in flight there
    if (ost != RPCA_OK) return ost;
    drop_graphs(b);
    b->seeded = false;
    b->runs = 0;
    b->jobs.assign(jobs, jobs + njobs);
    b->js.assign((size_t)njobs, BatchJobState{});

    // checks and workspace layout
    std::vector<std::vector<int64_t>> Ic((size_t)njobs), Jc((size_t)njobs);
    size_t off = 0;
    for (int64_t j = 0; j < njobs; ++j) {
        const rpca_job &J = b->jobs[j];
        BatchJobState &S = b->js[j];
        const std::string nm = "batch job " + std::to_string(j);
        if (!J.M || !J.L || !J.S || !J.seed_rows || !J.seed_cols)
            return set_status(ctx, RPCA_ERR_ARG, nm + ": NULL pointer");
        if (J.m < 1 || J.n < 1 || J.ldm < J.m || J.ldl < J.m || J.lds < J.m)
            return set_status(ctx, RPCA_ERR_ARG, nm + ": bad sizes or leading dimensions");
        if (J.r < 1 || J.p < 1 || J.q < 1 || J.p > J.m || J.q > J.n || J.r > std::min(J.p, J.q))
            return set_status(ctx, RPCA_ERR_ARG, nm + ": need 1 <= r <= min(p, q), p <= m, q <= n");
        if ((const void *)J.L == (const void *)J.S || (const void *)J.L == (const void *)J.M ||
            (const void *)J.S == (const void *)J.M)
            return set_status(ctx, RPCA_ERR_ARG, nm + ": L, S and M must be distinct buffers");
        std::vector<int64_t> I, Jv;
        int st = fetch_sorted(ctx, J.seed_rows, J.p, J.m, nm + " seed_rows", I, b->bs);
        if (st != RPCA_OK) return st;
        if ((st = fetch_sorted(ctx, J.seed_cols, J.q, J.n, nm + " seed_cols", Jv, b->bs)) != RPCA_OK) return st;
        Ic[j] = complement_sorted(I, J.m);
        Jc[j] = complement_sorted(Jv, J.n);
        S.mc = (int64_t)Ic[j].size();
        S.nc = (int64_t)Jc[j].size();
        // filter form of each side; the completion's rank class
        // lane form: small seeds, and regression offsets (column j: j ldm, row
        // i: i) that fit 32-bit byte offsets
        const bool lane_r = J.r <= tun.lane_max_r;
        const bool cols32 = (J.n - 1) * J.ldm * 4 + 4 <= (int64_t)UINT32_MAX;
        const bool rows32 = (J.m - 1) * 4 + 4 <= (int64_t)UINT32_MAX;
        S.lane_cols = lane_r && cols32 && J.p <= tun.lane_max_p &&
                      lane_class((int)J.p, J.r, lane_lpr(tun, J.p)) >= 0;
        S.lane_rows = lane_r && rows32 && J.q <= tun.lane_max_p &&
                      lane_class((int)J.q, J.r, lane_lpr(tun, J.q)) >= 0;
        for (int rr = 1; rr <= J.r; ++rr) {   // any seed rank up to r must have a kernel
            if ((!S.lane_cols && S.nc > 0 && !filter_supported(ctx, (int)J.p, rr, o.precision)) ||
                (!S.lane_rows && S.mc > 0 && !filter_supported(ctx, (int)J.q, rr, o.precision)))
                return set_status(ctx, RPCA_ERR_UNSUPPORTED, nm + ": seed size outside the built kernel classes");
        }
        S.R4 = (J.r + 3) / 4 * 4;
        if (S.R4 > 64) return set_status(ctx, RPCA_ERR_UNSUPPORTED, nm + ": rank above 64");
        S.o_Ic = off; off = align_up(off + (size_t)S.mc * 8, 256);
        S.o_Jc = off; off = align_up(off + (size_t)S.nc * 8, 256);
        S.o_U = off;  off = align_up(off + (size_t)J.p * J.r * 8, 256);
        S.o_sig = off; off = align_up(off + (size_t)J.r * 8, 256);
        S.o_V = off;  off = align_up(off + (size_t)J.q * J.r * 8, 256);
        S.o_Qt = off; off = align_up(off + (size_t)S.nc * J.r * 4, 256);
        S.o_Pt = off; off = align_up(off + (size_t)S.mc * J.r * 4, 256);
        S.o_it = off; off = align_up(off + (size_t)(S.nc + S.mc) * 4, 256);
        S.o_F = off;
        if (S.R4 <= 8) off = align_up(off + (size_t)(J.m + J.n) * S.R4 * 4, 256);
    }
    int st = ensure_buf(ctx, b->ws, std::max<size_t>(off, 256));
    if (st != RPCA_OK) return st;
    for (int64_t j = 0; j < njobs; ++j) {
        const BatchJobState &S = b->js[j];
        if (S.mc) RPCA_HIP_TRY(ctx, hipMemcpyAsync(b->at(S.o_Ic), Ic[j].data(), S.mc * 8, hipMemcpyHostToDevice, b->bs));
        if (S.nc) RPCA_HIP_TRY(ctx, hipMemcpyAsync(b->at(S.o_Jc), Jc[j].data(), S.nc * 8, hipMemcpyHostToDevice, b->bs));
    }
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));
    return RPCA_OK;
}

extern "C" {

void rpca_batch_tuning_default(rpca_batch_tuning *t)
{
    if (!t) return;
    t->lane_max_p = kLaneMaxP;
    t->lane_max_r = kLaneMaxR;
    t->lane_split2_p = 32;
    t->lane_split4_p = 64;
    t->filter_waves_per_cu = 8;
    t->recon_cols_per_wave = 32;
    t->order = 0;
    t->graph = 1;
    t->seed_batched = 1;
    t->recon_waves_per_cu = 4;
}

int rpca_batch_create(rpca_ctx_t ctx, const rpca_job *jobs, int64_t njobs, const rpca_opts *opts,
                      const rpca_batch_tuning *tuning, rpca_batch_t *out)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    if (!out) return set_status(ctx, RPCA_ERR_ARG, "batch: NULL output handle");
    *out = nullptr;
    if (!jobs || njobs < 1) return set_status(ctx, RPCA_ERR_ARG, "batch: need at least one job");
    if (!opts) return set_status(ctx, RPCA_ERR_ARG, "batch: NULL opts");
    rpca_batch_tuning tun;
    rpca_batch_tuning_default(&tun);
    if (tuning) tun = *tuning;
    int st = RPCA_OK;
    rpca_batch *b = batch_new(ctx, *opts, tun, &st);
    if (!b) return st;
    if ((st = batch_plan(b, jobs, njobs, nullptr)) != RPCA_OK) {
        rpca_batch_destroy(b);
        return st;
    }
    *out = b;
    return RPCA_OK;
}

int rpca_batch_seed(rpca_batch_t b, hipStream_t stream)
{
    if (!b) return RPCA_ERR_ARG;
    rpca_ctx *ctx = b->ctx;
    ctx->last_error.clear();
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));
    int ost = order_after(b, stream);      // M may still be in flight there
    if (ost != RPCA_OK) return ost;
    b->seeded = false;
    drop_graphs(b);
    int worst = RPCA_OK;
    std::string worst_msg;
    auto note = [&](size_t j, int st, const std::string &msg) -> int {
        if (st < 0) return set_status(ctx, st, "batch job " + std::to_string(j) + ": " + msg);
        if (st > 0 && worst == RPCA_OK) {
            worst = st;
            worst_msg = "batch job " + std::to_string(j) + ": " + msg;
        }
        return RPCA_OK;
    };
    auto dU = [&](size_t j) { return reinterpret_cast<double *>(b->at(b->js[j].o_U)); };
    auto dsig = [&](size_t j) { return reinterpret_cast<double *>(b->at(b->js[j].o_sig)); };
    auto dV = [&](size_t j) { return reinterpret_cast<double *>(b->at(b->js[j].o_V)); };

    // small seed blocks: all in one launch of the batched solver
    std::vector<size_t> small;
    std::vector<SmallSeedArgs> args;
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        const rpca_job &J = b->jobs[j];
        if (!b->tun.seed_batched || !seed_small_fits(ctx, J.p, J.q)) continue;
        small.push_back(j);
        args.push_back(SmallSeedArgs{J.M, J.ldm, J.seed_rows, J.seed_cols, J.p, J.q, J.r, dU(j),
                                     dsig(j), dV(j)});
    }
    if (!small.empty()) {
        const auto t0 = std::chrono::steady_clock::now();
        int st = ensure_buf(ctx, b->seed_ws, seed_small_workspace(args.data(), (int)args.size()));
        if (st != RPCA_OK) return st;
        std::vector<SeedOut> outs(small.size());
        std::vector<int> sts(small.size());
        st = run_seed_small(ctx, args.data(), (int)args.size(), b->opts, b->seed_ws.ptr, outs.data(),
                            sts.data(), b->bs);
        if (st != RPCA_OK) return st;
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (size_t k = 0; k < small.size(); ++k) {
            BatchJobState &S = b->js[small[k]];
            S.so = outs[k];
            S.seed_status = sts[k];
            S.t_seed_ms = ms;              // one launch serves them all
            const char *what = sts[k] == RPCA_ERR_SEED ? "the recovered seed has rank 0"
                             : sts[k] == RPCA_ERR_NUMERIC ? "non-finite entry in the seed block"
                             : sts[k] == RPCA_WARN_RANK ? "rank of L^s differs from the target"
                             : "seed tolerance not met";
            if ((st = note(small[k], sts[k], what)) != RPCA_OK) return st;
        }
    }
    std::vector<char> done(b->jobs.size(), 0), fell_back(b->jobs.size(), 0);
    for (size_t j : small) done[j] = 1;
    // larger blocks (up to 512 x 512): one launch of the device-resident
    // subspace-iteration solver, one workgroup each.  Every such block takes
    // it, however many the batch holds, so that a request's result does not
    // depend on what it is batched with.
    std::vector<size_t> large;
    args.clear();
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        const rpca_job &J = b->jobs[j];
        if (done[j] || !b->tun.seed_batched || b->opts.seed_route == 1 || !seed_large_fits(ctx, J.p, J.q))
            continue;
        large.push_back(j);
        args.push_back(SmallSeedArgs{J.M, J.ldm, J.seed_rows, J.seed_cols, J.p, J.q, J.r, dU(j),
                                     dsig(j), dV(j)});
    }
    if (!large.empty()) {
        const auto t0 = std::chrono::steady_clock::now();
        int st = ensure_buf(ctx, b->seed_ws, seed_large_workspace(args.data(), (int)args.size()));
        if (st != RPCA_OK) return st;
        std::vector<SeedOut> outs(large.size());
        std::vector<int> sts(large.size());
        st = run_seed_large(ctx, args.data(), (int)args.size(), b->opts, b->seed_ws.ptr, outs.data(),
                            sts.data(), b->bs);
        if (st != RPCA_OK) return st;
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (size_t k = 0; k < large.size(); ++k) {
            if (outs[k].fallback) {                  // taken again by the route below
                fell_back[large[k]] = 1;
                continue;
            }
            BatchJobState &S = b->js[large[k]];
            S.so = outs[k];
            S.seed_status = seed_status_message(ctx, sts[k], outs[k], b->jobs[large[k]].r);
            S.t_seed_ms = ms;
            done[large[k]] = 1;
            if ((st = note(large[k], S.seed_status, ctx->last_error)) != RPCA_OK) return st;
        }
    }
    // the others on the eigen-decomposition route.  It synchronises with the
    // host at every ALM step and leaves most of the chip idle, so up to
    // kSeedHelpers blocks run side by side, each on a helper context of its
    // own (BLAS handle, workspace, stream) made once per batch object; a
    // block's result does not depend on the helper that runs it.
    rpca_opts eig = b->opts;
    eig.seed_route = 1;
    std::vector<size_t> rest;
    for (size_t j = 0; j < b->jobs.size(); ++j)
        if (!done[j]) rest.push_back(j);
    const size_t want = std::min(rest.size(), (size_t)kSeedHelpers);
    while (want >= 2 && b->helpers.size() < want) {
        rpca_ctx *h = nullptr;
        hipStream_t hs = nullptr;
        if (rpca_ctx_create(ctx->device, &h) != RPCA_OK) break;
        if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) {
            rpca_ctx_destroy(h);
            break;
        }
        b->helpers.push_back(h);
        b->hstreams.push_back(hs);
    }
    const size_t nh = want >= 2 ? std::min(want, b->helpers.size()) : 0;
    std::vector<std::string> msgs(rest.size());
    auto one = [&](size_t i, rpca_ctx *c, hipStream_t sm) {
        const size_t j = rest[i];
        const rpca_job &J = b->jobs[j];
        BatchJobState &S = b->js[j];
        const auto t0 = std::chrono::steady_clock::now();
        S.so = SeedOut{};
        S.seed_status = run_seed(c, J.M, J.ldm, J.seed_rows, J.p, J.seed_cols, J.q, J.r, eig, dU(j),
                                 dsig(j), dV(j), &S.so, sm);
        if (fell_back[j]) S.so.route = RPCA_SEED_ROUTE_FELL_BACK;
        S.t_seed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        msgs[i] = c->last_error;
    };
    if (nh >= 2) {
        // the helpers' streams do not wait on the batch's: everything queued
        // there (the inputs' ordering, the launches above) is finished first
        RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));
        std::atomic<size_t> next{0};
        auto work = [&](size_t h) {
            (void)hipSetDevice(ctx->device);
            for (size_t i; (i = next.fetch_add(1)) < rest.size();) one(i, b->helpers[h], b->hstreams[h]);
            (void)hipStreamSynchronize(b->hstreams[h]);
        };
        std::vector<std::thread> threads;
        for (size_t h = 1; h < nh; ++h) threads.emplace_back(work, h);
        work(0);
        for (auto &t : threads) t.join();
    } else {
        for (size_t i = 0; i < rest.size(); ++i) one(i, ctx, b->bs);
    }
    for (size_t i = 0; i < rest.size(); ++i) {
        int st = note(rest[i], b->js[rest[i]].seed_status, msgs[i]);
        if (st != RPCA_OK) return st;
    }
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));
    int st = build_tables(b);
    if (st != RPCA_OK) return st;
    b->seeded = true;
    b->runs = 0;
    if (worst != RPCA_OK) return set_status(ctx, worst, worst_msg);
    ctx->last_error.clear();
    return RPCA_OK;
}

int rpca_batch_run(rpca_batch_t b, hipStream_t stream)
{
    if (!b) return RPCA_ERR_ARG;
    rpca_ctx *ctx = b->ctx;
    ctx->last_error.clear();
    if (!b->seeded) return set_status(ctx, RPCA_ERR_ARG, "batch: run before a successful rpca_batch_seed");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    // order after the caller's stream, run on the batch's stream, order back
    RPCA_HIP_TRY(ctx, hipEventRecord(b->ev[3], stream));
    RPCA_HIP_TRY(ctx, hipStreamWaitEvent(b->bs, b->ev[3], 0));
    int st;
    if (b->tun.graph && b->runs >= 1 && !b->exec[0]) {
        // capture once the first (eager) run has sized every workspace
        for (int g = 0; g < 2; ++g) {
            RPCA_HIP_TRY(ctx, hipStreamBeginCapture(b->bs, hipStreamCaptureModeThreadLocal));
            st = g == 0 ? enqueue_filter(b, b->bs) : enqueue_recon(b, b->bs);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(b->bs, &graph);
            if (st != RPCA_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                drop_graphs(b);
                return st;
            }
            if (e != hipSuccess) {
                drop_graphs(b);
                return set_status(ctx, RPCA_ERR_DEVICE, std::string("batch: graph capture: ") + hipGetErrorString(e));
            }
            b->graph[g] = graph;
            if (hipGraphInstantiate(&b->exec[g], graph, nullptr, nullptr, 0) != hipSuccess) {
                drop_graphs(b);
                return set_status(ctx, RPCA_ERR_DEVICE, "batch: hipGraphInstantiate failed");
            }
        }
    }
    RPCA_HIP_TRY(ctx, hipEventRecord(b->ev[0], b->bs));
    if (b->exec[0]) {
        RPCA_HIP_TRY(ctx, hipGraphLaunch(b->exec[0], b->bs));
        RPCA_HIP_TRY(ctx, hipEventRecord(b->ev[1], b->bs));
        RPCA_HIP_TRY(ctx, hipGraphLaunch(b->exec[1], b->bs));
    } else {
        if ((st = enqueue_filter(b, b->bs)) != RPCA_OK) return st;
        RPCA_HIP_TRY(ctx, hipEventRecord(b->ev[1], b->bs));
        if ((st = enqueue_recon(b, b->bs)) != RPCA_OK) return st;
    }
    RPCA_HIP_TRY(ctx, hipEventRecord(b->ev[2], b->bs));
    RPCA_HIP_TRY(ctx, hipStreamWaitEvent(stream, b->ev[2], 0));
    ++b->runs;
    return RPCA_OK;
}

int rpca_batch_job_info(rpca_batch_t b, int64_t job, rpca_info *info)
{
    if (!b) return RPCA_ERR_ARG;
    rpca_ctx *ctx = b->ctx;
    ctx->last_error.clear();
    if (!info || job < 0 || job >= (int64_t)b->jobs.size())
        return set_status(ctx, RPCA_ERR_ARG, "batch: bad job index or NULL info");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));
    const BatchJobState &S = b->js[job];
    std::vector<int32_t> its((size_t)(S.nc + S.mc));
    IterSummary is;
    if (b->runs > 0 && !its.empty()) {
        RPCA_HIP_TRY(ctx, hipMemcpyAsync(its.data(), b->at(S.o_it), its.size() * 4, hipMemcpyDeviceToHost, b->bs));
        RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));
        is = summarize_iters(its.data(), its.size());
    }
    const int64_t total = is.total, bad = is.not_converged;
    const int32_t kmax = is.max;
    float tf = 0, tr = 0;
    if (b->runs > 0) {
        (void)hipEventElapsedTime(&tf, b->ev[0], b->ev[1]);
        (void)hipEventElapsedTime(&tr, b->ev[1], b->ev[2]);
    }
    info->r_used = S.so.r_used;
    info->seed_iters = S.so.iters;
    info->seed_converged = S.so.converged;
    info->seed_route = S.so.route;
    info->filt_iters_max = kmax;
    info->filt_iters_total = total;
    info->filt_not_converged = bad;
    info->t_seed_ms = S.t_seed_ms;
    info->t_filter_ms = tf;
    info->t_reconstruct_ms = tr;
    if (is.nonfinite)
        return set_status(ctx, RPCA_ERR_NUMERIC, "job " + std::to_string(job) + ": " +
                                                     std::to_string(is.nonfinite) +
                                                     " regressions read a non-finite entry of M");
    return S.seed_status > 0 ? S.seed_status : (bad ? RPCA_WARN_NOT_CONVERGED : RPCA_OK);
}

int rpca_batch_job_factors(rpca_batch_t b, int64_t job, double *U, double *sigma, double *V)
{
    if (!b) return RPCA_ERR_ARG;
    rpca_ctx *ctx = b->ctx;
    ctx->last_error.clear();
    if (job < 0 || job >= (int64_t)b->jobs.size() || !U || !sigma || !V)
        return set_status(ctx, RPCA_ERR_ARG, "batch: bad job index or NULL buffer");
    if (!b->seeded) return set_status(ctx, RPCA_ERR_ARG, "batch: factors before a successful rpca_batch_seed");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));
    const rpca_job &J = b->jobs[job];
    const BatchJobState &S = b->js[job];
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(U, b->at(S.o_U), (size_t)J.p * J.r * 8, hipMemcpyDeviceToDevice, b->bs));
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(sigma, b->at(S.o_sig), (size_t)J.r * 8, hipMemcpyDeviceToDevice, b->bs));
    RPCA_HIP_TRY(ctx, hipMemcpyAsync(V, b->at(S.o_V), (size_t)J.q * J.r * 8, hipMemcpyDeviceToDevice, b->bs));
    RPCA_HIP_TRY(ctx, hipStreamSynchronize(b->bs));
    return RPCA_OK;
}

int rpca_batch_destroy(rpca_batch_t b)
{
    if (!b) return RPCA_ERR_ARG;
    (void)hipSetDevice(b->ctx->device);
    if (b->bs) (void)hipStreamSynchronize(b->bs);
    drop_graphs(b);
    for (DevBuf *d : {&b->ws, &b->tables, &b->seed_ws})
        if (d->ptr) (void)hipFree(d->ptr);
    if (b->wctx) {
        if (b->wctx->aux) (void)hipStreamSynchronize(b->wctx->aux);
        for (DevBuf *d : {&b->wctx->factors, &b->wctx->xbuf_ws, &b->wctx->frag_ws, &b->wctx->scratch,
                          &b->wctx->solve_ws, &b->wctx->seed_ws})
            if (d->ptr) (void)hipFree(d->ptr);
        for (auto &e : b->wctx->pev)
            if (e) (void)hipEventDestroy(e);
        if (b->wctx->aux) (void)hipStreamDestroy(b->wctx->aux);
        delete b->wctx;
    }
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    for (size_t h = 0; h < b->helpers.size(); ++h) {
        (void)hipStreamSynchronize(b->hstreams[h]);
        (void)hipStreamDestroy(b->hstreams[h]);
        rpca_ctx_destroy(b->helpers[h]);
    }
    if (b->bs) (void)hipStreamDestroy(b->bs);
    delete b;
    return RPCA_OK;
}

} // extern "C"
