// Served form: a request loop over the batched form.
//
// Requests (one rpca_job each) enter a FIFO queue.  Each of `workers` host
// threads owns a context (its own rocBLAS handle and workspace), one batch
// plan that is re-planned for every batch (so its device buffers only grow:
// no allocation or free, hence no device-wide synchronisation, in steady
// state) and a non-blocking stream.  A free worker admits requests from the
// head of the queue while the HBM footprint of all admitted, unfinished
// requests stays within the budget (a request larger than the budget is
// admitted alone), up to max_batch of them and to its share of the queue
// (queued requests / workers, rounded up, so a burst is spread over the
// workers instead of becoming one long batch), and runs steps 2-5 for them as
// one batch on its stream.  Requests that arrive while batches are on the GPU are
// taken by the next free worker, so batches of different workers overlap on
// the device.  A batch that fails as a whole (a bad index array, a seed of
// rank 0) is retried one request at a time, so one bad request never fails
// the others.
#include "rpca_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

struct Request {
    rpca_job job{};
    size_t footprint = 0;
    bool done = false;
    rpca_request_info info{};
};

// Device bytes a request keeps busy while admitted: its M, L and S, and the
// batch workspace it needs (indices, seed factors and seed solver matrices,
// filter outputs and iteration counts, completion factors).
size_t footprint_of(const rpca_job &J)
{
    const size_t mn = (size_t)J.m * J.n;
    const size_t R4 = (size_t)((J.r + 3) / 4 * 4);
    const size_t mnc = (size_t)(J.m + J.n);
    return 12 * mn + mnc * (8 + 4 * (size_t)J.r + 4 + 4 * R4) + 8 * (size_t)(J.p + J.q + 1) * J.r +
           24 * (size_t)J.p * J.q + (1 << 20);
}

double now_ms(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

} // namespace

struct rpca_server {
    int device = 0;
    rpca_opts opts{};
    rpca_batch_tuning tun{};
    rpca_server_opts so{};
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Request> reqs;
    int64_t next_ticket = 1;
    size_t inflight = 0;
    rpca_server_stats stats{};
    bool stop = false;
    std::vector<std::thread> workers;
    std::string error;

    bool admissible_locked() const
    {
        if (queue.empty()) return false;
        const Request &R = reqs.at(queue.front());
        return inflight == 0 || inflight + R.footprint <= (size_t)so.hbm_budget_bytes;
    }
};

namespace {

thread_local std::string g_server_error;

// Steps 2-5 for the jobs of one batch on the worker's plan; fills statuses
// and infos.  Returns the status of the batch as a whole.
int run_batch(rpca_batch *b, rpca_ctx *ctx, const std::vector<rpca_job> &jobs,
              std::vector<int> &status, std::vector<rpca_info> &info)
{
    const int64_t n = (int64_t)jobs.size();
    int st = batch_plan(b, jobs.data(), n, nullptr);
    if (st < 0) return st;
    st = rpca_batch_seed(b, nullptr);
    if (st < 0) return st;
    st = rpca_batch_run(b, batch_stream(b));
    if (st < 0) return st;
    for (int64_t k = 0; k < n; ++k) {
        status[k] = rpca_batch_job_info(b, k, &info[k]);
        // a job whose input holds Inf / NaN fails alone; the others stand
        if (status[k] < 0 && status[k] != RPCA_ERR_NUMERIC) return status[k];
    }
    (void)ctx;
    return RPCA_OK;
}

void worker_main(rpca_server *s, int index)
{
    rpca_ctx *ctx = nullptr;
    int st = rpca_ctx_create(s->device, &ctx);
    rpca_batch *b = nullptr;
    if (st == RPCA_OK) b = batch_new(ctx, s->opts, s->tun, &st);
    const std::string setup_error = st == RPCA_OK ? "" : (ctx ? ctx->last_error : "context creation failed");
    (void)index;
    for (;;) {
        std::vector<int64_t> mine;
        std::vector<rpca_job> jobs;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->admissible_locked() || (s->stop && s->queue.empty()); });
            // this worker's share of the queue: what is queued split over all
            // workers (busy ones take theirs when they come back), so a burst
            // becomes several batches running side by side
            const size_t nw = (size_t)s->so.workers;
            const int share = (int)std::min<size_t>((size_t)s->so.max_batch, (s->queue.size() + nw - 1) / nw);
            if (s->queue.empty()) break;           // stop requested and nothing left
            while (!s->queue.empty() && (int)mine.size() < std::max(1, share)) {
                Request &R = s->reqs.at(s->queue.front());
                if (!(s->inflight == 0 || s->inflight + R.footprint <= (size_t)s->so.hbm_budget_bytes))
                    break;
                s->inflight += R.footprint;
                s->stats.peak_inflight_bytes = std::max(s->stats.peak_inflight_bytes, (double)s->inflight);
                R.info.t_admit_ms = now_ms(s->t0);
                mine.push_back(s->queue.front());
                jobs.push_back(R.job);
                s->queue.pop_front();
            }
            ++s->stats.batches;
        }
        const int64_t n = (int64_t)mine.size();
        std::vector<int> status((size_t)n, RPCA_ERR_DEVICE);
        std::vector<rpca_info> info((size_t)n);
        std::vector<std::string> msg((size_t)n);
        if (!b) {
            for (auto &m : msg) m = setup_error;
        } else if (run_batch(b, ctx, jobs, status, info) < 0) {
            // isolate the failing request(s): one at a time
            for (int64_t k = 0; k < n; ++k) {
                std::vector<rpca_job> one{jobs[k]};
                std::vector<int> s1(1, RPCA_ERR_DEVICE);
                std::vector<rpca_info> i1(1);
                const int st1 = run_batch(b, ctx, one, s1, i1);
                status[k] = st1 < 0 ? st1 : s1[0];
                info[k] = i1[0];
                if (status[k] != RPCA_OK) msg[k] = ctx->last_error;
            }
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            const double t = now_ms(s->t0);
            for (int64_t k = 0; k < n; ++k) {
                Request &R = s->reqs.at(mine[k]);
                R.info.status = status[k];
                R.info.batch_size = (int32_t)n;
                R.info.info = info[k];
                R.info.t_done_ms = t;
                R.done = true;
                s->inflight -= R.footprint;
                ++s->stats.completed;
                if (status[k] < 0) ++s->stats.failed;
            }
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();                 // budget freed
    }
    if (b) {
        // the plan's workspace context is owned by the plan
        rpca_batch_destroy(b);
    }
    if (ctx) rpca_ctx_destroy(ctx);
}

} // namespace

extern "C" {

void rpca_server_opts_default(rpca_server_opts *o)
{
    if (!o) return;
    o->hbm_budget_bytes = 200e9;
    o->workers = 3;
    o->max_batch = 64;
}

int rpca_server_create(int device, const rpca_opts *opts, const rpca_batch_tuning *tuning,
                       const rpca_server_opts *sopts, rpca_server_t *out)
{
    g_server_error.clear();
    if (!out || !opts) {
        g_server_error = "server: NULL argument";
        return RPCA_ERR_ARG;
    }
    *out = nullptr;
    rpca_server_opts so;
    rpca_server_opts_default(&so);
    if (sopts) so = *sopts;
    if (!(so.hbm_budget_bytes > 0) || so.workers < 1 || so.workers > 16 || so.max_batch < 1) {
        g_server_error = "server: bad server options";
        return RPCA_ERR_ARG;
    }
    rpca_batch_tuning tun;
    rpca_batch_tuning_default(&tun);
    if (tuning) tun = *tuning;
    tun.graph = 0;                      // every batch is planned once and run once
    // check the options and tuning once, on a probe context
    rpca_ctx *probe = nullptr;
    int st = rpca_ctx_create(device, &probe);
    if (st != RPCA_OK) {
        g_server_error = rpca_last_error(nullptr);
        return st;
    }
    st = check_opts(probe, *opts);
    if (st == RPCA_OK) st = batch_check_tuning(probe, tun);
    if (st != RPCA_OK) {
        g_server_error = "server: " + probe->last_error;
        rpca_ctx_destroy(probe);
        return st;
    }
    rpca_ctx_destroy(probe);
    rpca_server *s = new rpca_server();
    s->device = device;
    s->opts = *opts;
    s->tun = tun;
    s->so = so;
    s->t0 = std::chrono::steady_clock::now();
    for (int w = 0; w < so.workers; ++w) s->workers.emplace_back(worker_main, s, w);
    *out = s;
    return RPCA_OK;
}

const char *rpca_server_error(rpca_server_t s)
{
    return s ? s->error.c_str() : g_server_error.c_str();
}

int rpca_server_submit(rpca_server_t s, const rpca_job *job, int64_t *ticket)
{
    if (!s) return RPCA_ERR_ARG;
    if (!job || !ticket) {
        s->error = "server: NULL argument";
        return RPCA_ERR_ARG;
    }
    const rpca_job &J = *job;
    if (!J.M || !J.L || !J.S || !J.seed_rows || !J.seed_cols || J.m < 1 || J.n < 1 ||
        J.ldm < J.m || J.ldl < J.m || J.lds < J.m || J.r < 1 || J.p < 1 || J.q < 1 || J.p > J.m ||
        J.q > J.n || J.r > std::min(J.p, J.q)) {
        s->error = "server: bad job (pointers, sizes or rank)";
        return RPCA_ERR_ARG;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            s->error = "server: shutting down";
            return RPCA_ERR_ARG;
        }
        const int64_t t = s->next_ticket++;
        Request &R = s->reqs[t];
        R.job = J;
        R.footprint = footprint_of(J);
        R.info.t_submit_ms = now_ms(s->t0);
        s->queue.push_back(t);
        ++s->stats.submitted;
        *ticket = t;
    }
    s->cv_work.notify_one();
    return RPCA_OK;
}

int rpca_server_wait(rpca_server_t s, int64_t ticket, rpca_request_info *info)
{
    if (!s) return RPCA_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        s->error = "server: unknown ticket";
        return RPCA_ERR_ARG;
    }
    s->cv_done.wait(lk, [&] { return it->second.done; });
    if (info) *info = it->second.info;
    const int st = it->second.info.status;
    s->reqs.erase(it);
    return st < 0 ? st : RPCA_OK;
}

int rpca_server_poll(rpca_server_t s, int64_t ticket, int32_t *done)
{
    if (!s || !done) return RPCA_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        s->error = "server: unknown ticket";
        return RPCA_ERR_ARG;
    }
    *done = it->second.done ? 1 : 0;
    return RPCA_OK;
}

int rpca_server_get_stats(rpca_server_t s, rpca_server_stats *stats)
{
    if (!s || !stats) return RPCA_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *stats = s->stats;
    stats->queued = (int64_t)s->queue.size();
    stats->inflight_bytes = (double)s->inflight;
    return RPCA_OK;
}

int rpca_server_destroy(rpca_server_t s)
{
    if (!s) return RPCA_ERR_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();      // the queue drains first
    delete s;
    return RPCA_OK;
}

} // extern "C"
