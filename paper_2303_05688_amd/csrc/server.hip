// Batched searches and a continuous-batching request loop.
//
// A worker pool: each worker owns a context (workspace arenas) and a HIP
// stream, so searches on different workers overlap on the device.  Requests
// wait in arrival order; a free worker takes the oldest one whose bytes,
// added to those budgeted for running requests and the workspace idle
// workers keep, fit the HBM budget, so small requests pass a large one that
// does not fit yet.  Once the oldest request has waited longer than the age
// bound, nothing passes it: workers then start it as soon as it fits.  Idle
// workers give their workspace back when a request needs room.  A result is
// handed over once (poll or wait) and then forgotten.  The batch entry point
// runs a pool over a fixed request list, largest estimated cost first.
#include "asci_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <thread>
#include <unordered_map>
#include <unordered_set>

namespace asci {

namespace {

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t c2(int64_t x) { return x * (x - 1) / 2; }

}  // namespace

int64_t request_pairs(const asci_request &r)
{
    const int64_t n = r.norb, na = r.nalpha, nb = r.nbeta, va = n - na, vb = n - nb;
    const int64_t per = na * va + nb * vb + c2(na) * c2(va) + c2(nb) * c2(vb) + na * va * nb * vb;
    const int64_t nq = (r.opt.ncore > 0 && r.opt.ncore < r.ndets) ? r.opt.ncore : r.ndets;
    return nq * per;
}

int64_t request_footprint(const asci_request &r, uint64_t cap_records, int finish_cap)
{
    const int W = r.norb <= 32 ? 1 : 2;
    const int L = r.nalpha < 3 ? r.nalpha : 3;
    // number of classes: C(n - na + L, L)
    int64_t ncls = 1;
    for (int i = 1; i <= L; ++i) ncls = ncls * (r.norb - r.nalpha + i) / i;
    const int64_t nq = (r.opt.ncore > 0 && r.opt.ncore < r.ndets) ? r.opt.ncore : r.ndets;
    const uint64_t P = (uint64_t)request_pairs(r);
    uint64_t Pb = std::min<uint64_t>(P, cap_records);
    if (r.opt.pair_buffer_bytes > 0) Pb = std::min<uint64_t>(Pb, (uint64_t)r.opt.pair_buffer_bytes / (2 * (8 * W + 8)));
    Pb = std::max<uint64_t>(Pb, 1) + Pb / 8;  // a class may overshoot the cap
    const uint64_t nc = (uint64_t)std::min<int64_t>(ncls, 2048);
    const uint64_t E = nc * (uint64_t)nq;
    const uint64_t k = (uint64_t)std::max<int64_t>(r.k, 1);
    const uint64_t pool = std::min<uint64_t>(P + 1, std::max<uint64_t>(4 * k, Pb) + k);
    const uint64_t setup = (uint64_t)r.ndets * 128 + (uint64_t)nq * 64 + (uint64_t)ncls * 16 +
                           (uint64_t)(2 * r.norb * r.norb + r.norb) * 8 + (1 << 20);
    const uint64_t main = E * 8 + Pb * (2 * (8 * W + 8)) + Pb * (8 * W + 16) + bucket_workspace_bytes(Pb, nc, W, finish_cap) +
                          pool * ((8 * W + 8) * 2 + 12) + std::min(k, pool) * 24 + (1 << 20);
    const uint64_t tables = spin_table_plan(r.norb, r.nalpha, r.nbeta, P, true).bytes;
    return (int64_t)(setup + main + tables);
}

// Argument checks of a request before it is queued (the checks of the search
// entry points): sizes, options, and for a device request its buffers.
static void check_request(const asci_request &r, bool device)
{
    check_common(r.norb, r.nalpha, r.nbeta, r.ndets);
    require(r.k >= 1, ASCI_EINVAL, "k must be >= 1");
    (void)resolve(&r.opt);
    if (device)
        require(r.h && r.eri && r.dets && r.coeffs && r.out_dets && r.out_scores, ASCI_EINVAL,
                "null buffer in a request");
}

// ---------------------------------------------------------------- the pool
struct Job {
    asci_request req;
    uint64_t ticket;
    double t_submit;
    int64_t footprint;
    int64_t pairs;
};

struct WorkerState {
    std::unique_ptr<asci_ctx> ctx;
    hipStream_t stream = nullptr;
    int64_t resident = 0;  // workspace the worker keeps between requests
    int64_t reserved = 0;  // bytes budgeted while running
    bool busy = false;
    std::thread th;
};

class Pool {
  public:
    Pool(int device, int64_t budget, int slots, bool fake, double ns_per_byte, int finish_cap)
        : device_(device), budget_(budget), fake_(fake), ns_per_byte_(ns_per_byte), finish_cap_(finish_cap)
    {
        slots = std::max(1, std::min(slots, 16));
        cap_records_ = (uint64_t)std::max<int64_t>(1 << 20, std::min<int64_t>(1ll << 30, budget / slots / 160));
        ws_.resize((size_t)slots);
        for (auto &w : ws_) {
            w = std::make_unique<WorkerState>();
            if (!fake_) {
                ASCI_HIP(hipSetDevice(device_));
                w->ctx = std::make_unique<asci_ctx>();
                w->ctx->device = device_;
                w->ctx->finish_cap = finish_cap;
                ASCI_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
            }
        }
        for (size_t i = 0; i < ws_.size(); ++i) ws_[i]->th = std::thread([this, i] { loop((int)i); });
    }

    // work queued on `after` before this call completes before any worker
    // starts what is submitted next (the pool must be idle)
    void order_after(hipStream_t after)
    {
        if (fake_ || !after) return;
        ASCI_HIP(hipSetDevice(device_));
        hipEvent_t ready = nullptr;
        ASCI_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        ASCI_HIP(hipEventRecord(ready, after));
        for (auto &w : ws_) ASCI_HIP(hipStreamWaitEvent(w->stream, ready, 0));
        ASCI_HIP(hipEventDestroy(ready));
    }

    // forget finished tickets whose results were not collected
    void forget(const std::vector<uint64_t> &tickets)
    {
        std::unique_lock<std::mutex> lk(mu_);
        for (uint64_t t : tickets) {
            done_.erase(t);
            live_.erase(t);
        }
    }

    ~Pool()
    {
        {
            std::unique_lock<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_work_.notify_all();
        for (auto &w : ws_)
            if (w->th.joinable()) w->th.join();
        for (auto &w : ws_)
            if (w->stream) (void)hipStreamDestroy(w->stream);
    }

    // the request as this pool runs it: pair buffer capped at cap_records_
    // records, then halved while the whole workspace exceeds the budget (its
    // other parts, such as the class x core matrix and the spin tables, do
    // not shrink with the pair buffer), down to 2^20 records
    asci_request shaped(const asci_request &r) const
    {
        asci_request q = r;
        const int64_t rec = r.norb <= 32 ? 32 : 48;  // ping-pong keys + values per record
        int64_t cap = (int64_t)cap_records_;
        if (q.opt.pair_buffer_bytes > 0) cap = std::max<int64_t>(1, std::min<int64_t>(cap, q.opt.pair_buffer_bytes / rec));
        q.opt.pair_buffer_bytes = cap * rec;
        while (cap > (1 << 20) && request_footprint(q, cap_records_, finish_cap_) > budget_) {
            cap = std::max<int64_t>(cap / 2, 1 << 20);
            q.opt.pair_buffer_bytes = cap * rec;
        }
        return q;
    }

    int64_t footprint(const asci_request &r) const { return request_footprint(shaped(r), cap_records_, finish_cap_); }

    int submit(const asci_request &r, uint64_t *ticket)
    {
        check_request(r, !fake_);
        Job j;
        j.req = shaped(r);
        j.pairs = request_pairs(r);
        j.footprint = request_footprint(j.req, cap_records_, finish_cap_);
        std::unique_lock<std::mutex> lk(mu_);
        j.ticket = next_ticket_++;
        *ticket = j.ticket;
        live_.insert(j.ticket);
        ++submitted_;
        if (first_submit_ < 0) first_submit_ = now_ms();
        if (j.footprint > budget_) {
            ++rejected_;
            asci_result res{};
            res.status = ASCI_ENOMEM;
            done_[j.ticket] = res;
            cv_done_.notify_all();
            return ASCI_ENOMEM;
        }
        j.t_submit = now_ms();
        queue_.push_back(j);
        cv_work_.notify_all();
        return ASCI_OK;
    }

    // a finished request's result is handed over once, then forgotten
    int poll(uint64_t t, asci_result *res, bool block)
    {
        std::unique_lock<std::mutex> lk(mu_);
        if (live_.find(t) == live_.end()) return ASCI_EINVAL;  // unknown, or already handed over
        for (;;) {
            auto it = done_.find(t);
            if (it != done_.end()) {
                if (res) *res = it->second;
                done_.erase(it);
                live_.erase(t);
                return ASCI_OK;
            }
            if (!block) return ASCI_EAGAIN;
            cv_done_.wait(lk);
        }
    }

    void set_age_bound(double ms)
    {
        std::unique_lock<std::mutex> lk(mu_);
        age_ms_ = ms;
        cv_work_.notify_all();
    }

    size_t pending() const
    {
        std::unique_lock<std::mutex> lk(mu_);
        return done_.size() + live_.size();
    }

    void drain()
    {
        std::unique_lock<std::mutex> lk(mu_);
        cv_done_.wait(lk, [&] { return queue_.empty() && running_ == 0; });
    }

    // free the workspaces of the idle workers (they grow again on demand)
    void trim()
    {
        std::unique_lock<std::mutex> lk(mu_);
        for (auto &w : ws_)
            if (!w->busy) release_locked(*w);
    }

    // the HBM the pool may use: what is free now plus what its workers hold
    void set_budget(int64_t free_bytes)
    {
        std::unique_lock<std::mutex> lk(mu_);
        int64_t held = 0;
        for (auto &w : ws_) held += w->resident;
        budget_ = free_bytes + held;
        cap_records_ = (uint64_t)std::max<int64_t>(
            1 << 20, std::min<int64_t>(1ll << 30, budget_ / (int64_t)ws_.size() / 160));
    }

    void stats(asci_server_stats *st)
    {
        std::unique_lock<std::mutex> lk(mu_);
        std::vector<double> l = lat_;
        std::sort(l.begin(), l.end());
        auto pct = [&](double p) {
            if (l.empty()) return 0.0;
            size_t i = (size_t)std::ceil(p * (double)l.size());
            return l[std::min(l.size() - 1, i ? i - 1 : 0)];
        };
        double sum = 0;
        for (double x : l) sum += x;
        st->submitted = submitted_;
        st->completed = completed_;
        st->failed = failed_;
        st->rejected = rejected_;
        st->max_running = max_running_;
        st->peak_bytes = peak_bytes_;
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        st->mean_ms = l.empty() ? 0.0 : sum / (double)l.size();
        st->wall_s = (first_submit_ >= 0 && last_done_ >= 0) ? (last_done_ - first_submit_) * 1e-3 : 0.0;
        st->contributions = contributions_;
        st->bypassed = bypassed_;
        st->held_results = (int64_t)done_.size();
    }

  private:
    int64_t committed_locked() const
    {
        int64_t c = 0;
        for (auto &w : ws_) c += w->busy ? std::max(w->reserved, w->resident) : w->resident;
        return c;
    }

    // bytes this worker would hold for a job of footprint fp
    int64_t need_for(const WorkerState &w, int64_t fp) const { return std::max(w.resident, fp); }

    void release_locked(WorkerState &w)
    {
        if (!fake_ && w.ctx) {
            (void)hipSetDevice(device_);
            w.ctx->setup.release();
            w.ctx->main.release();
            w.ctx->tables.release();
        }
        w.resident = 0;
    }

    // whether a job of footprint fp fits next to the running ones if worker
    // wi takes it (idle workspaces are given back when that makes room)
    bool fits_locked(WorkerState &me, int64_t fp)
    {
        auto fits = [&] { return committed_locked() - me.resident + need_for(me, fp) <= budget_; };
        if (!fits() && me.resident > fp) release_locked(me);
        if (!fits()) {
            for (auto &w : ws_)
                if (!w->busy && w.get() != &me && w->resident > 0) release_locked(*w);
        }
        return fits();
    }

    // the queue position worker wi starts next, or npos: the oldest job that
    // fits; only the oldest once it has waited longer than the age bound
    static constexpr size_t npos = ~size_t(0);
    static constexpr size_t kScan = 64;  // jobs looked at past the head
    size_t choose_locked(int wi)
    {
        if (queue_.empty()) return npos;
        WorkerState &me = *ws_[(size_t)wi];
        const bool head_old = now_ms() - queue_.front().t_submit > age_ms_;
        const size_t lim = head_old ? 1 : std::min(queue_.size(), kScan);
        for (size_t q = 0; q < lim; ++q)
            if (fits_locked(me, queue_[q].footprint)) {
                if (q > 0) ++bypassed_;
                return q;
            }
        return npos;
    }

    void loop(int wi)
    {
        WorkerState &me = *ws_[(size_t)wi];
        if (!fake_) (void)hipSetDevice(device_);
        for (;;) {
            Job j;
            {
                std::unique_lock<std::mutex> lk(mu_);
                size_t pick = npos;
                // re-checked at least every few ms: the head's age changes the choice
                while (!stop_ && (pick = choose_locked(wi)) == npos)
                    cv_work_.wait_for(lk, std::chrono::milliseconds(5));
                if (stop_ && queue_.empty()) return;
                if (stop_ && (pick = choose_locked(wi)) == npos) return;
                j = queue_[pick];
                queue_.erase(queue_.begin() + (std::ptrdiff_t)pick);
                me.busy = true;
                me.reserved = need_for(me, j.footprint);
                ++running_;
                max_running_ = std::max<int64_t>(max_running_, running_);
                peak_bytes_ = std::max(peak_bytes_, committed_locked());
            }
            const double t_run = now_ms();
            asci_result res{};
            res.status = ASCI_OK;
            if (fake_) {
                std::this_thread::sleep_for(std::chrono::nanoseconds((int64_t)(j.footprint * ns_per_byte_)));
                res.count = j.req.k;
            } else {
                try {
                    const asci_request &r = j.req;
                    require(r.norb >= 1 && r.norb <= 64 && r.k >= 1 && r.ndets >= 1, ASCI_EINVAL, "bad request");
                    asci_options o;
                    asci_options_default(&o);
                    o = r.opt;
                    SearchArgs in{r.h, r.eri, r.norb, r.nalpha, r.nbeta, r.dets, r.coeffs, r.ndets, r.E0, o};
                    SearchOut out;
                    out.k = r.k;
                    out.out_dets = r.out_dets;
                    out.out_scores = r.out_scores;
                    search_device(me.ctx.get(), in, out, me.stream);
                    res.count = out.count;
                } catch (const Error &e) {
                    res.status = e.code;
                } catch (const std::bad_alloc &) {
                    res.status = ASCI_ENOMEM;
                } catch (const std::exception &) {
                    res.status = ASCI_EDEVICE;
                }
            }
            const double t_end = now_ms();
            res.latency_ms = t_end - j.t_submit;
            res.run_ms = t_end - t_run;
            res.contributions = j.pairs;
            {
                std::unique_lock<std::mutex> lk(mu_);
                me.busy = false;
                me.reserved = 0;
                me.resident = fake_ ? std::max(me.resident, j.footprint)
                                    : (int64_t)(me.ctx->setup.capacity() + me.ctx->main.capacity() +
                                                me.ctx->tables.capacity());
                --running_;
                done_[j.ticket] = res;
                if (res.status == ASCI_OK) {
                    ++completed_;
                    contributions_ += j.pairs;
                    lat_.push_back(res.latency_ms);
                } else {
                    ++failed_;
                }
                last_done_ = t_end;
            }
            cv_done_.notify_all();
            cv_work_.notify_all();
        }
    }

    int device_;
    int64_t budget_;
    bool fake_;
    double ns_per_byte_;
    uint64_t cap_records_ = 1 << 26;
    int finish_cap_ = 4096;
    std::vector<std::unique_ptr<WorkerState>> ws_;
    mutable std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::deque<Job> queue_;
    std::unordered_map<uint64_t, asci_result> done_;  // finished, not yet handed over
    std::unordered_set<uint64_t> live_;               // submitted, not yet handed over
    double age_ms_ = 250.0;
    int64_t bypassed_ = 0;
    uint64_t next_ticket_ = 1;
    bool stop_ = false;
    int64_t running_ = 0, max_running_ = 0, peak_bytes_ = 0;
    int64_t submitted_ = 0, completed_ = 0, failed_ = 0, rejected_ = 0, contributions_ = 0;
    double first_submit_ = -1, last_done_ = -1;
    std::vector<double> lat_;
};

}  // namespace asci

struct asci_server {
    std::unique_ptr<asci::Pool> pool;
};

using namespace asci;

namespace {

int srv_fail(const Error &e) { return e.code; }

int64_t device_budget(int device)
{
    size_t fr = 0, tt = 0;
    ASCI_HIP(hipSetDevice(device));
    ASCI_HIP(hipMemGetInfo(&fr, &tt));
    return (int64_t)((double)fr * 0.8);
}

}  // namespace

extern "C" {

int64_t asci_request_footprint(const asci_request *req)
{
    if (!req) return -1;
    return request_footprint(*req, (uint64_t)1 << 30);
}

int asci_server_create(int device, int64_t hbm_budget, int slots, asci_server **out)
{
    try {
        require(out != nullptr && hbm_budget > 0 && slots >= 1, ASCI_EINVAL, "bad server arguments");
        int ndev = 0;
        ASCI_HIP(hipGetDeviceCount(&ndev));
        require(device >= 0 && device < ndev, ASCI_EINVAL, "no such device");
        auto *s = new asci_server();
        s->pool = std::make_unique<Pool>(device, hbm_budget, slots, false, 0.0, 4096);
        *out = s;
        return ASCI_OK;
    } catch (const Error &e) {
        return srv_fail(e);
    } catch (const std::bad_alloc &) {
        return ASCI_ENOMEM;
    } catch (const std::exception &) {
        return ASCI_EDEVICE;
    }
}

int asci_server_create_fake(int64_t hbm_budget, int slots, double ns_per_byte, asci_server **out)
{
    try {
        require(out != nullptr && hbm_budget > 0 && slots >= 1 && ns_per_byte >= 0, ASCI_EINVAL,
                "bad server arguments");
        auto *s = new asci_server();
        s->pool = std::make_unique<Pool>(0, hbm_budget, slots, true, ns_per_byte, 4096);
        *out = s;
        return ASCI_OK;
    } catch (const Error &e) {
        return srv_fail(e);
    } catch (const std::bad_alloc &) {
        return ASCI_ENOMEM;
    } catch (const std::exception &) {
        return ASCI_EDEVICE;
    }
}

int asci_server_submit(asci_server *srv, const asci_request *req, uint64_t *ticket)
{
    if (!srv || !req || !ticket) return ASCI_EINVAL;
    try {
        return srv->pool->submit(*req, ticket);
    } catch (const Error &e) {
        return srv_fail(e);
    } catch (const std::bad_alloc &) {
        return ASCI_ENOMEM;
    } catch (const std::exception &) {
        return ASCI_EDEVICE;
    }
}

int asci_server_set_param(asci_server *srv, const char *name, double value)
{
    if (!srv || !name) return ASCI_EINVAL;
    if (std::string(name) == "age_ms") {
        if (!(value >= 0.0)) return ASCI_EINVAL;
        srv->pool->set_age_bound(value);
        return ASCI_OK;
    }
    return ASCI_EINVAL;
}

int64_t asci_server_footprint(asci_server *srv, const asci_request *req)
{
    if (!srv || !req) return -1;
    return srv->pool->footprint(*req);
}

int asci_server_poll(asci_server *srv, uint64_t ticket, asci_result *res)
{
    if (!srv) return ASCI_EINVAL;
    return srv->pool->poll(ticket, res, false);
}

int asci_server_wait(asci_server *srv, uint64_t ticket, asci_result *res)
{
    if (!srv) return ASCI_EINVAL;
    return srv->pool->poll(ticket, res, true);
}

int asci_server_get_stats(asci_server *srv, asci_server_stats *st)
{
    if (!srv || !st) return ASCI_EINVAL;
    srv->pool->stats(st);
    return ASCI_OK;
}

int asci_server_destroy(asci_server *srv)
{
    if (!srv) return ASCI_OK;
    srv->pool->drain();
    delete srv;
    return ASCI_OK;
}

int asci_search_batch(asci_ctx *ctx, const asci_request *reqs, int nreq, asci_result *res, void *stream)
{
    try {
        require(ctx != nullptr && (nreq == 0 || (reqs && res)), ASCI_EINVAL, "null argument");
        require(nreq >= 0, ASCI_EINVAL, "nreq must be >= 0");
        if (nreq == 0) return ASCI_OK;
        const hipStream_t st = (hipStream_t)stream;
        if (!ctx->batch_pool || ctx->batch_pool_slots != ctx->batch_slots ||
            ctx->batch_pool_cap != ctx->finish_cap) {
            if (ctx->batch_pool) ctx->batch_pool_free(ctx->batch_pool);
            ctx->batch_pool = nullptr;
            const int64_t budget = device_budget(ctx->device);
            ctx->batch_pool = new Pool(ctx->device, budget, ctx->batch_slots, false, 0.0, ctx->finish_cap);
            ctx->batch_pool_free = [](void *p) { delete static_cast<Pool *>(p); };
            ctx->batch_pool_trim = [](void *p) { static_cast<Pool *>(p)->trim(); };
            ctx->batch_pool_slots = ctx->batch_slots;
            ctx->batch_pool_cap = ctx->finish_cap;
        }
        Pool &pool = *static_cast<Pool *>(ctx->batch_pool);
        ASCI_HIP(hipSetDevice(ctx->device));
        ASCI_HIP(hipStreamSynchronize(st));  // work queued on `stream` finishes first
        // requests of at least batch_solo_pairs pairs fill the GPU on their own:
        // they run one at a time on ctx, with its whole workspace, after the
        // rest.  Of the rest, requests inside the asynchronous search's scope
        // whose workspace fits a share of the free HBM run as one captured
        // graph on `stream` (batch_graph = 1); the others on the worker
        // streams, at the same time.
        std::vector<int> gidx, pidx, solo;
        size_t limit = 0;
        if (ctx->batch_graph) {
            size_t fr = 0, tt = 0;
            ASCI_HIP(hipMemGetInfo(&fr, &tt));
            limit = (size_t)((double)fr * 0.4) / (size_t)std::max(ctx->batch_slots, 1);
        }
        for (int i = 0; i < nreq; ++i) {
            if (ctx->batch_solo_pairs > 0 && request_pairs(reqs[i]) >= ctx->batch_solo_pairs) {
                solo.push_back(i);
                continue;
            }
            size_t b = 0;
            if (ctx->batch_graph) {
                try {
                    check_request(reqs[i], true);
                    b = graph_request_bytes(reqs[i], ctx->finish_cap, ctx->spin_tables != 0);
                } catch (const Error &) {
                    b = 0;  // the worker path reports it
                }
            }
            if (b > 0 && b <= limit) gidx.push_back(i);
            else pidx.push_back(i);
        }
        // without requests for ctx itself its workspaces are idle during the
        // batch: their HBM goes to the workers
        if (solo.empty()) {
            ctx->setup.release();
            ctx->main.release();
            ctx->tables.release();
        }
        pool.order_after(st);  // before the graph: the workers do not wait for it
        const double t0 = now_ms();
        if (!gidx.empty()) {
            if (!ctx->graph_batch) {
                ctx->graph_batch = new GraphBatch();
                ctx->graph_batch_free = [](void *p) { delete static_cast<GraphBatch *>(p); };
            }
            graph_batch_launch(*static_cast<GraphBatch *>(ctx->graph_batch), ctx->device, reqs, gidx,
                               ctx->batch_slots, ctx->finish_cap, ctx->spin_tables, st);
        }
        pool.set_budget(device_budget(ctx->device));
        std::stable_sort(pidx.begin(), pidx.end(),
                         [&](int a, int b) { return request_pairs(reqs[a]) > request_pairs(reqs[b]); });
        std::vector<uint64_t> tickets((size_t)nreq, 0);
        int rc = ASCI_OK;
        for (int i : pidx) {
            int r;
            try {
                r = pool.submit(reqs[i], &tickets[(size_t)i]);
            } catch (const Error &e) {  // rejected by the argument checks: never queued
                r = e.code;
                tickets[(size_t)i] = 0;
                res[i] = asci_result{};
                res[i].status = r;
            }
            if (r != ASCI_OK && rc == ASCI_OK) rc = r;
        }
        for (int i : pidx) {
            if (tickets[(size_t)i] == 0) continue;
            pool.poll(tickets[(size_t)i], &res[i], true);
            if (res[i].status != ASCI_OK && rc == ASCI_OK) rc = res[i].status;
        }
        if (!gidx.empty()) {
            ASCI_HIP(hipStreamSynchronize(st));
            const double t1 = now_ms();
            std::vector<asci_async_result> ar;
            graph_batch_results(*static_cast<GraphBatch *>(ctx->graph_batch), gidx.size(), ar);
            for (size_t j = 0; j < gidx.size(); ++j) {
                asci_result &r = res[gidx[j]];
                r = asci_result{};
                r.status = ar[j].status;
                r.count = ar[j].count;
                r.latency_ms = r.run_ms = t1 - t0;
                r.contributions = request_pairs(reqs[gidx[j]]);
                if (r.status != ASCI_OK && rc == ASCI_OK) rc = r.status;
            }
        }
        pool.forget(tickets);
        // the requests that fill the GPU alone, largest first, on ctx (a search
        // on ctx first frees the idle workers' workspaces)
        std::stable_sort(solo.begin(), solo.end(),
                         [&](int a, int b) { return request_pairs(reqs[a]) > request_pairs(reqs[b]); });
        for (int i : solo) {
            const asci_request &r = reqs[i];
            asci_result &out = res[i];
            out = asci_result{};
            const double t_run = now_ms();
            try {
                check_request(r, true);
                SearchArgs in{r.h, r.eri, r.norb, r.nalpha, r.nbeta, r.dets, r.coeffs, r.ndets, r.E0, resolve(&r.opt)};
                SearchOut so;
                so.k = r.k;
                so.out_dets = r.out_dets;
                so.out_scores = r.out_scores;
                search_device(ctx, in, so, st);
                out.count = so.count;
                out.status = ASCI_OK;
                out.contributions = request_pairs(r);
            } catch (const Error &e) {
                out.status = e.code;
            } catch (const std::bad_alloc &) {
                out.status = ASCI_ENOMEM;
            }
            const double t_end = now_ms();
            out.run_ms = t_end - t_run;
            out.latency_ms = t_end - t0;
            if (out.status != ASCI_OK && rc == ASCI_OK) rc = out.status;
        }
        return rc;
    } catch (const Error &e) {
        return srv_fail(e);
    } catch (const std::bad_alloc &) {
        return ASCI_ENOMEM;
    } catch (const std::exception &) {
        return ASCI_EDEVICE;
    }
}

int asci_autotune(asci_ctx *ctx, const asci_request *sample, int nsample, int64_t *best_slots,
                  int64_t *best_finish_cap)
{
    try {
        require(ctx != nullptr && sample != nullptr && nsample >= 1, ASCI_EINVAL, "bad arguments");
        // every shape of the sample gets its own finish capacity (synchronous
        // searches on ctx); the batch configuration is left as it is
        int tuned = 0;
        int rc = asci_tune_shapes(ctx, sample, nsample, &tuned);
        if (rc != ASCI_OK) return rc;
        int big = 0;
        for (int i = 1; i < nsample; ++i)
            if (request_pairs(sample[i]) > request_pairs(sample[big])) big = i;
        int cap = 0;
        rc = asci_tune_lookup(ctx->device, sample[big].norb, sample[big].nalpha, request_pairs(sample[big]), &cap);
        if (rc != ASCI_OK) return rc;
        if (best_slots) *best_slots = ctx->batch_slots;
        if (best_finish_cap) *best_finish_cap = cap ? cap : ctx->finish_cap;
        return ASCI_OK;
    } catch (const Error &e) {
        return srv_fail(e);
    } catch (const std::bad_alloc &) {
        return ASCI_ENOMEM;
    } catch (const std::exception &) {
        return ASCI_EDEVICE;
    }
}

}  // extern "C"
