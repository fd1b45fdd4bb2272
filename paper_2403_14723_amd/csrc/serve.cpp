// Serving loop: continuous batching of meshing requests on one GPU.
//
// Requests (a triangulation each) are copied at submit and queued.  The server runs `lanes`, each an internal context with
// its own stream, a fixed device arena and a thread of its own.  A lane's
// thread admits as many queued requests as fit the arena (their exact device
// footprint) up to max_batch, builds their half-edge structures and
// launches one batched meshing run.  While it
// runs, the other lanes take the requests that keep arriving, so uploads,
// builds, runs and downloads of different batches overlap.  When a lane's
// kernels finish, its outputs are copied to pinned host blocks (exact sizes,
// known from the run's counts); when the copies finish, every request of the
// batch completes with a host-resident result and the lane's arena is reset.
// Latency runs from submit to that point.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "runtime_internal.h"

using namespace gprt;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    uint64_t ticket = 0;
    int32_t *xy = nullptr, *tri = nullptr;   // pinned copies of the inputs
    size_t xy_cap = 0, tri_cap = 0;          // their blocks' real sizes
    int32_t nv = 0, nt = 0;
    size_t footprint = 0;   // build bytes; the batch adds its meshing bytes
    Clock::time_point t_submit;
    bool done = false;
    bool waited = false;   // a gpolylla_serve_wait call holds the ticket
    int status = GP_OK;
    gp_result *result = nullptr;
};

// Pinned host blocks for results; outlives the server while results hold
// blocks.  A request may get a free block of up to twice its size; a block
// always comes back at its real size.  At most kCap bytes are kept free
// (blocks beyond that are freed).
struct PinnedPool {
    static constexpr size_t kCap = (size_t)4 << 30;
    std::mutex mu;
    std::multimap<size_t, void *> free_;   // by real size
    size_t bytes = 0;                      // held in free_
    // A block of at least n bytes; *cap: its real size.
    void *take(size_t n, size_t *cap) {
        n = align_up(n ? n : kAlign);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = free_.lower_bound(n);
            if (it != free_.end() && it->first <= 2 * n) {
                void *p = it->second;
                *cap = it->first;
                bytes -= it->first;
                free_.erase(it);
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        *cap = n;
        return p;
    }
    // Returns block p of real size cap (as take reported it).
    void give(void *p, size_t cap) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (bytes + cap <= kCap) {
                bytes += cap;
                free_.emplace(cap, p);
                return;
            }
        }
        (void)hipHostFree(p);
    }
    ~PinnedPool() {
        for (auto &kv : free_) (void)hipHostFree(kv.second);
    }
};

struct Lane {
    gp_ctx *ctx = nullptr;
    enum State { FREE, RUNNING, COPYING } state = FREE;
    std::vector<Request *> reqs;
    std::vector<gp_mesh *> meshes;
    std::vector<gp_result *> dev;          // device results of the batch
    std::vector<void *> blocks;            // pinned block per request
    std::vector<size_t> block_bytes;       // its real size
    std::vector<gp_result_info> infos;
    hipEvent_t copied = nullptr;
};

double pct(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double k = q * (double)(v.size() - 1);
    const size_t i = (size_t)k;
    const double f = k - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

struct gp_server {
    int device = 0;
    gp_serve_opts opts{};
    size_t lane_bytes = 0;
    std::vector<Lane> lanes;
    std::shared_ptr<PinnedPool> pinned = std::make_shared<PinnedPool>();   // results
    // requests' inputs: pinned, so that the builds' uploads are asynchronous
    // copies at full link speed; reused after the requests complete
    PinnedPool inputs;
    std::vector<std::thread> workers;   // one per lane
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t next_ticket = 1;
    bool stopping = false;
    // statistics
    int64_t submitted = 0, completed = 0, rejected = 0, failed = 0, batches = 0, tri_done = 0;
    std::vector<double> lat_ms;
    Clock::time_point t_first, t_last;
    bool have_first = false;
};

namespace {

void give_inputs(gp_server *s, Request *r) {
    if (r->xy) s->inputs.give(r->xy, r->xy_cap);
    if (r->tri) s->inputs.give(r->tri, r->tri_cap);
    r->xy = r->tri = nullptr;
}

void complete(gp_server *s, Request *r, int status, gp_result *res) {
    give_inputs(s, r);   // the build has read them
    const auto now = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    r->status = status;
    r->result = res;
    r->done = true;
    if (status == GP_OK) {
        s->completed++;
        s->tri_done += r->nt;
        s->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
        s->t_last = now;
    } else {
        s->failed++;
    }
    s->cv_done.notify_all();
}

// Launches `batch` on lane L: build every mesh, then one batched run.
void launch(gp_server *s, Lane &L, std::vector<Request *> &batch) {
    L.reqs.clear();
    L.meshes.clear();
    const int n = (int)batch.size();
    std::vector<const int32_t *> xy(n), tri(n);
    std::vector<int32_t> nv(n), nt(n);
    std::vector<gp_mesh *> ms(n, nullptr);
    std::vector<int> st(n, GP_OK);
    for (int i = 0; i < n; i++) {
        xy[i] = batch[i]->xy;
        tri[i] = batch[i]->tri;
        nv[i] = batch[i]->nv;
        nt[i] = batch[i]->nt;
    }
    // every build of the batch, with two host checks in all
    const int b = build_many(L.ctx, n, xy.data(), nv.data(), tri.data(), nt.data(), 0, ms.data(), st.data());
    for (int i = 0; i < n; i++) {
        const int rc = b != GP_OK ? b : st[i];
        if (rc != GP_OK) {
            complete(s, batch[i], rc, nullptr);
            continue;
        }
        L.reqs.push_back(batch[i]);
        L.meshes.push_back(ms[i]);
    }
    if (L.reqs.empty()) {
        L.ctx->pool.reset();
        return;
    }
    L.dev.assign(L.reqs.size(), nullptr);
    const int rc = gpolylla_mesh_batch(L.ctx, L.meshes.data(), (int32_t)L.meshes.size(), GP_ASYNC, L.dev.data());
    if (rc != GP_OK) {
        for (Request *r : L.reqs) complete(s, r, rc, nullptr);
        for (gp_mesh *m : L.meshes) gpolylla_mesh_free(m);
        L.reqs.clear();
        L.meshes.clear();
        L.ctx->pool.reset();
        return;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->batches++;
    }
    L.state = Lane::RUNNING;
}

// Kernels done: copy every output to a pinned block.
void start_copies(gp_server *s, Lane &L) {
    const size_t n = L.reqs.size();
    L.blocks.assign(n, nullptr);
    L.block_bytes.assign(n, 0);
    L.infos.assign(n, gp_result_info{});
    hipStream_t st = L.ctx->stream;
    for (size_t i = 0; i < n; i++) {
        gp_result_info &info = L.infos[i];
        int rc = gpolylla_result_info(L.dev[i], &info);
        if (rc == GP_OK) {
            info.loops_only = s->opts.loops_only ? 1 : 0;
            const size_t links = info.loops_only ? 0 : 2 * (size_t)info.nh;
            const size_t words = links + (size_t)info.npoly + (size_t)info.npoly + 1 + (size_t)info.nloop_he;
            L.blocks[i] = s->pinned->take(4 * words, &L.block_bytes[i]);
            if (!L.blocks[i]) rc = GP_ENOMEM;
        }
        if (rc == GP_OK) {
            gp_result_dev dv{};
            gpolylla_result_device(L.dev[i], &dv);
            int32_t *b = static_cast<int32_t *>(L.blocks[i]);
            // block: [next | prev] seeds loop_off loop_he
            const size_t nh = info.loops_only ? 0 : (size_t)info.nh, P = (size_t)info.npoly,
                         F = (size_t)info.nloop_he;
            hipError_t e = hipSuccess;
            if (nh) e = hipMemcpyAsync(b, dv.next, 4 * nh, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && nh) e = hipMemcpyAsync(b + nh, dv.prev, 4 * nh, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && P) e = hipMemcpyAsync(b + 2 * nh, dv.seeds, 4 * P, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b + 2 * nh + P, dv.loop_off, 4 * (P + 1), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && F)
                e = hipMemcpyAsync(b + 2 * nh + 2 * P + 1, dv.loop_he, 4 * F, hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                rc = GP_EHIP;
            }
        }
        if (rc != GP_OK) {
            if (L.blocks[i]) s->pinned->give(L.blocks[i], L.block_bytes[i]);
            L.blocks[i] = nullptr;
            L.infos[i].nt = -1;   // failed
            L.infos[i].nv = rc;
        }
    }
    if (hipEventRecord(L.copied, st) != hipSuccess) (void)hipGetLastError();
    L.state = Lane::COPYING;
}

// Copies done: hand out host results, free the device side, reset the arena.
void finish(gp_server *s, Lane &L) {
    const size_t n = L.reqs.size();
    for (size_t i = 0; i < n; i++) {
        Request *r = L.reqs[i];
        const gp_result_info &info = L.infos[i];
        if (info.nt < 0 || !L.blocks[i]) {
            complete(s, r, info.nt < 0 ? (int)info.nv : GP_EHIP, nullptr);
            continue;
        }
        gp_result *x = new gp_result();
        x->host = true;
        x->hinfo = info;
        x->nt = (int32_t)info.nt;
        x->nv = (int32_t)info.nv;
        x->nflipped = info.nflipped;
        int32_t *b = static_cast<int32_t *>(L.blocks[i]);
        const size_t nh = info.loops_only ? 0 : (size_t)info.nh, P = (size_t)info.npoly;
        x->next_o = info.loops_only ? nullptr : b;
        x->prev_o = info.loops_only ? nullptr : b + nh;
        x->seeds = b + 2 * nh;
        x->loop_off = b + 2 * nh + P;
        x->loop_he = b + 2 * nh + 2 * P + 1;
        std::shared_ptr<PinnedPool> pool = s->pinned;
        void *blk = L.blocks[i];
        size_t bytes = L.block_bytes[i];
        x->on_free = [pool, blk, bytes]() { pool->give(blk, bytes); };
        complete(s, r, GP_OK, x);
    }
    for (gp_result *d : L.dev) gpolylla_result_free(d);
    for (gp_mesh *m : L.meshes) gpolylla_mesh_free(m);
    L.dev.clear();
    L.meshes.clear();
    L.reqs.clear();
    (void)gpolylla_ctx_sync(L.ctx);   // host side of the run (events, retired runs)
    L.ctx->pool.reset();
    L.state = Lane::FREE;
}

// Device bytes of a batch on one lane: every build plus the batched run.
size_t batch_bytes(const gp::LaunchCfg &cfg, const std::vector<Request *> &b, const Request *extra) {
    std::vector<int32_t> nts;
    size_t sum = 0;
    for (const Request *r : b) {
        nts.push_back(r->nt);
        sum += r->footprint;
    }
    if (extra) {
        nts.push_back(extra->nt);
        sum += extra->footprint;
    }
    return sum + batch_footprint(cfg, nts.data(), (int)nts.size());
}

// One lane's thread: admit a batch, build and mesh it, copy the results out,
// hand them over, repeat; on stop, drain the queue first.
void lane_main(gp_server *s, Lane *L) {
    DeviceGuard g(s->device);
    while (true) {
        std::vector<Request *> batch;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [s] { return s->stopping || !s->queue.empty(); });
            if (s->queue.empty()) break;   // stopping, nothing left
            // admission by footprint: as many queued requests as fit
            while (!s->queue.empty() && (int)batch.size() < s->opts.max_batch) {
                Request *r = s->queue.front();
                if (batch_bytes(L->ctx->cfg, batch, r) > s->lane_bytes) break;
                batch.push_back(r);
                s->queue.pop_front();
            }
            if (batch.empty()) {
                // submit rejects requests larger than a lane, so an empty lane
                // fits the first one; never spin on one that does not
                Request *r = s->queue.front();
                s->queue.pop_front();
                lk.unlock();
                complete(s, r, GP_ETOOBIG, nullptr);
                continue;
            }
            if (!s->queue.empty()) s->cv_work.notify_one();   // work left for another lane
        }
        launch(s, *L, batch);
        if (L->state != Lane::RUNNING) continue;   // every build failed
        if (hipStreamSynchronize(L->ctx->stream) != hipSuccess) (void)hipGetLastError();
        start_copies(s, *L);
        if (hipEventSynchronize(L->copied) != hipSuccess) (void)hipGetLastError();
        finish(s, *L);
    }
}

}  // namespace

extern "C" {

int gpolylla_serve_start(gp_ctx *ctx, const gp_serve_opts *opts, gp_server **out) {
    if (!ctx || !out) return GP_EINVAL;
    *out = nullptr;
    gp_serve_opts o{};
    o.pool_bytes = (size_t)16 << 30;
    o.max_batch = 64;
    o.max_queue = 4096;
    o.n_lanes = 2;
    if (opts) {
        if (opts->pool_bytes) o.pool_bytes = opts->pool_bytes;
        if (opts->max_batch > 0) o.max_batch = opts->max_batch;
        if (opts->max_queue > 0) o.max_queue = opts->max_queue;
        if (opts->n_lanes > 0) o.n_lanes = opts->n_lanes;
        o.loops_only = opts->loops_only ? 1 : 0;
    }
    if (o.n_lanes > 8) return GP_EINVAL;
    gp_server *s = new (std::nothrow) gp_server();
    if (!s) return GP_ENOMEM;
    s->device = ctx->device;
    s->opts = o;
    s->lane_bytes = o.pool_bytes / (size_t)o.n_lanes;
    DeviceGuard g(s->device);
    s->lanes.resize(o.n_lanes);
    for (Lane &L : s->lanes) {
        gp_ctx_opts co{};
        int rc = gpolylla_ctx_create(ctx->device, &co, &L.ctx);
        if (rc == GP_OK) {
            L.ctx->cfg = ctx->cfg;
            rc = L.ctx->pool.make_arena(s->lane_bytes);
        }
        if (rc == GP_OK && hipEventCreateWithFlags(&L.copied, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            rc = GP_EHIP;
        }
        if (rc != GP_OK) {
            for (Lane &M : s->lanes) {
                if (M.ctx) gpolylla_ctx_destroy(M.ctx);
                if (M.copied) (void)hipEventDestroy(M.copied);
            }
            delete s;
            return rc;
        }
    }
    for (Lane &L : s->lanes) s->workers.emplace_back(lane_main, s, &L);
    *out = s;
    return GP_OK;
}

int gpolylla_serve_submit_at(gp_server *s, const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
                             int64_t arrival_ns, uint64_t *ticket) {
    if (!s || !ticket || nv < 0 || nt < 0 || (nv > 0 && !xy) || (nt > 0 && !tri)) return GP_EINVAL;
    if (3ll * nt >= (1ll << 31)) return GP_ERANGE;
    const auto now = Clock::now();
    const auto arrival = Clock::time_point(std::chrono::nanoseconds(arrival_ns));
    if (arrival_ns > 0 && arrival > now) return GP_EINVAL;   // not arrived yet
    Request *r = new (std::nothrow) Request();
    if (!r) return GP_ENOMEM;
    r->nv = nv;
    r->nt = nt;
    r->footprint = build_footprint(nv, nt, false);
    const int32_t one = nt;
    const size_t alone = r->footprint + batch_footprint(s->lanes[0].ctx->cfg, &one, 1);
    r->t_submit = arrival_ns > 0 ? arrival : now;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete r;
            return GP_EINVAL;
        }
        if (alone > s->lane_bytes) {
            s->rejected++;
            delete r;
            return GP_ETOOBIG;
        }
        if ((int)s->queue.size() >= s->opts.max_queue) {
            s->rejected++;
            delete r;
            return GP_EAGAIN;
        }
    }
    r->xy = static_cast<int32_t *>(s->inputs.take(8 * (size_t)nv, &r->xy_cap));
    r->tri = static_cast<int32_t *>(s->inputs.take(12 * (size_t)nt, &r->tri_cap));
    if (!r->xy || !r->tri) {
        give_inputs(s, r);
        delete r;
        return GP_ENOMEM;
    }
    if (nv) std::memcpy(r->xy, xy, 8 * (size_t)nv);
    if (nt) std::memcpy(r->tri, tri, 12 * (size_t)nt);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {   // stopped while the inputs were copied: the lanes may be gone
            give_inputs(s, r);
            delete r;
            return GP_EINVAL;
        }
        r->ticket = s->next_ticket++;
        s->reqs[r->ticket] = r;
        s->queue.push_back(r);
        s->submitted++;
        if (!s->have_first) {
            s->t_first = r->t_submit;
            s->have_first = true;
        }
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return GP_OK;
}

int gpolylla_serve_submit(gp_server *s, const int32_t *xy, int32_t nv, const int32_t *tri, int32_t nt,
                          uint64_t *ticket) {
    return gpolylla_serve_submit_at(s, xy, nv, tri, nt, 0, ticket);
}

int gpolylla_serve_wait(gp_server *s, uint64_t ticket, int32_t timeout_ms, gp_result **out) {
    if (!s || !out) return GP_EINVAL;
    *out = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return GP_EINVAL;
    Request *r = it->second;
    // one waiter per ticket: the one that returns with the result deletes
    // the request, so a second waiter is turned away here
    if (r->waited) return GP_EINVAL;
    r->waited = true;
    auto pred = [r] { return r->done; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, pred);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
        r->waited = false;   // the ticket can be waited for again
        return GP_ETIMEDOUT;
    }
    const int st = r->status;
    *out = r->result;
    s->reqs.erase(it);
    delete r;
    return st;
}

int gpolylla_serve_stats(gp_server *s, gp_serve_stats *st) {
    if (!s || !st) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = gp_serve_stats{};
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->rejected = s->rejected;
    st->failed = s->failed;
    st->batches = s->batches;
    st->in_flight = s->submitted - s->completed - s->failed;
    st->p50_ms = pct(s->lat_ms, 0.50);
    st->p99_ms = pct(s->lat_ms, 0.99);
    double mean = 0;
    for (double v : s->lat_ms) mean += v;
    st->mean_ms = s->lat_ms.empty() ? 0.0 : mean / (double)s->lat_ms.size();
    st->max_ms = s->lat_ms.empty() ? 0.0 : *std::max_element(s->lat_ms.begin(), s->lat_ms.end());
    if (s->have_first && s->completed) {
        const double secs = std::chrono::duration<double>(s->t_last - s->t_first).count();
        st->mtri_s = secs > 0 ? (double)s->tri_done / secs / 1e6 : 0.0;
    }
    return GP_OK;
}

int gpolylla_serve_reset_stats(gp_server *s) {
    if (!s) return GP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->lat_ms.clear();
    s->completed = s->failed = s->rejected = s->batches = s->tri_done = 0;
    // requests not finished yet (queued or on a lane) count as submitted, so
    // that in_flight stays exact as they complete
    int64_t pending = 0;
    for (const auto &kv : s->reqs) pending += kv.second->done ? 0 : 1;
    s->submitted = pending;
    s->have_first = false;
    return GP_OK;
}

int gpolylla_serve_stop(gp_server *s) {
    if (!s) return GP_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (std::thread &t : s->workers)
        if (t.joinable()) t.join();
    {
        DeviceGuard g(s->device);
        for (Lane &L : s->lanes) {
            if (L.ctx) gpolylla_ctx_destroy(L.ctx);
            if (L.copied) (void)hipEventDestroy(L.copied);
        }
    }
    // requests never waited for: drop their results
    for (auto &kv : s->reqs) {
        if (kv.second->result) gpolylla_result_free(kv.second->result);
        delete kv.second;
    }
    delete s;
    return GP_OK;
}

}  // extern "C"
