// Request loop for count jobs (include/escape.h, esc_server_*).
//
// Continuous batching over a pool of pipeline contexts: every worker owns one
// esc_ctx (its own stream and device buffers), so up to max_inflight launches
// run on the device at once.  A free worker takes the head of the queue and,
// when it is small, every following queued request of the same k that still
// fits, and runs them as one batched launch (the disjoint-union pipeline);
// a large request runs alone.  A launch is admitted only when its estimated
// HBM footprint fits beside the launches already in flight, so requests that
// arrive while others run are admitted as workers and memory free up.  Each
// request's CSR is copied at submission and uploaded with its launch; results
// are exact 128-bit counts.
#include <stdlib.h>
#include <string.h>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

// Batches whose graphs all have at most this many vertices run the per-source
// passes a source per wave (per-wave LDS tables over a graph's keys).
constexpr int32_t PW_MAX_N = 4096;
#include <vector>
#include "device.h"
#include "ctx.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    uint64_t ticket;
    int32_t n;
    int k;
    std::vector<int32_t> rp, col;
    uint64_t wedges;           // sum_v C(d(v),2), for the footprint estimate
    uint64_t cost = 0;         // predicted device work (see work_cost), once priced
    bool priced = false;       // cost is set
    bool pricing = false;      // the pricing thread holds it (not deleted meanwhile)
    bool taken = false;        // its result was collected while it was being priced
    double t_submit = 0, t_done = 0;
    esc_status status = ESC_OK;
    bool done = false;
    esc_u128 out[45];
};

}  // namespace

struct esc_server {
    int device;
    size_t budget;             // admission budget (bytes of estimated footprint in flight)
    size_t reserved = 0;       // estimated footprint of the launches in flight
    int32_t small_n;           // requests up to this size may share a launch
    int max_group;             // requests per batched launch
    int nwg;                   // workgroups of the per-source kernels (table footprint)
    uint64_t cost_cap;         // predicted work of one grouped launch at most (a request alone may pass it)
    size_t max_queue = 1 << 20;   // requests waiting at most; esc_submit returns ESC_EBUSY beyond
    std::mutex mu;
    std::condition_variable cv;        // queue, memory or stop changed
    std::condition_variable cv_done;   // a request finished
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, Req *> reqs;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::vector<esc_ctx *> ctxs;
    std::vector<std::thread> workers;
    std::deque<Req *> unpriced;   // submitted, cost not yet computed (pricing thread)
    std::thread pricer;
    // statistics
    uint64_t completed = 0, launches = 0, batched_requests = 0;
    int running = 0, peak_running = 0;
    size_t peak_reserved = 0;
};

namespace {

// Device bytes one launch holds, from the buffers the pipeline allocates:
// CSR copies and the relabelled CSR with its arc arrays (~ 64 B per vertex,
// 160 B per edge), triangle lists (8 B per list entry, six entries per
// triangle, bounded through T <= W/3), and the per-workgroup dense tables of
// the largest graph (24 B per entry and workgroup).
size_t footprint(const std::vector<Req *> &grp, int nwg) {
    size_t bytes = 0;
    int64_t nmax = 0;
    for (const Req *r : grp) {
        const int64_t m = (int64_t)r->col.size() / 2;
        bytes += 64 * (size_t)(r->n + 1) + 160 * (size_t)m + 16 * (size_t)r->wedges;
        if (r->n > nmax) nmax = r->n;
    }
    bytes += 24 * (size_t)nmax * (size_t)nwg + ((size_t)64 << 20);
    return bytes;
}

// Predicted device work of a request, in visited list entries: the wedges W
// (pair passes) plus the directed 3-paths i <- a -> b -> j of the degree
// order with the j closing a triangle, sum over arcs a -> b of
// (d+(a) - 1) d+(b) (5-cycle pass), the two work terms of Thm fivevertex
// that are known before counting (Fig. predict fits the running time
// linearly in W, D, DP and DBP).  Ids outside [0, n) are skipped: the device
// rejects such input.
uint64_t work_cost(int32_t n, const int32_t *rp, const int32_t *col, uint64_t w) {
    std::vector<int32_t> dplus((size_t)n + 1, 0);
    auto later = [&](int32_t a, int32_t b) {   // b after a in the degree order
        const int32_t da = rp[a + 1] - rp[a], db = rp[b + 1] - rp[b];
        return db > da || (db == da && b > a);
    };
    for (int32_t v = 0; v < n; v++)
        for (int32_t p = rp[v]; p < rp[v + 1]; p++) {
            const int32_t u = col[p];
            if (u >= 0 && u < n && later(v, u)) dplus[v]++;
        }
    uint64_t dp = 0;
    for (int32_t b = 0; b < n; b++) {
        if (dplus[b] == 0) continue;
        uint64_t s = 0;
        for (int32_t p = rp[b]; p < rp[b + 1]; p++) {
            const int32_t a = col[p];
            if (a >= 0 && a < n && later(a, b) && dplus[a] > 0) s += (uint64_t)(dplus[a] - 1);
        }
        dp += s * (uint64_t)dplus[b];
    }
    return w + dp;
}

// Host-side shape checks at submission; the device checks the rest (every
// launch runs with ESC_F_VALIDATE).
esc_status check_shape(int32_t n, const int32_t *rp, const int32_t *col) {
    if (n < 0 || !rp) return ESC_EINVAL;
    if (rp[0] != 0) return ESC_ERANGE;
    for (int32_t v = 0; v < n; v++)
        if (rp[v + 1] < rp[v]) return ESC_ERANGE;
    if (rp[n] & 1) return ESC_ENOTSIMPLE;
    if (rp[n] > 0 && !col) return ESC_EINVAL;
    return ESC_OK;
}

// One launch: a single request alone, or a group as one batched call.
void run_group(esc_server *s, esc_ctx *c, std::vector<Req *> &grp) {
    const int k = grp[0]->k;
    const uint32_t flags = ESC_F_VALIDATE;
    if (grp.size() == 1) {
        Req *r = grp[0];
        r->status = esc_count_subgraphs(c, r->n, r->rp.data(), r->col.empty() ? nullptr : r->col.data(), k, flags,
                                        r->out, nullptr);
        return;
    }
    const int32_t G = (int32_t)grp.size();
    std::vector<int64_t> vo(G + 1, 0), ao(G + 1, 0);
    for (int32_t g = 0; g < G; g++) {
        vo[g + 1] = vo[g] + grp[g]->n;
        ao[g + 1] = ao[g] + (int64_t)grp[g]->col.size();
    }
    std::vector<int32_t> rp((size_t)(vo[G] + G)), col((size_t)ao[G] + 1);
    for (int32_t g = 0; g < G; g++) {
        memcpy(rp.data() + vo[g] + g, grp[g]->rp.data(), sizeof(int32_t) * (grp[g]->n + 1));
        if (!grp[g]->col.empty())
            memcpy(col.data() + ao[g], grp[g]->col.data(), sizeof(int32_t) * grp[g]->col.size());
    }
    const int cnt = k == 4 ? 11 : 45;
    std::vector<esc_u128> rows((size_t)G * cnt);
    esc_status st = run_batched_device(c, G, vo.data(), ao.data(), rp.data(), col.data(), k, flags, nullptr);
    if (st == ESC_OK) st = batched_copy_u128(c, rows.data());
    if (st == ESC_OK) st = call_finish(c, 0, 0, 0);
    if (st == ESC_OK) {
        for (int32_t g = 0; g < G; g++) {
            memcpy(grp[g]->out, rows.data() + (size_t)g * cnt, sizeof(esc_u128) * cnt);
            grp[g]->status = ESC_OK;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->batched_requests += G;
        return;
    }
    // a failed batch (one invalid request poisons its launch): every member
    // again on its own, so that each gets its own status
    for (Req *r : grp)
        r->status = esc_count_subgraphs(c, r->n, r->rp.data(), r->col.empty() ? nullptr : r->col.data(), k, flags,
                                        r->out, nullptr);
}

void worker(esc_server *s, esc_ctx *c) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
        if (s->queue.empty()) {
            if (s->stopping) break;
            continue;
        }
        // the launch: the head, plus queued requests of the same k and size
        // class (graphs of at most PW_MAX_N vertices batch apart from larger
        // ones, so their launches take the per-wave passes); requests that
        // do not match stay queued for the next free worker
        std::vector<Req *> grp{s->queue.front()};
        std::vector<size_t> pos{0};
        size_t est = footprint(grp, s->nwg);
        uint64_t gcost = grp[0]->cost;
        if (grp[0]->n <= s->small_n) {
            const bool tiny = grp[0]->n <= PW_MAX_N;
            const size_t scan = s->queue.size() < (size_t)4 * s->max_group ? s->queue.size() : (size_t)4 * s->max_group;
            for (size_t i = 1; i < scan && (int)grp.size() < s->max_group; i++) {
                Req *r = s->queue[i];
                if (r->k != grp[0]->k || r->n > s->small_n || (r->n <= PW_MAX_N) != tiny) continue;
                if (!r->priced) continue;   // joins a later launch once priced
                if (gcost + r->cost > s->cost_cap) break;   // the launch holds enough work
                gcost += r->cost;
                grp.push_back(r);
                size_t e2 = footprint(grp, s->nwg);
                if (e2 > s->budget) { grp.pop_back(); break; }
                est = e2;
                pos.push_back(i);
            }
        }
        if (grp.size() == 1 && est > s->budget) {
            // cannot fit even alone: fail it without holding up the queue
            Req *r = grp[0];
            s->queue.pop_front();
            r->status = ESC_ENOMEM;
            r->t_done = now_s();
            r->done = true;
            s->completed++;
            s->cv_done.notify_all();
            continue;
        }
        if (s->reserved > 0 && s->reserved + est > s->budget) {
            s->cv.wait(lk);   // until a launch in flight releases its memory
            continue;
        }
        for (size_t j = pos.size(); j-- > 0;) s->queue.erase(s->queue.begin() + (ptrdiff_t)pos[j]);
        s->reserved += est;
        s->running++;
        if (s->running > s->peak_running) s->peak_running = s->running;
        if (s->reserved > s->peak_reserved) s->peak_reserved = s->reserved;
        s->launches++;
        lk.unlock();
        run_group(s, c, grp);
        const double t = now_s();
        lk.lock();
        s->reserved -= est;
        s->running--;
        for (Req *r : grp) {
            r->t_done = t;
            r->done = true;
            s->completed++;
        }
        s->cv.notify_all();
        s->cv_done.notify_all();
    }
}

esc_status take_result(esc_server *s, Req *r, esc_u128 *out, double *seconds) {
    esc_status st = r->status;
    if (st == ESC_OK && out) memcpy(out, r->out, sizeof(esc_u128) * (r->k == 4 ? 11 : 45));
    if (seconds) *seconds = r->t_done - r->t_submit;
    s->reqs.erase(r->ticket);
    if (r->pricing) r->taken = true;   // the pricing thread deletes it when done
    else delete r;
    return st;
}

// Prices submitted requests off the submitting thread: work_cost is O(m)
// host work, which a burst of submissions would otherwise pay in line.
// The head of the queue runs without a price (a request alone may exceed
// the cap); a request joins another's launch only once priced.
void pricer(esc_server *s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv.wait(lk, [&] { return s->stopping || !s->unpriced.empty(); });
        if (s->unpriced.empty()) {
            if (s->stopping) break;
            continue;
        }
        std::vector<Req *> batch;
        while (!s->unpriced.empty() && batch.size() < 64) {
            Req *r = s->unpriced.front();
            s->unpriced.pop_front();
            r->pricing = true;
            batch.push_back(r);
        }
        lk.unlock();
        for (Req *r : batch) r->cost = work_cost(r->n, r->rp.data(), r->col.data(), r->wedges);
        lk.lock();
        for (Req *r : batch) {
            r->priced = true;
            r->pricing = false;
            if (r->taken) delete r;
        }
        s->cv.notify_all();   // priced requests may now join launches
    }
}

}  // namespace

extern "C" esc_status esc_server_start(esc_ctx *ctx, int max_inflight, esc_server **out) {
    if (!ctx || !out || max_inflight < 1 || max_inflight > 64) return ESC_EINVAL;
    *out = nullptr;
    esc_server *s = new (std::nothrow) esc_server();
    if (!s) return ESC_ENOMEM;
    s->device = ctx->device;
    s->nwg = pair_wgs(ctx);
    s->small_n = 1 << 20;
    s->max_group = 256;
    s->cost_cap = (uint64_t)1 << 38;   // some 0.5 s of device work on MI355X
    size_t budget = ctx->budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipSetDevice(ctx->device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return ESC_EDEVICE;
        }
        budget = fr / 2;
    }
    s->budget = budget;
    for (int i = 0; i < max_inflight; i++) {
        esc_ctx *c = nullptr;
        esc_status st = esc_create(&c, ctx->device, 0);
        if (st != ESC_OK) {
            for (esc_ctx *x : s->ctxs) esc_destroy(x);
            delete s;
            return st;
        }
        s->ctxs.push_back(c);
    }
    for (esc_ctx *c : s->ctxs) s->workers.emplace_back(worker, s, c);
    s->pricer = std::thread(pricer, s);
    *out = s;
    return ESC_OK;
}

extern "C" esc_status esc_submit(esc_server *s, int32_t n, const int32_t *row_ptr, const int32_t *col, int k,
                                 uint64_t *ticket) {
    if (!s || !ticket || (k != 4 && k != 5)) return ESC_EINVAL;
    ESC_TRY(check_shape(n, row_ptr, col));
    Req *r = new (std::nothrow) Req();
    if (!r) return ESC_ENOMEM;
    r->n = n;
    r->k = k;
    r->rp.assign(row_ptr, row_ptr + (size_t)n + 1);
    if (row_ptr[n] > 0) r->col.assign(col, col + row_ptr[n]);
    uint64_t w = 0;
    for (int32_t v = 0; v < n; v++) {
        uint64_t d = (uint64_t)(row_ptr[v + 1] - row_ptr[v]);
        w += d * (d - (d > 0)) / 2;
    }
    r->wedges = w;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
        delete r;
        return ESC_EINVAL;
    }
    if (s->queue.size() >= s->max_queue) {   // back-pressure
        delete r;
        return ESC_EBUSY;
    }
    r->ticket = s->next_ticket++;
    s->reqs[r->ticket] = r;
    s->queue.push_back(r);
    s->unpriced.push_back(r);
    *ticket = r->ticket;
    s->cv.notify_all();
    return ESC_OK;
}

extern "C" esc_status esc_poll(esc_server *s, uint64_t ticket, esc_u128 *out, int *done, double *seconds) {
    if (!s || !done) return ESC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return ESC_EINVAL;
    if (!it->second->done) {
        *done = 0;
        return ESC_OK;
    }
    *done = 1;
    return take_result(s, it->second, out, seconds);
}

extern "C" esc_status esc_wait(esc_server *s, uint64_t ticket, esc_u128 *out, double *seconds) {
    if (!s) return ESC_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return ESC_EINVAL;
    Req *r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    return take_result(s, r, out, seconds);
}

extern "C" esc_status esc_server_stats(esc_server *s, uint64_t *out) {
    if (!s || !out) return ESC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    out[0] = s->completed;
    out[1] = s->launches;
    out[2] = s->batched_requests;
    out[3] = (uint64_t)s->peak_running;
    out[4] = (uint64_t)s->peak_reserved;
    out[5] = (uint64_t)s->budget;
    out[6] = (uint64_t)s->queue.size();
    out[7] = (uint64_t)s->ctxs.size();
    return ESC_OK;
}

extern "C" esc_status esc_server_stop(esc_server *s) {
    if (!s) return ESC_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv.notify_all();
    }
    for (std::thread &t : s->workers) t.join();
    if (s->pricer.joinable()) s->pricer.join();
    for (esc_ctx *c : s->ctxs) esc_destroy(c);
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
    return ESC_OK;
}
