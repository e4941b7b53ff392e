// Serving: a request loop with continuous batching.
//
// Requests (a lattice size and decomposition, MCS count, rates) are queued by
// okpz_server_submit from any thread.  A native worker thread owns the GPU
// work: it admits queued requests in arrival order while their HBM footprint
// fits the budget and a member slot is free, creating a flat lattice for each
// as a member of the batch of its block scheme (a batch holds one scheme, so
// the worker keeps one per scheme); it then advances every member by up to
// `chunk` MCS with one persistent launch per non-empty batch, all on the
// server's stream (a "tick"), retires the members that
// have finished (final moments, optional copy of the final sites, lattice
// freed), and goes round again.  Requests arriving while others run join at
// the next tick, so their work overlaps on the device.  Lattice state stays
// resident on the GPU from admission to retirement.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>

#include "internal.hpp"

using namespace okpz_host;

namespace {

struct Request {
    uint64_t id;
    okpz_params prm;
    uint64_t n_mcs;
    double p, q;
    uint8_t *sites_out;  // caller's L*L buffer or NULL
    double t_submit;
};

struct Member {
    Request req;
    okpz_lattice *lat = nullptr;
    int32_t slot = -1;  // slot in the batch of its block scheme
    uint64_t left = 0;
    uint64_t bytes = 0;
    double t_start = 0;
};

// Device bytes one admitted request holds: the packed lattice and its
// measurement buffers (anchors, per-band partials, totals).
uint64_t footprint(const okpz_params &p)
{
    const uint64_t L = p.L;
    return L * L / 4 + L * sizeof(int32_t) + (L / 4) * okpz::kMomentFields * sizeof(int64_t) +
           2 * okpz::kMomentFields * sizeof(int64_t);
}

}  // namespace

struct okpz_server {
    okpz_server_config cfg;
    hipStream_t stream = nullptr;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    // shared with submitters
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> queue;
    std::deque<okpz_result> results;
    uint64_t next_id = 0;
    uint64_t submitted = 0, finished = 0;
    bool stop = false;
    int status = OKPZ_OK;  // first error of the worker
    // worker-owned: one batch per block scheme (DT, DB, DTr)
    okpz_batch *batch[3] = {nullptr, nullptr, nullptr};
    std::vector<Member> members;
    uint64_t bytes_in_use = 0;
    okpz_server_stats stats;  // guarded by mu
    std::thread worker;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void finish(okpz_server *s, Member &m, int status)
{
    okpz_result r;
    std::memset(&r, 0, sizeof(r));
    r.id = m.req.id;
    r.status = status;
    r.L = m.req.prm.L;
    r.n_mcs = m.req.n_mcs;
    r.t_submit = m.req.t_submit;
    r.t_start = m.t_start;
    if (status == OKPZ_OK && m.lat) {
        status = okpz_measure(m.lat, &r.moments);
        if (status == OKPZ_OK && m.req.sites_out) status = okpz_get_sites(m.lat, m.req.sites_out);
        r.status = status;
    }
    r.t_finish = s->now();
    if (m.slot >= 0) (void)okpz_batch_remove(s->batch[m.req.prm.block_scheme], m.slot);
    if (m.lat) (void)okpz_destroy(m.lat);
    s->bytes_in_use -= m.bytes;
    std::lock_guard<std::mutex> g(s->mu);
    s->results.push_back(r);
    s->finished += 1;
    s->cv.notify_all();
}

void drop_batches(okpz_server *s)
{
    for (okpz_batch *&b : s->batch)
        if (b) {
            (void)okpz_batch_destroy(b);
            b = nullptr;
        }
}

// Admit queued requests in arrival order while they fit.
void admit(okpz_server *s)
{
    for (;;) {
        Request req;
        {
            std::lock_guard<std::mutex> g(s->mu);
            if (s->queue.empty()) return;
            const Request &head = s->queue.front();
            if (s->members.size() >= s->cfg.max_members ||
                s->bytes_in_use + footprint(head.prm) > s->cfg.hbm_budget)
                return;
            req = head;
            s->queue.pop_front();
        }
        Member m;
        m.req = req;
        m.left = req.n_mcs;
        m.bytes = footprint(req.prm);
        m.t_start = s->now();
        s->bytes_in_use += m.bytes;
        int rc = okpz_create(&req.prm, s->stream, &m.lat);
        if (rc == OKPZ_OK) rc = okpz_batch_add(s->batch[req.prm.block_scheme], m.lat, &m.slot);
        if (rc != OKPZ_OK) {
            finish(s, m, rc);
            continue;
        }
        s->members.push_back(m);
        std::lock_guard<std::mutex> g(s->mu);
        s->stats.admitted += 1;
        s->stats.max_members = std::max<uint64_t>(s->stats.max_members, s->members.size());
    }
}

// The three per-scheme batches, configured as the server asks; on failure
// none is left.
int make_batches(okpz_server *s)
{
    int rc = OKPZ_OK;
    for (int b = 0; b < 3 && rc == OKPZ_OK; ++b) {
        rc = okpz_batch_create(s->stream, &s->batch[b]);
        if (rc == OKPZ_OK)
            rc = okpz_batch_config(s->batch[b], s->cfg.threads, s->cfg.grid, s->cfg.use_graph && s->stream);
    }
    if (rc != OKPZ_OK) drop_batches(s);
    return rc;
}

void worker_main(okpz_server *s)
{
    (void)hipSetDevice(s->device);
    std::vector<uint64_t> n[3];
    std::vector<double> p[3], q[3];
    for (;;) {
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv.wait(g, [&] { return s->stop || !s->queue.empty() || !s->members.empty(); });
            if (s->stop && s->members.empty()) return;
        }
        admit(s);
        if (s->members.empty()) continue;
        for (int b = 0; b < 3; ++b) {
            uint32_t nslots = 0;
            (void)okpz_batch_size(s->batch[b], &nslots);
            n[b].assign(nslots, 0);
            p[b].assign(nslots, 0.0);
            q[b].assign(nslots, 0.0);
        }
        uint64_t attempts = 0;
        for (const Member &m : s->members) {
            const int b = m.req.prm.block_scheme;
            const uint64_t k = std::min<uint64_t>(m.left, s->cfg.chunk_mcs);
            n[b][m.slot] = k;
            p[b][m.slot] = m.req.p;
            q[b][m.slot] = m.req.q;
            attempts += (uint64_t)m.req.prm.L * m.req.prm.L * k;
        }
        const double t_launch = s->now();
        // one launch per scheme that has members, queued back to back on the
        // stream, then one wait for all of them
        int rc = OKPZ_OK;
        for (int b = 0; b < 3 && rc == OKPZ_OK; ++b)
            if (!n[b].empty()) rc = okpz_batch_run(s->batch[b], n[b].data(), p[b].data(), q[b].data());
        for (int b = 0; b < 3 && rc == OKPZ_OK; ++b)  // every batch's own error flag
            if (!n[b].empty()) rc = okpz_batch_sync(s->batch[b]);
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stats.busy_seconds += s->now() - t_launch;
            s->stats.ticks += 1;
            if (rc == OKPZ_OK) s->stats.attempts += attempts;
        }
        if (rc != OKPZ_OK) {
            // the batches cannot continue: fail every member and start afresh
            for (Member &m : s->members) finish(s, m, rc);
            s->members.clear();
            drop_batches(s);
            std::lock_guard<std::mutex> g(s->mu);
            if (s->status == OKPZ_OK) s->status = rc;
            if (make_batches(s) != OKPZ_OK) {
                s->stop = true;
                s->cv.notify_all();
                return;
            }
            continue;
        }
        std::vector<Member> keep;
        keep.reserve(s->members.size());
        for (Member &m : s->members) {
            m.left -= std::min<uint64_t>(m.left, s->cfg.chunk_mcs);
            if (m.left == 0)
                finish(s, m, OKPZ_OK);
            else
                keep.push_back(m);
        }
        s->members.swap(keep);
    }
}

}  // namespace

extern "C" {

int okpz_server_create(const okpz_server_config *cfg, void *hip_stream, okpz_server **out)
{
    if (!cfg || !out) return OKPZ_EINVAL;
    *out = nullptr;
    if (cfg->max_members == 0 || cfg->chunk_mcs == 0 || cfg->hbm_budget == 0) return OKPZ_EINVAL;
    okpz_server *s = new (std::nothrow) okpz_server();
    if (!s) return OKPZ_ENOMEM;
    s->cfg = *cfg;
    s->stream = (hipStream_t)hip_stream;
    std::memset(&s->stats, 0, sizeof(s->stats));
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return OKPZ_EHIP;
    }
    const int rc = make_batches(s);
    if (rc != OKPZ_OK) {
        delete s;
        return rc;
    }
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        drop_batches(s);
        delete s;
        return OKPZ_ENOMEM;
    }
    *out = s;
    return OKPZ_OK;
}

int okpz_server_submit(okpz_server *s, const okpz_params *prm, uint64_t n_mcs, double p, double q,
                       uint8_t *sites_out, uint64_t *id)
{
    if (!s || !prm || !id) return OKPZ_EINVAL;
    const int rc = check_params(prm);
    if (rc != OKPZ_OK) return rc;
    if (prm->device_layer != OKPZ_DEVICE_DT)
        return fail_with(OKPZ_EINVAL, "okpz_server_submit: the dead-border control runs on single lattices only");
    if (n_mcs == 0 || n_mcs > kMcsLimit) return OKPZ_EINVAL;
    if (!(p >= 0.0 && p <= 1.0 && q >= 0.0 && q <= 1.0)) return OKPZ_EINVAL;
    if (footprint(*prm) > s->cfg.hbm_budget) return OKPZ_ENOMEM;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return OKPZ_ESTATE;
    Request r;
    r.id = s->next_id++;
    r.prm = *prm;
    r.n_mcs = n_mcs;
    r.p = p;
    r.q = q;
    r.sites_out = sites_out;
    r.t_submit = s->now();
    s->queue.push_back(r);
    s->submitted += 1;
    *id = r.id;
    s->cv.notify_all();
    return OKPZ_OK;
}

int okpz_server_poll(okpz_server *s, okpz_result *out, uint32_t max, uint32_t *n)
{
    if (!s || !n || (max && !out)) return OKPZ_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    uint32_t k = 0;
    while (k < max && !s->results.empty()) {
        out[k++] = s->results.front();
        s->results.pop_front();
    }
    *n = k;
    return OKPZ_OK;
}

int okpz_server_drain(okpz_server *s, double timeout_seconds)
{
    if (!s) return OKPZ_EINVAL;
    std::unique_lock<std::mutex> g(s->mu);
    const bool ok = s->cv.wait_for(g, std::chrono::duration<double>(timeout_seconds),
                                   [&] { return s->finished == s->submitted; });
    if (!ok) return OKPZ_ESTATE;
    return s->status;
}

int okpz_server_get_stats(okpz_server *s, okpz_server_stats *out)
{
    if (!s || !out) return OKPZ_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->stats;
    out->submitted = s->submitted;
    out->finished = s->finished;
    out->queued = s->queue.size();
    out->clock = s->now();
    return OKPZ_OK;
}

int okpz_server_destroy(okpz_server *s)
{
    if (!s) return OKPZ_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->queue.clear();  // queued requests are dropped; running ones finish
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    drop_batches(s);
    delete s;
    return OKPZ_OK;
}

}  // extern "C"
