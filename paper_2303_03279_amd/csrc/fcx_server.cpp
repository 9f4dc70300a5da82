// Serving form: many concurrent sessions, continuous batching.
//
// Admission: a session is opened only if its device footprint fits the
// server's HBM budget (FCX_E_BUSY otherwise).  Submission copies the trial
// into pinned host memory (checking it is finite in the same pass) and
// queues it on its session.  A builder thread forms ticks: every session with
// queued trials contributes its oldest ones -- up to FCX_SERVER_MAX_GROUP
// finite trials in submission order, coalesced into one pass over the
// session's running sums (read once, the trials applied in order, written
// once), or a non-finite trial alone, which the device then rejects as a
// plain push would.  The tick uploads those trials and runs the whole update
// of all of them as five batched launches (spectra, z-scores, power sums,
// pair update with its COR blocks, commit) whose workgroups drain a shared
// list of (session, block) items.  Trials that arrive while a tick runs go
// into the next tick, which is queued behind it on the stream (at most two
// ticks in flight), so the device is never idle while work is waiting.  A
// completion thread waits for each tick's event and stamps its trials done.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fcx_host.h"

namespace fcx {

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Submission {
    uint64_t ticket;
    Session *s;
    void *pinned;
    size_t bytes;
    double t_submit;
    bool finite;     // checked on the host while copying
};

// one session's share of a tick: its trials, applied in order in one pass
struct Group {
    Session *s;
    std::vector<Submission> subs;
};

struct TickBuffers {
    // host (pinned) and device copies of the descriptors and item lists
    SessDev<float> *h_desc = nullptr, *d_desc = nullptr;
    int4 *h_items = nullptr, *d_items = nullptr;
    size_t desc_cap = 0, item_cap = 0;
    hipEvent_t uploaded = nullptr;   // inputs, descriptors and items of the tick are on the device
    hipEvent_t started = nullptr;    // the tick's first kernel may start (timing)
    hipEvent_t done = nullptr;       // its last kernel finished (timing)
};

struct Tick {
    std::vector<Group> groups;
    int buf = 0;
};

struct Server {
    int64_t budget = 0, used = 0;
    int device = 0;
    hipStream_t stream = nullptr;        // kernels
    hipStream_t copy_stream = nullptr;   // host-to-device uploads, overlapping the previous tick
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_slot;
    std::map<uint64_t, Session *> sessions;             // by id, for deterministic order
    std::unordered_map<Session *, std::deque<Submission>> queues;
    std::unordered_map<uint64_t, double> latency;       // finished tickets
    std::unordered_map<uint64_t, bool> pending_tickets;
    std::deque<Tick> inflight;
    TickBuffers bufs[2];
    bool buf_busy[2] = {false, false};
    uint64_t next_ticket = 1;
    int64_t outstanding = 0;
    bool stop = false;
    bool failed = false;
    std::multimap<size_t, void *> pinned_pool;
    std::thread builder, completer;
    bool hold = false;      // fcx_server_hold: queue submissions, form no tick
    int64_t n_ticks = 0, n_trials = 0, max_group = 0;   // statistics
    double busy_ms = 0.0;   // summed device time of the ticks (start to done, one stream)
};

// device bytes a served session holds: the plain session plus one input
// buffer of FCX_SERVER_MAX_GROUP trials per tick buffer (uploads of one tick
// overlap the other tick's kernels)
static size_t tick_input_bytes(const BufferPlan &p) { return p.xbuf * (size_t)FCX_SERVER_MAX_GROUP; }

static int64_t served_footprint(const BufferPlan &p)
{
    return (int64_t)p.total() + 2 * (int64_t)tick_input_bytes(p);
}

static std::mutex g_srv_mu;
static std::unordered_map<uint64_t, Server *> g_srv;
static uint64_t g_srv_next = 1;

static Server *lookup_server(fcx_server *h)
{
    std::lock_guard<std::mutex> lk(g_srv_mu);
    auto it = g_srv.find((uint64_t)(uintptr_t)h);
    return it == g_srv.end() ? nullptr : it->second;
}

static hipError_t ensure_capacity(TickBuffers &b, size_t ndesc, size_t nitems)
{
    hipError_t e = hipSuccess;
    if (ndesc > b.desc_cap) {
        // freed and cleared first, so a failed allocation leaves nothing to
        // free twice
        if (b.h_desc) hipHostFree(b.h_desc);
        if (b.d_desc) hipFree(b.d_desc);
        b.h_desc = nullptr;
        b.d_desc = nullptr;
        b.desc_cap = 0;
        size_t cap = ndesc * 2;
        if ((e = hipHostMalloc((void **)&b.h_desc, cap * sizeof(SessDev<float>), hipHostMallocDefault)) != hipSuccess)
            return e;
        if ((e = hipMalloc((void **)&b.d_desc, cap * sizeof(SessDev<float>))) != hipSuccess) return e;
        b.desc_cap = cap;
    }
    if (nitems > b.item_cap) {
        if (b.h_items) hipHostFree(b.h_items);
        if (b.d_items) hipFree(b.d_items);
        b.h_items = nullptr;
        b.d_items = nullptr;
        b.item_cap = 0;
        size_t cap = nitems * 2;
        if ((e = hipHostMalloc((void **)&b.h_items, cap * sizeof(int4), hipHostMallocDefault)) != hipSuccess)
            return e;
        if ((e = hipMalloc((void **)&b.d_items, cap * sizeof(int4))) != hipSuccess) return e;
        b.item_cap = cap;
    }
    return e;
}

// enqueue one tick (called by the builder with the server lock released)
static hipError_t run_tick(Server *sv, Tick &tk)
{
    TickBuffers &b = sv->bufs[tk.buf];
    const int ns = (int)tk.groups.size();
    // item counts per kernel
    size_t n_sp = 0, n_zn = 0, n_psd = 0, n_pair = 0;
    // pair items are grouped by the session's kernel class: one batched
    // launch per class present, with that class's LDS
    std::vector<int> cls(ns);
    size_t cls_n[PAIR_CLASSES] = {}, cls_lds[PAIR_CLASSES] = {};
    for (int k = 0; k < ns; ++k) {
        Session *s = tk.groups[k].s;
        const int nt = (int)tk.groups[k].subs.size();
        const Geometry &g = s->g;
        cls[k] = pair_kernel_class(session_dev<float>(s, s->xbuf, g.M));
        const uint32_t sm = s->cfg.metrics & 0x7Fu;
        if (sm) {
            n_sp += (size_t)nt * ((g.N + 15) / 16) * ((g.B * g.L + 15) / 16);
            n_psd += (size_t)(g.B * g.N + 255) / 256;
            const size_t l = nt > 1 ? (size_t)nt * pair_lds_bytes(pair_chunk_bins_mt(g.B, g.L, 4, sm, nt), g.L, 4, sm)
                                    : pair_lds_bytes(pair_chunk_bins(g.B, g.L, 4, sm), g.L, 4, sm);
            if (l > cls_lds[cls[k]]) cls_lds[cls[k]] = l;
        }
        if (s->cfg.metrics & M_COR) n_zn += (size_t)nt * ((g.N + 3) / 4);
        const size_t np = (size_t)g.ntiles * SLICES;  // spectral sums and COR blocks of every tile slice
        cls_n[cls[k]] += np;
        n_pair += np;
    }
    const size_t n_items = n_sp + n_zn + n_psd + n_pair;
    hipError_t e = ensure_capacity(b, ns, n_items);
    if (e != hipSuccess) return e;
    int4 *it_sp = b.h_items, *it_zn = it_sp + n_sp, *it_psd = it_zn + n_zn, *it_pair = it_psd + n_psd;
    size_t cls_off[PAIR_CLASSES + 1] = {};
    for (int c = 0; c < PAIR_CLASSES; ++c) cls_off[c + 1] = cls_off[c] + cls_n[c];
    size_t cls_fill[PAIR_CLASSES];
    for (int c = 0; c < PAIR_CLASSES; ++c) cls_fill[c] = cls_off[c];
    size_t a = 0, z = 0, p = 0;
    for (int k = 0; k < ns; ++k) {
        Session *s = tk.groups[k].s;
        const int nt = (int)tk.groups[k].subs.size();
        const Geometry &g = s->g;
        // each tick buffer has its own device input per session; the last
        // tick that used this buffer has finished, so the upload can run
        // while the other buffer's tick computes.  Trial t of the group at
        // t * N * M floats.
        char *xb = (char *)s->xtick[tk.buf];
        for (int t = 0; t < nt; ++t) {
            const Submission &sb = tk.groups[k].subs[t];
            e = hipMemcpyAsync(xb + (size_t)t * sb.bytes, sb.pinned, sb.bytes, hipMemcpyHostToDevice,
                               sv->copy_stream);
            if (e != hipSuccess) return e;
        }
        b.h_desc[k] = session_dev<float>(s, xb, g.M);
        b.h_desc[k].nt = nt;
        const bool spectral = (s->cfg.metrics & 0x7Fu) != 0;
        if (spectral) {
            for (int t = 0; t < nt; ++t)
                for (int by = 0; by < (g.B * g.L + 15) / 16; ++by)
                    for (int bx = 0; bx < (g.N + 15) / 16; ++bx) it_sp[a++] = make_int4(k, bx, by, t);
            for (int bx = 0; bx < (g.B * g.N + 255) / 256; ++bx) it_psd[p++] = make_int4(k, bx, 0, 0);
        }
        if (s->cfg.metrics & M_COR)
            for (int t = 0; t < nt; ++t)
                for (int bx = 0; bx < (g.N + 3) / 4; ++bx) it_zn[z++] = make_int4(k, bx, 0, t);
        for (int t = 0; t < g.ntiles * SLICES; ++t) it_pair[cls_fill[cls[k]]++] = make_int4(k, t, 0, 0);
    }
    if ((e = hipMemcpyAsync(b.d_desc, b.h_desc, ns * sizeof(SessDev<float>), hipMemcpyHostToDevice,
                            sv->copy_stream)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(b.d_items, b.h_items, n_items * sizeof(int4), hipMemcpyHostToDevice,
                            sv->copy_stream)) != hipSuccess)
        return e;
    if ((e = hipEventRecord(b.uploaded, sv->copy_stream)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(sv->stream, b.uploaded, 0)) != hipSuccess) return e;
    if ((e = hipEventRecord(b.started, sv->stream)) != hipSuccess) return e;
    const int4 *d_sp = b.d_items, *d_zn = d_sp + n_sp, *d_psd = d_zn + n_zn, *d_pair = d_psd + n_psd;
    if ((e = launch_batched(FCX_B_SPECTRA, b.d_desc, d_sp, (int)n_sp, 0, sv->stream)) != hipSuccess) return e;
    if ((e = launch_batched(FCX_B_ZNORM, b.d_desc, d_zn, (int)n_zn, 0, sv->stream)) != hipSuccess) return e;
    if ((e = launch_batched(FCX_B_PSD, b.d_desc, d_psd, (int)n_psd, 0, sv->stream)) != hipSuccess) return e;
    for (int c = 0; c < PAIR_CLASSES; ++c)
        if (cls_n[c] &&
            (e = launch_batched_pair(c, b.d_desc, d_pair + cls_off[c], (int)cls_n[c], cls_lds[c], sv->stream)) !=
                hipSuccess)
            return e;
    if ((e = launch_batched(FCX_B_COMMIT, b.d_desc, nullptr, ns, 0, sv->stream)) != hipSuccess) return e;
    return hipEventRecord(b.done, sv->stream);
}

static void builder_main(Server *sv)
{
    hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv_work.wait(lk, [&] {
            if (sv->stop) return true;
            if (sv->hold || (sv->buf_busy[0] && sv->buf_busy[1])) return false;
            for (auto &kv : sv->queues)
                if (!kv.second.empty()) return true;
            return false;
        });
        if (sv->stop) return;
        Tick tk;
        tk.buf = sv->buf_busy[0] ? 1 : 0;
        for (auto &kv : sv->sessions) {  // deterministic order: by session id
            auto qit = sv->queues.find(kv.second);
            if (qit == sv->queues.end() || qit->second.empty()) continue;
            auto &q = qit->second;
            Group gr;
            gr.s = kv.second;
            // the oldest trials, in order: a run of finite ones, or a
            // non-finite one alone (the device rejects it)
            if (!q.front().finite) {
                gr.subs.push_back(q.front());
                q.pop_front();
            } else {
                const Session *ss = kv.second;
                const int lim = std::min(FCX_SERVER_MAX_GROUP,
                                         pair_group_max(ss->g.L, 4, ss->cfg.metrics & 0x7Fu));
                while (!q.empty() && q.front().finite && (int)gr.subs.size() < lim) {
                    gr.subs.push_back(q.front());
                    q.pop_front();
                }
            }
            sv->n_trials += (int64_t)gr.subs.size();
            if ((int64_t)gr.subs.size() > sv->max_group) sv->max_group = (int64_t)gr.subs.size();
            tk.groups.push_back(std::move(gr));
        }
        sv->n_ticks += 1;
        sv->buf_busy[tk.buf] = true;
        lk.unlock();
        const hipError_t e = run_tick(sv, tk);
        lk.lock();
        if (e != hipSuccess) sv->failed = true;
        sv->inflight.push_back(std::move(tk));
        sv->cv_done.notify_all();
    }
}

static void completer_main(Server *sv)
{
    hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv_done.wait(lk, [&] { return sv->stop || !sv->inflight.empty(); });
        if (sv->inflight.empty() && sv->stop) return;
        Tick tk = std::move(sv->inflight.front());
        sv->inflight.pop_front();
        lk.unlock();
        hipEventSynchronize(sv->bufs[tk.buf].done);
        const double t = now_s();
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sv->bufs[tk.buf].started, sv->bufs[tk.buf].done) != hipSuccess) ms = 0.f;
        lk.lock();
        sv->busy_ms += ms;
        for (auto &gr : tk.groups)
            for (auto &sb : gr.subs) {
                sv->latency[sb.ticket] = t - sb.t_submit;
                sv->pending_tickets.erase(sb.ticket);
                sv->pinned_pool.insert({sb.bytes, sb.pinned});
                sv->outstanding -= 1;
            }
        sv->buf_busy[tk.buf] = false;
        sv->cv_work.notify_all();
        sv->cv_slot.notify_all();
    }
}

static bool session_idle(Server *sv, Session *s)
{
    auto it = sv->queues.find(s);
    if (it != sv->queues.end() && !it->second.empty()) return false;
    for (auto &tk : sv->inflight)
        for (auto &gr : tk.groups)
            if (gr.s == s) return false;
    return true;
}

}  // namespace fcx

// Wait until a served session has no queued or unfinished trial, so a read
// of its state sees every trial submitted before it (the builder thread
// enqueues the session's next tick only for trials submitted after that).
fcx_status fcx::server_wait_idle(Session *s)
{
    Server *sv = (Server *)s->server;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->hold) {   // the caller needs the session's trials applied
        sv->hold = false;
        sv->cv_work.notify_all();
    }
    sv->cv_slot.wait(lk, [&] { return session_idle(sv, s) || sv->failed; });
    return sv->failed ? FCX_E_DEVICE : FCX_OK;
}

namespace fcx {

}  // namespace fcx

using namespace fcx;

extern "C" {

int64_t fcx_server_footprint_bytes(const fcx_config *cfg)
{
    Geometry g;
    if (make_geometry(cfg, &g) != FCX_OK || g.f64 || (cfg->metrics & M_XCOR)) return -1;
    g.R = g.W + FCX_SERVER_MAX_GROUP;
    return served_footprint(make_plan(*cfg, g));
}

fcx_status fcx_server_create(int64_t hbm_budget_bytes, fcx_server **out)
{
    if (!out || hbm_budget_bytes <= 0) return FCX_E_INVAL;
    *out = nullptr;
    Server *sv = new (std::nothrow) Server();
    if (!sv) return FCX_E_NOMEM;
    sv->budget = hbm_budget_bytes;
    if (hipGetDevice(&sv->device) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
        delete sv;
        return FCX_E_DEVICE;
    }
    if (hipStreamCreateWithFlags(&sv->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(sv->stream);
        delete sv;
        return FCX_E_DEVICE;
    }
    for (auto &b : sv->bufs)
        if (hipEventCreateWithFlags(&b.done, hipEventDefault) != hipSuccess ||
            hipEventCreateWithFlags(&b.started, hipEventDefault) != hipSuccess ||
            hipEventCreateWithFlags(&b.uploaded, hipEventDisableTiming) != hipSuccess) {
            for (auto &c : sv->bufs) {
                if (c.done) (void)hipEventDestroy(c.done);
                if (c.started) (void)hipEventDestroy(c.started);
                if (c.uploaded) (void)hipEventDestroy(c.uploaded);
            }
            (void)hipStreamDestroy(sv->copy_stream);
            (void)hipStreamDestroy(sv->stream);
            delete sv;
            return FCX_E_DEVICE;
        }
    sv->builder = std::thread(builder_main, sv);
    sv->completer = std::thread(completer_main, sv);
    std::lock_guard<std::mutex> lk(g_srv_mu);
    const uint64_t id = g_srv_next++;
    g_srv[id] = sv;
    *out = (fcx_server *)(uintptr_t)id;
    return FCX_OK;
}

fcx_status fcx_server_open(fcx_server *h, const fcx_config *cfg, fcx_session **out)
{
    Server *sv = lookup_server(h);
    if (!sv || !out) return FCX_E_INVAL;
    *out = nullptr;
    Geometry g;
    fcx_status st = make_geometry(cfg, &g);
    if (st != FCX_OK) return st;
    if (g.f64 || (cfg->metrics & M_XCOR)) return FCX_E_INVAL;  // served sessions: float32, no XCOR
    g.R = g.W + FCX_SERVER_MAX_GROUP;   // room for a coalesced group's new trials
    const int64_t fp = served_footprint(make_plan(*cfg, g));
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->used + fp > sv->budget) return FCX_E_BUSY;
        sv->used += fp;  // reserve before allocating
    }
    Session *s = new (std::nothrow) Session();
    if (!s) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->used -= fp;
        return FCX_E_NOMEM;
    }
    s->cfg = *cfg;
    s->g = g;
    s->plan = make_plan(*cfg, g);
    s->stream = sv->stream;
    s->own_stream = false;
    s->device = sv->device;
    s->server = sv;
    st = session_alloc(s);
    for (int k = 0; k < 2 && st == FCX_OK; ++k) {
        if (hipMalloc(&s->xtick[k], tick_input_bytes(s->plan)) == hipSuccess)
            s->allocs.push_back(s->xtick[k]);
        else
            st = FCX_E_NOMEM;
    }
    if (st != FCX_OK) {
        session_free(s);
        delete s;
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->used -= fp;
        return st;
    }
    const uint64_t id = register_session(s);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->sessions[id] = s;
        sv->queues[s];
    }
    *out = (fcx_session *)(uintptr_t)id;
    return FCX_OK;
}

fcx_status fcx_server_submit(fcx_server *h, fcx_session *hs, const void *x, int64_t ld, uint64_t *ticket)
{
    Server *sv = lookup_server(h);
    if (!sv || !x || !ticket) return FCX_E_INVAL;
    fcx_status st;
    Session *s = lookup_session(hs, &st);
    if (!s) return st;
    if (s->server != sv || ld < s->g.M) return FCX_E_INVAL;
    const size_t row = (size_t)s->g.M * 4;
    const size_t bytes = row * s->g.N;
    void *pin = nullptr;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->failed) return FCX_E_DEVICE;
        auto it = sv->pinned_pool.find(bytes);
        if (it != sv->pinned_pool.end()) {
            pin = it->second;
            sv->pinned_pool.erase(it);
        }
    }
    if (!pin && hipHostMalloc(&pin, bytes, hipHostMallocDefault) != hipSuccess) return FCX_E_NOMEM;
    const char *src = (const char *)x;
    if ((size_t)ld * 4 == row) {
        memcpy(pin, src, bytes);
    } else {
        for (int i = 0; i < s->g.N; ++i) memcpy((char *)pin + i * row, src + (size_t)i * ld * 4, row);
    }
    // Inf or NaN anywhere: exponent bits all ones (an integer OR-reduction
    // over the copy, which is still in cache)
    uint32_t allones = 0;
    const uint32_t *w = (const uint32_t *)pin;
    const size_t n = bytes / 4;
    for (size_t k = 0; k < n; ++k) allones |= (uint32_t)((w[k] & 0x7f800000u) == 0x7f800000u);
    std::lock_guard<std::mutex> lk(sv->mu);
    const uint64_t t = sv->next_ticket++;
    sv->queues[s].push_back({t, s, pin, bytes, now_s(), allones == 0});
    sv->pending_tickets[t] = true;
    sv->outstanding += 1;
    *ticket = t;
    sv->cv_work.notify_all();
    return FCX_OK;
}

fcx_status fcx_server_poll(fcx_server *h, uint64_t ticket, int *done, double *latency_s)
{
    Server *sv = lookup_server(h);
    if (!sv || !done) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->failed) return FCX_E_DEVICE;
    auto it = sv->latency.find(ticket);
    if (it != sv->latency.end()) {
        *done = 1;
        if (latency_s) *latency_s = it->second;
        return FCX_OK;
    }
    if (sv->pending_tickets.count(ticket)) {
        *done = 0;
        return FCX_OK;
    }
    return FCX_E_INVAL;
}

fcx_status fcx_server_drain(fcx_server *h)
{
    Server *sv = lookup_server(h);
    if (!sv) return FCX_E_INVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->hold && sv->outstanding > 0) return FCX_E_BUSY;   // would never finish
    sv->cv_slot.wait(lk, [&] { return sv->outstanding == 0 || sv->failed; });
    return sv->failed ? FCX_E_DEVICE : FCX_OK;
}

fcx_status fcx_server_usage(fcx_server *h, int64_t *used, int64_t *left, int32_t *n_sessions)
{
    Server *sv = lookup_server(h);
    if (!sv) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (used) *used = sv->used;
    if (left) *left = sv->budget - sv->used;
    if (n_sessions) *n_sessions = (int32_t)sv->sessions.size();
    return FCX_OK;
}

fcx_status fcx_server_hold(fcx_server *h, int hold)
{
    Server *sv = lookup_server(h);
    if (!sv) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->hold = hold != 0;
    sv->cv_work.notify_all();
    return FCX_OK;
}

fcx_status fcx_server_counts(fcx_server *h, int64_t *ticks, int64_t *trials, int64_t *max_group, double *busy_ms)
{
    Server *sv = lookup_server(h);
    if (!sv) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (ticks) *ticks = sv->n_ticks;
    if (trials) *trials = sv->n_trials;
    if (max_group) *max_group = sv->max_group;
    if (busy_ms) *busy_ms = sv->busy_ms;
    return FCX_OK;
}

fcx_status fcx_server_close_session(fcx_server *h, fcx_session *hs)
{
    Server *sv = lookup_server(h);
    if (!sv) return FCX_E_INVAL;
    fcx_status st;
    Session *s = lookup_session(hs, &st);
    if (!s) return st;
    if (s->server != sv) return FCX_E_INVAL;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->hold) {
            sv->hold = false;
            sv->cv_work.notify_all();
        }
        sv->cv_slot.wait(lk, [&] { return session_idle(sv, s) || sv->failed; });
        sv->sessions.erase(s->id);
        sv->queues.erase(s);
        sv->used -= served_footprint(s->plan);
    }
    s = unregister_session(hs, &st);
    if (!s) return st;
    session_free(s);
    delete s;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->cv_work.notify_all();
    return FCX_OK;
}

fcx_status fcx_server_destroy(fcx_server *h)
{
    Server *sv = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_srv_mu);
        auto it = g_srv.find((uint64_t)(uintptr_t)h);
        if (it == g_srv.end()) return FCX_E_INVAL;
        sv = it->second;
        g_srv.erase(it);
    }
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->hold = false;
        sv->cv_work.notify_all();
        sv->cv_slot.wait(lk, [&] { return sv->outstanding == 0 || sv->failed; });
        sv->stop = true;
        sv->cv_work.notify_all();
        sv->cv_done.notify_all();
    }
    sv->builder.join();
    sv->completer.join();
    (void)hipStreamSynchronize(sv->copy_stream);
    (void)hipStreamSynchronize(sv->stream);
    std::vector<Session *> left;
    for (auto &kv : sv->sessions) left.push_back(kv.second);
    for (Session *s : left) {
        fcx_status st;
        unregister_session((fcx_session *)(uintptr_t)s->id, &st);
        session_free(s);
        delete s;
    }
    for (auto &kv : sv->pinned_pool) hipHostFree(kv.second);
    for (auto &b : sv->bufs) {
        if (b.h_desc) hipHostFree(b.h_desc);
        if (b.d_desc) hipFree(b.d_desc);
        if (b.h_items) hipHostFree(b.h_items);
        if (b.d_items) hipFree(b.d_items);
        if (b.done) (void)hipEventDestroy(b.done);
        if (b.started) (void)hipEventDestroy(b.started);
        if (b.uploaded) (void)hipEventDestroy(b.uploaded);
    }
    (void)hipStreamDestroy(sv->copy_stream);
    (void)hipStreamDestroy(sv->stream);
    delete sv;
    return FCX_OK;
}

}  // extern "C"
