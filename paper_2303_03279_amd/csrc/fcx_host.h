// Host-side session state shared by the single-session API and the server.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/fcx.h"
#include "fcx_internal.h"

namespace fcx {

struct BufferPlan {
    // device byte sizes of every buffer a session allocates
    size_t ring = 0, psd = 0, plane = 0, gsum = 0, out = 0, ctl = 0, wtw = 0, lamw = 0, tiles = 0;
    size_t zring = 0, rsum = 0, xbuf = 0;
    size_t xtw = 0, xtwi = 0, xspec = 0, xpair = 0, xrho = 0, xtail = 0, xg = 0, xtm = 0, xval = 0,
           xsum = 0;   // XCOR
    int nplanes = 0;
    bool planes_used[NPLANES] = {false, false, false, false, false, false};
    bool g_used = false;
    bool u_fixed = false, g_narrow = false;
    int ufix_bits = 0;
    size_t uplane = 0;   // bytes of each unit-phasor plane
    size_t total() const;
};

struct Geometry {
    int N = 0, M = 0, W = 0, F = 0, B = 0, L = 0, klo = 0, khi = 0, nT = 0, ntiles = 0, Mz = 0;
    int xL = 0, xF = 0;   // XCOR lag limit and FFT length
    int R = 0;            // ring slots: W + 1 (a served session: W + FCX_SERVER_MAX_GROUP, so a
                          // coalesced group never overwrites a slot it still evicts)
    bool f64 = false;
    size_t esz = 4;
    size_t P = 0;
};

struct PendingTiming {
    int kernel;
    hipEvent_t a, b;
};

struct Session {
    uint64_t id = 0;
    fcx_config cfg{};
    Geometry g;
    BufferPlan plan;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;

    // device buffers
    void *ring = nullptr;
    double *psd = nullptr;
    void *plane[NPLANES] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    void *gsum = nullptr;
    void *out = nullptr;
    DevCtl *ctl = nullptr;
    void *wtw = nullptr;
    double *lamw = nullptr;
    int2 *tiles = nullptr;
    float *zring = nullptr;
    void *zbf = nullptr;   // BF16 z-scored window of the BF16 COR batch, allocated on first use
    double *rsum = nullptr;
    void *xbuf = nullptr;
    void *xtick[2] = {nullptr, nullptr};   // served sessions: each tick buffer's input of up to
                                           // FCX_SERVER_MAX_GROUP trials
    double2 *xtw = nullptr;
    float2 *xtwi = nullptr;
    float2 *xspec = nullptr, *xpair = nullptr;
    float *xrho = nullptr, *xval = nullptr, *xtm = nullptr;
    int2 *xtail = nullptr;
    double *xg = nullptr;
    double *xsum = nullptr;
    std::vector<void *> allocs;

    // pinned host staging for host-resident trials (two buffers, each
    // guarded by the event of its last upload)
    void *pinned[2] = {nullptr, nullptr};
    hipEvent_t pinned_ev[2] = {nullptr, nullptr};
    bool pinned_busy[2] = {false, false};
    int pinned_next = 0;

    int64_t reported_rejected = 0;
    bool stale = false;   // running sums not yet built for the window (after a batch pass)

    // timing
    bool timing = false;
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> free_events;
    int64_t launches[FCX_K_COUNT] = {0};
    double total_ms[FCX_K_COUNT] = {0};

    // serving
    void *server = nullptr;
    std::mutex mu;   // serialises calls on one session
};

// validation and planning (fcx_host.cpp)
fcx_status make_geometry(const fcx_config *cfg, Geometry *g);
BufferPlan make_plan(const fcx_config &cfg, const Geometry &g);
fcx_status session_alloc(Session *s);  // allocates per plan, uploads tables
void session_free(Session *s);
template <typename T> SessDev<T> session_dev(const Session *s, const void *x, long long ldx);
fcx_status session_enqueue_push(Session *s, const void *xdev, long long ldx);

// served sessions: wait until the session has no queued or unfinished trial
// (fcx_server.cpp)
fcx_status server_wait_idle(Session *s);

// handle table
uint64_t register_session(Session *s);
Session *lookup_session(fcx_session *h, fcx_status *st);
Session *unregister_session(fcx_session *h, fcx_status *st);

}  // namespace fcx
