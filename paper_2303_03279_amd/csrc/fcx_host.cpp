// Host side of the fcx C ABI: configuration, band plan, tapers, buffer
// planning, the session handle table, and the push / read entry points.
#include "fcx_host.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <new>
#include <unordered_map>

namespace fcx {

#define HIP_OK(call)                                   \
    do {                                               \
        if ((call) != hipSuccess) return FCX_E_DEVICE; \
    } while (0)

// ---------------------------------------------------------------------------
// band plan: bins floor(f F / fs) for both edges, inclusive, clamped to the
// one-sided range [0, F/2]
// ---------------------------------------------------------------------------
static void band_edges(const fcx_config *c, int *lo, int *hi)
{
    const double F = c->n_fft;
    long long a = (long long)floor(c->f_lo_hz * F / c->fs_hz + 1e-9);
    long long b = (long long)floor(c->f_hi_hz * F / c->fs_hz + 1e-9);
    if (a < 0) a = 0;
    if (b > c->n_fft / 2) b = c->n_fft / 2;
    *lo = (int)a;
    *hi = (int)b;
}

fcx_status make_geometry(const fcx_config *c, Geometry *g)
{
    if (!c || c->struct_size != sizeof(fcx_config)) return FCX_E_INVAL;
    if (c->n_nodes < 2 || c->n_nodes > 65536) return FCX_E_INVAL;
    if (c->n_samples < 2 || c->n_samples > 8192) return FCX_E_INVAL;
    if (c->window_trials < 1 || c->window_trials > 32767) return FCX_E_INVAL;
    if (c->n_fft < c->n_samples || c->n_fft > (1 << 20)) return FCX_E_INVAL;
    if (!(c->fs_hz > 0.0) || !isfinite(c->fs_hz)) return FCX_E_INVAL;
    if (!isfinite(c->f_lo_hz) || !isfinite(c->f_hi_hz) || c->f_lo_hz < 0.0 || c->f_hi_hz < c->f_lo_hz)
        return FCX_E_INVAL;
    if (c->metrics == 0 || (c->metrics & ~0x1FFu)) return FCX_E_INVAL;
    if (c->xcor_max_lag < 0 || c->xcor_max_lag > c->n_samples - 1) return FCX_E_INVAL;
    if (c->elem != FCX_ELEM_F32 && c->elem != FCX_ELEM_F64) return FCX_E_INVAL;
    if (c->gram_precision < FCX_GRAM_FP32 || c->gram_precision > FCX_GRAM_BF16X3) return FCX_E_INVAL;
    int L = 1;
    if (c->taper == FCX_TAPER_DPSS) {
        if (c->dpss_k < 1 || c->dpss_k > 8) return FCX_E_INVAL;
        if (!(c->dpss_nw > 0.0) || c->dpss_nw >= c->n_samples / 2.0) return FCX_E_INVAL;
        L = c->dpss_k;
    } else if (c->taper != FCX_TAPER_HANN) {
        return FCX_E_INVAL;
    }
    int lo, hi;
    band_edges(c, &lo, &hi);
    if (hi < lo) return FCX_E_INVAL;
    g->N = c->n_nodes;
    g->M = c->n_samples;
    g->W = c->window_trials;
    g->R = g->W + 1;
    g->F = c->n_fft;
    g->klo = lo;
    g->khi = hi;
    g->B = hi - lo + 1;
    g->L = L;
    g->nT = (g->N + TILE - 1) / TILE;
    g->ntiles = g->nT * (g->nT + 1) / 2;
    g->Mz = (g->M + ZPAD - 1) / ZPAD * ZPAD;
    g->f64 = c->elem == FCX_ELEM_F64;
    g->esz = g->f64 ? 8 : 4;
    g->P = (size_t)g->N * (g->N - 1) / 2;
    if (c->metrics & M_XCOR) {
        // linear correlation at lags -L..L from a circular one of length F
        g->xL = c->xcor_max_lag > 0 ? c->xcor_max_lag : g->M - 1;
        int F = 256;
        while (F < g->M + g->xL) F *= 2;
        if (F > XCOR_MAX_F) return FCX_E_INVAL;
        g->xF = F;
    }
    return FCX_OK;
}

size_t BufferPlan::total() const
{
    size_t t = ring + psd + gsum + out + ctl + wtw + lamw + tiles + zring + rsum + xbuf;
    t += xtw + xtwi + xspec + xpair + xrho + xtail + xg + xtm + xval + xsum;
    for (int i = 0; i < NPLANES; ++i)
        if (planes_used[i]) t += (i == P_URE || i == P_UIM) ? uplane : plane;
    return t;
}

// Unit-phasor sums of FP32 sessions are kept as int32 multiples of 2^-k with
// W * 2^k <= 2^30, exact under add/remove; FP64 sessions and windows longer
// than 256 trials keep FP64 sums.
static int ufix_bits_for(int W)
{
    int c = 0;
    while ((1 << c) < W) ++c;   // ceil(log2 W)
    return 30 - c;
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

BufferPlan make_plan(const fcx_config &c, const Geometry &g)
{
    BufferPlan p;
    const uint32_t m = c.metrics;
    const size_t slots = (size_t)g.R;
    const size_t elems = (size_t)g.ntiles * g.B * TILE_PAIRS;
    const bool spectral = (m & 0x7Fu) != 0;
    if (spectral) {
        p.ring = align256(slots * g.B * g.L * g.N * 2 * g.esz);
        p.psd = align256((size_t)g.B * g.N * 8);
        p.planes_used[P_SRE] = m & M_COH;
        p.planes_used[P_SIM] = m & (M_COH | M_IMCOH | M_WPLI | M_DSWPLI);
        p.planes_used[P_URE] = m & M_PLV;
        p.planes_used[P_UIM] = m & M_PLV;
        p.planes_used[P_A] = m & (M_WPLI | M_DSWPLI);
        p.planes_used[P_Q] = m & M_DSWPLI;
        for (int i = 0; i < NPLANES; ++i) p.nplanes += p.planes_used[i] ? 1 : 0;
        p.plane = align256(elems * 8);
        p.u_fixed = !g.f64 && g.W <= 256;
        p.ufix_bits = p.u_fixed ? ufix_bits_for(g.W) : 0;
        p.uplane = align256(elems * (p.u_fixed ? 4 : 8));
        p.g_used = m & (M_PLI | M_USPLI);
        p.g_narrow = g.W <= 127;
        p.gsum = p.g_used ? align256(elems * (p.g_narrow ? 1 : 2)) : 0;
        p.wtw = align256((size_t)g.L * g.B * g.M * 2 * g.esz);
        p.lamw = align256((size_t)g.L * 8);
    }
    p.out = align256(((m & M_XCOR) ? 9 : 8) * g.P * g.esz);
    p.ctl = align256(2 * sizeof(DevCtl));   // live control + replay control
    p.tiles = align256((size_t)g.ntiles * sizeof(int2));
    if (m & (M_COR | M_XCOR)) p.zring = align256(slots * g.N * g.Mz * 4);
    if (m & M_COR) p.rsum = align256((size_t)g.ntiles * TILE_PAIRS * 8);
    if (m & M_XCOR) {
        const size_t np = (size_t)(g.N + 1) / 2;   // node pairs (2p, 2p + 1)
        p.xtw = align256((size_t)g.xF * 16);
        p.xtwi = align256((size_t)xcor_tw_len(g.xF) * 8);
        p.xspec = align256(2 * np * (g.xF / 2 + 1) * 8);
        p.xpair = align256(np * g.xF * 8);
        p.xrho = align256(2 * np * g.xF * 4);
        p.xtail = align256(2 * np * 8);
        p.xg = align256(2 * np * g.Mz * 8);
        p.xtm = align256((size_t)g.ntiles * TILE_PAIRS * 4);
        p.xval = align256(slots * g.ntiles * TILE_PAIRS * 4);
        p.xsum = align256((size_t)g.ntiles * TILE_PAIRS * 8);
    }
    p.xbuf = align256((size_t)g.N * g.M * g.esz);
    return p;
}

// ---------------------------------------------------------------------------
// tapers
// ---------------------------------------------------------------------------
// exp(-2 pi i r / F): the angle is reduced to a quadrant and then to at most
// pi/4, so multiples of pi/2 come out exact (the DC and Nyquist bins stay
// exactly real) and large r loses no accuracy.
static void unit_root(long long r, long long F, double *c, double *s)
{
    r %= F;
    if (r < 0) r += F;
    const long long q = (4 * r) / F;          // quadrant
    const long long rem = 4 * r - q * F;      // angle within it: (pi/2) rem / F
    double cc, ss;
    if (rem == 0) {
        cc = 1.0;
        ss = 0.0;
    } else if (2 * rem <= F) {
        const double a = (M_PI / 2.0) * (double)rem / (double)F;
        cc = cos(a);
        ss = sin(a);
    } else {
        const double b = (M_PI / 2.0) * (double)(F - rem) / (double)F;
        cc = sin(b);
        ss = cos(b);
    }
    double rc, rs;  // rotate by q quarter turns
    switch (q & 3) {
    case 0: rc = cc; rs = ss; break;
    case 1: rc = -ss; rs = cc; break;
    case 2: rc = -cc; rs = -ss; break;
    default: rc = ss; rs = -cc; break;
    }
    *c = rc;
    *s = -rs;
}

// Symmetric tridiagonal eigenpairs for the DPSS: Sturm-sequence bisection for
// the K largest eigenvalues, then inverse iteration with a pivoted
// tridiagonal solve for each eigenvector.
static int sturm_below(const std::vector<double> &d, const std::vector<double> &e2, double x)
{
    int cnt = 0;
    double q = 1.0;
    const size_t n = d.size();
    for (size_t i = 0; i < n; ++i) {
        q = d[i] - x - (i ? e2[i] / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

static void tridiag_solve(const std::vector<double> &d, const std::vector<double> &e, double shift,
                          std::vector<double> &x)
{
    // Gaussian elimination with partial pivoting on (T - shift I) x = b,
    // e[i] couples i-1 and i.
    const size_t n = d.size();
    std::vector<double> dl(n, 0.0), dd(n), du(n, 0.0), du2(n, 0.0);
    for (size_t i = 0; i < n; ++i) dd[i] = d[i] - shift;
    for (size_t i = 0; i + 1 < n; ++i) {
        du[i] = e[i + 1];
        dl[i] = e[i + 1];
    }
    for (size_t i = 0; i + 1 < n; ++i) {
        if (fabs(dd[i]) >= fabs(dl[i])) {
            if (dd[i] == 0.0) dd[i] = 1e-300;
            const double f = dl[i] / dd[i];
            dd[i + 1] -= f * du[i];
            x[i + 1] -= f * x[i];
            dl[i] = 0.0;
        } else {
            const double f = dd[i] / dl[i];
            dd[i] = dl[i];
            const double t = dd[i + 1];
            dd[i + 1] = du[i] - f * t;
            if (i + 2 < n) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du2[i];
            }
            du[i] = t;
            std::swap(x[i], x[i + 1]);
            x[i + 1] -= f * x[i];
        }
    }
    if (dd[n - 1] == 0.0) dd[n - 1] = 1e-300;
    x[n - 1] /= dd[n - 1];
    if (n > 1) x[n - 2] = (x[n - 2] - du[n - 2] * x[n - 1]) / dd[n - 2];
    for (long long i = (long long)n - 3; i >= 0; --i)
        x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / dd[i];
}

static fcx_status dpss_impl(int M, double NW, int K, double *tapers, double *ratios)
{
    if (M < 2 || K < 1 || K > M || !(NW > 0.0) || NW >= M / 2.0) return FCX_E_INVAL;
    const double Wb = NW / M;
    std::vector<double> d(M), e(M, 0.0), e2(M, 0.0);
    for (int n = 0; n < M; ++n) {
        const double h = (M - 1 - 2.0 * n) / 2.0;
        d[n] = h * h * cos(2.0 * M_PI * Wb);
    }
    for (int n = 1; n < M; ++n) {
        e[n] = 0.5 * n * (double)(M - n);
        e2[n] = e[n] * e[n];
    }
    double lo = 1e300, hi = -1e300;
    for (int n = 0; n < M; ++n) {
        const double r = (n ? fabs(e[n]) : 0.0) + (n + 1 < M ? fabs(e[n + 1]) : 0.0);
        lo = std::min(lo, d[n] - r);
        hi = std::max(hi, d[n] + r);
    }
    std::vector<double> x(M);
    for (int k = 0; k < K; ++k) {
        // eigenvalue with exactly M-1-k eigenvalues below it
        const int target = M - 1 - k;
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 1e-15 * std::max(1.0, fabs(a) + fabs(b)); ++it) {
            const double mid = 0.5 * (a + b);
            if (sturm_below(d, e2, mid) <= target)
                a = mid;
            else
                b = mid;
        }
        const double lam = 0.5 * (a + b);
        for (int n = 0; n < M; ++n) x[n] = 1.0 + 0.01 * sin(0.37 * n + k);
        for (int it = 0; it < 4; ++it) {
            tridiag_solve(d, e, lam, x);
            double nrm = 0.0;
            for (int n = 0; n < M; ++n) nrm += x[n] * x[n];
            nrm = sqrt(nrm);
            for (int n = 0; n < M; ++n) x[n] /= nrm;
        }
        // sign: even orders positive sum, odd orders positive first
        // significant sample (square above max(1e-7, 1/M))
        double sum = 0.0;
        for (int n = 0; n < M; ++n) sum += x[n];
        bool flip = false;
        if (k % 2 == 0) {
            flip = sum < 0.0;
        } else {
            const double th = std::max(1e-7, 1.0 / M);
            for (int n = 0; n < M; ++n)
                if (x[n] * x[n] > th) {
                    flip = x[n] < 0.0;
                    break;
                }
        }
        for (int n = 0; n < M; ++n) tapers[(size_t)k * M + n] = flip ? -x[n] : x[n];
        // concentration in the band |f| < W: w^T A w with the sinc kernel
        double conc = 0.0;
        const double *w = tapers + (size_t)k * M;
        std::vector<double> sk(M);
        sk[0] = 2.0 * Wb;
        for (int m = 1; m < M; ++m) sk[m] = sin(2.0 * M_PI * Wb * m) / (M_PI * m);
        for (int i = 0; i < M; ++i) {
            double acc = 0.0;
            for (int j = 0; j < M; ++j) acc += sk[i > j ? i - j : j - i] * w[j];
            conc += w[i] * acc;
        }
        ratios[k] = conc;
    }
    return FCX_OK;
}

// ---------------------------------------------------------------------------
// handle table: ids are never reused, so a closed handle stays recognisable
// ---------------------------------------------------------------------------
static std::mutex g_tab_mu;
static std::unordered_map<uint64_t, Session *> g_tab;
static uint64_t g_next_id = 1;

uint64_t register_session(Session *s)
{
    std::lock_guard<std::mutex> lk(g_tab_mu);
    s->id = g_next_id++;
    g_tab[s->id] = s;
    return s->id;
}

Session *lookup_session(fcx_session *h, fcx_status *st)
{
    const uint64_t id = (uint64_t)(uintptr_t)h;
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_tab.find(id);
    if (it == g_tab.end()) {
        *st = (id > 0 && id < g_next_id) ? FCX_E_CLOSED : FCX_E_INVAL;
        return nullptr;
    }
    *st = FCX_OK;
    return it->second;
}

Session *unregister_session(fcx_session *h, fcx_status *st)
{
    const uint64_t id = (uint64_t)(uintptr_t)h;
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_tab.find(id);
    if (it == g_tab.end()) {
        *st = (id > 0 && id < g_next_id) ? FCX_E_CLOSED : FCX_E_INVAL;
        return nullptr;
    }
    Session *s = it->second;
    g_tab.erase(it);
    *st = FCX_OK;
    return s;
}

// ---------------------------------------------------------------------------
// allocation
// ---------------------------------------------------------------------------
static fcx_status dalloc(Session *s, size_t bytes, void **p)
{
    *p = nullptr;
    if (bytes == 0) return FCX_OK;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return FCX_E_NOMEM;
    }
    s->allocs.push_back(*p);
    if (hipMemsetAsync(*p, 0, bytes, s->stream) != hipSuccess) return FCX_E_DEVICE;
    return FCX_OK;
}

void session_free(Session *s)
{
    if (s->stream) hipStreamSynchronize(s->stream);
    for (void *p : s->allocs) hipFree(p);
    s->allocs.clear();
    for (int i = 0; i < 2; ++i) {
        if (s->pinned[i]) hipHostFree(s->pinned[i]);
        if (s->pinned_ev[i]) hipEventDestroy(s->pinned_ev[i]);
        s->pinned[i] = nullptr;
        s->pinned_ev[i] = nullptr;
    }
    for (auto &pt : s->pending) {
        hipEventDestroy(pt.a);
        hipEventDestroy(pt.b);
    }
    s->pending.clear();
    for (auto ev : s->free_events) hipEventDestroy(ev);
    s->free_events.clear();
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
    s->stream = nullptr;
}

template <typename T>
static void fill_tables(const Session *s, std::vector<T> &wtw, std::vector<double> &lamw)
{
    const Geometry &g = s->g;
    std::vector<double> taper((size_t)g.L * g.M), lam(g.L, 1.0);
    if (s->cfg.taper == FCX_TAPER_DPSS) {
        dpss_impl(g.M, s->cfg.dpss_nw, g.L, taper.data(), lam.data());
    } else {
        for (int n = 0; n < g.M; ++n) {
            double c, sn;
            unit_root(n, g.M, &c, &sn);
            taper[n] = 0.5 - 0.5 * c;
        }
    }
    double lsum = 0.0;
    for (int l = 0; l < g.L; ++l) lsum += lam[l];
    lamw.resize(g.L);
    for (int l = 0; l < g.L; ++l) lamw[l] = lam[l] / lsum;
    wtw.assign((size_t)g.L * g.B * g.M * 2, (T)0);
    for (int l = 0; l < g.L; ++l)
        for (int b = 0; b < g.B; ++b) {
            const long long k = g.klo + b;
            for (int n = 0; n < g.M; ++n) {
                double c, sn;
                unit_root(k * n, g.F, &c, &sn);
                const size_t o = (((size_t)l * g.B + b) * g.M + n) * 2;
                wtw[o] = (T)(taper[(size_t)l * g.M + n] * c);
                wtw[o + 1] = (T)(taper[(size_t)l * g.M + n] * sn);
            }
        }
}

fcx_status session_alloc(Session *s)
{
    const Geometry &g = s->g;
    const BufferPlan &p = s->plan;
    fcx_status st;
#define ALLOC(field, bytes)                                        \
    do {                                                           \
        void *tmp_ = nullptr;                                      \
        if ((st = dalloc(s, (bytes), &tmp_)) != FCX_OK) return st; \
        s->field = (decltype(s->field))tmp_;                       \
    } while (0)
    ALLOC(ring, p.ring);
    ALLOC(psd, p.psd);
    for (int i = 0; i < NPLANES; ++i)
        if (p.planes_used[i]) ALLOC(plane[i], (i == P_URE || i == P_UIM) ? p.uplane : p.plane);
    if (p.g_used) ALLOC(gsum, p.gsum);
    ALLOC(out, p.out);
    ALLOC(ctl, p.ctl);
    ALLOC(wtw, p.wtw);
    ALLOC(lamw, p.lamw);
    ALLOC(tiles, p.tiles);
    ALLOC(zring, p.zring);
    ALLOC(rsum, p.rsum);
    ALLOC(xbuf, p.xbuf);
    ALLOC(xtw, p.xtw);
    ALLOC(xtwi, p.xtwi);
    ALLOC(xspec, p.xspec);
    ALLOC(xpair, p.xpair);
    ALLOC(xrho, p.xrho);
    ALLOC(xtail, p.xtail);
    ALLOC(xg, p.xg);
    ALLOC(xtm, p.xtm);
    ALLOC(xval, p.xval);
    ALLOC(xsum, p.xsum);
#undef ALLOC
    if (p.xtw) {
        std::vector<double2> tw(g.xF);
        for (int m = 0; m < g.xF; ++m) {
            double c, sn;
            unit_root(m, g.xF, &c, &sn);
            tw[m] = make_double2(c, sn);
        }
        HIP_OK(hipMemcpyAsync(s->xtw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, s->stream));
        // inverse-FFT pass twiddles exp(+2 pi i r k / (R NS)) = conj(exp(-2 pi i r k (F / (R NS)) / F))
        std::vector<float2> twi;
        for (int i = 0; i < xcor_npass(g.xF); ++i) {
            const int R = xcor_pass_r(g.xF, i), NS = xcor_pass_ns(g.xF, i);
            for (int r = 1; r < R; ++r)
                for (int k = 0; k < NS; ++k) {
                    const double2 w = tw[(size_t)r * k * (g.xF / (R * NS))];
                    twi.push_back(make_float2((float)w.x, (float)-w.y));
                }
        }
        HIP_OK(hipMemcpyAsync(s->xtwi, twi.data(), twi.size() * sizeof(float2), hipMemcpyHostToDevice, s->stream));
        HIP_OK(hipMemsetAsync(s->xsum, 0, p.xsum, s->stream));
        HIP_OK(hipStreamSynchronize(s->stream));
    }
    // tile list: upper-triangle tiles in row-major order
    std::vector<int2> tl;
    tl.reserve(g.ntiles);
    for (int a = 0; a < g.nT; ++a)
        for (int b = a; b < g.nT; ++b) tl.push_back(make_int2(a, b));
    HIP_OK(hipMemcpyAsync(s->tiles, tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice, s->stream));
    if (p.wtw) {
        std::vector<double> lamw;
        if (g.f64) {
            std::vector<double> wtw;
            fill_tables<double>(s, wtw, lamw);
            HIP_OK(hipMemcpyAsync(s->wtw, wtw.data(), wtw.size() * 8, hipMemcpyHostToDevice, s->stream));
        } else {
            std::vector<float> wtw;
            fill_tables<float>(s, wtw, lamw);
            HIP_OK(hipMemcpyAsync(s->wtw, wtw.data(), wtw.size() * 4, hipMemcpyHostToDevice, s->stream));
        }
        HIP_OK(hipMemcpyAsync(s->lamw, lamw.data(), lamw.size() * 8, hipMemcpyHostToDevice, s->stream));
        HIP_OK(hipStreamSynchronize(s->stream));  // host tables go out of scope
    }
    for (int i = 0; i < 2; ++i) {
        HIP_OK(hipEventCreateWithFlags(&s->pinned_ev[i], hipEventDisableTiming));
    }
    HIP_OK(hipStreamSynchronize(s->stream));
    return FCX_OK;
}

template <typename T> SessDev<T> session_dev(const Session *s, const void *x, long long ldx)
{
    SessDev<T> d;
    const Geometry &g = s->g;
    d.N = g.N;
    d.M = g.M;
    d.W = g.W;
    d.B = g.B;
    d.L = g.L;
    d.nT = g.nT;
    d.ntiles = g.ntiles;
    d.Mz = g.Mz;
    d.metrics = s->cfg.metrics;
    d.has_cor = (s->cfg.metrics & M_COR) != 0;
    d.tiles = s->tiles;
    d.ring = (T *)s->ring;
    d.psd = s->psd;
    for (int i = 0; i < NPLANES; ++i) d.plane[i] = s->plane[i];
    d.gsum = s->gsum;
    d.u_fixed = s->plan.u_fixed ? 1 : 0;
    d.ufix_bits = s->plan.ufix_bits;
    d.g_narrow = s->plan.g_narrow ? 1 : 0;
    d.out = (T *)s->out;
    d.ctl = s->ctl;
    d.wtw = (const T *)s->wtw;
    d.lamw = s->lamw;
    d.x = x;
    d.ldx = ldx;
    d.zring = s->zring;
    d.zbf = s->zbf;
    d.rsum = s->rsum;
    d.kbase = -1;
    d.nt = 1;
    d.R = g.R;
    d.xL = g.xL;
    d.xF = g.xF;
    d.xtw = s->xtw;
    d.xtwi = s->xtwi;
    d.xspec = s->xspec;
    d.xpair = s->xpair;
    d.xrho = s->xrho;
    d.xtail = s->xtail;
    d.xg = s->xg;
    d.xtm = s->xtm;
    d.xval = s->xval;
    d.xsum = s->xsum;
    return d;
}
template SessDev<float> session_dev<float>(const Session *, const void *, long long);
template SessDev<double> session_dev<double>(const Session *, const void *, long long);

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
static hipEvent_t get_event(Session *s)
{
    if (!s->free_events.empty()) {
        hipEvent_t e = s->free_events.back();
        s->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

static fcx_status resolve_timing(Session *s)
{
    if (s->pending.empty()) return FCX_OK;
    HIP_OK(hipStreamSynchronize(s->stream));
    for (auto &pt : s->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pt.a, pt.b) == hipSuccess) {
            s->launches[pt.kernel] += 1;
            s->total_ms[pt.kernel] += ms;
        }
        s->free_events.push_back(pt.a);
        s->free_events.push_back(pt.b);
    }
    s->pending.clear();
    return FCX_OK;
}

struct TimedLaunch {
    Session *s;
    int kernel;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(Session *s_, int k) : s(s_), kernel(k)
    {
        if (s->timing) {
            a = get_event(s);
            b = get_event(s);
            hipEventRecord(a, s->stream);
        }
    }
    ~TimedLaunch()
    {
        if (a) {
            hipEventRecord(b, s->stream);
            s->pending.push_back({kernel, a, b});
            if (s->pending.size() > 4096) resolve_timing(s);
        }
    }
};

template <typename T> static fcx_status enqueue_push_t(Session *s, const void *xdev, long long ldx)
{
    const SessDev<T> d = session_dev<T>(s, xdev, ldx);
    const bool spectral = (s->cfg.metrics & 0x7Fu) != 0;
    if (spectral) {
        TimedLaunch t(s, FCX_K_SPECTRA);
        HIP_OK(launch_spectra<T>(d, s->stream));
    }
    if (s->cfg.metrics & (M_COR | M_XCOR)) {  // also checks finiteness (time-domain-only sessions)
        TimedLaunch t(s, FCX_K_ZNORM);
        HIP_OK(launch_znorm<T>(d, s->stream));
    }
    if (spectral) {
        TimedLaunch t(s, FCX_K_PSD);
        HIP_OK(launch_psd<T>(d, s->stream));
    }
    if (s->cfg.metrics & (0x7Fu | M_COR)) {
        // spectral running sums and COR Gram blocks of every pair tile
        TimedLaunch t(s, FCX_K_PAIR_UPDATE);
        HIP_OK(launch_pair_update<T>(d, s->stream));
    }
    if (s->cfg.metrics & M_XCOR) {
        TimedLaunch t(s, FCX_K_XCOR);
        HIP_OK(launch_xcor<T>(d, s->stream));
    }
    HIP_OK(launch_commit(s->ctl, s->stream));
    return FCX_OK;
}

fcx_status session_enqueue_push(Session *s, const void *xdev, long long ldx)
{
    return s->g.f64 ? enqueue_push_t<double>(s, xdev, ldx) : enqueue_push_t<float>(s, xdev, ldx);
}

// stage a host trial through pinned memory into the session's device buffer
static fcx_status upload_host_trial(Session *s, const void *x, int64_t ld)
{
    const Geometry &g = s->g;
    const size_t row = (size_t)g.M * g.esz;
    const size_t bytes = row * g.N;
    const int k = s->pinned_next;
    s->pinned_next ^= 1;
    if (!s->pinned[k]) {
        if (hipHostMalloc(&s->pinned[k], bytes, hipHostMallocDefault) != hipSuccess) {
            s->pinned[k] = nullptr;
            return FCX_E_NOMEM;
        }
    }
    if (s->pinned_busy[k]) HIP_OK(hipEventSynchronize(s->pinned_ev[k]));
    const char *src = (const char *)x;
    char *dst = (char *)s->pinned[k];
    if ((size_t)ld * g.esz == row) {
        memcpy(dst, src, bytes);
    } else {
        for (int i = 0; i < g.N; ++i) memcpy(dst + i * row, src + (size_t)i * ld * g.esz, row);
    }
    HIP_OK(hipMemcpyAsync(s->xbuf, dst, bytes, hipMemcpyHostToDevice, s->stream));
    HIP_OK(hipEventRecord(s->pinned_ev[k], s->stream));
    s->pinned_busy[k] = true;
    return FCX_OK;
}

// Rebuild every running sum from the cached window in one pass per kernel
// (power sums; pair planes, COR sums and networks), the trials added oldest
// first with the sliding update's own per-trial terms.  XCOR keeps its
// per-trial path: its window sum is zeroed and each cached trial's maxima are
// recomputed and added, driven by a private control block.
template <typename T> static fcx_status rebuild_window(Session *s, long long pushed)
{
    const Geometry &g = s->g;
    const BufferPlan &p = s->plan;
    const long long K = pushed < g.W ? pushed : g.W;
    const long long first = pushed - K;
    SessDev<T> d = session_dev<T>(s, nullptr, 0);
    const bool spectral = (s->cfg.metrics & 0x7Fu) != 0;
    if (K == 0) {   // an empty window: every sum is zero
        if (p.psd) HIP_OK(hipMemsetAsync(s->psd, 0, p.psd, s->stream));
        for (int i = 0; i < NPLANES; ++i)
            if (s->plane[i])
                HIP_OK(hipMemsetAsync(s->plane[i], 0, (i == P_URE || i == P_UIM) ? p.uplane : p.plane, s->stream));
        if (s->gsum) HIP_OK(hipMemsetAsync(s->gsum, 0, p.gsum, s->stream));
        if (s->rsum) HIP_OK(hipMemsetAsync(s->rsum, 0, p.rsum, s->stream));
    } else {
        if (spectral) HIP_OK(launch_psd_rebuild<T>(d, first, (int)K, s->stream));
        if (s->cfg.metrics & (0x7Fu | M_COR)) HIP_OK(launch_pair_rebuild<T>(d, first, (int)K, s->stream));
    }
    if (s->xsum) {
        HIP_OK(hipMemsetAsync(s->xsum, 0, p.xsum, s->stream));
        d.ctl = s->ctl + 1;
        d.kbase = first;
        for (long long t = first; t < pushed; ++t) {
            HIP_OK(launch_set_ctl(d.ctl, t, s->stream));
            HIP_OK(launch_xcor<T>(d, s->stream));
        }
    }
    HIP_OK(hipStreamSynchronize(s->stream));
    return FCX_OK;
}

static fcx_status read_ctl(Session *s, DevCtl *c)
{
    if (s->server) {
        // a served session: every trial submitted so far is applied first
        const fcx_status st = server_wait_idle(s);
        if (st != FCX_OK) return st;
    }
    HIP_OK(hipStreamSynchronize(s->stream));
    HIP_OK(hipMemcpy(c, s->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost));
    return FCX_OK;
}

// running sums of the current window rebuilt from the ring (after a batch
// pass, or on request)
static fcx_status rebuild_sums(Session *s)
{
    DevCtl c;
    fcx_status st = read_ctl(s, &c);
    if (st != FCX_OK) return st;
    st = s->g.f64 ? rebuild_window<double>(s, c.pushed) : rebuild_window<float>(s, c.pushed);
    if (st == FCX_OK) s->stale = false;
    return st;
}

static fcx_status take_rejections(Session *s, const DevCtl &c)
{
    if (c.rejected > s->reported_rejected) {
        s->reported_rejected = c.rejected;
        return FCX_E_NONFINITE;
    }
    return FCX_OK;
}

}  // namespace fcx

using namespace fcx;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *fcx_status_str(fcx_status st)
{
    switch (st) {
    case FCX_OK: return "ok";
    case FCX_E_INVAL: return "invalid argument";
    case FCX_E_NOMEM: return "out of memory";
    case FCX_E_DEVICE: return "HIP runtime error";
    case FCX_E_NOTREADY: return "not enough trials";
    case FCX_E_BUSY: return "HBM budget exhausted";
    case FCX_E_CLOSED: return "session closed";
    case FCX_E_NONFINITE: return "trial rejected: non-finite sample";
    }
    return "unknown status";
}

void fcx_config_init(fcx_config *c)
{
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->struct_size = sizeof(fcx_config);
    c->window_trials = 1;
    c->fs_hz = 1000.0;
    c->taper = FCX_TAPER_HANN;
    c->metrics = 0xFFu;
    c->gram_precision = FCX_GRAM_FP32;
    c->elem = FCX_ELEM_F32;
}

int32_t fcx_band_bins(const fcx_config *cfg, int32_t *k_lo, int32_t *k_hi)
{
    Geometry g;
    if (make_geometry(cfg, &g) != FCX_OK) return -1;
    if (k_lo) *k_lo = g.klo;
    if (k_hi) *k_hi = g.khi;
    return g.B;
}

int64_t fcx_footprint_bytes(const fcx_config *cfg)
{
    Geometry g;
    if (make_geometry(cfg, &g) != FCX_OK) return -1;
    return (int64_t)make_plan(*cfg, g).total();
}

int64_t fcx_pair_update_bytes(const fcx_config *cfg)
{
    Geometry g;
    if (make_geometry(cfg, &g) != FCX_OK) return -1;
    const BufferPlan p = make_plan(*cfg, g);
    int64_t per_pair_bin = 0;
    for (int i = 0; i < NPLANES; ++i)
        if (p.planes_used[i]) per_pair_bin += (i == P_URE || i == P_UIM) ? (p.u_fixed ? 4 : 8) : 8;
    if (p.g_used) per_pair_bin += p.g_narrow ? 1 : 2;
    int64_t per_pair = 0;
    for (int m = 0; m < 7; ++m)
        if (cfg->metrics & (1u << m)) per_pair += (int64_t)g.esz;
    if (cfg->metrics & M_COR) per_pair += 2 * 8 + (int64_t)g.esz;
    return (int64_t)g.P * (2 * per_pair_bin * g.B + per_pair);
}

fcx_status fcx_dpss(int32_t M, double NW, int32_t K, double *tapers, double *ratios)
{
    if (!tapers || !ratios) return FCX_E_INVAL;
    return dpss_impl(M, NW, K, tapers, ratios);
}

fcx_status fcx_open(const fcx_config *cfg, void *hip_stream, fcx_session **out)
{
    if (!out) return FCX_E_INVAL;
    *out = nullptr;
    Geometry g;
    fcx_status st = make_geometry(cfg, &g);
    if (st != FCX_OK) return st;
    Session *s = new (std::nothrow) Session();
    if (!s) return FCX_E_NOMEM;
    s->cfg = *cfg;
    s->g = g;
    s->plan = make_plan(*cfg, g);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return FCX_E_DEVICE;
    }
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return FCX_E_DEVICE;
        }
        s->own_stream = true;
    }
    st = session_alloc(s);
    if (st != FCX_OK) {
        session_free(s);
        delete s;
        return st;
    }
    *out = (fcx_session *)(uintptr_t)register_session(s);
    return FCX_OK;
}

fcx_status fcx_push_trial(fcx_session *h, const void *x, int64_t ld, int x_on_device)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    if (s->server) return FCX_E_INVAL;  // served sessions take trials through the server
    if (!x || ld < s->g.M) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stale && (st = rebuild_sums(s)) != FCX_OK) return st;
    const void *xdev = x;
    long long ldx = ld;
    if (!x_on_device) {
        st = upload_host_trial(s, x, ld);
        if (st != FCX_OK) return st;
        xdev = s->xbuf;
        ldx = s->g.M;
    }
    return session_enqueue_push(s, xdev, ldx);
}

fcx_status fcx_push_batch(fcx_session *h, const void *x, int64_t n_trials, int64_t trial_stride, int64_t ld,
                          int x_on_device)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    if (s->server) return FCX_E_INVAL;
    if (!x || n_trials < 1 || n_trials > s->g.W || ld < s->g.M || trial_stride < ld * s->g.N)
        return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const BufferPlan &p = s->plan;
    const Geometry &g = s->g;
    const size_t es = g.esz;
    // empty window: the batch trials go to ring slots 0 .. n_trials-1
    HIP_OK(hipMemsetAsync(s->ctl, 0, sizeof(DevCtl), s->stream));
    s->reported_rejected = 0;
    if (g.f64) {
        // FP64 sessions: zero the sums and add the trials one by one
        if (p.psd) HIP_OK(hipMemsetAsync(s->psd, 0, p.psd, s->stream));
        for (int i = 0; i < NPLANES; ++i)
            if (s->plane[i])
                HIP_OK(hipMemsetAsync(s->plane[i], 0, (i == P_URE || i == P_UIM) ? p.uplane : p.plane, s->stream));
        if (s->gsum) HIP_OK(hipMemsetAsync(s->gsum, 0, p.gsum, s->stream));
        if (s->rsum) HIP_OK(hipMemsetAsync(s->rsum, 0, p.rsum, s->stream));
        if (s->xsum) HIP_OK(hipMemsetAsync(s->xsum, 0, p.xsum, s->stream));
        for (int64_t k = 0; k < n_trials; ++k) {
            const void *xk = (const char *)x + (size_t)k * trial_stride * es;
            long long ldk = ld;
            if (!x_on_device) {
                if ((st = upload_host_trial(s, xk, ld)) != FCX_OK) return st;
                xk = s->xbuf;
                ldk = g.M;
            }
            if ((st = session_enqueue_push(s, xk, ldk)) != FCX_OK) return st;
        }
        s->stale = false;
        return FCX_OK;
    }
    // FP32 sessions: spectra of every trial into the ring, then one batch
    // pass with the Gram sums on the matrix cores
    if ((s->cfg.metrics & M_COR) && s->cfg.gram_precision == FCX_GRAM_BF16 && !s->zbf &&
        (st = dalloc(s, (size_t)g.W * g.N * g.Mz * 2, &s->zbf)) != FCX_OK)
        return st;
    SessDev<float> d = session_dev<float>(s, nullptr, 0);
    const bool spectral = (s->cfg.metrics & 0x7Fu) != 0, cor = (s->cfg.metrics & M_COR) != 0;
    const bool zneed = (s->cfg.metrics & (M_COR | M_XCOR)) != 0;   // XCOR comes from the rebuild
    if (x_on_device && n_trials <= 65535) {
        // every trial is already in device memory: one launch each for the
        // spectra and the z-scored samples of all of them (trial k -> slot k)
        d.x = x;
        d.ldx = ld;
        if (spectral) HIP_OK(launch_spectra_batch<float>(d, (int)n_trials, trial_stride, s->stream));
        if (zneed) HIP_OK(launch_znorm_batch<float>(d, (int)n_trials, trial_stride, s->stream));
    } else {
        for (int64_t k = 0; k < n_trials; ++k) {
            const void *xk = (const char *)x + (size_t)k * trial_stride * es;
            long long ldk = ld;
            if (!x_on_device) {
                if ((st = upload_host_trial(s, xk, ld)) != FCX_OK) return st;
                xk = s->xbuf;
                ldk = g.M;
            }
            d.x = xk;
            d.ldx = ldk;
            HIP_OK(launch_set_pushed(s->ctl, k, s->stream));
            if (spectral) HIP_OK(launch_spectra<float>(d, s->stream));
            if (zneed) HIP_OK(launch_znorm<float>(d, s->stream));
        }
    }
    const int prec = s->cfg.gram_precision;
    if (spectral) {
        HIP_OK(launch_psd_batch(d, (int)n_trials, s->stream));
        TimedLaunch t(s, FCX_K_PAIR_BATCH);
        HIP_OK(launch_pair_batch(d, (int)n_trials, prec, s->stream));
    }
    if (cor) {
        TimedLaunch t(s, FCX_K_COR);
        HIP_OK(launch_cor_batch(d, (int)n_trials, prec, s->stream));
    }
    HIP_OK(launch_batch_commit(s->ctl, n_trials, s->stream));
    s->stale = true;  // the running sums do not hold this window yet
    return FCX_OK;
}

fcx_status fcx_sync(fcx_session *h)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    DevCtl c;
    st = read_ctl(s, &c);
    if (st != FCX_OK) return st;
    return take_rejections(s, c);
}

fcx_status fcx_read_network(fcx_session *h, uint32_t metric, void *out, int64_t out_len, int out_on_device,
                            int per_bin, int32_t *k_trials_out)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    if (!out || metric == 0 || (metric & (metric - 1)) || !(metric & s->cfg.metrics)) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const Geometry &g = s->g;
    const bool bins = per_bin && metric != M_COR && metric != M_XCOR;
    const size_t need = bins ? (size_t)g.B * g.P : g.P;
    if (out_len < (int64_t)need) return FCX_E_INVAL;
    DevCtl c;
    st = read_ctl(s, &c);
    if (st != FCX_OK) return st;
    const int64_t K = c.pushed < g.W ? c.pushed : g.W;
    if (k_trials_out) *k_trials_out = (int32_t)K;
    if (K == 0) return FCX_E_NOTREADY;
    int mi = 0;
    while (!((metric >> mi) & 1u)) ++mi;
    const hipMemcpyKind kind = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (!bins) {
        // XCOR is not part of the batch pass: its window sum comes from the rebuild
        if (metric == M_XCOR && s->stale && (st = rebuild_sums(s)) != FCX_OK) return st;
        const char *src = (const char *)s->out + (size_t)mi * g.P * g.esz;
        HIP_OK(hipMemcpy(out, src, g.P * g.esz, kind));
    } else {
        if (s->stale && (st = rebuild_sums(s)) != FCX_OK) return st;
        void *dst = out;
        void *tmp = nullptr;
        if (!out_on_device) {
            if (hipMalloc(&tmp, need * g.esz) != hipSuccess) return FCX_E_NOMEM;
            dst = tmp;
        }
        hipError_t e;
        if (g.f64)
            e = launch_finalize_bins<double>(session_dev<double>(s, nullptr, 0), metric, (double *)dst, s->stream);
        else
            e = launch_finalize_bins<float>(session_dev<float>(s, nullptr, 0), metric, (float *)dst, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess && tmp) e = hipMemcpy(out, tmp, need * g.esz, hipMemcpyDeviceToHost);
        if (tmp) hipFree(tmp);
        if (e != hipSuccess) return FCX_E_DEVICE;
    }
    const fcx_status rej = take_rejections(s, c);
    if (rej != FCX_OK) return rej;
    if (K < 2 && (metric == M_USPLI || metric == M_DSWPLI)) return FCX_E_NOTREADY;
    return FCX_OK;
}

fcx_status fcx_resync(fcx_session *h)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    return rebuild_sums(s);
}

fcx_status fcx_close(fcx_session *h)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    if (s->server) return FCX_E_INVAL;  // close through fcx_server_close_session
    s = unregister_session(h, &st);
    if (!s) return st;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        session_free(s);
    }
    delete s;
    return FCX_OK;
}

fcx_status fcx_session_stream(fcx_session *h, void **hip_stream)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    if (!hip_stream) return FCX_E_INVAL;
    *hip_stream = (void *)s->stream;
    return FCX_OK;
}

fcx_status fcx_session_counts(fcx_session *h, int64_t *accepted, int64_t *rejected)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    DevCtl c;
    st = read_ctl(s, &c);
    if (st != FCX_OK) return st;
    if (accepted) *accepted = c.pushed;
    if (rejected) *rejected = c.rejected;
    return FCX_OK;
}

fcx_status fcx_set_timing(fcx_session *h, int enable)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    st = resolve_timing(s);
    s->timing = enable != 0;
    for (int k = 0; k < FCX_K_COUNT; ++k) {
        s->launches[k] = 0;
        s->total_ms[k] = 0.0;
    }
    return st;
}

fcx_status fcx_kernel_time(fcx_session *h, int kernel, int64_t *launches, double *total_ms)
{
    fcx_status st;
    Session *s = lookup_session(h, &st);
    if (!s) return st;
    if (kernel < 0 || kernel >= FCX_K_COUNT) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    st = resolve_timing(s);
    if (st != FCX_OK) return st;
    if (launches) *launches = s->launches[kernel];
    if (total_ms) *total_ms = s->total_ms[kernel];
    return FCX_OK;
}

fcx_status fcx_probe_copy(void *dst, const void *src, int64_t n_bytes, void *hip_stream)
{
    if (!dst || !src || n_bytes <= 0 || (n_bytes % 16)) return FCX_E_INVAL;
    return launch_copy_probe(dst, src, n_bytes, (hipStream_t)hip_stream) == hipSuccess ? FCX_OK : FCX_E_DEVICE;
}

fcx_status fcx_probe_rmw(void *buf, int64_t n_elems, void *hip_stream)
{
    if (!buf || n_elems <= 0) return FCX_E_INVAL;
    return launch_rmw_probe(buf, n_elems, (hipStream_t)hip_stream) == hipSuccess ? FCX_OK : FCX_E_DEVICE;
}

fcx_status fcx_probe_mfma(int32_t kind, int32_t iters, float *out, double *flops, void *hip_stream)
{
    if (kind < 0 || kind > 2 || iters <= 0 || !out || !flops) return FCX_E_INVAL;
    return launch_mfma_probe(kind, iters, out, flops, (hipStream_t)hip_stream) == hipSuccess ? FCX_OK
                                                                                            : FCX_E_DEVICE;
}

}  // extern "C"
