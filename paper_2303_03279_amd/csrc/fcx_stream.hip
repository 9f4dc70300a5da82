// Stream front end: what feeds pushes from a continuous multichannel stream
// (the noise-reduction and averaging plug-ins of the online pipeline,
// Sec. 2.5).  Per pushed block of every data channel:
//
//   k_fir_block   FFT convolution with a linear-phase FIR, two channels per
//                 transform (x_c + i x_c+1; the filter's response is
//                 Hermitian, so the inverse transform returns both filtered
//                 channels as its real and imaginary parts), overlap-add of
//                 the convolution tail into the next block; the filtered
//                 block goes into a ring of recent samples
//   k_trig_scan   rising edges of the trigger channel (prev < thr <= cur), in
//                 sample order (wavefront ballots)
//   k_cut_trials  the filtered samples of every completed trial window
//
// The filter design (windowed sinc, Hamming window, odd length) is on the
// host.  The output lags the input by the filter's group delay D = (T-1)/2;
// trial windows are shifted by D so that they cover the raw times
// n0 - pre .. n0 + post - 1 around an event at n0.
#include "fcx_device.h"
#include "fcx_fft.h"

#include <math.h>
#include <string.h>

#include <deque>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "fcx.h"

#pragma clang fp contract(off)

namespace fcx {

constexpr int ST = 256;          // threads of the filter workgroup
constexpr int STREAM_MAX_F = 4096;

struct StreamDev {
    int C, Bl, T, F, H;        // channels, block length, taps, FFT length, ring length (power of 2)
    long long n_out;           // filtered samples before this block (the ring position)
    const float2 *tw;          // [F] exp(-2 pi i m / F)
    const float2 *hf;          // [F] filter response, times 1/F
    float *tail;               // [C][T-1] overlap-add carry
    float *ring;               // [C][H] recent filtered samples
};

// One workgroup per channel pair: the forward transform is the inverse one
// applied to the conjugate input, conjugated back.
template <int F>
__global__ __launch_bounds__(ST) void k_fir_block(StreamDev s, const float *__restrict__ x, long long ld, float *y)
{
    __shared__ float2 Z[F];
    const int c0 = 2 * blockIdx.x, c1 = c0 + 1;
    const bool two = c1 < s.C;
    const int Bl = s.Bl, TL = s.T - 1;
    for (int n = threadIdx.x; n < F; n += ST) {
        float a = 0.f, b = 0.f;
        if (n < Bl) {
            a = x[(size_t)c0 * ld + n];
            if (two) b = x[(size_t)c1 * ld + n];
        }
        Z[n] = make_float2(a, -b);                       // conj(x_c0 + i x_c1)
    }
    __syncthreads();
    ifft_wg<F, ST>(Z, s.tw);
    for (int k = threadIdx.x; k < F; k += ST) {
        const float2 u = Z[k];
        Z[k] = cmulf(make_float2(u.x, -u.y), s.hf[k]);   // X(k) H(k) / F
    }
    __syncthreads();
    ifft_wg<F, ST>(Z, s.tw);
    // overlap-add: the block's first T-1 outputs receive the carried tail;
    // the new tail is this block's convolution beyond Bl plus what is left
    // of the old tail
    float *t0 = s.tail + (size_t)c0 * TL, *t1 = s.tail + (size_t)c1 * TL;
    float *r0 = s.ring + (size_t)c0 * s.H, *r1 = s.ring + (size_t)c1 * s.H;
    const unsigned hm = (unsigned)s.H - 1u;
    for (int n = threadIdx.x; n < Bl; n += ST) {
        float v0 = Z[n].x, v1 = Z[n].y;
        if (n < TL) {
            v0 += t0[n];
            if (two) v1 += t1[n];
        }
        const unsigned p = (unsigned)((s.n_out + n) & hm);
        r0[p] = v0;
        if (two) r1[p] = v1;
        if (y) {
            y[(size_t)c0 * Bl + n] = v0;
            if (two) y[(size_t)c1 * Bl + n] = v1;
        }
    }
    // the new tail is assembled in LDS: every old tail value (read above and
    // here) is read before the barrier, every new one written after it
    for (int n = threadIdx.x; n < TL; n += ST) {
        if (Bl + n < TL) {
            float2 v = Z[Bl + n];
            v.x += t0[Bl + n];
            if (two) v.y += t1[Bl + n];
            Z[Bl + n] = v;
        }
    }
    __syncthreads();
    for (int n = threadIdx.x; n < TL; n += ST) {
        const float2 v = Z[Bl + n];
        t0[n] = v.x;
        if (two) t1[n] = v.y;
    }
}

// rising edges in the block, in order; ev[0] = count, ev[1..] = indices
__global__ __launch_bounds__(64) void k_trig_scan(const float *__restrict__ trig, int Bl, float thr, float *last,
                                                 long long base, long long *ev)
{
    const int lane = threadIdx.x;
    long long cnt = 0;
    float prev_last = *last;
    for (int n0 = 0; n0 < Bl; n0 += 64) {
        const int n = n0 + lane;
        const float cur = n < Bl ? trig[n] : -INFINITY;
        const float prev = n == 0 ? prev_last : (n < Bl ? trig[n - 1] : -INFINITY);
        const bool edge = n < Bl && prev < thr && cur >= thr;
        const unsigned long long m = __ballot(edge);
        if (edge) {
            const int rank = __popcll(m & ((1ull << lane) - 1ull));
            ev[1 + cnt + rank] = base + n;
        }
        cnt += __popcll(m);
    }
    if (lane == 0) {
        ev[0] = cnt;
        *last = trig[Bl - 1];
    }
}

// trials[k][c][t] = ring[c][(start_k + t) mod H]
__global__ __launch_bounds__(256) void k_cut_trials(const float *__restrict__ ring, int C, int H, int len,
                                                   const long long *__restrict__ starts, float *trials)
{
    const int k = blockIdx.y, c = blockIdx.x;
    const long long a = starts[k];
    const unsigned hm = (unsigned)H - 1u;
    for (int t = threadIdx.x; t < len; t += 256)
        trials[((size_t)k * C + c) * len + t] = ring[(size_t)c * H + (unsigned)((a + t) & hm)];
}

}  // namespace fcx

using namespace fcx;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct fcx_stream {
    fcx_stream_config cfg{};
    std::vector<double> taps;
    hipStream_t st = nullptr;
    int device = 0;
    int F = 0, H = 0, D = 0;
    long long n_in = 0;                 // raw samples consumed
    float2 *tw = nullptr, *hf = nullptr;
    float *tail = nullptr, *ring = nullptr, *last = nullptr;
    long long *ev = nullptr, *starts = nullptr;
    size_t starts_cap = 0;
    std::vector<long long> h_ev;
    std::deque<long long> pending;      // detected events whose window is not complete yet
    std::mutex mu;
};

namespace {
std::mutex g_st_mu;
std::unordered_map<uint64_t, fcx_stream *> g_streams;
uint64_t g_st_next = 1;

fcx_stream *lookup_stream(fcx_stream *h)
{
    std::lock_guard<std::mutex> lk(g_st_mu);
    auto it = g_streams.find((uint64_t)(uintptr_t)h);
    return it == g_streams.end() ? nullptr : it->second;
}

void stream_free(fcx_stream *s)
{
    void *bufs[] = {s->tw, s->hf, s->tail, s->ring, s->last, s->ev, s->starts};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
}

}  // namespace

extern "C" {

fcx_status fcx_fir_design(int32_t kind, double fs_hz, double f1_hz, double f2_hz, double transition_hz,
                          int32_t n_taps, double *taps, int32_t cap, int32_t *n_taps_out)
{
    if (!(fs_hz > 0.0) || !(f1_hz > 0.0) || f1_hz >= fs_hz / 2.0) return FCX_E_INVAL;
    if (kind == FCX_FIR_BANDPASS && !(f2_hz > f1_hz && f2_hz < fs_hz / 2.0)) return FCX_E_INVAL;
    if (kind < FCX_FIR_LOWPASS || kind > FCX_FIR_BANDPASS) return FCX_E_INVAL;
    int T = n_taps;
    if (T <= 0) {
        if (!(transition_hz > 0.0)) return FCX_E_INVAL;
        const double t = ceil(3.3 * fs_hz / transition_hz);
        if (t > 1e6) return FCX_E_INVAL;
        T = (int)t;
        if (T % 2 == 0) ++T;
    }
    if (T < 3 || T % 2 == 0) return FCX_E_INVAL;
    if (n_taps_out) *n_taps_out = T;
    if (!taps || cap < T) return taps ? FCX_E_INVAL : FCX_OK;
    const double D = (T - 1) / 2.0;
    auto sinc = [](double v) { return v == 0.0 ? 1.0 : sin(M_PI * v) / (M_PI * v); };
    auto ideal_lp = [&](double fc, int n) { return 2.0 * fc / fs_hz * sinc(2.0 * fc / fs_hz * (n - D)); };
    double f0 = 0.0;
    for (int n = 0; n < T; ++n) {
        const double w = 0.54 - 0.46 * cos(2.0 * M_PI * n / (T - 1));
        double v;
        if (kind == FCX_FIR_LOWPASS) {
            v = ideal_lp(f1_hz, n);
        } else if (kind == FCX_FIR_HIGHPASS) {
            v = (n == (int)D ? 1.0 : 0.0) - ideal_lp(f1_hz, n);
        } else {
            v = ideal_lp(f2_hz, n) - ideal_lp(f1_hz, n);
        }
        taps[n] = v * w;
    }
    f0 = kind == FCX_FIR_LOWPASS ? 0.0 : (kind == FCX_FIR_HIGHPASS ? fs_hz / 2.0 : 0.5 * (f1_hz + f2_hz));
    double g = 0.0;
    for (int n = 0; n < T; ++n) g += taps[n] * cos(2.0 * M_PI * f0 / fs_hz * (n - D));
    if (g == 0.0) return FCX_E_INVAL;
    for (int n = 0; n < T; ++n) taps[n] /= g;
    return FCX_OK;
}

fcx_status fcx_stream_open(const fcx_stream_config *cfg, void *hip_stream, fcx_stream **out)
{
    if (!out) return FCX_E_INVAL;
    *out = nullptr;
    if (!cfg || cfg->struct_size != sizeof(fcx_stream_config) || !cfg->taps) return FCX_E_INVAL;
    if (cfg->n_channels < 1 || cfg->n_channels > 65536 || cfg->block_len < 1 || cfg->n_taps < 1 ||
        cfg->n_taps % 2 == 0 || cfg->pre_samples < 0 || cfg->post_samples < 1 ||
        !isfinite(cfg->trigger_threshold))
        return FCX_E_INVAL;
    int F = 256;
    while (F < cfg->block_len + cfg->n_taps - 1) F *= 2;
    if (F > STREAM_MAX_F) return FCX_E_INVAL;
    const long long need = (long long)cfg->pre_samples + cfg->post_samples + cfg->block_len;
    long long H = 256;
    while (H < need) H *= 2;
    if (H > (1 << 24)) return FCX_E_INVAL;
    fcx_stream *s = new (std::nothrow) fcx_stream();
    if (!s) return FCX_E_NOMEM;
    s->cfg = *cfg;
    s->taps.assign(cfg->taps, cfg->taps + cfg->n_taps);
    s->cfg.taps = nullptr;
    s->st = (hipStream_t)hip_stream;
    s->F = F;
    s->H = (int)H;
    s->D = (cfg->n_taps - 1) / 2;
    const int C = cfg->n_channels, TL = cfg->n_taps - 1;
    bool ok = hipGetDevice(&s->device) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->tw, F * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->hf, F * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->tail, ((size_t)(C + 1) * (TL > 0 ? TL : 1)) * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->ring, (size_t)(C + 1) * H * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->last, sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->ev, (size_t)(cfg->block_len + 1) * sizeof(long long)) == hipSuccess;
    if (!ok) {
        stream_free(s);
        delete s;
        return FCX_E_NOMEM;
    }
    // twiddles and the filter response H(k) / F (FP64 DFT of the taps)
    std::vector<float2> tw(F), hf(F);
    for (int m = 0; m < F; ++m) {
        double c, sn;
        root_of_unity(m, F, &c, &sn);
        tw[m] = make_float2((float)c, (float)sn);
    }
    for (int k = 0; k < F; ++k) {
        double re = 0.0, im = 0.0;
        for (int n = 0; n < cfg->n_taps; ++n) {
            double c, sn;
            root_of_unity((long long)k * n, F, &c, &sn);
            re += s->taps[n] * c;
            im += s->taps[n] * sn;
        }
        hf[k] = make_float2((float)(re / F), (float)(im / F));
    }
    const float neg = -INFINITY;
    ok = hipMemcpyAsync(s->tw, tw.data(), F * sizeof(float2), hipMemcpyHostToDevice, s->st) == hipSuccess &&
         hipMemcpyAsync(s->hf, hf.data(), F * sizeof(float2), hipMemcpyHostToDevice, s->st) == hipSuccess &&
         hipMemsetAsync(s->tail, 0, (size_t)(C + 1) * (TL > 0 ? TL : 1) * sizeof(float), s->st) == hipSuccess &&
         hipMemsetAsync(s->ring, 0, (size_t)(C + 1) * H * sizeof(float), s->st) == hipSuccess &&
         hipMemcpyAsync(s->last, &neg, sizeof(float), hipMemcpyHostToDevice, s->st) == hipSuccess &&
         hipStreamSynchronize(s->st) == hipSuccess;
    if (!ok) {
        stream_free(s);
        delete s;
        return FCX_E_DEVICE;
    }
    s->h_ev.resize(cfg->block_len + 1);
    std::lock_guard<std::mutex> lk(g_st_mu);
    const uint64_t id = g_st_next++;
    g_streams[id] = s;
    *out = (fcx_stream *)(uintptr_t)id;
    return FCX_OK;
}

fcx_status fcx_stream_push(fcx_stream *h, const float *x, int64_t ld, const float *trig, float *y, float *trials,
                           int32_t cap, int32_t *n_trials, int32_t *n_dropped)
{
    fcx_stream *s = lookup_stream(h);
    if (!s) return FCX_E_CLOSED;
    const fcx_stream_config &c = s->cfg;
    if (!x || !trig || ld < c.block_len || cap < 0 || (cap > 0 && !trials)) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    StreamDev d;
    d.C = c.n_channels;
    d.Bl = c.block_len;
    d.T = c.n_taps;
    d.F = s->F;
    d.H = s->H;
    d.n_out = s->n_in;   // filtered sample index n holds raw time n - D
    d.tw = s->tw;
    d.hf = s->hf;
    d.tail = s->tail;
    d.ring = s->ring;
    const dim3 grid((unsigned)((c.n_channels + 1) / 2)), blk(ST);
    switch (s->F) {
    case 256: hipLaunchKernelGGL(k_fir_block<256>, grid, blk, 0, s->st, d, x, (long long)ld, y); break;
    case 512: hipLaunchKernelGGL(k_fir_block<512>, grid, blk, 0, s->st, d, x, (long long)ld, y); break;
    case 1024: hipLaunchKernelGGL(k_fir_block<1024>, grid, blk, 0, s->st, d, x, (long long)ld, y); break;
    case 2048: hipLaunchKernelGGL(k_fir_block<2048>, grid, blk, 0, s->st, d, x, (long long)ld, y); break;
    default: hipLaunchKernelGGL(k_fir_block<4096>, grid, blk, 0, s->st, d, x, (long long)ld, y); break;
    }
    hipLaunchKernelGGL(k_trig_scan, dim3(1), dim3(64), 0, s->st, trig, c.block_len, c.trigger_threshold, s->last,
                       (long long)s->n_in, s->ev);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(s->h_ev.data(), s->ev, s->h_ev.size() * sizeof(long long), hipMemcpyDeviceToHost, s->st) !=
            hipSuccess ||
        hipStreamSynchronize(s->st) != hipSuccess)
        return FCX_E_DEVICE;
    s->n_in += c.block_len;
    for (long long k = 0; k < s->h_ev[0]; ++k) s->pending.push_back(s->h_ev[1 + k]);
    // completed windows, in event order
    std::vector<long long> starts;
    int dropped = 0;
    const long long avail = s->n_in;   // filtered samples so far
    while (!s->pending.empty()) {
        const long long n0 = s->pending.front();
        if (n0 - c.pre_samples < 0) {   // the window starts before the stream
            s->pending.pop_front();
            ++dropped;
            continue;
        }
        if (n0 + c.post_samples + s->D > avail) break;   // later events end later
        s->pending.pop_front();
        if ((int)starts.size() < cap)
            starts.push_back(n0 - c.pre_samples + s->D);
        else
            ++dropped;
    }
    if (n_trials) *n_trials = (int32_t)starts.size();
    if (n_dropped) *n_dropped = dropped;
    if (!starts.empty()) {
        if (starts.size() > s->starts_cap) {
            if (s->starts) (void)hipFree(s->starts);
            s->starts = nullptr;
            s->starts_cap = 0;
            if (hipMalloc((void **)&s->starts, starts.size() * sizeof(long long)) != hipSuccess) return FCX_E_NOMEM;
            s->starts_cap = starts.size();
        }
        const int len = c.pre_samples + c.post_samples;
        if (hipMemcpyAsync(s->starts, starts.data(), starts.size() * sizeof(long long), hipMemcpyHostToDevice,
                           s->st) != hipSuccess)
            return FCX_E_DEVICE;
        hipLaunchKernelGGL(k_cut_trials, dim3((unsigned)c.n_channels, (unsigned)starts.size()), dim3(256), 0, s->st,
                           s->ring, c.n_channels, s->H, len, s->starts, trials);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s->st) != hipSuccess) return FCX_E_DEVICE;
    }
    return FCX_OK;
}

fcx_status fcx_stream_close(fcx_stream *h)
{
    fcx_stream *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_st_mu);
        auto it = g_streams.find((uint64_t)(uintptr_t)h);
        if (it == g_streams.end()) return FCX_E_CLOSED;
        s = it->second;
        g_streams.erase(it);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        (void)hipStreamSynchronize(s->st);
        stream_free(s);
    }
    delete s;
    return FCX_OK;
}

}  // extern "C"
