// Time-resolved phase connectivity from the analytic signal (the approach the
// paper sets against its own in Sec. 4): per segment of N nodes x M samples
//
//   k_analytic     one workgroup per node pair: the two real segments as one
//                  complex transform of F points (x_a + i x_b, zero padded),
//                  separated by conjugate symmetry, each multiplied by the
//                  analytic filter response G[k] = m[k] H[k] / F (H the FIR's
//                  DFT, m = 1 at DC and F/2, 2 at the positive frequencies,
//                  0 above), two inverse transforms; samples D .. D + M - 1
//                  of the result go to z [M][N] (sample-major, complex)
//   per window     the window sum of |z_i|^2 (k_psd_batch) and the pair pass
//                  of the batch path (k_pair_batch): the cross-spectrum Gram
//                  on the matrix cores and the sign / |Im| / Im^2 sums on the
//                  vector units, with the window's samples in the role of the
//                  trials (one bin, one taper)
#include "fcx_device.h"
#include "fcx_fft.h"

#include <math.h>

#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "fcx.h"

#pragma clang fp contract(off)

namespace fcx {

constexpr int HT = 256;               // threads of the transform workgroup
constexpr int HILBERT_MAX_F = 4096;

template <int F>
__global__ __launch_bounds__(HT) void k_analytic(int N, int M, int D, const float *__restrict__ x, long long ld,
                                              const float2 *__restrict__ tw, const float2 *__restrict__ g,
                                              float2 *__restrict__ z)
{
    __shared__ float2 A[F];
    __shared__ float2 Bz[F];
    constexpr int PER = F / HT;
    const int c0 = 2 * blockIdx.x, c1 = c0 + 1;
    const bool two = c1 < N;
    for (int n = threadIdx.x; n < F; n += HT) {
        float a = 0.f, b = 0.f;
        if (n < M) {
            a = x[(size_t)c0 * ld + n];
            if (two) b = x[(size_t)c1 * ld + n];
        }
        A[n] = make_float2(a, -b);                        // conj(x_a + i x_b)
    }
    __syncthreads();
    ifft_wg<F, HT>(A, tw);                                // A[k] = conj(P[k]), P the DFT of x_a + i x_b
    // X_a[k] = (P[k] + conj P[F-k]) / 2, X_b[k] = (P[k] - conj P[F-k]) / 2i
    float2 za[PER], zb[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = threadIdx.x + q * HT;
        za[q] = make_float2(0.f, 0.f);
        zb[q] = za[q];
        if (k <= F / 2) {
            const float2 u = A[k], v = A[(F - k) & (F - 1)];
            const float2 xa = make_float2(0.5f * (u.x + v.x), 0.5f * (v.y - u.y));
            const float2 xb = make_float2(0.5f * (-u.y - v.y), 0.5f * (v.x - u.x));
            const float2 gk = g[k];
            za[q] = cmulf(xa, gk);
            zb[q] = cmulf(xb, gk);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = threadIdx.x + q * HT;
        A[k] = za[q];
        Bz[k] = zb[q];
    }
    __syncthreads();
    ifft_wg<F, HT>(A, tw);
    ifft_wg<F, HT>(Bz, tw);
    for (int t = threadIdx.x; t < M; t += HT) {
        z[(size_t)t * N + c0] = A[t + D];
        if (two) z[(size_t)t * N + c1] = Bz[t + D];
    }
}

}  // namespace fcx

using namespace fcx;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct fcx_hilbert {
    fcx_hilbert_config cfg{};
    std::vector<double> taps;
    hipStream_t st = nullptr;
    int F = 0, D = 0, K = 0, hop = 0, n_win = 0;
    float2 *tw = nullptr, *g = nullptr, *z = nullptr;
    double *psd = nullptr, *lamw = nullptr;
    int2 *tiles = nullptr;
    DevCtl *ctl = nullptr;
    SessDev<float> dev{};
    std::mutex mu;
};

namespace {
std::mutex g_h_mu;
std::unordered_map<uint64_t, fcx_hilbert *> g_hilberts;
uint64_t g_h_next = 1;

fcx_hilbert *lookup_hilbert(fcx_hilbert *h)
{
    std::lock_guard<std::mutex> lk(g_h_mu);
    auto it = g_hilberts.find((uint64_t)(uintptr_t)h);
    return it == g_hilberts.end() ? nullptr : it->second;
}

void hilbert_free(fcx_hilbert *s)
{
    void *bufs[] = {s->tw, s->g, s->z, s->psd, s->lamw, s->tiles, s->ctl};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
}
}  // namespace

extern "C" {

fcx_status fcx_hilbert_open(const fcx_hilbert_config *cfg, void *hip_stream, fcx_hilbert **out)
{
    if (!out) return FCX_E_INVAL;
    *out = nullptr;
    if (!cfg || cfg->struct_size != sizeof(fcx_hilbert_config) || !cfg->taps) return FCX_E_INVAL;
    const int N = cfg->n_nodes, M = cfg->n_samples, T = cfg->n_taps;
    if (N < 2 || N > 65536 || M < 1 || T < 1 || T % 2 == 0 || (long long)M + T - 1 > HILBERT_MAX_F) return FCX_E_INVAL;
    if (cfg->metrics == 0 || (cfg->metrics & ~0x7Fu)) return FCX_E_INVAL;
    if (cfg->gram_precision < FCX_GRAM_FP32 || cfg->gram_precision > FCX_GRAM_BF16X3) return FCX_E_INVAL;
    const int K = cfg->win_len == 0 ? M : cfg->win_len;
    const int hop = cfg->win_hop == 0 ? K : cfg->win_hop;
    if (K < 1 || K > M || hop < 1) return FCX_E_INVAL;
    for (int n = 0; n < T; ++n)
        if (!isfinite(cfg->taps[n])) return FCX_E_INVAL;
    int F = 256;
    while (F < M + T - 1) F *= 2;
    fcx_hilbert *s = new (std::nothrow) fcx_hilbert();
    if (!s) return FCX_E_NOMEM;
    s->cfg = *cfg;
    s->taps.assign(cfg->taps, cfg->taps + T);
    s->cfg.taps = nullptr;
    s->st = (hipStream_t)hip_stream;
    s->F = F;
    s->D = (T - 1) / 2;
    s->K = K;
    s->hop = hop;
    s->n_win = 1 + (M - K) / hop;
    const int nT = (N + TILE - 1) / TILE;
    const int ntiles = nT * (nT + 1) / 2;
    bool ok = hipMalloc((void **)&s->tw, F * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->g, F * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->z, (size_t)M * N * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->psd, (size_t)N * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->lamw, sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->tiles, (size_t)ntiles * sizeof(int2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->ctl, sizeof(DevCtl)) == hipSuccess;
    if (!ok) {
        hilbert_free(s);
        delete s;
        return FCX_E_NOMEM;
    }
    // twiddles; G[k] = m[k] H[k] / F on 0..F/2 (FP64 DFT of the taps), 0 above
    std::vector<float2> tw(F), g(F, make_float2(0.f, 0.f));
    for (int m = 0; m < F; ++m) {
        double c, sn;
        root_of_unity(m, F, &c, &sn);
        tw[m] = make_float2((float)c, (float)sn);
    }
    for (int k = 0; k <= F / 2; ++k) {
        double re = 0.0, im = 0.0;
        for (int n = 0; n < T; ++n) {
            double c, sn;
            root_of_unity((long long)k * n, F, &c, &sn);
            re += s->taps[n] * c;
            im += s->taps[n] * sn;
        }
        const double w = (k == 0 || k == F / 2 ? 1.0 : 2.0) / F;
        g[k] = make_float2((float)(re * w), (float)(im * w));
    }
    std::vector<int2> tl;
    tl.reserve(ntiles);
    for (int a = 0; a < nT; ++a)
        for (int b = a; b < nT; ++b) tl.push_back(make_int2(a, b));
    const double one = 1.0;
    const DevCtl c0{};
    ok = hipMemcpyAsync(s->tw, tw.data(), F * sizeof(float2), hipMemcpyHostToDevice, s->st) == hipSuccess &&
         hipMemcpyAsync(s->g, g.data(), F * sizeof(float2), hipMemcpyHostToDevice, s->st) == hipSuccess &&
         hipMemcpyAsync(s->tiles, tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice, s->st) ==
             hipSuccess &&
         hipMemcpyAsync(s->lamw, &one, sizeof(double), hipMemcpyHostToDevice, s->st) == hipSuccess &&
         hipMemcpyAsync(s->ctl, &c0, sizeof(DevCtl), hipMemcpyHostToDevice, s->st) == hipSuccess &&
         hipStreamSynchronize(s->st) == hipSuccess;
    if (!ok) {
        hilbert_free(s);
        delete s;
        return FCX_E_DEVICE;
    }
    // the pair pass sees the analytic samples as K "trials" of one bin and
    // one taper; ring and out are set per window
    SessDev<float> &d = s->dev;
    d.N = N;
    d.M = M;
    d.W = K;
    d.B = 1;
    d.L = 1;
    d.nT = nT;
    d.ntiles = ntiles;
    d.metrics = cfg->metrics;
    d.tiles = s->tiles;
    d.psd = s->psd;
    d.lamw = s->lamw;
    d.ctl = s->ctl;
    d.kbase = 0;
    std::lock_guard<std::mutex> lk(g_h_mu);
    const uint64_t id = g_h_next++;
    g_hilberts[id] = s;
    *out = (fcx_hilbert *)(uintptr_t)id;
    return FCX_OK;
}

fcx_status fcx_hilbert_info(fcx_hilbert *h, int32_t *n_windows, int32_t *fft_len)
{
    fcx_hilbert *s = lookup_hilbert(h);
    if (!s) return FCX_E_CLOSED;
    if (n_windows) *n_windows = s->n_win;
    if (fft_len) *fft_len = s->F;
    return FCX_OK;
}

fcx_status fcx_hilbert_run(fcx_hilbert *h, const float *x, int64_t ld, float *out, float *z)
{
    fcx_hilbert *s = lookup_hilbert(h);
    if (!s) return FCX_E_CLOSED;
    const int N = s->cfg.n_nodes, M = s->cfg.n_samples;
    if (!x || !out || ld < M) return FCX_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const dim3 grid((unsigned)((N + 1) / 2)), blk(HT);
    switch (s->F) {
    case 256: hipLaunchKernelGGL(k_analytic<256>, grid, blk, 0, s->st, N, M, s->D, x, (long long)ld, s->tw, s->g, s->z); break;
    case 512: hipLaunchKernelGGL(k_analytic<512>, grid, blk, 0, s->st, N, M, s->D, x, (long long)ld, s->tw, s->g, s->z); break;
    case 1024: hipLaunchKernelGGL(k_analytic<1024>, grid, blk, 0, s->st, N, M, s->D, x, (long long)ld, s->tw, s->g, s->z); break;
    case 2048: hipLaunchKernelGGL(k_analytic<2048>, grid, blk, 0, s->st, N, M, s->D, x, (long long)ld, s->tw, s->g, s->z); break;
    default: hipLaunchKernelGGL(k_analytic<4096>, grid, blk, 0, s->st, N, M, s->D, x, (long long)ld, s->tw, s->g, s->z); break;
    }
    if (hipGetLastError() != hipSuccess) return FCX_E_DEVICE;
    const size_t P = (size_t)N * (N - 1) / 2;
    SessDev<float> d = s->dev;
    for (int w = 0; w < s->n_win; ++w) {
        d.ring = (float *)(s->z + (size_t)w * s->hop * N);
        d.out = out + (size_t)w * 7 * P;
        if (launch_psd_batch(d, s->K, s->st) != hipSuccess ||
            launch_pair_batch(d, s->K, s->cfg.gram_precision, s->st) != hipSuccess)
            return FCX_E_DEVICE;
    }
    if (z && hipMemcpyAsync(z, s->z, (size_t)M * N * sizeof(float2), hipMemcpyDeviceToDevice, s->st) != hipSuccess)
        return FCX_E_DEVICE;
    return FCX_OK;
}

fcx_status fcx_hilbert_close(fcx_hilbert *h)
{
    fcx_hilbert *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_h_mu);
        auto it = g_hilberts.find((uint64_t)(uintptr_t)h);
        if (it == g_hilberts.end()) return FCX_E_CLOSED;
        s = it->second;
        g_hilberts.erase(it);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        (void)hipStreamSynchronize(s->st);
        hilbert_free(s);
    }
    delete s;
    return FCX_OK;
}

}  // extern "C"
