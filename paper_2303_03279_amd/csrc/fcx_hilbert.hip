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
//   windows        FP32 Gram with overlapping windows (blocks of at least 8
//                  samples, at most 3 windows open): k_window_psd and one pass of
//                  k_hilbert_windows over blocks of gcd(L, H) samples, each
//                  block's sums added to the windows holding it; otherwise per
//                  window the window sum of |z_i|^2 (k_psd_batch) and the pair
//                  pass of the batch path (k_pair_batch1).  Both take Re of
//                  the cross-spectrum Gram (and the unit-phasor Gram) on the
//                  matrix cores, and Im(z_i conj z_j) exact-rounded in FP64
//                  with its sign, |Im|, Im^2 and Im sums on the vector units,
//                  with the window's samples in the role of the trials (one
//                  bin, one taper)
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

// ---------------------------------------------------------------------------
// Overlapping windows in one pass (FP32 Gram).  The sample axis is cut into
// blocks of Bk = gcd(L, H) samples; a window is bl = L / Bk consecutive blocks
// and windows start every bh = H / Bk blocks.  Every block's sums are
// computed once, in 32-sample chunks staged through LDS (Re S and the phasor
// Gram on the matrix cores; Im, its sign, |Im| and Im^2 sums in FP64 on the
// vector units), and added to
// each of the NWO = ceil(bl / bh) (2 or 3) windows that hold it; a window's
// metrics are written when its last block is done.
// ---------------------------------------------------------------------------
constexpr int HW_CC = 32;            // samples per staged chunk
constexpr int HW_LD = HW_CC + 1;     // LDS row stride in float2

struct HWin {
    int Bk, bl, bh, nwin, nblk;
    const double *psd;   // [nwin][N] window power sums
    float *out;          // [nwin][7][P]
};

// window power sums: psd[w][i] = sum over the window's samples of |z_i|^2
__global__ __launch_bounds__(256) void k_window_psd(const float2 *__restrict__ z, int N, int L, int H, double *psd)
{
    const int i = blockIdx.x * 256 + threadIdx.x, w = blockIdx.y;
    if (i >= N) return;
    double p = 0.0;
    for (int t = w * H; t < w * H + L; ++t) {
        const float2 v = z[(size_t)t * N + i];
        p += (double)v.x * v.x + (double)v.y * v.y;
    }
    psd[(size_t)w * N + i] = p;
}

template <int NWO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NWO == 2 ? 2 : 1))) void k_hilbert_windows(
    SessDev<float> s, HWin hw)
{
    __shared__ float2 Xs[64 * HW_LD];
    __shared__ float2 Us[64 * HW_LD];
    __shared__ double2 Xd[32 * HW_LD];   // the row nodes again in FP64, for the vector sums
    const int tile = blockIdx.x >> 2, qd = blockIdx.x & 3;
    const int2 tt = s.tiles[tile];
    const int R0 = tt.x * TILE + 32 * (qd >> 1), C0 = tt.y * TILE + 32 * (qd & 1);
    const int N = s.N;
    if (R0 >= N || R0 >= min(C0 + 31, N - 1)) return;   // no pair i < j < N here
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int wr = w >> 1, wc = w & 1;
    const int arow = 16 * wr + lr;           // LDS node of this lane's A fragment
    const int bcol = 32 + 16 * wc + lr;      // LDS node of this lane's B fragment = its pairs' column
    const int j = C0 + 16 * wc + lr;
    int rows[4];                             // accumulator element k: row 4 lg + k of the wave's block
#pragma unroll
    for (int k = 0; k < 4; ++k) rows[k] = 16 * wr + 4 * lg + k;
    const uint32_t mm = s.metrics;
    const bool needU = mm & M_PLV;
    const float2 *z = (const float2 *)s.ring;   // [M][N]
    const size_t P = (size_t)N * (N - 1) / 2;
    const int K = hw.bl * hw.Bk;
    const double Kd = (double)K;

    // open windows: slot q holds window wid[q] (-1: none)
    int wid[NWO];
    float wsr[NWO][4], wur[NWO][4], wui[NWO][4];
    int wg[NWO][4];
    double wsi[NWO][4], wa[NWO][4], wq[NWO][4];
#pragma unroll
    for (int q = 0; q < NWO; ++q) wid[q] = -1;

    for (int blk = 0; blk < hw.nblk; ++blk) {
        if (blk % hw.bh == 0 && blk / hw.bh < hw.nwin) {   // a window starts here
            const int wn = blk / hw.bh;
#pragma unroll
            for (int q = 0; q < NWO; ++q)
                if (q == wn % NWO) {
                    wid[q] = wn;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        wsr[q][k] = wur[q][k] = wui[q][k] = 0.f;
                        wg[q][k] = 0;
                        wsi[q][k] = wa[q][k] = wq[q][k] = 0.0;
                    }
                }
        }
        floatx4 sre = {0.f, 0.f, 0.f, 0.f}, ure = sre, uim = sre;
        int G[4] = {0, 0, 0, 0};
        double Sb[4] = {0.0, 0.0, 0.0, 0.0}, Ab[4] = {0.0, 0.0, 0.0, 0.0}, Qb[4] = {0.0, 0.0, 0.0, 0.0};
        const int tb = blk * hw.Bk;
        for (int t0 = tb; t0 < tb + hw.Bk; t0 += HW_CC) {
            const int nk = min(HW_CC, tb + hw.Bk - t0);
            __syncthreads();
            // consecutive lanes take consecutive nodes of one sample
            for (int e = threadIdx.x; e < 64 * HW_CC; e += 256) {
                const int node = e & 63, col = e >> 6;
                const int g = node < 32 ? R0 + node : C0 + node - 32;
                float2 v = make_float2(0.f, 0.f), u = v;
                if (col < nk && g < N) {
                    v = z[(size_t)(t0 + col) * N + g];
                    if (needU) {
                        const double m2 = (double)v.x * v.x + (double)v.y * v.y;
                        const double r = m2 > 0.0 ? rsqrt(m2) : 0.0;
                        u.x = (float)(v.x * r);
                        u.y = (float)(v.y * r);
                    }
                }
                Xs[node * HW_LD + col] = v;
                if (node < 32) Xd[node * HW_LD + col] = make_double2(v.x, v.y);
                if (needU) Us[node * HW_LD + col] = u;
            }
            __syncthreads();
            // each MFMA step (4 samples) is followed by the vector sums of the
            // same samples; sample t's operands are loaded while sample t - 1
            // is summed (columns past the samples are 0 and add nothing; the
            // pad column HW_CC is loaded but never summed)
            auto mfma_step = [&](int st) {
                {
                    const float2 a = Xs[arow * HW_LD + 4 * st + lg];
                    const float2 bb = Xs[bcol * HW_LD + 4 * st + lg];
                    sre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, sre, 0, 0, 0);
                    sre = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, sre, 0, 0, 0);
                }
                if (needU) {
                    const float2 a = Us[arow * HW_LD + 4 * st + lg];
                    const float2 bb = Us[bcol * HW_LD + 4 * st + lg];
                    ure = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bb.x, ure, 0, 0, 0);
                    ure = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.y, ure, 0, 0, 0);
                    uim = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bb.x, uim, 0, 0, 0);
                    uim = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.x, bb.y, uim, 0, 0, 0);
                }
            };
            auto ldt = [&](int t, double2 (&xr)[4], float2 &xc) {
#pragma unroll
                for (int k = 0; k < 4; ++k) xr[k] = Xd[rows[k] * HW_LD + t];
                xc = Xs[bcol * HW_LD + t];
            };
            auto sum_t = [&](const double2 (&xr)[4], float2 xc) {
                const double jx = xc.x, jy = xc.y;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    // Im(z_i conj z_j) exact-rounded in FP64 (both products exact; never -0); sums in FP64
                    const double ci = __builtin_fma(xr[k].y, jx, __builtin_fma(-xr[k].x, jy, 0.0));
                    G[k] += sign_of_f64(ci);
                    Ab[k] = Ab[k] + fabs(ci);
                    Qb[k] = __builtin_fma(ci, ci, Qb[k]);
                    Sb[k] = Sb[k] + ci;
                }
            };
            double2 ra[4], rb[4];
            float2 ca, cb;
            ldt(0, ra, ca);
            for (int t = 0; t < nk; t += 2) {
                if ((t & 3) == 0) mfma_step(t >> 2);
                ldt(t + 1, rb, cb);
                sum_t(ra, ca);
                ldt(min(t + 2, HW_CC), ra, ca);
                sum_t(rb, cb);
            }
        }
        // the block into every open window, then the windows that end here
#pragma unroll
        for (int q = 0; q < NWO; ++q) {
            if (wid[q] < 0) continue;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                wsr[q][k] += sre[k];
                wsi[q][k] += Sb[k];
                wur[q][k] += ure[k];
                wui[q][k] += uim[k];
                wg[q][k] += G[k];
                wa[q][k] += Ab[k];
                wq[q][k] += Qb[k];
            }
            if (blk != wid[q] * hw.bh + hw.bl - 1) continue;
            const int wn = wid[q];
            wid[q] = -1;
            const double *ps = hw.psd + (size_t)wn * N;
            float *out = hw.out + (size_t)wn * 7 * P;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = R0 + rows[k];
                if (!(i < j && j < N)) continue;
                const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
                const double Sr = wsr[q][k], Si = wsi[q][k], A = wa[q][k], Q = wq[q][k];
                const double pp = ps[i] * ps[j];
                if (mm & M_COH) out[idx] = pp > 0.0 ? (float)sqrt((Sr * Sr + Si * Si) / pp) : 0.f;
                if (mm & M_IMCOH) out[P + idx] = pp > 0.0 ? (float)(Si / sqrt(pp)) : 0.f;
                if (mm & M_PLV) {
                    const double ur = wur[q][k], ui = wui[q][k];
                    out[2 * P + idx] = (float)(sqrt(ur * ur + ui * ui) / Kd);
                }
                const double pli = fabs((double)wg[q][k]) / Kd;
                if (mm & M_PLI) out[3 * P + idx] = (float)pli;
                if (mm & M_WPLI) out[4 * P + idx] = A > 0.0 ? ratio_t<float>(fabs(Si), A) : 0.f;
                if (mm & M_USPLI) out[5 * P + idx] = K >= 2 ? (float)((Kd * pli * pli - 1.0) / (Kd - 1.0)) : NAN;
                if (mm & M_DSWPLI) {
                    const double dd = A * A - Q;
                    out[6 * P + idx] = K >= 2 ? (dd != 0.0 ? ratio_t<float>(Si * Si - Q, dd) : 0.f) : NAN;
                }
            }
        }
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
    // one pass over overlapping windows (FP32 Gram): blocks of Bk samples,
    // windows of bl blocks every bh blocks, nwo windows open at a time
    int Bk = 0, bl = 0, bh = 0, nblk = 0, nwo = 0;
    float2 *tw = nullptr, *g = nullptr, *z = nullptr;
    double *psd = nullptr, *lamw = nullptr, *wpsd = nullptr;
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
    void *bufs[] = {s->tw, s->g, s->z, s->psd, s->lamw, s->tiles, s->ctl, s->wpsd};
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
    {
        int a = K, b = hop;
        while (b) {
            const int t = a % b;
            a = b;
            b = t;
        }
        const int Bk = a, bl = K / Bk, bh = hop / Bk, nwo = (bl + bh - 1) / bh;
        if (cfg->gram_precision == FCX_GRAM_FP32 && hop < K && Bk >= 8 && nwo <= 3) {
            s->Bk = Bk;
            s->bl = bl;
            s->bh = bh;
            s->nwo = nwo;
            s->nblk = (s->n_win - 1) * bh + bl;
        }
    }
    const int nT = (N + TILE - 1) / TILE;
    const int ntiles = nT * (nT + 1) / 2;
    bool ok = hipMalloc((void **)&s->tw, F * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->g, F * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->z, (size_t)M * N * sizeof(float2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->psd, (size_t)N * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->lamw, sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->tiles, (size_t)ntiles * sizeof(int2)) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->ctl, sizeof(DevCtl)) == hipSuccess;
    if (s->nwo) ok = ok && hipMalloc((void **)&s->wpsd, (size_t)s->n_win * N * sizeof(double)) == hipSuccess;
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
    d.nt = 1;
    d.R = K + 1;
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
    if (s->nwo) {
        d.ring = (float *)s->z;
        HWin hw{s->Bk, s->bl, s->bh, s->n_win, s->nblk, s->wpsd, out};
        hipLaunchKernelGGL(k_window_psd, dim3((unsigned)((N + 255) / 256), (unsigned)s->n_win), dim3(256), 0, s->st,
                           (const float2 *)s->z, N, s->K, s->hop, s->wpsd);
        const dim3 pg((unsigned)(d.ntiles * 4)), pb(256);
        if (s->nwo == 2)
            hipLaunchKernelGGL(k_hilbert_windows<2>, pg, pb, 0, s->st, d, hw);
        else
            hipLaunchKernelGGL(k_hilbert_windows<3>, pg, pb, 0, s->st, d, hw);
        if (hipGetLastError() != hipSuccess) return FCX_E_DEVICE;
    }
    for (int w = 0; w < (s->nwo ? 0 : s->n_win); ++w) {
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
