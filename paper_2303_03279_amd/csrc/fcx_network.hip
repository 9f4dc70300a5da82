// Network post-processing on the device: what the online display consumes
// after every update (results sections and the online pipeline: each network
// is normalised by its maximum edge weight, only the strongest fraction of
// edges is shown, and nodes are sized by their degree in that thresholded
// network).
//
// On a packed upper-triangle FP32 network w[P]:
//   k_sel_scan    max |w| over the finite edges and their count
//   k_sel_init    k = min(ceil(f P), finite edges)
//   k_sel_hist    \  four passes of an 8-bit radix select on the bits of
//   k_sel_pick    /  |w| (monotone for non-negative floats): the exact key T
//                    of the k-th strongest edge
//   k_sel_nodes   one wavefront per node: degree and strength over its N-1
//                 edges (ascending partner, FP64 sum)
//   k_sel_apply   w / max and the selected flags (|w| >= T), counted
// Every edge tied with T is selected, so the selected set is unique.
#include "fcx_device.h"

#include <math.h>
#include <string.h>

#include "fcx.h"

#pragma clang fp contract(off)

namespace fcx {

struct SelCtl {
    unsigned int maxbits;       // max |w| as float bits
    unsigned int prefix, mask;  // radix-select state: key bits found so far
    unsigned int none;          // k == 0: nothing is selected
    long long k, k_left;
    unsigned long long n_finite, n_selected;
    unsigned int hist[256];
};

constexpr int SEL_THREADS = 256;

__device__ __forceinline__ bool sel_key(float v, unsigned int &key)
{
    if (!isfinite(v)) return false;
    key = __float_as_uint(fabsf(v));
    return true;
}

__global__ __launch_bounds__(SEL_THREADS) void k_sel_scan(const float *__restrict__ w, long long P, SelCtl *c)
{
    __shared__ unsigned int smax[SEL_THREADS];
    __shared__ unsigned long long scnt[SEL_THREADS];
    unsigned int mx = 0;
    unsigned long long nf = 0;
    for (long long e = (long long)blockIdx.x * SEL_THREADS + threadIdx.x; e < P; e += (long long)gridDim.x * SEL_THREADS) {
        unsigned int key;
        if (sel_key(w[e], key)) {
            mx = max(mx, key);
            ++nf;
        }
    }
    smax[threadIdx.x] = mx;
    scnt[threadIdx.x] = nf;
    __syncthreads();
    for (int s = SEL_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + s]);
            scnt[threadIdx.x] += scnt[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&c->maxbits, smax[0]);
        atomicAdd(&c->n_finite, scnt[0]);
    }
}

__global__ void k_sel_init(SelCtl *c, double fraction, long long P)
{
    if (threadIdx.x == 0) {
        const double kk = ceil(fraction * (double)P);
        long long k = (long long)kk;
        if (k > (long long)c->n_finite) k = (long long)c->n_finite;
        c->k = k;
        c->k_left = k;
        c->none = k <= 0;
        c->prefix = 0;
        c->mask = 0;
    }
}

__global__ __launch_bounds__(SEL_THREADS) void k_sel_hist(const float *__restrict__ w, long long P, SelCtl *c,
                                                        int shift)
{
    __shared__ unsigned int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const unsigned int prefix = c->prefix, mask = c->mask;
    if (!c->none) {
        for (long long e = (long long)blockIdx.x * SEL_THREADS + threadIdx.x; e < P;
             e += (long long)gridDim.x * SEL_THREADS) {
            unsigned int key;
            if (sel_key(w[e], key) && (key & mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&c->hist[threadIdx.x], h[threadIdx.x]);
}

// picks the digit of the k_left-th largest key among those with the prefix,
// then clears the histogram for the next pass
__global__ void k_sel_pick(SelCtl *c, int shift)
{
    if (threadIdx.x == 0 && !c->none) {
        long long cum = 0;
        for (int d = 255; d >= 0; --d) {
            const long long h = c->hist[d];
            if (cum + h >= c->k_left) {
                c->prefix |= (unsigned int)d << shift;
                c->mask |= 255u << shift;
                c->k_left -= cum;
                break;
            }
            cum += h;
        }
    }
    __syncthreads();
    c->hist[threadIdx.x] = 0;
}

__device__ __forceinline__ bool sel_take(float v, const SelCtl &c, unsigned int T)
{
    unsigned int key;
    return sel_key(v, key) && !c.none && key >= T;
}

__device__ __forceinline__ float sel_norm(float v, float m)
{
    if (m > 0.f) return v / m;
    return isfinite(v) ? 0.f : v;
}

__global__ __launch_bounds__(SEL_THREADS) void k_sel_nodes(const float *__restrict__ w, int N, const SelCtl *c,
                                                         int *degree, float *strength)
{
    const int i = blockIdx.x * (SEL_THREADS / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= N) return;
    const unsigned int T = c->prefix;
    const float m = __uint_as_float(c->maxbits);
    int deg = 0;
    double str = 0.0;
    for (int j = lane; j < N; j += 64) {
        if (j == i) continue;
        const int a = min(i, j), b = max(i, j);
        const long long e = (long long)a * (2LL * N - a - 1) / 2 + (b - a - 1);
        const float v = w[e];
        if (sel_take(v, *c, T)) {
            ++deg;
            str += (double)fabsf(sel_norm(v, m));
        }
    }
    deg = (int)wave_sum((double)deg);
    str = wave_sum(str);
    if (lane == 0) {
        if (degree) degree[i] = deg;
        if (strength) strength[i] = (float)str;
    }
}

__global__ __launch_bounds__(SEL_THREADS) void k_sel_apply(const float *w, long long P, SelCtl *c, float *w_norm,
                                                         unsigned char *selected)
{
    __shared__ unsigned long long scnt[SEL_THREADS];
    const unsigned int T = c->prefix;
    const float m = __uint_as_float(c->maxbits);
    unsigned long long ns = 0;
    for (long long e = (long long)blockIdx.x * SEL_THREADS + threadIdx.x; e < P; e += (long long)gridDim.x * SEL_THREADS) {
        const float v = w[e];
        const bool t = sel_take(v, *c, T);
        ns += t;
        if (selected) selected[e] = t;
        if (w_norm) w_norm[e] = sel_norm(v, m);
    }
    scnt[threadIdx.x] = ns;
    __syncthreads();
    for (int s = SEL_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) scnt[threadIdx.x] += scnt[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&c->n_selected, scnt[0]);
}

}  // namespace fcx

using namespace fcx;

extern "C" fcx_status fcx_network_select(int32_t n_nodes, const float *w, double fraction, float *w_norm,
                                         uint8_t *selected, int32_t *degree, float *strength,
                                         fcx_select_info *info, void *hip_stream)
{
    if (n_nodes < 2 || n_nodes > 65536 || !w || !(fraction >= 0.0 && fraction <= 1.0)) return FCX_E_INVAL;
    const long long P = (long long)n_nodes * (n_nodes - 1) / 2;
    hipStream_t st = (hipStream_t)hip_stream;
    SelCtl *c = nullptr;
    if (hipMalloc((void **)&c, sizeof(SelCtl)) != hipSuccess) return FCX_E_NOMEM;
    fcx_status rs = FCX_OK;
    long long blocks = (P + SEL_THREADS - 1) / SEL_THREADS;
    if (blocks > 4096) blocks = 4096;
    const dim3 grid((unsigned)blocks), blk(SEL_THREADS);
    SelCtl h;
    bool ok = hipMemsetAsync(c, 0, sizeof(SelCtl), st) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_sel_scan, grid, blk, 0, st, w, P, c);
        hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(64), 0, st, c, fraction, P);
        for (int shift = 24; shift >= 0; shift -= 8) {
            hipLaunchKernelGGL(k_sel_hist, grid, blk, 0, st, w, P, c, shift);
            hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, st, c, shift);
        }
        if (degree || strength)
            hipLaunchKernelGGL(k_sel_nodes, dim3((n_nodes + 3) / 4), blk, 0, st, w, n_nodes, c, degree, strength);
        // last: w_norm may overwrite w
        hipLaunchKernelGGL(k_sel_apply, grid, blk, 0, st, w, P, c, w_norm, selected);
        ok = hipGetLastError() == hipSuccess && hipMemcpyAsync(&h, c, sizeof(SelCtl), hipMemcpyDeviceToHost, st) ==
                                                     hipSuccess && hipStreamSynchronize(st) == hipSuccess;
    }
    if (!ok) rs = FCX_E_DEVICE;
    (void)hipFree(c);
    if (rs == FCX_OK && info) {
        float mx, th;
        memcpy(&mx, &h.maxbits, sizeof(float));
        memcpy(&th, &h.prefix, sizeof(float));
        info->max_abs = mx;
        info->threshold = h.none ? INFINITY : th;
        info->k = h.k;
        info->n_finite = (int64_t)h.n_finite;
        info->n_selected = (int64_t)h.n_selected;
    }
    return rs;
}
