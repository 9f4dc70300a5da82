// Network post-processing on the device: what the online display consumes
// after every update (results sections and the online pipeline: each network
// is normalised by its maximum edge weight, only the strongest fraction of
// edges is shown, and nodes are sized by their degree in that thresholded
// network).
//
// On a packed upper-triangle FP32 network w[P]:
//   k_sel_scan    max |w| over the finite edges, their count, and the
//                 histogram of the first digit of the radix select below
//   k_sel_pick    (first) k = min(ceil(f P), finite edges); then for each of
//   k_sel_hist    the three digits (11, 10, 10 bits) of a radix select on the
//                 bits of |w| (monotone for non-negative floats), the digit
//                 of the k-th strongest edge: the exact key T
//   k_sel_rows    one wavefront per row of the triangle: w / max, the
//                 selected flags (|w| >= T), their count, and the degree and
//                 strength of both ends of every selected edge
//   k_sel_node_out  degree and strength out
// Every edge tied with T is selected, so the selected set is unique.
#include "fcx_device.h"

#include <math.h>
#include <string.h>

#include <stddef.h>

#include <mutex>
#include <new>
#include <unordered_map>

#include "fcx.h"

#pragma clang fp contract(off)

namespace fcx {

// Block results are spread over SEL_SLOTS copies of every counter (slot =
// block index mod SEL_SLOTS) so that no single address takes one atomic per
// block; the single-block kernels fold the slots.
constexpr int SEL_SLOTS = 16;
constexpr int SEL_THREADS = 256;
constexpr int SEL_BINS = 2048;     // largest digit: 11 bits
constexpr int SEL_MAX_NODES = 65536;
constexpr int SEL_MAX_BLOCKS = 2048;          // grid of the streaming passes
constexpr double SEL_FIX = 4294967296.0;      // 2^32
constexpr unsigned long long SEL_DEG1 = 1ull << 48;

// the part the host reads back after a call
struct SelHead {
    unsigned int maxbits;       // max |w| as float bits
    unsigned int prefix, mask;  // radix-select state: key bits found so far
    unsigned int none;          // k == 0: nothing is selected
    long long k, k_left;
    unsigned long long n_finite, n_selected;
    unsigned long long slot_ns[SEL_SLOTS];
};

struct SelCtl {
    SelHead h;
    unsigned int blk_max[SEL_MAX_BLOCKS];        // per scan block: max key, finite count
    unsigned long long blk_nf[SEL_MAX_BLOCKS];
    unsigned int hist[SEL_SLOTS][SEL_BINS];
    // per node: selected edges (bits 63..48) and strength in units of 2^-32
    // (bits 47..0; at most 65535 edges of |w_norm| <= 1 fit without carry)
    unsigned long long node[SEL_MAX_NODES];
};

__device__ __forceinline__ bool sel_key(float v, unsigned int &key)
{
    if (!isfinite(v)) return false;
    key = __float_as_uint(fabsf(v));
    return true;
}

// Element e of w, loaded as float4 where the array allows (VEC: w is 16-byte
// aligned); the loop covers the whole array: P4 = P / 4 vectors, then the
// P mod 4 tail by the first block.
template <bool VEC, typename F>
__device__ __forceinline__ void sel_for_each(const float *__restrict__ w, long long P, F &&f)
{
    const long long stride = (long long)gridDim.x * SEL_THREADS;
    const long long t0 = (long long)blockIdx.x * SEL_THREADS + threadIdx.x;
    if (VEC) {
        const long long P4 = P >> 2;
        const float4 *w4 = (const float4 *)w;
        // four independent vector loads in flight per thread
        long long q = t0;
        for (; q + 3 * stride < P4; q += 4 * stride) {
            float4 v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = w4[q + r * stride];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long e = 4 * (q + r * stride);
                f(e, v[r].x);
                f(e + 1, v[r].y);
                f(e + 2, v[r].z);
                f(e + 3, v[r].w);
            }
        }
        for (; q < P4; q += stride) {
            const float4 v = w4[q];
            f(4 * q, v.x);
            f(4 * q + 1, v.y);
            f(4 * q + 2, v.z);
            f(4 * q + 3, v.w);
        }
        if (blockIdx.x == 0 && threadIdx.x < (P & 3)) {
            const long long e = 4 * P4 + threadIdx.x;
            f(e, w[e]);
        }
    } else {
        for (long long e = t0; e < P; e += stride) f(e, w[e]);
    }
}

// The scan also takes the histogram of the first digit (bits 30..20 of
// every finite key: no prefix yet), so the first select pass needs no read
// of its own.
template <bool VEC>
__global__ __launch_bounds__(SEL_THREADS) void k_sel_scan(const float *__restrict__ w, long long P, int N, SelCtl *c)
{
    for (int i = blockIdx.x * SEL_THREADS + threadIdx.x; i < N; i += gridDim.x * SEL_THREADS) c->node[i] = 0;
    __shared__ unsigned int smax[SEL_THREADS / 64];
    __shared__ unsigned long long scnt[SEL_THREADS / 64];
    __shared__ unsigned int h[SEL_BINS];
    for (int d = threadIdx.x; d < SEL_BINS; d += SEL_THREADS) h[d] = 0;
    __syncthreads();
    unsigned int mx = 0;
    unsigned long long nf = 0;
    sel_for_each<VEC>(w, P, [&](long long, float v) {
        unsigned int key;
        if (sel_key(v, key)) {
            mx = max(mx, key);
            ++nf;
            atomicAdd(&h[key >> 20], 1u);
        }
    });
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, (unsigned int)__shfl_xor((int)mx, o));
        nf += (unsigned long long)__shfl_xor((long long)nf, o);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smax[wv] = mx;
        scnt[wv] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < SEL_THREADS / 64; ++q) {
            mx = max(mx, smax[q]);
            nf += scnt[q];
        }
        c->blk_max[blockIdx.x] = mx;
        c->blk_nf[blockIdx.x] = nf;
    }
    unsigned int *g = c->hist[blockIdx.x % SEL_SLOTS];
    for (int d = threadIdx.x; d < SEL_BINS; d += SEL_THREADS)
        if (h[d]) atomicAdd(&g[d], h[d]);
}

// the single-block kernel that folds the histograms and picks a digit
constexpr int PICK_THREADS = 1024;

// folds the scan blocks' partials (nblk of them) and sets up the selection;
// called by every thread of the pick kernel of the first pass
__device__ __forceinline__ void sel_init(SelCtl *c, int nblk, double fraction, long long P)
{
    __shared__ unsigned int smax[PICK_THREADS / 64];
    __shared__ unsigned long long scnt[PICK_THREADS / 64];
    unsigned int mx = 0;
    unsigned long long nf = 0;
    for (int b = threadIdx.x; b < nblk; b += PICK_THREADS) {
        mx = max(mx, c->blk_max[b]);
        nf += c->blk_nf[b];
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, (unsigned int)__shfl_xor((int)mx, o));
        nf += (unsigned long long)__shfl_xor((long long)nf, o);
    }
    if ((threadIdx.x & 63) == 0) {
        smax[threadIdx.x >> 6] = mx;
        scnt[threadIdx.x >> 6] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < PICK_THREADS / 64; ++q) {
            mx = max(mx, smax[q]);
            nf += scnt[q];
        }
        c->h.maxbits = mx;
        c->h.n_finite = nf;
        const double kk = ceil(fraction * (double)P);
        long long k = (long long)kk;
        if (k > (long long)nf) k = (long long)nf;
        c->h.k = k;
        c->h.k_left = k;
        c->h.none = k <= 0;
        c->h.prefix = 0;
        c->h.mask = 0;
    }
    __syncthreads();
}

// LDS histogram of the digit (key >> shift) & (nb - 1) of the keys that
// carry the prefix found so far.  The key's sign bit is always 0, so three
// passes of 11, 10 and 10 bits cover it; the first pass's 2048 bins spread
// the keys of a [-1, 1] network over many bins (few same-address atomics).
template <bool VEC>
__global__ __launch_bounds__(SEL_THREADS) void k_sel_hist(const float *__restrict__ w, long long P, SelCtl *c,
                                                        int shift, int nb)
{
    __shared__ unsigned int h[SEL_BINS];
    for (int d = threadIdx.x; d < nb; d += SEL_THREADS) h[d] = 0;
    __syncthreads();
    const unsigned int prefix = c->h.prefix, mask = c->h.mask, dm = (unsigned int)nb - 1u;
    if (!c->h.none)
        sel_for_each<VEC>(w, P, [&](long long, float v) {
            unsigned int key;
            if (sel_key(v, key) && (key & mask) == prefix) atomicAdd(&h[(key >> shift) & dm], 1u);
        });
    __syncthreads();
    unsigned int *g = c->hist[blockIdx.x % SEL_SLOTS];
    for (int d = threadIdx.x; d < nb; d += SEL_THREADS)
        if (h[d]) atomicAdd(&g[d], h[d]);
}

// picks the digit of the k_left-th largest key among those with the prefix:
// thread t sums the slots of its run of nb / PICK_THREADS bins, a suffix
// scan over the runs (within each wavefront by shuffles, then over the
// wavefront totals) finds the run that holds the k_left-th key, whose
// thread walks its bins from the top; then the histograms are cleared for
// the next pass
__global__ __launch_bounds__(PICK_THREADS) void k_sel_pick(SelCtl *c, int shift, int nb, int nblk, double fraction,
                                                         long long P)
{
    __shared__ unsigned long long wsum[PICK_THREADS / 64];
    if (nblk > 0) sel_init(c, nblk, fraction, P);   // first pass: the scan's partials
    const int per = nb / PICK_THREADS, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // read before any later barrier: one thread rewrites k_left at the end
    const bool none = c->h.none;
    const long long kl = c->h.k_left;
    unsigned int tot[SEL_BINS / PICK_THREADS];
    unsigned long long r = 0;
    for (int q = 0; q < per; ++q) {
        const int d = threadIdx.x * per + q;
        unsigned int t = 0;
#pragma unroll
        for (int sl = 0; sl < SEL_SLOTS; ++sl) t += c->hist[sl][d];
        tot[q] = t;
        r += t;
    }
    // inclusive suffix sum over the threads (runs in ascending bin order)
    unsigned long long incl = r;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long v = __shfl_down(incl, o, 64);
        if (lane + o < 64) incl += v;
    }
    if (lane == 0) wsum[wv] = incl;   // the wavefront's total
    __syncthreads();
    for (int q = wv + 1; q < PICK_THREADS / 64; ++q) incl += wsum[q];
    if (!none) {
        const long long above = (long long)(incl - r);
        if (above < kl && (long long)incl >= kl) {   // exactly one run holds the k_left-th key
            long long cum = above;
            for (int q = per - 1; q >= 0; --q) {
                const long long hd = tot[q];
                if (cum + hd >= kl) {
                    const int d = threadIdx.x * per + q;
                    c->h.prefix |= (unsigned int)d << shift;
                    c->h.mask |= (unsigned int)(nb - 1) << shift;
                    c->h.k_left = kl - cum;
                    break;
                }
                cum += hd;
            }
        }
    }
    for (int sl = 0; sl < SEL_SLOTS; ++sl)
        for (int d = threadIdx.x; d < nb; d += PICK_THREADS) c->hist[sl][d] = 0;
}

// zero the part of a control block that must start at zero (everything but
// the per-node counters, which the scan pass clears for the first N nodes);
// a kernel rather than a memset, so the sequence can be captured in a graph
__global__ __launch_bounds__(SEL_THREADS) void k_sel_clear(SelCtl *c)
{
    unsigned long long *p = (unsigned long long *)c;
    constexpr size_t n = offsetof(SelCtl, node) / sizeof(unsigned long long);
    for (size_t i = blockIdx.x * (size_t)SEL_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * SEL_THREADS)
        p[i] = 0ull;
}

__device__ __forceinline__ bool sel_take(float v, bool none, unsigned int T)
{
    unsigned int key;
    return sel_key(v, key) && !none && key >= T;
}

__device__ __forceinline__ float sel_norm(float v, float m)
{
    if (m > 0.f) return v / m;
    return isfinite(v) ? 0.f : v;
}

// One wavefront per row i of the packed triangle (its edges (i, j), j > i,
// are contiguous): the normalised network and the flags, the selected count,
// and the degrees and strengths of both ends.  The row's own share is summed
// over the wavefront; the partners' shares go straight to their counters.
// A selected edge adds one edge and its |w_norm| in units of 2^-32 (exact
// for |w_norm| >= 2^-9) to one 64-bit counter per end, so the sums do not
// depend on the order of the atomics.
__global__ __launch_bounds__(SEL_THREADS) void k_sel_rows(const float *w, int N, SelCtl *c, float *w_norm,
                                                        unsigned char *selected, int nodes)
{
    __shared__ unsigned long long scnt[SEL_THREADS / 64];
    const int i = blockIdx.x * (SEL_THREADS / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // the selection state is read once: the byte stores below may alias it
    const unsigned int T = c->h.prefix;
    const float m = __uint_as_float(c->h.maxbits);
    const bool none = c->h.none;
    unsigned long long ns = 0;
    if (i < N - 1) {
        const long long r0 = (long long)i * (2LL * N - i - 1) / 2 - (i + 1);   // e = r0 + j
        int deg = 0;
        double str = 0.0;
        // eight loads in flight per lane (the edges are visited in the same order)
        for (int j0 = i + 1 + lane; j0 < N; j0 += 8 * 64) {
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + 64 * q;
                v[q] = j < N ? w[r0 + j] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = j0 + 64 * q;
                if (j >= N) break;
                const long long e = r0 + j;
                const bool t = sel_take(v[q], none, T);
                const float nv = sel_norm(v[q], m);
                if (selected) selected[e] = t;
                if (w_norm) w_norm[e] = nv;
                if (t) {
                    ++ns;
                    if (nodes) {
                        ++deg;
                        const float a = fabsf(nv);
                        str += (double)a;
                        atomicAdd(&c->node[j], SEL_DEG1 + (unsigned long long)rint((double)a * SEL_FIX));
                    }
                }
            }
        }
        if (nodes) {
            for (int o = 32; o > 0; o >>= 1) {
                deg += __shfl_xor(deg, o);
                str += __shfl_xor(str, o);
            }
            if (lane == 0 && deg)
                atomicAdd(&c->node[i], SEL_DEG1 * (unsigned long long)deg + (unsigned long long)rint(str * SEL_FIX));
        }
    }
    for (int o = 32; o > 0; o >>= 1) ns += (unsigned long long)__shfl_xor((long long)ns, o);
    if (lane == 0) scnt[threadIdx.x >> 6] = ns;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < SEL_THREADS / 64; ++q) ns += scnt[q];
        if (ns) atomicAdd(&c->h.slot_ns[blockIdx.x % SEL_SLOTS], ns);
    }
}

__global__ __launch_bounds__(SEL_THREADS) void k_sel_node_out(const SelCtl *c, int N, int *degree, float *strength)
{
    const int i = blockIdx.x * SEL_THREADS + threadIdx.x;
    if (i >= N) return;
    const unsigned long long v = c->node[i];
    if (degree) degree[i] = (int)(v >> 48);
    if (strength) strength[i] = (float)((double)(v & (SEL_DEG1 - 1)) / SEL_FIX);
}

}  // namespace fcx

using namespace fcx;

namespace {
// One control block per device, allocated on first use and kept; calls on a
// device are serialised on it.
std::mutex g_sel_mu;
std::unordered_map<int, SelCtl *> g_sel_ctl;

// The allocation-free variant's control block: one file-scope device array
// (each device holds its own copy until the process ends).  In host code the
// name is only a stand-in; the device address comes from hipGetSymbolAddress
// on the device's first call and is kept per device.
static_assert(offsetof(SelCtl, node) % sizeof(unsigned long long) == 0, "control block layout");
constexpr int SEL_NOALLOC_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[sizeof(SelCtl)];
std::mutex g_na_mu;
SelCtl *g_na_ptr[SEL_NOALLOC_DEVICES];

fcx_status sel_check(int32_t n_nodes, const float *w, double fraction)
{
    if (n_nodes < 2 || n_nodes > SEL_MAX_NODES || !w || !(fraction >= 0.0 && fraction <= 1.0)) return FCX_E_INVAL;
    return FCX_OK;
}

// Enqueue the selection on st with control block c; with info non-NULL, read
// the head back (waits for the stream).
fcx_status sel_run(SelCtl *c, int32_t n_nodes, const float *w, double fraction, float *w_norm, uint8_t *selected,
                   int32_t *degree, float *strength, fcx_select_info *info, hipStream_t st)
{
    const long long P = (long long)n_nodes * (n_nodes - 1) / 2;
    const bool vec = ((uintptr_t)w & 15) == 0;   // float4 loads in the scan and histogram passes
    long long blocks = ((vec ? P / 4 : P) + SEL_THREADS - 1) / SEL_THREADS;
    if (blocks > SEL_MAX_BLOCKS) blocks = SEL_MAX_BLOCKS;
    if (blocks < 1) blocks = 1;
    const dim3 grid((unsigned)blocks), blk(SEL_THREADS);
    hipLaunchKernelGGL(k_sel_clear, dim3(64), blk, 0, st, c);
    if (vec)
        hipLaunchKernelGGL(k_sel_scan<true>, grid, blk, 0, st, w, P, (int)n_nodes, c);
    else
        hipLaunchKernelGGL(k_sel_scan<false>, grid, blk, 0, st, w, P, (int)n_nodes, c);
    // digits of 11, 10 and 10 bits (bits 30..20, 19..10, 9..0); the scan
    // took the first digit's histogram, and the first pick also sets up k
    const int shifts[3] = {20, 10, 0}, bins[3] = {2048, 1024, 1024};
    for (int pass = 0; pass < 3; ++pass) {
        if (pass > 0) {
            if (vec)
                hipLaunchKernelGGL(k_sel_hist<true>, grid, blk, 0, st, w, P, c, shifts[pass], bins[pass]);
            else
                hipLaunchKernelGGL(k_sel_hist<false>, grid, blk, 0, st, w, P, c, shifts[pass], bins[pass]);
        }
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(PICK_THREADS), 0, st, c, shifts[pass], bins[pass],
                           pass == 0 ? (int)blocks : 0, fraction, P);
    }
    // last: w_norm may overwrite w
    const int nodes = degree || strength;
    hipLaunchKernelGGL(k_sel_rows, dim3((n_nodes + 3) / 4), blk, 0, st, w, n_nodes, c, w_norm, selected, nodes);
    if (nodes)
        hipLaunchKernelGGL(k_sel_node_out, dim3((n_nodes + SEL_THREADS - 1) / SEL_THREADS), blk, 0, st, c, n_nodes,
                           degree, strength);
    if (hipGetLastError() != hipSuccess) return FCX_E_DEVICE;
    if (!info) return FCX_OK;
    SelHead h{};
    if (hipMemcpyAsync(&h, &c->h, sizeof(SelHead), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return FCX_E_DEVICE;
    float mx, th;
    memcpy(&mx, &h.maxbits, sizeof(float));
    memcpy(&th, &h.prefix, sizeof(float));
    unsigned long long ns = 0;
    for (int q = 0; q < SEL_SLOTS; ++q) ns += h.slot_ns[q];
    info->max_abs = mx;
    info->threshold = h.none ? INFINITY : th;
    info->k = h.k;
    info->n_finite = (int64_t)h.n_finite;
    info->n_selected = (int64_t)ns;
    return FCX_OK;
}
}  // namespace

extern "C" fcx_status fcx_network_select(int32_t n_nodes, const float *w, double fraction, float *w_norm,
                                         uint8_t *selected, int32_t *degree, float *strength,
                                         fcx_select_info *info, void *hip_stream)
{
    fcx_status rc = sel_check(n_nodes, w, fraction);
    if (rc != FCX_OK) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FCX_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_sel_mu);
    SelCtl *&c = g_sel_ctl[dev];
    if (!c && hipMalloc((void **)&c, sizeof(SelCtl)) != hipSuccess) {
        c = nullptr;
        return FCX_E_NOMEM;
    }
    // this entry point always reports back (info may still be NULL)
    fcx_select_info tmp;
    return sel_run(c, n_nodes, w, fraction, w_norm, selected, degree, strength, info ? info : &tmp,
                   (hipStream_t)hip_stream);
}

extern "C" fcx_status fcx_network_select_noalloc(int32_t n_nodes, const float *w, double fraction, float *w_norm,
                                                 uint8_t *selected, int32_t *degree, float *strength,
                                                 fcx_select_info *info, void *hip_stream)
{
    fcx_status rc = sel_check(n_nodes, w, fraction);
    if (rc != FCX_OK) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FCX_E_DEVICE;
    if (dev < 0 || dev >= SEL_NOALLOC_DEVICES) return FCX_E_INVAL;
    SelCtl *c = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_na_mu);
        if (!g_na_ptr[dev]) {
            // first call on this device (current): the device address of its copy
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FCX_E_DEVICE;
            g_na_ptr[dev] = (SelCtl *)p;
        }
        c = g_na_ptr[dev];
    }
    return sel_run(c, n_nodes, w, fraction, w_norm, selected, degree, strength, info, (hipStream_t)hip_stream);
}
