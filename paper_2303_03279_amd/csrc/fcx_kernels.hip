// HIP kernels of the sliding-window connectivity update for gfx950.
//
// One push of a trial runs, in stream order:
//   k_spectra      taper x band-limited DFT of every node into the ring slot of
//                  the new trial (the per-trial spectrum of the CSD/PSD eqs.),
//                  flags non-finite input
//   k_znorm        z-scored samples of the trial into the COR sample ring
//   k_psd          running per-node power sums: + new trial, - evicted trial
//   k_pair_update  per pair tile: the per-trial Pearson r of the new and the
//                  evicted trial as 16x16x4 FP32 MFMA Gram blocks into the COR
//                  running sum; then per bin the running sums of CSD, unit
//                  phasors, sign(Im), |Im| and Im^2 (+ new, - evicted), the
//                  seven spectral metrics and their band mean (the hot kernel)
//   k_commit       accept the trial (or count the rejection)
//
// Nothing is reordered across trials: an evicted trial's contribution is
// recomputed from the cached spectra with exactly the instructions that added
// it, so add and remove cancel bit for bit before the FP64 rounding of the
// running sum itself.
#include "fcx_device.h"

#include <math.h>

#pragma clang fp contract(off)

namespace fcx {

// ---------------------------------------------------------------------------
// spectra: X[b][l][i] = sum_n (w_l[n] e^{-2 pi i k_b n / F}) x_i[n]
// A workgroup owns 16 nodes and 16 (taper, bin) outputs per node; samples are
// staged through LDS 256 at a time and summed in blocks of 256 (four
// interleaved chains per block, block sums added to the total) to keep the
// FP32 rounding growth small.
// ---------------------------------------------------------------------------
constexpr int SP_NODES = 16;
constexpr int SP_CH = 256;

template <typename T>
__device__ __forceinline__ void spectra_body(const SessDev<T> &s, int bx, int by, T (*xs)[SP_CH + 1], int slot)
{
    const int t = threadIdx.x;
    const int node0 = bx * SP_NODES;
    const int nl = t & (SP_NODES - 1);
    const int bl = by * (256 / SP_NODES) + (t / SP_NODES);   // l * B + b
    const int BL = s.B * s.L;
    const bool active = bl < BL && node0 + nl < s.N;
    const T *x = (const T *)s.x;
    const T *tw = s.wtw + (size_t)(active ? bl : 0) * s.M * 2;
    T acc_re = 0, acc_im = 0;
    int bad = 0;
    for (int n0 = 0; n0 < s.M; n0 += SP_CH) {
        for (int e = t; e < SP_NODES * SP_CH; e += 256) {
            const int r = e / SP_CH, c = e % SP_CH;
            const int node = node0 + r, n = n0 + c;
            T v = 0;
            if (node < s.N && n < s.M) {
                v = x[(size_t)node * s.ldx + n];
                if (!finite_v(v)) bad = 1;
            }
            xs[r][c] = v;
        }
        __syncthreads();
        if (active) {
            // four independent chains over samples c = 4q + r, joined at the
            // end of the block
            const int nmax = min(SP_CH, s.M - n0);
            T pr[4] = {0, 0, 0, 0}, pi[4] = {0, 0, 0, 0};
            int c = 0;
#pragma unroll 4
            for (; c + 4 <= nmax; c += 4) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const T xv = xs[nl][c + r];
                    pr[r] = fma(xv, tw[2 * (n0 + c + r)], pr[r]);
                    pi[r] = fma(xv, tw[2 * (n0 + c + r) + 1], pi[r]);
                }
            }
            for (int r = 0; c < nmax; ++c, ++r) {
                const T xv = xs[nl][c];
                pr[r] = fma(xv, tw[2 * (n0 + c)], pr[r]);
                pi[r] = fma(xv, tw[2 * (n0 + c) + 1], pi[r]);
            }
            acc_re += (pr[0] + pr[1]) + (pr[2] + pr[3]);
            acc_im += (pi[0] + pi[1]) + (pi[2] + pi[3]);
        }
        __syncthreads();
    }
    if (bad) s.ctl->bad = 1;
    if (active) {
        const int l = bl / s.B, b = bl % s.B;
        const size_t o = (((size_t)slot * s.B + b) * s.L + l) * s.N + node0 + nl;
        typedef typename V2<T>::t T2;
        T2 v;
        v.x = acc_re;
        v.y = acc_im;
        ((T2 *)s.ring)[o] = v;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_spectra(SessDev<T> s)
{
    __shared__ T xs[SP_NODES][SP_CH + 1];
    spectra_body(s, blockIdx.x, blockIdx.y, xs, (int)(s.ctl->pushed % (long long)s.R));
}

// a batch of trials resident on the device: trial blockIdx.z (at x + z * stride
// elements) into ring slot z
template <typename T>
__global__ __launch_bounds__(256) void k_spectra_batch(SessDev<T> s, long long stride)
{
    __shared__ T xs[SP_NODES][SP_CH + 1];
    SessDev<T> d = s;
    d.x = (const T *)s.x + (size_t)blockIdx.z * stride;
    spectra_body(d, blockIdx.x, blockIdx.y, xs, (int)blockIdx.z);
}

template <typename T> hipError_t launch_spectra(const SessDev<T> &s, hipStream_t st)
{
    dim3 grid((s.N + SP_NODES - 1) / SP_NODES, (s.B * s.L + 15) / 16);
    hipLaunchKernelGGL(k_spectra<T>, grid, dim3(256), 0, st, s);
    return hipGetLastError();
}

template <typename T> hipError_t launch_spectra_batch(const SessDev<T> &s, int K, long long stride, hipStream_t st)
{
    dim3 grid((s.N + SP_NODES - 1) / SP_NODES, (s.B * s.L + 15) / 16, K);
    hipLaunchKernelGGL(k_spectra_batch<T>, grid, dim3(256), 0, st, s, stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// z-scored samples for COR: z = (x - mean) / ||x - mean|| (0 for a constant
// row), so that the Pearson r of a trial is the plain dot product z_i . z_j.
// One wavefront per node; rows padded with zeros to Mz.
// ---------------------------------------------------------------------------
constexpr int ZN_REG = 16;   // rows of up to 64 * ZN_REG samples are held in registers

template <typename T>
__device__ __forceinline__ void znorm_body(const SessDev<T> &s, int bx, int slot)
{
    const int lane = threadIdx.x & 63;
    const int node = bx * 4 + (threadIdx.x >> 6);
    if (node >= s.N) return;
    const T *xr = (const T *)s.x + (size_t)node * s.ldx;
    float *z = s.zring + ((size_t)slot * s.N + node) * s.Mz;
    double sum = 0.0;
    int bad = 0;
    if (s.M <= 64 * ZN_REG) {
        // the row is read once into registers; the sums run in the same order
        // as the three passes below, so the results are the same
        T v[ZN_REG];
#pragma unroll
        for (int r = 0; r < ZN_REG; ++r) {
            const int n = lane + 64 * r;
            v[r] = n < s.M ? xr[n] : (T)0;
        }
#pragma unroll
        for (int r = 0; r < ZN_REG; ++r)
            if (lane + 64 * r < s.M) {
                if (!finite_v(v[r])) bad = 1;
                sum += (double)v[r];
            }
        if (bad) s.ctl->bad = 1;
        const double mean = wave_sum(sum) / (double)s.M;
        double ss = 0.0;
#pragma unroll
        for (int r = 0; r < ZN_REG; ++r)
            if (lane + 64 * r < s.M) {
                const double d = (double)v[r] - mean;
                ss += d * d;
            }
        ss = wave_sum(ss);
        const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
#pragma unroll
        for (int r = 0; r < ZN_REG; ++r) {
            const int n = lane + 64 * r;
            if (n < s.Mz) z[n] = n < s.M ? (float)(((double)v[r] - mean) * inv) : 0.0f;
        }
        for (int n = lane + 64 * ZN_REG; n < s.Mz; n += 64) z[n] = 0.0f;
        return;
    }
    for (int n = lane; n < s.M; n += 64) {
        const T v = xr[n];
        if (!finite_v(v)) bad = 1;
        sum += (double)v;
    }
    if (bad) s.ctl->bad = 1;
    const double mean = wave_sum(sum) / (double)s.M;
    double ss = 0.0;
    for (int n = lane; n < s.M; n += 64) {
        const double d = (double)xr[n] - mean;
        ss += d * d;
    }
    ss = wave_sum(ss);
    const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    for (int n = lane; n < s.Mz; n += 64) z[n] = n < s.M ? (float)(((double)xr[n] - mean) * inv) : 0.0f;
}

template <typename T>
__global__ __launch_bounds__(256) void k_znorm(SessDev<T> s)
{
    znorm_body(s, blockIdx.x, (int)(s.ctl->pushed % (long long)s.R));
}

template <typename T>
__global__ __launch_bounds__(256) void k_znorm_batch(SessDev<T> s, long long stride)
{
    SessDev<T> d = s;
    d.x = (const T *)s.x + (size_t)blockIdx.y * stride;
    znorm_body(d, blockIdx.x, (int)blockIdx.y);
}

template <typename T> hipError_t launch_znorm(const SessDev<T> &s, hipStream_t st)
{
    hipLaunchKernelGGL(k_znorm<T>, dim3((s.N + 3) / 4), dim3(256), 0, st, s);
    return hipGetLastError();
}

template <typename T> hipError_t launch_znorm_batch(const SessDev<T> &s, int K, long long stride, hipStream_t st)
{
    hipLaunchKernelGGL(k_znorm_batch<T>, dim3((s.N + 3) / 4, K), dim3(256), 0, st, s, stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// running power sums: P[b][i] += PSD_new - PSD_evicted (FP64)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double trial_psd(const SessDev<T> &s, int slot, int b, int i)
{
    typedef typename V2<T>::t T2;
    const T2 *ring = (const T2 *)s.ring;
    double p = 0.0;
    for (int l = 0; l < s.L; ++l) {
        const T2 v = ring[(((size_t)slot * s.B + b) * s.L + l) * s.N + i];
        const double re = v.x, im = v.y;
        p += s.lamw[l] * (re * re + im * im);
    }
    return p;
}

template <typename T>
__device__ __forceinline__ void psd_body(const SessDev<T> &s, int bx)
{
    if (s.ctl->bad) return;
    const int e = bx * 256 + threadIdx.x;
    if (e >= s.B * s.N) return;
    const int b = e / s.N, i = e % s.N;
    double v = s.psd[e];
    for (int t = 0; t < s.nt; ++t) {   // a coalesced group: its trials in order
        const PushView pv = push_view(s, s.ctl->pushed + t);
        v = v + trial_psd(s, pv.slot_new, b, i);
        if (pv.has_old) v = v - trial_psd(s, pv.slot_old, b, i);
    }
    s.psd[e] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_psd(SessDev<T> s)
{
    psd_body(s, blockIdx.x);
}

template <typename T> hipError_t launch_psd(const SessDev<T> &s, hipStream_t st)
{
    hipLaunchKernelGGL(k_psd<T>, dim3((s.B * s.N + 255) / 256), dim3(256), 0, st, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pair update (the hot kernel)
//
// The pair state of a session is stored per 64x64 tile of the upper triangle,
// as planes [tile][bin][row][col].  A workgroup of 256 threads (4 wavefronts)
// owns one 16-row slice of a tile: lane = column j, wavefront w handles rows
// w, w+4, w+8, w+12 of the slice.  For each chunk of bins, the node data of
// the 16 row and 64 column nodes (new and evicted spectra, unit phasors,
// 1/sqrt(P)) are staged in LDS; the running sums stream from HBM once per
// push (the next bin's sums are loaded while the current bin is computed),
// are updated, written back, and the per-bin metrics are accumulated into the
// band mean, written once per pair.  Several slices share a CU, so one slice's
// MFMA (COR) phase overlaps the others' streaming.
//
// Storage of the running sums: CSD (re, im), |Im| and Im^2 sums in FP64; the
// unit-phasor sums of FP32 sessions in 32-bit fixed point with 2^-k resolution
// (u_fixed), so that adding and later removing a trial's phasor cancels
// exactly; sign sums in int8 when W <= 127, else int16.
// ---------------------------------------------------------------------------
// LDS per staged node and bin: new and evicted spectra (all tapers), their
// unit phasors (single taper with PLV) and 1/sqrt(P) (COH, IMCOH)
__host__ __device__ int pair_node_bytes(int L, int elem_bytes, uint32_t metrics)
{
    return 2 * L * 2 * elem_bytes + ((L == 1 && (metrics & M_PLV)) ? 2 * 2 * elem_bytes : 0) +
           ((metrics & (M_COH | M_IMCOH)) ? 8 : 0);
}

__host__ __device__ int pair_chunk_bins(int B, int L, int elem_bytes, uint32_t metrics)
{
    int cb = PAIR_LDS_BYTES / (PAIR_NODES * pair_node_bytes(L, elem_bytes, metrics));
    if (cb < 1) cb = 1;
    return cb < B ? cb : B;
}

__host__ __device__ size_t pair_lds_bytes(int CB, int L, int elem_bytes, uint32_t metrics)
{
    return (size_t)CB * PAIR_NODES * pair_node_bytes(L, elem_bytes, metrics);
}

// COR part of a slice: r_ij(trial) = z_i . z_j for the new and the evicted
// trial as v_mfma_f32_16x16x4f32 blocks.  Wavefront w owns the 16x16 block of
// the slice's rows and columns 16w..16w+15 of the tile.  Lane l feeds row
// (l & 15) of its block with the 4 consecutive samples 4*(l >> 4) .. +3 of
// each 16-sample step (one float4 load; the same sample permutation on both
// operands leaves every dot product unchanged).  The operands of the next
// COR_DEPTH steps are in flight while a step's MFMAs issue, so the chain of
// dependent L2 round trips is COR_DEPTH times shorter than the step count.
// The new and the evicted trial are contracted separately so the evicted r is
// bit-identical to the r added.
#ifndef FCX_COR_DEPTH
#define FCX_COR_DEPTH 2
#endif
constexpr int COR_DEPTH = FCX_COR_DEPTH;

// one trial's r block of a 16x16 COR block: the MFMA chain of cor_block over
// the z-scored samples (steps in order, components x, y, z, w), so the
// result is the bits cor_block adds for that trial
template <typename T>
__device__ __forceinline__ floatx4 cor_chain(const SessDev<T> &s, int slot, int row, int col, int lg, int steps)
{
    const int N = s.N, Mz = s.Mz;
    const float4 *rn = (const float4 *)(s.zring + ((size_t)slot * N + row) * Mz) + lg;
    const float4 *cn = (const float4 *)(s.zring + ((size_t)slot * N + col) * Mz) + lg;
    floatx4 an = {0.f, 0.f, 0.f, 0.f};
    float4 a[COR_DEPTH], b[COR_DEPTH];
#pragma unroll
    for (int d = 0; d < COR_DEPTH; ++d) {
        const int o = 4 * min(d, steps - 1);
        a[d] = rn[o];
        b[d] = cn[o];
    }
    for (int st = 0; st < steps; st += COR_DEPTH) {
#pragma unroll
        for (int d = 0; d < COR_DEPTH; ++d) {
            if (st + d >= steps) break;
            const float4 x = a[d], y = b[d];
            const int o = 4 * min(st + d + COR_DEPTH, steps - 1);
            a[d] = rn[o];
            b[d] = cn[o];
            an = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.x, an, 0, 0, 0);
            an = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, y.y, an, 0, 0, 0);
            an = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, y.z, an, 0, 0, 0);
            an = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, y.w, an, 0, 0, 0);
        }
    }
    return an;
}


template <typename T>
__device__ __forceinline__ void cor_block(const SessDev<T> &s, const PushView &pv, int tile, int sub, int J0,
                                          int R0, int w)
{
    const int N = s.N, Mz = s.Mz;
    const int C0 = J0 + 16 * w;
    if (R0 >= N || C0 >= N || R0 >= C0 + 15) return;   // no pair i < j < N in this block
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int row = R0 + lr, col = C0 + lr;
    const bool rv = row < N, cv = col < N, old = pv.has_old;
    const float4 *rn = (const float4 *)(s.zring + ((size_t)pv.slot_new * N + (rv ? row : 0)) * Mz) + lg;
    const float4 *cn = (const float4 *)(s.zring + ((size_t)pv.slot_new * N + (cv ? col : 0)) * Mz) + lg;
    const float4 *ro = (const float4 *)(s.zring + ((size_t)pv.slot_old * N + (rv ? row : 0)) * Mz) + lg;
    const float4 *co = (const float4 *)(s.zring + ((size_t)pv.slot_old * N + (cv ? col : 0)) * Mz) + lg;
    floatx4 an = {0.f, 0.f, 0.f, 0.f}, ao = {0.f, 0.f, 0.f, 0.f};
    const int steps = Mz / 16;
    // Loads are unconditional: a lane past N reads row 0 of the slot (its
    // pointer is clamped above), which only feeds output rows / columns that
    // are never stored, and a step past the end re-reads the last step.
    float4 a[COR_DEPTH], b[COR_DEPTH], a2[COR_DEPTH] = {}, b2[COR_DEPTH] = {};   // slot d: step st + d
    auto fetch = [&](int d, int stp) {
        const int o = 4 * min(stp, steps - 1);
        a[d] = rn[o];
        b[d] = cn[o];
        if (old) {
            a2[d] = ro[o];
            b2[d] = co[o];
        }
    };
#pragma unroll
    for (int d = 0; d < COR_DEPTH; ++d) fetch(d, d);
    for (int st = 0; st < steps; st += COR_DEPTH) {
#pragma unroll
        for (int d = 0; d < COR_DEPTH; ++d) {
            if (st + d >= steps) break;
            const float4 x = a[d], y = b[d], x2 = a2[d], y2 = b2[d];
            fetch(d, st + d + COR_DEPTH);   // refill the slot with the step COR_DEPTH ahead
            an = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.x, an, 0, 0, 0);
            an = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, y.y, an, 0, 0, 0);
            an = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, y.z, an, 0, 0, 0);
            an = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, y.w, an, 0, 0, 0);
            if (old) {
                ao = __builtin_amdgcn_mfma_f32_16x16x4f32(x2.x, y2.x, ao, 0, 0, 0);
                ao = __builtin_amdgcn_mfma_f32_16x16x4f32(x2.y, y2.y, ao, 0, 0, 0);
                ao = __builtin_amdgcn_mfma_f32_16x16x4f32(x2.z, y2.z, ao, 0, 0, 0);
                ao = __builtin_amdgcn_mfma_f32_16x16x4f32(x2.w, y2.w, ao, 0, 0, 0);
            }
        }
    }
    const size_t P = (size_t)N * (N - 1) / 2;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // accumulator element k of lane l: row 4*(l>>4)+k, column l&15
        const int ri = 16 * sub + 4 * lg + k, cj = 16 * w + lr;
        const int i = R0 + 4 * lg + k, j = C0 + lr;
        if (!(i < j && j < N)) continue;
        const size_t e = (size_t)tile * TILE_PAIRS + (size_t)ri * TILE + cj;
        double R = s.rsum[e] + (double)an[k];
        if (old) R = R - (double)ao[k];
        s.rsum[e] = R;
        const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
        s.out[7 * P + idx] = (T)(R / (double)pv.K);
    }
}

// Bins of a pair whose running-sum loads are issued together (1: the next
// bin's loads are in flight while the current bin is computed).  Measured
// best per variant on the 5000-node and 10000-node pushes: 8 for a single
// taper without COR, 6 with COR (its operand ring takes registers), 4 for
// multitaper sums, 2 for FP64 sessions.  FCX_BIN_GROUP overrides all.
template <typename T, int LT, int COR> constexpr int bin_group()
{
#ifdef FCX_BIN_GROUP
    return FCX_BIN_GROUP;
#else
    return sizeof(T) == 8 ? 2 : (LT != 1 ? 4 : (COR ? 6 : 8));
#endif
}

// running sums of one (pair, bin) as held in the planes
struct PairState {
    double sre, sim, ure, uim, a, q;
    int uqr, uqi, g;
};

// ---- one trial's terms: shared by the sliding update and the rebuild, so
// ---- that a trial removed later cancels the bits it added
//
// Unit phasor X / |X| (0 for X = 0) of a staged spectrum value; the
// magnitude is formed in FP64 so that tiny amplitudes cannot underflow.
template <typename T> __device__ __forceinline__ typename V2<T>::t unit_phasor(typename V2<T>::t x)
{
    typename V2<T>::t u;
    const double m2 = (double)x.x * x.x + (double)x.y * x.y;
    const double r = m2 > 0.0 ? rsqrt(m2) : 0.0;
    u.x = (T)(x.x * r);
    u.y = (T)(x.y * r);
    return u;
}

// The trial's CSD X_i conj(X_j) (taper-combined) of row node r and column
// node c from staged values: taper l of node n at X[l * PAIR_NODES + n] (the
// columns after the SLICE_ROWS rows).  FP32 operands give exact FP64 products.
template <typename T>
__device__ __forceinline__ void trial_csd(const typename V2<T>::t *X, int r, int c, int L, const double *lamw,
                                          double &cr, double &ci)
{
    cr = 0.0;
    ci = 0.0;
    for (int l = 0; l < L; ++l) {
        const typename V2<T>::t a = X[(size_t)l * PAIR_NODES + r], b = X[(size_t)l * PAIR_NODES + SLICE_ROWS + c];
        const double re = (double)a.x * b.x + (double)a.y * b.y;
        const double im = (double)a.y * b.x - (double)a.x * b.y;
        if (L == 1) {
            cr = re;
            ci = im;
        } else {
            cr += lamw[l] * re;
            ci += lamw[l] * im;
        }
    }
}

// The trial's unit-phasor product: single taper from the staged phasors
// U[n] (in the session's precision), several tapers the unit phasor of the
// taper-combined CSD
template <typename T>
__device__ __forceinline__ void trial_uprod(const typename V2<T>::t *U, int r, int c, int L, double cr, double ci,
                                            double &ur, double &ui)
{
    if (L == 1) {
        const typename V2<T>::t a = U[r], b = U[SLICE_ROWS + c];
        const T nr = a.x * b.x + a.y * b.y, ni = a.y * b.x - a.x * b.y;
        ur = nr;
        ui = ni;
    } else {
        const double m2 = cr * cr + ci * ci;
        const double rm = m2 > 0.0 ? rsqrt_t<T>(m2) : 0.0;
        ur = cr * rm;
        ui = ci * rm;
    }
}

// a phasor component as the fixed-point integer of the sums: u * 2^k is exact
// in FP32, so the integer of an evicted trial equals the one it added
__device__ __forceinline__ int ufix_of(double u, float uscale) { return (int)rintf((float)u * uscale); }

// The seven spectral metrics of one (pair, bin) from its sums, added to the
// band sums acc[7] (metric order COH IMCOH PLV PLI WPLI USPLI DSWPLI).
// srij = 1/sqrt(P_i P_j); ur, ui the phasor sums as values.
template <typename T>
__device__ __forceinline__ void bin_metrics(uint32_t mm, const PairState &st, double srij, T ur, T ui, int K,
                                            T (&acc)[7])
{
    const T Kt = (T)K;
    const T invK = (T)(1.0 / (double)K);
    const T invKm1 = K >= 2 ? (T)(1.0 / (double)(K - 1)) : (T)0;
    if (mm & (M_COH | M_IMCOH)) {
        if (mm & M_COH) acc[0] += sqrt_ratio<T>((st.sre * st.sre + st.sim * st.sim) * srij * srij);
        if (mm & M_IMCOH) acc[1] += (T)(st.sim * srij);
    }
    if (mm & M_PLV) acc[2] += sqrt_t<T>(ur * ur + ui * ui) * invK;   // |U| <= K: safe in the session's precision
    if (mm & (M_PLI | M_USPLI)) {
        const T pli = (T)abs(st.g) * invK;
        if (mm & M_PLI) acc[3] += pli;
        if (mm & M_USPLI) acc[5] += K >= 2 ? (Kt * pli * pli - (T)1) * invKm1 : (T)NAN;
    }
    if (mm & M_WPLI) acc[4] += st.a > 0.0 ? ratio_t<T>(fabs(st.sim), st.a) : (T)0;
    if (mm & M_DSWPLI) {
        const double dd = st.a * st.a - st.q;
        acc[6] += K >= 2 ? (dd != 0.0 ? ratio_t<T>(st.sim * st.sim - st.q, dd) : (T)0) : (T)NAN;
    }
}

// SPEC != 0 fixes the spectral metric set at compile time (the branches on
// it fold away); LT != 0 fixes the taper count; COR = 1 / 0 compiles the COR
// part in / out (-1: decided by the session's metric bits).  SPEC = 0, LT = 0,
// COR = -1 is the general kernel.  The COR part runs after the spectral sums.
template <typename T, uint32_t SPEC, int LT, int COR, int UG, bool OLD>
__device__ __forceinline__ void pair_slice_body(const SessDev<T> &s, const PushView &pv, int item, int CB, char *lds)
{
    typedef typename V2<T>::t T2;
    const int tile = item / SLICES, sub = item % SLICES;
    const int tid = threadIdx.x;
    const int c = tid & (TILE - 1);
    const int w = tid >> 6;
    const int2 tt = s.tiles[tile];
    const int I0 = tt.x * TILE, J0 = tt.y * TILE;
    const int R0 = I0 + SLICE_ROWS * sub;
    const int N = s.N, B = s.B, L = LT ? LT : s.L;
    constexpr bool has_old = OLD;
    const int K = pv.K;
    const int slot_new = pv.slot_new, slot_old = pv.slot_old;
    const uint32_t mm = SPEC ? SPEC : (s.metrics & 0x7Fu);   // spectral metrics
    const bool needSre = mm & M_COH;
    const bool needSim = mm & (M_COH | M_IMCOH | M_WPLI | M_DSWPLI);
    const bool needU = mm & M_PLV;
    const bool needG = mm & (M_PLI | M_USPLI);
    const bool needA = mm & (M_WPLI | M_DSWPLI);
    const bool needQ = mm & M_DSWPLI;
    const bool ufix = UG >= 0 ? (UG & 1) != 0 : s.u_fixed != 0;
    const bool g8 = UG >= 0 ? (UG & 2) != 0 : s.g_narrow != 0;
    const float uscale = ldexpf(1.0f, s.ufix_bits);
    const double uinv = ldexp(1.0, -s.ufix_bits);
    const T2 *ring = (const T2 *)s.ring;
    // Per-workgroup buffer resources over this tile of every plane (uniform
    // base, range = the tile); pair slots are addressed by 32-bit byte
    // offsets within the tile, so no per-lane 64-bit address arithmetic.
    const size_t tb = (size_t)tile * B * TILE_PAIRS;
    const int usz = ufix ? 4 : 8, gsz = g8 ? 1 : 2;
    const uint32_t tpairs = (uint32_t)B * TILE_PAIRS;
    // a plane the metric set does not use gets an empty range
    auto plane_rsrc = [&](bool need, void *plane, int esz) {
        return tile_rsrc(need ? (char *)plane + tb * esz : nullptr, need ? tpairs * (uint32_t)esz : 0u);
    };
    const Rsrc rSre = plane_rsrc(needSre, s.plane[P_SRE], 8);
    const Rsrc rSim = plane_rsrc(needSim, s.plane[P_SIM], 8);
    const Rsrc rUre = plane_rsrc(needU, s.plane[P_URE], usz);
    const Rsrc rUim = plane_rsrc(needU, s.plane[P_UIM], usz);
    const Rsrc rA = plane_rsrc(needA, s.plane[P_A], 8);
    const Rsrc rQ = plane_rsrc(needQ, s.plane[P_Q], 8);
    const Rsrc rG = plane_rsrc(needG, s.gsum, gsz);

    const T uinvT = (T)uinv;
    const size_t P = (size_t)N * (N - 1) / 2;

    const bool with_cor = COR > 0 || (COR < 0 && (s.metrics & M_COR));
    if (!mm) {   // COR-only session: no spectral sums
        if (with_cor) cor_block(s, pv, tile, sub, J0, R0, w);
        return;
    }

    // LDS layout as sized by pair_node_bytes
    const bool stageU = L == 1 && needU;
    T2 *Xn = (T2 *)lds;
    T2 *Xo = Xn + (size_t)CB * L * PAIR_NODES;
    T2 *Un = Xo + (size_t)CB * L * PAIR_NODES;
    T2 *Uo = Un + (stageU ? (size_t)CB * PAIR_NODES : 0);
    double *SR = (double *)(Uo + (stageU ? (size_t)CB * PAIR_NODES : 0));

    auto load_state = [&](uint32_t e) {
        PairState st;
        st.sre = needSre ? buf_ld_f64(rSre, e * 8u) : 0.0;
        st.sim = needSim ? buf_ld_f64(rSim, e * 8u) : 0.0;
        st.ure = (needU && !ufix) ? buf_ld_f64(rUre, e * 8u) : 0.0;
        st.uim = (needU && !ufix) ? buf_ld_f64(rUim, e * 8u) : 0.0;
        st.uqr = (needU && ufix) ? buf_ld_i32(rUre, e * 4u) : 0;
        st.uqi = (needU && ufix) ? buf_ld_i32(rUim, e * 4u) : 0;
        st.a = needA ? buf_ld_f64(rA, e * 8u) : 0.0;
        st.q = needQ ? buf_ld_f64(rQ, e * 8u) : 0.0;
        st.g = needG ? (g8 ? buf_ld_i8(rG, e) : buf_ld_i16(rG, e * 2u)) : 0;
        return st;
    };

    int ci = 0;
    for (int b0 = 0; b0 < B; b0 += CB, ++ci) {
        const int nb = min(CB, B - b0);
        const bool last_chunk = b0 + CB >= B;
        // node index nl: 0..15 the slice's rows, 16..79 the tile's columns
        for (int e = tid; e < nb * L * PAIR_NODES; e += PAIR_THREADS) {
            const int nl = e % PAIR_NODES, bl = e / PAIR_NODES;
            const int l = bl % L, bb = bl / L;
            const int node = nl < SLICE_ROWS ? R0 + nl : J0 + nl - SLICE_ROWS;
            T2 xn, xo;
            xn.x = xn.y = xo.x = xo.y = 0;
            if (node < N) {
                xn = ring[(((size_t)slot_new * B + b0 + bb) * L + l) * N + node];
                if (has_old) xo = ring[(((size_t)slot_old * B + b0 + bb) * L + l) * N + node];
            }
            Xn[(size_t)bl * PAIR_NODES + nl] = xn;
            Xo[(size_t)bl * PAIR_NODES + nl] = xo;
            if (stageU) {
                Un[(size_t)bb * PAIR_NODES + nl] = unit_phasor<T>(xn);
                Uo[(size_t)bb * PAIR_NODES + nl] = unit_phasor<T>(xo);
            }
        }
        if (mm & (M_COH | M_IMCOH)) {
            for (int e = tid; e < nb * PAIR_NODES; e += PAIR_THREADS) {
                const int nl = e % PAIR_NODES, bb = e / PAIR_NODES;
                const int node = nl < SLICE_ROWS ? R0 + nl : J0 + nl - SLICE_ROWS;
                double sr = 0.0;
                if (node < N) {
                    const double p = s.psd[(size_t)(b0 + bb) * N + node];
                    sr = p > 0.0 ? rsqrt(p) : 0.0;
                }
                SR[e] = sr;
            }
        }
        __syncthreads();

#pragma unroll 1
        for (int q = 0; q < SLICE_ROWS / 4; ++q) {
            const int r = 4 * q + w;                 // row within the slice
            const int rt = SLICE_ROWS * sub + r;     // row within the tile
            const int i = R0 + r, j = J0 + c;
            if (!(i < j && j < N)) continue;
            const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
            // band sums accumulate in bin order; a later bin chunk resumes the
            // partial sum the previous chunk stored, so the result does not
            // depend on how the band is split into chunks
            T acc[7];
#pragma unroll
            for (int m = 0; m < 7; ++m) acc[m] = (ci > 0 && (mm & (1u << m))) ? s.out[(size_t)m * P + idx] : (T)0;
            const uint32_t e0 = (uint32_t)((b0 * TILE + rt) * TILE + c);   // slot within the tile
            // one bin of the pair: update its running sums from the loaded
            // state, store them, add the bin's metrics to the band sums
            auto bin_step = [&](int bb, PairState st) {
                const uint32_t e = e0 + (uint32_t)bb * TILE_PAIRS;
                double cnr, cni, cor_ = 0.0, coi = 0.0;
                trial_csd<T>(Xn + (size_t)bb * L * PAIR_NODES, r, c, L, s.lamw, cnr, cni);
                if (has_old) trial_csd<T>(Xo + (size_t)bb * L * PAIR_NODES, r, c, L, s.lamw, cor_, coi);
                if (needSre) {
                    st.sre = st.sre + cnr;
                    if (has_old) st.sre = st.sre - cor_;
                    buf_st_f64(rSre, e * 8u, st.sre);
                }
                if (needSim) {
                    st.sim = st.sim + cni;
                    if (has_old) st.sim = st.sim - coi;
                    buf_st_f64(rSim, e * 8u, st.sim);
                }
                if (needU) {
                    double unr, uni, uor = 0.0, uoi = 0.0;
                    trial_uprod<T>(Un + (size_t)bb * PAIR_NODES, r, c, L, cnr, cni, unr, uni);
                    if (has_old) trial_uprod<T>(Uo + (size_t)bb * PAIR_NODES, r, c, L, cor_, coi, uor, uoi);
                    if (ufix) {
                        st.uqr += ufix_of(unr, uscale);
                        st.uqi += ufix_of(uni, uscale);
                        if (has_old) {
                            st.uqr -= ufix_of(uor, uscale);
                            st.uqi -= ufix_of(uoi, uscale);
                        }
                        buf_st_i32(rUre, e * 4u, st.uqr);
                        buf_st_i32(rUim, e * 4u, st.uqi);
                    } else {
                        st.ure = st.ure + unr;
                        st.uim = st.uim + uni;
                        if (has_old) {
                            st.ure = st.ure - uor;
                            st.uim = st.uim - uoi;
                        }
                        buf_st_f64(rUre, e * 8u, st.ure);
                        buf_st_f64(rUim, e * 8u, st.uim);
                    }
                }
                if (needG) {
                    st.g = st.g + sgn_of(cni);
                    if (has_old) st.g -= sgn_of(coi);
                    if (g8)
                        buf_st_i8(rG, e, st.g);
                    else
                        buf_st_i16(rG, e * 2u, st.g);
                }
                if (needA) {
                    st.a = st.a + fabs(cni);
                    if (has_old) st.a = st.a - fabs(coi);
                    buf_st_f64(rA, e * 8u, st.a);
                }
                if (needQ) {
                    st.q = st.q + cni * cni;
                    if (has_old) st.q = st.q - coi * coi;
                    buf_st_f64(rQ, e * 8u, st.q);
                }
                // metrics of this bin, into the band mean
                const double srij = (mm & (M_COH | M_IMCOH))
                                        ? SR[bb * PAIR_NODES + r] * SR[bb * PAIR_NODES + SLICE_ROWS + c] : 0.0;
                const T ur = ufix ? (T)st.uqr * uinvT : (T)st.ure;
                const T ui = ufix ? (T)st.uqi * uinvT : (T)st.uim;
                bin_metrics<T>(mm, st, srij, ur, ui, K, acc);
            };
            constexpr int BIN_GROUP = bin_group<T, LT, COR>();
            if constexpr (BIN_GROUP <= 1) {
                // software pipelining: the next bin's sums are in flight
                // while this bin is computed
                PairState cur = load_state(e0);
                for (int bb = 0; bb < nb; ++bb) {
                    PairState nxt = cur;
                    if (bb + 1 < nb) nxt = load_state(e0 + (uint32_t)(bb + 1) * TILE_PAIRS);
                    bin_step(bb, cur);
                    cur = nxt;
                }
            } else {
                // groups of bins: all loads of a group are issued before its
                // first bin is computed
                for (int g0 = 0; g0 < nb; g0 += BIN_GROUP) {
                    PairState st[BIN_GROUP];
#pragma unroll
                    for (int k = 0; k < BIN_GROUP; ++k)
                        if (g0 + k < nb) st[k] = load_state(e0 + (uint32_t)(g0 + k) * TILE_PAIRS);
#pragma unroll
                    for (int k = 0; k < BIN_GROUP; ++k)
                        if (g0 + k < nb) bin_step(g0 + k, st[k]);
                }
            }
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                if (!(mm & (1u << m))) continue;
                s.out[(size_t)m * P + idx] = last_chunk ? acc[m] / (T)B : acc[m];
            }
        }
        __syncthreads();
    }
    if (with_cor) cor_block(s, pv, tile, sub, J0, R0, w);
}

// One slice of a pair tile: the evicting and the non-evicting push are
// separate compile-time bodies (the choice is uniform across the launch).
template <typename T, uint32_t SPEC, int LT, int COR, int UG>
__device__ __forceinline__ void pair_item(const SessDev<T> &s, int item, long long tp, int CB, char *lds)
{
    const int tile = item / SLICES, sub = item % SLICES;
    const int2 tt = s.tiles[tile];
    const int R0 = tt.x * TILE + SLICE_ROWS * sub, J0 = tt.y * TILE;
    if (R0 >= s.N || R0 >= min(J0 + TILE - 1, s.N - 1)) return;   // no pair i < j < N in this slice
    const PushView pv = push_view(s, tp);
    if (pv.has_old)
        pair_slice_body<T, SPEC, LT, COR, UG, true>(s, pv, item, CB, lds);
    else
        pair_slice_body<T, SPEC, LT, COR, UG, false>(s, pv, item, CB, lds);
}

// ---------------------------------------------------------------------------
// A served session's coalesced group: the s.nt trials queued behind each
// other are applied in one pass over the state, in submission order, with
// the per-trial terms and the add-then-remove order of the single push, so
// the sums equal those of pushing the trials one by one; every state element
// is read and written once per group and the networks are finalised once,
// after the last trial.  Bins are staged in chunks of CB with all nt trials
// (new and evicted spectra, unit phasors).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void cor_block_mt(const SessDev<T> &s, long long tp0, int tile, int sub, int J0, int R0,
                                             int w)
{
    const int N = s.N, Mz = s.Mz;
    const int C0 = J0 + 16 * w;
    if (R0 >= N || C0 >= N || R0 >= C0 + 15) return;   // no pair i < j < N in this block
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    const int row = R0 + lr, col = C0 + lr;
    const int rr = row < N ? row : 0, cc = col < N ? col : 0;
    const int steps = Mz / 16;
    const size_t P = (size_t)N * (N - 1) / 2;
    double R[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int ri = 16 * sub + 4 * lg + k, cj = 16 * w + lr;
        const int i = R0 + 4 * lg + k, j = C0 + lr;
        R[k] = (i < j && j < N) ? s.rsum[(size_t)tile * TILE_PAIRS + (size_t)ri * TILE + cj] : 0.0;
    }
    int K = 0;
    for (int t = 0; t < s.nt; ++t) {
        const PushView pv = push_view(s, tp0 + t);
        const floatx4 an = cor_chain(s, pv.slot_new, rr, cc, lg, steps);
        floatx4 ao = {0.f, 0.f, 0.f, 0.f};
        if (pv.has_old) ao = cor_chain(s, pv.slot_old, rr, cc, lg, steps);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            R[k] = R[k] + (double)an[k];
            if (pv.has_old) R[k] = R[k] - (double)ao[k];
        }
        K = pv.K;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int ri = 16 * sub + 4 * lg + k, cj = 16 * w + lr;
        const int i = R0 + 4 * lg + k, j = C0 + lr;
        if (!(i < j && j < N)) continue;
        s.rsum[(size_t)tile * TILE_PAIRS + (size_t)ri * TILE + cj] = R[k];
        const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
        s.out[7 * P + idx] = (T)(R[k] / (double)K);
    }
}

template <typename T, uint32_t SPEC, int LT, int COR, int UG>
__device__ __forceinline__ void pair_slice_mt(const SessDev<T> &s, long long tp0, int item, int CB, char *lds)
{
    typedef typename V2<T>::t T2;
    const int tile = item / SLICES, sub = item % SLICES;
    const int tid = threadIdx.x, c = tid & (TILE - 1), w = tid >> 6;
    const int2 tt = s.tiles[tile];
    const int J0 = tt.y * TILE, R0 = tt.x * TILE + SLICE_ROWS * sub;
    const int N = s.N, B = s.B, L = LT ? LT : s.L, nt = s.nt;
    const uint32_t mm = SPEC ? SPEC : (s.metrics & 0x7Fu);
    const bool needSre = mm & M_COH;
    const bool needSim = mm & (M_COH | M_IMCOH | M_WPLI | M_DSWPLI);
    const bool needU = mm & M_PLV;
    const bool needG = mm & (M_PLI | M_USPLI);
    const bool needA = mm & (M_WPLI | M_DSWPLI);
    const bool needQ = mm & M_DSWPLI;
    const bool ufix = UG >= 0 ? (UG & 1) != 0 : s.u_fixed != 0;
    const bool g8 = UG >= 0 ? (UG & 2) != 0 : s.g_narrow != 0;
    const float uscale = ldexpf(1.0f, s.ufix_bits);
    const T uinvT = (T)ldexp(1.0, -s.ufix_bits);
    const bool with_cor = COR > 0 || (COR < 0 && (s.metrics & M_COR));
    const bool stageU = L == 1 && needU;
    const T2 *ring = (const T2 *)s.ring;
    const size_t P = (size_t)N * (N - 1) / 2;
    const int K = push_view(s, tp0 + nt - 1).K;
    if (!mm) {
        if (with_cor) cor_block_mt(s, tp0, tile, sub, J0, R0, w);
        return;
    }
    const size_t tb = (size_t)tile * B * TILE_PAIRS;
    const int usz = ufix ? 4 : 8, gsz = g8 ? 1 : 2;
    const uint32_t tpairs = (uint32_t)B * TILE_PAIRS;
    auto plane_rsrc = [&](bool need, void *plane, int esz) {
        return tile_rsrc(need ? (char *)plane + tb * esz : nullptr, need ? tpairs * (uint32_t)esz : 0u);
    };
    const Rsrc rSre = plane_rsrc(needSre, s.plane[P_SRE], 8);
    const Rsrc rSim = plane_rsrc(needSim, s.plane[P_SIM], 8);
    const Rsrc rUre = plane_rsrc(needU, s.plane[P_URE], usz);
    const Rsrc rUim = plane_rsrc(needU, s.plane[P_UIM], usz);
    const Rsrc rA = plane_rsrc(needA, s.plane[P_A], 8);
    const Rsrc rQ = plane_rsrc(needQ, s.plane[P_Q], 8);
    const Rsrc rG = plane_rsrc(needG, s.gsum, gsz);
    // LDS: new and evicted spectra [nt][CB][L][nodes], their unit phasors
    // [nt][CB][nodes], 1/sqrt(P) [CB][nodes]
    T2 *Xn = (T2 *)lds;
    T2 *Xo = Xn + (size_t)nt * CB * L * PAIR_NODES;
    T2 *Un = Xo + (size_t)nt * CB * L * PAIR_NODES;
    T2 *Uo = Un + (stageU ? (size_t)nt * CB * PAIR_NODES : 0);
    double *SR = (double *)(Uo + (stageU ? (size_t)nt * CB * PAIR_NODES : 0));
    int ci = 0;
    for (int b0 = 0; b0 < B; b0 += CB, ++ci) {
        const int nb = min(CB, B - b0);
        const bool last_chunk = b0 + CB >= B;
        const int per = nb * L * PAIR_NODES;
        for (int e = tid; e < nt * per; e += PAIR_THREADS) {
            const int t = e / per, r = e % per;
            const int nl = r % PAIR_NODES, bl = r / PAIR_NODES;
            const int l = bl % L, bb = bl / L;
            const int node = nl < SLICE_ROWS ? R0 + nl : J0 + nl - SLICE_ROWS;
            const PushView pv = push_view(s, tp0 + t);
            T2 xn, xo;
            xn.x = xn.y = xo.x = xo.y = 0;
            if (node < N) {
                xn = ring[(((size_t)pv.slot_new * B + b0 + bb) * L + l) * N + node];
                if (pv.has_old) xo = ring[(((size_t)pv.slot_old * B + b0 + bb) * L + l) * N + node];
            }
            Xn[((size_t)t * nb * L + bl) * PAIR_NODES + nl] = xn;
            Xo[((size_t)t * nb * L + bl) * PAIR_NODES + nl] = xo;
            if (stageU) {
                Un[((size_t)t * nb + bb) * PAIR_NODES + nl] = unit_phasor<T>(xn);
                Uo[((size_t)t * nb + bb) * PAIR_NODES + nl] = unit_phasor<T>(xo);
            }
        }
        if (mm & (M_COH | M_IMCOH)) {
            for (int e = tid; e < nb * PAIR_NODES; e += PAIR_THREADS) {
                const int nl = e % PAIR_NODES, bb = e / PAIR_NODES;
                const int node = nl < SLICE_ROWS ? R0 + nl : J0 + nl - SLICE_ROWS;
                double sr = 0.0;
                if (node < N) {
                    const double p = s.psd[(size_t)(b0 + bb) * N + node];
                    sr = p > 0.0 ? rsqrt(p) : 0.0;
                }
                SR[e] = sr;
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int q = 0; q < SLICE_ROWS / 4; ++q) {
            const int r = 4 * q + w, rt = SLICE_ROWS * sub + r;
            const int i = R0 + r, j = J0 + c;
            if (!(i < j && j < N)) continue;
            const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
            T acc[7];
#pragma unroll
            for (int m = 0; m < 7; ++m) acc[m] = (ci > 0 && (mm & (1u << m))) ? s.out[(size_t)m * P + idx] : (T)0;
            // the state loads of MT_GROUP bins go out together before their
            // trials are applied (their latency overlaps)
            constexpr int MT_GROUP = 4;
            for (int g0 = 0; g0 < nb; g0 += MT_GROUP) {
            PairState sg[MT_GROUP];
#pragma unroll
            for (int k = 0; k < MT_GROUP; ++k) {
                if (g0 + k >= nb) break;
                const uint32_t e = (uint32_t)(((b0 + g0 + k) * TILE + rt) * TILE + c);
                PairState &st = sg[k];
                st.sre = needSre ? buf_ld_f64(rSre, e * 8u) : 0.0;
                st.sim = needSim ? buf_ld_f64(rSim, e * 8u) : 0.0;
                st.ure = (needU && !ufix) ? buf_ld_f64(rUre, e * 8u) : 0.0;
                st.uim = (needU && !ufix) ? buf_ld_f64(rUim, e * 8u) : 0.0;
                st.uqr = (needU && ufix) ? buf_ld_i32(rUre, e * 4u) : 0;
                st.uqi = (needU && ufix) ? buf_ld_i32(rUim, e * 4u) : 0;
                st.a = needA ? buf_ld_f64(rA, e * 8u) : 0.0;
                st.q = needQ ? buf_ld_f64(rQ, e * 8u) : 0.0;
                st.g = needG ? (g8 ? buf_ld_i8(rG, e) : buf_ld_i16(rG, e * 2u)) : 0;
            }
#pragma unroll
            for (int k = 0; k < MT_GROUP; ++k) {
                const int bb = g0 + k;
                if (bb >= nb) break;
                const uint32_t e = (uint32_t)(((b0 + bb) * TILE + rt) * TILE + c);
                PairState &st = sg[k];
                for (int t = 0; t < nt; ++t) {
                    const bool old = push_view(s, tp0 + t).has_old;
                    const size_t xo = ((size_t)t * nb * L + (size_t)bb * L) * PAIR_NODES;
                    const size_t uo = ((size_t)t * nb + bb) * PAIR_NODES;
                    double cnr, cni, cor_ = 0.0, coi = 0.0;
                    trial_csd<T>(Xn + xo, r, c, L, s.lamw, cnr, cni);
                    if (old) trial_csd<T>(Xo + xo, r, c, L, s.lamw, cor_, coi);
                    if (needSre) {
                        st.sre = st.sre + cnr;
                        if (old) st.sre = st.sre - cor_;
                    }
                    if (needSim) {
                        st.sim = st.sim + cni;
                        if (old) st.sim = st.sim - coi;
                    }
                    if (needU) {
                        double unr, uni, uor = 0.0, uoi = 0.0;
                        trial_uprod<T>(Un + uo, r, c, L, cnr, cni, unr, uni);
                        if (old) trial_uprod<T>(Uo + uo, r, c, L, cor_, coi, uor, uoi);
                        if (ufix) {
                            st.uqr += ufix_of(unr, uscale);
                            st.uqi += ufix_of(uni, uscale);
                            if (old) {
                                st.uqr -= ufix_of(uor, uscale);
                                st.uqi -= ufix_of(uoi, uscale);
                            }
                        } else {
                            st.ure = st.ure + unr;
                            st.uim = st.uim + uni;
                            if (old) {
                                st.ure = st.ure - uor;
                                st.uim = st.uim - uoi;
                            }
                        }
                    }
                    if (needG) {
                        st.g = st.g + sgn_of(cni);
                        if (old) st.g -= sgn_of(coi);
                    }
                    if (needA) {
                        st.a = st.a + fabs(cni);
                        if (old) st.a = st.a - fabs(coi);
                    }
                    if (needQ) {
                        st.q = st.q + cni * cni;
                        if (old) st.q = st.q - coi * coi;
                    }
                }
                if (needSre) buf_st_f64(rSre, e * 8u, st.sre);
                if (needSim) buf_st_f64(rSim, e * 8u, st.sim);
                if (needU) {
                    if (ufix) {
                        buf_st_i32(rUre, e * 4u, st.uqr);
                        buf_st_i32(rUim, e * 4u, st.uqi);
                    } else {
                        buf_st_f64(rUre, e * 8u, st.ure);
                        buf_st_f64(rUim, e * 8u, st.uim);
                    }
                }
                if (needG) {
                    if (g8)
                        buf_st_i8(rG, e, st.g);
                    else
                        buf_st_i16(rG, e * 2u, st.g);
                }
                if (needA) buf_st_f64(rA, e * 8u, st.a);
                if (needQ) buf_st_f64(rQ, e * 8u, st.q);
                const double srij = (mm & (M_COH | M_IMCOH))
                                        ? SR[bb * PAIR_NODES + r] * SR[bb * PAIR_NODES + SLICE_ROWS + c] : 0.0;
                const T ur = ufix ? (T)st.uqr * uinvT : (T)st.ure;
                const T ui = ufix ? (T)st.uqi * uinvT : (T)st.uim;
                bin_metrics<T>(mm, st, srij, ur, ui, K, acc);
            }
            }
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                if (!(mm & (1u << m))) continue;
                s.out[(size_t)m * P + idx] = last_chunk ? acc[m] / (T)B : acc[m];
            }
        }
        __syncthreads();
    }
    if (with_cor) cor_block_mt(s, tp0, tile, sub, J0, R0, w);
}

template <typename T, uint32_t SPEC, int LT, int COR, int UG>
__global__ __launch_bounds__(PAIR_THREADS) void k_pair_update(SessDev<T> s, int CB)
{
    extern __shared__ __align__(16) char lds[];
    if (s.ctl->bad) return;
    pair_item<T, SPEC, LT, COR, UG>(s, xcd_item(blockIdx.x, gridDim.x), s.ctl->pushed, CB, lds);
}

// Compile-time variants of the pair update.  An FP32 session maps to one
// class: its metric set (all spectral metrics with one or three tapers, COH
// only, WPLI only, all spectral metrics with any taper count, or any set),
// COR in or out, and its storage widths (fixed-point phasor sums with 8- or
// 16-bit sign sums, or decided at run time).  The single-session launch and
// the batched serving launch use the same class, so a session's result does
// not depend on the path that ran it.
#define FCX_PAIR_SPECS(X) X(0, 0x7Fu, 1) X(1, M_COH, 1) X(2, M_WPLI, 1) X(3, 0x7Fu, 3) X(4, 0x7Fu, 0) X(5, 0u, 0)

template <uint32_t SPEC, int LT, int COR, int UG> struct PairVariant {
    static constexpr uint32_t spec = SPEC;
    static constexpr int lt = LT, cor = COR, ug = UG;
};

int pair_kernel_class(const SessDev<float> &s)
{
    const uint32_t spec = s.metrics & 0x7Fu;
    int si;
    if (s.L == 1 && spec == 0x7Fu)
        si = 0;
    else if (s.L == 1 && spec == M_COH)
        si = 1;
    else if (s.L == 1 && spec == M_WPLI)
        si = 2;
    else if (s.L == 3 && spec == 0x7Fu)
        si = 3;
    else if (spec == 0x7Fu)
        si = 4;
    else
        si = 5;
    const int cor = (s.metrics & M_COR) ? 1 : 0;
    const int ug = (s.u_fixed && s.g_narrow) ? 0 : (s.u_fixed ? 1 : 2);
    return (si * 2 + cor) * 3 + ug;
}

// calls f(PairVariant<...>{}) for class cls; false for an unknown class
template <typename F> static bool dispatch_pair_class(int cls, F &&f)
{
    if (cls < 0 || cls >= PAIR_CLASSES) return false;
    const int ugi = cls % 3, cor = (cls / 3) % 2, si = cls / 6;
#define FCX_UG(SPEC, LT, C)                       \
    if (ugi == 0)                                 \
        f(PairVariant<SPEC, LT, C, 3>{});         \
    else if (ugi == 1)                            \
        f(PairVariant<SPEC, LT, C, 1>{});         \
    else                                          \
        f(PairVariant<SPEC, LT, C, -1>{});
#define FCX_SPEC(I, SPEC, LT)   \
    if (si == I) {              \
        if (cor) {              \
            FCX_UG(SPEC, LT, 1) \
        } else {                \
            FCX_UG(SPEC, LT, 0) \
        }                       \
        return true;            \
    }
    FCX_PAIR_SPECS(FCX_SPEC)
#undef FCX_SPEC
#undef FCX_UG
    return false;
}

template <typename T> hipError_t launch_pair_update(const SessDev<T> &s, hipStream_t st)
{
    const uint32_t spec = s.metrics & 0x7Fu;
    const int CB = pair_chunk_bins(s.B, s.L, (int)sizeof(T), spec);
    const size_t lds = spec ? pair_lds_bytes(CB, s.L, (int)sizeof(T), spec) : 0;
    const dim3 grid(s.ntiles * SLICES), blk(PAIR_THREADS);
    if constexpr (sizeof(T) == 4) {
        dispatch_pair_class(pair_kernel_class(s), [&](auto v) {
            using V = decltype(v);
            hipLaunchKernelGGL((k_pair_update<float, V::spec, V::lt, V::cor, V::ug>), grid, blk, lds, st, s, CB);
        });
    } else {
        // FP64 sessions: the general kernel, COR in or out
        if (s.metrics & M_COR)
            hipLaunchKernelGGL((k_pair_update<T, 0u, 0, 1, -1>), grid, blk, lds, st, s, CB);
        else
            hipLaunchKernelGGL((k_pair_update<T, 0u, 0, 0, -1>), grid, blk, lds, st, s, CB);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// rebuild: every running sum of the window recomputed from the cached trials
// in one pass (after a batch pass, or on request), instead of replaying the
// window push by push.  Per (pair, bin) the K cached trials are added oldest
// first with the same per-trial terms as the sliding update (trial_csd,
// trial_uprod, ufix_of, the same FP64 additions), so the sums are bit for bit
// those a replay from zero gives, and a trial evicted later cancels exactly
// what it added.  Each state element is written once; the trials' spectra
// stream through LDS TT at a time, one bin after the other.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_psd_rebuild(SessDev<T> s, long long first, int K)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= s.B * s.N) return;
    const int b = e / s.N, i = e % s.N;
    double v = 0.0;
    for (int t = 0; t < K; ++t) v = v + trial_psd(s, (int)((first + t) % (long long)s.R), b, i);
    s.psd[e] = v;
}

template <typename T> hipError_t launch_psd_rebuild(const SessDev<T> &s, long long first, int K, hipStream_t st)
{
    hipLaunchKernelGGL(k_psd_rebuild<T>, dim3((s.B * s.N + 255) / 256), dim3(256), 0, st, s, first, K);
    return hipGetLastError();
}

// the COR sums of a whole 64x64 tile rebuilt from the window's cached
// z-scored samples: per 16x16 block and trial the same MFMA chain as the
// sliding update (cor_chain: steps in order, components x, y, z, w, the same
// lane layout), each trial's block added to the FP64 sums in trial order, so
// the sums are bit for bit those of a replay.  The tile's 64 row nodes are
// staged in LDS CRB_CH samples at a time (the next chunk loaded into
// registers meanwhile); wavefront w reads its 16 column nodes once per step,
// two steps ahead, for the tile's four row blocks, whose four chains run side
// by side.  Each trial's samples are read once per tile instead of once per
// 16x16 block.
constexpr int CRB_CH = 128;             // samples per staged chunk
constexpr int CRB_LD = CRB_CH + 4;     // LDS row stride in floats

template <typename T>
__global__ __launch_bounds__(256) void k_cor_rebuild(SessDev<T> s, long long first, int K)
{
    __shared__ __align__(16) float Zr[TILE * CRB_LD];
    const int tile = xcd_item(blockIdx.x, gridDim.x);
    const int2 tt = s.tiles[tile];
    const int N = s.N, Mz = s.Mz;
    const int R0 = tt.x * TILE, J0 = tt.y * TILE;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
    const int C0 = J0 + 16 * w, col = C0 + lr;
    // row block b (tile rows 16b..16b+15) holds a pair i < j < N with these columns
    bool act[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int Rb = R0 + 16 * b;
        act[b] = !(Rb >= N || C0 >= N || Rb >= C0 + 15);
    }
    double R[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int k = 0; k < 4; ++k) R[b][k] = 0.0;
    // the (trial, chunk) sequence; the next chunk's rows are loaded into
    // registers while the current one is contracted, and a chunk's column
    // values are loaded before its rows are stored
    const int nch = (Mz + CRB_CH - 1) / CRB_CH, total = K * nch;
    // thread tid stages float4 q = tid mod QPR of rows tid / QPR + u RPR
    // (u < RPT); float4s past the row's Mz samples are 0
    constexpr int QPR = CRB_CH / 4, RPR = 256 / QPR, RPT = TILE / RPR;
    const int sq = tid % QPR, sr = tid / QPR;
    auto zslot = [&](int t) { return s.zring + (size_t)((first + t) % (long long)s.R) * N * Mz; };
    auto load_rows = [&](int ix, float4 (&v)[RPT]) {
        const int t = ix / nch, c0 = (ix - t * nch) * CRB_CH;
        const bool ok = ix < total && c0 + 4 * sq < Mz;
        const float *zs = zslot(ok ? t : 0) + c0 + 4 * sq;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int g = R0 + sr + RPR * u;
            v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (ok && g < N) v[u] = *(const float4 *)(zs + (size_t)g * Mz);
        }
    };
    float4 rows[RPT];
    load_rows(0, rows);
    floatx4 an[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) an[b] = (floatx4){0.f, 0.f, 0.f, 0.f};
    for (int ix = 0; ix < total; ++ix) {
        const int t = ix / nch, ci = ix - t * nch, c0 = ci * CRB_CH, nq = min(CRB_CH, Mz - c0) / 4;
        // a lane past N reads column 0, which only feeds columns never stored
        const float4 *cn = (const float4 *)(zslot(t) + (size_t)(col < N ? col : 0) * Mz + c0) + lg;
        const int ns = nq / 4;   // 16-sample steps in this chunk
        // the column values two steps ahead are in flight while a step's MFMAs issue
        float4 y0 = cn[0], y1 = cn[4 * min(1, ns - 1)];
        __syncthreads();   // the previous chunk's readers are done
#pragma unroll
        for (int u = 0; u < RPT; ++u) *(float4 *)(Zr + (sr + RPR * u) * CRB_LD + 4 * sq) = rows[u];
        __syncthreads();
        load_rows(ix + 1, rows);
        for (int st = 0; st < ns; ++st) {
            const float4 y = y0, y2 = cn[4 * min(st + 2, ns - 1)];
            y0 = y1;
            y1 = y2;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (!act[b]) continue;
                const float4 x = *(const float4 *)(Zr + (16 * b + lr) * CRB_LD + 16 * st + 4 * lg);
                an[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.x, an[b], 0, 0, 0);
                an[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, y.y, an[b], 0, 0, 0);
                an[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, y.z, an[b], 0, 0, 0);
                an[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, y.w, an[b], 0, 0, 0);
            }
        }
        if (ci == nch - 1) {   // the trial's blocks, into the sums in trial order
#pragma unroll
            for (int b = 0; b < 4; ++b) {
#pragma unroll
                for (int k = 0; k < 4; ++k) R[b][k] = R[b][k] + (double)an[b][k];
                an[b] = (floatx4){0.f, 0.f, 0.f, 0.f};
            }
        }
    }
    const size_t P = (size_t)N * (N - 1) / 2;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (!act[b]) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // accumulator element k of lane l: row 4*(l>>4)+k, column l&15 of the block
            const int ri = 16 * b + 4 * lg + k, cj = 16 * w + lr;
            const int i = R0 + ri, j = C0 + lr;
            if (!(i < j && j < N)) continue;
            s.rsum[(size_t)tile * TILE_PAIRS + (size_t)ri * TILE + cj] = R[b][k];
            const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
            s.out[7 * P + idx] = (T)(R[b][k] / (double)K);
        }
    }
}

// LDS of the rebuild: TT trials x L tapers of the 80 staged nodes, their
// unit phasors (single taper with PLV), 1/sqrt(P) of the nodes
__host__ __device__ static int rebuild_trial_bytes(int L, int elem_bytes, uint32_t metrics)
{
    return PAIR_NODES * 2 * elem_bytes * (L + ((L == 1 && (metrics & M_PLV)) ? 1 : 0));
}

template <typename T, uint32_t SPEC, int LT, int COR, int UG>
__global__ __launch_bounds__(PAIR_THREADS) void k_pair_rebuild(SessDev<T> s, long long first, int K, int TT)
{
    extern __shared__ __align__(16) char lds[];
    typedef typename V2<T>::t T2;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int tile = item / SLICES, sub = item % SLICES;
    const int2 tt2 = s.tiles[tile];
    const int N = s.N, B = s.B, L = LT ? LT : s.L;
    const int J0 = tt2.y * TILE, R0 = tt2.x * TILE + SLICE_ROWS * sub;
    if (R0 >= N || R0 >= min(J0 + TILE - 1, N - 1)) return;   // no pair i < j < N in this slice
    const int tid = threadIdx.x, c = tid & (TILE - 1), w = tid >> 6;
    const uint32_t mm = SPEC ? SPEC : (s.metrics & 0x7Fu);
    const bool needSre = mm & M_COH;
    const bool needSim = mm & (M_COH | M_IMCOH | M_WPLI | M_DSWPLI);
    const bool needU = mm & M_PLV;
    const bool needG = mm & (M_PLI | M_USPLI);
    const bool needA = mm & (M_WPLI | M_DSWPLI);
    const bool needQ = mm & M_DSWPLI;
    const bool ufix = UG >= 0 ? (UG & 1) != 0 : s.u_fixed != 0;
    const bool g8 = UG >= 0 ? (UG & 2) != 0 : s.g_narrow != 0;
    const float uscale = ldexpf(1.0f, s.ufix_bits);
    const T uinvT = (T)ldexp(1.0, -s.ufix_bits);
    const bool stageU = L == 1 && needU;
    const T2 *ring = (const T2 *)s.ring;
    const size_t P = (size_t)N * (N - 1) / 2;
    if (mm) {
        T2 *X = (T2 *)lds;                                  // [TT][L][PAIR_NODES]
        T2 *U = X + (size_t)TT * L * PAIR_NODES;            // [TT][PAIR_NODES]
        double *SR = (double *)(U + (stageU ? (size_t)TT * PAIR_NODES : 0));
        T acc[4][7];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < 7; ++m) acc[q][m] = (T)0;
        for (int b = 0; b < B; ++b) {
            PairState st[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                st[q].sre = st[q].sim = st[q].ure = st[q].uim = st[q].a = st[q].q = 0.0;
                st[q].uqr = st[q].uqi = st[q].g = 0;
            }
            for (int t0 = 0; t0 < K; t0 += TT) {
                const int nt = min(TT, K - t0);
                __syncthreads();
                for (int e = tid; e < nt * L * PAIR_NODES; e += PAIR_THREADS) {
                    const int nl = e % PAIR_NODES, tl = e / PAIR_NODES;
                    const int l = tl % L, t = tl / L;
                    const int node = nl < SLICE_ROWS ? R0 + nl : J0 + nl - SLICE_ROWS;
                    const long long slot = (first + t0 + t) % (long long)s.R;
                    T2 x;
                    x.x = x.y = 0;
                    if (node < N) x = ring[(((size_t)slot * B + b) * L + l) * N + node];
                    X[(size_t)tl * PAIR_NODES + nl] = x;
                    if (stageU) U[(size_t)t * PAIR_NODES + nl] = unit_phasor<T>(x);
                }
                if (t0 == 0 && (mm & (M_COH | M_IMCOH))) {
                    for (int nl = tid; nl < PAIR_NODES; nl += PAIR_THREADS) {
                        const int node = nl < SLICE_ROWS ? R0 + nl : J0 + nl - SLICE_ROWS;
                        double sr = 0.0;
                        if (node < N) {
                            const double p = s.psd[(size_t)b * N + node];
                            sr = p > 0.0 ? rsqrt(p) : 0.0;
                        }
                        SR[nl] = sr;
                    }
                }
                __syncthreads();
                // trial by trial, the lane's four pairs side by side (each pair's
                // sums still in trial order); pairs outside i < j < N are summed
                // too, from staged values (zeros past N), and never written
                for (int t = 0; t < nt; ++t) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = 4 * q + w;
                        PairState &z = st[q];
                        double cnr, cni;
                        trial_csd<T>(X + (size_t)t * L * PAIR_NODES, r, c, L, s.lamw, cnr, cni);
                        if (needSre) z.sre = z.sre + cnr;
                        if (needSim) z.sim = z.sim + cni;
                        if (needU) {
                            double unr, uni;
                            trial_uprod<T>(U + (size_t)t * PAIR_NODES, r, c, L, cnr, cni, unr, uni);
                            if (ufix) {
                                z.uqr += ufix_of(unr, uscale);
                                z.uqi += ufix_of(uni, uscale);
                            } else {
                                z.ure = z.ure + unr;
                                z.uim = z.uim + uni;
                            }
                        }
                        if (needG) z.g = z.g + sgn_of(cni);
                        if (needA) z.a = z.a + fabs(cni);
                        if (needQ) z.q = z.q + cni * cni;
                    }
                }
            }
            // the bin's sums, written once, and its metrics into the band means
            const size_t tb = ((size_t)tile * B + b) * TILE_PAIRS;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 4 * q + w, i = R0 + r, j = J0 + c;
                if (!(i < j && j < N)) continue;
                const size_t e = tb + (size_t)(SLICE_ROWS * sub + r) * TILE + c;
                const PairState &z = st[q];
                if (needSre) ((double *)s.plane[P_SRE])[e] = z.sre;
                if (needSim) ((double *)s.plane[P_SIM])[e] = z.sim;
                if (needU) {
                    if (ufix) {
                        ((int *)s.plane[P_URE])[e] = z.uqr;
                        ((int *)s.plane[P_UIM])[e] = z.uqi;
                    } else {
                        ((double *)s.plane[P_URE])[e] = z.ure;
                        ((double *)s.plane[P_UIM])[e] = z.uim;
                    }
                }
                if (needG) {
                    if (g8)
                        ((signed char *)s.gsum)[e] = (signed char)z.g;
                    else
                        ((short *)s.gsum)[e] = (short)z.g;
                }
                if (needA) ((double *)s.plane[P_A])[e] = z.a;
                if (needQ) ((double *)s.plane[P_Q])[e] = z.q;
                const double srij = (mm & (M_COH | M_IMCOH)) ? SR[r] * SR[SLICE_ROWS + c] : 0.0;
                const T ur = ufix ? (T)z.uqr * uinvT : (T)z.ure;
                const T ui = ufix ? (T)z.uqi * uinvT : (T)z.uim;
                bin_metrics<T>(mm, z, srij, ur, ui, K, acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 4 * q + w, i = R0 + r, j = J0 + c;
            if (!(i < j && j < N)) continue;
            const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
#pragma unroll
            for (int m = 0; m < 7; ++m)
                if (mm & (1u << m)) s.out[(size_t)m * P + idx] = acc[q][m] / (T)B;
        }
    }
}

template <typename T> hipError_t launch_pair_rebuild(const SessDev<T> &s, long long first, int K, hipStream_t st)
{
    if (K <= 0) return hipSuccess;
    const uint32_t spec = s.metrics & 0x7Fu;
    const int per = rebuild_trial_bytes(s.L, (int)sizeof(T), spec);
    int TT = (PAIR_LDS_BYTES - PAIR_NODES * 8) / per;
    TT = TT < 1 ? 1 : (TT > K ? K : TT);
    const size_t lds = (size_t)TT * per + PAIR_NODES * 8;
    const dim3 grid(s.ntiles * SLICES), blk(PAIR_THREADS);
    if (spec) {
        if constexpr (sizeof(T) == 4) {
            dispatch_pair_class(pair_kernel_class(s), [&](auto v) {
                using V = decltype(v);
                hipLaunchKernelGGL((k_pair_rebuild<float, V::spec, V::lt, V::cor, V::ug>), grid, blk, lds, st, s,
                                   first, K, TT);
            });
        } else {
            hipLaunchKernelGGL((k_pair_rebuild<T, 0u, 0, 0, -1>), grid, blk, lds, st, s, first, K, TT);
        }
    }
    if (s.metrics & M_COR) hipLaunchKernelGGL(k_cor_rebuild<T>, dim3(s.ntiles), dim3(256), 0, st, s, first, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// commit: the only writer of the accepted-trial counter
// ---------------------------------------------------------------------------
__global__ void k_commit(DevCtl *c)
{
    if (threadIdx.x == 0) {
        if (c->bad)
            c->rejected = c->rejected + 1;
        else
            c->pushed = c->pushed + 1;
        c->bad = 0;
    }
}

hipError_t launch_commit(DevCtl *ctl, hipStream_t st)
{
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(64), 0, st, ctl);
    return hipGetLastError();
}

// replay control: point a private DevCtl at one cached trial
__global__ void k_set_ctl(DevCtl *c, long long pushed)
{
    if (threadIdx.x == 0) {
        c->pushed = pushed;
        c->bad = 0;
        c->rejected = 0;
    }
}

hipError_t launch_set_ctl(DevCtl *ctl, long long pushed, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, st, ctl, pushed);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-bin finalisation of one spectral metric from the running sums:
// out[b][P].  One thread per (tile, bin, pair slot).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_finalize_bins(SessDev<T> s, uint32_t metric, T *out)
{
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t total = (size_t)s.ntiles * s.B * TILE_PAIRS;
    if (e >= total) return;
    const int c = (int)(e % TILE), r = (int)((e / TILE) % TILE);
    const int b = (int)((e / TILE_PAIRS) % s.B);
    const int tile = (int)(e / ((size_t)TILE_PAIRS * s.B));
    const int2 tt = s.tiles[tile];
    const int N = s.N;
    const int i = tt.x * TILE + r, j = tt.y * TILE + c;
    if (!(i < j && j < N)) return;
    const long long tp = s.ctl->pushed;
    const int K = tp >= s.W ? s.W : (int)tp;
    const double Kd = (double)K;
    const size_t P = (size_t)N * (N - 1) / 2;
    const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(j - i - 1);
    const double pi_ = s.psd[(size_t)b * N + i], pj_ = s.psd[(size_t)b * N + j];
    const double den = sqrt(pi_ * pj_);
    const double *pl[NPLANES];
    for (int k = 0; k < NPLANES; ++k) pl[k] = (const double *)s.plane[k];
    auto usum = [&](int k) {
        return s.u_fixed ? (double)((const int *)s.plane[k])[e] * ldexp(1.0, -s.ufix_bits) : pl[k][e];
    };
    auto gsum = [&]() {
        return s.g_narrow ? (double)((const signed char *)s.gsum)[e] : (double)((const short *)s.gsum)[e];
    };
    double v = 0.0;
    switch (metric) {
    case M_COH: {
        const double a = pl[P_SRE][e], bb = pl[P_SIM][e];
        v = den > 0.0 ? sqrt(a * a + bb * bb) / den : 0.0;
        break;
    }
    case M_IMCOH: v = den > 0.0 ? pl[P_SIM][e] / den : 0.0; break;
    case M_PLV: {
        const double a = usum(P_URE), bb = usum(P_UIM);
        v = sqrt(a * a + bb * bb) / Kd;
        break;
    }
    case M_PLI: v = fabs(gsum()) / Kd; break;
    case M_USPLI: {
        const double pli = fabs(gsum()) / Kd;
        v = K >= 2 ? (Kd * pli * pli - 1.0) / (Kd - 1.0) : NAN;
        break;
    }
    case M_WPLI: {
        const double A = pl[P_A][e];
        v = A > 0.0 ? fabs(pl[P_SIM][e]) / A : 0.0;
        break;
    }
    case M_DSWPLI: {
        const double A = pl[P_A][e], Q = pl[P_Q][e], S = pl[P_SIM][e];
        const double dd = A * A - Q;
        v = K >= 2 ? (dd != 0.0 ? (S * S - Q) / dd : 0.0) : NAN;
        break;
    }
    default: break;
    }
    out[(size_t)b * P + idx] = (T)v;
}

template <typename T>
hipError_t launch_finalize_bins(const SessDev<T> &s, uint32_t metric, T *out, hipStream_t st)
{
    const size_t total = (size_t)s.ntiles * s.B * TILE_PAIRS;
    hipLaunchKernelGGL(k_finalize_bins<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, s,
                       metric, out);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched launches of the serving path: one launch drains a list of work
// items of many sessions (persistent-style grid-stride over the list).  Each
// item runs the same device body as the single-session kernels, so a
// session's result does not depend on what else shares the launch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void kb_spectra(const SessDev<float> *S, const int4 *items, int n)
{
    __shared__ float xs[SP_NODES][SP_CH + 1];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        SessDev<float> d = S[w.x];
        // trial w.w of the session's group: input rows N x ldx apart, ring slot
        // of that trial
        d.x = (const float *)d.x + (size_t)w.w * d.N * d.ldx;
        spectra_body(d, w.y, w.z, xs, (int)((d.ctl->pushed + w.w) % (long long)d.R));
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void kb_znorm(const SessDev<float> *S, const int4 *items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        SessDev<float> d = S[w.x];
        d.x = (const float *)d.x + (size_t)w.w * d.N * d.ldx;
        znorm_body(d, w.y, (int)((d.ctl->pushed + w.w) % (long long)d.R));
    }
}

__global__ __launch_bounds__(256) void kb_psd(const SessDev<float> *S, const int4 *items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        psd_body(S[w.x], w.y);
    }
}

template <uint32_t SPEC, int LT, int COR, int UG>
__global__ __launch_bounds__(PAIR_THREADS) void kb_pair_update(const SessDev<float> *S, const int4 *items, int n)
{
    extern __shared__ __align__(16) char lds[];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SessDev<float> &s = S[w.x];
        if (s.ctl->bad) continue;
        if (s.nt > 1) {
            const int tile = w.y / SLICES, sub = w.y % SLICES;
            const int2 tt = s.tiles[tile];
            const int R0 = tt.x * TILE + SLICE_ROWS * sub, J0 = tt.y * TILE;
            if (!(R0 >= s.N || R0 >= min(J0 + TILE - 1, s.N - 1)))
                pair_slice_mt<float, SPEC, LT, COR, UG>(
                    s, s.ctl->pushed, w.y, pair_chunk_bins_mt(s.B, s.L, 4, s.metrics & 0x7Fu, s.nt), lds);
        } else {
            pair_item<float, SPEC, LT, COR, UG>(s, w.y, s.ctl->pushed,
                                                pair_chunk_bins(s.B, s.L, 4, s.metrics & 0x7Fu), lds);
        }
        __syncthreads();
    }
}

__global__ void kb_commit(const SessDev<float> *S, int n)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i < n) {
        DevCtl *c = S[i].ctl;
        if (c->bad)
            c->rejected = c->rejected + 1;
        else
            c->pushed = c->pushed + S[i].nt;
        c->bad = 0;
    }
}

static unsigned persistent_grid(int n, int cap)
{
    return (unsigned)(n < cap ? (n > 0 ? n : 1) : cap);
}

hipError_t launch_batched(int which, const SessDev<float> *S, const int4 *items, int n, size_t lds,
                          hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    switch (which) {
    case FCX_B_SPECTRA:
        hipLaunchKernelGGL(kb_spectra, dim3(persistent_grid(n, 1 << 20)), dim3(256), 0, st, S, items, n);
        break;
    case FCX_B_ZNORM:
        hipLaunchKernelGGL(kb_znorm, dim3(persistent_grid(n, 1 << 20)), dim3(256), 0, st, S, items, n);
        break;
    case FCX_B_PSD:
        hipLaunchKernelGGL(kb_psd, dim3(persistent_grid(n, 1 << 20)), dim3(256), 0, st, S, items, n);
        break;
    case FCX_B_COMMIT:
        hipLaunchKernelGGL(kb_commit, dim3((n + 63) / 64), dim3(64), 0, st, S, n);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batched_pair(int cls, const SessDev<float> *S, const int4 *items, int n, size_t lds,
                               hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const bool ok = dispatch_pair_class(cls, [&](auto v) {
        using V = decltype(v);
        hipLaunchKernelGGL((kb_pair_update<V::spec, V::lt, V::cor, V::ug>), dim3(persistent_grid(n, 1 << 20)),
                           dim3(PAIR_THREADS), lds, st, S, items, n);
    });
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// HBM copy probe (16-byte vector loads/stores, grid-stride)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_copy_probe(float4 *__restrict__ dst, const float4 *__restrict__ src,
                                                    size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

hipError_t launch_copy_probe(void *dst, const void *src, int64_t n_bytes, hipStream_t st)
{
    const size_t n = (size_t)n_bytes / 16;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_copy_probe, dim3((unsigned)blocks), dim3(256), 0, st, (float4 *)dst,
                       (const float4 *)src, n);
    return hipGetLastError();
}

// Read-modify-write probe of the pair state layout of an FP32 all-8 session:
// per element four FP64 planes, two int32 planes and one int8 plane (41
// bytes), each element of each plane read and written once per launch, with
// the non-temporal hint the pair update uses on its planes.  It bounds what
// streaming the state alone can reach on this device.
__global__ __launch_bounds__(256) void k_rmw_probe(char *base, size_t n)
{
    double *d = (double *)base;
    int *q = (int *)(d + 4 * n);
    signed char *g = (signed char *)(q + 2 * n);
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        double v[4];
        int w[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(d + k * n + i);
#pragma unroll
        for (int k = 0; k < 2; ++k) w[k] = __builtin_nontemporal_load(q + k * n + i);
        const signed char c = __builtin_nontemporal_load(g + i);
#pragma unroll
        for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v[k] + 1.0, d + k * n + i);
#pragma unroll
        for (int k = 0; k < 2; ++k) __builtin_nontemporal_store(w[k] + 1, q + k * n + i);
        __builtin_nontemporal_store((signed char)(c + 1), g + i);
    }
}

hipError_t launch_rmw_probe(void *buf, int64_t n_elems, hipStream_t st)
{
    size_t blocks = ((size_t)n_elems + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_rmw_probe, dim3((unsigned)blocks), dim3(256), 0, st, (char *)buf, (size_t)n_elems);
    return hipGetLastError();
}

// Matrix-core probe: every wavefront runs `iters` rounds of independent
// MFMA chains on register operands (no memory traffic inside the loop) and
// writes one value per lane at the end so the work stays live.
//   kind 0: v_mfma_f32_16x16x4_f32, 8 chains (2048 flop each)
//   kind 1: v_mfma_f32_32x32x2_f32, 4 chains (4096 flop each)
//   kind 2: v_mfma_f32_16x16x32_bf16, 8 chains (16384 flop each)
constexpr int MFMA_PROBE_BLOCKS = 2048;
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int KIND> __global__ __launch_bounds__(256) void k_mfma_probe(float *out, int iters)
{
    const int lane = threadIdx.x & 63;
    const float a = 1.0f + lane * 1e-3f, b = 1.0f - lane * 1e-3f;
    float r = 0.f;
    if constexpr (KIND == 0) {
        floatx4 acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = (floatx4){0.f, 0.f, 0.f, (float)j};
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 8; ++j) r += acc[j][0] + acc[j][3];
    } else if constexpr (KIND == 1) {
        floatx16 acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[j][e] = (float)(j + e);
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) r += acc[j][0] + acc[j][15];
    } else {
        bf16x8 va, vb;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            va[e] = (__bf16)(a + e * 1e-2f);
            vb[e] = (__bf16)(b - e * 1e-2f);
        }
        floatx4 acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = (floatx4){0.f, 0.f, 0.f, (float)j};
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, acc[j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 8; ++j) r += acc[j][0] + acc[j][3];
    }
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = r;
}

hipError_t launch_mfma_probe(int kind, int iters, float *out, double *flops, hipStream_t st)
{
    const dim3 grid(MFMA_PROBE_BLOCKS), blk(256);
    const double waves = (double)MFMA_PROBE_BLOCKS * 4;
    switch (kind) {
    case 0:
        hipLaunchKernelGGL(k_mfma_probe<0>, grid, blk, 0, st, out, iters);
        *flops = waves * iters * 8 * 2048.0;
        break;
    case 1:
        hipLaunchKernelGGL(k_mfma_probe<1>, grid, blk, 0, st, out, iters);
        *flops = waves * iters * 4 * 4096.0;
        break;
    default:
        hipLaunchKernelGGL(k_mfma_probe<2>, grid, blk, 0, st, out, iters);
        *flops = waves * iters * 8 * 16384.0;
        break;
    }
    return hipGetLastError();
}

// explicit instantiations
#define FCX_INST(T)                                                                          \
    template hipError_t launch_spectra<T>(const SessDev<T> &, hipStream_t);                   \
    template hipError_t launch_psd<T>(const SessDev<T> &, hipStream_t);                       \
    template hipError_t launch_pair_update<T>(const SessDev<T> &, hipStream_t);               \
    template hipError_t launch_pair_rebuild<T>(const SessDev<T> &, long long, int, hipStream_t); \
    template hipError_t launch_psd_rebuild<T>(const SessDev<T> &, long long, int, hipStream_t); \
    template hipError_t launch_znorm<T>(const SessDev<T> &, hipStream_t);                     \
    template hipError_t launch_spectra_batch<T>(const SessDev<T> &, int, long long, hipStream_t); \
    template hipError_t launch_znorm_batch<T>(const SessDev<T> &, int, long long, hipStream_t);   \
    template hipError_t launch_finalize_bins<T>(const SessDev<T> &, uint32_t, T *, hipStream_t);
FCX_INST(float)
FCX_INST(double)

}  // namespace fcx
