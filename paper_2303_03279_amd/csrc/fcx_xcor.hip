// XCOR, the cross-correlation metric of the time-domain section, computed the
// way the implementation section describes it: spectra of the signals,
// their product, back to the time domain, then the largest correlation over
// the lags.  Per push, for the trial at the push's ring slot:
//
//   k_xcor_node   per node, from its z-scored samples z (zero mean, unit
//                 energy, already in the COR sample ring): the energies
//                 S(tau) = sum_{t >= tau} z(t)^2 for tau = 0..L (FP64 sums),
//                 stored as 1/sqrt(S(tau)) in FP32 (0 for S = 0), and the
//                 spectrum Z(f) = sum_t z(t) e^{-2 pi i f t/F}, f = 0..F/2,
//                 F a power of two >= M + L (FP64 sums, FP32 out)
//   k_xcor_pair   per pair tile row: for two columns at a time, the product
//                 spectra of the pairs are packed as H1 + i H2 (both
//                 Hermitian), one in-LDS inverse FFT of length F yields both
//                 circular correlations c1 = Re, c2 = Im, which equal the
//                 linear ones at lags -L..L since F >= M + L; then
//                   XCOR(tau)  = c(tau) / sqrt(S_i(tau) E_j)        tau = 0..L
//                   XCOR(-tau) = c(F - tau) / sqrt(S_j(tau) E_i)    tau = 1..L
//                 (0 where the product of energies is 0), the maximum over
//                 the 2L+1 lags, and the window sum: + this trial's maximum,
//                 - the evicted trial's maximum kept in a ring of per-trial
//                 values, so add and remove cancel exactly.
//
// The inverse FFT is a radix-4 Stockham (autosorting) transform, with one
// radix-2 stage when log2 F is odd, done by one wavefront in its own LDS
// buffer: every stage loads its butterflies' inputs, then stores the outputs
// in place; the wavefronts of a workgroup share the row node's data and the
// twiddles and never wait for each other.
#include "fcx_device.h"

#include <math.h>

#pragma clang fp contract(off)

namespace fcx {

constexpr int XT = 256;   // threads of both XCOR kernels

// ---------------------------------------------------------------------------
// node pass: one workgroup per node
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(XT) void k_xcor_node(SessDev<T> s)
{
    __shared__ float z[XCOR_MAX_F];
    __shared__ double suf[XCOR_MAX_F];
    if (s.ctl->bad) return;
    const int node = blockIdx.x, tid = threadIdx.x;
    const int M = s.M, L = s.xL, F = s.xF;
    const PushView pv = push_view(s, s.ctl->pushed);
    const float *zr = s.zring + ((size_t)pv.slot_new * s.N + node) * s.Mz;
    for (int t = tid; t < M; t += XT) z[t] = zr[t];
    __syncthreads();
    if (tid == 0) {
        double acc = 0.0;
        for (int t = M - 1; t >= 0; --t) {
            acc += (double)z[t] * (double)z[t];
            suf[t] = acc;
        }
    }
    __syncthreads();
    float *so = s.xsuf + (size_t)node * (L + 1);
    for (int t = tid; t <= L; t += XT) so[t] = suf[t] > 0.0 ? (float)(1.0 / sqrt(suf[t])) : 0.f;
    float2 *xo = s.xspec + (size_t)node * (F / 2 + 1);
    const unsigned fm = (unsigned)F - 1u;
    for (int f = tid; f <= F / 2; f += XT) {
        double re = 0.0, im = 0.0;
        for (int t = 0; t < M; ++t) {
            const float2 w = s.xtw[((unsigned)f * (unsigned)t) & fm];
            re += (double)z[t] * (double)w.x;
            im += (double)z[t] * (double)w.y;
        }
        xo[f] = make_float2((float)re, (float)im);
    }
}

// ---------------------------------------------------------------------------
// pair pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place inverse DFT (no 1/F) of Z[F] in LDS by one wavefront.  The LDS
// operations of a wavefront are performed in order, so a stage's loads (all
// lanes) precede its stores; the wave barriers keep the compiler from moving
// LDS accesses across the phase boundaries.
template <int F>
__device__ __forceinline__ void ifft_wave(float2 *Z, const float2 *tw, int lane)
{
    constexpr int NB4 = F / 4;                           // radix-4 butterflies per stage
    constexpr int PER4 = NB4 / 64;
#pragma unroll
    for (int Ns = 1; Ns * 4 <= F; Ns *= 4) {
        float2 v[PER4][4];
        const int step = F / (4 * Ns);
#pragma unroll
        for (int q = 0; q < PER4; ++q) {
            const int j = lane + q * 64;
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float2 a = Z[j + r * NB4];
                if (r && Ns > 1) {                       // the first stage's twiddles are 1
                    float2 w = tw[r * k * step];
                    w.y = -w.y;                          // inverse: exp(+2 pi i m / F)
                    a = cmul(a, w);
                }
                v[q][r] = a;
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < PER4; ++q) {
            const int j = lane + q * 64;
            const int k = j & (Ns - 1);
            const float2 a0 = v[q][0], a1 = v[q][1], a2 = v[q][2], a3 = v[q][3];
            const float2 t0 = make_float2(a0.x + a2.x, a0.y + a2.y);
            const float2 t1 = make_float2(a0.x - a2.x, a0.y - a2.y);
            const float2 t2 = make_float2(a1.x + a3.x, a1.y + a3.y);
            const float2 d = make_float2(a1.x - a3.x, a1.y - a3.y);
            const float2 t3 = make_float2(-d.y, d.x);    // +i (a1 - a3)
            const int o = (j / Ns) * Ns * 4 + k;
            Z[o] = make_float2(t0.x + t2.x, t0.y + t2.y);
            Z[o + Ns] = make_float2(t1.x + t3.x, t1.y + t3.y);
            Z[o + 2 * Ns] = make_float2(t0.x - t2.x, t0.y - t2.y);
            Z[o + 3 * Ns] = make_float2(t1.x - t3.x, t1.y - t3.y);
        }
        __builtin_amdgcn_wave_barrier();
    }
    constexpr bool odd = (F & 0x55555555) == 0;          // log2 F odd: a last radix-2 stage
    if constexpr (odd) {
        constexpr int NB2 = F / 2;
        constexpr int PER2 = NB2 / 64;
        float2 v0[PER2], v1[PER2];
#pragma unroll
        for (int q = 0; q < PER2; ++q) {
            const int j = lane + q * 64;
            float2 w = tw[j];
            w.y = -w.y;
            v0[q] = Z[j];
            v1[q] = cmul(Z[j + NB2], w);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < PER2; ++q) {
            const int j = lane + q * 64;
            Z[j] = make_float2(v0[q].x + v1[q].x, v0[q].y + v1[q].y);
            Z[j + NB2] = make_float2(v0[q].x - v1[q].x, v0[q].y - v1[q].y);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// waves per workgroup of the pair kernel (each has its own transform
// buffer), and whether the twiddles are staged in LDS (up to F = 1024; the
// 2048-point kernel reads them from the cache to keep three workgroups per CU)
template <int F> constexpr int xcor_waves() { return F >= 2048 ? 2 : 4; }
template <int F> constexpr bool xcor_tw_lds() { return F <= 1024; }

// One workgroup per (tile, row of the tile): row node i against the tile's
// columns j > i.  The row's spectrum, energies and the twiddles are shared in
// LDS; each wavefront takes two columns at a time into its own transform.
// Up to F = 1024 the global loads of a job are issued early: this job's
// column energies and the next job's column spectra go into registers before
// the transform, so their latency overlaps it.  NL = lag registers per lane:
// (L + 1) <= 64 NL.
template <int F> constexpr bool xcor_prefetch() { return F <= 1024; }

template <typename T, int F, int NL>
__global__ __launch_bounds__(64 * xcor_waves<F>()) __attribute__((amdgpu_waves_per_eu(F == 1024 && NL == 8 ? 3 : 1)))
void k_xcor_pair(SessDev<T> s)
{
    constexpr int NW = xcor_waves<F>();
    constexpr int NF = (F / 2 + 1 + 63) / 64;   // spectrum bins per lane
    __shared__ float2 Zw[NW][F];
    __shared__ float2 Rsp[F / 2 + 1];
    __shared__ float Rsuf[F];
    __shared__ float2 tws[xcor_tw_lds<F>() ? F : 1];
    if (s.ctl->bad) return;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int tile = item / TILE, r = item % TILE;
    const int2 tt = s.tiles[tile];
    const int N = s.N, L = s.xL, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i = tt.x * TILE + r, J0 = tt.y * TILE;
    if (i >= N) return;
    const int jlo = max(J0, i + 1), jhi = min(J0 + TILE, N);
    if (jlo >= jhi) return;
    const PushView pv = push_view(s, s.ctl->pushed);
    for (int f = tid; f <= F / 2; f += 64 * NW) Rsp[f] = s.xspec[(size_t)i * (F / 2 + 1) + f];
    for (int t = tid; t <= L; t += 64 * NW) Rsuf[t] = s.xsuf[(size_t)i * (L + 1) + t];
    if constexpr (xcor_tw_lds<F>())
        for (int m = tid; m < F; m += 64 * NW) tws[m] = s.xtw[m];
    __syncthreads();
    float2 *Z = Zw[wv];
    const float rEi = Rsuf[0];   // 1/sqrt of node i's energy (0 if none)
    const float invF = 1.0f / (float)F;
    const size_t TP = (size_t)s.ntiles * TILE_PAIRS;
    const size_t P = (size_t)N * (N - 1) / 2;
    // column spectra of a job (j, j + 1 or none) into registers
    float2 b1[xcor_prefetch<F>() ? NF : 1], b2[xcor_prefetch<F>() ? NF : 1];
    auto load_spec = [&](int j) {
        const int j2 = j + 1 < jhi ? j + 1 : -1;
        const float2 *c1p = s.xspec + (size_t)j * (F / 2 + 1);
        const float2 *c2p = s.xspec + (size_t)(j2 >= 0 ? j2 : j) * (F / 2 + 1);
#pragma unroll
        for (int q = 0; q < NF; ++q) {
            const int f = lane + 64 * q;
            b1[q] = make_float2(0.f, 0.f);
            b2[q] = b1[q];
            if (f <= F / 2) {
                b1[q] = c1p[f];
                if (j2 >= 0) b2[q] = c2p[f];
            }
        }
    };
    // Z = H1 + i H2 over the full circle, H = X_i conj(X_j) (Hermitian)
    auto put = [&](int f, float2 a, float2 c1, float2 c2) {
        const float h1r = a.x * c1.x + a.y * c1.y, h1i = a.y * c1.x - a.x * c1.y;
        const float h2r = a.x * c2.x + a.y * c2.y, h2i = a.y * c2.x - a.x * c2.y;
        Z[f] = make_float2(h1r - h2i, h1i + h2r);
        if (f > 0 && f < F / 2) Z[F - f] = make_float2(h1r + h2i, h2r - h1i);
    };
    int j = jlo + 2 * wv;
    if constexpr (xcor_prefetch<F>())
        if (j < jhi) load_spec(j);
    for (; j < jhi; j += 2 * NW) {
        const int j2 = j + 1 < jhi ? j + 1 : -1;
        if constexpr (xcor_prefetch<F>()) {
#pragma unroll
            for (int q = 0; q < NF; ++q) {
                const int f = lane + 64 * q;
                if (f <= F / 2) put(f, Rsp[f], b1[q], b2[q]);
            }
        } else {
            const float2 *c1p = s.xspec + (size_t)j * (F / 2 + 1);
            const float2 *c2p = s.xspec + (size_t)(j2 >= 0 ? j2 : j) * (F / 2 + 1);
            for (int f = lane; f <= F / 2; f += 64)
                put(f, Rsp[f], c1p[f], j2 >= 0 ? c2p[f] : make_float2(0.f, 0.f));
        }
        // this job's column energies, then the next job's spectra
        const float *s1 = s.xsuf + (size_t)j * (L + 1);
        const float *s2 = s.xsuf + (size_t)(j2 >= 0 ? j2 : j) * (L + 1);
        const float rE1 = s1[0], rE2 = j2 >= 0 ? s2[0] : 0.f;
        float e1[xcor_prefetch<F>() ? NL : 1], e2[xcor_prefetch<F>() ? NL : 1];
        if constexpr (xcor_prefetch<F>()) {
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int tau = lane + 64 * q;
                e1[q] = tau <= L ? s1[tau] : 0.f;
                e2[q] = tau <= L && j2 >= 0 ? s2[tau] : 0.f;
            }
        }
        if constexpr (xcor_prefetch<F>())
            if (j + 2 * NW < jhi) load_spec(j + 2 * NW);
        __builtin_amdgcn_wave_barrier();
        ifft_wave<F>(Z, xcor_tw_lds<F>() ? tws : s.xtw, lane);
        // largest XCOR over the lags, both pairs
        // XCOR = c / F * (1/sqrt S_advanced(tau)) * (1/sqrt E_other)
        float best1 = -INFINITY, best2 = -INFINITY;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int tau = lane + 64 * q;
            if (tau <= L) {
                const float2 p = Z[tau];
                const float ri = Rsuf[tau];
                best1 = fmaxf(best1, p.x * invF * ri * rE1);
                best2 = fmaxf(best2, p.y * invF * ri * rE2);
                if (tau > 0) {
                    const float2 qv = Z[F - tau];
                    float f1, f2;
                    if constexpr (xcor_prefetch<F>()) {
                        f1 = e1[q];
                        f2 = e2[q];
                    } else {
                        f1 = s1[tau];
                        f2 = j2 >= 0 ? s2[tau] : 0.f;
                    }
                    best1 = fmaxf(best1, qv.x * invF * f1 * rEi);
                    if (j2 >= 0) best2 = fmaxf(best2, qv.y * invF * f2 * rEi);
                }
            }
        }
        best1 = wave_max(best1);
        best2 = wave_max(best2);
        if (lane < 2) {
            const int jj = lane == 0 ? j : j2;
            if (jj >= 0) {
                const float v = lane == 0 ? best1 : best2;
                const size_t e = (size_t)tile * TILE_PAIRS + (size_t)r * TILE + (jj - J0);
                double sum = s.xsum[e] + (double)v;
                if (pv.has_old) sum = sum - (double)s.xval[(size_t)pv.slot_old * TP + e];
                s.xsum[e] = sum;
                s.xval[(size_t)pv.slot_new * TP + e] = v;
                const size_t idx = (size_t)i * (2 * (size_t)N - i - 1) / 2 + (size_t)(jj - i - 1);
                s.out[8 * P + idx] = (T)(sum / (double)pv.K);
            }
        }
        __builtin_amdgcn_wave_barrier();   // Z is rebuilt for the next columns
    }
}

template <typename T> hipError_t launch_xcor(const SessDev<T> &s, hipStream_t st)
{
    hipLaunchKernelGGL(k_xcor_node<T>, dim3(s.N), dim3(XT), 0, st, s);
    const dim3 grid((unsigned)(s.ntiles * TILE));
    // lag registers: half the transform when the lags fit, else all of it
    const bool half = s.xL + 1 <= s.xF / 2;
    const dim3 b256(64 * xcor_waves<256>()), b512(64 * xcor_waves<512>()), b1k(64 * xcor_waves<1024>()),
        b2k(64 * xcor_waves<2048>());
    switch (s.xF) {
    case 256:
        if (half) hipLaunchKernelGGL((k_xcor_pair<T, 256, 2>), grid, b256, 0, st, s);
        else hipLaunchKernelGGL((k_xcor_pair<T, 256, 4>), grid, b256, 0, st, s);
        break;
    case 512:
        if (half) hipLaunchKernelGGL((k_xcor_pair<T, 512, 4>), grid, b512, 0, st, s);
        else hipLaunchKernelGGL((k_xcor_pair<T, 512, 8>), grid, b512, 0, st, s);
        break;
    case 1024:
        if (half) hipLaunchKernelGGL((k_xcor_pair<T, 1024, 8>), grid, b1k, 0, st, s);
        else hipLaunchKernelGGL((k_xcor_pair<T, 1024, 16>), grid, b1k, 0, st, s);
        break;
    case 2048:
        if (half) hipLaunchKernelGGL((k_xcor_pair<T, 2048, 16>), grid, b2k, 0, st, s);
        else hipLaunchKernelGGL((k_xcor_pair<T, 2048, 32>), grid, b2k, 0, st, s);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_xcor<float>(const SessDev<float> &, hipStream_t);
template hipError_t launch_xcor<double>(const SessDev<double> &, hipStream_t);

}  // namespace fcx
