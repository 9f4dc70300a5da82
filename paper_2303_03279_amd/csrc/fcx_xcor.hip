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
//                 F a power of two >= M + L (FP64 sums and phasors, FP32 out)
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
// The inverse FFT is a mixed-radix Stockham (autosorting) transform done by
// one wavefront in its own LDS buffer: three passes of radix 16, 16 and 4 at
// F = 1024 (radix-16 butterflies in registers), each loading its
// butterflies' inputs, then storing the outputs in place; the wavefronts of
// a workgroup share the row node's data and the twiddles and never wait for
// each other.
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
    // bin f: sum_t z(t) exp(-2 pi i f t / F), the phasor advanced by one
    // FP64 rotation per sample and restarted from its exact value at the
    // start of each of XSEG segments (independent chains; the rounding of
    // the rotation grows by at most a few hundred FP64 ulps).  The bins
    // 1..F/2-1 go round the threads; f = 0 and f = F/2, whose phasors are
    // exactly +-1, are plain sums over the same segments, taken by the last
    // thread, which has the fewest rotating bins
    constexpr int XSEG = 4;
    float2 *xo = s.xspec + (size_t)node * (F / 2 + 1);
    const int seg = (M + XSEG - 1) / XSEG;
    for (int f = 1 + tid; f < F / 2; f += XT) {
        double sr, ci0;
        sincospi(-2.0 * (double)f / (double)F, &sr, &ci0);   // one-sample rotation (cos ci0, sin sr)
        double re[XSEG], im[XSEG], cr[XSEG], cs[XSEG];
#pragma unroll
        for (int g = 0; g < XSEG; ++g) {
            const int m = (int)(((long long)f * (long long)(g * seg)) % F);
            sincospi(-2.0 * (double)m / (double)F, &cs[g], &cr[g]);
            re[g] = 0.0;
            im[g] = 0.0;
        }
        for (int u = 0; u < seg; ++u) {
#pragma unroll
            for (int g = 0; g < XSEG; ++g) {
                const int t = g * seg + u;
                if (t < M) {
                    const double v = (double)z[t];
                    re[g] += v * cr[g];
                    im[g] += v * cs[g];
                    const double nr = cr[g] * ci0 - cs[g] * sr;
                    cs[g] = cr[g] * sr + cs[g] * ci0;
                    cr[g] = nr;
                }
            }
        }
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int g = 0; g < XSEG; ++g) {
            tr += re[g];
            ti += im[g];
        }
        xo[f] = make_float2((float)tr, (float)ti);
    }
    if (tid == XT - 1) {
        double d[XSEG], q[XSEG];   // f = 0: sum z(t); f = F/2: sum (-1)^t z(t)
#pragma unroll
        for (int g = 0; g < XSEG; ++g) {
            d[g] = 0.0;
            q[g] = 0.0;
            for (int t = g * seg; t < min(M, (g + 1) * seg); ++t) {
                const double v = (double)z[t];
                d[g] += v;
                q[g] += (t & 1) ? -v : v;
            }
        }
        double td = 0.0, tq = 0.0;
#pragma unroll
        for (int g = 0; g < XSEG; ++g) {
            td += d[g];
            tq += q[g];
        }
        xo[0] = make_float2((float)td, 0.f);
        xo[F / 2] = make_float2((float)tq, 0.f);
        // suffix energies, FP64, one thread (deterministic order)
        double acc = 0.0;
        for (int t = M - 1; t >= 0; --t) {
            acc += (double)z[t] * (double)z[t];
            suf[t] = acc;
        }
    }
    __syncthreads();
    float *so = s.xsuf + (size_t)node * (L + 1);
    for (int t = tid; t <= L; t += XT) so[t] = suf[t] > 0.0 ? (float)(1.0 / sqrt(suf[t])) : 0.f;
}

// ---------------------------------------------------------------------------
// pair pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// A transform buffer holds element m at m + m / 32: the pad after every 32
// elements (256 bytes) spreads the strided stores of the early passes over
// the LDS banks.
constexpr int XPAD_SHIFT = 5;
__host__ __device__ constexpr int xpad(int m) { return m + (m >> XPAD_SHIFT); }
template <int F> constexpr int xbuf_len() { return F + (F >> XPAD_SHIFT); }

// exp(+2 pi i m / 16), m = 0..7
__constant__ const float W16_RE[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                      0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
__constant__ const float W16_IM[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                                      1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};

// In-register inverse DFT of R = 4, 8 or 16 points: y_m = sum_r v_r
// exp(+2 pi i r m / R), split into even and odd halves down to radix 4.
template <int R>
__device__ __forceinline__ void idft_reg(float2 (&v)[R])
{
    if constexpr (R == 4) {
        const float2 t0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        const float2 t1 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        const float2 t2 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        const float2 d = make_float2(v[1].x - v[3].x, v[1].y - v[3].y);
        const float2 t3 = make_float2(-d.y, d.x);    // +i (v1 - v3)
        v[0] = make_float2(t0.x + t2.x, t0.y + t2.y);
        v[1] = make_float2(t1.x + t3.x, t1.y + t3.y);
        v[2] = make_float2(t0.x - t2.x, t0.y - t2.y);
        v[3] = make_float2(t1.x - t3.x, t1.y - t3.y);
    } else {
        constexpr int H = R / 2;
        float2 e[H], o[H];
#pragma unroll
        for (int m = 0; m < H; ++m) {
            e[m] = v[2 * m];
            o[m] = v[2 * m + 1];
        }
        idft_reg<H>(e);
        idft_reg<H>(o);
#pragma unroll
        for (int m = 0; m < H; ++m) {
            const int w = m * (16 / R);                  // exp(+2 pi i m / R) = W16^(16 m / R)
            const float2 t = cmul(o[m], make_float2(W16_RE[w], W16_IM[w]));
            v[m] = make_float2(e[m].x + t.x, e[m].y + t.y);
            v[m + H] = make_float2(e[m].x - t.x, e[m].y - t.y);
        }
    }
}

// One pass of radix R of the in-place Stockham (autosorting) inverse FFT by
// one wavefront; NS = product of the radices before it.  Butterfly j takes
// Z[j + r F/R] (times exp(+2 pi i r k / (R NS)), k = j mod NS) and writes
// its R-point DFT to Z[(j / NS) NS R + k + m NS].  A wavefront's LDS
// operations are performed in order, so all loads of the pass precede its
// stores; the wave barriers keep the compiler from moving LDS accesses
// across the phase boundaries.  With the pad every 32 elements both address
// patterns are one base plus constants (F / R and NS are multiples of 32, or
// NS < 32 with k + (m NS mod 32) < 32).
template <int F, int R, int NS>
__device__ __forceinline__ void xpass(float2 *Z, const float2 *tw, int lane)
{
    constexpr int NB = F / R;                   // butterflies
    constexpr int PER = NB / 64;                // per lane
    constexpr int STEP = F / (R * NS);          // twiddle stride
    static_assert(NB % 64 == 0 && NB % 32 == 0, "butterflies per lane");
    float2 v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = lane + 64 * q;
        const int k = j & (NS - 1);
        const float2 *zi = Z + xpad(j);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float2 a = zi[r * NB + ((r * NB) >> XPAD_SHIFT)];
            if (NS > 1 && r) {
                float2 w = tw[r * k * STEP];
                w.y = -w.y;                             // inverse: exp(+2 pi i m / F)
                a = cmul(a, w);
            }
            v[q][r] = a;
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = lane + 64 * q;
        const int k = j & (NS - 1);
        idft_reg<R>(v[q]);
        float2 *zo = Z + xpad((j / NS) * NS * R + k);
#pragma unroll
        for (int m = 0; m < R; ++m) zo[m * NS + ((m * NS) >> XPAD_SHIFT)] = v[q][m];
    }
    __builtin_amdgcn_wave_barrier();
}

// In-place inverse DFT (no 1/F) of the padded Z[F] in LDS by one wavefront:
// radices 4-4-4-4 (F = 256), 8-8-8 (512), 16-16-4 (1024), 16-16-8 (2048).
template <int F>
__device__ __forceinline__ void ifft_wave(float2 *Z, const float2 *tw, int lane)
{
    if constexpr (F == 256) {
        xpass<F, 4, 1>(Z, tw, lane);
        xpass<F, 4, 4>(Z, tw, lane);
        xpass<F, 4, 16>(Z, tw, lane);
        xpass<F, 4, 64>(Z, tw, lane);
    } else if constexpr (F == 512) {
        xpass<F, 8, 1>(Z, tw, lane);
        xpass<F, 8, 8>(Z, tw, lane);
        xpass<F, 8, 64>(Z, tw, lane);
    } else if constexpr (F == 1024) {
        xpass<F, 16, 1>(Z, tw, lane);
        xpass<F, 16, 16>(Z, tw, lane);
        xpass<F, 4, 256>(Z, tw, lane);
    } else {
        static_assert(F == 2048, "transform length");
        xpass<F, 16, 1>(Z, tw, lane);
        xpass<F, 16, 16>(Z, tw, lane);
        xpass<F, 8, 256>(Z, tw, lane);
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
// the transform, so their latency overlaps it.  NL = F / 128 lag registers
// per lane (L + 1 <= F / 2).
template <int F> constexpr bool xcor_prefetch() { return F <= 1024; }

template <typename T, int F, int NL>
__global__ __launch_bounds__(64 * xcor_waves<F>()) __attribute__((amdgpu_waves_per_eu(F == 1024 ? 3 : 1)))
void k_xcor_pair(SessDev<T> s)
{
    constexpr int NW = xcor_waves<F>();
    constexpr int NF = (F / 2 + 1 + 63) / 64;   // spectrum bins per lane
    __shared__ float2 Zw[NW][xbuf_len<F>()];
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
        const float h1r = __builtin_fmaf(a.x, c1.x, a.y * c1.y), h1i = __builtin_fmaf(a.y, c1.x, -(a.x * c1.y));
        const float h2r = __builtin_fmaf(a.x, c2.x, a.y * c2.y), h2i = __builtin_fmaf(a.y, c2.x, -(a.x * c2.y));
        Z[xpad(f)] = make_float2(h1r - h2i, h1i + h2r);
        if (f > 0 && f < F / 2) Z[xpad(F - f)] = make_float2(h1r + h2i, h2r - h1i);
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
                const float2 p = Z[xpad(tau)];
                const float ri = Rsuf[tau];
                best1 = fmaxf(best1, p.x * invF * ri * rE1);
                best2 = fmaxf(best2, p.y * invF * ri * rE2);
                if (tau > 0) {
                    const float2 qv = Z[xpad(F - tau)];
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
    // lag registers: L <= M - 1 and M + L <= F give L + 1 <= F / 2
    if (2 * (s.xL + 1) > s.xF) return hipErrorInvalidValue;
    switch (s.xF) {
    case 256: hipLaunchKernelGGL((k_xcor_pair<T, 256, 2>), grid, dim3(64 * xcor_waves<256>()), 0, st, s); break;
    case 512: hipLaunchKernelGGL((k_xcor_pair<T, 512, 4>), grid, dim3(64 * xcor_waves<512>()), 0, st, s); break;
    case 1024: hipLaunchKernelGGL((k_xcor_pair<T, 1024, 8>), grid, dim3(64 * xcor_waves<1024>()), 0, st, s); break;
    case 2048: hipLaunchKernelGGL((k_xcor_pair<T, 2048, 16>), grid, dim3(64 * xcor_waves<2048>()), 0, st, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_xcor<float>(const SessDev<float> &, hipStream_t);
template hipError_t launch_xcor<double>(const SessDev<double> &, hipStream_t);

}  // namespace fcx
